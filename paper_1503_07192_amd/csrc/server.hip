// Continuous-batching query server on a resident index (declarations and
// contracts in include/spq.h).  Batched answering of many queries at once is
// the extension the paper leaves to future work (Section 5); each launch is
// Algorithm 2 over a batch of pairs.
//
// Requests (host arrays of query pairs) queue in arrival order.  A worker
// thread owns the device side: a fixed set of slots (one HIP stream each) and
// one device pool plus one pinned host pool of the memory budget, carved by a
// first-fit arena that gates every launch (a launch starts only once its
// buffers are allocated there).  Whenever a slot is free and the arena can
// hold a launch, the requests at the head of the queue are coalesced into one
// launch of spq_query_batch: as many pairs as fit in the slot's capacity and
// in the largest free region, a request cut only when the room left cannot
// hold it whole.  Requests that arrive while others run are admitted as soon
// as a slot and memory free up, and their launches overlap on the device.
// The worker polls each slot's event and scatters the answers into the
// requests' own output arrays; a request's latency is the time its last
// answers were scattered minus the time it was submitted.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/spq.h"
#include "spq_internal.h"

namespace {

constexpr int64_t PAIR_BYTES = 12;  // v1, v2, answer as int32
constexpr int64_t ALIGN = 256;

spq_status fail(spq_status s, const std::string& msg) {
  return static_cast<spq_status>(spq::set_error(s, msg.c_str()));
}

// First-fit allocator of byte ranges in [0, size), ALIGN-byte units.
class Arena {
 public:
  explicit Arena(int64_t size) {
    size -= size % ALIGN;
    if (size > 0) holes_.emplace(0, size);
  }
  int64_t largest() const {
    int64_t b = 0;
    for (const auto& h : holes_) b = std::max(b, h.second);
    return b;
  }
  int64_t alloc(int64_t bytes) {  // offset, or -1 when no hole is large enough
    bytes = (std::max<int64_t>(bytes, 1) + ALIGN - 1) / ALIGN * ALIGN;
    for (auto it = holes_.begin(); it != holes_.end(); ++it) {
      if (it->second < bytes) continue;
      const int64_t off = it->first, len = it->second;
      holes_.erase(it);
      if (len > bytes) holes_.emplace(off + bytes, len - bytes);
      live_[off] = bytes;
      return off;
    }
    return -1;
  }
  void free(int64_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return;
    int64_t lo = off, len = it->second;
    live_.erase(it);
    auto nx = holes_.lower_bound(lo);
    if (nx != holes_.end() && lo + len == nx->first) {  // merge with the next hole
      len += nx->second;
      nx = holes_.erase(nx);
    }
    if (nx != holes_.begin()) {  // and with the previous one
      auto pv = std::prev(nx);
      if (pv->first + pv->second == lo) {
        lo = pv->first;
        len += pv->second;
        holes_.erase(pv);
      }
    }
    holes_.emplace(lo, len);
  }

 private:
  std::map<int64_t, int64_t> holes_;  // offset -> length, disjoint, unmerged never adjacent
  std::map<int64_t, int64_t> live_;   // offset -> length
};

struct Req {
  int64_t q = 0;
  const int32_t *v1 = nullptr, *v2 = nullptr;
  int32_t* out = nullptr;
  int64_t issued = 0, filled = 0;  // pairs handed to launches / answered
  double arrival = 0, done_at = -1;
  bool done = false;
};

struct Part {
  Req* r;
  int64_t lo, hi;  // pairs [lo, hi) of r
};

struct Launch {
  bool busy = false;
  int64_t off = 0, q = 0;  // arena offset (bytes) and pairs
  std::vector<Part> parts;
};

}  // namespace

struct spq_server {
  const spq_index* idx = nullptr;
  int device = 0;
  int32_t slots = 0;
  int64_t slot_pairs = 0;
  int32_t* d_pool = nullptr;  // device pool
  int32_t* h_pool = nullptr;  // pinned host pool, same size and offsets
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<Launch> inflight;  // per slot; worker only
  std::unique_ptr<Arena> arena;  // worker only
  std::chrono::steady_clock::time_point t0;
  std::thread worker;

  // everything below under mu
  std::mutex mu;
  std::condition_variable cv;  // submissions, completions, failure, stop
  std::deque<Req*> queue;      // requests with pairs not yet handed to a launch
  std::map<int64_t, std::unique_ptr<Req>> reqs;  // ticket -> request, until collected
  int64_t next_ticket = 1;
  bool stop = false;
  spq_status failed = SPQ_OK;  // first device error; the server stops serving
  std::string failure;
  int64_t launches = 0, pairs = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void set_failed(spq_status st, const std::string& msg) {
    std::lock_guard<std::mutex> lock(mu);
    if (failed == SPQ_OK) {
      failed = st;
      failure = msg;
    }
    cv.notify_all();
  }
  bool admit_one();
  bool complete();
  void run();
};

// One launch from the head of the queue on a free slot; false if none starts.
bool spq_server::admit_one() {
  int slot = -1;
  for (int s = 0; s < slots && slot < 0; s++)
    if (!inflight[s].busy) slot = s;
  if (slot < 0) return false;
  const int64_t room = std::min(slot_pairs, arena->largest() / PAIR_BYTES);
  if (room <= 0) return false;
  Launch& L = inflight[slot];
  int64_t take = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (failed != SPQ_OK) return false;
    while (!queue.empty() && take < room) {
      Req* r = queue.front();
      const int64_t left = r->q - r->issued;
      if (take > 0 && left > room - take) break;
      const int64_t cnt = std::min(left, room - take);
      L.parts.push_back({r, r->issued, r->issued + cnt});
      r->issued += cnt;
      take += cnt;
      if (r->issued < r->q) break;
      queue.pop_front();
    }
  }
  if (take == 0) return false;
  // fits: largest() is a multiple of ALIGN and take * PAIR_BYTES <= largest()
  const int64_t off = arena->alloc(take * PAIR_BYTES);
  L.busy = true;
  L.off = off;
  L.q = take;
  int32_t* h = h_pool + off / 4;
  int32_t* d = d_pool + off / 4;
  int64_t pos = 0;
  for (const Part& p : L.parts) {
    std::memcpy(h + pos, p.r->v1 + p.lo, sizeof(int32_t) * (p.hi - p.lo));
    std::memcpy(h + take + pos, p.r->v2 + p.lo, sizeof(int32_t) * (p.hi - p.lo));
    pos += p.hi - p.lo;
  }
  hipStream_t s = streams[slot];
  spq_status st = SPQ_OK;
  std::string msg;
  hipError_t e = hipMemcpyAsync(d, h, sizeof(int32_t) * 2 * take, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    st = spq_query_batch(idx, take, d, d + take, d + 2 * take, s);
    if (st != SPQ_OK) msg = spq_last_error();
  }
  if (e == hipSuccess && st == SPQ_OK)
    e = hipMemcpyAsync(h + 2 * take, d + 2 * take, sizeof(int32_t) * take, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && st == SPQ_OK) e = hipEventRecord(events[slot], s);
  if (e != hipSuccess || st != SPQ_OK) {
    // nothing of this launch will be scattered: wait for what was queued, then drop it
    (void)hipStreamSynchronize(s);
    arena->free(off);
    L.parts.clear();
    L.busy = false;
    if (st == SPQ_OK) {
      st = SPQ_EDEVICE;
      msg = std::string("server launch: ") + hipGetErrorString(e);
    }
    set_failed(st, msg);
    return false;
  }
  std::lock_guard<std::mutex> lock(mu);
  launches++;
  pairs += take;
  return true;
}

// Scatters the answers of the launches that finished; true if any did.
bool spq_server::complete() {
  bool any = false;
  for (int s = 0; s < slots; s++) {
    Launch& L = inflight[s];
    if (!L.busy) continue;
    const hipError_t e = hipEventQuery(events[s]);
    if (e == hipErrorNotReady) continue;
    if (e == hipSuccess) {
      const int32_t* ans = h_pool + L.off / 4 + 2 * L.q;
      const double t = now();
      int64_t pos = 0;
      std::lock_guard<std::mutex> lock(mu);
      for (const Part& p : L.parts) {
        std::memcpy(p.r->out + p.lo, ans + pos, sizeof(int32_t) * (p.hi - p.lo));
        pos += p.hi - p.lo;
        p.r->filled += p.hi - p.lo;
        if (p.r->filled == p.r->q) {
          p.r->done_at = t;
          p.r->done = true;
        }
      }
    } else {
      set_failed(SPQ_EDEVICE, std::string("server launch: ") + hipGetErrorString(e));
    }
    arena->free(L.off);
    L.parts.clear();
    L.busy = false;
    any = true;
  }
  if (any) cv.notify_all();
  return any;
}

void spq_server::run() {
  const hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) set_failed(SPQ_EDEVICE, std::string("server: ") + hipGetErrorString(e));
  for (;;) {
    const bool progressed = complete() | admit_one();
    while (admit_one()) {
    }
    bool idle = true;
    for (const Launch& L : inflight) idle = idle && !L.busy;
    std::unique_lock<std::mutex> lock(mu);
    // stop once every submitted pair is answered (or the server failed)
    if (stop && idle && (queue.empty() || failed != SPQ_OK)) break;
    if (idle && (queue.empty() || failed != SPQ_OK)) {
      cv.wait(lock, [&] { return stop || (!queue.empty() && failed == SPQ_OK); });
    } else if (!progressed) {
      lock.unlock();
      std::this_thread::yield();  // launches in flight: poll their events again
    }
  }
}

extern "C" {

spq_status spq_server_create(const spq_index* idx, int32_t slots, int64_t slot_pairs,
                             int64_t mem_bytes, spq_server** out) {
  if (!out) return fail(SPQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!idx) return fail(SPQ_EINVAL, "index is NULL");
  if (slots < 1 || slots > 64) return fail(SPQ_EINVAL, "slots must be in [1, 64]");
  if (slot_pairs < 1) return fail(SPQ_EINVAL, "slot_pairs < 1");
  if (mem_bytes < ALIGN || mem_bytes > (int64_t(1) << 36))
    return fail(SPQ_EINVAL, "mem_bytes must be in [256 B, 64 GiB]");
  spq_stats st;
  const spq_status ss = spq_index_stats(idx, &st);  // also waits for the build
  if (ss != SPQ_OK) return ss;
  std::unique_ptr<spq_server> S(new spq_server());
  S->idx = idx;
  S->slots = slots;
  S->slot_pairs = slot_pairs;
  const int64_t mem = mem_bytes - mem_bytes % ALIGN;
  S->arena.reset(new Arena(mem));
  S->inflight.resize(slots);
  hipError_t e = hipGetDevice(&S->device);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&S->d_pool), mem);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S->h_pool), mem);
  for (int i = 0; i < slots && e == hipSuccess; i++) {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);  // default priority
    if (e != hipSuccess) break;
    S->streams.push_back(s);
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) S->events.push_back(ev);
  }
  if (e != hipSuccess) {
    spq_server_destroy(S.release());
    return fail(e == hipErrorOutOfMemory ? SPQ_ENOMEM : SPQ_EDEVICE,
                std::string("server set-up: ") + hipGetErrorString(e));
  }
  S->t0 = std::chrono::steady_clock::now();
  spq_server* p = S.get();
  S->worker = std::thread([p] { p->run(); });
  *out = S.release();
  return SPQ_OK;
}

spq_status spq_server_submit(spq_server* S, int64_t q, const int32_t* v1, const int32_t* v2,
                             int32_t* out, int64_t* ticket) {
  if (!S || !ticket) return fail(SPQ_EINVAL, "null argument");
  if (q < 0) return fail(SPQ_EINVAL, "q < 0");
  if (q > 0 && (!v1 || !v2 || !out)) return fail(SPQ_EINVAL, "null query array");
  std::unique_ptr<Req> r(new Req());
  r->q = q;
  r->v1 = v1;
  r->v2 = v2;
  r->out = out;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    if (S->failed != SPQ_OK) return fail(S->failed, S->failure);
    r->arrival = S->now();
    if (q == 0) {
      r->done = true;
      r->done_at = r->arrival;
    } else {
      S->queue.push_back(r.get());
    }
    *ticket = S->next_ticket++;
    S->reqs[*ticket] = std::move(r);
  }
  S->cv.notify_all();
  return SPQ_OK;
}

spq_status spq_server_poll(spq_server* S, int64_t ticket, int32_t wait, int32_t* done,
                           double* latency_s) {
  if (!S || !done) return fail(SPQ_EINVAL, "null argument");
  std::unique_lock<std::mutex> lock(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(SPQ_EINVAL, "unknown or already collected ticket");
  Req* r = it->second.get();
  if (wait) S->cv.wait(lock, [&] { return r->done || S->failed != SPQ_OK; });
  if (!r->done && S->failed != SPQ_OK) return fail(S->failed, S->failure);
  *done = r->done ? 1 : 0;
  if (latency_s) *latency_s = r->done ? r->done_at - r->arrival : -1.0;
  if (r->done) S->reqs.erase(it);
  return SPQ_OK;
}

spq_status spq_server_stats(spq_server* S, int64_t* launches, int64_t* pairs) {
  if (!S) return fail(SPQ_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  if (launches) *launches = S->launches;
  if (pairs) *pairs = S->pairs;
  return SPQ_OK;
}

void spq_server_destroy(spq_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : S->events) (void)hipEventDestroy(e);
  if (S->d_pool) (void)hipFree(S->d_pool);
  if (S->h_pool) (void)hipHostFree(S->h_pool);
  delete S;
}

}  // extern "C"
