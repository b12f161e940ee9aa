// C-ABI of the shortest-path query library: index construction (Algorithm 1),
// batched queries (Algorithm 2), inspection and test hooks.  Declarations and
// their contracts are in include/spq.h.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/spq.h"
#include "spq_internal.h"

using spq::u32;

namespace {

thread_local std::string g_err;

spq_status fail(spq_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      return fail(e_ == hipErrorOutOfMemory ? SPQ_ENOMEM : SPQ_EDEVICE,                \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    }                                                                                  \
  } while (0)

// Device memory pool.  Index buffers are large (up to ~130 GB) and a fresh
// hipMalloc of memory freed a moment earlier costs about a second per 100 GB
// on this device, so a freed index hands its blocks back to this cache and
// the next build reuses them.  spq_release_cached_memory() returns them.
struct Pool {
  std::mutex mu;
  std::unordered_map<void*, std::pair<int, size_t>> live;  // ptr -> (device, bytes)
  std::multimap<std::pair<int, size_t>, void*> idle;       // (device, bytes) -> ptr
};

Pool& pool() {
  static Pool* p = new Pool();  // lives until the process ends
  return *p;
}

size_t pool_round(size_t b) {
  const size_t big = size_t(1) << 21;
  return b < big ? (b + 255) & ~size_t(255) : (b + big - 1) & ~(big - 1);
}

void pool_drop_idle(int dev) {  // caller holds the lock
  Pool& P = pool();
  for (auto it = P.idle.begin(); it != P.idle.end();) {
    if (dev < 0 || it->first.first == dev) {
      (void)hipFree(it->second);
      it = P.idle.erase(it);
    } else {
      ++it;
    }
  }
}

hipError_t pool_alloc(void** out, size_t bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  bytes = pool_round(bytes);
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  auto it = P.idle.lower_bound({dev, bytes});
  if (it != P.idle.end() && it->first.first == dev && it->first.second <= bytes + bytes / 4) {
    *out = it->second;
    P.live[*out] = it->first;
    P.idle.erase(it);
    return hipSuccess;
  }
  e = hipMalloc(out, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    pool_drop_idle(dev);
    e = hipMalloc(out, bytes);
  }
  if (e == hipSuccess) P.live[*out] = {dev, bytes};
  return e;
}

void pool_release(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) {
    (void)hipFree(p);
    return;
  }
  P.idle.insert({it->second, p});
  P.live.erase(it);
}

// Streams for the lookahead's side work, graph capture and host-array
// queries.  Creating and destroying a stream costs about 56 us on this
// device: nothing next to a build, but more than half of a one-pair
// spq_query_batch_host call (about 71 us with a stream of its own, 30 us with
// one from here).  A freed index hands its streams back (after its work has
// finished), a host query as soon as its stream has drained, and later calls
// on the same device take them again.
struct StreamPool {
  std::mutex mu;
  std::multimap<int, hipStream_t> idle;  // device -> stream
};

StreamPool& stream_pool() {
  static StreamPool* p = new StreamPool();  // lives until the process ends
  return *p;
}

hipError_t stream_take(hipStream_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    StreamPool& P = stream_pool();
    std::lock_guard<std::mutex> lock(P.mu);
    auto it = P.idle.find(dev);
    if (it != P.idle.end()) {
      *out = it->second;
      P.idle.erase(it);
      return hipSuccess;
    }
  }
  return hipStreamCreateWithFlags(out, hipStreamNonBlocking);  // default priority
}

// s must have no queued work left
void stream_give(int dev, hipStream_t s) {
  if (!s) return;
  StreamPool& P = stream_pool();
  std::lock_guard<std::mutex> lock(P.mu);
  P.idle.insert({dev, s});
}

template <typename T>
hipError_t dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  return pool_alloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)count);
}

int64_t round_up(int64_t x, int64_t t) { return (x + t - 1) / t * t; }

// Rows of v valid ones that the composition kernels relax: whole 128-tiles,
// but in the last, partial tile a wave skips its 16 rows of a half when they
// all lie past the valid ones (a wave holds rows 16w .. 16w+15 and
// 64+16w .. 64+16w+15 of the tile).
double mp_rows(int32_t v) {
  const int32_t rem = v % 128;
  double rows = (double)(v - rem);
  if (rem)
    for (int w = 0; w < 4; w++) rows += (16 * w < rem ? 16 : 0) + (64 + 16 * w < rem ? 16 : 0);
  return rows;
}

// Columns of v valid ones that the composition kernels relax: whole
// 128-tiles, and of the last, partial tile its first half alone when that
// holds them all.
double mp_cols(int32_t v) {
  const int32_t rem = v % 128;
  return (double)(v - rem) + (rem == 0 ? 0 : rem <= 64 ? 64 : 128);
}

}  // namespace

// Fixed staging of spq_query_batch_host_static: v1, v2 and the answers of one
// call, SPQ_STATIC_PAIRS int32 each, on every device the library runs on.
// Host code never passes this symbol to a kernel or a copy: it takes the
// device address hipGetSymbolAddress gives for the current device (once per
// device, kept in g_static).
static __device__ __align__(256) int32_t scratch[3 * SPQ_STATIC_PAIRS];

namespace {

constexpr int kMaxDevices = 64;

struct StaticScratch {
  std::once_flag once;
  hipError_t init = hipSuccess;
  int32_t* ptr = nullptr;         // scratch on this device
  std::atomic<bool> busy{false};  // a call holds the array
};

StaticScratch g_static[kMaxDevices];

}  // namespace

int spq::set_error(int s, const char* msg) { return fail(static_cast<spq_status>(s), msg); }

struct spq_index {
  int device = 0;
  int32_t n = 0, k = 0, V = 0, Vp = 0, tile = 128, pivot = 256, max_comp = 0, max_nb = 0;
  int32_t cpivot = 256;  // pivot rows of the 128-tile closures (components, groups, BG2, BG3)
  int64_t m = 0, comp_elems = 0;
  std::vector<int32_t> h_cnt, h_nb, h_off, h_bgoff, h_P, h_order;
  std::vector<int64_t> h_moff;
  std::vector<unsigned long long> h_sumc;
  // device memory owned by the index
  int32_t *comp = nullptr, *local = nullptr, *nb = nullptr, *off = nullptr, *bgoff = nullptr;
  int32_t *P = nullptr, *order = nullptr, *bgcomp = nullptr, *bglocal = nullptr;
  int32_t *cnt = nullptr, *fill = nullptr;
  int64_t* moff = nullptr;
  uint8_t* flag = nullptr;
  unsigned long long *sumc = nullptr, *total = nullptr;
  u32 *err = nullptr, *members = nullptr, *M = nullptr, *BG = nullptr;
  u32* vrec = nullptr;
  int64_t* gT = nullptr;           // [groups] first element of each group's band in H
  std::vector<int64_t> h_gT;
  // groups (all components in group 0 for the flat store)
  int32_t method = 1, ngroups = 1, cpg = 1, Vgp = 0, V2 = 0, m2pmax = 0, nbig = 0;
  int64_t V2p = 0, h_elems = 0;
  std::vector<int32_t> h_grp, h_gbg0, h_gV, h_m2, h_b2off;
  std::vector<int64_t> h_pairbase;
  int32_t *grp = nullptr, *gbg0 = nullptr, *gV = nullptr, *bgrow = nullptr, *bgnb = nullptr;
  int32_t *bggrp = nullptr, *b2list = nullptr, *b2rank = nullptr, *m2 = nullptr, *b2off = nullptr;
  uint8_t* flag2 = nullptr;
  u32 *Mg = nullptr, *R = nullptr, *XT = nullptr, *BG2 = nullptr, *H = nullptr;
  int64_t* pairbase = nullptr;
  // the composition's positions: per group its width (B2 vertices padded to
  // a multiple of 4, then the others), their bound Vrp and the table
  int32_t Vrp = 0;
  std::vector<int32_t> h_W;
  int32_t* pos = nullptr;
  // level 3 (closure of BG2 by super-groups of gpt groups)
  int32_t nT = 0, gpt = 0, V3gp = 0, V3 = 0, m3pmax = 0;
  int64_t V3p = 0;
  std::vector<int32_t> h_tbase, h_tsize, h_m3, h_b3off;
  int32_t *tbase = nullptr, *tsize = nullptr, *b3list = nullptr, *b3rank = nullptr, *m3 = nullptr;
  int32_t* pos3 = nullptr;  // the super-groups' positions
  int32_t* b3off = nullptr;
  uint8_t* flag3 = nullptr;
  // composition pair lists (level 2 or share, level 3)
  int2 *plist = nullptr, *plist3 = nullptr;
  int32_t npairs = 0, chunk = 0;
  u32 *M3 = nullptr, *R3 = nullptr, *XT3 = nullptr, *BG3 = nullptr;
  // share mode
  int32_t share_comps = 0, share_groups = 0, S2 = 0, bf_rounds = 0;
  int64_t S2p = 0;
  u32 *A = nullptr, *DT = nullptr, *bfflag = nullptr, *bfstamp = nullptr;
  int32_t *bfcnt = nullptr, *bflist = nullptr;
  // the blocks' boundary B3 (rows the rounds keep settled) and the rest
  uint8_t *sb_flag = nullptr, *sb_flagn = nullptr;
  int32_t *sb_list = nullptr, *sb_nlist = nullptr, *sb_rank = nullptr, *sb_nrank = nullptr;
  int32_t *sb_m = nullptr, *sb_n = nullptr;
  u32 *sb_A3 = nullptr, *sb_Aout = nullptr;
  std::vector<int32_t> h_sbm, h_sbn;
  // Bellman-Ford blocks (runs of groups): first level-2 id, size, first
  // group, and the block of every group
  int32_t bgpt = 1, nblk = 0, bpmax = 0;
  std::vector<int32_t> h_boff, h_bsize, h_bfirst, h_gblk;
  int32_t *boff = nullptr, *bsize = nullptr, *bfirst = nullptr, *gblk = nullptr;
  std::vector<int32_t> h_gfirst;  // first component of every group
  bool group_bg = false;          // groups formed by size
  int4* xe = nullptr;
  int32_t* xcount = nullptr;
  // exactness certificate (total weight >= INF)
  bool certify = false;
  int32_t *bgvert = nullptr, *label = nullptr, *bglabel = nullptr;
  u32* cert = nullptr;  // [4]: changed, bad, max APSP(C), max BG
  u32 cert_mc = 0, cert_mbg = 0;
  // lookahead of the flat rounds: side stream and its two sync events
  hipStream_t side = nullptr;
  hipStream_t part1 = nullptr;  // flat rounds: part 1 of every round beside part 2
  hipEvent_t la_sync[3] = {};
  hipEvent_t ev[5] = {};
  bool events = false;
  std::vector<hipEvent_t> prof;  // pairs around the BG interior-tile launches
  double relax_comp = 0, relax_bg = 0, relax_comp_exec = 0, relax_bg_exec = 0, relax_inner = 0;
  int64_t inner_launches = 0;
  // SPQ_GRAPH: captured Phase 2-3 work, replayed by spq_reweight_index on
  // the index's own copies of the edges
  bool graph = false, fused_cert = false, valid = true;
  hipStream_t cap = nullptr;
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  int64_t graph_nodes = 0;
  int32_t reweights = 0;
  int32_t *eu_own = nullptr, *ev_own = nullptr, *w_own = nullptr;
  // SPQ_PATHS: adjacency (rowptr[n+1], (neighbour, edge) pairs) and weights
  bool paths = false;
  int64_t* rowptr = nullptr;
  int2* adj = nullptr;
  unsigned long long* adeg = nullptr;
  int32_t* w_copy = nullptr;        // own copy of the weights (without SPQ_GRAPH)
  const int32_t* w_path = nullptr;  // the weights the walk reads (w_copy or w_own)

  ~spq_index() {
    if (events) {
      (void)hipEventSynchronize(ev[4]);
      for (auto& e : ev) (void)hipEventDestroy(e);
    }
    for (auto& e : prof) (void)hipEventDestroy(e);
    for (auto& e : la_sync)
      if (e) (void)hipEventDestroy(e);
    // no queued work of this index may still use its memory or its streams
    // once they are cached
    (void)hipDeviceSynchronize();
    stream_give(device, side);
    stream_give(device, part1);
    for (auto x : execs) (void)hipGraphExecDestroy(x);
    for (auto g : graphs) (void)hipGraphDestroy(g);
    stream_give(device, cap);
    void* ptrs[] = {comp, local, nb,   off,  bgoff, P,     order, bgcomp,  bglocal,
                    cnt,  fill,  moff, flag, sumc,  total, err,   members, M,      BG,
                    vrec, gT,    grp,   gbg0, gV,   bgrow, bgnb,  bggrp, b2list,  b2rank, m2,
                    b2off, flag2, Mg,  R,    XT,    BG2,   H,     pairbase, pos,
                    bgvert, label, bglabel, cert, A,    DT,    bfflag,  bfstamp, bfcnt, bflist,
                    sb_flag, sb_flagn, sb_list, sb_nlist, sb_rank, sb_nrank, sb_m, sb_n, sb_A3, sb_Aout,
                    xe, xcount, boff, bsize, bfirst, gblk,
                    eu_own, ev_own, w_own, tbase, tsize, b3list, b3rank, m3, b3off, flag3,
                    M3, R3, XT3, BG3, plist, plist3, rowptr, adj, adeg, w_copy, pos3};
    for (void* p : ptrs) pool_release(p);
  }
};

// Queues body(stream): directly on s, or (SPQ_GRAPH) captured on the index's
// capture stream into a HIP graph that is instantiated, launched on s and
// kept for spq_reweight_index.  body must queue device work only (no
// allocation, no host copy, no synchronization, no memset).
template <typename F>
static hipError_t graph_segment(spq_index* X, hipStream_t s, F&& body) {
  if (!X->graph) return body(s);
  hipError_t e = hipStreamBeginCapture(X->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  const hipError_t eb = body(X->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(X->cap, &g);
  if (g) X->graphs.push_back(g);
  if (eb != hipSuccess) return eb;
  if (e != hipSuccess) return e;
  size_t nodes = 0;
  e = hipGraphGetNodes(g, nullptr, &nodes);
  if (e != hipSuccess) return e;
  X->graph_nodes += (int64_t)nodes;
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) return e;
  X->execs.push_back(x);
  return hipGraphLaunch(x, s);
}

// Pair list of a composition (rows groups [0, rows) against groups [first,
// G), first = the row group itself when `upper`), uploaded to *dev, and the
// pairs per launch: the XT buffer holds one slot of slot_elems words per
// pair of a launch, within 1/32 of the composition's output clamped to
// [256 MiB, 4 GiB], at least one slot.
static hipError_t make_pairs(int32_t rows, int32_t G, bool upper, int64_t slot_elems,
                             int64_t out_elems, int2** dev, int32_t* npairs, int32_t* chunk,
                             hipStream_t s, const std::vector<uint8_t>* swap = nullptr) {
  const int64_t count = upper ? (int64_t)rows * (2 * (int64_t)G - rows + 1) / 2 : (int64_t)rows * G;
  if (count > 0x7fffffff) return hipErrorOutOfMemory;  // pair list beyond int32 indexing
  std::vector<int2> h;
  h.reserve((size_t)count);
  // swap (optional, rows x G flags in this order): pairs computed through
  // the row group's boundary (PAIR_SWAP)
  for (int32_t a1 = 0; a1 < rows; a1++)
    for (int32_t a2 = upper ? a1 : 0; a2 < G; a2++)
      h.push_back(swap && (*swap)[h.size()] ? make_int2(a2, a1 | spq::PAIR_SWAP) : make_int2(a1, a2));
  *npairs = (int32_t)h.size();
  // pairs per launch: XT slots within 4 GiB, and the grid's y dimension
  const int64_t budget = std::min<int64_t>((int64_t)1 << 30,
                                           std::max<int64_t>((int64_t)1 << 26, out_elems / 32));
  const int64_t fit = budget / std::max<int64_t>(slot_elems, 1);
  *chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)*npairs, fit, 65535}));
  hipError_t e = dalloc(dev, std::max<int64_t>(*npairs, 1));
  if (e != hipSuccess || h.empty()) return e;
  return hipMemcpyAsync(*dev, h.data(), sizeof(int2) * h.size(), hipMemcpyHostToDevice, s);
}

// The composition's positions from the level-2 boundary counts: widths and
// their bound Vrp (a multiple of 128).
static void set_positions(spq_index* X) {
  X->h_W.resize(X->ngroups);
  int64_t wmax = 0;
  for (int32_t g = 0; g < X->ngroups; g++) {
    X->h_W[g] = (int32_t)round_up(X->h_m2[g], 4) + X->h_gV[g] - X->h_m2[g];
    wmax = std::max<int64_t>(wmax, X->h_W[g]);
  }
  X->Vrp = (int32_t)std::max<int64_t>(128, round_up(wmax, 128));
}

// Executed relaxations of a pair's two products, the first over B2(a1)
// (rows B2(a2), columns: a1's vertices outside B2(a1); its B2 columns are
// copied from D2), the second over B2(a2) (rows: a1's positions, columns:
// a2's vertices outside B2(a2)).
static double xt_relax(const spq_index* X, int32_t a1, int32_t a2) {
  return mp_rows(X->h_m2[a2]) * mp_cols(X->h_gV[a1] - X->h_m2[a1]) * (double)round_up(X->h_m2[a1], 16);
}
static double y_relax(const spq_index* X, int32_t a1, int32_t a2) {
  return mp_rows(X->h_W[a1]) * mp_cols(X->h_gV[a2] - X->h_m2[a2]) * (double)round_up(X->h_m2[a2], 16);
}

// The query kernel locates a pair block from the two vertex records alone:
// band of S1 + |S1| * (first BG id of S2, minus that of S1 in the full store).
// The pair table built for the composition must agree with it.
static bool bands_match(const spq_index* X, int32_t row_groups, bool share) {
  const int32_t G = X->ngroups;
  for (int32_t a1 = 0; a1 < row_groups; a1++)
    for (int32_t a2 = share ? 0 : a1; a2 < G; a2++)
      if (X->h_pairbase[(size_t)a1 * G + a2] !=
          X->h_gT[a1] + (int64_t)X->h_gV[a1] * (X->h_gbg0[a2] - (share ? 0 : X->h_gbg0[a1])))
        return false;
  return true;
}

// Share mode (after level 1): Bellman-Ford over blocks of groups from the
// share's level-2 vertices, then the composition for the share's groups
// against all groups.  blk_opt: groups per block (> 0), 0 auto, -1 one.
// Synchronous (one small readback per round).
static spq_status build_share(spq_index* X, spq::HierArgs& ha, int64_t m, bool profile, int32_t blk_opt,
                              hipStream_t s) {
  const int32_t G = X->ngroups, Vgp = X->Vgp;
  if (((int64_t)std::max<int64_t>(X->V2p, 128) + 31) / 32 > 65535)
    return fail(SPQ_EINVAL, "share mode supports at most 2,097,120 level-2 vertices");
  X->share_groups = X->h_grp[X->share_comps - 1] + 1;
  X->S2 = X->h_b2off[X->share_groups];
  X->S2p = round_up(std::max<int32_t>(X->S2, 1), 128);
  X->h_pairbase.assign((size_t)G * G, -1);
  X->h_elems = 0;
  for (int32_t a1 = 0; a1 < X->share_groups; a1++)
    for (int32_t a2 = 0; a2 < G; a2++) {
      X->h_pairbase[(size_t)a1 * G + a2] = X->h_elems;
      X->h_elems += (int64_t)X->h_gV[a1] * X->h_gV[a2];
    }
  if (!bands_match(X, X->share_groups, true)) return fail(SPQ_EDEVICE, "internal: band layout");
  const int64_t V2p = std::max<int64_t>(X->V2p, 128);
  X->V2p = V2p;
  // Bellman-Ford blocks: runs of bgpt groups (auto: a power of two of groups,
  // about 1,024 level-2 vertices per block)
  int32_t bgpt = 1;
  if (blk_opt > 0) {
    bgpt = std::min(blk_opt, G);
  } else if (blk_opt == 0) {
    const double avg = std::max(1.0, (double)X->V2 / G);
    while (bgpt * 2 <= G && bgpt * 2 * avg <= 1024.0 * 1.41) bgpt *= 2;
  }
  X->bgpt = bgpt;
  // Blocks: the groups that start in each run of bgpt x (components per
  // group) consecutive components, so that a group cut in halves does not
  // shift the later blocks (groups formed by size: runs of bgpt groups).
  X->h_gblk.resize(G);
  for (int32_t g = 0; g < G; g++)
    X->h_gblk[g] = X->group_bg ? g / bgpt : (int32_t)(X->h_gfirst[g] / ((int64_t)bgpt * X->cpg));
  X->nblk = X->h_gblk[G - 1] + 1;
  if (X->nblk > 65535) return fail(SPQ_EINVAL, "more than 65,535 Bellman-Ford blocks");
  const int32_t NB = X->nblk;
  X->h_bfirst.assign(NB + 1, G);
  for (int32_t g = G - 1; g >= 0; g--) X->h_bfirst[X->h_gblk[g]] = g;
  bool multi = false;
  X->h_boff.assign(NB + 1, 0);
  X->h_bsize.assign(NB, 0);
  int32_t bmax = 0;
  for (int32_t t = 0; t < NB; t++) {
    if (X->h_bfirst[t] >= X->h_bfirst[t + 1]) return fail(SPQ_EDEVICE, "internal: empty block");
    multi |= X->h_bfirst[t + 1] - X->h_bfirst[t] > 1;
    X->h_boff[t] = X->h_b2off[X->h_bfirst[t]];
    X->h_bsize[t] = X->h_b2off[X->h_bfirst[t + 1]] - X->h_boff[t];
    bmax = std::max(bmax, X->h_bsize[t]);
  }
  X->h_boff[NB] = X->V2;
  X->bpmax = (int32_t)std::max<int64_t>(128, round_up(bmax, 128));
  const int32_t BP = X->bpmax;
  if (multi) X->relax_bg_exec += NB * spq::dense_fw_exec_relax(BP / 128, 128, X->cpivot);
  HIP_TRY(hipMemcpyAsync(X->b2off, X->h_b2off.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(dalloc(&X->boff, NB + 1));
  HIP_TRY(dalloc(&X->bsize, NB));
  HIP_TRY(hipMemcpyAsync(X->boff, X->h_boff.data(), sizeof(int32_t) * (NB + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(X->bsize, X->h_bsize.data(), sizeof(int32_t) * NB, hipMemcpyHostToDevice, s));
  HIP_TRY(dalloc(&X->bfirst, NB + 1));
  HIP_TRY(dalloc(&X->gblk, G));
  HIP_TRY(hipMemcpyAsync(X->bfirst, X->h_bfirst.data(), sizeof(int32_t) * (NB + 1), hipMemcpyHostToDevice,
                         s));
  HIP_TRY(hipMemcpyAsync(X->gblk, X->h_gblk.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
  set_positions(X);
  const int32_t Vrp = X->Vrp;
  // R's last row is read up to 127 words past its end (the second product's
  // column tiles start past the B2 positions)
  HIP_TRY(dalloc(&X->R, (int64_t)G * X->m2pmax * Vrp + 128));
  HIP_TRY(dalloc(&X->pos, (int64_t)G * Vrp));
  // each output block (S1, S2) through the cheaper boundary: through B2(S2)
  // or, S1 and S2 exchanged, through B2(S1) (its first product then reads D2
  // transposed, which is the Bellman-Ford table)
  auto cost = [&](int32_t a, int32_t b) { return xt_relax(X, a, b) + y_relax(X, a, b); };
  std::vector<uint8_t> swap((size_t)X->share_groups * G, 0);
  for (int32_t a1 = 0; a1 < X->share_groups; a1++)
    for (int32_t a2 = 0; a2 < G; a2++)
      swap[(size_t)a1 * G + a2] = a1 != a2 && cost(a2, a1) < cost(a1, a2);
  HIP_TRY(make_pairs(X->share_groups, G, false, (int64_t)X->m2pmax * Vrp, X->h_elems, &X->plist,
                     &X->npairs, &X->chunk, s, &swap));
  HIP_TRY(dalloc(&X->XT, (int64_t)X->chunk * X->m2pmax * Vrp));
  HIP_TRY(dalloc(&X->A, (int64_t)NB * BP * BP));
  // the Bellman-Ford matrix carries 128 spare rows: a row tile may start at
  // the last block's last level-2 id
  HIP_TRY(dalloc(&X->DT, (V2p + 128) * X->S2p));
  // D2 = DT transposed, one column panel of S2p x m2pmax per group
  HIP_TRY(dalloc(&X->BG2, (int64_t)G * X->S2p * X->m2pmax));
  HIP_TRY(dalloc(&X->H, X->h_elems));
  HIP_TRY(dalloc(&X->pairbase, (int64_t)G * G));
  HIP_TRY(dalloc(&X->xe, 2 * std::max<int64_t>(m, 1)));
  HIP_TRY(dalloc(&X->xcount, 1));
  // dirty flags, two rounds' worth: per block one word per column tile of
  // 128 share sources and one "any" word
  const int32_t ntc = (int32_t)(X->S2p / 128), fs = ntc + 1;
  HIP_TRY(dalloc(&X->bfflag, 2 * (int64_t)NB * fs));
  // rows lowered per (block, column tile), two rounds' worth, and the round
  // stamps that keep a row from being listed twice in one round
  HIP_TRY(dalloc(&X->bfcnt, 2 * (int64_t)NB * ntc));
  HIP_TRY(dalloc(&X->bfstamp, V2p * ntc));
  HIP_TRY(dalloc(&X->sb_flag, V2p));
  HIP_TRY(dalloc(&X->sb_flagn, V2p));
  HIP_TRY(dalloc(&X->sb_list, (int64_t)NB * BP));
  HIP_TRY(dalloc(&X->sb_nlist, (int64_t)NB * BP));
  HIP_TRY(dalloc(&X->sb_rank, V2p));
  HIP_TRY(dalloc(&X->sb_nrank, V2p));
  HIP_TRY(dalloc(&X->sb_m, NB));
  HIP_TRY(dalloc(&X->sb_n, NB));
  HIP_TRY(hipMemsetAsync(X->bfstamp, 0xff, sizeof(u32) * V2p * ntc, s));
  HIP_TRY(hipMemsetAsync(X->xcount, 0, sizeof(int32_t), s));
  HIP_TRY(hipMemsetAsync(X->DT + V2p * X->S2p, 0xff, 128 * X->S2p * sizeof(u32), s));
  HIP_TRY(hipMemcpyAsync(X->pairbase, X->h_pairbase.data(), sizeof(int64_t) * G * G,
                         hipMemcpyHostToDevice, s));
  ha.m2pmax = X->m2pmax; ha.V2 = X->V2; ha.V2p = V2p; ha.b2off = X->b2off; ha.R = X->R;
  ha.XT = X->XT; ha.BG2 = X->BG2; ha.H = X->H; ha.pairbase = X->pairbase;
  ha.pos = X->pos; ha.Vrp = Vrp;
  ha.plist = X->plist; ha.npairs = X->npairs; ha.chunk = X->chunk;
  ha.share_groups = X->share_groups; ha.S2 = X->S2; ha.S2p = X->S2p; ha.DT = X->DT;
  ha.D2t = X->DT; ha.d2tld = X->S2p;
  ha.xe = X->xe; ha.xcount = X->xcount;
  const spq::ShareBlocks blk{NB, BP, multi, X->bfirst, X->gblk, X->boff, X->bsize, X->A};
  HIP_TRY(spq::launch_share_prepare(ha, blk, s));
  HIP_TRY(spq::launch_share_b3_lists(ha, blk, X->sb_flag, X->sb_flagn, X->sb_list, X->sb_nlist,
                                     X->sb_rank, X->sb_nrank, X->sb_m, X->sb_n, s));
  int32_t nxe = 0;
  X->h_sbm.assign(NB, 0);
  X->h_sbn.assign(NB, 0);
  HIP_TRY(hipMemcpyAsync(&nxe, X->xcount, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(X->h_sbm.data(), X->sb_m, sizeof(int32_t) * NB, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(X->h_sbn.data(), X->sb_n, sizeof(int32_t) * NB, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int32_t m3max = 0, n3max = 0;
  for (int32_t t = 0; t < NB; t++) {
    m3max = std::max(m3max, X->h_sbm[t]);
    n3max = std::max(n3max, X->h_sbn[t]);
  }
  const int32_t B3P = (int32_t)std::max<int64_t>(128, round_up(m3max, 128));
  const int32_t N3P = (int32_t)std::max<int64_t>(128, round_up(n3max, 128));
  HIP_TRY(dalloc(&X->bflist, 2 * (int64_t)NB * ntc * B3P));
  HIP_TRY(dalloc(&X->sb_A3, (int64_t)NB * B3P * B3P));
  HIP_TRY(dalloc(&X->sb_Aout, (int64_t)NB * B3P * N3P));
  const spq::ShareB3 b3{B3P, N3P, X->sb_m, X->sb_n, X->sb_list, X->sb_nlist, X->sb_rank,
                        X->sb_A3, X->sb_Aout};
  HIP_TRY(spq::launch_share_b3_gather(blk, b3, s));
  // The blocks holding share sources start dirty on every column tile.  Their
  // rows start closed (DT's initial rows are rows of the closed A), so the
  // first intra step has no row to multiply: cross edges move first.
  std::vector<u32> hd((size_t)NB * fs, 0);
  std::vector<int32_t> hc((size_t)NB * ntc, 0);
  for (int32_t t = 0; t < NB && X->h_boff[t] < X->S2; t++)
    for (int32_t c = 0; c < fs; c++) hd[(size_t)t * fs + c] = 1;
  HIP_TRY(hipMemcpyAsync(X->bfflag, hd.data(), sizeof(u32) * NB * fs, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(X->bfcnt, hc.data(), sizeof(int32_t) * NB * ntc, hipMemcpyHostToDevice, s));
  // Rounds are queued ahead of the host: a round needs only the flags the
  // previous one left on the device, so up to BF_AHEAD rounds are in flight
  // while the host reads back (pinned, behind an event) the flags of the
  // oldest one, for the relaxation count and to see when nothing is dirty.
  // The rounds queued after the one that leaves nothing dirty find no dirty
  // tile and no cross edge to relax: they change nothing.
  constexpr int BF_AHEAD = 3, SLOTS = BF_AHEAD + 1;
  const size_t fwords = (size_t)NB * fs, cwords = (size_t)NB * ntc;
  struct Readback {
    u32* host = nullptr;
    hipEvent_t ev[SLOTS] = {};
    ~Readback() {
      for (auto& e : ev)
        if (e) {
          (void)hipEventSynchronize(e);
          (void)hipEventDestroy(e);
        }
      if (host) (void)hipHostFree(host);
    }
  } rb;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&rb.host), sizeof(u32) * SLOTS * (fwords + cwords)));
  for (auto& e : rb.ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  u32* dbuf[2] = {X->bfflag, X->bfflag + (int64_t)NB * fs};
  int32_t* cbuf[2] = {X->bfcnt, X->bfcnt + (int64_t)NB * ntc};
  int32_t* lbuf[2] = {X->bflist, X->bflist + (int64_t)NB * ntc * B3P};
  // executed relaxations of a round from the flags and counts it starts
  // with: a dirty (block, tile) multiplies its B3 row tiles by the rows
  // listed for it
  auto count = [&](const u32* fl, const int32_t* cn) {
    for (int32_t t = 0; t < NB; t++)
      for (int32_t c = 0; c < ntc; c++) {
        const int32_t cc = cn[(size_t)t * ntc + c];
        if (cc == 0 || !fl[(size_t)t * fs + c]) continue;
        const int32_t kk = cc == spq::BF_ALL_ROWS ? X->h_sbm[t] : cc;
        X->relax_bg_exec += (double)((X->h_sbm[t] + 127) / 128) * 128.0 * 128.0 *
                            (double)round_up(kk, 16);
      }
  };
  count(hd.data(), hc.data());
  int64_t issued = 0, consumed = 0;
  for (;;) {
    while (issued - consumed < BF_AHEAD) {
      if (issued >= 100000) return fail(SPQ_EDEVICE, "Bellman-Ford over blocks did not settle");
      const int in = (int)(issued & 1), out = in ^ 1;
      const spq::BfRound r{dbuf[in], dbuf[out], cbuf[in], lbuf[in], cbuf[out], lbuf[out],
                           X->bfstamp, (u32)(issued + 1)};
      HIP_TRY(hipMemsetAsync(dbuf[out], 0, sizeof(u32) * fwords, s));
      HIP_TRY(hipMemsetAsync(cbuf[out], 0, sizeof(int32_t) * cwords, s));
      HIP_TRY(spq::launch_share_round(ha, blk, b3, nxe, r, s));
      u32* slot = rb.host + (size_t)(issued % SLOTS) * (fwords + cwords);
      HIP_TRY(hipMemcpyAsync(slot, dbuf[out], sizeof(u32) * fwords, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(slot + fwords, cbuf[out], sizeof(int32_t) * cwords, hipMemcpyDeviceToHost,
                             s));
      HIP_TRY(hipEventRecord(rb.ev[issued % SLOTS], s));
      issued++;
    }
    HIP_TRY(hipEventSynchronize(rb.ev[consumed % SLOTS]));
    const u32* fl = rb.host + (size_t)(consumed % SLOTS) * (fwords + cwords);
    const int32_t* cn = reinterpret_cast<const int32_t*>(fl + fwords);
    consumed++;
    bool any = false;
    for (int32_t t = 0; t < NB; t++) any |= fl[(size_t)t * fs + ntc] != 0;
    if (!any) break;
    count(fl, cn);  // the next round's work
  }
  X->bf_rounds = (int32_t)consumed;
  // the rows outside B3 from the settled B3 rows
  HIP_TRY(spq::launch_share_final(ha, blk, b3, s));
  for (int32_t t = 0; t < NB; t++)
    if (X->h_sbm[t] > 0)
      X->relax_bg_exec += (double)((X->h_sbn[t] + 127) / 128) * ntc * 128.0 * 128.0 *
                          (double)round_up(X->h_sbm[t], 16);
  for (int32_t p1 = 0; p1 < X->share_groups; p1++)
    for (int32_t p2 = 0; p2 < G; p2++) {
      const bool sw = swap[(size_t)p1 * G + p2];
      const int32_t a1 = sw ? p2 : p1, a2 = sw ? p1 : p2;  // the products' roles
      X->relax_bg_exec += xt_relax(X, a1, a2);
      const double y = y_relax(X, a1, a2);
      X->relax_bg_exec += y;
      X->relax_inner += y;
    }
  X->inner_launches = (X->npairs + X->chunk - 1) / X->chunk;
  if (profile) {
    X->prof.resize(2 * X->inner_launches);
    for (auto& e : X->prof) HIP_TRY(hipEventCreate(&e));
    ha.evt = X->prof.data();
  }
  HIP_TRY(spq::launch_share_compose(ha, X->DT, s));
  return SPQ_OK;
}

// Connected components of G and their label on every BG vertex (needed by the
// exactness certificate).  Synchronous: one small readback per round.
static spq_status cc_labels(spq_index* X, int64_t m, const int32_t* eu, const int32_t* ev,
                            hipStream_t s) {
  const int32_t n = X->n;
  HIP_TRY(dalloc(&X->label, n));
  HIP_TRY(dalloc(&X->bglabel, X->V));
  HIP_TRY(dalloc(&X->cert, 4));
  HIP_TRY(hipMemsetAsync(X->cert, 0, 4 * sizeof(u32), s));
  HIP_TRY(spq::launch_cc_init(n, X->label, s));
  u32 changed = 1;
  int rounds = 0;
  while (changed) {
    if (++rounds > 256) return fail(SPQ_ERANGE, "connected components did not settle");
    HIP_TRY(hipMemsetAsync(X->cert, 0, sizeof(u32), s));
    HIP_TRY(spq::launch_cc_round(m, eu, ev, n, X->label, X->cert, s));
    HIP_TRY(hipMemcpyAsync(&changed, X->cert, sizeof(u32), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  HIP_TRY(spq::launch_bg_label(X->V, X->bgvert, X->label, X->bglabel, s));
  return SPQ_OK;
}

// The exactness certificate (range.hip) when the total edge weight reaches
// SPQ_INF; cc_labels must have run.  For the two-level store the BG check
// runs inside the composition kernel when that kernel was given the labels
// (fused_cert); otherwise here.  Synchronous.
static spq_status certify(spq_index* X, hipStream_t s) {
  if (!X->certify) return SPQ_OK;
  spq::CertArgs c{};
  c.bg_checked = X->method == 2 && X->fused_cert;
  c.V = X->V; c.ngroups = X->ngroups; c.Vgp = X->Vgp; c.Vp = X->Vp; c.comp_elems = X->comp_elems;
  c.M = X->M; c.BG = X->BG; c.H = X->method == 2 ? X->H : nullptr; c.bgvert = X->bgvert;
  c.label = X->label; c.gV = X->gV; c.gbg0 = X->gbg0; c.bgrow = X->bgrow; c.bgnb = X->bgnb;
  c.bglocal = X->bglocal; c.pairbase = X->pairbase; c.bglabel = X->bglabel;
  c.bad = X->cert + 1; c.mc = X->cert + 2; c.mbg = X->cert + 3;
  HIP_TRY(spq::launch_certificate(c, s));
  u32 h[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(h, X->cert, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[1]) return fail(SPQ_ERANGE, "a BG distance between connected vertices reaches SPQ_INF");
  if (2ull * h[2] + h[3] >= (unsigned long long)SPQ_INF)
    return fail(SPQ_ERANGE, "query sums could reach SPQ_INF (max APSP(C) " + std::to_string(h[2]) +
                                ", max BG " + std::to_string(h[3]) + ")");
  X->cert_mc = h[2];
  X->cert_mbg = h[3];
  return SPQ_OK;
}

// Pool blocks of a hook, released when it returns, after its stream has
// drained (also on an early error return, when copies may still be queued).
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t st) : s(st) {}
  template <typename T>
  hipError_t get(T** p, int64_t count) {
    hipError_t e = dalloc(p, count);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  ~Scratch() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(s);
    for (void* p : ptrs) pool_release(p);
  }
};

extern "C" {

const char* spq_last_error(void) { return g_err.c_str(); }

spq_status spq_build_index(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                           const int32_t* w, const int32_t* part, int32_t k,
                           const spq_build_opts* opts, void* stream, spq_index** out) {
  g_err.clear();
  if (!out) return fail(SPQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || m < 0 || k < 1) return fail(SPQ_EINVAL, "need n >= 1, m >= 0, k >= 1");
  if (k > n) return fail(SPQ_EINVAL, "k > n: some component would be empty");
  if (!part || (m > 0 && (!eu || !ev || !w))) return fail(SPQ_EINVAL, "null input array");
  if (n > 0x7fffffff - 1) return fail(SPQ_EINVAL, "n too large");
  int tile = 128;
  bool profile = false, plain = false;
  int32_t method_opt = 0, group_comps = 0, share_comps = 0, inner_kc = 0;
  bool lookahead = true, use_graph = false, use_paths = false;
  int32_t level3_opt = 0, group_bg = 0, pivot = 0;
  if (opts) {
    if (opts->bg_tile != 0 && opts->bg_tile != 64 && opts->bg_tile != 128)
      return fail(SPQ_EINVAL, "bg_tile must be 0, 64 or 128");
    if (opts->bg_tile) tile = opts->bg_tile;
    pivot = opts->bg_pivot;
    if (pivot != 0 && pivot != tile && pivot != 2 * tile && pivot != 4 * tile)
      return fail(SPQ_EINVAL, "bg_pivot must be 0 or 1, 2 or 4 tiles");
    profile = opts->profile != 0;
    plain = opts->plain != 0;
    method_opt = opts->bg_method;
    group_comps = opts->group_comps;
    if (method_opt < 0 || method_opt > 2) return fail(SPQ_EINVAL, "bg_method must be 0, 1 or 2");
    if (group_comps < 0) return fail(SPQ_EINVAL, "group_comps < 0");
    share_comps = opts->share_comps;
    if (share_comps < 0 || share_comps > k) return fail(SPQ_EINVAL, "share_comps outside [0, k]");
    if (share_comps == k) share_comps = 0;
    if (share_comps > 0 && method_opt == 1)
      return fail(SPQ_EINVAL, "a share needs the two-level method");
    inner_kc = opts->inner_kc;
    if (inner_kc != 0 && inner_kc != 16 && inner_kc != 32)
      return fail(SPQ_EINVAL, "inner_kc must be 0, 16 or 32");
    if (opts->flags & ~(SPQ_NO_LOOKAHEAD | SPQ_GRAPH | SPQ_PATHS))
      return fail(SPQ_EINVAL, "unknown flags");
    use_paths = (opts->flags & SPQ_PATHS) != 0;
    lookahead = !(opts->flags & SPQ_NO_LOOKAHEAD);
    use_graph = (opts->flags & SPQ_GRAPH) != 0;
    level3_opt = opts->level3_groups;
    group_bg = opts->group_bg;
    if (group_bg < 0) return fail(SPQ_EINVAL, "group_bg < 0");
    if (level3_opt < -1) return fail(SPQ_EINVAL, "level3_groups must be -1, 0 or positive");
    if (use_graph && (share_comps > 0 || profile))
      return fail(SPQ_EINVAL, "SPQ_GRAPH cannot be combined with share_comps or profile");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  spq_index* X = new spq_index();
  auto guard = [&](spq_status st) {
    delete X;
    return st;
  };
  X->n = n;
  X->k = k;
  X->m = m;
  X->tile = tile;
  // default: four-tile blocks for the flat BG closure (measured 388 against
  // 408 ms on a 27,904-wide matrix), two-tile blocks for the other closures
  // (four measured 10 ms slower on the 256-group composition's closures)
  X->pivot = pivot ? pivot : 4 * tile;
  X->cpivot = pivot ? pivot / tile * 128 : 256;
  X->graph = use_graph;
  {
    hipError_t e = hipGetDevice(&X->device);
    if (e != hipSuccess) return guard(fail(SPQ_EDEVICE, hipGetErrorString(e)));
  }
#define TRY(expr)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return guard(fail(e_ == hipErrorOutOfMemory ? SPQ_ENOMEM : SPQ_EDEVICE,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_)));               \
  } while (0)

  for (auto& e : X->ev) TRY(hipEventCreate(&e));
  X->events = true;
  TRY(hipEventRecord(X->ev[0], s));

  // ---- boundary detection and sizes (device), then the plan (host)
  TRY(dalloc(&X->cnt, k));
  TRY(dalloc(&X->nb, k));
  TRY(dalloc(&X->flag, n));
  TRY(dalloc(&X->sumc, k));
  TRY(dalloc(&X->total, 1));
  TRY(dalloc(&X->err, 1));
  TRY(hipMemsetAsync(X->cnt, 0, sizeof(int32_t) * k, s));
  TRY(hipMemsetAsync(X->nb, 0, sizeof(int32_t) * k, s));
  TRY(hipMemsetAsync(X->flag, 0, n, s));
  TRY(hipMemsetAsync(X->sumc, 0, sizeof(unsigned long long) * k, s));
  TRY(hipMemsetAsync(X->total, 0, sizeof(unsigned long long), s));
  TRY(hipMemsetAsync(X->err, 0, sizeof(u32), s));
  spq::PartArgs pa{};
  pa.n = n; pa.k = k; pa.m = m;
  pa.eu = eu; pa.ev = ev; pa.w = w; pa.part = part;
  pa.cnt = X->cnt; pa.nb = X->nb; pa.flag = X->flag; pa.sumc = X->sumc;
  pa.total = X->total; pa.err = X->err;
  TRY(spq::launch_partition_scan(pa, s));
  u32 herr = 0;
  unsigned long long htotal = 0;
  X->h_cnt.resize(k);
  X->h_nb.resize(k);
  X->h_sumc.resize(k);
  TRY(hipMemcpyAsync(&herr, X->err, sizeof(u32), hipMemcpyDeviceToHost, s));
  TRY(hipMemcpyAsync(&htotal, X->total, sizeof(htotal), hipMemcpyDeviceToHost, s));
  TRY(hipMemcpyAsync(X->h_cnt.data(), X->cnt, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
  TRY(hipMemcpyAsync(X->h_nb.data(), X->nb, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
  TRY(hipMemcpyAsync(X->h_sumc.data(), X->sumc, sizeof(unsigned long long) * k,
                     hipMemcpyDeviceToHost, s));
  TRY(hipStreamSynchronize(s));
  if (herr & spq::ERR_PART) return guard(fail(SPQ_EINVAL, "part[v] outside [0, k)"));
  if (herr & spq::ERR_VERTEX) return guard(fail(SPQ_EINVAL, "edge endpoint outside [0, n)"));
  if (herr & spq::ERR_WEIGHT) return guard(fail(SPQ_EINVAL, "edge weight outside [0, SPQ_INF)"));
  for (int32_t c = 0; c < k; c++)
    if (X->h_cnt[c] == 0) return guard(fail(SPQ_EINVAL, "component " + std::to_string(c) + " is empty"));
  // Every finite distance is at most the total edge weight, so below SPQ_INF
  // all sums stay exact.  Otherwise the build certifies its result (range.hip),
  // which needs every component's own weight below SPQ_INF.
  if (htotal >= (unsigned long long)SPQ_INF) {
    X->certify = true;
    if (share_comps > 0)
      return guard(fail(SPQ_ERANGE, "total edge weight " + std::to_string(htotal) +
                                        " reaches SPQ_INF; a share build needs it below"));
    for (int32_t c = 0; c < k; c++)
      if (X->h_sumc[c] >= (unsigned long long)SPQ_INF)
        return guard(fail(SPQ_ERANGE, "edge weights inside component " + std::to_string(c) +
                                          " reach SPQ_INF; distances might not fit in int32"));
  }

  X->h_off.assign(k + 1, 0);
  X->h_bgoff.assign(k + 1, 0);
  X->h_P.resize(k);
  X->h_moff.resize(k);
  for (int32_t c = 0; c < k; c++) {
    X->h_off[c + 1] = X->h_off[c] + X->h_cnt[c];
    X->h_bgoff[c + 1] = X->h_bgoff[c] + X->h_nb[c];
    // components above BIG_COMP vertices are closed by the multi-workgroup
    // blocked rounds (128-tiles); the rest one workgroup each
    const bool big = X->h_cnt[c] > spq::BIG_COMP;
    X->h_P[c] = (int32_t)round_up(X->h_cnt[c], big ? 128 : spq::COMP_TILE);
    X->h_moff[c] = X->comp_elems;
    X->comp_elems += (int64_t)X->h_P[c] * X->h_P[c];
    X->max_comp = std::max(X->max_comp, X->h_cnt[c]);
    X->max_nb = std::max(X->max_nb, X->h_nb[c]);
    X->relax_comp += (double)X->h_cnt[c] * X->h_cnt[c] * X->h_cnt[c];
    if (big) {
      X->relax_comp_exec += spq::dense_fw_exec_relax(X->h_P[c] / 128, 128, X->cpivot);
      X->nbig++;
    } else {
      // one workgroup runs the blocked rounds on 64-tiles, i <= j interior tiles only
      const int64_t ntc = X->h_P[c] / spq::COMP_TILE;
      X->relax_comp_exec += (double)ntc * 64.0 * 64.0 * 64.0 *
                            (1.0 + (ntc - 1) + (double)(ntc - 1) * ntc / 2.0);
    }
  }
  X->V = X->h_bgoff[k];
  X->relax_bg = (double)X->V * X->V * X->V;
  X->method = method_opt ? method_opt : (X->V > 32768 || share_comps > 0 ? 2 : 1);
  X->share_comps = share_comps;
  int32_t cpg = k;
  if (X->method == 2) {
    if (group_comps > 0) {
      cpg = std::min(group_comps, k);
    } else {
      // about 4,096 BG vertices per group, a power of two of components
      const double avg_nb = std::max(1.0, (double)X->V / k);
      cpg = 1;
      while (cpg * 2 <= k && cpg * 2 * avg_nb <= 4096.0 * 1.41) cpg *= 2;
    }
  }
  // groups = runs of consecutive components: cpg each, or (group_bg) as many
  // as keep the group within group_bg BG vertices
  std::vector<int32_t> gstart;
  if (X->method == 2 && group_bg > 0) {
    int32_t held = 0;
    for (int32_t c = 0; c < k; c++) {
      if (gstart.empty() || (held > 0 && held + X->h_nb[c] > group_bg)) {
        gstart.push_back(c);
        held = 0;
      }
      held += X->h_nb[c];
    }
  } else {
    for (int32_t c = 0; c < k; c += cpg) gstart.push_back(c);
    // Every group matrix is padded to the widest group (whole 128-tiles).
    // In a share build, when a few groups reach one tile past almost all the
    // others (grid2048, 16 components per group: 6 of 1,024 above 896 BG
    // vertices), they are cut in halves of consecutive components until they
    // fit the tile count of the 99th percentile, so the others are not
    // padded for them.  (The Bellman-Ford blocks follow the component
    // ranges, not the group count, so the cut shifts none of them.)
    if (X->method == 2 && share_comps > 0 && gstart.size() >= 100) {
      std::vector<int32_t> sorted;
      for (size_t g = 0; g < gstart.size(); g++)
        sorted.push_back(X->h_bgoff[g + 1 < gstart.size() ? gstart[g + 1] : k] -
                         X->h_bgoff[gstart[g]]);
      std::sort(sorted.begin(), sorted.end());
      const int64_t cap = round_up(std::max<int32_t>(1, sorted[(sorted.size() * 99) / 100]), 128);
      if (cap < round_up(sorted.back(), 128)) {
        std::vector<int32_t> cut;
        std::vector<std::pair<int32_t, int32_t>> todo;
        for (size_t g = 0; g < gstart.size(); g++) {
          todo.emplace_back(gstart[g], g + 1 < gstart.size() ? gstart[g + 1] : k);
          while (!todo.empty()) {
            const auto r = todo.back();
            todo.pop_back();
            if (r.second - r.first > 1 && X->h_bgoff[r.second] - X->h_bgoff[r.first] > cap) {
              const int32_t mid = r.first + (r.second - r.first) / 2;
              todo.emplace_back(mid, r.second);  // the lower half first
              todo.emplace_back(r.first, mid);
            } else {
              cut.push_back(r.first);
            }
          }
        }
        gstart.swap(cut);
      }
    }
  }
  X->group_bg = X->method == 2 && group_bg > 0;
  X->h_gfirst = gstart;
  X->ngroups = (int32_t)gstart.size();
  gstart.push_back(k);
  // group pairs index launch grids (up to ngroups^2 workgroups per launch of
  // the certificate check, ngroups along a grid's y dimension elsewhere)
  if (X->ngroups > 32768)
    return guard(fail(SPQ_EINVAL, "more than 32,768 groups: raise group_comps or group_bg"));
  X->cpg = cpg;
  X->h_grp.resize(k);
  X->h_gbg0.resize(X->ngroups);
  X->h_gV.resize(X->ngroups);
  for (int32_t g = 0; g < X->ngroups; g++) {
    for (int32_t c = gstart[g]; c < gstart[g + 1]; c++) X->h_grp[c] = g;
    X->h_gbg0[g] = X->h_bgoff[gstart[g]];
    X->h_gV[g] = X->h_bgoff[gstart[g + 1]] - X->h_gbg0[g];
    X->Vgp = std::max<int32_t>(X->Vgp, (int32_t)round_up(X->h_gV[g], 128));
  }
  if (X->method == 1) {
    X->Vp = (int32_t)round_up(X->V, tile);
    const int64_t nt = X->Vp / tile;
    X->relax_bg_exec = spq::dense_fw_exec_relax(nt, tile, X->pivot, &X->relax_inner);
    if (X->relax_inner > 0) {
      X->inner_launches = spq::fw_rounds_count((int)nt, tile, X->pivot);
    }
  } else {
    X->Vgp = std::max<int32_t>(X->Vgp, 128);
    // the composition stores a group pair's block with 32-bit offsets
    if (X->Vgp > 32768)
      return guard(fail(SPQ_EINVAL, "a group holds more than 32,768 BG vertices: lower "
                                    "group_comps or group_bg"));
    X->relax_bg_exec = X->ngroups * spq::dense_fw_exec_relax(X->Vgp / 128, 128, X->cpivot);
  }
  X->h_order.resize(k);
  std::iota(X->h_order.begin(), X->h_order.end(), 0);
  std::stable_sort(X->h_order.begin(), X->h_order.end(),
                   [&](int32_t a, int32_t b) { return X->h_P[a] > X->h_P[b]; });

  // ---- index memory
  TRY(dalloc(&X->comp, n));
  TRY(dalloc(&X->local, n));
  TRY(dalloc(&X->off, k + 1));
  TRY(dalloc(&X->bgoff, k + 1));
  TRY(dalloc(&X->P, k));
  TRY(dalloc(&X->order, k));
  TRY(dalloc(&X->moff, k));
  TRY(dalloc(&X->bgcomp, X->V));
  TRY(dalloc(&X->bglocal, X->V));
  TRY(dalloc(&X->bgvert, X->V));
  TRY(dalloc(&X->fill, k));
  TRY(dalloc(&X->members, n));
  TRY(dalloc(&X->vrec, spq::VREC_WORDS * (int64_t)n));
  TRY(dalloc(&X->M, X->comp_elems));
  if (X->method == 1 && X->Vp > 0) TRY(dalloc(&X->BG, (int64_t)X->Vp * X->Vp));
  TRY(dalloc(&X->grp, k));
  TRY(dalloc(&X->gbg0, X->ngroups));
  TRY(dalloc(&X->gV, X->ngroups));
  TRY(hipMemcpyAsync(X->grp, X->h_grp.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->gbg0, X->h_gbg0.data(), sizeof(int32_t) * X->ngroups, hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->gV, X->h_gV.data(), sizeof(int32_t) * X->ngroups, hipMemcpyHostToDevice, s));
  // band of each group in the blocked store: the full store keeps group pairs
  // S1 <= S2 (rows of S1 against S1 .. last), a share keeps share groups
  // against all groups, the flat method one group
  X->h_gT.assign(X->ngroups, 0);
  {
    const int32_t sg = share_comps > 0 ? X->h_grp[share_comps - 1] + 1 : X->ngroups;
    int64_t t = 0;
    for (int32_t g = 0; g < sg; g++) {
      X->h_gT[g] = t;
      t += (int64_t)X->h_gV[g] * (share_comps > 0 ? X->V : X->V - X->h_gbg0[g]);
    }
  }
  TRY(dalloc(&X->gT, X->ngroups));
  TRY(hipMemcpyAsync(X->gT, X->h_gT.data(), sizeof(int64_t) * X->ngroups, hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->off, X->h_off.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->bgoff, X->h_bgoff.data(), sizeof(int32_t) * (k + 1), hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->P, X->h_P.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->order, X->h_order.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
  TRY(hipMemcpyAsync(X->moff, X->h_moff.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
  TRY(hipMemsetAsync(X->fill, 0, sizeof(int32_t) * k, s));
  if (X->graph) {
    // the captured kernels read the index's own copies of the edges
    TRY(dalloc(&X->eu_own, m));
    TRY(dalloc(&X->ev_own, m));
    TRY(dalloc(&X->w_own, m));
    if (m > 0) {
      TRY(hipMemcpyAsync(X->eu_own, eu, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
      TRY(hipMemcpyAsync(X->ev_own, ev, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
      TRY(hipMemcpyAsync(X->w_own, w, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
    }
    eu = X->eu_own;
    ev = X->ev_own;
    w = X->w_own;
    TRY(stream_take(&X->cap));
  }

  if (use_paths) {
    // adjacency for the path walk; the weights it reads follow reweighting
    if (m > 0x7fffffff) return guard(fail(SPQ_EINVAL, "SPQ_PATHS needs m < 2^31"));
    X->paths = true;
    TRY(dalloc(&X->rowptr, (int64_t)n + 1));
    TRY(dalloc(&X->adj, 2 * m));
    TRY(dalloc(&X->adeg, n));
    TRY(hipMemsetAsync(X->adeg, 0, sizeof(unsigned long long) * n, s));
    TRY(spq::launch_adjacency(n, m, eu, ev, X->adeg, X->rowptr, X->adj, s));
    if (X->graph) {
      X->w_path = X->w_own;
    } else {
      TRY(dalloc(&X->w_copy, m));
      if (m > 0) TRY(hipMemcpyAsync(X->w_copy, w, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s));
      X->w_path = X->w_copy;
    }
  }

  // ---- renumbering (Section 4, Fig. 1)
  pa.off = X->off; pa.bgoff = X->bgoff; pa.fill = X->fill; pa.members = X->members;
  pa.comp = X->comp; pa.local = X->local; pa.bgcomp = X->bgcomp; pa.bglocal = X->bglocal;
  pa.moff = X->moff; pa.P = X->P; pa.vrec = X->vrec; pa.grp = X->grp; pa.gbg0 = X->gbg0;
  pa.gV = X->gV; pa.gT = X->gT; pa.bgvert = X->bgvert;
  TRY(spq::launch_renumber(pa, s));
  if (X->certify) {
    spq_status cs = cc_labels(X, m, eu, ev, s);
    if (cs != SPQ_OK) return guard(cs);
  }
  TRY(hipEventRecord(X->ev[1], s));

  // ---- Phase 2: APSP(C) for every component
  spq::CompArgs ca{};
  ca.k = k; ca.m = m; ca.eu = eu; ca.ev = ev; ca.w = w; ca.comp = X->comp; ca.local = X->local;
  ca.P = X->P; ca.moff = X->moff; ca.M = X->M;
  auto phase2 = [&](hipStream_t st) -> hipError_t {
    hipError_t e = spq::launch_components(ca, st);
    if (plain) {
      // order[] lists components largest first: the big ones lead
      for (int32_t b = 0; b < X->nbig && e == hipSuccess; b++) {
        const int32_t c = X->h_order[b];
        e = spq::launch_dense_fw(X->M + X->h_moff[c], X->h_P[c], 128, X->h_P[c] / 128, st, nullptr,
                                 inner_kc, X->cpivot);
      }
    } else {
      // runs of consecutive big components of one padded size lie back to
      // back in M (offsets follow the ids): one batched closure per run
      for (int32_t c = 0; c < k && e == hipSuccess;) {
        if (X->h_cnt[c] <= spq::BIG_COMP) {
          c++;
          continue;
        }
        const int32_t P = X->h_P[c];
        int32_t c2 = c + 1;
        while (c2 < k && c2 - c < 65535 && X->h_cnt[c2] > spq::BIG_COMP && X->h_P[c2] == P) c2++;
        e = spq::launch_dense_fw_batch(X->M + X->h_moff[c], P, 128, P / 128, c2 - c, (int64_t)P * P, st,
                                       nullptr, inner_kc, X->cpivot);
        c = c2;
      }
    }
    if (e != hipSuccess) return e;
    if (plain) {
      for (int32_t c = X->nbig; c < k && e == hipSuccess; c++)
        e = spq::launch_comp_fw(1, X->order + c, X->P, X->moff, X->M, st);
    } else {
      e = spq::launch_comp_fw(k - X->nbig, X->order + X->nbig, X->P, X->moff, X->M, st);
    }
    if (e == hipSuccess && !X->graph) e = hipEventRecord(X->ev[2], st);
    return e;
  };
  if (X->graph) {
    // one graph covers the phases: no split of their device time
    TRY(hipEventRecord(X->ev[2], s));
    TRY(hipEventRecord(X->ev[3], s));
  }

  // ---- Phase 3: BG and its all-pairs distances
  if (X->method == 2) {
    spq::HierArgs ha{};
    const int32_t G = X->ngroups, V = X->V, Vgp = X->Vgp;
    TRY(dalloc(&X->Mg, (int64_t)G * Vgp * Vgp));
    TRY(dalloc(&X->flag2, V));
    TRY(dalloc(&X->b2list, (int64_t)G * Vgp));
    TRY(dalloc(&X->b2rank, V));
    TRY(dalloc(&X->m2, G));
    TRY(dalloc(&X->b2off, G + 1));
    TRY(dalloc(&X->bgrow, V));
    TRY(dalloc(&X->bgnb, V));
    TRY(dalloc(&X->bggrp, V));
    // level-2 boundary flags depend on the edges only and are only ever set
    if (V > 0) TRY(hipMemsetAsync(X->flag2, 0, V, s));
    ha.V = V; ha.ngroups = G; ha.Vgp = Vgp; ha.m = m; ha.kc = inner_kc; ha.pivot = X->cpivot;
    ha.eu = eu; ha.ev = ev; ha.w = w; ha.comp = X->comp; ha.local = X->local; ha.bgoff = X->bgoff;
    ha.nb = X->nb; ha.bgcomp = X->bgcomp; ha.bglocal = X->bglocal; ha.P = X->P; ha.moff = X->moff;
    ha.M = X->M; ha.grp = X->grp; ha.gbg0 = X->gbg0; ha.gV = X->gV; ha.bgrow = X->bgrow;
    ha.bgnb = X->bgnb; ha.bggrp = X->bggrp; ha.Mg = X->Mg; ha.flag2 = X->flag2; ha.b2list = X->b2list;
    ha.b2rank = X->b2rank; ha.m2 = X->m2;
    // the closures of this path (the groups' and super-groups' batches, BG2
    // or BG3) run with the lookahead of the flat method; a share build keeps
    // to one stream
    if (lookahead && X->share_comps == 0) {
      TRY(stream_take(&X->side));
      for (auto& e : X->la_sync) TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ha.side = X->side;
      ha.sync = X->la_sync;
    }
    TRY(graph_segment(X, s, [&](hipStream_t st) -> hipError_t {
      hipError_t e = phase2(st);
      if (e == hipSuccess && !X->graph) e = hipEventRecord(X->ev[3], st);
      if (e == hipSuccess) e = spq::launch_hier_level1(ha, st);
      return e;
    }));
    X->h_m2.resize(G);
    TRY(hipMemcpyAsync(X->h_m2.data(), X->m2, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    X->h_b2off.assign(G + 1, 0);
    int32_t m2max = 0;
    for (int32_t g = 0; g < G; g++) {
      X->h_b2off[g + 1] = X->h_b2off[g] + X->h_m2[g];
      m2max = std::max(m2max, X->h_m2[g]);
    }
    X->V2 = X->h_b2off[G];
    X->V2p = round_up(X->V2, 128);
    X->m2pmax = (int32_t)std::max<int64_t>(128, round_up(m2max, 128));
    if (X->share_comps > 0) {
      spq_status ss = build_share(X, ha, m, profile, level3_opt, s);
      if (ss != SPQ_OK) return guard(ss);
      TRY(hipEventRecord(X->ev[4], s));
      *out = X;
      return SPQ_OK;
    }
    X->h_pairbase.assign((size_t)G * G, 0);
    for (int32_t a1 = 0; a1 < G; a1++)
      for (int32_t a2 = a1; a2 < G; a2++) {
        X->h_pairbase[(size_t)a1 * G + a2] = X->h_elems;
        X->h_elems += (int64_t)X->h_gV[a1] * X->h_gV[a2];
      }
    if (!bands_match(X, G, false)) return guard(fail(SPQ_EDEVICE, "internal: band layout"));
    // level 3: BG2 above 16,384 vertices (or as asked) is closed by super-groups
    if (X->V2 > 0 && level3_opt >= 0) {
      int32_t gpt = 0;
      if (level3_opt > 0) {
        gpt = std::min(level3_opt, G);
      } else if (X->V2 > 16384) {
        // about 4,096 BG2 vertices per super-group, a power of two of groups
        const double avg = (double)X->V2 / G;
        gpt = 1;
        while (gpt * 2 <= G && gpt * 2 * avg <= 4096.0 * 1.41) gpt *= 2;
        if (gpt >= G) gpt = 0;
      }
      if (gpt > 0) {
        X->gpt = gpt;
        X->nT = (G + gpt - 1) / gpt;
        X->h_tbase.resize(X->nT);
        X->h_tsize.resize(X->nT);
        int32_t tmax = 0;
        for (int32_t t = 0; t < X->nT; t++) {
          X->h_tbase[t] = X->h_b2off[t * gpt];
          X->h_tsize[t] = X->h_b2off[std::min((t + 1) * gpt, G)] - X->h_tbase[t];
          tmax = std::max(tmax, X->h_tsize[t]);
        }
        X->V3gp = (int32_t)std::max<int64_t>(128, round_up(tmax, 128));
      }
    }
    // executed relaxations of level 2 (its BG2 closure is counted with level 3)
    if (X->V2p > 0 && X->nT == 0)
      X->relax_bg_exec += spq::dense_fw_exec_relax(X->V2p / 128, 128, X->cpivot);
    set_positions(X);
    const int32_t Vrp = X->Vrp;
    for (int32_t a1 = 0; a1 < G; a1++)
      for (int32_t a2 = a1; a2 < G; a2++) {
        if (X->V2p > 0) X->relax_bg_exec += xt_relax(X, a1, a2);
        const double y = y_relax(X, a1, a2);
        X->relax_bg_exec += y;
        X->relax_inner += y;
      }
    TRY(make_pairs(G, G, true, (int64_t)X->m2pmax * Vrp, X->h_elems, &X->plist, &X->npairs,
                   &X->chunk, s));
    X->inner_launches = (X->npairs + X->chunk - 1) / X->chunk;
    if (profile) {
      X->prof.resize(2 * X->inner_launches);
      for (auto& e : X->prof) TRY(hipEventCreate(&e));
      ha.evt = X->prof.data();
    }
    TRY(hipMemcpyAsync(X->b2off, X->h_b2off.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, s));
    // R's last row is read up to 127 words past its end (the second
    // product's column tiles start past the B2 positions)
    TRY(dalloc(&X->R, (int64_t)G * X->m2pmax * Vrp + 128));
    TRY(dalloc(&X->pos, (int64_t)G * Vrp));
    TRY(dalloc(&X->XT, (int64_t)X->chunk * X->m2pmax * Vrp));
    if (X->V2p > 0) TRY(dalloc(&X->BG2, X->V2p * X->V2p));
    TRY(dalloc(&X->H, X->h_elems));
    TRY(dalloc(&X->pairbase, (int64_t)G * G));
    TRY(hipMemcpyAsync(X->pairbase, X->h_pairbase.data(), sizeof(int64_t) * G * G,
                       hipMemcpyHostToDevice, s));
    ha.m2pmax = X->m2pmax; ha.V2 = X->V2; ha.V2p = X->V2p; ha.b2off = X->b2off; ha.R = X->R;
    ha.XT = X->XT; ha.BG2 = X->BG2; ha.H = X->H; ha.pairbase = X->pairbase;
    ha.pos = X->pos; ha.Vrp = Vrp;
    ha.plist = X->plist; ha.npairs = X->npairs; ha.chunk = X->chunk;
    if (X->certify) {
      ha.bglabel = X->bglabel;
      ha.cert_bad = X->cert + 1;
      ha.cert_mbg = X->cert + 3;
      X->fused_cert = true;
    }
    if (X->nT == 0) {
      TRY(graph_segment(X, s, [&](hipStream_t st) -> hipError_t {
        hipError_t e = spq::launch_hier_level2_prep(ha, st);
        if (e == hipSuccess) e = spq::launch_hier_level2_close(ha, st);
        if (e == hipSuccess) e = spq::launch_hier_level2_compose(ha, st);
        return e;
      }));
    } else {
      const int32_t nT = X->nT, V3gp = X->V3gp;
      TRY(dalloc(&X->tbase, nT));
      TRY(dalloc(&X->tsize, nT));
      TRY(dalloc(&X->M3, (int64_t)nT * V3gp * V3gp));
      TRY(dalloc(&X->flag3, X->V2));
      TRY(dalloc(&X->b3list, (int64_t)nT * V3gp));
      TRY(dalloc(&X->b3rank, X->V2));
      TRY(dalloc(&X->m3, nT));
      TRY(dalloc(&X->b3off, nT + 1));
      TRY(hipMemcpyAsync(X->tbase, X->h_tbase.data(), sizeof(int32_t) * nT, hipMemcpyHostToDevice, s));
      TRY(hipMemcpyAsync(X->tsize, X->h_tsize.data(), sizeof(int32_t) * nT, hipMemcpyHostToDevice, s));
      // level-3 boundary flags depend on the edges only and are only ever set
      TRY(hipMemsetAsync(X->flag3, 0, X->V2, s));
      spq::L3Args la{};
      la.nT = nT; la.gpt = X->gpt; la.V3gp = V3gp; la.kc = inner_kc; la.pivot = X->cpivot; la.m = m; la.V2p = X->V2p;
      la.eu = eu; la.ev = ev; la.w = w; la.comp = X->comp; la.local = X->local; la.bgoff = X->bgoff;
      la.grp = X->grp; la.b2off = X->b2off; la.b2rank = X->b2rank; la.BG2 = X->BG2;
      la.tbase = X->tbase; la.tsize = X->tsize; la.M3 = X->M3; la.flag3 = X->flag3;
      la.b3list = X->b3list; la.b3rank = X->b3rank; la.m3 = X->m3;
      la.side = ha.side; la.sync = ha.sync;
      TRY(graph_segment(X, s, [&](hipStream_t st) -> hipError_t {
        hipError_t e = spq::launch_hier_level2_prep(ha, st);
        if (e == hipSuccess) e = spq::launch_level3_a(la, st);
        return e;
      }));
      X->h_m3.resize(nT);
      TRY(hipMemcpyAsync(X->h_m3.data(), X->m3, sizeof(int32_t) * nT, hipMemcpyDeviceToHost, s));
      TRY(hipStreamSynchronize(s));
      X->h_b3off.assign(nT + 1, 0);
      int32_t m3max = 0;
      for (int32_t t = 0; t < nT; t++) {
        X->h_b3off[t + 1] = X->h_b3off[t] + X->h_m3[t];
        m3max = std::max(m3max, X->h_m3[t]);
      }
      X->V3 = X->h_b3off[nT];
      X->V3p = round_up(X->V3, 128);
      X->m3pmax = (int32_t)std::max<int64_t>(128, round_up(m3max, 128));
      // the super-groups' positions (B3 vertices first, as the groups' at
      // level 2): widths and their bound V3rp
      std::vector<int32_t> w3(nT);
      int64_t w3max = 0;
      for (int32_t t = 0; t < nT; t++) {
        w3[t] = (int32_t)round_up(X->h_m3[t], 4) + X->h_tsize[t] - X->h_m3[t];
        w3max = std::max<int64_t>(w3max, w3[t]);
      }
      const int32_t V3rp = (int32_t)std::max<int64_t>(128, round_up(w3max, 128));
      // executed relaxations of level 3 (the first product over T1's
      // vertices outside B3, its B3 positions being copied; the second over
      // T2's vertices outside B3)
      X->relax_bg_exec += nT * spq::dense_fw_exec_relax(V3gp / 128, 128, X->cpivot);
      if (X->V3p > 0) X->relax_bg_exec += spq::dense_fw_exec_relax(X->V3p / 128, 128, X->cpivot);
      for (int32_t t1 = 0; t1 < nT; t1++)
        for (int32_t t2 = t1; t2 < nT; t2++) {
          if (X->V3p > 0)
            X->relax_bg_exec += mp_rows(X->h_m3[t2]) * mp_cols(X->h_tsize[t1] - X->h_m3[t1]) *
                                (double)round_up(X->h_m3[t1], 16);
          X->relax_bg_exec += mp_rows(w3[t1]) * mp_cols(X->h_tsize[t2] - X->h_m3[t2]) *
                              (double)round_up(X->h_m3[t2], 16);
        }
      TRY(hipMemcpyAsync(X->b3off, X->h_b3off.data(), sizeof(int32_t) * (nT + 1),
                         hipMemcpyHostToDevice, s));
      // R3's last row is read up to 127 words past its end (as R's)
      TRY(dalloc(&X->R3, (int64_t)nT * X->m3pmax * V3rp + 128));
      TRY(dalloc(&X->pos3, (int64_t)nT * V3rp));
      int32_t np3 = 0, ch3 = 0;
      TRY(make_pairs(nT, nT, true, (int64_t)X->m3pmax * V3rp, X->V2p * X->V2p / 2, &X->plist3,
                     &np3, &ch3, s));
      TRY(dalloc(&X->XT3, (int64_t)ch3 * X->m3pmax * V3rp));
      la.plist = X->plist3; la.npairs = np3; la.chunk = ch3;
      la.pos3 = X->pos3; la.V3rp = V3rp;
      if (X->V3p > 0) TRY(dalloc(&X->BG3, X->V3p * X->V3p));
      la.V3 = X->V3; la.V3p = X->V3p; la.m3pmax = X->m3pmax; la.b3off = X->b3off; la.R3 = X->R3;
      la.XT3 = X->XT3; la.BG3 = X->BG3; la.side = ha.side; la.sync = ha.sync;
      TRY(graph_segment(X, s, [&](hipStream_t st) -> hipError_t {
        hipError_t e = spq::launch_level3_b(la, st);
        if (e == hipSuccess) e = spq::launch_hier_level2_compose(ha, st);
        return e;
      }));
    }
    TRY(hipEventRecord(X->ev[4], s));
    spq_status cs = certify(X, s);
    if (cs != SPQ_OK) return guard(cs);
    *out = X;
    return SPQ_OK;
  }
  spq::BgArgs ba{};
  ba.V = X->V; ba.Vp = X->Vp; ba.m = m; ba.eu = eu; ba.ev = ev; ba.w = w;
  ba.comp = X->comp; ba.local = X->local; ba.bgoff = X->bgoff; ba.nb = X->nb;
  ba.bgcomp = X->bgcomp; ba.bglocal = X->bglocal; ba.P = X->P; ba.moff = X->moff;
  ba.M = X->M; ba.BG = X->BG;
  if (profile && X->inner_launches > 0) {
    X->prof.resize(2 * X->inner_launches);
    for (auto& e : X->prof) TRY(hipEventCreate(&e));
  }
  // the blocked store the queries read (one group: the whole V x V matrix)
  const int32_t V = X->V;
  TRY(dalloc(&X->bgrow, V));
  TRY(dalloc(&X->bgnb, V));
  TRY(dalloc(&X->bggrp, V));
  X->h_elems = (int64_t)V * V;
  TRY(dalloc(&X->H, X->h_elems));
  TRY(dalloc(&X->pairbase, 1));
  TRY(hipMemsetAsync(X->pairbase, 0, sizeof(int64_t), s));
  const bool la = lookahead && X->Vp / tile > 1;
  if (la) {
    TRY(stream_take(&X->side));
    TRY(stream_take(&X->part1));
    for (auto& e : X->la_sync) TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  hipEvent_t* pev = X->prof.empty() ? nullptr : X->prof.data();
  TRY(graph_segment(X, s, [&](hipStream_t st) -> hipError_t {
    hipError_t e = phase2(st);
    if (e == hipSuccess) e = spq::launch_bg_assembly(ba, st);
    if (e == hipSuccess && !X->graph) e = hipEventRecord(X->ev[3], st);
    if (e != hipSuccess) return e;
    if (la)
      e = spq::launch_dense_fw_lookahead(X->BG, X->Vp, tile, X->Vp / tile, st, X->side, X->la_sync,
                                         pev, inner_kc, X->pivot, X->part1);
    else
      e = spq::launch_dense_fw(X->BG, X->Vp, tile, X->Vp / tile, st, pev, inner_kc, X->pivot);
    if (e != hipSuccess) return e;
    return spq::launch_flat_store(V, X->Vp, X->BG, X->bgcomp, X->bgoff, X->nb, X->grp, X->gbg0,
                                  X->bgrow, X->bgnb, X->bggrp, X->bglocal, X->H, st);
  }));
  TRY(hipEventRecord(X->ev[4], s));
#undef TRY
  spq_status cs = certify(X, s);
  if (cs != SPQ_OK) return guard(cs);
  *out = X;
  return SPQ_OK;
}

// Replays the captured Phase 2-3 graphs with new weights (see spq.h).
spq_status spq_reweight_index(spq_index* X, const int32_t* w, void* stream) {
  g_err.clear();
  if (!X) return fail(SPQ_EINVAL, "index is NULL");
  if (!X->graph) return fail(SPQ_EINVAL, "index was built without SPQ_GRAPH");
  if (!X->valid) return fail(SPQ_ERANGE, "index invalidated by a failed reweight");
  if (X->m > 0 && !w) return fail(SPQ_EINVAL, "w is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int32_t k = X->k;
  HIP_TRY(hipStreamWaitEvent(s, X->ev[4], 0));
  HIP_TRY(hipEventRecord(X->ev[0], s));
  // validate the new weights and sum them, per component and in total
  HIP_TRY(hipMemsetAsync(X->sumc, 0, sizeof(unsigned long long) * k, s));
  HIP_TRY(hipMemsetAsync(X->total, 0, sizeof(unsigned long long), s));
  HIP_TRY(hipMemsetAsync(X->err, 0, sizeof(u32), s));
  spq::PartArgs pa{};
  pa.n = X->n; pa.k = k; pa.m = X->m; pa.eu = X->eu_own; pa.ev = X->ev_own; pa.w = w;
  pa.part = X->comp; pa.flag = X->flag; pa.sumc = X->sumc; pa.total = X->total; pa.err = X->err;
  HIP_TRY(spq::launch_edges_scan(pa, s));
  u32 herr = 0;
  unsigned long long htotal = 0;
  HIP_TRY(hipMemcpyAsync(&herr, X->err, sizeof(u32), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&htotal, X->total, sizeof(htotal), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(X->h_sumc.data(), X->sumc, sizeof(unsigned long long) * k,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr & spq::ERR_WEIGHT) return fail(SPQ_EINVAL, "edge weight outside [0, SPQ_INF)");
  if (herr) return fail(SPQ_EDEVICE, "edge scan reported an inconsistent index");
  const bool cert = htotal >= (unsigned long long)SPQ_INF;
  if (cert)
    for (int32_t c = 0; c < k; c++)
      if (X->h_sumc[c] >= (unsigned long long)SPQ_INF)
        return fail(SPQ_ERANGE, "edge weights inside component " + std::to_string(c) +
                                    " reach SPQ_INF; distances might not fit in int32");
  // commit: from here on the index holds the new weights
  if (X->m > 0)
    HIP_TRY(hipMemcpyAsync(X->w_own, w, sizeof(int32_t) * X->m, hipMemcpyDeviceToDevice, s));
  X->certify = cert;
  if (cert) {
    if (!X->label) {
      spq_status cs = cc_labels(X, X->m, X->eu_own, X->ev_own, s);
      if (cs != SPQ_OK) {
        X->valid = false;
        return cs;
      }
    }
    HIP_TRY(hipMemsetAsync(X->cert, 0, 4 * sizeof(u32), s));
  }
  HIP_TRY(hipEventRecord(X->ev[1], s));
  HIP_TRY(hipEventRecord(X->ev[2], s));
  HIP_TRY(hipEventRecord(X->ev[3], s));
  for (hipGraphExec_t x : X->execs) HIP_TRY(hipGraphLaunch(x, s));
  HIP_TRY(hipEventRecord(X->ev[4], s));
  spq_status cs = certify(X, s);
  if (cs != SPQ_OK) {
    X->valid = false;
    return cs;
  }
  X->reweights++;
  return SPQ_OK;
}

spq_status spq_query_batch(const spq_index* X, int64_t q, const int32_t* v1, const int32_t* v2,
                           int32_t* out, void* stream) {
  if (!X) return fail(SPQ_EINVAL, "index is NULL");
  if (!X->valid) return fail(SPQ_ERANGE, "index invalidated by a failed reweight");
  if (q < 0) return fail(SPQ_EINVAL, "q < 0");
  if (q == 0) return SPQ_OK;
  if (!v1 || !v2 || !out) return fail(SPQ_EINVAL, "null query array");
  spq::QueryArgs a{};
  a.q = q; a.v1 = v1; a.v2 = v2; a.out = out; a.n = X->n;
  a.vrec = X->vrec; a.M = X->M; a.H = X->H; a.share_comps = X->share_comps;
  HIP_TRY(spq::launch_query(a, reinterpret_cast<hipStream_t>(stream)));
  return SPQ_OK;
}

spq_status spq_query_paths(const spq_index* X, int64_t q, const int32_t* v1, const int32_t* v2,
                           int32_t max_len, int32_t* paths, int32_t* lens, void* stream) {
  if (!X) return fail(SPQ_EINVAL, "index is NULL");
  if (!X->paths) return fail(SPQ_EINVAL, "index was built without SPQ_PATHS");
  if (!X->valid) return fail(SPQ_ERANGE, "index invalidated by a failed reweight");
  if (q < 0 || max_len < 1) return fail(SPQ_EINVAL, "need q >= 0 and max_len >= 1");
  if (q == 0) return SPQ_OK;
  if (!v1 || !v2 || !paths || !lens) return fail(SPQ_EINVAL, "null array");
  spq::QueryArgs a{};
  a.q = q; a.v1 = v1; a.v2 = v2; a.n = X->n;
  a.vrec = X->vrec; a.M = X->M; a.H = X->H; a.share_comps = X->share_comps;
  HIP_TRY(spq::launch_paths(a, max_len, X->rowptr, X->adj, X->w_path, paths, lens,
                            reinterpret_cast<hipStream_t>(stream)));
  return SPQ_OK;
}

spq_status spq_query_batch_host(const spq_index* X, int64_t q, const int32_t* v1, const int32_t* v2,
                                int32_t* out) {
  if (!X) return fail(SPQ_EINVAL, "index is NULL");
  if (!X->valid) return fail(SPQ_ERANGE, "index invalidated by a failed reweight");
  if (q < 0) return fail(SPQ_EINVAL, "q < 0");
  if (q == 0) return SPQ_OK;
  if (!v1 || !v2 || !out) return fail(SPQ_EINVAL, "null query array");
  int32_t* d = nullptr;
  HIP_TRY(dalloc(&d, 3 * q));
  hipStream_t s = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = stream_take(&s);
  // the index may still be building on another stream
  if (e == hipSuccess) e = hipStreamWaitEvent(s, X->ev[4], 0);
  if (e == hipSuccess) e = hipMemcpyAsync(d, v1, sizeof(int32_t) * q, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d + q, v2, sizeof(int32_t) * q, hipMemcpyHostToDevice, s);
  spq_status st = SPQ_OK;
  if (e == hipSuccess) {
    st = spq_query_batch(X, q, d, d + q, d + 2 * q, s);
    if (st == SPQ_OK)
      e = hipMemcpyAsync(out, d + 2 * q, sizeof(int32_t) * q, hipMemcpyDeviceToHost, s);
  }
  if (s) {
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    if (es == hipSuccess)
      stream_give(dev, s);
    else
      (void)hipStreamDestroy(s);
  }
  pool_release(d);  // the stream has drained: nothing queued uses d any more
  if (st != SPQ_OK) return st;
  HIP_TRY(e);
  return SPQ_OK;
}

// spq_query_batch_host through the fixed staging array (see spq.h): no
// allocation, caller's stream, SPQ_EBUSY while another call holds the array.
spq_status spq_query_batch_host_static(const spq_index* X, int64_t q, const int32_t* v1,
                                       const int32_t* v2, int32_t* out, void* stream) {
  if (!X) return fail(SPQ_EINVAL, "index is NULL");
  if (!X->valid) return fail(SPQ_ERANGE, "index invalidated by a failed reweight");
  if (q < 0) return fail(SPQ_EINVAL, "q < 0");
  if (q > SPQ_STATIC_PAIRS)
    return fail(SPQ_EINVAL, "q = " + std::to_string(q) + " exceeds SPQ_STATIC_PAIRS (" +
                                std::to_string(SPQ_STATIC_PAIRS) + ")");
  if (q == 0) return SPQ_OK;
  if (!v1 || !v2 || !out) return fail(SPQ_EINVAL, "null query array");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SPQ_EINVAL, "device id beyond the library's table");
  StaticScratch& S = g_static[dev];
  std::call_once(S.once, [&S] {
    void* p = nullptr;
    S.init = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (S.init == hipSuccess) S.ptr = static_cast<int32_t*>(p);
  });
  if (S.init != hipSuccess || !S.ptr)
    return fail(SPQ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(S.init != hipSuccess ? S.init : hipErrorUnknown));
  if (S.busy.exchange(true)) return fail(SPQ_EBUSY, "the static query staging is in use on this device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t* d1 = S.ptr;
  int32_t* d2 = S.ptr + SPQ_STATIC_PAIRS;
  int32_t* dout = S.ptr + 2 * (int64_t)SPQ_STATIC_PAIRS;
  const size_t bytes = sizeof(int32_t) * (size_t)q;
  // the index may still be building on another stream
  hipError_t e = hipStreamWaitEvent(s, X->ev[4], 0);
  if (e == hipSuccess) e = hipMemcpyAsync(d1, v1, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d2, v2, bytes, hipMemcpyHostToDevice, s);
  spq_status st = SPQ_OK;
  if (e == hipSuccess) {
    st = spq_query_batch(X, q, d1, d2, dout, s);
    if (st == SPQ_OK) e = hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, s);
  }
  // the array is free again only once nothing queued uses it
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  S.busy.store(false);
  if (st != SPQ_OK) return st;
  HIP_TRY(e);
  return SPQ_OK;
}

// The build from host arrays: staged in pool memory, built on a cached
// stream of the library, waited for (see spq.h).
spq_status spq_build_index_host(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                                const int32_t* w, const int32_t* part, int32_t k,
                                const spq_build_opts* opts, spq_index** out) {
  g_err.clear();
  if (!out) return fail(SPQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || m < 0 || k < 1) return fail(SPQ_EINVAL, "need n >= 1, m >= 0, k >= 1");
  if (!part || (m > 0 && (!eu || !ev || !w))) return fail(SPQ_EINVAL, "null input array");
  int32_t* d = nullptr;
  HIP_TRY(dalloc(&d, 3 * m + n));
  hipStream_t s = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = stream_take(&s);
  const size_t eb = sizeof(int32_t) * (size_t)m;
  if (e == hipSuccess && m > 0) e = hipMemcpyAsync(d, eu, eb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m > 0) e = hipMemcpyAsync(d + m, ev, eb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m > 0) e = hipMemcpyAsync(d + 2 * m, w, eb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d + 3 * m, part, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s);
  spq_status st = SPQ_OK;
  if (e == hipSuccess) st = spq_build_index(n, m, d, d + m, d + 2 * m, d + 3 * m, k, opts, s, out);
  if (s) {
    // the build reads the staged arrays until its queued work is done
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    if (es == hipSuccess)
      stream_give(dev, s);
    else
      (void)hipStreamDestroy(s);
  }
  pool_release(d);
  if (st != SPQ_OK) return st;
  if (e != hipSuccess) {
    spq_free_index(*out);
    *out = nullptr;
  }
  HIP_TRY(e);
  return SPQ_OK;
}

spq_status spq_index_stats(const spq_index* X, spq_stats* st) {
  if (!X || !st) return fail(SPQ_EINVAL, "null argument");
  std::memset(st, 0, sizeof(*st));
  st->n = X->n; st->k = X->k; st->m = X->m; st->v_bg = X->V; st->v_bg_padded = X->Vp;
  st->max_comp = X->max_comp; st->max_boundary = X->max_nb;
  st->comp_bytes = X->comp_elems * 4;
  st->bg_bytes = (int64_t)X->h_elems * 4;
  st->relax_comp = X->relax_comp;
  st->relax_bg = X->relax_bg;
  st->relax_comp_exec = X->relax_comp_exec;
  st->relax_bg_exec = X->relax_bg_exec;
  st->relax_dominant = X->relax_inner;
  st->dominant_launches = X->inner_launches;
  st->bg_method = X->method;
  st->ngroups = X->ngroups;
  st->v_bg2 = X->V2;
  st->share_comps = X->share_comps;
  st->share_groups = X->share_groups;
  st->bf_rounds = X->bf_rounds;
  st->bf_block_groups = X->share_comps > 0 ? X->bgpt : 0;
  st->graphs = (int32_t)X->execs.size();
  st->reweights = X->reweights;
  st->graph_nodes = X->graph_nodes;
  st->groups3 = X->nT;
  st->v_bg3 = X->V3;
  if (X->method == 2) st->v_bg_padded = X->Vgp;
  HIP_TRY(hipEventSynchronize(X->ev[4]));
  for (size_t i = 0; i + 1 < X->prof.size(); i += 2) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, X->prof[i], X->prof[i + 1]));
    st->ms_dominant += ms;
  }
  HIP_TRY(hipEventElapsedTime(&st->ms_partition, X->ev[0], X->ev[1]));
  HIP_TRY(hipEventElapsedTime(&st->ms_components, X->ev[1], X->ev[2]));
  HIP_TRY(hipEventElapsedTime(&st->ms_bg_assembly, X->ev[2], X->ev[3]));
  HIP_TRY(hipEventElapsedTime(&st->ms_bg_apsp, X->ev[3], X->ev[4]));
  return SPQ_OK;
}

spq_status spq_index_layout(const spq_index* X, int32_t* comp, int32_t* local, int32_t* nb,
                            int32_t* off, int32_t* bgoff) {
  if (!X) return fail(SPQ_EINVAL, "index is NULL");
  HIP_TRY(hipEventSynchronize(X->ev[4]));
  if (comp) HIP_TRY(hipMemcpy(comp, X->comp, sizeof(int32_t) * X->n, hipMemcpyDeviceToHost));
  if (local) HIP_TRY(hipMemcpy(local, X->local, sizeof(int32_t) * X->n, hipMemcpyDeviceToHost));
  if (nb) std::memcpy(nb, X->h_nb.data(), sizeof(int32_t) * X->k);
  if (off) std::memcpy(off, X->h_off.data(), sizeof(int32_t) * (X->k + 1));
  if (bgoff) std::memcpy(bgoff, X->h_bgoff.data(), sizeof(int32_t) * (X->k + 1));
  return SPQ_OK;
}

spq_status spq_index_component(const spq_index* X, int32_t c, int32_t* out) {
  if (!X || !out) return fail(SPQ_EINVAL, "null argument");
  if (c < 0 || c >= X->k) return fail(SPQ_EINVAL, "component id out of range");
  HIP_TRY(hipEventSynchronize(X->ev[4]));
  const int32_t N = X->h_cnt[c], P = X->h_P[c];
  HIP_TRY(hipMemcpy2D(out, sizeof(int32_t) * N, X->M + X->h_moff[c], sizeof(int32_t) * P,
                      sizeof(int32_t) * N, N, hipMemcpyDeviceToHost));
  return SPQ_OK;
}

spq_status spq_index_bg_rows(const spq_index* X, int32_t row0, int32_t nrows, int32_t* out) {
  if (!X || !out) return fail(SPQ_EINVAL, "null argument");
  if (row0 < 0 || nrows < 0 || (int64_t)row0 + nrows > X->V)
    return fail(SPQ_EINVAL, "BG rows out of range");
  if (nrows == 0) return SPQ_OK;
  HIP_TRY(hipEventSynchronize(X->ev[4]));
  // rows are gathered from the blocked store the queries read
  if (X->share_comps > 0 &&
      (int64_t)row0 + nrows > X->h_gbg0[X->share_groups - 1] + X->h_gV[X->share_groups - 1])
    return fail(SPQ_EINVAL, "BG rows outside the share");
  u32* tmp = nullptr;
  HIP_TRY(dalloc(&tmp, X->V));
  spq::HierArgs ha{};
  ha.share_groups = X->share_groups;
  ha.V = X->V; ha.ngroups = X->ngroups; ha.bggrp = X->bggrp; ha.bgrow = X->bgrow; ha.bgnb = X->bgnb;
  ha.bglocal = X->bglocal; ha.gV = X->gV; ha.pairbase = X->pairbase; ha.H = X->H;
  hipError_t e = hipSuccess;
  for (int32_t r = 0; r < nrows && e == hipSuccess; r++) {
    e = spq::launch_hier_row(ha, row0 + r, tmp, nullptr);
    if (e == hipSuccess)
      e = hipMemcpy(out + (int64_t)r * X->V, tmp, sizeof(int32_t) * X->V, hipMemcpyDeviceToHost);
  }
  pool_release(tmp);
  HIP_TRY(e);
  return SPQ_OK;
}

void spq_free_index(spq_index* X) { delete X; }

void spq_release_cached_memory(void) {
  {
    Pool& P = pool();
    std::lock_guard<std::mutex> lock(P.mu);
    pool_drop_idle(-1);
  }
  StreamPool& S = stream_pool();
  std::lock_guard<std::mutex> lock(S.mu);
  for (auto& it : S.idle) (void)hipStreamDestroy(it.second);
  S.idle.clear();
}

spq_status spq_fw_components(int32_t count, const int32_t* size, const int64_t* off,
                             const int32_t* ld, int32_t* data, void* stream) {
  if (count < 0 || (count > 0 && (!size || !off || !ld || !data)))
    return fail(SPQ_EINVAL, "bad arguments");
  if (count == 0) return SPQ_OK;
  for (int32_t i = 0; i < count; i++)
    if (size[i] < 1 || ld[i] < size[i] || ld[i] % spq::COMP_TILE || off[i] < 0 || off[i] % 4)
      return fail(SPQ_EINVAL, "matrix " + std::to_string(i) + ": bad size, ld or offset");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int32_t> order(count);
  std::iota(order.begin(), order.end(), 0);
  int32_t *d_order = nullptr, *d_P = nullptr;
  int64_t* d_off = nullptr;
  HIP_TRY(dalloc(&d_order, count));
  HIP_TRY(dalloc(&d_P, count));
  HIP_TRY(dalloc(&d_off, count));
  HIP_TRY(hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_P, ld, sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_off, off, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
  HIP_TRY(spq::launch_comp_fw(count, d_order, d_P, d_off, reinterpret_cast<u32*>(data), s));
  HIP_TRY(hipStreamSynchronize(s));
  pool_release(d_order);
  pool_release(d_P);
  pool_release(d_off);
  return SPQ_OK;
}

spq_status spq_fw_dense(int32_t v, int32_t ld, int32_t tile, int32_t pivot, int32_t kc,
                        int32_t* data, void* stream) {
  if (tile != 64 && tile != 128) return fail(SPQ_EINVAL, "tile must be 64 or 128");
  if (pivot != 0 && pivot != tile && pivot != 2 * tile && pivot != 4 * tile)
    return fail(SPQ_EINVAL, "pivot must be 0 or 1, 2 or 4 tiles");
  if (kc != 0 && kc != 16 && kc != 32) return fail(SPQ_EINVAL, "kc must be 0, 16 or 32");
  if (v < 0 || ld < v || ld % tile || (v > 0 && !data)) return fail(SPQ_EINVAL, "bad v or ld");
  if (v == 0) return SPQ_OK;
  HIP_TRY(spq::launch_dense_fw(reinterpret_cast<u32*>(data), ld, tile, ld / tile,
                               reinterpret_cast<hipStream_t>(stream), nullptr, kc, pivot));
  return SPQ_OK;
}

// Group-level composition products on caller buffers (see spq.h).
spq_status spq_minplus_batched(int32_t layout, int32_t groups, const int32_t* nv, const int32_t* nk,
                               int32_t vp, int32_t kp, const int32_t* R, const int32_t* D,
                               const int32_t* Dt, int64_t ldd, const int32_t* M, int32_t npairs,
                               const int32_t* pairs, int32_t assoc, int32_t cb, int32_t* out,
                               int64_t ldo, void* stream) {
  if (layout != SPQ_MP_BLOCKED && layout != SPQ_MP_DENSE) return fail(SPQ_EINVAL, "bad layout");
  if (assoc < 0 || assoc > 2 || (assoc && layout != SPQ_MP_BLOCKED))
    return fail(SPQ_EINVAL, "assoc must be 0, or 1 or 2 with SPQ_MP_BLOCKED");
  if (groups < 1 || groups > 4096) return fail(SPQ_EINVAL, "groups must be in [1, 4096]");
  if (vp < 128 || vp % 128 || kp < 128 || kp % 128)
    return fail(SPQ_EINVAL, "vp and kp must be positive multiples of 128");
  if (vp > 32768) return fail(SPQ_EINVAL, "vp above 32,768");
  if (!nv || !nk || !R || !M || !out || npairs < 0 || (npairs > 0 && !pairs))
    return fail(SPQ_EINVAL, "null argument or npairs < 0");
  std::vector<int32_t> koff(groups + 1, 0), voff(groups + 1, 0);
  for (int32_t g = 0; g < groups; g++) {
    if (nv[g] < 1 || nv[g] > vp || nk[g] < 0 || nk[g] > kp)
      return fail(SPQ_EINVAL, "group " + std::to_string(g) + ": nv outside [1, vp] or nk outside [0, kp]");
    koff[g + 1] = koff[g] + nk[g];
    voff[g + 1] = voff[g] + nv[g];
  }
  if (koff[groups] > 0 && (!D || ldd < koff[groups] || (assoc && !Dt)))
    return fail(SPQ_EINVAL, "D (or Dt) is NULL or ldd below the total boundary rows");
  if (layout == SPQ_MP_BLOCKED && cb < 1) return fail(SPQ_EINVAL, "cb < 1");
  if (layout == SPQ_MP_DENSE && ldo < voff[groups]) return fail(SPQ_EINVAL, "ldo below the total vertices");
  std::vector<int2> plist(npairs);
  std::vector<int64_t> pairbase((size_t)groups * groups, -1);
  int64_t obase = 0;
  for (int32_t p = 0; p < npairs; p++) {
    const int32_t s1 = pairs[2 * p], s2 = pairs[2 * p + 1];
    if (s1 < 0 || s1 >= groups || s2 < 0 || s2 >= groups)
      return fail(SPQ_EINVAL, "pair " + std::to_string(p) + ": group outside [0, groups)");
    if (pairbase[(size_t)s1 * groups + s2] >= 0)
      return fail(SPQ_EINVAL, "pair " + std::to_string(p) + " repeats an earlier pair");
    pairbase[(size_t)s1 * groups + s2] = obase;
    obase += (int64_t)nv[s1] * nv[s2];
    // through B2(S1) instead of B2(S2): the products' roles exchanged
    auto cost = [&](int32_t a, int32_t b) {
      return mp_rows(nk[b]) * mp_cols(nv[a]) * (double)round_up(nk[a], 16) +
             mp_rows(nv[a]) * mp_cols(nv[b]) * (double)round_up(nk[b], 16);
    };
    const bool sw = s1 != s2 && (assoc == 2 || (assoc == 1 && cost(s2, s1) < cost(s1, s2)));
    plist[p] = sw ? make_int2(s2, s1 | spq::PAIR_SWAP) : make_int2(s1, s2);
  }
  if (npairs == 0) return SPQ_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // pairs per launch: XT slots of kp x vp words within 256 MiB
  const int64_t slot = (int64_t)kp * vp;
  const int32_t chunk =
      (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)npairs, 65535, ((int64_t)1 << 26) / slot}));
  Scratch sc(s);
  int2* d_plist = nullptr;
  int32_t *d_nk = nullptr, *d_nv = nullptr, *d_koff = nullptr, *d_voff = nullptr;
  u32* d_xt = nullptr;
  HIP_TRY(sc.get(&d_plist, npairs));
  HIP_TRY(sc.get(&d_nk, groups));
  HIP_TRY(sc.get(&d_nv, groups));
  HIP_TRY(sc.get(&d_koff, groups + 1));
  HIP_TRY(sc.get(&d_voff, groups + 1));
  HIP_TRY(sc.get(&d_xt, (int64_t)chunk * slot));
  HIP_TRY(hipMemcpyAsync(d_plist, plist.data(), sizeof(int2) * npairs, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_nk, nk, sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_nv, nv, sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_koff, koff.data(), sizeof(int32_t) * (groups + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_voff, voff.data(), sizeof(int32_t) * (groups + 1), hipMemcpyHostToDevice, s));
  // a D with no rows is never read; the kernels still take a valid pointer
  const u32* dD = reinterpret_cast<const u32*>(koff[groups] > 0 ? D : R);
  const int64_t ld = koff[groups] > 0 ? ldd : 1;
  if (layout == SPQ_MP_DENSE) {
    spq::L3Args a{};
    a.V3gp = vp; a.m3pmax = kp; a.m3 = d_nk; a.tsize = d_nv; a.b3off = d_koff; a.tbase = d_voff;
    a.BG3 = const_cast<u32*>(dD); a.V3p = ld;
    a.R3 = const_cast<u32*>(reinterpret_cast<const u32*>(R));
    a.M3 = const_cast<u32*>(reinterpret_cast<const u32*>(M));
    a.XT3 = d_xt; a.BG2 = reinterpret_cast<u32*>(out); a.V2p = ldo;
    a.plist = d_plist; a.npairs = npairs; a.chunk = chunk;
    HIP_TRY(spq::launch_level3_compose(a, s));
  } else {
    // every group cut into consecutive components of cb vertices: per vertex
    // its component's first index, size and its own index inside it
    const int32_t V = voff[groups];
    std::vector<int32_t> row(V), cnb(V), loc(V);
    for (int32_t g = 0; g < groups; g++)
      for (int32_t x = 0; x < nv[g]; x++) {
        const int32_t r0 = x - x % cb;
        row[voff[g] + x] = r0;
        cnb[voff[g] + x] = std::min(cb, nv[g] - r0);
        loc[voff[g] + x] = x % cb;
      }
    int32_t *d_row = nullptr, *d_cnb = nullptr, *d_loc = nullptr;
    int64_t* d_pb = nullptr;
    HIP_TRY(sc.get(&d_row, V));
    HIP_TRY(sc.get(&d_cnb, V));
    HIP_TRY(sc.get(&d_loc, V));
    HIP_TRY(sc.get(&d_pb, (int64_t)groups * groups));
    HIP_TRY(hipMemcpyAsync(d_row, row.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_cnb, cnb.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_loc, loc.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_pb, pairbase.data(), sizeof(int64_t) * groups * groups,
                           hipMemcpyHostToDevice, s));
    spq::HierArgs a{};
    a.ngroups = groups; a.Vgp = vp; a.m2pmax = kp; a.m2 = d_nk; a.gV = d_nv; a.b2off = d_koff;
    a.gbg0 = d_voff; a.BG2 = const_cast<u32*>(dD); a.V2p = ld;
    a.R = const_cast<u32*>(reinterpret_cast<const u32*>(R));
    a.Mg = const_cast<u32*>(reinterpret_cast<const u32*>(M));
    a.XT = d_xt; a.H = reinterpret_cast<u32*>(out); a.pairbase = d_pb;
    a.bgrow = d_row; a.bgnb = d_cnb; a.bglocal = d_loc;
    a.D2t = koff[groups] > 0 && Dt ? reinterpret_cast<const u32*>(Dt) : dD; a.d2tld = ld;
    a.plist = d_plist; a.npairs = npairs; a.chunk = chunk;
    HIP_TRY(spq::launch_hier_level2_compose(a, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return SPQ_OK;
}

// The in-place product of the share's Bellman-Ford rounds on caller buffers
// (see spq.h).
spq_status spq_minplus_rows(int32_t groups, const int32_t* nk, int32_t kp, const int32_t* A,
                            int32_t* C, int64_t ldc, const int32_t* cnt, const int32_t* rows,
                            const int32_t* own, void* stream) {
  if (groups < 1 || groups > 65535) return fail(SPQ_EINVAL, "groups must be in [1, 65535]");
  if (kp < 128 || kp % 128) return fail(SPQ_EINVAL, "kp must be a positive multiple of 128");
  if (ldc < 128 || ldc % 128) return fail(SPQ_EINVAL, "ldc must be a positive multiple of 128");
  if (!nk || !A || !C || !cnt) return fail(SPQ_EINVAL, "null argument");
  std::vector<int32_t> koff(groups + 1, 0);
  int64_t listed = 0;
  for (int32_t g = 0; g < groups; g++) {
    if (nk[g] < 0 || nk[g] > kp) return fail(SPQ_EINVAL, "nk outside [0, kp]");
    if (cnt[g] > nk[g]) return fail(SPQ_EINVAL, "more listed rows than rows in a group");
    koff[g + 1] = koff[g] + nk[g];
    if (cnt[g] > 0) listed += cnt[g];
  }
  if (listed > 0 && !rows) return fail(SPQ_EINVAL, "rows is NULL");
  const int32_t ntc = (int32_t)(ldc / 128);
  std::vector<u32> dirty((size_t)groups * (ntc + 1), 1u);
  std::vector<int32_t> hc((size_t)groups * ntc);
  std::vector<int32_t> hl((size_t)groups * ntc * kp, 0);
  std::vector<int32_t> ho((size_t)groups * kp, 0);
  for (int32_t g = 0, at = 0; g < groups; g++) {
    for (int32_t r = 0; r < nk[g]; r++) {
      const int32_t c = own ? own[koff[g] + r] : koff[g] + r;
      if (c < 0) return fail(SPQ_EINVAL, "negative row in own");
      ho[(size_t)g * kp + r] = c;
    }
    const int32_t c = cnt[g] < 0 ? spq::BF_ALL_ROWS : cnt[g];
    for (int32_t t = 0; t < ntc; t++) {
      hc[(size_t)g * ntc + t] = c;
      for (int32_t i = 0; i < std::max(cnt[g], 0); i++) {
        const int32_t r = rows[at + i];
        if (r < 0 || r >= nk[g]) return fail(SPQ_EINVAL, "listed row outside its group");
        hl[((size_t)g * ntc + t) * kp + i] = r;
      }
    }
    at += std::max(cnt[g], 0);
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Scratch sc(s);
  int32_t *d_nk = nullptr, *d_zero = nullptr, *d_own = nullptr, *d_cnt = nullptr, *d_list = nullptr;
  u32* d_dirty = nullptr;
  const std::vector<int32_t> zero(groups, 0);
  HIP_TRY(sc.get(&d_nk, groups));
  HIP_TRY(sc.get(&d_zero, groups));
  HIP_TRY(sc.get(&d_own, (int64_t)groups * kp));
  HIP_TRY(sc.get(&d_cnt, (int64_t)groups * ntc));
  HIP_TRY(sc.get(&d_list, (int64_t)groups * ntc * kp));
  HIP_TRY(sc.get(&d_dirty, (int64_t)groups * (ntc + 1)));
  HIP_TRY(hipMemcpyAsync(d_nk, nk, sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_zero, zero.data(), sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_own, ho.data(), sizeof(int32_t) * ho.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_cnt, hc.data(), sizeof(int32_t) * hc.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_list, hl.data(), sizeof(int32_t) * hl.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_dirty, dirty.data(), sizeof(u32) * dirty.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(spq::launch_bf_rows(groups, kp, kp, ldc, d_nk, d_zero, d_own,
                              reinterpret_cast<const u32*>(A), reinterpret_cast<u32*>(C), d_dirty,
                              d_cnt, d_list, s));
  HIP_TRY(hipStreamSynchronize(s));
  return SPQ_OK;
}

spq_status spq_minplus_gather(int32_t groups, const int32_t* nk, const int32_t* nout, int32_t kp,
                              int32_t np, const int32_t* Aout, int32_t* C, int64_t ldc,
                              const int32_t* own, const int32_t* out, void* stream) {
  if (groups < 1 || groups > 65535) return fail(SPQ_EINVAL, "groups must be in [1, 65535]");
  if (kp < 128 || kp % 128 || np < 128 || np % 128)
    return fail(SPQ_EINVAL, "kp and np must be positive multiples of 128");
  if (ldc < 128 || ldc % 128) return fail(SPQ_EINVAL, "ldc must be a positive multiple of 128");
  if (!nk || !nout || !Aout || !C) return fail(SPQ_EINVAL, "null argument");
  const int32_t L = std::max(kp, np);
  std::vector<int32_t> ho((size_t)groups * L, 0), hq((size_t)groups * L, 0);
  int64_t ak = 0, ao = 0;
  for (int32_t g = 0; g < groups; g++) {
    if (nk[g] < 0 || nk[g] > kp || nout[g] < 0 || nout[g] > np)
      return fail(SPQ_EINVAL, "nk outside [0, kp] or nout outside [0, np]");
    if ((nk[g] > 0 && !own) || (nout[g] > 0 && !out)) return fail(SPQ_EINVAL, "null row list");
    for (int32_t k = 0; k < nk[g]; k++) {
      if (own[ak + k] < 0) return fail(SPQ_EINVAL, "negative row in own");
      ho[(size_t)g * L + k] = own[ak + k];
    }
    for (int32_t i = 0; i < nout[g]; i++) {
      if (out[ao + i] < 0) return fail(SPQ_EINVAL, "negative row in out");
      hq[(size_t)g * L + i] = out[ao + i];
    }
    ak += nk[g];
    ao += nout[g];
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Scratch sc(s);
  int32_t *d_nk = nullptr, *d_nout = nullptr, *d_zero = nullptr, *d_own = nullptr, *d_out = nullptr;
  const std::vector<int32_t> zero(groups, 0);
  HIP_TRY(sc.get(&d_nk, groups));
  HIP_TRY(sc.get(&d_nout, groups));
  HIP_TRY(sc.get(&d_zero, groups));
  HIP_TRY(sc.get(&d_own, (int64_t)groups * L));
  HIP_TRY(sc.get(&d_out, (int64_t)groups * L));
  HIP_TRY(hipMemcpyAsync(d_nk, nk, sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_nout, nout, sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_zero, zero.data(), sizeof(int32_t) * groups, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_own, ho.data(), sizeof(int32_t) * ho.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_out, hq.data(), sizeof(int32_t) * hq.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(spq::launch_bf_gather(groups, L, kp, np, ldc, d_nk, d_nout, d_zero, d_own, d_out,
                                reinterpret_cast<const u32*>(Aout), reinterpret_cast<u32*>(C), s));
  HIP_TRY(hipStreamSynchronize(s));
  return SPQ_OK;
}

// Measured VALU issue rates (see spq.h).
spq_status spq_valu_rates(double* out, void* stream) {
  if (!out) return fail(SPQ_EINVAL, "out is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 8 * std::max(cus, 1);
  u32* buf = nullptr;
  HIP_TRY(dalloc(&buf, (int64_t)blocks * 256));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int iters[4] = {4000, 4000, 1000, 1000};
  for (int kind = 0; kind < 4 && e == hipSuccess; kind++) {
    e = spq::launch_valu_probe(kind, blocks, iters[kind] / 4, buf, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = spq::launch_valu_probe(kind, blocks, iters[kind], buf, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const double lanes = (double)blocks * 256.0;
    const double work = kind < 2 ? lanes * iters[kind] * 32.0 : lanes * 64.0 * 16.0 * iters[kind];
    if (e == hipSuccess) out[kind] = ms > 0 ? work / (ms * 1e-3) : 0.0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  pool_release(buf);
  HIP_TRY(e);
  return SPQ_OK;
}

}  // extern "C"
