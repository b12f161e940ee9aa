"""Continuous-batching query serving on a resident index.

Requests (batches of query pairs) arrive over time.  The server is the
library's own (``spq.Server``, spq_server_* in the C ABI): a native worker
thread keeps a FIFO admission queue and a fixed set of slots, each slot one
HIP stream.  Every launch's device buffers (pairs in, distances out) and their
pinned staging are carved out of one device pool and one pinned pool of the
memory budget's size by a first-fit allocator: a launch is admitted only when
its buffers can be allocated there (memory-based admission), and they return
to the pools when it completes.  Whenever a slot is free, the requests at the
head of the queue are coalesced into one launch of ``spq_query_batch`` on that
slot, as many as fit in the slot's pair capacity and in the largest free
region.  Several slots are in flight at once, so requests that arrive while
others run are admitted as soon as a slot and memory free up, and their work
overlaps on the device.  A request's latency is its completion time minus
its arrival time.

``Scheduler`` and ``Arena`` below are the same admission policy in Python,
driven by an executor interface (``submit / done / result``): the tests run
them on the CPU against a fake executor, where the policy's decisions can be
checked step by step.  ``run_native`` replays an arrival stream against the
library's server.

The paper answers queries one at a time and lists parallel queries as future
work (Section 5, Conclusion); ``OneAtATime`` is that mode, kept as the
comparator.
"""
from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field

import numpy as np

BYTES_PER_PAIR = 12  # v1, v2, out as int32


@dataclass
class Request:
    rid: int
    arrival: float          # seconds since the stream start
    v1: np.ndarray
    v2: np.ndarray
    result: np.ndarray | None = None
    done_at: float | None = None
    launches: list = field(default_factory=list)

    @property
    def size(self):
        return len(self.v1)


def poisson_stream(rng, rate_pairs: float, nreq: int, n: int, max_log2: float = 16.0,
                   lo: int = 0, hi: int | None = None, sources=None):
    """Open-loop arrivals: batch sizes floor(2**U(0, max_log2)) (1 .. 65,536),
    uniform random pairs, exponential gaps at rate_pairs / E[batch] requests/s.
    v1 is uniform in [lo, hi), or over the array `sources` when given (a
    share's vertices); v2 uniform in [0, n)."""
    hi = n if hi is None else hi
    sizes = np.floor(2.0 ** rng.uniform(0.0, max_log2, nreq)).astype(np.int64)
    mean_b = (2.0 ** max_log2 - 1.0) / (max_log2 * np.log(2.0))  # E[2^U]
    gaps = rng.exponential(mean_b / rate_pairs, nreq)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(nreq):
        b = int(sizes[i])
        if sources is None:
            v1 = rng.integers(lo, hi, b).astype(np.int32)
        else:
            v1 = np.asarray(sources)[rng.integers(0, len(sources), b)].astype(np.int32)
        v2 = rng.integers(0, n, b).astype(np.int32)
        reqs.append(Request(i, float(t[i]), v1, v2))
    return reqs


class Arena:
    """First-fit allocator of byte ranges in [0, size), in ALIGN-byte units:
    the admission gate of the server (a launch runs only once its buffers
    are allocated here) over the executor's device and pinned pools."""

    ALIGN = 256

    def __init__(self, size: int):
        self.size = size - size % self.ALIGN
        self.holes = [(0, self.size)] if self.size > 0 else []   # (offset, length), sorted
        self.live = {}   # offset -> length
        self.used = 0

    def largest(self) -> int:
        return max((h[1] for h in self.holes), default=0)

    def alloc(self, nbytes: int):
        """Offset of a free range of at least nbytes, or None."""
        n = -(-max(nbytes, 1) // self.ALIGN) * self.ALIGN
        for i, (off, ln) in enumerate(self.holes):
            if ln >= n:
                if ln == n:
                    del self.holes[i]
                else:
                    self.holes[i] = (off + n, ln - n)
                self.live[off] = n
                self.used += n
                return off
        return None

    def free(self, off: int):
        n = self.live.pop(off)
        self.used -= n
        holes = self.holes
        i = 0
        while i < len(holes) and holes[i][0] < off:
            i += 1
        holes.insert(i, (off, n))
        # merge with the following and the preceding hole
        if i + 1 < len(holes) and holes[i][0] + holes[i][1] == holes[i + 1][0]:
            holes[i] = (holes[i][0], holes[i][1] + holes[i + 1][1])
            del holes[i + 1]
        if i > 0 and holes[i - 1][0] + holes[i - 1][1] == holes[i][0]:
            holes[i - 1] = (holes[i - 1][0], holes[i - 1][1] + holes[i][1])
            del holes[i]


class Scheduler:
    """Admission, coalescing and completion on top of an executor.  The
    executor's ``arena`` (its memory pools; a fresh Arena of mem_budget bytes
    if it has none) decides admission."""

    def __init__(self, executor, slots: int, slot_pairs: int, mem_budget: int):
        if slots < 1 or slot_pairs < 1 or mem_budget < Arena.ALIGN:
            raise ValueError("need at least one slot and memory for one pair")
        self.ex = executor
        self.nslots = slots
        self.slot_pairs = slot_pairs
        self.arena = getattr(executor, "arena", None) or Arena(mem_budget)
        if self.arena.size > mem_budget:
            raise ValueError("the executor's pool is larger than the memory budget")
        self.mem_budget = mem_budget
        self.free = list(range(slots))
        self.inflight = {}  # slot -> (handle, [(req, lo, hi)], bytes)
        self.queue = collections.deque()
        self.launches = 0
        self.launch_sizes = []

    def enqueue(self, req: Request):
        """Queues a request; one larger than a slot or than the memory budget
        is served in pieces, in order."""
        req.result = np.empty(req.size, np.int32)
        req._issued = 0   # pairs handed to launches
        req._filled = 0   # pairs whose results came back
        if req.size == 0:
            req.done_at = req.arrival
            return
        self.queue.append(req)

    def _admit_one(self):
        """Coalesces queue-head requests into one launch on a free slot.  A
        request is cut only when the room left in the launch (slot capacity,
        memory budget) cannot hold it whole."""
        if not self.free or not self.queue:
            return False
        room = min(self.slot_pairs, self.arena.largest() // BYTES_PER_PAIR)
        if room <= 0:
            return False
        parts, take = [], 0
        while self.queue and take < room:
            req = self.queue[0]
            left = req.size - req._issued
            if take > 0 and left > room - take:
                break
            cnt = min(left, room - take)
            parts.append((req, req._issued, req._issued + cnt))
            req._issued += cnt
            take += cnt
            if req._issued == req.size:
                self.queue.popleft()
            else:
                break
        slot = self.free.pop()
        v1 = np.concatenate([r.v1[l:h] for r, l, h in parts])
        v2 = np.concatenate([r.v2[l:h] for r, l, h in parts])
        off = self.arena.alloc(take * BYTES_PER_PAIR)   # fits: take <= largest hole / 12
        handle = self.ex.submit(slot, v1, v2, off)
        self.inflight[slot] = (handle, parts, off)
        self.launches += 1
        self.launch_sizes.append(take)
        for r, l, h in parts:
            r.launches.append(self.launches)
        return True

    def admit(self):
        n = 0
        while self._admit_one():
            n += 1
        return n

    def complete(self, now_fn):
        """Collects finished slots; returns the requests completed."""
        finished = []
        for slot in list(self.inflight):
            handle, parts, off = self.inflight[slot]
            if not self.ex.done(handle):
                continue
            out = self.ex.result(handle)
            t = now_fn()
            pos = 0
            for r, l, h in parts:
                r.result[l:h] = out[pos:pos + (h - l)]
                pos += h - l
                r._filled += h - l
                if r._filled == r.size:
                    r.done_at = t
                    finished.append(r)
            del self.inflight[slot]
            self.arena.free(off)
            self.free.append(slot)
        return finished

    @property
    def mem_used(self):
        return self.arena.used

    def busy(self):
        return bool(self.inflight) or bool(self.queue)


def run_stream(sched: Scheduler, reqs, clock=None, spin=True):
    """Replays the arrival times in real time (or on the given clock).  The
    cyclic garbage collector is paused while requests are in flight (a full
    collection in the middle of the loop delays every request behind it) and
    run once afterwards."""
    clock = clock or time.perf_counter
    t0 = clock()
    now = lambda: clock() - t0
    i, done = 0, []
    was_enabled = gc.isenabled()
    gc.disable()
    try:
        while i < len(reqs) or sched.busy():
            t = now()
            while i < len(reqs) and reqs[i].arrival <= t:
                sched.enqueue(reqs[i])
                i += 1
            done += sched.complete(now)
            sched.admit()
            if not spin and i < len(reqs) and not sched.busy():
                time.sleep(max(0.0, reqs[i].arrival - now()))
    finally:
        if was_enabled:
            gc.enable()
        gc.collect()
    return done


def summarize(reqs, sched=None, server_stats=None):
    lat = np.array([r.done_at - r.arrival for r in reqs])
    pairs = sum(r.size for r in reqs)
    span = max(r.done_at for r in reqs) - min(r.arrival for r in reqs)
    # the offered load this sample of sizes and gaps actually carried
    arr = max(r.arrival for r in reqs) - min(r.arrival for r in reqs)
    out = {"requests": len(reqs), "pairs": int(pairs), "span_s": span,
           "queries_per_s": pairs / span if span > 0 else float("inf"),
           "offered_realized_pairs_per_s": pairs / arr if arr > 0 else float("inf"),
           "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
           "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
           "latency_ms_mean": float(lat.mean() * 1e3)}
    if sched is not None:
        out["launches"] = sched.launches
        out["pairs_per_launch"] = float(np.mean(sched.launch_sizes)) if sched.launch_sizes else 0.0
    if server_stats is not None:
        out["launches"] = server_stats["launches"]
        out["pairs_per_launch"] = server_stats["pairs"] / max(1, server_stats["launches"])
    return out


# ------------------------------------------------------------- native server
def run_native(server, reqs, clock=time.perf_counter):
    """Replays the arrival times in real time against ``server`` (an
    ``spq.Server``): each request is submitted at its arrival time, then every
    one is collected.  done_at = submission time + the server's own latency
    (completion minus submission), so a submission that lags its arrival
    time counts against the request.  The cyclic garbage collector is paused
    meanwhile."""
    t0 = clock()
    sent = []
    was_enabled = gc.isenabled()
    gc.disable()
    try:
        for r in reqs:
            while clock() - t0 < r.arrival:
                pass
            at = clock() - t0
            sent.append((r, server.submit(r.v1, r.v2), at))
        for r, ticket, at in sent:
            r.result, lat = server.poll(ticket, wait=True)
            r.done_at = at + lat
    finally:
        if was_enabled:
            gc.enable()
        gc.collect()
    return reqs


class OneAtATime:
    """The paper's mode: every pair is its own launch, one after another."""

    def __init__(self, index):
        import torch
        from . import spq
        self.torch, self.spq, self.index = torch, spq, index
        self.h = torch.empty(3, dtype=torch.int32, pin_memory=True)
        self.d = torch.empty(3, dtype=torch.int32, device="cuda")

    def run(self, reqs, clock=time.perf_counter):
        torch = self.torch
        s = torch.cuda.current_stream()
        t0 = clock()
        for r in reqs:
            while clock() - t0 < r.arrival:
                pass
            r.result = np.empty(r.size, np.int32)
            for i in range(r.size):
                self.h[0], self.h[1] = int(r.v1[i]), int(r.v2[i])
                self.d.copy_(self.h, non_blocking=True)
                self.spq.query_batch(self.index, self.d[0:1], self.d[1:2], self.d[2:3], stream=s)
                self.h.copy_(self.d, non_blocking=True)
                s.synchronize()
                r.result[i] = int(self.h[2])
            r.done_at = clock() - t0
        return reqs


# ------------------------------------------------------------------ main
def main(argv=None):
    """Serving measurement on the Delaunay index (1M points, 4,096 parts)."""
    import argparse
    import json
    import torch
    from . import spq, workloads as W

    p = argparse.ArgumentParser()
    p.add_argument("--rates", default="1e5,1e6,1e7")
    p.add_argument("--requests", type=int, default=2000)
    p.add_argument("--low-rate-requests", type=int, default=300,
                   help="requests at rates below 1e6 pairs/s (their arrivals are slow)")
    p.add_argument("--slots", type=int, default=4)
    p.add_argument("--slot-pairs", type=int, default=65536)
    p.add_argument("--mem-mib", type=float, default=64.0)
    p.add_argument("--one-at-a-time-requests", type=int, default=20)
    p.add_argument("--workload", default="delaunay1m", choices=["delaunay1m", "grid256d"])
    args = p.parse_args(argv)
    torch.cuda.set_device(0)
    g = W.delaunay1m() if args.workload == "delaunay1m" else W.grid256d(queries=0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    import os
    cache = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
    idx = spq.build_index(g["n"], dev(g["eu"]), dev(g["ev"]), dev(g["w"]), dev(g["part"]), g["k"],
                          tune_cache=cache)
    torch.cuda.synchronize()
    st = spq.index_stats(idx)
    print("index built: n=%d V_BG=%d method=%d groups=%d bg_bytes=%.1f GB" % (
        g["n"], st["v_bg"], st["bg_method"], st["ngroups"], st["bg_bytes"] / 1e9), flush=True)
    rng = np.random.default_rng(W.SEED_BASE + 5)
    report = {"workload": args.workload, "n": g["n"], "k": g["k"], "v_bg": st["v_bg"],
              "slots": args.slots, "slot_pairs": args.slot_pairs, "mem_mib": args.mem_mib,
              "rates": {}}
    mem = int(args.mem_mib * 2**20)
    for rate in [float(x) for x in args.rates.split(",")]:
        nreq = args.requests if rate >= 1e6 else args.low_rate_requests
        reqs = poisson_stream(rng, rate, nreq, g["n"])
        server = spq.Server(idx, args.slots, args.slot_pairs, mem)
        done = run_native(server, reqs)
        res = summarize(done, server_stats=server.stats())
        server.close()
        # each request alone must give the same answers as inside the mix
        same = 0
        for r in reqs:
            alone = spq.query_batch(idx, dev(r.v1), dev(r.v2)).cpu().numpy()
            same += int(np.array_equal(alone, r.result))
        res["alone_equals_mix"] = "%d/%d" % (same, len(reqs))
        res["offered_pairs_per_s"] = rate
        report["rates"]["%g" % rate] = res
        print(json.dumps({"rate": rate, **res}), flush=True)
    one = poisson_stream(rng, 1e5, args.one_at_a_time_requests, g["n"], max_log2=10.0)
    OneAtATime(idx).run(one)
    report["one_at_a_time"] = summarize(one)
    report["one_at_a_time"]["batch_sizes"] = "floor(2^U(0,10)) at 1e5 pairs/s offered"
    print(json.dumps({"one_at_a_time": report["one_at_a_time"]}), flush=True)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
