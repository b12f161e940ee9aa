"""Benchmark: one step = the whole hot path on one batch of synthetic input.

A step builds the index (boundary + renumbering, APSP of every component,
BG assembly, distances in BG) and answers one batch of query pairs.  The
default workload is the largest one that fits one GPU: the 2048x2048 grid
with 10% of its edges deleted (4.19M vertices, 16,384 components of 16x16),
built as one GPU's share (all APSP(C), BG rows of components [0, 512)),
then 10M query pairs with v1 in the share.  Inputs are resident in HBM
before timing.

Prints ONE JSON line.  `value` is min-plus relaxations executed per second
over the whole step (queries included in the time); `index_build_ms` is the
build alone and `query_batch_ms_p50/p99` the batch, both from HIP events.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 2.4 GHz.  A relaxation c = min(c, a+b) is one v_add_u32
# and half a v_min3_u32 (two candidates folded per min3): 1.5 VALU
# instructions.  The published fp32 vector peak, 157.3 TFLOP/s, is 128
# lanes per CU per clock (an FMA counts two flops); at that rate for every
# 32-bit instruction a relaxation costs 1.5 / 128 CU-clocks: 5.24e13
# relaxations/s, the peak the roofline fraction is taken against.  At 64
# lanes per CU per clock for v_min3_u32 and 128 for v_add_u32 (what
# spq_valu_rates measures on the box: the add above 64 lanes per clock, the
# min3 below it) the bound would be 3.93e13: reported beside it as the lower
# end of the band.
LANE_CYCLES_PER_S = 256 * 64 * 2.4e9
RELAX_PEAK = 256 * 2.4e9 * 128 / 1.5
RELAX_PEAK_LOW = LANE_CYCLES_PER_S * 1.0
HBM_PEAK = 8.0e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="grid2048", choices=sorted(WORKLOADS))
    p.add_argument("--queries", type=int, default=None)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-probe", action="store_true",
                   help="run one 256 MiB device copy first (calibrates HBM byte counters)")
    p.add_argument("--no-serve", action="store_true",
                   help="skip the continuous-batching serving run after the timed region")
    return p.parse_args()


WORKLOADS = {
    "grid256d": dict(
        queries=100_000,
        desc="grid256d: 256x256 grid + random cell diagonals, weights U[1,1000], 1,024 blocks "
             "of 8x8, %d uniform query pairs"),
    "delaunay1m": dict(
        queries=100_000,
        desc="delaunay1m: Delaunay triangulation of 1M uniform points, weight rint(length*1e6), "
             "4,096 recursive-bisection parts, two-level BG, %d uniform query pairs"),
    "grid2048": dict(
        queries=10_000_000,
        desc="grid2048: 2048x2048 grid minus 10%% of edges (connected), lognormal weights, 16,384 "
             "blocks of 16x16; one GPU's share = BG rows of components [0,512); %d pairs with v1 "
             "in the share"),
}


def recorded_traffic(name, work):
    """HBM bytes per launch of a kernel, from the committed counter summary
    profiles/pmc_<name>.md, if the sources it names still hash to the ones it
    was measured on and a launch does the same work (relaxations or queries)
    as in that run."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_%s.md" % name)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        k, _, v = line.partition(":")
        if k in ("traffic_bytes_per_launch", "work_per_launch", "sources", "source_sha256"):
            rec[k] = v.strip()
    if len(rec) < 4:
        return None
    csrc = os.path.join(ROOT, "paper_1503_07192_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in rec["sources"].split())
    if rec["source_sha256"] != hashlib.sha256(src).hexdigest():
        return None
    if abs(float(rec["work_per_launch"]) - work) > 1e-9 * max(1.0, work):
        return None
    return float(rec["traffic_bytes_per_launch"])


TUNE_CACHE = os.path.join(ROOT, "paper_1503_07192_amd", "tune_cache.json")


def make_workload(name, queries):
    """The graph and its build options.  grid256d closes BG by flat
    Floyd-Warshall (the workload's definition; the two-level method is timed
    beside it); the others take the autotuner's choice for this device."""
    from paper_1503_07192_amd import workloads as W
    if name == "grid256d":
        return W.grid256d(queries=queries), {}
    if name == "delaunay1m":
        return W.delaunay1m(queries=queries), {"tune_cache": TUNE_CACHE}
    g = W.grid2048(queries=queries)
    return g, {"share_comps": g["share_k"], "tune_cache": TUNE_CACHE}


def cpu_baseline(g, st, budget_s):
    """The oracle as it stands (built -O3 -march=native on this host), timed on
    a bounded sample of the same workload: component Floyd-Warshalls on all
    threads and on one, Dijkstra in BG from sampled sources where BG is small
    enough for the oracle, and one Dijkstra on G per query."""
    import oracle
    oracle.configure(native=True)
    threads = max(1, min(16, os.cpu_count() or 1))
    n, k = g["n"], g["k"]
    rng = np.random.default_rng(0)
    order = rng.permutation(k)

    def fw_sample(count, nthreads):
        comps = np.sort(order[:count])
        t0 = time.perf_counter()
        members, apsp = oracle.component_apsp(n, g["eu"], g["ev"], g["w"], g["part"], k,
                                              comps=comps, nthreads=nthreads)
        return comps, members, apsp, time.perf_counter() - t0

    def budgeted(nthreads, seconds):
        # a first sample fixes the rate; later ones grow until the sample
        # fills most of the budget (or covers every component)
        c = min(k, 64 * nthreads)
        comps, members, apsp, t = fw_sample(c, nthreads)
        while t < 0.7 * seconds and c < k:
            c = int(min(k, max(c + 1, c * seconds / max(t, 1e-3))))
            comps, members, apsp, t = fw_sample(c, nthreads)
        return comps, members, apsp, t

    comps, members, apsp, t_comp = budgeted(threads, budget_s * 0.3)
    relax_sample = float(sum(len(m) ** 3 for m in members))
    res = {"value": relax_sample / t_comp, "unit": "relax/s", "cores": threads, "kind": "oracle",
           "build": "gcc -O3 -march=native",
           "sample": "Floyd-Warshall of %d of %d components (%.3g relaxations, %.2f s, %d threads)"
                     % (len(comps), k, relax_sample, t_comp, threads)}
    comps1, members1, _, t1 = budgeted(1, budget_s * 0.15)
    res["value_1thread"] = float(sum(len(m) ** 3 for m in members1)) / t1
    res["sample"] += "; one thread: %d components in %.2f s" % (len(comps1), t1)
    res["component_phase_s"] = float(st["relax_comp"]) / res["value"]
    if k <= 1024 and len(comps) == k:
        # the paper's Phase 3: Dijkstra in BG from a budgeted number of sources
        bg_ids, bverts, bu, bv, bw = oracle.boundary_graph(n, g["eu"], g["ev"], g["w"], g["part"],
                                                           k, members, apsp)
        V = len(bg_ids)
        t0 = time.perf_counter()
        oracle.bg_apsp(bg_ids, bu, bv, bw, sources=np.arange(min(64, V)), nthreads=threads)
        per_src = (time.perf_counter() - t0) / min(64, V)
        nsrc = int(min(V, max(64, budget_s * 0.3 / max(per_src, 1e-6))))
        t0 = time.perf_counter()
        oracle.bg_apsp(bg_ids, bu, bv, bw, sources=np.arange(nsrc), nthreads=threads)
        t_bg = (time.perf_counter() - t0) * V / nsrc
        res["index_build_s"] = t_comp + t_bg
        res["sample"] += ("; Dijkstra in BG from %d of %d sources, scaled: whole index in %.1f s"
                          % (nsrc, V, t_comp + t_bg))
    # the paper's comparison for queries: one Dijkstra per query on G
    nq = threads
    t0 = time.perf_counter()
    oracle.dijkstra(n, g["eu"], g["ev"], g["w"], g["v1"][:nq], nthreads=threads)
    t = time.perf_counter() - t0
    if t < budget_s * 0.25:
        nq = int(min(len(g["v1"]), max(nq + 1, nq * budget_s * 0.25 / max(t, 1e-3))))
        t0 = time.perf_counter()
        oracle.dijkstra(n, g["eu"], g["ev"], g["w"], g["v1"][:nq], nthreads=threads)
        t = time.perf_counter() - t0
    res["queries_per_s"] = nq / t
    res["query_sample"] = "Dijkstra on G from %d query sources, %d threads, %.2f s" % (
        nq, threads, t)
    return res


T_START = time.perf_counter()


def progress(msg):
    """One line per finished phase on stderr (stdout holds only the result)."""
    print("bench: %s (%.1f s)" % (msg, time.perf_counter() - T_START), file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the index of one GPU's share is built and "
              "queried locally; multi-GPU sharding is not part of this build.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1503_07192_amd import spq, workloads as W

    torch.cuda.set_device(0)
    wl = WORKLOADS[args.workload]
    nq = args.queries or wl["queries"]
    g, build_kw = make_workload(args.workload, nq)
    progress("workload %s generated" % args.workload)
    tuned = None
    if build_kw.get("tune_cache"):
        from paper_1503_07192_amd import autotune
        tuned = autotune.lookup(build_kw["tune_cache"], g["n"], g["m"], g["k"],
                                build_kw.get("share_comps", 0))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    eu, ev, w, part = dev(g["eu"]), dev(g["ev"]), dev(g["w"]), dev(g["part"])
    v1, v2 = dev(g["v1"]), dev(g["v2"])
    out = torch.empty_like(v1)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()

    def step(record):
        eb, e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        eb.record(stream)
        idx = spq.build_index(g["n"], eu, ev, w, part, g["k"], profile=True, stream=stream,
                              **build_kw)
        e0.record(stream)
        spq.query_batch(idx, v1, v2, out, stream=stream)
        e1.record(stream)
        st = spq.index_stats(idx)
        e1.synchronize()
        if record is not None:
            st["ms_build"] = eb.elapsed_time(e0)
            st["ms_query"] = e0.elapsed_time(e1)
            record.append(st)
        idx.free()

    for i in range(args.warmup):
        step(None)
        progress("warm-up step %d done" % (i + 1))
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress("%d timed steps done" % args.steps)

    st = recs[-1]
    relax = st["relax_comp_exec"] + st["relax_bg_exec"]
    ms_step = elapsed * 1e3 / args.steps
    q = len(g["v1"])
    mq = np.array([r["ms_query"] for r in recs])
    mb = np.array([r["ms_build"] for r in recs])
    # dominant kernel: the BG interior-tile launches, timed with HIP events on
    # the build stream inside the timed steps
    inner_ms = np.array([r["ms_dominant"] for r in recs])
    launches = st["dominant_launches"]
    avg_launch_ms = float(np.median(inner_ms)) / launches
    per_launch = st["relax_dominant"] / launches
    inner_rate = per_launch / (avg_launch_ms * 1e-3)
    kernel = ("k_fw_inner (BG interior tiles, 128x128, K chunk 16)" if st["bg_method"] == 1 else
              "k_mp_y (two-level composition product, 128x128 tiles, K chunk 16)")

    # the other BG method on the same workload, after the timed region: same
    # answers (checked on the whole query batch), different work
    alt = None
    if args.workload == "grid256d":
        ref = out.clone()
        for method in (2,):   # with the autotuner's options for this workload
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            idx = spq.build_index(g["n"], eu, ev, w, part, g["k"], bg_method=method,
                                  tune_cache=TUNE_CACHE, stream=stream)
            spq.query_batch(idx, v1, v2, out, stream=stream)
            torch.cuda.synchronize()
            t_alt = time.perf_counter() - t1
            ast = spq.index_stats(idx)
            alt = {"bg_method": "two-level", "groups": ast["ngroups"], "v_bg2": ast["v_bg2"],
                   "step_ms": t_alt * 1e3, "ms_bg": ast["ms_bg_apsp"],
                   "relax_executed": ast["relax_comp_exec"] + ast["relax_bg_exec"],
                   "answers_identical": bool(torch.equal(ref, out))}
            idx.free()

    # the build captured as HIP graphs, then replays of those graphs with other
    # weights and back (spq_reweight_index); the last replay restores the
    # workload's weights, so its answers must equal the timed steps'
    graph = None
    if not st["share_comps"]:
        ref = out.clone()
        w2 = torch.remainder(w, 997) + 1
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        idx = spq.build_index(g["n"], eu, ev, w, part, g["k"], graph=True, stream=stream,
                              **build_kw)
        torch.cuda.synchronize()
        t_cap = time.perf_counter() - t1
        reps = []
        for wr in (w2, w, w2, w):
            t1 = time.perf_counter()
            spq.reweight(idx, wr, stream=stream)
            torch.cuda.synchronize()
            reps.append((time.perf_counter() - t1) * 1e3)
        spq.query_batch(idx, v1, v2, out, stream=stream)
        torch.cuda.synchronize()
        gst = spq.index_stats(idx)
        graph = {"build_ms": t_cap * 1e3, "reweight_ms_p50": float(np.median(reps)),
                 "reweight_ms": reps, "graphs": gst["graphs"], "graph_nodes": gst["graph_nodes"],
                 "answers_identical": bool(torch.equal(ref, out))}
        idx.free()

    # the plain comparators, after the timed region: one launch per component
    # for APSP(C), and one query per launch
    idx = spq.build_index(g["n"], eu, ev, w, part, g["k"], plain=True, paths=True, stream=stream,
                          **build_kw)
    plain_st = spq.index_stats(idx)
    progress("comparison builds done")
    lay = spq.index_layout(idx)
    layout_tables = (lay["comp"], lay["nb"])
    # shortest paths (vertex sequences) for the first 1,000 pairs
    npath = min(1000, q)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _, plens = spq.query_paths(idx, v1[:npath], v2[:npath], 16384, stream=stream)
    e1.record(stream)
    e1.synchronize()
    plens = plens.cpu().numpy()
    paths_res = {"pairs": npath, "ms": e0.elapsed_time(e1),
                 "paths_per_s": npath / (e0.elapsed_time(e1) * 1e-3),
                 "mean_vertices": float(plens[plens > 0].mean()) if (plens > 0).any() else 0.0,
                 "found": int((plens > 0).sum()), "unreachable": int((plens == 0).sum())}
    # the same batch again on this (warm) index: caches and TLB hold its tables
    warm = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        spq.query_batch(idx, v1, v2, out, stream=stream)
        e1.record(stream)
        e1.synchronize()
        warm.append(e0.elapsed_time(e1))
    lat = []
    for i in range(200):
        a, b = v1[i:i + 1], v2[i:i + 1]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        spq.query_batch(idx, a, b, out[i:i + 1], stream=stream)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1) * 1e3)
    idx.free()
    lat = np.array(lat)

    # continuous batching on a resident index of the same workload, after the
    # timed region: open-loop Poisson arrivals of 1 .. 65,536 pairs, slots and
    # memory-gated admission (the library's server); every checked request must give the
    # same answers alone as in the mix
    served = None
    if not args.no_serve:
        from paper_1503_07192_amd import serve as SV
        idx = spq.build_index(g["n"], eu, ev, w, part, g["k"], stream=stream, **build_kw)
        torch.cuda.synchronize()
        srcs = (np.flatnonzero(g["part"] < st["share_comps"]).astype(np.int32)
                if st["share_comps"] else None)
        rng = np.random.default_rng(W.SEED_BASE + 5)
        mem = 64 << 20
        served = {"server": "spq_server (native worker thread)", "slots": 4,
                  "slot_pairs": 65536, "mem_mib": 64, "rates": {}}
        for rate, nreq in ((1e6, 300), (1e7, 1000)):
            reqs = SV.poisson_stream(rng, rate, nreq, g["n"], sources=srcs)
            server = spq.Server(idx, 4, 65536, mem)
            done = SV.run_native(server, reqs)
            res = SV.summarize(done, server_stats=server.stats())
            server.close()
            same = sum(int(np.array_equal(spq.query_batch(idx, dev(r.v1), dev(r.v2)).cpu().numpy(),
                                          r.result)) for r in reqs[:100])
            res["alone_equals_mix"] = "%d/%d" % (same, min(100, len(reqs)))
            served["rates"]["%g" % rate] = res
        idx.free()

    # bytes the query kernel must move per pair: both row prefixes, the BG
    # block, the ids and the result (12), the two 48-byte vertex records read
    # as the 16 bytes a pair uses, and d_C1(v1, v2) when C1 = C2
    comp_of, nb_of = layout_tables
    c1, c2 = comp_of[g["v1"]], comp_of[g["v2"]]
    nb1, nb2 = nb_of[c1].astype(np.float64), nb_of[c2].astype(np.float64)
    qbytes_total = float(np.sum(4 * (nb1 + nb1 * nb2 + nb2) + 12 + 16 + 4 * (c1 == c2)))
    qbytes = qbytes_total / q

    line = {
        "metric": "min-plus relaxations/s (index build); queries/s + p50/p99 query latency",
        "value": relax * args.steps / elapsed,
        "unit": "relax/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": wl["desc"] % q, "name": args.workload,
                   "n": g["n"], "m": g["m"], "k": g["k"], "v_bg": st["v_bg"], "queries": q,
                   "bg_method": "flat" if st["bg_method"] == 1 else "two-level",
                   "groups": st["ngroups"], "v_bg2": st["v_bg2"],
                   "groups3": st["groups3"], "v_bg3": st["v_bg3"], "bf_rounds": st["bf_rounds"],
                   "share_comps": st["share_comps"], "bg_bytes": st["bg_bytes"],
                   "tuned_options": tuned},
        "phase_ms": {key: float(np.median([r[key] for r in recs]))
                     for key in ("ms_partition", "ms_components", "ms_bg_assembly",
                                 "ms_bg_apsp", "ms_query")},
        "relax_per_step": relax,
        "index_build_ms": float(np.median(mb)),
        "index_build_ms_p99": float(np.percentile(mb, 99)),
        "index_build_relax_per_s": relax / (np.median(mb) * 1e-3),
        "queries_per_s": q / (np.median(mq) * 1e-3),
        "queries_per_s_warm": q / (np.median(warm) * 1e-3),
        "query_batch_ms_p50": float(np.percentile(mq, 50)),
        "query_batch_ms_p99": float(np.percentile(mq, 99)),
        "other_bg_method": alt,
        "paths": paths_res,
        "graph_build": graph,
        "plain_components_ms": plain_st["ms_components"],
        "batched_components_ms": float(np.median([r["ms_components"] for r in recs])),
        "served": served,
        "single_query_us_p50": float(np.percentile(lat, 50)),
        "single_query_us_p99": float(np.percentile(lat, 99)),
        # the batched forms against the plain GPU path (one launch per
        # component; one pair per query launch, back to back)
        "speedup_vs_plain": {
            "components": plain_st["ms_components"] /
                          max(1e-9, float(np.median([r["ms_components"] for r in recs]))),
            "queries": (q / (np.median(mq) * 1e-3)) / (1e6 / float(np.percentile(lat, 50)))},
        # context only: the paper's cluster (300 nodes, 2x Xeon E5-2670 + 2x
        # Tesla M2090 each) answered one query at a time in 0.25-2 ms on an
        # unspecified 256k-vertex planar graph, 500-4,000 queries/s
        "paper_context_queries_per_s": [500, 4000],
        "roofline": {"bound": "alu", "kernel": kernel,
                     "achieved": inner_rate / 1e12, "peak": RELAX_PEAK / 1e12,
                     "unit": "Trelax/s", "frac": inner_rate / RELAX_PEAK,
                     "peak_band": {"low": RELAX_PEAK_LOW / 1e12, "high": RELAX_PEAK / 1e12,
                                   "frac_high_to_low": [inner_rate / RELAX_PEAK,
                                                        inner_rate / RELAX_PEAK_LOW]},
                     "traffic": recorded_traffic(("k_fw_inner_" if st["bg_method"] == 1 else "k_mp_y_")
                                                 + args.workload, per_launch),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a 256 MiB copy)",
                     "launches_per_step": launches, "avg_launch_ms": avg_launch_ms,
                     "relax_per_launch": per_launch},
        "query_roofline": {"bound": "hbm", "achieved": qbytes_total / (np.median(mq) * 1e-3) / 1e9,
                           "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                           "frac": qbytes_total / (np.median(mq) * 1e-3) / HBM_PEAK,
                           "frac_warm": qbytes_total / (np.median(warm) * 1e-3) / HBM_PEAK,
                           "bytes_per_query": qbytes,
                           "traffic": recorded_traffic("k_query_" + args.workload, float(q)),
                           "traffic_unit": "HBM bytes per launch of the step's batch (rocprofv3 "
                                           "FETCH_SIZE + WRITE_SIZE, scaled by a 256 MiB copy)"},
    }
    # instruction issue rates behind the peak, measured after the timed region
    progress("query latencies and serving done")
    vr = spq.valu_rates(stream)
    line["valu_rates"] = {
        "v_add_u32_lane_ops_per_s": vr["v_add_u32"], "v_min3_u32_lane_ops_per_s": vr["v_min3_u32"],
        "per_nominal_lane_cycle": {"v_add_u32": vr["v_add_u32"] / LANE_CYCLES_PER_S,
                                   "v_min3_u32": vr["v_min3_u32"] / LANE_CYCLES_PER_S},
        "relax_loop_per_s": vr["relax_loop"], "relax_loop_frac": vr["relax_loop"] / RELAX_PEAK,
        "relax_regs_per_s": vr["relax_regs"], "relax_regs_frac": vr["relax_regs"] / RELAX_PEAK}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, st, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
