"""How the index and its queries change with the number of components k.

The paper reports (its Figs. 3 and 4, for a cluster) that Phase 2 dominates
preprocessing at small k and Phase 3 (BG) at large k, and that memory per node
falls as k grows.  This study builds the index of one graph for several k on
one GPU and records, per k: |B(C)|, V_BG, the bytes of APSP(C) and of the BG
store, the device time of Phase 2 and of the BG closure, and the time of a
batch of queries (first batch after the build, then the same batch again).

The graph is grid256d's (256 x 256 grid with random cell diagonals, weights
U[1,1000]); the partitions are square blocks of side 64, 32, 16, 8 and 4
(k = 16 .. 4,096).  Every index is checked to give the same answers as the
first one on the query batch.

    python -m paper_1503_07192_amd.study > study.json
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def run(blocks=(64, 32, 16, 8, 4), queries=100_000, log=print, answers=False):
    """One row per block side; with answers=True each row also holds the
    query batch (v1, v2) and that index's answers (numpy)."""
    import torch
    from . import spq, workloads as W
    g = W.grid256d(queries=queries)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    eu, ev, w = dev(g["eu"]), dev(g["ev"]), dev(g["w"])
    v1, v2 = dev(g["v1"]), dev(g["v2"])
    rows, ref = [], None
    for b in blocks:
        part_np, k = W.block_partition(256, 256, b, b)
        part = dev(part_np)
        # one build to warm the allocator, then the measured one
        spq.build_index(g["n"], eu, ev, w, part, k).free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx = spq.build_index(g["n"], eu, ev, w, part, k)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        st = spq.index_stats(idx)
        out = torch.empty_like(v1)
        ts = []
        for _ in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            spq.query_batch(idx, v1, v2, out)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ans = out.cpu().numpy()
        if ref is None:
            ref = ans
        row = {"block": b, "k": k, "component_vertices": b * b, "v_bg": st["v_bg"],
               "mean_boundary": st["v_bg"] / k, "bg_method": "flat" if st["bg_method"] == 1 else "two-level",
               "groups": st["ngroups"], "comp_bytes": st["comp_bytes"], "bg_bytes": st["bg_bytes"],
               "build_ms": build_ms, "ms_components": st["ms_components"],
               "ms_bg": st["ms_bg_apsp"], "relax_executed": st["relax_comp_exec"] + st["relax_bg_exec"],
               "query_ms_first": ts[0], "query_ms_again": float(np.median(ts[1:])),
               "queries": len(g["v1"]), "answers_identical": bool(np.array_equal(ans, ref))}
        log(json.dumps(row))
        if answers:
            row["v1"], row["v2"], row["answers"] = g["v1"], g["v2"], ans
        rows.append(row)
        idx.free()
    return rows


def main(argv=None):
    import torch
    p = argparse.ArgumentParser()
    p.add_argument("--queries", type=int, default=100_000)
    args = p.parse_args(argv)
    torch.cuda.set_device(0)
    run(queries=args.queries, log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
