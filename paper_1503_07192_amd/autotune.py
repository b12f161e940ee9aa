"""Autotuner for the index build.

The build options that change speed but never results are timed on the
workload itself and the fastest set is stored in a JSON cache keyed by the
device architecture and a size class of the problem:

* flat Floyd-Warshall on BG: tile side (64, 128) x interior K chunk (16, 32);
* two-level BG: consecutive components per group (8 .. 256) x K chunk, and
  on large BG (above 65,536 vertices) super-groups of 8 or 32 groups for the
  level-3 closure of BG2 at 16 and 32 components per group;
* share builds: consecutive components per group (8 .. 64) x groups per
  block of the Bellman-Ford over BG2 (1, 2, 4, 8), K chunk 16.
  Groups formed by size (``group_bg``) are not tried: on partitions numbered
  by recursive bisection or along a Z-order curve they cut across the aligned runs of
  2^j components that make a group compact, and measured 1.5-10x slower.

Every candidate must give bit-identical answers on a query sample (checked),
so picking one is purely a speed decision.  ``build_index(..., tune_cache=)``
reads the cache.

    python -m paper_1503_07192_amd.autotune --workload grid256d --cache tune.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np


def device_key() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def size_key(n: int, m: int, k: int, share_comps: int) -> str:
    return "n%d_m%d_k%d_%s" % (round(math.log2(max(n, 1))), round(math.log2(max(m, 1))),
                               round(math.log2(max(k, 1))), "share" if share_comps else "full")


def lookup(path: str, n: int, m: int, k: int, share_comps: int = 0) -> dict:
    """Tuned options for this device and size class ({} if none)."""
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return dict(data.get(device_key(), {}).get(size_key(n, m, k, share_comps), {}).get("best", {}))


def candidates(v_bg: int, k: int, share_comps: int):
    out = []
    if v_bg <= 32768 and not share_comps:
        for tile in (128, 64):
            for kc in (16, 32):
                for pt in (2, 4):
                    out.append({"bg_method": 1, "bg_tile": tile, "inner_kc": kc, "bg_pivot": pt * tile})
    cpg = 8
    if share_comps:
        while cpg <= min(64, k):
            for blk in (1, 2, 4, 8):
                out.append({"bg_method": 2, "group_comps": cpg, "level3_groups": blk,
                            "inner_kc": 16})
            cpg *= 2
        return out
    while cpg <= min(256, k):
        for kc in (16, 32):
            out.append({"bg_method": 2, "group_comps": cpg, "inner_kc": kc})
        if v_bg > 65536 and cpg in (16, 32):
            # BG2 closed by super-groups of fewer or more groups than the
            # automatic choice (about 4,096 BG2 vertices each)
            for l3 in (8, 32):
                out.append({"bg_method": 2, "group_comps": cpg, "inner_kc": 16,
                            "level3_groups": l3})
        cpg *= 2
    return out


def tune(g: dict, path: str | None = None, share_comps: int = 0, sample: int = 20000,
         max_bg_bytes: float = 200e9, log=print):
    import torch
    from . import spq
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()
    eu, ev, w, part = dev(g["eu"]), dev(g["ev"]), dev(g["w"]), dev(g["part"])
    rng = np.random.default_rng(7)
    if share_comps:
        sv = np.flatnonzero(g["part"] < share_comps)
        v1 = sv[rng.integers(0, len(sv), sample)].astype(np.int32)
    else:
        v1 = rng.integers(0, g["n"], sample).astype(np.int32)
    v2 = rng.integers(0, g["n"], sample).astype(np.int32)
    q1, q2 = dev(v1), dev(v2)
    probe = spq.build_index(g["n"], eu, ev, w, part, g["k"], share_comps=share_comps,
                            bg_method=2 if share_comps else 0)
    v_bg = spq.index_stats(probe)["v_bg"]
    probe.free()
    results, ref = [], None
    for opt in candidates(v_bg, g["k"], share_comps):
        if opt["bg_method"] == 1 and 4.0 * v_bg * v_bg > max_bg_bytes:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            idx = spq.build_index(g["n"], eu, ev, w, part, g["k"], share_comps=share_comps, **opt)
            torch.cuda.synchronize()
        except spq.SpqError as e:
            log("  %s: %s" % (opt, e))
            continue
        ms = (time.perf_counter() - t0) * 1e3
        ans = spq.query_batch(idx, q1, q2).cpu().numpy()
        idx.free()
        if ref is None:
            ref = ans
        elif not np.array_equal(ans, ref):
            raise RuntimeError("candidate %s changed the answers" % opt)
        results.append({"opts": opt, "build_ms": ms})
        log("  %-60s %9.1f ms" % (json.dumps(opt), ms))
    best = min(results, key=lambda r: r["build_ms"])
    entry = {"best": best["opts"], "build_ms": best["build_ms"], "v_bg": v_bg, "tried": results}
    if path:
        data = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
        data.setdefault(device_key(), {})[size_key(g["n"], g["m"], g["k"], share_comps)] = entry
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return entry


def main(argv=None):
    import torch
    from . import workloads as W
    p = argparse.ArgumentParser()
    p.add_argument("--workload", default="grid256d", choices=["grid32", "grid256d", "delaunay1m",
                                                               "grid2048"])
    p.add_argument("--cache", default="tune_cache.json")
    args = p.parse_args(argv)
    torch.cuda.set_device(0)
    share = 0
    if args.workload == "grid32":
        g = W.grid32()
    elif args.workload == "grid256d":
        g = W.grid256d(queries=0)
    elif args.workload == "delaunay1m":
        g = W.delaunay1m()
    else:
        g = W.grid2048(queries=0)
        share = g["share_k"]
    print("autotune %s on %s" % (args.workload, device_key()), flush=True)
    e = tune(g, args.cache, share_comps=share, log=lambda s: print(s, flush=True))
    print(json.dumps({"workload": args.workload, "best": e["best"], "build_ms": e["build_ms"]}),
          flush=True)


if __name__ == "__main__":
    main()
