#!/usr/bin/env python3
"""Throughput of the Interval Tree Matching hot path on one MI355X.

A step is one whole pass of the hot path over the workload's inputs, which
are resident in device memory before timing starts: build the per-dimension
interval trees over the subscriptions (sort + tree + maxupper), match every
update (BITS counts, update order, count traversal, scan, fill traversal,
segment sort) into a preallocated output, and release the trees.  As in the
paper's measurements, preprocessing (the tree build) is inside the timed
step.

Prints ONE JSON line: pairs/s (value), regions/s, the roofline of the
dominant kernel (its launch durations measured with HIP events on the
stream it is launched on, during the timed steps) and the CPU oracle's rate
on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM3E peak of one MI355X (bytes/s) and its vector ALU issue rate: 256 CUs x
# 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per second.
HBM_PEAK_GBS = 8000.0
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--traversal", default="auto", choices=["auto", "lane", "tile"])
    ap.add_argument("--workload", default="d2_uniform", choices=["d2_uniform", "d2_hotspot"])
    ap.add_argument("--path", default="both", choices=["plain", "learned", "both"],
                    help="plain two-pass, learned single-pass, or both (value = faster)")
    ap.add_argument("--predictor", default="",
                    help="saved predictor (.npz); default: train one before timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="updates in the oracle's timed sample (0 = auto)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: every node here exposes a single MI355X and "
              "the matcher has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    t0 = time.time()
    if args.workload == "d2_uniform":
        inst = W.uniform_2d_1m(1)
        wname, seed = "d2_N1e6_alpha1_uniform", 1
    else:
        inst = W.hotspot_2d(2)
        wname, seed = "d2_N1e6_hotspots_alpha100", 2
    log(f"workload {wname} generated in {time.time() - t0:.2f}s: d={inst.d} n={inst.n} "
        f"m={inst.m}")
    dev = lambda a: torch.from_numpy(a).cuda()
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)

    pred, train_rep = None, None
    if args.path in ("learned", "both"):
        if args.predictor:
            pred = P.Predictor.load(args.predictor)
        else:
            from paper_1309_3458_amd import learn
            pred, train_rep = learn.train_predictor(n_inst=32, per_instance=16000, epochs=20)
            log(f"predictor trained: {train_rep}")

    # size the output once (untimed), then reuse it
    t = P.build(s_lo, s_hi)
    K0 = int(P.match(t, u_lo, u_hi, traversal=args.traversal).numel())
    t.free()
    out = torch.empty(K0 + 1, dtype=torch.int64, device="cuda")
    log(f"K = {K0}")

    def step_plain():
        t = P.build(s_lo, s_hi)
        keys = P.match(t, u_lo, u_hi, traversal=args.traversal, out=out)
        t.free()
        return keys.numel()

    info = {}

    def step_learned():
        t = P.build(s_lo, s_hi)
        keys = P.match_learned(t, u_lo, u_hi, pred, traversal=args.traversal, out=out, info=info)
        t.free()
        return keys.numel()

    def timed(step, name):
        for i in range(args.warmup):
            K = step()
        torch.cuda.synchronize()
        # which traversal kernel dominates: one step with every launch evented
        P.prof_enable(True)
        step()
        torch.cuda.synchronize()
        prof = P.prof_read()
        P.prof_enable(False)
        dom = max((k for k in prof if k.startswith("traverse")), key=lambda k: prof[k][0])
        log(f"[{name}] per-kernel ms (one step): "
            + json.dumps({k: round(v[0], 4) for k, v in sorted(prof.items())}))
        # timed region: HIP events only around the dominant kernel's launches
        P.prof_enable(True, only=dom)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            K = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dprof = P.prof_read()
        P.prof_enable(False)
        assert K == K0
        dms, dn = dprof[dom]
        return {"ms_per_step": (t1 - t0) * 1e3 / args.steps, "dominant": dom,
                "dominant_avg_ms": dms / dn, "per_kernel_ms": prof}

    res = {}
    if args.path in ("plain", "both"):
        res["plain"] = timed(step_plain, "plain")
    if args.path in ("learned", "both"):
        res["learned"] = timed(step_learned, "learned")
        res["learned"]["overflowed"] = info.get("overflowed")
        res["learned"]["slots"] = info.get("slots")
    best = min(res, key=lambda k: res[k]["ms_per_step"])
    ms_step = res[best]["ms_per_step"]
    pairs_s = K0 / (ms_step / 1e3)
    regions_s = (inst.n + inst.m) / (ms_step / 1e3)
    dom, dom_avg_ms = res[best]["dominant"], res[best]["dominant_avg_ms"]

    # Dominant kernel: one traversal pass.  Its unit of work is the per-
    # dimension candidate test of Algorithm 3 (an update against a
    # subscription that meets it in the probe dimension), 2*d float compares
    # each.  Candidates per pass = sum_j min_k c_{j,k} (exact BITS counts,
    # recomputed here on the host).
    ks = [np.sort(inst.s_lo[k]) for k in range(inst.d)]
    he = [np.sort(inst.s_hi[k]) for k in range(inst.d)]
    c = np.stack([np.searchsorted(ks[k], inst.u_hi[k], side="right")
                  - np.searchsorted(he[k], inst.u_lo[k], side="left") for k in range(inst.d)])
    cand = float(c.min(axis=0).sum())
    ops = cand * 2 * inst.d
    achieved = ops / (dom_avg_ms / 1e3) / 1e9
    roofline = {"bound": "alu", "achieved": round(achieved, 1), "peak": ALU_PEAK_GOPS,
                "unit": "Gop/s", "frac": round(achieved / ALU_PEAK_GOPS, 4), "traffic": None,
                "kernel": dom, "kernel_avg_ms": round(dom_avg_ms, 4),
                "candidates_per_launch": int(cand)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = min(os.cpu_count() or 1, 16)
        sample = args.cpu_sample or (inst.m if args.workload == "d2_uniform" else 2000)
        t0 = time.perf_counter()
        ok = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo[:, :sample], inst.u_hi[:, :sample],
                        threads=cores)
        dt = time.perf_counter() - t0
        cpu = {"value": round(len(ok) / dt, 1), "unit": "pairs/s", "cores": cores,
               "kind": "oracle",
               "sample": f"all {inst.n} subscriptions x first {sample} updates, tree build "
                         f"included, {dt:.2f}s, {len(ok)} pairs"}

    paths = {k: {"ms_per_step": round(v["ms_per_step"], 4),
                 "pairs_per_s": round(K0 / (v["ms_per_step"] / 1e3), 1),
                 **({"overflowed": v.get("overflowed"), "slots": v.get("slots")}
                    if k == "learned" else {})}
             for k, v in res.items()}
    if "plain" in res and "learned" in res:
        paths["learned_speedup_vs_plain"] = round(
            res["plain"]["ms_per_step"] / res["learned"]["ms_per_step"], 4)
    rec = {
        "metric": "matched pairs/sec + regions/sec at d=2 N=1M alpha=1; p99 latency (serving)",
        "value": round(pairs_s, 1),
        "unit": "pairs/s",
        "regions_per_s": round(regions_s, 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "d": inst.d, "n": inst.n, "m": inst.m,
                   "seed": seed, "K": int(K0), "traversal": args.traversal, "path": best},
        "paths": paths,
        "predictor": ({"val_under_rate": train_rep["val_under_rate"],
                       "val_mae_log1p": round(train_rep["val_mae_log1p"], 4),
                       "delta": round(train_rep["delta"], 4), "train_s": train_rep["train_s"]}
                      if train_rep else None),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
