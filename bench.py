#!/usr/bin/env python3
"""Throughput of the Interval Tree Matching hot path on one MI355X.

A step is one whole pass of the hot path over the workload's inputs, which
are resident in device memory before timing starts: build the per-dimension
interval trees over the subscriptions (sort + tree + maxupper), match every
update (BITS counts, update order, count traversal, scan, fill traversal,
segment sort) into a preallocated output, and release the trees.  As in the
paper's measurements, preprocessing (the tree build) is inside the timed
step; the match alone on a resident tree is reported beside it.

Workloads:
  d2_uniform (default)  d=2, 500,000 subscriptions + 500,000 updates, square
                        side 1000 on [0, 1e6)^2 (alpha = 1), seed 1
  d3_uniform            d=3, 500,000 + 500,000 cubes, side 1e6*(1/1e6)^(1/3)
                        (alpha = 1), seed 1
  d2_hotspot            d=2, 500,000 + 500,000 boxes around 16 Gaussian
                        hotspots, log-normal sides (median 1e4), seed 2
  batch256              256 independent instances (N log-uniform in
                        [1e3, 2e5], d in {1,2,3}, alpha log-uniform in
                        [0.01, 100], seed 3), one graph replay per step
  sweep_1d              the paper's experiment on the GPU: d=1, N from 5e4
                        to 5e5, alpha in {0.01, 1, 100}; ITM (build +
                        match) beside GPU Brute-Force and Sort-Based
                        Matching
  sweep_fig7            the time surface of the paper's Fig. 7 on the GPU: ITM
                        build + match for d=1, N from 5e4 to 5e5 and alpha
                        over 0 < alpha <= 100 (0.01 .. 100, half-decade steps)
  dynamic               dynamic DDM on the d=2, 10^6-box workload: moves of 1% of
                        the updates or of the subscriptions (resident trees
                        and result, only the moved extents' pairs recomputed)
                        against a full build + match of the moved sets
  hbm_copy              a plain device-to-device copy of 1 GiB per step
                        (calibrates the HBM traffic counters)
  serve                 open-loop Poisson arrivals (2000/s, d=3, N
                        log-uniform in [1e3, 1e6], alpha log-uniform in
                        [0.01, 100], seed 4) into the serving loop with
                        learned sizing; p50/p99 latency arrival -> host

Prints ONE JSON line: pairs/s (value), regions/s, per-step statistics, the
roofline of the dominant kernel (its launch durations measured with HIP
events on the stream it is launched on) and the CPU oracle's rate on the
host.  The default workload's line also carries the learned single pass
against the plain two-pass path on the hotspot workload
(hotspot_learned_vs_plain: times, speedup, identical bytes).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM3E peak of one MI355X (bytes/s) and its vector ALU issue rate: 256 CUs x
# 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per second.
HBM_PEAK_GBS = 8000.0
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
METRIC = "matched pairs/sec + regions/sec at d=2 N=1M alpha=1; p99 latency (serving)"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--traversal", default="auto", choices=["auto", "lane", "tile"])
    ap.add_argument("--workload", default="d2_uniform",
                    choices=["d2_uniform", "d2_hotspot", "d3_uniform", "batch256", "serve", "hbm_copy",
                             "sweep_1d", "sweep_fig7", "dynamic"])
    ap.add_argument("--duration", type=float, default=60.0,
                    help="serve: seconds of Poisson arrivals (the schedule is cut, not rescaled)")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: arrivals per second")
    ap.add_argument("--workers", type=int, default=8, help="serve: concurrent requests")
    ap.add_argument("--batch-max", type=int, default=0,
                    help="serve: small requests matched together (0 = library default, 1 = off)")
    ap.add_argument("--batch-small", type=int, default=0,
                    help="serve: largest n + m of a request that may be batched (0 = default)")
    ap.add_argument("--deliver-device", action="store_true",
                    help="serve: results stay in device memory (no PCIe copy)")
    ap.add_argument("--compact", action="store_true",
                    help="serve: host results as subscription ids + update offsets")
    ap.add_argument("--n-hi", type=float, default=1e6,
                    help="serve: largest request size N (the schedule's log-uniform range "
                         "is [1e3, n_hi])")
    ap.add_argument("--path", default="both", choices=["plain", "learned", "both"],
                    help="plain two-pass, learned single-pass, or both (value = faster)")
    ap.add_argument("--predictor", default="",
                    help="saved predictor file (Predictor.save); default: train one before timing")
    ap.add_argument("--tuning", default="",
                    help="batch256: tuning table (JSON); default: the packaged table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hotspot", action="store_true",
                    help="d2_uniform: skip the learned-vs-plain comparison on the hotspot "
                         "workload")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="updates in the oracle's timed sample (0 = auto)")
    return ap.parse_args()


def step_stats(ms):
    return {"mean": round(statistics.fmean(ms), 4), "median": round(statistics.median(ms), 4),
            "min": round(min(ms), 4)}


def candidates(inst):
    """Per-dimension candidate tests of one traversal pass: sum over updates
    of the smallest exact per-dimension count (closed BITS identity)."""
    import numpy as np
    c = None
    for k in range(inst.d):
        lo, hi = np.sort(inst.s_lo[k]), np.sort(inst.s_hi[k])
        ck = np.searchsorted(lo, inst.u_hi[k], side="right") \
            - np.searchsorted(hi, inst.u_lo[k], side="left")
        c = ck if c is None else np.minimum(c, ck)
    return float(c.sum())


# HBM traffic counters (rocprofv3 FETCH_SIZE, WRITE_SIZE; KiB per dispatch)
# of the default workload's plain path, calibrated by a 1 GiB device copy
# (FETCH x 2.000, WRITE x 1.000: the copy's FETCH_SIZE reads half its bytes).
# They hold only for the kernel sources they were taken on: `sha` is the
# SHA-256 (first 16 hex digits) of the files in TRAFFIC_SOURCES, and a build
# from other sources reports the traffic as null (the hash is moved to new
# sources only when every kernel the step launches compiles to the same
# code object, which the profile records).  `kernel` is the dominant
# kernel's own launch; `step` sums every kernel of one build + match step.
TRAFFIC_SOURCES = ("paper_1309_3458_amd/csrc/match.hip", "paper_1309_3458_amd/csrc/traverse.h",
                   "paper_1309_3458_amd/csrc/ddm_internal.h", "paper_1309_3458_amd/csrc/tree.hip",
                   "paper_1309_3458_amd/csrc/tree_dev.h", "paper_1309_3458_amd/csrc/sort_scan.hip")
TRAFFIC = {
    ("d2_N1e6_alpha1_uniform", "plain", "traverse_tile_count_stash"): {
        "sha": "909628ee2e08fdfe", "kernel_fetch_kib": 118650.9, "kernel_write_kib": 31364.4,
        "step_fetch_kib": 238170.7, "step_write_kib": 189257.5, "step_kernel_us": 328.3,
        "profile": "profiles/traffic_d2_N1e6_alpha1_pmc.md"},
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def sources_sha():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_entry(wname, path, kernel):
    t = TRAFFIC.get((wname, path, kernel))
    if not t or t["sha"] is None or t["sha"] != sources_sha():
        return None
    return t


def compulsory_bytes_count_pass(inst, K):
    """Bytes one count pass of Algorithm 4 must move at least, whatever its
    design: every subscription record of the probe tree read once (2d floats
    + a 4-byte id), every update's 2d bounds read, a 4-byte count written per
    update and each of the K hits kept (a 12-byte entry: key and rank)."""
    d = inst.d
    return (8 * d + 4) * inst.n + 8 * d * inst.m + 4 * inst.m + 12 * K


def roofline_record(inst, K, cand, dom, dom_avg_ms, wname, path):
    """The roofline object of the dominant kernel (the count traversal).

    bound "hbm": the pass does no dense arithmetic, so its roofline is HBM
    bandwidth; `achieved` = the compulsory bytes of the pass per launch over
    the launch's duration.  Beside it: the measured FETCH+WRITE traffic per
    launch and as a fraction of peak, the same fraction over a whole step,
    and the compare rate of the candidate tests against the vector ALU issue
    rate (secondary: the pass is bound by the latency of its dependent
    block-scan chain, not by either unit)."""
    sec = dom_avg_ms / 1e3
    algo = compulsory_bytes_count_pass(inst, K)
    achieved = algo / sec / 1e9
    t = traffic_entry(wname, path, dom)
    traffic = None
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
         "kernel": dom, "kernel_avg_ms": round(dom_avg_ms, 4),
         "algorithmic_bytes_per_launch": int(algo)}
    if t:
        traffic = (t["kernel_fetch_kib"] * FETCH_SCALE + t["kernel_write_kib"] * WRITE_SCALE) * 1024
        r["traffic"] = round(traffic, 1)
        r["measured_gbs"] = round(traffic / sec / 1e9, 1)
        r["measured_frac_hbm_peak"] = round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)
        st = (t["step_fetch_kib"] * FETCH_SCALE + t["step_write_kib"] * WRITE_SCALE) * 1024
        r["step_traffic"] = round(st, 1)
        r["step_kernel_us"] = t["step_kernel_us"]
        r["step_measured_frac_hbm_peak"] = round(
            st / (t["step_kernel_us"] / 1e6) / 1e9 / HBM_PEAK_GBS, 4)
        r["counters"] = t["profile"]
    else:
        r["traffic_note"] = "counters not taken on these kernel sources"
    r["target_measured_frac"] = 0.40
    ops = cand * 2 * inst.d
    alu = ops / sec / 1e9
    r["alu"] = {"achieved": round(alu, 1), "peak": ALU_PEAK_GOPS, "unit": "Gop/s",
                "frac": round(alu / ALU_PEAK_GOPS, 4), "candidates_per_launch": int(cand),
                "what": "2d float compares per probe-dimension candidate"}
    return r


def roofline_alu(cand, ops, dom, dom_avg_ms, traffic=None):
    # Unit of work of a traversal pass: the per-dimension candidate test of
    # Algorithm 4 (an update against a subscription that meets it in the probe
    # dimension), 2*d float compares each.
    achieved = ops / (dom_avg_ms / 1e3) / 1e9
    r = {"bound": "alu", "achieved": round(achieved, 1), "peak": ALU_PEAK_GOPS,
         "unit": "Gop/s", "frac": round(achieved / ALU_PEAK_GOPS, 4), "traffic": traffic,
         "kernel": dom, "kernel_avg_ms": round(dom_avg_ms, 4),
         "candidates_per_launch": int(cand)}
    if traffic:
        r["traffic_gbs"] = round(traffic / (dom_avg_ms / 1e3) / 1e9, 1)
        r["traffic_frac_hbm_peak"] = round(r["traffic_gbs"] / HBM_PEAK_GBS, 4)
    return r


def cpu_info():
    """Host cores the oracle may use and what they are.  On the GPU hosts
    one GPU's share of the CPU is 16 cores (OMP_NUM_THREADS is set to it);
    nproc and the CPU model are recorded beside it."""
    share = os.environ.get("OMP_NUM_THREADS")
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    cores = int(share) if share and share.isdigit() and int(share) > 0 else aff
    cores = max(1, min(cores, aff))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, {"nproc": os.cpu_count(), "affinity_cores": aff,
                   "omp_num_threads": share, "cpu_model": model}


def evented_steps(step, steps):
    """Run `steps` steps with a HIP event between consecutive steps on the
    current stream; returns (wall ms per step, per-step ms list, last K)."""
    import gc
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    # no collector pause of the host inside the timed region
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        K = None
        for i in range(steps):
            K = step()
            ev[i + 1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        gc.enable()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return (t1 - t0) * 1e3 / steps, per, K


def oracle_rate(inst, cores, sample, what):
    import oracle
    t0 = time.perf_counter()
    ok = oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo[:, :sample], inst.u_hi[:, :sample],
                    threads=cores)
    dt = time.perf_counter() - t0
    return {"value": round(len(ok) / dt, 1), "unit": "pairs/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{what}: all {inst.n} subscriptions x first {sample} updates, tree "
                      f"build included, {dt:.2f}s, {len(ok)} pairs"}


def hotspot_paths(pred, steps, warmup):
    """The learned single pass against the plain two-pass path on the hotspot
    workload (d=2, 500,000 + 500,000 boxes around 16 Gaussian hotspots,
    log-normal sides with median 1e4, seed 2), in build + match steps:
    per-path time, speedup, overflowed updates, and that the two outputs are
    identical element by element."""
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import workloads as W

    inst = W.hotspot_2d(2)
    dev = lambda a: torch.from_numpy(a).cuda()
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
    t = P.build(s_lo, s_hi)
    out = P.match(t, u_lo, u_hi)
    K = out.numel()
    other = torch.empty_like(out)
    info = {}
    P.match_learned(t, u_lo, u_hi, pred, out=other, info=info)
    same = bool(torch.equal(out, other))
    t.free()
    del other

    def step(path):
        tt = P.build(s_lo, s_hi)
        if path == "plain":
            k = P.match(tt, u_lo, u_hi, out=out).numel()
        else:
            k = P.match_learned(tt, u_lo, u_hi, pred, out=out).numel()
        tt.free()
        return k

    res = {}
    for path in ("plain", "learned"):
        for _ in range(warmup):
            step(path)
        wall, per, k = evented_steps(lambda: step(path), steps)
        assert k == K
        res[path] = {"ms_per_step": round(wall, 3), "step_ms": step_stats(per),
                     "pairs_per_s": round(K / (wall / 1e3), 1)}
    del out
    torch.cuda.synchronize()
    return {"workload": "d2_N1e6_hotspots_alpha100", "seed": 2, "K": int(K), **res,
            "learned_speedup_vs_plain": round(res["plain"]["ms_per_step"] /
                                              res["learned"]["ms_per_step"], 4),
            "identical_bytes": same, "overflowed": info.get("overflowed"),
            "slots": info.get("slots")}


def bench_single(args):
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import workloads as W

    t0 = time.time()
    if args.workload == "d2_uniform":
        inst = W.uniform_2d_1m(1)
        wname, seed = "d2_N1e6_alpha1_uniform", 1
    elif args.workload == "d3_uniform":
        inst = W.uniform_instance(1, 500_000, 500_000, 3, W.side_for_alpha(1.0, 1_000_000, 3))
        wname, seed = "d3_N1e6_alpha1_uniform", 1
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
    out = torch.empty(K0 + 1, dtype=torch.int64, device="cuda")
    log(f"K = {K0}")

    # the match alone on a resident tree (untimed region)
    for _ in range(args.warmup):
        P.match(t, u_lo, u_hi, traversal=args.traversal, out=out)
    _, per_match, _ = evented_steps(
        lambda: P.match(t, u_lo, u_hi, traversal=args.traversal, out=out).numel(), args.steps)
    t.free()

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
            step()
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
        wall, per, K = evented_steps(step, args.steps)
        dprof = P.prof_read()
        P.prof_enable(False)
        assert K == K0
        dms, dn = dprof[dom]
        return {"ms_per_step": wall, "step_ms": step_stats(per), "dominant": dom,
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
    cand = candidates(inst)
    roofline = roofline_record(inst, K0, cand, res[best]["dominant"],
                               res[best]["dominant_avg_ms"], wname, best)

    cpu = None
    if not args.no_cpu_baseline:
        cores, host = cpu_info()
        sample = args.cpu_sample or (inst.m if args.workload == "d2_uniform" else 2000)
        cpu = oracle_rate(inst, cores, sample, wname)
        # the plain sequential oracle on a tenth of the sample
        one = oracle_rate(inst, 1, max(1, sample // 10), wname)
        cpu["single_thread"] = {"value": one["value"], "sample": one["sample"]}
        cpu.update(host)

    hot = None
    if args.workload == "d2_uniform" and pred is not None and not args.no_hotspot:
        hot = hotspot_paths(pred, steps=min(args.steps, 10), warmup=2)
        log(f"hotspot: {json.dumps(hot)}")

    paths = {k: {"ms_per_step": round(v["ms_per_step"], 4), "step_ms": v["step_ms"],
                 "pairs_per_s": round(K0 / (v["ms_per_step"] / 1e3), 1),
                 **({"overflowed": v.get("overflowed"), "slots": v.get("slots")}
                    if k == "learned" else {})}
             for k, v in res.items()}
    if "plain" in res and "learned" in res:
        paths["learned_speedup_vs_plain"] = round(
            res["plain"]["ms_per_step"] / res["learned"]["ms_per_step"], 4)
    return {
        "metric": METRIC,
        "value": round(K0 / (ms_step / 1e3), 1),
        "unit": "pairs/s",
        "regions_per_s": round((inst.n + inst.m) / (ms_step / 1e3), 1),
        "ms_per_step": round(ms_step, 4),
        "step_ms": res[best]["step_ms"],
        "match_only_ms": step_stats(per_match),
        "dtype": "f32",
        "config": {"workload": wname, "d": inst.d, "n": inst.n, "m": inst.m,
                   "seed": seed, "K": int(K0), "traversal": args.traversal, "path": best},
        "paths": paths,
        "predictor": ({"val_under_rate": train_rep["val_under_rate"],
                       "val_mae_log1p": round(train_rep["val_mae_log1p"], 4),
                       "delta": round(train_rep["delta"], 4), "train_s": train_rep["train_s"]}
                      if train_rep else None),
        "hotspot_learned_vs_plain": hot,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def bench_batch(args):
    import numpy as np
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import tune
    from paper_1309_3458_amd import workloads as W

    t0 = time.time()
    specs = W.batch_specs(3, 256)
    insts = [W.instance_from_spec(s) for s in specs]
    log(f"batch256 generated in {time.time() - t0:.2f}s: "
        f"sum n={sum(i.n for i in insts)} sum m={sum(i.m for i in insts)}")
    dev = lambda a: torch.from_numpy(a).cuda()
    tens = [(dev(i.s_lo), dev(i.s_hi), dev(i.u_lo), dev(i.u_hi)) for i in insts]
    table = tune.Table.load(args.tuning or tune.DEFAULT_TABLE)
    qpts, wpc = table.qpts(specs), table.waves_per_cu
    K0 = tune.batch_total(tens, qpts)
    out = torch.empty(K0, dtype=torch.int64, device="cuda")
    log(f"K = {K0}; tuned classes {len(table.qpt_map)}, waves/CU {wpc}")
    b = P.Batch(tens, K0, qpts=qpts, waves_per_cu=wpc, use_graph=True, out=out)

    def step():
        b.run()
        return K0

    for _ in range(args.warmup):
        step()
    wall, per, _ = evented_steps(step, args.steps)
    tot, _ = b.result()
    assert tot == K0
    b.free()

    # per-kernel durations: the same sequence launched eagerly, every launch
    # evented once, then HIP events around the dominant traversal only
    e = P.Batch(tens, K0, qpts=qpts, waves_per_cu=wpc, use_graph=False, out=out)
    e.run()
    torch.cuda.synchronize()
    P.prof_enable(True)
    e.run()
    torch.cuda.synchronize()
    prof = P.prof_read()
    P.prof_enable(False)
    dom = max((k for k in prof if k.startswith("batch_traverse")), key=lambda k: prof[k][0])
    log("[batch] per-kernel ms (one eager step): "
        + json.dumps({k: round(v[0], 4) for k, v in sorted(prof.items())}))
    P.prof_enable(True, only=dom)
    eager_wall, _, _ = evented_steps(lambda: e.run(), args.steps)
    dprof = P.prof_read()
    P.prof_enable(False)
    e.result()
    e.free()
    dms, dn = dprof[dom]
    cands = [candidates(i) for i in insts]
    ops = sum(c * 2 * i.d for c, i in zip(cands, insts))
    roofline = roofline_alu(sum(cands), ops, dom, dms / dn)
    roofline["timing"] = "eager launches of the same sequence"

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores, host = cpu_info()
        # a bounded sample: whole instances in a fixed shuffled order until
        # ~10 s of oracle time
        order = np.random.default_rng(11).permutation(len(insts))
        pairs, dt, used = 0, 0.0, 0
        for i in order:
            inst = insts[i]
            t1 = time.perf_counter()
            pairs += len(oracle.itm(inst.s_lo, inst.s_hi, inst.u_lo, inst.u_hi, threads=cores))
            dt += time.perf_counter() - t1
            used += 1
            if dt > 10.0:
                break
        cpu = {"value": round(pairs / dt, 1), "unit": "pairs/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{used} whole instances of batch256 in a fixed shuffled order, "
                         f"{dt:.2f}s, {pairs} pairs", **host}

    n_tot = sum(i.n + i.m for i in insts)
    return {
        "metric": METRIC,
        "value": round(K0 / (wall / 1e3), 1),
        "unit": "pairs/s",
        "regions_per_s": round(n_tot / (wall / 1e3), 1),
        "ms_per_step": round(wall, 4),
        "step_ms": step_stats(per),
        "eager_ms_per_step": round(eager_wall, 4),
        "dtype": "f32",
        "config": {"workload": "batch256_N1e3-2e5_d1-3_alpha0.01-100", "instances": 256,
                   "seed": 3, "K": int(K0), "regions": int(n_tot), "graph": True,
                   "waves_per_cu": wpc,
                   "qpt_hist": {str(q): qpts.count(q) for q in sorted(set(qpts))}},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def bench_serve(args):
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import learn, serve
    from paper_1309_3458_amd import workloads as W

    sched = W.serving_schedule(seed=4, rate=args.rate, duration_s=args.duration,
                               n_hi=args.n_hi)
    log(f"schedule: {len(sched)} requests over {args.duration}s")
    if args.predictor:
        pred, rep = P.Predictor.load(args.predictor), None
    else:
        pred, rep = learn.train_predictor(n_inst=32, per_instance=16000, epochs=20)
        log(f"predictor trained: {rep}")
    srv = P.Server(predictor=pred, workers=args.workers, host_pool=4 << 30,
                   batch_max=args.batch_max, batch_small=args.batch_small,
                   deliver_device=args.deliver_device, compact=args.compact)
    # warm-up on a different schedule (allocator caches, code objects)
    warm = W.serving_schedule(seed=104, rate=args.rate, duration_s=0.5, n_hi=args.n_hi)
    serve.run(srv, warm, sample_every=10 ** 9)
    st = serve.run(srv, sched, sample_every=100, log=log)
    srv.close()
    log(f"served: { {k: v for k, v in st.items() if k != 'samples'} }")
    if st["n_errors"]:
        raise SystemExit(f"serving errors: {st['errors']}")
    # identity of sampled results with the requests alone (and the oracle on
    # the small ones); the oracle's time on those is the CPU baseline
    import oracle
    cores, host = cpu_info()
    alone = serve.check_alone(st["samples"], sched)
    t_or, p_or, n_or = 0.0, 0, 0
    for i in sorted(st["samples"]):
        spec = sched[i].spec
        if spec.N > 200_000 or len(st["samples"][i]) > 2_000_000 or t_or > 10.0:
            continue
        h = [x.cpu().numpy() for x in W.device_instance(spec)]
        t0 = time.perf_counter()
        ref = oracle.itm(h[0], h[1], h[2], h[3], threads=cores)
        t_or += time.perf_counter() - t0
        assert (ref == st["samples"][i]).all() and len(ref) == len(st["samples"][i])
        p_or += len(ref)
        n_or += 1
    torch.cuda.synchronize()
    return {
        "metric": METRIC,
        "value": st["pairs_per_s"],
        "unit": "pairs/s",
        "regions_per_s": st["regions_per_s"],
        "ms_per_step": round(st["span_s"] * 1e3, 3),
        "latency_ms": st["latency_ms"],
        "latency_from_submit_ms": st["latency_from_submit_ms"],
        "queue_wait_ms": st["queue_wait_ms"],
        "service_ms": st["service_ms"],
        "client_late_ms": st["client_late_ms"],
        "dtype": "f32",
        "config": {"workload": f"serve_poisson_d3_N1e3-{args.n_hi:.0e}_alpha0.01-100", "seed": 4,
                   "rate_per_s": args.rate, "duration_s": args.duration,
                   "requests": st["requests"], "completed": st["completed"],
                   "pairs": st["pairs"], "regions": st["regions"], "workers": args.workers,
                   "learned_sizing": True,
                   "inputs": "generated in device memory just before arrival",
                   "results": "device memory" if args.deliver_device else "pinned host memory",
                   "batch_max": args.batch_max, "batch_small": args.batch_small,
                   "compact_results": args.compact},
        "checks": {"sampled_equal_alone": alone, "sampled_equal_oracle": n_or},
        "hbm_peak_bytes": st["hbm_peak_bytes"],
        "roofline": None,
        "cpu_baseline": ({"value": round(p_or / t_or, 1), "unit": "pairs/s", "cores": cores,
                          "kind": "oracle",
                          "sample": f"{n_or} sampled requests (every 100th, N <= 2e5), "
                                    f"{t_or:.2f}s, {p_or} pairs", **host}
                         if t_or > 0 else None),
    }


def bench_sweep(args):
    """Sec. V's experiment (d = 1, n = m = N/2, uniform lower ends on [0, L),
    common length alpha L / N) on the GPU: ITM build + match per step, and
    Brute-Force Matching (Algorithm 2) and Sort-Based Matching (Algorithm 3)
    on the same inputs."""
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import workloads as W

    rows = []
    dev = lambda a: torch.from_numpy(a).cuda()
    for N in (50_000, 100_000, 200_000, 300_000, 400_000, 500_000):
        for alpha in (0.01, 1.0, 100.0):
            n, m = W.split_regions(N)
            inst = W.uniform_instance([5, N, int(alpha * 100)], n, m, 1,
                                      W.side_for_alpha(alpha, N, 1))
            s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
            t = P.build(s_lo, s_hi)
            K = int(P.match(t, u_lo, u_hi).numel())
            t.free()
            out = torch.empty(max(K, 1), dtype=torch.int64, device="cuda")

            def step():
                t = P.build(s_lo, s_hi)
                k = P.match(t, u_lo, u_hi, out=out).numel()
                t.free()
                return k

            for _ in range(args.warmup):
                step()
            wall, per, k2 = evented_steps(step, args.steps)
            assert k2 == K
            bf = lambda: P.match_brute(s_lo, s_hi, u_lo, u_hi, out=out).numel()
            bf()
            bwall, bper, kb = evented_steps(bf, 3)
            assert kb == K
            sb = lambda: P.match_sbm(s_lo, s_hi, u_lo, u_hi, out=out).numel()
            for _ in range(args.warmup):
                sb()
            swall, sper, ks = evented_steps(sb, args.steps)
            assert ks == K
            rows.append({"N": N, "alpha": alpha, "K": K, "itm_ms": step_stats(per),
                         "brute_ms": step_stats(bper), "sbm_ms": step_stats(sper),
                         "itm_pairs_per_s": round(K / (wall / 1e3), 1),
                         "speedup_itm_vs_brute": round(bwall / wall, 2),
                         "speedup_itm_vs_sbm": round(swall / wall, 2)})
            log(f"N={N} alpha={alpha}: K={K} ITM {wall:.4f} ms, SBM {swall:.4f} ms, "
                f"BF {bwall:.3f} ms")
    last = [r for r in rows if r["N"] == 500_000 and r["alpha"] == 100.0][0]
    return {"metric": "ITM build+match time, d=1 sweep of the paper's experiment",
            "value": last["itm_pairs_per_s"], "unit": "pairs/s",
            "ms_per_step": last["itm_ms"]["mean"], "dtype": "f32",
            "config": {"workload": "sweep_1d_N5e4-5e5_alpha0.01-1-100",
                       "value_at": "N=5e5 alpha=100"},
            "sweep": rows, "roofline": None, "cpu_baseline": None}


def bench_fig7(args):
    """Fig. 7 of Sec. V on the GPU: ITM (build + match, one step each) over
    N in {50, 100, ..., 500} x 10^3 extents (n = m = N/2, d = 1, uniform lower
    ends, common length alpha L / N) and alpha from 0.01 to 100 in
    half-decade steps.  The mean time per step of every cell, K and pairs/s
    go into the JSON line; a markdown table of the times goes to stderr."""
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import workloads as W

    Ns = [50_000 * i for i in range(1, 11)]
    alphas = [0.01, 0.03, 0.1, 0.3, 1.0, 3.0, 10.0, 30.0, 100.0]
    steps = min(args.steps, 10)
    dev = lambda a: torch.from_numpy(a).cuda()
    rows = []
    for N in Ns:
        for alpha in alphas:
            n, m = W.split_regions(N)
            inst = W.uniform_instance([7, N, int(round(alpha * 100))], n, m, 1,
                                      W.side_for_alpha(alpha, N, 1))
            s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
            t = P.build(s_lo, s_hi)
            K = int(P.match(t, u_lo, u_hi).numel())
            t.free()
            out = torch.empty(max(K, 1), dtype=torch.int64, device="cuda")

            def step():
                t = P.build(s_lo, s_hi)
                k = P.match(t, u_lo, u_hi, out=out).numel()
                t.free()
                return k

            for _ in range(min(args.warmup, 2)):
                step()
            wall, per, k2 = evented_steps(step, steps)
            assert k2 == K
            rows.append({"N": N, "alpha": alpha, "K": K, "ms": step_stats(per),
                         "pairs_per_s": round(K / (wall / 1e3), 1)})
    head = "| N \\ alpha | " + " | ".join(f"{a:g}" for a in alphas) + " |"
    log("ITM build + match, mean ms per step (d = 1, one MI355X)")
    log(head)
    log("|" + "---|" * (len(alphas) + 1))
    for N in Ns:
        cells = [f"{r['ms']['mean']:.3f}" for r in rows if r["N"] == N]
        log(f"| {N} | " + " | ".join(cells) + " |")
    last = [r for r in rows if r["N"] == Ns[-1] and r["alpha"] == alphas[-1]][0]
    return {"metric": "ITM build+match time over (N, alpha), d=1 (Fig. 7 of the paper)",
            "value": last["pairs_per_s"], "unit": "pairs/s", "ms_per_step": last["ms"]["mean"],
            "dtype": "f32",
            "config": {"workload": "sweep_fig7_d1_N5e4-5e5_alpha0.01-100",
                       "value_at": "N=5e5 alpha=100", "steps_per_cell": steps},
            "grid": rows, "roofline": None, "cpu_baseline": None}


def bench_dynamic(args):
    """Dynamic DDM (the paper's dynamic scenario) on the d=2, 500,000 +
    500,000 squares workload (alpha = 1, seed 1): each step moves 1% of one
    set (updates and subscriptions alternately) to new uniform positions;
    the resident matcher recomputes only the moved extents' pairs.  Beside it:
    a full build + match of the same sets."""
    import numpy as np
    import torch

    import paper_1309_3458_amd as P
    from paper_1309_3458_amd import workloads as W

    inst = W.uniform_2d_1m(1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dy = P.Dynamic(dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi))
    rng = np.random.default_rng(11)
    c = inst.m // 100
    side = np.float32(inst.side)
    moves = []
    for i in range(args.warmup + args.steps):
        which = i % 2
        ids = dev(rng.choice(inst.n if which == 0 else inst.m, c, replace=False).astype(np.int32))
        lo = rng.uniform(0, 1e6, (2, c)).astype(np.float32)
        moves.append((which, ids, dev(lo), dev((lo + side).astype(np.float32))))
    it = iter(moves)
    for _ in range(args.warmup):
        dy.move(*next(it))
    wall, per, K = evented_steps(lambda: dy.move(*next(it)), args.steps)
    s_lo, s_hi, u_lo, u_hi = dev(inst.s_lo), dev(inst.s_hi), dev(inst.u_lo), dev(inst.u_hi)
    out = torch.empty(K + (1 << 16), dtype=torch.int64, device="cuda")

    def full():
        t = P.build(s_lo, s_hi)
        k = P.match(t, u_lo, u_hi, out=out).numel()
        t.free()
        return k

    for _ in range(args.warmup):
        full()
    fwall, fper, _ = evented_steps(full, args.steps)
    dy.free()
    return {"metric": "dynamic DDM: time per move of 1% of one set (resident trees and result)",
            "value": round(wall, 4), "unit": "ms", "ms_per_step": round(wall, 4),
            "higher_is_better": False, "dtype": "f32",
            "config": {"workload": "dynamic_d2_N1e6_alpha1_move1pct", "seed": 1,
                       "moved_per_step": c, "K_after": int(K)},
            "step_ms": step_stats(per), "full_rematch_ms": step_stats(fper),
            "speedup_vs_full_rematch": round(fwall / wall, 2),
            "roofline": None, "cpu_baseline": None}


def bench_copy(args):
    """1 GiB device-to-device copy per step: the reference kernel whose
    FETCH_SIZE / WRITE_SIZE counters calibrate the traffic of the others."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    wall, per, _ = evented_steps(lambda: b.copy_(a), args.steps)
    gbs = 2 * nbytes / (wall / 1e3) / 1e9
    return {"metric": "device copy bandwidth (read + write bytes / s)", "value": round(gbs, 1),
            "unit": "GB/s", "ms_per_step": round(wall, 4), "step_ms": step_stats(per),
            "dtype": "u8", "config": {"workload": "hbm_copy_1GiB", "bytes_read": nbytes,
                                      "bytes_written": nbytes},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
            "cpu_baseline": None}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: every node here exposes a single MI355X and "
              "the matcher has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch256":
        rec = bench_batch(args)
    elif args.workload == "serve":
        rec = bench_serve(args)
    elif args.workload == "hbm_copy":
        rec = bench_copy(args)
    elif args.workload == "sweep_1d":
        rec = bench_sweep(args)
    elif args.workload == "sweep_fig7":
        rec = bench_fig7(args)
    elif args.workload == "dynamic":
        rec = bench_dynamic(args)
    else:
        rec = bench_single(args)
    head = {"metric": rec.pop("metric"), "value": rec.pop("value"), "unit": rec.pop("unit"),
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": rec.pop("ms_per_step"),
            "higher_is_better": rec.pop("higher_is_better", True),
            "scaling": "weak", "vs_baseline": None, "dtype": rec.pop("dtype"),
            "data": "synthetic", "config": rec.pop("config")}
    head.update(rec)
    print(json.dumps(head), flush=True)


if __name__ == "__main__":
    main()
