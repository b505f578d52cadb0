"""Open-loop serving driver: Poisson arrivals of match requests into a Server.

Every request of a pre-drawn schedule is submitted at its arrival time;
its coordinates are generated in device memory shortly before.  Latency is
measured from the scheduled arrival to the result in host memory, on the
server's own CLOCK_MONOTONIC timestamps, so a client that falls behind the
schedule is charged to the latency, not hidden.
"""
from __future__ import annotations

import math
import threading
import time

import numpy as np

from . import workloads as W


def percentile(x, q):
    if not len(x):
        return float("nan")
    return float(np.percentile(np.asarray(x, dtype=np.float64), q))


def run(server, schedule, sample_every: int = 100, lead_s: float = 0.5, log=None,
        sample_max_pairs: int = 20_000_000, sample_bytes: int = 4 << 30,
        lookahead_s: float = 1.0):
    """Serve `schedule` (a list of workloads.Request) on `server`.

    Three threads: the generator draws each request's coordinates in device
    memory up to `lookahead_s` before its arrival (the data a real client
    would have ready when it sends the request); the submitter hands each
    request to the server at its scheduled arrival time; the drain thread
    collects completions.  Latency runs from the scheduled arrival to the
    result in host memory (and, separately, from the moment the request was
    handed to the server, which excludes any lag of the client's own
    generation on the shared GPU).  Returns a dict of statistics plus `samples`:
    {request index: keys (uint64)} for every sample_every-th request (up to
    sample_max_pairs pairs each and sample_bytes in all), for identity
    checks after the run.
    """
    import collections

    import torch
    gen_stream = torch.cuda.Stream()
    sub_stream = torch.cuda.Stream()
    ready = collections.deque()
    cv = threading.Condition()
    ticket_of = {}
    lat, lat_sub, wait, service, K, regions, late = [], [], [], [], [], [], []
    submit_ns = {}
    samples = {}
    kept = [0]
    errors = []
    n_req = len(schedule)
    t0 = time.monotonic_ns() + int(lead_s * 1e9)
    la = int(lookahead_s * 1e9)

    def generator():
        with torch.cuda.stream(gen_stream):
            for i, rq in enumerate(schedule):
                target = t0 + int(rq.arrival_s * 1e9) - la
                dt = (target - time.monotonic_ns()) / 1e9
                if dt > 0:
                    time.sleep(dt)
                tens = W.device_instance(rq.spec)
                ev = torch.cuda.Event()
                ev.record(gen_stream)
                with cv:
                    ready.append((i, tens, ev))
                    cv.notify()

    def submitter():
        for i, rq in enumerate(schedule):
            target = t0 + int(rq.arrival_s * 1e9)
            with cv:
                while not ready or ready[0][0] != i:
                    cv.wait()
                _, tens, ev = ready.popleft()
            dt = (target - time.monotonic_ns()) / 1e9
            if dt > 0:
                time.sleep(dt)
            ev.synchronize()
            now = time.monotonic_ns()
            late.append(max(0, now - target) / 1e6)
            t = server.submit(*tens, arrival_ns=target, stream=sub_stream)
            submit_ns[i] = now
            ticket_of[t] = i

    def drain():
        got = 0
        while got < n_req:
            for t in server.wait_any(50):
                while t not in ticket_of:  # submit returned but not recorded yet
                    time.sleep(0)
                i = ticket_of[t]
                r = server.result(t, copy=False)
                if (i % sample_every == 0 and r["status"] == 0 and r["count"] <= sample_max_pairs
                        and kept[0] + 8 * r["count"] <= sample_bytes):
                    r = server.result(t, copy=True)
                    kept[0] += 8 * r["count"]
                if r["status"] != 0:
                    errors.append((i, r["status"], r.get("detail", "")))
                else:
                    lat.append((r["t_done_ns"] - r["t_arrival_ns"]) / 1e6)
                    lat_sub.append((r["t_done_ns"] - submit_ns.get(i, r["t_arrival_ns"])) / 1e6)
                    wait.append((r["t_start_ns"] - r["t_arrival_ns"]) / 1e6)
                    service.append((r["t_done_ns"] - r["t_start_ns"]) / 1e6)
                    K.append(r["count"])
                    regions.append(schedule[i].spec.N)
                    if "pairs" in r:
                        samples[i] = r["pairs"]
                    elif "sub_ids" in r:
                        samples[i] = (r["sub_ids"], r["upd_offsets"])
                server.release(t)
                got += 1
                if log and got % 5000 == 0:
                    log(f"served {got}/{n_req}: p50 {percentile(lat, 50):.2f} ms "
                        f"p99 {percentile(lat, 99):.2f} ms, {server.stats()}")

    threads = [threading.Thread(target=f, daemon=True) for f in (drain, generator, submitter)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    t_end = time.monotonic_ns()
    span_s = (t_end - t0) / 1e9
    st = server.stats()

    def pct(x):
        return {"p50": round(percentile(x, 50), 3), "p99": round(percentile(x, 99), 3),
                "mean": round(float(np.mean(x)) if x else math.nan, 3),
                "max": round(max(x) if x else math.nan, 3)}

    return {
        "requests": n_req, "completed": len(lat), "errors": errors[:10],
        "n_errors": len(errors),
        "latency_ms": pct(lat), "latency_from_submit_ms": pct(lat_sub),
        "queue_wait_ms": pct(wait), "service_ms": pct(service),
        "client_late_ms": {"p99": round(percentile(late, 99), 3),
                           "max": round(max(late) if late else math.nan, 3)},
        "pairs": int(sum(K)), "regions": int(sum(regions)), "span_s": round(span_s, 3),
        "pairs_per_s": round(sum(K) / span_s, 1), "regions_per_s": round(sum(regions) / span_s, 1),
        "hbm_peak_bytes": st["hbm_peak"],
        "samples": samples,
    }


def keys_from_compact(sub_ids, upd_offsets):
    """The 64-bit keys (update << 32) | subscription of a compact result
    (subscription ids plus update offsets), for comparisons."""
    m = len(upd_offsets) - 1
    upd = np.repeat(np.arange(m, dtype=np.uint64), np.diff(upd_offsets).astype(np.int64))
    return (upd << np.uint64(32)) | np.asarray(sub_ids).astype(np.uint64)


def check_alone(samples, schedule):
    """Every sampled result equals the same request matched alone on the GPU
    (ddm_build + ddm_match, nothing else running).  Compact samples are
    replaced by their keys.  Returns the number of requests checked."""
    import torch

    import paper_1309_3458_amd as P
    checked = 0
    for i, got in sorted(samples.items()):
        if isinstance(got, tuple):  # compact result
            got = keys_from_compact(*got)
            samples[i] = got
        s_lo, s_hi, u_lo, u_hi = W.device_instance(schedule[i].spec)
        t = P.build(s_lo, s_hi)
        want = P.match(t, u_lo, u_hi).cpu().numpy().view(np.uint64)
        t.free()
        if not np.array_equal(got, want):
            raise AssertionError(f"request {i}: served result differs from the result alone")
        checked += 1
    torch.cuda.synchronize()
    return checked
