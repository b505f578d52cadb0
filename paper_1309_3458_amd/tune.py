"""Launch-parameter autotuner for the batched matcher.

Two parameters of a batch change its speed but never its bytes (the batch
tests run every value):

* qpt, the updates per traversal work item (16, 32 or 64), chosen per
  instance class (N bucket = floor(log2 N), d, alpha bucket =
  round(log10 alpha)): dense classes favour full 64-update tiles, sparse ones
  with short candidate ranges can prefer narrower tiles whose enclosing
  interval is tighter;
* waves_per_cu, 0 for one wavefront per tile or the occupancy of a
  persistent traversal grid, chosen for the whole workload.

The tuner times graph replays of the batch on the current GPU and writes a
JSON table: {"device": ..., "waves_per_cu": W, "qpt": {"lg,d,la": q, ...},
"timings": {...}}.  Classes missing from a table get qpt 64.

    python -m paper_1309_3458_amd.tune --out paper_1309_3458_amd/tuning/batch_gfx950.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(PKG, "tuning", "batch_gfx950.json")
QPTS = (16, 32, 64)
WAVES = (0, 8, 16, 24)


def bucket(N: int, d: int, alpha: float) -> str:
    lg = int(math.floor(math.log2(max(int(N), 2))))
    la = int(round(math.log10(alpha)))
    return f"{lg},{int(d)},{la}"


class Table:
    def __init__(self, qpt=None, waves_per_cu: int = 0, device: str = "", timings=None):
        self.qpt_map = dict(qpt or {})
        self.waves_per_cu = int(waves_per_cu)
        self.device = device
        self.timings = timings or {}

    @classmethod
    def load(cls, path: str = DEFAULT_TABLE) -> "Table":
        if not os.path.exists(path):
            return cls()
        with open(path) as f:
            t = json.load(f)
        return cls(t.get("qpt"), t.get("waves_per_cu", 0), t.get("device", ""),
                   t.get("timings"))

    def save(self, path: str):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump({"device": self.device, "waves_per_cu": self.waves_per_cu,
                       "qpt": dict(sorted(self.qpt_map.items())), "timings": self.timings},
                      f, indent=1, sort_keys=True)
            f.write("\n")

    def qpt(self, N: int, d: int, alpha: float) -> int:
        return int(self.qpt_map.get(bucket(N, d, alpha), 64))

    def qpts(self, specs) -> list[int]:
        return [self.qpt(s.N, s.d, s.alpha) for s in specs]


def _tensors(insts):
    import torch
    dev = lambda a: torch.from_numpy(a).cuda()
    return [(dev(i.s_lo), dev(i.s_hi), dev(i.u_lo), dev(i.u_hi)) for i in insts]


def batch_total(tens, qpts=None) -> int:
    """Exact number of pairs of a batch (a run with zero capacity)."""
    import paper_1309_3458_amd as P
    b = P.Batch(tens, 0, use_graph=False, qpts=qpts)
    b.run()
    try:
        b.result()
    except P.DDMError as e:
        if e.code != -3:
            raise
    tot = b.total
    b.free()
    return tot


def time_batch(tens, K: int, qpts=None, waves_per_cu: int = 0, reps: int = 10,
               out=None) -> float:
    """Mean ms of a graph replay of the batch."""
    import torch
    import paper_1309_3458_amd as P
    b = P.Batch(tens, K, qpts=qpts, waves_per_cu=waves_per_cu, use_graph=True, out=out)
    b.run()
    b.run()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.run()
    e.record()
    torch.cuda.synchronize()
    tot, _ = b.result()
    assert tot == K
    b.free()
    return s.elapsed_time(e) / reps


def _class_instances(key: str, count: int, seed: int):
    """`count` uniform instances drawn inside one class."""
    import numpy as np
    from . import workloads as W
    lg, d, la = (int(x) for x in key.split(","))
    rng = np.random.default_rng([seed, lg, d, la + 10])
    insts = []
    for i in range(count):
        N = max(4, 2 * int(2 ** rng.uniform(lg, lg + 1) / 2))
        alpha = 10 ** rng.uniform(la - 0.5, la + 0.5)
        n, m = W.split_regions(N)
        insts.append(W.uniform_instance([seed, lg, d, la + 10, i], n, m, d,
                                        W.side_for_alpha(alpha, N, d)))
    return insts


def tune(specs, per_class: int = 4, reps: int = 10, seed: int = 500, log=print) -> Table:
    """Tune qpt for every class present in `specs`, then waves_per_cu on the
    whole set of specs with the chosen qpts."""
    import torch
    from . import workloads as W
    keys = sorted({bucket(s.N, s.d, s.alpha) for s in specs})
    table = Table(device=torch.cuda.get_device_name(0))
    for key in keys:
        tens = _tensors(_class_instances(key, per_class, seed))
        K = batch_total(tens)
        ms = {q: time_batch(tens, K, [q] * len(tens), reps=reps) for q in QPTS}
        best = min(ms, key=ms.get)
        table.qpt_map[key] = best
        table.timings[key] = {str(q): round(v, 4) for q, v in ms.items()}
        log(f"class {key}: K={K} " + " ".join(f"q{q}={v:.3f}ms" for q, v in ms.items())
            + f" -> {best}")
        del tens
    insts = [W.instance_from_spec(s) for s in specs]
    tens = _tensors(insts)
    qpts = table.qpts(specs)
    K = batch_total(tens, qpts)
    out = torch.empty(K, dtype=torch.int64, device="cuda")
    ms = {w: time_batch(tens, K, qpts, w, reps=reps, out=out) for w in WAVES}
    ms64 = time_batch(tens, K, None, 0, reps=reps, out=out)
    table.waves_per_cu = min(ms, key=ms.get)
    table.timings["waves_per_cu"] = {str(w): round(v, 4) for w, v in ms.items()}
    table.timings["untuned_q64_w0"] = round(ms64, 4)
    log(f"whole workload K={K}: " + " ".join(f"w{w}={v:.3f}ms" for w, v in ms.items())
        + f" -> {table.waves_per_cu}; untuned (qpt 64, one wave per tile) {ms64:.3f}ms")
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--seed", type=int, default=3, help="seed of the batched workload")
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--per-class", type=int, default=4)
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(PKG))
    import torch
    from . import workloads as W
    assert torch.cuda.is_available(), "the tuner times kernels on a GPU"
    t0 = time.time()
    table = tune(W.batch_specs(a.seed, a.count), a.per_class, a.reps,
                 log=lambda s: print(s, flush=True))
    table.save(a.out)
    print(f"wrote {a.out} ({len(table.qpt_map)} classes, {time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    main()
