"""Autotuner for the launch shapes (run on the GPU).

Times the library at a grid of shapes and writes tuned.json next to this
file; the binding then gives every plan the tuned shape for its own state
dimension, length and quadrature class (so a plan's result never depends on
the batch it runs in):

  * segments: chain segments per plan, per state dimension n and length N
    (the depth of the marginals/mean-solve sweeps is about
    2 N / segments + 2 segments block steps).

The expectation kernel needs no table: its factors per workgroup are
chosen per launch from the batch and never change results.

Usage: python -m paper_2411_03416_amd.autotune [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _time_solve(pg, probs, iters, reps=3, **kw):
    import torch
    ctx = pg.pgvimp_create(probs, use_graph=True, **kw)
    pg.pgvimp_solve(ctx, iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pg.pgvimp_solve(ctx, iters)
    dt = (time.perf_counter() - t0) / reps
    pg.pgvimp_destroy(ctx)
    return dt


def tune(quick=False):
    import paper_2411_03416_amd as pg
    import workloads
    out = {"segments": {}, "device": None}
    import torch
    out["device"] = torch.cuda.get_device_name(0)
    Ns = [50, 150, 400, 750, 1000] if not quick else [50, 750]
    for n, maker in ((4, lambda s, N: workloads.config1_problem(s, N=N)),
                     (6, lambda s, N: workloads.point3d_problem(s, N=N)),
                     (14, lambda s, N: workloads.arm_problem(s, N=N))):
        rows = []
        for N in Ns:
            if n == 14 and N > 400:
                continue
            plans = [maker(k, N) for k in range(8 if n < 14 else 2)]
            for p in plans:
                p["n_iters"] = 3
                p.pop("segments", None)
            cands = sorted({c for c in (4, 8, 12, 16, 24, 32, 48, 64) if c <= max(1, N // 2)})
            best = None
            for c in cands:
                for p in plans:
                    p["segments"] = c
                dt = _time_solve(pg, plans, 3)
                print(f"n={n} N={N} segments={c}: {dt * 1e3:.2f} ms", flush=True)
                if best is None or dt < best[1]:
                    best = (c, dt)
            rows.append([N, best[0]])
        out["segments"][str(n)] = rows
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    args = ap.parse_args()
    res = tune(args.quick)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))
