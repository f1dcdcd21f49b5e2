"""Benchmark of the P-GVIMP hot path on one MI355X.

Workload (default): 32 seeded point-robot plans, N = 750 support states
each, 500 x 500 FP32 SDF maps of 40 discs/boxes, Gauss-Hermite p = 5 on
(x, y), 20 proximal iterations.  One step = one full solve of the batch:
prior build, initial marginals and 20 iterations (expectations, step-size
selection, update, marginals) for all 32 plans, captured in one HIP graph.
The primary mode is mixed precision (FP32 quadrature, FP64 elsewhere); the
plain FP64 path is timed beside it.

Prints ONE JSON line.  `value` = factor expectations per second over the
whole path (32 x 750 factors x 20 iterations per step / step time).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor-expectations/s + plans/s with p50/p99 latency, mixed vs plain FP64 GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plans", type=int, default=32)
    ap.add_argument("--N", type=int, default=750)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip plans/s of configs 0, 2 and 3")
    ap.add_argument("--configs-only", action="store_true", help="only plans/s of configs 0, 2 and 3")
    ap.add_argument("--segments", type=int, default=0)
    ap.add_argument("--group", type=int, default=0, help="factors per expectation workgroup (0 = per launch)")
    ap.add_argument("--trial-width", type=int, default=0, help="trial step sizes per window (0 = library default)")
    ap.add_argument("--trial-slots", type=int, default=0, help="widest trial window (0 = library default)")
    ap.add_argument("--trial-lookahead", type=int, default=0,
                    help="first window = previous trial count + this (0 = full first window)")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving mix (Poisson arrivals of configs 0-3) instead of the batch solve")
    ap.add_argument("--qps-list", type=float, nargs="*", default=None, help="offered loads of --serve's sweep")
    ap.add_argument("--requests", type=int, default=2000, help="measured requests of --serve")
    ap.add_argument("--warmup-requests", type=int, default=200)
    ap.add_argument("--hbm-budget-gib", type=float, default=16.0, help="--serve's admission budget")
    ap.add_argument("--serve-max-n", type=int, default=1000)
    ap.add_argument("--serial-sample", type=int, default=100, help="requests of the serial FP64 baseline")
    ap.add_argument("--serve-timeout", type=float, default=300.0)
    ap.add_argument("--sweep-plans", type=int, nargs="*", default=None, help="plan counts of --expect-sweep")
    ap.add_argument("--sweep-prec", choices=("mixed", "fp64", "both"), default="both",
                    help="precisions of --expect-sweep")
    ap.add_argument("--sweep-reps", type=int, default=20, help="timed launches per --expect-sweep point")
    ap.add_argument("--sweep-maps", choices=("shared", "distinct"), default="shared",
                    help="--expect-sweep: plans k and k+32 share a map, or every plan has its own copy")
    ap.add_argument("--expect-sweep", action="store_true",
                    help="time the expectation kernel alone over a batch sweep (32 plans, growing N)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="the shapes of the paper's efficiency tables (Sec. 7.1) instead of the headline line")
    ap.add_argument("--tables-iters", type=int, default=20, help="iterations of the whole-optimisation table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 512 MiB copy kernel once (known traffic, to scale memory counters)")
    return ap.parse_args()


def serve(args, pg):
    """Serving mix (config 4): Poisson arrivals of requests drawn from
    configs 0-3 with N ~ U{50..max_N} (state dimensions 4, 6, 14), up to 256
    plans live, admission by an HBM budget; warm-up requests first, the
    measured ones after.  The offered load is swept upward until the served
    plans/s fall below 90 % of it (saturation); then mixed and FP64 are
    served at 70 % of the saturated rate, and the serial FP64 baseline (one
    plan at a time, back to back) is timed on a sample of the same stream."""
    import workloads
    from paper_2411_03416_amd.serve import ServingEngine
    warm, count = args.warmup_requests, args.requests
    budget = int(args.hbm_budget_gib * (1 << 30))
    base = workloads.serving_mix(seed=0, count=warm + count, qps=1.0, n_range=(50, args.serve_max_n), map_pool=16)
    for _, p in base:
        p["n_iters"] = min(p["n_iters"], args.iters)
    print(f"serve: {len(base)} requests generated", flush=True)

    def at(qps):
        return [(t / qps, p) for t, p in base]

    def run(qps, prec):
        eng = ServingEngine(precision=prec, hbm_budget=budget, max_concurrent=256, chunk=2,
                            max_N=args.serve_max_n)
        m, _ = eng.run(at(qps), timeout_s=args.serve_timeout, measured_from=warm)
        eng.close()
        m["qps"] = qps
        print(f"serve: {qps:.1f} QPS {'mixed' if prec == pg.MIXED else 'fp64'}: {m['plans_per_s']:.1f} plans/s, "
              f"p50 {m['p50_ms']} ms, p99 {m['p99_ms']} ms, completed {m['completed']}/{m['requests']}", flush=True)
        return m

    sweep, sat = [], None
    for q in (args.qps_list or [25.0, 50.0, 100.0, 200.0, 400.0, 800.0]):
        m = run(q, pg.MIXED)
        sweep.append(m)
        # saturated: requests left unanswered at the time limit, or the
        # served rate below 90 % of the offered one (a request the library
        # rejects is answered, with its error)
        if m["completed"] + m["errors"] < m["requests"] or m["plans_per_s"] < 0.9 * q:
            sat = m["plans_per_s"]
            break
    if sat is None:
        sat = max(m["plans_per_s"] for m in sweep)
    q70 = 0.7 * sat
    mixed = run(q70, pg.MIXED)
    fp64 = run(q70, pg.FP64)
    # serial FP64: one plan at a time, back to back, on the first requests
    sample = [(0.0, p) for _, p in base[warm:warm + args.serial_sample]]
    eng = ServingEngine(precision=pg.FP64, hbm_budget=budget, serial=True, max_N=args.serve_max_n)
    t0 = time.perf_counter()
    _, recs = eng.run(sample, timeout_s=args.serve_timeout)
    wall = time.perf_counter() - t0
    eng.close()
    svc = np.array([r["done"] - r.get("admitted", r["done"]) for r in recs if "done" in r and "error" not in r])
    serial = {"plans_per_s": len(svc) / wall if wall > 0 else 0.0, "sample": len(sample),
              "service_p50_ms": float(np.percentile(svc, 50) * 1e3) if svc.size else None,
              "service_p99_ms": float(np.percentile(svc, 99) * 1e3) if svc.size else None}
    print(f"serve: serial FP64 {serial['plans_per_s']:.2f} plans/s on {len(sample)} requests", flush=True)
    out = {"metric": METRIC + " (serving mix)", "value": mixed["plans_per_s"], "unit": "plans/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32 quadrature + fp64",
           "config": {"workload": f"serving mix: Poisson arrivals, configs 0-3, N ~ U{{50..{args.serve_max_n}}}, "
                                  f"{warm} warm-up + {count} measured requests, 256 concurrent, HBM budget "
                                  f"{args.hbm_budget_gib} GiB", "qps": q70},
           "saturation_plans_per_s": sat, "sweep": sweep, "mixed": mixed, "fp64": fp64, "serial_fp64": serial}
    print(json.dumps(out), flush=True)


def expect_sweep(args, pg):
    """Expectation kernel alone (config 1 shape: point robot, 500x500 maps,
    p = 5, N = 750) over a batch sweep of the number of plans (the 32 seeded
    maps repeated), mixed and FP64.  (Longer chains at dt = 0.1 make the
    prior numerically singular, so the batch grows in plans.)
    Achieved HBM rate = 88 B per factor (mean 2 + covariance 3 doubles in,
    E + g 2 + H 3 doubles out) / mean launch time; the SDF gathers (4 cells x
    4 B per node, 25 nodes) and FP32 node flops (~1.1 kFLOP) are reported
    beside it."""
    import numpy as np
    import torch
    import workloads
    rows = []
    base = [workloads.config1_problem(seed=k) for k in range(32)]
    N = 750
    for n_plans in ((32, 128, 512, 2048, 8192) if not args.sweep_plans else tuple(args.sweep_plans)):
        probs = []
        for k in range(n_plans):
            q = dict(base[k % 32])
            q["n_iters"] = 1
            if args.sweep_maps == "distinct" and k >= 32:
                # the same obstacles, offset by a small constant per plan: a
                # map of its own on the device for every plan
                q["sdf"] = base[k % 32]["sdf"] + np.float32(1e-4 * (k // 32))
            if args.group:
                q["expect_group"] = args.group
            probs.append(q)
        for name, prec in (("mixed", pg.MIXED), ("fp64", pg.FP64)):
            if args.sweep_prec not in ("both", name):
                continue
            ctx = pg.pgvimp_create(probs, precision=prec, use_graph=False, trial_width=1)
            pg.pgvimp_expect_all(ctx, 3)
            pg.pgvimp_profile(ctx, True)
            pg.pgvimp_kernel_times(ctx, reset=True)
            pg.pgvimp_expect_all(ctx, args.sweep_reps)
            kt = pg.pgvimp_kernel_times(ctx, reset=True)
            pg.pgvimp_destroy(ctx)
            torch.cuda.synchronize()
            ms = kt["expect"][0]
            f = n_plans * N
            rows.append({"factors": f, "precision": name, "maps": args.sweep_maps, "group": args.group or "auto",
                         "ms": ms,
                         "factors_per_s": f / (ms * 1e-3),
                         "hbm_GBs": 88.0 * f / (ms * 1e-3) / 1e9, "hbm_frac": 88.0 * f / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "gather_GBs": 400.0 * f / (ms * 1e-3) / 1e9,
                         "fp32_tflops": 1100.0 * f / (ms * 1e-3) / 1e12})
            print(json.dumps(rows[-1]), flush=True)
    out = {"metric": "expectation kernel alone, batch sweep", "unit": "factor-expectations/s", "n_gpus": 1,
           "data": "synthetic", "config": {"workload": "point robot, 500x500 maps, GH p=5, N=750, plans swept"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def make_batch(n_plans, N, iters):
    import workloads
    probs = []
    for k in range(n_plans):
        p = workloads.config1_problem(seed=k, N=N)
        p["n_iters"] = iters
        probs.append(p)
    return probs


def timed_solve(pg, probs, precision, steps, warmup, iters, segments=0, group=0, profile=True, trial_width=0,
                trial_lookahead=0, trial_slots=0):
    """Create one context for the batch, warm up, then time `steps` solves,
    each one HIP graph replay.  With profile, the same number of solves is
    then run with HIP events around every kernel on the context's stream
    (launched directly, since events inside a graph cannot be timed) to get
    each kernel's mean duration."""
    import torch
    if segments or group:
        # explicit shapes override the tuned per-plan ones
        probs = [dict(p) for p in probs]
        for p in probs:
            if segments:
                p["segments"] = segments
            if group:
                p["expect_group"] = group
    ctx = pg.pgvimp_create(probs, precision=precision, use_graph=True, segments=segments, expect_group=group,
                           trial_width=trial_width, trial_lookahead=trial_lookahead, trial_slots=trial_slots)
    for _ in range(warmup):
        pg.pgvimp_solve(ctx, iters)
    torch.cuda.synchronize()
    step_ms, trials = [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        st = pg.pgvimp_solve(ctx, iters)
        step_ms.append(1e3 * (time.perf_counter() - s0))
        trials += sum(v["trials_total"] for v in st.values())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = None
    evals = prof_trials = 0
    if profile:
        pg.pgvimp_profile(ctx, True)
        pg.pgvimp_kernel_times(ctx, reset=True)
        t1 = time.perf_counter()
        for _ in range(steps):
            sp = pg.pgvimp_solve(ctx, iters)
            evals += sum(v["evals_total"] for v in sp.values())
            prof_trials += sum(v["trials_total"] for v in sp.values())
        kt = pg.pgvimp_kernel_times(ctx, reset=True)
        kt["eager_ms_per_step"] = 1e3 * (time.perf_counter() - t1) / steps
        pg.pgvimp_profile(ctx, False)
    status = [v["status"] for v in st.values()]
    seg, group_used = pg.pgvimp_launch_shape(ctx, probs[0]["N"])
    pg.pgvimp_destroy(ctx)
    return {"wall_s": wall, "step_ms": step_ms, "trials": trials, "kt": kt, "status": status,
            "segments": seg, "group": group_used, "evals": evals, "prof_trials": prof_trials}


KERNEL_SOURCE = {"trial_kernel": ["chain_impl.h", "coop.h", "blockmath.h"], "expect_kernel": ["expect.hip"]}


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/<kernel>_config1_counters.txt: FETCH_SIZE and WRITE_SIZE
    per launch, each scaled by the factor a 512 MiB copy kernel reads), or
    None when the summary is missing or was taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_config1_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for name in KERNEL_SOURCE[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2411_03416_amd", "csrc", name), "rb").read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def expect_plateau():
    """The expectation kernel at its batch plateau, from the committed counter
    summary (profiles/expect_kernel_batch_counters.txt, 8192 plans x 750
    factors): the busy fraction of the unit that binds it (the texture data
    unit returning the grid gathers) beside HBM and VALU issue; None when the
    summary is missing or was taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "expect_kernel_batch_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for name in KERNEL_SOURCE["expect_kernel"]:
        h.update(open(os.path.join(ROOT, "paper_2411_03416_amd", "csrc", name), "rb").read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    try:
        return {"kernel": "expect_lane_kernel<float,2,5,point2d>", "factors_per_launch": 6144000,
                "factors_per_s": float(kv["factors_per_s"]), "bound": "gather data path (texture data unit)",
                "frac": float(kv["td_busy_frac"]), "addresser_busy_frac": float(kv["ta_busy_frac"]),
                "hbm_frac": float(kv["hbm_GBs"]) * 1e9 / (HBM_PEAK_GBS * 1e9),
                "valu_issue_frac": float(kv["valu_issue_frac"]),
                "source": "profiles/expect_kernel_batch_counters.txt"}
    except (KeyError, ValueError):
        return None


def pct(xs, q):
    xs = sorted(xs)
    k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[k]


_CPU_SAMPLE = """
import sys, time
sys.path.insert(0, {root!r})
import workloads
from oracle import prior, prox
p = workloads.config1_problem(seed={seed}, N={N})
t0 = time.perf_counter()
pri = prior.build_prior(p)
st = prox.init_state(p, pri)
for _ in range({iters}):
    st, _, _ = prox.prox_iteration(p, pri, st)
print(time.perf_counter() - t0)
"""


_TABLE_CPU = """
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import workloads
from oracle import collision, gbp, prior, prox
p = workloads.{make}
p["quadrature"] = "sparse"
p["gh_points"] = {level}
pri = prior.build_prior(p)
out = {{}}
t0 = time.perf_counter()
st = prox.init_state(p, pri)
out["gbp_s"] = time.perf_counter() - t0
# every stride-th factor, scaled to all of them (the arm's take ~0.5 s each)
ci = np.asarray(p["coll_index"])
every = collision.collision_states(p)
sample = every[::{stride}]
t0 = time.perf_counter()
for i in sample:
    collision.factor_expectation(p, st["mu"][i][ci], st["Sig"][i][np.ix_(ci, ci)])
out["expect_s"] = (time.perf_counter() - t0) * len(every) / len(sample)
out["expect_sampled"] = int(len(sample))
if {iteration}:
    t0 = time.perf_counter()
    prox.prox_iteration(p, pri, st)
    out["iteration_s"] = time.perf_counter() - t0
print(json.dumps(out))
"""


def paper_tables(args, pg):
    """The shapes of the paper's efficiency tables (Sec. 7.1) on one MI355X,
    on synthetic maps and a synthetic 7-joint chain (the paper's maps and
    WAM model are not available), one trajectory per row:
      expected collision cost (Table cost_time_comparison): N = 750, Smolyak
        level 10 on the 2-D and 3-D point robots' positions, level 6 on the
        arm's 7 joints; GPU = one expectation launch (kernel time from HIP
        events), FP64 and mixed; CPU = the oracle's expectations of the same
        marginals, one thread (serial);
      marginal covariances (Table Inverse_comparison): precisions of
        dimension 5000 (n = 4, N = 1250), 4998 (n = 6, N = 833) and 4998
        (n = 14, N = 357), the GP prior's K^-1; GPU GBP = pgvimp_marginals
        with no outputs (chain kernel and plan bookkeeping, wall clock);
        brute force = the dense inverse of the same matrix: torch.linalg.inv
        (LU) and the Cholesky inverse on the GPU (FP64, hipSOLVER) and
        numpy.linalg.inv on the host (all threads), and the oracle's serial
        GBP;
      whole optimisation (Table total_cost_time_comparison): the expected
        cost rows' problems, prior build + initial marginals + `tables_iters`
        iterations (the paper does not print its count) with pgvimp_solve,
        FP64 and mixed; CPU = the oracle's time for one iteration, times the
        iteration count (a full serial run takes minutes per row); for the
        arm, whose oracle expectations take ~0.5 s per factor, the
        expectations of every 38th factor scaled to all, and the whole run
        bounded below by the expectations alone."""
    import numpy as np
    import torch
    import workloads
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")

    def cpu_leg(make, iteration, level=2, stride=1):
        if args.no_cpu:
            return None
        print(f"tables: oracle leg {make}", flush=True)
        r = subprocess.run([sys.executable, "-c", _TABLE_CPU.format(root=ROOT, make=make, iteration=iteration,
                                                                    level=level, stride=stride)],
                           capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            return {"error": r.stderr[-400:]}
        return json.loads(r.stdout.strip().splitlines()[-1])

    # (problem, Smolyak level, oracle sampling stride, oracle iteration timed)
    rows = {"point2d": ("config1_problem(seed=0, N=750)", 10, 1, True),
            "point3d": ("point3d_problem(0, N=750)", 10, 3, True),
            "arm": ("arm_problem(0, N=750)", 6, 38, False)}
    t1, t3 = {}, {}
    for name, (make, level, stride, whole) in rows.items():
        prob = eval("workloads." + make)
        prob.update(quadrature="sparse", gh_points=level, n_iters=args.tables_iters)
        print(f"tables: {name} level {level}", flush=True)
        r1 = {"N": prob["N"], "rule": f"Smolyak level {level}"}
        r3 = {"N": prob["N"], "iters": args.tables_iters}
        for pname, prec in (("mixed", pg.MIXED), ("fp64", pg.FP64)):
            ctx = pg.pgvimp_create([prob], precision=prec, use_graph=False)
            pg.pgvimp_expect_all(ctx, 2)
            pg.pgvimp_profile(ctx, True)
            pg.pgvimp_kernel_times(ctx, reset=True)
            pg.pgvimp_expect_all(ctx, 10)
            r1[pname + "_ms"] = pg.pgvimp_kernel_times(ctx, reset=True)["expect"][0]
            print(f"tables: {name} {pname} expectations {r1[pname + '_ms']:.3f} ms", flush=True)
            pg.pgvimp_profile(ctx, False)
            # one solve, kernels launched directly (a graph would be captured
            # for this single run); every kernel has run once already
            # (prior build and marginals at creation, expectations above)
            res = {}
            dt = _timed(lambda: res.update(pg.pgvimp_solve(ctx, args.tables_iters)), 1)
            r3[pname + "_s"] = dt
            r3[pname + "_status"] = res[0]["status"]
            r3[pname + "_E_coll"] = res[0]["E_coll"]
            print(f"tables: {name} {pname} solve {dt:.3f} s", flush=True)
            pg.pgvimp_destroy(ctx)
        cpu = cpu_leg(make, whole, level, stride)
        if cpu is not None and "error" not in cpu:
            r1["cpu_oracle_ms"] = 1e3 * cpu["expect_s"]
            r1["cpu_oracle_sample"] = f"{cpu['expect_sampled']} of {prob['N']} factors, scaled"
            if whole:
                r3["cpu_oracle_s_per_iteration"] = cpu["iteration_s"]
                r3["cpu_oracle_s_estimate"] = cpu["iteration_s"] * args.tables_iters
            else:
                # the expectations alone: a lower bound of the serial run
                r3["cpu_oracle_s_lower_bound"] = cpu["expect_s"] * args.tables_iters
        elif cpu is not None:
            r1["cpu_error"] = cpu["error"]
        t1[name], t3[name] = r1, r3
    t2 = {}
    for name, make in (("point2d", "config1_problem(seed=0, N=1250)"), ("point3d", "point3d_problem(0, N=833)"),
                       ("arm", "arm_problem(0, N=357)")):
        prob = eval("workloads." + make)
        print(f"tables: marginals {name}", flush=True)
        ctx = pg.pgvimp_create([prob], precision=pg.FP64, use_graph=False)
        lib = pg._abi.load()

        def gbp():
            pg._check(lib.pgvimp_marginals(ctx.handle, 0, None, None, None), ctx.handle)

        gbp()
        row = {"dim": prob["N"] * prob["n"], "n": prob["n"], "N": prob["N"], "gpu_gbp_ms": 1e3 * _timed(gbp, 20)}
        _, D, U = pg.pgvimp_get_state(ctx, 0)
        pg.pgvimp_destroy(ctx)
        n, N = prob["n"], prob["N"]
        L = np.zeros((N * n, N * n))
        for i in range(N):
            L[i * n:(i + 1) * n, i * n:(i + 1) * n] = D[i]
            if i < N - 1:
                L[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = U[i]
                L[(i + 1) * n:(i + 2) * n, i * n:(i + 1) * n] = U[i].T
        Lg = torch.from_numpy(L).cuda()
        # the default linear-algebra backend's triangular solves fail to get
        # their workspace at this size on this stack; hipSOLVER's do not
        torch.backends.cuda.preferred_linalg_library("cusolver")
        torch.linalg.inv(Lg)
        row["gpu_dense_inverse_ms"] = 1e3 * _timed(lambda: torch.linalg.inv(Lg), 5)
        torch.cholesky_inverse(torch.linalg.cholesky(Lg))
        row["gpu_dense_cholesky_inverse_ms"] = 1e3 * _timed(lambda: torch.cholesky_inverse(torch.linalg.cholesky(Lg)),
                                                            5)
        del Lg
        t0 = time.perf_counter()
        np.linalg.inv(L)
        row["cpu_dense_inverse_ms"] = 1e3 * (time.perf_counter() - t0)
        cpu = cpu_leg(make, False)
        if cpu is not None and "error" not in cpu:
            row["cpu_oracle_gbp_ms"] = 1e3 * cpu["gbp_s"]
        t2[name] = row
    out = {"metric": "paper-shape tables (Sec. 7.1)", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "one trajectory per row; Smolyak levels 10/10/6; N = 750; precisions of "
                                  "dimension 5000/4998/4998"},
           "expected_collision_cost": t1, "marginal_covariances": t2, "whole_optimisation": t3,
           "cpu_model": _cpu_model(), "nproc": os.cpu_count()}
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, iters_sample=20, max_cores=16):
    """The oracle as it stands on the same workload, timed on the host (it
    never touches the GPU): plans of the config-1 batch, each prior build +
    iters_sample iterations in a child process pinned to one BLAS/OpenMP
    thread.  First one plan on one core, then one plan per core on every
    host core at once (plan-parallel): factor expectations per second of
    the whole solve."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")

    def run(seeds):
        procs = [subprocess.Popen([sys.executable, "-c", _CPU_SAMPLE.format(root=ROOT, N=N, iters=iters_sample,
                                                                             seed=k)],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
                 for k in seeds]
        t0 = time.perf_counter()
        outs = [p.communicate(timeout=900) for p in procs]
        wall = time.perf_counter() - t0
        if any(p.returncode != 0 for p in procs):
            return None, next(o[1] for o, p in zip(outs, procs) if p.returncode != 0)[-500:]
        return wall, [float(o[0].strip().splitlines()[-1]) for o in outs]

    wall1, t1 = run([0])
    if wall1 is None:
        return {"value": None, "error": t1}
    cores = max(1, min(os.cpu_count() or 1, max_cores))
    wallc, tc = run(list(range(cores)))
    if wallc is None:
        return {"value": None, "error": tc}
    model = _cpu_model()
    return {"value": cores * N * iters_sample / wallc, "unit": "factor-expectations/s", "cores": cores,
            "kind": "oracle", "plans_per_s": cores / wallc, "cpu_model": model, "nproc": os.cpu_count(),
            "sample": f"{cores} of the {N}-state plans at once, one per core (plan-parallel), each prior build + "
                      f"{iters_sample} iterations, numpy/scipy FP64 one thread each: {wallc:.1f} s wall",
            "one_core": {"value": N * iters_sample / t1[0], "plans_per_s": 1.0 / t1[0], "cores": 1,
                         "sample": f"1 plan: {t1[0]:.1f} s"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(plans are independent and would shard by request, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import paper_2411_03416_amd as pg
    if args.calibrate_copy:
        import torch
        # a plain copy kernel of known traffic (512 MiB read, 512 MiB written):
        # a dtype-converting copy runs as a kernel, a same-dtype one may not
        src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty(512 << 20, dtype=torch.int8, device="cuda")
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.serve:
        serve(args, pg)
        return
    if args.expect_sweep:
        expect_sweep(args, pg)
        return
    if args.paper_tables:
        paper_tables(args, pg)
        return
    if args.configs_only:
        print(json.dumps({"metric": "plans/s of configs 0, 2 and 3", "n_gpus": 1, "data": "synthetic",
                          "configs": config_rates(pg)}), flush=True)
        return

    probs = make_batch(args.plans, args.N, args.iters)
    B, N, K = args.plans, args.N, args.iters
    n = probs[0]["n"]
    mixed = timed_solve(pg, probs, pg.MIXED, args.steps, args.warmup, K, args.segments, args.group,
                        trial_width=args.trial_width, trial_lookahead=args.trial_lookahead,
                        trial_slots=args.trial_slots)
    ms = 1e3 * mixed["wall_s"] / args.steps
    factors_per_step = B * N * K
    value = factors_per_step / (ms / 1e3)
    out = {
        "metric": METRIC, "value": value, "unit": "factor-expectations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32 quadrature + fp64", "data": "synthetic",
        "config": {"workload": f"point robot, {B} seeded maps 500x500 (40 discs/boxes), N={N}, GH p=5, "
                               f"{K} prox iterations per solve, one HIP graph per solve",
                   "plans": B, "N": N, "iters": K, "n": n, "segments": mixed["segments"],
                   "expect_group": mixed["group"]},
        "plans_per_s": B / (ms / 1e3),
        "latency_ms": {"p50": pct(mixed["step_ms"], 50), "p99": pct(mixed["step_ms"], 99)},
        "status_ok": all(s == 0 for s in mixed["status"]),
    }
    kt = mixed["kt"]
    if kt and kt["expect"][1] and kt["trial"][1]:
        # expectation kernel: 88 B per factor of HBM traffic that the method
        # must move (marginal mean 2 + covariance 3 doubles in; E, g (2),
        # H (3) doubles out)
        exp_ms = kt["expect"][0]
        exp_bytes = 88.0 * B * N
        exp_gbs = exp_bytes / (exp_ms * 1e-3) / 1e9
        # trial kernel, per (evaluated step size, state): the GBP sweep of the
        # trial precision reads D_i, U_i and writes Sigma_ii, Sigma_{i,i+1} with
        # messages (48 n^2 B) and the update + mean solve moves (6 n^2 + 4 n)
        # doubles: 1664 B for n = 4 (HBM bound at batch); FP64 ~18 n^3 flops
        # Units are the method's own trials (the step sizes that halving one
        # at a time would evaluate); the speculative step sizes of each
        # concurrent window are reported beside them as waste.
        trial_ms, trial_launches = kt["trial"]
        unit_bytes = 48.0 * n * n + 8.0 * (6 * n * n + 4 * n)
        units_per_launch = mixed["prof_trials"] * N / trial_launches
        evals_per_launch = mixed["evals"] * N / trial_launches
        bytes_per_launch = unit_bytes * units_per_launch
        trial_gbs = bytes_per_launch / (trial_ms * 1e-3) / 1e9
        totals = {k: v[0] * v[1] for k, v in kt.items() if isinstance(v, tuple)}
        tot = sum(totals.values())
        rtrial = {"kernel": "trial_kernel<4>", "bound": "hbm", "achieved": trial_gbs, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": trial_gbs / HBM_PEAK_GBS, "traffic": counter_traffic("trial_kernel"),
                  "avg_ms": trial_ms, "bytes_per_launch": bytes_per_launch, "unit_bytes": unit_bytes,
                  "units_per_launch": units_per_launch, "evaluated_per_launch": evals_per_launch,
                  "speculative_frac": 1.0 - units_per_launch / max(evals_per_launch, 1e-300),
                  "fp64_tflops": 18.0 * n ** 3 * units_per_launch / (trial_ms * 1e-3) / 1e12}
        rexp = {"kernel": "expect_kernel<float,2,5,point2d>", "bound": "hbm", "achieved": exp_gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": exp_gbs / HBM_PEAK_GBS,
                "traffic": counter_traffic("expect_kernel"), "avg_ms": exp_ms, "bytes_per_launch": exp_bytes,
                "note": "24k factors per launch: latency-bound; the batch sweep (--expect-sweep) gives the plateau",
                "plateau": expect_plateau()}
        dominant = max(totals, key=totals.get)
        out["roofline"] = rtrial if dominant == "trial" else rexp
        out["roofline_expect"] = rexp
        out["kernel_share"] = {k: v / tot for k, v in totals.items()}
        out["kernel_avg_ms"] = {k: v[0] for k, v in kt.items() if isinstance(v, tuple)}
        out["eager_ms_per_step"] = kt["eager_ms_per_step"]
    if not args.no_fp64:
        f64 = timed_solve(pg, probs, pg.FP64, max(2, args.steps // 2), 1, K, args.segments, args.group,
                          profile=False, trial_width=args.trial_width, trial_lookahead=args.trial_lookahead,
                          trial_slots=args.trial_slots)
        ms64 = 1e3 * f64["wall_s"] / max(2, args.steps // 2)
        out["fp64"] = {"value": factors_per_step / (ms64 / 1e3), "ms_per_step": ms64,
                       "plans_per_s": B / (ms64 / 1e3),
                       "latency_ms": {"p50": pct(f64["step_ms"], 50), "p99": pct(f64["step_ms"], 99)}}
        # serial FP64: the same plans solved one at a time
        ser = timed_solve(pg, probs[:1], pg.FP64, 3, 1, K, args.segments, args.group, profile=False)
        ser_ms = 1e3 * ser["wall_s"] / 3
        out["serial_fp64"] = {"plans_per_s": 1.0 / (ser_ms / 1e3), "ms_per_plan": ser_ms}
        if not args.no_configs:
            out["configs"] = config_rates(pg)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(N)
    print(json.dumps(out), flush=True)


def _timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def config_rates(pg):
    """Plans/s of the other configurations, mixed and plain FP64, one step =
    one solve of the batch (prior build, initial marginals, iterations):
      config 0: 32 point-robot plans, N = 50, GH p = 3, 20 iterations;
      config 2: 8 arm plans (n = 14), N = 100, GH p = 2 on 7 joints, 20 iterations;
      config 3: 64 quadrotor plans, N ~ U{100..300}, 10 rounds of statistical
                linearisation (Alg. 2) x 15 iterations."""
    import workloads
    out = {}
    for name, make, count, iters, steps in (("config0", workloads.config0_problem, 32, 20, 5),
                                             ("config2", workloads.config2_problem, 8, 20, 1)):
        probs = [make(seed=k) for k in range(count)]
        row = {"plans": count, "N": probs[0]["N"], "iters": iters}
        for pname, prec in (("mixed", pg.MIXED), ("fp64", pg.FP64)):
            ctx = pg.pgvimp_create(probs, precision=prec, use_graph=True)
            pg.pgvimp_solve(ctx, iters)
            dt = _timed(lambda: pg.pgvimp_solve(ctx, iters), steps)
            st = pg.pgvimp_solve(ctx, iters)
            pg.pgvimp_destroy(ctx)
            row[pname] = {"plans_per_s": count / dt, "ms_per_step": 1e3 * dt,
                          "factor_expectations_per_s": count * probs[0]["N"] * iters / dt,
                          "status_ok": all(v["status"] == 0 for v in st.values())}
        out[name] = row
    probs = [workloads.config3_problem(seed=k) for k in range(64)]
    row = {"plans": 64, "N_range": [min(p["N"] for p in probs), max(p["N"] for p in probs)],
           "rounds": probs[0]["n_rounds"], "iters_per_round": probs[0]["n_iters"]}
    for pname, prec in (("mixed", pg.MIXED), ("fp64", pg.FP64)):
        ctx = pg.pgvimp_create(probs, precision=prec, use_graph=True)
        failed = set()

        def solve():
            for r in range(probs[0]["n_rounds"]):
                if r == 0:
                    for k, p in enumerate(probs):
                        try:
                            pg.ipgvimp_begin(ctx, k, p)
                        except pg.PgvimpError:
                            # a linearised prior that is not positive definite
                            # ends this plan (its budget is spent); the others go on
                            failed.add(k)
                            pg.pgvimp_set_budget(ctx, k, 0)
                else:
                    # later rounds: every live plan in shared launches
                    live = [k for k in range(len(probs)) if k not in failed]
                    for k, code in zip(live, pg.ipgvimp_next_round_many(ctx, live, probs[0])):
                        if code != pg.OK:
                            failed.add(k)
                pg.pgvimp_prox_step(ctx, probs[0]["n_iters"])
        dt = _timed(solve, 1)
        pg.pgvimp_destroy(ctx)
        row[pname] = {"plans_per_s": 64 / dt, "ms_per_step": 1e3 * dt, "plans_ended_early": len(failed)}
    out["config3"] = row
    return out


if __name__ == "__main__":
    main()
