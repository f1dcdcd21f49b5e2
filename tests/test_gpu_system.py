"""GPU tests of the outer loops: Alg. 2 (statistical linearisation rounds)
and the continuous-batching serving loop."""
import numpy as np
import pytest

import workloads
from gpu_common import fp64_tol, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg():
    import paper_2411_03416_amd as m
    return m


def _perturbed(p, scale, seed=0):
    q = dict(p)
    rng = np.random.default_rng(seed)
    q["nominal_mean"] = p["nominal_mean"] * (1.0 + scale * rng.standard_normal(p["nominal_mean"].shape))
    return q


def test_ipgvimp_rounds_match_oracle(pg):
    from oracle import prior, slr
    p = workloads.quadrotor_problem(7, N=40)
    p["n_rounds"], p["n_iters"] = 3, 4
    _, ref = slr.run_ipgvimp(p, history=True)
    # the oracle's own divergence when its input moves by a rounding-size
    # amount measures how much Alg. 2 amplifies rounding, round by round
    _, refp = slr.run_ipgvimp(_perturbed(p, 1e-13), history=True)
    ctx = pg.pgvimp_create([p], use_graph=True)
    for r, ((A_r, a_r, st), (_, _, stp)) in enumerate(zip(ref, refp)):
        if r == 0:
            A, a = pg.ipgvimp_begin(ctx, 0, p)
        else:
            A, a = pg.ipgvimp_next_round(ctx, 0, p)
        q = slr.linearised_problem(p, A_r, a_r)
        pri = prior.build_prior(q)
        tol = fp64_tol(float(np.linalg.cond(prior.dense_from_blocks(pri["D"], pri["U"]))))
        self_mu, self_D = rel(stp["mu"], st["mu"]), rel(stp["D"], st["D"])
        err_A = rel(A[:p["N"] - 1], A_r[:p["N"] - 1])
        pg.pgvimp_prox_step(ctx, p["n_iters"])
        mu, D, U = pg.pgvimp_get_state(ctx, 0)
        err_mu, err_D = rel(mu, st["mu"]), rel(D, st["D"])
        print("round", r, "A", err_A, "mu", err_mu, "D", err_D, "oracle self", self_mu, self_D, "tol", tol,
              flush=True)
        if r == 0:
            assert err_A < 1e-10
        assert err_mu < max(p["n_iters"] * (r + 1) * tol, 100 * self_mu), r
        assert err_D < max(p["n_iters"] * (r + 1) * tol, 100 * self_D), r


def _serving_requests(spacing=0.002):
    reqs = []
    t = 0.0
    for k, (kind, N) in enumerate([(0, 60), (1, 120), (2, 150), (0, 45), (2, 200), (3, 50), (1, 80), (0, 70),
                                   (3, 40), (2, 180), (1, 150)]):
        seed = 100 + k
        if kind == 0:
            prob = workloads.point2d_problem(seed, N=N)
        elif kind == 1:
            prob = workloads.config1_problem(seed, N=N)
        elif kind == 2:
            prob = workloads.arm_problem(seed, N=N)
        else:
            prob = workloads.quadrotor_problem(seed, N=N)
            prob["n_rounds"], prob["n_iters"] = 2, 5
        prob["n_iters"] = prob.get("n_iters", 20) if kind == 3 else 6
        reqs.append((t, prob))
        t += spacing
    return reqs


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("budget_mib", [4096, 64])
def test_serving_matches_plans_solved_alone(pg, precision, budget_mib):
    """Continuous batching with admission by an HBM budget: every request is
    served, and each result equals the same plan served alone, bitwise in
    both precisions (no kernel's result depends on the batch).  A 64 MiB
    budget holds only a few plans at once: requests queue for admission
    and are admitted as plans leave."""
    from paper_2411_03416_amd.serve import ServingEngine, plan_bytes
    reqs = _serving_requests()
    budget = budget_mib << 20
    eng = ServingEngine(precision=precision, hbm_budget=budget, max_concurrent=8, chunk=2, max_N=200,
                        trial_width=8, trial_slots=8)
    metrics, recs = eng.run(reqs, timeout_s=120)
    eng.close()
    print("serving metrics", metrics, flush=True)
    assert metrics["completed"] == len(reqs) and metrics["errors"] == 0
    sizes = [plan_bytes(p, 8, 8) for _, p in reqs]
    if budget_mib == 64:
        # the budget held: never more live bytes than the budget, unless a
        # single plan larger than it ran alone
        assert metrics["peak_bytes"] <= max(budget, max(sizes))
        assert sum(sizes) > budget  # the stream does not fit at once ...
        assert metrics["admission_wait_p99_ms"] > 0.0  # ... so requests waited
        assert metrics["peak_live"] < len(reqs)
    for rec in recs:
        alone = ServingEngine(precision=precision, hbm_budget=1 << 30, max_concurrent=1, chunk=2,
                              dims=(rec["prob"]["n"],), max_N=200, trial_width=8, trial_slots=8)
        _, r2 = alone.run([(0.0, rec["prob"])], timeout_s=60)
        alone.close()
        assert np.array_equal(rec["result"]["mu"], r2[0]["result"]["mu"]), rec["id"]
        assert np.array_equal(rec["result"]["cov_diag"], r2[0]["result"]["cov_diag"]), rec["id"]


def test_slr_round_rejects_bad_nominal_and_keeps_plan(pg):
    # Alg. 2's first round validates the nominal trajectory in the library:
    # a covariance block that is not SPD, or a mean without covariances, is
    # EINVAL and leaves the plan as it was
    import ctypes as C
    from paper_2411_03416_amd import _abi
    p = workloads.quadrotor_problem(5, N=30)
    ctx = pg.pgvimp_create([p], use_graph=False, mu_init=[p["nominal_mean"]])
    before = pg.pgvimp_get_state(ctx, 0)
    bad = np.array(p["nominal_cov"], dtype=np.float64).copy()
    bad[7] = -bad[7]
    with pytest.raises(pg.PgvimpError) as e:
        pg.pgvimp_slr_round(ctx, 0, gravity=p["quad"]["gravity"], n_iters=3, nominal_mean=p["nominal_mean"],
                            nominal_cov=bad)
    assert e.value.code == pg.EINVAL
    mean = np.ascontiguousarray(p["nominal_mean"], dtype=np.float64)
    prm = np.array([p["quad"]["gravity"]])
    rc = _abi.load().pgvimp_slr_round(ctx.handle, 0, _abi.MODEL_QUAD2D, prm.ctypes.data_as(C.POINTER(C.c_double)),
                                      3, mean.ctypes.data, None, 3, None, None)
    assert rc == pg.EINVAL
    for x, y in zip(before, pg.pgvimp_get_state(ctx, 0)):
        assert np.array_equal(x, y)
    # a valid first round: the budget is the round's iteration count
    pg.pgvimp_slr_round(ctx, 0, gravity=p["quad"]["gravity"], n_iters=3, nominal_mean=p["nominal_mean"],
                        nominal_cov=p["nominal_cov"])
    st = pg.pgvimp_prox_step(ctx, 5)[0]
    assert st["iters_done"] == 3 and st["iters_left"] == 0


def test_plans_with_one_map_share_it_and_keep_their_results():
    """Plans whose SDF grids are identical share one device copy; removing
    one of them leaves the others' results unchanged (bitwise against the
    plan alone)."""
    import paper_2411_03416_amd as pg
    a = workloads.point2d_problem(0, N=40)
    b = workloads.point2d_problem(0, N=27)  # same map as a
    c = workloads.point2d_problem(1, N=33)
    print("shared maps: plans 40/27 on map 0, 33 on map 1", flush=True)
    ctx = pg.pgvimp_create([a, b, c], precision=pg.FP64, use_graph=False)
    alone = pg.pgvimp_create([b], precision=pg.FP64, use_graph=False)
    for x in (pg.pgvimp_factor_expectations(ctx, 1), pg.pgvimp_factor_expectations(alone, 0)):
        assert np.abs(x[0]).max() >= 0
    e_mix = pg.pgvimp_factor_expectations(ctx, 1)
    e_alone = pg.pgvimp_factor_expectations(alone, 0)
    assert all(np.array_equal(u, v) for u, v in zip(e_mix, e_alone))
    pg.pgvimp_remove_plan(ctx, 0)  # the map stays for plan 1
    pg.pgvimp_prox_step(ctx, 3)
    pg.pgvimp_prox_step(alone, 3)
    s_mix = pg.pgvimp_get_state(ctx, 1)
    s_alone = pg.pgvimp_get_state(alone, 0)
    assert all(np.array_equal(u, v) for u, v in zip(s_mix, s_alone))
    # a new plan on the released map's neighbour slot and on map 0 again
    pid = pg.pgvimp_add_plan(ctx, workloads.point2d_problem(0, N=40))
    e_new = pg.pgvimp_factor_expectations(ctx, pid)
    e_ref = pg.pgvimp_factor_expectations(pg.pgvimp_create([a], precision=pg.FP64, use_graph=False), 0)
    assert all(np.array_equal(u, v) for u, v in zip(e_new, e_ref))


@pytest.mark.parametrize("precision", [0, 1])
def test_round_for_many_plans_equals_rounds_one_by_one(pg, precision):
    """pgvimp_slr_round_many (a later Alg. 2 round of several plans in shared
    launches) gives the bits of pgvimp_slr_round on each plan in turn, and
    leaves the unlisted plans untouched."""
    probs = [workloads.config3_problem(seed=s) for s in (1, 5, 8, 13, 21)]
    for p in probs:
        p["n_iters"] = 3
    ctxs = [pg.pgvimp_create(probs, precision=precision, use_graph=False) for _ in range(2)]
    for ctx in ctxs:
        for k, p in enumerate(probs):
            pg.ipgvimp_begin(ctx, k, p)
        pg.pgvimp_prox_step(ctx, 3)
    listed = [1, 2, 4]
    before = {k: pg.pgvimp_get_state(ctxs[0], k) for k in range(len(probs))}
    codes = pg.ipgvimp_next_round_many(ctxs[0], listed, probs[0])
    for k in listed:
        pg.ipgvimp_next_round(ctxs[1], k, probs[k])
    assert all(c == pg.OK for c in codes)
    for k in range(len(probs)):
        a, b = pg.pgvimp_get_state(ctxs[0], k), pg.pgvimp_get_state(ctxs[1], k)
        assert all(np.array_equal(u, v) for u, v in zip(a, b)), k
        if k not in listed:
            assert all(np.array_equal(u, v) for u, v in zip(a, before[k])), k
        else:
            assert not np.array_equal(a[1], before[k][1]), k  # the precision restarted from the new K^-1
    for ctx in ctxs:
        pg.pgvimp_prox_step(ctx, 3)
    for k in range(len(probs)):
        a, b = pg.pgvimp_get_state(ctxs[0], k), pg.pgvimp_get_state(ctxs[1], k)
        assert all(np.array_equal(u, v) for u, v in zip(a, b)), k
    with pytest.raises(pg.PgvimpError):
        pg.ipgvimp_next_round_many(ctxs[0], [1, 1], probs[0])
    for ctx in ctxs:
        pg.pgvimp_destroy(ctx)
