"""GPU tests of the outer loops: Alg. 2 (statistical linearisation rounds)
and the continuous-batching serving loop."""
import numpy as np
import pytest

import workloads
from gpu_common import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg():
    import paper_2411_03416_amd as m
    return m


def test_ipgvimp_rounds_match_oracle(pg):
    from oracle import slr
    p = workloads.quadrotor_problem(7, N=40)
    p["n_rounds"], p["n_iters"] = 3, 4
    ctx = pg.pgvimp_create([p], use_graph=True)
    pg.ipgvimp_begin(ctx, 0, p)
    pg.pgvimp_prox_step(ctx, p["n_iters"])
    for _ in range(p["n_rounds"] - 1):
        pg.ipgvimp_next_round(ctx, 0, p)
        pg.pgvimp_prox_step(ctx, p["n_iters"])
    mu, D, U = pg.pgvimp_get_state(ctx, 0)
    st, rounds = slr.run_ipgvimp(p)
    err_mu, err_D = rel(mu, st["mu"]), rel(D, st["D"])
    print("i-P-GVIMP gpu vs oracle: mu", err_mu, "D", err_D)
    # the Grammians of the quadrotor are ill-conditioned (cond ~1e9): allow
    # that much rounding growth over the rounds
    assert err_mu < 1e-5 and err_D < 1e-5


def test_serving_matches_plans_solved_alone(pg):
    from paper_2411_03416_amd.serve import ServingEngine
    reqs = []
    t = 0.0
    for k, (kind, N) in enumerate([(0, 60), (1, 120), (0, 45), (2, 30), (3, 50), (1, 80), (0, 70), (3, 40)]):
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
        t += 0.002
    eng = ServingEngine(precision=pg.FP64, hbm_budget=3 << 30, max_plans=8, chunk=2, max_N=200)
    metrics, recs = eng.run(reqs, timeout_s=120)
    eng.close()
    print("serving metrics", metrics)
    assert metrics["completed"] == len(reqs)
    # each result equals the same plan served alone (bitwise in FP64)
    for rec in recs:
        alone = ServingEngine(precision=pg.FP64, hbm_budget=1 << 30, max_plans=1, chunk=2,
                              dims=(rec["prob"]["n"],), max_N=200)
        _, r2 = alone.run([(0.0, rec["prob"])], timeout_s=60)
        alone.close()
        assert np.array_equal(rec["result"]["mu"], r2[0]["result"]["mu"]), rec["id"]
        assert np.array_equal(rec["result"]["cov_diag"], r2[0]["result"]["cov_diag"]), rec["id"]
