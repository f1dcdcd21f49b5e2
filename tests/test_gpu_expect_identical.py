"""Collision-factor expectations (Sec. 4.1 eq. gradients_psid, Sec. 4.3) on
identical inputs: the oracle integrates exactly the marginals N(mu_i,
Sigma_ii) that the GPU reads (the GPU's own mean and marginal covariances,
read back through the C ABI), so the comparison measures the expectation
kernel alone and not the conditioning of the marginals.

Per factor i the bound is relative to the size of the sums that the rule
forms (all weights are positive).  A node's cost psi = w h^2 carries an
absolute rounding error of about 2 w h u M, where M bounds the magnitudes
that enter h (the margin, the grid values and the coordinates) and u is the
unit roundoff; summed with the weights this is at most 2 u M sqrt(w E) by
Cauchy-Schwarz.  So with e_i = E_ref + M sqrt(w E_ref), |xi| <= xmax and
Linv = L_i^-1:
    |E - E_ref|        <= tol * e_i,
    |g - g_ref|_inf    <= tol * e_i * xmax * |Linv|,
    |H - H_ref|_inf    <= tol * e_i * (xmax^2 + 1) * |Linv|^2,
with tol = 1e-12 in FP64 mode (about 1e4 u).  Mixed mode (FP32 nodes, SDF
and cost, u = 6e-8) is held to 1e-5 per factor on the same scales and to
5e-5 normwise per plan (the Stein Hessian subtracts E[psi] I from a sum of
its own size).
"""
import numpy as np
import pytest

import workloads
from gpu_common import rel
from oracle import collision, gh

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMIX = 1e-5


@pytest.fixture(scope="module")
def pg():
    import paper_2411_03416_amd as m
    return m


def _factor_errors(p, mu, S, E, g, H):
    """Worst per-factor error ratios (error / bound at tol = 1) for E, g, H."""
    ci = np.asarray(p["coll_index"])
    d = ci.size
    xmax = float(np.abs(gh.gh_rule(p["gh_points"])[0]).max())
    grid = np.asarray(p["sdf"], dtype=np.float64)
    M = (np.abs(grid).max() + max(grid.shape) * p["cell"] + np.abs(p["origin"]).max()
         + p["hinge_eps"] + np.abs(p["sphere_radius"]).max())
    w = p["obs_weight"]
    Er, gr, Hr = collision.collision_expectations(p, mu, S)
    worst = np.zeros(3)
    for i in collision.collision_states(p):
        Sc = S[i][np.ix_(ci, ci)]
        Li = np.linalg.inv(np.linalg.cholesky(Sc))
        nl = np.abs(Li).sum(axis=1).max()  # |Linv|_inf
        e = max(Er[i] + M * np.sqrt(w * Er[i]), 1e-300)
        worst[0] = max(worst[0], abs(E[i] - Er[i]) / e)
        worst[1] = max(worst[1], np.abs(g[i][ci] - gr[i][ci]).max() / (e * xmax * nl))
        worst[2] = max(worst[2], np.abs(H[i][np.ix_(ci, ci)] - Hr[i][np.ix_(ci, ci)]).max()
                       / (e * (xmax ** 2 + 1) * nl ** 2))
    assert np.all(E[np.setdiff1d(np.arange(p["N"]), collision.collision_states(p))] == 0.0)
    return worst, (Er, gr, Hr)


def _check_plan(pg, ctx, plan, p, tol, label):
    mu, _, _ = pg.pgvimp_get_state(ctx, plan)
    S, _, _ = pg.pgvimp_marginals(ctx, plan)
    E, g, H, _ = pg.pgvimp_factor_expectations(ctx, plan)
    worst, (Er, gr, Hr) = _factor_errors(p, mu, S, E, g, H)
    norm = (rel(E, Er), rel(g, gr), rel(H, Hr))
    print(f"{label}: per-factor/bound {worst[0]:.2e} {worst[1]:.2e} {worst[2]:.2e}; "
          f"normwise {norm[0]:.2e} {norm[1]:.2e} {norm[2]:.2e}", flush=True)
    assert np.abs(Er).max() > 0, "the workload must activate hinge terms"
    assert worst.max() < tol, (label, worst)
    assert max(norm) < (tol if tol == TOL64 else 5 * tol), (label, norm)
    return worst, norm


@pytest.mark.parametrize("precision", [0, 1])
def test_config1_all_factors_identical_inputs(pg, precision):
    """All 32 x 750 factors of the benchmark workload, at the initial state
    and after three iterations, in the benchmark's launch configuration."""
    probs = [workloads.config1_problem(seed=k) for k in range(32)]
    print(f"config 1 identical inputs, precision {precision}", flush=True)
    ctx = pg.pgvimp_create(probs, precision=precision, use_graph=True)
    tol = TOL64 if precision == 0 else TOLMIX
    for stage in ("initial", "after 3 iterations"):
        if stage != "initial":
            pg.pgvimp_solve(ctx, 3)
        for k, p in enumerate(probs):
            _check_plan(pg, ctx, k, p, tol, f"plan {k} {stage}")
    pg.pgvimp_destroy(ctx)


# seeds whose straight-line initial state crosses obstacles (active hinges)
@pytest.mark.parametrize("p_gh", [1, 2, 3, 4, 5, 6, 7, 8, 10])
@pytest.mark.parametrize("precision", [0, 1])
def test_point2d_every_rule(pg, p_gh, precision):
    p = workloads.point2d_problem(2, N=37, gh_points=p_gh)
    ctx = pg.pgvimp_create([p], precision=precision, use_graph=False)
    _check_plan(pg, ctx, 0, p, TOL64 if precision == 0 else TOLMIX, f"point2d p={p_gh} prec={precision}")


@pytest.mark.parametrize("p_gh", [2, 3, 4, 5])
@pytest.mark.parametrize("precision", [0, 1])
def test_point3d_every_rule(pg, p_gh, precision):
    p = workloads.point3d_problem(2, N=29, gh_points=p_gh)
    ctx = pg.pgvimp_create([p], precision=precision, use_graph=False)
    _check_plan(pg, ctx, 0, p, TOL64 if precision == 0 else TOLMIX, f"point3d p={p_gh} prec={precision}")


@pytest.mark.parametrize("p_gh,N", [(2, 9), (3, 3)])
@pytest.mark.parametrize("precision", [0, 1])
def test_arm_every_rule(pg, p_gh, N, precision):
    p = workloads.arm_problem(0, N=N, gh_points=p_gh)
    ctx = pg.pgvimp_create([p], precision=precision, use_graph=False)
    _check_plan(pg, ctx, 0, p, TOL64 if precision == 0 else TOLMIX, f"arm p={p_gh} prec={precision}")


@pytest.mark.parametrize("precision", [0, 1])
def test_interior_only_and_grid_clamping(pg, precision):
    """coll_states = interior (the end states carry no collision factor) and
    nodes outside the map (the clamp holds the boundary value): the mean is
    moved so that the first states sit beyond the grid's corner."""
    p = workloads.point2d_problem(2, N=41, gh_points=4)
    p["coll_states"] = "interior"
    ctx = pg.pgvimp_create([p], precision=precision, use_graph=False)
    mu, D, U = pg.pgvimp_get_state(ctx, 0)
    mu = mu.copy()
    mu[:8, 0] -= 1.6  # x below the origin for the first states
    mu[:8, 1] -= 1.2
    mu[-5:, 0] += 2.5  # beyond the far edge (map is 10 m wide)
    pg.pgvimp_set_state(ctx, 0, mu, D, U)
    S, _, _ = pg.pgvimp_marginals(ctx, 0)
    assert mu[:8, :2].min() < -0.5 and mu[-5:, 0].max() > 10.5
    E, _, _, _ = pg.pgvimp_factor_expectations(ctx, 0)
    assert E[0] == 0.0 and E[-1] == 0.0
    _check_plan(pg, ctx, 0, p, TOL64 if precision == 0 else TOLMIX, f"interior+clamp prec={precision}")


def test_mixed_rule_of_one_point_is_not_centred(pg):
    """p = 1: the rule does not integrate xi xi^T, so the mixed-mode centring
    must be off; H = -E[psi] Sigma^-1 as in FP64."""
    p = workloads.point2d_problem(2, N=37, gh_points=1)
    ctx = pg.pgvimp_create([p], precision=1, use_graph=False)
    _, _, H, _ = pg.pgvimp_factor_expectations(ctx, 0)
    assert np.abs(H).max() > 0
    _check_plan(pg, ctx, 0, p, TOLMIX, "point2d p=1 mixed")


@pytest.mark.parametrize("kind,p_gh", [("point2d", 3), ("point2d", 5), ("point2d", 10), ("point3d", 3)])
@pytest.mark.parametrize("precision", [0, 1])
def test_workgroup_shapes_give_the_same_bits(pg, kind, p_gh, precision):
    """The launch shape is chosen per launch from the batch: one factor per
    thread (256 per workgroup) and the staged shapes (32-128 factors per
    workgroup) must give bitwise identical results, so a plan's result does
    not depend on the batch it runs in."""
    make = workloads.point2d_problem if kind == "point2d" else workloads.point3d_problem
    p = make(2, N=300, gh_points=p_gh)
    print(f"shapes {kind} p={p_gh} precision={precision}", flush=True)
    outs = []
    for group in (256, 128, 64, 32):
        ctx = pg.pgvimp_create([p], precision=precision, use_graph=False, expect_group=group)
        outs.append(pg.pgvimp_factor_expectations(ctx, 0))
        pg.pgvimp_destroy(ctx)
    assert np.abs(outs[0][0]).max() > 0
    for o in outs[1:]:
        assert all(np.array_equal(u, v) for u, v in zip(outs[0], o))


@pytest.mark.parametrize("p_gh,quad", [(2, "tensor"), (3, "tensor"), (3, "sparse")])
@pytest.mark.parametrize("precision", [0, 1])
def test_arm_workgroup_shapes_give_the_same_bits(pg, p_gh, quad, precision):
    """The arm's launch takes 8 factors per workgroup for small batches (the
    default) and 32 otherwise; both shapes must give bitwise identical
    results (several chunks of nodes per factor for the 3^7 rule)."""
    p = workloads.arm_problem(1, N=40, gh_points=p_gh)
    p["quadrature"] = quad
    print(f"arm shapes p={p_gh} {quad} precision={precision}", flush=True)
    outs = []
    for group in (0, 32):
        ctx = pg.pgvimp_create([p], precision=precision, use_graph=False, expect_group=group)
        outs.append(pg.pgvimp_factor_expectations(ctx, 0))
        pg.pgvimp_destroy(ctx)
    assert np.abs(outs[0][0]).max() > 0
    assert all(np.array_equal(u, v) for u, v in zip(outs[0], outs[1]))


def _sparse_factor_errors(p, mu, S, E, g, H, mixed):
    """_factor_errors for a sparse rule, whose weights can be negative: the
    sums are bounded by the rule with |W|, so E_ref becomes
    E_abs = sum |W| psi and the node term M sqrt(w E) becomes
    M sqrt(w sum|W| E_abs) (Cauchy-Schwarz with weights |W|).  In mixed mode
    the rule is rounded to FP32 and the centring by c = psi(mu) relies on
    sum W = 1 and sum W xi xi^T = I, which then hold to about u sum |W|;
    c sum |W| joins the scale.  sum |W| is 19 and 181 for level 10 in 2 and
    3 dimensions and 3653 for level 6 in 7: the FP32 sums of a high-level
    rule cancel that much, which the normwise errors printed here show."""
    ci = np.asarray(p["coll_index"])
    pts, wts = gh.rule("sparse", p["gh_points"], ci.size)
    wabs = np.abs(wts)
    xmax = max(float(np.abs(pts).max()), 1.0)  # level 1 is the single node xi = 0
    grid = np.asarray(p["sdf"], dtype=np.float64)
    M = (np.abs(grid).max() + max(grid.shape) * p["cell"] + np.abs(p["origin"]).max()
         + p["hinge_eps"] + np.abs(p["sphere_radius"]).max())
    w = p["obs_weight"]
    Er, gr, Hr = collision.collision_expectations(p, mu, S)
    worst = np.zeros(3)
    for i in collision.collision_states(p):
        Sc = S[i][np.ix_(ci, ci)]
        L = np.linalg.cholesky(Sc)
        Li = np.linalg.inv(L)
        nl = np.abs(Li).sum(axis=1).max()
        mc = mu[i][ci]
        Eabs = float(np.sum(wabs * collision.collision_cost(p, pts @ L.T + mc[None, :])))
        e = Eabs + M * np.sqrt(w * wabs.sum() * Eabs)
        if mixed:
            e += abs(float(collision.collision_cost(p, mc[None, :])[0])) * wabs.sum()
        e = max(e, 1e-300)
        worst[0] = max(worst[0], abs(E[i] - Er[i]) / e)
        worst[1] = max(worst[1], np.abs(g[i][ci] - gr[i][ci]).max() / (e * xmax * nl))
        worst[2] = max(worst[2], np.abs(H[i][np.ix_(ci, ci)] - Hr[i][np.ix_(ci, ci)]).max()
                       / (e * (xmax ** 2 + 1) * nl ** 2))
    return worst, (Er, gr, Hr)


# Smolyak levels of the paper's experiments (10 for the point robots, 6 for
# the arm) and low levels (k = 1: the single node xi = 0, no centring)
@pytest.mark.parametrize("kind,k,N", [("point2d", 1, 37), ("point2d", 3, 37), ("point2d", 10, 37),
                                      ("point3d", 2, 29), ("point3d", 10, 29), ("arm", 3, 5), ("arm", 6, 3)])
@pytest.mark.parametrize("precision", [0, 1])
def test_sparse_rules_identical_inputs(pg, kind, k, N, precision):
    """Sec. 4.3 Lemma 1: the expectations with the Smolyak rule built on the
    host (merged nodes, negative weights) against the oracle's own sparse
    rule on the marginals the GPU reads."""
    make = {"point2d": workloads.point2d_problem, "point3d": workloads.point3d_problem,
            "arm": workloads.arm_problem}[kind]
    p = make(2 if kind != "arm" else 0, N=N, gh_points=k)
    p["quadrature"] = "sparse"
    print(f"sparse {kind} k={k} precision={precision}", flush=True)
    ctx = pg.pgvimp_create([p], precision=precision, use_graph=False)
    mu, _, _ = pg.pgvimp_get_state(ctx, 0)
    S, _, _ = pg.pgvimp_marginals(ctx, 0)
    E, g, H, _ = pg.pgvimp_factor_expectations(ctx, 0)
    worst, (Er, gr, Hr) = _sparse_factor_errors(p, mu, S, E, g, H, precision == 1)
    norm = (rel(E, Er), rel(g, gr), rel(H, Hr))
    print(f"  per-factor/bound {worst[0]:.2e} {worst[1]:.2e} {worst[2]:.2e}; "
          f"normwise {norm[0]:.2e} {norm[1]:.2e} {norm[2]:.2e}", flush=True)
    assert np.abs(Er).max() > 0, "the workload must activate hinge terms"
    tol = TOL64 if precision == 0 else TOLMIX
    assert worst.max() < tol, worst
    pg.pgvimp_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_sparse_and_tensor_plans_in_one_batch(pg, precision):
    """Plans with tensor rules and sparse rules of two levels share one
    context and one solve; each plan's expectations equal those it gets
    alone (the launch filters plans by rule, and sparse plans of every
    level run in one launch)."""
    probs = []
    for k, quad in ((4, "tensor"), (10, "sparse"), (5, "sparse"), (10, "tensor")):
        p = workloads.point2d_problem(3, N=60, gh_points=k)
        p["quadrature"] = quad
        probs.append(p)
    ctx = pg.pgvimp_create(probs, precision=precision, use_graph=False)
    both = [pg.pgvimp_factor_expectations(ctx, k) for k in range(len(probs))]
    pg.pgvimp_solve(ctx, 2)
    after = [pg.pgvimp_get_state(ctx, k)[0] for k in range(len(probs))]
    pg.pgvimp_destroy(ctx)
    for k, p in enumerate(probs):
        c1 = pg.pgvimp_create([p], precision=precision, use_graph=False)
        alone = pg.pgvimp_factor_expectations(c1, 0)
        assert all(np.array_equal(u, v) for u, v in zip(both[k], alone)), k
        pg.pgvimp_solve(c1, 2)
        assert np.array_equal(pg.pgvimp_get_state(c1, 0)[0], after[k]), k
        pg.pgvimp_destroy(c1)
