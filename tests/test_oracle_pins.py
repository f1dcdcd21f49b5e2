"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself:
closed forms, invariants, special cases that reduce to a textbook result, or
brute force on tiny inputs.
"""
import math
import os

import numpy as np
import pytest

import workloads
from oracle import collision, fk, gbp, gh, prior, prox, sdf, slr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# Gauss-Hermite rule (Sec. 4.3 steps 1-3)
# ----------------------------------------------------------------------------
def _golden_gh():
    rules = {}
    env = {"sqrt": math.sqrt}
    with open(os.path.join(GOLDEN, "gh_closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, x, w = [t.strip() for t in line.split("|")]
            rules.setdefault(int(p), []).append((eval(x, env), eval(w, env)))
    return rules


def test_gh_matches_closed_forms():
    for p, rows in _golden_gh().items():
        xi, w = gh.gh_rule(p)
        np.testing.assert_allclose(xi, [r[0] for r in rows], rtol=0, atol=1e-14)
        np.testing.assert_allclose(w, [r[1] for r in rows], rtol=1e-14, atol=0)


def test_gh_matches_library_rule_and_moments():
    from numpy.polynomial.hermite_e import hermegauss
    for p in range(1, 13):
        xi, w = gh.gh_rule(p)
        x2, w2 = hermegauss(p)
        np.testing.assert_allclose(xi, x2, atol=1e-12)
        np.testing.assert_allclose(w, w2 / math.sqrt(2 * math.pi), rtol=1e-11, atol=1e-300)
        assert abs(w.sum() - 1.0) < 1e-14
        for k in range(0, 2 * p):
            exact = 0.0 if k % 2 else float(np.prod(np.arange(k - 1, 0, -2)) if k else 1.0)
            scale = np.sum(np.abs(w * xi ** k))
            assert abs(np.sum(w * xi ** k) - exact) <= 1e-13 * max(1.0, scale)


def _gauss_moment_1d(mean, var, k):
    """E[y^k] for y ~ N(mean, var) by the binomial expansion."""
    s = 0.0
    for j in range(0, k + 1, 2):
        dfact = float(np.prod(np.arange(j - 1, 0, -2))) if j else 1.0
        s += math.comb(k, j) * mean ** (k - j) * var ** (j / 2) * dfact
    return s


@pytest.mark.parametrize("p,d", [(2, 2), (3, 2), (4, 3), (5, 2), (2, 7)])
def test_tensor_rule_exact_for_low_degree(p, d):
    rng = np.random.default_rng(p * 10 + d)
    m = rng.normal(size=d)
    Mx = rng.normal(size=(d, d))
    P = Mx @ Mx.T + 0.5 * np.eye(d)
    for _ in range(4):
        a = rng.normal(size=d)
        for k in range(0, 2 * p):
            val = gh.expect(lambda x: (x @ a) ** k, m, P, p)
            ref = _gauss_moment_1d(a @ m, a @ P @ a, k)
            assert abs(val - ref) <= 1e-10 * max(1.0, abs(ref)), (k, val, ref)
    # a mixed monomial of degree 2p-1 across two coordinates (Isserlis)
    if d >= 2 and p >= 2:
        val = gh.expect(lambda x: x[:, 0] * x[:, 1], m, P, p)
        assert abs(val - (P[0, 1] + m[0] * m[1])) < 1e-12


# ----------------------------------------------------------------------------
# Stein-form factor expectations (Sec. 4.1 eq. gradients_psid)
# ----------------------------------------------------------------------------
def _rand_spd(rng, d, scale=1.0):
    M = rng.normal(size=(d, d))
    return scale * (M @ M.T / d + 0.3 * np.eye(d))


@pytest.mark.parametrize("d", [2, 3, 7])
def test_stein_quadratic_is_exact(d):
    rng = np.random.default_rng(d)
    mu, S = rng.normal(size=d), _rand_spd(rng, d)
    c, W = rng.normal(size=d), _rand_spd(rng, d)
    cost = lambda x: 0.5 * np.einsum("ka,ab,kb->k", x - c, W, x - c)  # noqa: E731
    prob = {"gh_points": 3}
    E, g, H = collision.factor_expectation(prob, mu, S, p=3, cost=cost)
    assert abs(E - 0.5 * (np.trace(W @ S) + (mu - c) @ W @ (mu - c))) < 1e-11
    np.testing.assert_allclose(g, W @ (mu - c), atol=1e-11)
    np.testing.assert_allclose(H, W, atol=1e-10)
    # two points per axis are not enough for the degree-4 Hessian integrand
    _, _, H2 = collision.factor_expectation(prob, mu, S, p=2, cost=lambda x: cost(x) ** 2)
    _, _, H3 = collision.factor_expectation(prob, mu, S, p=5, cost=lambda x: cost(x) ** 2)
    assert np.abs(H2 - H3).max() > 1e-3


def test_affine_sdf_closed_form():
    prob = workloads.affine_sdf_problem()
    a, b = prob["affine"]
    w = prob["obs_weight"]
    kappa = prob["hinge_eps"] - b
    rng = np.random.default_rng(1)
    for _ in range(5):
        mu = rng.uniform(5.0, 25.0, size=2)
        S = _rand_spd(rng, 2, 0.05)
        E, g, H = collision.factor_expectation(prob, mu, S, p=3)
        r = kappa - a @ mu
        assert abs(E - w * (r * r + a @ S @ a)) < 1e-9 * abs(E)
        np.testing.assert_allclose(g, -2 * w * r * a, rtol=1e-10)
        # the Stein form subtracts E[psi] Sigma^-1 from a term of the same size:
        # rounding leaves an absolute error of order eps |E| ||Sigma^-1||
        tol = 64 * np.finfo(float).eps * abs(E) * np.linalg.norm(np.linalg.inv(S))
        np.testing.assert_allclose(H, 2 * w * np.outer(a, a), rtol=0, atol=tol)


def test_bilinear_field_quadrature_converges_exactly():
    # field c0 + c1 x + c2 y + c3 x y on a dyadic grid: bilinear interpolation
    # reproduces it, psi = w (K - f)^2 has degree 4: E, g exact for p >= 3,
    # the Hessian for p >= 4.
    g_, cell = 128, 0.125
    xs = cell * np.arange(g_)
    X, Y = np.meshgrid(xs, xs)
    c = (-3.0, 0.25, 0.5, -0.015625)
    grid = (c[0] + c[1] * X + c[2] * Y + c[3] * X * Y).astype(np.float32)
    assert np.array_equal(grid.astype(np.float64), c[0] + c[1] * X + c[2] * Y + c[3] * X * Y)
    prob = {"coll_kind": "point2d", "sdf": grid, "origin": np.zeros(3), "cell": cell,
            "hinge_eps": 100.0, "obs_weight": 1.0, "sphere_radius": np.zeros(1)}
    mu, S = np.array([7.3, 6.1]), np.array([[0.09, 0.02], [0.02, 0.05]])
    out = {p: collision.factor_expectation(prob, mu, S, p=p) for p in (3, 4, 5, 6)}
    for p in (4, 5, 6):
        assert abs(out[p][0] - out[3][0]) < 1e-12 * abs(out[3][0])
        np.testing.assert_allclose(out[p][1], out[3][1], rtol=1e-12)
    for p in (5, 6):
        np.testing.assert_allclose(out[p][2], out[4][2], rtol=1e-11, atol=1e-9)
    # bilinear interpolation itself is exact for the field
    pts = np.random.default_rng(0).uniform(1, 14, size=(50, 2))
    np.testing.assert_allclose(sdf.bilinear(grid, np.zeros(3), cell, pts),
                               c[0] + c[1] * pts[:, 0] + c[2] * pts[:, 1] + c[3] * pts[:, 0] * pts[:, 1],
                               rtol=1e-13, atol=1e-13)


def test_trilinear_reproduces_trilinear_field():
    g_, cell = 16, 0.25
    ax = cell * np.arange(g_)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    f = lambda x, y, z: 1.0 + 0.5 * x - 0.25 * y + 0.125 * z + 0.0625 * x * y * z - 0.5 * y * z  # noqa: E731
    grid = f(X, Y, Z).astype(np.float32)
    assert np.array_equal(grid.astype(np.float64), f(X, Y, Z))
    pts = np.random.default_rng(3).uniform(0.1, 3.6, size=(40, 3))
    np.testing.assert_allclose(sdf.trilinear(grid, np.zeros(3), cell, pts),
                               f(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=1e-12, atol=1e-12)
    # clamping holds the boundary value outside the grid
    v = sdf.trilinear(grid, np.zeros(3), cell, np.array([[-5.0, 1.0, 1.0]]))
    assert abs(v[0] - f(0.0, 1.0, 1.0)) < 1e-12


def test_sdf_matches_hand_interpolation():
    grid = np.array([[0.0, 1.0, 4.0], [2.0, 3.0, 5.0]], dtype=np.float32)  # [gy=2, gx=3]
    v = sdf.bilinear(grid, np.zeros(3), 0.5, np.array([[0.25, 0.25], [0.75, 0.0], [9.0, 9.0]]))
    assert abs(v[0] - 1.5) < 1e-15  # centre of cell (0,0): mean of 0,1,2,3
    assert abs(v[1] - 2.5) < 1e-15  # halfway between 1 and 4 on row 0
    assert abs(v[2] - 5.0) < 1e-15  # clamped to the far corner


# ----------------------------------------------------------------------------
# Prior (Sec. 2.2, Alg. 1)
# ----------------------------------------------------------------------------
def test_van_loan_matches_double_integrator_closed_form():
    for dof in (2, 3, 7):
        A, a, B = workloads.double_integrator(dof)
        Phi, abar, Q = prior.discretize(A, a, B, 0.8 * np.eye(dof), 0.1)
        Phi_c, Q_c = prior.lti_double_integrator_closed_form(dof, 0.8, 0.1)
        np.testing.assert_allclose(Phi, Phi_c, atol=1e-15)
        np.testing.assert_allclose(Q, Q_c, rtol=1e-13, atol=1e-17)
        assert np.all(abar == 0)


def test_van_loan_matches_quadrature_of_the_grammian():
    rng = np.random.default_rng(5)
    n, m, dt = 4, 2, 0.3
    A = rng.normal(size=(n, n))
    a = rng.normal(size=n)
    B = rng.normal(size=(n, m))
    Qc = _rand_spd(rng, m)
    Phi, abar, Q = prior.discretize(A, a, B, Qc, dt)
    # composite Simpson rule of the defining integrals, with e^{As} from eigh-free series
    import scipy.linalg
    s = np.linspace(0.0, dt, 2001)
    wts = np.ones_like(s)
    wts[1:-1:2], wts[2:-1:2] = 4, 2
    wts *= (s[1] - s[0]) / 3
    Qn = sum(wk * scipy.linalg.expm(A * sk) @ B @ Qc @ B.T @ scipy.linalg.expm(A * sk).T for sk, wk in zip(s, wts))
    an = sum(wk * scipy.linalg.expm(A * sk) @ a for sk, wk in zip(s, wts))
    np.testing.assert_allclose(Q, Qn, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(abar, an, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Phi, scipy.linalg.expm(A * dt), rtol=1e-13)


def test_prior_blocks_match_dense_factor_assembly():
    p = workloads.quadrotor_problem(3, N=9)
    rng = np.random.default_rng(0)
    p["ltv"] = True
    p["A"] = rng.normal(size=(8, 6, 6)) * 0.5
    p["a"] = rng.normal(size=(8, 6))
    # a full-rank noise input keeps every Grammian well conditioned
    p["m"] = 6
    p["Qc"] = _rand_spd(rng, 6)
    p["B"] = rng.normal(size=(8, 6, 6))
    pri = prior.build_prior(p)
    Kd, eta_d = prior.dense_prior_precision(p)
    # normwise: Q of a random drift is ill-conditioned, so single entries of
    # K^-1 cancel to far below its norm
    Kb = prior.dense_from_blocks(pri["D"], pri["U"])
    assert np.linalg.norm(Kb - Kd) < 1e-13 * np.linalg.norm(Kd)
    assert np.linalg.norm(pri["eta"].reshape(-1) - eta_d) < 1e-13 * np.linalg.norm(eta_d)
    mu_d = np.linalg.solve(Kd, eta_d)
    assert np.linalg.norm(pri["mu_bar"].reshape(-1) - mu_d) < 1e-6 * np.linalg.norm(mu_d)


def test_banded_solve_and_matvec():
    rng = np.random.default_rng(2)
    N, n = 7, 3
    D, U = _rand_chain(rng, N, n)
    x = rng.normal(size=(N, n))
    M = prior.dense_from_blocks(D, U)
    np.testing.assert_allclose(prior.block_matvec(D, U, x).reshape(-1), M @ x.reshape(-1), rtol=1e-13)
    np.testing.assert_allclose(prior.banded_solve(D, U, prior.block_matvec(D, U, x)), x, rtol=1e-10)


# ----------------------------------------------------------------------------
# GBP (Sec. 5.1)
# ----------------------------------------------------------------------------
def _rand_chain(rng, N, n):
    """Random SPD block-tridiagonal precision."""
    J = rng.normal(size=(N * n, N * n))
    M = np.zeros((N * n, N * n))
    for i in range(N):
        for j in range(max(0, i - 1), min(N, i + 2)):
            M[i * n:(i + 1) * n, j * n:(j + 1) * n] = J[i * n:(i + 1) * n, j * n:(j + 1) * n]
    M = M @ M.T + 0.5 * np.eye(N * n)  # pentadiagonal in blocks; keep the tridiagonal part
    D = np.array([M[i * n:(i + 1) * n, i * n:(i + 1) * n] for i in range(N)])
    U = np.array([M[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] for i in range(N - 1)])
    D = D + 2 * n * np.eye(n)[None]  # diagonal dominance keeps the band SPD
    return D, U


@pytest.mark.parametrize("N,n", [(1, 2), (2, 3), (5, 4), (8, 4), (6, 2)])
def test_gbp_equals_dense_inverse(N, n):
    rng = np.random.default_rng(N * 7 + n)
    D, U = _rand_chain(rng, N, n)
    Sig, Soff, ld = gbp.gbp_marginals(D, U)
    Sd, Sod, ldd, sign = gbp.dense_marginals(D, U)
    assert sign > 0
    np.testing.assert_allclose(Sig, Sd, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(Soff, Sod, rtol=1e-11, atol=1e-13)
    assert abs(ld - ldd) < 1e-11 * max(1, abs(ldd))


def test_gbp_prior_marginals_and_band_identity():
    p = workloads.config0_problem(0)
    pri = prior.build_prior(p)
    Sig, Soff, ld = gbp.gbp_marginals(pri["D"], pri["U"])
    Sd, Sod, ldd, _ = gbp.dense_marginals(pri["D"], pri["U"])
    scale = np.abs(Sd).max()
    assert np.abs(Sig - Sd).max() < 1e-9 * scale
    assert np.abs(Soff - Sod).max() < 1e-9 * scale
    assert abs(ld - ldd) < 1e-9 * abs(ldd)


def test_gbp_detects_indefinite():
    rng = np.random.default_rng(9)
    D, U = _rand_chain(rng, 5, 3)
    D[3] -= 100 * np.eye(3)
    with pytest.raises(gbp.NotPositiveDefinite) as e:
        gbp.gbp_marginals(D, U)
    assert e.value.index <= 3


# ----------------------------------------------------------------------------
# KL and prior factor costs
# ----------------------------------------------------------------------------
def test_kl_banded_matches_dense_and_is_zero_on_self():
    rng = np.random.default_rng(4)
    N, n = 5, 3
    D0, U0 = _rand_chain(rng, N, n)
    D1, U1 = _rand_chain(rng, N, n)
    mu0, mu1 = rng.normal(size=(N, n)), rng.normal(size=(N, n))
    S1, So1, ld1 = gbp.gbp_marginals(D1, U1)
    S0, So0, ld0 = gbp.gbp_marginals(D0, U0)
    kl = prox.kl_banded(mu1, S1, So1, ld1, mu0, D0, U0, ld0)
    ref = prox.kl_dense(mu1.reshape(-1), np.linalg.inv(prior.dense_from_blocks(D1, U1)),
                        mu0.reshape(-1), np.linalg.inv(prior.dense_from_blocks(D0, U0)))
    assert abs(kl - ref) < 1e-10 * abs(ref)
    assert abs(prox.kl_banded(mu0, S0, So0, ld0, mu0, D0, U0, ld0)) < 1e-10


def test_kl_step_equals_textbook_kl():
    p = workloads.config0_problem(3)
    p["N"] = 12
    pri = prior.build_prior(p)
    st = prox.init_state(p, pri)
    rng = np.random.default_rng(1)
    H = np.zeros((12, 4, 4))
    for i in range(12):
        Hi = _rand_spd(rng, 2, 50.0)
        H[i, :2, :2] = Hi
    g = rng.normal(size=(12, 4)) * 10
    for beta in (1.0, 0.25, 1e-3):
        Dn, Un, MD, MU, rhs = prox.trial(p, pri, st, g, H, beta)
        Sig, Soff, ld = gbp.gbp_marginals(Dn, Un)
        mu = prior.banded_solve(MD, MU, rhs)
        k1 = prox.kl_step(p, pri, st, H, beta, mu, Sig, Soff, ld)
        ref = prox.kl_dense(mu.reshape(-1), np.linalg.inv(prior.dense_from_blocks(Dn, Un)),
                            st["mu"].reshape(-1), np.linalg.inv(prior.dense_from_blocks(st["D"], st["U"])))
        assert abs(k1 - ref) < 1e-7 * max(1.0, abs(ref)), (beta, k1, ref)


def test_prior_costs_match_quadrature_over_pairwise_marginals():
    p = workloads.config0_problem(1)
    p["N"] = 6
    pri = prior.build_prior(p)
    rng = np.random.default_rng(0)
    D, U = _rand_chain(rng, 6, 4)
    Sig, Soff, _ = gbp.gbp_marginals(D, U)
    mu = rng.normal(size=(6, 4))
    costs = prox.prior_factor_costs(p, pri, mu, Sig, Soff)
    for i in range(5):
        m = np.concatenate([mu[i], mu[i + 1]])
        P = np.block([[Sig[i], Soff[i]], [Soff[i].T, Sig[i + 1]]])
        Phi, W, ab = pri["Phi"][i], pri["Qinv"][i], pri["abar"][i]

        def f(x):
            r = x[:, 4:] - x[:, :4] @ Phi.T - ab
            return 0.5 * np.einsum("ka,ab,kb->k", r, W, r)
        assert abs(gh.expect(f, m, P, 2) - costs[1 + i]) < 1e-9 * abs(costs[1 + i])
    Ws = np.linalg.inv(p["Sig_start"])
    ref0 = gh.expect(lambda x: 0.5 * np.einsum("ka,ab,kb->k", x - p["mu_start"], Ws, x - p["mu_start"]), mu[0], Sig[0], 2)
    assert abs(ref0 - costs[0]) < 1e-9 * abs(ref0)


# ----------------------------------------------------------------------------
# Proximal iteration (Theorem 1, Alg. 1)
# ----------------------------------------------------------------------------
def test_obstacle_free_iteration_follows_scalar_recursion():
    T, beta = 1.7, 0.6
    p = workloads.free_problem(n_dof=2, N=9, temperature=T, beta_max=beta)
    p["kl_bound"] = math.inf
    pri = prior.build_prior(p)
    N, n = p["N"], p["n"]
    rng = np.random.default_rng(0)
    mu0 = pri["mu_bar"] + rng.normal(size=(N, n))
    st = prox.init_state(p, pri, mu0)
    alpha, dev = 1.0, mu0 - pri["mu_bar"]
    for _ in range(12):
        st, stats, (E, g, H) = prox.prox_iteration(p, pri, st)
        assert stats["status"] == 0 and stats["beta"] == beta and np.all(E == 0)
        dev = alpha / (beta + alpha) * dev
        alpha = (beta + alpha) / (beta * T + 1.0)
        np.testing.assert_allclose(st["D"], alpha * pri["D"], rtol=1e-12)
        np.testing.assert_allclose(st["U"], alpha * pri["U"], rtol=1e-12)
        np.testing.assert_allclose(st["mu"] - pri["mu_bar"], dev, rtol=1e-7, atol=1e-9)
    # the limit is the closed-form posterior N(mu_bar, T K)
    for _ in range(60):
        st, _, _ = prox.prox_iteration(p, pri, st)
    np.testing.assert_allclose(st["D"], pri["D"] / T, rtol=1e-12)
    Kd, eta = prior.dense_prior_precision(p)
    np.testing.assert_allclose(st["mu"].reshape(-1), np.linalg.solve(Kd, eta), rtol=1e-8, atol=1e-8)


def test_quadratic_cost_fixed_point():
    T = 1.5
    p = workloads.affine_sdf_problem(N=8, temperature=T, beta_max=1.0)
    p["kl_bound"] = math.inf
    a, b = p["affine"]
    w, kappa = p["obs_weight"], p["hinge_eps"] - b
    pri = prior.build_prior(p)
    st = prior_state = prox.init_state(p, pri)  # noqa: F841
    for _ in range(150):
        st, stats, (E, g, H) = prox.prox_iteration(p, pri, st)
        assert stats["status"] == 0
    N, n = p["N"], p["n"]
    G = np.zeros((N, n, n))
    G[:, :2, :2] = 2 * w * np.outer(a, a)
    rhs = pri["eta"].copy()
    rhs[:, :2] += 2 * w * kappa * a
    np.testing.assert_allclose(st["D"], (pri["D"] + G) / T, rtol=1e-10, atol=1e-8)
    np.testing.assert_allclose(st["U"], pri["U"] / T, rtol=1e-10, atol=1e-8)
    mu_star = np.linalg.solve(prior.dense_from_blocks(pri["D"] + G, pri["U"]), rhs.reshape(-1))
    np.testing.assert_allclose(st["mu"].reshape(-1), mu_star, rtol=1e-9, atol=1e-9)
    # fixed-point residual of Theorem 1 at convergence
    E, g, H = collision.collision_expectations(p, st["mu"], st["Sig"])
    res_mu = prior.block_matvec(pri["D"], pri["U"], st["mu"] - pri["mu_bar"]) + g
    assert np.abs(res_mu).max() < 1e-6 * np.abs(g).max()


def test_step_size_rule_halves_until_positive_definite():
    p = workloads.config0_problem(0)
    p["kl_bound"] = math.inf
    pri = prior.build_prior(p)
    st = prox.init_state(p, pri)
    new, stats, (E, g, H) = prox.prox_iteration(p, pri, st)
    # every rejected trial must have been indefinite, the accepted one PD
    beta = p["beta_max"]
    for t in range(stats["trials"] - 1):
        Dn, Un, *_ = prox.trial(p, pri, st, g, H, beta)
        with pytest.raises(gbp.NotPositiveDefinite):
            gbp.gbp_marginals(Dn, Un)
        beta /= 2
    assert beta == stats["beta"]
    assert np.all(np.linalg.eigvalsh(prior.dense_from_blocks(new["D"], new["U"])) > 0)


def test_kl_bound_is_respected_and_state_unchanged_on_failure():
    p = workloads.config0_problem(2)
    pri = prior.build_prior(p)
    st = prox.init_state(p, pri)
    new, stats, _ = prox.prox_iteration(p, pri, st)
    assert stats["status"] == 0 and stats["kl"] <= p["kl_bound"]
    p2 = dict(p, max_bisect=1, kl_bound=1e-12)
    same, stats2, _ = prox.prox_iteration(p2, pri, st)
    assert stats2["status"] == -4 and same is st


# ----------------------------------------------------------------------------
# SLR (Sec. 6.2) and forward kinematics
# ----------------------------------------------------------------------------
def test_slr_recovers_affine_maps_exactly():
    rng = np.random.default_rng(3)
    A0, a0 = rng.normal(size=(6, 6)), rng.normal(size=6)
    xbar, S = rng.normal(size=6), _rand_spd(rng, 6, 0.2)
    for p in (2, 3):
        A, a = slr.slr(lambda x: x @ A0.T + a0, xbar, S, p)
        np.testing.assert_allclose(A, A0, atol=1e-11)
        np.testing.assert_allclose(a, a0, atol=1e-11)


def test_slr_quadrotor_matches_gaussian_closed_forms():
    params = {"gravity": 9.81}
    xbar = np.array([1.0, 2.0, 0.4, 0.7, -0.3, 0.2])
    s2 = np.array([0.1, 0.2, 0.05, 0.03, 0.04, 0.02])
    S = np.diag(s2)
    A, a = slr.slr(lambda x: slr.quadrotor_drift(x, params), xbar, S, 12)
    m, v = xbar[2], s2[2]
    Ec, Es = math.cos(m) * math.exp(-v / 2), math.sin(m) * math.exp(-v / 2)
    fbar = A @ xbar + a
    vx, vz, w, g = xbar[3], xbar[4], xbar[5], 9.81
    ref = np.array([vx * Ec - vz * Es, vx * Es + vz * Ec, w, vz * w - g * Es, -vx * w - g * Ec, 0.0])
    np.testing.assert_allclose(fbar, ref, atol=1e-12)
    # Stein: with independent coordinates A = E[Jacobian of f]
    np.testing.assert_allclose(A[0, 2], -vx * Es - vz * Ec, atol=1e-12)
    np.testing.assert_allclose(A[3, 2], -g * Ec, atol=1e-12)
    np.testing.assert_allclose(A[0, 3], Ec, atol=1e-12)
    np.testing.assert_allclose(A[3, 5], vz, atol=1e-12)
    # vanishing covariance gives the Jacobian
    A0, _ = slr.slr(lambda x: slr.quadrotor_drift(x, params), xbar, 1e-14 * np.eye(6), 3)
    J = np.zeros((6, 6))
    c, s = math.cos(m), math.sin(m)
    J[0, 2], J[0, 3], J[0, 4] = -vx * s - vz * c, c, -s
    J[3, 2], J[3, 4], J[3, 5] = -g * c, w, vz
    np.testing.assert_allclose(A0[[0, 3]], J[[0, 3]], atol=1e-6)


def test_fk_straight_chain_and_rotations():
    chain = workloads.arm_chain(workloads._rng(0))
    c = fk.sphere_centres(np.zeros(7), chain)
    L = chain["link_len"]
    cum = np.concatenate([[0.0], np.cumsum(L)])
    for s, (link, frac) in enumerate(zip(chain["sphere_link"], chain["sphere_frac"])):
        ref = np.array(chain["base"]) + np.array([0.0, 0.0, cum[link] + frac * L[link]])
        np.testing.assert_allclose(c[s], ref, atol=1e-15)
    for ax in range(3):
        R = fk.rot(ax, 0.7)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-15)
        assert abs(np.linalg.det(R) - 1) < 1e-15


def test_fk_matches_rodrigues_composition():
    chain = workloads.arm_chain(workloads._rng(1))
    q = np.random.default_rng(2).uniform(-1.5, 1.5, 7)

    def rodrigues(k, th):
        K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
    R, o, frames = np.eye(3), np.array(chain["base"], dtype=float), []
    for k in range(7):
        axis = np.eye(3)[int(chain["axes"][k])]
        R = R @ rodrigues(axis, q[k])
        frames.append((R.copy(), o.copy()))
        o = o + R[:, 2] * chain["link_len"][k]
    ref = [frames[l][1] + frames[l][0][:, 2] * f * chain["link_len"][l]
           for l, f in zip(chain["sphere_link"], chain["sphere_frac"])]
    np.testing.assert_allclose(fk.sphere_centres(q, chain), np.array(ref), atol=1e-14)
