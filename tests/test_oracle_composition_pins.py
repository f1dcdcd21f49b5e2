"""Pins of the oracle's composed costs and drivers against closed forms.

Each test fixes a value of an oracle function by mathematics that does not
re-use the oracle's own formula:
  * the 3-D point robot's expected hinge cost on an affine field (the cost is
    then an exact quadratic, Sec. 4.1 eq. gradients_psid has closed forms);
  * the arm's cost composition (forward kinematics -> trilinear lookup ->
    per-sphere hinge with its own radius -> sum over spheres) on an affine
    field, at the straight configuration and in expectation over a Gaussian
    on one joint, where trigonometric Gaussian moments give E[psi] exactly;
  * one and two rounds of Alg. 2 with a drift whose statistical linear
    regression (Sec. 6.2 eqs. SLR_best_ai, SLR_best_Ai) is known in closed
    form and differs from state to state, so the interval each regression is
    held on is checked;
  * the entropy of q against a library routine on the dense covariance.
"""
import math

import numpy as np
import pytest
import scipy.stats

import workloads
from gpu_common import rand_chain
from oracle import collision, gbp, prior, prox, slr


def _rand_spd(rng, d, scale):
    M = rng.normal(size=(d, d))
    return scale * (M @ M.T / d + 0.3 * np.eye(d))


# ----------------------------------------------------------------------------
# 3-D point robot on an affine field
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("p_gh", [3, 4])
def test_point3d_affine_field_closed_form(p_gh):
    prob = workloads.affine_sdf3_problem(gh_points=p_gh)
    a, b = prob["affine"]
    w = prob["obs_weight"]
    kappa = prob["hinge_eps"] - b
    rng = np.random.default_rng(11)
    for _ in range(4):
        mu = rng.uniform(2.5, 5.5, size=3)
        S = _rand_spd(rng, 3, 0.04)
        E, g, H = collision.factor_expectation(prob, mu, S)
        r = kappa - a @ mu
        E_ref = w * (r * r + a @ S @ a)
        assert abs(E - E_ref) < 1e-12 * E_ref
        # g = L^-T sum W psi xi sums terms of size E to a result of size |g|:
        # rounding leaves an absolute error of order eps E ||L^-1||
        Li = np.linalg.norm(np.linalg.inv(np.linalg.cholesky(S)), 2)
        np.testing.assert_allclose(g, -2.0 * w * r * a, rtol=0, atol=64 * np.finfo(float).eps * E * Li)
        tol = 64 * np.finfo(float).eps * abs(E) * np.linalg.norm(np.linalg.inv(S))
        np.testing.assert_allclose(H, 2.0 * w * np.outer(a, a), rtol=0, atol=tol)


def test_point3d_affine_field_through_the_trajectory_expectations():
    # the embedding into the 6-dim state: only the position block is set
    prob = workloads.affine_sdf3_problem(N=5)
    a, b = prob["affine"]
    w, kappa = prob["obs_weight"], prob["hinge_eps"] - b
    rng = np.random.default_rng(3)
    mu = rng.uniform(2.5, 5.5, size=(5, 6))
    Sig = np.array([_rand_spd(rng, 6, 0.03) for _ in range(5)])
    E, g, H = collision.collision_expectations(prob, mu, Sig)
    for i in range(5):
        r = kappa - a @ mu[i, :3]
        assert abs(E[i] - w * (r * r + a @ Sig[i, :3, :3] @ a)) < 1e-12 * E[i]
        np.testing.assert_allclose(g[i, :3], -2.0 * w * r * a, rtol=1e-11)
        assert np.all(g[i, 3:] == 0.0) and np.all(H[i, 3:, :] == 0.0) and np.all(H[i, :, 3:] == 0.0)


# ----------------------------------------------------------------------------
# Arm on an affine field
# ----------------------------------------------------------------------------
def _straight_chain_centres(chain):
    """Sphere centres at q = 0: every joint frame is the identity, so sphere
    s sits at the base plus the lengths of the links before its own plus its
    fraction of its own link, all along z."""
    lens = np.asarray(chain["link_len"])
    out = []
    for link, frac in zip(chain["sphere_link"], chain["sphere_frac"]):
        z = lens[:link].sum() + frac * lens[link]
        out.append(np.asarray(chain["base"]) + np.array([0.0, 0.0, z]))
    return np.array(out)


def test_arm_cost_at_straight_configuration():
    prob = workloads.arm_affine_problem()
    a, b = prob["affine"]
    w, eps = prob["obs_weight"], prob["hinge_eps"]
    r = np.asarray(prob["sphere_radius"])
    assert len(set(r.tolist())) == len(r), "radii must be distinct for this pin"
    c = _straight_chain_centres(prob["fk"])
    expected = w * np.sum((eps + r - (c @ a + b)) ** 2)
    got = collision.collision_cost(prob, np.zeros((1, 7)))[0]
    assert abs(got - expected) < 1e-13 * expected


def _trig_moments(m, v):
    """Gaussian moments of sin and cos for theta ~ N(m, v)."""
    e1, e2 = math.exp(-v / 2.0), math.exp(-2.0 * v)
    return {
        "s": math.sin(m) * e1, "c": math.cos(m) * e1,
        "ss": 0.5 * (1.0 - math.cos(2 * m) * e2), "cc": 0.5 * (1.0 + math.cos(2 * m) * e2),
        "sc": 0.5 * math.sin(2 * m) * e2,
    }


@pytest.mark.slow
def test_arm_expected_cost_one_joint_closed_form():
    # Only joint 1 (local y axis) varies: theta ~ N(m, s^2).  Spheres on link
    # 0 stay put; a sphere on link k >= 1 sits at o1 + z_s (sin t, 0, cos t),
    # o1 = base + (0, 0, l_0), z_s its distance along the chain from joint 1.
    # On the affine field h_s = alpha_s - z_s (a_x sin t + a_z cos t), so
    # E[h_s^2] follows from the Gaussian moments of sin and cos.  GH with 4
    # points is exact to degree 7; with s = 0.05 the rule's error on these
    # moments is below 1e-13 relative.
    prob = workloads.arm_affine_problem(gh_points=4)
    ch = prob["fk"]
    a, b = prob["affine"]
    w, eps = prob["obs_weight"], prob["hinge_eps"]
    r = np.asarray(prob["sphere_radius"])
    lens = np.asarray(ch["link_len"])
    m, s = 0.4, 0.05
    mu = np.zeros(7)
    mu[1] = m
    Sig = np.diag(np.full(7, 1e-30))
    Sig[1, 1] = s * s
    E, _, _ = collision.factor_expectation(prob, mu, Sig)
    mom = _trig_moments(m, s * s)
    o1 = np.asarray(ch["base"]) + np.array([0.0, 0.0, lens[0]])
    total = 0.0
    for k, (link, frac) in enumerate(zip(ch["sphere_link"], ch["sphere_frac"])):
        kappa = eps + r[k] - b
        if link == 0:
            c = np.asarray(ch["base"]) + np.array([0.0, 0.0, frac * lens[0]])
            total += (kappa - a @ c) ** 2
            continue
        z = lens[1:link].sum() + frac * lens[link]
        alpha = kappa - a @ o1
        ax, az = a[0], a[2]
        total += (alpha ** 2 - 2.0 * alpha * z * (ax * mom["s"] + az * mom["c"])
                  + z * z * (ax * ax * mom["ss"] + 2.0 * ax * az * mom["sc"] + az * az * mom["cc"]))
    expected = w * total
    assert abs(E - expected) < 1e-12 * expected, (E, expected)


# ----------------------------------------------------------------------------
# Alg. 2 with a drift whose regression is known in closed form
# ----------------------------------------------------------------------------
def _quadratic_drift_problem(N=12):
    p = workloads.free_problem(n_dof=2, N=N)
    n = p["n"]
    rng = np.random.default_rng(5)
    A0 = np.array(p["A"], dtype=np.float64) + 0.05 * rng.normal(size=(n, n))
    a0 = 0.1 * rng.normal(size=n)
    c, k = 0.03, 2

    def drift(x):
        return x @ A0.T + a0[None, :] + c * np.outer(x[:, 0] ** 2, np.eye(n)[k])

    def regression(m, S):
        # y = A0 x + a0 + c x_0^2 e_k under x ~ N(m, S):
        # Cov(x_0^2, x) = 2 m_0 S[0, :], so A = A0 + 2 c m_0 e_k e_0^T and
        # a = E[y] - A m = a0 + c (S_00 - m_0^2) e_k
        A = A0.copy()
        A[k, 0] += 2.0 * c * m[0]
        a = a0.copy()
        a[k] += c * (S[0, 0] - m[0] ** 2)
        return A, a

    t = np.linspace(0.0, 1.0, N)[:, None]
    p["nominal_mean"] = (1.0 - t) * p["mu_start"][None, :] + t * p["mu_goal"][None, :]
    p["nominal_cov"] = np.array([(0.01 + 0.002 * i) * np.eye(n) for i in range(N)])
    p["slr_points"] = 2
    p["n_iters"] = 3
    p["kl_bound"] = math.inf
    return p, drift, regression


def _ltv_from(p, A_t, a_t):
    q = dict(p)
    N = p["N"]
    q["ltv"] = True
    q["A"] = np.array(A_t[:N - 1])
    q["a"] = np.array(a_t[:N - 1])
    q["B"] = np.repeat(np.asarray(p["B"])[None], N - 1, axis=0)
    return q


def test_alg2_rounds_follow_closed_form_regression():
    p, drift, regression = _quadratic_drift_problem()
    N = p["N"]
    st, rounds = slr.run_ipgvimp(p, n_rounds=2, history=True, drift=drift)
    mu, Sig = p["nominal_mean"], p["nominal_cov"]
    for rnd, (A_t, a_t, st_r) in enumerate(rounds):
        ref = [regression(mu[i], Sig[i]) for i in range(N)]
        A_ref = np.array([x[0] for x in ref])
        a_ref = np.array([x[1] for x in ref])
        assert np.abs(A_t - A_ref).max() < 1e-12, rnd
        assert np.abs(a_t - a_ref).max() < 1e-12, rnd
        # the round runs P-GVIMP on the LTV model that holds state i's
        # regression on [t_i, t_{i+1}), from its mean, with the precision
        # restarted from that model's K^-1
        q = _ltv_from(p, A_ref, a_ref)
        pri = prior.build_prior(q)
        st_ref = prox.init_state(q, pri, mu)
        for _ in range(p["n_iters"]):
            st_ref, _, _ = prox.prox_iteration(q, pri, st_ref)
        scale = np.abs(st_ref["mu"]).max()
        assert np.abs(st_r["mu"] - st_ref["mu"]).max() < 1e-10 * scale, rnd
        assert np.abs(st_r["D"] - st_ref["D"]).max() < 1e-10 * np.abs(st_ref["D"]).max(), rnd
        mu, Sig = st_ref["mu"], st_ref["Sig"]
    assert st is rounds[-1][2]


def test_alg2_regression_varies_along_the_trajectory():
    # the pin above only checks the hold interval if the regressions differ
    p, _, regression = _quadratic_drift_problem()
    A = [regression(p["nominal_mean"][i], p["nominal_cov"][i])[0] for i in range(p["N"])]
    assert min(np.abs(A[i + 1] - A[i]).max() for i in range(p["N"] - 1)) > 1e-4


# ----------------------------------------------------------------------------
# Entropy of q
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N,n", [(1, 2), (5, 4), (9, 3)])
def test_entropy_matches_dense_gaussian(N, n):
    rng = np.random.default_rng(N * 10 + n)
    D, U = rand_chain(rng, N, n)
    _, _, logdet = gbp.gbp_marginals(D, U)
    st = {"mu": np.zeros((N, n)), "logdet": logdet}
    dense = prior.dense_from_blocks(D, U)
    ref = scipy.stats.multivariate_normal(mean=np.zeros(N * n), cov=np.linalg.inv(dense)).entropy()
    assert abs(prox.entropy(st) - ref) < 1e-11 * max(1.0, abs(ref))


# ----------------------------------------------------------------------------
# Cost breakdown of the objective (Sec. 2.2): J(q) = E[psi] - T H(q)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("temperature", [1.0, 3.5])
def test_objective_gap_is_temperature_times_kl_to_the_posterior(temperature):
    """Without obstacles psi is the GP prior's quadratic, whose tempered
    posterior is q* = N(mu_bar, T K); the objective then satisfies
    J(q) - J(q*) = T KL(q || q*) for every Gaussian q.  KL on the dense
    matrices (numpy slogdet and inverse) pins the prior costs, the entropy
    and the sign and scale of the entropy cost together."""
    prob = workloads.free_problem(n_dof=2, N=6, temperature=temperature)
    pri = prior.build_prior(prob)
    N, n = prob["N"], prob["n"]
    rng = np.random.default_rng(4)
    D, U = rand_chain(rng, N, n)
    mu = pri["mu_bar"] + rng.normal(size=(N, n))

    def state(mu, D, U):
        S, So, ld = gbp.gbp_marginals(D, U)
        return {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}

    q = state(mu, D, U)
    qs = state(pri["mu_bar"], pri["D"] / temperature, pri["U"] / temperature)
    cq, cs = prox.cost_breakdown(prob, pri, q), prox.cost_breakdown(prob, pri, qs)
    assert cq["E_coll"] == 0.0 and cs["E_coll"] == 0.0
    Lam = prior.dense_from_blocks(D, U)
    Kinv = prior.dense_from_blocks(pri["D"], pri["U"])
    Sq = np.linalg.inv(Lam)
    Ss = temperature * np.linalg.inv(Kinv)
    d = (mu - pri["mu_bar"]).ravel()
    kl = 0.5 * (np.trace(np.linalg.solve(Ss, Sq)) + d @ np.linalg.solve(Ss, d) - N * n
                + np.linalg.slogdet(Ss)[1] - np.linalg.slogdet(Sq)[1])
    assert abs((cq["total"] - cs["total"]) - temperature * kl) < 1e-9 * max(1.0, abs(temperature * kl))
    # the entropy cost is -T H(q) with H the Gaussian entropy
    H = scipy.stats.multivariate_normal(mean=np.zeros(N * n), cov=Sq).entropy()
    assert abs(cq["entropy_cost"] + temperature * H) < 1e-9 * abs(H)
