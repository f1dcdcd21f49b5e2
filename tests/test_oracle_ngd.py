"""Pins of the oracle's natural-gradient step (Sec. 3.1(d), eq. ngd_proximal).

The step is natural-gradient descent on the objective J(q) = E[psi] - T H(q)
of Sec. 2.2.  The first test builds it from its definition alone: the
Fisher information of the Gaussian family in natural parameters from
Isserlis' theorem (the covariance of the sufficient statistics), and the
gradient of J by central differences of the oracle's own cost breakdown
(pinned elsewhere by J(q) - J(q*) = T KL(q || q*)).  The others check what
the natural-gradient step must do on a Gaussian target, its agreement with
Theorem 1 to first order in the step size, and the fixed point the two rules
share.
"""
import numpy as np
import pytest

import workloads
from gpu_common import rand_chain
from oracle import gbp, prior, prox


def _surrogate(rng, N, n):
    """A quadratic stand-in for the collision cost, psi_c(x) = 1/2 x^T Hc x +
    g0^T x with Hc block diagonal (one block per state, as the collision
    factors are), so E[psi_c], its mean gradient g = Hc mu + g0 and
    H = 2 dE/dSigma = Hc are exact."""
    Hc = np.zeros((N, n, n))
    for i in range(N):
        A = rng.normal(size=(n, n))
        Hc[i] = A @ A.T + 0.5 * np.eye(n)
    g0 = rng.normal(size=(N, n))
    return Hc, g0


def _objective(prob, pri, Hc, g0, mu, Sigma):
    """J(q) = E[psi_prior] + E[psi_c] - T H(q) for a dense Gaussian (mu [N,n],
    Sigma dense), through the oracle's cost breakdown of the band."""
    N, n = mu.shape
    S = np.array([Sigma[i * n:(i + 1) * n, i * n:(i + 1) * n] for i in range(N)])
    So = np.array([Sigma[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] for i in range(N - 1)])
    st = {"mu": mu, "Sig": S, "Soff": So, "logdet": -np.linalg.slogdet(Sigma)[1]}
    c = prox.cost_breakdown(prob, pri, st)
    x = mu.ravel()
    Hd = np.zeros((N * n, N * n))
    for i in range(N):
        Hd[i * n:(i + 1) * n, i * n:(i + 1) * n] = Hc[i]
    e_c = 0.5 * np.trace(Hd @ Sigma) + 0.5 * x @ Hd @ x + g0.ravel() @ x
    return c["total"] + e_c


def _fisher_natural(mu, Sigma):
    """Fisher information of N(mu, Sigma) in the natural coordinates
    v = (theta1, theta2_ij for i <= j), log q = theta1^T x + x^T theta2 x - A:
    the covariance of the sufficient statistics (x_a; x_i^2; 2 x_i x_j, i < j)
    by Isserlis' theorem."""
    d = mu.size
    pairs = [(i, j) for i in range(d) for j in range(i, d)]
    m = d + len(pairs)
    G = np.zeros((m, m))
    G[:d, :d] = Sigma
    for b, (i, j) in enumerate(pairs):
        f = 1.0 if i == j else 2.0
        for a in range(d):
            G[a, d + b] = G[d + b, a] = f * (mu[i] * Sigma[a, j] + mu[j] * Sigma[a, i])
        for c, (k, l) in enumerate(pairs):
            f2 = f * (1.0 if k == l else 2.0)
            cov = (Sigma[i, k] * Sigma[j, l] + Sigma[i, l] * Sigma[j, k]
                   + mu[i] * mu[k] * Sigma[j, l] + mu[i] * mu[l] * Sigma[j, k]
                   + mu[j] * mu[k] * Sigma[i, l] + mu[j] * mu[l] * Sigma[i, k])
            G[d + b, d + c] = f2 * cov
    return G, pairs


@pytest.mark.parametrize("temperature,beta", [(1.0, 0.3), (0.7, 0.45)])
def test_ngd_step_is_the_fisher_preconditioned_gradient(temperature, beta):
    prob = workloads.free_problem(n_dof=2, N=2, temperature=temperature)
    prob["update"] = "ngd"
    pri = prior.build_prior(prob)
    N, n = prob["N"], prob["n"]
    rng = np.random.default_rng(11)
    Hc, g0 = _surrogate(rng, N, n)
    D, U = rand_chain(rng, N, n)
    mu = pri["mu_bar"] + 0.3 * rng.normal(size=(N, n))
    Lam = prior.dense_from_blocks(D, U)
    Sigma = np.linalg.inv(Lam)
    d = N * n
    G, pairs = _fisher_natural(mu.ravel(), Sigma)
    theta1 = Lam @ mu.ravel()
    theta2 = -0.5 * Lam
    v = np.concatenate([theta1, [theta2[i, j] for i, j in pairs]])

    def unpack(v):
        t2 = np.zeros((d, d))
        for b, (i, j) in enumerate(pairs):
            t2[i, j] = t2[j, i] = v[d + b]
        L = -2.0 * t2
        S = np.linalg.inv(L)
        return (S @ v[:d]).reshape(N, n), S, L

    def J(v):
        m, S, _ = unpack(v)
        return _objective(prob, pri, Hc, g0, m, S)

    grad = np.zeros_like(v)
    for k in range(v.size):
        h = 1e-5 * max(1.0, abs(v[k]))
        e = np.zeros_like(v)
        e[k] = h
        grad[k] = (J(v + e) - J(v - e)) / (2 * h)
    v1 = v - beta * np.linalg.solve(G, grad)
    mu_ref, _, Lam_ref = unpack(v1)

    S, So, ld = gbp.gbp_marginals(D, U)
    st = {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}
    g = np.einsum("iab,ib->ia", Hc, mu) + g0
    Dn, Un, MD, MU, rhs = prox.trial(prob, pri, st, g, Hc, beta)
    mu1 = prior.banded_solve(MD, MU, rhs)
    Lam1 = prior.dense_from_blocks(Dn, Un)
    assert np.abs(Lam1 - Lam_ref).max() < 1e-6 * np.abs(Lam_ref).max()
    assert np.abs(mu1 - mu_ref).max() < 1e-6 * max(1.0, np.abs(mu_ref).max())


@pytest.mark.parametrize("temperature", [1.0, 0.5, 2.0])
def test_ngd_step_of_size_one_over_t_reaches_the_gaussian_target(temperature):
    """Without obstacles psi is the GP prior's quadratic and the target is
    the tempered posterior N(mu_bar, T K); one natural-gradient step of size
    1 / T lands on it from any Gaussian."""
    prob = workloads.free_problem(n_dof=2, N=7, temperature=temperature)
    prob["update"] = "ngd"
    pri = prior.build_prior(prob)
    N, n = prob["N"], prob["n"]
    rng = np.random.default_rng(5)
    D, U = rand_chain(rng, N, n)
    mu = pri["mu_bar"] + rng.normal(size=(N, n))
    S, So, ld = gbp.gbp_marginals(D, U)
    st = {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}
    Dn, Un, MD, MU, rhs = prox.trial(prob, pri, st, np.zeros((N, n)), np.zeros((N, n, n)), 1.0 / temperature)
    mu1 = prior.banded_solve(MD, MU, rhs)
    Kinv = prior.dense_from_blocks(pri["D"], pri["U"])
    Lam1 = prior.dense_from_blocks(Dn, Un)
    assert np.abs(Lam1 - Kinv / temperature).max() < 1e-12 * np.abs(Kinv).max()
    assert np.abs(mu1 - pri["mu_bar"]).max() < 1e-9 * np.abs(pri["mu_bar"]).max()


def test_ngd_and_theorem_1_agree_to_first_order():
    """Both rules move q along the same direction for small steps: their
    difference shrinks like beta^2 (halving beta quarters it) while the step
    itself shrinks like beta.  Small means beta |K^-1| << 1: the start and
    goal factors make K^-1 of order 1e4."""
    prob = workloads.free_problem(n_dof=2, N=6, temperature=0.8)
    pri = prior.build_prior(prob)
    N, n = prob["N"], prob["n"]
    rng = np.random.default_rng(2)
    Hc, g0 = _surrogate(rng, N, n)
    D, U = rand_chain(rng, N, n)
    mu = pri["mu_bar"] + 0.5 * rng.normal(size=(N, n))
    S, So, ld = gbp.gbp_marginals(D, U)
    st = {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}
    g = np.einsum("iab,ib->ia", Hc, mu) + g0

    def both(beta):
        out = []
        for rule in ("prox", "ngd"):
            Dn, Un, MD, MU, rhs = prox.trial(dict(prob, update=rule), pri, st, g, Hc, beta)
            out.append((prior.dense_from_blocks(Dn, Un), prior.banded_solve(MD, MU, rhs)))
        return out

    diffs = []
    for beta in (4e-6, 2e-6, 1e-6):
        (L0, m0), (L1, m1) = both(beta)
        diffs.append((np.abs(L1 - L0).max(), np.abs(m1 - m0).max()))
        assert np.abs(m1 - m0).max() < 1e-4 * np.abs(m0 - mu).max()
    for a, b in zip(diffs, diffs[1:]):
        for x, y in zip(a, b):
            assert 3.5 < x / y < 4.5, diffs


def test_ngd_and_theorem_1_share_the_fixed_point():
    """For a quadratic cost the optimum q* has Lambda* = (K^-1 + Hc) / T and
    (K^-1 + Hc) mu* = eta - g0; both rules leave it in place at any step
    size."""
    prob = workloads.free_problem(n_dof=2, N=5, temperature=0.6)
    pri = prior.build_prior(prob)
    N, n = prob["N"], prob["n"]
    rng = np.random.default_rng(9)
    Hc, g0 = _surrogate(rng, N, n)
    D = (pri["D"] + Hc) / prob["temperature"]
    U = pri["U"] / prob["temperature"]
    mu = prior.banded_solve(pri["D"] + Hc, pri["U"], pri["eta"] - g0)
    S, So, ld = gbp.gbp_marginals(D, U)
    st = {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}
    g = np.einsum("iab,ib->ia", Hc, mu) + g0
    for rule in ("prox", "ngd"):
        for beta in (0.05, 0.7, 3.0):
            Dn, Un, MD, MU, rhs = prox.trial(dict(prob, update=rule), pri, st, g, Hc, beta)
            m1 = prior.banded_solve(MD, MU, rhs)
            assert np.abs(Dn - D).max() < 1e-12 * np.abs(D).max(), (rule, beta)
            assert np.abs(Un - U).max() < 1e-12 * np.abs(D).max(), (rule, beta)
            assert np.abs(m1 - mu).max() < 1e-10 * max(1.0, np.abs(mu).max()), (rule, beta)


@pytest.mark.parametrize("temperature,beta", [(1.0, 0.4), (1.0, 1.0), (0.5, 1.9), (2.0, 0.9), (0.8, 3.0)])
def test_ngd_step_kl_equals_the_dense_kl(temperature, beta):
    """The step rule's KL (rearranged with Lambda_k = (Lambda' - beta (K^-1 +
    H)) / (1 - beta T), plain near beta T = 1) against numpy's dense KL."""
    prob = dict(workloads.free_problem(n_dof=2, N=5, temperature=temperature), update="ngd")
    pri = prior.build_prior(prob)
    N, n = prob["N"], prob["n"]
    rng = np.random.default_rng(3)
    Hc, g0 = _surrogate(rng, N, n)
    D, U = rand_chain(rng, N, n)
    mu = pri["mu_bar"] + 0.2 * rng.normal(size=(N, n))
    S, So, ld = gbp.gbp_marginals(D, U)
    st = {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}
    g = np.einsum("iab,ib->ia", Hc, mu) + g0
    Dn, Un, MD, MU, rhs = prox.trial(prob, pri, st, g, Hc, beta)
    Lam1 = prior.dense_from_blocks(Dn, Un)
    assert np.linalg.eigvalsh(Lam1).min() > 0
    S1, So1, ld1 = gbp.gbp_marginals(Dn, Un)
    mu1 = prior.banded_solve(MD, MU, rhs)
    kl = prox.kl_step(prob, pri, st, Hc, beta, mu1, S1, So1, ld1)
    Sq = np.linalg.inv(Lam1)
    Sk = np.linalg.inv(prior.dense_from_blocks(D, U))
    dense = prox.kl_dense(mu1.ravel(), Sq, mu.ravel(), Sk)
    assert abs(kl - dense) < 1e-8 * max(1.0, abs(dense)), (kl, dense)


def test_unknown_update_rule_is_rejected():
    prob = workloads.free_problem(n_dof=2, N=5)
    pri = prior.build_prior(prob)
    st = prox.init_state(prob, pri, pri["mu_bar"] + 0.2)
    N, n = prob["N"], prob["n"]
    H = np.zeros((N, n, n))
    with pytest.raises(ValueError):
        prox.trial(dict(prob, update="sgd"), pri, st, np.zeros((N, n)), H, 0.4)
