"""The Gauss-Hermite expectations of the hinge collision cost (Sec. 4.1 eq.
gradients_psid, Sec. 4.3) against Monte Carlo: the hinge is not smooth, so a
rule of p points per axis only approximates E[psi], grad_mu and 2 grad_Sigma;
at p = 30 the oracle's tensor rule must agree with a seeded 2-million-sample
estimate of the same three quantities (Stein form, sample covariance of the
integrands) within five standard errors, and the rule's own change from
p = 20 to p = 30 must be small against the values.  This pins the quadrature
of the non-smooth cost against the truth up to sampling error."""
import numpy as np

import workloads
from oracle import collision


def _near_obstacle(p):
    """A mean inside the hinge band (sdf between 0.05 and 0.15 m) of a
    seeded map, so the hinge is active on part of the Gaussian only."""
    grid = np.asarray(p["sdf"], dtype=np.float64)
    ys, xs = np.where((grid > 0.05) & (grid < 0.15))
    k = len(xs) // 2
    return np.array([xs[k] * p["cell"] + p["origin"][0], ys[k] * p["cell"] + p["origin"][1]])


def _monte_carlo(p, mu, Sig, M, seed):
    rng = np.random.default_rng(seed)
    L = np.linalg.cholesky(Sig)
    x = rng.standard_normal((M, 2)) @ L.T + mu
    psi = collision.collision_cost(p, x)
    dx = x - mu
    Si = np.linalg.inv(Sig)
    # per-sample integrands of E[psi], Sigma^-1 E[(x-mu) psi] and
    # Sigma^-1 E[(x-mu)(x-mu)^T psi] Sigma^-1 - E[psi] Sigma^-1
    f0 = psi
    f1 = (dx * psi[:, None]) @ Si.T
    y = dx @ Si.T  # Sigma^-1 (x - mu)
    f2 = (y[:, :, None] * y[:, None, :] * psi[:, None, None]).reshape(M, 4) - psi[:, None] * Si.reshape(1, 4)
    est = [f.mean(axis=0) for f in (f0, f1, f2)]
    se = [f.std(axis=0) / np.sqrt(M) for f in (f0, f1, f2)]
    return est, se


def test_hinge_expectations_match_monte_carlo():
    p = workloads.config0_problem(seed=0)
    mu = _near_obstacle(p)
    Sig = np.array([[0.09, 0.03], [0.03, 0.05]])
    E30, g30, H30 = collision.factor_expectation(p, mu, Sig, p=30)
    E20, g20, H20 = collision.factor_expectation(p, mu, Sig, p=20)
    (Em, gm, Hm), (sE, sg, sH) = _monte_carlo(p, mu, Sig, 2_000_000, seed=7)
    assert E30 > 100.0, "the hinge must be active"
    assert abs(E30 - Em) <= 5 * sE
    assert np.all(np.abs(g30 - gm) <= 5 * sg)
    assert np.all(np.abs(H30.ravel() - Hm) <= 5 * sH)
    # the rule itself has settled: p = 20 -> 30 moves the results by well
    # under a percent of their size
    assert abs(E30 - E20) <= 5e-3 * abs(E30)
    assert np.abs(g30 - g20).max() <= 5e-3 * np.abs(g30).max()
    assert np.abs(H30 - H20).max() <= 5e-3 * np.abs(H30).max()
