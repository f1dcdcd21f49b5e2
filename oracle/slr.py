"""Statistical linear regression and the i-P-GVIMP outer loop (Sec. 6, Alg. 2).

SLR (eqs. SLR_objective, SLR_best_ai, SLR_best_Ai) finds the affine model
y ~ A x + a minimising E||f(x) - A x - a||^2 under x ~ N(xbar, Sigbar):
    A = P_yx P_xx^-1,  a = E[f] - A E[x],
    P_yx = E[(f - E f)(x - E x)^T],  P_xx = E[(x - E x)(x - E x)^T],
with every expectation taken by the tensor Gauss-Hermite rule.

Reading of the paper: the regression is applied to the continuous drift of
the uncontrolled SDE (u = 0) at each support state's marginal, giving
(A_t, a_t) held constant on the interval that starts at that state; the
LTV prior is then rebuilt from them (Alg. 2 feeds Alg. 1).  After each
linearisation the precision restarts from the new K^-1 and the mean is
kept; the first round starts from the nominal trajectory.
"""
from __future__ import annotations

import numpy as np

from . import gh, prior as prior_mod, prox


def quadrotor_drift(x, params):
    """Drift of eq. planar_quad with u = 0; x [K, 6] = (x, z, phi, vx, vz, phidot)."""
    g = params["gravity"]
    phi, vx, vz, w = x[:, 2], x[:, 3], x[:, 4], x[:, 5]
    c, s = np.cos(phi), np.sin(phi)
    return np.stack([vx * c - vz * s, vx * s + vz * c, w,
                     vz * w - g * s, -vx * w - g * c, np.zeros_like(phi)], axis=1)


def slr(f, xbar, Sigbar, p):
    """(A, a) of the statistical linear regression of f about N(xbar, Sigbar)."""
    n = xbar.shape[0]
    L = np.linalg.cholesky(Sigbar)
    pts, wts = gh.tensor_rule(p, n)
    x = pts @ L.T + xbar[None, :]
    y = f(x)
    Ex = wts @ x
    Ey = wts @ y
    Pyx = np.einsum("k,ka,kb->ab", wts, y - Ey, x - Ex)
    Pxx = np.einsum("k,ka,kb->ab", wts, x - Ex, x - Ex)
    A = Pyx @ np.linalg.inv(Pxx)
    return A, Ey - A @ Ex


def slr_trajectory(f, mu, Sig_diag, p):
    """SLR at every support state: A [N,n,n], a [N,n]."""
    N, n = mu.shape
    A = np.zeros((N, n, n))
    a = np.zeros((N, n))
    for i in range(N):
        A[i], a[i] = slr(f, mu[i], Sig_diag[i], p)
    return A, a


def linearised_problem(prob, A_t, a_t):
    """LTV copy of prob with (A_i, a_i) = SLR at state i, i = 0..N-2."""
    q = dict(prob)
    N = prob["N"]
    q["ltv"] = True
    q["A"] = A_t[:N - 1].copy()
    q["a"] = a_t[:N - 1].copy()
    B = prob["B"] if np.ndim(prob["B"]) == 2 else prob["B"][0]
    q["B"] = np.repeat(np.asarray(B)[None], N - 1, axis=0)
    return q


def run_ipgvimp(prob, n_rounds=None, n_iters=None, history=False, drift=None):
    """Alg. 2: alternate SLR and P-GVIMP; returns the final state and the
    list of (A_t, a_t) per round (with history=True, (A_t, a_t, state after
    the round's iterations) per round).  drift (a callable on [K, n] points)
    replaces the quadrotor drift of the problem when given."""
    f = drift if drift is not None else (lambda x: quadrotor_drift(x, prob["quad"]))  # noqa: E731
    mu = np.array(prob["nominal_mean"], dtype=np.float64)
    Sig = np.array(prob["nominal_cov"], dtype=np.float64)
    n_rounds = prob["n_rounds"] if n_rounds is None else n_rounds
    n_iters = prob["n_iters"] if n_iters is None else n_iters
    rounds = []
    st = None
    for _ in range(n_rounds):
        A_t, a_t = slr_trajectory(f, mu, Sig, prob["slr_points"])
        q = linearised_problem(prob, A_t, a_t)
        pri = prior_mod.build_prior(q)
        st = prox.run(q, n_iters=n_iters, pri=pri, mu0=mu)
        rounds.append((A_t, a_t, st) if history else (A_t, a_t))
        mu, Sig = st["mu"], st["Sig"]
    return st, rounds
