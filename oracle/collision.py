"""Collision factors and their Gaussian expectations.

Collision cost (Sec. 4.1 eq. collision_factorization, Sec. 2.2): the cost
factorises over support states, psi(x) = sum_i psi_i(x_i), with
psi_i = ||h(x_i)||^2 weighted by a scalar.  The paper never writes h; the
readings used here are
  * h_s = max(0, eps + r_s - sdf(c_s(x))) per collision sphere s, with c_s
    the sphere centre (the point itself for a point robot, forward
    kinematics for the arm) and eps the hinge margin ("r + eps_sdf");
  * psi_i = w * sum_s h_s^2 with a scalar weight w (no factor 1/2, no dt);
  * every support state carries a collision factor.

Per-factor expectations (Sec. 4.1 eq. gradients_psid, restricted to the
factor's marginal by eq. mapping_from_joint_to_factor and Sec. 4.2):
    grad_mu   = Sigma^-1 E[(x - mu) psi]
    grad_Sigma = -1/2 Sigma^-1 E[psi] + 1/2 Sigma^-1 E[(x-mu)(x-mu)^T psi] Sigma^-1
with the expectations over N(mu_i, Sigma_i) taken by the tensor Gauss-Hermite
rule (Sec. 4.3).  The update of Theorem 1 uses 2 grad_Sigma, returned here
as "hess" (it equals E[Hessian of psi] by Stein's lemma).  The derivative-
free form is used because the hinge is not smooth.
"""
from __future__ import annotations

import numpy as np

from . import fk, gh, sdf


def collision_cost(prob, x):
    """psi at configuration points x [K, d] -> [K]."""
    kind = prob["coll_kind"]
    eps, w = prob["hinge_eps"], prob["obs_weight"]
    if kind in ("point2d", "point3d"):
        if kind == "point2d":
            dist = sdf.bilinear(prob["sdf"], prob["origin"], prob["cell"], x[:, :2])
        else:
            dist = sdf.trilinear(prob["sdf"], prob["origin"], prob["cell"], x[:, :3])
        h = np.maximum(0.0, eps + prob["sphere_radius"][0] - dist)
        return w * h * h
    if kind == "arm3d":
        c = fk.sphere_centres(x, prob["fk"])  # [K, S, 3]
        dist = sdf.trilinear(prob["sdf"], prob["origin"], prob["cell"], c)
        h = np.maximum(0.0, eps + prob["sphere_radius"][None, :] - dist)
        return w * np.sum(h * h, axis=1)
    if kind == "none":
        return np.zeros(x.shape[0])
    raise ValueError(kind)


def factor_expectation(prob, mu_c, Sig_c, p=None, cost=None):
    """E[psi], grad_mu and 2 grad_Sigma for one factor marginal N(mu_c, Sig_c).

    cost, if given, replaces the collision cost (a callable on [K, d] points).
    """
    p = prob["gh_points"] if p is None else p
    mu_c = np.asarray(mu_c, dtype=np.float64)
    d = mu_c.shape[0]
    L = np.linalg.cholesky(Sig_c)
    pts, wts = gh.rule(prob.get("quadrature", "tensor"), p, d)
    x = pts @ L.T + mu_c[None, :]
    psi = collision_cost(prob, x) if cost is None else cost(x)
    dx = x - mu_c[None, :]
    E0 = np.sum(wts * psi)
    E1 = np.einsum("k,k,ka->a", wts, psi, dx)
    E2 = np.einsum("k,k,ka,kb->ab", wts, psi, dx, dx)
    Sinv = np.linalg.inv(Sig_c)
    grad = Sinv @ E1
    grad_Sigma = -0.5 * Sinv * E0 + 0.5 * Sinv @ E2 @ Sinv
    return E0, grad, 2.0 * grad_Sigma


def collision_states(prob):
    """Indices of the support states that carry a collision factor."""
    if prob.get("coll_states", "all") == "interior":
        return np.arange(1, prob["N"] - 1)
    return np.arange(prob["N"])


def collision_expectations(prob, mu, Sig_diag, p=None):
    """Per-state E [N], gradient [N,n] and 2 grad_Sigma [N,n,n], embedded
    into the full state (zeros outside the configuration coordinates)."""
    N, n = prob["N"], prob["n"]
    ci = np.asarray(prob["coll_index"])
    E = np.zeros(N)
    g = np.zeros((N, n))
    H = np.zeros((N, n, n))
    if prob["coll_kind"] == "none":
        return E, g, H
    for i in collision_states(prob):
        e, gi, Hi = factor_expectation(prob, mu[i][ci], Sig_diag[i][np.ix_(ci, ci)], p)
        E[i] = e
        g[i][ci] = gi
        H[i][np.ix_(ci, ci)] = Hi
    return E, g, H
