"""KL-proximal iteration (Theorem 1 eq. mu_Sigma_update, Alg. 1, App. C).

State: mean mu [N,n] and precision Lambda as block-tridiagonal blocks
(D [N,n,n], U [N-1,n,n]), plus the GBP marginals of Lambda.

Update for a step size beta (Theorem 1, with the entropy temperature T of
the objective E[psi] - T H(q) carried through the same derivation; T = 1
gives the printed theorem):
    Lambda' = (beta (K^-1 + H) + Lambda_k) / (beta T + 1)
    (K^-1 + Lambda_k / beta) mu' = -g + K^-1 mu_bar + Lambda_k mu_k / beta
where g and H = 2 grad_Sigma psi_d are the collision-factor expectations
mapped back to the joint (eq. gradients_psid_factorize; each factor only
touches its own state's diagonal block).

Step size (Alg. 1, App. C): start at beta_max and halve until Lambda' is
positive definite and KL(q' || q_k) <= kl_bound, at most max_bisect trials;
if no trial passes the state is left unchanged.  The paper prints neither
the bound nor the bisection constants; halving from beta_max is the reading
used.  The KL is evaluated in the rearranged form of kl_step.

Natural-gradient variant (Sec. 3.1(d), eq. ngd_proximal; problem key
"update" = "ngd"): the proximal term is the symmetric KL, whose second-order
form is the Fisher metric, so the step is natural-gradient descent on
J(q) = E[psi] - T H(q).  Read in the natural parameters (Lambda mu,
-Lambda / 2), where the Fisher-preconditioned gradient is the gradient with
respect to the mean parameters (mu, Sigma + mu mu^T):
    Lambda' = Lambda_k + beta (K^-1 + H - T Lambda_k)
    Lambda' mu' = Lambda_k mu_k - beta [(K^-1 mu_k - eta + g) - (K^-1 + H - T Lambda_k) mu_k]
The step size follows the same halving rule (Lambda' positive definite and
KL(q' || q_k) <= kl_bound); see kl_step for how its KL is evaluated.

Initial state (not stated in the paper): mu_0 = mu_bar, Lambda_0 = K^-1.
"""
from __future__ import annotations

import math

import numpy as np

from . import collision, gbp, prior as prior_mod


def prior_factor_costs(prob, pri, mu, Sig, Soff):
    """Expected prior factor costs [N+1] = [start, transitions..., goal],
    each 1/2 E[r^T W r] in closed form: 1/2 (tr(W Cov r) + rbar^T W rbar)."""
    N = prob["N"]
    out = np.zeros(N + 1)
    Ws = np.linalg.inv(prob["Sig_start"])
    r = mu[0] - prob["mu_start"]
    out[0] = 0.5 * (np.trace(Ws @ Sig[0]) + r @ Ws @ r)
    for i in range(N - 1):
        Phi, W = pri["Phi"][i], pri["Qinv"][i]
        rb = mu[i + 1] - Phi @ mu[i] - pri["abar"][i]
        C = Sig[i + 1] - Soff[i].T @ Phi.T - Phi @ Soff[i] + Phi @ Sig[i] @ Phi.T
        out[1 + i] = 0.5 * (np.trace(W @ C) + rb @ W @ rb)
    Wg = np.linalg.inv(prob["Sig_goal"])
    r = mu[N - 1] - prob["mu_goal"]
    out[N] = 0.5 * (np.trace(Wg @ Sig[N - 1]) + r @ Wg @ r)
    return out


def kl_banded(mu1, Sig1, Soff1, logdet1, mu0, D0, U0, logdet0):
    """KL(N(mu1, Sigma1) || N(mu0, Lambda0^-1)) using only the band of
    Lambda0 and the marginal blocks of Sigma1:
    1/2 [tr(Lambda0 Sigma1) + d^T Lambda0 d - dim + log det Lambda1 - log det Lambda0]."""
    N, n = mu1.shape
    tr = np.einsum("iab,iba->", D0, Sig1)
    if N > 1:
        tr += 2.0 * np.einsum("iab,iab->", U0, Soff1)
    d = mu1 - mu0
    quad = np.sum(d * prior_mod.block_matvec(D0, U0, d))
    return 0.5 * (tr + quad - N * n + logdet1 - logdet0)


def kl_step(prob, pri, st, H, beta, mu1, Sig1, Soff1, logdet1):
    """KL(q_{k+1} || q_k) for the step of size beta, evaluated stably.

    Same quantity as kl_banded.  Because Lambda_k = (beta T + 1) Lambda' -
    beta (K^-1 + H) exactly and tr(Lambda' Sigma') = dim, the trace term is
    tr(Lambda_k Sigma') - dim = beta (T dim - tr((K^-1 + H) Sigma')); this
    avoids subtracting dim from a sum of terms many orders of magnitude
    larger (the precision of a long, loosely pinned trajectory has a
    condition number near 1e10, which leaves the textbook form with an
    absolute error of several nats).
    """
    N, n = mu1.shape
    T = prob["temperature"]
    scale = 1.0
    if update_rule(prob) == "ngd":
        # natural-gradient step: Lambda_k = (Lambda' - beta (K^-1 + H)) / (1 - beta T),
        # so the same trace term divided by 1 - beta T.  Near beta T = 1,
        # Lambda' hardly involves Lambda_k and the plain form is used.
        scale = 1.0 - beta * T
        if abs(scale) < 0.25:
            return kl_banded(mu1, Sig1, Soff1, logdet1, st["mu"], st["D"], st["U"], st["logdet"])
    trKH = np.einsum("iab,iba->", pri["D"] + H, Sig1)
    if N > 1:
        trKH += 2.0 * np.einsum("iab,iab->", pri["U"], Soff1)
    d = mu1 - st["mu"]
    quad = np.sum(d * prior_mod.block_matvec(st["D"], st["U"], d))
    return 0.5 * (beta * (T * N * n - trKH) / scale + quad + logdet1 - st["logdet"])


def kl_dense(mu1, S1, mu0, S0):
    """Textbook Gaussian KL(N(mu1,S1) || N(mu0,S0)) on dense matrices."""
    k = mu1.shape[0]
    S0inv = np.linalg.inv(S0)
    d = mu1 - mu0
    return 0.5 * (np.trace(S0inv @ S1) + d @ S0inv @ d - k
                  + np.linalg.slogdet(S0)[1] - np.linalg.slogdet(S1)[1])


def init_state(prob, pri, mu0=None):
    """mu_0 = mu_bar (or a given mean), Lambda_0 = K^-1, with its marginals."""
    mu = pri["mu_bar"].copy() if mu0 is None else np.array(mu0, dtype=np.float64)
    D, U = pri["D"].copy(), pri["U"].copy()
    Sig, Soff, logdet = gbp.gbp_marginals(D, U)
    return {"mu": mu, "D": D, "U": U, "Sig": Sig, "Soff": Soff, "logdet": logdet}


def update_rule(prob):
    """'prox' (Theorem 1, the default) or 'ngd' (Sec. 3.1(d))."""
    rule = prob.get("update", "prox")
    if rule not in ("prox", "ngd"):
        raise ValueError(f"unknown update rule {rule!r}")
    return rule


def trial_ngd(prob, pri, st, g, H, beta):
    """Precision and mean of the natural-gradient step for one step size
    (Sec. 3.1(d)); returns the same tuple as trial, the mean system being
    Lambda' mu' = rhs."""
    T = prob["temperature"]
    # dJ/dm2 = 1/2 (K^-1 + H) - T/2 Lambda_k, as blocks of 2 dJ/dm2
    GD = pri["D"] + H - T * st["D"]
    GU = pri["U"] - T * st["U"]
    # dJ/dm1 = dJ/dmu - 2 dJ/dm2 mu_k
    grad_mu = prior_mod.block_matvec(pri["D"], pri["U"], st["mu"]) - pri["eta"] + g
    grad_m1 = grad_mu - prior_mod.block_matvec(GD, GU, st["mu"])
    # natural parameters (Lambda mu, -Lambda / 2) step by -beta (dJ/dm1, dJ/dm2)
    Dn = st["D"] + beta * GD
    Un = st["U"] + beta * GU
    rhs = prior_mod.block_matvec(st["D"], st["U"], st["mu"]) - beta * grad_m1
    return Dn, Un, Dn, Un, rhs


def trial(prob, pri, st, g, H, beta):
    """Precision and mean of Theorem 1 for one step size (or of the
    natural-gradient step when the problem asks for it)."""
    if update_rule(prob) == "ngd":
        return trial_ngd(prob, pri, st, g, H, beta)
    T = prob["temperature"]
    Dn = (beta * (pri["D"] + H) + st["D"]) / (beta * T + 1.0)
    Un = (beta * pri["U"] + st["U"]) / (beta * T + 1.0)
    MD = pri["D"] + st["D"] / beta
    MU = pri["U"] + st["U"] / beta
    rhs = -g + pri["eta"] + prior_mod.block_matvec(st["D"], st["U"], st["mu"]) / beta
    return Dn, Un, MD, MU, rhs


def prox_iteration(prob, pri, st):
    """One iteration of Alg. 1: expectations, step-size selection, update.

    Returns (new_state, stats).  stats['status'] is 0 on success and -4 if
    no step size passed (state unchanged)."""
    E, g, H = collision.collision_expectations(prob, st["mu"], st["Sig"])
    costs = prior_factor_costs(prob, pri, st["mu"], st["Sig"], st["Soff"])
    beta = prob["beta_max"]
    bound = prob["kl_bound"]
    stats = {"E_coll": float(np.sum(E)), "E_prior": float(np.sum(costs)),
             "logdet": st["logdet"], "status": -4, "beta": 0.0, "kl": math.nan,
             "trials": 0}
    for t in range(int(prob["max_bisect"])):
        stats["trials"] = t + 1
        Dn, Un, MD, MU, rhs = trial(prob, pri, st, g, H, beta)
        try:
            Sig, Soff, logdet = gbp.gbp_marginals(Dn, Un)
        except gbp.NotPositiveDefinite:
            beta *= 0.5
            continue
        mu = prior_mod.banded_solve(MD, MU, rhs)
        kl = kl_step(prob, pri, st, H, beta, mu, Sig, Soff, logdet)
        if not (kl <= bound):
            beta *= 0.5
            continue
        stats.update(status=0, beta=beta, kl=float(kl))
        new = {"mu": mu, "D": Dn, "U": Un, "Sig": Sig, "Soff": Soff, "logdet": logdet}
        return new, stats, (E, g, H)
    return st, stats, (E, g, H)


def entropy(st):
    """Entropy of q: dim/2 (1 + log 2 pi) - 1/2 log det Lambda."""
    N, n = st["mu"].shape
    return 0.5 * N * n * (1.0 + math.log(2.0 * math.pi)) - 0.5 * st["logdet"]


def cost_breakdown(prob, pri, st):
    """The objective of Sec. 2.2, J(q) = E[psi] - T H(q), split as the paper's
    cost tables do: E_prior (sum of the prior factors' expected costs),
    E_coll (sum of the collision factors'), entropy_cost = -T H(q) and their
    sum total = J(q), at the state st (mean, precision, marginals)."""
    E, _, _ = collision.collision_expectations(prob, st["mu"], st["Sig"])
    e_prior = float(np.sum(prior_factor_costs(prob, pri, st["mu"], st["Sig"], st["Soff"])))
    e_coll = float(np.sum(E))
    ent = -prob["temperature"] * entropy(st)
    return {"E_prior": e_prior, "E_coll": e_coll, "entropy_cost": ent, "total": e_prior + e_coll + ent}


def run(prob, n_iters=None, pri=None, mu0=None, history=False):
    """Run the proximal iteration from the initial state; returns the final
    state (and the list of per-iteration states/stats when history=True)."""
    pri = prior_mod.build_prior(prob) if pri is None else pri
    st = init_state(prob, pri, mu0)
    n_iters = prob["n_iters"] if n_iters is None else n_iters
    hist = []
    for _ in range(n_iters):
        st, stats, _ = prox_iteration(prob, pri, st)
        if history:
            hist.append((st, stats))
    return (st, hist) if history else st
