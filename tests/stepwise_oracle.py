"""Oracle side of the step-by-step parity tests (imported by worker
processes; no GPU).

One task = one proximal iteration (Alg. 1) of the oracle from a state that
the GPU produced: its mean and precision blocks and its own K^-1 (the
precision right after a prior build), so that the comparison measures one
step of each implementation and not the divergence of two long runs.  The
same step is also run from that input perturbed entry by entry by up to
2 n units of roundoff (relative 2 n 2^-53, random sign and size; n = the
state dimension, 2 n = the band width of the block-tridiagonal precision):
a backward-stable banded factorization or solve returns the exact result of
an input perturbed that much, so the change it causes is the floor of what
two FP64 implementations of the step can agree to.
"""
from __future__ import annotations

import functools

import numpy as np

import workloads
from oracle import collision, gbp, prior, prox, slr


@functools.lru_cache(maxsize=8)
def problem(kind, seed):
    """The configuration's problem; kind "<config>_ngd" takes the
    natural-gradient step (Sec. 3.1(d)) instead of Theorem 1's."""
    base, _, rule = kind.partition("_")
    p = {"config0": workloads.config0_problem, "config1": workloads.config1_problem,
         "config2": workloads.config2_problem, "config3": workloads.config3_problem}[base](seed=seed)
    if rule:
        p = dict(p, update=rule)
    return p


def _perturb(rng, x, n, sym=False):
    y = x * (1.0 + 2 * n * 2.0 ** -53 * rng.uniform(-1.0, 1.0, size=x.shape))
    if sym:
        y = 0.5 * (y + np.swapaxes(y, -1, -2))
    return y


def _step(p, pri, mu, D, U, at_trial=0):
    """One iteration of Alg. 1 with the oracle's own functions in the order of
    prox.prox_iteration, recording every trial's step size, positive
    definiteness and KL divergence up to the accepted one (so that a
    disputed decision can be examined).  With at_trial > 0 the update of
    that trial (1-based) is also returned as "forced" (whether or not the
    rule accepts it), and the trials run at least that far."""
    S, So, ld = gbp.gbp_marginals(D, U)
    st = {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So, "logdet": ld}
    _, g, H = collision.collision_expectations(p, mu, S)
    beta = p["beta_max"]
    out = {"mu": mu, "D": D, "U": U, "beta": 0.0, "trials": int(p["max_bisect"]), "status": -4, "trial_log": []}
    for t in range(int(p["max_bisect"])):
        Dn, Un, MD, MU, rhs = prox.trial(p, pri, st, g, H, beta)
        if t + 1 == at_trial:
            out["forced"] = {"mu": prior.banded_solve(MD, MU, rhs), "D": Dn, "U": Un}
        try:
            Sn, Son, ldn = gbp.gbp_marginals(Dn, Un)
        except gbp.NotPositiveDefinite:
            out["trial_log"].append((beta, False, float("nan")))
            beta *= 0.5
            continue
        mun = prior.banded_solve(MD, MU, rhs)
        kl = float(prox.kl_step(p, pri, st, H, beta, mun, Sn, Son, ldn))
        out["trial_log"].append((beta, True, kl))
        if kl <= p["kl_bound"] and out["status"] != 0:
            out.update(mu=mun, D=Dn, U=Un, beta=beta, trials=t + 1, status=0)
        if out["status"] == 0 and t + 1 >= at_trial:
            break
        beta *= 0.5
    return out


def one_step(task):
    """task: kind, seed, mu, D, U (the GPU's state k), KD, KU (the GPU's K^-1)
    and, for the quadrotor, A, a (the GPU's linearisation of the round).
    Returns the oracle's state k + 1 from that input and from the perturbed
    input."""
    p = problem(task["kind"], task["seed"])
    if "A" in task:
        p = slr.linearised_problem(p, task["A"], task["a"])
    if "temperature" in task:
        p = dict(p, temperature=task["temperature"])
    pri = dict(prior.build_prior(p))
    rng = np.random.default_rng(task.get("rng", 0))
    out = {}
    for name, pert in (("ref", False), ("pert", True)):
        mu, D, U, KD, KU = task["mu"], task["D"], task["U"], task["KD"], task["KU"]
        if pert:
            n = mu.shape[1]
            mu, D, U = _perturb(rng, mu, n), _perturb(rng, D, n, sym=True), _perturb(rng, U, n)
            KD, KU = _perturb(rng, KD, n, sym=True), _perturb(rng, KU, n)
        q = dict(pri)
        q["D"], q["U"] = KD, KU
        out[name] = _step(p, q, mu, D, U, task.get("gpu_trials", 0))
        # the cost breakdown of the input state (Sec. 2.2 objective)
        S, So, ld = gbp.gbp_marginals(D, U)
        out[name]["costs"] = prox.cost_breakdown(p, q, {"mu": mu, "D": D, "U": U, "Sig": S, "Soff": So,
                                                         "logdet": ld})
    return out


def slr_round(task):
    """The oracle's statistical linearisation (Sec. 6.2) about the GPU's
    marginals (mean mu, diagonal covariance blocks S) for the quadrotor, and
    the same from the marginals perturbed by 2 n roundoffs per entry (the
    floor: the regression divides by covariances whose condition number
    grows along the iteration)."""
    p = problem(task["kind"], task["seed"])
    f = lambda x: slr.quadrotor_drift(x, p["quad"])  # noqa: E731
    rng = np.random.default_rng(task.get("rng", 0))
    mu, S = np.asarray(task["mu"]), np.asarray(task["S"])
    n = mu.shape[1]
    ref = slr.slr_trajectory(f, mu, S, p["slr_points"])
    pert = slr.slr_trajectory(f, _perturb(rng, mu, n), _perturb(rng, S, n, sym=True), p["slr_points"])
    return ref, pert


def errors(gpu, ref, pert):
    """Normwise and worst-block relative differences of the GPU's step and
    of the perturbed oracle step (the floor), per block family."""
    out = {}
    for k in ("mu", "D", "U"):
        g, r, q = (np.asarray(x[k]) for x in (gpu, ref, pert))
        if r.size == 0:
            continue
        nr = max(np.linalg.norm(r), 1e-300)
        blk = lambda x: np.linalg.norm((x - r).reshape(r.shape[0], -1), axis=1) / np.maximum(  # noqa: E731
            np.linalg.norm(r.reshape(r.shape[0], -1), axis=1), 1e-300)
        out[k] = {"err": float(np.linalg.norm(g - r) / nr), "floor": float(np.linalg.norm(q - r) / nr),
                  "err_blk": float(blk(g).max()), "floor_blk": float(blk(q).max())}
    return out


def decision_tie(ref, pert, gpu_trials, bound, mixed):
    """Whether a GPU step-size decision that differs from the oracle's is a
    tie of the step rule, that is, not decided by the numbers: at the first
    trial where the two disagree the oracle's KL lies within the measured
    floor of the bound (ten times the change the perturbed input makes to
    it there, or ten times its largest relative change over the trials of
    the iteration times its value), or the perturbed input flips the oracle's own positive-definiteness
    there, or the disputed trial is the first positive definite one of the
    halving sequence, or a trial computed a negative KL (in the
    last two cases the trial precision is at the edge of positive
    definiteness and its marginals, log det and KL are not resolved in FP64).
    In mixed mode the FP32 rounding of the collision Hessians moves the trace
    term tr(H Sigma') (of order 1e5) by up to about one nat, so the margin
    there adds 10 % of the bound."""
    t = min(gpu_trials, ref["trials"]) - 1
    kls = [kl for run in (ref, pert) for _, pd, kl in run["trial_log"] if pd]
    if any(kl < -1e-9 * max(1.0, abs(bound)) for kl in kls):
        return True
    if t >= len(ref["trial_log"]):
        return False
    if t >= len(pert["trial_log"]):
        return True  # the perturbed input already decided differently
    _, pd_r, kl_r = ref["trial_log"][t]
    _, pd_p, kl_p = pert["trial_log"][t]
    if pd_r != pd_p:
        return True
    if not pd_r:
        return False
    if not any(pd for _, pd, _ in ref["trial_log"][:t]):
        return True  # first positive definite trial
    # the KL's resolution: its change under the perturbation at this trial,
    # or its largest relative change over the iteration's trials
    rel = max((abs(a[2] - b[2]) / max(abs(a[2]), 1e-300) for a, b in zip(ref["trial_log"], pert["trial_log"])
               if a[1] and b[1]), default=0.0)
    margin = 10.0 * max(abs(kl_r - kl_p), rel * abs(kl_r)) + (1e-1 if mixed else 1e-12) * abs(bound)
    return abs(kl_r - bound) <= margin
