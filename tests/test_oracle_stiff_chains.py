"""The oracle's chain marginals (Sec. 5.1, GBP) on the stiff priors of the
workloads, against the exact selected inverse computed at 50 significant
digits (block elimination in mpmath: the forward pivots P_i = D_i -
U_{i-1}^T P_{i-1}^-1 U_{i-1} and the backward recursion Sigma_i = P_i^-1 +
G_i Sigma_{i+1} G_i^T, G_i = P_i^-1 U_i, which are exact in exact
arithmetic).  The per-block relative errors bound what FP64 parity against
the oracle can show on these chains: about 1e-10 on the point-robot and arm
priors and 1e-8 on the quadrotor's linearised prior, whose input matrix has
rank 2 (the one-sided sweep that the GPU runs, done in numpy FP64, measures
1.3e-9 there)."""
import numpy as np
import pytest

import workloads
from oracle import gbp, prior, slr

mp = pytest.importorskip("mpmath")


def exact_marginals(D, U, digits=50):
    mp.mp.dps = digits
    N, n = D.shape[0], D.shape[1]
    Dm = [mp.matrix(D[i].tolist()) for i in range(N)]
    Um = [mp.matrix(U[i].tolist()) for i in range(N - 1)]
    Pinv, G = [None] * N, [None] * N
    P = Dm[0]
    for i in range(N):
        Pinv[i] = P ** -1
        if i + 1 < N:
            G[i] = Pinv[i] * Um[i]
            P = Dm[i + 1] - Um[i].T * G[i]
    S = [None] * N
    S[N - 1] = Pinv[N - 1]
    for i in range(N - 2, -1, -1):
        S[i] = Pinv[i] + G[i] * S[i + 1] * G[i].T
    return np.array([[[float(S[i][a, b]) for b in range(n)] for a in range(n)] for i in range(N)])


def worst_block_error(D, U):
    ref = exact_marginals(D, U)
    got = gbp.gbp_marginals(D, U)[0]
    return max(np.abs(got[i] - ref[i]).max() / np.abs(ref[i]).max() for i in range(len(ref)))


def test_point_robot_prior():
    pri = prior.build_prior(workloads.config1_problem(seed=0, N=200))
    assert worst_block_error(pri["D"], pri["U"]) < 2e-9


def test_arm_prior():
    pri = prior.build_prior(workloads.config2_problem(seed=0))
    assert worst_block_error(pri["D"], pri["U"]) < 1e-9


def test_quadrotor_linearised_prior():
    p = workloads.config3_problem(seed=0)
    drift = lambda x: slr.quadrotor_drift(x, p["quad"])  # noqa: E731
    A_t, a_t = slr.slr_trajectory(drift, np.array(p["nominal_mean"]), np.array(p["nominal_cov"]),
                                  p["slr_points"])
    pri = prior.build_prior(slr.linearised_problem(p, A_t, a_t))
    assert worst_block_error(pri["D"], pri["U"]) < 5e-8
