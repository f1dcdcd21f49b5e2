"""Gaussian belief propagation on the chain (Sec. 5.1).

Only the covariance is wanted, so the zero-mean Gaussian
r(x) ~ exp(-1/2 x^T Lambda x) is used (eq. zero_mean_Gaussian).  Lambda is
split into unary factors with the diagonal blocks D_i and pairwise factors
carrying only the off-diagonal blocks U_i = Lambda_{i,i+1}.  All messages
are Gaussian, so a message is its precision matrix:

  variable -> pairwise factor (eq. messages, first line): the product of the
      other incoming messages, i.e. precision D_i + (message from the other
      side).
  pairwise factor -> variable (eq. messages, second line): marginalise the
      sending variable out of the pairwise potential times that variable's
      message; for potential [[0, U],[U^T, 0]] and incoming precision P this
      is the Schur complement -U^T P^{-1} U (forward) or -U R^{-1} U^T
      (backward).
  belief (eq. belief_lambda): Lambda_b_i = D_i + F_i + G_i, the sum of all
      incoming precisions; Sigma_ii = Lambda_b_i^{-1}.

The pairwise marginal covariance Sigma_{i,i+1} (not written in the paper,
needed by the pairwise prior factors and the KL trace) is read off the
belief of the pairwise factor, whose precision is
[[D_i + F_i, U_i], [U_i^T, D_{i+1} + G_{i+1}]].  On a chain GBP is exact.
The forward precisions P_i = D_i + F_i are the pivots of the block
Cholesky factorisation, so log det Lambda = sum_i log det P_i and Lambda is
positive definite iff every P_i is.
"""
from __future__ import annotations

import numpy as np


class NotPositiveDefinite(Exception):
    def __init__(self, index):
        super().__init__(f"precision not positive definite at state {index}")
        self.index = index


def _chol(M, i):
    try:
        return np.linalg.cholesky(M)
    except np.linalg.LinAlgError:
        raise NotPositiveDefinite(i) from None


def gbp_marginals(D, U):
    """Marginal covariances of N(0, Lambda^-1) with Lambda = blocks (D, U).

    Returns (Sig_diag [N,n,n], Sig_off [N-1,n,n], logdet Lambda).
    Raises NotPositiveDefinite if Lambda is not positive definite.
    """
    D = np.asarray(D, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    N, n = D.shape[0], D.shape[1]
    F = np.zeros((N, n, n))  # message from pairwise factor (i-1,i) into x_i
    G = np.zeros((N, n, n))  # message from pairwise factor (i,i+1) into x_i
    logdet = 0.0
    for i in range(N):
        P = D[i] + F[i]
        L = _chol(P, i)
        logdet += 2.0 * np.sum(np.log(np.diag(L)))
        if i + 1 < N:
            F[i + 1] = -U[i].T @ np.linalg.solve(P, U[i])
    for i in range(N - 1, 0, -1):
        R = D[i] + G[i]
        G[i - 1] = -U[i - 1] @ np.linalg.solve(R, U[i - 1].T)
    Sig = np.zeros((N, n, n))
    for i in range(N):
        Sig[i] = np.linalg.inv(D[i] + F[i] + G[i])
        Sig[i] = 0.5 * (Sig[i] + Sig[i].T)
    Soff = np.zeros((max(N - 1, 0), n, n))
    for i in range(N - 1):
        pair = np.block([[D[i] + F[i], U[i]], [U[i].T, D[i + 1] + G[i + 1]]])
        Soff[i] = np.linalg.inv(pair)[:n, n:]
    return Sig, Soff, logdet


def dense_marginals(D, U):
    """Brute-force reference: blocks of the dense inverse and dense log det."""
    from .prior import dense_from_blocks
    M = dense_from_blocks(D, U)
    S = np.linalg.inv(M)
    N, n = D.shape[0], D.shape[1]
    Sig = np.array([S[i * n:(i + 1) * n, i * n:(i + 1) * n] for i in range(N)])
    Soff = np.array([S[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] for i in range(N - 1)])
    sign, logdet = np.linalg.slogdet(M)
    return Sig, Soff.reshape(max(N - 1, 0), n, n), logdet, sign
