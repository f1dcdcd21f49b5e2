"""Shared helpers for the GPU parity tests (inputs are seeded and synthetic;
expected values come from the oracle only)."""
import numpy as np


def rel(a, b):
    """Normwise relative difference ||a - b|| / ||b|| over a whole block family."""
    a = np.ravel(np.asarray(a, dtype=np.float64))
    b = np.ravel(np.asarray(b, dtype=np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rand_chain(rng, N, n, dominance=2.0):
    """Random SPD block-tridiagonal precision (D [N,n,n], U [N-1,n,n])."""
    D = np.zeros((N, n, n))
    U = np.zeros((max(N - 1, 0), n, n))
    for i in range(N):
        M = rng.normal(size=(n, n))
        D[i] = M @ M.T / n + (dominance + 1.0) * np.eye(n)
    for i in range(N - 1):
        U[i] = rng.normal(size=(n, n)) * 0.5
    # enforce block diagonal dominance: D_i - sum of neighbouring |U| norms > 0
    for i in range(N):
        s = 0.0
        if i > 0:
            s += np.linalg.norm(U[i - 1], 2)
        if i < N - 1:
            s += np.linalg.norm(U[i], 2)
        D[i] += s * np.eye(n)
    return D, U


def fp64_tol(kappa):
    """FP64 parity bound for quantities derived from a precision matrix with
    condition number kappa: 1e-10 where kappa * eps is small, otherwise a
    bound that grows with kappa * eps (both sides carry that much rounding)."""
    return max(1e-10, 64.0 * kappa * np.finfo(float).eps)
