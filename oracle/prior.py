"""GP prior of the linear(ised) SDE (Sec. 2.2 eq. dynamics_linear, Alg. 1).

The prior process dX = (A_t X + a_t) dt + B_t dW, discretised on support
states t_0..t_{N-1} (N states, N-1 intervals of length dt; A_t, a_t, B_t
held constant on each interval), gives per interval
    x_{i+1} = Phi_i x_i + abar_i + w_i,   w_i ~ N(0, Q_i),
with Phi_i = e^{A dt}, abar_i = int_0^dt e^{A s} ds a and the Grammian
Q_i = int_0^dt e^{A s} B Qc B^T e^{A^T s} ds.  Phi and abar come from the
exponential of [[A, a], [0, 0]] dt; Q from Van Loan's block exponential of
[[-A, B Qc B^T], [0, A^T]] dt (Van Loan 1978), both evaluated with
scipy's matrix exponential.

The path prior N(mu_bar, K) has a block-tridiagonal precision K^-1 that is
the sum of the start factor N(x_0; mu_s, Sig_s), the goal factor
N(x_{N-1}; mu_g, Sig_g) and the transition factors above.  Blocks:
D[i] = (i,i) block, U[i] = (i,i+1) block; eta = K^-1 mu_bar.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def discretize(A, a, B, Qc, dt):
    """Phi, abar, Q of one interval by matrix exponentials."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    M1 = np.zeros((n + 1, n + 1))
    M1[:n, :n] = A
    M1[:n, n] = a
    E1 = scipy.linalg.expm(M1 * dt)
    Phi = E1[:n, :n]
    abar = E1[:n, n]
    BQB = B @ Qc @ B.T
    M2 = np.zeros((2 * n, 2 * n))
    M2[:n, :n] = -A
    M2[:n, n:] = BQB
    M2[n:, n:] = A.T
    E2 = scipy.linalg.expm(M2 * dt)
    Phi_vl = E2[n:, n:].T
    Q = Phi_vl @ E2[:n, n:]
    Q = 0.5 * (Q + Q.T)
    return Phi, abar, Q


def lti_double_integrator_closed_form(dof, qc, dt):
    """Closed-form Phi and Q of the constant-velocity prior (white-noise
    acceleration with density qc I): Phi = [[I, dt I], [0, I]],
    Q = [[dt^3/3, dt^2/2], [dt^2/2, dt]] (x) qc I."""
    I = np.eye(dof)
    Phi = np.block([[I, dt * I], [np.zeros((dof, dof)), I]])
    Q = np.block([[dt ** 3 / 3 * qc * I, dt ** 2 / 2 * qc * I],
                  [dt ** 2 / 2 * qc * I, dt * qc * I]])
    return Phi, Q


def interval_models(prob):
    """(A_i, a_i, B_i) for i = 0..N-2."""
    N = prob["N"]
    if prob.get("ltv", False):
        return [(prob["A"][i], prob["a"][i], prob["B"][i]) for i in range(N - 1)]
    return [(prob["A"], prob["a"], prob["B"])] * (N - 1)


def build_prior(prob):
    """Discretise every interval and sum the factors into K^-1 and eta."""
    N, n = prob["N"], prob["n"]
    Phi = np.zeros((max(N - 1, 0), n, n))
    abar = np.zeros((max(N - 1, 0), n))
    Q = np.zeros((max(N - 1, 0), n, n))
    for i, (A, a, B) in enumerate(interval_models(prob)):
        Phi[i], abar[i], Q[i] = discretize(A, a, B, prob["Qc"], prob["dt"])
    Qinv = np.array([np.linalg.inv(q) for q in Q]).reshape(Q.shape)
    D = np.zeros((N, n, n))
    U = np.zeros((max(N - 1, 0), n, n))
    eta = np.zeros((N, n))
    Ss = np.linalg.inv(prob["Sig_start"])
    Sg = np.linalg.inv(prob["Sig_goal"])
    D[0] += Ss
    eta[0] += Ss @ prob["mu_start"]
    D[N - 1] += Sg
    eta[N - 1] += Sg @ prob["mu_goal"]
    for i in range(N - 1):
        # residual r = x_{i+1} - Phi x_i - abar with precision Qinv
        D[i] += Phi[i].T @ Qinv[i] @ Phi[i]
        D[i + 1] += Qinv[i]
        U[i] += -Phi[i].T @ Qinv[i]
        eta[i] += -Phi[i].T @ Qinv[i] @ abar[i]
        eta[i + 1] += Qinv[i] @ abar[i]
    mu_bar = banded_solve(D, U, eta)
    return {"Phi": Phi, "abar": abar, "Q": Q, "Qinv": Qinv, "D": D, "U": U,
            "eta": eta, "mu_bar": mu_bar}


def dense_from_blocks(D, U):
    """Dense symmetric matrix from diagonal blocks D and super-diagonal U."""
    N, n = D.shape[0], D.shape[1]
    M = np.zeros((N * n, N * n))
    for i in range(N):
        M[i * n:(i + 1) * n, i * n:(i + 1) * n] = D[i]
    for i in range(N - 1):
        M[i * n:(i + 1) * n, (i + 1) * n:(i + 2) * n] = U[i]
        M[(i + 1) * n:(i + 2) * n, i * n:(i + 1) * n] = U[i].T
    return M


def dense_prior_precision(prob):
    """K^-1 and eta assembled densely as J^T W J and J^T W r0 from explicit
    factor Jacobians (an independent assembly used to pin build_prior)."""
    N, n = prob["N"], prob["n"]
    rows_J, rows_W, rows_r = [], [], []
    E0 = np.zeros((n, N * n))
    E0[:, :n] = np.eye(n)
    rows_J.append(E0)
    rows_W.append(np.linalg.inv(prob["Sig_start"]))
    rows_r.append(prob["mu_start"])
    for i, (A, a, B) in enumerate(interval_models(prob)):
        Phi, abar, Q = discretize(A, a, B, prob["Qc"], prob["dt"])
        J = np.zeros((n, N * n))
        J[:, i * n:(i + 1) * n] = -Phi
        J[:, (i + 1) * n:(i + 2) * n] = np.eye(n)
        rows_J.append(J)
        rows_W.append(np.linalg.inv(Q))
        rows_r.append(abar)
    EN = np.zeros((n, N * n))
    EN[:, (N - 1) * n:] = np.eye(n)
    rows_J.append(EN)
    rows_W.append(np.linalg.inv(prob["Sig_goal"]))
    rows_r.append(prob["mu_goal"])
    J = np.vstack(rows_J)
    W = scipy.linalg.block_diag(*rows_W)
    r0 = np.concatenate(rows_r)
    return J.T @ W @ J, J.T @ W @ r0


def banded_solve(D, U, rhs):
    """Solve the block-tridiagonal SPD system (D, U) x = rhs with LAPACK's
    banded Cholesky (scipy.linalg.solveh_banded); rhs is [N, n]."""
    N, n = D.shape[0], D.shape[1]
    u = 2 * n - 1  # number of super-diagonals of the scalar band
    ab = np.zeros((u + 1, N * n))
    M = lambda i, j: _block_entry(D, U, n, i, j)  # noqa: E731
    for j in range(N * n):
        for i in range(max(0, j - u), j + 1):
            ab[u + i - j, j] = M(i, j)
    x = scipy.linalg.solveh_banded(ab, np.asarray(rhs).reshape(-1), lower=False)
    return x.reshape(N, n)


def _block_entry(D, U, n, i, j):
    bi, bj = i // n, j // n
    ri, rj = i % n, j % n
    if bi == bj:
        return D[bi][ri, rj]
    if bj == bi + 1:
        return U[bi][ri, rj]
    if bi == bj + 1:
        return U[bj][rj, ri]
    return 0.0


def block_matvec(D, U, x):
    """y = M x for the block-tridiagonal symmetric M = (D, U)."""
    y = np.einsum("iab,ib->ia", D, x)
    if U.shape[0]:
        y[:-1] += np.einsum("iab,ib->ia", U, x[1:])
        y[1:] += np.einsum("iba,ib->ia", U, x[:-1])
    return y
