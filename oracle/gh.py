"""Gauss-Hermite quadrature (Sec. 4.3, steps 1-3 and eq. GH_quadrature_matmul).

Readings of the paper:
  * The Hermite family is the probabilists' He_p (weight = standard normal
    density), so the rule integrates against N(0, I) and its weights sum to 1.
  * The printed weight formula lacks the square on He_{p-1}; as printed it
    gives a negative weight for p = 3.  The weight used is
        W_i = p! / (p^2 * He_{p-1}(xi_i)^2).
  * In the multi-dimensional rule the square root of P is the lower Cholesky
    factor L (P = L L^T), and the points are the tensor product of the
    one-dimensional points, the first coordinate varying fastest.
  * Sparse grids (Sec. 4.3 Lemma 1): Smolyak's combination of tensor rules
    built from the 1-D Gauss-Hermite rules, as in the cited Heiss-Winschel
    construction: level k (the paper's precision degree k_q) is exact for
    every polynomial of total degree <= 2k - 1.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from numpy.polynomial import hermite_e


def hermite_he(k: int, x):
    """Probabilists' Hermite polynomial He_k(x) by its three-term recurrence
    He_{j+1} = x He_j - j He_{j-1}, He_0 = 1, He_1 = x."""
    x = np.asarray(x, dtype=np.float64)
    h_prev = np.ones_like(x)
    if k == 0:
        return h_prev
    h = x.copy()
    for j in range(1, k):
        h_prev, h = h, x * h - j * h_prev
    return h


def gh_rule(p: int):
    """Step 1: the p roots of He_p (sigma points); step 2: their weights."""
    if p < 1:
        raise ValueError("p must be >= 1")
    coeffs = np.zeros(p + 1)
    coeffs[p] = 1.0
    xi = np.sort(np.real(hermite_e.hermeroots(coeffs)))
    # polish the roots with Newton steps on the recurrence (dHe_p = p He_{p-1})
    for _ in range(3):
        xi = xi - hermite_he(p, xi) / (p * hermite_he(p - 1, xi))
    w = math.factorial(p) / (p * p * hermite_he(p - 1, xi) ** 2)
    return xi, w


def tensor_rule(p: int, d: int):
    """Tensor-product points [p^d, d] and weights [p^d]; coordinate 0 fastest."""
    xi, w = gh_rule(p)
    idx = np.indices((p,) * d).reshape(d, -1)[::-1].T  # rows: (j_0, ..., j_{d-1}), j_0 fastest
    pts = xi[idx]
    wts = np.prod(w[idx], axis=1)
    return pts, wts


def expect(phi, m, P, p: int):
    """Step 3: int phi(x) N(x; m, P) dx ~ sum_j W_j phi(L xi_j + m).

    phi maps an [K, d] array of points to [K, ...] values.
    """
    m = np.asarray(m, dtype=np.float64)
    d = m.shape[0]
    L = np.linalg.cholesky(np.asarray(P, dtype=np.float64))
    pts, wts = tensor_rule(p, d)
    x = pts @ L.T + m[None, :]
    vals = np.asarray(phi(x), dtype=np.float64)
    return np.tensordot(wts, vals, axes=(0, 0))


def smolyak_rule(k: int, d: int):
    """Sparse-grid rule of level k in d dimensions: points [M, d], weights [M].

    A(k, d) = sum over q = max(0, k - d) .. k - 1 of
              (-1)^(k-1-q) C(d-1, k-1-q) sum over i in N^d, i_j >= 1,
              |i| = d + q, of the tensor rule U_{i_1} x ... x U_{i_d},
    U_i being the i-point Gauss-Hermite rule (exact to degree 2i - 1).
    Points that several tensor rules share (only coordinates equal to the
    exact zero of odd rules coincide) are merged by adding their weights.
    Points are listed in the order they first appear; weights may be
    negative."""
    if k < 1 or d < 1:
        raise ValueError("k and d must be >= 1")
    acc = {}
    order = []
    for q in range(max(0, k - d), k):
        coef = (-1) ** (k - 1 - q) * math.comb(d - 1, k - 1 - q)
        for levels in itertools.product(range(1, q + 2), repeat=d):
            if sum(levels) != d + q:
                continue
            rules = [gh_rule(i) for i in levels]
            for combo in itertools.product(*[range(i) for i in levels]):
                x = tuple(float(rules[a][0][combo[a]]) for a in range(d))
                w = coef * math.prod(float(rules[a][1][combo[a]]) for a in range(d))
                if x not in acc:
                    acc[x] = 0.0
                    order.append(x)
                acc[x] += w
    pts = np.array(order, dtype=np.float64).reshape(-1, d)
    wts = np.array([acc[x] for x in order], dtype=np.float64)
    return pts, wts


def rule(kind: str, p: int, d: int):
    """The d-dimensional rule of a problem: 'tensor' (p points per axis) or
    'sparse' (Smolyak level p)."""
    return smolyak_rule(p, d) if kind == "sparse" else tensor_rule(p, d)
