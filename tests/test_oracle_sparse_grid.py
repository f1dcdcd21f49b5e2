"""Pins of the oracle's Smolyak sparse-grid rule (Sec. 4.3 Lemma 1).

* a hand-worked level-2 rule in 2-D (tests/golden/smolyak_k2_d2.txt);
* exactness for every monomial of total degree <= 2k - 1 against the
  moments of the standard normal (E[x^m] = (m-1)!! for even m, 0 for odd),
  and failure for some monomial of degree 2k (so the level is not higher);
* in one dimension the level-k rule is the k-point Gauss-Hermite rule;
* the expectation of a quadratic collision cost on an affine field is the
  closed form whatever rule integrates it (both rules are exact there).
"""
import itertools
import math
import os

import numpy as np
import pytest

import workloads
from oracle import collision, gbp, gh, prior

HERE = os.path.dirname(os.path.abspath(__file__))


def normal_moment(alpha):
    out = 1.0
    for m in alpha:
        if m % 2:
            return 0.0
        out *= math.prod(range(m - 1, 0, -2)) if m > 0 else 1.0
    return out


def monomials(d, degree):
    for alpha in itertools.product(range(degree + 1), repeat=d):
        if sum(alpha) <= degree:
            yield alpha


def test_level_two_in_two_dimensions_matches_hand_construction():
    ref = np.loadtxt(os.path.join(HERE, "golden", "smolyak_k2_d2.txt"))
    x, w = gh.smolyak_rule(2, 2)
    got = {tuple(p): wi for p, wi in zip(x, w)}
    assert len(got) == len(ref)
    for row in ref:
        assert abs(got[(row[0], row[1])] - row[2]) < 1e-15


@pytest.mark.parametrize("k,d", [(2, 3), (3, 2), (3, 4), (4, 3), (5, 2), (3, 7), (4, 5)])
def test_exact_to_total_degree_2k_minus_1(k, d):
    x, w = gh.smolyak_rule(k, d)
    assert abs(w.sum() - 1.0) < 1e-13
    for alpha in monomials(d, 2 * k - 1):
        val = float(np.sum(w * np.prod(x ** np.array(alpha), axis=1)))
        assert abs(val - normal_moment(alpha)) < 1e-10 * max(1.0, normal_moment(alpha)), (k, d, alpha, val)
    # some monomial of degree 2k is missed (for d >= 2 the rule is not a
    # tensor rule of k points, which would be exact there)
    misses = [alpha for alpha in itertools.product(range(2 * k + 1), repeat=d) if sum(alpha) == 2 * k
              and abs(float(np.sum(w * np.prod(x ** np.array(alpha), axis=1))) - normal_moment(alpha)) > 1e-8]
    assert misses


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_one_dimension_is_the_gauss_hermite_rule(k):
    x, w = gh.smolyak_rule(k, 1)
    xg, wg = gh.gh_rule(k)
    order = np.argsort(x[:, 0])
    np.testing.assert_allclose(x[order, 0], xg, atol=1e-14)
    np.testing.assert_allclose(w[order], wg, atol=1e-14)


def test_fewer_points_than_the_tensor_rule_in_seven_dimensions():
    # the reason for sparse grids (Sec. 4.3): level 6 in 7-D against 6^7
    x, w = gh.smolyak_rule(6, 7)
    assert len(w) < 6 ** 7 / 30
    assert np.min(w) < 0  # negative weights


@pytest.mark.parametrize("k", [3, 4])
def test_affine_field_closed_form_with_sparse_rule(k):
    p = workloads.affine_sdf_problem(N=6)
    p["quadrature"], p["gh_points"] = "sparse", k
    a, b = p["affine"]
    w, kappa = p["obs_weight"], p["hinge_eps"] - b
    pri = prior.build_prior(p)
    S, _, _ = gbp.gbp_marginals(pri["D"], pri["U"])
    E, g, H = collision.collision_expectations(p, pri["mu_bar"], S)
    r = kappa - pri["mu_bar"][:, :2] @ a
    Ec = w * (r ** 2 + np.einsum("a,iab,b->i", a, S[:, :2, :2], a))
    np.testing.assert_allclose(E, Ec, rtol=1e-12)
    np.testing.assert_allclose(g[:, :2], -2 * w * r[:, None] * a[None, :], rtol=1e-10, atol=1e-10)
    # the Stein form subtracts E[psi] Sigma^-1 from a term of its size
    # (Sigma ~ 1e-4 I here), as with the tensor rule
    np.testing.assert_allclose(H[:, :2, :2], np.repeat((2 * w * np.outer(a, a))[None], 6, axis=0),
                               rtol=1e-6, atol=1e-6)
