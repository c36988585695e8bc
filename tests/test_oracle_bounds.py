"""Pins of the oracle's error-control bounds (section 3, "Upper and Lower
Bounds"; rounding algorithm of the supplementary material) to facts that do
not come from the oracle itself: marginal invariants of the rounding, a
hand-derived rounding, weak duality against the exact transport value of the
assignment problem, and strong duality at an LP optimum.
"""
import math

import numpy as np
import pytest
from scipy.optimize import linprog

import pdgen
from oracle import bounds, ground, matching, sinkhorn


def test_rounding_hand_example():
    """P = ones(2, 2), r = (1, 3), c = (2, 2), worked by hand: X = (1/2, 1),
    Y = (1, 1), e_r = (0, 1), e_c = (1/2, 1/2), F = [[1/2, 1/2], [3/2, 3/2]]."""
    F = bounds.round_to_feasible(np.ones((2, 2)), [1.0, 3.0], [2.0, 2.0])
    np.testing.assert_allclose(F, [[0.5, 0.5], [1.5, 1.5]], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rounding_marginals_and_feasible_fixed_point(seed):
    """F(P) lies in Pi(r, c) and is non-negative; a plan already in Pi(r, c)
    is returned unchanged."""
    rng = np.random.default_rng(seed)
    P = rng.random((7, 5)) * (rng.random((7, 5)) < 0.7)
    r = rng.random(7) + 0.1
    c = rng.random(5) + 0.1
    c *= r.sum() / c.sum()
    F = bounds.round_to_feasible(P, r, c)
    np.testing.assert_allclose(F.sum(axis=1), r, rtol=1e-13)
    np.testing.assert_allclose(F.sum(axis=0), c, rtol=1e-13)
    assert np.all(F >= -1e-15)
    G = np.outer(r, c) / r.sum()
    np.testing.assert_allclose(bounds.round_to_feasible(G, r, c), G, rtol=1e-14)


def _pair(seed, d, n1, n2):
    rng = np.random.default_rng(seed)
    D1 = pdgen.gen(rng, n1)
    D2 = pdgen.gen(rng, n2)
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    exact = matching.ot_assignment(matching.hist_points(h1, d), matching.hist_points(h2, d))
    return h1, h2, exact


@pytest.mark.parametrize("seed,gamma,iters", [(0, 1e-2, 5), (1, 5e-3, 40), (2, 2e-3, 200), (3, 1e-2, 1)])
def test_bounds_bracket_exact_value(seed, gamma, iters):
    """m_t <= L_C(a, b) <= M_t for any t (weak duality / feasibility of the
    rounded plan), with L_C from the assignment problem of Proposition 1; the
    rounded plan has exactly the marginals (a, b)."""
    d = 10
    h1, h2, exact = _pair(seed, d, 6, 9)
    C = ground.dense_cost(d)
    r = sinkhorn.sinkhorn(h1, h2, gamma, max_iter=iters, C=C)
    a, b = ground.marginals(h1, h2)
    up = bounds.upper_bound(r.log_u, r.log_v, a, b, C, gamma)
    lo = bounds.lower_bound(r.log_u, a, b, C, gamma)
    assert lo <= exact + 1e-12 and exact <= up + 1e-12, (lo, exact, up)
    F = bounds.round_to_feasible(bounds.dense_plan(r.log_u, r.log_v, C, gamma), a, b)
    np.testing.assert_allclose(F.sum(axis=1), a, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(F.sum(axis=0), b, rtol=1e-12, atol=1e-12)


def test_bounds_close_at_small_gamma():
    """With a small gamma run to a tight marginal error the two bounds pinch the
    exact value (the error-control statement of section 3)."""
    d = 10
    h1, h2, exact = _pair(5, d, 7, 8)
    C = ground.dense_cost(d)
    gamma = 5e-4
    r = sinkhorn.sinkhorn(h1, h2, gamma, tol=1e-9, max_iter=20000, C=C)
    a, b = ground.marginals(h1, h2)
    up = bounds.upper_bound(r.log_u, r.log_v, a, b, C, gamma)
    lo = bounds.lower_bound(r.log_u, a, b, C, gamma)
    assert lo <= exact <= up
    assert up - lo <= 0.02 * exact, (lo, exact, up)


def test_dual_bound_strong_duality_at_lp_optimum():
    """At an optimal dual pair of the transport LP (scipy's linprog on the
    supports) the c-transform bound equals L_C exactly, and it never falls
    below the dual objective of the pair it starts from."""
    d = 8
    h1, h2, exact = _pair(7, d, 5, 6)
    C = ground.dense_cost(d)
    a, b = ground.marginals(h1, h2)
    ia, ib = np.flatnonzero(a > 0), np.flatnonzero(b > 0)
    na, nb = len(ia), len(ib)
    # max <alpha, a> + <beta, b>  s.t.  alpha_i + beta_j <= C_ij
    A = np.zeros((na * nb, na + nb))
    for p, i in enumerate(range(na)):
        A[p * nb:(p + 1) * nb, i] = 1.0
        A[p * nb:(p + 1) * nb, na:] = np.eye(nb)
    rhs = C[np.ix_(ia, ib)].ravel()
    lp = linprog(-np.concatenate([a[ia], b[ib]]), A_ub=A, b_ub=rhs, bounds=(None, None), method="highs")
    assert lp.status == 0
    assert math.isclose(-lp.fun, exact, rel_tol=1e-9, abs_tol=1e-12)
    alpha = np.full(a.shape, -np.inf)
    alpha[ia] = lp.x[:na]
    val = bounds.dual_bound(alpha, a, b, C)
    assert math.isclose(val, exact, rel_tol=1e-9, abs_tol=1e-12), (val, exact)
    # any feasible start: the transformed pair does at least as well
    rng = np.random.default_rng(0)
    al = rng.normal(size=na) * 0.05
    be = np.min(C[np.ix_(ia, ib)] - al[:, None], axis=0) - rng.random(nb) * 0.01
    alpha2 = np.full(a.shape, -np.inf)
    alpha2[ia] = al
    assert bounds.dual_bound(alpha2, a, b, C) >= a[ia] @ al + b[ib] @ be - 1e-12
    assert bounds.dual_bound(alpha2, a, b, C) <= exact + 1e-12


def test_c_transform_one_dimensional_example():
    """A 3-point space with C = |x - y| worked by hand: alpha = (0, 1, -inf)
    gives alpha^c = (0, -1, 0)."""
    C = np.abs(np.subtract.outer([0.0, 1.0, 2.0], [0.0, 1.0, 2.0]))
    np.testing.assert_array_equal(bounds.c_transform([0.0, 1.0, -np.inf], C), [0.0, -1.0, 0.0])
