"""Pins of the FP64 oracle to facts that do not come from the oracle itself.

Each test names the passage of the paper (or the piece of mathematics) it
checks.  None of these touch the GPU library.
"""
import json
import math
import os

import numpy as np
import pytest

import pdgen
from oracle import barycenter, ground, kmeans, matching, separable, sinkhorn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_diag(rng, n, d=None):
    b = rng.random(n)
    t = np.minimum(b + rng.random(n) * (1 - b), 1.0)
    pts = np.stack([b, t], 1)
    if d is not None:                       # snap to grid cells (exact discretisation)
        pts = np.floor(pts * d) / d
    return pts.astype(np.float32)


# --- ground space -----------------------------------------------------------

@pytest.mark.parametrize("p", [1.0, 2.0, 3.0])
def test_dense_cost_is_geometry(p):
    """C entries equal ||x - y||_p^p between cell corners and the distance to the
    orthogonal projection on the diagonal (section 2, d_p; section 3, cost C)."""
    d = 5
    C = ground.dense_cost(d, p)
    rng = np.random.default_rng(1)
    for _ in range(50):
        i, j, k, l = rng.integers(0, d, 4)
        x = np.array([i / d, j / d])
        y = np.array([k / d, l / d])
        assert math.isclose(C[i * d + j, k * d + l], np.sum(np.abs(x - y) ** p), rel_tol=1e-14, abs_tol=1e-15)
        proj = np.full(2, x.mean())          # orthogonal projection on {s = t}
        cd = np.sum(np.abs(x - proj) ** p)
        assert math.isclose(C[i * d + j, d * d], cd, rel_tol=1e-14, abs_tol=1e-15)
        assert math.isclose(C[d * d, i * d + j], cd, rel_tol=1e-14, abs_tol=1e-15)
    assert C[d * d, d * d] == 0.0
    np.testing.assert_array_equal(C, C.T)


def test_discretize_cells_and_errors():
    """Point (b, t) -> cell (floor(b d), floor(t d)), 1.0 -> last cell (supplementary, discretisation)."""
    h = ground.discretize(np.array([[0.0, 0.0], [0.5, 0.99], [1.0, 1.0], [0.5, 0.99]], np.float32), 4)
    assert h[0, 0] == 1 and h[2, 3] == 2 and h[3, 3] == 1 and h.sum() == 4
    for bad in ([[0.6, 0.5]], [[-0.1, 0.5]], [[0.2, 1.5]], [[np.nan, 0.5]]):
        with pytest.raises(ValueError):
            ground.discretize(np.array(bad, np.float32), 4)
    # float32 values at cell boundaries: decision in exact arithmetic
    v = np.nextafter(np.float32(0.5), np.float32(0))
    assert ground.discretize(np.array([[v, v]], np.float32), 100)[49, 49] == 1


# --- Propositions 2 and 3 ---------------------------------------------------

@pytest.mark.parametrize("d", [4, 7, 32])
def test_prop2_separable_apply_equals_dense(d):
    """Proposition 2: the separable K application equals the dense (d^2+1) kernel."""
    gamma = 0.05
    rng = np.random.default_rng(d)
    C = ground.dense_cost(d)
    K = np.exp(-C / gamma)
    k, _, kd, _ = separable.tables(d, gamma)
    U = rng.random((d, d)) * rng.random((d, d))      # not symmetric on purpose
    ud = 0.7
    dense = K @ np.append(U.ravel(), ud)
    W, Wd = separable.apply_K(U, ud, k, kd)
    np.testing.assert_allclose(W.ravel(), dense[:-1], rtol=1e-13, atol=0)
    assert math.isclose(Wd, dense[-1], rel_tol=1e-13)


@pytest.mark.parametrize("d", [4, 7, 32])
def test_prop3_separable_cost_equals_dense(d):
    """Proposition 3: the separable transport cost equals <diag(u) K diag(v), C>."""
    gamma = 0.05
    rng = np.random.default_rng(100 + d)
    C = ground.dense_cost(d)
    K = np.exp(-C / gamma)
    k, m, kd, md = separable.tables(d, gamma)
    U, V = rng.random((d, d)), rng.random((d, d))
    ud, vd = 0.3, 1.9
    u, v = np.append(U.ravel(), ud), np.append(V.ravel(), vd)
    dense = np.sum(u[:, None] * K * v[None, :] * C)
    sep = separable.transport_cost(U, ud, V, vd, k, m, md)
    assert math.isclose(sep, dense, rel_tol=1e-13)


def test_kernel_symmetric_and_marginals():
    """K = K^T (C symmetric, section 3) and the marginals of P = diag(u) K diag(v) are
    u * (K v) and v * (K^T u) (supplementary, proof of Proposition 4)."""
    d, gamma = 6, 0.1
    C = ground.dense_cost(d)
    K = np.exp(-C / gamma)
    np.testing.assert_array_equal(K, K.T)
    rng = np.random.default_rng(3)
    u, v = rng.random(d * d + 1), rng.random(d * d + 1)
    P = u[:, None] * K * v[None, :]
    np.testing.assert_allclose(P.sum(1), u * (K @ v), rtol=1e-14)
    np.testing.assert_allclose(P.sum(0), v * (K.T @ u), rtol=1e-14)


# --- Proposition 1 and exact distances -------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_prop1_ot_equals_partial_matching(seed):
    """Proposition 1: L_C(D1 + R D2, D2 + R D1) equals d_p^p, the minimum over
    partial matchings (brute-force enumeration of the definition)."""
    rng = np.random.default_rng(seed)
    D1 = _rand_diag(rng, int(rng.integers(0, 5)))
    D2 = _rand_diag(rng, int(rng.integers(1, 5)))
    for p in (1.0, 2.0):
        bf = matching.dp_bruteforce(D1, D2, p)
        ot = matching.ot_assignment(D1, D2, p)
        assert math.isclose(bf, ot, rel_tol=1e-12, abs_tol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_gamma_to_zero_bound(seed):
    """S^gamma at convergence approaches L_C as gamma -> 0 within the error bound
    2 gamma n log n + dist(P, Pi) ||C||_inf of section 3."""
    d = 10
    rng = np.random.default_rng(seed)
    D1, D2 = _rand_diag(rng, 3, d), _rand_diag(rng, 4, d)
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    L = matching.ot_assignment(matching.hist_points(h1, d), matching.hist_points(h2, d))
    C = ground.dense_cost(d)
    n = h1.sum() + h2.sum()
    gaps = []
    for gamma in (1e-2, 3e-3, 1e-3):
        r = sinkhorn.sinkhorn(h1, h2, gamma, tol=1e-8, max_iter=200000, C=C)
        bound = 2 * gamma * n * math.log(n) + r.err * n * C.max()
        assert abs(r.cost - L) <= bound
        assert r.cost >= L - r.err * n * C.max() - 1e-12     # feasible up to the marginal error
        gaps.append(abs(r.cost - L))
    assert gaps[-1] <= 0.05 * max(L, 1e-3) + 1e-9


@pytest.mark.parametrize("seed", range(3))
def test_discretization_error_bound(seed):
    """|d_p(D1, D2) - L_C(hist)^(1/p)| <= 2^(1/p) (1/d) (|D1|^(1/p) + |D2|^(1/p)):
    supplementary bound, with the per-point displacement of up to 1/d in each
    coordinate (the printed bound omits the 2^(1/p))."""
    rng = np.random.default_rng(seed)
    D1, D2 = _rand_diag(rng, 3), _rand_diag(rng, 3)
    for d, p in ((8, 2.0), (16, 2.0), (8, 1.0)):
        h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
        raw = matching.dp_bruteforce(D1, D2, p) ** (1 / p)
        disc = matching.ot_assignment(matching.hist_points(h1, d), matching.hist_points(h2, d), p) ** (1 / p)
        bound = 2 ** (1 / p) / d * (len(D1) ** (1 / p) + len(D2) ** (1 / p))
        assert abs(raw - disc) <= bound + 1e-12


# --- Algorithm 1 closed forms and invariants --------------------------------

@pytest.mark.parametrize("gamma", [1e-1, 1e-2, 1e-3])
def test_empty_diagram_closed_form(gamma):
    """D2 empty: the only feasible plan sends every point to the diagonal, so
    <P, C> = sum_cells a_ij c_Delta,ij for every gamma, exactly from iteration 2.
    d=50, gamma=1e-3 puts c_Delta/gamma up to 480 (range stress)."""
    d = 50
    D1 = pdgen.gen(np.random.default_rng(7), 60)
    h1 = ground.discretize(D1, d)
    h2 = np.zeros((d, d))
    exact = float(np.sum(h1 * ground.cost_diag(d)))
    C = ground.dense_cost(d)
    for T in (2, 3, 10):
        r = sinkhorn.sinkhorn(h1, h2, gamma, max_iter=T, C=C)
        assert math.isclose(r.cost, exact, rel_tol=1e-13)
        assert r.err < 1e-13


def test_mass_scaling_equivariance():
    """Scaling both marginals by s scales every plan and S by s; err/m is unchanged."""
    d, gamma = 12, 5e-3
    D1, D2 = pdgen.pair_single(3, 9, 11)
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    C = ground.dense_cost(d)
    r1 = sinkhorn.sinkhorn(h1, h2, gamma, max_iter=40, C=C)
    r2 = sinkhorn.sinkhorn(2.5 * h1, 2.5 * h2, gamma, max_iter=40, C=C)
    assert math.isclose(r2.cost, 2.5 * r1.cost, rel_tol=1e-12)
    assert math.isclose(r2.err, r1.err, rel_tol=1e-9)


def _converged(h1, h2, gamma, C, **kw):
    return sinkhorn.sinkhorn(h1, h2, gamma, tol=1e-12, max_iter=100000, C=C, **kw)


def test_symmetry_and_uniqueness_at_fixed_point():
    """P^gamma is unique (strictly convex problem, section 2): S(a,b) = S(b,a) and
    the fixed point does not depend on the initial v."""
    d, gamma = 12, 5e-3
    D1, D2 = pdgen.pair_single(5, 8, 13)
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    C = ground.dense_cost(d)
    r_ab = _converged(h1, h2, gamma, C)
    r_ba = _converged(h2, h1, gamma, C)
    rng = np.random.default_rng(0)
    r_init = _converged(h1, h2, gamma, C, log_v0=rng.normal(0, 3, d * d + 1))
    assert math.isclose(r_ab.cost, r_ba.cost, rel_tol=1e-9)
    assert math.isclose(r_ab.cost, r_init.cost, rel_tol=1e-9)


def test_diagonal_shift_invariance():
    """Shifting both diagrams by whole cells along (1,1) leaves C restricted to the
    support unchanged (C depends on index differences and j - i only)."""
    d, gamma = 14, 5e-3
    rng = np.random.default_rng(11)
    D1 = _rand_diag(rng, 6) * 0.6
    D2 = _rand_diag(rng, 7) * 0.6
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    s = 3
    g1, g2 = np.zeros_like(h1), np.zeros_like(h2)
    g1[s:, s:] = h1[: d - s, : d - s]
    g2[s:, s:] = h2[: d - s, : d - s]
    assert g1.sum() == h1.sum() and g2.sum() == h2.sum()
    C = ground.dense_cost(d)
    assert math.isclose(_converged(h1, h2, gamma, C).cost, _converged(g1, g2, gamma, C).cost, rel_tol=1e-9)


def test_fixed_point_marginals_and_plan():
    """At stopping the plan's marginals are within the reported error of a and b,
    and the reported cost is <P, C> of that plan."""
    d, gamma = 10, 1e-2
    D1, D2 = pdgen.pair_single(2, 7, 9)
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    C = ground.dense_cost(d)
    r = sinkhorn.sinkhorn(h1, h2, gamma, tol=1e-6, max_iter=5000, C=C)
    P = sinkhorn.plan(r, C, gamma)
    a, b = ground.marginals(h1, h2)
    dist = (np.abs(P.sum(1) - a).sum() + np.abs(P.sum(0) - b).sum()) / a.sum()
    assert dist <= 1e-6 and math.isclose(dist, r.err, rel_tol=1e-6, abs_tol=1e-12)
    assert math.isclose(np.sum(P * C), r.cost, rel_tol=1e-12)


def test_stabilised_scaling_matches_log_domain():
    """The absorbed scaling form and the log-sum-exp form run the same iterations:
    at a gamma that forces absorptions, costs agree at every checked iteration count."""
    d, gamma = 16, 1e-3
    D1 = np.array([[0.0, 0.95], [0.3, 0.4], [0.31, 0.45]], np.float32)   # (0, 0.95): c_Delta/gamma ~ 450
    D2 = np.array([[0.8, 0.85], [0.5, 0.55], [0.52, 0.9]], np.float32)
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    C = ground.dense_cost(d)
    a, b = ground.marginals(h1, h2)
    for T in (1, 5, 40):
        r = sinkhorn.solve(a, b, C, gamma, max_iter=T)
        cl, tl, el, _, _ = sinkhorn.solve_log(a, b, C, gamma, max_iter=T)
        assert tl == r.iters == T
        assert math.isclose(r.cost, cl, rel_tol=1e-10)
        assert math.isclose(r.err, el, rel_tol=1e-6, abs_tol=1e-13)
    assert sinkhorn.solve(a, b, C, gamma, max_iter=40).absorptions > 0


def test_log_domain_on_support_rows_matches_full():
    """Rows off supp(a) carry u = 0 in every iterate, so the log-sum-exp form
    restricted to the rows of supp(a) (all columns kept: the start v = 1 covers
    every column) runs the same iterations as the full stabilised form; the
    GPU tests use it at tiny gamma, where only the log form stays in range."""
    d, gamma = 12, 1e-3
    rng = np.random.default_rng(3)
    h1, h2 = ground.discretize(pdgen.gen(rng, 9), d), ground.discretize(pdgen.gen(rng, 7), d)
    C = ground.dense_cost(d)
    a, b = ground.marginals(h1, h2)
    sa = a > 0
    for T in (1, 6, 30):
        r = sinkhorn.solve(a, b, C, gamma, max_iter=T)
        cl, tl, el, _, _ = sinkhorn.solve_log(a[sa], b, C[sa, :], gamma, max_iter=T)
        assert tl == T
        assert math.isclose(r.cost, cl, rel_tol=1e-10)
        assert math.isclose(r.err, el, rel_tol=1e-6, abs_tol=1e-13)


def test_single_pair_reference_run():
    """Single pair, d=32, gamma=1e-2, 300 iterations: oracle and log-domain agree."""
    D1, D2 = pdgen.pair_single(0)
    d = 32
    h1, h2 = ground.discretize(D1, d), ground.discretize(D2, d)
    C = ground.dense_cost(d)
    r = sinkhorn.sinkhorn(h1, h2, 1e-2, max_iter=300, C=C)
    a, b = ground.marginals(h1, h2)
    cl, _, _, _, _ = sinkhorn.solve_log(a, b, C, 1e-2, max_iter=300)
    assert r.iters == 300
    assert math.isclose(r.cost, cl, rel_tol=1e-11)
    L = matching.ot_assignment(matching.hist_points(h1, d), matching.hist_points(h2, d))
    n = a.sum()
    assert abs(r.cost - L) <= 2 * 1e-2 * n * math.log(n) + r.err * n * C.max()


# --- Proposition 5 and Algorithm 2 ------------------------------------------

def test_prop5_gradient_finite_difference():
    """Proposition 5: d/dx L^gamma(x + R a, a + R x) = gamma (log u + log v_Delta),
    checked by central differences of <P, C> - gamma h(P) at the fixed point."""
    d, gamma = 6, 0.05
    C = ground.dense_cost(d)
    rng = np.random.default_rng(9)
    A = np.triu(rng.random((d, d)) < 0.3).astype(float)
    A[1, 3] += 1
    x = np.triu(np.full((d, d), 0.4)) + np.triu(rng.random((d, d))) * 0.2

    def objective(xx):
        a, b = ground.marginals(xx, A)
        r = sinkhorn.solve(a, b, C, gamma, tol=1e-14, max_iter=200000)
        return sinkhorn.entropic_objective(sinkhorn.plan(r, C, gamma), C, gamma), r

    _, r0 = objective(x)
    grad = gamma * (r0.log_u[: d * d] + r0.log_v[d * d]).reshape(d, d)
    eps = 1e-5
    for (i, j) in [(0, 0), (1, 4), (2, 2), (3, 5), (0, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[i, j] += eps
        xm[i, j] -= eps
        fd = (objective(xp)[0] - objective(xm)[0]) / (2 * eps)
        assert math.isclose(fd, grad[i, j], rel_tol=1e-5, abs_tol=1e-8)


def test_barycenter_lp_value():
    """Two one-point diagrams: the smoothed barycenter energy is bounded below by
    the exact barycenter energy (S^gamma >= L_C at convergence) and approaches it
    as gamma -> 0 (localization corollary; hand-derived value in the fixture)."""
    g = json.load(open(os.path.join(GOLDEN, "bary_two_points.json")))
    d = g["d"]
    hists = [ground.discretize(np.array(D, np.float32), d) for D in g["diagrams"]]
    C = ground.dense_cost(d)
    E_lp = g["lp_optimum_energy"]
    res = barycenter.barycenter(hists, 4e-3, lam=2.0, tol=1e-7, max_inner=200000,
                                max_outer=60, energy_rtol=1e-6, C=C)
    assert res.energy >= E_lp - 1e-6
    assert res.energy < 0.5 * res.energies[0]          # well below the uniform start
    i, j = g["optimal_cell"]
    assert res.z[i, j] == res.z.max()
    # Energies decrease along the multiplicative (mirror-descent) updates.
    e = np.array(res.energies)
    assert np.all(np.diff(e) <= 1e-6 * e[:-1])


def test_barycenter_energy_convexity():
    """E is convex (supplementary, convexity of E); so is its entropic version,
    checked along a segment between two histograms with the converged L^gamma."""
    d, gamma = 6, 0.02
    C = ground.dense_cost(d)
    rng = np.random.default_rng(4)
    hists = [np.triu(rng.integers(0, 2, (d, d))).astype(float) for _ in range(3)]
    mu0 = np.triu(rng.random((d, d))) * 2
    mu1 = np.triu(rng.random((d, d))) * 2

    def E(mu):
        tot = 0.0
        for h in hists:
            a, b = ground.marginals(mu, h)
            r = sinkhorn.solve(a, b, C, gamma, tol=1e-13, max_iter=100000)
            tot += sinkhorn.entropic_objective(sinkhorn.plan(r, C, gamma), C, gamma)
        return tot / len(hists)

    e0, e1 = E(mu0), E(mu1)
    for t in (0.25, 0.5, 0.75):
        assert E((1 - t) * mu0 + t * mu1) <= (1 - t) * e0 + t * e1 + 1e-10


def test_kmeans_assign_separated_clusters():
    """Section 5 k-means assignment: diagrams near one of two far-apart templates
    go to the centroid built from that template; ties go to the lowest index."""
    d = 10
    near = [ground.discretize(np.array([[0.05, 0.15], [0.1, 0.2]], np.float32), d),
            ground.discretize(np.array([[0.1, 0.15]], np.float32), d)]
    far = [ground.discretize(np.array([[0.6, 0.95]], np.float32), d)]
    cents = [near[0], far[0], near[0]]
    labels, dist, _ = kmeans.assign(near + far, cents, 1e-2, tol=1e-6)
    assert list(labels) == [0, 0, 1]
    assert dist[0, 0] == dist[0, 2]          # identical centroids: the tie goes to index 0


def test_barycenter_step_is_finite_difference_gradient():
    """Algorithm 2's update z <- z exp(-lambda grad) with grad the derivative of
    the mean regularised objective (1/N) sum_i L^gamma(z + R a_i, a_i + R z)
    (Proposition 5; gradient averaged over the diagrams).  The step of
    ``barycenter`` is compared with central differences of that objective,
    evaluated by ``entropic_objective`` of converged plans, which involves no
    gradient formula: a dropped diagonal-bin term, a wrong sign or a sum in
    place of the mean each move z by more than 20 %."""
    d, gamma, lam = 5, 0.05, 3.0
    C = ground.dense_cost(d)
    rng = np.random.default_rng(3)
    hists = [np.triu(rng.random((d, d)) < 0.35).astype(float) for _ in range(2)]
    hists[0][0, 2] += 1
    hists[1][3, 4] += 2
    z0 = barycenter.uniform_init(d, float(np.mean([h.sum() for h in hists])))
    r = barycenter.barycenter(hists, gamma, lam=lam, tol=1e-13, max_inner=500000, max_outer=2,
                              energy_rtol=0.0, z0=z0, C=C)
    assert r.outer == 2

    def L_mean(z):
        tot = 0.0
        for h in hists:
            a, b = ground.marginals(z, h)
            s = sinkhorn.solve(a, b, C, gamma, tol=1e-14, max_iter=500000)
            tot += sinkhorn.entropic_objective(sinkhorn.plan(s, C, gamma), C, gamma)
        return tot / len(hists)

    eps = 1e-6
    for i in range(d):
        for j in range(d):
            if j < i:
                assert r.z[i, j] == 0.0          # the multiplicative step keeps the support
                continue
            zp, zm = z0.copy(), z0.copy()
            zp[i, j] += eps
            zm[i, j] -= eps
            g = (L_mean(zp) - L_mean(zm)) / (2 * eps)
            assert math.isclose(r.z[i, j], z0[i, j] * math.exp(-lam * g), rel_tol=1e-7), (i, j)


def test_barycenter_single_diagram_concentrates_as_gamma_falls():
    """N = 1: the barycenter of one diagram is the diagram itself, so as gamma
    falls the smoothed barycenter puts more of its mass on the diagram's cells
    and its total mass approaches the diagram's (the diagonal-bin term of the
    gradient is what sets the mass)."""
    d = 8
    C = ground.dense_cost(d)
    h = ground.discretize(np.array([[1 / 8, 5 / 8], [2 / 8, 6 / 8]], np.float32), d)
    on, mass = [], []
    for g in (8e-3, 4e-3, 2e-3):
        r = barycenter.barycenter([h], g, lam=2.0, tol=1e-8, max_inner=200000, max_outer=80, energy_rtol=1e-7, C=C)
        on.append(float((r.z * (h > 0)).sum() / r.z.sum()))
        mass.append(float(r.z.sum()))
    assert on[0] < on[1] < on[2]
    assert mass[0] > mass[1] > mass[2] > h.sum()


def _two_families(d, n_each=3, seed=1):
    rng = np.random.default_rng(seed)

    def fam(center):
        out = []
        for _ in range(n_each):
            p = np.clip(np.array(center) + rng.normal(0, 0.02, (3, 2)), 0, 1)
            p[:, 1] = np.maximum(p[:, 1], p[:, 0])
            out.append(ground.discretize(p.astype(np.float32), d))
        return out

    return fam([0.1, 0.25]) + fam([0.55, 0.95])


@pytest.mark.parametrize("seed", [0, 3])
def test_lloyd_separates_two_families(seed):
    """Section 5 k-means on diagrams around two far-apart templates: the final
    partition is the two families, whatever the seeded initial centroids
    (seed 0 draws both from the same family).  Once the centroids are
    barycenters (every round after the first) the objective never rises, and
    it stays fixed once the partition does (same members, same barycenter)."""
    d, g = 10, 1e-2
    hists = _two_families(d)
    cents, labels, hist = kmeans.lloyd(hists, 2, 4, g, tol=1e-6, seed=seed, max_outer=8)
    assert len(set(labels[:3])) == 1 and len(set(labels[3:])) == 1 and labels[0] != labels[3]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist[1:], hist[2:]))
    assert hist[-1] == hist[-2]


def test_lloyd_empty_cluster_keeps_centroid():
    """Section 5 readings: ties go to the lowest centroid index, so of two
    identical initial centroids the second gets no member, and a cluster
    without members keeps its centroid."""
    d, g = 10, 1e-2
    hists = _two_families(d)
    hists = hists + [hists[0].copy()]          # diagram 6 duplicates diagram 0
    init = np.random.default_rng(11).choice(len(hists), size=3, replace=False)
    assert sorted(init.tolist()) == [0, 5, 6]
    c_dup = int(np.flatnonzero(init == 6)[0])
    c_orig = int(np.flatnonzero(init == 0)[0])
    assert c_orig < c_dup
    cents, labels, _ = kmeans.lloyd(hists, 3, 1, g, tol=1e-6, seed=11, max_outer=4)
    assert c_dup not in labels.tolist()
    np.testing.assert_array_equal(cents[c_dup], hists[6])


def test_lloyd_singleton_clusters():
    """k = N: every diagram starts as its own centroid, so the first
    assignment is a bijection and the first objective is the sum of the
    self-distances S(D, D) (each within the entropic bound 2 gamma m log m of
    the exact value 0)."""
    d, g = 10, 1e-2
    pts = ([[0.05, 0.25], [0.1, 0.3]], [[0.15, 0.55]], [[0.5, 0.95], [0.62, 0.9]], [[0.3, 0.45], [0.72, 0.85]])
    hists = [ground.discretize(np.array(p, np.float32), d) for p in pts]
    N = len(hists)
    cents, labels, hist = kmeans.lloyd(hists, N, 1, g, tol=1e-6, seed=2, max_outer=2)
    assert sorted(labels.tolist()) == list(range(N))
    C = ground.dense_cost(d)
    self_d = []
    for h in hists:
        a, b = ground.marginals(h, h)
        self_d.append(sinkhorn.solve(a, b, C, g, tol=1e-6, max_iter=1000).cost)
        m = 2 * h.sum()
        assert 0.0 <= self_d[-1] <= 2 * g * m * math.log(m)
    assert math.isclose(hist[0], sum(self_d), rel_tol=1e-12)


# --- Entropic sharpening (section 4, after Algorithm 2; readings in oracle/sharpen.py) ---

def test_sharpen_hits_the_target_entropy_and_keeps_mass_and_order():
    """The sharpened histogram has the target entropy (checked with scipy's own
    entropy routine), the same mass and support, the same order of its cells,
    and is a power of the input: log z' = beta log z + const on the support."""
    from scipy.stats import entropy as sp_entropy
    from oracle import sharpen
    rng = np.random.default_rng(4)
    z = np.triu(rng.gamma(0.7, 1.0, (12, 12)))
    z[z < 0.2] = 0.0
    h = sp_entropy(z[z > 0])
    for h0 in (h - 0.3, h - 1.0, 1.5):
        zs, beta = sharpen.sharpen(z, h0)
        pos = z > 0
        assert beta > 1.0
        assert abs(sp_entropy(zs[pos]) - h0) < 1e-10
        assert np.array_equal(zs > 0, pos)
        assert abs(zs.sum() - z.sum()) < 1e-12 * z.sum()
        order = np.argsort(z[pos], kind="stable")
        assert np.all(np.diff(zs[pos][order]) >= -1e-15)
        slope, icpt = np.polyfit(np.log(z[pos]), np.log(zs[pos]), 1)
        assert abs(slope - beta) < 1e-8 * beta
        assert np.allclose(np.log(zs[pos]), slope * np.log(z[pos]) + icpt, atol=1e-9)


def test_sharpen_two_cells_closed_form():
    """Two cells of masses x and 1 - x: the binary entropy of the sharpened
    split equals h0, and its split is x^b / (x^b + (1-x)^b)."""
    from oracle import sharpen
    x = 0.3
    z = np.array([[x, 1.0 - x]])
    h0 = 0.4
    zs, beta = sharpen.sharpen(z, h0)
    q = zs[0, 0]
    assert abs(-(q * math.log(q) + (1 - q) * math.log(1 - q)) - h0) < 1e-12
    assert abs(q - x ** beta / (x ** beta + (1 - x) ** beta)) < 1e-12


def test_sharpen_no_op_and_limits():
    """At or below the target nothing changes (beta = 1); a target at or below
    log n_max gives the even split over the maximal cells; a uniform histogram
    cannot be sharpened and is its own limit."""
    from oracle import sharpen
    z = np.array([[4.0, 1.0, 1.0], [0.0, 2.0, 4.0], [0.0, 0.0, 0.5]])
    zs, beta = sharpen.sharpen(z, sharpen.entropy(z) + 1e-9)
    assert beta == 1.0 and np.array_equal(zs, z)
    zs, beta = sharpen.sharpen(z, math.log(2.0))
    assert beta == math.inf
    np.testing.assert_allclose(zs, np.where(z == 4.0, z.sum() / 2, 0.0))
    u = np.ones((3, 3))
    zs, beta = sharpen.sharpen(u, 1.0)
    np.testing.assert_allclose(zs, u)
    assert sharpen.sharpen(np.zeros((2, 2)), 0.5)[1] == 1.0


def test_quantize_rounds_each_cell_to_counts():
    """Integer counts nearest to each cell's mass, halves upwards; an integer
    histogram is a fixed point; the total stays within half a point per
    positive cell of the mass."""
    from oracle import sharpen
    z = np.array([[0.49, 0.5, 1.5], [0.0, 2.49999, 3.0], [0.0, 0.0, 7.51]], np.float32)
    q = sharpen.quantize(z)
    np.testing.assert_array_equal(q, [[0, 1, 2], [0, 2, 3], [0, 0, 8]])
    h = np.array([[2.0, 0.0], [1.0, 5.0]], np.float32)
    np.testing.assert_array_equal(sharpen.quantize(h), h.astype(np.int64))
    rng = np.random.default_rng(2)
    r = np.float32(rng.gamma(0.5, 2.0, (20, 20)))
    assert abs(int(sharpen.quantize(r).sum()) - float(r.sum())) <= 0.5 * np.count_nonzero(r)
