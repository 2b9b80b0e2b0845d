"""Pins of the oracle's PDFB closure (data dual with the identity stand-in,
primal update, extrapolation): each checked against a property fixed by the
mathematics rather than by retyping the oracle's formulas."""
import numpy as np
import pytest
from scipy import stats

import synth
from oracle import closure, geometry, sara, step


def _ball_case(seed, ny=9, nx=7, L=4):
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((ny, nx, L))
    z = y + rng.standard_normal((ny, nx, L)) * np.array([0.1, 1.0, 3.0, 0.01])
    eps = np.array([2.0, 2.0, 2.0, 2.0])
    return rng, y, z, eps


def test_l2_ball_projection_variational_inequality():
    """p = proj_C(z) iff p in C and <z - p, q - p> <= 0 for every q in C
    (Table 1, projection onto the l2 ball, per channel)."""
    rng, y, z, eps = _ball_case(1)
    p = closure.project_l2_ball(z, y, eps)
    for l in range(z.shape[2]):
        d = p[..., l] - y[..., l]
        assert np.linalg.norm(d) <= eps[l] * (1 + 1e-12)
        for _ in range(200):
            u = rng.standard_normal(d.shape)
            q = y[..., l] + u / np.linalg.norm(u) * eps[l] * rng.uniform() ** (1.0 / u.size)
            assert np.sum((z[..., l] - p[..., l]) * (q - p[..., l])) <= 1e-12
    inside = np.linalg.norm(z - y, axis=(0, 1)) <= eps
    assert inside.any() and (~inside).any()
    np.testing.assert_array_equal(p[..., inside], z[..., inside])


def test_data_dual_is_distance_to_ball():
    """(I - proj_B)(z) has norm dist(z, B) = max(0, ||z - y|| - eps) and points
    along z - y (Alg. 2 data dual step with the identity operator)."""
    rng, y, z, eps = _ball_case(2)
    v0 = rng.standard_normal(z.shape)
    xc = z - v0
    v = closure.data_dual_update(v0, xc, y, eps)
    r = np.linalg.norm(z - y, axis=(0, 1))
    np.testing.assert_allclose(np.linalg.norm(v, axis=(0, 1)), np.maximum(0.0, r - eps), atol=1e-12)
    for l in range(z.shape[2]):
        if r[l] > eps[l]:
            cos = np.sum(v[..., l] * (z[..., l] - y[..., l])) / (np.linalg.norm(v[..., l]) * r[l])
            assert cos == pytest.approx(1.0, abs=1e-12)


def test_l2_ball_radius_is_chi_square_quantile():
    """eps^2 = sigma^2 (M + 2 sqrt(M)) is the chi-square(M) mean plus sqrt(2)
    standard deviations (Sec. 2.2): its CDF tends to Phi(sqrt 2)."""
    sigma = 0.7
    for m, tol in ((10 ** 4, 0.01), (10 ** 6, 0.002)):
        e = closure.l2_ball_radius(sigma, m)
        assert stats.chi2.cdf((e / sigma) ** 2, m) == pytest.approx(stats.norm.cdf(np.sqrt(2.0)), abs=tol)


def test_primal_update_properties():
    """Projection onto the non-negative orthant, extrapolation 2X+ - X, and the
    relative variation (Alg. 2 primal step)."""
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, (8, 6, 3))
    g = rng.standard_normal(x.shape)
    v = rng.standard_normal(x.shape)
    xn, xc, xi = closure.primal_update(x, g, v, 0.33)
    assert (xn >= 0).all()
    free = x - 0.33 * (g + v) > 0
    np.testing.assert_allclose(xn[free], (x - 0.33 * (g + v))[free], rtol=0, atol=1e-15)
    assert (xn[~free] == 0).all()
    np.testing.assert_allclose(xc + x, 2 * xn, atol=1e-15)
    assert xi.shape == (1,)
    assert xi[0] == pytest.approx(np.sqrt(np.sum((xn - x) ** 2) / np.sum(x ** 2)), rel=1e-13)
    _, _, xi0 = closure.primal_update(np.zeros_like(x), g, v, 0.33)
    assert np.isinf(xi0[0])


def test_relative_variation_per_subcube():
    """Alg. 2 measures the relative variation of each spectral sub-problem on
    its own channels (channel-interleaved sub-cubes, Sec. 2.4.1): changing
    only the channels of sub-cube 1 leaves xi_0 = 0, and a zero sub-cube gives
    +inf whatever the others do."""
    rng = np.random.default_rng(4)
    x = rng.uniform(0.5, 1.0, (5, 4, 6))
    xn = x.copy()
    xn[..., 1::3] *= 1.5
    xi = closure.relative_variation(xn, x, C=3)
    assert xi[0] == 0.0 and xi[2] == 0.0
    assert xi[1] == pytest.approx(0.5, rel=1e-14)
    x[..., 2::3] = 0.0
    xi = closure.relative_variation(xn, x, C=3)
    assert np.isinf(xi[2]) and xi[0] == 0.0


def _objective(X, geom, mu, mu_bar, levels, L):
    f = 0.0
    for q, fc in enumerate(geom.facets):
        f += mu_bar * np.linalg.svd(step.facet_matrix(X, fc, list(range(L))), compute_uv=False).sum()
    A = sara.flatten(sara.analysis(X, levels))
    return f + mu * np.sqrt(np.sum(A * A, axis=1)).sum()


def test_pdfb_reaches_the_constrained_minimiser():
    """With unit weights the problem of Sec. 3 (facet nuclear norms + l21 SARA
    prior, l2-ball data constraint with the identity operator, X >= 0) is
    convex and tau (zeta ||D||^2 + kappa ||Psi||^2 + ||Phi||^2) = 0.99 < 1, so
    the iteration converges to a minimiser.  Checked with the optimality
    conditions of that problem and by a random search: no nearby feasible
    point has a lower objective."""
    ny, nx, L, levels = 16, 12, 3, 2
    geom = geometry.Geometry(ny, nx, 2, 2, 2, 2, levels)
    Xt = synth.blob_cube(ny, nx, L, 6, 123).astype(np.float64)
    rng = np.random.default_rng(5)
    sig = 0.02 * Xt.max()
    y = Xt + sig * rng.standard_normal(Xt.shape)
    eps = np.full(L, closure.l2_ball_radius(sig, ny * nx))
    I = sara.n_coefficients(ny, nx, levels)
    mu, mu_b = 0.05 * Xt.max(), 0.05 * Xt.max()
    theta, theta_bar = [np.ones(I)], [[np.ones(L) for _ in geom.facets]]
    mu_v, mu_bar = np.array([mu]), np.array([[mu_b] * geom.Q])
    x = np.zeros_like(y)
    xc = x.copy()
    P = [[np.zeros(f.nuc_shape + (L,)) for f in geom.facets]]
    W = [np.zeros((I, L))]
    v = np.zeros_like(y)
    for _ in range(500):
        x, xc, P, W, v, xi = closure.pdfb_iteration(x, xc, P, W, v, y, eps, theta, theta_bar, mu_v, mu_bar, geom)
    assert xi[0] < 1e-6
    assert (x >= 0).all()
    assert (np.linalg.norm(x - y, axis=(0, 1)) <= eps * (1 + 1e-5)).all()
    # Optimality (KKT) conditions of the convex problem, from the duals the
    # iteration carries: zeta P_q in the subdifferential of mu_bar ||.||_* at
    # D_q X (spectral norm <= mu_bar, Fenchel-Young equality), kappa W_i in that
    # of mu ||.||_2 at the analysis row, v in the normal cone of the ball, and
    # -(sum_q zeta S~_q^T D_q P_q + kappa Psi W + v) in the normal cone of the
    # orthant.  The gradient is re-assembled here from the windows and the
    # synthesis operator, both pinned on their own.
    G = np.zeros_like(x)
    for q, fc in enumerate(geom.facets):
        Dx = step.facet_matrix(x, fc, list(range(L)))
        Pq = P[0][q].reshape(-1, L)
        assert np.linalg.norm(Pq, 2) <= mu_b * (1 + 1e-6)
        assert np.sum(Pq * Dx) == pytest.approx(mu_b * np.linalg.svd(Dx, compute_uv=False).sum(), rel=1e-4)
        (y0, y1), (x0, x1) = fc.nuc_window
        G[y0:y1, x0:x1] += fc.window()[..., None] * P[0][q]
    A = sara.flatten(sara.analysis(x, levels))
    assert (np.linalg.norm(W[0], axis=1) <= mu * (1 + 1e-6)).all()
    assert np.sum(W[0] * A) == pytest.approx(mu * np.linalg.norm(A, axis=1).sum(), rel=1e-4)
    G += sara.synthesis(sara.unflatten(W[0], ny, nx, levels), ny, nx, levels)
    for l in range(L):
        assert np.sum(v[..., l] * (x[..., l] - y[..., l])) == pytest.approx(
            eps[l] * np.linalg.norm(v[..., l]), rel=1e-4)
    r = G + v
    scale = np.abs(G).max()
    pos = x > 1e-6 * Xt.max()
    assert np.abs(r[pos]).max() <= 1e-4 * scale
    if (~pos).any():
        assert r[~pos].min() >= -1e-4 * scale
    f0 = _objective(x, geom, mu, mu_b, levels, L)
    tried = 0
    for _ in range(150):
        xp = x + 1e-3 * Xt.max() * rng.standard_normal(x.shape)
        for _ in range(20):
            xp = np.maximum(xp, 0.0)
            d = xp - y
            xp = y + d * np.minimum(1.0, eps / np.linalg.norm(d, axis=(0, 1)))
        if (xp < 0).any():
            continue
        tried += 1
        assert _objective(xp, geom, mu, mu_b, levels, L) > f0
    assert tried > 100
