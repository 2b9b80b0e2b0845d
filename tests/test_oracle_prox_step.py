"""Pins of the oracle's proximal operators, dual updates, gather and heuristics.

Closed forms of Table 1, special cases (diagonal / rank-1 / zero / huge or zero
thresholds, one channel), brute force on tiny facets (LAPACK SVD vs Gram
eigendecomposition vs a cyclic Jacobi written here, and the prox objective
against random perturbations), the Moreau / Fenchel-Young identities of the
dual problem (Sec. 3.2), the reductions of Sec. 2.4 (Q = 1: HyperSARA step,
C = L with mu_bar = 0: SARA step), and the chi-distribution constants of the
heuristics.
"""
import numpy as np
import pytest

from oracle import geometry, heuristics, prox, sara, step

RNG = np.random.default_rng(11)


def sv(Z):
    return np.linalg.svd(Z, compute_uv=False)


# ---------------------------------------------------------------- Table 1

def test_soft_threshold():
    z = np.array([-3.0, -0.5, 0.0, 0.2, 2.0])
    assert np.allclose(prox.soft_threshold(z, 1.0), [-2.0, 0.0, 0.0, 0.0, 1.0])


def test_svt_diagonal_matrix():
    d = np.array([5.0, -3.0, 1.0, 0.5])
    Z = np.zeros((6, 4))
    Z[np.arange(4), np.arange(4)] = d
    t = np.array([1.0, 1.5, 2.0, 4.0])     # paired with |d| sorted descending
    P = prox.weighted_svt_complement(Z, t)
    expect = np.zeros((6, 4))
    expect[np.arange(4), np.arange(4)] = np.sign(d) * np.minimum(np.abs(d), t)
    assert np.allclose(P, expect, atol=1e-14)


def test_svt_rank_one():
    a, b = RNG.standard_normal(30), RNG.standard_normal(5)
    Z = np.outer(a, b)
    t = np.array([0.7, 0.8, 0.9, 0.95, 1.0])
    P = prox.weighted_svt_complement(Z, t)
    scale = min(1.0, t[0] / (np.linalg.norm(a) * np.linalg.norm(b)))
    assert np.allclose(P, scale * Z, atol=1e-13)


def test_svt_limits():
    Z = RNG.standard_normal((40, 6))
    assert np.allclose(prox.weighted_svt_complement(np.zeros((40, 6)), np.ones(6)), 0.0)
    assert np.allclose(prox.weighted_svt_complement(Z, np.full(6, 1e30)), Z, atol=1e-13)
    assert np.allclose(prox.weighted_svt_complement(Z, np.zeros(6)), 0.0, atol=1e-14)
    # equal thresholds: projection onto the spectral-norm ball of radius t
    t = 0.5 * sv(Z)[2]
    P = prox.weighted_svt_complement(Z, np.full(6, t))
    assert np.allclose(sv(P), np.minimum(sv(Z), t), atol=1e-13)
    # one channel: complement of the vector l2 shrink, z min(1, t / ||z||)
    z = RNG.standard_normal((40, 1))
    P = prox.weighted_svt_complement(z, np.array([0.3]))
    assert np.allclose(P, z * min(1.0, 0.3 / np.linalg.norm(z)), atol=1e-14)


def _jacobi_eig(A, sweeps=30):
    """Textbook cyclic Jacobi for a small symmetric matrix (brute-force check)."""
    A = A.copy()
    n = A.shape[0]
    V = np.eye(n)
    for _ in range(sweeps):
        off = np.sqrt(np.sum(A ** 2) - np.sum(np.diag(A) ** 2))
        if off < 1e-15 * np.linalg.norm(A):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if A[p, q] == 0.0:
                    continue
                th = (A[q, q] - A[p, p]) / (2 * A[p, q])
                t = np.sign(th) / (abs(th) + np.sqrt(th * th + 1)) if th != 0 else 1.0
                c = 1 / np.sqrt(t * t + 1)
                s = t * c
                J = np.eye(n)
                J[p, p] = J[q, q] = c
                J[p, q], J[q, p] = s, -s
                A = J.T @ A @ J
                V = V @ J
    return np.diag(A), V


def test_svt_brute_force_three_routes():
    # 5 x 4 pixel facet, 3 channels: LAPACK SVD, Gram eigendecomposition and a
    # cyclic Jacobi eigensolver give the same complement of the weighted SVT
    Z = RNG.standard_normal((20, 3))
    t = np.array([0.8, 1.2, 1.9])
    P1 = prox.weighted_svt_complement(Z, t)
    for lam, V in [np.linalg.eigh(Z.T @ Z), _jacobi_eig(Z.T @ Z)]:
        order = np.argsort(lam)[::-1]
        lam, V = lam[order], V[:, order]
        s = np.sqrt(np.maximum(lam, 0))
        h = np.minimum(1.0, t / s)
        P2 = Z @ (V * h) @ V.T
        assert np.allclose(P1, P2, atol=1e-12)


def test_weighted_svt_is_prox_point():
    # f(X) = sum_j t_j s_j(X), t non-descending: the weighted SVT minimises
    # f(X) + 0.5 ||X - Z||^2; compare with 10^4 random perturbations
    Z = RNG.standard_normal((8, 4)) * 2
    t = np.sort(RNG.uniform(0.5, 1.5, 4))
    X = prox.weighted_svt(Z, t)
    obj = lambda M: float(np.dot(t, sv(M))) + 0.5 * float(np.sum((M - Z) ** 2))
    base = obj(X)
    pert = RNG.standard_normal((10000, 8, 4))
    scales = 10.0 ** RNG.uniform(-4, 0, 10000)
    vals = [obj(X + s * d) for s, d in zip(scales, pert)]
    assert min(vals) >= base - 1e-12


def test_moreau_and_fenchel_young_nuclear():
    Z = RNG.standard_normal((50, 6)) * 3
    t = np.sort(RNG.uniform(0.5, 2.0, 6))
    Pp = prox.weighted_svt_complement(Z, t)
    Pr = prox.weighted_svt(Z, t)
    assert np.allclose(Pp + Pr, Z, atol=1e-13)
    assert np.all(sv(Pp) <= t[::-1].max() + 1e-12)
    # sigma_j(P+) = min(sigma_j, t_j)
    assert np.allclose(sv(Pp), np.sort(np.minimum(sv(Z), t))[::-1], atol=1e-12)
    # <prox, P+> = sum_j t_j sigma_j(prox)
    assert abs(float(np.sum(Pr * Pp)) - float(np.dot(t, sv(Pr)))) < 1e-11


def test_l21_closed_forms():
    U = RNG.standard_normal((100, 7))
    a = RNG.uniform(0.5, 3.0, 100)
    Wp = prox.l21_prox_complement(U, a)
    Pr = prox.l21_prox(U, a)
    assert np.allclose(Wp + Pr, U, atol=1e-14)
    assert np.all(np.linalg.norm(Wp, axis=1) <= a + 1e-13)
    # Fenchel-Young: <prox_i, W+_i> = a_i ||prox_i||
    assert np.allclose(np.sum(Pr * Wp, axis=1), a * np.linalg.norm(Pr, axis=1), atol=1e-12)
    # one channel: clip(u, -a, a), the complement of soft-thresholding
    u = RNG.standard_normal((100, 1)) * 2
    assert np.allclose(prox.l21_prox_complement(u, a)[:, 0], np.clip(u[:, 0], -a, a))
    assert np.allclose(prox.l21_prox(u, a)[:, 0], prox.soft_threshold(u[:, 0], a))
    # zero row stays zero
    U[3] = 0
    assert np.all(prox.l21_prox_complement(U, a)[3] == 0)


# ---------------------------------------------------------------- steps

def _small_problem(ny=64, nx=72, L=5, qy=2, qx=3, o=6, C=1, warm=False, seed=0):
    g = np.random.default_rng(seed)
    X = np.abs(g.standard_normal((ny, nx, L)))
    geom = geometry.Geometry(ny, nx, qy, qx, o, o, 4)
    chans = step.subcube_channels(L, C)
    I = sara.n_coefficients(ny, nx, 4)
    P = [[(g.standard_normal(f.nuc_shape + (len(ch),)) * 0.1 if warm
           else np.zeros(f.nuc_shape + (len(ch),))) for f in geom.facets] for ch in chans]
    W = [g.standard_normal((I, len(ch))) * 0.1 if warm else np.zeros((I, len(ch))) for ch in chans]
    theta = [g.uniform(0.5, 1, I) for _ in chans]
    tbar = [[np.sort(g.uniform(0.5, 1, len(ch))) for _ in geom.facets] for ch in chans]
    return X, geom, P, W, theta, tbar


def test_l21_huge_threshold_returns_kappa_x():
    # theta -> infinity with W = 0: W+ = Psi^dagger X, kappa Psi W+ = kappa X
    X, geom, P, W, theta, tbar = _small_problem()
    Wn, G = step.l21_dual_update(X, W, [np.full_like(theta[0], 1e30)], [1.0], 1.0)
    assert np.allclose(G, X, atol=1e-12)
    Wn, G = step.l21_dual_update(X, W, [np.full_like(theta[0], 1e30)], [1.0], 2.0)
    assert np.allclose(G, 2.0 * X, atol=1e-12)               # kappa scales the synthesis


def test_nuclear_huge_threshold_returns_window_squares():
    # t -> infinity with P = 0: P+ = D_q S~_q X, gather = zeta sum_q S~_q^T D_q^2 S~_q X
    X, geom, P, W, theta, tbar = _small_problem()
    Pn, G = step.nuclear_dual_update(X, P, tbar, [[1e30] * geom.Q], 2.0, geom)
    d2 = np.zeros(X.shape[:2])
    for f in geom.facets:
        (y0, y1), (x0, x1) = f.nuc_window
        d2[y0:y1, x0:x1] += f.window() ** 2
    assert np.allclose(G, 2.0 * d2[..., None] * X, atol=1e-12)   # zeta scales the gather
    # zero thresholds: P+ = 0
    Pn, G = step.nuclear_dual_update(X, P, tbar, [[0.0] * geom.Q], 1.0, geom)
    assert np.allclose(G, 0.0)


def test_single_facet_is_hypersara_step():
    # Q = 1, C = 1 (Sec. 2.4.2): D = 1 and the nuclear update is the SVT of the
    # whole cube reshaped to N x L
    X, _, _, _, theta, _ = _small_problem()
    ny, nx, L = X.shape
    geom = geometry.Geometry(ny, nx, 1, 1, 0, 0, 4)
    P = [[np.zeros((ny, nx, L))]]
    t = np.sort(RNG.uniform(0.5, 1, L))
    Pn, G = step.nuclear_dual_update(X, P, [[t]], [[0.7]], 1.0, geom)
    U, s, Vt = np.linalg.svd(X.reshape(-1, L), full_matrices=False)
    ref = (U * np.minimum(s, 0.7 * t)) @ Vt
    assert np.allclose(Pn[0][0].reshape(-1, L), ref, atol=1e-12)
    assert np.allclose(G.reshape(-1, L), ref, atol=1e-12)


def test_sara_reduction_channel_separable():
    # C = L and mu_bar = 0 (Sec. 2.4.1): every channel is its own sub-problem,
    # the nuclear part vanishes and the l21 shrink becomes a per-channel clip
    X, geom, _, _, _, _ = _small_problem(L=4)
    L = X.shape[2]
    I = sara.n_coefficients(X.shape[0], X.shape[1], 4)
    W = [np.zeros((I, 1)) for _ in range(L)]
    theta = [np.full(I, 1.0) for _ in range(L)]
    P = [[np.zeros(f.nuc_shape + (1,)) for f in geom.facets] for _ in range(L)]
    tb = [[np.ones(1) for _ in geom.facets] for _ in range(L)]
    Pn, Wn, G = step.facet_prox_step(X, P, W, theta, tb, [0.05] * L, [[0.0] * geom.Q] * L,
                                     1.0, 1.0, geom, C=L)
    for l in range(L):
        A = sara.flatten(sara.analysis(X[..., l:l + 1], 4))
        assert np.allclose(Wn[l], np.clip(A, -0.05, 0.05), atol=1e-14)
        ref = sara.synthesis(sara.unflatten(np.clip(A, -0.05, 0.05), *X.shape[:2], 4), *X.shape[:2], 4)
        assert np.allclose(G[..., l:l + 1], ref, atol=1e-13)


def test_l21_facet_grid_invariance():
    # the faceted l21 update and its synthesis + overlap-add do not depend on
    # the facet grid (exact faceting, Sec. 2.4.2)
    X, _, _, W, theta, _ = _small_problem(ny=300, nx=260, L=3)
    Wn, G = step.l21_dual_update(X, W, theta, [0.2], 1.0)
    for grid in [(2, 2), (3, 2)]:
        geom = geometry.Geometry(300, 260, grid[0], grid[1], 0, 0, 4)
        Gf = sara.faceted_synthesis(sara.unflatten(Wn[0], 300, 260, 4), geom, 4)
        assert np.allclose(Gf, G, atol=1e-12)


def test_interleaved_subcubes():
    # sub-cube c holds channels c, c + C, ... (Sec. 2.4.1); sub-cubes are independent
    assert step.subcube_channels(10, 3) == [[0, 3, 6, 9], [1, 4, 7], [2, 5, 8]]
    X, geom, P, W, theta, tbar = _small_problem(L=6, C=2, warm=True)
    Pn, Wn, G = step.facet_prox_step(X, P, W, theta, tbar, [0.1, 0.2], [[0.5] * geom.Q, [0.3] * geom.Q],
                                     1.0, 1.0, geom, C=2)
    Pn1, Wn1, G1 = step.facet_prox_step(X[..., 1::2], [P[1]], [W[1]], [theta[1]], [tbar[1]], [0.2],
                                        [[0.3] * geom.Q], 1.0, 1.0, geom, C=1)
    assert np.allclose(G[..., 1::2], G1)
    assert np.allclose(Wn[1], Wn1[0])


def test_step_moreau_identities():
    # dual-update outputs satisfy the conjugate constraints: every singular
    # value of P+_q is <= its threshold and every row of W+ has norm <= a theta_i
    X, geom, P, W, theta, tbar = _small_problem(warm=True)
    mu, mub = [0.3], [[0.9] * geom.Q]
    Pn, Wn, G = step.facet_prox_step(X, P, W, theta, tbar, mu, mub, 1.0, 1.0, geom)
    for q, f in enumerate(geom.facets):
        s = sv(Pn[0][q].reshape(-1, X.shape[2]))
        assert np.all(s <= mub[0][q] * tbar[0][q][::-1] + 1e-12)
    assert np.all(np.linalg.norm(Wn[0], axis=1) <= mu[0] * theta[0] + 1e-12)


# ---------------------------------------------------------------- heuristics

def test_chi_constants():
    # closed forms k = 1 (half-normal), k = 2 (Rayleigh) and the m + s values used
    # by the heuristics; m + s -> sqrt(k) for large k (Sec. 2.3.2)
    m, s = heuristics.chi_mean_std(1)
    assert abs(m - np.sqrt(2 / np.pi)) < 1e-14 and abs(s - np.sqrt(1 - 2 / np.pi)) < 1e-14
    m, s = heuristics.chi_mean_std(2)
    assert abs(m - np.sqrt(np.pi / 2)) < 1e-14
    for k, ref in [(10, 3.7821), (12, 4.0922), (20, 5.1192), (60, 8.4194), (64, 8.6745), (100, 10.6813)]:
        m, s = heuristics.chi_mean_std(k)
        assert abs(m + s - ref) < 1e-4
        # Monte-Carlo check of the chi distribution itself
        smp = np.sqrt(np.random.default_rng(k).chisquare(k, 400000))
        assert abs(smp.mean() - m) < 5e-3 and abs(smp.std() - s) < 5e-3
    m, s = heuristics.chi_mean_std(1e6)
    assert abs((m + s) / np.sqrt(1e6) - 1) < 1e-3


def test_heuristic_parameters():
    assert heuristics.mu_low_rank(2.0, 1000, 20) == pytest.approx(2.0 * np.sqrt(1000))
    assert heuristics.mu_sparsity(0.5, 20) == pytest.approx(0.5 * 5.1192, abs=1e-4)


def test_reweighting_weights_range_and_order():
    X, geom, _, _, _, _ = _small_problem()
    ub = [[0.5] * geom.Q]
    tb = heuristics.nuclear_weights(X, geom, ub)
    for w in tb[0]:
        assert np.all((w > 0) & (w <= 1)) and np.all(np.diff(w) >= 0)
    th = heuristics.l21_weights(X, [0.05])
    assert np.all((th[0] > 0) & (th[0] <= 1))
    # zero image: all weights equal one
    th0 = heuristics.l21_weights(np.zeros_like(X), [0.05])
    assert np.all(th0[0] == 1.0)
