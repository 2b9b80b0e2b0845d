"""Value pins of the oracle's reweighting weights (eqs. facet_hypersara_rank
and facet_hypersara_sparsity): closed forms on rank-one cubes and single
deltas, and identities that tie the weights back to the cube by another
route (sum of squared singular values = Frobenius norm of the windowed facet;
sum of squared coefficient-row norms = ||X||^2, the SARA dictionary being an
isometry).  Chosen so that a facet-index mix-up of upsilon_bar_{c,q}, a
missing window D_q, a wrong sub-cube's channels or a missing 1/3 all fail."""
import numpy as np
import pytest

import synth
from oracle import geometry, heuristics, sara


def _rank_one(ny, nx, b, seed):
    a = synth.rng(seed).uniform(0.1, 1.0, (ny, nx))
    return a, a[..., None] * np.asarray(b, dtype=np.float64)[None, None, :]


def test_rank_one_single_facet():
    """X = a b^T with one facet (Q = 1, D = 1): one singular value ||a|| ||b||,
    the others 0, so theta_bar = (ub / (||a|| ||b|| + ub), 1, ..., 1)."""
    b = np.array([0.3, 1.0, 0.7, 0.2, 0.5])
    a, X = _rank_one(12, 9, b, 1)
    geom = geometry.Geometry(12, 9, 1, 1, 0, 0, 2)
    ub = 0.37
    tb = heuristics.nuclear_weights(X, geom, [[ub]])[0][0]
    s1 = np.linalg.norm(a) * np.linalg.norm(b)
    assert tb[0] == pytest.approx(ub / (s1 + ub), rel=1e-13)
    np.testing.assert_allclose(tb[1:], 1.0, rtol=0, atol=1e-13)


def test_rank_one_windowed_facets_distinct_upsilon():
    """Two interleaved sub-cubes X_c = a b_c^T on a 3 x 2 facet grid with
    overlap: facet (c, q) sees (D_q a_q) b_c^T, whose one singular value is
    ||D_q a_q|| ||b_c||; every (c, q) has its own upsilon_bar."""
    L, C = 6, 2
    b = np.array([0.9, 0.2, 0.4, 1.1, 0.6, 0.3])
    a, X = _rank_one(30, 22, b, 2)
    geom = geometry.Geometry(30, 22, 3, 2, 4, 3, 2)
    ub = [[0.05 + 0.1 * (c * geom.Q + q) for q in range(geom.Q)] for c in range(C)]
    tb = heuristics.nuclear_weights(X, geom, ub, C=C)
    for c in range(C):
        bc = b[c::C]
        for q, f in enumerate(geom.facets):
            (y0, y1), (x0, x1) = f.nuc_window
            s1 = np.linalg.norm(f.window() * a[y0:y1, x0:x1]) * np.linalg.norm(bc)
            u = ub[c][q]
            assert tb[c][q][0] == pytest.approx(u / (s1 + u), rel=1e-12), (c, q)
            np.testing.assert_allclose(tb[c][q][1:], 1.0, rtol=0, atol=1e-12)


def test_nuclear_weights_sum_of_squares():
    """On a generic cube, sigma_j = ub (1 / theta_bar_j - 1) recovers the
    singular values of D_q S~_q X_c: their squares sum to its Frobenius norm,
    computed directly from the windowed pixels of the sub-cube's channels."""
    C, L = 2, 8
    X = synth.blob_cube(40, 36, L, 10, synth.BASE_SEED + 31).astype(np.float64)
    geom = geometry.Geometry(40, 36, 2, 3, 6, 5, 2)
    ub = [[1e-3 * (1 + c + 0.5 * q) for q in range(geom.Q)] for c in range(C)]
    tb = heuristics.nuclear_weights(X, geom, ub, C=C)
    for c in range(C):
        for q, f in enumerate(geom.facets):
            (y0, y1), (x0, x1) = f.nuc_window
            fro2 = np.sum((f.window()[..., None] * X[y0:y1, x0:x1, c::C]) ** 2)
            sig = ub[c][q] * (1.0 / tb[c][q] - 1.0)
            assert np.all(np.diff(sig) <= 1e-12 * sig[0])     # descending singular values
            assert np.sum(sig ** 2) == pytest.approx(fro2, rel=1e-9), (c, q)


def test_l21_weights_dirac_rows():
    """Dirac basis (identity / 3, Sec. 2.3.1): the weight of pixel i is
    upsilon / (||x_i|| / 3 + upsilon) over the sub-cube's channels."""
    C, L = 2, 6
    X = synth.blob_cube(20, 18, L, 6, synth.BASE_SEED + 32).astype(np.float64)
    ups = [0.02, 0.005]
    th = heuristics.l21_weights(X, ups, levels=2, C=C)
    I = sara.n_coefficients(20, 18, 2)
    for c in range(C):
        r = np.linalg.norm(X[..., c::C], axis=2).reshape(-1) / 3.0
        np.testing.assert_allclose(th[c][I - 20 * 18:], ups[c] / (r + ups[c]), rtol=1e-13)


def test_l21_weights_haar_delta():
    """A single delta x = delta_(y0, x0) b: the db1 (Haar) coefficients at level
    j are +-2^-j at (y0 >> j, x0 >> j) in each detail band (and 2^-J in the last
    low-low band), zero elsewhere, so those rows get upsilon / (2^-j ||b|| / 3 +
    upsilon) and every other db1 row gets 1."""
    ny, nx, L, J = 16, 12, 3, 3
    y0, x0 = 9, 6
    b = np.array([0.5, 1.2, 0.8])
    X = np.zeros((ny, nx, L))
    X[y0, x0] = b
    ups = 0.04
    th = heuristics.l21_weights(X, [ups], levels=J)[0]
    shapes = sara.band_shapes(ny, nx, J)
    off = 0
    for k in range(3 * J + 1):                      # db1: (lh, hl, hh) per level, then ll
        Ky, Kx = shapes[k]
        j = k // 3 + 1 if k < 3 * J else J
        want = np.ones((Ky, Kx))
        r = 2.0 ** -j * np.linalg.norm(b) / 3.0
        want[y0 >> j, x0 >> j] = ups / (r + ups)
        np.testing.assert_allclose(th[off:off + Ky * Kx].reshape(Ky, Kx), want, rtol=1e-13, err_msg=str(k))
        off += Ky * Kx


def test_l21_weights_isometry():
    """r_i = upsilon (1 / theta_i - 1) recovers the coefficient-row norms of
    Psi^dagger X_c; the dictionary is an isometry (Psi Psi^dagger = I, Sec.
    2.3.1), so sum_i r_i^2 = ||X_c||_F^2 for each sub-cube."""
    C, L = 2, 6
    X = synth.blob_cube(24, 20, L, 8, synth.BASE_SEED + 33).astype(np.float64)
    ups = [1e-4, 3e-4]
    th = heuristics.l21_weights(X, ups, levels=3, C=C)
    for c in range(C):
        r = ups[c] * (1.0 / th[c].astype(np.float64) - 1.0)
        assert np.sum(r ** 2) == pytest.approx(np.sum(X[..., c::C] ** 2), rel=1e-8), c
