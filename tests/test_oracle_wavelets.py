"""Pins of the oracle's Daubechies filters, DWT and SARA dictionary.

Every check here is fixed by mathematics or by the paper, not by the oracle
itself: closed-form filters, the orthonormality / moment conditions of the
Daubechies construction, the Haar special case, isometry and perfect
reconstruction (Sec. 2.3.1), the unit spectral norm used for kappa (Sec. 3.2),
and the faceting overlap range printed in Sec. 2.4.2.
"""
import json
import os
from math import sqrt

import numpy as np
import pytest

from oracle import dwt, filters, geometry, sara

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------- filters

def test_db1_db2_db3_closed_forms():
    # Haar and Daubechies' closed forms for N = 2, 3 (Daubechies 1988)
    assert np.allclose(filters.lowpass(1), [1 / sqrt(2), 1 / sqrt(2)], atol=1e-15)
    s3 = sqrt(3.0)
    db2 = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * sqrt(2))
    assert np.allclose(filters.lowpass(2), db2, atol=1e-15)
    r = sqrt(10.0)
    q = sqrt(5 + 2 * r)
    db3 = sqrt(2) / 32 * np.array([1 + r + q, 5 + r + 3 * q, 10 - 2 * r + 2 * q,
                                   10 - 2 * r - 2 * q, 5 + r - 3 * q, 1 + r - q])
    assert np.allclose(filters.lowpass(3), db3, atol=1e-14)


@pytest.mark.parametrize("N", range(1, 9))
def test_daubechies_conditions(N):
    h = filters.lowpass(N)
    g = filters.highpass(h)
    L = len(h)
    assert L == 2 * N
    assert abs(h.sum() - sqrt(2)) < 1e-14
    # double-shift orthonormality of h, of g, and h _|_ g
    for k in range(N):
        hh = sum(h[m] * h[m + 2 * k] for m in range(L - 2 * k))
        gg = sum(g[m] * g[m + 2 * k] for m in range(L - 2 * k))
        assert abs(hh - (k == 0)) < 1e-14 and abs(gg - (k == 0)) < 1e-14
    for k in range(-N + 1, N):
        hg = sum(h[m] * g[m + 2 * k] for m in range(L) if 0 <= m + 2 * k < L)
        assert abs(hg) < 1e-14
    # N vanishing moments of the wavelet: sum_m (-1)^m m^p h[m] = 0, p < N
    for p in range(N):
        mom = sum((-1) ** m * float(m) ** p * h[m] for m in range(L))
        assert abs(mom) < 1e-12 * max(1.0, float(L) ** p)
    # power-complementarity |m0(w)|^2 + |m0(w + pi)|^2 = 1
    w = np.linspace(0, np.pi, 257)
    m0 = lambda om: np.abs(np.exp(-1j * np.outer(om, np.arange(L))) @ h) ** 2 / 2
    assert np.max(np.abs(m0(w) + m0(w + np.pi) - 1)) < 1e-13


@pytest.mark.parametrize("N", range(2, 9))
def test_extremal_phase(N):
    # all zeros of sum_n h[n] z^n other than z = -1 lie strictly outside the unit
    # circle, i.e. the extremal-phase factor of Daubechies' construction
    h = filters.lowpass(N)
    # divide out the N-fold zero at z = -1 (descending powers for np.polydiv)
    q, r = np.polydiv(h[::-1], np.poly1d([1.0, 1.0]) ** N)
    assert np.max(np.abs(r)) < 1e-12
    zz = np.roots(q)
    assert len(zz) == N - 1 and np.all(np.abs(zz) > 1.0 + 1e-9)
    # and the energy is front-loaded (partial-energy property)
    e = np.cumsum(h ** 2)
    er = np.cumsum(h[::-1] ** 2)
    assert np.all(e >= er - 1e-14)


# ---------------------------------------------------------------- DWT

def test_haar_special_case():
    # db1 with n = 2^d: the level-d ll band is the sum over 2^d x 2^d blocks / 2^d
    rng = np.random.default_rng(1)
    x = rng.standard_normal((32, 48))
    h, g = filters.lowpass(1), filters.highpass(filters.lowpass(1))
    bands = dwt.wavedec2(x, h, g, 4)
    ll = bands[-1]
    ref = x.reshape(2, 16, 3, 16).sum(axis=(1, 3)) / 16
    assert np.allclose(ll, ref, atol=1e-13)
    # level-1 hh on 2x2 blocks [[a, b], [c, d]] is (a - b - c + d) / 2
    hh = bands[2]
    blk = x.reshape(16, 2, 24, 2)
    ref = (blk[:, 0, :, 0] - blk[:, 0, :, 1] - blk[:, 1, :, 0] + blk[:, 1, :, 1]) / 2
    assert np.allclose(hh, ref, atol=1e-13)


@pytest.mark.parametrize("N", [2, 5, 8])
def test_vanishing_moments_kill_polynomials(N):
    # detail coefficients whose support lies inside the signal vanish for
    # polynomials of degree < N
    h = filters.lowpass(N)
    g = filters.highpass(h)
    n = 64
    t = np.arange(n, dtype=np.float64) / n
    x = sum(t ** p for p in range(N))
    d = dwt.analysis_axis(x, g, 0)
    L = 2 * N
    interior = [k for k in range(len(d)) if 2 * k + 1 - (L - 1) >= 0 and 2 * k + 1 < n]
    assert np.max(np.abs(d[interior])) < 1e-10
    edge = [k for k in range(len(d)) if k not in interior]
    assert np.max(np.abs(d[edge])) > 1e-6     # zero extension creates edge details


@pytest.mark.parametrize("shape", [(7, 8), (33, 20), (40, 57)])
def test_sara_isometry_and_reconstruction(shape):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(shape + (3,))
    b = sara.analysis(x, 4)
    assert len(b) == 8 * 13 + 1
    energy = sum(float((bb ** 2).sum()) for bb in b)
    assert abs(energy - float((x ** 2).sum())) < 1e-12 * float((x ** 2).sum())
    assert np.max(np.abs(sara.synthesis(b, *shape, 4) - x)) < 1e-13
    # adjoint dot test <Psi^dagger x, w> = <x, Psi w>
    w = [rng.standard_normal(bb.shape) for bb in b]
    lhs = sum(float((bb * ww).sum()) for bb, ww in zip(b, w))
    rhs = float((x * sara.synthesis(w, *shape, 4)).sum())
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_spectral_norm_is_one_power_method():
    # kappa = 1 / ||Psi^dagger||_S^2 = 1 (Sec. 3.2); power method as in the
    # footnote of Sec. 2.3.1 (relative variation < 1e-4, <= 100 iterations)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((24, 30))
    val = 0.0
    for _ in range(100):
        x = x / np.linalg.norm(x)
        y = sara.synthesis(sara.analysis(x, 4), 24, 30, 4)
        new = float((x * y).sum())
        if abs(new - val) < 1e-4 * abs(new):
            val = new
            break
        val, x = new, y
    assert abs(1.0 / val - GOLDEN["kappa"]["value"]) < 1e-12


def test_coefficient_count():
    # I = sum over bands; the Dirac basis contributes N, every wavelet basis
    # at least N (expansive transform)
    ny, nx = 256, 256
    I = sara.n_coefficients(ny, nx, 4)
    shapes = sara.band_shapes(ny, nx, 4)
    assert len(shapes) == GOLDEN["sara_bases"]["value"] * 13 - 12
    assert shapes[-1] == (ny, nx)
    assert I == 650484          # 9.926 N for 256 x 256, db1..db8 at 4 levels


# ---------------------------------------------------------------- faceting

@pytest.mark.parametrize("grid", [(2, 2), (3, 2)])
def test_faceted_sara_equals_global(grid):
    rng = np.random.default_rng(4)
    ny, nx = 300, 260
    x = rng.standard_normal((ny, nx, 2))
    geom = geometry.Geometry(ny, nx, grid[0], grid[1], 0, 0, 4, E=225)
    A = sara.analysis(x, 4)
    Af = sara.faceted_analysis(x, geom, 4)
    assert max(float(np.max(np.abs(a - b))) for a, b in zip(A, Af)) == 0.0
    Y = sara.synthesis(A, ny, nx, 4)
    Yf = sara.faceted_synthesis(A, geom, 4)
    assert np.max(np.abs(Y - Yf)) < 1e-12


def _min_exact_E(n, Q):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, 16))
    A = sara.analysis(x, 4)

    def exact(E):
        g = geometry.Geometry(n, 16, Q, 1, 0, 0, 4, E=E)
        return max(float(np.max(np.abs(a - b)))
                   for a, b in zip(A, sara.faceted_analysis(x, g, 4))) == 0.0
    lo, hi = 0, 260
    while lo < hi:
        mid = (lo + hi) // 2
        if exact(mid):
            hi = mid
        else:
            lo = mid + 1
    return lo, exact


@pytest.mark.slow
@pytest.mark.parametrize("n", [1024, 1030, 1054])
def test_minimal_overlap_matches_paper_range(n):
    # Sec. 2.4.2: the overlap that makes faceting exact lies between
    # 15(2^d - 2) and 15(2^d - 1) pixels (d = 4 -> [210, 225]); with the causal
    # zero-extended convention it is 210 + (t mod 16) for a tile start t.
    rng_vals = GOLDEN["faceted_overlap_db8"]
    E, exact = _min_exact_E(n, 2)
    t = n // 2
    assert rng_vals["min"] <= E <= rng_vals["max"]
    assert E == 210 + t % 16
    assert not exact(E - 1)


def test_window_partition_of_unity():
    for (ny, nx, qy, qx, o) in [(256, 256, 2, 2, 32), (1024, 2048, 4, 4, 64), (100, 90, 3, 4, 7),
                                (64, 64, 4, 4, 0)]:
        g = geometry.Geometry(ny, nx, qy, qx, o, o)
        s = g.window_sum()
        assert np.max(np.abs(s - 1.0)) < 1e-15
        for f in g.facets:
            assert np.all(f.window() > 0)
            (ty0, ty1), (tx0, tx1) = f.tile
            (wy0, wy1), (wx0, wx1) = f.nuc_window
            # facets extend toward top/left only; edge facets keep the tile size
            assert wy1 == ty1 and wx1 == tx1
            assert wy0 == (ty0 - o if f.sy > 0 else ty0)
            assert wx0 == (tx0 - o if f.sx > 0 else tx0)
            if o == 0:
                assert np.all(f.window() == 1.0)


def test_ownership_partitions_every_band():
    g = geometry.Geometry(300, 260, 3, 2, 10, 10)
    shapes = sara.band_shapes(300, 260, 4)
    cover = [np.zeros(s, dtype=int) for s in shapes]
    for f in g.facets:
        for k, ((y0, y1), (x0, x1)) in enumerate(g.owned_rects(f)):
            cover[k][y0:y1, x0:x1] += 1
    assert all(np.all(c == 1) for c in cover)
