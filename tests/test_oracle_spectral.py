"""Pins of the overlapping spectral facets (oracle.spectral, the 100-channel
case read literally: the spatial overlap rule of Sec. 2.4.2 applied along the
spectral axis).

* the spectral windows cover every channel with weights summing to one, and
  extend o channels before each block but the first;
* no overlap: the plain step on contiguous sub-cubes, i.e. the plain
  (interleaved) step on the channel-permuted cube;
* one block: the plain step;
* a spatially and spectrally separable rank-one cube: every facet matrix is
  (D_q a)(d_c b)^T, whose singular value is known in closed form;
* the nuclear aggregation is the exact adjoint of the facet extraction.
"""
import numpy as np
import pytest

import synth
from oracle import geometry, sara, spectral, step

RNG = np.random.default_rng(29)


@pytest.mark.parametrize("L,C,o", [(100, 10, 2), (24, 3, 4), (7, 2, 1), (12, 4, 0)])
def test_spectral_windows_partition_unity(L, C, o):
    acc = np.zeros(L)
    blocks = spectral.block_channels(L, C)
    for c in range(C):
        chans, w = spectral.spectral_window(L, C, c, o)
        assert chans[-1] == blocks[c][-1]
        assert chans[0] == (blocks[c][0] - o if c > 0 else 0)
        assert np.all(w > 0)
        acc[chans] += w
    assert np.max(np.abs(acc - 1.0)) < 1e-15
    assert sorted(sum(blocks, [])) == list(range(L))


def make(C, Lb, o, seed=4, ny=48, nx=40):
    L = C * Lb
    geom = geometry.Geometry(ny, nx, 2, 2, 6, 5, 2)
    X = synth.blob_cube(ny, nx, L, 10, seed)
    I = sara.n_coefficients(ny, nx, 2)
    wins = [spectral.spectral_window(L, C, c, o)[0] for c in range(C)]
    P = [[0.05 * RNG.standard_normal(f.nuc_shape + (len(wins[c]),)) for f in geom.facets] for c in range(C)]
    W = [0.02 * RNG.standard_normal((I, Lb)) for _ in range(C)]
    theta = [synth.uniform_weights(I, seed + c) for c in range(C)]
    tbar = [[synth.sorted_weights(len(wins[c]), 60 + c * geom.Q + q) for q in range(geom.Q)] for c in range(C)]
    mu = 0.03 * (1.0 + 0.2 * np.arange(C))
    mub = 0.3 * (1.0 + 0.1 * np.arange(C * geom.Q)).reshape(C, geom.Q)
    return geom, X, P, W, theta, tbar, mu, mub


def test_no_overlap_is_the_plain_step_on_permuted_channels():
    C, Lb = 3, 4
    L = C * Lb
    geom, X, P, W, theta, tbar, mu, mub = make(C, Lb, 0)
    Pb, Wb, Gb = spectral.facet_prox_step(X, P, W, theta, tbar, mu, mub, 0.9, 1.1, geom, C, 0)
    # interleaved sub-cube c of the permuted cube = contiguous block c
    perm = np.empty(L, dtype=int)
    for c in range(C):
        for l in range(Lb):
            perm[c + l * C] = c * Lb + l
    Pi, Wi, Gi = step.facet_prox_step(X[..., perm], P, W, theta, tbar, mu, mub, 0.9, 1.1, geom, C=C)
    for c in range(C):
        for q in range(geom.Q):
            assert np.allclose(Pb[c][q], Pi[c][q], rtol=0, atol=1e-13)
        assert np.allclose(Wb[c], Wi[c], rtol=0, atol=1e-13)
    assert np.allclose(Gb[..., perm], Gi, rtol=0, atol=1e-12)


def test_one_block_is_the_plain_step():
    geom, X, P, W, theta, tbar, mu, mub = make(1, 6, 3)
    Pb, Wb, Gb = spectral.facet_prox_step(X, P, W, theta, tbar, mu, mub, 1.0, 1.0, geom, 1, 3)
    Pp, Wp, Gp = step.facet_prox_step(X, P, W, theta, tbar, mu, mub, 1.0, 1.0, geom, C=1)
    for q in range(geom.Q):
        assert np.allclose(Pb[0][q], Pp[0][q], rtol=0, atol=1e-13)
    assert np.allclose(Wb[0], Wp[0], rtol=0, atol=1e-13)
    assert np.allclose(Gb, Gp, rtol=0, atol=1e-12)


def test_separable_rank_one_cube():
    C, Lb, o = 3, 5, 2
    L = C * Lb
    ny, nx = 48, 40
    geom = geometry.Geometry(ny, nx, 2, 2, 6, 5, 2)
    a = RNG.random((ny, nx)) + 0.1
    b = RNG.random(L) + 0.5
    X = a[..., None] * b[None, None, :]
    I = sara.n_coefficients(ny, nx, 2)
    wins = [spectral.spectral_window(L, C, c, o) for c in range(C)]
    P = [[np.zeros(f.nuc_shape + (len(wins[c][0]),)) for f in geom.facets] for c in range(C)]
    W = [np.zeros((I, Lb)) for _ in range(C)]
    tbar = [[np.ones(len(wins[c][0])) for _ in geom.facets] for c in range(C)]
    t = 0.25
    Pn, _, _ = spectral.facet_prox_step(X, P, W, [np.ones(I)] * C, tbar, np.zeros(C), np.full((C, geom.Q), t),
                                        1.0, 1.0, geom, C, o)
    for c in range(C):
        chans, w = wins[c]
        for q, f in enumerate(geom.facets):
            (y0, y1), (x0, x1) = f.nuc_window
            u = (f.window() * a[y0:y1, x0:x1]).reshape(-1)
            v = w * b[chans]
            s1 = np.linalg.norm(u) * np.linalg.norm(v)
            assert s1 > t
            assert np.allclose(Pn[c][q].reshape(-1, len(chans)), (t / s1) * np.outer(u, v), rtol=0, atol=1e-13)


def test_nuclear_aggregation_is_the_adjoint_of_the_extraction():
    C, Lb, o = 3, 4, 2
    geom, X, P, W, theta, tbar, mu, mub = make(C, Lb, o)
    zeta = 0.7
    # mu = 0: W+ = 0, so G is the nuclear aggregation of P+ alone
    Pn, Wn, G = spectral.facet_prox_step(X, P, W, theta, tbar, np.zeros(C), mub, zeta, 1.0, geom, C, o)
    assert all(np.all(w == 0) for w in Wn)
    Y = RNG.standard_normal(X.shape)
    L = X.shape[2]
    rhs = 0.0
    for c in range(C):
        chans, w = spectral.spectral_window(L, C, c, o)
        for q, f in enumerate(geom.facets):
            rhs += zeta * np.sum(Pn[c][q].reshape(-1, len(chans)) * spectral.facet_matrix(Y, f, chans, w))
    assert abs(np.sum(G * Y) - rhs) <= 1e-11 * max(1.0, abs(rhs))
