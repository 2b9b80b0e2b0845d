"""Pins of the oracle's sampled-block step (oracle/blocks.py) against the full
oracle step on problems small enough to run whole: for blocks at the corner,
an edge, the interior and the far corner, with warm duals and with random or
cube-derived weights, the block's P+, the W+ rows its facets own and G on its
exact tiles equal the full step's (Sec. 2.4.2: the step is local, and the
faceted transform equals the global one)."""
import numpy as np
import pytest

import synth
from oracle import blocks, geometry, heuristics, sara, step

LEVELS = 2
E = 48          # >= 15 (2^2 - 1): exact faceting at two levels


def _problem(C, seed):
    ny, nx, L, qy, qx, o = 200, 168, 4 * C, 4, 3, 10
    X = synth.blob_cube(ny, nx, L, 30, synth.BASE_SEED + 500 + seed)
    geom = geometry.Geometry(ny, nx, qy, qx, o, o, LEVELS, E=E)
    sb = synth.sigma_bar(X)
    Lc = L // C
    mu = np.array([heuristics.mu_sparsity(sb, Lc)] * C)
    mub = [[heuristics.mu_low_rank(sb, f.n_rows, Lc) for f in geom.facets] for _ in range(C)]
    return X, geom, mu, mub


def _offsets(ny, nx):
    shapes = sara.band_shapes(ny, nx, LEVELS)
    return shapes, np.concatenate([[0], np.cumsum([a * b for a, b in shapes])])


@pytest.mark.parametrize("where", ["corner", "edge", "interior", "far_corner"])
@pytest.mark.parametrize("weights", ["given", "from_cube"])
def test_block_equals_full_step(where, weights):
    C = 2
    X, geom, mu, mub = _problem(C, {"corner": 0, "edge": 1, "interior": 2, "far_corner": 3}[where])
    ny, nx, L = X.shape
    Lc = L // C
    sy0, sx0, ky, kx = {"corner": (0, 0, 2, 2), "edge": (1, 1, 2, 2), "interior": (1, 0, 2, 3),
                        "far_corner": (2, 1, 2, 2)}[where]
    blk = blocks.make_block(geom, sy0, sx0, ky, kx)
    shapes, offs = _offsets(ny, nx)
    I = int(offs[-1])
    Kx = [b for _, b in shapes]

    # warm duals from the counter-based generator, for the full problem and the block
    Pfull = [[synth.warm_p_np(c * geom.Q + f.index, f.n_rows * Lc, synth.warm_p_scale(mub[c][f.index], f.n_rows))
              .reshape(f.nuc_shape + (Lc,)) for f in geom.facets] for c in range(C)]
    pos = np.arange(L, dtype=np.int64)
    Wfull = synth.warm_w_np(np.arange(I, dtype=np.int64)[:, None], pos[None, :],
                            1.0)  # unit amplitude, scaled per sub-cube below
    Wfull = [Wfull[:, c * Lc:(c + 1) * Lc].astype(np.float64) * synth.warm_w_scale(mu[c]) for c in range(C)]
    Wfull = [w.astype(np.float32) for w in Wfull]

    def P0(c, f):
        return Pfull[c][f.index]

    def W0(rr, cc, k, c):
        i = offs[k] + rr * Kx[k] + cc
        return Wfull[c][i]

    if weights == "given":
        th_full = [synth.uniform_weights(I, 900 + c) for c in range(C)]
        tb_full = [[synth.sorted_weights(Lc, 950 + c * geom.Q + q) for q in range(geom.Q)] for c in range(C)]

        def theta(rr, cc, k, c):
            return th_full[c][offs[k] + rr * Kx[k] + cc]

        def theta_bar(c, f):
            return tb_full[c][f.index]
    else:
        th_full = heuristics.l21_weights(X, mu, levels=LEVELS, C=C)
        tb_full = heuristics.nuclear_weights(X, geom, mub, C=C)
        theta = theta_bar = None

    ref_P, ref_W, ref_G = step.facet_prox_step(X, Pfull, Wfull, th_full, tb_full, mu, mub, 1.0, 1.0, geom, C=C)
    got = blocks.block_step(X, geom, blk, C, mu, mub, P0=P0, W0=W0, theta=theta, theta_bar=theta_bar)

    facets = blk.facets(geom)
    assert len(facets) == ky * kx
    for c in range(C):
        for f in facets:
            np.testing.assert_array_equal(got["P"][(c, f.index)], ref_P[c][f.index])
    for k, ((r0, r1), (c0, c1)) in enumerate(got["owned"]):
        assert r1 > r0 and c1 > c0
        full = np.concatenate([ref_W[c][offs[k]:offs[k + 1]].reshape(shapes[k] + (Lc,)) for c in range(C)], axis=2)
        np.testing.assert_allclose(got["W"][k], full[r0:r1, c0:c1], rtol=1e-12, atol=1e-14 * mu[0], err_msg=str(k))
    (gy0, gy1), (gx0, gx1) = got["tile"]
    assert gy1 > gy0 and gx1 > gx0
    np.testing.assert_allclose(got["G"], ref_G[gy0:gy1, gx0:gx1], rtol=1e-11, atol=1e-13 * np.abs(ref_G).max())


def test_block_rectangles():
    """The owned rectangles of all facets tile every band, and the sub-image
    starts at a multiple of 2^levels at least E above / left of the block."""
    X, geom, mu, mub = _problem(1, 4)
    ny, nx, _ = X.shape
    shapes, _ = _offsets(ny, nx)
    cover = [np.zeros(s, dtype=int) for s in shapes]
    for sy in range(geom.qy):
        for sx in range(geom.qx):
            blk = blocks.make_block(geom, sy, sx, 1, 1)
            assert blk.y0 % (1 << LEVELS) == 0 and blk.x0 % (1 << LEVELS) == 0
            ty, tx = geometry.tile_bounds(ny, geom.qy), geometry.tile_bounds(nx, geom.qx)
            assert blk.y0 == 0 or blk.y0 <= ty[sy] - E
            assert blk.x0 == 0 or blk.x0 <= tx[sx] - E
            for k, ((r0, r1), (c0, c1)) in enumerate(blocks.owned_rects(geom, blk)):
                cover[k][r0:r1, c0:c1] += 1
    assert all(np.all(cv == 1) for cv in cover)
