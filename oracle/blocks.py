"""The facet step on a sampled block of facets of a full-size problem (oracle).

TEST INFRASTRUCTURE ONLY.

A full-size cube (4096 x 4096 x 64 and the like) is beyond a plain FP64 oracle
in memory and time, but the step is local (Sec. 2.4.2): a facet's nuclear dual
depends only on its own window, the coefficients a facet owns depend only on
its SARA window (the faceted transform equals the global one), and the
gradient on a tile gathers only the facets whose windows cover it and the
coefficients owned by the tile's facet and its right / bottom neighbours (the
causal convention makes every dependency point to lower indices).  For a block
of ky x kx facets starting at facet (sy0, sx0) this module therefore computes,
exactly as the full problem would:

* P+ of every facet of the block (its full-problem window and apodisation);
* W+ of every coefficient row owned by a facet of the block;
* G on the tiles of the block whose right and bottom neighbours are in the
  block or outside the image.

The l21 part runs on a sub-image that starts at least E pixels above / left
of the block's first tile, at a multiple of 2^levels (so that the
sub-image's coefficient grids line up with the global ones: coefficient k of
level j of the sub-image is global coefficient k + y0 / 2^j), and ends at the
block's last tile.

Warm duals and the reweighting weights are supplied as callables, or the
weights are computed here from the cube (eqs. facet_hypersara_rank and
facet_hypersara_sparsity with upsilon = mu and upsilon_bar = mu_bar), exact on
everything compared.
"""
from dataclasses import dataclass
from types import SimpleNamespace

import numpy as np

from . import geometry, heuristics, prox, sara, step
from .filters import sara_filters


@dataclass
class Block:
    sy0: int
    sx0: int
    ky: int
    kx: int
    y0: int      # sub-image rows [y0, y1), columns [x0, x1)
    y1: int
    x0: int
    x1: int

    def facets(self, geom):
        return [f for f in geom.facets
                if self.sy0 <= f.sy < self.sy0 + self.ky and self.sx0 <= f.sx < self.sx0 + self.kx]


def make_block(geom, sy0, sx0, ky, kx):
    """The block of facets [sy0, sy0 + ky) x [sx0, sx0 + kx) and its sub-image."""
    if not (0 <= sy0 and sy0 + ky <= geom.qy and 0 <= sx0 and sx0 + kx <= geom.qx and ky > 0 and kx > 0):
        raise ValueError("block outside the facet grid")
    ty, tx = geometry.tile_bounds(geom.ny, geom.qy), geometry.tile_bounds(geom.nx, geom.qx)
    a = 1 << geom.levels

    def start(t):
        return 0 if t == 0 else max(0, (t - geom.E) // a * a)

    return Block(sy0, sx0, ky, kx, start(ty[sy0]), ty[sy0 + ky], start(tx[sx0]), tx[sx0 + kx])


def owned_rects(geom, blk):
    """Per band (storage order): the global rectangle of coefficients owned by
    the block's facets ((r0, r1), (c0, c1))."""
    rects = []
    for h, _ in sara_filters():
        oy = geometry.ownership_1d(geom.ny, geom.qy, len(h), geom.levels)
        ox = geometry.ownership_1d(geom.nx, geom.qx, len(h), geom.levels)
        for j in range(geom.levels):
            r = ((oy[j][blk.sy0], oy[j][blk.sy0 + blk.ky]), (ox[j][blk.sx0], ox[j][blk.sx0 + blk.kx]))
            rects += [r] * 3
        j = geom.levels - 1
        rects.append(((oy[j][blk.sy0], oy[j][blk.sy0 + blk.ky]), (ox[j][blk.sx0], ox[j][blk.sx0 + blk.kx])))
    ty, tx = geometry.tile_bounds(geom.ny, geom.qy), geometry.tile_bounds(geom.nx, geom.qx)
    rects.append(((ty[blk.sy0], ty[blk.sy0 + blk.ky]), (tx[blk.sx0], tx[blk.sx0 + blk.kx])))
    return rects


def band_levels(levels):
    """Level of every band in storage order (0 for the Dirac band)."""
    out = []
    for _ in range(8):
        out += [j + 1 for j in range(levels) for _ in range(3)] + [levels]
    return out + [0]


def exact_tile_rect(geom, blk):
    """Pixels ((r0, r1), (c0, c1)) on which G is exact: the block's tiles
    except its last row / column of tiles, unless those end at the image."""
    ty, tx = geometry.tile_bounds(geom.ny, geom.qy), geometry.tile_bounds(geom.nx, geom.qx)
    ey = blk.sy0 + blk.ky if blk.sy0 + blk.ky == geom.qy else blk.sy0 + blk.ky - 1
    ex = blk.sx0 + blk.kx if blk.sx0 + blk.kx == geom.qx else blk.sx0 + blk.kx - 1
    return (ty[blk.sy0], ty[ey]), (tx[blk.sx0], tx[ex])


def _sub_image(X, blk):
    return np.asarray(X[blk.y0:blk.y1, blk.x0:blk.x1], dtype=np.float64)


def block_weights(X, geom, blk, C, upsilon, upsilon_bar):
    """Reweighting weights from the cube X = X^(t) (eqs. facet_hypersara_rank
    and facet_hypersara_sparsity), exact for the block's facets and owned
    rows, as the callables block_step takes: theta(rows, cols, band, c) at
    global band positions (computed on the sub-image) and theta_bar(c, f).
    upsilon (C,); upsilon_bar [C][Q]."""
    facets = blk.facets(geom)
    tb = heuristics.nuclear_weights(X, SimpleNamespace(facets=facets),
                                    [[upsilon_bar[c][f.index] for f in facets] for c in range(C)], C=C)
    tb_of = {(c, f.index): tb[c][i] for c in range(C) for i, f in enumerate(facets)}
    Xs = _sub_image(X, blk)
    shapes = sara.band_shapes(Xs.shape[0], Xs.shape[1], geom.levels)
    lev = band_levels(geom.levels)
    th = heuristics.l21_weights(Xs, upsilon, levels=geom.levels, C=C)
    offs = np.concatenate([[0], np.cumsum([a * b for a, b in shapes])])
    bands = [[th[c][offs[k]:offs[k + 1]].reshape(shapes[k]) for k in range(len(shapes))] for c in range(C)]

    def theta(rr, cc, k, c):
        j = lev[k]
        return bands[c][k][rr - (blk.y0 >> j), cc - (blk.x0 >> j)]

    def theta_bar(c, f):
        return tb_of[(c, f.index)]

    return theta, theta_bar


def block_step(X, geom, blk, C, mu, mu_bar, zeta=1.0, kappa=1.0, P0=None, W0=None, theta=None, theta_bar=None):
    """The facet step restricted to a block (see the module docstring).

    X: the full cube (ny, nx, L); mu (C,); mu_bar [C][Q] (full facet order).
    P0(c, f) -> initial P of facet f (array nuc_shape + (L_c,)), or None: zero.
    W0(rows, cols, band, c) -> initial W of sub-cube c at the global band
      positions (rows, cols) (2-D index arrays; returns (..., L_c)), or None: zero.
    theta(rows, cols, band, c) -> l21 weights at global band positions, or
      None: computed from X with upsilon = mu (eq. facet_hypersara_sparsity).
    theta_bar(c, f) -> nuclear weights of facet f, or None: computed from X
      with upsilon_bar = mu_bar (eq. facet_hypersara_rank).  (block_weights
      gives both as callables, so that they can be computed apart.)

    Returns dict(P={(c, f.index): P+}, W=[per band: (rows, cols, L) array of
    W+ over the owned rectangle, channel positions c L_c + l], G=(rows, cols,
    L) over exact_tile_rect, theta_bar={(c, f.index): weights used},
    owned=owned_rects(...), tile=exact_tile_rect(...)).
    """
    X = np.asarray(X)
    L = X.shape[2]
    Lc = L // C
    chans = step.subcube_channels(L, C)
    levels = geom.levels
    facets = blk.facets(geom)
    out = dict(P={}, theta_bar={}, owned=owned_rects(geom, blk), tile=exact_tile_rect(geom, blk))
    (gy0, gy1), (gx0, gx1) = out["tile"]
    G = np.zeros((gy1 - gy0, gx1 - gx0, L))

    if theta is None or theta_bar is None:
        th_f, tb_f = block_weights(X, geom, blk, C, mu, mu_bar)
        theta = th_f if theta is None else theta
        theta_bar = tb_f if theta_bar is None else theta_bar

    # nuclear duals of the block's facets (Alg. 2 nuclear dual update)
    theta_bar_of = {(c, f.index): np.asarray(theta_bar(c, f), dtype=np.float64) for c in range(C) for f in facets}
    for c in range(C):
        for f in facets:
            shape = f.nuc_shape + (Lc,)
            Z = step.facet_matrix(X, f, chans[c])
            if P0 is not None:
                Z = Z + np.asarray(P0(c, f), dtype=np.float64).reshape(-1, Lc)
            t = (mu_bar[c][f.index] / zeta) * theta_bar_of[(c, f.index)]
            Pn = prox.weighted_svt_complement(Z, t).reshape(shape)
            out["P"][(c, f.index)] = Pn
            out["theta_bar"][(c, f.index)] = theta_bar_of[(c, f.index)]
            # facet back-projection onto the exact tiles
            (y0, y1), (x0, x1) = f.nuc_window
            a0, a1, b0, b1 = max(y0, gy0), min(y1, gy1), max(x0, gx0), min(x1, gx1)
            if a0 < a1 and b0 < b1:
                part = zeta * f.window()[..., None] * Pn
                G[a0 - gy0:a1 - gy0, b0 - gx0:b1 - gx0, chans[c]] += part[a0 - y0:a1 - y0, b0 - x0:b1 - x0]

    # l21 duals on the sub-image (Alg. 2 l21 dual update), then its synthesis
    Xs = _sub_image(X, blk)
    sny, snx = Xs.shape[:2]
    sub_shapes = sara.band_shapes(sny, snx, levels)
    lev = band_levels(levels)
    Isub = sum(a * b for a, b in sub_shapes)

    def sub_index(k):
        """Global (rows, cols) index grids of every position of band k of the sub-image."""
        j = lev[k]
        ry, rx = np.arange(sub_shapes[k][0]) + (blk.y0 >> j), np.arange(sub_shapes[k][1]) + (blk.x0 >> j)
        return np.meshgrid(ry, rx, indexing="ij")

    W = []
    thetas = []
    for c in range(C):
        wc = np.zeros((Isub, Lc))
        tc = np.zeros(Isub)
        off = 0
        for k, (a, b) in enumerate(sub_shapes):
            rr, cc = sub_index(k)
            if W0 is not None:
                wc[off:off + a * b] = np.asarray(W0(rr, cc, k, c), dtype=np.float64).reshape(a * b, Lc)
            tc[off:off + a * b] = np.asarray(theta(rr, cc, k, c), dtype=np.float64).reshape(a * b)
            off += a * b
        W.append(wc)
        thetas.append(tc)
    Wn, Gs = step.l21_dual_update(Xs, W, thetas, mu, kappa, levels, C=C)
    G += Gs[gy0 - blk.y0:gy1 - blk.y0, gx0 - blk.x0:gx1 - blk.x0]

    # W+ over the owned rectangles, in global coordinates
    out["W"] = []
    off = 0
    for k, (a, b) in enumerate(sub_shapes):
        j = lev[k]
        (r0, r1), (c0, c1) = out["owned"][k]
        s0, s1 = r0 - (blk.y0 >> j), r1 - (blk.y0 >> j)
        t0, t1 = c0 - (blk.x0 >> j), c1 - (blk.x0 >> j)
        assert 0 <= s0 <= s1 <= a and 0 <= t0 <= t1 <= b, (k, out["owned"][k], (a, b))
        blkw = np.concatenate([Wn[c][off:off + a * b].reshape(a, b, Lc)[s0:s1, t0:t1] for c in range(C)], axis=2)
        out["W"].append(blkw)
        off += a * b
    out["G"] = G
    return out
