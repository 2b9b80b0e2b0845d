"""Facet geometry of Faceted HyperSARA (oracle).

TEST INFRASTRUCTURE ONLY.

Sec. 2.4.2 ("Spatial faceting"):
* the image is cut into non-overlapping tiles; a facet is its tile extended
  toward the top and the left so that it overlaps its top/left neighbours;
  an edge facet with no neighbour on a side keeps the tile's size there;
* the low-rankness facets (selection S~_q) use an adjustable overlap and are
  weighted by D_q, a 2D triangular apodisation window (outer product of two 1D
  piecewise-linear windows) whose weights are positive and sum to one at
  every pixel over all facets;
* the sparsity facets (selection S_q) use the overlap that makes the faceted
  wavelet transform exact, between 15(2^d - 2) and 15(2^d - 1) pixels for
  d levels of db8.

Readings where the paper is silent:
* tile split along an axis of n pixels into Q tiles: t_s = floor(s n / Q);
* 1D window of facet s along an axis (overlap o): weight 1 on the tile except
  that the facet's own border [t_s - o, t_s) rises as (k+1)/(o+1) and the last o
  pixels of its tile (covered by the next facet's border) fall as
  1 - (k+1)/(o+1), k = 0 .. o-1;
* coefficient ownership per axis at level j: boundary b_j(s) =
  ceil((b_{j-1}(s) - 1) / 2) with b_0(s) = t_s, the first facet starting at 0
  and the last one owning the tail up to the band length; a facet owns a
  coefficient exactly when the highest-index input it depends on lies in that
  facet's tile (causal convention of the transform);
* SARA window along an axis: [max(0, t_s - E), t_{s+1}).
"""
from dataclasses import dataclass, field

import numpy as np

from . import dwt
from .filters import sara_filters


def tile_bounds(n, Q):
    return [(s * n) // Q for s in range(Q + 1)]


def window_1d(n, Q, s, o):
    """(start, stop, weights) of the low-rankness window of facet s on one axis."""
    t = tile_bounds(n, Q)
    a = t[s] - o if s > 0 else t[s]
    b = t[s + 1]
    w = np.ones(b - a, dtype=np.float64)
    if s > 0:
        for k in range(o):
            w[k] = (k + 1) / (o + 1)
    if s < Q - 1:
        base = b - o - a
        for k in range(o):
            w[base + k] = 1.0 - (k + 1) / (o + 1)
    return a, b, w


def ownership_1d(n, Q, L, levels):
    """Per level j = 1..levels, the list of Q+1 boundaries of owned coefficients."""
    t = tile_bounds(n, Q)
    out = []
    prev = list(t)
    length = n
    for _ in range(levels):
        K = dwt.out_len(length, L)
        cur = [0] + [-(-(prev[s] - 1) // 2) for s in range(1, Q)] + [K]
        out.append(cur)
        prev, length = cur, K
    return out


@dataclass
class Facet:
    index: int
    sy: int
    sx: int
    tile: tuple
    nuc_window: tuple
    wy: np.ndarray
    wx: np.ndarray
    sara_window: tuple

    @property
    def nuc_shape(self):
        (y0, y1), (x0, x1) = self.nuc_window
        return (y1 - y0, x1 - x0)

    @property
    def n_rows(self):
        a, b = self.nuc_shape
        return a * b

    def window(self):
        """D_q as a (ny~, nx~) array."""
        return np.outer(self.wy, self.wx)


@dataclass
class Geometry:
    ny: int
    nx: int
    qy: int
    qx: int
    oy: int
    ox: int
    levels: int = 4
    E: int = 225
    facets: list = field(default_factory=list)

    def __post_init__(self):
        ty, tx = tile_bounds(self.ny, self.qy), tile_bounds(self.nx, self.qx)
        for sy in range(self.qy):
            if sy > 0 and self.oy > ty[sy] - ty[sy - 1]:
                raise ValueError("overlap larger than the neighbouring tile")
        for sx in range(self.qx):
            if sx > 0 and self.ox > tx[sx] - tx[sx - 1]:
                raise ValueError("overlap larger than the neighbouring tile")
        if self.oy > min(ty[s + 1] - ty[s] for s in range(self.qy)) and self.qy > 1:
            raise ValueError("overlap larger than a tile")
        if self.ox > min(tx[s + 1] - tx[s] for s in range(self.qx)) and self.qx > 1:
            raise ValueError("overlap larger than a tile")
        self.facets = []
        for sy in range(self.qy):
            ay, by, wy = window_1d(self.ny, self.qy, sy, self.oy)
            for sx in range(self.qx):
                ax, bx, wx = window_1d(self.nx, self.qx, sx, self.ox)
                sara = ((max(0, ty[sy] - self.E) if sy > 0 else 0, ty[sy + 1]),
                        (max(0, tx[sx] - self.E) if sx > 0 else 0, tx[sx + 1]))
                self.facets.append(Facet(len(self.facets), sy, sx,
                                         ((ty[sy], ty[sy + 1]), (tx[sx], tx[sx + 1])),
                                         ((ay, by), (ax, bx)), wy, wx, sara))

    @property
    def Q(self):
        return self.qy * self.qx

    def owned_rects(self, f):
        """Owned rectangle of facet f in every band, in storage order."""
        rects = []
        for h, _ in sara_filters():
            oy = ownership_1d(self.ny, self.qy, len(h), self.levels)
            ox = ownership_1d(self.nx, self.qx, len(h), self.levels)
            for j in range(self.levels):
                r = ((oy[j][f.sy], oy[j][f.sy + 1]), (ox[j][f.sx], ox[j][f.sx + 1]))
                rects += [r] * 3
            j = self.levels - 1
            rects.append(((oy[j][f.sy], oy[j][f.sy + 1]), (ox[j][f.sx], ox[j][f.sx + 1])))
        rects.append(f.tile)
        return rects

    def window_sum(self):
        """sum_q S~_q^T D_q 1 (must be 1 everywhere)."""
        acc = np.zeros((self.ny, self.nx))
        for f in self.facets:
            (y0, y1), (x0, x1) = f.nuc_window
            acc[y0:y1, x0:x1] += f.window()
        return acc
