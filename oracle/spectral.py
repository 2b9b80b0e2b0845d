"""Spectral facets with overlap: the 100-channel case taken literally (oracle).

TEST INFRASTRUCTURE ONLY.

The paper's spectral sub-cubes are disjoint, channel-interleaved and
independent (Sec. 2.4.1).  A split of L channels into C contiguous blocks
whose low-rankness facets overlap by o channels is not in the paper; this
module is the reading used for it: the spatial overlap rule of Sec. 2.4.2
applied along the spectral axis.

* l21 term: block c holds the contiguous channels [c L/C, (c + 1) L/C); its
  rows span those channels only (the SARA part is the paper's, on contiguous
  sub-cubes).
* low-rankness term: the facet (c, q) matrix takes the spatial window of
  facet q and the spectral window of block c, which starts o channels before
  the block (none for the first block) and ends with the block.  Its weights
  are the triangular ramp of the spatial window on one axis: rising over the
  o channels before the block, falling over the block's last o channels
  (unless it is the last block), 1 elsewhere.  The spectral weights of the
  blocks then sum to one on every channel, as D_q does over the image.
  So Z_{c,q} = P_{c,q} + (D_q x d_c) S~_q X over those channels, and the
  aggregation adds zeta S~_q^T (D_q x d_c) P_{c,q} into them.

With o = 0 this is the plain step on contiguous sub-cubes; with C = 1 it is
the plain step.
"""
import numpy as np

from . import geometry, prox, sara


def block_channels(L, C):
    """Channels of each contiguous block (the l21 rows)."""
    t = geometry.tile_bounds(L, C)
    return [list(range(t[c], t[c + 1])) for c in range(C)]


def spectral_window(L, C, c, o):
    """(channels, weights) of the low-rankness window of block c."""
    a, b, w = geometry.window_1d(L, C, c, o)
    return list(range(a, b)), w


def facet_matrix(xcheck, f, chans, wts):
    """(D_q x d_c) S~_q X over the window's channels, as an (N~_q, |chans|) matrix."""
    (y0, y1), (x0, x1) = f.nuc_window
    xs = np.asarray(xcheck, dtype=np.float64)[y0:y1, x0:x1][..., chans]
    return (f.window()[..., None] * np.asarray(wts)[None, None, :] * xs).reshape(-1, len(chans))


def facet_prox_step(xcheck, P, W, theta, theta_bar, mu, mu_bar, zeta, kappa, geom, C, o):
    """The facet step with overlapping spectral facets.

    P[c][q]: (ny~_q, nx~_q, |window of c|); theta_bar[c][q]: (|window of c|,)
    ascending; W[c]: (I, L/C); theta[c]: (I,); mu (C,); mu_bar (C, Q).
    Returns (P_new, W_new, G) with G (ny, nx, L).
    """
    ny, nx, L = xcheck.shape
    G = np.zeros((ny, nx, L))
    P_new = []
    for c in range(C):
        chans, wts = spectral_window(L, C, c, o)
        row = []
        for q, f in enumerate(geom.facets):
            Z = np.asarray(P[c][q], dtype=np.float64).reshape(-1, len(chans)) + facet_matrix(xcheck, f, chans, wts)
            t = (mu_bar[c][q] / zeta) * np.asarray(theta_bar[c][q], dtype=np.float64)
            Pn = prox.weighted_svt_complement(Z, t).reshape(f.nuc_shape + (len(chans),))
            row.append(Pn)
            (y0, y1), (x0, x1) = f.nuc_window
            G[y0:y1, x0:x1][..., chans] += zeta * f.window()[..., None] * np.asarray(wts)[None, None, :] * Pn
        P_new.append(row)
    W_new = []
    for c, chans in enumerate(block_channels(L, C)):
        A = sara.flatten(sara.analysis(np.asarray(xcheck, dtype=np.float64)[..., chans], geom.levels))
        U = np.asarray(W[c], dtype=np.float64) + A
        Wn = prox.l21_prox_complement(U, (mu[c] / kappa) * np.asarray(theta[c], dtype=np.float64))
        W_new.append(Wn)
        G[..., chans] += kappa * sara.synthesis(sara.unflatten(Wn, ny, nx, geom.levels), ny, nx, geom.levels)
    return P_new, W_new, G
