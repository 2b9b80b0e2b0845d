"""SARA dictionary Psi^dagger and its adjoint Psi (oracle).

TEST INFRASTRUCTURE ONLY.

Sec. 2.3.1: Psi^dagger is the concatenation of D = 9 orthonormal bases (the
first eight Daubechies wavelets and the Dirac basis) divided by sqrt(D) = 3, so
that Psi Psi^dagger = I.  Every wavelet basis uses the same number of levels
(4 in every workload here).

Coefficient storage (a layout choice the paper does not fix): a flat list of
2D(+channel) bands, basis by basis (db1 ... db8, then Dirac); within a wavelet
basis, level by level from fine to coarse as (lh, hl, hh), followed by the
coarsest ll band.

The faceted variant follows Sec. 2.4.2: facet q applies the transform to the
pixels of its own window only (zero elsewhere) and keeps the coefficients it
owns; the adjoint zero-fills the coefficients it does not own, applies the
transposed transform and keeps the window's pixels, and the facet results are
overlap-added.  Its equality with the global transform is one of the pins.
"""
import numpy as np

from . import dwt
from .filters import sara_filters

NBASES = 9
SCALE = 1.0 / 3.0   # 1 / sqrt(9)


def band_shapes(ny, nx, levels):
    """Spatial shape of every band, in storage order."""
    shapes = []
    for h, _ in sara_filters():
        lv = dwt.level_shapes(ny, nx, len(h), levels)
        for (_, _, Ky, Kx) in lv:
            shapes += [(Ky, Kx)] * 3
        shapes.append(lv[-1][2:])
    shapes.append((ny, nx))
    return shapes


def n_coefficients(ny, nx, levels):
    """I: number of coefficient rows (positions) of Psi^dagger."""
    return sum(a * b for a, b in band_shapes(ny, nx, levels))


def analysis(x, levels=4):
    """Psi^dagger x: list of bands (each (Ky, Kx, ...)), scaled by 1/3."""
    bands = []
    for h, g in sara_filters():
        bands += [SCALE * b for b in dwt.wavedec2(x, h, g, levels)]
    bands.append(SCALE * np.asarray(x, dtype=np.float64))
    return bands


def synthesis(bands, ny, nx, levels=4):
    """Psi w = (1/3) (sum_b DWT_b^T w_b + w_dirac): the adjoint of `analysis`."""
    per = 3 * levels + 1
    out = None
    for b, (h, g) in enumerate(sara_filters()):
        part = dwt.waverec2_adjoint(bands[b * per:(b + 1) * per], h, g, ny, nx, levels)
        out = part if out is None else out + part
    out = out + bands[8 * per]
    return SCALE * out


def flatten(bands):
    """Concatenate bands as coefficient rows: (I, ...)."""
    return np.concatenate([b.reshape((-1,) + b.shape[2:]) for b in bands], axis=0)


def unflatten(flat, ny, nx, levels=4):
    """Inverse of `flatten` for a given image size."""
    out, off = [], 0
    for (a, b) in band_shapes(ny, nx, levels):
        out.append(flat[off:off + a * b].reshape((a, b) + flat.shape[1:]))
        off += a * b
    assert off == flat.shape[0]
    return out


# ---------------------------------------------------------------------------
# Explicit faceted variant (Sec. 2.4.2)

def faceted_analysis(x, geom, levels=4):
    """sum over facets of S_q^T-free local transforms: each facet transforms its
    SARA window alone and contributes only the coefficients it owns."""
    ny, nx = x.shape[:2]
    shapes = band_shapes(ny, nx, levels)
    out = [np.zeros(s + x.shape[2:]) for s in shapes]
    for f in geom.facets:
        (y0, y1), (x0, x1) = f.sara_window
        xw = np.zeros_like(x, dtype=np.float64)
        xw[y0:y1, x0:x1] = x[y0:y1, x0:x1]
        local = analysis(xw, levels)
        for k, (ry, rx) in enumerate(geom.owned_rects(f)):
            out[k][ry[0]:ry[1], rx[0]:rx[1]] = local[k][ry[0]:ry[1], rx[0]:rx[1]]
    return out


def faceted_synthesis(bands, geom, levels=4):
    """sum_q S_q^T Psi_q w_q with w_q the coefficients owned by facet q."""
    ny, nx = geom.ny, geom.nx
    trail = bands[0].shape[2:]
    out = np.zeros((ny, nx) + trail)
    for f in geom.facets:
        local = [np.zeros_like(b, dtype=np.float64) for b in bands]
        for k, (ry, rx) in enumerate(geom.owned_rects(f)):
            local[k][ry[0]:ry[1], rx[0]:rx[1]] = bands[k][ry[0]:ry[1], rx[0]:rx[1]]
        img = synthesis(local, ny, nx, levels)
        (y0, y1), (x0, x1) = f.sara_window
        out[y0:y1, x0:x1] += img[y0:y1, x0:x1]
    return out
