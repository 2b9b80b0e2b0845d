"""Zero-extended, expansive, separable 2D DWT and its adjoint (oracle).

TEST INFRASTRUCTURE ONLY.

The paper asks for orthonormal bases with Psi Psi^dagger = I (Sec. 2.3.1) and
an exact faceted implementation (Sec. 2.4.2) but does not state the boundary
extension.  The reading taken here is the zero-extended ("expansive")
transform with the causal index convention:

    a[k] = sum_{m=0}^{L-1} h[m] x[2k+1-m],   d[k] = sum_m g[m] x[2k+1-m],
    k = 0 .. K-1,  K = floor((n + L - 1) / 2),  x = 0 outside [0, n).

K is exactly the number of shifts k for which the filter support meets
[0, n), so the map x -> (a, d) is an isometry (A^T A = I) for every n and
every orthonormal filter pair.  Each coefficient depends only on inputs of
equal or lower index, which is what makes facets overlap only with their
top/left neighbours.

A level is applied along axis 0 (rows, y) and axis 1 (columns, x); a
multi-level transform recurses on the low-low band (Mallat pyramid).
Arrays are (ny, nx, ...) with any trailing (channel) axes.
"""
import numpy as np


def out_len(n, L):
    """Number of coefficients per band for an input of length n."""
    return (n + L - 1) // 2


def analysis_axis(x, f, axis):
    """One filter-and-decimate pass along `axis`: y[k] = sum_m f[m] x[2k+1-m]."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, 0)
    n, L = x.shape[0], len(f)
    K = out_len(n, L)
    # padded copy: xp[i + L - 1] = x[i]
    xp = np.zeros((n + 2 * L - 1,) + x.shape[1:], dtype=np.float64)
    xp[L - 1:L - 1 + n] = x
    y = np.zeros((K,) + x.shape[1:], dtype=np.float64)
    for m in range(L):
        # x[2k+1-m] = xp[2k + L - m]
        start = L - m
        y += f[m] * xp[start:start + 2 * K:2]
    return np.moveaxis(y, 0, axis)


def adjoint_axis(y, f, n, axis):
    """Exact transpose of `analysis_axis` for an input length n."""
    y = np.moveaxis(np.asarray(y, dtype=np.float64), axis, 0)
    K, L = y.shape[0], len(f)
    assert K == out_len(n, L)
    xp = np.zeros((n + 2 * L - 1,) + y.shape[1:], dtype=np.float64)
    for m in range(L):
        start = L - m
        xp[start:start + 2 * K:2] += f[m] * y
    x = xp[L - 1:L - 1 + n]
    return np.moveaxis(x, 0, axis)


def analysis_level(x, h, g):
    """One 2D level.  Returns (ll, lh, hl, hh); the first letter is the filter
    applied along rows (axis 0), the second the one along columns (axis 1)."""
    lo = analysis_axis(x, h, 0)
    hi = analysis_axis(x, g, 0)
    return (analysis_axis(lo, h, 1), analysis_axis(lo, g, 1),
            analysis_axis(hi, h, 1), analysis_axis(hi, g, 1))


def adjoint_level(ll, lh, hl, hh, h, g, ny, nx):
    """Transpose of `analysis_level` for an input of size ny x nx."""
    lo = adjoint_axis(ll, h, nx, 1) + adjoint_axis(lh, g, nx, 1)
    hi = adjoint_axis(hl, h, nx, 1) + adjoint_axis(hh, g, nx, 1)
    return adjoint_axis(lo, h, ny, 0) + adjoint_axis(hi, g, ny, 0)


def level_shapes(ny, nx, L, levels):
    """Input shape of every level and shape of its bands: [(ny_j, nx_j, Ky, Kx)]."""
    out = []
    for _ in range(levels):
        Ky, Kx = out_len(ny, L), out_len(nx, L)
        out.append((ny, nx, Ky, Kx))
        ny, nx = Ky, Kx
    return out


def wavedec2(x, h, g, levels):
    """Multi-level transform.  Returns the list of bands in storage order:
    [lh1, hl1, hh1, lh2, hl2, hh2, ..., lhJ, hlJ, hhJ, llJ]."""
    bands = []
    cur = x
    for _ in range(levels):
        ll, lh, hl, hh = analysis_level(cur, h, g)
        bands += [lh, hl, hh]
        cur = ll
    bands.append(cur)
    return bands


def waverec2_adjoint(bands, h, g, ny, nx, levels):
    """Adjoint of `wavedec2` (equal to its inverse on the image, since the
    transform is an isometry)."""
    shapes = level_shapes(ny, nx, len(h), levels)
    cur = bands[-1]
    for j in reversed(range(levels)):
        lh, hl, hh = bands[3 * j:3 * j + 3]
        nyj, nxj, _, _ = shapes[j]
        cur = adjoint_level(cur, lh, hl, hh, h, g, nyj, nxj)
    return cur
