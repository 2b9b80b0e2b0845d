"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds none of the method's arithmetic: it only draws random
numbers and lays out arrays.  It stands in for the paper's simulated Cyg A
cube and VLA data (Sec. 4.1), which are not available here.

Cube recipe (per-blob simplification of the power-law spectral model of
Sec. 4.1): X[n, l] = sum_b A_b exp(-|r_n - c_b|^2 / (2 s_b^2)) (nu_l / nu_1)^{alpha_b}
with centres c_b uniform over the image, widths s_b ~ U(1, 8) px, spectral
indices alpha_b ~ U(-1, 1), amplitudes log-uniform on [1e-3, 1]; every blob is
evaluated within 6 s_b of its centre.  Frequencies are uniform over
[2.052, 3.572] GHz (L <= 64) or [2.052, 3.636] GHz (L = 100), the bands of the
two experiments of Sec. 4.1.  The cube is drawn in float64 and rounded once to
float32; every consumer uses the rounded values.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    ny: int
    nx: int
    L: int
    qy: int
    qx: int
    overlap: int       # low-rankness overlap in pixels, toward top/left
    C: int = 1         # spectral sub-cubes (channel-interleaved)
    blobs: int = 50
    levels: int = 4
    seed_offset: int = 0

    @property
    def voxels(self):
        return self.ny * self.nx * self.L


WORKLOADS = {
    "cfg1_256x256x20": Workload("cfg1_256x256x20", 256, 256, 20, 2, 2, 32, 1, 50, 4, 1),
    "cfg2_1024x2048x20": Workload("cfg2_1024x2048x20", 1024, 2048, 20, 4, 4, 64, 1, 50, 4, 2),
    "cfg3_2048x2048x60": Workload("cfg3_2048x2048x60", 2048, 2048, 60, 8, 8, 26, 1, 3200, 4, 3),
    "cfg4_2048x2048x100_c10": Workload("cfg4_2048x2048x100_c10", 2048, 2048, 100, 8, 8, 26, 10, 3200, 4, 4),
    "cfg5_4096x4096x64": Workload("cfg5_4096x4096x64", 4096, 4096, 64, 16, 16, 128, 1, 12800, 4, 5),
}

BASE_SEED = 200307358


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def frequencies(L):
    hi = 3.636 if L == 100 else 3.572
    return np.linspace(2.052, hi, L)


def blob_cube(ny, nx, L, nblobs, seed):
    """float32 (ny, nx, L) sum of Gaussian blobs with power-law spectra."""
    g = rng(seed)
    cy = g.uniform(0, ny, nblobs)
    cx = g.uniform(0, nx, nblobs)
    s = g.uniform(1.0, 8.0, nblobs)
    alpha = g.uniform(-1.0, 1.0, nblobs)
    amp = 10.0 ** g.uniform(-3.0, 0.0, nblobs)
    nu = frequencies(L)
    X = np.zeros((ny, nx, L), dtype=np.float64)
    for b in range(nblobs):
        r = int(np.ceil(6 * s[b]))
        y0, y1 = max(0, int(cy[b]) - r), min(ny, int(cy[b]) + r + 1)
        x0, x1 = max(0, int(cx[b]) - r), min(nx, int(cx[b]) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        gy = np.exp(-((np.arange(y0, y1) - cy[b]) ** 2) / (2 * s[b] ** 2))
        gx = np.exp(-((np.arange(x0, x1) - cx[b]) ** 2) / (2 * s[b] ** 2))
        spec = amp[b] * (nu / nu[0]) ** alpha[b]
        X[y0:y1, x0:x1] += (gy[:, None] * gx[None, :])[..., None] * spec[None, None, :]
    return X.astype(np.float32)


def uniform_weights(n, seed, lo=0.5, hi=1.0):
    return rng(seed).uniform(lo, hi, n).astype(np.float32)


def sorted_weights(n, seed, lo=0.5, hi=1.0):
    """Ascending U(lo, hi) weights (float64), one draw per facet."""
    return np.sort(rng(seed).uniform(lo, hi, n))


def gaussian(shape, seed, scale):
    return (scale * rng(seed).standard_normal(shape)).astype(np.float32)


def sigma_bar(X):
    """Noise-level stand-in: 1e-3 max(X) (the paper's estimate needs the
    measurement operator, which is out of scope)."""
    return 1e-3 * float(np.max(X))


def workload_cube(w: Workload, variant="plain"):
    """X_check for a workload.  'plain': X; 'signed': 2 X_a - X_b with X_b from
    the next seed (the extrapolated iterate of Algorithm 2 can be negative)."""
    seed = BASE_SEED + w.seed_offset
    Xa = blob_cube(w.ny, w.nx, w.L, w.blobs, seed)
    if variant == "plain":
        return Xa
    Xb = blob_cube(w.ny, w.nx, w.L, w.blobs, seed + 1000)
    return (2.0 * Xa.astype(np.float64) - Xb).astype(np.float32)


def noisy_data(X, frac, seed):
    """Data of the denoising stand-in: y = X + sigma n, n ~ N(0, 1) i.i.d.,
    sigma = frac max|X|.  Returns (y float32, sigma)."""
    sigma = frac * float(np.max(np.abs(X)))
    n = rng(seed).standard_normal(X.shape)
    return (X.astype(np.float64) + sigma * n).astype(np.float32), sigma


# ---------------------------------------------------------------- counter-based values
# Warm duals of full-size problems are too large to draw on the host and ship
# to the device; instead each value is a fixed function of its index, which
# the host (numpy) and the device (torch) evaluate identically, so that a
# sampled block on the host sees exactly the values the device holds.

def hash32(i, j, seed):
    """32-bit integer hash of (i, j, seed) (T. Mueller's 0x45d9f3b
    xor-shift-multiply mixer applied to a linear combination of the
    counters).  i, j: int64 arrays (numpy) or tensors (torch) of values below
    2^31; every intermediate stays below 2^63.  Returns int64 in [0, 2^32)."""
    h = (i * 73856093 + j * 19349663 + seed * 83492791) & 0xFFFFFFFF
    h = ((h ^ (h >> 16)) * 0x45D9F3B) & 0xFFFFFFFF
    h = ((h ^ (h >> 16)) * 0x45D9F3B) & 0xFFFFFFFF
    return h ^ (h >> 16)


def hash_uniform_np(i, j, seed):
    """float64 in [-0.5, 0.5) from hash32 (numpy)."""
    h = hash32(np.asarray(i, dtype=np.int64), np.asarray(j, dtype=np.int64), int(seed))
    return h.astype(np.float64) / 4294967296.0 - 0.5


WARM_W_SEED, WARM_P_SEED = 71, 73


def warm_w_np(rows, positions, scale):
    """Warm l21 dual: W[i, p] = scale * u(i, p), u = hash_uniform(i, p, WARM_W_SEED),
    rounded once to float32.  rows: coefficient rows, positions: channel
    positions (broadcast against each other)."""
    return (float(scale) * hash_uniform_np(rows, positions, WARM_W_SEED)).astype(np.float32)


def warm_p_np(facet, n, scale):
    """Warm nuclear dual of facet f (flattened [ny~][nx~][L_c], n values):
    P[e] = scale * hash_uniform(e, f, WARM_P_SEED), rounded to float32."""
    return (float(scale) * hash_uniform_np(np.arange(n, dtype=np.int64), facet, WARM_P_SEED)).astype(np.float32)


def warm_w_scale(mu_c):
    """Amplitude of the warm l21 dual of sub-cube c: rows of norm about the
    threshold, so that both branches of the row shrink occur."""
    return 0.8 * float(mu_c)


def warm_p_scale(mu_bar_f, n_rows):
    """Amplitude of the warm nuclear dual of a facet with n_rows pixels."""
    return 0.3 * float(mu_bar_f) / np.sqrt(n_rows)


def facet_selection(C, Q, prob, seed):
    """Random draw of the facets whose duals a randomized step updates:
    (C, Q) booleans, each true with probability prob."""
    return rng(seed).random((C, Q)) < prob


def uv_coverage(M, seed, spread=0.35):
    """A synthetic uv-coverage standing in for the VLA coverages of Sec. 4.1:
    M points (omega_y, omega_x) in radians per pixel, radially concentrated
    toward the origin like an interferometer's (Gaussian radii of scale
    spread * pi, uniform angles), kept inside [-pi/2, pi/2)^2 so that the
    coverage scaled by the channel's frequency ratio (up to about 1.8 over
    the paper's bands) stays inside [-pi, pi)^2.  Includes conjugate-free
    points only (no symmetry imposed)."""
    r = rng(seed)
    out = np.empty((0, 2))
    while len(out) < M:
        rad = np.abs(r.standard_normal(2 * M)) * spread * np.pi
        ang = r.uniform(0, 2 * np.pi, 2 * M)
        pts = np.stack([rad * np.sin(ang), rad * np.cos(ang)], axis=1)
        pts = pts[np.all(np.abs(pts) < 0.5 * np.pi, axis=1)]
        out = np.concatenate([out, pts])
    return out[:M]


def channel_coverages(M, L, seed):
    """Per channel l, the reference coverage scaled by nu_l / nu_1 (Sec. 4.1:
    the coverage of channel l is the reference one scaled by the frequency
    ratio)."""
    base = uv_coverage(M, seed)
    nu = frequencies(L)
    return [base * (nu[l] / nu[0]) for l in range(L)]
