"""Proximal operators of Table 1 (oracle).

TEST INFRASTRUCTURE ONLY.

* soft-thresholding: prox_{a|.|_1}(z) = sgn(z) max(|z| - a, 0);
* singular value thresholding: prox_{a||.||_*}(Z) = U Diag(prox_{a|.|_1}(s)) V^T
  from the thin SVD Z = U Diag(s) V^T (LAPACK gesdd through numpy);
  the weighted version thresholds the j-th largest singular value with the
  j-th threshold t_j (reading: weights are paired with singular values in
  descending order of the latter, the pairing under which the weighted SVT
  is the exact proximal point for non-descending weights);
* l21 row shrink: prox_{a||.||_{2,1}}(Z) scales row n by max(||z_n|| - a, 0)/||z_n||;
  the weighted version uses a_i = a theta_i for row i.

The dual updates of Algorithm 2 use the complements I - prox, which are
provided directly in closed form:
* Z - prox_svt(Z) = U Diag(min(s, t)) V^T;
* z_i - prox_l21(z)_i = z_i min(1, a_i / ||z_i||), and 0 for a zero row.
"""
import numpy as np


def soft_threshold(z, a):
    z = np.asarray(z, dtype=np.float64)
    return np.sign(z) * np.maximum(np.abs(z) - a, 0.0)


def weighted_svt(Z, t):
    """prox of the weighted nuclear norm sum_j t_j s_j(.) at Z (t aligned with
    singular values in descending order)."""
    U, s, Vt = np.linalg.svd(np.asarray(Z, dtype=np.float64), full_matrices=False)
    t = np.asarray(t, dtype=np.float64)[:len(s)]
    return (U * np.maximum(s - t, 0.0)) @ Vt


def weighted_svt_complement(Z, t):
    """(I - prox_{sum t_j s_j})(Z) = U Diag(min(s, t)) V^T."""
    U, s, Vt = np.linalg.svd(np.asarray(Z, dtype=np.float64), full_matrices=False)
    t = np.asarray(t, dtype=np.float64)[:len(s)]
    return (U * np.minimum(s, t)) @ Vt


def l21_prox(Z, a):
    """Row shrink with per-row thresholds a (scalar or (rows,))."""
    Z = np.asarray(Z, dtype=np.float64)
    r = np.linalg.norm(Z, axis=1)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), r.shape)
    scale = np.zeros_like(r)
    nz = r > 0
    scale[nz] = np.maximum(r[nz] - a[nz], 0.0) / r[nz]
    return Z * scale[:, None]


def l21_prox_complement(Z, a):
    """(I - prox_{a||.||_{2,1}})(Z): row i scaled by min(1, a_i/||z_i||), zero rows stay 0."""
    Z = np.asarray(Z, dtype=np.float64)
    r = np.linalg.norm(Z, axis=1)
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), r.shape)
    scale = np.zeros_like(r)
    nz = r > 0
    scale[nz] = np.minimum(1.0, a[nz] / r[nz])
    return Z * scale[:, None]
