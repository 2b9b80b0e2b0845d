"""Reconstruction quality metrics of Sec. 4 (oracle).

TEST INFRASTRUCTURE ONLY.

Per channel l of a cube of shape (ny, nx, L), with x_ref the ground truth and
x the estimate (Sec. 4.3, reconstruction quality):

* SNR_l = 20 log10(||x_ref_l||_2 / ||x_ref_l - x_l||_2);
* SNR_log_l: the same on the term-wise log10(z / eps_l + 1) of both images,
  eps_l the per-channel noise level in image space (it sets the dynamic range).

Both are +inf when the estimate equals the reference, and are reported as
average and standard deviation over the channels.
"""
import numpy as np


def _db(num2, den2):
    """10 log10(num2 / den2) = 20 log10(sqrt(num2) / sqrt(den2)); +inf if den2 = 0."""
    num2 = np.asarray(num2, dtype=np.float64)
    den2 = np.asarray(den2, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(den2 > 0, 10.0 * np.log10(num2 / np.where(den2 > 0, den2, 1.0)), np.inf)


def snr(x_ref, x):
    """Per-channel SNR in dB, shape (L,)."""
    r = np.asarray(x_ref, dtype=np.float64)
    d = r - np.asarray(x, dtype=np.float64)
    return _db(np.sum(r * r, axis=(0, 1)), np.sum(d * d, axis=(0, 1)))


def snr_log(x_ref, x, eps):
    """Per-channel SNR of the log10(z / eps + 1) images, shape (L,)."""
    eps = np.asarray(eps, dtype=np.float64)
    a = np.log10(np.asarray(x_ref, dtype=np.float64) / eps + 1.0)
    b = np.log10(np.asarray(x, dtype=np.float64) / eps + 1.0)
    d = a - b
    return _db(np.sum(a * a, axis=(0, 1)), np.sum(d * d, axis=(0, 1)))


def summary(values):
    """(mean, standard deviation) over the channels."""
    v = np.asarray(values, dtype=np.float64)
    return float(np.mean(v)), float(np.std(v))
