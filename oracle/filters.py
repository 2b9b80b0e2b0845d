"""Daubechies extremal-phase filters (oracle; test infrastructure only).

The SARA dictionary uses "the first eight Daubechies wavelets" (Sec. 2.3.1).
The paper gives no coefficients, so they are derived here from the published
construction (Daubechies 1988): the squared modulus of the low-pass transfer
function is cos^{2N}(w/2) P(sin^2(w/2)) with

    P(y) = sum_{k=0}^{N-1} binom(N-1+k, k) y^k,

and the trigonometric polynomial with that modulus is obtained by spectral
factorisation (one root of each reciprocal pair z, 1/z is kept).

Orientation (not fixed by the paper): for every root y_k of P the root of
z^2 - (2 - 4 y_k) z + 1 = 0 *outside* the unit circle is kept, and h[n] is
sqrt(2) times the coefficient of z^n in ((1+z)/2)^N prod_k (z - r_k)/(1 - r_k).
This gives Daubechies' own form, e.g. db2 = [1+s3, 3+s3, 3-s3, 1-s3]/(4 sqrt 2)
with s3 = sqrt(3): the energy sits at the start of the filter.

The high-pass filter is g[m] = (-1)^m h[L-1-m], L = 2N.
"""
from math import comb, sqrt

import numpy as np


def daubechies_polynomial(N):
    """Coefficients (ascending powers of y) of P(y) = sum_k binom(N-1+k, k) y^k."""
    return np.array([comb(N - 1 + k, k) for k in range(N)], dtype=np.float64)


def lowpass(N):
    """Scaling filter h of dbN (length 2N), float64, sum(h) = sqrt(2)."""
    if N < 1:
        raise ValueError("N >= 1")
    p = daubechies_polynomial(N)
    # np.roots wants descending powers
    yroots = np.roots(p[::-1]) if N > 1 else np.array([], dtype=np.complex128)
    zroots = []
    for y in yroots:
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zroots.append(z1 if abs(z1) > 1.0 else z2)
    # polynomial in z, ascending coefficients
    poly = np.array([1.0 + 0j])
    for _ in range(N):
        poly = np.convolve(poly, np.array([0.5, 0.5]))
    for r in zroots:
        poly = np.convolve(poly, np.array([-r, 1.0])) / (1.0 - r)
    h = sqrt(2.0) * poly
    if np.max(np.abs(h.imag)) > 1e-10:
        raise AssertionError("spectral factor is not real")
    return h.real.copy()


def highpass(h):
    """g[m] = (-1)^m h[L-1-m] (quadrature mirror of h)."""
    L = len(h)
    return np.array([(-1) ** m * h[L - 1 - m] for m in range(L)], dtype=np.float64)


def sara_filters():
    """The eight (h, g) pairs of the SARA dictionary: db1 ... db8."""
    out = []
    for N in range(1, 9):
        h = lowpass(N)
        out.append((h, highpass(h)))
    return out
