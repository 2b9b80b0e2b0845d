"""Pins of the reconstruction metrics oracle (Sec. 4.3) against closed forms."""
import numpy as np
import pytest

from oracle import metrics


def cube(seed, shape=(9, 7, 4)):
    return np.random.default_rng(seed).uniform(0.1, 2.0, shape)


def test_snr_of_a_scaled_estimate_is_closed_form():
    # x = (1 + d_l) x_ref per channel -> SNR_l = -20 log10 |d_l| exactly
    r = cube(1)
    d = np.array([0.1, -0.01, 0.5, 1e-3])
    got = metrics.snr(r, r * (1.0 + d))
    np.testing.assert_allclose(got, -20.0 * np.log10(np.abs(d)), rtol=1e-12)


def test_snr_by_hand_on_a_tiny_case():
    r = np.zeros((1, 2, 1))
    r[0, :, 0] = [3.0, 4.0]                   # ||r|| = 5
    x = r.copy()
    x[0, 1, 0] = 4.5                          # ||r - x|| = 0.5
    assert metrics.snr(r, x)[0] == pytest.approx(20.0)


def test_exact_estimate_is_infinite():
    r = cube(2)
    assert np.all(np.isinf(metrics.snr(r, r)))
    assert np.all(np.isinf(metrics.snr_log(r, r, np.full(4, 0.3))))


def test_snr_log_tends_to_snr_for_a_large_noise_level():
    # log10(z / eps + 1) = z / (eps ln 10) + O(z^2 / eps^2): the ratio of norms
    # tends to the linear one as eps grows
    r = cube(3)
    x = r * np.exp(0.05 * np.random.default_rng(4).standard_normal(r.shape))  # positive, like the iterates
    lin = metrics.snr(r, x)
    np.testing.assert_allclose(metrics.snr_log(r, x, np.full(4, 1e6)), lin, rtol=1e-4)
    assert not np.allclose(metrics.snr_log(r, x, np.full(4, 1e-3)), lin, rtol=1e-2)


def test_snr_log_by_hand():
    # eps = 1, r = 9 -> log10(10) = 1; x = 99 -> log10(100) = 2: SNR_log = 20 log10(1 / 1) = 0
    r = np.full((1, 1, 1), 9.0)
    x = np.full((1, 1, 1), 99.0)
    assert metrics.snr_log(r, x, [1.0])[0] == pytest.approx(0.0, abs=1e-12)


def test_summary():
    m, s = metrics.summary([10.0, 20.0])
    assert m == 15.0 and s == 5.0
