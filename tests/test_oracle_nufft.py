"""Pins of the oracle's measurement operator and data-fidelity dual update
(oracle.nufft; Sec. 2.1 eq. model, Alg. 2 data-fidelity lines, eq.
prox_definition, Sec. 3.2 preconditioning and sub-iterations).

* the Kaiser-Bessel kernel's closed-form Fourier transform against numerical
  quadrature (the scaling Z depends on it);
* Phi against the brute-force centred DFT on small images (the NUFFT's error
  bound for a 7 x 7 kernel at 2x oversampling), a centred delta (all ones)
  and a shifted one (a phase ramp);
* the adjoint by the dot test Re <Phi x, v> = <x, Phi^dagger v>;
* the inverse sampling density: shared cells, the count of occupied cells;
* the projection in the U metric: z inside the ball, U = c I (Euclidean
  projection), the KKT / variational inequality for random points of the
  ball, and the forward-backward sub-iterations converging to it;
* the dual update with U = I reducing to the identity-metric closure
  formula, and its parts composed by hand.
"""
import numpy as np
import pytest

import synth
from oracle import nufft

RNG = np.random.default_rng(41)


def test_kb_fourier_closed_form_matches_quadrature():
    J = nufft.KB_WIDTH
    d = np.linspace(-J / 2, J / 2, 400001)
    psi = nufft.kb_kernel(d)
    for xi in (0.0, 0.03, 0.11, 0.2, 0.25):
        q = np.trapezoid(psi * np.cos(2 * np.pi * d * xi), d)
        assert abs(q / nufft.kb_fourier(xi) - 1.0) < 1e-9, xi
    # the kernel vanishes outside its support and is even
    assert nufft.kb_kernel(J / 2 + 1e-9) == 0.0
    assert nufft.kb_kernel(1.3) == nufft.kb_kernel(-1.3)


@pytest.mark.parametrize("ny,nx", [(32, 32), (16, 24)])
def test_nufft_matches_the_direct_dft(ny, nx):
    om = RNG.uniform(-np.pi, np.pi, (200, 2))
    x = RNG.standard_normal((ny, nx))
    op = nufft.Nufft(ny, nx, om)
    y, ref = op.forward(x), nufft.nudft(x, om)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-5


def test_nufft_of_deltas():
    ny, nx = 32, 16
    om = RNG.uniform(-np.pi, np.pi, (50, 2))
    op = nufft.Nufft(ny, nx, om)
    x = np.zeros((ny, nx))
    x[ny // 2, nx // 2] = 1.0           # the image centre: every visibility is 1
    assert np.max(np.abs(op.forward(x) - 1.0)) < 1e-5
    x[:] = 0.0
    x[ny // 2 + 3, nx // 2 - 5] = 1.0   # a shift (3, -5): exp(-i (3 w_y - 5 w_x))
    ref = np.exp(-1j * (3 * om[:, 0] - 5 * om[:, 1]))
    assert np.max(np.abs(op.forward(x) - ref)) < 1e-5


def test_nufft_adjoint_dot_test():
    ny, nx = 24, 32
    om = synth.uv_coverage(300, 3)
    op = nufft.Nufft(ny, nx, om)
    x = RNG.standard_normal((ny, nx))
    v = RNG.standard_normal(300) + 1j * RNG.standard_normal(300)
    lhs = np.real(np.vdot(op.forward(x), v))
    rhs = np.sum(x * op.adjoint(v))
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0)


def test_inverse_density():
    K1, K2 = 16, 16
    # three points in the cell of grid point (1, 2), one alone in (5, 5)
    w = 2 * np.pi / K1
    om = np.array([[1.0 * w, 2.0 * w], [1.2 * w, 1.9 * w], [0.8 * w, 2.3 * w], [5.0 * w, 5.0 * w]])
    U = nufft.inverse_density(om, K1, K2)
    assert np.allclose(U, [1 / 3, 1 / 3, 1 / 3, 1.0])
    om = synth.uv_coverage(2000, 5)
    U = nufft.inverse_density(om, 64, 64)
    cells = {(int(np.rint(a * 64 / (2 * np.pi))) % 64, int(np.rint(b * 64 / (2 * np.pi))) % 64) for a, b in om}
    assert abs(np.sum(U) - len(cells)) < 1e-9
    assert np.all(U > 0) and np.all(U <= 1)


def test_metric_projection():
    M = 60
    y = RNG.standard_normal(M) + 1j * RNG.standard_normal(M)
    eps = 0.7
    U = RNG.uniform(0.1, 1.0, M)
    # inside the ball: unchanged
    z = y + 0.3 * eps * (RNG.standard_normal(M) + 1j * RNG.standard_normal(M)) / np.sqrt(2 * M)
    assert np.allclose(nufft.project_ball_metric(z, y, eps, U), z)
    # outside: on the sphere, and U = c I gives the Euclidean projection
    z = y + 3.0 * (RNG.standard_normal(M) + 1j * RNG.standard_normal(M))
    assert np.allclose(nufft.project_ball_metric(z, y, eps, np.full(M, 0.4)), nufft.project_ball(z, y, eps),
                       atol=1e-12)
    p = nufft.project_ball_metric(z, y, eps, U)
    assert abs(np.linalg.norm(p - y) - eps) < 1e-10
    # variational inequality: Re <U (p - z), w - p> >= 0 for every w in the ball
    for _ in range(200):
        d = RNG.standard_normal(M) + 1j * RNG.standard_normal(M)
        w = y + d * (eps * RNG.uniform() / np.linalg.norm(d))
        assert np.real(np.vdot(U * (p - z), w - p)) >= -1e-10
    # forward-backward sub-iterations converge to it; zero sub-iterations: P_B(z)
    assert np.allclose(nufft.project_ball_metric_fb(z, y, eps, U, 0), nufft.project_ball(z, y, eps))
    e = [np.linalg.norm(nufft.project_ball_metric_fb(z, y, eps, U, n) - p) for n in (0, 1, 5, 50)]
    assert e[0] > e[1] > e[2] > e[3] or e[3] < 1e-13
    assert e[0] > 1e-2 and e[3] < 1e-12


def test_data_dual_update_with_identity_metric_and_by_hand():
    ny, nx, L, M = 16, 16, 3, 120
    covs = synth.channel_coverages(M, L, 7)
    ops = [nufft.Nufft(ny, nx, c) for c in covs]
    x = np.abs(RNG.standard_normal((ny, nx, L)))
    xc = x + 0.1 * RNG.standard_normal((ny, nx, L))
    y = [op.forward(x[..., l]) + 0.5 * (RNG.standard_normal(M) + 1j * RNG.standard_normal(M))
         for l, op in enumerate(ops)]
    v = [0.1 * (RNG.standard_normal(M) + 1j * RNG.standard_normal(M)) for _ in range(L)]
    eps = np.full(L, 2.0)
    eta = np.array([0.5, 1.0, 2.0])
    # U = I: v+ = (I - P_B)(v + Phi xcheck) whatever the number of sub-iterations
    ones = [np.ones(M)] * L
    for n_sub in (0, 3):
        vn, g, r = nufft.data_dual_update(x, xc, v, y, ones, eps, eta, n_sub, ops)
        for l in range(L):
            z = v[l] + ops[l].forward(xc[..., l])
            assert np.allclose(vn[l], z - nufft.project_ball(z, y[l], eps[l]), atol=1e-12)
            assert np.allclose(g[..., l], eta[l] * ops[l].adjoint(vn[l]), atol=1e-12)
            assert abs(r[l] - np.linalg.norm(y[l] - ops[l].forward(x[..., l]))) < 1e-10
    # a preconditioned update, composed by hand
    U = [nufft.inverse_density(c, 2 * ny, 2 * nx) for c in covs]
    vn, g, r = nufft.data_dual_update(x, xc, v, y, U, eps, eta, 4, ops)
    for l in range(L):
        z = v[l] / U[l] + ops[l].forward(xc[..., l])
        p = nufft.project_ball_metric_fb(z, y[l], eps[l], U[l], 4)
        assert np.allclose(vn[l], U[l] * (z - p), atol=1e-12)
