"""Pins of the oracle's outer reweighting loop (Alg. 1) and of the stopping
rule of each PDFB run (Alg. 2): degenerate cases with a known outcome, the
loop conditions checked against the recorded histories, the residual
against its definition, the loop structure (two passes = one pass resumed),
the per-sub-cube loops of Alg. 1 / Alg. 2 (sub-cubes are independent
sub-problems, Sec. 2.4.1), and the method's purpose on a noisy cube (the
estimate beats the data)."""
import numpy as np
import pytest

import synth
from fhs_cases import Problem
from oracle import closure, heuristics, metrics, solve


def _noisy(ny=40, nx=36, L=6, q=2, o=4, levels=2, seed=3, frac=0.05, C=1):
    pb = Problem(ny, nx, L, q, q, C, o, o, levels, seed=seed, blobs=8)
    y, sig = synth.noisy_data(pb.X, frac, synth.BASE_SEED + 5 + seed)
    eps = np.full(L, closure.l2_ball_radius(sig, ny * nx))
    ups = np.array([heuristics.mu_sparsity(sig, pb.Lc)] * C)
    return pb, y, eps, ups


def _solve(pb, y, eps, ups, x0=None, P=None, W=None, v=None, **kw):
    x0 = np.maximum(y, 0.0) if x0 is None else x0
    return solve.reweighting_solve(x0, pb.P if P is None else P, pb.W if W is None else W,
                                   np.zeros(y.shape) if v is None else v, y, eps, pb.mu, pb.mu_bar, ups, pb.mu_bar,
                                   pb.geom, C=pb.C, levels=pb.levels, **kw)


def test_zero_data_runs_every_iteration():
    """y = 0 from X = 0 with zero duals: every quantity stays zero, so the
    relative variations are +inf (X = 0), each run reaches the iteration cap
    and the outer loop makes all T passes; the first weights are all one
    (upsilon / (0 + upsilon))."""
    pb = Problem(24, 20, 4, 2, 2, 1, 2, 2, 2, zero=True)
    y = np.zeros((24, 20, 4))
    eps = np.full(4, 0.5)
    th_bar = heuristics.nuclear_weights(y, pb.geom, pb.mu_bar)
    th = heuristics.l21_weights(y, np.array([0.3]), levels=2)
    assert all(np.all(t == 1.0) for row in th_bar for t in row) and np.all(th[0] == 1.0)
    x, P, W, v, _, _, rep = _solve(pb, y, eps, np.array([0.3]), x0=np.zeros(y.shape), T=3, xi_rw=0.5,
                                   p_min=1, p_max=4, xi_tol=1.0)
    assert [len(h) for h in rep["runs"][0]] == [4, 4, 4]
    assert all(np.isinf(xi) for h in rep["runs"][0] for xi, _ in h) and all(np.isinf(rep["xi"][0]))
    assert not np.any(x) and not np.any(v) and not any(np.any(w) for w in W)


def _check_histories(rep, eps, C, p_min, p_max, xi_tol, res_factor):
    for c in range(C):
        bound = res_factor * np.linalg.norm(eps[c::C])
        for hist in rep["runs"][c]:
            n = len(hist)
            assert p_min <= n <= p_max
            done = [(xi <= xi_tol and r <= bound) for xi, r in hist]
            assert n == p_max or done[-1]
            assert not any(done[p_min - 1:n - 1])


@pytest.mark.parametrize("p_min,p_max,xi_tol,res_factor", [(2, 12, 1.2e-2, 1.01), (3, 40, 1e-2, 0.5), (2, 15, 1e-2, 1.01),
                                                           (1, 9, 0.0, 1.01), (5, 5, 1.0, 1e9)])
def test_stopping_rule_against_histories(p_min, p_max, xi_tol, res_factor):
    """Each run stops at the first p >= p_min where p = p_max or both xi_p <=
    xi_tol and ||r|| <= res_factor ||eps|| (Alg. 2 loop condition); the
    residual of the first iteration is ||y - X(0)|| of the run's input."""
    pb, y, eps, ups = _noisy()
    x0 = np.maximum(y, 0.0)
    _, _, _, _, _, _, rep = _solve(pb, y, eps, ups, x0=x0, T=2, xi_rw=0.0, p_min=p_min, p_max=p_max,
                                   xi_tol=xi_tol, res_factor=res_factor)
    assert rep["runs"][0][0][0][1] == pytest.approx(np.linalg.norm(y.astype(np.float64) - x0), rel=1e-14)
    _check_histories(rep, eps, 1, p_min, p_max, xi_tol, res_factor)


def test_stopping_rule_per_subcube():
    """With two sub-cubes each run's history obeys the loop condition of its
    own sub-problem: xi and ||r_c|| of its channels against ||eps_c|| (Alg. 2
    solves each spectral sub-problem); the first residual of sub-cube c is
    ||y_c - X_c(0)|| over its channels only."""
    pb, y, eps, ups = _noisy(L=8, C=2, seed=7)
    eps = eps * np.where(np.arange(8) % 2 == 0, 1.0, 1.7)   # unequal ball radii per sub-cube
    x0 = np.maximum(y, 0.0)
    kw = dict(p_min=2, p_max=30, xi_tol=1.5e-2, res_factor=1.01)
    _, _, _, _, _, _, rep = _solve(pb, y, eps, ups, x0=x0, T=2, xi_rw=0.0, **kw)
    for c in range(2):
        r0 = np.linalg.norm(y.astype(np.float64)[..., c::2] - x0[..., c::2])
        assert rep["runs"][c][0][0][1] == pytest.approx(r0, rel=1e-14)
    _check_histories(rep, eps, 2, kw["p_min"], kw["p_max"], kw["xi_tol"], kw["res_factor"])


def test_residual_bound_per_subcube():
    """The residual test of Alg. 2 uses the sub-cube's own l2-ball radii: with
    generous radii on sub-cube 0 and radii far below the noise on sub-cube 1,
    sub-cube 0 stops on its relative variation while sub-cube 1, whose
    residual never enters its bound, runs to the cap."""
    pb, y, eps, ups = _noisy(L=8, C=2, seed=10)
    eps = eps * np.where(np.arange(8) % 2 == 0, 3.0, 1e-3)
    kw = dict(T=1, xi_rw=0.0, p_min=2, p_max=16, xi_tol=2e-2, res_factor=1.01)
    _, _, _, _, _, _, rep = _solve(pb, y, eps, ups, **kw)
    assert len(rep["runs"][1][0]) == 16
    assert len(rep["runs"][0][0]) < 16
    _check_histories(rep, eps, 2, kw["p_min"], kw["p_max"], kw["xi_tol"], kw["res_factor"])


def test_subcubes_stop_independently():
    """Sub-cube 0 of a two-sub-cube problem has zero data and a zero start, so
    its relative variation stays +inf and each of its runs goes to the cap;
    sub-cube 1 is noisy and stops early on its own criteria.  The zero
    sub-cube stays zero, and the noisy one's result is that of a one-sub-cube
    solve on its own channels (eq. problem-split-subcube: independent
    sub-problems; Alg. 1 loops over c)."""
    pb, y, eps, ups = _noisy(L=8, C=2, seed=8)
    y = y.astype(np.float64)
    y[..., 0::2] = 0.0
    x0 = np.maximum(y, 0.0)
    kw = dict(T=2, xi_rw=0.0, p_min=2, p_max=14, xi_tol=2e-2, res_factor=1.01)
    x, P, W, v, th, thb, rep = _solve(pb, y, eps, ups, x0=x0, **kw)
    assert [len(h) for h in rep["runs"][0]] == [14, 14]
    n1 = [len(h) for h in rep["runs"][1]]
    assert all(n < 14 for n in n1), n1
    assert not np.any(x[..., 0::2]) and not np.any(v[..., 0::2]) and not np.any(W[0])
    assert not any(np.any(p) for p in P[0])
    # the same sub-problem alone
    p1 = Problem(pb.ny, pb.nx, pb.Lc, pb.geom.qy, pb.geom.qx, 1, pb.geom.oy, pb.geom.ox, pb.levels)
    p1.P, p1.W = [pb.P[1]], [pb.W[1]]
    p1.mu, p1.mu_bar = pb.mu[1:], pb.mu_bar[1:]
    x1, P1, W1, v1, th1, thb1, rep1 = _solve(p1, y[..., 1::2], eps[1::2], ups[1:], x0=x0[..., 1::2], **kw)
    assert [len(h) for h in rep1["runs"][0]] == n1
    np.testing.assert_array_equal(x[..., 1::2], x1)
    np.testing.assert_array_equal(v[..., 1::2], v1)
    np.testing.assert_array_equal(W[1], W1[0])
    np.testing.assert_array_equal(th[1], th1[0])
    for a, b in zip(P[1], P1[0]):
        np.testing.assert_array_equal(a, b)


def test_outer_loop_stops_on_relative_variation():
    """A bound above the first run's variation ends the loop after one pass; a
    zero bound runs all T passes (Alg. 1 loop condition)."""
    pb, y, eps, ups = _noisy()
    kw = dict(p_min=2, p_max=3, xi_tol=0.0)
    _, _, _, _, _, _, rep = _solve(pb, y, eps, ups, T=4, xi_rw=10.0, **kw)
    assert len(rep["runs"][0]) == 1 and rep["xi"][0][0] < 10.0
    _, _, _, _, _, _, rep = _solve(pb, y, eps, ups, T=3, xi_rw=0.0, **kw)
    assert len(rep["runs"][0]) == 3 and all(xi > 0 for xi in rep["xi"][0])


def test_outer_loop_per_subcube():
    """Each sub-cube ends its own reweighting loop: a zero sub-cube (relative
    variation +inf) makes all T passes while a noisy one whose first
    variation is below the bound stops after one (Alg. 1, loop inside
    'for c')."""
    pb, y, eps, ups = _noisy(L=8, C=2, seed=9)
    y = y.astype(np.float64)
    y[..., 0::2] = 0.0
    x0 = np.maximum(y, 0.0)
    _, _, _, _, _, _, rep = _solve(pb, y, eps, ups, x0=x0, T=3, xi_rw=10.0, p_min=2, p_max=3, xi_tol=0.0)
    assert len(rep["runs"][0]) == 3 and all(np.isinf(rep["xi"][0]))
    assert len(rep["runs"][1]) == 1 and rep["xi"][1][0] < 10.0


def test_two_passes_equal_one_pass_resumed():
    """Alg. 1 carries X, P, W and v from one pass to the next and recomputes
    the weights from X: two passes equal one pass, then one more pass started
    from its outputs."""
    pb, y, eps, ups = _noisy(seed=4)
    kw = dict(p_min=2, p_max=2, xi_tol=0.0, xi_rw=0.0)
    x2, P2, W2, v2, th2, thb2, _ = _solve(pb, y, eps, ups, T=2, **kw)
    x1, P1, W1, v1, _, _, _ = _solve(pb, y, eps, ups, T=1, **kw)
    xr, Pr, Wr, vr, thr, thbr, _ = _solve(pb, y, eps, ups, x0=x1, P=P1, W=W1, v=v1, T=1, **kw)
    np.testing.assert_array_equal(x2, xr)
    np.testing.assert_array_equal(v2, vr)
    np.testing.assert_array_equal(W2[0], Wr[0])
    np.testing.assert_array_equal(th2[0], thr[0])


def test_reweighting_solve_denoises():
    """The point of the method: on a noisy cube the estimate is closer to the
    truth than the data (Sec. 4.3 SNR), and reweighting passes do not undo it."""
    pb, y, eps, ups = _noisy()
    x, _, _, _, _, _, rep = _solve(pb, y, eps, ups, T=3, xi_rw=1e-3, p_min=3, p_max=30, xi_tol=1e-3)
    s_data, s_est = metrics.snr(pb.X, y).mean(), metrics.snr(pb.X, x).mean()
    assert s_est > s_data + 5.0, (s_data, s_est)
    assert rep["xi"][0][-1] < rep["xi"][0][0]


def test_residual_is_taken_on_the_iterate_entering_each_iteration():
    """Alg. 2 residual step: iteration p measures ||y - x|| on x^(p), the
    iterate it starts from, which is the output of a run capped at p
    iterations (runs are prefixes of each other)."""
    pb, y, eps, ups = _noisy(seed=5)
    kw = dict(T=1, xi_rw=0.0, xi_tol=0.0)
    hist = _solve(pb, y, eps, ups, p_min=4, p_max=4, **kw)[-1]["runs"][0][0]
    for k in range(1, 4):
        xk = _solve(pb, y, eps, ups, p_min=k, p_max=k, **kw)[0]
        assert hist[k][1] == pytest.approx(np.linalg.norm(y.astype(np.float64) - xk), rel=1e-13)


def test_each_run_restarts_the_extrapolation_at_its_input():
    """Each PDFB run starts with Xcheck = X of its input (Alg. 2
    initialisation), not with the previous run's extrapolated point: one
    iteration per run, composed by hand from the paper's steps (weights,
    facet step on Xcheck, data dual, primal update)."""
    from oracle import step
    pb, y, eps, ups = _noisy(seed=6)
    tau = 0.33
    x, P, W, v = np.maximum(y, 0.0).astype(np.float64), pb.P, pb.W, np.zeros(y.shape)
    for _ in range(2):
        thb = heuristics.nuclear_weights(x, pb.geom, pb.mu_bar)
        th = heuristics.l21_weights(x, ups, levels=pb.levels)
        P, W, G = step.facet_prox_step(x, P, W, th, thb, pb.mu, pb.mu_bar, 1.0, 1.0, pb.geom)
        v = closure.data_dual_update(v, x, y, eps)
        x = np.maximum(0.0, x - tau * (G + v))
    got = _solve(pb, y, eps, ups, T=2, xi_rw=0.0, p_min=1, p_max=1, xi_tol=0.0, tau=tau)
    np.testing.assert_allclose(got[0], x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(got[3], v, rtol=0, atol=1e-13)
