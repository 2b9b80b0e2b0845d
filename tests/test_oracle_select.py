"""Pins of the oracle's randomized facet step (Sec. 3.2: a random subset of the
facet dual variables is updated at an iteration).

* everything selected: the plain facet step;
* nothing selected: the duals are unchanged and G is the aggregation of the
  old duals, computed here through the explicit faceted synthesis;
* G is linear in the duals, and the duals of disjoint selections do not
  interact: G(S1) + G(S2) = G(S1 u S2) + G(empty);
* a selected facet's l21 dual equals its facet-local update, with the
  analysis of the facet's own SARA window (Sec. 2.4.2), and every other
  coefficient row keeps its value.
"""
import numpy as np
import pytest

import synth
from oracle import geometry, prox, sara, step

LEVELS = 2


def problem(C, seed=3):
    ny, nx, L = 64, 56, 4 * C
    geom = geometry.Geometry(ny, nx, 3, 2, 6, 6, LEVELS)
    X = synth.blob_cube(ny, nx, L, 12, seed)
    Lc = L // C
    r = np.random.default_rng(seed + 1)
    I = sara.n_coefficients(ny, nx, LEVELS)
    P = [[0.05 * r.standard_normal(f.nuc_shape + (Lc,)) for f in geom.facets] for _ in range(C)]
    W = [0.02 * r.standard_normal((I, Lc)) for _ in range(C)]
    theta = [synth.uniform_weights(I, seed + 2 + c) for c in range(C)]
    tbar = [[synth.sorted_weights(Lc, 40 + c * geom.Q + q) for q in range(geom.Q)] for c in range(C)]
    mu = np.full(C, 0.03)
    mub = np.full((C, geom.Q), 0.4) * (1.0 + 0.1 * np.arange(geom.Q))
    return geom, X, P, W, theta, tbar, mu, mub


def run(C, select, zeta=1.0, kappa=1.0):
    geom, X, P, W, theta, tbar, mu, mub = problem(C)
    return geom, X, P, W, step.facet_prox_step_select(X, P, W, theta, tbar, mu, mub, zeta, kappa, geom, select, C=C)


@pytest.mark.parametrize("C", [1, 2])
def test_all_selected_is_the_plain_step(C):
    geom, X, P, W, theta, tbar, mu, mub = problem(C)
    sel = np.ones((C, geom.Q), dtype=bool)
    Ps, Ws, Gs = step.facet_prox_step_select(X, P, W, theta, tbar, mu, mub, 0.8, 1.3, geom, sel, C=C)
    Pp, Wp, Gp = step.facet_prox_step(X, P, W, theta, tbar, mu, mub, 0.8, 1.3, geom, C=C)
    for c in range(C):
        for q in range(geom.Q):
            assert np.allclose(Ps[c][q], Pp[c][q], rtol=0, atol=1e-13)
        assert np.allclose(Ws[c], Wp[c], rtol=0, atol=1e-13)
    assert np.allclose(Gs, Gp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("C", [1, 2])
def test_nothing_selected_keeps_the_duals(C):
    geom, X, P, W, theta, tbar, mu, mub = problem(C)
    sel = np.zeros((C, geom.Q), dtype=bool)
    zeta, kappa = 0.7, 1.6
    Ps, Ws, G = step.facet_prox_step_select(X, P, W, theta, tbar, mu, mub, zeta, kappa, geom, sel, C=C)
    L = X.shape[2]
    chans = step.subcube_channels(L, C)
    ref = np.zeros(X.shape)
    for c in range(C):
        for q, f in enumerate(geom.facets):
            assert np.array_equal(Ps[c][q], P[c][q])
            (y0, y1), (x0, x1) = f.nuc_window
            ref[y0:y1, x0:x1][..., chans[c]] += zeta * f.window()[..., None] * P[c][q]
        assert np.array_equal(Ws[c], W[c])
        bands = sara.unflatten(W[c], geom.ny, geom.nx, LEVELS)
        ref[..., chans[c]] += kappa * sara.faceted_synthesis(bands, geom, LEVELS)
    assert np.allclose(G, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("C", [1, 2])
def test_disjoint_selections_add(C):
    geom = problem(C)[0]
    draw = synth.facet_selection(C, geom.Q, 0.5, 17)
    s1, s2 = draw, ~draw
    assert s1.any() and s2.any()
    G1 = run(C, s1)[-1][2]
    G2 = run(C, s2)[-1][2]
    Gall = run(C, np.ones_like(draw))[-1][2]
    Gnone = run(C, np.zeros_like(draw))[-1][2]
    assert np.allclose(G1 + G2, Gall + Gnone, rtol=0, atol=1e-11)


@pytest.mark.parametrize("C", [1, 2])
def test_selected_facets_take_their_local_update(C):
    geom, X, P, W, theta, tbar, mu, mub = problem(C)
    sel = synth.facet_selection(C, geom.Q, 0.5, 23)
    sel[0, 0], sel[-1, -1] = True, False
    Ps, Ws, _ = step.facet_prox_step_select(X, P, W, theta, tbar, mu, mub, 1.0, 1.0, geom, sel, C=C)
    L = X.shape[2]
    chans = step.subcube_channels(L, C)
    Lc = L // C
    for c in range(C):
        old = sara.unflatten(W[c], geom.ny, geom.nx, LEVELS)
        new = sara.unflatten(Ws[c], geom.ny, geom.nx, LEVELS)
        th = sara.unflatten(theta[c], geom.ny, geom.nx, LEVELS)
        owned = np.zeros(sara.n_coefficients(geom.ny, geom.nx, LEVELS), dtype=bool)
        for q, f in enumerate(geom.facets):
            # the facet's own transform: its SARA window alone (zero elsewhere)
            (y0, y1), (x0, x1) = f.sara_window
            xw = np.zeros((geom.ny, geom.nx, Lc))
            xw[y0:y1, x0:x1] = X[y0:y1, x0:x1][..., chans[c]]
            local = sara.analysis(xw, LEVELS)
            for k, ((r0, r1), (c0, c1)) in enumerate(geom.owned_rects(f)):
                got = new[k][r0:r1, c0:c1].reshape(-1, Lc)
                if sel[c, q]:
                    u = old[k][r0:r1, c0:c1].reshape(-1, Lc) + local[k][r0:r1, c0:c1].reshape(-1, Lc)
                    a = mu[c] * th[k][r0:r1, c0:c1].reshape(-1)
                    assert np.allclose(got, prox.l21_prox_complement(u, a), rtol=0, atol=1e-13)
                else:
                    assert np.array_equal(got, old[k][r0:r1, c0:c1].reshape(-1, Lc))
            if not sel[c, q]:
                assert np.array_equal(Ps[c][q], P[c][q])
            else:
                Z = P[c][q].reshape(-1, Lc) + step.facet_matrix(X, f, chans[c])
                ref = prox.weighted_svt_complement(Z, mub[c][q] * np.asarray(tbar[c][q]))
                assert np.allclose(Ps[c][q].reshape(-1, Lc), ref, rtol=0, atol=1e-13)
