"""Host-side checks of the full-size test plumbing (no GPU): the warm duals
written for the device equal the ones the sampled-block oracle evaluates, and
the extraction of a block's results from the library's packed layouts (P per
facet, W in global band order, G) selects exactly the values the oracle's
block step computes.  Runs the library's plan functions (host code) and torch
CPU tensors in place of device ones."""
import numpy as np
import pytest

import synth
from fhs_cases import block_errors, device_block_outputs, fill_warm_duals, random_weight_inputs, warm_oracle_inputs
from oracle import blocks, geometry, heuristics, sara, step

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")


@pytest.mark.parametrize("C", [1, 2])
def test_block_extraction_matches_oracle_layouts(C):
    ny, nx, L, qy, qx, o, lev = 200, 168, 4 * C, 4, 3, 10, 2
    geom = geometry.Geometry(ny, nx, qy, qx, o, o, lev)
    plan = fhs.Plan(ny, nx, L, qy, qx, C, o, o, lev)
    s = plan.sizes
    X = synth.blob_cube(ny, nx, L, 30, synth.BASE_SEED + 611)
    sb = synth.sigma_bar(X)
    mu, mub = plan.heuristics(sb)
    mub2 = np.asarray(mub).reshape(C, geom.Q)
    # the device fill (on CPU tensors) against the oracle-side callables
    p = torch.zeros(s["n_p"], dtype=torch.float32)
    w = torch.zeros(s["n_w"], dtype=torch.float32)
    fill_warm_duals(plan, p, w, mu, mub, chunk_rows=1000)
    P0, W0 = warm_oracle_inputs(geom, C, L, mu, mub2)
    Lc = L // C
    for c in range(C):
        for f in geom.facets:
            fi = plan.facet(c * geom.Q + f.index)
            n = f.n_rows * Lc
            assert np.array_equal(p[fi["poff"]:fi["poff"] + n].numpy(), P0(c, f).reshape(-1))
    shapes = sara.band_shapes(ny, nx, lev)
    wv = w.view(s["n_coef"], L).numpy()
    off = 0
    for k, (a, b) in enumerate(shapes):
        rr, cc = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
        for c in range(C):
            assert np.array_equal(wv[off:off + a * b, c * Lc:(c + 1) * Lc].reshape(a, b, Lc), W0(rr, cc, k, c))
        off += a * b
    # the full oracle step, packed into the library's layouts, seen through the extraction
    theta = synth.uniform_weights(s["n_theta"], 5)
    tbar = [synth.sorted_weights(Lc, 50 + f) for f in range(s["n_facets"])]
    Pw = [[P0(c, f) for f in geom.facets] for c in range(C)]
    Ww = [wv[:, c * Lc:(c + 1) * Lc].copy() for c in range(C)]
    th = [theta.reshape(C, -1)[c] for c in range(C)]
    tb = [[tbar[c * geom.Q + q] for q in range(geom.Q)] for c in range(C)]
    Pn, Wn, G = step.facet_prox_step(X, Pw, Ww, th, tb, mu, mub2, 1.0, 1.0, geom, C=C)
    pd = torch.zeros(s["n_p"], dtype=torch.float32)
    for c in range(C):
        for f in geom.facets:
            fi = plan.facet(c * geom.Q + f.index)
            pd[fi["poff"]:fi["poff"] + f.n_rows * Lc] = torch.from_numpy(Pn[c][f.index].reshape(-1).astype(np.float32))
    wd = torch.from_numpy(np.concatenate(Wn, axis=1).astype(np.float32).reshape(-1))
    gd = torch.from_numpy(G.astype(np.float32).reshape(-1))
    theta_f, theta_bar_f = random_weight_inputs(geom, C, theta, tbar)
    for spec in [(0, 0, 2, 2), (qy - 1, qx - 1, 1, 1), (1, qx - 1, 2, 1), (1, 1, 2, 2)]:
        blk = blocks.make_block(geom, *spec)
        got = device_block_outputs(plan, pd, wd, gd, geom, blk)
        ref = blocks.block_step(X, geom, blk, C, mu, mub2, P0=P0, W0=W0, theta=theta_f, theta_bar=theta_bar_f)
        for key, (e, m, n) in block_errors(got, ref).items():
            assert n > 0 and e < 1e-6 and m < 1e-5, (spec, key, e, m)
