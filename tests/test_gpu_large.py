"""Full-size workloads on the GPU, checked against the FP64 oracle on a
sampled block, and the 50-iteration HIP graph of the batched spectral case.

Sampled parity: the oracle runs the facet step on the top-left 3 x 3 facets
of the cube (same tile size, overlap and weights).  There it is exact for the
nuclear duals of the four facets whose right / bottom neighbours lie inside
the block (their windows and apodization are those of the full problem), for
the wavelet coefficients at level j with both indices below n_block / 2^j
(the causal transform reads only lower indices), and for the gradient on the
first tile (its facets are among those four, and its wavelet support ends
well inside the block).  Same bar as the other parity tests.
"""
import time

import numpy as np
import pytest

import synth
from fhs_cases import log, max_rel, rel_l2
from oracle import closure, geometry, sara, step

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = 1e-5
ELEM = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(name, got, ref):
    e, m = rel_l2(got, ref), max_rel(got, ref)
    log(f"    {name}: rel_l2={e:.3e} max_rel={m:.3e} ({np.asarray(ref).size} values)")
    assert e <= TOL, (name, e)
    assert m <= ELEM, (name, m)


def full_inputs(w):
    X = synth.workload_cube(w)
    plan = fhs.Plan(w.ny, w.nx, w.L, w.qy, w.qx, w.C, w.overlap, w.overlap, w.levels).attach_workspace()
    s = plan.sizes
    seed = synth.BASE_SEED + w.seed_offset
    theta = synth.uniform_weights(s["n_theta"], seed + 11)
    tbar = [synth.sorted_weights(plan.Lc, seed + 100 + f) for f in range(s["n_facets"])]
    mu, mub = plan.heuristics(synth.sigma_bar(X))
    return X, plan, theta, tbar, mu, mub


@pytest.mark.parametrize("wname", ["cfg4_2048x2048x100_c10", "cfg5_4096x4096x64", "cfg3_2048x2048x60"])
def test_sampled_block_parity(wname):
    w = synth.WORKLOADS[wname]
    log(f"[case] sampled 3x3-facet block parity, {wname}")
    X, plan, theta, tbar, mu, mub = full_inputs(w)
    s = plan.sizes
    p = torch.zeros(s["n_p"], dtype=torch.float32, device="cuda")
    wt = torch.zeros(s["n_w"], dtype=torch.float32, device="cuda")
    g = torch.empty(s["n_x"], dtype=torch.float32, device="cuda")
    plan.facet_prox_step(dev(X), p, wt, dev(theta), dev(np.concatenate(tbar)), dev(mu), dev(mub), 1.0, 1.0, g)
    torch.cuda.synchronize()
    log("    gpu step done")

    k, C, Lc, L, lev = 3, w.C, w.L // w.C, w.L, w.levels
    Q = w.qy * w.qx
    f00 = plan.facet(0)
    ys, xs = plan.facet((k - 1) * w.qx + (k - 1))["ty1"], plan.facet((k - 1) * w.qx + (k - 1))["tx1"]
    geom = geometry.Geometry(ys, xs, k, k, w.overlap, w.overlap, lev)
    full_bands = plan.bands()
    sub_bands = sara.band_shapes(ys, xs, lev)
    I_full, I_sub = s["n_coef"], sara.n_coefficients(ys, xs, lev)
    # theta of the block: the full problem's weight of the same band position
    th_full = theta.reshape(C, I_full)
    th_sub = np.zeros((C, I_sub), dtype=np.float32)
    off_s = 0
    for (rf, cf, off_f, _), (rs, cs) in zip(full_bands, sub_bands):
        th_sub[:, off_s:off_s + rs * cs] = th_full[:, off_f:off_f + rf * cf].reshape(C, rf, cf)[:, :rs, :cs] \
            .reshape(C, -1)
        off_s += rs * cs
    full_f = lambda c, sy, sx: c * Q + sy * w.qx + sx
    tb_sub = [[tbar[full_f(c, q // k, q % k)] for q in range(k * k)] for c in range(C)]
    mub_sub = [[mub[full_f(c, q // k, q % k)] for q in range(k * k)] for c in range(C)]
    P0 = [[np.zeros(f.nuc_shape + (Lc,)) for f in geom.facets] for _ in range(C)]
    W0 = [np.zeros((I_sub, Lc)) for _ in range(C)]
    t0 = time.time()
    Pn, Wn, G = step.facet_prox_step(X[:ys, :xs], P0, W0, list(th_sub), tb_sub, mu, mub_sub, 1.0, 1.0, geom, C=C)
    log(f"    oracle on {ys}x{xs}x{L} done in {time.time() - t0:.1f} s")

    # nuclear duals of the interior facets of the block
    got, ref = [], []
    for c in range(C):
        for sy in range(k - 1):
            for sx in range(k - 1):
                fi = plan.facet(full_f(c, sy, sx))
                n = (fi["wy1"] - fi["wy0"]) * (fi["wx1"] - fi["wx0"]) * Lc
                got.append(p[fi["poff"]:fi["poff"] + n].cpu().numpy())
                ref.append(Pn[c][sy * k + sx].reshape(-1))
    check("P+ (interior facets of the block)", np.concatenate(got), np.concatenate(ref))

    # wavelet coefficients below the block's exactness bound
    got, ref = [], []
    w2 = wt.view(I_full, L)
    off_s = 0
    for (rf, cf, off_f, level), (rs, cs) in zip(full_bands, sub_bands):
        j = max(level, 0)
        rv, cv = (ys >> j, xs >> j) if j > 0 else (ys, xs)
        rv, cv = min(rv, rs), min(cv, cs)
        got.append(w2[off_f:off_f + rf * cf].view(rf, cf, L)[:rv, :cv].cpu().numpy().reshape(-1, L))
        blk = np.concatenate([Wn[c][off_s:off_s + rs * cs].reshape(rs, cs, Lc)[:rv, :cv] for c in range(C)],
                             axis=2)
        ref.append(blk.reshape(-1, L))
        off_s += rs * cs
    check("W+ (exact region of every band)", np.concatenate(got), np.concatenate(ref))

    # gradient on the first tile
    ty1, tx1 = f00["ty1"], f00["tx1"]
    gg = g.view(w.ny, w.nx, L)[:ty1, :tx1].cpu().numpy()
    check("G (first tile)", gg, G[:ty1, :tx1])


def test_cfg4_graph_50_iterations():
    """2048 x 2048 x 100, 8 x 8 facets x 10 interleaved sub-cubes: 50 PDFB
    iterations (identity data term) as one HIP graph, replayed twice, equal
    bit for bit to 50 eager iterations."""
    w = synth.WORKLOADS["cfg4_2048x2048x100_c10"]
    log("[case] cfg4 graph of 50 iterations")
    X, plan, theta, tbar, mu, mub = full_inputs(w)
    y, sig = synth.noisy_data(X, 0.05, synth.BASE_SEED + 4077)
    eps = np.full(w.L, closure.l2_ball_radius(sig, w.ny * w.nx))
    x0 = np.maximum(y, 0.0).astype(np.float32)
    s = plan.sizes
    n = 50
    const = dict(y=dev(y), eps=dev(eps), theta=dev(theta), theta_bar=dev(np.concatenate(tbar)), mu=dev(mu),
                 mu_bar=dev(mub))
    del X, y

    def fresh():
        t = dict(x=dev(x0), xcheck=dev(x0), p=torch.zeros(s["n_p"], dtype=torch.float32, device="cuda"),
                 w=torch.zeros(s["n_w"], dtype=torch.float32, device="cuda"),
                 v=torch.zeros(s["n_x"], dtype=torch.float32, device="cuda"),
                 grad=torch.empty(s["n_x"], dtype=torch.float32, device="cuda"),
                 xi=torch.zeros(n * w.C, dtype=torch.float64, device="cuda"))
        return t, plan.pdfb_state(**t, **const)

    te, ste = fresh()
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(n):
        plan.pdfb_iteration(ste, i)
    torch.cuda.synchronize()
    t_eager = (time.time() - t0) / n
    log(f"    eager: {t_eager * 1e3:.2f} ms / iteration; xi[0]={te['xi'][0].item():.3e} "
        f"xi[-1]={te['xi'][-1].item():.3e}")
    assert torch.isfinite(te["xi"]).all()
    tg, stg = fresh()
    graph = plan.pdfb_graph(stg, n)
    for rep in range(2):
        if rep:
            for key, val in fresh()[0].items():
                tg[key].copy_(val)
        torch.cuda.synchronize()
        t0 = time.time()
        graph.launch()
        torch.cuda.synchronize()
        t_graph = (time.time() - t0) / n
        for key in ("x", "xcheck", "v", "p", "w", "xi"):
            assert torch.equal(tg[key], te[key]), (rep, key)
        log(f"    graph replay {rep}: {t_graph * 1e3:.2f} ms / iteration, identical to eager")
    graph.close()
