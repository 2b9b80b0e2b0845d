"""Full-size workloads on the GPU, checked against the FP64 oracle on sampled
blocks of facets, and the 50-iteration HIP graph of the batched spectral case.

Sampled parity (oracle/blocks.py): the step is local (Sec. 2.4.2), so the
oracle computes, on a block of facets and a sub-image reaching E pixels above /
left of it, exactly what the full problem gives for the block's facets (P+),
the coefficient rows they own (W+) and the tiles whose right / bottom
neighbours are in the block or outside the image (G).  Blocks: the top-left
corner, the bottom-right corner (the last facet: no falling ramp, owns the
band tails), a right-edge pair, and the 2 x 2 block around the brightest
pixel.  Inputs: zero duals with random weights (top-left), warm duals (from
the counter-based generator, identical on host and device) with random
weights at 2048^2, and at 4096^2 x 64 warm duals with the reweighting weights
of the cube itself (eqs. facet_hypersara_rank, facet_hypersara_sparsity;
fhs_reweight on the device, the oracle's own weights on the host).  Same bar as
the other parity tests: relative L2 <= 1e-5 per output and element-wise
<= 1e-4 of the largest magnitude.
"""
import time

import numpy as np
import pytest

import synth
from fhs_cases import (block_errors, device_block_outputs, fill_warm_duals, log, random_weight_inputs,
                       warm_oracle_inputs)
from oracle import blocks, closure, geometry

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = 1e-5
ELEM = 1e-4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def full_inputs(w):
    X = synth.workload_cube(w)
    plan = fhs.Plan(w.ny, w.nx, w.L, w.qy, w.qx, w.C, w.overlap, w.overlap, w.levels).attach_workspace()
    s = plan.sizes
    seed = synth.BASE_SEED + w.seed_offset
    theta = synth.uniform_weights(s["n_theta"], seed + 11)
    tbar = [synth.sorted_weights(plan.Lc, seed + 100 + f) for f in range(s["n_facets"])]
    mu, mub = plan.heuristics(synth.sigma_bar(X))
    return X, plan, theta, tbar, mu, mub


def bright_block(X, geom):
    """2 x 2 block of facets around the brightest pixel (summed over channels)."""
    iy, ix = np.unravel_index(np.argmax(np.sum(X, axis=2, dtype=np.float64)), X.shape[:2])
    ty, tx = geometry.tile_bounds(geom.ny, geom.qy), geometry.tile_bounds(geom.nx, geom.qx)
    sy = int(np.searchsorted(ty, iy, side="right")) - 1
    sx = int(np.searchsorted(tx, ix, side="right")) - 1
    return min(max(sy, 0), geom.qy - 2), min(max(sx, 0), geom.qx - 2), 2, 2


def block_spec(name, X, geom):
    if name == "top_left":
        return 0, 0, 2, 2
    if name == "bottom_right":
        return geom.qy - 1, geom.qx - 1, 1, 1
    if name == "right_edge":
        return geom.qy // 2 - 1, geom.qx - 1, 2, 1
    return bright_block(X, geom)


# (workload, input variant, block): variant "zero" = zero duals and random
# weights, "warm" = warm duals and random weights, "reweight" = warm duals and
# the cube's own reweighting weights
CASES = [
    ("cfg3_2048x2048x60", "zero", "top_left"),
    ("cfg3_2048x2048x60", "warm", "right_edge"),
    ("cfg3_2048x2048x60", "warm", "bright"),
    ("cfg4_2048x2048x100_c10", "zero", "top_left"),
    ("cfg4_2048x2048x100_c10", "warm", "bottom_right"),
    ("cfg4_2048x2048x100_c10", "warm", "bright"),
    ("cfg5_4096x4096x64", "zero", "top_left"),
    ("cfg5_4096x4096x64", "reweight", "bottom_right"),
    ("cfg5_4096x4096x64", "reweight", "right_edge"),
    ("cfg5_4096x4096x64", "reweight", "bright"),
]

_cache = {}


def gpu_run(wname, variant):
    """One facet step of the full workload on the device for an input variant,
    cached for the blocks that follow (one workload held at a time)."""
    key = (wname, variant)
    if key in _cache:
        return _cache[key]
    _cache.clear()
    torch.cuda.empty_cache()
    w = synth.WORKLOADS[wname]
    t0 = time.time()
    X, plan, theta, tbar, mu, mub = full_inputs(w)
    s = plan.sizes
    x = dev(X)
    p = torch.zeros(s["n_p"], dtype=torch.float32, device="cuda")
    wt = torch.zeros(s["n_w"], dtype=torch.float32, device="cuda")
    g = torch.empty(s["n_x"], dtype=torch.float32, device="cuda")
    th, tb = dev(theta), dev(np.concatenate(tbar))
    mu_d, mub_d = dev(mu), dev(mub)
    if variant != "zero":
        fill_warm_duals(plan, p, wt, mu, mub)
    if variant == "reweight":
        # X^(t) = Xcheck at the start of a run, upsilon = mu, upsilon_bar = mu_bar
        plan.reweight(x, mu_d, mub_d, th, tb)
    plan.facet_prox_step(x, p, wt, th, tb, mu_d, mub_d, 1.0, 1.0, g)
    torch.cuda.synchronize()
    log(f"    {wname} ({variant}): inputs and device step in {time.time() - t0:.1f} s")
    geom = geometry.Geometry(w.ny, w.nx, w.qy, w.qx, w.overlap, w.overlap, w.levels)
    _cache[key] = dict(w=w, X=X, plan=plan, theta=theta, tbar=tbar, mu=mu, mub=mub, p=p, wt=wt, g=g, geom=geom)
    return _cache[key]


@pytest.mark.parametrize("wname,variant,where", CASES, ids=[f"{a}-{b}-{c}" for a, b, c in CASES])
def test_sampled_block_parity(wname, variant, where):
    log(f"[case] sampled block parity {wname} {variant} {where}")
    r = gpu_run(wname, variant)
    w, X, plan, geom = r["w"], r["X"], r["plan"], r["geom"]
    C, Lc = w.C, w.L // w.C
    mub = np.asarray(r["mub"]).reshape(C, geom.Q)
    blk = blocks.make_block(geom, *block_spec(where, X, geom))
    got = device_block_outputs(plan, r["p"], r["wt"], r["g"], geom, blk)
    kw = {}
    if variant != "zero":
        kw["P0"], kw["W0"] = warm_oracle_inputs(geom, C, w.L, r["mu"], mub)
    if variant != "reweight":
        kw["theta"], kw["theta_bar"] = random_weight_inputs(geom, C, r["theta"], r["tbar"])
    t0 = time.time()
    ref = blocks.block_step(X, geom, blk, C, r["mu"], mub, **kw)
    log(f"    oracle on block {blk} in {time.time() - t0:.1f} s")
    for k, (e, m, n) in block_errors(got, ref).items():
        log(f"    {k}: rel_l2={e:.3e} max_rel={m:.3e} ({n} values)")
        assert e <= TOL, (k, e)
        assert m <= ELEM, (k, m)


def test_cfg4_graph_50_iterations():
    """2048 x 2048 x 100, 8 x 8 facets x 10 interleaved sub-cubes: 50 PDFB
    iterations (identity data term) as one HIP graph, replayed twice, equal
    bit for bit to 50 eager iterations."""
    _cache.clear()
    torch.cuda.empty_cache()
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
