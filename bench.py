#!/usr/bin/env python3
"""Throughput of the facet-wise regularization step (facet_prox_step) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = fhs_facet_prox_step over the whole cube: the weighted nuclear-norm
dual update of every facet, the weighted l21 dual update of every coefficient
row and the gather of both into the primal gradient (Alg. 2, facet loop and
facet part of the aggregation).  Default workload: the 4096 x 4096 x 64 cube
with 16 x 16 facets and 128-px overlap, its reweighting weights computed from
the cube itself (eqs. facet_hypersara_rank and facet_hypersara_sparsity, the
iterate entering a PDFB run), zero duals.  Inputs are seeded synthetic cubes
(see synth/), resident in HBM before timing.  Prints ONE JSON line:
value = voxels / s (N * L per step), a roofline entry for the dominant kernel
(timed live with HIP events on its launch stream), and the FP64 CPU oracle on
a bounded sample of facets as the CPU baseline, whose outputs also give the
relative error of the step's outputs (P+, W+, G) on those facets.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "cfg5_4096x4096x64"
REL_ERR_BOUND = 1e-5


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(plan, w, kernel, form):
    """Algorithmic HBM bytes of the launches of `kernel` in one step (every
    input it must read and every state output it must write, once; no halo
    re-reads, no intermediate low-low bands) and its launches per step.  In
    the batched form the Dirac band's dual update runs in the first level-1
    synthesis group; in the per-facet form it runs in the level-1 analysis,
    which is launched once per spatial facet."""
    bands = plan.bands()
    N, L, C, lev = w.ny * w.nx, w.L, w.C, w.levels
    per_basis = 3 * lev + 1
    fused = form == "batched"

    def band_rows(b, j):          # rows of one detail band of basis b, level j (1-based)
        return bands[b * per_basis + 3 * (j - 1)][0] * bands[b * per_basis + 3 * (j - 1)][1]

    if kernel == "analysis_l1":
        tot = N * L * 4                                   # Xcheck
        for b in range(8):
            r = band_rows(b, 1)
            tot += 3 * r * (2 * L * 4 + C * 4)            # level-1 detail bands: W read + write, theta
            if lev == 1:
                tot += r * (2 * L * 4 + C * 4)            # (one level: the low-low band is W too)
        if not fused:
            tot += N * (2 * L * 4 + C * 4)                # Dirac band: W read + write, theta
        return tot, 1 if fused else w.qy * w.qx
    raise ValueError(f"no algorithmic byte count for kernel {kernel}")


def step_bytes(plan):
    """Algorithmic bytes of one whole step: Xcheck once, P and W read + written,
    theta, G written (float32)."""
    s = plan.sizes
    return 4 * (s["n_x"] + 2 * s["n_p"] + 2 * s["n_w"] + s["n_theta"] + s["n_x"])


def traffic_from_profiles(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources in the same precision form; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("precision", "fp32") != precision:
        return None
    from paper_2003_07358_amd.profiling import source_hash
    files = d.get("sources")
    if d.get("source_hash") != source_hash(None if files in (None, "all") else files):
        return None
    return d.get("hbm_bytes_per_launch")


# ---------------------------------------------------------------- CPU leg (oracle)
_CPU = {}


def _cpu_facet(spec):
    """One facet of the sample, in a worker process with one BLAS thread: its
    weights (untimed), then the timed facet step on it (oracle)."""
    from threadpoolctl import threadpool_limits

    from oracle import blocks
    sy, sx, keep = spec
    X, geom, C, mu, mub = _CPU["X"], _CPU["geom"], _CPU["C"], _CPU["mu"], _CPU["mub"]
    with threadpool_limits(limits=1):
        blk = blocks.make_block(geom, sy, sx, 1, 1)
        th, tb = blocks.block_weights(X, geom, blk, C, mu, mub)
        t0 = time.perf_counter()
        out = blocks.block_step(X, geom, blk, C, mu, mub, theta=th, theta_bar=tb)
        dt = time.perf_counter() - t0
    res = {"sy": sy, "sx": sx, "seconds": dt}
    if keep:
        res["P"] = {k: v.astype(np.float32) for k, v in out["P"].items()}
        res["W"] = [v.astype(np.float32) for v in out["W"]]
        res["G"] = out["G"].astype(np.float32)
    return res


def cpu_leg(w, X, procs, keep):
    """The FP64 oracle (oracle/blocks.py: the facet step of one facet, exact
    for it) on a bounded sample of facets, one facet per process and one BLAS
    thread each (the paper runs one facet per core): the bottom-right corner
    facet and facets along the middle row.  Runs before the GPU is touched
    (the pool forks).  Returns (cpu_baseline entry, oracle outputs of the first
    `keep` facets)."""
    import multiprocessing as mp

    from oracle import geometry, heuristics
    geom = geometry.Geometry(w.ny, w.nx, w.qy, w.qx, w.overlap, w.overlap, w.levels)
    C, Lc = w.C, w.L // w.C
    from threadpoolctl import threadpool_limits

    import synth
    sb = synth.sigma_bar(X)
    mu = np.array([heuristics.mu_sparsity(sb, Lc)] * C)
    mub = [[heuristics.mu_low_rank(sb, f.n_rows, Lc) for f in geom.facets] for _ in range(C)]
    # the corner, then facets in raster order from the middle row's centre on
    order = [(w.qy - 1, w.qx - 1)]
    start = (w.qy // 2) * w.qx + w.qx // 2
    for k in range(w.qy * w.qx):
        sy, sx = divmod((start + k) % (w.qy * w.qx), w.qx)
        if (sy, sx) not in order:
            order.append((sy, sx))
    specs = order[:procs]
    _CPU.update(X=X, geom=geom, C=C, mu=mu, mub=mub)
    t0 = time.perf_counter()
    with threadpool_limits(limits=1), mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_cpu_facet, [(sy, sx, i < keep) for i, (sy, sx) in enumerate(specs)], chunksize=1)
    wall = time.perf_counter() - t0
    _CPU.clear()
    tiles = [f for f in geom.facets if (f.sy, f.sx) in set(specs)]
    vox = sum((f.tile[0][1] - f.tile[0][0]) * (f.tile[1][1] - f.tile[1][0]) for f in tiles) * w.L
    per = sorted(r["seconds"] for r in res)
    vox1 = vox / len(specs)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    entry = {"value": vox / per[-1], "unit": "voxels/s", "cores": procs, "kind": "oracle",
             "sample": (f"{len(specs)} of the {w.qy * w.qx} facets (the bottom-right corner, then from the centre "
                        f"on), one facet per process with 1 BLAS thread, all at once; per facet the step on its "
                        f"window (SARA window transform, row shrink, synthesis; nuclear SVD), timed alone "
                        f"(weights computed before); value = sampled voxels / slowest facet "
                        f"({per[-1]:.1f} s, pool wall {wall:.1f} s), the whole-cube rate extrapolated linearly by "
                        f"facet count"),
             "single_core_value": vox1 / per[len(per) // 2], "nproc": os.cpu_count(), "cpu_model": model}
    return entry, [r for r in res if "P" in r], geom


def rel_errors(plan, geom, p_d, w_d, g_d, refs):
    """Relative L2 (and max relative) error of P+, W+, G of the device step on
    the sampled facets against the oracle's."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from fhs_cases import block_errors, device_block_outputs
    from oracle import blocks
    got_all, ref_all = {"P": {}, "W": [], "G": []}, {"P": {}, "W": [], "G": []}
    for r in refs:
        blk = blocks.make_block(geom, r["sy"], r["sx"], 1, 1)
        got = device_block_outputs(plan, p_d, w_d, g_d, geom, blk)
        got_all["P"].update(got["P"])
        ref_all["P"].update(r["P"])
        got_all["W"] += got["W"]
        ref_all["W"] += r["W"]
        got_all["G"].append(got["G"].reshape(-1))
        ref_all["G"].append(r["G"].reshape(-1))
    got_all["G"] = np.concatenate(got_all["G"])
    ref_all["G"] = np.concatenate(ref_all["G"])
    errs = block_errors(got_all, ref_all)
    return {k: {"rel_l2": e, "max_rel": m, "values": n} for k, (e, m, n) in errs.items()}


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--kernel", default="analysis_l1", help="kernel reported in the roofline entry")
    ap.add_argument("--cpu-procs", type=int, default=16, help="oracle processes (one facet each)")
    ap.add_argument("--cpu-keep", type=int, default=4, help="sampled facets whose outputs give the rel-err")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weights", choices=("reweight", "random"), default="reweight",
                    help="reweight: theta, theta_bar from the cube (fhs_reweight); random: U(0.5, 1)")
    ap.add_argument("--precision", choices=("fp32", "mixed"), default="fp32",
                    help="fp32: filters, Gram and reconstruction accumulated in FP64 (default); mixed: the "
                         "l21 filters in FP32 and the Gram on BF16 MFMA (FHS_PRECISION_MIXED)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default launch shapes")
    ap.add_argument("--form", choices=("batched", "plain"), default="batched",
                    help="batched: every operator one launch over all facets (default); plain: the "
                         "per-facet execution form, one launch per facet and operator")
    ap.add_argument("--tuning", default=None, metavar="JSON",
                    help="fixed launch shapes (a JSON object as printed in the 'tuning' field) instead of autotuning")
    ap.add_argument("--tuning-cache", default=None, metavar="PATH",
                    help="JSON cache of autotuned launch shapes (a hit skips the tuning)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (the reference "
                         "dispatch that scales HBM counters read under rocprofv3 --pmc)")
    ap.add_argument("--data-block", action="store_true",
                    help="time the data-fidelity dual update (measurement operator, preconditioned l2-ball "
                         "projection) on a 1024x2048x20 cube instead of the facet step")
    ap.add_argument("--vis-per-channel", type=int, default=1 << 20)
    ap.add_argument("--n-sub", type=int, default=10, help="forward-backward sub-iterations of the projection")
    ap.add_argument("--pdfb-graph", type=int, default=0, metavar="N",
                    help="time N whole PDFB iterations (identity data term) captured in one HIP graph on the "
                         "workload (default workload then: 2048x2048x100, 10 sub-cubes)")
    ap.add_argument("--spectral-overlap", type=int, default=0, metavar="O",
                    help="with --pdfb-graph: contiguous sub-cubes whose low-rankness facets overlap by O channels")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of the "
              "facet step is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    if args.data_block:
        return data_block_bench(args)
    if args.pdfb_graph:
        return pdfb_graph_bench(args)

    import synth
    w = synth.WORKLOADS[args.workload]
    log(f"[bench] workload {w.name}: generating inputs")
    X = synth.workload_cube(w)

    cpu, refs, geom = None, [], None
    if not args.no_cpu_baseline:
        procs = max(1, min(args.cpu_procs, len(os.sched_getaffinity(0)), w.qy * w.qx))
        log(f"[bench] CPU oracle baseline: {procs} facets in {procs} processes")
        if args.weights != "reweight":
            log("[bench] (the oracle sample uses the cube's reweighting weights; rel-err is skipped)")
        cpu, refs, geom = cpu_leg(w, X, procs, args.cpu_keep if args.weights == "reweight" else 0)
        log(f"[bench] CPU: {cpu['value']:.3e} voxels/s ({cpu['sample']})")

    import torch

    import paper_2003_07358_amd as fhs
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    mixed = args.precision == "mixed"
    plan = fhs.Plan(w.ny, w.nx, w.L, w.qy, w.qx, w.C, w.overlap, w.overlap, w.levels,
                    precision=1 if mixed else 0).attach_workspace()
    s = plan.sizes
    mu, mub = plan.heuristics(synth.sigma_bar(X))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x_d, mu_d, mub_d = dev(X), dev(mu), dev(mub)
    if args.weights == "reweight":
        th_d = torch.empty(s["n_theta"], dtype=torch.float32, device="cuda")
        tb_d = torch.empty(s["n_theta_bar"], dtype=torch.float64, device="cuda")
        plan.reweight(x_d, mu_d, mub_d, th_d, tb_d)   # X^(t) = Xcheck, upsilon = mu, upsilon_bar = mu_bar
    else:
        seed = synth.BASE_SEED + w.seed_offset
        th_d = dev(synth.uniform_weights(s["n_theta"], seed + 11))
        tb_d = dev(np.concatenate([synth.sorted_weights(plan.Lc, seed + 100 + f) for f in range(s["n_facets"])]))
    kappa_hist = None
    if mixed and args.weights == "reweight":
        # kappa_q = s_1(Z_q) / min_j t_j of every facet at the first step (Z = D_q Xcheck): with
        # upsilon_bar = mu_bar, theta_bar_1 = mu_bar / (s_1 + mu_bar) and t_min = mu_bar theta_bar_1,
        # so kappa = (1 / theta_bar_1 - 1) / theta_bar_1 (from the FP64 weights)
        tb1 = tb_d.view(s["n_facets"], plan.Lc)[:, 0].cpu().numpy()
        kappa = (1.0 / tb1 - 1.0) / tb1
        edges = [0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, np.inf]
        counts, _ = np.histogram(np.log10(np.maximum(kappa, 1e-300)), bins=edges)
        kappa_hist = {"log10_kappa_bin_edges": edges[:-1] + ["inf"], "facets": counts.tolist(),
                      "min": float(kappa.min()), "median": float(np.median(kappa)), "max": float(kappa.max())}
        log(f"[bench] kappa per facet: min {kappa.min():.3e} median {np.median(kappa):.3e} max {kappa.max():.3e}")
    p_d = torch.zeros(s["n_p"], dtype=torch.float32, device="cuda")
    w_d = torch.zeros(s["n_w"], dtype=torch.float32, device="cuda")
    g_d = torch.empty(s["n_x"], dtype=torch.float32, device="cuda")
    del X

    plain = args.form == "plain"

    def one_step():
        plan.facet_prox_step(x_d, p_d, w_d, th_d, tb_d, mu_d, mub_d, 1.0, 1.0, g_d, plain=plain)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)          # one elementwise kernel: reads n * 4 B, writes n * 4 B
        torch.cuda.synchronize()
        log(f"[bench] calibration copy kernel: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst

    if args.tuning:
        plan.tuning = json.loads(args.tuning)
        log(f"[bench] fixed tuning {plan.tuning}")
    elif not args.no_autotune and not plain:
        # launch shapes picked on the workload itself (outside the timed region);
        # the duals it scribbles on are reset afterwards
        t0a = time.perf_counter()
        tuning = plan.autotune(x_d, p_d, w_d, th_d, tb_d, mu_d, mub_d, g_d, reps=5, cache=args.tuning_cache)
        p_d.zero_()
        w_d.zero_()
        torch.cuda.synchronize()
        log(f"[bench] autotune {time.perf_counter() - t0a:.1f} s: {tuning}")

    # outputs of one step from zero duals, against the oracle on the sampled facets
    rel = None
    if refs:
        one_step()
        torch.cuda.synchronize()
        rel = rel_errors(plan, geom, p_d, w_d, g_d, refs)
        rel["bound"] = REL_ERR_BOUND
        rel["sample"] = f"{len(refs)} facets of the CPU sample (incl. the bottom-right corner tile for G), zero duals"
        log(f"[bench] rel-err vs FP64 oracle: " + ", ".join(f"{k} {v['rel_l2']:.2e}" for k, v in rel.items()
                                                           if isinstance(v, dict)))
        p_d.zero_()
        w_d.zero_()

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    plan.profile(args.kernel, max_launches=max(16, 4 * args.steps) * (w.qy * w.qx if plain else 1))
    log(f"[bench] timing {args.steps} steps")
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        one_step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / args.steps
    kms, launches = plan.profile_read()
    plan.profile(None)
    value = w.voxels / (ms / 1e3)
    kb, per_step = kernel_bytes(plan, w, args.kernel, args.form)
    avg_launch_s = (kms / launches) / 1e3 if launches else float("nan")
    achieved = kb / per_step / avg_launch_s / 1e9
    frac = achieved / HBM_PEAK_GBS
    if not frac <= 1.0:
        raise SystemExit(f"roofline fraction {frac:.3f} > 1: the byte count or the launch timing is wrong")
    traffic = traffic_from_profiles(args.kernel, w.name, args.precision) if not plain else None
    sb = step_bytes(plan)
    log(f"[bench] {ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f}); {args.kernel}: "
        f"{kms / max(launches, 1):.3f} ms/launch ({launches} launches), {achieved:.0f} GB/s; step bytes "
        f"{sb / 1e9:.2f} GB -> {sb / (ms / 1e3) / 1e9:.0f} GB/s")
    out = {
        "metric": "facet-prox voxels/s at rel-err<=1e-5 vs FP64 oracle; % HBM/MFMA peak",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 / bf16 (l21 filters accumulated in f32; Gram bf16 on MFMA, f32 accumulation; eig and "
                  "reconstruction f64)" if mixed else "f32 (filters, Gram and reconstruction accumulated in f64)"),
        "data": "synthetic (seeded Gaussian-blob cube with power-law spectra)",
        "config": {"workload": w.name, "form": args.form, "ny": w.ny, "nx": w.nx, "channels": w.L,
                   "facets": [w.qy, w.qx], "overlap_px": w.overlap, "subcubes": w.C, "levels": w.levels,
                   "bases": "db1-db8+dirac", "weights": args.weights, "duals": "zero at the first step",
                   "precision": args.precision,
                   "parallelism": "single GPU"},
        "roofline": {"kernel": args.kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": frac, "traffic": traffic,
                     "bytes_per_launch": kb / per_step, "avg_launch_ms": kms / max(launches, 1)},
        "rel_err": rel,
        "kappa_hist": kappa_hist,
        "tuning": plan.tuning,
        "step_hbm": {"algorithmic_bytes": sb, "achieved_GBs": sb / (ms / 1e3) / 1e9,
                     "frac": sb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def data_block_bench(args):
    """One fhs_data_dual_update per step (Alg. 2 data-fidelity lines: two
    forward NUFFTs, the preconditioned projection by sub-iterations, the
    adjoint into the gradient) on the 1024 x 2048 x 20 cube with a synthetic
    coverage of vis_per_channel points per channel, scaled by the frequency
    ratio.  Prints one JSON line (visibilities per second)."""
    import torch

    import paper_2003_07358_amd as fhs
    import synth
    w = synth.WORKLOADS["cfg2_1024x2048x20"]
    X = synth.workload_cube(w)
    L, M = w.L, args.vis_per_channel
    log(f"[bench] data block: {w.ny}x{w.nx}x{L}, {M} visibilities per channel, {args.n_sub} sub-iterations")
    covs = synth.channel_coverages(M, L, synth.BASE_SEED + 77)
    dp = fhs.DataPlan(w.ny, w.nx, covs).attach_workspace()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x = dev(X)
    U = dev(dp.preconditioner().astype(np.float32))
    y = torch.empty(dp.m, dtype=torch.complex64, device="cuda")
    dp.forward(x, y)                                   # data: the cube's visibilities (plus a stand-in noise)
    g = torch.Generator(device="cuda").manual_seed(5)
    y += 0.01 * torch.randn(dp.m, dtype=torch.complex64, device="cuda", generator=g) * y.abs().mean()
    xc = x * 1.01
    v = torch.zeros(dp.m, dtype=torch.complex64, device="cuda")
    grad = torch.zeros_like(x)
    eps = torch.full((L,), 0.5, dtype=torch.float64, device="cuda") * torch.tensor(
        [float(torch.linalg.vector_norm(y[dp.voff[l]:dp.voff[l + 1]])) for l in range(L)], dtype=torch.float64,
        device="cuda") * 0.01
    eta = torch.ones(L, dtype=torch.float64, device="cuda")
    res = torch.zeros(L, dtype=torch.float64, device="cuda")

    def one():
        dp.dual_update(xc, x, v, y, U, eps, eta, args.n_sub, grad, res)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        one()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.steps
    N = w.ny * w.nx
    # algorithmic bytes of one call: the images read (xcheck, x) and the
    # gradient read and written, the visibilities (y, U read; v read and
    # written), and for each of the three 2D FFTs of the 2x2-oversampled grid
    # one read and one write of it
    algo = 4 * N * L * 4 + dp.m * (8 + 4 + 16) + 3 * 2 * (8 * 4 * N * L)
    achieved = algo / (ms / 1e3) / 1e9
    line = {"metric": "data-fidelity dual update (Alg. 2 data-fidelity lines) visibilities/s", "value": dp.m / (ms / 1e3),
            "unit": "visibilities/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FFT), f64 (sums)",
            "data": "synthetic (seeded blob cube, Gaussian-radius uv-coverage scaled per channel)",
            "config": {"workload": f"data_{w.ny}x{w.nx}x{L}_m{M}", "ny": w.ny, "nx": w.nx, "channels": L,
                       "visibilities": int(dp.m), "grid": [int(dp.K1), int(dp.K2)], "kernel": "Kaiser-Bessel 7x7",
                       "sub_iterations": args.n_sub},
            "roofline": {"kernel": "whole call", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "bytes_per_call": algo}}
    log(f"[bench] data block: {ms:.3f} ms per call, {dp.m / (ms / 1e3) / 1e9:.2f} G visibilities/s")
    print(json.dumps(line), flush=True)


def pdfb_graph_bench(args):
    """N whole PDFB iterations (facet step, identity data term, primal update,
    extrapolation; Alg. 2 with the denoising stand-in) captured in one HIP graph,
    replayed from the same start; value = voxels per second per iteration.
    With --spectral-overlap the sub-cubes are contiguous channel blocks whose
    low-rankness facets overlap by that many channels."""
    import torch

    import paper_2003_07358_amd as fhs
    import synth
    name = args.workload if args.workload != DEFAULT_WORKLOAD else "cfg4_2048x2048x100_c10"
    w = synth.WORKLOADS[name]
    o = args.spectral_overlap
    n = args.pdfb_graph
    X = synth.workload_cube(w)
    plan = fhs.Plan(w.ny, w.nx, w.L, w.qy, w.qx, w.C, w.overlap, w.overlap, w.levels,
                    spectral_overlap=o).attach_workspace()
    s = plan.sizes
    mu, mub = plan.heuristics(synth.sigma_bar(X))
    seed = synth.BASE_SEED + w.seed_offset
    theta = synth.uniform_weights(s["n_theta"], seed + 11)
    tbar = np.concatenate([synth.sorted_weights(plan.Ln, seed + 100 + f) for f in range(s["n_facets"])])
    y, sig = synth.noisy_data(X, 0.05, seed + 4077)
    npix = w.ny * w.nx
    eps = np.full(w.L, sig * np.sqrt(npix + 2.0 * np.sqrt(npix)))   # eps^2 = sigma^2 (N + 2 sqrt(N)), Sec. 2.2
    x0 = np.maximum(y, 0.0).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    const = dict(y=dev(y), eps=dev(eps), theta=dev(theta), theta_bar=dev(tbar), mu=dev(mu), mu_bar=dev(mub))
    del X, y
    t = dict(x=dev(x0), xcheck=dev(x0), p=torch.zeros(s["n_p"], dtype=torch.float32, device="cuda"),
             w=torch.zeros(s["n_w"], dtype=torch.float32, device="cuda"),
             v=torch.zeros(s["n_x"], dtype=torch.float32, device="cuda"),
             grad=torch.empty(s["n_x"], dtype=torch.float32, device="cuda"),
             xi=torch.zeros(n * w.C, dtype=torch.float64, device="cuda"))
    init = {k: v.clone() for k, v in t.items()}
    state = plan.pdfb_state(**t, **const)
    log(f"[bench] {name}: {n} PDFB iterations in one graph (spectral overlap {o})")
    graph = plan.pdfb_graph(state, n)
    times = []
    for rep in range(1 + max(1, args.steps // 10)):
        for k in t:
            t[k].copy_(init[k])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.launch()
        e1.record()
        torch.cuda.synchronize()
        if rep:
            times.append(e0.elapsed_time(e1) / n)
    graph.close()
    ms = float(np.median(times))
    xi = t["xi"].view(n, w.C).cpu().numpy()
    vox = w.ny * w.nx * w.L
    sb = step_bytes(plan) + 44 * vox           # the facet step plus the closure passes (32 + 12 B/voxel)
    achieved = sb / (ms / 1e3) / 1e9
    line = {"metric": "PDFB iterations (identity data term) in one HIP graph: voxels/s per iteration",
            "value": vox / (ms / 1e3), "unit": "voxels/s", "n_gpus": 1, "steps": n, "warmup": 1,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 (filters, Gram and reconstruction accumulated in f64)",
            "data": "synthetic (seeded Gaussian-blob cube with power-law spectra, 5 % noise)",
            "config": {"workload": name, "ny": w.ny, "nx": w.nx, "channels": w.L, "facets": [w.qy, w.qx],
                       "subcubes": w.C, "spectral": "contiguous blocks, overlap %d channels" % o if o else
                       "interleaved sub-cubes", "graph_iterations": n, "weights": "random",
                       "parallelism": "single GPU"},
            "roofline": {"kernel": "whole iteration", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "bytes_per_iteration": sb},
            "xi_first_last": [float(xi[0].max()), float(xi[-1].max())]}
    log(f"[bench] {ms:.3f} ms per iteration in the graph; xi {xi[0].max():.3e} -> {xi[-1].max():.3e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
