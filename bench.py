#!/usr/bin/env python3
"""Throughput of the facet-wise regularization step (facet_prox_step) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = fhs_facet_prox_step over the whole cube: the weighted nuclear-norm
dual update of every facet, the weighted l21 dual update of every coefficient
row and the gather of both into the primal gradient (Alg. 2, facet loop and
facet part of the aggregation).  Inputs are seeded synthetic cubes (see
synth/), resident in HBM before timing.  Prints ONE JSON line:
value = voxels / s (N * L per step), with a roofline entry for one kernel
(timed live with HIP events on the launch stream) and the FP64 CPU oracle
timed on a bounded sample as the CPU baseline.
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
DEFAULT_WORKLOAD = "cfg2_1024x2048x20"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(plan, w, kernel, fused=True):
    """Algorithmic HBM bytes of all launches of `kernel` in one step: every
    input the kernel must read and every output it must write, once.  fused:
    the Dirac band's dual update runs in the first level-1 synthesis group
    (the batched step), else in the level-1 analysis (the per-facet form)."""
    bands = plan.bands()
    N, L, C, lev = w.ny * w.nx, w.L, w.C, w.levels
    per_basis = 3 * lev + 1

    def band_rows(b, j):          # rows of one detail band of basis b, level j (1-based)
        return bands[b * per_basis + 3 * (j - 1)][0] * bands[b * per_basis + 3 * (j - 1)][1]

    if kernel == "analysis_l1":
        tot = N * L * 4                                   # cube
        for b in range(8):
            r = band_rows(b, 1)
            tot += 3 * r * (2 * L * 4 + C * 4)            # details: W read + write, theta
            tot += r * L * 4 * (2 if lev == 1 else 1)     # low-low: W rw (1 level) or written once
        if not fused:
            tot += N * (2 * L * 4 + C * 4)                # Dirac: W rw, theta
        return tot, 1
    if kernel in ("synth_final_a", "synth_final_b"):
        bs = range(0, 4) if kernel == "synth_final_a" else range(4, 8)
        tot = sum(4 * band_rows(b, 1) * L * 4 for b in bs)
        if kernel == "synth_final_a":
            tot += N * L * 4 * 2                          # Dirac W read + G write
            if fused:
                tot += N * (2 * L * 4 + C * 4)            # Xcheck, Dirac W write, theta
        else:
            tot += N * L * 4 * 2                          # G read + write
        return tot, 1
    raise ValueError(kernel)


def step_bytes(plan, w):
    """Algorithmic bytes of one whole step: Xcheck once, P and W read + written,
    theta, G written (float32)."""
    s = plan.sizes
    return 4 * (s["n_x"] + 2 * s["n_p"] + 2 * s["n_w"] + s["n_theta"] + s["n_x"])


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    from paper_2003_07358_amd.profiling import source_hash
    files = d.get("sources")
    if d.get("source_hash") != source_hash(None if files in (None, "all") else files):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, budget_s):
    """FP64 oracle on a bounded sample of the workload: the facet step restricted
    to the top-left block of facets (same facet sizes and overlap), grown until
    it takes about `budget_s` seconds; value in voxels per second."""
    from threadpoolctl import threadpool_info

    import synth
    from oracle import geometry, heuristics, sara, step
    X = synth.workload_cube(w)
    best = None
    for k in range(1, max(w.qy, w.qx) + 1):
        qy, qx = min(k, w.qy), min(k, w.qx)
        ny, nx = (w.ny * qy) // w.qy, (w.nx * qx) // w.qx
        geom = geometry.Geometry(ny, nx, qy, qx, w.overlap, w.overlap, w.levels)
        Xs = np.ascontiguousarray(X[:ny, :nx])
        I = sara.n_coefficients(ny, nx, w.levels)
        Lc = w.L // w.C
        sb = synth.sigma_bar(X)
        mu = [heuristics.mu_sparsity(sb, Lc)] * w.C
        mub = [[heuristics.mu_low_rank(sb, f.n_rows, Lc) for f in geom.facets] for _ in range(w.C)]
        P = [[np.zeros(f.nuc_shape + (Lc,), np.float32) for f in geom.facets] for _ in range(w.C)]
        W = [np.zeros((I, Lc), np.float32) for _ in range(w.C)]
        th = [synth.uniform_weights(I, 1 + c) for c in range(w.C)]
        tb = [[synth.sorted_weights(Lc, 7 + q) for q in range(geom.Q)] for _ in range(w.C)]
        t0 = time.perf_counter()
        step.facet_prox_step(Xs, P, W, th, tb, mu, mub, 1.0, 1.0, geom, C=w.C)
        dt = time.perf_counter() - t0
        best = (ny, nx, qy, qx, dt)
        if dt > budget_s / 3 or (qy == w.qy and qx == w.qx):
            break
    ny, nx, qy, qx, dt = best
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": ny * nx * w.L / dt, "unit": "voxels/s", "cores": int(threads), "kind": "oracle",
            "sample": f"top-left {qy}x{qx} facets ({ny}x{nx}x{w.L}) of the workload, one step, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--kernel", default="analysis_l1", help="kernel reported in the roofline entry")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default launch shapes")
    ap.add_argument("--form", choices=("batched", "plain"), default="batched",
                    help="batched: every operator one launch over all facets (default); plain: the "
                         "per-facet execution form, one launch per facet and operator")
    ap.add_argument("--tuning", default=None, metavar="JSON",
                    help="fixed launch shapes (a JSON object as printed in the 'tuning' field) instead of autotuning")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (the reference "
                         "dispatch that scales HBM counters read under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of the "
              "facet step is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2003_07358_amd as fhs
    import synth
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = synth.WORKLOADS[args.workload]
    log(f"[bench] workload {w.name}: generating inputs")
    X = synth.workload_cube(w)
    plan = fhs.Plan(w.ny, w.nx, w.L, w.qy, w.qx, w.C, w.overlap, w.overlap, w.levels).attach_workspace()
    s = plan.sizes
    mu, mub = plan.heuristics(synth.sigma_bar(X))
    seed = synth.BASE_SEED + w.seed_offset
    theta = synth.uniform_weights(s["n_theta"], seed + 11)
    tbar = np.concatenate([synth.sorted_weights(plan.Lc, seed + 100 + f) for f in range(s["n_facets"])])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x_d, th_d, tb_d, mu_d, mub_d = dev(X), dev(theta), dev(tbar), dev(mu), dev(mub)
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
        tuning = plan.autotune(x_d, p_d, w_d, th_d, tb_d, mu_d, mub_d, g_d, reps=5)
        p_d.zero_()
        w_d.zero_()
        torch.cuda.synchronize()
        log(f"[bench] autotune {time.perf_counter() - t0a:.1f} s: {tuning}")
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    plan.profile(args.kernel, max_launches=max(16, 4 * args.steps))
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
    voxels = w.voxels
    value = voxels / (ms / 1e3)
    kb, per_step = kernel_bytes(plan, w, args.kernel, fused=args.form == "batched")
    avg_launch_s = (kms / launches) / 1e3 if launches else float("nan")
    achieved = kb / per_step / avg_launch_s / 1e9
    traffic = traffic_from_profiles(args.kernel, w.name)
    sb = step_bytes(plan, w)
    log(f"[bench] {ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f}); {args.kernel}: "
        f"{kms / max(launches, 1):.3f} ms/launch, {achieved:.0f} GB/s; step bytes {sb / 1e9:.2f} GB "
        f"-> {sb / (ms / 1e3) / 1e9:.0f} GB/s")
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
        "dtype": "f32 (nuclear path f64-accumulated)",
        "data": "synthetic (seeded Gaussian-blob cube with power-law spectra)",
        "config": {"workload": w.name, "form": args.form, "ny": w.ny, "nx": w.nx, "channels": w.L,
                   "facets": [w.qy, w.qx],
                   "overlap_px": w.overlap, "subcubes": w.C, "levels": w.levels, "bases": "db1-db8+dirac",
                   "parallelism": "single GPU"},
        "roofline": {"kernel": args.kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": kb / per_step, "avg_launch_ms": kms / max(launches, 1)},
        "tuning": plan.tuning,
        "step_hbm": {"algorithmic_bytes": sb, "achieved_GBs": sb / (ms / 1e3) / 1e9,
                     "frac": sb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
