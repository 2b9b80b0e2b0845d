"""GPU parity of the PDFB iteration (facet step + data-fidelity dual with the
identity operator + primal update + extrapolation) against the FP64 oracle,
and of its HIP-graph capture against eager launches.

Bars: one closure call matches the oracle to 1e-6 (float64 arithmetic,
float32 storage); after k iterations every state array is within k * 1e-5
relative L2 (each step within 1e-5, carried through a non-expansive
iteration) -- the data dual v relative to the norm of the step's input
v + xcheck - y, since (I - proj) is 1-Lipschitz but v can be tiny next to
its input; the relative variation within 2k * 1e-5 absolute.  A graph replay
equals the same iterations launched eagerly bit for bit.
"""
import numpy as np
import pytest

import synth
from fhs_cases import Problem, log, rel_l2
from oracle import closure

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CLOSURE_CASES = {
    "ragged_101x77x6": (101, 77, 6),
    "cfg1_256x256x20": (256, 256, 20),
    "l100_64x48x100": (64, 48, 100),
    "l1_33x17x1": (33, 17, 1),
    "l256_9x5x256": (9, 5, 256),
}


@pytest.mark.parametrize("name", list(CLOSURE_CASES))
def test_closure_parity(name):
    ny, nx, L = CLOSURE_CASES[name]
    log(f"[case] closure {name}")
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, (ny, nx, L)).astype(np.float32)
    xc = (x + 0.1 * rng.standard_normal(x.shape)).astype(np.float32)
    v = (0.05 * rng.standard_normal(x.shape)).astype(np.float32)
    y = rng.uniform(0, 1, (ny, nx, L)).astype(np.float32)
    g = (0.3 * rng.standard_normal(x.shape)).astype(np.float32)
    # radii: half the channels with v + xcheck inside the ball, half outside
    r = np.linalg.norm((v.astype(np.float64) + xc - y), axis=(0, 1))
    eps = np.where(np.arange(L) % 2 == 0, 0.5 * r, 2.0 * r)
    C = next(c for c in range(1, L + 1) if L % c == 0 and L // c <= 64)
    plan = fhs.Plan(ny, nx, L, n_sub=C, levels=1 if min(ny, nx) < 16 else 4).attach_workspace()
    xt, xct, vt = dev(x), dev(xc), dev(v)
    xi = torch.zeros(C, dtype=torch.float64, device="cuda")
    plan.pdfb_closure(xt, xct, vt, dev(y), dev(eps), dev(g), 0.33, xi)
    vr = closure.data_dual_update(v, xc, y, eps)
    xr, xcr, xir = closure.primal_update(x, g, vr, 0.33, C)
    for nm, got, ref in (("v", host(vt), vr), ("x", host(xt), xr), ("xcheck", host(xct), xcr)):
        e = rel_l2(got, ref)
        log(f"    {nm}: rel_l2={e:.3e}")
        assert e <= 1e-6, (nm, e)
    xig = host(xi)
    log(f"    xi (C={C}) gpu={xig[:4]} oracle={xir[:4]}")
    np.testing.assert_allclose(xig, xir, rtol=1e-12, atol=1e-15)


def pdfb_problem(ny, nx, L, qy, qx, C, o, levels=4, seed=0, blobs=12, frac=0.05):
    pb = Problem(ny, nx, L, qy, qx, C, o, o, levels, seed=seed, blobs=blobs)
    y, sig = synth.noisy_data(pb.X, frac, synth.BASE_SEED + 77 + seed)
    eps = np.full(L, closure.l2_ball_radius(sig, ny * nx))
    x0 = np.maximum(y, 0.0).astype(np.float32)
    return pb, y, eps, x0


def gpu_state(plan, pb, y, eps, x0, n_xi):
    t = dict(x=dev(x0), xcheck=dev(x0), p=dev(pb.P_flat()), w=dev(pb.W_flat()),
             v=torch.zeros(x0.size, dtype=torch.float32, device="cuda"), y=dev(y), eps=dev(eps),
             theta=dev(pb.theta_flat()), theta_bar=dev(pb.theta_bar_flat()), mu=dev(pb.mu),
             mu_bar=dev(pb.mu_bar_flat()), grad=torch.empty(x0.size, dtype=torch.float32, device="cuda"),
             xi=torch.zeros(n_xi * pb.C, dtype=torch.float64, device="cuda"))
    return t, plan.pdfb_state(**t)


PDFB_CASES = {
    "q2x2_c2_64x64x12": dict(ny=64, nx=64, L=12, qy=2, qx=2, C=2, o=8),
    "q3x2_c1_90x70x8": dict(ny=90, nx=70, L=8, qy=3, qx=2, C=1, o=6),
}


@pytest.mark.parametrize("name", list(PDFB_CASES))
def test_pdfb_iterations_parity(name):
    log(f"[case] pdfb {name}")
    pb, y, eps, x0 = pdfb_problem(**PDFB_CASES[name])
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    K = 5
    t, st = gpu_state(plan, pb, y, eps, x0, K)
    x, xc = x0.astype(np.float64), x0.astype(np.float64)
    P, W, v = pb.P, pb.W, np.zeros(x0.shape)
    for k in range(1, K + 1):
        plan.pdfb_iteration(st, k - 1)
        z_norm = np.linalg.norm(v + xc - y)   # input of the data-dual step
        x, xc, P, W, v, xi = closure.pdfb_iteration(x, xc, P, W, v, y, eps, pb.theta, pb.theta_bar, pb.mu,
                                                    pb.mu_bar, pb.geom, C=pb.C)
        got = {n: host(t[n]) for n in ("x", "xcheck", "v", "p", "w")}
        ref = {"x": x, "xcheck": xc, "v": v,
               "p": np.concatenate([q.reshape(-1) for row in P for q in row]),
               "w": np.concatenate(W, axis=1)}
        for n in got:
            if n == "v":
                # v = (I - proj)(z) is 1-Lipschitz in z but can be tiny next to
                # it (z just outside the ball): measure its error on z's scale
                e = np.linalg.norm(got[n].reshape(-1) - ref[n].reshape(-1)) / z_norm
            else:
                e = rel_l2(got[n].reshape(-1), ref[n].reshape(-1))
            log(f"    it {k} {n}: rel err={e:.3e}")
            assert e <= k * 1e-5, (k, n, e)
        xig = host(t["xi"])[(k - 1) * pb.C:k * pb.C]
        log(f"    it {k} xi gpu={xig} oracle={xi}")
        assert np.all(np.abs(xig - xi) <= 2 * k * 1e-5)


def test_pdfb_graph_replays_match_eager():
    log("[case] graph vs eager, q2x2_c2_64x64x12, 6 iterations, 3 replays")
    pb, y, eps, x0 = pdfb_problem(**PDFB_CASES["q2x2_c2_64x64x12"])
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    n = 6
    te, ste = gpu_state(plan, pb, y, eps, x0, n)
    for i in range(n):
        plan.pdfb_iteration(ste, i)
    eager = {k: host(v).copy() for k, v in te.items()}
    tg, stg = gpu_state(plan, pb, y, eps, x0, n)
    init = {k: v.clone() for k, v in tg.items()}
    graph = plan.pdfb_graph(stg, n)
    for rep in range(3):
        for k in tg:
            tg[k].copy_(init[k])
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        for k in ("x", "xcheck", "v", "p", "w", "grad", "xi"):
            assert np.array_equal(host(tg[k]), eager[k]), (rep, k)
        # unrelated eager work between replays
        (tg["grad"] * 2.0).sum().item()
        log(f"    replay {rep}: identical")
    graph.close()
    assert np.isfinite(eager["xi"]).all() and (eager["xi"] > 0).all()


SOLVE_CASES = {
    # (case, x0, T, rw_tol, p_min, p_max, pdfb_tol, res_factor, zero_sub, eps_scale): runs that stop on
    # the relative variation, on the residual, and at the caps; sub-cubes that
    # stop at different iterations and passes (a zero sub-cube runs to the cap
    # beside a noisy one; unequal ball radii per sub-cube); the deciding values
    # are far from the bounds (checked on the oracle side)
    "xi_stop": ("q2x2_c2_64x64x12", "zero", 2, 0.0, 2, 12, 0.1, 1.01, None, None),
    "res_stop": ("q3x2_c1_90x70x8", "zero", 2, 0.0, 2, 12, 1.0, 1.01, None, None),
    "caps": ("q3x2_c1_90x70x8", "data", 2, 0.0, 2, 3, 0.0, 1.01, None, None),
    "outer_stop": ("q2x2_c2_64x64x12", "data", 3, 1.0, 1, 2, 0.0, 1.01, None, None),
    "zero_subcube": ("q2x2_c2_64x64x12", "data", 2, 0.0, 2, 14, 2e-2, 1.01, 0, None),
    "radii_per_subcube": ("q2x2_c2_64x64x12", "data", 1, 0.0, 2, 16, 2e-2, 1.01, None, (3.0, 1e-3)),
    "outer_per_subcube": ("q2x2_c2_64x64x12", "data", 3, 10.0, 2, 3, 0.0, 1.01, 0, None),
}


@pytest.mark.parametrize("name", list(SOLVE_CASES))
def test_reweighting_solve_parity(name):
    """Alg. 1 on the GPU (fhs_reweighting_solve) against the oracle's loops,
    one per sub-cube: the same number of runs and iterations per run for
    every sub-cube, and the state after K iterations in all within K * 1e-5
    (as for K plain iterations), the weights of the last pass included."""
    from oracle import solve
    case, start, T, rw_tol, p_min, p_max, pdfb_tol, res_factor, zero_sub, eps_scale = SOLVE_CASES[name]
    log(f"[case] reweighting solve {name}: {case} from {start}")
    pb, y, eps, x0 = pdfb_problem(**PDFB_CASES[case])
    C = pb.C
    if zero_sub is not None:
        y = y.copy()
        y[..., zero_sub::C] = 0.0
        x0 = np.maximum(y, 0.0).astype(np.float32)
    if eps_scale is not None:
        eps = eps * np.array([eps_scale[l % C] for l in range(pb.L)])
    if start == "zero":
        x0 = np.zeros_like(x0)
    kw = dict(T=T, xi_rw=rw_tol, p_min=p_min, p_max=p_max, xi_tol=pdfb_tol, res_factor=res_factor)
    x, P, W, v, th, thb, rep = solve.reweighting_solve(x0, pb.P, pb.W, np.zeros(x0.shape), y, eps, pb.mu, pb.mu_bar,
                                                       pb.mu, pb.mu_bar, pb.geom, C=C, levels=pb.levels, **kw)
    iters = [[len(h) for h in rep["runs"][c]] for c in range(C)]
    # every stopping decision of the oracle is taken with a wide margin
    for c in range(C):
        bound = res_factor * np.linalg.norm(eps[c::C])
        for h in rep["runs"][c]:
            for xi, r in h:
                assert pdfb_tol == 0.0 or np.isinf(xi) or abs(xi / pdfb_tol - 1.0) > 0.05
                assert abs(r / bound - 1.0) > 0.01
        assert all(rw_tol == 0.0 or np.isinf(xi) or abs(xi / rw_tol - 1.0) > 0.05 for xi in rep["xi"][c])
    log(f"    oracle: iterations per run and sub-cube {iters}, outer xi {rep['xi']}")

    plan = fhs.Plan(*pb.cfg).attach_workspace()
    t, st = gpu_state(plan, pb, y, eps, x0, p_max)
    x_prev = torch.empty(x0.size, dtype=torch.float32, device="cuda")
    got = plan.reweighting_solve(st, dev(pb.mu), dev(pb.mu_bar_flat()), x_prev, max_reweights=T, rw_tol=rw_tol,
                                 min_iter=p_min, max_iter=p_max, pdfb_tol=pdfb_tol, res_factor=res_factor)
    log(f"    gpu:    iterations per run and sub-cube {got['iters']}, outer xi {got['rw_xi']}")
    assert got["iters"] == iters and got["runs"] == max(len(i) for i in iters)
    assert got["iterations"] == sum(sum(i) for i in iters)
    K = max(sum(i) for i in iters)
    ref = {"x": x, "p": np.concatenate([q.reshape(-1) for row in P for q in row]), "w": np.concatenate(W, axis=1),
           "theta": np.concatenate(th), "theta_bar": np.concatenate([q for row in thb for q in row])}
    for n, r in ref.items():
        e = rel_l2(host(t[n]).reshape(-1), r.reshape(-1))
        log(f"    {n}: rel err={e:.3e}")
        assert e <= K * 1e-5, (n, e)
    ev = np.linalg.norm(host(t["v"]).reshape(-1) - v.reshape(-1)) / np.linalg.norm(y)
    log(f"    v: err / ||y|| = {ev:.3e}")
    assert ev <= K * 1e-5
    if zero_sub is not None:
        # the zero sub-cube stays exactly zero throughout
        xg = host(t["x"]).reshape(x0.shape)
        assert not np.any(xg[..., zero_sub::C])
    for c in range(C):
        for a, b in zip(got["rw_xi"][c], rep["xi"][c]):
            assert (np.isinf(a) and np.isinf(b)) or abs(a - b) <= 1e-3 * b


def test_resume_from_checkpoint_is_bitwise(tmp_path):
    """Four iterations in a row equal two, a checkpoint of the state written to
    disk and read back into fresh device arrays, and two more (the state that
    Alg. 1 carries: X, Xcheck, P, W, v)."""
    from paper_2003_07358_amd import checkpoint
    log("[case] checkpoint / resume, q3x2_c1_90x70x8, 2 + 2 iterations")
    pb, y, eps, x0 = pdfb_problem(**PDFB_CASES["q3x2_c1_90x70x8"])
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    ta, sta = gpu_state(plan, pb, y, eps, x0, 4)
    for i in range(4):
        plan.pdfb_iteration(sta, i)
    tb, stb = gpu_state(plan, pb, y, eps, x0, 4)
    for i in range(2):
        plan.pdfb_iteration(stb, i)
    keys = ("x", "xcheck", "p", "w", "v")
    checkpoint.save(tmp_path / "s.npz", plan, **{k: tb[k] for k in keys})
    tc, stc = gpu_state(plan, pb, y, eps, x0, 4)
    for k, v in checkpoint.load(tmp_path / "s.npz", plan).items():
        tc[k].copy_(v)
    for i in range(2, 4):
        plan.pdfb_iteration(stc, i)
    for k in keys + ("grad",):
        assert np.array_equal(host(ta[k]), host(tc[k])), k
    assert np.array_equal(host(ta["xi"])[2:], host(tc["xi"])[2:])


@pytest.mark.parametrize("L,with_log", [(20, True), (5, True), (64, False)])
def test_snr_matches_oracle(L, with_log):
    """Reconstruction SNR and log-scale SNR per channel (Sec. 4.3) against the
    oracle: the same float32 images, sums in float64 on both sides."""
    from oracle import metrics
    ny, nx = 37, 53
    plan = fhs.Plan(ny, nx, L, 1, 1, 1, 0, 0, 2).attach_workspace()
    rng = np.random.default_rng(11 + L)
    ref = rng.uniform(0.0, 3.0, (ny, nx, L)).astype(np.float32)
    est = (ref * np.exp(0.1 * rng.standard_normal(ref.shape))).astype(np.float32)
    est[0, 0, :] = ref[0, 0, :]
    eps = rng.uniform(0.01, 0.5, L)
    d_eps = torch.from_numpy(eps).cuda() if with_log else None
    snr, snr_log = plan.snr(torch.from_numpy(ref).cuda(), torch.from_numpy(est).cuda(), d_eps)
    np.testing.assert_allclose(snr.cpu().numpy(), metrics.snr(ref, est), rtol=1e-10)
    if with_log:
        np.testing.assert_allclose(snr_log.cpu().numpy(), metrics.snr_log(ref, est, eps), rtol=1e-10)
    # exact estimate -> +inf
    same, _ = plan.snr(torch.from_numpy(ref).cuda(), torch.from_numpy(ref).cuda())
    assert np.all(np.isinf(same.cpu().numpy()))
