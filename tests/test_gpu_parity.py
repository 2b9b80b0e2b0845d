"""GPU parity of every C-ABI compute call against the FP64 oracle.

Same seeded inputs on both sides (the oracle reads the float32 arrays promoted
to float64).  Bar: relative L2 error <= 1e-5 per output array (FP32 path; the
nuclear update accumulates in FP64), and an element-wise bound of 1e-4 of the
array's largest magnitude; integer-like invariants (zero in, zero out;
determinism) are exact.  Cases span several workgroup tiles, ragged sizes,
odd channel counts (Jacobi padding), interleaved sub-cubes, one facet,
zero overlap, 64 channels per sub-cube, shallow decompositions and warm /
signed inputs.
"""
import numpy as np
import pytest

from fhs_cases import Problem, log, max_rel, rel_l2
from oracle import sara, step

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = pytest.mark.gpu
TOL = 1e-5
ELEM = 1e-4

CASES = {
    "cfg1_256x256x20_q2x2_o32": dict(ny=256, nx=256, L=20, qy=2, qx=2, oy=32, ox=32),
    "ragged_101x77x6_q3x2_c2": dict(ny=101, nx=77, L=6, qy=3, qx=2, C=2, oy=7, ox=5, blobs=12),
    "lc64_70x45x64_q2x1": dict(ny=70, nx=45, L=64, qy=2, qx=1, oy=9, ox=0, blobs=8),
    "lc5_odd_48x40x5_q1x1": dict(ny=48, nx=40, L=5, blobs=6),
    "tiny_7x9x3_levels2": dict(ny=7, nx=9, L=3, levels=2, blobs=2),
    "c4_64x64x12_q4x4_o0": dict(ny=64, nx=64, L=12, qy=4, qx=4, C=4, blobs=10),
    # dense lane segments (L_c = 12 or 20): one sub-cube; two sub-cubes; seven
    # sub-cubes, whose segments do not fill the waves evenly
    "lc12_72x60x12_q2x2": dict(ny=72, nx=60, L=12, qy=2, qx=2, oy=8, ox=8, blobs=8),
    "c2_lc20_60x52x40_q2x1": dict(ny=60, nx=52, L=40, qy=2, qx=1, C=2, oy=6, ox=0, blobs=8),
    "c7_lc12_40x36x84": dict(ny=40, nx=36, L=84, C=7, blobs=6),
    # dense segments of even, non-multiple-of-4 widths (pair sums)
    "lc6_50x44x6_q2x2": dict(ny=50, nx=44, L=6, qy=2, qx=2, oy=6, ox=6, blobs=8),
    "c10_lc10_40x36x100_q2x2": dict(ny=40, nx=36, L=100, qy=2, qx=2, C=10, oy=4, ox=4, blobs=6),
    "c4_lc18_36x30x72_q2x1": dict(ny=36, nx=30, L=72, qy=2, qx=1, C=4, oy=4, ox=0, blobs=6),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(name, **kw):
    args = dict(CASES[name])
    args.update(kw)
    log(f"[case] {name} {kw}")
    pb = Problem(**args)
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    return pb, plan


def check(name, got, ref, tol=TOL):
    e, m = rel_l2(got, ref), max_rel(got, ref)
    log(f"    {name}: rel_l2={e:.3e} max_rel={m:.3e}")
    assert e <= tol, (name, e)
    assert m <= ELEM, (name, m)


@pytest.mark.parametrize("name", list(CASES))
def test_sara_analysis(name):
    pb, plan = make(name)
    w = torch.empty(plan.sizes["n_w"], dtype=torch.float32, device="cuda")
    plan.sara_analysis(dev(pb.X), w)
    check("Psi^dagger x", host(w).reshape(pb.I, pb.L), pb.oracle_analysis())


@pytest.mark.parametrize("name", list(CASES))
def test_sara_synthesis(name):
    pb, plan = make(name)
    rng = np.random.default_rng(7)
    wv = rng.standard_normal((pb.I, pb.L)).astype(np.float32)
    x0 = rng.standard_normal((pb.ny, pb.nx, pb.L)).astype(np.float32)
    xt = dev(x0)
    plan.sara_synthesis(dev(wv), xt, alpha=1.5, beta=0.5)
    ref = 0.5 * x0.astype(np.float64)
    for c, ch in enumerate(step.subcube_channels(pb.L, pb.C)):
        part = wv[:, c * pb.Lc:(c + 1) * pb.Lc].astype(np.float64)
        ref[..., ch] += 1.5 * sara.synthesis(sara.unflatten(part, pb.ny, pb.nx, pb.levels), pb.ny, pb.nx,
                                             pb.levels)
    check("beta x + alpha Psi w", host(xt), ref)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("warm", [False, True])
def test_l21_dual_update(name, warm):
    pb, plan = make(name, warm=warm)
    kappa = 1.0 if not warm else 0.8
    w = dev(pb.W_flat())
    g0 = np.random.default_rng(3).standard_normal((pb.ny, pb.nx, pb.L)).astype(np.float32)
    g = dev(g0)
    beta = 0.25 if warm else 0.0
    plan.l21_dual_update(dev(pb.X), w, dev(pb.theta_flat()), dev(pb.mu), kappa, g, beta)
    Wn, G = pb.oracle_l21(kappa)
    check("W+", host(w), np.concatenate(Wn, axis=1).reshape(-1))
    check("beta g + kappa Psi W+", host(g), beta * g0.astype(np.float64) + G)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("warm", [False, True])
def test_nuclear_dual_update(name, warm):
    pb, plan = make(name, warm=warm)
    zeta = 1.0 if not warm else 1.3
    p = dev(pb.P_flat())
    g0 = np.random.default_rng(4).standard_normal((pb.ny, pb.nx, pb.L)).astype(np.float32)
    g = dev(g0)
    beta = 0.5 if warm else 0.0
    plan.nuclear_dual_update(dev(pb.X), p, dev(pb.theta_bar_flat()), dev(pb.mu_bar_flat()), zeta, g, beta)
    Pn, G = pb.oracle_nuclear(zeta)
    ref = np.concatenate([q.reshape(-1) for row in Pn for q in row])
    check("P+", host(p), ref)
    check("beta g + zeta sum S~^T D P+", host(g), beta * g0.astype(np.float64) + G)


def test_nuclear_conditioning_sweep():
    """Error of the nuclear dual update against the oracle as the thresholds
    shrink and kappa = sigma_1 / min t grows to ~5e6 (the Gram route squares
    kappa; FP64 accumulation of the Gram and the reconstruction keeps every
    point within the 1e-5 bar)."""
    from oracle import step as ostep
    pb, plan = make("cfg1_256x256x20_q2x2_o32", warm=True)
    sig1 = max(np.linalg.svd(ostep.facet_matrix(pb.X, f, np.arange(pb.L)), compute_uv=False)[0]
               for f in pb.geom.facets)
    for scale in (1.0, 1e-1, 1e-2, 1e-3, 1e-4):
        mub = np.asarray(pb.mu_bar) * scale
        tmin = min(float(np.min(mub[0][q] * pb.theta_bar[0][q])) for q in range(pb.geom.Q))
        p = dev(pb.P_flat())
        g = torch.zeros(plan.sizes["n_x"], device="cuda")
        plan.nuclear_dual_update(dev(pb.X), p, dev(pb.theta_bar_flat()), dev(mub.reshape(-1)), 1.0, g, 0.0)
        Pn, G = ostep.nuclear_dual_update(pb.X, pb.P, pb.theta_bar, mub, 1.0, pb.geom, C=pb.C)
        ref = np.concatenate([q.reshape(-1) for row in Pn for q in row])
        kappa = sig1 / tmin
        e, eg = rel_l2(host(p), ref), rel_l2(host(g), G.reshape(-1))
        log(f"    threshold scale {scale:g}: kappa = {kappa:.3e}, P+ rel_l2 = {e:.3e}, G rel_l2 = {eg:.3e}")
        assert e <= TOL and eg <= TOL, (scale, kappa, e, eg)


def _nuclear_case(pb, plan, mub, zeta=1.0):
    p = dev(pb.P_flat())
    g = torch.zeros(plan.sizes["n_x"], device="cuda")
    plan.nuclear_dual_update(dev(pb.X), p, dev(pb.theta_bar_flat()), dev(np.asarray(mub).reshape(-1)), zeta, g, 0.0)
    Pn, G = step.nuclear_dual_update(pb.X, pb.P, pb.theta_bar, mub, zeta, pb.geom, C=pb.C)
    return host(p), np.concatenate([q.reshape(-1) for row in Pn for q in row]), host(g), G.reshape(-1)


def test_nuclear_threshold_zero_and_infinite():
    """t = 0 (mu_bar = 0): P+ = 0 exactly, so the gather adds nothing; t -> inf:
    nothing is thresholded, P+ = Z = P + D Xcheck (Table 1 SVT limits)."""
    pb, plan = make("ragged_101x77x6_q3x2_c2", warm=True)
    got, ref, g, G = _nuclear_case(pb, plan, np.zeros_like(np.asarray(pb.mu_bar)))
    assert not np.any(got) and not np.any(g) and not np.any(ref)
    got, ref, g, G = _nuclear_case(pb, plan, np.full_like(np.asarray(pb.mu_bar), 1e30))
    check("P+ (t = inf)", got, ref)
    check("G (t = inf)", g, G)


def test_nuclear_fewer_pixels_than_channels():
    """Facets of 12 to 20 pixels and 64 channels: J = min(N~_q, L_c) < L_c, the
    Gram is rank deficient and the components beyond the rank are zero."""
    pb = Problem(9, 8, 64, 2, 2, 1, 1, 1, 2, seed=3, blobs=4, warm=True)
    assert all(f.n_rows < 64 for f in pb.geom.facets)
    log(f"[case] 9x8x64, 2x2 facets: facet pixels {[f.n_rows for f in pb.geom.facets]}")
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    got, ref, g, G = _nuclear_case(pb, plan, pb.mu_bar)
    check("P+ (N~ < L_c)", got, ref)
    check("G (N~ < L_c)", g, G)


def test_nuclear_equal_weights_repeated_singular_values():
    """Z with repeated singular values (3, 3, 3, 1, 0.5, ...) and equal weights:
    the result, the projection of Z onto the spectral-norm ball of radius t,
    is unique whatever basis the eigensolver picks in the repeated
    eigenspace (Table 1 SVT; ties with equal weights)."""
    pb = Problem(24, 20, 8, 1, 1, 1, 0, 0, 2, zero=True)
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    rng = np.random.default_rng(21)
    f = pb.geom.facets[0]
    U, _ = np.linalg.qr(rng.standard_normal((f.n_rows, 8)))
    V, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    s = np.array([3.0, 3.0, 3.0, 1.0, 0.5, 0.25, 0.1, 0.05])
    pb.P = [[((U * s) @ V.T).reshape(f.nuc_shape + (8,)).astype(np.float32)]]
    pb.theta_bar = [[np.ones(8)]]
    log("[case] repeated singular values 3, 3, 3 with equal weights, t = 2")
    got, ref, g, G = _nuclear_case(pb, plan, np.array([[2.0]]))
    check("P+ (ties, equal weights)", got, ref)
    check("G (ties, equal weights)", g, G)


def test_sara_reduction_one_channel_per_subcube():
    """C = L (L_c = 1) with mu_bar = 0: the nuclear term vanishes and the step
    is channel by channel (the SARA reduction of the prior, Sec. 2.4); the
    l21 row norm is |u| and W+ = clip(u, -a, a)."""
    pb, plan = make("lc5_odd_48x40x5_q1x1", C=5, warm=True)
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.empty(plan.sizes["n_x"], dtype=torch.float32, device="cuda")
    mub = np.zeros_like(np.asarray(pb.mu_bar))
    plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                         dev(mub.reshape(-1)), 1.0, 1.0, g)
    Pn, Wn, G = step.facet_prox_step(pb.X, pb.P, pb.W, pb.theta, pb.theta_bar, pb.mu, mub, 1.0, 1.0, pb.geom, C=pb.C)
    assert not np.any(host(p))
    check("W+ (L_c = 1)", host(w), np.concatenate(Wn, axis=1).reshape(-1))
    check("G (L_c = 1)", host(g), G.reshape(-1))


@pytest.mark.parametrize("variant", ["plain", "signed"])
@pytest.mark.parametrize("warm", [False, True])
def test_facet_prox_step_cfg1(variant, warm):
    pb, plan = make("cfg1_256x256x20_q2x2_o32", variant=variant, warm=warm)
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.full((plan.sizes["n_x"],), float("nan"), device="cuda")   # overwritten, never read
    plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                         dev(pb.mu_bar_flat()), 1.0, 1.0, g)
    Pn, Wn, G = pb.oracle_step()
    check("P+", host(p), np.concatenate([q.reshape(-1) for row in Pn for q in row]))
    check("W+", host(w), np.concatenate(Wn, axis=1).reshape(-1))
    check("G", host(g), G.reshape(-1))


def test_reweight():
    pb, plan = make("ragged_101x77x6_q3x2_c2")
    from oracle import heuristics
    ups = np.array([0.05, 0.02])
    upb = np.linspace(0.5, 1.5, pb.C * pb.geom.Q)
    th = torch.empty(plan.sizes["n_theta"], dtype=torch.float32, device="cuda")
    tb = torch.empty(plan.sizes["n_theta_bar"], dtype=torch.float64, device="cuda")
    plan.reweight(dev(pb.X), dev(ups), dev(upb), th, tb)
    ref_t = np.concatenate(heuristics.l21_weights(pb.X, ups, pb.levels, pb.C))
    ref_b = heuristics.nuclear_weights(pb.X, pb.geom, upb.reshape(pb.C, -1), pb.C)
    check("theta", host(th), ref_t)
    check("theta_bar", host(tb), np.concatenate([t for row in ref_b for t in row]), tol=1e-8)


def test_zero_input_gives_zero():
    pb, plan = make("cfg1_256x256x20_q2x2_o32", zero=True)
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.full((plan.sizes["n_x"],), 7.0, device="cuda")
    plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                         dev(pb.mu_bar_flat()), 1.0, 1.0, g)
    assert np.all(host(p) == 0) and np.all(host(w) == 0) and np.all(host(g) == 0)


def test_bitwise_deterministic():
    pb, plan = make("ragged_101x77x6_q3x2_c2", warm=True)
    outs = []
    for _ in range(2):
        p, w = dev(pb.P_flat()), dev(pb.W_flat())
        g = torch.empty(plan.sizes["n_x"], device="cuda")
        plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                             dev(pb.mu_bar_flat()), 1.0, 1.0, g)
        outs.append((host(p), host(w), host(g)))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["cfg1_256x256x20_q2x2_o32", "ragged_101x77x6_q3x2_c2"])
def test_stream_schedules_agree(name):
    """One stream, or the nuclear chain on the side stream beside the wavelet
    chain: the same kernels on the same data, so the same bits."""
    pb, plan = make(name, warm=True)
    outs = []
    for conc in (0, 1):
        plan.tuning = {"concurrent": conc}
        p, w = dev(pb.P_flat()), dev(pb.W_flat())
        g = torch.empty(plan.sizes["n_x"], device="cuda")
        plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                             dev(pb.mu_bar_flat()), 1.0, 1.0, g)
        outs.append((host(p), host(w), host(g)))
    for o in outs[1:]:
        for nm, a, b in zip(("P+", "W+", "G"), o, outs[0]):
            assert np.array_equal(a, b), nm
    Pn, Wn, G = pb.oracle_step()
    check("G (side stream)", outs[1][2], G.reshape(-1))


@pytest.mark.slow
def test_facet_prox_step_cfg2_full():
    """1024 x 2048 x 20, 4 x 4 facets, 64-px overlap: the full FP64 oracle."""
    log("[case] cfg2_1024x2048x20_q4x4_o64 full oracle")
    pb = Problem(1024, 2048, 20, 4, 4, 1, 64, 64, 4, seed=2, blobs=50)
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.empty(plan.sizes["n_x"], device="cuda")
    plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                         dev(pb.mu_bar_flat()), 1.0, 1.0, g)
    gp, gw, gg = host(p), host(w), host(g)
    log("    gpu done; running oracle")
    Pn, Wn, G = pb.oracle_step()
    check("P+", gp, np.concatenate([q.reshape(-1) for row in Pn for q in row]))
    check("W+", gw, np.concatenate(Wn, axis=1).reshape(-1))
    check("G", gg, G.reshape(-1))


def test_autotune_keeps_results():
    """Launch shapes chosen by the autotuner change speed only: the tuned step
    matches the oracle and the default-shape step."""
    pb, plan = make("cfg1_256x256x20_q2x2_o32", warm=True)
    args = [dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu), dev(pb.mu_bar_flat())]
    x = dev(pb.X)

    def step():
        p, w = dev(pb.P_flat()), dev(pb.W_flat())
        g = torch.empty(plan.sizes["n_x"], device="cuda")
        plan.facet_prox_step(x, p, w, args[0], args[1], args[2], args[3], 1.0, 1.0, g)
        return host(p), host(w), host(g)

    ref = step()
    t0 = plan.tuning
    scratch = [dev(pb.P_flat()), dev(pb.W_flat()), torch.empty(plan.sizes["n_x"], device="cuda")]
    t1 = plan.autotune(x, scratch[0], scratch[1], *args, scratch[2], reps=1)
    log(f"    default {t0}\n    tuned   {t1}")
    got = step()
    for name, a, b in zip(("P+", "W+", "G"), got, ref):
        check(name + " (tuned vs default)", a, b, tol=1e-6)
    Pn, Wn, G = pb.oracle_step()
    check("P+", got[0], np.concatenate([q.reshape(-1) for row in Pn for q in row]))
    check("W+", got[1], np.concatenate(Wn, axis=1).reshape(-1))
    check("G", got[2], G.reshape(-1))


def test_autotune_cache(tmp_path):
    """A cache miss tunes and stores the shapes under the plan's key; a hit on
    a fresh plan of the same configuration sets them without timing."""
    import json
    pb, plan = make("ragged_101x77x6_q3x2_c2")
    cache = str(tmp_path / "tuning.json")
    args = [dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu), dev(pb.mu_bar_flat())]
    x = dev(pb.X)
    scratch = [dev(pb.P_flat()), dev(pb.W_flat()), torch.empty(plan.sizes["n_x"], device="cuda")]
    t1 = plan.autotune(x, scratch[0], scratch[1], *args, scratch[2], reps=1, cache=cache)
    entries = json.load(open(cache))
    assert entries == {plan.tuning_key(): t1}
    fresh = fhs.Plan(*pb.cfg).attach_workspace()
    fresh.tuning = {"nuc_seg": 16, "ana_phase": 1}          # differs from what is stored
    poison = [torch.full_like(a, float("nan")) for a in scratch]
    t2 = fresh.autotune(x, poison[0], poison[1], *args, poison[2], reps=1, cache=cache)
    assert t2 == t1
    assert all(torch.isnan(a).all() for a in poison)     # a hit runs nothing on the scratch arrays
    other = fhs.Plan(*pb.cfg, precision=1).attach_workspace()
    assert other.tuning_key() != plan.tuning_key()


@pytest.mark.parametrize("name", ["cfg1_256x256x20_q2x2_o32", "ragged_101x77x6_q3x2_c2", "c4_64x64x12_q4x4_o0"])
def test_per_facet_form_matches_batched(name):
    """The per-facet execution form computes the same step as the batched one
    (same kernels on each facet's own coefficients, pixels and window rows)."""
    pb, plan = make(name, warm=True)
    args = [dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu), dev(pb.mu_bar_flat())]
    x = dev(pb.X)
    out = []
    for plain in (False, True):
        p, w = dev(pb.P_flat()), dev(pb.W_flat())
        g = torch.empty(plan.sizes["n_x"], device="cuda")
        plan.facet_prox_step(x, p, w, *args, 1.0, 1.0, g, plain=plain)
        out.append((host(p), host(w), host(g)))
    for nm, a, b in zip(("P+", "W+", "G"), out[1], out[0]):
        log(f"    {nm}: max |plain - batched| = {np.max(np.abs(a - b)):.3e}")
        assert np.array_equal(a, b), nm


@pytest.mark.parametrize("name", ["cfg1_256x256x20_q2x2_o32", "ragged_101x77x6_q3x2_c2", "lc64_70x45x64_q2x1",
                                  "tiny_7x9x3_levels2"])
def test_direct_analysis_matches_staged(name):
    """The LDS-free analysis (taps, W and theta loaded into registers) gives the
    same coefficients, bit for bit, as the LDS-staged one, for every mode; so
    does either launch order (basis-major or tile-major)."""
    pb, plan = make(name, warm=True)
    x = dev(pb.X)
    outs = []
    # staged, direct at every level, mixed; tile-major order at every level and mixed
    for direct, order in ((0, 0), (63, 0), (0b0101, 0), (0, 63), (0b0110, 0b0011)):
        plan.tuning = {"ana_direct": direct, "ana_order": order}
        w0 = torch.empty(plan.sizes["n_w"], dtype=torch.float32, device="cuda")
        plan.sara_analysis(x, w0)
        w1, g1 = dev(pb.W_flat()), torch.empty(plan.sizes["n_x"], device="cuda")
        plan.l21_dual_update(x, w1, dev(pb.theta_flat()), dev(pb.mu), 1.0, g1)
        th = torch.empty(plan.sizes["n_theta"], dtype=torch.float32, device="cuda")
        tb = torch.empty(plan.sizes["n_theta_bar"], dtype=torch.float64, device="cuda")
        plan.reweight(x, dev(pb.mu), dev(pb.mu_bar_flat()), th, tb)
        outs.append([host(w0), host(w1), host(g1), host(th)])
    for o in outs[1:]:
        for nm, a, b in zip(("Psi^dagger x", "W+", "G", "theta"), o, outs[0]):
            log(f"    {nm}: max |direct - staged| = {np.max(np.abs(a - b)):.3e}")
            assert np.array_equal(a, b), nm
    check("W+ (direct)", outs[1][1], np.concatenate(pb.oracle_l21()[0], axis=1).reshape(-1))


def test_diagnostics_count_non_finite_facets():
    """A NaN in one facet's window makes that facet's Gram non-finite: the
    diagnostic counter names exactly the facets whose windows hold it (the
    pixel lies in the bottom-right tile only, inside no other window); clean
    inputs count nothing, and the eigensolver converges on every facet."""
    pb, plan = make("cfg1_256x256x20_q2x2_o32", warm=True)
    args = (dev(pb.theta_bar_flat()), dev(pb.mu_bar_flat()), 1.0)
    g = torch.zeros(plan.sizes["n_x"], device="cuda")
    plan.diagnostics(reset=True)
    plan.nuclear_dual_update(dev(pb.X), dev(pb.P_flat()), *args, g, 0.0)
    assert plan.diagnostics(reset=True) == {"eig_not_converged": 0, "gram_not_finite": 0}
    X = pb.X.copy()
    X[250, 250, 3] = np.nan
    plan.nuclear_dual_update(dev(X), dev(pb.P_flat()), *args, g, 0.0)
    d = plan.diagnostics(reset=True)
    log(f"    diagnostics with one NaN pixel: {d}")
    assert d == {"eig_not_converged": 0, "gram_not_finite": 1}
    assert plan.diagnostics() == {"eig_not_converged": 0, "gram_not_finite": 0}
