"""The mixed-precision form (FHS_PRECISION_MIXED) against the FP64 oracle,
beside the FP32 form: the l21 update's wavelet filters accumulated in FP32,
the facet Gram of BF16-rounded Z on BF16 MFMA with FP32 accumulation, the
eigendecomposition, sigma scaling and reconstruction in FP64.

Stated bounds (from the arithmetic; the measured errors are logged):
* W+ and the l21 part of G: FP32 accumulation of unit-norm filters over
  differences of neighbouring values, relative L2 <= 1e-4;
* P+ of facet q: rounding Z to BF16 (unit roundoff u = 2^-8) perturbs the
  Gram by ~2u ||Z||^2, its eigenvalues by as much (Weyl), and
  h_j = min(1, t_j / s_j) by ~u s_1^2 / t^2 near the threshold, so the
  facet's relative error is bounded by 4 u kappa_q^2 with
  kappa_q = s_1(Z_q) / min_j t_j (at least the FP32 form's 1e-5);
* G: the sum of both parts, bounded by the larger.
"""
import numpy as np
import pytest

from fhs_cases import Problem, log, rel_l2
from oracle import step

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = pytest.mark.gpu
U_BF16 = 2.0 ** -8

CASES = {
    "cfg1_256x256x20_q2x2_o32": dict(ny=256, nx=256, L=20, qy=2, qx=2, oy=32, ox=32),
    "ragged_101x77x6_q3x2_c2": dict(ny=101, nx=77, L=6, qy=3, qx=2, C=2, oy=7, ox=5, blobs=12),
    "lc64_70x45x64_q2x1": dict(ny=70, nx=45, L=64, qy=2, qx=1, oy=9, ox=0, blobs=8),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(pb, precision):
    plan = fhs.Plan(*pb.cfg, precision=precision).attach_workspace()
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.empty(plan.sizes["n_x"], dtype=torch.float32, device="cuda")
    plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                         dev(pb.mu_bar_flat()), 1.0, 1.0, g)
    torch.cuda.synchronize()
    return plan, p.cpu().numpy(), w.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("scale", [1.0, 100.0])
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_precision_bounds(name, scale):
    """scale multiplies the nuclear thresholds (100: small kappa, where the
    BF16 Gram's bound is tight)."""
    pb = Problem(**CASES[name], warm=True)
    pb.mu_bar = np.asarray(pb.mu_bar) * scale
    log(f"[case] mixed precision {name}, thresholds x{scale:g}")
    Pn, Wn, G = pb.oracle_step()
    out = {prec: run(pb, prec) for prec in (0, 1)}
    Lc, Q = pb.Lc, pb.geom.Q
    kappas, worst = [], 0.0
    for c in range(pb.C):
        for q, f in enumerate(pb.geom.facets):
            Z = np.asarray(pb.P[c][q], dtype=np.float64).reshape(-1, Lc) + \
                step.facet_matrix(pb.X, f, step.subcube_channels(pb.L, pb.C)[c])
            s1 = np.linalg.svd(Z, compute_uv=False)[0]
            t = pb.mu_bar[c][q] * np.asarray(pb.theta_bar[c][q])
            kappa = s1 / np.min(t)
            kappas.append(kappa)
            fi = out[1][0].facet(c * Q + q)
            n = f.n_rows * Lc
            ref = Pn[c][q].reshape(-1)
            e = rel_l2(out[1][1][fi["poff"]:fi["poff"] + n], ref)
            e32 = rel_l2(out[0][1][fi["poff"]:fi["poff"] + n], ref)
            bound = max(1e-5, 4 * U_BF16 * kappa ** 2)
            worst = max(worst, e / bound)
            log(f"    facet ({c},{q}): kappa {kappa:.3e}  P+ err mixed {e:.3e} (bound {bound:.2e})  fp32 {e32:.3e}")
            assert e32 <= 1e-5
            assert e <= bound, (c, q, kappa, e, bound)
    eW = {prec: rel_l2(out[prec][2], np.concatenate(Wn, axis=1).reshape(-1)) for prec in (0, 1)}
    eG = {prec: rel_l2(out[prec][3], G.reshape(-1)) for prec in (0, 1)}
    log(f"    W+ err: fp32 {eW[0]:.3e}  mixed {eW[1]:.3e};  G err: fp32 {eG[0]:.3e}  mixed {eG[1]:.3e};  "
        f"kappa range {min(kappas):.2e} .. {max(kappas):.2e}; worst P+ err / bound {worst:.3f}")
    assert eW[0] <= 1e-5 and eG[0] <= 1e-5
    assert eW[1] <= 1e-4
    assert eG[1] <= max(1e-4, 4 * U_BF16 * max(kappas) ** 2)


@pytest.mark.parametrize("L,C", [(6, 2), (20, 1), (64, 1), (40, 4)])
def test_bf16_gram_exact_on_representable_inputs(L, C):
    """Z exactly representable in BF16 (small integers, window D = 1 with no
    overlap, Xcheck = 0): the BF16 products are exact and their FP32 sums too,
    so the mixed form's P+ equals the FP32 form's up to the FP64
    eigensolver's rounding (checks the BF16 MFMA operand layout)."""
    pb = Problem(48, 40, L, 2, 2, C, 0, 0, 2, zero=True)
    rng = np.random.default_rng(31 + L)
    pb.P = [[rng.integers(-8, 9, f.nuc_shape + (pb.Lc,)).astype(np.float32) for f in pb.geom.facets]
            for _ in range(C)]
    pb.mu_bar = np.full((C, pb.geom.Q), 6.0)
    log(f"[case] BF16 Gram on integer Z, L={L}, C={C}")
    _, p32, _, _ = run(pb, 0)
    _, pmx, _, _ = run(pb, 1)
    e = rel_l2(pmx, p32)
    log(f"    P+ mixed vs fp32: rel_l2 {e:.3e}")
    assert e <= 1e-6


def test_mixed_precision_leaves_weights_and_fp32_form_alone():
    """The weights (fhs_reweight) keep the FP64 path in both forms, bit for
    bit; the FP32 form of a plan is unchanged by the existence of the mixed one."""
    pb = Problem(**CASES["cfg1_256x256x20_q2x2_o32"], warm=True)
    res = []
    for prec in (0, 1):
        plan = fhs.Plan(*pb.cfg, precision=prec).attach_workspace()
        th = torch.empty(plan.sizes["n_theta"], dtype=torch.float32, device="cuda")
        tb = torch.empty(plan.sizes["n_theta_bar"], dtype=torch.float64, device="cuda")
        plan.reweight(dev(pb.X), dev(pb.mu), dev(pb.mu_bar_flat()), th, tb)
        torch.cuda.synchronize()
        res.append((th.cpu().numpy(), tb.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
