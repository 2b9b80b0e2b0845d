"""GPU parity of the randomized facet step (fhs_facet_prox_step_select, Sec.
3.2: a random subset of the facet duals updated) against the oracle's
facet_prox_step_select, through the C ABI.

Bar: relative L2 error <= 1e-5 per output and an element-wise bound of 1e-4
of the largest magnitude, as for the plain step; the duals of unselected
facets (their P, and the coefficient rows they own in every band) must come
back bit for bit.  The draw is seeded and passed in.  Cases span several
tiles per band, ragged sizes, two sub-cubes and deep / shallow transforms;
edge draws: all facets (the plain step's results) and none (duals untouched,
G the aggregation of the old duals).
"""
import numpy as np
import pytest

import synth
from fhs_cases import Problem, log, max_rel, rel_l2
from oracle import sara, step

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = pytest.mark.gpu
TOL = 1e-5
ELEM = 1e-4

CASES = {
    "multi_tile_300x260x8_q3x3_o24": dict(ny=300, nx=260, L=8, qy=3, qx=3, oy=24, ox=24, blobs=30),
    "ragged_101x77x6_q3x2_c2": dict(ny=101, nx=77, L=6, qy=3, qx=2, C=2, oy=7, ox=5, blobs=12),
    "c4_64x64x12_q4x4_o0": dict(ny=64, nx=64, L=12, qy=4, qx=4, C=4, blobs=10),
    "lc20_128x96x20_q2x3_levels2": dict(ny=128, nx=96, L=20, qy=2, qx=3, oy=16, ox=12, levels=2, blobs=10),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run_select(pb, plan, sel, zeta=1.0, kappa=1.0):
    s = plan.sizes
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.empty(s["n_x"], dtype=torch.float32, device="cuda")
    seld = dev(np.asarray(sel, dtype=np.uint8).reshape(-1))
    plan.facet_prox_step_select(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                                dev(pb.mu_bar_flat()), zeta, kappa, seld, g)
    return host(p), host(w), host(g)


def check(pb, out, ref, sel, tag):
    Pd, Wd, Gd = out
    Pn, Wn, G = ref
    Pref = np.concatenate([q.reshape(-1) for row in Pn for q in row])
    Wref = np.concatenate(Wn, axis=1).reshape(-1)
    for name, a, b in (("P", Pd, Pref), ("W", Wd, Wref), ("G", Gd, G.reshape(-1))):
        e, m = rel_l2(a, b), max_rel(a, b)
        log(f"    {tag} {name}: rel_l2 {e:.2e} max {m:.2e}")
        assert e <= TOL and m <= ELEM, (tag, name, e, m)
    # the duals of unselected facets come back bit for bit
    P0, W0 = pb.P_flat(), pb.W_flat().reshape(pb.I, pb.L)
    Wv = Wd.reshape(pb.I, pb.L)
    geom, Lc = pb.geom, pb.Lc
    off = 0
    for c in range(pb.C):
        for q, f in enumerate(geom.facets):
            n = f.n_rows * Lc
            if not sel[c][q]:
                assert np.array_equal(Pd[off:off + n], P0[off:off + n]), (tag, "P kept", c, q)
            off += n
    shapes = sara.band_shapes(pb.ny, pb.nx, pb.levels)
    starts = np.concatenate([[0], np.cumsum([a * b for a, b in shapes])])
    for c in range(pb.C):
        cols = slice(c * Lc, (c + 1) * Lc)
        for q, f in enumerate(geom.facets):
            if sel[c][q]:
                continue
            for k, ((r0, r1), (c0, c1)) in enumerate(geom.owned_rects(f)):
                b = shapes[k][1]
                rows = (starts[k] + np.arange(r0, r1)[:, None] * b + np.arange(c0, c1)[None, :]).reshape(-1)
                assert np.array_equal(Wv[rows, cols], W0[rows, cols]), (tag, "W kept", c, q, k)


@pytest.mark.parametrize("prob", [0.5, 0.2])
@pytest.mark.parametrize("name", list(CASES))
def test_select_step_matches_oracle(name, prob):
    args = CASES[name]
    pb = Problem(**args, warm=True)
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    sel = synth.facet_selection(pb.C, pb.geom.Q, prob, 101 + int(100 * prob))
    sel[0, 0] = True
    log(f"[case] select {name} p={prob}: {int(sel.sum())} of {sel.size} facets")
    ref = step.facet_prox_step_select(pb.X, pb.P, pb.W, pb.theta, pb.theta_bar, pb.mu, pb.mu_bar, 0.9, 1.2,
                                      pb.geom, sel, C=pb.C)
    check(pb, run_select(pb, plan, sel, 0.9, 1.2), ref, sel, "random")


@pytest.mark.parametrize("name", ["multi_tile_300x260x8_q3x3_o24", "ragged_101x77x6_q3x2_c2"])
def test_select_all_and_none(name):
    pb = Problem(**CASES[name], warm=True)
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    log(f"[case] select all / none {name}")
    Q = pb.geom.Q
    for tag, sel in (("all", np.ones((pb.C, Q), dtype=bool)), ("none", np.zeros((pb.C, Q), dtype=bool))):
        ref = step.facet_prox_step_select(pb.X, pb.P, pb.W, pb.theta, pb.theta_bar, pb.mu, pb.mu_bar, 1.0, 1.0,
                                          pb.geom, sel, C=pb.C)
        out = run_select(pb, plan, sel)
        check(pb, out, ref, sel, tag)
        if tag == "none":
            assert np.array_equal(out[0], pb.P_flat()) and np.array_equal(out[1], pb.W_flat())
    # everything selected: the plain step's duals, bit for bit
    s = plan.sizes
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.empty(s["n_x"], dtype=torch.float32, device="cuda")
    plan.facet_prox_step(dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu),
                         dev(pb.mu_bar_flat()), 1.0, 1.0, g)
    Pa, Wa, Ga = run_select(pb, plan, np.ones((pb.C, Q), dtype=bool))
    assert np.array_equal(Pa, host(p)) and np.array_equal(Wa, host(w))
    assert rel_l2(Ga, host(g)) <= 1e-6


def test_select_rejects_missing_draw():
    pb = Problem(**CASES["c4_64x64x12_q4x4_o0"])
    plan = fhs.Plan(*pb.cfg).attach_workspace()
    s = plan.sizes
    bad = torch.zeros(s["n_facets"] + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(fhs.FhsError):
        plan.facet_prox_step_select(dev(pb.X), dev(pb.P_flat()), dev(pb.W_flat()), dev(pb.theta_flat()),
                                    dev(pb.theta_bar_flat()), dev(pb.mu), dev(pb.mu_bar_flat()), 1.0, 1.0, bad,
                                    torch.empty(s["n_x"], dtype=torch.float32, device="cuda"))
