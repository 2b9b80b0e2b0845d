"""The no-allocation entry point (fhs_facet_prox_step_noalloc) against the
workspace entry point (fhs_facet_prox_step): same outputs bit for bit, for two
calls in a row on plans with no workspace attached, the second smaller than
the first; a plan whose workspace exceeds the static scratch is rejected
before anything is launched."""
import numpy as np
import pytest

from fhs_cases import Problem, log, rel_l2

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _step(plan, pb, noalloc):
    p, w = dev(pb.P_flat()), dev(pb.W_flat())
    g = torch.full((plan.sizes["n_x"],), float("nan"), device="cuda")
    args = (dev(pb.X), p, w, dev(pb.theta_flat()), dev(pb.theta_bar_flat()), dev(pb.mu), dev(pb.mu_bar_flat()),
            1.0, 1.0, g)
    if noalloc:
        plan.facet_prox_step_noalloc(*args)
    else:
        plan.facet_prox_step(*args)
    torch.cuda.synchronize()
    return p.cpu().numpy(), w.cpu().numpy(), g.cpu().numpy()


def test_noalloc_step_matches_workspace_step():
    limit = fhs.lib().fhs_noalloc_scratch_bytes()
    cases = [dict(ny=256, nx=256, L=20, qy=2, qx=2, oy=32, ox=32, warm=True),
             dict(ny=101, nx=77, L=6, qy=3, qx=2, C=2, oy=7, ox=5, blobs=12, warm=True)]
    for k, case in enumerate(cases):
        log(f"[case] no-alloc call {k + 1}: {case}")
        pb = Problem(**case)
        plan = fhs.Plan(*pb.cfg)                      # no workspace attached
        need = plan.sizes["workspace_bytes"]
        assert 0 < need <= limit, (need, limit)
        got = _step(plan, pb, noalloc=True)
        ref = _step(fhs.Plan(*pb.cfg).attach_workspace(), pb, noalloc=False)
        for name, a, b in zip(("P+", "W+", "G"), got, ref):
            log(f"    {name}: identical={np.array_equal(a, b)} rel_l2={rel_l2(a, b):.3e}")
            assert np.array_equal(a, b), name
        Pn, Wn, G = pb.oracle_step()
        assert rel_l2(got[0], np.concatenate([q.reshape(-1) for row in Pn for q in row])) <= 1e-5
        assert rel_l2(got[1], np.concatenate(Wn, axis=1).reshape(-1)) <= 1e-5
        assert rel_l2(got[2], G.reshape(-1)) <= 1e-5


def test_noalloc_rejects_oversized_plan():
    plan = fhs.Plan(1024, 1024, 20, 4, 4, 1, 32, 32, 4)
    assert plan.sizes["workspace_bytes"] > fhs.lib().fhs_noalloc_scratch_bytes()
    z = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device="cuda")
    s = plan.sizes
    with pytest.raises(fhs.FhsError, match="static scratch"):
        plan.facet_prox_step_noalloc(z(s["n_x"]), z(s["n_p"]), z(s["n_w"]), z(s["n_theta"]),
                                     z(s["n_theta_bar"], torch.float64), z(1, torch.float64),
                                     z(s["n_facets"], torch.float64), 1.0, 1.0, z(s["n_x"]))
