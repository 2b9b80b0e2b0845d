"""CPU tests of the C-ABI library: it loads, exports every symbol that
include/fhs.h declares, and its host-side results (filters, chi moments,
heuristics, facet geometry, band layout, error paths) agree with the oracle.
No compute call is made (no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2003_07358_amd as fhs
from oracle import filters, geometry, heuristics, sara

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhs.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fhs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(fhs.library_path())
    names = declared_symbols()
    assert len(names) == 42
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(fhs.binding.SYMBOLS)


@pytest.mark.parametrize("N", range(1, 9))
def test_library_filters_match_oracle(N):
    # two independent derivations (Durand-Kerner in C++, companion-matrix roots
    # in numpy) of the same published construction
    assert np.max(np.abs(fhs.filter_taps(N) - filters.lowpass(N))) < 1e-14


def test_chi_and_heuristics_match_oracle():
    for k in (1, 2, 10, 20, 60, 64, 100):
        m, s = fhs.chi_mean_std(k)
        mo, so = heuristics.chi_mean_std(k)
        assert abs(m - mo) < 1e-12 and abs(s - so) < 1e-10
    p = fhs.Plan(256, 256, 20, 2, 2, 1, 32, 32, 4)
    g = geometry.Geometry(256, 256, 2, 2, 32, 32, 4)
    mu, mub = p.heuristics(0.01)
    assert abs(mu[0] - heuristics.mu_sparsity(0.01, 20)) < 1e-14
    for q, f in enumerate(g.facets):
        assert abs(mub[q] - heuristics.mu_low_rank(0.01, f.n_rows, 20)) < 1e-12


@pytest.mark.parametrize("case", [
    (256, 256, 20, 2, 2, 1, 32, 32, 4),
    (1024, 2048, 20, 4, 4, 1, 64, 64, 4),
    (101, 77, 6, 3, 2, 2, 7, 5, 4),
    (64, 64, 12, 4, 4, 3, 0, 0, 2),
    (300, 260, 4, 1, 1, 1, 0, 0, 4),
])
def test_plan_geometry_matches_oracle(case):
    ny, nx, L, qy, qx, C, oy, ox, lev = case
    p = fhs.Plan(ny, nx, L, qy, qx, C, oy, ox, lev)
    g = geometry.Geometry(ny, nx, qy, qx, oy, ox, lev)
    Lc = L // C
    assert p.sizes["n_facets"] == C * g.Q
    off = 0
    for c in range(C):
        for q, f in enumerate(g.facets):
            d = p.facet(c * g.Q + q)
            assert (d["c"], d["sy"], d["sx"]) == (c, f.sy, f.sx)
            assert ((d["ty0"], d["ty1"]), (d["tx0"], d["tx1"])) == f.tile
            assert ((d["wy0"], d["wy1"]), (d["wx0"], d["wx1"])) == f.nuc_window
            assert d["poff"] == off
            off += f.n_rows * Lc
    assert p.sizes["n_p"] == off
    shapes = sara.band_shapes(ny, nx, lev)
    bands = p.bands()
    assert len(bands) == len(shapes)
    start = 0
    for (rows, cols, first, level), s in zip(bands, shapes):
        assert (rows, cols) == s and first == start
        start += rows * cols
    assert p.sizes["n_coef"] == sara.n_coefficients(ny, nx, lev) == start
    assert p.sizes["n_w"] == start * L
    assert p.sizes["n_theta"] == start * C
    assert p.sizes["n_theta_bar"] == C * g.Q * Lc


@pytest.mark.parametrize("bad", [
    dict(ny=0, nx=8, nchan=2),
    dict(ny=8, nx=8, nchan=6, n_sub=4),           # C does not divide L
    dict(ny=8, nx=8, nchan=130),                  # > 64 channels per sub-cube
    dict(ny=64, nx=64, nchan=2, qy=4, qx=4, overlap_y=17, overlap_x=0),   # overlap > tile
    dict(ny=8, nx=8, nchan=2, levels=7),
    dict(ny=8, nx=8, nchan=2, qy=65),
])
def test_plan_rejects_invalid_configs(bad):
    with pytest.raises(fhs.FhsError):
        fhs.Plan(**bad)


def test_compute_without_workspace_is_an_error():
    # checked on the host before anything touches a device pointer
    lib = fhs.lib()
    p = fhs.Plan(16, 16, 2)
    rc = lib.fhs_sara_analysis(p._p, ctypes.c_void_p(0), ctypes.c_void_p(0), ctypes.c_void_p(0))
    assert rc == -5
    assert b"workspace" in lib.fhs_last_error()
    rc = lib.fhs_plan_set_workspace(p._p, ctypes.c_void_p(0), 0)
    assert rc == -1


def test_tuning_roundtrip_and_validation():
    plan = fhs.Plan(256, 256, 20, 2, 2, 1, 32, 32, 4)
    t = plan.tuning
    assert t["ana_rows"][:4] == [64, 64, 64, 64] and t["concurrent"] == 1 and t["fin_waves"] == 8
    assert t["nuc_seg"] in (16, 32, 64)
    plan.tuning = {"ana_rows": [32, 64, 128, 16, 64, 64], "fin_rows": 256, "nuc_seg": 16}
    t2 = plan.tuning
    assert t2["ana_rows"][:4] == [32, 64, 128, 16] and t2["fin_rows"] == 256 and t2["nuc_seg"] == 16
    for bad in ({"ana_rows": [12, 64, 64, 64, 64, 64]}, {"ana_phase": 3}, {"syn_rows": 20}, {"nuc_seg": 48},
                {"nuc_chunk_rows": 0}, {"concurrent": 2}, {"ana_direct": 64}, {"fin_waves": 5},
                {"ana_order": 64}):
        with pytest.raises(fhs.FhsError):
            plan.tuning = bad
    assert plan.tuning == t2   # a rejected setting leaves the plan unchanged


def test_data_plan_host_side_matches_oracle():
    """The data plan's host computations (no GPU): grid sizes and the inverse
    sampling density per channel against the oracle's."""
    import synth
    from oracle import nufft
    covs = synth.channel_coverages(700, 3, 11)
    covs[1] = covs[1][:0]                      # a channel without visibilities
    dp = fhs.DataPlan(32, 64, covs)
    assert (dp.K1, dp.K2, dp.m) == (64, 128, 1400)
    u = dp.preconditioner()
    for l, c in enumerate(covs):
        if len(c):
            ref = nufft.inverse_density(c, 64, 128)
            assert np.array_equal(u[dp.voff[l]:dp.voff[l + 1]], ref)
    with pytest.raises(fhs.FhsError):
        fhs.DataPlan(48, 64, covs)             # not a power of two
    with pytest.raises(fhs.FhsError):
        fhs.DataPlan(32, 64, [np.array([[np.nan, 0.0]])])
