"""ctypes binding of libfhs (include/fhs.h).

Argument marshalling only: sizes, dtypes and contiguity are checked against
the plan, then raw device pointers and the current HIP stream are passed to the
C ABI; every step of the computation runs in the library's HIP kernels.  There
is no fallback: if libfhs.so is missing, using the binding raises FhsError.
"""
import ctypes
import json
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfhs.so")
_lib = None


class FhsError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("ny", "nx", "nchan", "qy", "qx", "n_sub", "overlap_y", "overlap_x", "levels", "precision",
                 "spectral_overlap")]


class _DataConfig(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("ny", "nx", "nchan")]


class _Sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_x", "n_p", "n_coef", "n_w", "n_theta", "n_facets", "n_theta_bar", "n_bands",
                 "workspace_bytes")]


class _Tuning(ctypes.Structure):
    _fields_ = [("ana_rows", ctypes.c_int32 * 6)] + [(n, ctypes.c_int32) for n in
                ("ana_phase", "syn_rows", "fin_rows", "nuc_seg", "nuc_chunk_rows", "concurrent", "ana_direct",
                 "fin_waves", "ana_order")]


class _PdfbState(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("x", "xcheck", "p", "w", "v", "y", "eps", "theta", "theta_bar", "mu", "mu_bar", "grad", "xi")] + \
               [(n, ctypes.c_double) for n in ("zeta", "kappa", "tau")]


class _SolveParams(ctypes.Structure):
    _fields_ = [("max_reweights", ctypes.c_int32), ("rw_tol", ctypes.c_double), ("min_iter", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("pdfb_tol", ctypes.c_double), ("res_factor", ctypes.c_double)]


class _SolveReport(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_int32), ("iterations", ctypes.c_int64)]


SYMBOLS = {
    "fhs_version": (ctypes.c_int, []),
    "fhs_last_error": (ctypes.c_char_p, []),
    "fhs_filter": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "fhs_chi_mean_std": (ctypes.c_int, [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "fhs_plan_create": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_void_p)]),
    "fhs_plan_destroy": (None, [ctypes.c_void_p]),
    "fhs_plan_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Sizes)]),
    "fhs_plan_facet": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "fhs_plan_band": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "fhs_plan_heuristics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "fhs_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "fhs_plan_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "fhs_plan_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Tuning)]),
    "fhs_plan_autotune": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 8 + [ctypes.c_int32, ctypes.c_void_p]),
    "fhs_sara_analysis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_sara_synthesis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_void_p]),
    "fhs_l21_dual_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_float,
                                           ctypes.c_void_p]),
    "fhs_nuclear_dual_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p]),
    "fhs_facet_prox_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_facet_prox_step_plain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_facet_prox_step_select": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "fhs_facet_prox_step_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_noalloc_scratch_bytes": (ctypes.c_int64, []),
    "fhs_reweight": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_snr": (ctypes.c_int, [ctypes.c_void_p] * 7),
    "fhs_pdfb_closure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_pdfb_iteration": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_PdfbState), ctypes.c_int32,
                                          ctypes.c_void_p]),
    "fhs_reweighting_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_PdfbState), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_SolveParams),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(_SolveReport), ctypes.c_void_p]),
    "fhs_pdfb_graph_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_PdfbState), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "fhs_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_graph_destroy": (None, [ctypes.c_void_p]),
    "fhs_plan_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "fhs_plan_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                            ctypes.c_void_p]),
    "fhs_data_plan_create": (ctypes.c_int, [ctypes.POINTER(_DataConfig), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "fhs_data_plan_destroy": (None, [ctypes.c_void_p]),
    "fhs_data_plan_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "fhs_data_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "fhs_data_preconditioner": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fhs_nufft_forward": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "fhs_nufft_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_float, ctypes.c_void_p]),
    "fhs_data_dual_update": (ctypes.c_int, [ctypes.c_void_p] * 8 + [ctypes.c_int32] + [ctypes.c_void_p] * 3),
    "fhs_plan_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int64)]),
}

# kernel identifiers of fhs_plan_profile (include/fhs.h)
KERNELS = {
    "analysis_l1": 0, "analysis": 1, "synthesis": 2, "synth_final_a": 3, "synth_final_b": 4,
    "nuc_gram": 5, "nuc_eig": 6, "nuc_recon": 7, "nuc_gather": 8, "closure": 9,
}


def lib():
    """The loaded libfhs (raises FhsError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise FhsError(f"{_LIB_PATH} is missing: build it with `python -m paper_2003_07358_amd.build`")
        handle = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def library_path():
    return _LIB_PATH


def _check(rc):
    if rc != 0:
        raise FhsError(f"libfhs error {rc}: {lib().fhs_last_error().decode()}")


def _dptr(arr):
    return ctypes.cast(arr.ctypes.data, ctypes.POINTER(ctypes.c_double))


def filter_taps(N):
    """dbN scaling filter as derived by the library (host computation)."""
    out = np.zeros(2 * N, dtype=np.float64)
    _check(lib().fhs_filter(N, _dptr(out)))
    return out


def chi_mean_std(k):
    m, s = ctypes.c_double(), ctypes.c_double()
    _check(lib().fhs_chi_mean_std(float(k), ctypes.byref(m), ctypes.byref(s)))
    return m.value, s.value


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


class Plan:
    """Geometry of one problem (include/fhs.h, fhs_plan_create) plus its workspace."""

    def __init__(self, ny, nx, nchan, qy=1, qx=1, n_sub=1, overlap_y=0, overlap_x=0, levels=4, precision=0,
                 spectral_overlap=0):
        """precision: 0 = FHS_PRECISION_FP32, 1 = FHS_PRECISION_MIXED; spectral_overlap: channels
        by which the low-rankness facets of contiguous sub-cubes overlap (0: interleaved
        sub-cubes), see include/fhs.h."""
        self._lib = lib()
        self.cfg = _Config(ny, nx, nchan, qy, qx, n_sub, overlap_y, overlap_x, levels, precision,
                           spectral_overlap)
        handle = ctypes.c_void_p()
        _check(self._lib.fhs_plan_create(ctypes.byref(self.cfg), ctypes.byref(handle)))
        self._p = handle
        s = _Sizes()
        _check(self._lib.fhs_plan_sizes(self._p, ctypes.byref(s)))
        self.sizes = {n: getattr(s, n) for n, _ in _Sizes._fields_}
        self.ny, self.nx, self.L, self.C = ny, nx, nchan, n_sub
        self.Lc = nchan // n_sub
        self.Q = qy * qx
        self.levels = levels
        self.precision = precision
        self.spectral_overlap = spectral_overlap
        self.Ln = self.Lc + spectral_overlap  # columns of a facet matrix
        self.workspace = None

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value:
            self._lib.fhs_plan_destroy(p)
            self._p = None

    # ------------------------------------------------------------ host queries
    def facet(self, f):
        out = (ctypes.c_int64 * 12)()
        _check(self._lib.fhs_plan_facet(self._p, f, out))
        keys = ("c", "sy", "sx", "ty0", "ty1", "tx0", "tx1", "wy0", "wy1", "wx0", "wx1", "poff")
        return dict(zip(keys, list(out)))

    def band(self, k):
        out = (ctypes.c_int64 * 4)()
        _check(self._lib.fhs_plan_band(self._p, k, out))
        return tuple(out)

    def bands(self):
        return [self.band(k) for k in range(self.sizes["n_bands"])]

    def heuristics(self, sigma_bar):
        sb = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma_bar, dtype=np.float64), (self.C,)))
        mu = np.zeros(self.C)
        mub = np.zeros(self.sizes["n_facets"])
        _check(self._lib.fhs_plan_heuristics(self._p, _dptr(sb), _dptr(mu), _dptr(mub)))
        return mu, mub

    # ------------------------------------------------------------ launch shapes
    @property
    def tuning(self):
        t = _Tuning()
        _check(self._lib.fhs_plan_get_tuning(self._p, ctypes.byref(t)))
        d = {n: getattr(t, n) for n, _ in _Tuning._fields_}
        d["ana_rows"] = list(t.ana_rows)
        return d

    @tuning.setter
    def tuning(self, d):
        t = _Tuning()
        _check(self._lib.fhs_plan_get_tuning(self._p, ctypes.byref(t)))
        for n, v in d.items():
            if n == "ana_rows":
                for j, r in enumerate(v):
                    t.ana_rows[j] = int(r)
            else:
                setattr(t, n, int(v))
        _check(self._lib.fhs_plan_set_tuning(self._p, ctypes.byref(t)))

    def tuning_key(self, device=None):
        """Key of this plan's tuned launch shapes in a cache: device name,
        library version and the plan configuration."""
        import torch
        name = torch.cuda.get_device_name(device)
        c = self.cfg
        return (f"{name}|fhs{self._lib.fhs_version()}|{c.ny}x{c.nx}x{c.nchan}|q{c.qy}x{c.qx}|C{c.n_sub}|"
                f"o{c.overlap_y},{c.overlap_x}|lev{c.levels}|prec{c.precision}|so{c.spectral_overlap}")

    def autotune(self, xcheck, p, w, theta, theta_bar, mu, mu_bar, grad, reps=3, cache=None):
        """Times candidate launch shapes on these arrays and keeps the fastest
        (p, w and grad are overwritten: pass scratch copies).  cache: path of a
        JSON file of tuned shapes by tuning_key(); a hit sets the stored shapes
        without timing anything, a miss tunes and adds the result."""
        import torch
        self._need_ws()
        key = self.tuning_key(xcheck.device) if cache else None
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                entries = json.load(fh)
            if key in entries:
                self.tuning = entries[key]
                return self.tuning
        s = self.sizes
        _check(self._lib.fhs_plan_autotune(
            self._p, self._t(xcheck, s["n_x"], torch.float32, "xcheck"),
            self._t(p, s["n_p"], torch.float32, "p"), self._t(w, s["n_w"], torch.float32, "w"),
            self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"),
            self._t(mu, self.C, torch.float64, "mu"), self._t(mu_bar, s["n_facets"], torch.float64, "mu_bar"),
            self._t(grad, s["n_x"], torch.float32, "grad"), int(reps), _stream(xcheck)))
        if cache:
            entries = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    entries = json.load(fh)
            entries[key] = self.tuning
            tmp = f"{cache}.{os.getpid()}.tmp"
            with open(tmp, "w") as fh:
                json.dump(entries, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return self.tuning

    # ------------------------------------------------------------ device side
    def attach_workspace(self, device="cuda"):
        import torch
        nbytes = max(256, self.sizes["workspace_bytes"])
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        _check(self._lib.fhs_plan_set_workspace(self._p, ctypes.c_void_p(ws.data_ptr() + off), nbytes))
        return self

    def _t(self, t, n, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise FhsError(f"{name}: expected a device tensor")
        if t.dtype != dtype:
            raise FhsError(f"{name}: expected {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise FhsError(f"{name}: must be contiguous")
        if t.numel() != n:
            raise FhsError(f"{name}: expected {n} elements, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())

    def _need_ws(self):
        if self.workspace is None:
            raise FhsError("attach_workspace() first")

    def sara_analysis(self, x, w):
        import torch
        self._need_ws()
        s = self.sizes
        _check(self._lib.fhs_sara_analysis(self._p, self._t(x, s["n_x"], torch.float32, "x"),
                                           self._t(w, s["n_w"], torch.float32, "w"), _stream(x)))

    def sara_synthesis(self, w, x, alpha=1.0, beta=0.0):
        import torch
        self._need_ws()
        s = self.sizes
        _check(self._lib.fhs_sara_synthesis(self._p, self._t(w, s["n_w"], torch.float32, "w"),
                                            self._t(x, s["n_x"], torch.float32, "x"), float(alpha),
                                            float(beta), _stream(x)))

    def l21_dual_update(self, xcheck, w, theta, mu, kappa, grad, beta=0.0):
        import torch
        self._need_ws()
        s = self.sizes
        _check(self._lib.fhs_l21_dual_update(
            self._p, self._t(xcheck, s["n_x"], torch.float32, "xcheck"),
            self._t(w, s["n_w"], torch.float32, "w"), self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(mu, self.C, torch.float64, "mu"), float(kappa),
            self._t(grad, s["n_x"], torch.float32, "grad"), float(beta), _stream(xcheck)))

    def nuclear_dual_update(self, xcheck, p, theta_bar, mu_bar, zeta, grad, beta=0.0):
        import torch
        self._need_ws()
        s = self.sizes
        _check(self._lib.fhs_nuclear_dual_update(
            self._p, self._t(xcheck, s["n_x"], torch.float32, "xcheck"),
            self._t(p, s["n_p"], torch.float32, "p"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"),
            self._t(mu_bar, s["n_facets"], torch.float64, "mu_bar"), float(zeta),
            self._t(grad, s["n_x"], torch.float32, "grad"), float(beta), _stream(xcheck)))

    def facet_prox_step(self, xcheck, p, w, theta, theta_bar, mu, mu_bar, zeta, kappa, grad, plain=False):
        """plain=True: the per-facet execution form (fhs_facet_prox_step_plain)."""
        import torch
        self._need_ws()
        s = self.sizes
        fn = self._lib.fhs_facet_prox_step_plain if plain else self._lib.fhs_facet_prox_step
        _check(fn(
            self._p, self._t(xcheck, s["n_x"], torch.float32, "xcheck"),
            self._t(p, s["n_p"], torch.float32, "p"), self._t(w, s["n_w"], torch.float32, "w"),
            self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"),
            self._t(mu, self.C, torch.float64, "mu"),
            self._t(mu_bar, s["n_facets"], torch.float64, "mu_bar"), float(zeta), float(kappa),
            self._t(grad, s["n_x"], torch.float32, "grad"), _stream(xcheck)))

    def facet_prox_step_select(self, xcheck, p, w, theta, theta_bar, mu, mu_bar, zeta, kappa, select, grad):
        """fhs_facet_prox_step_select: the randomized step; select is a device
        uint8 tensor of n_facets flags (facet descriptor order)."""
        import torch
        self._need_ws()
        s = self.sizes
        _check(self._lib.fhs_facet_prox_step_select(
            self._p, self._t(xcheck, s["n_x"], torch.float32, "xcheck"),
            self._t(p, s["n_p"], torch.float32, "p"), self._t(w, s["n_w"], torch.float32, "w"),
            self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"),
            self._t(mu, self.C, torch.float64, "mu"),
            self._t(mu_bar, s["n_facets"], torch.float64, "mu_bar"), float(zeta), float(kappa),
            self._t(select, s["n_facets"], torch.uint8, "select"),
            self._t(grad, s["n_x"], torch.float32, "grad"), _stream(xcheck)))

    def facet_prox_step_noalloc(self, xcheck, p, w, theta, theta_bar, mu, mu_bar, zeta, kappa, grad):
        """fhs_facet_prox_step_noalloc: the step on the library's static device
        scratch (no workspace needed; plans whose workspace exceeds the
        scratch are rejected)."""
        import torch
        s = self.sizes
        _check(self._lib.fhs_facet_prox_step_noalloc(
            self._p, self._t(xcheck, s["n_x"], torch.float32, "xcheck"),
            self._t(p, s["n_p"], torch.float32, "p"), self._t(w, s["n_w"], torch.float32, "w"),
            self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"),
            self._t(mu, self.C, torch.float64, "mu"),
            self._t(mu_bar, s["n_facets"], torch.float64, "mu_bar"), float(zeta), float(kappa),
            self._t(grad, s["n_x"], torch.float32, "grad"), _stream(xcheck)))

    # ------------------------------------------------------------ PDFB iterations
    def pdfb_closure(self, x, xcheck, v, y, eps, grad, tau, xi):
        """Data-fidelity dual (identity operator), primal update, extrapolation;
        xi: a float64 device tensor of C elements receiving the relative
        variation of each sub-cube."""
        import torch
        self._need_ws()
        n = self.sizes["n_x"]
        _check(self._lib.fhs_pdfb_closure(
            self._p, self._t(x, n, torch.float32, "x"), self._t(xcheck, n, torch.float32, "xcheck"),
            self._t(v, n, torch.float32, "v"), self._t(y, n, torch.float32, "y"),
            self._t(eps, self.L, torch.float64, "eps"), self._t(grad, n, torch.float32, "grad"), float(tau),
            self._t(xi, self.C, torch.float64, "xi"), _stream(x)))

    def snr(self, x_ref, x, eps=None):
        """Per-channel reconstruction SNR in dB (float64 device tensor [L]) and,
        with noise levels eps (float64 [L]), the log-scale SNR (else None)."""
        import torch
        self._need_ws()
        n = self.sizes["n_x"]
        out = torch.empty(self.L, dtype=torch.float64, device=x.device)
        out_log = torch.empty(self.L, dtype=torch.float64, device=x.device) if eps is not None else None
        _check(self._lib.fhs_snr(
            self._p, self._t(x_ref, n, torch.float32, "x_ref"), self._t(x, n, torch.float32, "x"),
            self._t(eps, self.L, torch.float64, "eps") if eps is not None else None, self._t(out, self.L, torch.float64, "snr"),
            self._t(out_log, self.L, torch.float64, "snr_log") if out_log is not None else None, _stream(x)))
        return out, out_log

    def pdfb_state(self, x, xcheck, p, w, v, y, eps, theta, theta_bar, mu, mu_bar, grad, xi, zeta=1.0,
                   kappa=1.0, tau=0.33):
        """Checked state block for pdfb_iteration / pdfb_graph (xi: float64, C
        entries per iteration).  The state holds references to the tensors, so
        they live at least as long as it (and any graph captured from it)."""
        import torch
        s = self.sizes
        n = s["n_x"]
        if not (isinstance(xi, torch.Tensor) and xi.is_cuda and xi.dtype == torch.float64 and xi.is_contiguous()):
            raise FhsError("xi: expected a contiguous float64 device tensor")
        if xi.numel() < self.C or xi.numel() % self.C:
            raise FhsError("xi: expected a multiple of C entries (C per iteration)")
        st = _PdfbState(
            self._t(x, n, torch.float32, "x"), self._t(xcheck, n, torch.float32, "xcheck"),
            self._t(p, s["n_p"], torch.float32, "p"), self._t(w, s["n_w"], torch.float32, "w"),
            self._t(v, n, torch.float32, "v"), self._t(y, n, torch.float32, "y"),
            self._t(eps, self.L, torch.float64, "eps"), self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"),
            self._t(mu, self.C, torch.float64, "mu"), self._t(mu_bar, s["n_facets"], torch.float64, "mu_bar"),
            self._t(grad, n, torch.float32, "grad"), ctypes.c_void_p(xi.data_ptr()),
            float(zeta), float(kappa), float(tau))
        st.n_xi = xi.numel() // self.C
        st.device = x.device
        st.keep = (x, xcheck, p, w, v, y, eps, theta, theta_bar, mu, mu_bar, grad, xi)
        return st

    def pdfb_iteration(self, state, it=0):
        self._need_ws()
        if not 0 <= it < state.n_xi:
            raise FhsError("iteration index outside xi")
        import torch
        _check(self._lib.fhs_pdfb_iteration(self._p, ctypes.byref(state), int(it),
                                            ctypes.c_void_p(torch.cuda.current_stream(state.device).cuda_stream)))

    def reweighting_solve(self, state, upsilon, upsilon_bar, x_prev, max_reweights=5, rw_tol=1e-5, min_iter=10,
                          max_iter=2000, pdfb_tol=1e-5, res_factor=1.01):
        """Alg. 1 (fhs_reweighting_solve) on a pdfb_state whose theta and
        theta_bar tensors it overwrites; xi must hold max_iter * C entries.
        Every sub-cube runs its own loops.  Returns dict(runs, iterations,
        iters, rw_xi) with iters[c] (rw_xi[c]) the iteration counts (ending
        relative variations) of sub-cube c's passes."""
        import torch
        self._need_ws()
        if max_iter > state.n_xi:
            raise FhsError("xi must hold max_iter entries")
        s = self.sizes
        prm = _SolveParams(int(max_reweights), float(rw_tol), int(min_iter), int(max_iter), float(pdfb_tol),
                           float(res_factor))
        T, C = int(max_reweights), self.C
        iters = (ctypes.c_int32 * max(1, T * C))()
        rw = (ctypes.c_double * max(1, T * C))()
        rep = _SolveReport()
        _check(self._lib.fhs_reweighting_solve(
            self._p, ctypes.byref(state), self._t(upsilon, self.C, torch.float64, "upsilon"),
            self._t(upsilon_bar, s["n_facets"], torch.float64, "upsilon_bar"),
            self._t(x_prev, s["n_x"], torch.float32, "x_prev"), ctypes.byref(prm), iters, rw, ctypes.byref(rep),
            ctypes.c_void_p(torch.cuda.current_stream(state.device).cuda_stream)))
        per = [[iters[t * C + c] for t in range(T) if iters[t * C + c] > 0] for c in range(C)]
        xis = [[rw[t * C + c] for t in range(len(per[c]))] for c in range(C)]
        return dict(runs=rep.runs, iterations=rep.iterations, iters=per, rw_xi=xis)

    def pdfb_graph(self, state, n_iter):
        """HIP graph of n_iter iterations (xi[0 .. n_iter-1])."""
        self._need_ws()
        if not 1 <= n_iter <= state.n_xi:
            raise FhsError("n_iter must be in [1, len(xi)]")
        return Graph(self, state, n_iter)

    # ------------------------------------------------------------ diagnostics
    def profile(self, kernel, max_launches=4096):
        """Time every launch of `kernel` (name from KERNELS, or None to stop)."""
        kid = -1 if kernel is None else KERNELS[kernel]
        _check(self._lib.fhs_plan_profile(self._p, kid, max_launches))

    def diagnostics(self, reset=False):
        """dict(eig_not_converged, gram_not_finite): counters since the
        workspace was attached or last reset (synchronises the stream)."""
        import torch
        self._need_ws()
        out = (ctypes.c_int64 * 2)()
        _check(self._lib.fhs_plan_diagnostics(self._p, out, int(bool(reset)),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        return {"eig_not_converged": out[0], "gram_not_finite": out[1]}

    def profile_read(self):
        """(total ms, launches) since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(self._lib.fhs_plan_profile_read(self._p, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def reweight(self, x, upsilon, upsilon_bar, theta, theta_bar):
        import torch
        self._need_ws()
        s = self.sizes
        _check(self._lib.fhs_reweight(
            self._p, self._t(x, s["n_x"], torch.float32, "x"),
            self._t(upsilon, self.C, torch.float64, "upsilon"),
            self._t(upsilon_bar, s["n_facets"], torch.float64, "upsilon_bar"),
            self._t(theta, s["n_theta"], torch.float32, "theta"),
            self._t(theta_bar, s["n_theta_bar"], torch.float64, "theta_bar"), _stream(x)))


class Graph:
    """A captured sequence of PDFB iterations (fhs_pdfb_graph_create)."""

    def __init__(self, plan, state, n_iter):
        self._lib = plan._lib
        self._plan, self._state = plan, state   # keep both alive with the graph
        handle = ctypes.c_void_p()
        _check(self._lib.fhs_pdfb_graph_create(plan._p, ctypes.byref(state), int(n_iter), ctypes.byref(handle)))
        self._g = handle
        self.n_iter = n_iter

    def launch(self):
        import torch
        _check(self._lib.fhs_graph_launch(self._g, ctypes.c_void_p(
            torch.cuda.current_stream(self._state.device).cuda_stream)))

    def close(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value:
            self._lib.fhs_graph_destroy(g)
            self._g = None

    def __del__(self):
        self.close()


class DataPlan:
    """The measurement operator and the data dual update of one cube
    (include/fhs.h, fhs_data_plan_create): image ny x nx x L, per channel l the
    uv-points uv[l] (M_l x 2, radians per pixel)."""

    def __init__(self, ny, nx, uv):
        self._lib = lib()
        self.L = len(uv)
        self.ny, self.nx = ny, nx
        self.n_vis = np.array([len(u) for u in uv], dtype=np.int64)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(u, dtype=np.float64).reshape(-1, 2) for u in uv]))
        cfg = _DataConfig(ny, nx, self.L)
        handle = ctypes.c_void_p()
        _check(self._lib.fhs_data_plan_create(ctypes.byref(cfg), self.n_vis.ctypes.data_as(ctypes.c_void_p),
                                              flat.ctypes.data_as(ctypes.c_void_p), ctypes.byref(handle)))
        self._p = handle
        out = (ctypes.c_int64 * 4)()
        _check(self._lib.fhs_data_plan_sizes(self._p, out))
        self.m, self.workspace_bytes, self.K1, self.K2 = list(out)
        self.voff = np.concatenate([[0], np.cumsum(self.n_vis)])
        self.workspace = None

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value:
            self._lib.fhs_data_plan_destroy(p)
            self._p = None

    def attach_workspace(self, device="cuda"):
        import torch
        nbytes = max(256, self.workspace_bytes)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws
        _check(self._lib.fhs_data_plan_set_workspace(self._p, ctypes.c_void_p(ws.data_ptr() + off), nbytes))
        return self

    def preconditioner(self):
        """Inverse sampling density per visibility (host float64)."""
        u = np.empty(self.m, dtype=np.float64)
        _check(self._lib.fhs_data_preconditioner(self._p, u.ctypes.data_as(ctypes.c_void_p)))
        return u

    def _t(self, t, n, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise FhsError(f"{name}: expected a device tensor")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
            raise FhsError(f"{name}: expected a contiguous {dtype} tensor of {n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def _need_ws(self):
        if self.workspace is None:
            raise FhsError("attach_workspace() first")

    def forward(self, x, vis):
        """vis (complex64, m) = Phi x (x float32 [ny][nx][L])."""
        import torch
        self._need_ws()
        _check(self._lib.fhs_nufft_forward(self._p, self._t(x, self.ny * self.nx * self.L, torch.float32, "x"),
                                           self._t(vis, self.m, torch.complex64, "vis"), _stream(x)))

    def adjoint(self, vis, x, scale=None, beta=0.0):
        """x = beta x + scale_l Re(Phi_l^dagger vis)."""
        import torch
        self._need_ws()
        sc = self._t(scale, self.L, torch.float64, "scale") if scale is not None else None
        _check(self._lib.fhs_nufft_adjoint(self._p, self._t(vis, self.m, torch.complex64, "vis"),
                                           self._t(x, self.ny * self.nx * self.L, torch.float32, "x"), sc,
                                           float(beta), _stream(x)))

    def dual_update(self, xcheck, x, v, y, U, eps, eta, n_sub, grad, residual=None):
        """fhs_data_dual_update (Alg. 2 data-fidelity lines)."""
        import torch
        self._need_ws()
        n = self.ny * self.nx * self.L
        res = self._t(residual, self.L, torch.float64, "residual") if residual is not None else None
        _check(self._lib.fhs_data_dual_update(
            self._p, self._t(xcheck, n, torch.float32, "xcheck"), self._t(x, n, torch.float32, "x"),
            self._t(v, self.m, torch.complex64, "v"), self._t(y, self.m, torch.complex64, "y"),
            self._t(U, self.m, torch.float32, "U"), self._t(eps, self.L, torch.float64, "eps"),
            self._t(eta, self.L, torch.float64, "eta"), int(n_sub), self._t(grad, n, torch.float32, "grad"), res,
            _stream(x)))
