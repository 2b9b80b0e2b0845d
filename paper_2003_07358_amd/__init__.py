"""Faceted HyperSARA facet-wise regularization step (arXiv:2003.07358) on AMD
Instinct MI355X: the nuclear-norm and l21 dual updates of every spatio-spectral
facet and their gather into the primal gradient, as HIP kernels for gfx950
behind the C ABI of include/fhs.h.  This package is the thin Python binding.
"""
from .binding import DataPlan, FhsError, Plan, chi_mean_std, filter_taps, lib, library_path  # noqa: F401
