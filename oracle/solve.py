"""Outer reweighting loop (Alg. 1) around PDFB runs with the stopping rule of
Alg. 2 (oracle).

TEST INFRASTRUCTURE ONLY.

* Alg. 2, loop condition: iterate while p < P_min, or while p < P_max and
  either the relative variation xi of the iterate exceeds its bound or the
  data residual ||r|| exceeds res_factor ||eps|| (res_factor = 1.01 in the
  paper).  With the identity as measurement operator the residual of
  iteration p is r_l = ||y_l - x_l|| for the iterate x entering that
  iteration, and ||r|| = sqrt(sum_l r_l^2).  Each PDFB run starts its
  extrapolated iterate at the run's input (Xcheck <- X).
* Alg. 1: t = 0, xi = +inf; while t < T and xi > xi_rw: weights from X^(t)
  (eqs. facet_hypersara_rank and facet_hypersara_sparsity), one PDFB run
  warm-started from (X^(t), P, W, v), xi = ||X^(t+1) - X^(t)|| / ||X^(t)||
  (+inf if X^(t) = 0), t <- t + 1.

Readings: the relative-variation update and the counter increment close
each pass of the while loop (the printed layout sets them after it); all
spectral sub-cubes advance together and the criteria are taken over the
whole cube (for one sub-cube this is the algorithm as printed).
"""
import numpy as np

from . import closure, heuristics


def rel_var(x_new, x_old):
    n = np.linalg.norm(x_old)
    return np.linalg.norm(np.asarray(x_new, dtype=np.float64) - x_old) / n if n > 0 else np.inf


def pdfb_run(x, P, W, v, y, eps, theta, theta_bar, mu, mu_bar, geom, C=1, tau=0.33, zeta=1.0, kappa=1.0,
             p_min=10, p_max=2000, xi_tol=1e-5, res_factor=1.01):
    """Alg. 2 until its stopping rule holds.  Returns (x, P, W, v, hist) with
    hist = list of (xi, ||r||) per iteration."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xc = x.copy()
    eps_norm = np.linalg.norm(eps)
    hist = []
    p, xi, res = 0, np.inf, np.linalg.norm(y - x)
    while p < p_min or (p < p_max and (xi > xi_tol or res > res_factor * eps_norm)):
        res = np.linalg.norm(y - x)
        x, xc, P, W, v, xi = closure.pdfb_iteration(x, xc, P, W, v, y, eps, theta, theta_bar, mu, mu_bar, geom,
                                                    C=C, tau=tau, zeta=zeta, kappa=kappa)
        hist.append((xi, res))
        p += 1
    return x, P, W, v, hist


def reweighting_solve(x, P, W, v, y, eps, mu, mu_bar, upsilon, upsilon_bar, geom, C=1, levels=4, tau=0.33,
                      zeta=1.0, kappa=1.0, T=5, xi_rw=1e-5, **run):
    """Alg. 1.  upsilon [C], upsilon_bar [C][Q].  Returns (x, P, W, v, theta,
    theta_bar, report) with report = dict(runs=[hist per PDFB run],
    xi=[outer relative variation per run])."""
    x = np.asarray(x, dtype=np.float64)
    t, xi = 0, np.inf
    runs, xis = [], []
    theta = theta_bar = None
    while t < T and xi > xi_rw:
        theta_bar = heuristics.nuclear_weights(x, geom, upsilon_bar, C=C)
        theta = heuristics.l21_weights(x, upsilon, levels=levels, C=C)
        x_new, P, W, v, hist = pdfb_run(x, P, W, v, y, eps, theta, theta_bar, mu, mu_bar, geom, C=C, tau=tau,
                                        zeta=zeta, kappa=kappa, **run)
        xi = rel_var(x_new, x)
        x = x_new
        runs.append(hist)
        xis.append(xi)
        t += 1
    return x, P, W, v, theta, theta_bar, dict(runs=runs, xi=xis)
