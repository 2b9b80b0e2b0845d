"""Outer reweighting loop (Alg. 1) around PDFB runs with the stopping rule of
Alg. 2 (oracle).

TEST INFRASTRUCTURE ONLY.

The spectral sub-cubes are independent sub-problems (Sec. 2.4.1, eq.
problem-split-subcube): Alg. 1 runs its reweighting loop inside "for c = 1 to
C", and Alg. 2 solves one spectral sub-problem with that sub-cube's own
iteration counter, relative variation and residual.  This oracle therefore
takes the sub-cubes one after the other, each on its own channels
(c, c + C, c + 2C, ... of the cube), its own duals, data, noise levels,
weights and thresholds:

* Alg. 2, loop condition for sub-cube c: iterate while p < P_min, or while
  p < P_max and either xi_c = ||X_c^(p+1) - X_c^(p)|| / ||X_c^(p)|| exceeds its
  bound or ||r_c|| exceeds res_factor ||eps_c|| (res_factor = 1.01 in the
  paper), with ||eps_c|| the l2 norm of the sub-cube's l2-ball radii.  With
  the identity as measurement operator the residual of iteration p is
  r_{c,l} = ||y_l - x_l|| for the iterate x entering that iteration, and
  ||r_c|| = sqrt(sum_{l in c} r_{c,l}^2).  Each PDFB run starts its
  extrapolated iterate at the run's input (Xcheck_c <- X_c).
* Alg. 1 for sub-cube c: t = 0, xi = +inf; while t < T and xi > xi_rw:
  weights from X_c^(t) (eqs. facet_hypersara_rank and
  facet_hypersara_sparsity), one PDFB run warm-started from
  (X_c^(t), P_c, W_c, v_c), xi = ||X_c^(t+1) - X_c^(t)|| / ||X_c^(t)||
  (+inf if X_c^(t) = 0), t <- t + 1.

Reading: the relative-variation update and the counter increment close each
pass of the while loop (the printed layout sets them after it), and t, xi
start afresh for every sub-cube.
"""
import numpy as np

from . import closure, heuristics
from .step import subcube_channels


def rel_var(x_new, x_old):
    n = np.linalg.norm(x_old)
    return np.linalg.norm(np.asarray(x_new, dtype=np.float64) - x_old) / n if n > 0 else np.inf


def pdfb_run(x, P, W, v, y, eps, theta, theta_bar, mu, mu_bar, geom, tau=0.33, zeta=1.0, kappa=1.0,
             p_min=10, p_max=2000, xi_tol=1e-5, res_factor=1.01):
    """Alg. 2 on ONE spectral sub-problem until its stopping rule holds.
    x, v, y: (ny, nx, L_c); P: [Q] facet duals; W: (I, L_c); eps: (L_c,);
    theta: (I,); theta_bar: [Q] (L_c,); mu: scalar; mu_bar: [Q].
    Returns (x, P, W, v, hist) with hist = list of (xi, ||r||) per iteration."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xc = x.copy()
    eps_norm = np.linalg.norm(eps)
    P, W, th, thb, mub = [P], [W], [theta], [theta_bar], [mu_bar]
    hist = []
    p, xi, res = 0, np.inf, np.linalg.norm(y - x)
    while p < p_min or (p < p_max and (xi > xi_tol or res > res_factor * eps_norm)):
        res = np.linalg.norm(y - x)
        x, xc, P, W, v, xiv = closure.pdfb_iteration(x, xc, P, W, v, y, eps, th, thb, [mu], mub, geom, C=1,
                                                     tau=tau, zeta=zeta, kappa=kappa)
        xi = float(xiv[0])
        hist.append((xi, res))
        p += 1
    return x, P[0], W[0], v, hist


def subcube_solve(x, P, W, v, y, eps, mu, mu_bar, upsilon, upsilon_bar, geom, levels=4, tau=0.33, zeta=1.0,
                  kappa=1.0, T=5, xi_rw=1e-5, **run):
    """Alg. 1's loop for ONE sub-cube (arrays as in `pdfb_run`; upsilon scalar,
    upsilon_bar [Q]).  Returns (x, P, W, v, theta, theta_bar, runs, xis)."""
    x = np.asarray(x, dtype=np.float64)
    t, xi = 0, np.inf
    runs, xis = [], []
    theta = theta_bar = None
    while t < T and xi > xi_rw:
        theta_bar = heuristics.nuclear_weights(x, geom, [upsilon_bar], C=1)[0]
        theta = heuristics.l21_weights(x, [upsilon], levels=levels, C=1)[0]
        x_new, P, W, v, hist = pdfb_run(x, P, W, v, y, eps, theta, theta_bar, mu, mu_bar, geom, tau=tau, zeta=zeta,
                                        kappa=kappa, **run)
        xi = rel_var(x_new, x)
        x = x_new
        runs.append(hist)
        xis.append(xi)
        t += 1
    return x, P, W, v, theta, theta_bar, runs, xis


def reweighting_solve(x, P, W, v, y, eps, mu, mu_bar, upsilon, upsilon_bar, geom, C=1, levels=4, tau=0.33,
                      zeta=1.0, kappa=1.0, T=5, xi_rw=1e-5, **run):
    """Alg. 1 over the C interleaved sub-cubes of the cube (x, v, y: (ny, nx,
    L); P[c][q]; W[c]; eps (L,); mu, upsilon [C]; mu_bar, upsilon_bar [C][Q]).
    Returns (x, P, W, v, theta, theta_bar, report) with report =
    dict(runs=[[hist per PDFB run] per sub-cube], xi=[[outer relative
    variation per run] per sub-cube]).  A sub-cube whose weights were never
    computed (T = 0) reports None weights."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    L = x.shape[2]
    P, W = [list(row) for row in P], list(W)
    theta, theta_bar = [None] * C, [None] * C
    runs, xis = [], []
    for c, ch in enumerate(subcube_channels(L, C)):
        xc, Pc, Wc, vc, th, thb, r, xs = subcube_solve(
            x[..., ch], P[c], W[c], v[..., ch], y[..., ch], eps[ch], mu[c], mu_bar[c], upsilon[c], upsilon_bar[c],
            geom, levels=levels, tau=tau, zeta=zeta, kappa=kappa, T=T, xi_rw=xi_rw, **run)
        x[..., ch], v[..., ch] = xc, vc
        P[c], W[c], theta[c], theta_bar[c] = Pc, Wc, th, thb
        runs.append(r)
        xis.append(xs)
    return x, P, W, v, theta, theta_bar, dict(runs=runs, xi=xis)
