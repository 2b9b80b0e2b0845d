"""Rest of one PDFB iteration around the facet step (oracle).

TEST INFRASTRUCTURE ONLY.

The measurement operator is out of scope, so the data-fidelity block uses
the identity as a stand-in (denoising: y = X_true + noise), with the paper's
l2-ball constraint per channel and U = I, eta = 1:

* data dual (Alg. 2, data-fidelity dual update with Phi = I):
      v <- (I - proj_{B(y, eps)})(v + Xcheck),
  proj_{B(y, eps)}(z) = y + (z - y) / max(||z - y|| / eps, 1)   (Table 1);
* aggregation (aggregation): A = G + v, G the facet part;
* primal update (primal update) and extrapolation:
      X+ = max(0, X - tau A)  (projection onto the non-negative orthant, Table 1),
      Xcheck = 2 X+ - X;
* relative variation of each spectral sub-problem (Alg. 2 solves every
  sub-cube c on its own): xi_c = ||X+_c - X_c||_F / ||X_c||_F over the
  channels of sub-cube c (+inf if X_c = 0).

eps_l^2 = sigma_l^2 (M_l + 2 sqrt(M_l)) with M_l = N measurements per channel
(Sec. 2.2, noise statistics of the l2 ball).
"""
import numpy as np

from . import step


def l2_ball_radius(sigma, n):
    return np.sqrt(sigma ** 2 * (n + 2.0 * np.sqrt(n)))


def project_l2_ball(z, y, eps):
    """Per-channel projection of z onto B(y, eps); arrays (ny, nx, L), eps (L,)."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = z - y
    nrm = np.sqrt(np.sum(d * d, axis=(0, 1)))
    return y + d / np.maximum(nrm / np.asarray(eps, dtype=np.float64), 1.0)


def data_dual_update(v, xcheck, y, eps):
    z = np.asarray(v, dtype=np.float64) + np.asarray(xcheck, dtype=np.float64)
    return z - project_l2_ball(z, y, eps)


def relative_variation(x_new, x_old, C=1):
    """(C,) array: ||x_new_c - x_old_c||_F / ||x_old_c||_F per interleaved
    sub-cube c (channels c, c + C, ...), +inf where x_old_c = 0."""
    x_new = np.asarray(x_new, dtype=np.float64)
    x_old = np.asarray(x_old, dtype=np.float64)
    out = np.empty(C)
    for c in range(C):
        n = np.linalg.norm(x_old[..., c::C])
        out[c] = np.linalg.norm(x_new[..., c::C] - x_old[..., c::C]) / n if n > 0 else np.inf
    return out


def primal_update(x, grad, v, tau, C=1):
    """Returns (X+, Xcheck, xi) with xi the (C,) relative variations."""
    x = np.asarray(x, dtype=np.float64)
    xn = np.maximum(0.0, x - tau * (np.asarray(grad, dtype=np.float64) + np.asarray(v, dtype=np.float64)))
    return xn, 2.0 * xn - x, relative_variation(xn, x, C)


def pdfb_iteration(x, xcheck, P, W, v, y, eps, theta, theta_bar, mu, mu_bar, geom, C=1, tau=0.33, zeta=1.0,
                   kappa=1.0):
    """One iteration of Algorithm 2 with the identity data term, every
    sub-cube at once.  Returns (x, xcheck, P, W, v, xi), xi of shape (C,)."""
    P, W, G = step.facet_prox_step(xcheck, P, W, theta, theta_bar, mu, mu_bar, zeta, kappa, geom, C=C)
    v = data_dual_update(v, xcheck, y, eps)
    x, xcheck, xi = primal_update(x, G, v, tau, C)
    return x, xcheck, P, W, v, xi
