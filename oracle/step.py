"""One facet-wise regularization step of Algorithm 2 (oracle).

TEST INFRASTRUCTURE ONLY.

For every spectral sub-cube c and spatial facet q (Algorithm 2, facet loop):

  nuclear dual update (prox of Table 1):
      P_{c,q} <- (I - prox_{zeta^-1 mu_bar_{c,q} ||.||_{*,theta_bar_{c,q}}})(P_{c,q} + D_q S~_q X_c)
      with thresholds t_j = (mu_bar_{c,q} / zeta) theta_bar_{c,q,j};
      then P~_{c,q} = D_q P_{c,q} (facet back-projection; the printed
      "D_q^dagger P_c" is read as D_q P_{c,q}, D_q being real diagonal).

  l21 dual update (row shrink of Table 1):
      W_{c,q} <- (I - prox_{kappa^-1 mu_c ||.||_{2,1,theta_{c,q}}})(W_{c,q} + Psi_q^dagger S_q X_c)
      then W~_{c,q} = Psi_q W_{c,q} (facet synthesis).

  facet part of the aggregation:
      A_c = sum_q zeta S~_q^T P~_{c,q} + kappa S_q^T W~_{c,q}.

The faceted wavelet transform is exactly the global one (Sec. 2.4.2), so the
l21 update is computed here on the global transform; `sara.faceted_*` provide
the explicit faceted form that the tests pin against it.

facet_prox_step_select is the randomized form (Sec. 3.2): only a random
subset of the facets update their duals at an iteration, the draw being an
input.

Spectral sub-cubes (Sec. 2.4.1) are channel-interleaved: sub-cube c holds the
channels c, c + C, c + 2C, ... of the cube.

Data layout: X is (ny, nx, L); P[c][q] is (ny~_q, nx~_q, L_c); W[c] is (I, L_c)
in the coefficient order of `sara.flatten`; theta[c] is (I,); theta_bar[c][q]
is (L_c,) (ascending); mu is (C,); mu_bar is (C, Q).  Inputs are promoted to
float64 and every operation runs in float64.
"""
import numpy as np

from . import prox, sara


def subcube_channels(L, C):
    """Channel indices of each interleaved sub-cube."""
    return [list(range(c, L, C)) for c in range(C)]


def facet_matrix(xcheck, f, chans):
    """D_q S~_q X_c as an (N~_q, L_c) matrix (rows = pixels in row-major order)."""
    (y0, y1), (x0, x1) = f.nuc_window
    xs = np.asarray(xcheck, dtype=np.float64)[y0:y1, x0:x1][..., chans]
    return (f.window()[..., None] * xs).reshape(-1, len(chans))


def nuclear_dual_update(xcheck, P, theta_bar, mu_bar, zeta, geom, C=1):
    """Returns (P_new, G_nuc) with G_nuc = zeta sum_q S~_q^T D_q P_new_{c,q}."""
    ny, nx, L = xcheck.shape
    chans = subcube_channels(L, C)
    G = np.zeros((ny, nx, L))
    P_new = []
    for c in range(C):
        row = []
        for q, f in enumerate(geom.facets):
            shape = f.nuc_shape + (len(chans[c]),)
            Z = np.asarray(P[c][q], dtype=np.float64).reshape(-1, len(chans[c])) \
                + facet_matrix(xcheck, f, chans[c])
            t = (mu_bar[c][q] / zeta) * np.asarray(theta_bar[c][q], dtype=np.float64)
            Pn = prox.weighted_svt_complement(Z, t).reshape(shape)
            row.append(Pn)
            (y0, y1), (x0, x1) = f.nuc_window
            G[y0:y1, x0:x1][..., chans[c]] += zeta * f.window()[..., None] * Pn
        P_new.append(row)
    return P_new, G


def l21_dual_update(xcheck, W, theta, mu, kappa, levels=4, C=1):
    """Returns (W_new, G_l21) with G_l21 = kappa Psi W_new."""
    ny, nx, L = xcheck.shape
    chans = subcube_channels(L, C)
    G = np.zeros((ny, nx, L))
    W_new = []
    for c in range(C):
        A = sara.flatten(sara.analysis(np.asarray(xcheck, dtype=np.float64)[..., chans[c]], levels))
        U = np.asarray(W[c], dtype=np.float64) + A
        a = (mu[c] / kappa) * np.asarray(theta[c], dtype=np.float64)
        Wn = prox.l21_prox_complement(U, a)
        W_new.append(Wn)
        G[..., chans[c]] += kappa * sara.synthesis(sara.unflatten(Wn, ny, nx, levels), ny, nx, levels)
    return W_new, G


def facet_prox_step(xcheck, P, W, theta, theta_bar, mu, mu_bar, zeta, kappa, geom, C=1):
    """Both dual updates and the gather: returns (P_new, W_new, G)."""
    P_new, Gn = nuclear_dual_update(xcheck, P, theta_bar, mu_bar, zeta, geom, C)
    W_new, Gs = l21_dual_update(xcheck, W, theta, mu, kappa, geom.levels, C)
    return P_new, W_new, Gn + Gs


def facet_prox_step_select(xcheck, P, W, theta, theta_bar, mu, mu_bar, zeta, kappa, geom, select, C=1):
    """Randomized form of the facet step (Sec. 3.2, random selection of the
    facet dual variables updated at an iteration): only the facets (c, q) with
    select[c][q] true update their duals; the others keep them.  The facet
    duals of (c, q) are P_{c,q} and the l21 dual W_{c,q}, i.e. the coefficient
    rows facet q owns in every band (Sec. 2.4.2).  The aggregation sums the
    contributions of every facet's current duals.

    select: (C, Q) booleans (the random draw is an input).  Returns
    (P_new, W_new, G) in the layouts of facet_prox_step.
    """
    ny, nx, L = xcheck.shape
    chans = subcube_channels(L, C)
    levels = geom.levels
    P_new = []
    for c in range(C):
        row = []
        for q, f in enumerate(geom.facets):
            if select[c][q]:
                Lc = len(chans[c])
                Z = np.asarray(P[c][q], dtype=np.float64).reshape(-1, Lc) + facet_matrix(xcheck, f, chans[c])
                t = (mu_bar[c][q] / zeta) * np.asarray(theta_bar[c][q], dtype=np.float64)
                row.append(prox.weighted_svt_complement(Z, t).reshape(f.nuc_shape + (Lc,)))
            else:
                row.append(np.array(P[c][q], dtype=np.float64))
        P_new.append(row)
    W_new = []
    for c in range(C):
        # the update of every row, kept where the owning facet is selected
        A = sara.flatten(sara.analysis(np.asarray(xcheck, dtype=np.float64)[..., chans[c]], levels))
        U = np.asarray(W[c], dtype=np.float64) + A
        upd = sara.unflatten(prox.l21_prox_complement(U, (mu[c] / kappa) * np.asarray(theta[c], dtype=np.float64)),
                             ny, nx, levels)
        out = sara.unflatten(np.array(W[c], dtype=np.float64), ny, nx, levels)
        for q, f in enumerate(geom.facets):
            if not select[c][q]:
                continue
            for k, ((r0, r1), (c0, c1)) in enumerate(geom.owned_rects(f)):
                out[k][r0:r1, c0:c1] = upd[k][r0:r1, c0:c1]
        W_new.append(sara.flatten(out))
    G = np.zeros((ny, nx, L))
    for c in range(C):
        for q, f in enumerate(geom.facets):
            (y0, y1), (x0, x1) = f.nuc_window
            G[y0:y1, x0:x1][..., chans[c]] += zeta * f.window()[..., None] * P_new[c][q]
        G[..., chans[c]] += kappa * sara.synthesis(sara.unflatten(W_new[c], ny, nx, levels), ny, nx, levels)
    return P_new, W_new, G
