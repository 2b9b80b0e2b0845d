"""Regularisation parameters and reweighting weights (oracle).

TEST INFRASTRUCTURE ONLY.

* eq. heuristic_fhs_sparsity:  mu_c = upsilon_c = sigma_bar_c (m_chi(L_c) + s_chi(L_c)),
  with m_chi, s_chi the mean and standard deviation of a chi distribution with
  L_c degrees of freedom;
* eq. heuristic_fhs_low_rank:  mu_bar_{c,q} = upsilon_bar_{c,q}
  = sigma_bar_c sqrt(N~_q L_c / J_{c,q}),  J_{c,q} = min(N~_q, L_c);
* eq. facet_hypersara_rank:    theta_bar_j = upsilon_bar / (s_j(D_q S~_q X) + upsilon_bar);
* eq. facet_hypersara_sparsity: theta_i = upsilon / (||[Psi^dagger X]_i||_2 + upsilon).
"""
import numpy as np
from scipy.special import gammaln

from . import sara
from .step import facet_matrix, subcube_channels


def chi_mean_std(k):
    """Mean sqrt(2) Gamma((k+1)/2) / Gamma(k/2) and std sqrt(k - mean^2) of chi_k."""
    m = np.sqrt(2.0) * np.exp(gammaln((k + 1) / 2.0) - gammaln(k / 2.0))
    return m, np.sqrt(k - m * m)


def mu_sparsity(sigma_bar, Lc):
    m, s = chi_mean_std(Lc)
    return sigma_bar * (m + s)


def mu_low_rank(sigma_bar, n_rows, Lc):
    return sigma_bar * np.sqrt(n_rows * Lc / min(n_rows, Lc))


def nuclear_weights(xprev, geom, upsilon_bar, C=1):
    """theta_bar[c][q]: (L_c,) weights from the singular values of D_q S~_q X_c^{(t)}."""
    L = xprev.shape[2]
    chans = subcube_channels(L, C)
    out = []
    for c in range(C):
        row = []
        for q, f in enumerate(geom.facets):
            s = np.linalg.svd(facet_matrix(xprev, f, chans[c]), compute_uv=False)
            row.append(upsilon_bar[c][q] / (s + upsilon_bar[c][q]))
        out.append(row)
    return out


def l21_weights(xprev, upsilon, levels=4, C=1):
    """theta[c]: (I,) weights from the row norms of Psi^dagger X_c^{(t)}."""
    L = xprev.shape[2]
    chans = subcube_channels(L, C)
    out = []
    for c in range(C):
        A = sara.flatten(sara.analysis(np.asarray(xprev, dtype=np.float64)[..., chans[c]], levels))
        r = np.linalg.norm(A, axis=1)
        out.append(upsilon[c] / (r + upsilon[c]))
    return out
