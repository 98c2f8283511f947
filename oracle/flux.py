"""Moment fluxes and characteristic speeds (oracle, test infrastructure only).

* Flux (eq. "The ME equation", flux line): F_i = int u_x phi_i(u_bar) f du.
  With u_x = w + s_x u_bar_x and the quadrature in gauge coordinates,
  F_i = n sum_p sigma_p (w + s_x u_bar_{x,p}) phi_i(u_bar_p), n = beta_0.
* Characteristic speeds for local Lax--Friedrichs (eq. "The lax F"): the
  eigenvalues of dF/dM.  With f = exp(alpha . phi), dM/dalpha = B and
  dF/dalpha = C where B = sum w f phi phi^T and C = sum w f u_x phi phi^T, so
  the eigenvalues solve C v = lambda B v.  In gauge coordinates
  lambda = w + s_x mu with mu the generalized eigenvalues of
  (E_sigma[u_bar_x phi phi^T], E_sigma[phi phi^T]); solved with LAPACK.
"""

import numpy as np
import scipy.linalg

from . import maxent as _maxent


def fluxes(beta, g, nodes, Phi, logw):
    beta = np.asarray(beta, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    sig = _maxent.sigma(beta, Phi, logw)
    ux = nodes[:, 0]
    E = sig @ Phi
    Ex = (sig * ux[None, :]) @ Phi
    n = beta[:, 0]
    return n[:, None] * (g[:, :1] * E + g[:, 1:2] * Ex)


def char_speeds(beta, g, nodes, Phi, logw):
    """(lambda_min, lambda_max) per cell, physical units.

    Where B is not positive definite in FP64 (sigma concentrated on too few
    nodes) the eigenvalues are undefined; the cell then takes the bound
    |mu| <= max_p |u_x,p| that every eigenvalue of the pencil obeys, as the GPU
    path does (its MEM_ST_LAMBDA_FAIL)."""
    beta = np.asarray(beta, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    sig = _maxent.sigma(beta, Phi, logw)
    ux = nodes[:, 0]
    C = beta.shape[0]
    lo = np.empty(C)
    hi = np.empty(C)
    # E_sigma[phi phi^T] and E_sigma[u_bar_x phi phi^T], direct weighted sums
    Bs = _maxent.second_moments(sig, Phi)
    Cs = _maxent.second_moments(sig * ux[None, :], Phi)
    for c in range(C):
        B, Cx = Bs[c], Cs[c]
        try:
            mu = scipy.linalg.eigh(Cx, B, eigvals_only=True)
            m0, m1 = mu[0], mu[-1]
        except np.linalg.LinAlgError:
            m1 = np.max(np.abs(ux))
            m0 = -m1
        lo[c] = g[c, 0] + g[c, 1] * m0
        hi[c] = g[c, 0] + g[c, 1] * m1
    return lo, hi


def spectral_radius(beta, g, nodes, Phi, logw):
    lo, hi = char_speeds(beta, g, nodes, Phi, logw)
    return np.maximum(np.abs(lo), np.abs(hi))
