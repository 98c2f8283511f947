"""Gauge transformations for the oracle (test infrastructure only).

Gauge parameters (Sec. 3.3, eq. "Sufficient 35 ortho"): g = (w, s) in 1D and
g = (w_x, s_x, s_r) in 3D, with gauge coordinates
u_bar = ((u_x - w_x)/s_x, u_y/s_r, u_z/s_r).

* Hermite gauge (eqs. "The Hermite Gauge moments", "Hermite parameters"):
  w_H = E[u_x], s_{H,x}^2 = Var[u_x], s_{H,r}^2 = E[u_y^2 + u_z^2]/2.  The
  expectations of the needed monomials of u_bar are obtained from the moments
  by expanding each monomial in the orthonormal basis, with coefficients found
  by Gaussian projection (not by a hand-derived formula).
* Change of gauge T(g', g) (eq. "Change gauge M F"): phi(u_bar') = T phi(u_bar)
  as polynomials, u_bar' = a*u_bar + b per axis.  Built here by numerical
  projection T_ij = E_{z~N(0,I)}[phi_i(a*z + b) phi_j(z)], exact with 6 nodes
  per axis because the integrand has degree <= 8.
* M(g') = T(g', g) M(g); alpha(g') = T(g, g')^T alpha(g) (same equation), and
  beta'_i = alpha'_i for i >= 1 (eq. "form transformation"); beta'_0 = n.
"""

import numpy as np

from . import basis as _basis
from . import quadrature as _quad


def _proj_rule(dim, n=6):
    return _quad.tensor_rule(n, dim)


def monomial_coefficients(expo, dim):
    """c with prod_d u_d^{expo_d} = sum_i c_i phi_i(u) (degree <= 4)."""
    z, w = _proj_rule(dim)
    Phi = _basis.evaluate(z, dim)
    mono = np.prod(z ** np.asarray(expo)[None, :], axis=1)
    return (w * mono) @ Phi


def gauge_expectations(M, dim):
    """E_f[u_bar monomials] needed by the Hermite gauge, from moments M (C, K)."""
    n = M[:, 0]
    out = {}
    if dim == 1:
        keys = {"x": (1,), "xx": (2,)}
    else:
        keys = {"x": (1, 0, 0), "xx": (2, 0, 0), "yy": (0, 2, 0), "zz": (0, 0, 2)}
    for k, e in keys.items():
        out[k] = (M @ monomial_coefficients(e, dim)) / n
    return out


def hermite_gauge(M, g, dim):
    """Hermite gauge parameters g_H computed from moments M in gauge g."""
    M = np.asarray(M, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    ex = gauge_expectations(M, dim)
    gH = np.empty_like(g)
    gH[:, 0] = g[:, 0] + g[:, 1] * ex["x"]
    gH[:, 1] = g[:, 1] * np.sqrt(ex["xx"] - ex["x"] ** 2)
    if dim == 3:
        gH[:, 2] = g[:, 2] * np.sqrt(0.5 * (ex["yy"] + ex["zz"]))
    return gH


def _affine(g_to, g_from, dim):
    """u_bar(g_to) = a * u_bar(g_from) + b, per axis."""
    a = np.empty((g_to.shape[0], dim))
    b = np.zeros((g_to.shape[0], dim))
    a[:, 0] = g_from[:, 1] / g_to[:, 1]
    b[:, 0] = (g_from[:, 0] - g_to[:, 0]) / g_to[:, 1]
    if dim == 3:
        a[:, 1] = g_from[:, 2] / g_to[:, 2]
        a[:, 2] = a[:, 1]
    return a, b


def change_matrix(g_to, g_from, dim):
    """T(g_to, g_from): (C, K, K), by Gaussian projection."""
    g_to = np.atleast_2d(np.asarray(g_to, dtype=np.float64))
    g_from = np.atleast_2d(np.asarray(g_from, dtype=np.float64))
    z, w = _proj_rule(dim)
    Phi = _basis.evaluate(z, dim)
    a, b = _affine(g_to, g_from, dim)
    C = a.shape[0]
    K = Phi.shape[1]
    T = np.empty((C, K, K))
    for c in range(C):
        Phi_s = _basis.evaluate(z * a[c][None, :] + b[c][None, :], dim)
        T[c] = (Phi_s * w[:, None]).T @ Phi
    return T


def transform_moments(M, g_to, g_from, dim):
    T = change_matrix(g_to, g_from, dim)
    return np.einsum("cij,cj->ci", T, M)


def transform_beta(beta, g_to, g_from, dim):
    """beta in gauge g_from -> beta in gauge g_to (beta_0 = n kept)."""
    Tinv = change_matrix(g_from, g_to, dim)  # T(g, g')
    alpha = np.array(beta, dtype=np.float64, copy=True)
    alpha[:, 0] = 0.0  # alpha_0 only shifts the normalisation
    out = np.einsum("cji,cj->ci", Tinv, alpha)
    out[:, 0] = beta[:, 0]
    return out


def to_hermite_gauge(M, beta, g, dim):
    """ComputeGaugeParameters + GaugeTransformation of Alg. 2 (Step)."""
    gH = hermite_gauge(M, g, dim)
    MH = transform_moments(M, gH, g, dim)
    bH = None if beta is None else transform_beta(beta, gH, g, dim)
    return MH, bH, gH
