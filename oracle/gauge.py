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

import math

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


def _axis_projection(a, b, n=6):
    """t[c, k, l] = E_{z~N(0,1)}[p_k(a_c z + b_c) p_l(z)], p_k = He_k/sqrt(k!), k, l <= 4.

    One axis of the projection below, by an n-point Gauss--Hermite rule (exact:
    the integrand has degree <= 8)."""
    z, w = _quad.gauss_hermite(n)
    norm = np.sqrt([float(math.factorial(k)) for k in range(5)])
    P0 = _basis.hermite_e(4, z) / norm[:, None]                      # (5, n)
    Ps = _basis.hermite_e(4, a[:, None] * z[None, :] + b[:, None])   # (5, C, n)
    Ps = np.moveaxis(Ps, 0, 1) / norm[None, :, None]                 # (C, 5, n)
    return (Ps * w[None, None, :]) @ P0.T


def change_matrix(g_to, g_from, dim):
    """T(g_to, g_from): (C, K, K), by Gaussian projection.

    T_ij = E_{z~N(0,I)}[phi_i(a*z + b) phi_j(z)] over the tensor rule.  The
    basis and the rule are both tensor products, so the sum factorises into
    one projection per axis: T_(abc),(a'b'c') = t_x[a,a'] t_y[b,b'] t_z[c,c']."""
    g_to = np.atleast_2d(np.asarray(g_to, dtype=np.float64))
    g_from = np.atleast_2d(np.asarray(g_from, dtype=np.float64))
    a, b = _affine(g_to, g_from, dim)
    idx = np.asarray(_basis.multi_indices(dim))                      # (K, dim)
    T = None
    for d in range(dim):
        t = _axis_projection(a[:, d], b[:, d])                       # (C, 5, 5)
        f = t[:, idx[:, d][:, None], idx[:, d][None, :]]             # (C, K, K)
        T = f if T is None else T * f
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
