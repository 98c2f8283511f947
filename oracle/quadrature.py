"""Quadrature rules for the oracle (test infrastructure only).

The paper integrates over molecular velocity with a fixed rule
sum_p w_p f(u_p) (Sec. 3.1, eq. "Numerical integration").  Here the nodes are
tensor Gauss--Hermite nodes of the standard normal fixed in gauge coordinates.
To integrate against Lebesgue measure, the log weights carry the Gaussian
density back: log w~_p = log w_p + |u_p|^2/2 + (d/2) log(2 pi).

Two independent constructions of the 1D rule are provided so that tests can
pin one against the other: NumPy's ``hermegauss`` and a Golub--Welsch
eigen-solve of the Jacobi matrix of the probabilists' Hermite polynomials.
"""

import math

import numpy as np


def gauss_hermite(n):
    """1D probabilists' Gauss--Hermite rule for N(0,1), weights summing to 1."""
    x, w = np.polynomial.hermite_e.hermegauss(n)
    w = w / math.sqrt(2.0 * math.pi)
    return x.astype(np.float64), w.astype(np.float64)


def golub_welsch(n):
    """Same rule from the symmetric tridiagonal Jacobi matrix.

    The monic He_k satisfy x He_k = He_{k+1} + k He_{k-1}, so the Jacobi
    matrix has zero diagonal and off-diagonal sqrt(k).  Nodes are its
    eigenvalues; weights are the squared first components of the normalised
    eigenvectors (total mass 1 for a probability measure).
    """
    off = np.sqrt(np.arange(1, n, dtype=np.float64))
    J = np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(J)
    w = V[0, :] ** 2
    return x, w


def tensor_rule(n, dim):
    """Tensor-product rule: nodes (Q, dim), weights (Q,), Q = n**dim.

    Node ordering: the last axis varies fastest.
    """
    x, w = gauss_hermite(n)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    wgrids = np.meshgrid(*([w] * dim), indexing="ij")
    nodes = np.stack([g.reshape(-1) for g in grids], axis=1)
    weights = np.prod(np.stack([g.reshape(-1) for g in wgrids], axis=1), axis=1)
    return nodes, weights


def lebesgue_log_weights(nodes, weights):
    """log w~_p such that sum_p exp(log w~_p) g(u_p) ~ integral g(u) du."""
    dim = nodes.shape[1]
    return (np.log(weights) + 0.5 * np.sum(nodes ** 2, axis=1)
            + 0.5 * dim * math.log(2.0 * math.pi))
