"""Pins for the oracle's quadrature rule and basis (no GPU).

Quadrature (Sec. 3.1, eq. "Numerical integration"): Gauss--Hermite with N
nodes integrates x^k exactly against N(0,1) for k <= 2N-1, whose moments are
(k-1)!! for even k and 0 for odd k.  Two independent constructions must agree.
Basis (App. B, orthogonal form): orthonormal under N(0, I).
"""

import math

import numpy as np
import pytest

from oracle import basis, quadrature


def dfact(k):
    r = 1
    while k > 1:
        r *= k
        k -= 2
    return r


@pytest.mark.parametrize("n", [5, 12, 16, 24, 64])
def test_gauss_hermite_exact_on_polynomials(n):
    x, w = quadrature.gauss_hermite(n)
    assert abs(w.sum() - 1.0) < 1e-14
    for k in range(0, min(2 * n, 40)):
        exact = 0.0 if k % 2 else float(dfact(k - 1))
        got = np.sum(w * x ** k)
        scale = np.sum(w * np.abs(x) ** k)   # rounding scale of the sum
        assert abs(got - exact) <= 1e-13 * scale + 1e-15, (n, k, got, exact)


@pytest.mark.parametrize("n", [12, 16, 24])
def test_golub_welsch_matches_numpy_rule(n):
    x1, w1 = quadrature.gauss_hermite(n)
    x2, w2 = quadrature.golub_welsch(n)
    assert np.max(np.abs(x1 - x2)) < 1e-12
    assert np.max(np.abs(w1 - w2)) < 1e-14


def test_node_extent_matches_known_values():
    # largest probabilists' Gauss-Hermite nodes
    for n, xmax in [(12, 5.5009), (16, 6.6308), (24, 8.5078)]:
        x, _ = quadrature.gauss_hermite(n)
        assert abs(x.max() - xmax) < 1e-3


def test_basis_size_and_order():
    idx = basis.multi_indices(3)
    assert len(idx) == 35
    assert idx[:4] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    assert all(sum(e) <= 4 for e in idx)
    assert len(set(idx)) == 35
    assert basis.multi_indices(1) == [(0,), (1,), (2,), (3,), (4,)]


def test_hermite_recurrence_matches_numpy_hermite_e():
    x = np.linspace(-7, 7, 41)
    H = basis.hermite_e(8, x)
    for n in range(9):
        c = np.zeros(n + 1); c[n] = 1
        ref = np.polynomial.hermite_e.hermeval(x, c)
        assert np.allclose(H[n], ref, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("dim,n", [(1, 16), (3, 12), (3, 5)])
def test_basis_orthonormal_under_quadrature(dim, n):
    nodes, w = quadrature.tensor_rule(n, dim)
    Phi = basis.evaluate(nodes, dim)
    G = (Phi * w[:, None]).T @ Phi
    assert np.max(np.abs(G - np.eye(Phi.shape[1]))) < 1e-13


def test_lebesgue_weights_integrate_gaussian_density():
    # sum exp(logw~) * N(x;0,I) = 1 and a shifted/scaled Gaussian integrates to 1
    nodes, w = quadrature.tensor_rule(12, 3)
    lw = quadrature.lebesgue_log_weights(nodes, w)
    s = 1.1
    dens = np.exp(-0.5 * np.sum((nodes / s) ** 2, axis=1)) / ((2 * math.pi) ** 1.5 * s ** 3)
    assert abs(np.sum(np.exp(lw) * dens) - 1.0) < 1e-6
