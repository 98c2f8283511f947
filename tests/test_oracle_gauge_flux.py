"""Pins for the oracle's gauge transforms, fluxes and characteristic speeds.

* T(g', g) (eq. "Change gauge M F") is checked as the polynomial identity
  phi(u_bar') = T phi(u_bar) at random points, and against the Hermite
  connection formula He_n(a x + b) = sum_k C(n,k) a^k He_k(x) h_{n-k}(b; a^2-1)
  written out here; T(g, g) = I and T(g, g') T(g', g) = I.
* Hermite gauge (eq. "The Hermite Gauge moments"): after the transform the
  first-, second-degree x moments and the radial second moment vanish.
* Gauge invariance of the model: transformed beta gives the same exponent up to
  a constant at any physical velocity, and the same physical moments.
* Flux of a Maxwellian equals the Euler fluxes; characteristic speeds of a
  Maxwellian in its Hermite gauge are w + s_x * (roots of He_1..He_5), the
  largest sqrt(5 + sqrt(10)); every speed lies within the node span.
"""

import math

import numpy as np
import pytest

import mem_inputs
from oracle import basis, flux, gauge, kinetics, maxent


def _h(m, b, c):
    return sum(math.comb(m, 2 * j) * max(1, math.prod(range(2 * j - 1, 0, -2)))
               * c ** j * b ** (m - 2 * j) for j in range(m // 2 + 1))


def _t1d(a, b):
    t = np.zeros((5, 5))
    for n in range(5):
        for k in range(n + 1):
            t[n, k] = (math.comb(n, k) * a ** k * _h(n - k, b, a * a - 1.0)
                       * math.sqrt(math.factorial(k) / math.factorial(n)))
    return t


def test_change_matrix_is_polynomial_identity():
    rng = np.random.default_rng(21)
    g1 = np.array([[0.7, 1.3, 0.8]]); g2 = np.array([[-0.4, 0.9, 1.6]])
    T = gauge.change_matrix(g2, g1, 3)[0]
    u = rng.normal(size=(50, 3)) * 2.0  # physical velocities
    ub1 = np.stack([(u[:, 0] - g1[0, 0]) / g1[0, 1], u[:, 1] / g1[0, 2], u[:, 2] / g1[0, 2]], 1)
    ub2 = np.stack([(u[:, 0] - g2[0, 0]) / g2[0, 1], u[:, 1] / g2[0, 2], u[:, 2] / g2[0, 2]], 1)
    lhs = basis.evaluate(ub2, 3)
    rhs = basis.evaluate(ub1, 3) @ T.T
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-9)


def test_change_matrix_matches_connection_formula():
    g1 = np.array([[0.3, 1.2, 0.7]]); g2 = np.array([[1.1, 0.8, 1.5]])
    T = gauge.change_matrix(g2, g1, 3)[0]
    ax, bx = g1[0, 1] / g2[0, 1], (g1[0, 0] - g2[0, 0]) / g2[0, 1]
    ar = g1[0, 2] / g2[0, 2]
    tx, tr = _t1d(ax, bx), _t1d(ar, 0.0)
    idx = basis.multi_indices(3)
    ref = np.array([[tx[a, a2] * tr[b, b2] * tr[c, c2] for (a2, b2, c2) in idx]
                    for (a, b, c) in idx])
    assert np.max(np.abs(T - ref)) < 1e-12


def test_change_matrix_identity_and_inverse():
    g1 = np.array([[0.3, 1.2, 0.7]]); g2 = np.array([[1.1, 0.8, 1.5]])
    assert np.max(np.abs(gauge.change_matrix(g1, g1, 3)[0] - np.eye(35))) < 1e-13
    P = gauge.change_matrix(g1, g2, 3)[0] @ gauge.change_matrix(g2, g1, 3)[0]
    assert np.max(np.abs(P - np.eye(35))) < 1e-12


def test_hermite_gauge_conditions_and_invariance(rule3):
    cells = mem_inputs.mott_smith_cells(8, config=2, replica=3)
    g0 = cells["g"].copy()
    g0[:, 0] += 0.7; g0[:, 1] *= 1.3; g0[:, 2] *= 0.8   # move to a non-Hermite gauge
    M0 = gauge.transform_moments(cells["M"], g0, cells["g"], 3)
    MH, _, gH = gauge.to_hermite_gauge(M0, None, g0, 3)
    i100, i200 = basis.index_of(3, (1, 0, 0)), basis.index_of(3, (2, 0, 0))
    i020, i002 = basis.index_of(3, (0, 2, 0)), basis.index_of(3, (0, 0, 2))
    assert np.max(np.abs(MH[:, i100])) < 1e-12
    assert np.max(np.abs(MH[:, i200])) < 1e-11
    assert np.max(np.abs(MH[:, i020] + MH[:, i002])) < 1e-11
    assert np.allclose(gH, cells["g"], rtol=1e-12)
    # physical quantities are gauge invariant
    a, b = kinetics.macroscopic(M0, g0), kinetics.macroscopic(MH, gH)
    for k in a:
        assert np.allclose(a[k], b[k], rtol=1e-11, atol=1e-11), k


def test_beta_transform_keeps_the_density(rule3):
    rng = np.random.default_rng(22)
    beta = mem_inputs.maxwellian_beta(1, 35, np.array([1.3]))
    beta[:, 1:] += 0.05 * rng.normal(size=(1, 34))
    g1 = np.array([[0.2, 1.1, 0.9]]); g2 = np.array([[0.9, 1.4, 1.2]])
    b2 = gauge.transform_beta(beta, g2, g1, 3)
    u = rng.normal(size=(40, 3))
    ub1 = np.stack([(u[:, 0] - g1[0, 0]) / g1[0, 1], u[:, 1] / g1[0, 2], u[:, 2] / g1[0, 2]], 1)
    ub2 = np.stack([(u[:, 0] - g2[0, 0]) / g2[0, 1], u[:, 1] / g2[0, 2], u[:, 2] / g2[0, 2]], 1)
    e1 = basis.evaluate(ub1, 3)[:, 1:] @ beta[0, 1:]
    e2 = basis.evaluate(ub2, 3)[:, 1:] @ b2[0, 1:]
    d = e1 - e2
    assert np.max(np.abs(d - d.mean())) < 1e-11  # equal up to the normaliser


def test_solution_invariance_across_gauges_converges_with_nodes():
    # (ii) moving the nodes with the gauge: agreement only to quadrature error,
    # shrinking as the rule is refined.  Target: moments of a decaying
    # exponential-family density (degree <= 3 perturbation, negative quartic
    # diagonal) integrated on a fine 30^3 rule, so a continuum solution exists.
    from oracle import quadrature
    rng = np.random.default_rng(5)
    bt = mem_inputs.maxwellian_beta(1, 35, np.array([1.2]))
    bt[:, 1:20] += 0.03 * rng.normal(size=(1, 19))
    for i, e in enumerate(basis.multi_indices(3)):
        if sum(e) == 4 and max(e) == 4:
            bt[:, i] = -0.04
    gA = np.array([[0.0, 1.0, 1.0]])
    nodes, w = quadrature.tensor_rule(30, 3)
    MA = maxent.model_moments(bt, basis.evaluate(nodes, 3),
                              quadrature.lebesgue_log_weights(nodes, w))
    gB = gA * np.array([1.0, 1.15, 0.9]) + np.array([0.2, 0.0, 0.0])
    MB = gauge.transform_moments(MA, gB, gA, 3)
    errs = []
    for nq in (8, 12, 16):
        nodes, w = quadrature.tensor_rule(nq, 3)
        Phi, lw = basis.evaluate(nodes, 3), quadrature.lebesgue_log_weights(nodes, w)
        bA = maxent.newton_solve(MA, mem_inputs.maxwellian_beta(1, 35, MA[:, 0]), Phi, lw)["beta"]
        bB = maxent.newton_solve(MB, gauge.transform_beta(bA, gB, gA, 3), Phi, lw)["beta"]
        errs.append(np.max(np.abs(gauge.transform_beta(bB, gA, gB, 3) - bA)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-5


def test_maxwellian_flux_is_euler_flux(rule3):
    for (n, v, T) in [(1.0, 3.873, 1.0), (3.0, 1.291, 3.6667), (0.7, -0.5, 2.0)]:
        M, g = kinetics.maxwellian_state(n, v, T)
        beta = maxent.maxwellian_beta(M, 3)
        F = flux.fluxes(beta, g, rule3["nodes"], rule3["Phi"], rule3["logw"])
        mac = kinetics.macroscopic(F, g)   # F is linear in f: reuse the monomial map
        # mass flux n v ; momentum flux n v^2 + n T ; energy flux n v (v^2/2 + 5T/2)
        assert F[0, 0] == pytest.approx(n * v, rel=1e-13)
        s = g[0, 1]
        c1 = gauge.monomial_coefficients((1, 0, 0), 3)
        c2 = gauge.monomial_coefficients((2, 0, 0), 3)
        cr = gauge.monomial_coefficients((0, 2, 0), 3) + gauge.monomial_coefficients((0, 0, 2), 3)
        Ex = F[0] @ c1; Exx = F[0] @ c2; Err = F[0] @ cr
        mom = v * F[0, 0] + s * Ex
        energy = 0.5 * (v * v * F[0, 0] + 2 * v * s * Ex + s * s * Exx + s * s * Err)
        assert mom == pytest.approx(n * v * v + n * T, rel=1e-12)
        assert energy == pytest.approx(n * v * (0.5 * v * v + 2.5 * T), rel=1e-12)
        del mac


def test_maxwellian_characteristic_speeds(rule3):
    M, g = kinetics.maxwellian_state(2.0, 1.5, 3.0)
    beta = maxent.maxwellian_beta(M, 3)
    lo, hi = flux.char_speeds(beta, g, rule3["nodes"], rule3["Phi"], rule3["logw"])
    mu = math.sqrt(5 + math.sqrt(10))
    assert hi[0] == pytest.approx(1.5 + math.sqrt(3.0) * mu, rel=1e-12)
    assert lo[0] == pytest.approx(1.5 - math.sqrt(3.0) * mu, rel=1e-12)


def test_characteristic_speeds_within_node_span(rule3):
    cells = mem_inputs.mott_smith_cells(4, config=2, replica=5)
    out = maxent.newton_solve(cells["M"], mem_inputs.maxwellian_beta(4, 35, cells["M"][:, 0]),
                              rule3["Phi"], rule3["logw"])
    lo, hi = flux.char_speeds(out["beta"], cells["g"], rule3["nodes"], rule3["Phi"], rule3["logw"])
    umax = np.max(np.abs(rule3["nodes"][:, 0]))
    g = cells["g"]
    assert np.all(hi <= g[:, 0] + g[:, 1] * umax + 1e-9)
    assert np.all(lo >= g[:, 0] - g[:, 1] * umax - 1e-9)
    assert np.all(hi > lo)


def test_speeds_take_the_node_span_bound_when_B_is_singular(rule3):
    # beta that puts essentially all mass on one node: B = E[phi phi^T] has rank 1
    # in FP64, the eigenvalues are undefined and the speeds take the bound
    # |mu| <= max_p |u_x,p| that every eigenvalue of the pencil obeys
    beta = np.zeros((1, 35))
    beta[0, 0] = 1.0
    beta[0, 1] = 400.0           # exponent 400 u_x: the largest-u_x nodes dominate
    g = np.array([[0.5, 2.0, 1.0]])
    lo, hi = flux.char_speeds(beta, g, rule3["nodes"], rule3["Phi"], rule3["logw"])
    umax = np.max(np.abs(rule3["nodes"][:, 0]))
    assert hi[0] == pytest.approx(0.5 + 2.0 * umax, rel=1e-12)
    assert lo[0] == pytest.approx(0.5 - 2.0 * umax, rel=1e-12)
