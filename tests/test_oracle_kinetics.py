"""Pins for the oracle's collision, shock set-up and time step (no GPU).

* Rankine--Hugoniot ratios (eq. "RH condition") for gamma = 5/3, and the jump
  conserves mass, momentum and energy fluxes of the Euler equations.
* ES-BGK relaxation (App. A) conserves n, n v_x and total energy; the target
  has the stated covariance; a Maxwellian is its own target; Pr = 1 gives the
  Maxwellian (plain BGK).
* Workload closed forms (``mem_inputs``): Gaussian Hermite moments equal the
  oracle's Gaussian quadrature.
* Alg. 2 with LLF: a uniform equilibrium is stationary; the update is
  conservative (interior fluxes telescope) up to the boundary fluxes.
"""

import math

import numpy as np
import pytest

import mem_inputs
from oracle import gauge, kinetics


@pytest.mark.parametrize("mach,ratio,v2,tr", [
    (1.2, 1.2973, 1.1942, 1.1948), (3.0, 3.0, 1.2910, 3.6667),
    (4.0, 3.3684, 1.5331, 5.8633), (10.0, 3.8835, 3.3243, 32.1231)])
def test_rankine_hugoniot_table(mach, ratio, v2, tr):
    (n1, v1, T1), (n2, vv2, T2) = kinetics.rankine_hugoniot(mach)
    assert n2 == pytest.approx(ratio, abs=1e-4)
    assert vv2 == pytest.approx(v2, abs=1e-4)
    assert T2 == pytest.approx(tr, abs=1e-4)
    # Euler flux conservation across the jump (p = n T)
    assert n1 * v1 == pytest.approx(n2 * vv2, rel=1e-13)
    assert n1 * v1 ** 2 + n1 * T1 == pytest.approx(n2 * vv2 ** 2 + n2 * T2, rel=1e-13)
    assert n1 * v1 * (0.5 * v1 ** 2 + 2.5 * T1) == pytest.approx(
        n2 * vv2 * (0.5 * vv2 ** 2 + 2.5 * T2), rel=1e-13)
    # Mach number definition v = sqrt(gamma T) Ma upstream
    assert v1 == pytest.approx(math.sqrt(5.0 / 3.0) * mach, rel=1e-14)


def test_inputs_rh_matches_oracle_rh():
    (a1, b1, c1), (a2, b2, c2) = mem_inputs.rankine_hugoniot(np.array([2.5]))
    (d1, e1, f1), (d2, e2, f2) = kinetics.rankine_hugoniot(2.5)
    assert np.allclose([a2[0], b2[0], c2[0]], [d2, e2, f2], rtol=1e-14)


def test_inputs_gaussian_moments_match_quadrature():
    rng = np.random.default_rng(31)
    C = 5
    n = rng.uniform(0.5, 2, C); v = rng.normal(size=C)
    Txx = rng.uniform(0.5, 3, C); Trr = rng.uniform(0.5, 3, C)
    g = np.stack([rng.normal(size=C), rng.uniform(0.7, 1.5, C), rng.uniform(0.7, 1.5, C)], 1)
    a = mem_inputs.gaussian_moments(n, v, Txx, Trr, g)
    b = kinetics.gaussian_moments(n, v, Txx, Trr, g)
    assert np.max(np.abs(a - b)) < 1e-12 * max(1.0, np.max(np.abs(a)))


def test_mott_smith_targets_are_in_hermite_gauge():
    cells = mem_inputs.mott_smith_cells(16, config=2, replica=1)
    gH = gauge.hermite_gauge(cells["M"], cells["g"], 3)
    assert np.allclose(gH, cells["g"], rtol=1e-12)


def _nonequilibrium_state():
    cells = mem_inputs.mott_smith_cells(6, config=2, replica=2)
    return cells["M"], cells["g"]


def test_collision_conserves_mass_momentum_energy():
    M, g = _nonequilibrium_state()
    a = kinetics.macroscopic(M, g)
    M2 = kinetics.collision(M, g, h=0.05)
    b = kinetics.macroscopic(M2, g)
    assert np.allclose(a["n"], b["n"], rtol=1e-13)
    assert np.allclose(a["n"] * a["v"], b["n"] * b["v"], rtol=1e-12)
    ea = a["n"] * (0.5 * a["v"] ** 2 + 1.5 * a["T"])
    eb = b["n"] * (0.5 * b["v"] ** 2 + 1.5 * b["T"])
    assert np.allclose(ea, eb, rtol=1e-12)
    # stress relaxes: |P_xx - nT| shrinks
    assert np.all(np.abs(b["Pxx"] - b["n"] * b["T"]) < np.abs(a["Pxx"] - a["n"] * a["T"]))


def test_es_bgk_target_covariance_and_limits():
    M, g = _nonequilibrium_state()
    Pr = 2.0 / 3.0
    Mt, _ = kinetics.es_bgk_target(M, g, Pr)
    a, b = kinetics.macroscopic(M, g), kinetics.macroscopic(Mt, g)
    # target carries n, v, T and Sigma_xx = T/Pr + (1 - 1/Pr) P_xx/n
    assert np.allclose(b["n"], a["n"], rtol=1e-13)
    assert np.allclose(b["v"], a["v"], rtol=1e-12)
    assert np.allclose(b["T"], a["T"], rtol=1e-12)
    sxx = a["T"] / Pr + (1 - 1 / Pr) * a["Pxx"] / a["n"]
    assert np.allclose(b["Pxx"] / b["n"], sxx, rtol=1e-12)
    assert np.allclose(b["qx"], 0.0, atol=1e-10)
    # a Maxwellian is its own target (equilibrium is the fixed point)
    mac = a
    Mmx = kinetics.gaussian_moments(mac["n"], mac["v"], mac["T"], mac["T"], g)
    Mmt, _ = kinetics.es_bgk_target(Mmx, g, Pr)
    assert np.max(np.abs(Mmt - Mmx)) < 1e-12
    # Pr = 1: Maxwellian with the same n, v, T (plain BGK)
    M1, _ = kinetics.es_bgk_target(M, g, 1.0)
    assert np.max(np.abs(M1 - Mmx)) < 1e-12


def test_relaxation_time_maxwell_molecules():
    # tau = mu/(Pr n T) with mu = sqrt(2/pi) T  ->  h/tau = h Pr n / sqrt(2/pi)
    M, g = _nonequilibrium_state()
    Mt, n = kinetics.es_bgk_target(M, g, 2.0 / 3.0)
    h = 0.01
    M2 = kinetics.collision(M, g, h)
    r = h * (2.0 / 3.0) * n / math.sqrt(2.0 / math.pi)
    assert np.allclose(M2, (1 - r)[:, None] * M + r[:, None] * Mt, rtol=1e-13, atol=1e-14)


def test_uniform_equilibrium_is_stationary():
    s = kinetics.ShockSolver(1.0 + 1e-12, 16, -8.0, 8.0, 2.0, nodes_1d=8)
    # Mach -> 1: upstream == downstream, uniform Maxwellian everywhere
    M0 = s.M.copy()
    for _ in range(3):
        s.step()
    assert np.max(np.abs(s.M - M0)) < 1e-9


def test_fv_update_is_conservative():
    s = kinetics.ShockSolver(3.0, 24, -6.0, 6.0, 3.0, nodes_1d=8)
    from oracle import flux
    M, g = s.M, s.g
    beta = s.beta
    F = flux.fluxes(beta, g, s.nodes, s.Phi, s.logw)
    rho = flux.spectral_radius(beta, g, s.nodes, s.Phi, s.logw)
    dt = s.dt
    M2 = s._fv(M, F, rho, dt)
    # mass (M_0 is gauge invariant): change equals boundary flux difference
    MLg, FLg, rL, _, _ = s.ghost_left
    MRg, FRg, rR, _, _ = s.ghost_right
    TL = gauge.change_matrix(g[:1], s.ghost_left[3][None], 3)[0]
    TR = gauge.change_matrix(g[-1:], s.ghost_right[3][None], 3)[0]
    fL = 0.5 * ((TL @ FLg)[0] + F[0, 0]) + 0.5 * max(rL, rho[0]) * ((TL @ MLg)[0] - M[0, 0])
    fR = 0.5 * (F[-1, 0] + (TR @ FRg)[0]) + 0.5 * max(rho[-1], rR) * (M[-1, 0] - (TR @ MRg)[0])
    dm = np.sum(M2[:, 0] - M[:, 0]) * s.dx
    assert dm == pytest.approx(dt * (fL - fR), rel=1e-10, abs=1e-13)


def test_unrepresentable_cell_takes_its_maxwellian():
    """On a positive discrete measure E[phi_k] lies between min_p and max_p of
    phi_k over the nodes: a target above the maximum is certainly not
    representable.  Such a cell takes the Maxwellian of its gauge; a Maxwellian
    cell beside it solves to the Maxwellian as usual."""
    from oracle import maxent
    s = kinetics.ShockSolver(1.5, 8, -4.0, 4.0, 2.0, nodes_1d=8)
    M = np.zeros((2, 35))            # Hermite moments of n N(0, I) in its own gauge
    M[:, 0] = (1.3, 0.7)
    k4 = [i for i, e in enumerate(basis_indices()) if e == (4, 0, 0)][0]
    M[1, k4] = 1.5 * M[1, 0] * np.max(s.Phi[:, k4])     # beyond every node value
    beta = s._solve(M, maxent.maxwellian_beta(M, 3))
    assert s.maxwell_cells.tolist() == [False, True]
    assert np.allclose(beta[1], maxent.maxwellian_beta(M[1:], 3)[0])
    assert np.allclose(beta[0], maxent.maxwellian_beta(M[:1], 3)[0], atol=1e-9)


def basis_indices():
    from oracle import basis
    return [tuple(e) for e in basis.multi_indices(3)]
