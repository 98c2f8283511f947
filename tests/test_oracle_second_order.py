"""Pins of the oracle's second-order interface fluxes (Sec. 3.4, eqs. "The lax W"
and "The FLIC").

* the van Leer limiter against its defining formula (r + |r|) / (1 + |r|) and
  its symmetry phi(r) / r = phi(1 / r);
* FLIC with the limiter forced to zero is the local Lax--Friedrichs step, which
  the oracle computes by a separate cell-centred route;
* a smooth pulse between two equal ghost states: mass, momentum and energy are
  conserved to rounding by LW and FLIC;
* order of accuracy on the same smooth, collisionless problem: halving dx (and
  dt with it) divides the two-step Lax--Wendroff error by about four and the
  LLF error by about two.
"""

import math

import numpy as np
import pytest

from oracle import kinetics


@pytest.mark.parametrize("r", [-3.0, -0.5, 0.0, 0.25, 1.0, 2.0, 7.5])
def test_van_leer_matches_its_definition(r):
    b = 0.3
    phi = kinetics.van_leer(np.array([r * b]), np.array([b]))[0]
    assert phi == pytest.approx((r + abs(r)) / (1.0 + abs(r)), abs=1e-15)
    if r > 0:   # symmetric limiter
        inv = kinetics.van_leer(np.array([b]), np.array([r * b]))[0]
        assert phi / r == pytest.approx(inv, rel=1e-14)


def test_van_leer_limits():
    a = np.array([1.0, 1.0, -2.0, 0.0, 5.0])
    b = np.array([1.0, -1.0, -2.0, 3.0, 0.0])
    assert np.allclose(kinetics.van_leer(a, b), [1.0, 0.0, 1.0, 0.0, 0.0])


def _pulse(n_cells, scheme, collide=False, amp=0.2, half=3.0, v0=0.5, width=0.8):
    x = -half + (np.arange(n_cells) + 0.5) * (2 * half / n_cells)
    n = 1.0 + amp * np.exp(-(x / width) ** 2)
    M = np.zeros((n_cells, 35))
    g = np.zeros((n_cells, 3))
    for c in range(n_cells):
        Mc, gc = kinetics.maxwellian_state(n[c], v0, 1.0)
        M[c], g[c] = Mc[0], gc[0]
    return kinetics.FVSolver(M, g, 2 * half / n_cells, (1.0, v0, 1.0), (1.0, v0, 1.0),
                             scheme=scheme, collide=collide)


def _totals(s):
    m = kinetics.macroscopic(s.M, s.g)
    n, v, T = m["n"], m["v"], m["T"]
    return np.array([np.sum(n), np.sum(n * v), np.sum(n * (0.5 * v * v + 1.5 * T))]) * s.dx


def _run_to(s, t_end):
    while s.t < t_end - 1e-14:
        s.dt = min(s.dt, t_end - s.t)
        s.step()


def test_flic_with_zero_limiter_is_llf(monkeypatch):
    a = kinetics.ShockSolver(3.0, 40, -4.0, 4.0, 1.5, scheme="llf")
    monkeypatch.setattr(kinetics, "van_leer", lambda x, y: np.zeros(np.broadcast(x, y).shape))
    b = kinetics.ShockSolver(3.0, 40, -4.0, 4.0, 1.5, scheme="flic")
    for _ in range(3):
        da, db = a.step(), b.step()
        assert db == pytest.approx(da, rel=1e-12)
    scale = np.maximum(1.0, np.abs(a.M))
    assert np.max(np.abs(a.M - b.M) / scale) < 1e-11
    assert not np.any(b.lw_failed)


@pytest.mark.parametrize("scheme", ["lw", "flic"])
def test_second_order_steps_conserve(scheme):
    # narrow enough that the boundary cells equal the ghosts to rounding
    s = _pulse(32, scheme, collide=True, width=0.5)
    tot0 = _totals(s)
    for _ in range(4):
        s.step()
    rel = np.abs(_totals(s) - tot0) / np.abs(tot0)
    assert np.all(rel < 1e-11), rel


def _density_error(coarse, fine):
    """L1 distance of coarse cell densities from the fine run averaged in pairs
    (density is the zeroth moment in every gauge)."""
    nf = fine.M[:, 0].reshape(-1, 2).mean(axis=1)
    return np.sum(np.abs(coarse.M[:, 0] - nf)) * coarse.dx


@pytest.mark.parametrize("scheme, lo, hi", [("lw", 3.3, 5.0), ("llf", 1.5, 2.6)])
def test_order_of_accuracy_on_a_smooth_pulse(scheme, lo, hi):
    t_end = 0.25
    runs = []
    for N in (24, 48, 96):
        s = _pulse(N, scheme)
        _run_to(s, t_end)
        assert s.t == pytest.approx(t_end, abs=1e-13)
        runs.append(s)
    e1 = _density_error(runs[0], runs[1])
    e2 = _density_error(runs[1], runs[2])
    ratio = e1 / e2
    print(f"\n[{scheme}] errors {e1:.3e} {e2:.3e} ratio {ratio:.2f} (order {math.log2(ratio):.2f})")
    assert lo < ratio < hi


@pytest.mark.parametrize("scheme", ["lw", "flic"])
def test_uniform_equilibrium_is_stationary_second_order(scheme):
    # Mach -> 1: one Maxwellian everywhere; the half-step states equal the cells'
    s = kinetics.ShockSolver(1.0 + 1e-12, 12, -6.0, 6.0, 2.0, nodes_1d=8, scheme=scheme)
    M0 = s.M.copy()
    for _ in range(3):
        s.step()
    assert np.max(np.abs(s.M - M0)) < 1e-9
    assert not np.any(s.lw_failed)
