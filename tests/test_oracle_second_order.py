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
  LLF error by about two;
* with the MaxEnt closure replaced by a linear map F = A M (all cells in one
  gauge), the two-step Lax--Wendroff update is the classical one-step stencil
  M - nu/2 A (M+ - M-) + nu^2/2 A^2 (M+ - 2M + M-), for both oracles;
* the FLIC limiter on a hand-computed sequence (each side's ratio binds
  somewhere), TVD for linear advection in either direction, and a mirrored
  FLIC step of the full nonlinear scheme returns the mirrored state.
"""

import math

import numpy as np
import pytest

from oracle import axisym, basis, kinetics, maxent
from oracle import flux as oflux


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


# ---- linear-closure pins ------------------------------------------------------
# With the closure replaced by beta = M and F = A beta, every flux of the scheme
# is linear and the update has a closed form.

def _linear_closure(monkeypatch, A, which):
    def fake_solve_k(M, beta, *a, **k):
        return dict(beta=np.array(M, copy=True), nonrealizable=np.zeros(len(M), bool))

    def fake_solve_a(M, g, beta, rule, **k):
        return dict(beta=np.array(M, copy=True), nonrealizable=np.zeros(len(M), bool))

    def fake_flux(beta, *a, **k):
        return np.asarray(beta) @ A.T

    if which == "kinetics":
        monkeypatch.setattr(maxent, "newton_solve", fake_solve_k)
        monkeypatch.setattr(oflux, "fluxes", fake_flux)
    else:
        monkeypatch.setattr(axisym, "solve", fake_solve_a)
        monkeypatch.setattr(axisym, "fluxes", fake_flux)


def _bare_solver(which, K, N, dx, scheme, ML, MR, A, lam):
    """A stepper object with N cells and two ghosts, every element in one gauge."""
    g = np.array([0.3, 1.1, 0.9])
    if which == "kinetics":
        s = object.__new__(kinetics.FVSolver)
        s.nodes, s.Phi, s.logw = None, None, None
        s.newton = {}
    else:
        s = object.__new__(axisym.ShockSolver)
        s.rule, s.newton = None, {}
    s.scheme, s.dx = scheme, dx
    s.g = np.repeat(g[None], N, axis=0)
    zb = np.zeros(K)
    s.ghost_left = (ML, A @ ML, lam, g.copy(), zb)
    s.ghost_right = (MR, A @ MR, lam, g.copy(), zb)
    return s


def _elements(s, M):
    return np.vstack([s.ghost_left[0][None], M, s.ghost_right[0][None]])


@pytest.mark.parametrize("which, K", [("kinetics", 35), ("axisym", 9)])
def test_two_step_lw_is_the_lax_wendroff_stencil(monkeypatch, which, K):
    rng = np.random.default_rng(11)
    N, dx, dt = 7, 0.2, 0.05
    A = rng.normal(size=(K, K)) / K + 1.5 * np.eye(K)
    # densities (component 0) stay positive at every half step: a half-step state
    # without positive density is not representable and keeps the LLF flux
    E0 = rng.normal(size=(N + 2, K))
    E0[:, 0] = 5.0 + np.abs(E0[:, 0])
    M = E0[1:-1]
    s = _bare_solver(which, K, N, dx, "lw", E0[0], E0[-1], A, 3.0)
    _linear_closure(monkeypatch, A, which)
    F = M @ A.T
    beta = np.zeros_like(M)
    rho = np.full(N, 3.0)
    got = s._fv2(M, F, beta, rho, dt)
    E = _elements(s, M)
    nu = dt / dx
    Mm, M0, Mp = E[:-2], E[1:-1], E[2:]
    want = (M0 - 0.5 * nu * (Mp - Mm) @ A.T
            + 0.5 * nu * nu * (Mp - 2.0 * M0 + Mm) @ (A @ A).T)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("which", ["kinetics", "axisym"])
def test_flic_limiter_on_a_hand_computed_sequence(monkeypatch, which):
    """Elements (ghost, 5 cells, ghost) carry u = 0, 1, 2, 4, 5, 5.5, 6 in every
    moment.  Interface j lies between elements j and j + 1; with d the jump
    across it, r_L = (jump one element to the left) / d and r_R = (jump one
    element to the right) / d, and the ghosts repeat beyond the ends:
      j = 0: r_L = 0 / 1           -> phi = 0
      j = 1: r_L = 1 / 1,  r_R = 2 / 1   -> min(1, 4/3) = 1
      j = 2: r_L = 1 / 2,  r_R = 1 / 2   -> 2/3
      j = 3: r_L = 2 / 1,  r_R = 0.5 / 1 -> min(4/3, 2/3) = 2/3
      j = 4: r_L = 1 / 0.5, r_R = 0.5 / 0.5 -> min(4/3, 1) = 1
      j = 5: r_R = 0 / 0.5          -> 0
    with van Leer's phi(r) = (r + |r|) / (1 + |r|)."""
    K = 35 if which == "kinetics" else 9
    a, lam, dx, dt = 1.0, 2.0, 0.1, 0.04
    A = a * np.eye(K)
    u = np.array([0.0, 1.0, 2.0, 4.0, 5.0, 5.5, 6.0])
    E = np.repeat(u[:, None], K, axis=1)
    s = _bare_solver(which, K, 5, dx, "flic", E[0], E[-1], A, lam)
    _linear_closure(monkeypatch, A, which)
    M = E[1:-1]
    f = s.interface_fluxes(M, M @ A.T, np.zeros_like(M), np.full(5, lam), dt)
    f = f[0] if isinstance(f, tuple) else f
    L, R = E[:-1], E[1:]
    f_lf = 0.5 * a * (L + R) + 0.5 * lam * (L - R)
    f_lw = a * (0.5 * (L + R) + 0.5 * (dt / dx) * a * (L - R))
    phi = (f - f_lf) / (f_lw - f_lf)
    want = np.array([0.0, 1.0, 2.0 / 3.0, 2.0 / 3.0, 1.0, 0.0])
    assert np.max(np.abs(phi - want[:, None])) < 1e-12


def _tv(E):
    return np.sum(np.abs(np.diff(E, axis=0)), axis=0)


@pytest.mark.parametrize("a", [1.0, -1.0])
def test_flic_is_tvd_for_linear_advection_either_way(monkeypatch, a):
    K = 35
    A = a * np.eye(K)
    N, dx = 40, 0.1
    dt = 0.8 * dx / abs(a)
    x = (np.arange(N) + 0.5) * dx
    prof = np.where((x > 1.0) & (x < 2.5), 1.0, 0.0) + 0.5 * np.exp(-((x - 3.2) / 0.2) ** 2)
    rng = np.random.default_rng(5)
    M = prof[:, None] * rng.uniform(0.5, 2.0, size=K)[None, :]
    out = {}
    for scheme in ("flic", "lw"):
        s = _bare_solver("kinetics", K, N, dx, scheme, M[0] * 0, M[-1] * 0, A, abs(a))
        _linear_closure(monkeypatch, A, "kinetics")
        out[scheme] = s._fv2(M, M @ A.T, np.zeros_like(M), np.full(N, abs(a)), dt)
    E0 = _elements(s, M)
    lo, hi = E0.min(axis=0), E0.max(axis=0)
    new = out["flic"]
    assert np.all(new >= lo - 1e-12) and np.all(new <= hi + 1e-12)
    assert np.all(_tv(_elements(s, new)) <= _tv(E0) + 1e-12)
    # the same data makes Lax--Wendroff overshoot: the check above has teeth
    assert np.any(out["lw"] > hi + 1e-3) or np.any(out["lw"] < lo - 1e-3)


def _mirror_sign(which):
    """(-1)^(degree in u_x) of each statistic: the sign it takes under u_x -> -u_x."""
    if which == "kinetics":
        return np.array([(-1.0) ** e[0] for e in basis.multi_indices(3)])
    return np.array([1.0, -1.0, 1.0, 1.0, -1.0, 1.0, 1.0, -1.0, 1.0])


@pytest.mark.parametrize("which", ["kinetics", "axisym"])
def test_flic_is_mirror_symmetric(monkeypatch, which):
    """x -> -x with u_x -> -u_x: moment i takes the sign P_i = (-1)^(x-degree),
    the elements come in reverse order, and the flux of the mirrored state is
    -P F.  A linear closure F = S M with that symmetry has S_ij = 0 unless P_i
    and P_j differ; S symmetric, so waves travel both ways at speeds +-mu.  One
    FLIC step of the mirrored elements must be the mirrored step.  With the
    printed one-sided ratio alone the limiter sees other neighbours: not so."""
    P = _mirror_sign(which)
    K = P.size
    rng = np.random.default_rng(8)
    S = rng.normal(size=(K, K))
    S = 0.5 * (S + S.T) * (P[:, None] != P[None, :])
    S /= np.max(np.abs(np.linalg.eigvalsh(S)))
    N, dx, lam = 12, 0.1, 1.0
    dt = 0.8 * dx / lam
    E = rng.normal(size=(N + 2, K)) * np.linspace(0.2, 1.5, N + 2)[:, None] ** 2
    E[:, 0] = 3.0 + np.abs(E[:, 0])
    Em = (E * P)[::-1]

    def step(Eh, limiter):
        s = _bare_solver(which, K, N, dx, "flic", Eh[0], Eh[-1], S, lam)
        _linear_closure(monkeypatch, S, which)
        monkeypatch.setattr(kinetics, "flic_limiter", limiter)
        M = Eh[1:-1]
        return s._fv2(M, M @ S.T, np.zeros_like(M), np.full(N, lam), dt)

    both = kinetics.flic_limiter
    one_sided = lambda dl, dm, dr: kinetics.van_leer(dl, dm)  # noqa: E731
    a, b = step(E, both), step(Em, both)
    assert np.max(np.abs(b - (a * P)[::-1])) < 1e-13
    a1, b1 = step(E, one_sided), step(Em, one_sided)
    assert np.max(np.abs(b1 - (a1 * P)[::-1])) > 1e-3
