"""Pins for the oracle's nine-statistic discretisation (no GPU).

* Block-wise Gauss--Legendre (end of Sec. 3.1): exact on polynomials of the
  rule's degree, against closed-form integrals over the box with the
  axisymmetric measure 2 pi u_r du_r du_x.
* Statistics (appendix on the 35-moment system, orthogonal form): orthonormal
  under the standard Maxwellian, inside the span of the 35 three-dimensional
  Hermite statistics (the 35 -> 9 reduction), and the printed eighth statistic
  is not orthogonal (the reading the oracle takes).
* Moments and fluxes of Maxwellians in arbitrary gauges (Sec. 3.1, Sec. 3.3)
  against closed-form Gaussian expectations; Hermite gauge of a Maxwellian.
* Alg. 1 on the nine statistics returns the closed-form Maxwellian
  multipliers; the integration-domain formula reproduces the paper's printed
  boxes (``tests/golden/axisym_domains.json``).
"""

import json
import math
import os

import numpy as np
import pytest

import mem_inputs
from oracle import axisym, basis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("order", [1, 2, 5, 8, 12, 16])
def test_gauss_legendre_exact(order):
    x, w = axisym.gauss_legendre(order)
    for k in range(2 * order):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


def test_blockwise_rule_exact_on_polynomials():
    lo, hi, rh = -3.1, 4.7, 5.3
    rule = axisym.blockwise_rule(lo, hi, rh, 3, 2, 4)
    assert rule["ux"].size == 3 * 2 * 16
    w = np.exp(rule["logw"])
    for a in range(8):
        for b in range(7):   # u_r^(b+1) must stay within degree 7 per axis
            num = np.sum(w * rule["ux"] ** a * rule["ur"] ** b)
            exact = (2 * math.pi * (hi ** (a + 1) - lo ** (a + 1)) / (a + 1)
                     * rh ** (b + 2) / (b + 2))
            assert abs(num - exact) <= 1e-12 * max(1.0, abs(exact))


def _wide_rule():
    return axisym.blockwise_rule(-22.0, 22.0, 22.0, 22, 11, 12)


def test_statistics_orthonormal_under_standard_maxwellian():
    rule = _wide_rule()
    f = np.exp(rule["logw"] - 0.5 * (rule["ux"] ** 2 + rule["ur"] ** 2)) / (2 * math.pi) ** 1.5
    Phi = axisym.statistics(rule["ux"], rule["ur"])
    G = (Phi * f[:, None]).T @ Phi
    assert np.max(np.abs(G - np.eye(9))) < 1e-12
    # the printed eighth statistic u_x (u_r^2 - 1)/2 is not orthogonal to u_x
    printed = 0.5 * rule["ux"] * (rule["ur"] ** 2 - 1.0)
    assert abs(np.sum(f * printed * rule["ux"]) - 0.5) < 1e-12


def test_statistics_in_span_of_3d_hermite_basis():
    rng = np.random.default_rng(7)
    u = rng.normal(size=(400, 3)) * 1.7
    P35 = basis.evaluate(u, 3)
    P9 = axisym.statistics(u[:, 0], np.sqrt(u[:, 1] ** 2 + u[:, 2] ** 2))
    coef, *_ = np.linalg.lstsq(P35, P9, rcond=None)
    assert np.max(np.abs(P35 @ coef - P9)) < 1e-10
    # symmetric in (u_y, u_z): swapping them leaves every statistic unchanged
    assert np.allclose(axisym.statistics(u[:, 0], np.hypot(u[:, 2], u[:, 1])), P9, atol=1e-13)


def _raw_gauss(mu, s2, kmax):
    m = [1.0, mu]
    for k in range(2, kmax + 1):
        m.append(mu * m[k - 1] + (k - 1) * s2 * m[k - 2])
    return m


def _closed_form(n, v, T, g, with_ux=False):
    """Closed-form n E[phi_i] (or n E[u_x phi_i]) for a Maxwellian, gauge g."""
    w, sx, sr = g
    mu, s2, th = (v - w) / sx, T / sx ** 2, T / sr ** 2
    mx = _raw_gauss(mu, s2, 6)
    Ey = [math.factorial(k) * th ** k for k in range(3)]
    # x-polynomials (coefficients of x^0..x^4) and y-polynomials of each statistic
    xp = {0: [1], 1: [0, 1], 2: [-1 / math.sqrt(2), 0, 1 / math.sqrt(2)],
          3: [0, -3 / math.sqrt(6), 0, 1 / math.sqrt(6)],
          4: [3 / math.sqrt(24), 0, -6 / math.sqrt(24), 0, 1 / math.sqrt(24)]}
    stats = [(0, [1]), (1, [1]), (2, [1]), (0, [-1, 1]), (3, [1]), (4, [1]),
             (0, [1, -2, 0.5]), (1, [-1, 1]), (2, [-1, 1])]
    out = []
    for xi, yp in stats:
        c = list(xp[xi])
        if with_ux:   # u_x = w + s_x x
            c = [w * a for a in c] + [0.0]
            for k, a in enumerate(xp[xi]):
                c[k + 1] += sx * a
        ex = sum(a * mx[k] for k, a in enumerate(c))
        ey = sum(a * Ey[k] for k, a in enumerate(yp))
        out.append(n * ex * ey)
    return np.array(out)


def _maxwellian_beta_in_gauge(n, v, T, g):
    w, sx, sr = g
    b = np.zeros(9)
    b[0] = n
    b[1] = -sx * (w - v) / T
    b[2] = -sx ** 2 / (math.sqrt(2) * T)
    b[3] = -sr ** 2 / T
    return b


CASES = [(1.0, 0.0, 1.0, (0.0, 1.0, 1.0)), (2.3, 1.7, 0.6, (1.2, 0.9, 0.7)),
         (0.4, -2.0, 3.1, (-1.5, 1.6, 2.1))]


@pytest.mark.parametrize("case", CASES)
def test_maxwellian_moments_and_fluxes_closed_form(case):
    n, v, T, g = case
    rule = _wide_rule()
    beta = _maxwellian_beta_in_gauge(n, v, T, g)[None, :]
    M = axisym.moments(beta, np.array([g]), rule)[0]
    F = axisym.fluxes(beta, np.array([g]), rule)[0]
    assert np.max(np.abs(M - _closed_form(n, v, T, g))) < 1e-10
    assert np.max(np.abs(F - _closed_form(n, v, T, g, with_ux=True))) < 1e-10
    # the shared input generator's closed form agrees
    Mi = mem_inputs.gaussian_moments9(np.array([n]), np.array([v]), np.array([T]),
                                      np.array([T]), np.array([g]))[0]
    assert np.max(np.abs(Mi - M)) < 1e-10
    gH = axisym.hermite_gauge(M[None, :], np.array([g]))[0]
    assert np.allclose(gH, [v, math.sqrt(T), math.sqrt(T)], atol=1e-10)


@pytest.mark.parametrize("case", CASES)
def test_solve_returns_maxwellian_multipliers(case):
    n, v, T, g = case
    rule = _wide_rule()
    M = _closed_form(n, v, T, g)[None, :]
    b0 = axisym.maxwellian_beta(np.array([n]), np.array([g]))
    r = axisym.solve(M, np.array([g]), b0, rule, tol_grad=1e-12, max_iter=100)
    assert r["converged"][0]
    assert np.max(np.abs(r["beta"][0] - _maxwellian_beta_in_gauge(n, v, T, g))) < 1e-8


def test_solve_mott_smith_cells_on_paper_box():
    cells = mem_inputs.mott_smith_cells9(12, replica=3)
    rule = axisym.blockwise_rule(**mem_inputs.AXI_MACH10_BOX)
    assert rule["ux"].size == 1536
    b0 = axisym.maxwellian_beta(cells["M"][:, 0], cells["g"])
    r = axisym.solve(cells["M"], cells["g"], b0, rule, tol_grad=1e-11, max_iter=200)
    assert np.all(r["converged"])
    res = axisym.moment_residual(r["beta"], cells["M"], cells["g"], rule)
    assert np.all(res <= 1e-11)
    # the certificate of Alg. 1: the gradient is zero, so the model reproduces M
    Mm = axisym.moments(r["beta"], cells["g"], rule)
    assert np.max(np.abs(Mm - cells["M"]) / cells["M"][:, :1]) < 1e-10


def test_integration_domain_reproduces_printed_boxes():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "axisym_domains.json")))
    for c in gold["cases"]:
        (n1, v1, T1), (n2, v2, T2) = mem_inputs.rankine_hugoniot(c["mach"])
        box = axisym.integration_domain(float(v1), float(T1), float(v2), float(T2),
                                        c["n_a"], c["n_b"], c["n_r"])
        assert [round(b, 1) for b in box] == c["box"]


G_A, G_B, G_C = (0.3, 1.1, 0.9), (-1.2, 1.7, 1.4), (2.0, 0.8, 1.3)


def test_change_matrix_group_and_identity():
    assert np.max(np.abs(axisym.change_matrix(G_A, G_A) - np.eye(9))) < 1e-13
    T = axisym.change_matrix(G_C, G_B) @ axisym.change_matrix(G_B, G_A)
    assert np.max(np.abs(T - axisym.change_matrix(G_C, G_A))) < 1e-12
    # lower triangular in (x degree, y degree): statistic (a, k) only draws on a' <= a, k' <= k
    deg = [(0, 0), (1, 0), (2, 0), (0, 1), (3, 0), (4, 0), (0, 2), (1, 1), (2, 1)]
    T = axisym.change_matrix(G_B, G_A)
    for i, (a, k) in enumerate(deg):
        for j, (a2, k2) in enumerate(deg):
            if a2 > a or k2 > k:
                assert abs(T[i, j]) < 1e-13


@pytest.mark.parametrize("case", CASES)
def test_change_of_gauge_moves_maxwellian_moments(case):
    n, v, T, _ = case
    Ma = _closed_form(n, v, T, G_A)
    Mb = axisym.change_matrix(G_B, G_A) @ Ma
    assert np.max(np.abs(Mb - _closed_form(n, v, T, G_B))) < 1e-11


def test_to_hermite_gauge_keeps_the_distribution():
    rule = _wide_rule()
    beta = _maxwellian_beta_in_gauge(1.2, 0.7, 1.4, G_A)
    beta[4] += 0.01
    beta[5] -= 0.004
    beta[8] += 0.003
    M = axisym.moments(beta[None, :], np.array([G_A]), rule)
    Mo, bo, gH = axisym.to_hermite_gauge(M, beta[None, :], np.array([G_A]))
    # the same distribution: its moments in the Hermite gauge from the moved beta
    M2 = axisym.moments(bo, gH, rule)
    assert np.max(np.abs(M2 - Mo)) < 1e-10
    # the Hermite gauge zeroes the first and the two second-degree moments
    assert np.max(np.abs(Mo[0, 1:4])) < 1e-12


def test_char_speeds_of_maxwellian_are_hermite_roots():
    # in its own Hermite gauge a Maxwellian makes x and y independent; the pencil
    # splits by y-degree into {1..x^4}, {1, x, x^2} (y - 1) and the y^2 block,
    # whose eigenvalues are the roots of He_5, He_3 and 0: the extremes are the
    # outermost root of He_5 (the five-point Gauss--Hermite node)
    rule = _wide_rule()
    n, v, T = 1.4, 0.8, 2.3
    g = (v, math.sqrt(T), math.sqrt(T))
    beta = _maxwellian_beta_in_gauge(n, v, T, g)[None, :]
    lam = axisym.char_speeds(beta, np.array([g]), rule)[0]
    r5 = math.sqrt(5.0 + math.sqrt(10.0))
    assert abs(lam[0] - (v - math.sqrt(T) * r5)) < 1e-9
    assert abs(lam[1] - (v + math.sqrt(T) * r5)) < 1e-9


def test_char_speeds_within_node_span():
    cells = mem_inputs.mott_smith_cells9(6, mach_lo=2.0, mach_hi=10.0, replica=8)
    rule = axisym.blockwise_rule(**mem_inputs.AXI_MACH10_BOX)
    sol = axisym.solve(cells["M"], cells["g"], axisym.maxwellian_beta(cells["M"][:, 0], cells["g"]),
                       rule, tol_grad=1e-10, max_iter=300)
    lam = axisym.char_speeds(sol["beta"], cells["g"], rule)
    assert np.all(lam[:, 0] >= rule["ux"].min() - 1e-9)
    assert np.all(lam[:, 1] <= rule["ux"].max() + 1e-9)
    assert np.all(lam[:, 0] < lam[:, 1])


def test_collision_conserves_and_relaxes_to_es_bgk():
    cells = mem_inputs.mott_smith_cells9(5, mach_lo=2.0, mach_hi=6.0, replica=9)
    M, g = cells["M"], cells["g"]
    mac0 = axisym.macroscopic(M, g)
    M1 = axisym.collision(M, g, 0.3)
    mac1 = axisym.macroscopic(M1, g)
    for k in ("n", "v", "T"):
        assert np.allclose(mac0[k], mac1[k], rtol=1e-12, atol=1e-12), k
    # the Gaussian moments match the shared closed form (Pr = 1: the Maxwellian)
    Mt = axisym.gaussian_moments(mac0["n"], mac0["v"], mac0["T"], mac0["T"], g)
    Mi = mem_inputs.gaussian_moments9(mac0["n"], mac0["v"], mac0["T"], mac0["T"], g)
    assert np.max(np.abs(Mt - Mi)) < 1e-11


def _small_shock():
    (n1, v1, T1), (n2, v2, T2) = mem_inputs.rankine_hugoniot(3.0)
    a_x, b_x, b_r = axisym.integration_domain(float(v1), float(T1), float(v2), float(T2), 10, 6, 6)
    box = dict(ux_lo=a_x, ux_hi=b_x, ur_hi=b_r, blocks_x=6, blocks_r=4, order=8)
    return box


def test_transport_is_conservative_in_the_interior():
    # T(g', g) keeps the mass row (phi_0 = 1 in every gauge), and both cells of a
    # face use the same LLF speed, so interior mass fluxes telescope: the total
    # mass changes only through the two boundary faces
    sh = axisym.ShockSolver(3.0, 24, -12.0, 12.0, 5.44, _small_shock())
    for _ in range(2):
        sh.step()
    F = axisym.fluxes(sh.beta, sh.g, sh.rule)
    rho = sh._rho(sh.beta)
    dt = sh.dt
    Mn = sh._fv(sh.M, F, rho, dt)
    MLg, FLg, rL, _, _ = sh.ghost_left
    MRg, FRg, rR, _, _ = sh.ghost_right
    fL = 0.5 * (FLg[0] + F[0, 0]) + 0.5 * max(rL, rho[0]) * (MLg[0] - sh.M[0, 0])
    fR = 0.5 * (F[-1, 0] + FRg[0]) + 0.5 * max(rho[-1], rR) * (sh.M[-1, 0] - MRg[0])
    dmass = np.sum(Mn[:, 0] - sh.M[:, 0]) * sh.dx
    assert abs(dmass - dt * (fL - fR)) < 1e-12 * np.sum(sh.M[:, 0])
    assert np.all(np.isfinite(Mn))


def test_uniform_equilibrium_is_stationary():
    box = _small_shock()
    sh = axisym.ShockSolver(3.0, 8, -4.0, 4.0, 5.44, box)
    (n1, v1, T1), _ = sh.states
    gg = np.array([[v1, math.sqrt(T1), math.sqrt(T1)]])
    sh.g = np.repeat(gg, 8, axis=0)
    sh.M = np.zeros((8, 9)); sh.M[:, 0] = n1
    sh.beta = axisym.maxwellian_beta(sh.M[:, 0], sh.g)
    # both ghosts upstream: the uniform upstream state must not move
    sh.ghost_right = sh.ghost_left
    sh.M = axisym.moments(sh.beta, sh.g, sh.rule)
    mac0 = axisym.macroscopic(sh.M, sh.g)
    sh.step()
    # the source and the re-gauging keep n, v, T; the higher moments move by the
    # box's quadrature error against the exact Gaussian target (~1e-5), which
    # leaves the two boundary cells a flux imbalance of that order times dt
    mac1 = axisym.macroscopic(sh.M, sh.g)
    for k in ("n", "v", "T"):
        assert np.max(np.abs(mac1[k] - mac0[k])) < 1e-7, k
        assert np.max(np.abs(mac1[k][1:-1] - mac0[k][1:-1])) < 1e-10, k


def test_second_order_interface_fluxes_reduce_to_lf():
    # with the limiter forced to zero FLIC is LF; the LF interface fluxes of the
    # second-order path equal those the LLF update uses
    sh = axisym.ShockSolver(3.0, 12, -6.0, 6.0, 5.44, _small_shock(), scheme="flic")
    F = axisym.fluxes(sh.beta, sh.g, sh.rule)
    rho = sh._rho(sh.beta)
    sh.scheme = "llf"
    Ml = sh._fv(sh.M, F, rho, sh.dt)
    M2 = sh._fv2(sh.M, F, sh.beta, rho, sh.dt)
    assert np.max(np.abs(Ml - M2)) < 1e-12
    sh.scheme = "flic"
    for _ in range(2):
        sh.step()
    assert np.all(np.isfinite(sh.M))


# ---- the two forms of the family and overflow (Sec. 2; Sec. 4.1, Fig. 1) ----

@pytest.fixture(scope="module")
def e1_rule():
    return axisym.blockwise_rule(**mem_inputs.E1_BOX)


def test_noncanonical_form_is_the_same_density(e1_rule):
    # alpha_0 = log beta_0 - log Z(beta), alpha_i = beta_i gives the same
    # moments as the canonical form, summed without any shift
    d = mem_inputs.overflow_samples(6, sigma=0.02, replica=3)
    beta = d["beta"].copy()
    beta[:, 5] = -np.abs(beta[:, 5]) - 0.01     # decaying quartic terms: finite sums
    beta[:, 6] = -np.abs(beta[:, 6]) - 0.01
    alpha = axisym.noncanonical_alpha(beta, d["g"], e1_rule)
    assert np.array_equal(alpha[:, 1:], beta[:, 1:])
    Mn = axisym.noncanonical_moments(alpha, d["g"], e1_rule)
    Mc = axisym.moments(beta, d["g"], e1_rule)
    assert np.max(np.abs(Mn - Mc) / beta[:, :1]) < 1e-12


def test_equilibrium_alpha_is_the_maxwellian_normalisation(e1_rule):
    # the non-canonical equilibrium is n (2 pi)^(-3/2) exp(-|u|^2/2): its
    # alpha_0 is the Maxwellian's normalisation up to the box quadrature error
    d = mem_inputs.overflow_samples(1)
    a = axisym.noncanonical_alpha(d["centre_beta"][None], d["g"], e1_rule)
    assert a[0, 0] == pytest.approx(-1.5 * (math.log(2.0 * math.pi) + 1.0), abs=1e-7)
    M = axisym.noncanonical_moments(d["centre_alpha"][None], d["g"], e1_rule)
    assert M[0, 0] == pytest.approx(1.0, abs=1e-7)


def test_overflow_classification_by_hand(e1_rule):
    d = mem_inputs.overflow_samples(1)
    a = np.tile(d["centre_alpha"], (3, 1))
    a[1, 5] += 0.1          # u_x^4 coefficient positive
    a[2, 6] += 0.1          # u_r^4 coefficient positive
    certain, safe = axisym.noncanonical_overflow(a, d["g"][[0, 0, 0]], e1_rule)
    assert safe[0] and not certain[0]
    # row 1: at the node nearest u_x = -30.7, u_r = 0 the exponent is about
    # alpha_0 - x^2/2 + 0.1 He_4(x)/sqrt24 with x ~ -30.7: far above log(FLT_MAX)
    x = e1_rule["ux"].min()
    by_hand = a[1, 0] - 0.5 * x * x + 0.1 * (x ** 4 - 6 * x * x + 3) / math.sqrt(24.0)
    assert by_hand > 1e4
    assert certain[1] and not safe[1]
    # row 2: y = u_r^2/2 ~ 578 at the outer radius, 0.1 (y^2/2 - 2y + 1) ~ 1.7e4
    assert certain[2] and not safe[2]


def test_overflow_free_samples_lie_in_the_third_quadrant(e1_rule):
    # Fig. 1(b): without the partition function the samples that stay finite
    # nearly all have both the u_x^4 and u_r^4 coefficients negative (a few
    # with a slightly positive one outweighed by the other terms); with it none
    # overflow
    d = mem_inputs.overflow_samples(256, replica=1)
    certain, safe = axisym.noncanonical_overflow(d["alpha"], d["g"], e1_rule)
    third = (d["alpha"][:, 5] < 0.0) & (d["alpha"][:, 6] < 0.0)
    assert np.mean(third[safe]) >= 0.9
    assert not np.any(safe & (d["alpha"][:, 5] > 0.01))
    assert certain.mean() > 0.5
    # canonical: log-sum-exp moments of every beta sample are finite
    M = axisym.moments(d["beta"], d["g"], e1_rule)
    assert np.all(np.isfinite(M))
