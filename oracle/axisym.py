"""The paper's own velocity discretisation for 1D flow (oracle).

Test infrastructure only.  For flow along x with cylindrical symmetry in
velocity the paper works with nine statistics of (u_x, u_r),
u_r = sqrt(u_y^2 + u_z^2), integrated over a truncated box (u_x, u_r) in
[a_x, b_x] x [0, b_r] with block-wise Gauss--Legendre quadrature:

* statistics: the orthogonal form of the nine-statistic system (appendix on the
  exponential family of the 35-moment system).  Written with x = u_bar_x and
  y = u_bar_r^2 / 2 they are products of probabilists' Hermite polynomials in
  x and Laguerre polynomials in y:
  1, x, He_2(x)/sqrt2, y - 1, He_3(x)/sqrt6, He_4(x)/sqrt24,
  y^2/2 - 2y + 1, x (y - 1), He_2(x)/sqrt2 (y - 1).
  Reading: the printed eighth statistic u_x (u_r^2 - 1)/2 is neither
  orthogonal to u_x nor of unit norm under the standard Maxwellian, although
  the paper calls the set orthogonal; it is read as u_x (u_r^2 - 2)/2, the
  product of the second and fourth statistics, which matches the factor
  (u_r^2 - 2) of the ninth.
* gauge (Sec. 3.3): u_bar = ((u_x - w_x)/s_x, u_r/s_r).  The quadrature nodes
  stay fixed in physical velocity, so every cell evaluates the statistics at
  its own u_bar_p (a per-cell Phi).
* quadrature (end of Sec. 3.1): the box is cut into equal blocks, each
  integrated with the tensor product of the 1D Gauss--Legendre rule.  The
  integrands are axisymmetric, so d^3u = 2 pi u_r du_r du_x and the weight of
  node p is 2 pi u_r,p times the product of the two scaled Gauss--Legendre
  weights (the integral over the angle is exact).
* integration domain (appendix on the normal-shock set-up): a_x, b_x, b_r from
  the upstream and downstream states with integer multipliers n_a, n_b, n_r.
* Hermite gauge of the nine moments (Sec. 3.3): w_H = w + s_x E[x],
  s_xH^2 = s_x^2 Var(x), s_rH^2 = s_r^2 E[u_bar_r^2]/2 with
  E[x^2] = sqrt2 M_2/n + 1 and E[u_bar_r^2] = 2 (M_3/n + 1).
* change of gauge (Sec. 3.3): T(g', g) by projection onto the orthonormal
  statistics with an exact Gauss--Hermite x Gauss--Laguerre rule.
* solve: Alg. 1 through ``maxent.newton_solve`` cell by cell, each with its
  own Phi (nodes fixed in physical velocity) and the common log weights.

Units are non-dimensional with m = k_B = 1, so sqrt(k_B T/m) = sqrt(T).
"""

import math

import numpy as np

from . import maxent

K9 = 9
SQ2 = math.sqrt(2.0)
SQ6 = math.sqrt(6.0)
SQ24 = math.sqrt(24.0)


def statistics(x, ur):
    """The nine statistics at gauge coordinates (x, u_bar_r): shape (..., 9)."""
    x = np.asarray(x, dtype=np.float64)
    ur = np.asarray(ur, dtype=np.float64)
    y = 0.5 * ur * ur
    he2 = x * x - 1.0
    he3 = x * x * x - 3.0 * x
    he4 = x ** 4 - 6.0 * x * x + 3.0
    return np.stack([np.ones_like(x), x, he2 / SQ2, y - 1.0, he3 / SQ6, he4 / SQ24,
                     0.5 * y * y - 2.0 * y + 1.0, x * (y - 1.0), he2 / SQ2 * (y - 1.0)], axis=-1)


def gauss_legendre(order):
    """1D Gauss--Legendre nodes and weights on [-1, 1] (NumPy's leggauss)."""
    x, w = np.polynomial.legendre.leggauss(order)
    return x.astype(np.float64), w.astype(np.float64)


def blockwise_rule(ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order):
    """Nodes (u_x, u_r) and log weights of the block-wise rule on the box.

    Nodes run over blocks in x (outer), blocks in r, then the Gauss--Legendre
    points in x, then in r.  log w_p = log(2 pi u_r,p hx hr wx wr) with the
    half-widths hx, hr of a block.
    """
    gx, gw = gauss_legendre(order)
    hx = 0.5 * (ux_hi - ux_lo) / blocks_x
    hr = 0.5 * ur_hi / blocks_r
    ux, ur, w = [], [], []
    for bx in range(blocks_x):
        cx = ux_lo + (2 * bx + 1) * hx
        for br in range(blocks_r):
            cr = (2 * br + 1) * hr
            for i in range(order):
                for j in range(order):
                    u_r = cr + hr * gx[j]
                    ux.append(cx + hx * gx[i])
                    ur.append(u_r)
                    w.append(2.0 * math.pi * u_r * hx * hr * gw[i] * gw[j])
    return dict(ux=np.array(ux), ur=np.array(ur), logw=np.log(np.array(w)))


def integration_domain(v_minus, T_minus, v_plus, T_plus, n_a, n_b, n_r):
    """(a_x, b_x, b_r) of the normal-shock set-up (m = k_B = 1)."""
    sm, sp = math.sqrt(T_minus), math.sqrt(T_plus)
    a_x = min(v_plus - n_a * sp, v_minus - n_a * sm)
    b_x = max(v_minus + n_b * sm, v_plus + n_b * sp)
    b_r = max(n_r * sm, n_r * sp)
    return a_x, b_x, b_r


def cell_phi(rule, g):
    """Phi of one cell in gauge g = (w_x, s_x, s_r): (P, 9)."""
    w, sx, sr = g
    return statistics((rule["ux"] - w) / sx, rule["ur"] / sr)


def moments(beta, g, rule):
    """M_i = beta_0 sum_p sigma_p phi_i(u_bar_p) per cell (Sec. 3.1)."""
    beta = np.asarray(beta, dtype=np.float64)
    out = np.empty((beta.shape[0], K9))
    for c in range(beta.shape[0]):
        out[c] = maxent.model_moments(beta[c:c + 1], cell_phi(rule, g[c]), rule["logw"])[0]
    return out


def fluxes(beta, g, rule):
    """F_i = beta_0 sum_p sigma_p u_x,p phi_i(u_bar_p), u_x in physical velocity."""
    beta = np.asarray(beta, dtype=np.float64)
    out = np.empty((beta.shape[0], K9))
    for c in range(beta.shape[0]):
        Phi = cell_phi(rule, g[c])
        sig = maxent.sigma(beta[c:c + 1], Phi, rule["logw"])[0]
        out[c] = beta[c, 0] * (sig * rule["ux"]) @ Phi
    return out


def moment_residual(beta, M, g, rule):
    """max_{i>=1} |E_sigma[phi_i] - M_i/n| in FP64, per cell."""
    beta = np.asarray(beta, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    r = np.empty(M.shape[0])
    for c in range(M.shape[0]):
        r[c] = maxent.moment_residual(beta[c:c + 1], M[c:c + 1], cell_phi(rule, g[c]),
                                      rule["logw"])[0]
    return r


def hermite_gauge(M, g):
    """Hermite gauge parameters from the nine moments in gauge g (Sec. 3.3)."""
    M = np.asarray(M, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = M[:, 0]
    m1 = M[:, 1] / n
    exx = SQ2 * M[:, 2] / n + 1.0
    err = 2.0 * (M[:, 3] / n + 1.0)
    wH = g[:, 0] + g[:, 1] * m1
    sxH = g[:, 1] * np.sqrt(exx - m1 * m1)
    srH = g[:, 2] * np.sqrt(err / 2.0)
    return np.stack([wH, sxH, srH], axis=1)


def maxwellian_beta(n, g):
    """Cold start: the Maxwellian of the cell's own Hermite gauge, beta_0 = n.

    exp(-x^2/2 - u_bar_r^2/2) = exp(-(He_2(x)/sqrt2)/sqrt2 - (y - 1)) up to a
    constant absorbed by log Z: beta_2 = -1/sqrt2, beta_3 = -1.
    """
    n = np.asarray(n, dtype=np.float64)
    beta = np.zeros((n.size, K9))
    beta[:, 0] = n
    beta[:, 2] = -1.0 / SQ2
    beta[:, 3] = -1.0
    return beta


def solve(M, g, beta_init, rule, **kw):
    """Alg. 1 per cell on the nine statistics; returns maxent.newton_solve's fields."""
    M = np.asarray(M, dtype=np.float64)
    keys = ("beta", "iters", "resid", "converged", "stagnated", "nonrealizable", "shifted")
    out = {k: [] for k in keys}
    for c in range(M.shape[0]):
        r = maxent.newton_solve(M[c:c + 1], np.asarray(beta_init[c:c + 1], np.float64),
                                cell_phi(rule, g[c]), rule["logw"], **kw)
        for k in keys:
            out[k].append(r[k][0])
    return {k: np.array(v) for k, v in out.items()}


def _xy_coords(g_to, g_from, x, y):
    """Gauge coordinates in g_to of the velocity whose g_from coordinates are
    (x, y = u_bar_r^2/2)."""
    w, sx, sr = g_from
    w2, sx2, sr2 = g_to
    x2 = (w + sx * x - w2) / sx2
    y2 = y * (sr / sr2) ** 2
    return x2, y2


def change_matrix(g_to, g_from):
    """T(g', g) with M(g') = T M(g) (Sec. 3.3, eq. "Change gauge M F").

    Built by projection: the statistics are orthonormal under x ~ N(0, 1),
    y ~ Exp(1), and phi_i(u_bar') is a polynomial in the span, so
    T_ij = E[phi_i(u_bar'(x, y)) phi_j(x, y)], integrated exactly with
    Gauss--Hermite in x and Gauss--Laguerre in y.
    """
    xh, wh = np.polynomial.hermite_e.hermegauss(12)
    wh = wh / math.sqrt(2.0 * math.pi)
    yl, wl = np.polynomial.laguerre.laggauss(8)
    X, Y = np.meshgrid(xh, yl, indexing="ij")
    W = np.outer(wh, wl).ravel()
    X, Y = X.ravel(), Y.ravel()
    Pj = statistics(X, np.sqrt(2.0 * Y))
    x2, y2 = _xy_coords(g_to, g_from, X, Y)
    Pi = statistics(x2, np.sqrt(2.0 * y2))
    return (Pi * W[:, None]).T @ Pj


def to_hermite_gauge(M, beta, g):
    """Moments (and multipliers) moved into the Hermite gauge of M (Sec. 3.3).

    M' = T(g_H, g) M; beta'_i = sum_j T(g, g_H)_ji beta_j for i >= 1, beta'_0 = beta_0.
    """
    M = np.asarray(M, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    gH = hermite_gauge(M, g)
    Mo = np.empty_like(M)
    bo = None if beta is None else np.array(beta, dtype=np.float64, copy=True)
    for c in range(M.shape[0]):
        Mo[c] = change_matrix(gH[c], g[c]) @ M[c]
        if bo is not None:
            Ti = change_matrix(g[c], gH[c])
            bo[c, 1:] = (Ti.T @ np.asarray(beta[c], np.float64))[1:]
    return Mo, bo, gH


def char_speeds(beta, g, rule):
    """(min, max) eigenvalue of dF/dM per cell (the local Lax--Friedrichs speeds
    of Sec. 3.4): the extreme generalised eigenvalues of (E[x phi phi^T],
    E[phi phi^T]) in gauge coordinates, mapped to physical velocity
    w_x + s_x lambda.  scipy's generalised symmetric eigen-solver."""
    import scipy.linalg
    beta = np.asarray(beta, dtype=np.float64)
    out = np.empty((beta.shape[0], 2))
    for c in range(beta.shape[0]):
        w, sx, sr = g[c]
        Phi = cell_phi(rule, g[c])
        sig = maxent.sigma(beta[c:c + 1], Phi, rule["logw"])[0]
        x = (rule["ux"] - w) / sx
        B = (Phi * sig[:, None]).T @ Phi
        C = (Phi * (sig * x)[:, None]).T @ Phi
        ev = scipy.linalg.eigh(C, B, eigvals_only=True)
        out[c] = (w + sx * ev[0], w + sx * ev[-1])
    return out


# ---- the time step of Alg. 2 on the nine statistics --------------------------
def macroscopic(M, g):
    """n, v_x, T, P_xx/n and P_rr/n (= (P_yy + P_zz)/2n) from the nine moments."""
    M = np.asarray(M, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = M[:, 0]
    ex = M[:, 1] / n
    exx = SQ2 * M[:, 2] / n + 1.0
    err = 2.0 * (M[:, 3] / n + 1.0)          # E[u_bar_r^2]
    w, sx, sr = g[:, 0], g[:, 1], g[:, 2]
    pxx = sx ** 2 * (exx - ex ** 2)
    prr = 0.5 * sr ** 2 * err
    return dict(n=n, v=w + sx * ex, T=(pxx + 2.0 * prr) / 3.0, pxx=pxx, prr=prr)


def gaussian_moments(n, v, Sxx, Srr, g, rule_1d=16):
    """Nine moments in gauge g of n N((v,0,0), diag(Sxx, Srr, Srr)), by
    Gauss--Hermite in x and Gauss--Laguerre in y (exact for these degrees)."""
    xh, wh = np.polynomial.hermite_e.hermegauss(rule_1d)
    wh = wh / math.sqrt(2.0 * math.pi)
    yl, wl = np.polynomial.laguerre.laggauss(rule_1d)
    out = np.empty((len(n), K9))
    for c in range(len(n)):
        ux = v[c] + math.sqrt(Sxx[c]) * xh            # physical u_x
        y = Srr[c] * yl                                # u_r^2/2 for u_y, u_z ~ N(0, Srr)
        X, Y = np.meshgrid((ux - g[c][0]) / g[c][1], y / g[c][2] ** 2, indexing="ij")
        W = np.outer(wh, wl)
        out[c] = n[c] * np.einsum("ij,ijk->k", W, statistics(X, np.sqrt(2.0 * Y)))
    return out


def collision(M, g, h, prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi)):
    """ES-BGK relaxation over h (appendix on the ES-BGK model): M <- (1 - h/tau) M
    + (h/tau) M~, M~ the Gaussian with Sigma = T/Pr + (1 - 1/Pr) P/n,
    tau = mu_ref/(Pr n) (Maxwell molecules)."""
    mac = macroscopic(M, g)
    Sxx = mac["T"] / prandtl + (1.0 - 1.0 / prandtl) * mac["pxx"]
    Srr = mac["T"] / prandtl + (1.0 - 1.0 / prandtl) * mac["prr"]
    Mt = gaussian_moments(mac["n"], mac["v"], Sxx, Srr, np.asarray(g, np.float64))
    tau = mu_ref / (prandtl * mac["n"])
    r = (h / tau)[:, None]
    return (1.0 - r) * M + r * Mt


class ShockSolver:
    """Alg. 2 with local Lax--Friedrichs fluxes on the nine statistics: a normal
    shock between two fixed ghost Maxwellians, cells in their Hermite gauges,
    neighbour moments and fluxes moved into each cell's gauge by T(g_i, g_j),
    the ES-BGK source in two half steps around the transport (Sec. 3.4)."""

    def __init__(self, mach, n_cells, x_lo, x_hi, thickness, box, cfl=0.5,
                 prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi), newton=None,
                 scheme="llf"):
        import mem_inputs
        if scheme not in ("llf", "lw", "flic"):
            raise ValueError("scheme must be llf, lw or flic")
        self.scheme = scheme
        self.rule = blockwise_rule(**box)
        self.cfl, self.prandtl, self.mu_ref = cfl, prandtl, mu_ref
        self.newton = dict(tol_grad=1e-11, max_iter=300)
        if newton:
            self.newton.update(newton)
        (n1, v1, T1), (n2, v2, T2) = mem_inputs.rankine_hugoniot(mach)
        n1, v1, T1, n2, v2, T2 = (float(a) for a in (n1, v1, T1, n2, v2, T2))
        gm = np.array([[0.5 * (v1 + v2), 1.0, 1.0]])
        Mm = mem_inputs.gaussian_moments9(np.array([n1]), np.array([v1]), np.array([T1]),
                                          np.array([T1]), gm)[0]
        Mp = mem_inputs.gaussian_moments9(np.array([n2]), np.array([v2]), np.array([T2]),
                                          np.array([T2]), gm)[0]
        self.dx = (x_hi - x_lo) / n_cells
        x = x_lo + self.dx * (np.arange(n_cells) + 0.5)
        th = thickness / 2.0
        frac = ((np.tanh(x / th) - math.tanh(x_lo / th))
                / (math.tanh(x_hi / th) - math.tanh(x_lo / th)) - 0.5)
        M0 = (Mp - Mm)[None, :] * frac[:, None] + 0.5 * (Mp + Mm)[None, :]
        self.M, _, self.g = to_hermite_gauge(M0, None, np.repeat(gm, n_cells, axis=0))
        self.beta = maxwellian_beta(self.M[:, 0], self.g)
        self.states = ((n1, v1, T1), (n2, v2, T2))
        gh = []
        for (n, v, T) in self.states:
            gg = np.array([[v, math.sqrt(T), math.sqrt(T)]])
            bg = maxwellian_beta(np.array([n]), gg)
            Mg = moments(bg, gg, self.rule)
            Fg = fluxes(bg, gg, self.rule)
            lam = char_speeds(bg, gg, self.rule)[0]
            gh.append((Mg[0], Fg[0], float(np.max(np.abs(lam))), gg[0], bg[0]))
        self.ghost_left, self.ghost_right = gh
        self.t = 0.0
        self.beta = self._solve(self.M, self.beta)
        self.dt = self._dt(self._rho(self.beta))

    def _solve(self, M, beta):
        """Alg. 1 per cell; a cell the box cannot represent takes the Maxwellian
        of its gauge (the GPU step applies the same rule)."""
        out = solve(M, self.g, beta, self.rule, **self.newton)
        b = out["beta"].copy()
        bad = out["nonrealizable"] | ~np.all(np.isfinite(b), axis=1)
        if np.any(bad):
            b[bad] = maxwellian_beta(M[bad, 0], self.g[bad])
        return b

    def _rho(self, beta):
        lam = char_speeds(beta, self.g, self.rule)
        return np.max(np.abs(lam), axis=1)

    def _dt(self, rho):
        rmax = max(np.max(rho), self.ghost_left[2], self.ghost_right[2])
        return self.cfl * self.dx / rmax

    def _fv(self, M, F, rho, dt):
        N = M.shape[0]
        g = self.g
        MLg, FLg, rL, gL, _ = self.ghost_left
        MRg, FRg, rR, gR, _ = self.ghost_right
        out = np.empty_like(M)
        for i in range(N):
            if i > 0:
                Tl = change_matrix(g[i], g[i - 1]); Ml, Fl, rl = Tl @ M[i - 1], Tl @ F[i - 1], rho[i - 1]
            else:
                Tl = change_matrix(g[i], gL); Ml, Fl, rl = Tl @ MLg, Tl @ FLg, rL
            if i < N - 1:
                Tr = change_matrix(g[i], g[i + 1]); Mr, Fr, rr = Tr @ M[i + 1], Tr @ F[i + 1], rho[i + 1]
            else:
                Tr = change_matrix(g[i], gR); Mr, Fr, rr = Tr @ MRg, Tr @ FRg, rR
            lm, lp = max(rl, rho[i]), max(rho[i], rr)
            f_minus = 0.5 * (Fl + F[i]) + 0.5 * lm * (Ml - M[i])
            f_plus = 0.5 * (F[i] + Fr) + 0.5 * lp * (M[i] - Mr)
            out[i] = M[i] + dt / self.dx * (f_minus - f_plus)
        return out

    def interface_fluxes(self, M, F, beta, rho, dt):
        """Flux at each of the N + 1 interfaces (Sec. 3.4: LF, two-step LW, FLIC
        with the per-moment van Leer limiter), interface j between elements j
        and j + 1 of [left ghost, cells, right ghost], in the gauge of element
        j + 1.  One MaxEnt solve per interface; an interface whose half-step
        state cannot be solved keeps F_LF."""
        from .kinetics import flic_limiter
        MLg, FLg, rL, gL, bL = self.ghost_left
        MRg, FRg, rR, gR, bR = self.ghost_right
        Me = np.vstack([MLg[None], M, MRg[None]])
        Fe = np.vstack([FLg[None], F, FRg[None]])
        ge = np.vstack([gL[None], self.g, gR[None]])
        be = np.vstack([bL[None], beta, bR[None]])
        re = np.concatenate([[rL], rho, [rR]])
        N = M.shape[0]
        out = np.empty((N + 1, K9))
        Mh = np.empty((N + 1, K9))
        for j in range(N + 1):
            L, R = j, j + 1
            T = change_matrix(ge[R], ge[L])
            ML, FL = T @ Me[L], T @ Fe[L]
            lam = max(re[L], re[R])
            out[j] = 0.5 * (FL + Fe[R]) + 0.5 * lam * (ML - Me[R])
            Mh[j] = 0.5 * (ML + Me[R]) + 0.5 * (dt / self.dx) * (FL - Fe[R])
        if self.scheme == "llf":
            return out
        sol = solve(Mh, ge[1:], be[1:], self.rule, **self.newton)
        for j in range(N + 1):
            L, R = j, j + 1
            bh = sol["beta"][j]
            if (sol["nonrealizable"][j] or not np.all(np.isfinite(bh))
                    or not np.all(np.isfinite(Mh[j])) or not Mh[j, 0] > 0):
                continue
            f_lw = fluxes(bh[None, :], ge[R][None, :], self.rule)[0]
            if self.scheme == "lw":
                phi = np.ones(K9)
            else:
                # the ghosts continue beyond both boundaries
                LL, RR = max(L - 1, 0), min(R + 1, N + 1)
                ML = change_matrix(ge[R], ge[L]) @ Me[L]
                MLL = change_matrix(ge[R], ge[LL]) @ Me[LL]
                MRR = change_matrix(ge[R], ge[RR]) @ Me[RR] if RR != R else Me[R]
                phi = flic_limiter(ML - MLL, Me[R] - ML, MRR - Me[R])
            out[j] = out[j] + phi * (f_lw - out[j])
        return out

    def _fv2(self, M, F, beta, rho, dt):
        """Conservative update from the interface fluxes: cell i receives the
        flux of its left face as given (its own gauge) and that of its right
        face moved into its gauge by T(g_i, g_{i+1})."""
        f = self.interface_fluxes(M, F, beta, rho, dt)
        gR = self.ghost_right[3]
        out = np.empty_like(M)
        for i in range(M.shape[0]):
            gn = self.g[i + 1] if i + 1 < M.shape[0] else gR
            fr = change_matrix(self.g[i], gn) @ f[i + 1]
            out[i] = M[i] + dt / self.dx * (f[i] - fr)
        return out

    def step(self):
        dt = self.dt
        M = collision(self.M, self.g, 0.5 * dt, self.prandtl, self.mu_ref)
        beta = self._solve(M, self.beta)
        F = fluxes(beta, self.g, self.rule)
        rho = self._rho(beta)
        dt = min(dt, self._dt(rho))
        M = self._fv(M, F, rho, dt) if self.scheme == "llf" else self._fv2(M, F, beta, rho, dt)
        M = collision(M, self.g, 0.5 * dt, self.prandtl, self.mu_ref)
        self.M, self.beta, self.g = to_hermite_gauge(M, beta, self.g)
        self.t += dt
        self.dt = self._dt(rho)
        return dt


# ---- the two forms of the family and overflow (Sec. 2, the canonical form;
# Sec. 4.1, Fig. 1) ---------------------------------------------------------------
# canonical:     f = beta_0 exp(beta_i phi_i - log Z(beta)),
# non-canonical: f = exp(alpha_0 + alpha_i phi_i), with alpha_0 = log beta_0 -
# log Z(beta) and alpha_i = beta_i for the same density.

LOG_FLT_MAX = math.log(float(np.finfo(np.float32).max))   # 88.72...


def noncanonical_alpha(beta, g, rule):
    """Non-canonical parameters of the densities given canonically."""
    beta = np.asarray(beta, dtype=np.float64)
    alpha = beta.copy()
    for c in range(beta.shape[0]):
        lz = maxent.log_partition(beta[c:c + 1], cell_phi(rule, g[c]), rule["logw"])[0]
        alpha[c, 0] = math.log(beta[c, 0]) - lz
    return alpha


def _noncanonical_exponents(alpha, Phi):
    """alpha_0 + alpha_i phi_i(u_p), i >= 1: (C, P)."""
    return alpha[:, :1] + alpha[:, 1:] @ Phi[:, 1:].T


def noncanonical_moments(alpha, g, rule):
    """M_j = sum_p w_p exp(alpha_0 + alpha_i phi_i(u_p)) phi_j(u_p), the plain
    sum with no shift of the exponent (FP64)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    out = np.empty((alpha.shape[0], K9))
    for c in range(alpha.shape[0]):
        Phi = cell_phi(rule, g[c])
        e = _noncanonical_exponents(alpha[c:c + 1], Phi)[0] + rule["logw"]
        out[c] = np.exp(e) @ Phi
    return out


def noncanonical_overflow(alpha, g, rule, margin=1.0):
    """Whether the FP32 evaluation of the non-canonical moments (exp of each
    exponent, times w_p, times phi_j, summed) overflows, decided in FP64.

    Returns (certain, safe): certain where some exponent exceeds
    log(FLT_MAX) + margin (exp itself is infinite there); safe where every
    exponent and, for every j, log sum_p w_p exp(.) |phi_j| stay below
    log(FLT_MAX) - margin (no product and no partial sum can reach FLT_MAX).
    Samples in neither class sit within the margin, where FP32 rounding of the
    exponent decides."""
    alpha = np.asarray(alpha, dtype=np.float64)
    C = alpha.shape[0]
    certain = np.zeros(C, dtype=bool)
    safe = np.zeros(C, dtype=bool)
    for c in range(C):
        Phi = cell_phi(rule, g[c])
        e = _noncanonical_exponents(alpha[c:c + 1], Phi)[0]
        emax = e.max()
        lt = e + rule["logw"]
        q = lt.max()
        with np.errstate(divide="ignore"):
            lsum = q + np.log(np.exp(lt - q) @ np.abs(Phi))   # log sum_p w e |phi_j|
        certain[c] = emax > LOG_FLT_MAX + margin
        safe[c] = emax < LOG_FLT_MAX - margin and np.all(lsum < LOG_FLT_MAX - margin)
    return certain, safe
