"""Collision, normal-shock set-up and the finite-volume time step (oracle).

Test infrastructure only.  3D velocity space, 35-moment basis, 1D transport
along x.  Paper passages followed:

* macroscopic quantities n, v, T, pressure tensor and heat flux (Sec. 2.1 and
  App. A, eq. "Pressure, Stress, and Heat flux"), obtained from moments by
  expanding each velocity monomial in the basis (coefficients by projection);
* ES-BGK target (App. A, eq. "The ES BGK model"): Gaussian with
  Sigma = (1/Pr) T I + (1 - 1/Pr) P/n, restricted -- as the paper's statistics
  {1, u_x, u_x^2, u_r^2} for the target are (App. B) -- to the axisymmetric
  form (v_x, Sigma_xx, Sigma_rr = (Sigma_yy + Sigma_zz)/2);  its moments are
  integrated with Gauss--Hermite in the Gaussian's own coordinates (exact for
  polynomials);  relaxation time from mu/Pr = n T tau with Maxwell-molecule
  viscosity mu = mu_ref T (eqs. "Maxwell viscosity coef", "The ES BGK
  viscosity");
* operator-split relaxation M <- (1 - h/tau) M + (h/tau) M~ (eq. "source
  update");
* Rankine--Hugoniot states (eq. "RH condition") with the non-dimensionalisation
  m = 1, rho_- = 1, v_- = sqrt(gamma) Ma, T_- = 1 (eq. "Non-dim");
* tanh initial profile between M_- and M_+ (eq. "Mx ini");
* local Lax--Friedrichs flux and conservative update in each cell's own gauge,
  neighbours moved into it by T (eqs. "The lax F", "The ME equation fvm 2",
  "The lax F convert");
* second-order interface fluxes (Sec. 3.4): two-step Lax--Wendroff (eq. "The
  lax W": half-step interface moments, their MaxEnt solve, the flux of that
  solution) and FLIC (eq. "The FLIC": LLF plus a van Leer-limited share of
  the Lax--Wendroff correction, the ratio r taken per moment);
* Alg. 2 Step: Collision(dt/2), Transport(dt), Collision(dt/2), then the
  Hermite-gauge update.

Readings for the second-order fluxes with per-cell gauges (the paper states the
schemes for one gauge): each interface is evaluated once, in the gauge of the
cell to its right (the right ghost for the last one), from its neighbours
moved into that gauge; the cell to its left receives the same flux moved into
its own gauge by T, so the update stays conservative.  The half-step state is
solved from the right cell's beta.  Where it cannot be represented (the solve
certifies non-realizability or does not stay finite) the interface takes the
LLF flux.  The limiter is the van Leer function (r + |r|)/(1 + |r|); the
printed denominator 1 + r agrees with it for r >= 0 and only differs where
the numerator is zero.  The printed ratio r looks one element upwind for waves
moving in +x; the scheme is a centred one, and the moment system carries waves
in both directions (behind a shock, the subsonic side), so the limiter takes
the smaller of phi(r_L) and phi(r_R), r_R being the same ratio one element to
the right (``flic_limiter``).  Then it is TVD for either direction of motion
and the step is symmetric under x -> -x.  The ghost states continue beyond the
boundaries, so the first and the last interface have phi = 0.

Reading for the step size (paper gives only a CFL relation): the step taken at
step k is CFL*dx/max rho from the characteristic speeds of the transport of
step k-1 (ghost cells included); the first step uses a solve of the initial
state.
"""

import math

import numpy as np

from . import basis as _basis
from . import flux as _flux
from . import gauge as _gauge
from . import maxent as _maxent
from . import quadrature as _quad

DIM = 3


def macroscopic(M, g):
    """n, v_x, T, P_xx, P_yy, P_zz, q_x from moments M in gauge g (3D)."""
    M = np.asarray(M, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = M[:, 0]

    def E(expo):
        return (M @ _gauge.monomial_coefficients(expo, DIM)) / n

    ex, exx, eyy, ezz = E((1, 0, 0)), E((2, 0, 0)), E((0, 2, 0)), E((0, 0, 2))
    exxx, exyy, exzz = E((3, 0, 0)), E((1, 2, 0)), E((1, 0, 2))
    w, sx, sr = g[:, 0], g[:, 1], g[:, 2]
    v = w + sx * ex
    Pxx = n * sx ** 2 * (exx - ex ** 2)
    Pyy = n * sr ** 2 * eyy
    Pzz = n * sr ** 2 * ezz
    T = (Pxx + Pyy + Pzz) / (3.0 * n)
    # q_x = 1/2 n E[c_x |c|^2], c = (sx (ux - ex), sr uy, sr uz)
    cxxx = exxx - 3 * ex * exx + 2 * ex ** 3
    cxrr = (exyy + exzz) - ex * (eyy + ezz)
    qx = 0.5 * n * (sx ** 3 * cxxx + sx * sr ** 2 * cxrr)
    return dict(n=n, v=v, T=T, Pxx=Pxx, Pyy=Pyy, Pzz=Pzz, qx=qx)


def gaussian_moments(n, v, Sxx, Srr, g, nq=5):
    """Moments in gauge g of n * N((v, 0, 0), diag(Sxx, Srr, Srr)) by quadrature.

    The integrand is a polynomial of degree <= 4 in the Gaussian's own
    coordinates, so nq >= 3 points per axis integrate it exactly."""
    n, v, Sxx, Srr = (np.atleast_1d(np.asarray(a, dtype=np.float64))
                      for a in (n, v, Sxx, Srr))
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    z, w = _quad.tensor_rule(nq, DIM)
    C, P = n.shape[0], z.shape[0]
    # velocities of the Gaussian's nodes, then their gauge coordinates: (C, P, 3)
    u = np.empty((C, P, DIM))
    u[:, :, 0] = v[:, None] + np.sqrt(Sxx)[:, None] * z[None, :, 0]
    u[:, :, 1] = np.sqrt(Srr)[:, None] * z[None, :, 1]
    u[:, :, 2] = np.sqrt(Srr)[:, None] * z[None, :, 2]
    ub = np.empty_like(u)
    ub[:, :, 0] = (u[:, :, 0] - g[:, None, 0]) / g[:, None, 1]
    ub[:, :, 1] = u[:, :, 1] / g[:, None, 2]
    ub[:, :, 2] = u[:, :, 2] / g[:, None, 2]
    Phi = _basis.evaluate(ub.reshape(-1, DIM), DIM).reshape(C, P, -1)
    return n[:, None] * np.einsum("p,cpi->ci", w, Phi)


def es_bgk_target(M, g, prandtl):
    mac = macroscopic(M, g)
    n, T = mac["n"], mac["T"]
    Sxx = T / prandtl + (1.0 - 1.0 / prandtl) * mac["Pxx"] / n
    Srr = T / prandtl + (1.0 - 1.0 / prandtl) * 0.5 * (mac["Pyy"] + mac["Pzz"]) / n
    return gaussian_moments(n, mac["v"], Sxx, Srr, g), n


def collision(M, g, h, prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi)):
    """M <- (1 - h/tau) M + (h/tau) M~, tau = mu_ref/(Pr n) (Maxwell molecules)."""
    Mt, n = es_bgk_target(M, g, prandtl)
    tau = mu_ref / (prandtl * n)
    r = (h / tau)[:, None]
    return (1.0 - r) * M + r * Mt


def rankine_hugoniot(mach, gamma=5.0 / 3.0):
    """(n, v, T) upstream and downstream, non-dimensional (m=1, n_-=1, T_-=1)."""
    m2 = mach * mach
    ratio = (gamma + 1) * m2 / ((gamma - 1) * m2 + 2)
    tr = ((2 * gamma * m2 - (gamma - 1)) * ((gamma - 1) * m2 + 2)
          / ((gamma + 1) ** 2 * m2))
    v1 = math.sqrt(gamma) * mach
    return (1.0, v1, 1.0), (ratio, v1 / ratio, tr)


def maxwellian_state(n, v, T):
    """Moments, beta and Hermite gauge of a Maxwellian (moments by quadrature)."""
    g = np.array([[v, math.sqrt(T), math.sqrt(T)]])
    M = gaussian_moments(n, v, T, T, g)
    return M, g


def shock_initial(mach, n_cells, x_lo, x_hi, thickness, gamma=5.0 / 3.0):
    """Cell-centred tanh profile of eq. "Mx ini" (moments interpolated in a common gauge)."""
    (n1, v1, T1), (n2, v2, T2) = rankine_hugoniot(mach, gamma)
    gm = np.array([[0.5 * (v1 + v2), 1.0, 1.0]])
    Mm = gaussian_moments(n1, v1, T1, T1, gm)[0]
    Mp = gaussian_moments(n2, v2, T2, T2, gm)[0]
    dx = (x_hi - x_lo) / n_cells
    x = x_lo + dx * (np.arange(n_cells) + 0.5)
    th = thickness / 2.0
    frac = ((np.tanh(x / th) - math.tanh(x_lo / th))
            / (math.tanh(x_hi / th) - math.tanh(x_lo / th)) - 0.5)
    M = (Mp - Mm)[None, :] * frac[:, None] + 0.5 * (Mp + Mm)[None, :]
    g = np.repeat(gm, n_cells, axis=0)
    return M, g, dx


SCHEMES = ("llf", "lw", "flic")


def van_leer(a, b):
    """Van Leer limiter phi(r) = (r + |r|) / (1 + |r|) at r = a / b, elementwise.

    For a b > 0 this is 2 a / (a + b); it is zero where a and b differ in sign
    or either is zero."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros(np.broadcast(a, b).shape)
    pos = a * b > 0
    out[pos] = 2.0 * a[pos] / (a[pos] + b[pos])
    return out


def flic_limiter(d_left, d_mid, d_right):
    """FLIC limiter per moment: min(phi(r_L), phi(r_R)) with the van Leer phi,
    r_L = d_left / d_mid and r_R = d_right / d_mid, where d_mid is the jump
    across the interface and d_left, d_right the jumps one element upwind of it
    on either side (eq. "The FLIC" prints r_L, the upwind ratio of waves moving
    in +x; r_R is the upwind ratio of waves moving in -x)."""
    return np.minimum(van_leer(d_left, d_mid), van_leer(d_right, d_mid))


class FVSolver:
    """Oracle time stepper (Alg. 2) for one 1D problem: cells in their Hermite
    gauges between two fixed ghost Maxwellians.  scheme: "llf", "lw" or "flic";
    collide=False leaves out the relaxation (pure transport)."""

    def __init__(self, M0, g0, dx, left, right, nodes_1d=12, cfl=0.5,
                 prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi), newton=None,
                 scheme="llf", collide=True):
        if scheme not in SCHEMES:
            raise ValueError(f"scheme must be one of {SCHEMES}")
        self.scheme, self.collide = scheme, collide
        self.nodes, w = _quad.tensor_rule(nodes_1d, DIM)
        self.logw = _quad.lebesgue_log_weights(self.nodes, w)
        self.Phi = _basis.evaluate(self.nodes, DIM)
        self.cfl, self.prandtl, self.mu_ref = cfl, prandtl, mu_ref
        self.newton = dict(tol_grad=1e-11, max_iter=100)
        if newton:
            self.newton.update(newton)
        self.dx = dx
        self.M, _, self.g = _gauge.to_hermite_gauge(M0, None, g0, DIM)
        self.beta = _maxent.maxwellian_beta(self.M, DIM)
        # ghost cells: Maxwellians (n, v, T) in their own gauge
        gh = []
        for (n, v, T) in (left, right):
            Mg, gg = maxwellian_state(n, v, T)
            bg = self._solve(Mg, _maxent.maxwellian_beta(Mg, DIM))
            Fg = _flux.fluxes(bg, gg, self.nodes, self.Phi, self.logw)
            rg = _flux.spectral_radius(bg, gg, self.nodes, self.Phi, self.logw)
            gh.append((Mg[0], Fg[0], rg[0], gg[0], bg[0]))
        self.ghost_left, self.ghost_right = gh
        self._start()

    def _start(self):
        self.t = 0.0
        self.beta = self._solve(self.M, self.beta)
        rho = _flux.spectral_radius(self.beta, self.g, self.nodes, self.Phi, self.logw)
        self.dt = self._dt(rho)

    def _solve(self, M, beta):
        """Alg. 1 per cell.  Where the nodes cannot represent a cell's moments (the
        solve certifies non-realizability, or its iterate is not finite) the cell
        takes the Maxwellian of its gauge, so that fluxes and speeds stay defined
        (the paper integrates over a wide fixed velocity box and does not meet this
        case; the GPU step applies the same rule)."""
        out = _maxent.newton_solve(M, beta, self.Phi, self.logw, **self.newton)
        self.last_solve = out
        b = out["beta"]
        ok_M = np.all(np.isfinite(M), axis=1) & (M[:, 0] > 0)
        bad = ok_M & (out["nonrealizable"] | ~np.all(np.isfinite(b), axis=1))
        if np.any(bad):
            b = b.copy()
            b[bad] = _maxent.maxwellian_beta(M[bad], DIM)
        self.maxwell_cells = bad
        return b

    def _dt(self, rho):
        rmax = max(np.max(rho), self.ghost_left[2], self.ghost_right[2])
        return self.cfl * self.dx / rmax

    def _fv(self, M, F, rho, dt):
        N = M.shape[0]
        g = self.g
        MLg, FLg, rL, gL, _ = self.ghost_left
        MRg, FRg, rR, gR, _ = self.ghost_right
        # neighbour data (left and right), each in its own gauge
        Ml = np.vstack([MLg[None], M[:-1]]); Fl = np.vstack([FLg[None], F[:-1]])
        gl = np.vstack([gL[None], g[:-1]]); rl = np.concatenate([[rL], rho[:-1]])
        Mr = np.vstack([M[1:], MRg[None]]); Fr = np.vstack([F[1:], FRg[None]])
        gr = np.vstack([g[1:], gR[None]]); rr = np.concatenate([rho[1:], [rR]])
        Tl = _gauge.change_matrix(g, gl, DIM)
        Tr = _gauge.change_matrix(g, gr, DIM)
        Ml = np.einsum("cij,cj->ci", Tl, Ml); Fl = np.einsum("cij,cj->ci", Tl, Fl)
        Mr = np.einsum("cij,cj->ci", Tr, Mr); Fr = np.einsum("cij,cj->ci", Tr, Fr)
        lm = np.maximum(rl, rho)[:, None]
        lp = np.maximum(rho, rr)[:, None]
        f_minus = 0.5 * (Fl + F) + 0.5 * lm * (Ml - M)
        f_plus = 0.5 * (F + Fr) + 0.5 * lp * (M - Mr)
        return M + dt / self.dx * (f_minus - f_plus)

    def interface_fluxes(self, M, F, beta, rho, dt):
        """Numerical flux at each of the N + 1 interfaces (Sec. 3.4, eqs. "The
        lax F", "The lax W", "The FLIC"), interface j between element j and
        j + 1 of [left ghost, cells, right ghost], in the gauge of element j + 1.
        Returns (fluxes, lw_failed mask)."""
        MLg, FLg, rL, gL, bL = self.ghost_left
        MRg, FRg, rR, gR, bR = self.ghost_right
        Me = np.vstack([MLg[None], M, MRg[None]])
        Fe = np.vstack([FLg[None], F, FRg[None]])
        ge = np.vstack([gL[None], self.g, gR[None]])
        be = np.vstack([bL[None], beta, bR[None]])
        re = np.concatenate([[rL], rho, [rR]])
        N = M.shape[0]
        R = np.arange(1, N + 2)
        L = R - 1
        LL = np.maximum(L - 1, 0)   # the left ghost continues beyond the boundary
        gI = ge[R]
        TL = _gauge.change_matrix(gI, ge[L], DIM)
        ML = np.einsum("cij,cj->ci", TL, Me[L])
        FL = np.einsum("cij,cj->ci", TL, Fe[L])
        MR, FR = Me[R], Fe[R]
        lam = np.maximum(re[L], re[R])[:, None]
        f_lf = 0.5 * (FL + FR) + 0.5 * lam * (ML - MR)
        failed = np.zeros(N + 1, dtype=bool)
        if self.scheme == "llf":
            return f_lf, failed
        # two-step Lax--Wendroff: half-step interface state, its MaxEnt solve
        Mh = 0.5 * (ML + MR) + 0.5 * (dt / self.dx) * (FL - FR)
        out = _maxent.newton_solve(Mh, be[R], self.Phi, self.logw, **self.newton)
        bh = out["beta"]
        failed = (out["nonrealizable"] | ~np.all(np.isfinite(bh), axis=1)
                  | ~np.all(np.isfinite(Mh), axis=1) | ~(Mh[:, 0] > 0))
        bh = np.where(failed[:, None], be[R], bh)
        f_lw = _flux.fluxes(bh, gI, self.nodes, self.Phi, self.logw)
        if self.scheme == "lw":
            phi = np.ones_like(f_lw)
        else:
            # the ratio on either side of the interface, each moved into its gauge;
            # the ghost states continue beyond both boundaries
            RR = np.minimum(R + 1, N + 1)
            TLL = _gauge.change_matrix(gI, ge[LL], DIM)
            MLL = np.einsum("cij,cj->ci", TLL, Me[LL])
            TRR = _gauge.change_matrix(gI, ge[RR], DIM)
            MRR = np.einsum("cij,cj->ci", TRR, Me[RR])
            MRR[RR == R] = MR[RR == R]
            phi = flic_limiter(ML - MLL, MR - ML, MRR - MR)
        f = f_lf + phi * (f_lw - f_lf)
        f[failed] = f_lf[failed]
        return f, failed

    def _fv2(self, M, F, beta, rho, dt):
        """Conservative update from interface fluxes: cell n takes interface n
        (already in its gauge) and interface n + 1 moved from the gauge of its
        right neighbour (eq. "The ME equation fvm 2")."""
        f, failed = self.interface_fluxes(M, F, beta, rho, dt)
        self.lw_failed = failed
        gR = self.ghost_right[3]
        g_right = np.vstack([self.g[1:], gR[None]])
        T = _gauge.change_matrix(self.g, g_right, DIM)
        f_plus = np.einsum("cij,cj->ci", T, f[1:])
        return M + dt / self.dx * (f[:-1] - f_plus)

    def step(self):
        dt = self.dt
        M = self.M
        if self.collide:
            M = collision(M, self.g, 0.5 * dt, self.prandtl, self.mu_ref)
        beta = self._solve(M, self.beta)
        F = _flux.fluxes(beta, self.g, self.nodes, self.Phi, self.logw)
        rho = _flux.spectral_radius(beta, self.g, self.nodes, self.Phi, self.logw)
        # the transport (and the second collision half) never exceed the CFL
        # limit of this step's own speeds; dt came from the previous step's
        dt = min(dt, self._dt(rho))
        if self.scheme == "llf":
            M = self._fv(M, F, rho, dt)
        else:
            M = self._fv2(M, F, beta, rho, dt)
        if self.collide:
            M = collision(M, self.g, 0.5 * dt, self.prandtl, self.mu_ref)
        self.M, self.beta, self.g = _gauge.to_hermite_gauge(M, beta, self.g, DIM)
        self.t += dt
        self.dt = self._dt(rho)
        return dt


class ShockSolver(FVSolver):
    """Oracle time stepper for one normal-shock problem (App. D set-up)."""

    def __init__(self, mach, n_cells, x_lo, x_hi, thickness, nodes_1d=12,
                 cfl=0.5, prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi),
                 gamma=5.0 / 3.0, newton=None, scheme="llf"):
        self.rh = rankine_hugoniot(mach, gamma)
        M0, g0, dx = shock_initial(mach, n_cells, x_lo, x_hi, thickness, gamma)
        super().__init__(M0, g0, dx, self.rh[0], self.rh[1], nodes_1d=nodes_1d, cfl=cfl,
                         prandtl=prandtl, mu_ref=mu_ref, newton=newton, scheme=scheme)
