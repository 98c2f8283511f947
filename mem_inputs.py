"""Seeded synthetic workloads for the MEM hot path.

This module is the only one read by both the FP64 oracle (``oracle/``) and the
HIP library's users (tests, ``bench.py``).  It holds the random draws and the
physical description of each workload -- Gaussian mixtures, shock states,
initial profiles -- but none of the method's arithmetic: no partition function,
no MaxEnt solve, no gauge transform, no flux.

Target moments of Gaussian (mixture) states are the *definition* of the input
and are written in closed form: for X ~ N(mu, s^2),
E[He_n(X)] = h_n(mu; s^2 - 1) with h_n(b; c) = sum_j C(n, 2j) (2j-1)!! c^j b^(n-2j).
Moments are returned in FP64 and in the orthonormal Hermite basis
phi_(a,b,c)(u_bar) = He_a He_b He_c / sqrt(a! b! c!), a+b+c <= 4, ordered by total
degree then lexicographically descending; gauge coordinates
u_bar = ((u_x - w)/s_x, u_y/s_r, u_z/s_r).

Workloads (seed = 1000*config + replica):

1. ``config1_candidates``: 1D, 5 moments; per cell n ~ U(0.5, 2),
   v ~ N(0, 1), T ~ U(0.5, 2), perturbation of the He_3/He_4 multipliers of
   the standardised Maxwellian: c3 ~ N(0, 0.05), c4 = -|N(0, 0.05)|.  A pool
   of candidates in a fixed order; the targets (64-node quadrature of the
   perturbed density) are built by whoever evaluates the density.
2. ``mott_smith_cells``: 3D, 35 moments; Mach ~ U(lo, hi), mixing weight
   nu ~ U(0, 1), gamma = 5/3; f = (1-nu) f_M(upstream) + nu f_M(downstream)
   with Rankine--Hugoniot downstream states; targets in the mixture's exact
   Hermite gauge (its mean and standard deviations).
3. ``shock_problem``: Mach-3 normal shock, tanh initial profile of the
   upstream/downstream Maxwellian moments in a common gauge, Maxwellian
   boundary states in their own gauges.
5. ``ragged_batch``: many shock problems with log-uniform cell counts.
6. ``mott_smith_cells9``: the Mott-Smith mixtures of workload 2 on the paper's
   nine statistics of (u_x, u_r), by default at Mach 10 (the paper's Mach-10
   shock; its box ``AXI_MACH10_BOX``).
7. ``overflow_samples``: parameters drawn around the equilibrium n = 1, v = 0,
   T = 1 (standard deviation 0.1 in every component) in the canonical and in
   the non-canonical form of the nine-statistic family, on the box
   ``E1_BOX`` (the overflow experiment of Sec. 4.1, Fig. 1).
"""

import math

import numpy as np

GAMMA = 5.0 / 3.0
MU_REF = math.sqrt(2.0 / math.pi)   # viscosity at T = 1 for Kn = 1 (non-dim units)


def seed_for(config, replica=0):
    return 1000 * config + replica


def multi_indices(dim, degree=4):
    out = []
    for tot in range(degree + 1):
        if dim == 1:
            out.append((tot,))
            continue
        for a in range(tot, -1, -1):
            for b in range(tot - a, -1, -1):
                out.append((a, b, tot - a - b))
    return out


def _double_factorial_odd(k):
    """(2j-1)!! for k = 2j-1 >= -1."""
    r = 1
    while k > 1:
        r *= k
        k -= 2
    return r


def hermite_gauss_moment(m, mean, var):
    """E[He_m(X)] for X ~ N(mean, var), elementwise over arrays."""
    mean = np.asarray(mean, dtype=np.float64)
    c = np.asarray(var, dtype=np.float64) - 1.0
    out = np.zeros(np.broadcast(mean, c).shape)
    for j in range(m // 2 + 1):
        coef = math.comb(m, 2 * j) * _double_factorial_odd(2 * j - 1)
        out = out + coef * c ** j * mean ** (m - 2 * j)
    return out


def gaussian_moments(n, v, Txx, Trr, g):
    """Moments in gauge g of n * N((v,0,0), diag(Txx, Trr, Trr)); arrays over cells."""
    n, v, Txx, Trr = (np.asarray(a, dtype=np.float64) for a in (n, v, Txx, Trr))
    g = np.asarray(g, dtype=np.float64)
    mx = (v - g[:, 0]) / g[:, 1]
    vx = Txx / g[:, 1] ** 2
    vr = Trr / g[:, 2] ** 2
    hx = [hermite_gauss_moment(k, mx, vx) for k in range(5)]
    hr = [hermite_gauss_moment(k, 0.0 * mx, vr) for k in range(5)]
    idx = multi_indices(3)
    M = np.empty((n.shape[0], len(idx)))
    for i, (a, b, c) in enumerate(idx):
        norm = math.sqrt(math.factorial(a) * math.factorial(b) * math.factorial(c))
        M[:, i] = n * hx[a] * hr[b] * hr[c] / norm
    return M


def rankine_hugoniot(mach, gamma=GAMMA):
    """Upstream/downstream (n, v, T); non-dimensional m = 1, n_- = 1, T_- = 1."""
    mach = np.asarray(mach, dtype=np.float64)
    m2 = mach * mach
    ratio = (gamma + 1) * m2 / ((gamma - 1) * m2 + 2)
    tr = ((2 * gamma * m2 - (gamma - 1)) * ((gamma - 1) * m2 + 2)
          / ((gamma + 1) ** 2 * m2))
    v1 = math.sqrt(gamma) * mach
    one = np.ones_like(mach)
    return (one, v1, one), (ratio, v1 / ratio, tr)


# --------------------------------------------------------------------------
# workload 1: 1D perturbed Maxwellians (targets built by the density evaluator)
# --------------------------------------------------------------------------
def mixture_1d(n_cells, replica=0):
    """1D two-Gaussian mixtures given in their own Hermite gauge (closed form).

    Weights nu ~ U(0, 1), densities n ~ U(0.5, 2), component means ~ N(0, 1),
    variances ~ U(0.5, 2).  Returns M [n_cells][5] (orthonormal He_k / sqrt(k!)
    moments times the density) and g [n_cells][2] = (mean, standard deviation).
    """
    rng = np.random.default_rng(seed_for(1, 100 + replica))
    n = rng.uniform(0.5, 2.0, n_cells)
    nu = rng.uniform(0.0, 1.0, n_cells)
    v1, v2 = rng.normal(0.0, 1.0, n_cells), rng.normal(0.0, 1.0, n_cells)
    T1, T2 = rng.uniform(0.5, 2.0, n_cells), rng.uniform(0.5, 2.0, n_cells)
    mean = (1 - nu) * v1 + nu * v2
    var = (1 - nu) * (T1 + v1 ** 2) + nu * (T2 + v2 ** 2) - mean ** 2
    s = np.sqrt(var)
    M = np.zeros((n_cells, 5))
    for k in range(5):
        e1 = hermite_gauss_moment(k, (v1 - mean) / s, T1 / var)
        e2 = hermite_gauss_moment(k, (v2 - mean) / s, T2 / var)
        M[:, k] = n * ((1 - nu) * e1 + nu * e2) / math.sqrt(math.factorial(k))
    return dict(M=M, g=np.stack([mean, s], axis=1))


def config1_candidates(n_pool=4096, replica=0):
    rng = np.random.default_rng(seed_for(1, replica))
    n = rng.uniform(0.5, 2.0, n_pool)
    v = rng.normal(0.0, 1.0, n_pool)
    T = rng.uniform(0.5, 2.0, n_pool)
    c3 = rng.normal(0.0, 0.05, n_pool)
    c4 = -np.abs(rng.normal(0.0, 0.05, n_pool))
    return dict(n=n, v=v, T=T, c3=c3, c4=c4)


# --------------------------------------------------------------------------
# workload 2 / 4: Mott-Smith mixtures in their Hermite gauge
# --------------------------------------------------------------------------
def mott_smith_cells(n_cells, mach_lo=1.5, mach_hi=10.0, config=2, replica=0):
    rng = np.random.default_rng(seed_for(config, replica))
    mach = rng.uniform(mach_lo, mach_hi, n_cells)
    nu = rng.uniform(0.0, 1.0, n_cells)
    (n1, v1, T1), (n2, v2, T2) = rankine_hugoniot(mach)
    a1, a2 = (1.0 - nu) * n1, nu * n2
    N = a1 + a2
    mean = (a1 * v1 + a2 * v2) / N
    varx = (a1 * (T1 + v1 ** 2) + a2 * (T2 + v2 ** 2)) / N - mean ** 2
    varr = (a1 * T1 + a2 * T2) / N
    g = np.stack([mean, np.sqrt(varx), np.sqrt(varr)], axis=1)
    M = ((1.0 - nu)[:, None] * gaussian_moments(n1, v1, T1, T1, g)
         + nu[:, None] * gaussian_moments(n2, v2, T2, T2, g))
    return dict(M=M, g=g, mach=mach, nu=nu)


def maxwellian_beta(n_cells, K, n=None):
    """Cold start: the Maxwellian in the cell's Hermite gauge (beta_0 = n)."""
    beta = np.zeros((n_cells, K))
    if n is not None:
        beta[:, 0] = n
    idx = multi_indices(3 if K == 35 else 1)
    for i, e in enumerate(idx):
        if sum(e) == 2 and max(e) == 2:
            beta[:, i] = -1.0 / math.sqrt(2.0)
    return beta


# --------------------------------------------------------------------------
# workload 3 / 5: normal shocks
# --------------------------------------------------------------------------
def shock_problem(mach=3.0, n_cells=1000, x_lo=-20.0, x_hi=20.0, thickness=5.44):
    """Initial moments (common gauge), boundary Maxwellians and grid spacing."""
    (n1, v1, T1), (n2, v2, T2) = (tuple(float(x) for x in s)
                                  for s in rankine_hugoniot(np.array(mach)))
    gm = np.array([[0.5 * (v1 + v2), 1.0, 1.0]])
    Mm = gaussian_moments(np.array([n1]), np.array([v1]), np.array([T1]), np.array([T1]), gm)[0]
    Mp = gaussian_moments(np.array([n2]), np.array([v2]), np.array([T2]), np.array([T2]), gm)[0]
    dx = (x_hi - x_lo) / n_cells
    x = x_lo + dx * (np.arange(n_cells) + 0.5)
    th = thickness / 2.0
    frac = ((np.tanh(x / th) - math.tanh(x_lo / th))
            / (math.tanh(x_hi / th) - math.tanh(x_lo / th)) - 0.5)
    M = (Mp - Mm)[None, :] * frac[:, None] + 0.5 * (Mp + Mm)[None, :]
    g = np.repeat(gm, n_cells, axis=0)
    gL = np.array([v1, math.sqrt(T1), math.sqrt(T1)])
    gR = np.array([v2, math.sqrt(T2), math.sqrt(T2)])
    ML = np.zeros(35); ML[0] = n1
    MR = np.zeros(35); MR[0] = n2
    return dict(M=M, g=g, dx=dx, x=x, M_left=ML, M_right=MR, g_left=gL, g_right=gR,
                states=((n1, v1, T1), (n2, v2, T2)))


def ragged_batch(n_problems=2048, lo=64, hi=4096, mach_lo=1.2, mach_hi=10.0,
                 dx=1.0, thickness=10.0, replica=0):
    """Independent shocks with log-uniform cell counts, concatenated."""
    rng = np.random.default_rng(seed_for(5, replica))
    counts = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_problems))).astype(np.int64)
    mach = rng.uniform(mach_lo, mach_hi, n_problems)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    probs = []
    for p in range(n_problems):
        half = 0.5 * counts[p] * dx
        probs.append(shock_problem(mach[p], int(counts[p]), -half, half, thickness))
    return dict(counts=counts, mach=mach, offsets=offsets, problems=probs, dx=dx)


# --------------------------------------------------------------------------
# the paper's own discretisation: nine statistics of (u_x, u_r) on a
# block-wise Gauss--Legendre box fixed in physical velocity
# --------------------------------------------------------------------------
# The Mach-10 shock set-up: box [-24.8, 31.4] x [0, 28.1], 6 x 4 blocks of
# 8 x 8 Gauss--Legendre points (1536 nodes).
AXI_MACH10_BOX = dict(ux_lo=-24.8, ux_hi=31.4, ur_hi=28.1, blocks_x=6, blocks_r=4, order=8)


def gaussian_moments9(n, v, Txx, Trr, g):
    """Nine moments in gauge g of n * N((v,0,0), diag(Txx, Trr, Trr)).

    With x = u_bar_x ~ N(mu, s^2) and y = u_bar_r^2/2 ~ Exp(mean theta),
    theta = Trr/s_r^2, independent: E[He_k(x)] = h_k(mu; s^2 - 1),
    E[y - 1] = theta - 1, E[y^2/2 - 2y + 1] = (theta - 1)^2.  Statistic order:
    1, x, He_2/sqrt2, y-1, He_3/sqrt6, He_4/sqrt24, y^2/2-2y+1, x(y-1),
    He_2/sqrt2 (y-1).
    """
    n, v, Txx, Trr = (np.asarray(a, dtype=np.float64) for a in (n, v, Txx, Trr))
    g = np.asarray(g, dtype=np.float64)
    mx = (v - g[:, 0]) / g[:, 1]
    hx = [hermite_gauss_moment(k, mx, Txx / g[:, 1] ** 2) for k in range(5)]
    th = Trr / g[:, 2] ** 2
    l1, l2 = th - 1.0, (th - 1.0) ** 2
    one = np.ones_like(mx)
    cols = [one, hx[1], hx[2] / math.sqrt(2.0), l1, hx[3] / math.sqrt(6.0),
            hx[4] / math.sqrt(24.0), l2, hx[1] * l1, hx[2] / math.sqrt(2.0) * l1]
    return n[:, None] * np.stack(cols, axis=1)


def mott_smith_cells9(n_cells, mach_lo=10.0, mach_hi=10.0, config=6, replica=0):
    """Mott-Smith mixtures (as ``mott_smith_cells``) on the nine statistics,
    in the mixture's exact Hermite gauge."""
    rng = np.random.default_rng(seed_for(config, replica))
    mach = rng.uniform(mach_lo, mach_hi, n_cells)
    nu = rng.uniform(0.0, 1.0, n_cells)
    (n1, v1, T1), (n2, v2, T2) = rankine_hugoniot(mach)
    a1, a2 = (1.0 - nu) * n1, nu * n2
    N = a1 + a2
    mean = (a1 * v1 + a2 * v2) / N
    varx = (a1 * (T1 + v1 ** 2) + a2 * (T2 + v2 ** 2)) / N - mean ** 2
    varr = (a1 * T1 + a2 * T2) / N
    g = np.stack([mean, np.sqrt(varx), np.sqrt(varr)], axis=1)
    M = ((1.0 - nu)[:, None] * gaussian_moments9(n1, v1, T1, T1, g)
         + nu[:, None] * gaussian_moments9(n2, v2, T2, T2, g))
    return dict(M=M, g=g, mach=mach, nu=nu)


# --------------------------------------------------------------------------
# overflow experiment (Sec. 4.1, Fig. 1): random parameters about equilibrium
# --------------------------------------------------------------------------
# Box [-30.7, 37.3] x [0, 34.0], 16 x 16 blocks of 8 x 8 Gauss--Legendre
# points (16,384 nodes), trivial gauge (0, 1, 1).
E1_BOX = dict(ux_lo=-30.7, ux_hi=37.3, ur_hi=34.0, blocks_x=16, blocks_r=16, order=8)


def overflow_samples(n_samples, sigma=0.1, config=7, replica=0):
    """Parameters of the nine-statistic family about the equilibrium n = 1,
    v = 0, T = 1 in the gauge (0, 1, 1).

    The equilibrium density n (2 pi)^(-3/2) exp(-|u|^2 / 2) written with the
    statistics (He_2(x)/sqrt2 and y - 1 carry -|u|^2/2 up to a constant):
      canonical      beta  = (n, 0, -1/sqrt2, -1, 0, 0, 0, 0, 0),
      non-canonical  alpha = (log n - 3/2 (log(2 pi) + 1), 0, -1/sqrt2, -1, 0, ...),
    alpha_0 being the log of the Maxwellian's normalisation.  Every component
    of each form gets an independent N(0, sigma^2) draw (separate draws for
    the two forms)."""
    rng = np.random.default_rng(seed_for(config, replica))
    centre_b = np.array([1.0, 0.0, -1.0 / math.sqrt(2.0), -1.0, 0, 0, 0, 0, 0])
    centre_a = centre_b.copy()
    centre_a[0] = -1.5 * (math.log(2.0 * math.pi) + 1.0)
    beta = centre_b + sigma * rng.normal(size=(n_samples, 9))
    alpha = centre_a + sigma * rng.normal(size=(n_samples, 9))
    return dict(beta=beta, alpha=alpha, g=np.tile([0.0, 1.0, 1.0], (n_samples, 1)),
                centre_beta=centre_b, centre_alpha=centre_a)
