"""Mesh convergence of the second-order scheme on the paper's own
discretisation (Sec. 4.6, Fig. 6): the Mach-4 normal shock with FLIC on the
nine statistics, at 125, 250, 500 and 1000 cells, stepped together as one
batch (mem_axi_step_batch) until the finest grid reaches t = 40, long after the
profile has settled.  The steady density profiles, centred where n crosses the
mean of the end states, converge as the grid is refined."""
import math

import numpy as np
import pytest
import torch

import mem_inputs
import paper_2303_02898_amd as mem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# the Mach-4 box and domain of the cell-count study
BOX4 = dict(ux_lo=-22.7, ux_hi=16.1, ur_hi=14.5, blocks_x=6, blocks_r=4, order=8)
X_LO, X_HI, THICKNESS = -16.3, 16.3, 5.44


def _tanh_profile(N, states):
    """Moments of the tanh profile between the two states in the gauge
    (mean speed, 1, 1), that gauge, and dx."""
    (n1, v1, T1), (n2, v2, T2) = states
    dx = (X_HI - X_LO) / N
    x = X_LO + dx * (np.arange(N) + 0.5)
    th = THICKNESS / 2.0
    frac = ((np.tanh(x / th) - math.tanh(X_LO / th))
            / (math.tanh(X_HI / th) - math.tanh(X_LO / th)) - 0.5)
    gm = np.array([[0.5 * (v1 + v2), 1.0, 1.0]])
    Mm = mem_inputs.gaussian_moments9(np.array([n1]), np.array([v1]), np.array([T1]),
                                      np.array([T1]), gm)[0]
    Mp = mem_inputs.gaussian_moments9(np.array([n2]), np.array([v2]), np.array([T2]),
                                      np.array([T2]), gm)[0]
    M = (Mp - Mm)[None, :] * frac[:, None] + 0.5 * (Mp + Mm)[None, :]
    return M, np.repeat(gm, N, axis=0), dx


def test_flic_mesh_convergence_on_the_paper_box():
    Ns = [125, 250, 500, 1000]
    print(f"\n[gpu] mesh study: Mach-4 FLIC on the box, {Ns} cells in one batch", flush=True)
    states = tuple(tuple(float(a) for a in s) for s in mem_inputs.rankine_hugoniot(4.0))
    (n1, _, _), (n2, _, _) = states
    parts = [_tanh_profile(N, states) for N in Ns]
    r = mem.AxiRule(**BOX4)
    Md = torch.tensor(np.concatenate([p[0] for p in parts]).astype(np.float32), device=DEV)
    gd = torch.tensor(np.concatenate([p[1] for p in parts]).astype(np.float32), device=DEV)
    r.gauge(Md, None, gd)
    b0 = np.zeros((Md.shape[0], 9), np.float32)
    b0[:, 2] = -1.0 / math.sqrt(2.0)
    b0[:, 3] = -1.0
    bd = torch.tensor(b0, device=DEV)
    bd[:, 0] = Md[:, 0]
    off = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
    P = len(Ns)
    offd = torch.tensor(off, device=DEV)
    dxd = torch.tensor([p[2] for p in parts], dtype=torch.float32, device=DEV)
    ghd = torch.tensor([[a for s in states for a in s]] * P, dtype=torch.float32, device=DEV)
    t = torch.zeros(P, device=DEV)
    dt = torch.zeros(P, device=DEV)
    st = torch.zeros(int(off[-1]), dtype=torch.int32, device=DEV)
    r.reserve(int(off[-1]), P)
    args = (Md, bd, gd, t, dt, offd, dxd, ghd)
    r.step_batch(*args, n_steps=0, scheme="flic")
    steps = 0
    while t.min().item() < 40.0 and steps < 200000:
        r.step_batch(*args, n_steps=5000, status=st, scheme="flic", use_graph=True)
        steps += 5000
        print(f"  {steps} steps, t = {np.round(t.cpu().numpy(), 2).tolist()}", flush=True)
    M = Md.cpu().numpy().astype(np.float64)
    s = st.cpu().numpy()
    r.close()
    assert t.min().item() >= 40.0
    assert np.all(np.isfinite(M))
    assert np.all(s & (mem.ST_CONVERGED | mem.ST_STAGNATED)), "every last solve ends usable"
    # centred density profiles on a common grid
    xs = np.linspace(-8.0, 8.0, 801)
    mid = 0.5 * (n1 + n2)
    prof = []
    for p, N in enumerate(Ns):
        n = M[off[p]:off[p + 1], 0]
        x = X_LO + parts[p][2] * (np.arange(N) + 0.5)
        k = int(np.argmax(n >= mid))
        xc = x[k - 1] + (mid - n[k - 1]) * (x[k] - x[k - 1]) / (n[k] - n[k - 1])
        prof.append(np.interp(xs + xc, x, n))
    d = [float(np.max(np.abs(prof[p] - prof[p + 1])) / (n2 - n1)) for p in range(P - 1)]
    order = [math.log2(d[p] / d[p + 1]) for p in range(P - 2)]
    print(f"  max |n_N - n_2N| / (n2 - n1): {['%.2e' % v for v in d]}, observed order "
          f"{['%.2f' % v for v in order]}", flush=True)
    assert d[0] > d[1] > d[2]
    assert min(order) >= 1.0
    assert d[-1] <= 5e-4
