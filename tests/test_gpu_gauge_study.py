"""The gauge experiment of Sec. 4.3 (the Hermite gauge against a fixed one),
on the 35-moment Gauss-Hermite discretisation: upstream
Maxwellians of normal shocks for Mach 2..12 (n = 1, T = 1, v = sqrt(5/3) Ma),
solved in FP32 from the uniform start (beta_i = 0 for i >= 1) once in the
Hermite gauge of each state and once in the fixed gauge (0, 1, 1), against the
FP64 oracle's solution of the same discrete problems.

What the paper reports and this checks: in the Hermite gauge the iteration
count does not depend on the Mach number and the FP32 parameters sit close to
FP64; without the gauge the solve is slower and less accurate and, here, the
12^3 Gauss-Hermite nodes stop representing the state from Mach 4 on (Mach >= 5
certified by both sides).
"""

import math

import numpy as np
import pytest
import torch

import mem_inputs
import paper_2303_02898_amd as mem
from oracle import basis, maxent, quadrature

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ctx3():
    c = mem.Context(3, 12)
    yield c
    c.close()


def _study(ctx, gauge):
    machs = np.arange(2, 13, dtype=np.float64)
    v = math.sqrt(5.0 / 3.0) * machs
    N = machs.size
    w = v if gauge == "hermite" else np.zeros(N)
    g = np.stack([w, np.ones(N), np.ones(N)], axis=1)
    M = mem_inputs.gaussian_moments(np.ones(N), v, np.ones(N), np.ones(N), g)
    b0 = np.zeros((N, 35))
    b0[:, 0] = 1.0
    Md = torch.tensor(M.astype(np.float32), device=DEV)
    bd = torch.tensor(b0.astype(np.float32), device=DEV)
    it = torch.zeros(N, dtype=torch.int32, device=DEV)
    rs = torch.zeros(N, device=DEV)
    st = torch.zeros(N, dtype=torch.int32, device=DEV)
    ctx.solve(Md, bd, iters=it, resid=rs, status=st)
    torch.cuda.synchronize()
    nodes, wq = quadrature.tensor_rule(12, 3)
    logw = quadrature.lebesgue_log_weights(nodes, wq)
    Phi = basis.evaluate(nodes, 3)
    o = maxent.newton_solve(M, b0, Phi, logw, tol_grad=1e-12, max_iter=400)
    beta = bd.cpu().numpy().astype(np.float64)
    mse = np.mean((beta[:, 1:] - o["beta"][:, 1:]) ** 2, axis=1)
    return machs, it.cpu().numpy(), st.cpu().numpy(), rs.cpu().numpy(), beta, o, mse


def test_hermite_gauge_is_mach_independent_and_accurate(ctx3):
    machs, it, st, rs, beta, o, mse = _study(ctx3, "hermite")
    print(f"\n[hermite] iterations {it.tolist()}, log10 MSE {np.round(np.log10(mse), 2).tolist()}")
    assert np.all(o["converged"])
    assert np.all(st & mem.ST_CONVERGED)
    assert it.max() - it.min() <= 1 and it.max() <= 13
    assert np.all(rs <= 2e-6)
    assert np.all(np.log10(mse) < -11.5)
    # the solution is the state's Maxwellian (closed form in its own gauge)
    assert np.allclose(beta[:, [4, 7, 9]], -math.sqrt(0.5), atol=1e-4)
    assert np.max(np.abs(np.delete(beta[:, 1:], [3, 6, 8], axis=1))) < 1e-4


def test_fixed_gauge_is_slower_less_accurate_and_fails_at_high_mach(ctx3):
    machs, it_h, _, _, _, _, mse_h = _study(ctx3, "hermite")
    machs, it, st, rs, beta, o, mse = _study(ctx3, "lab")
    print(f"\n[fixed gauge] iterations {it.tolist()}, status {[hex(s) for s in st]}, "
          f"log10 MSE {np.round(np.log10(mse + 1e-300), 2).tolist()}")
    # Mach 2: converges, but FP32 lands further from FP64: by 1.5 orders of
    # magnitude in the MSE with the persistent solver's sum-factorised
    # assembly (over 2 with the MFMA assembly, whose rounding differs)
    assert st[0] & mem.ST_CONVERGED and it[0] >= it_h[0]
    assert math.log10(mse[0]) > math.log10(mse_h[0]) + 1.0
    # Mach 3: converges in FP64 only, after more iterations than in the Hermite gauge
    assert o["converged"][1] and o["iters"][1] > 13
    assert it[1] > it_h[1]
    # Mach >= 4: no FP32 solution; where the oracle certifies non-realizability the
    # GPU reports it too
    assert not np.any(st[2:] & mem.ST_CONVERGED)
    assert np.all(o["nonrealizable"][3:])
    assert np.all(st[3:] & mem.ST_NONREALIZABLE)


def test_gauge_study_on_the_paper_box():
    """Sec. 4.3 on the paper's own box ([-30.7, 37.3] x [0, 34.0], 16 x 16 blocks
    of 8 x 8 Gauss-Legendre points): upstream Maxwellians of Mach 2..12 solved in
    FP32 by the nine-statistic solver from the uniform distribution (beta_i = 0,
    i >= 1), once in the Hermite gauge of each state and once in the fixed gauge
    (0, 1, 1), tolerance 1e-6, against the FP64 oracle of the same problems.
    The paper states its experiment with the Maxwell family {1, u_x, u_x^2,
    u_r^2}; the nine statistics contain it, so the solution is the same with the
    other five multipliers at zero.  As in Fig. 3: in the Hermite gauge the
    iterations stay within a narrow band and FP32 lands on FP64; in the fixed
    gauge they climb and scatter with the Mach number and FP32 drifts far from
    FP64 (from about Mach 7 on it does not converge)."""
    from oracle import axisym
    box = mem_inputs.E1_BOX
    r = mem.AxiRule(**box)
    orule = axisym.blockwise_rule(**box)
    machs = np.arange(2, 13, dtype=np.float64)
    N = machs.size
    v = math.sqrt(5.0 / 3.0) * machs
    out = {}
    for gauge in ("hermite", "fixed"):
        w = v if gauge == "hermite" else np.zeros(N)
        g = np.stack([w, np.ones(N), np.ones(N)], axis=1)
        M = mem_inputs.gaussian_moments9(np.ones(N), v, np.ones(N), np.ones(N), g)
        b0 = np.zeros((N, 9))
        b0[:, 0] = 1.0
        o = axisym.solve(M, g, b0, orule, tol_grad=1e-12, max_iter=500)
        assert np.all(o["converged"])
        opts = mem.default_opts(tol_grad=1e-6, max_iter=500)
        Md = torch.tensor(M.astype(np.float32), device=DEV)
        gd = torch.tensor(g.astype(np.float32), device=DEV)
        bd = torch.tensor(b0.astype(np.float32), device=DEV)
        it, rs, st = r.solve(Md, gd, bd, opts=opts)
        torch.cuda.synchronize()
        beta = bd.cpu().numpy().astype(np.float64)
        lmse = np.log10(np.mean((beta[:, 1:] - o["beta"][:, 1:]) ** 2, axis=1) + 1e-300)
        out[gauge] = (it.cpu().numpy(), st.cpu().numpy(), lmse)
        print(f"\n[box gauge study, {gauge}] iterations {it.cpu().tolist()}, log10 MSE "
              f"{np.round(lmse, 2).tolist()}")
    r.close()
    it_h, st_h, l_h = out["hermite"]
    it_f, st_f, l_f = out["fixed"]
    assert np.all(st_h & mem.ST_CONVERGED)
    assert l_h.max() < -13.0
    assert it_h.max() <= 35 and it_h.max() - it_h.min() <= 10
    assert l_f[0] < -10.0                       # Mach 2 still converges without the gauge
    assert np.all(l_f[machs >= 7] > -4.0)       # far from FP64 beyond Mach 7
    assert not np.all(st_f & mem.ST_CONVERGED)
    assert np.sum(it_f > it_h) >= 8
