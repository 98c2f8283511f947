"""GPU parity of the mixed-precision (BF16 / FP16 hi+lo) assembly and solve.

The moment columns (0, j) come from FP32 products, so E[phi] keeps the FP32
error bound; the other pair columns of S = sigma . Psi are sums of hi*hi +
hi*lo + lo*hi 16-bit products with FP32 accumulation, whose representation
error is bounded per node:
  BF16 (8 significant bits per part): |d(sigma Psi)| <= 4 * 2^-18 sigma |Psi|;
  FP16 (11 bits, subnormals below 2^-14, node scale 2^k_p):
      |d(sigma Psi)| <= 4 * 2^-22 sigma |Psi| + sigma min(|Psi|, 2^-25 2^k_p)
                        + |Psi| min(sigma, 2^-25 2^-k_p).
The solve must meet the same bars as the FP32 path: residual <= 1e-5
(FP32-floor-aware) and beta within 1e-4 of the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import mem_inputs
import paper_2303_02898_amd as mem
from oracle import basis, maxent

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PRECS = ("bf16x3", "fp16x3")


def dev(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.fixture(scope="module", params=PRECS)
def ctxm(request):
    print(f"\n[gpu] creating 3D context (12^3 nodes, {request.param})", flush=True)
    c = mem.Context(3, 12, request.param)
    c.prec_name = request.param
    yield c
    c.close()


def _decaying_beta(rng, C):
    beta = mem_inputs.maxwellian_beta(C, 35, rng.uniform(0.5, 2.0, C))
    beta[:, 1:20] += 0.05 * rng.normal(size=(C, 19))
    for i, e in enumerate(basis.multi_indices(3)):
        if sum(e) == 4 and max(e) == 4:
            beta[:, i] = -0.04
    return f32(beta)


def test_mixed_dual_within_split_bound(ctxm, rule3):
    rng = np.random.default_rng(111)
    C = 200
    beta = _decaying_beta(rng, C)
    logZ, E, H = ctxm.dual(dev(beta))
    torch.cuda.synchronize()
    Phi, logw, w = rule3["Phi"], rule3["logw"], rule3["w"]
    sig = maxent.sigma(beta, Phi, logw)
    E_o = sig @ Phi
    H_o = maxent.hessian(beta, np.repeat(beta[:, :1], 35, 1), Phi, logw)[:, 1:, 1:]
    u = 2.0 ** -24
    de = 36 * u * (np.abs(logw)[None, :] + np.abs(beta[:, 1:]) @ np.abs(Phi[:, 1:]).T)
    # moments: FP32 products, same bound as the FP32 path
    bound_E = (sig * de) @ np.abs(Phi) + 1728 * u * (sig @ np.abs(Phi))
    errE = np.abs(E.cpu().numpy() - E_o)
    print(f"[{ctxm.prec_name}] E err/bound max {np.max(errE / bound_E):.3f}")
    assert np.all(errE <= bound_E + 1e-7)
    # pair columns: split-representation bound + FP32 exponent and sums
    aP = np.abs(Phi[:, 1:])
    pair = aP[:, :, None] * aP[:, None, :]                       # |Psi_p,ij|, (Q, 34, 34)
    A = np.einsum("cp,pij->cij", sig * (1.0 + de), pair)         # sum_p sigma_p |Psi|
    if ctxm.prec_name == "bf16x3":
        rep = 4 * 2.0 ** -18 * A
    else:
        k = np.clip(np.floor(-np.log2(w)), 0, 15)
        # subnormal parts: absolute error 2^-25 in scaled units, never more than the value
        d_psi = np.minimum(pair, (2.0 ** -25 * 2.0 ** k)[:, None, None])
        d_sig = np.minimum(sig, (2.0 ** -25 * 2.0 ** -k)[None, :])
        rep = (4 * 2.0 ** -22 * A + np.einsum("cp,pij->cij", sig, d_psi)
               + np.einsum("cp,pij->cij", d_sig, pair))
    fp32 = np.einsum("cp,pij->cij", sig * de, pair) + 1728 * u * A
    # H = S_ij / S_00 - E_i E_j: the E_i E_j term carries the FP32 moment bound
    ee = bound_E[:, 1:, None] * np.abs(E_o[:, None, 1:]) + np.abs(E_o[:, 1:, None]) * bound_E[:, None, 1:]
    bound_H = 2.0 * (rep + fp32 + ee) + 1e-7
    errH = np.abs(H.cpu().numpy() - H_o)
    ratio = errH / bound_H
    print(f"[{ctxm.prec_name}] H err max {errH.max():.2e}, err/bound max {ratio.max():.3f}")
    assert np.all(ratio <= 1.0)


def _solve(ctx, M, b0):
    bg = dev(b0)
    iters, resid, status = ctx.solve(dev(M), bg)
    torch.cuda.synchronize()
    return (bg.cpu().numpy().astype(np.float64), iters.cpu().numpy(), resid.cpu().numpy(),
            status.cpu().numpy())


@pytest.mark.parametrize("config,mach", [(2, (1.5, 10.0)), (4, (5.0, 10.0))])
def test_mixed_solve_matches_oracle(ctxm, rule3, config, mach):
    C = 333
    cells = mem_inputs.mott_smith_cells(C, mach[0], mach[1], config=config, replica=7)
    M = f32(cells["M"])
    b0 = f32(mem_inputs.maxwellian_beta(C, 35, M[:, 0]))
    beta, it, res, st = _solve(ctxm, M, b0)
    ref = maxent.newton_solve(M, b0, rule3["Phi"], rule3["logw"])
    good = ref["converged"]
    bad = ref["nonrealizable"]
    assert np.all(good | bad)
    conv = (st & mem.ST_CONVERGED) != 0
    assert np.mean(conv[good]) >= 0.99
    assert np.all(st[good & ~conv] & mem.ST_STAGNATED)
    assert not np.any(conv[bad])
    sel = good & conv
    r = maxent.moment_residual(beta[sel], M[sel], rule3["Phi"], rule3["logw"])
    floor = maxent.moment_residual(f32(ref["beta"][sel]), M[sel], rule3["Phi"], rule3["logw"])
    bar = np.maximum(1e-5, 2.0 * floor)
    scale = np.maximum(1.0, np.max(np.abs(ref["beta"][sel]), axis=1))
    berr = np.max(np.abs(beta[sel] - ref["beta"][sel]), axis=1) / scale
    print(f"[{ctxm.prec_name} config {config}] converged {conv[good].mean():.3f} of "
          f"{good.sum()} realizable; r max {r.max():.2e} (r/bar {np.max(r / bar):.2f}); "
          f"beta err max {berr.max():.2e}; iterations mean {it.mean():.1f} max {it.max()}",
          flush=True)
    assert np.all(r <= bar)
    assert berr.max() <= 1e-4
    # the library's own residual is the compensated one: it must agree with FP64
    dr = np.abs(res[sel] - r)
    print(f"[{ctxm.prec_name} config {config}] |resid - r_fp64| max {dr.max():.2e}")
    assert np.all(dr <= 2e-7 + 0.01 * r)


def test_mixed_full_size_sampled(ctxm, rule3):
    """The full mixed-precision workload (262,144 Mott-Smith cells, Mach 5-10,
    12^3 nodes) in one solve: its own compensated residual on every cell, and
    48 sampled cells against the FP64 oracle at the same bars as the FP32 path."""
    C = 262144
    cells = mem_inputs.mott_smith_cells(C, 5.0, 10.0, config=4, replica=0)
    M = f32(cells["M"])
    b0 = f32(mem_inputs.maxwellian_beta(C, 35, M[:, 0]))
    print(f"\n[{ctxm.prec_name} full] {C} cells", flush=True)
    beta, it, res, st = _solve(ctxm, M, b0)
    conv = (st & mem.ST_CONVERGED) != 0
    nonreal = (st & mem.ST_NONREALIZABLE) != 0
    print(f"[{ctxm.prec_name} full] converged {conv.mean():.5f}, certified non-realizable "
          f"{nonreal.mean():.5f}, fp64 direction {np.mean((st & mem.ST_FP64) != 0):.4f}, "
          f"iterations mean {it.mean():.2f} max {it.max()}", flush=True)
    assert np.all(res[conv] <= 1e-5)
    assert np.mean(conv | nonreal) >= 0.99
    rng = np.random.default_rng(48)
    idx = np.sort(rng.choice(C, 48, replace=False))
    ref = maxent.newton_solve(M[idx], b0[idx], rule3["Phi"], rule3["logw"])
    good, bad = ref["converged"], ref["nonrealizable"]
    assert np.all(good | bad)
    assert not np.any(conv[idx][bad])
    sel = good & conv[idx]
    assert sel.sum() >= 0.95 * good.sum()
    Ms, bs, rs = M[idx][sel], beta[idx][sel], ref["beta"][sel]
    r = maxent.moment_residual(bs, Ms, rule3["Phi"], rule3["logw"])
    floor = maxent.moment_residual(f32(rs), Ms, rule3["Phi"], rule3["logw"])
    bar = np.maximum(1e-5, 2.0 * floor)
    scale = np.maximum(1.0, np.max(np.abs(rs), axis=1))
    berr = np.max(np.abs(bs - rs), axis=1) / scale
    print(f"[{ctxm.prec_name} full] sample: {sel.sum()} of {good.sum()} realizable converged; "
          f"r max {r.max():.2e}; beta err max {berr.max():.2e}", flush=True)
    assert np.all(r <= bar)
    assert berr.max() <= 1e-4
    dr = np.abs(res[idx][sel] - r)
    assert np.all(dr <= 2e-7 + 0.01 * r)


def test_mixed_precision_steps_match_oracle(ctxm):
    """mem_step on a mixed-precision context: the cells' Newton Hessians come from
    the hi+lo 16-bit assembly, gradients, fluxes and speeds stay FP32.  Mach-3
    shock, 240 cells, 8 steps, against the oracle's FP64 steps."""
    from oracle import kinetics
    args = (3.0, 240, -12.0, 12.0, 3.0)
    problem = mem_inputs.shock_problem(*args)
    M = problem["M"].astype(np.float32)
    g = problem["g"].astype(np.float32)
    Md = torch.tensor(M, device=DEV)
    gd = torch.tensor(g, device=DEV)
    ctxm.gauge(Md, None, gd)
    bd = torch.tensor(mem_inputs.maxwellian_beta(M.shape[0], 35, Md[:, 0].cpu().numpy())
                      .astype(np.float32), device=DEV)
    batch = mem.ShockBatch([0, M.shape[0]], [problem["dx"]], problem["M_left"][None],
                           problem["M_right"][None], problem["g_left"][None],
                           problem["g_right"][None], device=DEV)
    t = torch.zeros(1, device=DEV)
    dt = torch.zeros(1, device=DEV)
    status = torch.zeros(M.shape[0], dtype=torch.int32, device=DEV)
    ctxm.step(batch, Md, bd, gd, t, dt, 8, status=status)
    torch.cuda.synchronize()
    ora = kinetics.ShockSolver(*args, nodes_1d=12)
    dts = [ora.step() for _ in range(8)]
    assert t.item() == pytest.approx(sum(dts), rel=1e-5)
    mg = kinetics.macroscopic(Md.cpu().numpy().astype(np.float64), gd.cpu().numpy().astype(np.float64))
    mo = kinetics.macroscopic(ora.M, ora.g)
    err = max(np.max(np.abs(mg[k] - mo[k]) / np.abs(mo[k])) for k in ("n", "v", "T"))
    print(f"\n[{ctxm.prec_name} step] n, v, T rel err {err:.2e}")
    assert err < 1e-4
    st = status.cpu().numpy()
    assert not np.any(st & (mem.ST_NONFINITE | mem.ST_NONREALIZABLE | mem.ST_LAMBDA_FAIL))
