"""GPU test of the allocation-free solve (mem_maxent_solve_noalloc) through the
C ABI: two calls in a row, the second with fewer cells, each checked against
mem_maxent_solve on the same inputs and against the FP64 oracle to the solve's
parity bars (relative moment residual <= 1e-5 evaluated in FP64 at the GPU's
beta, beta within 1e-4 of the oracle's), plus the size limit."""

import numpy as np
import pytest
import torch

import mem_inputs
import paper_2303_02898_amd as mem
from oracle import basis, maxent, quadrature

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


@pytest.fixture(scope="module")
def rule3():
    nodes, w = quadrature.tensor_rule(12, 3)
    return dict(Phi=basis.evaluate(nodes, 3), logw=quadrature.lebesgue_log_weights(nodes, w))


def _one_call(ctx, M, b0, rule, tag, replica, opts):
    C = M.shape[0]
    print(f"\n[noalloc] {tag}: {C} Mott-Smith cells (replica {replica})", flush=True)
    Md = dev(M)
    b_ref, b_na = dev(b0), dev(b0)
    _, r_ref, st_ref = ctx.solve(Md, b_ref, opts=opts)
    _, r_na, st_na = ctx.solve_noalloc(Md, b_na, opts=opts)
    torch.cuda.synchronize()
    st_ref, st_na = st_ref.cpu().numpy(), st_na.cpu().numpy()
    bref, bna = b_ref.cpu().numpy().astype(np.float64), b_na.cpu().numpy().astype(np.float64)
    conv_ref = (st_ref & mem.ST_CONVERGED) != 0
    conv_na = (st_na & mem.ST_CONVERGED) != 0
    print(f"[noalloc] {tag}: converged {conv_na.mean():.4f} (mem_maxent_solve {conv_ref.mean():.4f})")
    # same kernels: the two entry points agree to the solve's bars
    both = conv_ref & conv_na
    assert both.mean() >= 0.97
    scale = np.maximum(1.0, np.max(np.abs(bref[both]), axis=1))
    d = np.max(np.abs(bna[both] - bref[both]), axis=1) / scale
    print(f"[noalloc] {tag}: |beta_noalloc - beta_solve| / max(1, |beta|) max {d.max():.2e}")
    assert d.max() <= 1e-4
    assert np.all(r_na.cpu().numpy()[conv_na] <= 1e-5)
    # against the oracle on a sample of the converged cells
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(np.nonzero(conv_na)[0], min(48, int(conv_na.sum())), replace=False))
    ref = maxent.newton_solve(M[idx], b0[idx], rule["Phi"], rule["logw"])
    good = ref["converged"]
    r64 = maxent.moment_residual(bna[idx][good], M[idx][good], rule["Phi"], rule["logw"])
    floor = maxent.moment_residual(f32(ref["beta"][good]), M[idx][good], rule["Phi"], rule["logw"])
    bar = np.maximum(1e-5, 2.0 * floor)
    berr = (np.max(np.abs(bna[idx][good] - ref["beta"][good]), axis=1)
            / np.maximum(1.0, np.max(np.abs(ref["beta"][good]), axis=1)))
    print(f"[noalloc] {tag}: oracle sample {good.sum()}: r/bar max {np.max(r64 / bar):.2f}, "
          f"beta err max {berr.max():.2e}")
    assert np.all(r64 <= bar)
    assert berr.max() <= 1e-4


def test_noalloc_solve_matches_solve_twice(rule3):
    ctx = mem.Context(3, 12)
    try:
        opts = mem.default_opts(check_every=0)   # no stream synchronisation inside the call
        for tag, C, rep in (("first call", 3000, 5), ("second call, smaller", 700, 6)):
            cells = mem_inputs.mott_smith_cells(C, config=2, replica=rep)
            M = f32(cells["M"])
            b0 = f32(mem_inputs.maxwellian_beta(C, 35, M[:, 0]))
            _one_call(ctx, M, b0, rule3, tag, rep, opts)
        # beyond the static scratch: an error, nothing launched, beta untouched
        n = 8193
        M = torch.zeros(n, 35, device=DEV)
        M[:, 0] = 1.0
        b = torch.zeros(n, 35, device=DEV)
        with pytest.raises(mem.MemError):
            ctx.solve_noalloc(M, b)
        torch.cuda.synchronize()
        assert float(b.abs().max()) == 0.0
    finally:
        ctx.close()
