#!/usr/bin/env python3
"""Throughput of the 35-moment maximal-entropy dual solve on one MI355X.

Workload (one "step" = one full solve of the batch, cold start):
  65,536 independent cells, 35-moment basis (orthonormal Hermite products of
  total degree <= 4), 12^3 = 1728 Gauss--Hermite nodes in gauge coordinates,
  FP32 (or the mixed BF16/FP16 hi+lo assembly with --prec).  Cell states are
  Mott-Smith mixtures of upstream/downstream Maxwellians (Mach ~ U(1.5, 10),
  gamma = 5/3, mixing weight ~ U(0, 1)) given as FP64 targets in each
  mixture's Hermite gauge, rounded to FP32; the solve starts from the
  Maxwellian multipliers.  Inputs are resident in HBM before timing.

value = solves/s counting only cells that finish converged with a relative
moment residual <= 1e-5 (the library's compensated residual, which agrees with
FP64 to ~1e-7; the parity tests evaluate it in FP64 with the oracle).

Prints ONE JSON line.  Single-GPU build: --gpus above 1 exits with a message.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "35-moment MaxEnt solves/s at rel. residual ≤1e-5, FP32 vs mixed; cell-steps/s"
MFMA_PEAK = {"fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0}
# FP32 vector peak (MI355X published, 256 CUs at 2.4 GHz) counts packed FP32,
# two FMAs per lane per clock.  The kernels are built without packed FP32
# instructions, so the attainable vector rate is 256 CUs x 4 SIMDs x 16 lanes x
# 2 flop x 2.4 GHz = 78.6 TFLOP/s.
FP32_VECTOR_PEAK = 157.3
FP32_VECTOR_UNPACKED = 78.6
# the method's work per cell-iteration in its dense form (exponent pass, the
# sigma . Psi assembly GEMM of 2 x 1728 x 630 flop, Cholesky, solves, one
# line-search trial): what the list loop executes, and what the persistent
# kernel's sum factorisation computes with fewer operations
DENSE_FLOP_ITER = 2.43e6
# k_newton_wave, algorithmic flops per assembled cell-iteration at 12^3 nodes
# (lower bound): the sum-factorised Hessian assembly (46,848 FMA: 25,920 +
# 15,120 + 5,808 over the three axes), the exponent of sigma (5 FMA per node,
# shared by the full step's line-search trial and the next assembly), the
# Cholesky of the 34 x 34 Newton matrix ((34^3 - 34) / 6 = 6,545 FMA) and its
# two triangular solves (2 x 34 x 33 / 2 = 1,122 FMA); exp, the coefficient
# builds and backtracking trials are not counted
WAVE_FLOP_ITER = 2.0 * (25920 + 15120 + 5808 + 5 * 1728 + 6545 + 1122)

# HBM bytes per launch from two rocprofv3 runs of this bench's solve (65,536
# cells): --pmc FETCH_SIZE, then --pmc WRITE_SIZE, KiB per dispatch, each scaled
# by what the counter reads for a 1 GiB device-to-device copy (--copy-mib 1024:
# FETCH x 2.0, WRITE x 1.0).  Each figure describes one version of its kernel and
# of the Newton loop that launches it: the source texts are pinned by hash, and
# any other version reports null.
#  * k_assemble3 on the list loop (launch parameters 2,512): averaged over the
#    timed solve's 24 launches, the first one empty (the cells start at their
#    gauge's Maxwellian and take the first pass in closed form);
#  * k_newton_wave: one launch per solve (12 waves per CU), the run's one launch.
ASM_TRAFFIC = {
    "kernel_sha256": "167e9e156928e32203a2cce7d44770e14e6078e247a24d4e9d1db43bf23a0910",
    "fetch_kib": 30730.8, "fetch_scale": 1.99995,
    "write_kib": 63904.4, "write_scale": 1.0,
    "cells": 65536, "tuning": [2, 512],
}
WAVE_TRAFFIC = {
    "kernel_sha256": "311f5b120e56592825f8e11cdb7fc618d9bf7ebd3b437bcb0aed9d9150813717",
    "fetch_kib": 18926.2, "fetch_scale": 1.99995,
    "write_kib": 197486.7, "write_scale": 1.0,
    "cells": 65536,
}
# the figures depend on the kernels and on the Newton loop that launches them
_ASM_SRC = (("paper_2303_02898_amd/csrc/k_solve3.hip",
             "// assembly: S[cell][col] = sum_p sigma_p Psi[p][col] on FP32 MFMA",
             "// S[cell] = sum over splits"),
            ("paper_2303_02898_amd/csrc/k_solve3.hip",
             "int assembly_splits(", "hipError_t launch_assemble5("),
            ("paper_2303_02898_amd/csrc/api.cpp",
             "mem_err_t newton3(", "// Process-wide tuning results"))
_WAVE_SRC = (("paper_2303_02898_amd/csrc/k_solve3.hip",
              "__device__ __forceinline__ float rl(float v, int src)",
              "// Lm: this wave's LDS copy of L"),
             ("paper_2303_02898_amd/csrc/k_solve3.hip",
              "// Column `lane` of H = S/s00 - E E^T", "constexpr int DIR_WAVES"),
             ("paper_2303_02898_amd/csrc/k_solve3.hip",
              "// Unordered pair (p, q) of one-dimensional Hermite indices",
              "hipError_t launch_set_ctr("),
             ("paper_2303_02898_amd/csrc/k_solve3.hip",
              "hipError_t launch_newton_wave(", "hipError_t launch_unpack3("),
             ("paper_2303_02898_amd/csrc/api.cpp",
              "mem_err_t newton3(", "// Process-wide tuning results"))


def strict_json(v):
    """The bench line as strict JSON: a non-finite float (a conditioning bound
    whose Cholesky failed, say) is written as the string "inf", "-inf" or
    "nan"."""
    if isinstance(v, float) and not math.isfinite(v):
        return "nan" if v != v else ("inf" if v > 0 else "-inf")
    if isinstance(v, dict):
        return {k: strict_json(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [strict_json(x) for x in v]
    return v


def source_sha(spans):
    """sha256 of the given source spans (None if one is not found)."""
    h = hashlib.sha256()
    try:
        for path, begin, end in spans:
            with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), path)) as f:
                txt = f.read()
            a = txt.index(begin)
            h.update(txt[a:txt.index(end, a)].encode())
    except (OSError, ValueError):
        return None
    return h.hexdigest()


def measured_traffic(t, spans, prec, cells):
    """Calibrated HBM bytes per launch, or None when they were not measured for
    this kernel version and workload."""
    if prec != "fp32" or cells != t["cells"] or source_sha(spans) != t["kernel_sha256"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def cpu_baseline(M, b0, n_sample):
    """The FP64 oracle on a bounded sample of the same workload (host cores)."""
    from oracle import basis, maxent, quadrature
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()
                       if d.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    try:
        import torch   # the oracle's dense sums run on torch's CPU threads
        threads = max(threads, torch.get_num_threads())
    except Exception:
        pass
    nodes, w = quadrature.tensor_rule(12, 3)
    Phi, logw = basis.evaluate(nodes, 3), quadrature.lebesgue_log_weights(nodes, w)
    Ms = M[:n_sample].astype(np.float64)
    bs = b0[:n_sample].astype(np.float64)
    t0 = time.perf_counter()
    out = maxent.newton_solve(Ms, bs, Phi, logw, tol_grad=1e-10)
    el = time.perf_counter() - t0
    ok = int(np.sum(out["converged"]))
    res = {"value": ok / el, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
           "sample": f"first {n_sample} cells of the same 65,536-cell batch, FP64 NumPy "
                     f"Alg. 1 to max|G| <= 1e-10, {el:.1f} s wall"}
    # the same oracle on one thread (BLAS and torch), a smaller sample
    try:
        import torch
        from threadpoolctl import threadpool_limits
        n1 = max(1, n_sample // 8)
        tt = torch.get_num_threads()
        torch.set_num_threads(1)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            o1 = maxent.newton_solve(Ms[:n1], bs[:n1], Phi, logw, tol_grad=1e-10)
            el1 = time.perf_counter() - t0
        torch.set_num_threads(tt)
        res["single_thread"] = {"value": int(np.sum(o1["converged"])) / el1, "unit": "solves/s",
                                "cores": 1, "sample": f"first {n1} cells, {el1:.1f} s wall"}
    except Exception as exc:   # threadpoolctl missing: leave it out
        res["single_thread"] = {"error": str(exc)}
    # the oracle's time step beside the shock workloads: Mach-3 shock, 240 cells,
    # 4 LLF steps after the set-up (cell-steps/s, warm solves)
    from oracle import kinetics
    sh = kinetics.ShockSolver(3.0, 240, -12.0, 12.0, 3.0, nodes_1d=12)
    t0 = time.perf_counter()
    for _ in range(4):
        sh.step()
    el2 = time.perf_counter() - t0
    res["time_step"] = {"value": 240 * 4 / el2, "unit": "cell-steps/s",
                        "sample": f"Mach-3 shock, 240 cells, 4 LLF steps, FP64, {el2:.1f} s wall"}
    # the oracle on the paper's own discretisation (nine statistics, Mach-10 box)
    import mem_inputs
    from oracle import axisym
    rule = axisym.blockwise_rule(**mem_inputs.AXI_MACH10_BOX)
    cells = mem_inputs.mott_smith_cells9(AXI_CELLS)
    na = 256
    Ma, ga = cells["M"][:na].astype(np.float32), cells["g"][:na].astype(np.float32)
    t0 = time.perf_counter()
    oa = axisym.solve(Ma.astype(np.float64), ga.astype(np.float64),
                      axisym.maxwellian_beta(Ma[:, 0].astype(np.float64), ga), rule,
                      tol_grad=1e-10, max_iter=300)
    el3 = time.perf_counter() - t0
    res["axi_solve"] = {"value": float(np.sum(oa["converged"])) / el3, "unit": "solves/s",
                        "sample": f"first {na} cells of the nine-statistic Mach-10 batch, FP64 "
                                  f"Alg. 1 cell by cell to max|G| <= 1e-10, {el3:.1f} s wall"}
    return res


# the paper's own discretisation: Mach-10 Mott-Smith cells on its Mach-10 box
AXI_CELLS = 65536
# algorithmic flops per node: exponent (8 FMAs in FP64) per pass; the 45 sums
# (sigma, 8 sigma phi_i, 36 sigma phi_i phi_j: 8 products, 9 adds, 36 FMAs)
# per assembly pass
AXI_FLOP_LSE = 16
AXI_FLOP_ASM = 16 + 89
# unpacked FP32 / FP64 vector FMA rate: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
VALU_PEAK_TFLOPS = 78.6


def _axi_shock_init(mach, n_cells):
    """Tanh profile of a normal shock on [-47.1, 47.1] (thickness 15.7): moments
    in the gauge (mean speed, 1, 1), that gauge, the ghost states and dx."""
    import math
    import mem_inputs
    (n1, v1, T1), (n2, v2, T2) = mem_inputs.rankine_hugoniot(mach)
    n1, v1, T1, n2, v2, T2 = (float(a) for a in (n1, v1, T1, n2, v2, T2))
    x_lo, x_hi, th = -47.1, 47.1, 15.7 / 2.0
    dx = (x_hi - x_lo) / n_cells
    x = x_lo + dx * (np.arange(n_cells) + 0.5)
    frac = ((np.tanh(x / th) - math.tanh(x_lo / th))
            / (math.tanh(x_hi / th) - math.tanh(x_lo / th)) - 0.5)
    gm = np.array([[0.5 * (v1 + v2), 1.0, 1.0]])
    Mm = mem_inputs.gaussian_moments9(np.array([n1]), np.array([v1]), np.array([T1]),
                                      np.array([T1]), gm)[0]
    Mp = mem_inputs.gaussian_moments9(np.array([n2]), np.array([v2]), np.array([T2]),
                                      np.array([T2]), gm)[0]
    M0 = (Mp - Mm)[None, :] * frac[:, None] + 0.5 * (Mp + Mm)[None, :]
    return M0, np.repeat(gm, n_cells, axis=0), ((n1, v1, T1), (n2, v2, T2)), dx


def _axi_start_beta(torch, Md):
    """Maxwellian multipliers of each cell's gauge (the solves' cold start)."""
    b0 = np.zeros((Md.shape[0], 9), np.float32)
    b0[:, 2] = -1.0 / np.sqrt(2.0)
    b0[:, 3] = -1.0
    bd = torch.tensor(b0, device=Md.device)
    bd[:, 0] = Md[:, 0]
    return bd


def _axi_shock_rate(mem, torch, dev, rule, n_cells=150, steps=400, scheme="llf"):
    """Alg. 2 steps of the Mach-10 shock on the nine statistics (wall time)."""
    M0, g0, ((n1, v1, T1), (n2, v2, T2)), dx = _axi_shock_init(10.0, n_cells)
    Md = torch.tensor(M0.astype(np.float32), device=dev)
    gd = torch.tensor(g0.astype(np.float32), device=dev)
    rule.gauge(Md, None, gd)
    bd = _axi_start_beta(torch, Md)
    t = torch.zeros(1, device=dev)
    dt = torch.zeros(1, device=dev)
    st = torch.zeros(n_cells, dtype=torch.int32, device=dev)
    cm = torch.zeros(1, device=dev)   # conditioning monitor, on in the timed steps
    args = (Md, bd, gd, t, dt, dx, (n1, v1, T1), (n2, v2, T2))
    rule.reserve(n_cells)
    rule.step(*args, n_steps=0, status=st, scheme=scheme)
    rule.step(*args, n_steps=20, status=st, scheme=scheme, use_graph=True, cond_max=cm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rule.step(*args, n_steps=steps, status=st, scheme=scheme, use_graph=True, cond_max=cm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    Mh = Md.cpu().numpy()
    sh = st.cpu().numpy()
    return {"workload": f"Mach-10 normal shock, {n_cells} cells on [-47.1, 47.1], tanh "
                        f"thickness 15.7, {scheme.upper()} in local gauges with ES-BGK halves, "
                        "same box, hipGraph replay",
            "steps": steps, "ms_per_step": 1e3 * el / steps,
            "cell_steps_per_s": n_cells * steps / el, "t": float(t.item()),
            "finite": bool(np.all(np.isfinite(Mh))),
            "density_ends": [float(Mh[0, 0]), float(Mh[-1, 0])],
            "cond_bound": float(cm.item()),
            "last_step_cells": {k: float(np.mean((sh & bit) != 0)) for k, bit in
                                (("converged", mem.ST_CONVERGED), ("stagnated", mem.ST_STAGNATED),
                                 ("fp64_direction", mem.ST_FP64),
                                 ("nonrealizable", mem.ST_NONREALIZABLE))}}


def _axi_shock_batch_rate(mem, torch, dev, rule, n_problems=256, steps=100, scheme="llf"):
    """Alg. 2 steps of a ragged batch of normal shocks on the nine statistics in
    one mem_axi_step_batch: Mach numbers spread over [6, 10], 100 to 200 cells
    each, every problem with its own dx, ghosts, t and dt (wall time)."""
    rng = np.random.default_rng(2303)
    machs = np.linspace(6.0, 10.0, n_problems)
    cells = rng.integers(100, 201, n_problems)
    inits = [_axi_shock_init(float(m), int(c)) for m, c in zip(machs, cells)]
    Md = torch.tensor(np.concatenate([i[0] for i in inits]).astype(np.float32), device=dev)
    gd = torch.tensor(np.concatenate([i[1] for i in inits]).astype(np.float32), device=dev)
    rule.gauge(Md, None, gd)
    bd = _axi_start_beta(torch, Md)
    off = torch.tensor(np.concatenate([[0], np.cumsum(cells)]).astype(np.int64), device=dev)
    dxd = torch.tensor([i[3] for i in inits], dtype=torch.float32, device=dev)
    ghd = torch.tensor([[a for st in i[2] for a in st] for i in inits], dtype=torch.float32,
                       device=dev)
    n = int(cells.sum())
    t = torch.zeros(n_problems, device=dev)
    dt = torch.zeros(n_problems, device=dev)
    st = torch.zeros(n, dtype=torch.int32, device=dev)
    rule.reserve(n, n_problems)
    args = (Md, bd, gd, t, dt, off, dxd, ghd)
    rule.step_batch(*args, n_steps=0, status=st, scheme=scheme)
    rule.step_batch(*args, n_steps=10, status=st, scheme=scheme, use_graph=True)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rule.step_batch(*args, n_steps=steps, status=st, scheme=scheme, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"workload": f"{n_problems} normal shocks, Mach 6-10, 100-200 cells each "
                        f"({n} cells) on [-47.1, 47.1], {scheme.upper()} in local gauges with "
                        "ES-BGK halves, same box, one batched hipGraph replay per step",
            "problems": n_problems, "cells": n, "steps": steps, "ms_per_step": 1e3 * el / steps,
            "cell_steps_per_s": n * steps / el,
            "finite": bool(torch.isfinite(Md).all().item()),
            "t_range": [float(t.min().item()), float(t.max().item())]}


def paper_discretisation(mem, torch, dev, reps=5):
    """Alg. 1 on the paper's nine statistics and block-wise Gauss--Legendre box."""
    import mem_inputs
    box = mem_inputs.AXI_MACH10_BOX
    cells = mem_inputs.mott_smith_cells9(AXI_CELLS)
    C = AXI_CELLS
    rule = mem.AxiRule(**box)
    P = rule.n_nodes
    Md = torch.tensor(cells["M"].astype(np.float32), device=dev)
    gd = torch.tensor(cells["g"].astype(np.float32), device=dev)
    # cold start: the Maxwellian of each cell's own Hermite gauge
    b0 = np.zeros((C, 9), np.float32)
    b0[:, 0] = cells["M"][:, 0]
    b0[:, 2] = -1.0 / np.sqrt(2.0)
    b0[:, 3] = -1.0
    b0d = torch.tensor(b0, device=dev)
    bg = b0d.clone()
    it = torch.zeros(C, dtype=torch.int32, device=dev)
    rs = torch.zeros(C, dtype=torch.float32, device=dev)
    st = torch.zeros(C, dtype=torch.int32, device=dev)
    rule.solve(Md, gd, bg, None, it, rs, st)   # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        bg.copy_(b0d)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rule.solve(Md, gd, bg, None, it, rs, st)   # one kernel launch
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    # the paper's Mach-10 shock on its own discretisation: 150 cells on
    # [-47.1, 47.1], tanh thickness 15.7, the same box; LLF steps
    shock = _axi_shock_rate(mem, torch, dev, rule)
    shock_flic = _axi_shock_rate(mem, torch, dev, rule, scheme="flic")
    batch = _axi_shock_batch_rate(mem, torch, dev, rule)
    batch_flic = _axi_shock_batch_rate(mem, torch, dev, rule, scheme="flic")
    rule.close()
    ms = float(np.mean(times))
    s = st.cpu().numpy()
    conv = (s & mem.ST_CONVERGED) != 0
    good = conv & (rs.cpu().numpy() <= 1e-5)
    iters = it.cpu().numpy().astype(np.float64)
    # every Newton iteration is one assembly pass and at least one exponent pass
    flop = P * (np.sum(iters) * (AXI_FLOP_ASM + AXI_FLOP_LSE) + C * AXI_FLOP_LSE)
    achieved = flop / (ms * 1e-3) / 1e12
    return {"workload": f"nine-statistic Alg. 1, {C} Mach-10 Mott-Smith cells in their Hermite "
                        f"gauge, box [{box['ux_lo']}, {box['ux_hi']}] x [0, {box['ur_hi']}], "
                        f"{box['blocks_x']}x{box['blocks_r']} blocks of {box['order']}x"
                        f"{box['order']} Gauss-Legendre points ({P} nodes), FP32 with a compensated "
                        "final residual, cold start",
            "ms_per_solve": ms, "solves_per_s": float(np.sum(good)) / (ms * 1e-3),
            "converged_fraction": float(np.mean(conv)),
            "stagnated_fraction": float(np.mean((s & mem.ST_STAGNATED) != 0)),
            "iterations_mean": float(iters.mean()), "iterations_max": int(iters.max()),
            "shock_llf": shock, "shock_flic": shock_flic,
            "shock_batch_llf": batch, "shock_batch_flic": batch_flic,
            "roofline": {"bound": "alu", "kernel": "k_axi_solve", "achieved": achieved,
                         "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / VALU_PEAK_TFLOPS,
                         "flop_note": "lower bound: one exponent pass per iteration counted, "
                                      "statistics evaluation and exp not counted"}}


def run_solves(mem, ctx, Md, b0d, steps, warmup, tune=True):
    """Time `steps` cold-start solves of the resident batch; kernel times live.

    With tune, mem_autotune first picks the launch parameters on this batch
    (outside the timed region)."""
    import torch
    tuning = ctx.autotune(Md, b0d) if tune else ctx.tuning()
    C = Md.shape[0]
    bg = torch.empty_like(b0d)
    iters = torch.zeros(C, dtype=torch.int32, device=Md.device)
    resid = torch.zeros(C, dtype=torch.float32, device=Md.device)
    status = torch.zeros(C, dtype=torch.int32, device=Md.device)
    opts = mem.default_opts()
    for _ in range(warmup):
        bg.copy_(b0d)
        ctx.solve(Md, bg, opts, iters, resid, status)
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bg.copy_(b0d)
        ctx.solve(Md, bg, opts, iters, resid, status)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = status.cpu().numpy()
    rs = resid.cpu().numpy()
    it = iters.cpu().numpy()
    ok = ((st & mem.ST_CONVERGED) != 0) & (rs <= 1e-5)
    prof = {k: ctx.profile_read(k) for k in ("assemble", "direction", "lse", "wave")}
    ctx.profile(False)
    asm_ms, asm_n = prof["assemble"]
    wave_ms, wave_n = prof["wave"]
    # assembled cell-iterations: a cell that starts exactly at the Maxwellian of
    # its gauge takes its first direction in closed form (no assembly)
    b0 = b0d.cpu().numpy()
    maxw = np.zeros((1, b0.shape[1]), dtype=np.float32)
    maxw[0, [4, 7, 9]] = np.float32(-np.sqrt(0.5))
    closed = np.all(b0[:, 1:] == maxw[:, 1:], axis=1) & (it >= 1)
    assembled = float(np.sum(it - closed.astype(it.dtype)))
    total_flop = 2.0 * 1728 * 630 * assembled * steps
    wave_flop = WAVE_FLOP_ITER * assembled * steps
    return dict(
        value=int(ok.sum()) * steps / elapsed, ms=1e3 * elapsed / steps, ok=ok, it=it, st=st,
        assembled_cell_iterations=assembled,
        asm_tflops=total_flop / (asm_ms * 1e-3) / 1e12 if asm_ms > 0 else 0.0, tuning=tuning,
        asm_launches=asm_n, asm_avg_ms=asm_ms / max(asm_n, 1),
        wave_tflops=wave_flop / (wave_ms * 1e-3) / 1e12 if wave_ms > 0 else 0.0,
        wave_launches=wave_n, wave_avg_ms=wave_ms / max(wave_n, 1),
        kernel_ms={k: v[0] / steps for k, v in prof.items()}, beta=bg)


def passes(mem, torch, ctx, Md, gd, r, reps=20):
    """Achieved HBM bandwidth of the exp (log-sum-exp + line search) and flux passes
    against the 8 TB/s peak.  Both are arithmetic-bound by design: the exponent is
    sum-factorised (a few FMAs per node from the 1D tables in LDS), so a cell moves
    a few hundred bytes against ~10^4 node evaluations."""
    n = Md.shape[0]
    beta = r["beta"]
    F, lam = ctx.flux(beta, gd)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.flux(beta, gd)
    e1.record()
    torch.cuda.synchronize()
    flux_ms = e0.elapsed_time(e1) / reps
    flux_bytes = 4 * n * (35 + 3 + 35 + 2)            # beta, g in; F, (lam_min, lam_max) out
    # line search per live cell-iteration: beta, dbeta, M, L, G.dbeta, list in;
    # beta, log Z, L, alpha out (the 1D node tables stay in LDS / L2)
    lse_bytes = 4 * float(r["it"].sum()) * (35 + 36 + 35 + 3 + 35 + 3)
    lse_ms = r["kernel_ms"]["lse"]
    exp_lse = ({"kernels": "k_lse3 (log-sum-exp pass and Armijo trials)",
                "ms_per_solve": lse_ms, "bytes_per_cell_iteration": 4 * 147,
                "achieved_GBps": lse_bytes / (lse_ms * 1e-3) / 1e9, "peak_GBps": 8000.0,
                "bound": "valu (sum-factorised exponent)"} if lse_ms > 0 else
               {"kernels": "inside k_newton_wave (the persistent Newton loop): no separate "
                           "exponent pass"})
    return {
        "exp_lse": exp_lse,
        "flux": {"kernels": "k_flux3 + k_eig3 (moment fluxes and extreme speeds)",
                 "cells": n, "ms": flux_ms, "bytes_per_cell": 4 * 75,
                 "achieved_GBps": flux_bytes / (flux_ms * 1e-3) / 1e9, "peak_GBps": 8000.0,
                 "bound": "valu (quadrature over 1728 nodes per cell)"},
    }


def mixed_comparison(mem, torch, dev, cells, steps, warmup):
    """FP32 vs BF16x3 vs FP16x3 on the Mach 5-10 Mott-Smith workload."""
    import mem_inputs
    ms = mem_inputs.mott_smith_cells(cells, 5.0, 10.0, config=4, replica=0)
    M32 = ms["M"].astype(np.float32)
    b032 = mem_inputs.maxwellian_beta(cells, 35, M32[:, 0].astype(np.float64)).astype(np.float32)
    Md = torch.tensor(M32, device=dev)
    b0d = torch.tensor(b032, device=dev)
    out = {"workload": f"3D 35-moment MaxEnt dual solve, {cells} Mott-Smith cells "
                       "(Mach U(5,10), nu U(0,1)), 12^3 nodes, cold start",
           "cells": cells}
    base = None
    beta32 = None
    for prec in ("fp32", "fp32_list", "bf16x3", "fp16x3"):
        ctx = mem.Context(3, 12, "fp32" if prec == "fp32_list" else prec)
        ctx.reserve(cells)
        if prec == "fp32_list":
            # the same FP32 solve on the list-compacted loop with the MFMA assembly
            ctx.set_tuning(dir_waves=2, split_want=512, solver=0)
        r = run_solves(mem, ctx, Md, b0d, steps, warmup, tune=prec != "fp32_list")
        # per-moment residual G_k = E[phi_k]/E[phi_0] - M_k/n of the converged cells,
        # evaluated in compensated arithmetic (agrees with FP64 to a few 1e-8)
        G = ctx.moment_residual(Md, r["beta"]).abs().cpu().numpy()
        beta = r["beta"].cpu().numpy().astype(np.float64)
        ctx.close()
        ok = r["ok"]
        if base is None:
            base = r["value"]
            beta32, ok32 = beta, ok
        both = ok & ok32
        scale = np.maximum(1.0, np.abs(beta32[both]).max(axis=1))
        out[prec] = {"solves_per_s": r["value"], "ms_per_solve": r["ms"],
                     "newton_loop": "persistent" if r["tuning"].get("solver") == 1 else "list/MFMA",
                     "speedup_vs_fp32": r["value"] / base if base else None,
                     "speedup_vs_fp32_list": (r["value"] / out["fp32_list"]["solves_per_s"]
                                              if "fp32_list" in out else None),
                     "converged_fraction": float(ok.mean()),
                     "iterations_mean": float(r["it"].mean()), "iterations_max": int(r["it"].max()),
                     "assemble_ms_per_solve": r["kernel_ms"]["assemble"],
                     "assemble_algorithmic_tflops": r["asm_tflops"],
                     "residual_max": float(G[ok].max()),
                     "residual_per_moment_max": [float(f"{v:.3g}") for v in G[ok].max(axis=0)[1:]],
                     "residual_per_moment_p99": [float(f"{v:.3g}")
                                                 for v in np.percentile(G[ok], 99, axis=0)[1:]],
                     "beta_vs_fp32_max": float(np.max(np.abs(beta[both] - beta32[both]).max(axis=1)
                                                      / scale))}
    return out


def shock_setup(mem, torch, dev, ctx, probs, dx, use_graph, iter_hist=None, flux_scheme="llf",
                cond_max=None, status_counts=None, budget=8):
    """Device state and batch for a list of shock problems (gauge applied)."""
    import mem_inputs
    M = np.concatenate([p["M"] for p in probs]).astype(np.float32)
    g = np.concatenate([p["g"] for p in probs]).astype(np.float32)
    counts = [p["M"].shape[0] for p in probs]
    off = np.concatenate([[0], np.cumsum(counts)])
    Md, gd = torch.tensor(M, device=dev), torch.tensor(g, device=dev)
    ctx.gauge(Md, None, gd)
    bd = torch.tensor(mem_inputs.maxwellian_beta(M.shape[0], 35, Md[:, 0].cpu().numpy())
                      .astype(np.float32), device=dev)
    batch = mem.ShockBatch(off, dx, np.stack([p["M_left"] for p in probs]),
                           np.stack([p["M_right"] for p in probs]),
                           np.stack([p["g_left"] for p in probs]),
                           np.stack([p["g_right"] for p in probs]), device=dev,
                           use_graph=use_graph, iter_hist=iter_hist, flux_scheme=flux_scheme,
                           cond_max=cond_max, status_counts=status_counts,
                           newton_per_step=budget)
    P = len(probs)
    return batch, Md, bd, gd, torch.zeros(P, device=dev), torch.zeros(P, device=dev)


def shock_steady(mem, torch, dev, max_steps, scheme="llf", cells=1000):
    """Mach-3 normal shock on [-20, 20]: step rate and time to steady state."""
    import mem_inputs
    ctx = mem.Context(3, 12)
    pr = mem_inputs.shock_problem(3.0, cells, -20.0, 20.0, 5.44)
    b, M, be, g, t, dt = shock_setup(mem, torch, dev, ctx, [pr], [pr["dx"]], True,
                                     flux_scheme=scheme)
    ctx.step(b, M, be, g, t, dt, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(b, M, be, g, t, dt, 500)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / 500
    (n1, v1, T1), (n2, v2, T2) = pr["states"]
    prev = M[:, 0].clone()
    steps, change = 510, float("inf")
    t0 = time.perf_counter()
    while steps < max_steps and change > 2e-5:
        ctx.step(b, M, be, g, t, dt, 100)
        steps += 100
        cur = M[:, 0].clone()
        change = (cur - prev).abs().max().item() / (n2 - n1)
        prev = cur
    wall = time.perf_counter() - t0
    n = M[:, 0].cpu().numpy()
    ctx.close()
    # density thickness (n+ - n-) / max |dn/dx|, in upstream mean free paths
    thick = (n2 - n1) / (np.max(np.abs(np.diff(n))) / pr["dx"])
    names = {"llf": "LLF", "lw": "two-step Lax-Wendroff", "flic": "FLIC (van Leer)"}
    return {"workload": f"Mach-3 normal shock, {cells} cells on [-20, 20] (upstream mean free "
                        f"path 1), ES-BGK Pr 2/3, {names[scheme]}, CFL 0.5, 12^3 nodes, 8 Newton "
                        "iterations per solve, hipGraph replay",
            "ms_per_step": ms, "cell_steps_per_s": cells / (ms * 1e-3),
            "steady": {"criterion": "max |n(k+100) - n(k)| / (n+ - n-) <= 2e-5",
                       "steps": steps, "t": float(t.item()), "wall_s": wall + ms * 510e-3,
                       "last_change": change, "reached": change <= 2e-5,
                       "n_ends": [float(n[0]), float(n[-1])], "n_rankine_hugoniot": [n1, n2],
                       "density_thickness_mfp": float(thick),
                       "finite": bool(np.isfinite(n).all())}}


def gauge_study(mem, torch, dev):
    """Upstream Maxwellians of Mach 2..12 solved in FP32 from the uniform start,
    in each state's Hermite gauge and in the fixed gauge (0, 1, 1)."""
    import math
    import mem_inputs
    ctx = mem.Context(3, 12)
    machs = np.arange(2, 13, dtype=np.float64)
    v = math.sqrt(5.0 / 3.0) * machs
    N = machs.size
    out = {"workload": "upstream Maxwellians n = 1, T = 1, Mach 2..12, 12^3 nodes, FP32, "
                       "start beta_i = 0 (i >= 1)", "mach": machs.tolist()}
    names = [(mem.ST_CONVERGED, "converged"), (mem.ST_STAGNATED, "stagnated"),
             (mem.ST_NONREALIZABLE, "nonrealizable"), (mem.ST_MAXITER, "maxiter")]
    for gauge in ("hermite", "fixed"):
        w = v if gauge == "hermite" else np.zeros(N)
        g = np.stack([w, np.ones(N), np.ones(N)], axis=1)
        M = mem_inputs.gaussian_moments(np.ones(N), v, np.ones(N), np.ones(N), g)
        b = np.zeros((N, 35), dtype=np.float32)
        b[:, 0] = 1.0
        Md = torch.tensor(M.astype(np.float32), device=dev)
        bd = torch.tensor(b, device=dev)
        it = torch.zeros(N, dtype=torch.int32, device=dev)
        rs = torch.zeros(N, device=dev)
        st = torch.zeros(N, dtype=torch.int32, device=dev)
        ctx.solve(Md, bd, iters=it, resid=rs, status=st)
        torch.cuda.synchronize()
        stv = st.cpu().numpy()
        row = {"iterations": it.cpu().tolist(), "residual": [float(x) for x in rs.cpu()],
               "status": [next((nm for bit, nm in names if s & bit), hex(int(s))) for s in stv]}
        if gauge == "hermite":
            # the answer is the state's Maxwellian: -1/sqrt(2) on the three squares, else 0
            ref = np.zeros((N, 34))
            ref[:, [3, 6, 8]] = -math.sqrt(0.5)
            row["beta_error_max"] = float(np.max(np.abs(bd.cpu().numpy()[:, 1:] - ref)))
        out[gauge] = row
    ctx.close()
    return out


def cond_study(mem, torch, dev):
    """Conditioning against resolution (the paper's cell-count study): Mach-4
    shock on [-16.3, 16.3], run to t = 10, then the largest in-kernel lower bound
    of cond(H) (at each cell's solution) over the next 200 steps."""
    import mem_inputs
    ctx = mem.Context(3, 12)
    out = {"workload": "Mach-4 normal shock on [-16.3, 16.3], tanh thickness 5.44, ES-BGK, "
                       "12^3 nodes; in-kernel lower bound of cond(H) at each cell's solution "
                       "(power and inverse iterations), over steps t > 10 "
                       "(200 steps)", "runs": []}
    for scheme, cells in (("llf", 125), ("llf", 250), ("llf", 500), ("llf", 1000),
                          ("flic", 125), ("flic", 250)):
        pr = mem_inputs.shock_problem(4.0, cells, -16.3, 16.3, 5.44)
        cm = torch.zeros(1, device=dev)
        b, M, be, g, t, dt = shock_setup(mem, torch, dev, ctx, [pr], [pr["dx"]], True,
                                         flux_scheme=scheme, cond_max=cm)
        steps = 0
        while t.item() < 10.0 and steps < 20000:
            ctx.step(b, M, be, g, t, dt, 100)
            steps += 100
            if steps % 1000 == 0 and not torch.isfinite(M).all().item():
                break
        cm.zero_()
        ctx.step(b, M, be, g, t, dt, 200)
        torch.cuda.synchronize()
        out["runs"].append({"scheme": scheme, "cells": cells, "dx": pr["dx"],
                            "cond_bound_max": float(cm.item()), "t": float(t.item()),
                            "finite": bool(torch.isfinite(M).all().item())})
    ctx.close()
    return out


def ragged_rate(mem, torch, dev, steps):
    """2048 independent shocks, log-uniform cell counts in [64, 4096]: cell-steps/s."""
    import mem_inputs
    rb = mem_inputs.ragged_batch(2048)
    ctx = mem.Context(3, 12)
    # the Newton budget per step of the oracle parity test of this workload
    budget = 40
    hist = torch.zeros(budget + 1, dtype=torch.int64, device=dev)
    counts = torch.zeros(9, dtype=torch.int64, device=dev)
    b, M, be, g, t, dt = shock_setup(mem, torch, dev, ctx, rb["problems"], [rb["dx"]] * 2048, True,
                                     iter_hist=hist, status_counts=counts, budget=budget)
    status = torch.zeros(b.n_cells, dtype=torch.int32, device=dev)
    ctx.step(b, M, be, g, t, dt, 1, status=status)
    torch.cuda.synchronize()
    hist.zero_()
    counts.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(b, M, be, g, t, dt, steps, status=status)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx_loop = "persistent" if ctx.tuning().get("solver") == 1 else "list/MFMA"
    ctx.close()
    st = status.cpu().numpy()
    off = b.offsets.cpu().numpy()
    fin = torch.isfinite(M).all(dim=1).cpu().numpy() & (M[:, 0] > 0).cpu().numpy()
    mx = (st & mem.ST_MAXWELL_FLUX) != 0
    prob_mx = np.array([mx[off[p]:off[p + 1]].any() for p in range(2048)])
    prob_fin = np.array([fin[off[p]:off[p + 1]].all() for p in range(2048)])
    h = hist.cpu().numpy().astype(np.int64)
    cnt = counts.cpu().numpy().astype(np.int64)
    cell_steps = b.n_cells * steps
    # cell-steps that ended MAXITER (an unconverged beta) or stepped with the
    # Maxwellian of their gauge are reported apart and not counted as solved
    apart = int(cnt[1]) + int(cnt[8])
    cdf = np.cumsum(h) / max(int(h.sum()), 1)
    pct = {f"p{q}": int(np.searchsorted(cdf, q / 100.0)) for q in (50, 90, 99)}
    return {"workload": f"2048 normal shocks (Mach U(1.2,10), tanh initial profiles), cell counts "
                        f"log-uniform in [64, 4096] ({b.n_cells} cells), dx = 1, {steps} steps, "
                        f"Newton budget {budget} per step, hipGraph replay",
            "newton_loop": ctx_loop,
            "cells": b.n_cells, "steps": steps, "ms_per_step": 1e3 * el / steps,
            "cell_steps_per_s": (cell_steps - apart) / el,
            "cell_steps_per_s_all": cell_steps / el,
            "cell_steps_by_status": {
                "total": cell_steps, "converged": int(cnt[0]), "maxiter": int(cnt[1]),
                "stagnated": int(cnt[2]), "fp64_direction": int(cnt[4]),
                "nonfinite": int(cnt[5]), "nonrealizable": int(cnt[6]),
                "maxwell_flux": int(cnt[8]),
                "note": "cell_steps_per_s leaves out the maxiter and maxwell_flux cell-steps"},
            "newton_iterations": {
                "per_cell_step_histogram": h.tolist(),
                "budget": budget,
                "mean": float((h * np.arange(budget + 1)).sum() / max(int(h.sum()), 1)),
                **pct, "max": int(np.nonzero(h)[0].max()) if h.any() else 0},
            "problems_finite": int(prob_fin.sum()),
            "maxwell_flux": {
                "cells": int(mx.sum()), "problems": int(prob_mx.sum()),
                "lowest_mach": float(rb["mach"][prob_mx].min()) if prob_mx.any() else None,
                "note": "cells whose moments the 12^3 Gauss-Hermite nodes cannot represent "
                        "(solve certifies non-realizability) step with the Maxwellian of "
                        "their gauge"}}


def latency_1d(mem, torch, dev, calls=200):
    """1D 5-moment solves of 1024 cells (16 nodes): wall time per call, on the
    perturbed-multiplier workload (targets committed by
    tests/golden/make_config1_targets.py, moved into each cell's Hermite gauge on
    the GPU) and on two-Gaussian mixtures."""
    import mem_inputs
    with open(os.path.join(ROOT, "tests", "golden", "config1_targets.json")) as f:
        c1 = json.load(f)
    mix = mem_inputs.mixture_1d(1024)
    ctx = mem.Context(1, 16)
    out = {}
    for name, M, g, gauge in (("perturbed_multipliers", np.asarray(c1["M"]), np.asarray(c1["g"]),
                               True),
                              ("two_gaussian_mixtures", mix["M"], mix["g"], False)):
        Md = torch.tensor(M.astype(np.float32), device=dev)
        gd = torch.tensor(g.astype(np.float32), device=dev)
        if gauge:
            ctx.gauge(Md, None, gd)
        b0d = torch.zeros(Md.shape[0], 5, device=dev)
        b0d[:, 0] = Md[:, 0]
        b0d[:, 2] = -1.0 / np.sqrt(2.0)
        bg = b0d.clone()
        it, rs, st = ctx.solve(Md, bg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            bg.copy_(b0d)
            ctx.solve(Md, bg, None, it, rs, st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        conv = float(np.mean((st.cpu().numpy() & mem.ST_CONVERGED) != 0))
        out[name] = {"us_per_call": 1e6 * el / calls, "solves_per_s": Md.shape[0] * calls / el,
                     "converged_fraction": conv,
                     "iterations_mean": float(it.float().mean().item())}
    ctx.close()
    out["workload"] = ("1D 5-moment solve, 1024 cells, 16 Gauss-Hermite nodes in each cell's "
                       "Hermite gauge, cold start from the gauge Maxwellian: the perturbed-"
                       "multiplier targets (n ~ U(0.5, 2), v ~ N(0, 1), T ~ U(0.5, 2), He_3/He_4 "
                       "multipliers ~ N(0, 0.05)), and two-Gaussian mixtures")
    out["us_per_call"] = out["perturbed_multipliers"]["us_per_call"]
    out["solves_per_s"] = out["perturbed_multipliers"]["solves_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=65536)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--cpu-sample", type=int, default=6144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-cells", type=int, default=262144,
                    help="cells of the FP32-vs-mixed comparison (0 = skip)")
    ap.add_argument("--ragged-steps", type=int, default=200)
    ap.add_argument("--shock-max-steps", type=int, default=40000)
    ap.add_argument("--only-paper-discretisation", action="store_true",
                    help="run only the nine-statistic leg and print it (for profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 1D, shock and ragged-batch measurements")
    ap.add_argument("--tuning", default=None, metavar="DIR_WAVES,SPLIT_WANT",
                    help="fixed launch parameters instead of the autotuner (e.g. to profile "
                         "exactly the launches a tuned run timed)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (a known-size "
                         "kernel for calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the cell "
              "batch would be sharded across GPUs without communication.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import mem_inputs
    import paper_2303_02898_amd as mem

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.only_paper_discretisation:
        print(json.dumps(strict_json({"paper_discretisation": paper_discretisation(mem, torch, dev)}),
                         allow_nan=False),
              flush=True)
        return
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    C = args.cells
    cells = mem_inputs.mott_smith_cells(C, config=2, replica=0)
    M32 = cells["M"].astype(np.float32)
    b032 = mem_inputs.maxwellian_beta(C, 35, M32[:, 0].astype(np.float64)).astype(np.float32)
    ctx = mem.Context(3, 12, args.prec)
    ctx.reserve(C)
    Md = torch.tensor(M32, device=dev)
    b0d = torch.tensor(b032, device=dev)
    if args.tuning:
        dw, sw = (int(v) for v in args.tuning.split(","))
        ctx.set_tuning(dir_waves=dw, split_want=sw)
    r = run_solves(mem, ctx, Md, b0d, args.steps, args.warmup, tune=not args.tuning)
    pass_rates = passes(mem, torch, ctx, Md, torch.tensor(cells["g"].astype(np.float32),
                                                           device=dev), r)
    wave = r["tuning"].get("solver") == 1 and args.prec == "fp32"
    # the same workload on the list-compacted Newton loop with the MFMA assembly
    rl = rl128 = None
    if wave:
        ctx.set_tuning(dir_waves=2, split_want=512, solver=0)
        rl = run_solves(mem, ctx, Md, b0d, args.steps, args.warmup, tune=False)
        # the assembly's other workgroup size: 128 cells (eight waves) per node tile
        ctx.set_tuning(dir_waves=2, split_want=512, solver=0, asm_waves=8)
        rl128 = run_solves(mem, ctx, Md, b0d, args.steps, args.warmup, tune=False)
    ctx.close()
    peak = MFMA_PEAK[args.prec]

    def mfma_roofline(rr):
        return {
            "bound": "mfma",
            "kernel": "k_assemble3 (sigma . Psi, 630 pair columns)" if args.prec == "fp32"
                      else "k_assemble3m (sigma . Psi, hi+lo 16-bit products)",
            "achieved": rr["asm_tflops"],
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": rr["asm_tflops"] / peak,
            "traffic": measured_traffic(ASM_TRAFFIC, _ASM_SRC, args.prec, C),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_tuning": ASM_TRAFFIC["tuning"],
            "flop_per_cell_iteration": 2.0 * 1728 * 630,
            "assembled_cell_iterations_per_step": rr["assembled_cell_iterations"],
            "launches": rr["asm_launches"],
            "avg_launch_ms": rr["asm_avg_ms"],
        }

    if wave:
        # same cell-iterations and kernel time, priced at the dense formulation's work
        dense_rate = r["wave_tflops"] * DENSE_FLOP_ITER / WAVE_FLOP_ITER
        roof = {
            "bound": "alu",
            "kernel": "k_newton_wave (persistent Newton loop, one wavefront per cell, "
                      "sum-factorised assembly)",
            "achieved": r["wave_tflops"],
            "peak": FP32_VECTOR_UNPACKED,
            "peak_note": "FP32 vector without packed instructions (the kernels are compiled without them): "
                         "256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz",
            "unit": "TFLOP/s",
            "frac": r["wave_tflops"] / FP32_VECTOR_UNPACKED,
            "frac_of_packed_fp32_peak": r["wave_tflops"] / FP32_VECTOR_PEAK,
            "dense_equivalent": {
                "flop_per_cell_iteration": DENSE_FLOP_ITER,
                "achieved": dense_rate,
                "frac_of_fp32_peak": dense_rate / FP32_VECTOR_PEAK,
                "note": "the method's per-iteration work in its dense form (assembly as the "
                        "sigma . Psi GEMM), divided by the same kernel time: the rate at which "
                        "the persistent kernel delivers what the dense formulation would "
                        "execute"},
            "traffic": measured_traffic(WAVE_TRAFFIC, _WAVE_SRC, args.prec, C),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "flop_per_cell_iteration": WAVE_FLOP_ITER,
            "flop_note": "lower bound: sum-factorised assembly, the exponent of sigma (which "
                         "also serves the full step's line-search trial), the 34 x 34 "
                         "Cholesky and its two triangular solves per assembled "
                         "cell-iteration; exp, coefficient builds and backtracking trials "
                         "not counted",
            "assembled_cell_iterations_per_step": r["assembled_cell_iterations"],
            "launches": r["wave_launches"],
            "avg_launch_ms": r["wave_avg_ms"],
        }
    else:
        roof = mfma_roofline(r)

    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else args.prec,
        "data": "synthetic",
        "config": {
            "workload": f"3D 35-moment MaxEnt dual solve, {C} Mott-Smith cells "
                        "(Mach U(1.5,10), nu U(0,1), gamma 5/3), 12^3 Gauss-Hermite nodes, "
                        "cold start from the Maxwellian, Alg. 1 to max|G|<=2e-6",
            "cells": C, "nodes": 1728, "basis": 35, "prec": args.prec,
        },
        "roofline": roof,
        "solver": {
            "converged_fraction": float(r["ok"].mean()),
            "iterations_mean": float(r["it"].mean()),
            "iterations_max": int(r["it"].max()),
            "fp64_direction_fraction": float(np.mean((r["st"] & mem.ST_FP64) != 0)),
            "tuning": r["tuning"],
            "newton_loop": "persistent (k_newton_wave)" if wave else "list/MFMA",
            "kernel_ms_per_step": {"assemble": r["kernel_ms"]["assemble"],
                                   "direction": r["kernel_ms"]["direction"],
                                   "lse_linesearch": r["kernel_ms"]["lse"],
                                   "newton_wave": r["kernel_ms"]["wave"]},
        },
    }
    if rl is not None:
        line["mfma_path"] = {
            "workload": "the same solve on the list-compacted Newton loop (launches per pass, "
                        "MFMA assembly), launch parameters 2,512",
            "solves_per_s": rl["value"], "ms_per_step": rl["ms"],
            "converged_fraction": float(rl["ok"].mean()),
            "iterations_mean": float(rl["it"].mean()),
            "roofline": mfma_roofline(rl),
            "assembly_cells_per_workgroup": {
                str(cells): {"avg_launch_ms": rr["asm_avg_ms"], "tflops": rr["asm_tflops"],
                             "solves_per_s": rr["value"]}
                for cells, rr in ((64, rl), (128, rl128))}}
    line["passes"] = pass_rates
    if args.mixed_cells > 0:
        line["mixed"] = mixed_comparison(mem, torch, dev, args.mixed_cells, 3, 1)
    if not args.no_extras:
        line["latency_1d"] = latency_1d(mem, torch, dev)
        line["paper_discretisation"] = paper_discretisation(mem, torch, dev)
        line["gauge_study"] = gauge_study(mem, torch, dev)
        line["cond_study"] = cond_study(mem, torch, dev)
        line["shock"] = shock_steady(mem, torch, dev, args.shock_max_steps)
        # second order at the paper's resolutions (0.13-0.63 mean free paths per
        # cell), against LLF on the same grid
        line["shock_flic"] = {"flic": shock_steady(mem, torch, dev, args.shock_max_steps, "flic", 250),
                              "llf_same_grid": shock_steady(mem, torch, dev, args.shock_max_steps,
                                                            "llf", 250)}
        if args.ragged_steps > 0:
            line["ragged"] = ragged_rate(mem, torch, dev, args.ragged_steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(M32, b032, args.cpu_sample)
    print(json.dumps(strict_json(line), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
