"""Pins for the oracle's canonical form, dual objective and Newton (no GPU).

* Maxwellian in its Hermite gauge: beta = -1/sqrt(2) on the three pure
  second-degree statistics reproduces M = n e_0 exactly on any tensor GH rule
  with >= 3 nodes (the exponent is -|u|^2/2 + const, so sigma_p = w_p).
* Gradient and Hessian of L (App. C) against central finite differences of L
  and of the gradient; the Hessian is SPD; dM/dbeta = beta_0 H (Sec. 3.3,
  eq. "moments vs parameter jacob").
* Alg. 1 reaches the FP64 floor on Mott-Smith cells, from different starts to
  the same beta (strict convexity), with quadratic convergence at the end.
"""

import numpy as np
import pytest

import mem_inputs
from oracle import basis, maxent, quadrature, workloads


def test_maxwellian_closed_form_is_exact(rule3):
    M = np.zeros((3, 35)); M[:, 0] = [0.5, 1.0, 3.0]
    beta = maxent.maxwellian_beta(M, 3)
    r = maxent.moment_residual(beta, M, rule3["Phi"], rule3["logw"])
    assert np.max(r) < 1e-14
    sig = maxent.sigma(beta, rule3["Phi"], rule3["logw"])
    assert np.allclose(sig, rule3["w"][None, :], rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("n", [3, 4, 7])
def test_maxwellian_exact_small_rules(n):
    nodes, w = quadrature.tensor_rule(n, 3)
    Phi = basis.evaluate(nodes, 3)
    lw = quadrature.lebesgue_log_weights(nodes, w)
    M = np.zeros((1, 35)); M[0, 0] = 1.7
    r = maxent.moment_residual(maxent.maxwellian_beta(M, 3), M, Phi, lw)
    assert r[0] < 1e-13


def _random_state(rng, C=3, scale=0.15):
    beta = mem_inputs.maxwellian_beta(C, 35, n=rng.uniform(0.5, 2.0, C))
    # perturb the degree <= 3 multipliers (indices 1..19); a negative quartic diagonal keeps
    # the density decaying
    beta[:, 1:20] += scale * rng.normal(size=(C, 19)) * 0.3
    for i, e in enumerate(basis.multi_indices(3)):
        if sum(e) == 4 and max(e) == 4:
            beta[:, i] = -0.05
    return beta


def test_gradient_matches_finite_differences(rule3):
    rng = np.random.default_rng(11)
    beta = _random_state(rng, C=2)
    M = maxent.model_moments(beta, rule3["Phi"], rule3["logw"])
    M[:, 1:] += 0.01 * rng.normal(size=(2, 34))  # gradient non-zero
    G = maxent.gradient(beta, M, rule3["Phi"], rule3["logw"])
    h = 1e-6
    for j in [1, 3, 5, 12, 20, 34]:
        bp = beta.copy(); bp[:, j] += h
        bm = beta.copy(); bm[:, j] -= h
        fd = (maxent.objective(bp, M, rule3["Phi"], rule3["logw"])
              - maxent.objective(bm, M, rule3["Phi"], rule3["logw"])) / (2 * h)
        assert np.allclose(fd, G[:, j], rtol=1e-6, atol=1e-8), j
    # beta_0 component: G_0 = n - n^2/beta_0 (zero at beta_0 = n)
    assert np.allclose(G[:, 0], 0.0, atol=1e-14)


def test_hessian_matches_jacobian_of_gradient_and_is_spd(rule3):
    rng = np.random.default_rng(12)
    beta = _random_state(rng, C=2)
    M = maxent.model_moments(beta, rule3["Phi"], rule3["logw"])
    H = maxent.hessian(beta, M, rule3["Phi"], rule3["logw"])
    h = 1e-5
    for j in [1, 2, 4, 10, 19, 34]:
        bp = beta.copy(); bp[:, j] += h
        bm = beta.copy(); bm[:, j] -= h
        fd = (maxent.gradient(bp, M, rule3["Phi"], rule3["logw"])
              - maxent.gradient(bm, M, rule3["Phi"], rule3["logw"])) / (2 * h)
        assert np.allclose(fd[:, 1:], H[:, 1:, j], rtol=1e-6, atol=1e-7), j
    for c in range(2):
        ev = np.linalg.eigvalsh(H[c, 1:, 1:])
        assert ev[0] > 0
        assert np.allclose(H[c], H[c].T, atol=1e-13)
    assert np.allclose(H[:, 0, 0], 1.0)  # n^2/beta_0^2 at beta_0 = n


def test_moment_jacobian_is_beta0_times_hessian(rule3):
    rng = np.random.default_rng(13)
    beta = _random_state(rng, C=1)
    M = maxent.model_moments(beta, rule3["Phi"], rule3["logw"])
    H = maxent.hessian(beta, M, rule3["Phi"], rule3["logw"])
    h = 1e-6
    for j in [1, 7, 25]:
        bp = beta.copy(); bp[:, j] += h
        bm = beta.copy(); bm[:, j] -= h
        fd = (maxent.model_moments(bp, rule3["Phi"], rule3["logw"])
              - maxent.model_moments(bm, rule3["Phi"], rule3["logw"])) / (2 * h)
        assert np.allclose(fd[0, 1:], beta[0, 0] * H[0, 1:, j], rtol=1e-6, atol=1e-8)


def test_printed_residual_sign_is_never_positive(rule3):
    # reading of Alg. 1: 0.5*dbeta.G <= 0 always, so res = -0.5*dbeta.G is used
    rng = np.random.default_rng(14)
    beta = _random_state(rng, C=1)
    M = maxent.model_moments(beta, rule3["Phi"], rule3["logw"])
    M[:, 1:] += 0.02 * rng.normal(size=(1, 34))
    G = maxent.gradient(beta, M, rule3["Phi"], rule3["logw"])[0, 1:]
    H = maxent.hessian(beta, M, rule3["Phi"], rule3["logw"])[0, 1:, 1:]
    d = -np.linalg.solve(H, G)
    assert 0.5 * d @ G < 0


def test_shifted_cholesky_on_indefinite_matrix():
    A = np.diag([1.0, 2.0, -1e-4, 3.0])
    L, lam = maxent._shifted_cholesky(A, 1e-3, 10.0)
    assert lam == pytest.approx(1e-3)
    assert np.allclose(L @ L.T, A + lam * np.eye(4))
    L2, lam2 = maxent._shifted_cholesky(np.eye(3), 1e-3, 10.0)
    assert lam2 == 0.0


def test_newton_reaches_fp64_floor_on_mott_smith(rule3):
    cells = mem_inputs.mott_smith_cells(24, config=2, replica=7)
    M = cells["M"]
    out = maxent.newton_solve(M, mem_inputs.maxwellian_beta(24, 35, M[:, 0]),
                              rule3["Phi"], rule3["logw"])
    assert out["converged"].all()
    assert np.max(out["resid"]) < 1e-12
    r = maxent.moment_residual(out["beta"], M, rule3["Phi"], rule3["logw"])
    assert np.max(r) < 1e-12
    assert np.max(out["iters"]) <= 40


def test_newton_solution_unique_from_other_start(rule3):
    cells = mem_inputs.mott_smith_cells(6, config=2, replica=8)
    M = cells["M"]
    b1 = maxent.newton_solve(M, mem_inputs.maxwellian_beta(6, 35, M[:, 0]),
                             rule3["Phi"], rule3["logw"])["beta"]
    start = mem_inputs.maxwellian_beta(6, 35, M[:, 0])
    start[:, 1:4] = 0.3  # a shifted Gaussian start
    b2 = maxent.newton_solve(M, start, rule3["Phi"], rule3["logw"], max_iter=400)["beta"]
    assert np.max(np.abs(b1 - b2)) < 1e-8


def test_newton_quadratic_convergence(rule3):
    cells = mem_inputs.mott_smith_cells(1, mach_lo=4.0, mach_hi=4.0, config=2, replica=9)
    M = cells["M"]
    beta = mem_inputs.maxwellian_beta(1, 35, M[:, 0])
    hist = []
    for k in range(1, 30):
        out = maxent.newton_solve(M, beta, rule3["Phi"], rule3["logw"], max_iter=k,
                                  tol_grad=0.0)
        hist.append(out["resid"][0])
        if hist[-1] < 1e-13:
            break
    # final steps: r_{k+1} <= C r_k^2 with a modest constant
    tail = [h for h in hist if 1e-13 < h < 1e-2]
    assert len(tail) >= 2
    for a, b in zip(tail[:-1], tail[1:]):
        assert b <= 50.0 * a * a + 1e-14


def test_config1_recovers_generating_beta(rule1):
    cand = mem_inputs.config1_candidates(2048)
    M, g, bgen = workloads.config1_targets(cand, 256)
    # targets are already in the generating gauge; solve at 16 nodes
    out = maxent.newton_solve(M, maxent.maxwellian_beta(M, 1), rule1["Phi"], rule1["logw"])
    assert out["converged"].all()
    err = np.max(np.abs(out["beta"] - bgen), axis=1)
    assert np.median(err) < 1e-4
    assert np.max(err) < 5e-3


def test_dual_value_lower_bound_at_solutions(rule3):
    # at a minimiser: logZ - beta.M/n = sum sigma log w~ - sum sigma log sigma >= min log w~
    cells = mem_inputs.mott_smith_cells(16, config=2, replica=12)
    M = cells["M"]
    out = maxent.newton_solve(M, mem_inputs.maxwellian_beta(16, 35, M[:, 0]),
                              rule3["Phi"], rule3["logw"])
    ok = out["converged"]
    v = maxent.dual_value(out["beta"][ok], M[ok], rule3["Phi"], rule3["logw"])
    sig = maxent.sigma(out["beta"][ok], rule3["Phi"], rule3["logw"])
    ent = -np.sum(sig * np.log(np.maximum(sig, 1e-300)), axis=1)
    assert np.allclose(v, sig @ rule3["logw"] + ent, rtol=1e-9, atol=1e-9)
    assert np.all(v >= np.min(rule3["logw"]))


def test_target_outside_node_hull_is_certified_nonrealizable(rule1):
    # mean velocity beyond the largest node: no distribution on the nodes has it
    M = np.array([[1.0, 7.0, 0.0, 0.0, 0.0]])
    out = maxent.newton_solve(M, maxent.maxwellian_beta(M, 1), rule1["Phi"], rule1["logw"])
    assert out["nonrealizable"][0] and not out["converged"][0]


def test_committed_config1_targets_are_the_oracles():
    """tests/golden/config1_targets.json (read by the bench's 1D leg) holds
    exactly what its oracle-only script computes."""
    import hashlib
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(here, "config1_targets.json")) as f:
        d = json.load(f)
    with open(os.path.join(here, "make_config1_targets.py"), "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest() == d["script_sha256"]
    M, g, b = workloads.config1_targets(mem_inputs.config1_candidates(4096), d["cells"])
    assert np.array_equal(np.asarray(d["M"]), M)
    assert np.array_equal(np.asarray(d["g"]), g)
    assert np.array_equal(np.asarray(d["beta_generating"]), b)
