"""Canonical-form exponential family, dual objective and modified Newton (oracle).

Test infrastructure only.  Follows, in the paper's notation:

* canonical form f = beta_0 exp(beta_i phi_i - log Z), i >= 1 (Sec. 2.2);
* log Z by the log-sum-exp trick over the quadrature nodes, with
  Q = max_p {beta_i phi_i(u_p) + log w_p} subtracted (Sec. 3.1, eq. "MLE
  optimization goal log sum exp"); sigma_p = exp(beta_i phi_i(u_p) + log w_p
  - log Z) is the discrete probability of node p (eq. "Numerical integration
  moments");
* dual objective L = log Z - beta_i M_i/n - n^2 (log beta_0 - beta_0/n),
  its gradient, and the Hessian: H_00 = n^2/beta_0^2, H_ij = Cov(phi_i, phi_j)
  for i, j >= 1, zero otherwise (App. C, eqs. "MLE optimization goal",
  "MLE optimization goal hessian", "correlation");
* Alg. 1: Newton with the Hessian shifted by lambda*I until Cholesky succeeds
  (lambda = 1e-3, x10), backtracking line search alpha = 1, 1/2, ... with at
  most 26 trials, and the Armijo test with the floating-point tolerance
  (c = 5e-4, atol = 5e-6, rtol = 5e-5).

Readings of the paper (also listed in the design doc): the convergence residual is
taken as res = -1/2 dbeta.G = 1/2 G^T (H+lambda I)^-1 G >= 0 (the printed
1/2 dbeta.grad L is never positive); beta_0 is held at n, which zeroes G_0 and
decouples the 0-block, so the Newton system is the (K-1)x(K-1) block; the
oracle stops on max_{i>=1} |G_i| <= tol_grad so that it reaches the FP64 floor.

Moments and the Hessian are direct weighted sums over nodes (Phi^T diag(sigma)
Phi), never a table of basis products.  The large dense sums and exponentials
run as plain PyTorch CPU operations in FP64 (threaded); the rest is NumPy.

Realizability on the node set (Sec. 2.3 discusses when beta exists): at a
minimiser sigma* matches the targets, so
    logZ(beta*) - beta*.M/n = sum_p sigma*_p log w~_p - sum_p sigma*_p log sigma*_p
                            >= min_p log w~_p.
An iterate whose value logZ - beta.M/n falls below min_p log w~_p therefore
certifies that the discrete dual has no minimiser (the targets lie outside the
moment set of distributions on the nodes); such cells stop as non-realizable.
"""

import numpy as np
import torch

def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))


def _exponent(beta, Phi, logw):
    """e[c, p] = sum_{i>=1} beta_i phi_i(u_p) + log w~_p (torch, FP64)."""
    return _t(beta[:, 1:]) @ _t(Phi[:, 1:]).T + _t(logw)[None, :]


def log_partition(beta, Phi, logw):
    """log Z(beta) by log-sum-exp.  beta: (C, K) with column 0 = beta_0 (unused)."""
    e = _exponent(beta, Phi, logw)
    q = torch.max(e, dim=1).values
    return (q + torch.log(torch.sum(torch.exp(e - q[:, None]), dim=1))).numpy()


def sigma(beta, Phi, logw, logZ=None):
    """Discrete probabilities sigma[c, p]."""
    if logZ is None:
        logZ = log_partition(beta, Phi, logw)
    e = _exponent(beta, Phi, logw)
    return torch.exp(e - _t(logZ)[:, None]).numpy()


def expectations(beta, Phi, logw):
    """E_sigma[phi_i] for every cell: (C, K)."""
    return sigma(beta, Phi, logw) @ Phi


def model_moments(beta, Phi, logw):
    """M_i(beta) = beta_0 sum_p sigma_p phi_i(u_p)."""
    return beta[:, :1] * expectations(beta, Phi, logw)


def second_moments(sig, Phi):
    """E_sigma[phi_i phi_j]: (C, K, K); row i is (sigma * phi_i) @ Phi over the nodes."""
    s, P = _t(sig), _t(Phi)
    C, K = s.shape[0], P.shape[1]
    out = torch.empty((C, K, K), dtype=torch.float64)
    for i in range(K):
        out[:, i, :] = (s * P[:, i]) @ P
    return out.numpy()


def objective(beta, M, Phi, logw):
    """Dual objective L(beta; M, phi) (App. C)."""
    n = M[:, 0]
    b0 = beta[:, 0]
    logZ = log_partition(beta, Phi, logw)
    return (logZ - np.sum(beta[:, 1:] * M[:, 1:], axis=1) / n
            - n ** 2 * (np.log(b0) - b0 / n))


def dual_value(beta, M, Phi, logw):
    """logZ(beta) - sum_{i>=1} beta_i M_i/n (L without its constant beta_0 term)."""
    return log_partition(beta, Phi, logw) - np.sum(beta[:, 1:] * M[:, 1:], axis=1) / M[:, 0]


def gradient(beta, M, Phi, logw):
    """dL/dbeta: G_0 = n - n^2/beta_0, G_i = E[phi_i] - M_i/n."""
    n = M[:, 0]
    E = expectations(beta, Phi, logw)
    G = E - M / n[:, None]
    G[:, 0] = n - n ** 2 / beta[:, 0]
    return G


def hessian(beta, M, Phi, logw):
    """d2L/dbeta2 (App. C): block-diagonal with the covariance block."""
    n = M[:, 0]
    sig = sigma(beta, Phi, logw)
    E = sig @ Phi
    S = second_moments(sig, Phi)
    H = S - E[:, :, None] * E[:, None, :]
    H[:, 0, :] = 0.0
    H[:, :, 0] = 0.0
    H[:, 0, 0] = n ** 2 / beta[:, 0] ** 2
    return H


def maxwellian_beta(M, dim):
    """Multipliers of the Maxwellian in its own Hermite gauge.

    With phi_(2) = (u^2 - 1)/sqrt(2) per axis, exp(-|u|^2/2) corresponds to
    beta = -1/sqrt(2) on each pure second-degree statistic (the constant is
    absorbed by log Z).  beta_0 = n.
    """
    from .basis import multi_indices
    idx = multi_indices(dim)
    beta = np.zeros((M.shape[0], len(idx)))
    beta[:, 0] = M[:, 0]
    for i, e in enumerate(idx):
        if sum(e) == 2 and max(e) == 2:
            beta[:, i] = -1.0 / np.sqrt(2.0)
    return beta


def _shifted_cholesky(H, lambda0, lambda_mul, max_shifts=60):
    """Alg. 1: Cholesky of H, else of H + lambda I with lambda growing x10."""
    try:
        return np.linalg.cholesky(H), 0.0
    except np.linalg.LinAlgError:
        pass
    lam = lambda0
    eye = np.eye(H.shape[0])
    for _ in range(max_shifts):
        try:
            return np.linalg.cholesky(H + lam * eye), lam
        except np.linalg.LinAlgError:
            lam *= lambda_mul
    return None, lam


def newton_solve(M, beta_init, Phi, logw, tol_grad=1e-12, tol_dec=0.0,
                 max_iter=200, max_ls=25, c=5e-4, atol=5e-6, rtol=5e-5,
                 lambda0=1e-3, lambda_mul=10.0, alpha_min=1e-6, want_cond=False):
    """Alg. 1 for a batch of independent cells (FP64).

    Returns dict with beta (C, K), iters, resid (max_{i>=1}|G_i| at the
    returned beta), converged, stagnated, nonrealizable (certified by the
    lower bound min_p log w~_p on the dual value at a minimiser), shifted
    (lambda used at least once), cond (condition number of the last
    unshifted covariance block).
    """
    M = np.asarray(M, dtype=np.float64)
    C, K = M.shape
    n = M[:, 0]
    beta = np.array(beta_init, dtype=np.float64, copy=True)
    beta[:, 0] = n
    dbeta = np.zeros_like(beta)
    alpha = np.ones(C)
    iters = np.zeros(C, dtype=np.int64)
    resid = np.full(C, np.inf)
    converged = np.zeros(C, dtype=bool)
    stagnated = np.zeros(C, dtype=bool)
    shifted = np.zeros(C, dtype=bool)
    nonreal = np.zeros(C, dtype=bool)
    cond = np.zeros(C)
    active = np.ones(C, dtype=bool)
    lmin = np.min(logw)

    for _ in range(max_iter + 1):
        act = np.nonzero(active)[0]
        if act.size == 0:
            break
        b, d, m = beta[act], dbeta[act], M[act]
        # --- BackTrackingLineSearch (alpha = 1, 1/2, ...; Armijo with tolerance)
        L0 = objective(b, m, Phi, logw)
        g0 = gradient(b, m, Phi, logw)
        a = np.full(act.size, 2.0)
        sat = np.zeros(act.size, dtype=bool)
        for _s in range(max_ls + 1):
            todo = ~sat
            if not todo.any():
                break
            a[todo] *= 0.5
            step = a[todo, None] * d[todo]
            gradD = -c * np.sum(g0[todo] * step, axis=1)
            LD = L0[todo] - objective(b[todo] + step, m[todo], Phi, logw)
            sat[todo] = (LD - gradD) >= -(atol + rtol * np.abs(LD))
        b = b + a[:, None] * d
        b[:, 0] = m[:, 0]
        beta[act] = b
        alpha[act] = a
        # --- Hessian and gradient at the updated beta (one sigma evaluation)
        sig = sigma(b, Phi, logw)
        E = sig @ Phi
        G = E[:, 1:] - m[:, 1:] / m[:, :1]
        H = second_moments(sig, Phi)[:, 1:, 1:] - E[:, 1:, None] * E[:, None, 1:]
        r = np.max(np.abs(G), axis=1)
        resid[act] = r
        newd = np.zeros((act.size, K))
        res = np.zeros(act.size)
        # Cholesky of every unshifted block at once; where any block needs the
        # lambda shift, every cell takes the per-cell loop below instead
        try:
            Lb = np.linalg.cholesky(H) if act.size else None
        except np.linalg.LinAlgError:
            Lb = None
        if Lb is not None:
            w = np.linalg.solve(Lb, -G[:, :, None])
            newd[:, 1:] = np.linalg.solve(np.swapaxes(Lb, 1, 2), w)[:, :, 0]
            res = 0.5 * np.sum(w[:, :, 0] ** 2, axis=1)
            if want_cond:
                ev = np.linalg.eigvalsh(H)
                with np.errstate(divide="ignore"):
                    cond[act] = np.where(ev[:, 0] > 0, ev[:, -1] / ev[:, 0], np.inf)
        for j in range(act.size if Lb is None else 0):
            Lh, lam = _shifted_cholesky(H[j], lambda0, lambda_mul)
            if lam > 0:
                shifted[act[j]] = True
            if Lh is None:
                res[j] = np.nan
                continue
            w = np.linalg.solve(Lh, -G[j])
            newd[j, 1:] = np.linalg.solve(Lh.T, w)
            res[j] = 0.5 * np.dot(w, w)
            if want_cond:
                ev = np.linalg.eigvalsh(H[j])
                cond[act[j]] = ev[-1] / ev[0] if ev[0] > 0 else np.inf
        dbeta[act] = newd
        iters[act] += 1
        done_grad = r <= tol_grad
        done_dec = res <= tol_dec
        stag = a <= alpha_min
        below = dual_value(b, m, Phi, logw) < lmin
        fin = done_grad | done_dec | stag | below | ~np.isfinite(res)
        converged[act] = done_grad | done_dec
        nonreal[act] = below & ~(done_grad | done_dec)
        stagnated[act] = stag & ~(done_grad | done_dec) & ~below
        active[act[fin]] = False
        over = iters > max_iter
        active &= ~over
    return dict(beta=beta, iters=iters, resid=resid, converged=converged,
                stagnated=stagnated, nonrealizable=nonreal, shifted=shifted, cond=cond,
                alpha=alpha)


def moment_residual(beta, M, Phi, logw):
    """Relative moment residual r = max_{i>=1} |E_sigma[phi_i] - M_i/n| (FP64)."""
    beta = np.asarray(beta, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    E = expectations(beta, Phi, logw)
    return np.max(np.abs(E[:, 1:] - M[:, 1:] / M[:, :1]), axis=1)
