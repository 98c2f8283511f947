// 1D velocity (5-moment) maximal-entropy solve and Hermite gauge on gfx950.
//
// With K = 5 and at most 64 nodes every quantity of one cell fits in
// registers, so one thread runs the whole of Alg. 1 for its cell: log-sum-exp
// pass (Sec. 3.1), moments and the 4 x 4 covariance Hessian (App. C),
// Cholesky with the lambda*I shift, Newton direction and the Armijo
// backtracking line search.  The node table (phi_0..phi_4, log w~) is staged
// in LDS once per workgroup.
#include <cfloat>
#include <cmath>

#include "mem_internal.h"

namespace memk {

namespace {

struct Lse1 { float logZ, L; };

__device__ __forceinline__ Lse1 lse1(const float* sT, int Q, const float* bt, const float* mn) {
  float mx = -FLT_MAX, sm = 0.f;
  for (int q = 0; q < Q; ++q) {
    const float* r = sT + q * 8;
    const float e = r[5] + bt[1] * r[1] + bt[2] * r[2] + bt[3] * r[3] + bt[4] * r[4];
    if (e > mx) { sm *= __expf(mx - e); mx = e; }
    sm += __expf(e - mx);
  }
  const float lz = mx + __logf(sm);
  return {lz, lz - (bt[1] * mn[1] + bt[2] * mn[2] + bt[3] * mn[3] + bt[4] * mn[4])};
}

// Cholesky of a 4 x 4 SPD matrix (lower, in place); false on a bad pivot
template <typename T>
__device__ __forceinline__ bool chol4(T (&A)[4][4], T& dmin, T& dmax) {
  dmin = (T)3.0e38f; dmax = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T d = A[k][k];
#pragma unroll
    for (int j = 0; j < k; ++j) d -= A[k][j] * A[k][j];
    if (!(d > 0) || !isfinite(d)) return false;
    dmin = d < dmin ? d : dmin; dmax = d > dmax ? d : dmax;
    const T lkk = sqrt(d);
    A[k][k] = lkk;
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      T s = A[i][k];
#pragma unroll
      for (int j = 0; j < k; ++j) s -= A[i][j] * A[k][j];
      A[i][k] = s / lkk;
    }
  }
  return true;
}

// direction d = -(L L^T)^-1 G and decrement 1/2 |L^-1 G|^2
template <typename T>
__device__ __forceinline__ void solve4(const T (&L)[4][4], const T (&G)[4], T (&d)[4], T& res) {
  T w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T s = -G[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= L[i][k] * w[k];
    w[i] = s / L[i][i];
  }
  res = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) res += w[i] * w[i];
  res *= (T)0.5;
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    T s = w[i];
#pragma unroll
    for (int k = i + 1; k < 4; ++k) s -= L[k][i] * d[k];
    d[i] = s / L[i][i];
  }
}

}  // namespace

__global__ __launch_bounds__(128) void k_solve1(int64_t n, int Q, const float* __restrict__ tab,
                                                const float* __restrict__ M,
                                                float* __restrict__ beta, SolveParams p,
                                                int32_t* iters_out, float* resid_out,
                                                uint32_t* status_out) {
  __shared__ float sT[Q1MAX * 8];
  for (int i = threadIdx.x; i < Q * 8; i += blockDim.x) sT[i] = tab[i];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float m[5], b[5];
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    m[k] = M[c * 5 + k];
    b[k] = beta[c * 5 + k];
    fin = fin && isfinite(m[k]) && (k == 0 || isfinite(b[k]));
  }
  uint32_t st = 0;
  int it = 0;
  float r = INFINITY;
  if (!fin) st = MEM_ST_NONFINITE;
  else if (!(m[0] > 0.f)) st = MEM_ST_NONREALIZABLE;
  if (st == 0) {
    const float nn = m[0];
    float mn[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) mn[k] = m[k] / nn;
    b[0] = nn;
    Lse1 cur = lse1(sT, Q, b, mn);
    float d[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    float alpha = 1.f, gdot = 0.f;
    for (;;) {
      if (it > 0) {  // BackTrackingLineSearch of Alg. 1
        float a = 1.f;
        for (int s = 0;; ++s) {
          float bt[5];
#pragma unroll
          for (int k = 0; k < 5; ++k) bt[k] = b[k] + a * d[k];
          const Lse1 tr = lse1(sT, Q, bt, mn);
          const float LD = cur.L - tr.L;
          const float gradD = -p.c * a * gdot;
          const bool sat = (LD - gradD) >= -(p.atol + p.rtol * fabsf(LD));
          if (sat || s >= p.max_ls) {
#pragma unroll
            for (int k = 1; k < 5; ++k) b[k] = bt[k];
            cur = tr;
            alpha = a;
            break;
          }
          a *= 0.5f;
        }
      }
      // moments, gradient and covariance Hessian at b
      float E[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, S2[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) S2[i][j] = 0.f;
      for (int q = 0; q < Q; ++q) {
        const float* rw = sT + q * 8;
        const float e = rw[5] + b[1] * rw[1] + b[2] * rw[2] + b[3] * rw[3] + b[4] * rw[4];
        const float sg = __expf(e - cur.logZ);
#pragma unroll
        for (int i = 0; i < 5; ++i) E[i] += sg * rw[i];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j) S2[i][j] += sg * rw[i + 1] * rw[j + 1];
      }
      const float inv0 = 1.f / E[0];
      float G[4], H[4][4];
      r = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        G[i] = E[i + 1] * inv0 - mn[i + 1];
        r = fmaxf(r, fabsf(G[i]));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = i > j ? i : j, bb = i > j ? j : i;
          H[i][j] = S2[a][bb] * inv0 - (E[i + 1] * inv0) * (E[j + 1] * inv0);
        }
      ++it;
      float dd[4], res = 0.f;
      bool ok;
      {
        float A[4][4], dmin, dmax;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) A[i][j] = H[i][j];
        ok = chol4(A, dmin, dmax);
        if (p.fp64_ratio > 0.f && (!ok || dmin < p.fp64_ratio * dmax)) {
          // FP64 direction for a small pivot ratio, with the lambda*I shift
          double Ad[4][4], Gd[4], ddd[4], rs, dn, dx;
          st |= MEM_ST_FP64;
          double lam = 0.0;
          for (int tries = 0; tries < 41; ++tries) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j) Ad[i][j] = (double)H[i][j] + (i == j ? lam : 0.0);
            ok = chol4(Ad, dn, dx);
            if (ok) break;
            lam = tries == 0 ? (double)p.lambda0 : lam * (double)p.lambda_mul;
            st |= MEM_ST_SHIFTED;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) Gd[i] = (double)G[i];
          solve4(Ad, Gd, ddd, rs);
#pragma unroll
          for (int i = 0; i < 4; ++i) dd[i] = (float)ddd[i];
          res = (float)rs;
        } else {
          float lam = p.lambda0;
          for (int tries = 0; tries < 40 && !ok; ++tries, lam *= p.lambda_mul) {
            st |= MEM_ST_SHIFTED;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j) A[i][j] = H[i][j] + (i == j ? lam : 0.f);
            ok = chol4(A, dmin, dmax);
          }
          solve4(A, G, dd, res);
        }
      }
      gdot = 0.f;
      bool dfin = ok;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        d[i + 1] = dd[i];
        gdot += G[i] * dd[i];
        dfin = dfin && isfinite(dd[i]);
      }
      if (r <= p.tol_grad || (res <= p.tol_dec && r <= p.tol_loose)) { st |= MEM_ST_CONVERGED; break; }
      if (cur.L < p.lmin) { st |= MEM_ST_NONREALIZABLE; break; }  // no minimiser exists
      if (p.beta_max > 0.f && fmaxf(fmaxf(fabsf(b[1]), fabsf(b[2])), fmaxf(fabsf(b[3]), fabsf(b[4]))) > p.beta_max) {
        st |= MEM_ST_NONREALIZABLE;
        break;
      }
      if (!isfinite(r) || !dfin) { st |= MEM_ST_NONFINITE; break; }
      if (alpha <= p.alpha_min) { st |= MEM_ST_STAGNATED; break; }
      if (it >= p.max_iter) { st |= MEM_ST_MAXITER; break; }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) beta[c * 5 + k] = b[k];
  }
  if (iters_out) iters_out[c] = it;
  if (resid_out) resid_out[c] = r;
  if (status_out) status_out[c] = st;
}

// ---- 1D Hermite gauge ---------------------------------------------------------
// h_m(b; c) = E[He_m(X)], X ~ N(b, 1 + c)
__device__ __forceinline__ void hpoly(float b, float c, float (&h)[5]) {
  h[0] = 1.f;
  h[1] = b;
  h[2] = b * b + c;
  h[3] = b * b * b + 3.f * b * c;
  h[4] = b * b * b * b + 6.f * b * b * c + 3.f * c * c;
}

// t[n][k]: phi_n(a x + b) = sum_k t[n][k] phi_k(x) for the orthonormal He basis
__device__ __forceinline__ void conn1d(float a, float b, float (&t)[5][5]) {
  const float binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                             {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
  const float sfact[5] = {1.f, 1.f, 1.41421356237f, 2.44948974278f, 4.89897948557f};
  float h[5];
  hpoly(b, a * a - 1.f, h);
  float ak[5] = {1.f, a, a * a, a * a * a, a * a * a * a};
#pragma unroll
  for (int nn = 0; nn < 5; ++nn)
#pragma unroll
    for (int k = 0; k < 5; ++k)
      t[nn][k] = k <= nn ? binom[nn][k] * ak[k] * h[nn - k] * sfact[k] / sfact[nn] : 0.f;
}

__global__ void k_gauge1(int64_t n, float* __restrict__ M, float* __restrict__ beta,
                         float* __restrict__ g) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float m[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) m[k] = M[c * 5 + k];
  const float w = g[c * 2], s = g[c * 2 + 1];
  const float nn = m[0];
  if (!(nn > 0.f) || !(s > 0.f)) return;
  const float m1 = m[1] / nn;
  const float exx = (1.41421356237f * m[2] + nn) / nn;
  const float var = exx - m1 * m1;
  if (!(var > 0.f) || !isfinite(var)) return;
  const float wH = w + s * m1, sH = s * sqrtf(var);
  float t[5][5];
  conn1d(s / sH, (w - wH) / sH, t);   // T(g_H, g)
  float mo[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k <= i; ++k) acc += t[i][k] * m[k];
    mo[i] = acc;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) M[c * 5 + k] = mo[k];
  if (beta) {
    float ti[5][5], b[5];
    conn1d(sH / s, (wH - w) / s, ti);   // T(g, g_H); alpha' = T^T alpha
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = beta[c * 5 + k];
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      float acc = 0.f;
#pragma unroll
      for (int j = i; j < 5; ++j) acc += ti[j][i] * b[j];
      beta[c * 5 + i] = acc;
    }
  }
  g[c * 2] = wH;
  g[c * 2 + 1] = sH;
}

hipError_t launch_solve1(mem_ctx_t c, int64_t n, const float* M, float* beta,
                         const SolveParams& p, int32_t* iters, float* resid, uint32_t* status,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_solve1<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(n, c->Q, c->d_tab1, M, beta, p, iters, resid,
                                                       status);
  return hipGetLastError();
}

hipError_t launch_gauge1(mem_ctx_t c, int64_t n, float* M, float* beta, float* g, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  (void)c;
  k_gauge1<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, M, beta, g);
  return hipGetLastError();
}

}  // namespace memk
