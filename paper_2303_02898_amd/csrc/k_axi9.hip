// The paper's own velocity discretisation on gfx950: nine statistics of
// (u_x, u_r) for 1D flow with cylindrical symmetry (appendix on the 35-moment
// system, orthogonal form), integrated with block-wise Gauss--Legendre over a
// truncated box fixed in physical velocity (end of Sec. 3.1).
//
// Because the nodes do not move with the gauge, every cell evaluates the
// statistics at its own u_bar_p = ((u_x,p - w_x)/s_x, u_r,p/s_r) (Sec. 3.3):
// there is no Phi shared by the batch and the moment/Hessian assembly is a
// per-cell weighted Gram matrix of 9 columns (45 distinct sums), work for the
// vector ALU rather than the matrix cores.  One wave runs the whole of Alg. 1
// for one cell: the lanes stride over the nodes, the 45 sums are reduced
// through LDS in a fixed order, and every lane then holds the same 8 x 8
// Hessian, factorises it and takes the same uniform decisions.
//
// Statistics, x = u_bar_x and y = u_bar_r^2/2 (Hermite in x, Laguerre in y):
//   1, x, He_2/sqrt2, y-1, He_3/sqrt6, He_4/sqrt24, y^2/2-2y+1, x(y-1),
//   He_2/sqrt2 (y-1).
#include <cfloat>
#include <cmath>

#include "dfloat.h"
#include "mem_internal.h"

namespace memk {

namespace {

constexpr int NA = 45;          // sum sigma, 8 first moments, 36 second moments
constexpr int AXW = 1;          // waves (cells) per workgroup: a slow cell holds only its own slot
constexpr int RSTRIDE = NA;     // odd row stride of the reduction area: no bank conflicts

struct AxGauge { float w, isx, isr; };

// Exponent lw_p + sum_i beta_i phi_i(u_bar_p) and the statistics at node p, in
// FP32.  The exponent adds terms of size ~10 that largely cancel where sigma
// is not small, so its absolute rounding error is relative error of sigma.
// Two things keep it near 1e-6 there:
//  * the coordinate u_x - w: the node's u_x arrives as hi + lo (the FP32
//    rounding of the FP64 node and its remainder), and hi - w is exact when the
//    two are within a factor of two (or rounded relative to the difference,
//    which then puts sigma far out in the tail), so x carries relative error
//    ~1e-7 instead of the 1e-6 absolute that rounding u_x alone would leave at
//    Mach-10 velocities;
//  * the sum itself: with x accurate, its rounding is ~(|lw| + sum |b_i phi_i|)
//    2^-24 ~ 1e-6 where sigma matters.
// The statistics used in the sums are the same FP32 values.
__device__ __forceinline__ float expo9(const float4& nd, const AxGauge& g, const float (&b)[9],
                                       float (&f)[9]) {
  const float x = ((nd.x - g.w) + nd.w) * g.isx;
  const float t = nd.y * g.isr;
  const float y = 0.5f * t * t;
  const float x2 = x * x;
  const float ym = y - 1.f;
  const float p2 = (x2 - 1.f) * 0.70710678118654752f;
  f[0] = 1.f;
  f[1] = x;
  f[2] = p2;
  f[3] = ym;
  f[4] = x * (x2 - 3.f) * 0.40824829046386302f;
  f[5] = fmaf(x2, x2 - 6.f, 3.f) * 0.20412414523193151f;
  f[6] = fmaf(0.5f * y, y, fmaf(-2.f, y, 1.f));
  f[7] = x * ym;
  f[8] = p2 * ym;
  float e = nd.z;
#pragma unroll
  for (int i = 1; i < 9; ++i) e = fmaf(b[i], f[i], e);
  return e;
}

// The cell's gauge (FP32: the statistics are defined with exactly these values).
__device__ __forceinline__ AxGauge ax_gauge(const float* gin, int64_t c) {
  return {gin[c * 3], 1.f / gin[c * 3 + 1], 1.f / gin[c * 3 + 2]};
}

// log Z(b) by the log-sum-exp of Sec. 3.1: a running (max, scaled sum) per
// lane over groups of four nodes (one rescale per group), then a butterfly
// over the wave.  Every lane returns the same value.
__device__ float lse9(const float4* __restrict__ tab, int P, const AxGauge& g, const float (&b)[9],
                      int lane) {
  float mx = -FLT_MAX, sm = 0.f;
  for (int q0 = lane; q0 < P; q0 += 4 * 64) {
    float e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = q0 + 64 * k;
      float f[9];
      e[k] = q < P ? expo9(tab[q], g, b, f) : -INFINITY;
    }
    const float m = fmaxf(fmaxf(mx, fmaxf(e[0], e[1])), fmaxf(e[2], e[3]));
    float s = sm * __expf(mx - m);
#pragma unroll
    for (int k = 0; k < 4; ++k) s += __expf(e[k] - m);
    sm = s;
    mx = m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float om = __shfl_xor(mx, off), os = __shfl_xor(sm, off);
    const float m = fmaxf(mx, om);
    sm = sm * __expf(mx - m) + os * __expf(om - m);
    mx = m;
  }
  return mx + __logf(sm);
}

// The 45 sums of sigma, sigma phi_i and sigma phi_i phi_j (1 <= i <= j <= 8) at
// b with sigma_p = exp(e_p - logZ), reduced over the wave in a fixed order;
// every lane gets all 45 in A.
__device__ void assemble9(const float4* __restrict__ tab, int P, const AxGauge& g,
                          const float (&b)[9], float logZ, int lane, float* red,
                          float (&A)[NA]) {
#pragma unroll
  for (int k = 0; k < NA; ++k) A[k] = 0.f;
  // the next node's entry is loaded one step ahead (one wave per SIMD leaves
  // no other wave to cover the load latency)
  float4 nd = lane < P ? tab[lane] : make_float4(0.f, 1.f, 0.f, 0.f);
  for (int q = lane; q < P; q += 64) {
    const float4 cur = nd;
    if (q + 64 < P) nd = tab[q + 64];
    float f[9];
    const float s = __expf(expo9(cur, g, b, f) - logZ);
    A[0] += s;
    float t[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      t[i] = s * f[i];
      A[i] += t[i];
    }
    int k = 9;
#pragma unroll
    for (int i = 1; i < 9; ++i)
#pragma unroll
      for (int j = i; j < 9; ++j) {
        A[k] = fmaf(t[i], f[j], A[k]);
        ++k;
      }
  }
#pragma unroll
  for (int k = 0; k < NA; ++k) red[lane * RSTRIDE + k] = A[k];
  __builtin_amdgcn_wave_barrier();
  float tot = 0.f;
  if (lane < NA)
    for (int l = 0; l < 64; ++l) tot += red[l * RSTRIDE + lane];
  __builtin_amdgcn_wave_barrier();
  if (lane < NA) red[64 * RSTRIDE + lane] = tot;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int k = 0; k < NA; ++k) A[k] = red[64 * RSTRIDE + k];
  __builtin_amdgcn_wave_barrier();
}

// Packed lower triangle of an 8 x 8 matrix: entry (i, j), j <= i, at PK(i, j).
__host__ __device__ constexpr int PK(int i, int j) { return i * (i + 1) / 2 + j; }
// Upper-triangle position of E_sigma[phi_i phi_j] (1 <= i <= j <= 8 as 0-based
// i <= j < 8) among the 45 sums.
__host__ __device__ constexpr int UA(int i, int j) { return 9 + 8 * i - i * (i - 1) / 2 + (j - i); }

// Cholesky of an 8 x 8 SPD matrix in packed lower storage (in place); false on
// a bad pivot
template <typename T>
__device__ __forceinline__ bool chol8(T (&A)[36], T& dmin, T& dmax) {
  dmin = (T)3.0e38f; dmax = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    T d = A[PK(k, k)];
#pragma unroll
    for (int j = 0; j < k; ++j) d -= A[PK(k, j)] * A[PK(k, j)];
    if (!(d > 0) || !isfinite(d)) return false;
    dmin = d < dmin ? d : dmin; dmax = d > dmax ? d : dmax;
    const T lkk = sqrt(d);
    A[PK(k, k)] = lkk;
#pragma unroll
    for (int i = k + 1; i < 8; ++i) {
      T s = A[PK(i, k)];
#pragma unroll
      for (int j = 0; j < k; ++j) s -= A[PK(i, j)] * A[PK(k, j)];
      A[PK(i, k)] = s / lkk;
    }
  }
  return true;
}

// Lower bound of cond(H) for the conditioning monitor (Sec. 3.5), H SPD in
// packed storage with its Cholesky factor L (packed) and smallest pivot dmin:
// for unit vectors v, u, |H v| <= lambda_max and |H^-1 u| <= 1 / lambda_min,
// so |H v| |H^-1 u| <= cond(H).  v and u come from CE_ITERS steps of power and
// inverse iteration from (1, ..., 1)/sqrt 8; the bound max_i H_ii / dmin (every
// pivot lies between the extreme eigenvalues) is folded in.
constexpr int CE_ITERS = 6;
__device__ __forceinline__ float cond_est8(const float (&H)[36], const float (&L)[36],
                                           float dmin) {
  float v[8], u[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = u[i] = 0.35355339059327376f;
  float nv = 0.f, nu = 0.f;
  for (int k = 0; k < CE_ITERS; ++k) {
    float w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < 8; ++j) s += H[i >= j ? PK(i, j) : PK(j, i)] * v[j];
      w[i] = s;
    }
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) q += w[i] * w[i];
    nv = sqrtf(q);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = w[i] / nv;
    // w = (L L^T)^-1 u
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float s = u[i];
#pragma unroll
      for (int j = 0; j < i; ++j) s -= L[PK(i, j)] * w[j];
      w[i] = s / L[PK(i, i)];
    }
#pragma unroll
    for (int i = 7; i >= 0; --i) {
      float s = w[i];
#pragma unroll
      for (int j = i + 1; j < 8; ++j) s -= L[PK(j, i)] * w[j];
      w[i] = s / L[PK(i, i)];
    }
    q = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) q += w[i] * w[i];
    nu = sqrtf(q);
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = w[i] / nu;
  }
  float hmax = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) hmax = fmaxf(hmax, H[PK(i, i)]);
  const float est = nv * nu;
  return isfinite(est) ? fmaxf(est, hmax / dmin) : INFINITY;
}

// direction d = -(L L^T)^-1 G and decrement 1/2 |L^-1 G|^2 (L packed)
template <typename T>
__device__ __forceinline__ void solve8(const T (&L)[36], const T (&G)[8], T (&d)[8], T& res) {
  T w[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    T s = -G[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= L[PK(i, k)] * w[k];
    w[i] = s / L[PK(i, i)];
  }
  res = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) res += w[i] * w[i];
  res *= (T)0.5;
#pragma unroll
  for (int i = 7; i >= 0; --i) {
    T s = w[i];
#pragma unroll
    for (int k = i + 1; k < 8; ++k) s -= L[PK(k, i)] * d[k];
    d[i] = s / L[PK(i, i)];
  }
}

// The same two steps in FP64 on a wave's LDS area (all lanes hold the same
// values): the rare FP64 direction then costs no registers, which keeps the
// kernel at three waves per SIMD without spills.
__device__ __forceinline__ bool chol8_lds(double* A, double& dmin, double& dmax) {
  dmin = 3.0e38; dmax = 0.0;
  for (int k = 0; k < 8; ++k) {
    double d = A[PK(k, k)];
    for (int j = 0; j < k; ++j) d -= A[PK(k, j)] * A[PK(k, j)];
    if (!(d > 0.0) || !isfinite(d)) return false;
    dmin = d < dmin ? d : dmin; dmax = d > dmax ? d : dmax;
    const double lkk = sqrt(d);
    A[PK(k, k)] = lkk;
    for (int i = k + 1; i < 8; ++i) {
      double t = A[PK(i, k)];
      for (int j = 0; j < k; ++j) t -= A[PK(i, j)] * A[PK(k, j)];
      A[PK(i, k)] = t / lkk;
    }
  }
  return true;
}

__device__ __forceinline__ double solve8_lds(const double* L, const double* G, double* w, double* d) {
  for (int i = 0; i < 8; ++i) {
    double t = -G[i];
    for (int k = 0; k < i; ++k) t -= L[PK(i, k)] * w[k];
    w[i] = t / L[PK(i, i)];
  }
  double res = 0.0;
  for (int i = 0; i < 8; ++i) res += w[i] * w[i];
  for (int i = 7; i >= 0; --i) {
    double t = w[i];
    for (int k = i + 1; k < 8; ++k) t -= L[PK(k, i)] * d[k];
    d[i] = t / L[PK(i, i)];
  }
  return 0.5 * res;
}

// FP32 residual floor.  A residual that has not halved for AX_FLOOR_WINDOW
// iterations has reached the rounding floor of the FP32 moments.  Where that
// floor lies at or below half of tol_grad_loose the cell is converged: the
// moments carry ~1e-6 of FP32 evaluation error (see expo9), so its residual in exact arithmetic stays within tol_grad_loose.
// A floor above that ends the cell as stagnated after AX_STALL_WINDOW
// iterations below AX_STALL_GATE.  Above the gate there is no such window:
// on a wide box the damped phase of Newton from the Maxwellian start can keep
// the residual from halving for 30-40 iterations (the FP64 oracle shows the
// same), and only the step-size and iteration-budget exits apply.
constexpr int AX_FLOOR_WINDOW = 6;
constexpr int AX_STALL_WINDOW = 20;
constexpr float AX_STALL_GATE = 1e-3f;

struct Lse9 { float logZ, L; };

__device__ __forceinline__ Lse9 value9(const float4* tab, int P, const AxGauge& g, const float (&b)[9],
                                       const float (&mn)[9], int lane) {
  const float lz = lse9(tab, P, g, b, lane);
  float bm = 0.f;
#pragma unroll
  for (int i = 1; i < 9; ++i) bm = fmaf(b[i], mn[i], bm);
  return {lz, lz - bm};
}

// Double-float constants 1/sqrt(2), 1/sqrt(6), 1/sqrt(24): the FP32 rounding
// and its remainder.
constexpr double RS2 = 0.70710678118654752440, RS6 = 0.40824829046386301637,
                 RS24 = 0.20412414523193150818;
constexpr dfl C_RS2{(float)RS2, (float)(RS2 - (double)(float)RS2)};
constexpr dfl C_RS6{(float)RS6, (float)(RS6 - (double)(float)RS6)};
constexpr dfl C_RS24{(float)RS24, (float)(RS24 - (double)(float)RS24)};

// Compensated gradient G_i = E_sigma[phi_i] - M_i / n (i = 1..8) at b, all in
// FP32 arithmetic: coordinates, statistics and exponent in double-float from
// the hi + lo parts of the nodes (tab for u_x, lo for u_r and log w), the
// gauge scales 1/s as quotient + remainder, sigma = exp(e - shift) (1 + e_lo),
// and double-float sums reduced over the wave in a fixed order.  The shift
// only keeps exp in range (it cancels in the quotients).  Returns max |G_i|;
// every lane gets G.
__device__ float grad9_acc(const float4* __restrict__ tab, const float2* __restrict__ lo, int P,
                           float gw, float gsx, float gsr, const float (&b)[9], float shift,
                           const float (&m)[9], int lane, float (&G)[8]) {
#pragma clang fp contract(off)
  const dfl isx = df_recip(gsx), isr = df_recip(gsr);
  dfl S[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) S[i] = {0.f, 0.f};
  for (int q = lane; q < P; q += 64) {
    const float4 nd = tab[q];
    const float2 nl = lo[q];
    float xs, xe;
    two_sum(nd.x, -gw, xs, xe);
    const dfl x = df_mul(df_norm({xs, xe + nd.w}), isx);
    const dfl t = df_mul({nd.y, nl.x}, isr);
    dfl y = df_mul(t, t);
    y = {0.5f * y.h, 0.5f * y.l};
    const dfl x2 = df_mul(x, x);
    const dfl ym = df_plus(y, -1.f);
    dfl f[9];
    f[1] = x;
    f[2] = df_mul(df_plus(x2, -1.f), C_RS2);
    f[3] = ym;
    f[4] = df_mul(df_mul(x, df_plus(x2, -3.f)), C_RS6);
    f[5] = df_mul(df_plus(df_mul(x2, df_plus(x2, -6.f)), 3.f), C_RS24);
    dfl y2 = df_mul(y, y);
    y2 = {0.5f * y2.h, 0.5f * y2.l};
    dfl f6 = y2;
    df_add(f6, {-2.f * y.h, -2.f * y.l});
    f[6] = df_plus(df_norm(f6), 1.f);
    f[7] = df_mul(x, ym);
    f[8] = df_mul(f[2], ym);
    dfl e = {nd.z, nl.y};
#pragma unroll
    for (int i = 1; i < 9; ++i) df_acc1(e, b[i], f[i]);
    e = df_plus(df_norm(e), -shift);
    if (e.h < -80.f) continue;  // weight below 1e-34: no measurable moment
    const float ex = expf(e.h);
    const float sg = fmaf(ex, e.l, ex);
    df_add(S[0], {sg, 0.f});
#pragma unroll
    for (int i = 1; i < 9; ++i) df_acc1(S[i], sg, f[i]);
  }
  // butterfly over the wave: the same fixed order on every lane
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const dfl o = {__shfl_xor(S[i].h, off), __shfl_xor(S[i].l, off)};
      df_add(S[i], o);
    }
  const float h0 = S[0].h, l0 = S[0].l, inv0 = 1.f / h0;
  const float nn = m[0];
  float r = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    // quotients as q1 + q2 with q2 from the exact remainder (fma)
    const float e1 = S[i + 1].h * inv0;
    const float e2 = (fmaf(-e1, h0, S[i + 1].h) + (S[i + 1].l - e1 * l0)) * inv0;
    const float m1 = m[i + 1] / nn;
    const float m2 = fmaf(-m1, nn, m[i + 1]) / nn;
    G[i] = (e1 - m1) + (e2 - m2);
    r = fmaxf(r, fabsf(G[i]));
  }
  return isfinite(r) ? r : INFINITY;
}

}  // namespace

__global__ __launch_bounds__(64 * AXW) void k_axi_solve(int64_t n, int P,
                                                        const float4* __restrict__ tab,
                                                        const float* __restrict__ M,
                                                        const float* __restrict__ gin,
                                                        float* __restrict__ beta, SolveParams p,
                                                        int32_t* iters_out, float* resid_out,
                                                        uint32_t* status_out, float* cond_out) {
  __shared__ __align__(16) float sred[AXW][65 * RSTRIDE];
  __shared__ float sHk[AXW][36];  // the last FP32 Hessian, for the refinement
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * AXW + wv;
  if (c >= n) return;  // whole waves leave; no workgroup barrier follows
  float* red = sred[wv];
  float m[9], b[9];
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    m[k] = M[c * 9 + k];
    b[k] = beta[c * 9 + k];
    fin = fin && isfinite(m[k]) && (k == 0 || isfinite(b[k]));
  }
  const float gw = gin[c * 3], gsx = gin[c * 3 + 1], gsr = gin[c * 3 + 2];
  fin = fin && isfinite(gw) && isfinite(gsx) && isfinite(gsr);
  uint32_t st = 0;
  int it = 0;
  float r = INFINITY;
  // conditioning monitor (Sec. 3.5): cond_est8 of the FP32 Hessian at the
  // solve's last iterate (a lower bound of cond(H)); +inf where its Cholesky
  // fails; 0 for a cell that never assembled one
  float cmon = 0.f;
  if (!fin) st = MEM_ST_NONFINITE;
  else if (!(m[0] > 0.f) || !(gsx > 0.f) || !(gsr > 0.f)) st = MEM_ST_NONREALIZABLE;
  if (st == 0) {
    const AxGauge g{gw, 1.f / gsx, 1.f / gsr};
    const float nn = m[0];
    float mn[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) mn[k] = m[k] / nn;
    b[0] = nn;
    Lse9 cur = value9(tab, P, g, b, mn, lane);
    float d[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = 0.f;
    float alpha = 1.f, gdot = 0.f, rbest = INFINITY;
    int itbest = 0;
    for (;;) {
      if (it > 0) {  // BackTrackingLineSearch of Alg. 1
        float a = 1.f;
        for (int s = 0;; ++s) {
          float bt[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) bt[k] = b[k] + a * d[k];
          const Lse9 tr = value9(tab, P, g, bt, mn, lane);
          const float LD = cur.L - tr.L;
          const float gradD = -p.c * a * gdot;
          const bool sat = (LD - gradD) >= -(p.atol + p.rtol * fabsf(LD));
          if (sat || s >= p.max_ls) {
#pragma unroll
            for (int k = 1; k < 9; ++k) b[k] = bt[k];
            cur = tr;
            alpha = a;
            break;
          }
          a *= 0.5f;
        }
      }
      // moments, gradient and covariance Hessian at b (App. C)
      float A[NA];
      assemble9(tab, P, g, b, cur.logZ, lane, red, A);
      const float inv0 = 1.f / A[0];
      float E[8], G[8], Hp[36];
      r = 0.f;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        E[i] = A[1 + i] * inv0;
        G[i] = E[i] - mn[1 + i];
        r = fmaxf(r, fabsf(G[i]));
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) Hp[PK(i, j)] = A[UA(j, i)] * inv0 - E[i] * E[j];
      if (lane < 36) sHk[wv][lane] = Hp[lane];
      ++it;
      if (r < 0.5f * rbest) { rbest = r; itbest = it; }
      float dd[8], res = 0.f;
      bool ok;
      {
        float Af[36], dmin, dmax;
#pragma unroll
        for (int k = 0; k < 36; ++k) Af[k] = Hp[k];
        ok = chol8(Af, dmin, dmax);
        if (p.fp64_ratio > 0.f && (!ok || dmin < p.fp64_ratio * dmax)) {
          // FP64 direction for a small pivot ratio, with the lambda*I shift,
          // on the (now idle) reduction area: A[36], G[8], w[8], d[8]
          double* Ad = reinterpret_cast<double*>(red);
          double* Gd = Ad + 36;
          double dn, dx;
          st |= MEM_ST_FP64;
          double lam = 0.0;
          for (int tries = 0; tries < 41; ++tries) {
            for (int i = 0; i < 8; ++i)
              for (int j = 0; j <= i; ++j)
                Ad[PK(i, j)] = (double)Hp[PK(i, j)] + (i == j ? lam : 0.0);
            __builtin_amdgcn_wave_barrier();
            ok = chol8_lds(Ad, dn, dx);
            __builtin_amdgcn_wave_barrier();
            if (ok) break;
            lam = tries == 0 ? (double)p.lambda0 : lam * (double)p.lambda_mul;
            st |= MEM_ST_SHIFTED;
          }
          for (int i = 0; i < 8; ++i) Gd[i] = (double)G[i];
          __builtin_amdgcn_wave_barrier();
          res = (float)solve8_lds(Ad, Gd, Gd + 8, Gd + 16);
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int i = 0; i < 8; ++i) dd[i] = (float)Gd[16 + i];
          __builtin_amdgcn_wave_barrier();
        } else {
          float lam = p.lambda0;
          for (int tries = 0; tries < 40 && !ok; ++tries, lam *= p.lambda_mul) {
            st |= MEM_ST_SHIFTED;
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
              for (int j = 0; j <= i; ++j) Af[PK(i, j)] = Hp[PK(i, j)] + (i == j ? lam : 0.f);
            ok = chol8(Af, dmin, dmax);
          }
          solve8(Af, G, dd, res);
        }
      }
      gdot = 0.f;
      bool dfin = ok;
      float bmax = 0.f;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        d[i + 1] = dd[i];
        gdot += G[i] * dd[i];
        dfin = dfin && isfinite(dd[i]);
        bmax = fmaxf(bmax, fabsf(b[i + 1]));
      }
      if (r <= p.tol_grad || (res <= p.tol_dec && r <= p.tol_loose) ||
          (r <= 0.5f * p.tol_loose && it - itbest >= AX_FLOOR_WINDOW)) {
        st |= MEM_ST_CONVERGED;
        break;
      }
      if (cur.L < p.lmin) { st |= MEM_ST_NONREALIZABLE; break; }  // no minimiser exists
      if (p.beta_max > 0.f && bmax > p.beta_max) { st |= MEM_ST_NONREALIZABLE; break; }
      if (!isfinite(r) || !dfin) { st |= MEM_ST_NONFINITE; break; }
      if (alpha <= p.alpha_min ||
          (r <= AX_STALL_GATE &&
           it - itbest >= (p.stall_window > 0 ? p.stall_window : AX_STALL_WINDOW))) {
        st |= MEM_ST_STAGNATED;
        break;
      }
      if (it >= p.max_iter) { st |= MEM_ST_MAXITER; break; }
    }
    if (cond_out && it > 0) {  // the Hessian of the last direction, kept in sHk
      __builtin_amdgcn_wave_barrier();
      float Hk[36], Lk[36], dmin, dmax;
#pragma unroll
      for (int k = 0; k < 36; ++k) Lk[k] = Hk[k] = sHk[wv][k];
      cmon = chol8(Lk, dmin, dmax) ? cond_est8(Hk, Lk, dmin) : INFINITY;
    }
    // Compensated refinement (as the 35-moment path): the FP32 iteration stops
    // where its own rounding hides the residual; a cell that ended converged or
    // at that floor takes Newton corrections with the double-float gradient
    // and the last FP32 Hessian, keeping the best multipliers, and its final
    // status and residual are the compensated ones.
    if (p.refine > 0 && (st & (MEM_ST_CONVERGED | MEM_ST_STAGNATED)) &&
        !(st & (MEM_ST_NONFINITE | MEM_ST_NONREALIZABLE))) {
      __builtin_amdgcn_wave_barrier();
      float Lf[36], dmin, dmax;
#pragma unroll
      for (int k = 0; k < 36; ++k) Lf[k] = sHk[wv][k];
      bool okf = chol8(Lf, dmin, dmax);
      const float2* lo = reinterpret_cast<const float2*>(tab + P);
      float Ga[8];
      float ra = grad9_acc(tab, lo, P, gw, gsx, gsr, b, cur.logZ, m, lane, Ga);
      float bb[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) bb[k] = b[k];
      float rb = ra;
      for (int ref = 0; okf && !(ra <= p.tol_grad) && ref < p.refine; ++ref) {
        float dd[8], res;
        solve8(Lf, Ga, dd, res);
        bool fin = true;
#pragma unroll
        for (int i = 0; i < 8; ++i) fin = fin && isfinite(dd[i]);
        if (!fin) break;
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i + 1] += dd[i];
        ra = grad9_acc(tab, lo, P, gw, gsx, gsr, b, cur.logZ, m, lane, Ga);
        if (ra < rb) {
          rb = ra;
#pragma unroll
          for (int k = 0; k < 9; ++k) bb[k] = b[k];
        }
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) b[k] = bb[k];
      r = rb;
      st = rb <= p.tol_loose ? (st & ~MEM_ST_STAGNATED) | MEM_ST_CONVERGED
                             : (st & ~MEM_ST_CONVERGED) | MEM_ST_STAGNATED;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) beta[c * 9 + k] = b[k];
    if (iters_out) iters_out[c] = it;
    if (resid_out) resid_out[c] = r;
    if (status_out) status_out[c] = st;
    if (cond_out) cond_out[c] = cmon;
  }
}

// Moments and fluxes from multipliers (Sec. 3.1; flux line of the moment
// equations): M_i = beta_0 E_sigma[phi_i], F_i = beta_0 E_sigma[u_x phi_i] with
// u_x the physical velocity of the node; E_sigma normalised by sum_p sigma_p.
__global__ __launch_bounds__(64 * AXW) void k_axi_moments(int64_t n, int P,
                                                          const float4* __restrict__ tab,
                                                          const float* __restrict__ beta,
                                                          const float* __restrict__ gin,
                                                          float* __restrict__ M, float* __restrict__ F) {
  __shared__ float sred[AXW][65 * 19];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * AXW + wv;
  if (c >= n) return;
  float* red = sred[wv];
  float b[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) b[k] = beta[c * 9 + k];
  const AxGauge g = ax_gauge(gin, c);
  const float lz = lse9(tab, P, g, b, lane);
  float acc[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) acc[k] = 0.f;
  for (int q = lane; q < P; q += 64) {
    const float4 nd = tab[q];
    float f[9];
    const float s = __expf(expo9(nd, g, b, f) - lz);
    const float su = s * (nd.x + nd.w);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      acc[i] = fmaf(s, f[i], acc[i]);
      acc[9 + i] = fmaf(su, f[i], acc[9 + i]);
    }
  }
#pragma unroll
  for (int k = 0; k < 18; ++k) red[lane * 19 + k] = acc[k];
  __builtin_amdgcn_wave_barrier();
  if (lane < 18) {
    float tot = 0.f;
    for (int l = 0; l < 64; ++l) tot += red[l * 19 + lane];
    red[64 * 19 + lane] = tot;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < 9) {
    const float s0 = red[64 * 19];
    const float scale = (float)b[0] / s0;
    if (M) M[c * 9 + lane] = red[64 * 19 + lane] * scale;
    if (F) F[c * 9 + lane] = red[64 * 19 + 9 + lane] * scale;
  }
}

// ---- change of gauge (Sec. 3.3) ------------------------------------------------
// Statistic i is p_a(x) l_k(y) with p_a = He_a/sqrt(a!) and l_0 = 1,
// l_1 = y - 1, l_2 = y^2/2 - 2y + 1; (a, k) per index:
__constant__ int AX_A[9] = {0, 1, 2, 0, 3, 4, 0, 1, 2};
__constant__ int AX_K[9] = {0, 0, 0, 1, 0, 0, 2, 1, 1};

// p_n(a x + b) = sum_k t[n][k] p_k(x): t = C(n,k) a^k h_{n-k}(b; a^2 - 1) sqrt(k!/n!),
// h_m(b; c) = E[He_m(X)], X ~ N(b, 1 + c)
__device__ __forceinline__ void conn_x(float a, float b, float (&t)[5][5]) {
  const float c = a * a - 1.0f;
  const float h[5] = {1.0f, b, b * b + c, b * b * b + 3.0f * b * c,
                       b * b * b * b + 6.0f * b * b * c + 3.0f * c * c};
  const float binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                              {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
  const float sf[5] = {1.0f, 1.0f, 1.41421356237309505f, 2.44948974278317810f,
                        4.89897948556635620f};
  float ak = 1.0f;
  float apow[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) { apow[k] = ak; ak *= a; }
#pragma unroll
  for (int n = 0; n < 5; ++n)
#pragma unroll
    for (int k = 0; k < 5; ++k)
      t[n][k] = k <= n ? binom[n][k] * apow[k] * h[n - k] * sf[k] / sf[n] : 0.0f;
}

// l_k(c y) = sum_k' r[k][k'] l_k'(y) (dilation of the radial variable)
__device__ __forceinline__ void conn_y(float c, float (&r)[3][3]) {
  r[0][0] = 1.0f; r[0][1] = 0.0f; r[0][2] = 0.0f;
  r[1][0] = c - 1.0f; r[1][1] = c; r[1][2] = 0.0f;
  r[2][0] = (c - 1.0f) * (c - 1.0f); r[2][1] = 2.0f * c * (c - 1.0f); r[2][2] = c * c;
}

// T(g', g)_ij = t[a_i][a_j] r[k_i][k_j] with a = s_x/s_x', b = (w - w')/s_x',
// c = (s_r/s_r')^2
__device__ __forceinline__ float tij(const float (&t)[5][5], const float (&r)[3][3], int i,
                                      int j) {
  return t[AX_A[i]][AX_A[j]] * r[AX_K[i]][AX_K[j]];
}

// One thread per cell: Hermite gauge of the nine moments, M <- T(g_H, g) M,
// beta_i <- sum_j T(g, g_H)_ji beta_j (i >= 1), g <- g_H.  Cells with n <= 0,
// a non-positive variance or non-finite values are left unchanged.
__global__ void k_axi_gauge(int64_t n, float* __restrict__ M, float* __restrict__ beta,
                            float* __restrict__ g) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float m[9];
  bool fin = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    m[k] = M[c * 9 + k];
    fin = fin && isfinite(m[k]);
  }
  const float w = g[c * 3], sx = g[c * 3 + 1], sr = g[c * 3 + 2];
  if (!fin || !(m[0] > 0.0f) || !(sx > 0.0f) || !(sr > 0.0f)) return;
  const float m1 = m[1] / m[0];
  const float exx = 1.41421356237309505f * m[2] / m[0] + 1.0f;
  const float err = 2.0f * (m[3] / m[0] + 1.0f);
  const float vx = exx - m1 * m1;
  if (!(vx > 0.0f) || !(err > 0.0f) || !isfinite(vx) || !isfinite(err)) return;
  const float wH = w + sx * m1, sxH = sx * sqrtf(vx), srH = sr * sqrtf(0.5f * err);
  float t[5][5], r[3][3];
  conn_x(sx / sxH, (w - wH) / sxH, t);
  conn_y((sr / srH) * (sr / srH), r);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 9; ++j) acc += tij(t, r, i, j) * m[j];
    M[c * 9 + i] = (float)acc;
  }
  if (beta) {
    float b[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) b[k] = beta[c * 9 + k];
    conn_x(sxH / sx, (wH - w) / sx, t);
    conn_y((srH / sr) * (srH / sr), r);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      float acc = 0.0f;
#pragma unroll
      for (int j = 1; j < 9; ++j) acc += tij(t, r, j, i) * b[j];
      beta[c * 9 + i] = (float)acc;
    }
  }
  g[c * 3] = (float)wH;
  g[c * 3 + 1] = (float)sxH;
  g[c * 3 + 2] = (float)srH;
}

// ---- characteristic speeds (Sec. 3.4) ----------------------------------------
// dF/dM has the eigenvalues of the pencil (C, B), B = E[phi phi^T] and
// C = E[x phi phi^T] in gauge coordinates x = u_bar_x; physical speeds are
// w_x + s_x lambda, and the scheme needs the extreme two.  One wave per cell
// accumulates the 2 x 45 sums, reduced in LDS.  Every lane then runs the same
// FP32 arithmetic on the same sums, in registers: B = L L^T, A = L^-1 C L^-T,
// Householder reduction of A to tridiagonal form (Golub & Van Loan, Sec. 8.3),
// and a multisection of the Gershgorin interval with Sturm counts (Sec. 8.4):
// 32 lanes bracket the smallest eigenvalue and 32 the largest, each round
// narrowing both brackets 33-fold.  A pencil whose B is not positive definite
// leaves the node span [min u_x, max u_x] as the speeds (every eigenvalue lies
// there).
constexpr int SP_NS = 90;
constexpr int SP_ROW = SP_NS + 1;  // odd row stride
constexpr int SP_ROUNDS = 6;       // 33^6 > 1e9: the brackets end at FP32 resolution

// Number of eigenvalues below sig of the symmetric tridiagonal (d, e) (Sturm
// count by the LDL^T pivots; a zero pivot is replaced by a tiny negative one).
__device__ __forceinline__ int sturm9(const float (&d)[9], const float (&e2)[8], float sig) {
  int cnt = 0;
  float q = d[0] - sig;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (i > 0) q = d[i] - sig - e2[i - 1] / q;
    if (fabsf(q) < 1e-30f) q = -1e-30f;
    cnt += q < 0.f ? 1 : 0;
  }
  return cnt;
}

__global__ __launch_bounds__(64) void k_axi_speeds(int64_t n, int P, const float4* __restrict__ tab,
                                                   const float* __restrict__ beta,
                                                   const float* __restrict__ gin, float ux_min,
                                                   float ux_max, float* __restrict__ lam) {
  __shared__ __align__(16) float red[65 * SP_ROW];
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  float b[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) b[k] = beta[c * 9 + k];
  const AxGauge g = ax_gauge(gin, c);
  const float lz = lse9(tab, P, g, b, lane);
  float acc[SP_NS];
#pragma unroll
  for (int k = 0; k < SP_NS; ++k) acc[k] = 0.f;
  for (int q = lane; q < P; q += 64) {
    const float4 nd = tab[q];
    float f[9];
    const float sg = __expf(expo9(nd, g, b, f) - lz);
    const float x = f[1];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float t = sg * f[i];
      const float tx = t * x;
#pragma unroll
      for (int j = i; j < 9; ++j) {
        acc[k] = fmaf(t, f[j], acc[k]);
        acc[45 + k] = fmaf(tx, f[j], acc[45 + k]);
        ++k;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < SP_NS; ++k) red[lane * SP_ROW + k] = acc[k];
  __syncthreads();
  for (int k = lane; k < SP_NS; k += 64) {
    float t = 0.f;
    for (int l = 0; l < 64; ++l) t += red[l * SP_ROW + k];
    red[64 * SP_ROW + k] = t;
  }
  __syncthreads();
  const float* S = red + 64 * SP_ROW;
  float Lb[9][9], Y[9][9];
  {
    int k = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
      for (int j = i; j < 9; ++j) {
        Lb[i][j] = Lb[j][i] = S[k];
        Y[i][j] = Y[j][i] = S[45 + k];
        ++k;
      }
  }
  // B = L L^T (L in the lower triangle of Lb)
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    float d = Lb[k][k];
#pragma unroll
    for (int j = 0; j < k; ++j) d = fmaf(-Lb[k][j], Lb[k][j], d);
    ok = ok && d > 0.f && isfinite(d);
    const float l = sqrtf(fmaxf(d, FLT_MIN));
    const float il = 1.f / l;
    Lb[k][k] = l;
#pragma unroll
    for (int i = k + 1; i < 9; ++i) {
      float t = Lb[i][k];
#pragma unroll
      for (int j = 0; j < k; ++j) t = fmaf(-Lb[i][j], Lb[k][j], t);
      Lb[i][k] = t * il;
    }
  }
  // Y = L^-1 C (column by column, in place), then A = L^-1 Y^T: column j of A
  // solves against row j of Y; A is symmetric, its lower triangle is kept
  float A[9][9];
#pragma unroll
  for (int j = 0; j < 9; ++j)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float t = Y[i][j];
#pragma unroll
      for (int m = 0; m < i; ++m) t = fmaf(-Lb[i][m], Y[m][j], t);
      Y[i][j] = t / Lb[i][i];
    }
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    float z[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float t = Y[j][i];
#pragma unroll
      for (int m = 0; m < i; ++m) t = fmaf(-Lb[i][m], z[m], t);
      z[i] = t / Lb[i][i];
    }
#pragma unroll
    for (int i = j; i < 9; ++i) A[i][j] = A[j][i] = z[i];
  }
  // Householder tridiagonalisation: H = I - beta v v^T on rows/columns k+1..8,
  // A <- H A H = A - v q^T - q v^T with p = beta A v, q = p - (beta/2)(v.p) v
  float dg[9], e2[8], ea[8];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    float s2 = 0.f;
#pragma unroll
    for (int i = k + 1; i < 9; ++i) s2 = fmaf(A[i][k], A[i][k], s2);
    const float x0 = A[k + 1][k];
    const float xn = sqrtf(s2);
    const float alpha = x0 >= 0.f ? -xn : xn;
    const float vtv = 2.f * (s2 - alpha * x0);
    dg[k] = A[k][k];
    if (vtv > 1e-30f) {
      float v[9];
#pragma unroll
      for (int i = k + 1; i < 9; ++i) v[i] = A[i][k];
      v[k + 1] = x0 - alpha;
      const float beta = 2.f / vtv;
      float pv[9], vp = 0.f;
#pragma unroll
      for (int i = k + 1; i < 9; ++i) {
        float t = 0.f;
#pragma unroll
        for (int j = k + 1; j < 9; ++j) t = fmaf(A[i][j], v[j], t);
        pv[i] = beta * t;
        vp = fmaf(v[i], pv[i], vp);
      }
      const float kk = 0.5f * beta * vp;
#pragma unroll
      for (int i = k + 1; i < 9; ++i) pv[i] = fmaf(-kk, v[i], pv[i]);
#pragma unroll
      for (int i = k + 1; i < 9; ++i)
#pragma unroll
        for (int j = k + 1; j <= i; ++j)
          A[i][j] = A[j][i] = A[i][j] - v[i] * pv[j] - pv[i] * v[j];
      ea[k] = alpha;
    } else {
      ea[k] = x0;
    }
  }
  dg[7] = A[7][7];
  dg[8] = A[8][8];
  ea[7] = A[8][7];
  float glo = FLT_MAX, ghi = -FLT_MAX;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float r = (i > 0 ? fabsf(ea[i - 1]) : 0.f) + (i < 8 ? fabsf(ea[i]) : 0.f);
    glo = fminf(glo, dg[i] - r);
    ghi = fmaxf(ghi, dg[i] + r);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) e2[i] = ea[i] * ea[i];
  ok = ok && isfinite(glo) && isfinite(ghi);
  float lo = ux_min, hi = ux_max;
  if (ok) {
    // multisection: lanes 0-31 bracket the smallest eigenvalue, lanes 32-63
    // the largest (count(sig) = number of eigenvalues below sig)
    const float pad = 1e-6f * fmaxf(fabsf(glo), fabsf(ghi)) + 1e-30f;
    float a0 = glo - pad, a1 = ghi + pad, c0 = a0, c1 = a1;
    const int j = lane & 31;
    const bool upper = lane >= 32;
    for (int round = 0; round < SP_ROUNDS; ++round) {
      const float l0 = upper ? c0 : a0, l1 = upper ? c1 : a1;
      const float sig = l0 + (l1 - l0) * ((float)(j + 1) / 33.f);
      const int cnt = sturm9(dg, e2, sig);
      const uint64_t bm = __ballot(!upper && cnt >= 1);
      const uint64_t bx = __ballot(upper && cnt <= 8) >> 32;
      const float wa = a1 - a0, wc = c1 - c0;
      if (bm != 0ull) {
        const int jm = __builtin_ctzll(bm);  // smallest sig above the eigenvalue
        a1 = a0 + wa * ((float)(jm + 1) / 33.f);
        a0 = a0 + wa * ((float)jm / 33.f);
      } else {
        a0 = a0 + wa * (32.f / 33.f);
      }
      if (bx != 0ull) {
        const int jx = 63 - __builtin_clzll(bx);  // largest sig at or below it
        c0 = c0 + wc * ((float)(jx + 1) / 33.f);
        c1 = jx == 31 ? c1 : c0 + wc * (1.f / 33.f);
      } else {
        c1 = c0 + wc * (1.f / 33.f);
      }
    }
    const float emin = 0.5f * (a0 + a1), emax = 0.5f * (c0 + c1);
    const float gw = gin[c * 3], gsx = gin[c * 3 + 1];
    if (isfinite(emin) && isfinite(emax)) {
      lo = fmaxf(fmaf(gsx, emin, gw), ux_min);
      hi = fminf(fmaf(gsx, emax, gw), ux_max);
    }
  }
  if (lane == 0) {
    lam[c * 2] = lo;
    lam[c * 2 + 1] = hi;
  }
}

// Moments of the non-canonical form f = exp(alpha_0 + alpha_i phi_i), the
// comparison of Sec. 4.1: M_j = sum_p w_p exp(alpha_0 + alpha_i phi_i(u_bar_p))
// phi_j(u_bar_p) summed in plain FP32 with no shift of the exponent, so that
// exp overflows wherever the exponent exceeds log(FLT_MAX) -- the failure the
// canonical form's log-sum-exp removes.  One wave per parameter row.
__global__ __launch_bounds__(64) void k_axi_moments_nc(int64_t n, int P,
                                                       const float4* __restrict__ tab,
                                                       const float* __restrict__ alpha,
                                                       const float* __restrict__ gin,
                                                       float* __restrict__ M) {
  __shared__ float red[65 * 9];
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  if (c >= n) return;
  float a[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) a[k] = alpha[c * 9 + k];
  const AxGauge g = ax_gauge(gin, c);
  float acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.f;
  for (int q = lane; q < P; q += 64) {
    const float4 nd = tab[q];
    float f[9];
    (void)expo9(nd, g, a, f);
    float e = a[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) e = fmaf(a[i], f[i], e);
    const float v = expf(e) * expf(nd.z);
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = fmaf(v, f[k], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) red[lane * 9 + k] = acc[k];
  __syncthreads();
  if (lane < 9) {
    float t = 0.f;
    for (int l = 0; l < 64; ++l) t += red[l * 9 + lane];
    M[c * 9 + lane] = t;
  }
}

hipError_t launch_axi_moments_nc(int64_t n, int P, const float4* tab, const float* alpha,
                                 const float* g, float* M, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axi_moments_nc<<<(unsigned)n, 64, 0, s>>>(n, P, tab, alpha, g, M);
  return hipGetLastError();
}

// ---- batches of shock problems -------------------------------------------------
// Problem p owns cells [off[p], off[p+1]) and interface rows
// [off[p] + p, off[p+1] + p] (one more than its cells); its ghosts are rows 2p
// (left) and 2p + 1 (right) of the ghost arrays, and scal[2p], scal[2p + 1]
// hold its dt used and next dt.  Every index below is clamped into its array,
// so offsets that break the layout give wrong numbers, never a stray access.

// Cell range of problem p, clamped to [0, n) and non-empty.
__device__ __forceinline__ void ax_range(const AxBatch& b, int p, int64_t& lo, int64_t& hi) {
  lo = b.off[p];
  hi = b.off[p + 1];
  lo = lo < 0 ? 0 : (lo > b.n - 1 ? b.n - 1 : lo);
  hi = hi < lo + 1 ? lo + 1 : (hi > b.n ? b.n : hi);
}

// The problem of each cell (the last p with off[p] <= c) and of each
// interface row (the last p with off[p] + p <= i), by bisection.
__global__ void k_axi_maps(AxBatch b, int32_t* __restrict__ pid, int32_t* __restrict__ pidI) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b.n + b.P) return;
  auto last_le = [&](int64_t x, bool iface) {
    int lo = 0, hi = b.P - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (b.off[mid] + (iface ? mid : 0) <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  if (t < b.n) pid[t] = last_le(t, false);
  pidI[t] = last_le(t, true);
}

// One problem's descriptors from scalars: off = {0, n}, dx, ghost states.
__global__ void k_axi_single(int64_t n, float dx, float nl, float vl, float Tl, float nr, float vr,
                             float Tr, int64_t* __restrict__ off, float* __restrict__ dxo,
                             float* __restrict__ gs) {
  if (threadIdx.x == 0) {
    off[0] = 0;
    off[1] = n;
    dxo[0] = dx;
    gs[0] = nl; gs[1] = vl; gs[2] = Tl;
    gs[3] = nr; gs[4] = vr; gs[5] = Tr;
  }
}

// The two ghost Maxwellians of every problem in their own Hermite gauges:
// beta = (n, 0, -1/sqrt2, -1, 0, ...), g = (v, sqrt T, sqrt T); ghost row r is
// side r % 2 of problem r / 2, from gs[p][6] = left (n, v, T), right (n, v, T).
__global__ void k_axi_ghosts(int P, const float* __restrict__ gs, float* __restrict__ gB,
                             float* __restrict__ gG) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * P) return;
  const float* st = gs + (r / 2) * 6 + (r % 2) * 3;
  const float mb[9] = {st[0], 0.f, -0.70710678118654752f, -1.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 9; ++k) gB[r * 9 + k] = mb[k];
  gG[r * 3] = st[1];
  gG[r * 3 + 1] = sqrtf(st[2]);
  gG[r * 3 + 2] = sqrtf(st[2]);
}

hipError_t launch_axi_prologue(const AxBatch& b, const float* gs, int32_t* pid, int32_t* pidI,
                               float* gB, float* gG, hipStream_t s) {
  const int64_t rows = b.n + b.P;
  k_axi_maps<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(b, pid, pidI);
  k_axi_ghosts<<<(unsigned)((2 * b.P + 63) / 64), 64, 0, s>>>(b.P, gs, gB, gG);
  return hipGetLastError();
}

hipError_t launch_axi_single(int64_t n, float dx, const float* left, const float* right,
                             int64_t* off, float* dxo, float* gs, hipStream_t s) {
  k_axi_single<<<1, 64, 0, s>>>(n, dx, left[0], left[1], left[2], right[0], right[1], right[2],
                                off, dxo, gs);
  return hipGetLastError();
}

hipError_t launch_axi_speeds(int64_t n, int P, const float4* tab, const float* beta, const float* g,
                             float ux_min, float ux_max, float* lam, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axi_speeds<<<(unsigned)n, 64, 0, s>>>(n, P, tab, beta, g, ux_min, ux_max, lam);
  return hipGetLastError();
}

// ---- the time step of Alg. 2 (Sec. 3.4; ES-BGK source of the appendix) -------
// ES-BGK relaxation over f * dt of the cell's problem (dtp[pid * stride]):
// M <- (1 - r) M + r M~, r = h/tau,
// tau = mu_ref/(Pr n); M~ the Gaussian n N((v,0,0), diag(Sxx, Srr, Srr)),
// Sigma = T/Pr + (1 - 1/Pr) P/n, in the cell's gauge: x ~ N(mu, var) gives
// E[He_k(x)] = h_k(mu; var - 1), y ~ Exp(theta) gives E[l_1] = theta - 1 and
// E[l_2] = (theta - 1)^2.  One thread per cell.
__global__ void k_axi_collide(AxBatch b, float* __restrict__ M, const float* __restrict__ g,
                              const float* __restrict__ dtp, int stride, float f, float prandtl,
                              float mu_ref) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.n) return;
  float m[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = M[c * 9 + k];
  const float w = g[c * 3], sx = g[c * 3 + 1], sr = g[c * 3 + 2];
  const float nn = m[0];
  if (!(nn > 0.0f) || !isfinite(nn)) return;
  const float ex = m[1] / nn;
  const float exx = 1.41421356237309505f * m[2] / nn + 1.0f;
  const float err = 2.0f * (m[3] / nn + 1.0f);
  const float pxx = sx * sx * (exx - ex * ex), prr = 0.5f * sr * sr * err;
  const float T = (pxx + 2.0f * prr) / 3.0f;
  const float Pr = prandtl;
  const float sxx = T / Pr + (1.0f - 1.0f / Pr) * pxx, srr = T / Pr + (1.0f - 1.0f / Pr) * prr;
  const float mu = ex;  // (v - w)/s_x with v = w + s_x E[x]
  const float cv = sxx / (sx * sx) - 1.0f;
  const float hx[5] = {1.0f, mu, mu * mu + cv, mu * mu * mu + 3.0f * mu * cv,
                        mu * mu * mu * mu + 6.0f * mu * mu * cv + 3.0f * cv * cv};
  const float px[5] = {hx[0], hx[1], hx[2] * 0.70710678118654752f, hx[3] * 0.40824829046386302f,
                        hx[4] * 0.20412414523193151f};
  const float th = srr / (sr * sr);
  const float ly[3] = {1.0f, th - 1.0f, (th - 1.0f) * (th - 1.0f)};
  const float r = f * dtp[b.pid[c] * stride] * Pr * nn / mu_ref;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float mt = nn * px[AX_A[i]] * ly[AX_K[i]];
    M[c * 9 + i] = (1.0f - r) * m[i] + r * mt;
  }
}

// Cells the box cannot represent (the solve ended NONREALIZABLE or NONFINITE on
// finite targets) take the Maxwellian of their gauge, so that fluxes and speeds
// stay defined.
__global__ void k_axi_fix(int64_t n, const float* __restrict__ M, float* __restrict__ beta,
                          const uint32_t* __restrict__ st) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  if (!(st[c] & (MEM_ST_NONREALIZABLE | MEM_ST_NONFINITE))) return;
  const float nn = M[c * 9];
  if (!(nn > 0.f) || !isfinite(nn)) return;
  const float mb[9] = {nn, 0.f, -0.70710678118654752f, -1.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 9; ++k) beta[c * 9 + k] = mb[k];
}

// dt of this step, per problem (one workgroup each): min(previous dt,
// cfl dx / max speed) over its cells and ghosts; scal[2p] = dt used,
// scal[2p + 1] = cfl dx / max speed (the next step's dt).  With init,
// dt[p] <- cfl dx / max speed and nothing else.
__global__ __launch_bounds__(256) void k_axi_dt(AxBatch b, const float* __restrict__ lam,
                                                const float* __restrict__ glam, float cfl,
                                                float* __restrict__ dt, float* __restrict__ scal,
                                                int init) {
  __shared__ float sm[256];
  const int p = blockIdx.x;
  int64_t lo, hi;
  ax_range(b, p, lo, hi);
  float r = 0.f;
  for (int64_t c = lo + threadIdx.x; c < hi; c += 256)
    r = fmaxf(r, fmaxf(fabsf(lam[c * 2]), fabsf(lam[c * 2 + 1])));
  if (threadIdx.x < 2) {
    const float* gl = glam + (2 * p + threadIdx.x) * 2;
    r = fmaxf(r, fmaxf(fabsf(gl[0]), fabsf(gl[1])));
  }
  sm[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float dn = cfl * b.dx[p] / sm[0];
    if (init) {
      dt[p] = dn;
    } else {
      scal[2 * p] = fminf(dt[p], dn);
      scal[2 * p + 1] = dn;
    }
  }
}

__device__ __forceinline__ void axi_T(const float* gto, const float* gfrom, float (&t)[5][5],
                                      float (&r)[3][3]) {
  const float sxt = gto[1], sx = gfrom[1], srt = gto[2], sr = gfrom[2];
  conn_x(sx / sxt, (gfrom[0] - gto[0]) / sxt, t);
  conn_y((sr / srt) * (sr / srt), r);
}

// LLF in local gauges: neighbour moments and fluxes moved into the cell's gauge
// by T(g_i, g_j); both cells of a face use max(rho_i, rho_j), rho = max |lam|.
// The first and last cell of a problem face its ghosts (ghost rows 2p, 2p + 1).
__global__ void k_axi_fv(AxBatch b, const float* __restrict__ M, const float* __restrict__ F,
                         const float* __restrict__ lam, const float* __restrict__ g,
                         const float* __restrict__ gM, const float* __restrict__ gF,
                         const float* __restrict__ glam, const float* __restrict__ gG,
                         const float* __restrict__ scal, float* __restrict__ Mout) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.n) return;
  const int p = b.pid[c];
  int64_t lo, hi;
  ax_range(b, p, lo, hi);
  const float dt = scal[2 * p];
  const float dx = b.dx[p];
  auto rho_of = [](const float* l) { return fmaxf(fabsf(l[0]), fabsf(l[1])); };
  const float ri = rho_of(lam + c * 2);
  float acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = M[c * 9 + k];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const bool ghost = side == 0 ? (c <= lo) : (c >= hi - 1);
    const int64_t j = side == 0 ? c - 1 : c + 1;
    const int gr = 2 * p + side;
    const float* Mj = ghost ? gM + gr * 9 : M + j * 9;
    const float* Fj = ghost ? gF + gr * 9 : F + j * 9;
    const float* gj = ghost ? gG + gr * 3 : g + j * 3;
    const float rj = rho_of(ghost ? glam + gr * 2 : lam + j * 2);
    const float a = fmaxf(ri, rj);
    float t[5][5], r[3][3];
    axi_T(g + c * 3, gj, t, r);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float mj = 0.0f, fj = 0.0f;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float tk = tij(t, r, i, k);
        mj += tk * Mj[k];
        fj += tk * Fj[k];
      }
      const float mi = M[c * 9 + i], fi = F[c * 9 + i];
      // left face: + dt/dx (1/2 (F_l + F_i) + 1/2 a (M_l - M_i));
      // right face: - dt/dx (1/2 (F_i + F_r) + 1/2 a (M_i - M_r))
      const float face = side == 0 ? 0.5f * (fj + fi) + 0.5f * a * (mj - mi)
                                    : -(0.5f * (fi + fj) + 0.5f * a * (mi - mj));
      acc[i] += dt / dx * face;
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Mout[c * 9 + k] = (float)acc[k];
}

// ---- second-order fluxes (Sec. 3.4: two-step LW, FLIC) ------------------------
// Elements e = 0..n+1 of a problem of n cells are [left ghost, cells, right
// ghost]; its interface j lies between elements j and j + 1 and works in the
// gauge of element j + 1.
struct AxElem { const float *M, *F, *g, *b, *lam; };
__device__ __forceinline__ AxElem axi_elem(int64_t e, int64_t n, const float* M, const float* F,
                                           const float* g, const float* beta, const float* lam,
                                           const float* gM, const float* gF, const float* gG,
                                           const float* gB, const float* glam) {
  if (e == 0) return {gM, gF, gG, gB, glam};
  if (e == n + 1) return {gM + 9, gF + 9, gG + 3, gB + 9, glam + 2};
  const int64_t c = e - 1;
  return {M + c * 9, F + c * 9, g + c * 3, beta + c * 9, lam + c * 2};
}

// One thread per interface: F_LF and the half-step state
// Mh = (M_L + M_R)/2 + dt/(2 dx) (F_L - F_R) in the right element's gauge, the
// per-moment van Leer limiter of FLIC (1 for LW), and the right element's
// gauge and multipliers as the interface solve's gauge and start.
__global__ void k_axi_iface(AxBatch b, const float* __restrict__ M0, const float* __restrict__ F0,
                            const float* __restrict__ lam0, const float* __restrict__ g0,
                            const float* __restrict__ beta0, const float* __restrict__ gM0,
                            const float* __restrict__ gF0, const float* __restrict__ glam0,
                            const float* __restrict__ gG0, const float* __restrict__ gB0,
                            const float* __restrict__ scal, int flic,
                            float* __restrict__ fLF, float* __restrict__ Mh,
                            float* __restrict__ gI, float* __restrict__ bI,
                            float* __restrict__ phi) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= b.n + b.P) return;
  const int p = b.pidI[row];
  int64_t lo, hi;
  ax_range(b, p, lo, hi);
  const int64_t n = hi - lo;  // the problem's cells
  int64_t j = row - lo - p;   // its interface
  j = j < 0 ? 0 : (j > n ? n : j);
  const float dt = scal[2 * p];
  const float dx = b.dx[p];
  // the problem's cells and ghost rows
  const float *M = M0 + lo * 9, *F = F0 + lo * 9, *g = g0 + lo * 3, *beta = beta0 + lo * 9,
              *lam = lam0 + lo * 2;
  const float *gM = gM0 + 2 * p * 9, *gF = gF0 + 2 * p * 9, *gG = gG0 + 2 * p * 3,
              *gB = gB0 + 2 * p * 9, *glam = glam0 + 2 * p * 2;
  const AxElem L = axi_elem(j, n, M, F, g, beta, lam, gM, gF, gG, gB, glam);
  const AxElem R = axi_elem(j + 1, n, M, F, g, beta, lam, gM, gF, gG, gB, glam);
  const AxElem LL = axi_elem(j > 0 ? j - 1 : 0, n, M, F, g, beta, lam, gM, gF, gG, gB, glam);
  // the ghosts repeat beyond both ends
  const bool rr_is_r = j + 1 > n;
  const AxElem RR = axi_elem(rr_is_r ? j + 1 : j + 2, n, M, F, g, beta, lam, gM, gF, gG, gB, glam);
  auto rho_of = [](const float* l) { return fmaxf(fabsf(l[0]), fabsf(l[1])); };
  const float a = fmaxf(rho_of(L.lam), rho_of(R.lam));
  float t[5][5], r[3][3], t2[5][5], r2[3][3], t3[5][5], r3[3][3];
  axi_T(R.g, L.g, t, r);
  axi_T(R.g, LL.g, t2, r2);
  axi_T(R.g, RR.g, t3, r3);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    float ml = 0.0f, fl = 0.0f, mll = 0.0f, mrr = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float tk = tij(t, r, i, k);
      ml += tk * L.M[k];
      fl += tk * L.F[k];
      mll += tij(t2, r2, i, k) * LL.M[k];
      mrr += tij(t3, r3, i, k) * RR.M[k];
    }
    const float mr = R.M[i], fr = R.F[i];
    if (rr_is_r) mrr = mr;
    fLF[row * 9 + i] = 0.5f * (fl + fr) + 0.5f * a * (ml - mr);
    Mh[row * 9 + i] = 0.5f * (ml + mr) + 0.5f * (dt / dx) * (fl - fr);
    float ph = 1.0f;
    if (flic) {  // van Leer on both sides: 2 a / (a + b) for a b > 0, else 0; the smaller
      const float da = ml - mll, db = mr - ml, dc = mrr - mr;
      const float pl = da * db > 0.0f ? 2.0f * da / (da + db) : 0.0f;
      const float pr = dc * db > 0.0f ? 2.0f * dc / (dc + db) : 0.0f;
      ph = fminf(pl, pr);
    }
    phi[row * 9 + i] = (float)ph;
    bI[row * 9 + i] = R.b[i];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) gI[row * 3 + k] = R.g[k];
}

// Blend F = F_LF + phi (F_LW - F_LF) (F_LF where the interface solve failed)
// and apply: cell c takes its left face (interface row c + p) as given and its
// right face (row c + p + 1) moved into its gauge by T(g_c, g_{c+1}).
__global__ void k_axi_fv2(AxBatch b, const float* __restrict__ M, const float* __restrict__ g,
                          const float* __restrict__ gG, const float* __restrict__ fLF,
                          const float* __restrict__ fLW, const float* __restrict__ phi,
                          const uint32_t* __restrict__ stI, const float* __restrict__ scal,
                          float* __restrict__ Mout) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.n) return;
  const int p = b.pid[c];
  int64_t lo, hi;
  ax_range(b, p, lo, hi);
  const float dt = scal[2 * p];
  const float dx = b.dx[p];
  auto face = [&](int64_t j, int i) {
    const bool bad = (stI[j] & (MEM_ST_NONREALIZABLE | MEM_ST_NONFINITE)) != 0;
    const float lf = fLF[j * 9 + i];
    return bad ? lf : lf + phi[j * 9 + i] * (fLW[j * 9 + i] - lf);
  };
  const float* gn = c + 1 < hi ? g + (c + 1) * 3 : gG + (2 * p + 1) * 3;
  float t[5][5], r[3][3];
  axi_T(g + c * 3, gn, t, r);
  const int64_t fl = c + p;  // the left face's interface row
  float fr[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) fr[k] = face(fl + 1, k);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) acc += tij(t, r, i, k) * fr[k];
    Mout[c * 9 + i] = M[c * 9 + i] + dt / dx * (face(fl, i) - acc);
  }
}

hipError_t launch_axi_iface(const AxBatch& b, const float* M, const float* F, const float* lam,
                            const float* g, const float* beta, const float* gM, const float* gF,
                            const float* glam, const float* gG, const float* gB,
                            const float* scal, int flic, float* fLF, float* Mh, float* gI,
                            float* bI, float* phi, hipStream_t s) {
  k_axi_iface<<<(unsigned)((b.n + b.P + 127) / 128), 128, 0, s>>>(
      b, M, F, lam, g, beta, gM, gF, glam, gG, gB, scal, flic, fLF, Mh, gI, bI, phi);
  return hipGetLastError();
}

hipError_t launch_axi_fv2(const AxBatch& b, const float* M, const float* g, const float* gG,
                          const float* fLF, const float* fLW, const float* phi,
                          const uint32_t* stI, const float* scal, float* Mout, hipStream_t s) {
  if (b.n <= 0) return hipSuccess;
  k_axi_fv2<<<(unsigned)((b.n + 127) / 128), 128, 0, s>>>(b, M, g, gG, fLF, fLW, phi, stI, scal,
                                                         Mout);
  return hipGetLastError();
}

__global__ void k_axi_finish(int P, float* __restrict__ t, float* __restrict__ dt,
                             const float* __restrict__ scal) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) {
    t[p] += scal[2 * p];
    dt[p] = scal[2 * p + 1];
  }
}

hipError_t launch_axi_collide(const AxBatch& b, float* M, const float* g, const float* dtp,
                              int stride, float f, float prandtl, float mu_ref, hipStream_t s) {
  if (b.n <= 0) return hipSuccess;
  k_axi_collide<<<(unsigned)((b.n + 255) / 256), 256, 0, s>>>(b, M, g, dtp, stride, f, prandtl,
                                                             mu_ref);
  return hipGetLastError();
}

hipError_t launch_axi_fix(int64_t n, const float* M, float* beta, const uint32_t* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axi_fix<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, M, beta, st);
  return hipGetLastError();
}

hipError_t launch_axi_dt(const AxBatch& b, const float* lam, const float* glam, float cfl,
                         float* dt, float* scal, int init, hipStream_t s) {
  k_axi_dt<<<(unsigned)b.P, 256, 0, s>>>(b, lam, glam, cfl, dt, scal, init);
  return hipGetLastError();
}

hipError_t launch_axi_fv(const AxBatch& b, const float* M, const float* F, const float* lam,
                         const float* g, const float* gM, const float* gF, const float* glam,
                         const float* gG, const float* scal, float* Mout, hipStream_t s) {
  if (b.n <= 0) return hipSuccess;
  k_axi_fv<<<(unsigned)((b.n + 127) / 128), 128, 0, s>>>(b, M, F, lam, g, gM, gF, glam, gG, scal,
                                                        Mout);
  return hipGetLastError();
}

hipError_t launch_axi_finish(int P, float* t, float* dt, const float* scal, hipStream_t s) {
  k_axi_finish<<<(unsigned)((P + 63) / 64), 64, 0, s>>>(P, t, dt, scal);
  return hipGetLastError();
}

hipError_t launch_axi_gauge(int64_t n, float* M, float* beta, float* g, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axi_gauge<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, M, beta, g);
  return hipGetLastError();
}

hipError_t launch_axi_solve(int64_t n, int P, const float4* tab, const float* M, const float* g,
                            float* beta, const SolveParams& p, int32_t* iters, float* resid,
                            uint32_t* status, hipStream_t s, float* cond) {
  if (n <= 0) return hipSuccess;
  k_axi_solve<<<(unsigned)((n + AXW - 1) / AXW), 64 * AXW, 0, s>>>(n, P, tab, M, g, beta, p, iters,
                                                                 resid, status, cond);
  return hipGetLastError();
}

// cond_max[p] = max(cond_max[p], max over the problem's cells of cond[c]), as
// an unsigned max of the float bits (all values >= 0); a wave whose cells all
// belong to one problem makes one atomic.
__global__ void k_axi_cond_max(AxBatch b, const float* __restrict__ cond, uint32_t* out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = c < b.n;
  const float r = in ? cond[c] : 0.f;
  const uint32_t v = (in && r >= 0.f) ? __float_as_uint(r) : 0u;
  const int p = in ? b.pid[c] : -1;
  const int p0 = __shfl(p, 0);
  if (__all(!in || p == p0)) {
    uint32_t m = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0 && p0 >= 0 && m > 0u) atomicMax(&out[p0], m);
  } else if (in && v > 0u) {
    atomicMax(&out[p], v);
  }
}

hipError_t launch_axi_cond_max(const AxBatch& b, const float* cond, float* cond_max,
                               hipStream_t s) {
  if (b.n <= 0) return hipSuccess;
  k_axi_cond_max<<<(unsigned)((b.n + 255) / 256), 256, 0, s>>>(
      b, cond, reinterpret_cast<uint32_t*>(cond_max));
  return hipGetLastError();
}

hipError_t launch_axi_moments(int64_t n, int P, const float4* tab, const float* beta,
                              const float* g, float* M, float* F, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_axi_moments<<<(unsigned)((n + AXW - 1) / AXW), 64 * AXW, 0, s>>>(n, P, tab, beta, g, M, F);
  return hipGetLastError();
}

}  // namespace memk
