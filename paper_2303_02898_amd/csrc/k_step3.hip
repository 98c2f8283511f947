// Gauge, flux, characteristic speeds, collision and finite-volume kernels for
// the 3D 35-moment system with transport along x (Sec. 3.3-3.4, App. A, Alg. 2).
//
// Change of gauge (eq. "Change gauge M F"): per axis u_bar' = a u_bar + b with
// a = s/s', b = (w - w')/s' (b = 0 on the transverse axes).  For the
// orthonormal Hermite basis the 1D connection is
//   phi_n(a x + b) = sum_{k<=n} C(n,k) a^k h_{n-k}(b; a^2-1) sqrt(k!/n!) phi_k(x),
// with h_m(b; c) = E[He_m(X)], X ~ N(b, 1 + c); the 3D matrix is the
// Kronecker product of the three axis matrices, applied axis by axis on the
// total-degree-<=4 index set (which the lower-triangular factors preserve).
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "mem_internal.h"

namespace memk {

// basis index of (a, b, c): degree offset + position within the degree
__host__ __device__ constexpr int bidx(int a, int b, int c) {
  return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 +
         (b + c) * (b + c + 1) / 2 + c;
}

__device__ __forceinline__ void hpoly3(float b, float c, float (&h)[5]) {
  h[0] = 1.f;
  h[1] = b;
  h[2] = b * b + c;
  h[3] = b * b * b + 3.f * b * c;
  h[4] = b * b * b * b + 6.f * b * b * c + 3.f * c * c;
}

__device__ __forceinline__ void conn(float a, float b, float (&t)[5][5]) {
  const float binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                             {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
  const float sfact[5] = {1.f, 1.f, 1.41421356237f, 2.44948974278f, 4.89897948557f};
  float h[5];
  hpoly3(b, a * a - 1.f, h);
  const float ak[5] = {1.f, a, a * a, a * a * a, a * a * a * a};
#pragma unroll
  for (int n = 0; n < 5; ++n)
#pragma unroll
    for (int k = 0; k < 5; ++k)
      t[n][k] = k <= n ? binom[n][k] * ak[k] * h[n - k] * sfact[k] / sfact[n] : 0.f;
}

// v <- (t along axis AX) v, or its transpose
template <int AX, bool TR>
__device__ __forceinline__ void axis_apply(const float (&t)[5][5], float (&v)[K3]) {
  float o[K3];
#pragma unroll
  for (int a = 0; a <= 4; ++a)
#pragma unroll
    for (int b = 0; b <= 4 - a; ++b)
#pragma unroll
      for (int c = 0; c <= 4 - a - b; ++c) {
        const int x = AX == 0 ? a : (AX == 1 ? b : c);
        const int rest = a + b + c - x;
        float acc = 0.f;
        if (!TR) {
#pragma unroll
          for (int x2 = 0; x2 <= x; ++x2) {
            const int i = AX == 0 ? bidx(x2, b, c) : (AX == 1 ? bidx(a, x2, c) : bidx(a, b, x2));
            acc += t[x][x2] * v[i];
          }
        } else {
#pragma unroll
          for (int x2 = x; x2 <= 4 - rest; ++x2) {
            const int i = AX == 0 ? bidx(x2, b, c) : (AX == 1 ? bidx(a, x2, c) : bidx(a, b, x2));
            acc += t[x2][x] * v[i];
          }
        }
        o[bidx(a, b, c)] = acc;
      }
#pragma unroll
  for (int i = 0; i < K3; ++i) v[i] = o[i];
}

// v <- T(g_to, g_from) v
__device__ __forceinline__ void change_gauge(float (&v)[K3], const float* gto, const float* gfrom) {
  float tx[5][5], tr[5][5];
  conn(gfrom[1] / gto[1], (gfrom[0] - gto[0]) / gto[1], tx);
  conn(gfrom[2] / gto[2], 0.f, tr);
  axis_apply<0, false>(tx, v);
  axis_apply<1, false>(tr, v);
  axis_apply<2, false>(tr, v);
}

// ---- Hermite gauge ------------------------------------------------------------
__device__ __forceinline__ bool hermite_params(const float (&m)[K3], const float* g, float* gH) {
  const float n = m[0];
  if (!(n > 0.f)) return false;
  const float s2 = 1.41421356237f;
  const float m1 = m[bidx(1, 0, 0)] / n;
  const float exx = (s2 * m[bidx(2, 0, 0)] + n) / n;
  const float err = (s2 * (m[bidx(0, 2, 0)] + m[bidx(0, 0, 2)]) + 2.f * n) / n;
  const float vx = exx - m1 * m1;
  if (!(vx > 0.f) || !(err > 0.f) || !isfinite(vx) || !isfinite(err)) return false;
  gH[0] = g[0] + g[1] * m1;
  gH[1] = g[1] * sqrtf(vx);
  gH[2] = g[2] * sqrtf(0.5f * err);
  return true;
}

__global__ __launch_bounds__(128) void k_gauge3(int64_t n, float* __restrict__ M, float* __restrict__ beta,
                         float* __restrict__ g) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float m[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) m[k] = M[c * K3 + k];
  const float gg[3] = {g[c * 3], g[c * 3 + 1], g[c * 3 + 2]};
  if (!(gg[1] > 0.f) || !(gg[2] > 0.f)) return;
  float gH[3];
  if (!hermite_params(m, gg, gH)) return;
  change_gauge(m, gH, gg);
#pragma unroll
  for (int k = 0; k < K3; ++k) M[c * K3 + k] = m[k];
  if (beta) {
    // alpha(g_H) = T(g, g_H)^T alpha(g); beta_i = alpha_i for i >= 1
    float b[K3];
#pragma unroll
    for (int k = 0; k < K3; ++k) b[k] = k == 0 ? 0.f : beta[c * K3 + k];
    float tx[5][5], tr[5][5];
    conn(gH[1] / gg[1], (gH[0] - gg[0]) / gg[1], tx);
    conn(gH[2] / gg[2], 0.f, tr);
    axis_apply<0, true>(tx, b);
    axis_apply<1, true>(tr, b);
    axis_apply<2, true>(tr, b);
#pragma unroll
    for (int k = 1; k < K3; ++k) beta[c * K3 + k] = b[k];
  }
  g[c * 3] = gH[0];
  g[c * 3 + 1] = gH[1];
  g[c * 3 + 2] = gH[2];
}

// ---- fluxes from the assembled moments --------------------------------------------
// F_i = n (w E[phi_i] + s_x E[u_bar_x phi_i]); phi_1 = u_bar_x so E[u_bar_x phi_i]
// is the (1, i) pair column of S.
// F_i = n (w E[phi_i] + s_x E[u_x phi_i]) from rows of S (flux_rows = 0: pair
// columns (0, i) and (1, i), phi_(100) = u_x) or of the 128-column flux operand
// (flux_rows = 1: E[phi_i] in columns 0..34, E[u_x phi_i] in 35..69).
__global__ void k_flux3(int64_t n, const float* __restrict__ S, const float* __restrict__ beta,
                        const float* __restrict__ g, float* __restrict__ F, int flux_rows) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const float* Sc = S + c * (flux_rows ? NC5 : NCOL);
  const float inv0 = 1.f / Sc[0];
  const float nn = beta[c * K3];
  const float w = g[c * 3], sx = g[c * 3 + 1];
  for (int i = 0; i < K3; ++i) {
    const float e = Sc[i] * inv0;
    const int xc = flux_rows ? K3 + i : (i == 0 ? 1 : pair_col(1, i));
    F[c * K3 + i] = nn * (w * e + sx * Sc[xc] * inv0);
  }
}

// ---- characteristic speeds -------------------------------------------------------
// Eigenvalues of dF/dM solve C v = mu B v with B = E[phi phi^T], C = E[u_bar_x
// phi phi^T] (35 x 35, phi_0 included); lambda = w + s_x mu.  One wavefront per
// cell, lane j holding column j of the current matrix in registers:
//   * Cholesky B = L L^T (column k of the current matrix, pivot included,
//     shared through LDS; column k of L stored in the same row);
//   * A = L^-1 C L^-T by two lane-parallel forward substitutions (each lane
//     solves for its own column), the transposes through LDS;
//   * Householder tridiagonalisation of A (Householder vector and p - K v
//     shared through LDS, lane-parallel rank-2 updates);
//   * extreme eigenvalues of the tridiagonal matrix by multisection: every
//     lane evaluates a Sturm count at its own shift, the two halves of the
//     wave bracketing the two extremes, 32 subintervals each per round.
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int EIG_WAVES = 4;
constexpr int EST = 36;  // row stride of the per-wave LDS matrices

__device__ __forceinline__ float rlf(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ float wmin(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ float wmax(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// An empty asm that reads and writes every entry of a 35-value column, so
// that the values exist in registers at this point of the program.
__device__ __forceinline__ void eig_keep(float (&v)[K3]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
               "+v"(v[6]), "+v"(v[7]), "+v"(v[8]));
  asm volatile("" : "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
               "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]));
  asm volatile("" : "+v"(v[18]), "+v"(v[19]), "+v"(v[20]), "+v"(v[21]), "+v"(v[22]),
               "+v"(v[23]), "+v"(v[24]), "+v"(v[25]), "+v"(v[26]));
  asm volatile("" : "+v"(v[27]), "+v"(v[28]), "+v"(v[29]), "+v"(v[30]), "+v"(v[31]),
               "+v"(v[32]), "+v"(v[33]), "+v"(v[34]));
}

// Three wavefronts per SIMD (at most 168 VGPRs; one cold 16-byte spill) hide
// more of the per-step LDS and reduction latency than two.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_eig3(int64_t n, const float* __restrict__ S,
                                              const float* __restrict__ S5,
                                              const int32_t* __restrict__ ux_src,
                                              const float2* __restrict__ ux_w,
                                              const float* __restrict__ g, float umax,
                                              float* __restrict__ out, int radius_only,
                                              uint32_t* status) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * EIG_WAVES + wv;
  if (c >= n) return;  // whole wave
  __shared__ __align__(16) float sbuf[EIG_WAVES][2 * K3 * EST];  // S, C rows; then L and T
  __shared__ __align__(16) float svec[EIG_WAVES][5][EST];       // 1/L_kk, v, q, d, e
  float* W = sbuf[wv];
  float* Lm = W;              // row k = column k of L
  float* T = W + K3 * EST;    // transposes
  float* invd = svec[wv][0];
  float* vb = svec[wv][1];
  float* qb = svec[wv][2];
  float* dd = svec[wv][3];
  float* ee = svec[wv][4];
  {
    // S in the rows that become L, the S5 row behind the area that becomes T
    const f4* s4 = reinterpret_cast<const f4*>(S + c * NCOL);
    const f4* x4 = reinterpret_cast<const f4*>(S5 + c * NC5);
    f4* w4 = reinterpret_cast<f4*>(W);
    for (int i = lane; i < NCOL / 4; i += 64) w4[i] = s4[i];
    if (lane < NC5 / 4) w4[(K3 * EST + NCOL) / 4 + lane] = x4[lane];
  }
  __builtin_amdgcn_wave_barrier();
  // C = E[u_x phi phi^T] in packed pair order into the T area (read only after
  // the Cholesky, so that one 35-value column is live at a time): each entry is
  // two weighted entries of S or S5 (Hermite three-term recurrence)
  for (int q = lane; q < NPAIR; q += 64) {
    const int sr = ux_src[q];
    const float2 wq = ux_w[q];
    const int s1 = sr & 0xffff, s2 = sr >> 16;
    const float v1 = s1 < 1024 ? W[s1] : T[NCOL + s1 - 1024];
    const float v2 = s2 < 1024 ? W[s2] : T[NCOL + s2 - 1024];
    T[q] = fmaf(wq.x, v1, wq.y * v2);
  }
  __builtin_amdgcn_wave_barrier();
  const float inv0 = 1.f / W[0];
  bool ok = isfinite(inv0) && inv0 > 0.f;
  const int j = lane < K3 ? lane : 0;
  float a[K3], x[K3];
#pragma unroll
  for (int i = 0; i < K3; ++i) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    a[i] = W[pair_col(lo, hi)] * inv0;
  }
  __builtin_amdgcn_wave_barrier();  // the S rows become L

  // Cholesky of B, right-looking: step k writes column k of the current matrix
  // to LDS, reads it back with aligned broadcast reads (pivot included), updates
  // the trailing columns unpredicated (multiplier 0 on lanes <= k) and then
  // stores column k of L in the same row
  float dinv = 1.f;
#pragma unroll
  for (int k = 0; k < K3; ++k) {
    float* row = Lm + k * EST;
    if (lane < K3) row[lane] = a[k];
    __builtin_amdgcn_wave_barrier();
    float u[EST];
    const f4* r4 = reinterpret_cast<const f4*>(row);
#pragma unroll
    for (int q = k / 4; q < EST / 4; ++q) {
      const f4 v = r4[q];
      u[4 * q] = v[0]; u[4 * q + 1] = v[1]; u[4 * q + 2] = v[2]; u[4 * q + 3] = v[3];
    }
    const float d = u[k];
    ok = ok && d > 0.f && isfinite(d);
    const float inv = __builtin_amdgcn_rsqf(d);
    if (lane == k) dinv = inv;
    const float cj = lane > k ? a[k] * (inv * inv) : 0.f;
#pragma unroll
    for (int i = k + 1; i < K3; ++i) a[i] = fmaf(-u[i], cj, a[i]);
    __builtin_amdgcn_wave_barrier();
    if (lane < K3) row[lane] = lane >= k ? a[k] * inv : 0.f;  // L[lane][k]
    // materialise the updated column here: left to itself the compiler turns the
    // right-looking update into a left-looking one (each entry recomputed when
    // first needed) and keeps every earlier step's row and multiplier alive
    eig_keep(a);
    asm volatile("" : "+v"(dinv));
    __builtin_amdgcn_wave_barrier();
  }
  if (lane < K3) invd[lane] = dinv;
#pragma unroll
  for (int i = 0; i < K3; ++i) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    x[i] = T[pair_col(lo, hi)] * inv0;
  }
  __builtin_amdgcn_wave_barrier();  // the Sx staging becomes T
  // forward substitution L y = x on this lane's column (rows of L read 16 bytes
  // at a time)
  auto fsolve = [&](float (&y)[K3]) {
#pragma unroll
    for (int k = 0; k < K3; ++k) {
      const float yk = y[k] * invd[k];
      y[k] = yk;
      const f4* r4 = reinterpret_cast<const f4*>(Lm + k * EST);
#pragma unroll
      for (int q = (k + 1) / 4; q < EST / 4; ++q) {
        const f4 v = r4[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = 4 * q + t;
          if (i > k && i < K3) y[i] = fmaf(-v[t], yk, y[i]);
        }
      }
      eig_keep(y);  // keep the substitution column-oriented (see the Cholesky)
    }
  };
  // column j of the transpose: T[j][i] = y[i] written by lane j, read back as T[i][j]
  auto transpose = [&](float (&y)[K3], bool average) {
    if (lane < K3) {
#pragma unroll
      for (int i = 0; i < K3; ++i) T[lane * EST + i] = y[i];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < K3; ++i) {
      const float t = T[i * EST + j];
      y[i] = average ? 0.5f * (y[i] + t) : t;
    }
    __builtin_amdgcn_wave_barrier();
  };
  fsolve(x);              // column j of Y = L^-1 C
  transpose(x, false);    // column j of Y^T (C symmetric: Y^T = C L^-T)
  fsolve(x);              // column j of A = L^-1 C L^-T
  transpose(x, true);     // symmetrised against rounding

  // Householder tridiagonalisation: d_k = A[k][k], e_k = A[k+1][k] of the result.
  // Lane i holds column i, so its x[k] is A[i][k]: every lane contributes its own
  // entry of the reflector, the norm is a wave reduction.
  const bool in = lane < K3;
#pragma unroll
  for (int k = 0; k < K3 - 2; ++k) {
    const float xk = x[k];
    const float vl = (lane > k && in) ? xk : 0.f;
    const float sig = wsum(vl * vl);
    const float x0 = rlf(xk, k + 1);
    if (lane == 0) dd[k] = rlf(xk, k);
    const float nx = sqrtf(sig);
    const float al = x0 > 0.f ? -nx : nx;
    const float v1 = x0 - al;           // first entry of the Householder vector
    const float vn = sig - x0 * x0 + v1 * v1;
    if (lane == 0) ee[k] = al;
    if (nx > 0.f && vn > 0.f) {
      const float bet = 2.f / vn;
      const float vj = lane == k + 1 ? v1 : vl;
      if (lane < EST) vb[lane] = vj;
      __builtin_amdgcn_wave_barrier();
      float vv[EST];
      const f4* v4 = reinterpret_cast<const f4*>(vb);
#pragma unroll
      for (int q = (k + 1) / 4; q < EST / 4; ++q) {
        const f4 v = v4[q];
        vv[4 * q] = v[0]; vv[4 * q + 1] = v[1]; vv[4 * q + 2] = v[2]; vv[4 * q + 3] = v[3];
      }
      float w = 0.f;
#pragma unroll
      for (int i = k + 1; i < K3; ++i) w = fmaf(x[i], vv[i], w);
      const float pj = (lane > k && in) ? bet * w : 0.f;
      const float Kc = 0.5f * bet * wsum(vj * pj);
      const float qj = pj - Kc * vj;
      if (lane < EST) qb[lane] = qj;
      __builtin_amdgcn_wave_barrier();
      const f4* q4 = reinterpret_cast<const f4*>(qb);
#pragma unroll
      for (int q = (k + 1) / 4; q < EST / 4; ++q) {
        const f4 qv = q4[q];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = 4 * q + t;
          if (i > k && i < K3) x[i] = x[i] - (vv[i] * qj + qv[t] * vj);
        }
      }
    }
    eig_keep(x);
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == K3 - 2) { dd[K3 - 2] = x[K3 - 2]; ee[K3 - 2] = x[K3 - 1]; }
  if (lane == K3 - 1) dd[K3 - 1] = x[K3 - 1];
  __builtin_amdgcn_wave_barrier();

  // Gershgorin bracket, then multisection with Sturm counts
  float glo = FLT_MAX, ghi = -FLT_MAX;
  if (lane < K3) {
    const float r = (lane > 0 ? fabsf(ee[lane - 1]) : 0.f) + (lane < K3 - 1 ? fabsf(ee[lane]) : 0.f);
    glo = dd[lane] - r;
    ghi = dd[lane] + r;
  }
  glo = wmin(glo);
  ghi = wmax(ghi);
  // Sturm count below xs (number of negative pivots of T - xs I), with d_k and
  // e_k^2 in registers and the hardware reciprocal in place of the division
  float dk[K3], e2[K3 - 1];
#pragma unroll
  for (int i = 0; i < K3; ++i) dk[i] = dd[i];
#pragma unroll
  for (int i = 0; i < K3 - 1; ++i) e2[i] = ee[i] * ee[i];
  auto count_below = [&](float xs) {
    int cnt = 0;
    float q = dk[0] - xs;
    if (q == 0.f) q = -1e-30f;
    cnt += q < 0.f;
#pragma unroll
    for (int i = 1; i < K3; ++i) {
      q = fmaf(-e2[i - 1], __builtin_amdgcn_rcpf(q), dk[i] - xs);
      if (q == 0.f) q = -1e-30f;
      cnt += q < 0.f;
    }
    return cnt;
  };
  // Both extremes at once: lanes 0..31 bracket the smallest eigenvalue (first x
  // with count >= 1), lanes 32..63 the largest (first x with count >= K); each
  // half samples 32 shifts per round, its last lane the bracket's upper end,
  // where count >= need always holds.
  float lo2[2] = {glo, glo}, hi2[2] = {ghi, ghi};
  const int half = lane >> 5, sub = lane & 31;
  const int need = half ? K3 : 1;
  for (int round = 0; round < 5; ++round) {
    const float lo = half ? lo2[1] : lo2[0], hi = half ? hi2[1] : hi2[0];
    const float wdt = hi - lo;
    const float xs = sub == 31 ? hi : lo + wdt * (float)(sub + 1) * (1.f / 32.f);
    const unsigned long long m = __ballot(count_below(xs) >= need);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const unsigned int mh = (unsigned int)(m >> (32 * h));
      if (mh == 0u) continue;
      const int f = __ffs((int)mh) - 1;
      const float w2 = hi2[h] - lo2[h];
      const float nh = f == 31 ? hi2[h] : lo2[h] + w2 * (float)(f + 1) * (1.f / 32.f);
      lo2[h] = lo2[h] + w2 * (float)f * (1.f / 32.f);
      hi2[h] = nh;
    }
  }
  float mu_lo = 0.f, mu_hi = 0.f;
  if (ok) {
    mu_lo = 0.5f * (lo2[0] + hi2[0]);
    mu_hi = 0.5f * (lo2[1] + hi2[1]);
    ok = isfinite(mu_lo) && isfinite(mu_hi);
    // C v = mu B v with B, C weighted sums over the nodes: every eigenvalue is a
    // Rayleigh quotient of u_bar_x, so |mu| <= max_p |u_bar_x,p| for any beta;
    // a value beyond that is rounding of an ill-conditioned B
    mu_lo = fmaxf(mu_lo, -umax);
    mu_hi = fminf(mu_hi, umax);
  }
  if (!ok) {  // bound |mu| <= max_p |u_bar_x,p|
    mu_lo = -umax;
    mu_hi = umax;
  }
  if (lane == 0) {
    if (!ok && status) status[c] |= MEM_ST_LAMBDA_FAIL;
    const float w = g[c * 3], sx = g[c * 3 + 1];
    const float l0 = w + sx * mu_lo, l1 = w + sx * mu_hi;
    if (radius_only) out[c] = fmaxf(fabsf(l0), fabsf(l1));
    else { out[c * 2] = l0; out[c * 2 + 1] = l1; }
  }
}

// ---- ES-BGK collision -----------------------------------------------------------
__global__ __launch_bounds__(128) void k_collide3(int64_t n, float* __restrict__ M, const float* __restrict__ g,
                           float h_scalar, const float* __restrict__ dt_prob,
                           const int32_t* __restrict__ prob, float prandtl, float mu_ref) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float m[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) m[k] = M[c * K3 + k];
  const float nn = m[0];
  if (!(nn > 0.f)) return;
  const float w = g[c * 3], sx = g[c * 3 + 1], sr = g[c * 3 + 2];
  const float s2 = 1.41421356237f;
  const float m1 = m[bidx(1, 0, 0)] / nn;
  const float exx = (s2 * m[bidx(2, 0, 0)] + nn) / nn;
  const float eyy = (s2 * m[bidx(0, 2, 0)] + nn) / nn;
  const float ezz = (s2 * m[bidx(0, 0, 2)] + nn) / nn;
  const float v = w + sx * m1;
  const float pxx = sx * sx * (exx - m1 * m1);       // P_xx / n
  const float prr = 0.5f * sr * sr * (eyy + ezz);    // (P_yy + P_zz) / (2n)
  const float T = (pxx + 2.f * prr) / 3.f;
  const float ip = 1.f / prandtl;
  const float Sxx = T * ip + (1.f - ip) * pxx;
  const float Srr = T * ip + (1.f - ip) * prr;
  float hx[5], hr[5];
  hpoly3((v - w) / sx, Sxx / (sx * sx) - 1.f, hx);
  hpoly3(0.f, Srr / (sr * sr) - 1.f, hr);
  const float sfact[5] = {1.f, 1.f, 1.41421356237f, 2.44948974278f, 4.89897948557f};
  const float h = dt_prob ? 0.5f * dt_prob[prob[c]] : h_scalar;
  const float tau = mu_ref / (prandtl * nn);
  const float rr = h / tau;
#pragma unroll
  for (int a = 0; a <= 4; ++a)
#pragma unroll
    for (int b = 0; b <= 4 - a; ++b)
#pragma unroll
      for (int cc = 0; cc <= 4 - a - b; ++cc) {
        const int i = bidx(a, b, cc);
        const float mt = nn * hx[a] * hr[b] * hr[cc] / (sfact[a] * sfact[b] * sfact[cc]);
        M[c * K3 + i] = (1.f - rr) * m[i] + rr * mt;
      }
}

// ---- local Lax--Friedrichs update in each cell's gauge ----------------------------------
__global__ __launch_bounds__(64) void k_fv3(int64_t n, const float* __restrict__ M, const float* __restrict__ F,
                      const float* __restrict__ rho, const float* __restrict__ g,
                      const int32_t* __restrict__ prob, const int64_t* __restrict__ off,
                      const float* __restrict__ dx, const float* __restrict__ dt,
                      const float* __restrict__ gM, const float* __restrict__ gF,
                      const float* __restrict__ gR, const float* __restrict__ gG,
                      float* __restrict__ Mnew) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int p = prob[c];
  const bool first = c == off[p], last = c == off[p + 1] - 1;
  const float* gc = g + c * 3;
  const float* gl = first ? gG + (2 * p) * 3 : g + (c - 1) * 3;
  const float* gr = last ? gG + (2 * p + 1) * 3 : g + (c + 1) * 3;
  const float* Ml = first ? gM + (int64_t)(2 * p) * K3 : M + (c - 1) * K3;
  const float* Fl = first ? gF + (int64_t)(2 * p) * K3 : F + (c - 1) * K3;
  const float* Mr = last ? gM + (int64_t)(2 * p + 1) * K3 : M + (c + 1) * K3;
  const float* Fr = last ? gF + (int64_t)(2 * p + 1) * K3 : F + (c + 1) * K3;
  const float rl = first ? gR[2 * p] : rho[c - 1];
  const float rr = last ? gR[2 * p + 1] : rho[c + 1];
  const float rc = rho[c];
  const float lm = fmaxf(rl, rc), lp = fmaxf(rc, rr);
  const float k = dt[p] / dx[p];
  float acc[K3];
#pragma unroll
  for (int i = 0; i < K3; ++i) acc[i] = M[c * K3 + i];
  // F_{n-1/2} = (F_l + F_c)/2 + lm/2 (M_l - M_c); F_{n+1/2} = (F_c + F_r)/2 + lp/2 (M_c - M_r)
  // contribution to M_c: k (F_{n-1/2} - F_{n+1/2})
  //   = k/2 [F_l - F_r] + k/2 [lm M_l + lp M_r] - k/2 (lm + lp) M_c
#pragma unroll
  for (int i = 0; i < K3; ++i) acc[i] -= 0.5f * k * (lm + lp) * M[c * K3 + i];
#pragma unroll 1
  for (int side = 0; side < 2; ++side) {
    const float* gn = side ? gr : gl;
    const float* Mn = side ? Mr : Ml;
    const float* Fn = side ? Fr : Fl;
    const float lam = side ? lp : lm;
    const float sgn = side ? -1.f : 1.f;
    float tx[5][5], tr[5][5];
    conn(gn[1] / gc[1], (gn[0] - gc[0]) / gc[1], tx);
    conn(gn[2] / gc[2], 0.f, tr);
    float v[K3];
#pragma unroll
    for (int i = 0; i < K3; ++i) v[i] = lam * Mn[i] + sgn * Fn[i];
    axis_apply<0, false>(tx, v);
    axis_apply<1, false>(tr, v);
    axis_apply<2, false>(tr, v);
#pragma unroll
    for (int i = 0; i < K3; ++i) acc[i] += 0.5f * k * v[i];
  }
#pragma unroll
  for (int i = 0; i < K3; ++i) Mnew[c * K3 + i] = acc[i];
}

// ---- second-order interface fluxes (two-step Lax--Wendroff, FLIC) -----------------------
// Interfaces of problem p are numbered off[p] + p ... off[p + 1] + p: interface
// c + p lies left of cell c, off[p + 1] + p is the right boundary.  Each one is
// evaluated in the gauge of the element to its right (cell or right ghost).
// Per interface: the LLF flux, the Lax--Wendroff half-step moments (to be solved),
// the right element's beta as the solve's start, that gauge and, for FLIC, the
// van Leer limiter per moment.  Ghost rows: 2p left, 2p + 1 right.
__global__ __launch_bounds__(64) void k_iface3(int64_t n, int P, const float* __restrict__ M,
                      const float* __restrict__ F, const float* __restrict__ beta,
                      const float* __restrict__ rho, const float* __restrict__ g,
                      const int32_t* __restrict__ prob, const int64_t* __restrict__ off,
                      const float* __restrict__ dx, const float* __restrict__ dt,
                      const float* __restrict__ gM, const float* __restrict__ gF,
                      const float* __restrict__ gB, const float* __restrict__ gR,
                      const float* __restrict__ gG, int flic, float* __restrict__ hM,
                      float* __restrict__ hB, float* __restrict__ hG, float* __restrict__ hLF,
                      float* __restrict__ hPhi) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n + P) return;
  int p;
  int64_t r, l, ll, iface;  // element indices; -1 = left ghost, -2 = right ghost
  if (t < n) {
    r = t;
    p = prob[r];
    l = r - 1 >= off[p] ? r - 1 : -1;
    ll = r - 2 >= off[p] ? r - 2 : -1;
    iface = r + p;
  } else {
    p = (int)(t - n);
    r = -2;
    l = off[p + 1] - 1;
    ll = l - 1 >= off[p] ? l - 1 : -1;
    iface = off[p + 1] + p;
  }
  const int64_t gl_row = 2 * (int64_t)p, gr_row = 2 * (int64_t)p + 1;
  auto row = [&](const float* cells, const float* ghosts, int64_t e, int w) -> const float* {
    return e >= 0 ? cells + e * w : ghosts + (e == -1 ? gl_row : gr_row) * w;
  };
  const float* gI = row(g, gG, r, 3);
  const float* gl = row(g, gG, l, 3);
  const float* MR = row(M, gM, r, K3);
  const float* FR = row(F, gF, r, K3);
  const float rr = r >= 0 ? rho[r] : gR[gr_row];
  const float rl = l >= 0 ? rho[l] : gR[gl_row];
  const float lam = fmaxf(rl, rr);
  const float k = dt[p] / dx[p];
  float ml[K3];
  {
    const float* src = row(M, gM, l, K3);
#pragma unroll
    for (int i = 0; i < K3; ++i) ml[i] = src[i];
  }
  change_gauge(ml, gI, gl);
  if (flic) {
    // the element beyond r on the right (the right ghost repeats past the end)
    const int64_t rr = (r >= 0 && r + 1 < off[p + 1]) ? r + 1 : -2;
    float u[K3], v[K3];
    {
      const float* src = row(M, gM, ll, K3);
#pragma unroll
      for (int i = 0; i < K3; ++i) u[i] = src[i];
      change_gauge(u, gI, row(g, gG, ll, 3));
    }
    if (rr == r) {
#pragma unroll
      for (int i = 0; i < K3; ++i) v[i] = MR[i];
    } else {
      const float* src = row(M, gM, rr, K3);
#pragma unroll
      for (int i = 0; i < K3; ++i) v[i] = src[i];
      change_gauge(v, gI, row(g, gG, rr, 3));
    }
    // van Leer phi(r) = (r + |r|) / (1 + |r|) on both sides of the interface:
    // r_L = (M_l - M_ll) / (M_r - M_l), r_R = (M_rr - M_r) / (M_r - M_l); the
    // smaller one is taken (waves in either direction)
#pragma unroll
    for (int i = 0; i < K3; ++i) {
      const float a = ml[i] - u[i], b = MR[i] - ml[i], c = v[i] - MR[i];
      const float pl = a * b > 0.f ? 2.f * a / (a + b) : 0.f;
      const float pr = c * b > 0.f ? 2.f * c / (c + b) : 0.f;
      hPhi[iface * K3 + i] = fminf(pl, pr);
    }
  }
  float fl[K3];
  {
    const float* src = row(F, gF, l, K3);
#pragma unroll
    for (int i = 0; i < K3; ++i) fl[i] = src[i];
  }
  change_gauge(fl, gI, gl);
#pragma unroll
  for (int i = 0; i < K3; ++i) {
    const float mr = MR[i], fr = FR[i];
    hLF[iface * K3 + i] = 0.5f * (fl[i] + fr) + 0.5f * lam * (ml[i] - mr);
    hM[iface * K3 + i] = 0.5f * (ml[i] + mr) + 0.5f * k * (fl[i] - fr);
  }
  const float* bR = row(beta, gB, r, K3);
#pragma unroll
  for (int i = 0; i < K3; ++i) hB[iface * K3 + i] = bR[i];
  for (int i = 0; i < 3; ++i) hG[iface * 3 + i] = gI[i];
}

// Conservative update from interface fluxes: cell c takes interface c + p (in its
// own gauge) and interface c + p + 1 moved from its right neighbour's gauge.  The
// interface flux is LLF + phi (LW - LLF), phi = 1 for Lax--Wendroff; an interface
// whose half-step solve failed (not representable, not finite) keeps LLF.
__device__ __forceinline__ void iface_flux(int64_t i, const float* __restrict__ hLF,
                                           const float* __restrict__ hF,
                                           const float* __restrict__ hPhi,
                                           const uint32_t* __restrict__ st, float (&f)[K3]) {
  float lw[K3];
  bool ok = !(st[i] & (MEM_ST_NONREALIZABLE | MEM_ST_NONFINITE));
#pragma unroll
  for (int j = 0; j < K3; ++j) {
    lw[j] = hF[i * K3 + j];
    f[j] = hLF[i * K3 + j];
    ok = ok && isfinite(lw[j]);
  }
  if (!ok) return;
#pragma unroll
  for (int j = 0; j < K3; ++j) f[j] += (hPhi ? hPhi[i * K3 + j] : 1.f) * (lw[j] - f[j]);
}

__global__ __launch_bounds__(64) void k_fv3i(int64_t n, const float* __restrict__ M,
                      const float* __restrict__ g, const int32_t* __restrict__ prob,
                      const int64_t* __restrict__ off, const float* __restrict__ dx,
                      const float* __restrict__ dt, const float* __restrict__ gG,
                      const float* __restrict__ hLF, const float* __restrict__ hF,
                      const float* __restrict__ hPhi, const uint32_t* __restrict__ st,
                      float* __restrict__ Mnew) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int p = prob[c];
  const bool last = c == off[p + 1] - 1;
  const float* gr = last ? gG + (2 * (int64_t)p + 1) * 3 : g + (c + 1) * 3;
  const float k = dt[p] / dx[p];
  float fp[K3];
  iface_flux(c + p + 1, hLF, hF, hPhi, st, fp);
  change_gauge(fp, g + c * 3, gr);
  float fm[K3];
  iface_flux(c + p, hLF, hF, hPhi, st, fm);
#pragma unroll
  for (int i = 0; i < K3; ++i) Mnew[c * K3 + i] = M[c * K3 + i] + k * (fm[i] - fp[i]);
}

// ---- batch book-keeping ---------------------------------------------------------------
__global__ void k_prob_map(const int64_t* __restrict__ off, int P, int32_t* __restrict__ prob) {
  const int p = blockIdx.x;
  if (p >= P) return;
  for (int64_t c = off[p] + threadIdx.x; c < off[p + 1]; c += blockDim.x) prob[c] = p;
}

__global__ void k_ghost_pack(int P, const float* __restrict__ ML, const float* __restrict__ MR,
                             const float* __restrict__ gL, const float* __restrict__ gR,
                             float* gM, float* gB, float* gG) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  for (int side = 0; side < 2; ++side) {
    const float* m = side ? MR + (int64_t)p * K3 : ML + (int64_t)p * K3;
    const float* gg = side ? gR + p * 3 : gL + p * 3;
    const int64_t o = 2 * (int64_t)p + side;
    for (int k = 0; k < K3; ++k) {
      gM[o * K3 + k] = m[k];
      const bool sq = (k == bidx(2, 0, 0) || k == bidx(0, 2, 0) || k == bidx(0, 0, 2));
      gB[o * K3 + k] = k == 0 ? m[0] : (sq ? -0.70710678118f : 0.f);
    }
    for (int k = 0; k < 3; ++k) gG[o * 3 + k] = gg[k];
  }
}

__global__ void k_rmax_init(int P, const float* __restrict__ gR, uint32_t* rmax) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  rmax[p] = __float_as_uint(fmaxf(gR[2 * p], gR[2 * p + 1]));
}

// Per-problem maximum of the spectral radii.  Neighbouring cells almost always
// belong to the same problem: a wave whose lanes share one problem reduces first
// and issues a single atomic, otherwise every lane issues its own.  Non-negative
// floats order like their bit patterns, hence the unsigned maximum.
__global__ void k_rho_max(int64_t n, const float* __restrict__ rho, const int32_t* __restrict__ prob,
                          uint32_t* rmax) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = c < n;
  const float r = in ? rho[c] : 0.f;
  const uint32_t v = (in && isfinite(r) && r >= 0.f) ? __float_as_uint(r) : 0u;
  const int p = in ? prob[c] : -1;
  const int p0 = __shfl(p, 0);
  if (__all(!in || p == p0)) {
    uint32_t m = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0 && p0 >= 0 && m > 0u) atomicMax(&rmax[p0], m);
  } else if (in && v > 0u) {
    atomicMax(&rmax[p], v);
  }
}

// Per-problem maximum of the cells' condition bounds (non-negative, +inf kept;
// NaN ignored), wave-aggregated as in k_rho_max.
__global__ void k_cond_max(int64_t n, const float* __restrict__ cond, const int32_t* __restrict__ prob,
                           uint32_t* out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = c < n;
  const float r = in ? cond[c] : 0.f;
  const uint32_t v = (in && r >= 0.f) ? __float_as_uint(r) : 0u;
  const int p = in ? prob[c] : -1;
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

__global__ void k_zero(int64_t n, float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

// mode 0: set dt where dt <= 0; mode 1: t += dt, dt = CFL dx / max radius;
// both then reset the running maximum to the ghost radii.  mode 2: cap this
// step's dt by the CFL limit of the radii just computed (the transport and the
// second collision half use it), keeping the maximum for mode 1.
__global__ void k_dt3(int P, const float* __restrict__ dx, float cfl, float* t, float* dt,
                      uint32_t* rmax, const float* __restrict__ gR, int mode) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float r = __uint_as_float(rmax[p]);
  const float ndt = cfl * dx[p] / r;
  if (mode == 2) {
    if (ndt < dt[p]) dt[p] = ndt;
    return;
  }
  if (mode == 0) {
    if (!(dt[p] > 0.f)) dt[p] = ndt;
  } else {
    t[p] += dt[p];
    dt[p] = ndt;
  }
  rmax[p] = __float_as_uint(fmaxf(gR[2 * p], gR[2 * p + 1]));
}

__global__ void k_status_or(int64_t n, const uint32_t* __restrict__ src, uint32_t* dst) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) dst[c] |= src[c];
}

// Cells whose step solve could not represent the moments on the nodes take the
// Maxwellian of their gauge (standard normal in gauge coordinates: -1/sqrt(2)
// on the pure second-degree Hermite statistics, indices 4, 7, 9).
__global__ void k_maxwell_fallback(int64_t n, const float* __restrict__ M, float* __restrict__ beta,
                                   uint32_t* __restrict__ status_w) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint32_t st = status_w[c];
  if (!(st & (MEM_ST_NONREALIZABLE | MEM_ST_NONFINITE))) return;
  const float* m = M + c * K3;
  bool fin = m[0] > 0.f;
  for (int k = 0; k < K3; ++k) fin = fin && isfinite(m[k]);
  if (!fin) return;
  float* b = beta + c * K3;
  for (int k = 0; k < K3; ++k) b[k] = 0.f;
  b[0] = m[0];
  b[4] = b[7] = b[9] = -0.70710678118654752f;
  status_w[c] = st | MEM_ST_MAXWELL_FLUX;
}

// Cell-steps by outcome: counts[k] += number of cells with status bit 1 << k
// (k < 9), an LDS count per workgroup added to the device array at the end.
__global__ __launch_bounds__(256) void k_status_count(int64_t n, const uint32_t* __restrict__ st,
                                                      unsigned long long* counts) {
  __shared__ unsigned int sh[9];
  if (threadIdx.x < 9) sh[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
    const uint32_t v = st[c];
    for (int k = 0; k < 9; ++k)
      if (v & (1u << k)) atomicAdd(&sh[k], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 9 && sh[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)sh[threadIdx.x]);
}

// Distribution of per-cell Newton iterations of one step's solve: an LDS
// histogram per workgroup, added to the device histogram at the end.
__global__ __launch_bounds__(256) void k_iter_hist(int64_t n, const int32_t* __restrict__ iters,
                                                   int nbins, unsigned long long* hist) {
  extern __shared__ unsigned int sh_bins[];
  for (int i = threadIdx.x; i < nbins; i += 256) sh_bins[i] = 0u;
  __syncthreads();
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
    const int k = min(max(iters[c], 0), nbins - 1);
    atomicAdd(&sh_bins[k], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += 256)
    if (sh_bins[i]) atomicAdd(&hist[i], (unsigned long long)sh_bins[i]);
}

__global__ void k_copy(int64_t n, const float* __restrict__ src, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ---- conserved totals in FP64 ---------------------------------------------------------
__global__ void k_conserved(const int64_t* __restrict__ off, const float* __restrict__ dx,
                            const float* __restrict__ M, const float* __restrict__ g,
                            double* out) {
  const int p = blockIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t c = off[p] + threadIdx.x; c < off[p + 1]; c += blockDim.x) {
    const float* m = M + c * K3;
    const double nn = m[0];
    const double w = g[c * 3], sx = g[c * 3 + 1], sr = g[c * 3 + 2];
    const double r2 = 1.4142135623730951;
    const double m1 = m[bidx(1, 0, 0)] / nn;
    const double exx = (r2 * m[bidx(2, 0, 0)] + nn) / nn;
    const double err = (r2 * (m[bidx(0, 2, 0)] + m[bidx(0, 0, 2)]) + 2.0 * nn) / nn;
    const double v = w + sx * m1;
    const double trP = nn * (sx * sx * (exx - m1 * m1) + sr * sr * err);
    s0 += nn;
    s1 += nn * v;
    s2 += 0.5 * nn * v * v + 0.5 * trP;
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = s0; red[1][threadIdx.x] = s1; red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double h = dx[p];
    out[p * 3] = h * red[0][0];
    out[p * 3 + 1] = h * red[1][0];
    out[p * 3 + 2] = h * red[2][0];
  }
}

// ---- launchers ---------------------------------------------------------------------------
static inline unsigned nb(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_gauge3(mem_ctx_t c, int64_t n, float* M, float* beta, float* g, hipStream_t s) {
  (void)c;
  if (n <= 0) return hipSuccess;
  k_gauge3<<<nb(n, 128), 128, 0, s>>>(n, M, beta, g);
  return hipGetLastError();
}

hipError_t launch_flux3(mem_ctx_t c, int64_t n, const float* beta, const float* g, float* F,
                        float* out, bool want_lam, bool radius_only, uint32_t* status,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  // log Z at beta; then, with speeds, S = sigma . Psi and the degree-5 columns S5,
  // without, only the 128 flux columns
  SolveParams dummy{};
  hipError_t e = launch_lse3(c, n, nullptr, nullptr, n, nullptr, const_cast<float*>(beta), false,
                             dummy, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  if (!want_lam) {
    // fluxes only: the 70 columns E[phi_i], E[u_x phi_i] (128-column operand)
    if (!F) return hipSuccess;
    e = launch_assemble5(c, n, beta, c->d_psiF, c->w_S5, s);
    if (e != hipSuccess) return e;
    k_flux3<<<nb(n, 128), 128, 0, s>>>(n, c->w_S5, beta, g, F, 1);
    return hipGetLastError();
  }
  e = launch_assemble3(c, n, nullptr, nullptr, n, beta, c->d_psi, c->w_S, s);
  if (e != hipSuccess) return e;
  if (F) {
    k_flux3<<<nb(n, 128), 128, 0, s>>>(n, c->w_S, beta, g, F, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    e = launch_assemble5(c, n, beta, c->d_psi5, c->w_S5, s);
    if (e != hipSuccess) return e;
    double um = 0.0;
    for (int p = 0; p < c->Q; ++p) um = fmax(um, fabs(c->h_nodes[(size_t)p * 3]));
    k_eig3<<<nb(n, EIG_WAVES), 256, 0, s>>>(n, c->w_S, c->w_S5, c->d_ux_src, c->d_ux_w, g,
                                            (float)um, out, radius_only ? 1 : 0, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_collide3(mem_ctx_t c, int64_t n, float* M, const float* g, float h_scalar,
                           const float* dt_prob, const int32_t* prob, float prandtl, float mu_ref,
                           hipStream_t s) {
  (void)c;
  if (n <= 0) return hipSuccess;
  k_collide3<<<nb(n, 128), 128, 0, s>>>(n, M, g, h_scalar, dt_prob, prob, prandtl, mu_ref);
  return hipGetLastError();
}

hipError_t launch_fv3(mem_ctx_t c, int64_t n, const float* M, const float* F, const float* rho,
                      const float* g, const int32_t* prob, const int64_t* offsets, const float* dx,
                      const float* dt, float* Mnew, int P, hipStream_t s) {
  (void)P;
  if (n <= 0) return hipSuccess;
  k_fv3<<<nb(n, 64), 64, 0, s>>>(n, M, F, rho, g, prob, offsets, dx, dt, c->w_gM, c->w_gF, c->w_gR,
                                 c->w_gG, Mnew);
  return hipGetLastError();
}

hipError_t launch_iface3(mem_ctx_t c, int64_t n, int P, const float* M, const float* F,
                        const float* beta, const float* rho, const float* g, const int32_t* prob,
                        const int64_t* offsets, const float* dx, const float* dt, bool flic,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_iface3<<<nb(n + P, 64), 64, 0, s>>>(n, P, M, F, beta, rho, g, prob, offsets, dx, dt, c->w_gM,
                                        c->w_gF, c->w_gB, c->w_gR, c->w_gG, flic ? 1 : 0, c->w_hM,
                                        c->w_hB, c->w_hG, c->w_hLF, c->w_hPhi);
  return hipGetLastError();
}

hipError_t launch_fv3i(mem_ctx_t c, int64_t n, const float* M, const float* g, const int32_t* prob,
                       const int64_t* offsets, const float* dx, const float* dt, bool flic,
                       float* Mnew, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fv3i<<<nb(n, 64), 64, 0, s>>>(n, M, g, prob, offsets, dx, dt, c->w_gG, c->w_hLF, c->w_hF,
                                  flic ? c->w_hPhi : nullptr, c->w_status, Mnew);
  return hipGetLastError();
}

hipError_t launch_prob_map(mem_ctx_t c, const int64_t* offsets, int P, int32_t* prob,
                           hipStream_t s) {
  (void)c;
  if (P <= 0) return hipSuccess;
  k_prob_map<<<P, 256, 0, s>>>(offsets, P, prob);
  return hipGetLastError();
}

hipError_t launch_ghost_pack(mem_ctx_t c, const mem_batch_t* b, hipStream_t s) {
  const int P = b->n_problems;
  k_ghost_pack<<<nb(P, 128), 128, 0, s>>>(P, b->M_left, b->M_right, b->g_left, b->g_right, c->w_gM,
                                          c->w_gB, c->w_gG);
  return hipGetLastError();
}

hipError_t launch_rho_max(mem_ctx_t c, int64_t n, const float* rho, const int32_t* prob, int P,
                          hipStream_t s) {
  (void)P;
  if (n <= 0) return hipSuccess;
  k_rho_max<<<nb(n, 256), 256, 0, s>>>(n, rho, prob, c->w_rmax);
  return hipGetLastError();
}

hipError_t launch_zero(int64_t n, float* x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_zero<<<nb(n, 256), 256, 0, s>>>(n, x);
  return hipGetLastError();
}

hipError_t launch_cond_max(int64_t n, const float* cond, const int32_t* prob, float* out,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_cond_max<<<nb(n, 256), 256, 0, s>>>(n, cond, prob, reinterpret_cast<uint32_t*>(out));
  return hipGetLastError();
}

hipError_t launch_dt_update(mem_ctx_t c, int P, const float* dx, float cfl, float* t, float* dt,
                            bool advance_t, hipStream_t s) {
  k_dt3<<<nb(P, 128), 128, 0, s>>>(P, dx, cfl, t, dt, c->w_rmax, c->w_gR, advance_t ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_dt_cap(mem_ctx_t c, int P, const float* dx, float cfl, float* dt,
                         hipStream_t s) {
  k_dt3<<<nb(P, 128), 128, 0, s>>>(P, dx, cfl, nullptr, dt, c->w_rmax, c->w_gR, 2);
  return hipGetLastError();
}

hipError_t launch_rmax_init(mem_ctx_t c, int P, hipStream_t s) {
  k_rmax_init<<<nb(P, 128), 128, 0, s>>>(P, c->w_gR, c->w_rmax);
  return hipGetLastError();
}

hipError_t launch_maxwell_fallback(mem_ctx_t c, int64_t n, const float* M, float* beta,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_maxwell_fallback<<<nb(n, 256), 256, 0, s>>>(n, M, beta, c->w_status);
  return hipGetLastError();
}

hipError_t launch_status_count(int64_t n, const uint32_t* st, int64_t* counts, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(nb(n, 256), 1024);
  k_status_count<<<grid, 256, 0, s>>>(n, st, reinterpret_cast<unsigned long long*>(counts));
  return hipGetLastError();
}

hipError_t launch_iter_hist(int64_t n, const int32_t* iters, int nbins, int64_t* hist,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(nb(n, 256), 1024);
  k_iter_hist<<<grid, 256, (size_t)nbins * sizeof(unsigned int), s>>>(
      n, iters, nbins, reinterpret_cast<unsigned long long*>(hist));
  return hipGetLastError();
}

hipError_t launch_status_or(int64_t n, const uint32_t* src, uint32_t* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_status_or<<<nb(n, 256), 256, 0, s>>>(n, src, dst);
  return hipGetLastError();
}

hipError_t launch_copy(int64_t n, const float* src, float* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_copy<<<nb(n, 256), 256, 0, s>>>(n, src, dst);
  return hipGetLastError();
}

hipError_t launch_conserved(mem_ctx_t c, const mem_batch_t* b, const float* M, const float* g,
                            double* out, hipStream_t s) {
  (void)c;
  if (b->n_problems <= 0) return hipSuccess;
  k_conserved<<<b->n_problems, 256, 0, s>>>(b->cell_offsets, b->dx, M, g, out);
  return hipGetLastError();
}

}  // namespace memk
