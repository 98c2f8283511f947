// 3D (35-moment) maximal-entropy dual solve on gfx950.
//
// One Newton iteration of Alg. 1 is four launches over a work-list of live
// cells (cells that have not met a stopping test):
//   k_assemble3  : sigma_p = exp(beta.phi_p + log w~_p - log Z) for 16-node
//                  groups, the exponent itself an MFMA product of the node
//                  table with beta, then S = sigma . Psi on FP32 MFMA, where
//                  Psi[p][(i,j)] = phi_i phi_j(u_p) (630 pair columns + 10 pad).
//                  Row (0, j) of S gives E[phi_j]; the rest gives E[phi_i phi_j].
//   k_direction3 : Hessian H_ij = E[phi_i phi_j] - E_i E_j (App. C) and gradient
//                  G_i = E_i - M_i/n, Cholesky with the lambda*I shift, Newton
//                  direction, decrement, stopping tests; cells whose FP32 pivot
//                  ratio is below the threshold go to the FP64 kernel.
//   k_fallback3  : the same direction in FP64 (rare path).
//   k_lse3       : backtracking line search with the Armijo test of Alg. 1; each
//                  trial is one log-sum-exp pass (Sec. 3.1) over the nodes.
// beta_0 is held at n, which zeroes G_0 and decouples H_00 = n^2/beta_0^2, so
// the Newton system is the 34 x 34 covariance block.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "dfloat.h"
#include "mem_internal.h"

namespace memk {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Wait for every outstanding vector-memory load of this wave, direct-to-LDS
// loads included.
__device__ __forceinline__ void vm_wait_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Third descriptor word of a raw buffer resource on CDNA (gfx9 family).
constexpr int BUF_DW3 = 0x00020000;

// Generic -> LDS address space, for the direct global -> LDS loads.
__device__ __forceinline__ __attribute__((address_space(3))) void* lds_ptr(const void* p) {
  return (__attribute__((address_space(3))) void*)(p);
}

// Wave-aggregated append of `cell` to a work list.  Every lane of the wave
// must call it (it uses a ballot).
__device__ __forceinline__ void wave_append(bool pred, int cell, int32_t* list, int32_t* ctr) {
  unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(ctr, __popcll(mask));
  base = __shfl(base, leader);
  if (pred) {
    unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
    list[base + __popcll(below)] = cell;
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}


// --------------------------------------------------------------------------
// init: validate, beta_0 = n, seed the live list
// --------------------------------------------------------------------------
__global__ void k_init3(int64_t n, const float* __restrict__ M, float* __restrict__ beta,
                        float* alpha, int32_t* iters_w, uint32_t* status_w, float* resid_w,
                        float* rbest_w, int32_t* itbest_w,
                        int32_t* list, int32_t* ctr, int32_t* iters_out, float* resid_out,
                        uint32_t* status_out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = false;
  if (c < n) {
    const float* m = M + c * K3;
    float* b = beta + c * K3;
    bool fin = true;  // & rather than &&: the 70 loads issue together
#pragma unroll
    for (int k = 0; k < K3; ++k) fin = fin & isfinite(m[k]) & (k == 0 || isfinite(b[k]));
    uint32_t st = 0;
    if (!fin) st = MEM_ST_NONFINITE;
    else if (!(m[0] > 0.f)) st = MEM_ST_NONREALIZABLE;
    ok = st == 0;
    if (ok) b[0] = m[0];
    alpha[c] = 1.f;
    iters_w[c] = 0;
    status_w[c] = st;
    resid_w[c] = INFINITY;
    rbest_w[c] = INFINITY;
    itbest_w[c] = 0;
    if (!ok) {
      if (iters_out) iters_out[c] = 0;
      if (resid_out) resid_out[c] = INFINITY;
      if (status_out) status_out[c] = st;
    }
  }
  wave_append(ok, (int)c, list, ctr);
}

__global__ void k_set_ctr(int32_t* ctr, int n) {
  if (threadIdx.x < (unsigned)n) ctr[threadIdx.x] = 0;
}

// --------------------------------------------------------------------------
// log-sum-exp pass and the Armijo backtracking line search of Alg. 1
// --------------------------------------------------------------------------
// One wavefront per cell.  The exponent on the tensor grid factors axis by
// axis (sum factorisation, phi_(a,b,c) = h_a h_b h_c):
//   V[i][j][c] = sum_{a,b} beta_abc h_a(x_i) h_b(x_j),
//   e(i,j,l)   = lw_i + lw_j + lw_l + sum_c V[i][j][c] h_c(x_l),
// and it is linear in beta, so for the trial point beta + alpha dbeta the
// coefficients are V_beta + alpha V_dbeta: the factors are built once and each
// trial of the backtracking search costs 5 FMAs and one exp per node.
// t1 holds the one-dimensional tables (h_a(x_k) at [a n + k], lw_k at
// [5 n + k]); only the high parts are used here.
constexpr int NBC = 15;  // (b, c) with b + c <= 4
__device__ __forceinline__ int tri(int m) { return m * (m + 1) / 2; }
__device__ __forceinline__ int bidx3(int a, int b, int c) {
  const int t = a + b + c, m = b + c;
  return t * (t + 1) * (t + 2) / 6 + tri(m) + c;
}

// Partial log-sum-exp (max, sum) of this lane's node pairs (i, j), all l,
// for the coefficients V_beta + alpha V_dbeta.  NT = n when it is known at
// compile time (exponents of a pair kept in registers), 0 otherwise (two
// sweeps over l).
template <bool LS, int NT>
__device__ __forceinline__ void lse_pairs(int n, int lane, float alpha, const float* sH,
                                          const float* sVb, const float* sVd, float& mx,
                                          float& sm) {
  const int nn = NT > 0 ? NT : n;
  for (int q = lane; q < nn * nn; q += 64) {
    const int i = q / nn, j = q % nn;
    const float base = sH[5 * nn + i] + sH[5 * nn + j];
    float v[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = LS ? fmaf(alpha, sVd[q * 5 + c], sVb[q * 5 + c]) : sVb[q * 5 + c];
    auto ex = [&](int l) {
      float x = base + sH[5 * nn + l];
#pragma unroll
      for (int c = 0; c < 5; ++c) x = fmaf(v[c], sH[c * nn + l], x);
      return x;
    };
    if constexpr (NT > 0) {
      float e[NT];
      float gm = -FLT_MAX;
#pragma unroll
      for (int l = 0; l < NT; ++l) { e[l] = ex(l); gm = fmaxf(gm, e[l]); }
      if (gm > mx) { sm *= __expf(mx - gm); mx = gm; }
#pragma unroll
      for (int l = 0; l < NT; ++l) sm += __expf(e[l] - mx);
    } else {
      float gm = -FLT_MAX;
      for (int l = 0; l < nn; ++l) gm = fmaxf(gm, ex(l));
      if (gm > mx) { sm *= __expf(mx - gm); mx = gm; }
      for (int l = 0; l < nn; ++l) sm += __expf(ex(l) - mx);
    }
  }
}

template <bool LS, int NT>
__global__ __launch_bounds__(64) void k_lse3(
    const float2* __restrict__ t1, int n, const int32_t* __restrict__ list,
    const int32_t* __restrict__ ctr, int64_t ncell, const float* __restrict__ M,
    float* __restrict__ beta, const float* __restrict__ dbeta, float* __restrict__ logZ,
    float* __restrict__ Lval, float* __restrict__ alpha_w, const float* __restrict__ gdot,
    SolveParams p, int32_t* reset_a, int32_t* reset_b) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (reset_a) *reset_a = 0;
    if (reset_b) *reset_b = 0;
  }
  if (NT > 0) n = NT;
  const int64_t count = ctr ? (int64_t)(*ctr) : ncell;
  const int64_t slot = blockIdx.x;
  if (slot >= count) return;
  const int lane = threadIdx.x;
  const int64_t cell = list ? (int64_t)list[slot] : slot;
  extern __shared__ float dynf[];
  float* sB = dynf;               // [36] beta, then dbeta at [36..71]
  float* sH = dynf + 72;          // [6][n]: h_a(x_k), lw_k (high parts)
  float* sVb = sH + 6 * n;        // [n*n][5]
  float* sVd = sVb + n * n * 5;   // [n*n][5]

  const bool kin = lane >= 1 && lane < K3;
  const float bk = kin ? beta[cell * K3 + lane] : 0.f;
  const float dk = (LS && kin) ? dbeta[cell * 36 + lane] : 0.f;
  // M may be null (log Z only): the linear term of L is then dropped
  const float nn = M ? M[cell * K3] : 1.f;
  const float mk = (M && kin) ? M[cell * K3 + lane] / nn : 0.f;
  if (lane < 36) { sB[lane] = bk; sB[36 + lane] = dk; }
  for (int t = lane; t < 6 * n; t += 64) sH[t] = t1[t].x;
  __builtin_amdgcn_wave_barrier();
  // coefficients of pair (i, j): v_c = sum_{a+b+c<=4} beta_abc h_a(x_i) h_b(x_j),
  // straight from the 15 products h_a(x_i) h_b(x_j) with compile-time indices
  float bb[K3], bd[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) {
    bb[k] = sB[k];  // sB[0] = 0: beta_0 enters through log Z
    bd[k] = LS ? sB[36 + k] : 0.f;
  }
  for (int q = lane; q < n * n; q += 64) {
    const int i = q / n, j = q - (q / n) * n;
    float ha[5], hb[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) { ha[a] = sH[a * n + i]; hb[a] = sH[a * n + j]; }
    float vb[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, vd[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 5; ++a) {
#pragma unroll
      for (int b = 0; a + b < 5; ++b) {
        const float pab = ha[a] * hb[b];
#pragma unroll
        for (int c = 0; a + b + c < 5; ++c) {
          vb[c] = fmaf(bb[bidx3(a, b, c)], pab, vb[c]);
          if (LS) vd[c] = fmaf(bd[bidx3(a, b, c)], pab, vd[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sVb[q * 5 + c] = vb[c];
      if (LS) sVd[q * 5 + c] = vd[c];
    }
  }
  __builtin_amdgcn_wave_barrier();

  float L0 = 0.f, gd = 0.f;
  if (LS) { L0 = Lval[cell]; gd = gdot[cell]; }
  float alpha = 1.f;
  for (int s = 0;; ++s) {
    float mx = -FLT_MAX, sm = 0.f;
    lse_pairs<LS, NT>(n, lane, alpha, sH, sVb, sVd, mx, sm);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float om = __shfl_xor(mx, off), os = __shfl_xor(sm, off);
      const float nm = fmaxf(mx, om);
      sm = sm * __expf(mx - nm) + os * __expf(om - nm);
      mx = nm;
    }
    const float lz = mx + __logf(sm);
    const float bt = fmaf(alpha, dk, bk);
    const float Lt = lz - wave_sum(bt * mk);  // dual objective up to the beta_0 term
    if (!LS) {
      if (lane == 0) { logZ[cell] = lz; Lval[cell] = Lt; }
      return;
    }
    // Armijo test with the floating-point tolerance (Alg. 1, ArmijoCondition)
    const float LD = L0 - Lt;
    const float gradD = -p.c * alpha * gd;
    const bool sat = (LD - gradD) >= -(p.atol + p.rtol * fabsf(LD));
    if (sat || s >= p.max_ls) {  // the last trial is kept (Alg. 1)
      if (kin) beta[cell * K3 + lane] = bt;
      if (lane == 0) { logZ[cell] = lz; Lval[cell] = Lt; alpha_w[cell] = alpha; }
      return;
    }
    alpha *= 0.5f;
  }
}

// --------------------------------------------------------------------------
// assembly: S[cell][col] = sum_p sigma_p Psi[p][col] on FP32 MFMA
// --------------------------------------------------------------------------
// Split mode (nsplit > 1, few live cells): workgroup b takes tile b % ntile
// and node groups [split * ngroups / nsplit, (split + 1) * ngroups / nsplit)
// of split = b / ntile, and writes its partial sums to
// Sp[split][slot][NCOL]; k_sum_splits adds them in a fixed order.
// NB4 quadruples of 16-column blocks: 10 (S, 640 columns) or 2 (the 128
// columns of the degree-5 products used by the characteristic speeds).
// AW wavefronts of 16 cells per workgroup (4 or 8): a workgroup holds 16 AW
// cells, and its AW waves share each node half staged in LDS.
template <int NB4, int AW>
__global__ __launch_bounds__(64 * AW, 8 / AW) void k_assemble3(
    const float* __restrict__ phiA, const float* __restrict__ psi, int ngroups,
    const int32_t* __restrict__ list, const int32_t* __restrict__ ctr, int64_t n,
    const float* __restrict__ beta, const float* __restrict__ logZ, float* __restrict__ S,
    int ntile, int nsplit, float* __restrict__ Sp) {
  const int64_t count = ctr ? (int64_t)(*ctr) : n;
  constexpr int TW = 16 * AW;  // cells per workgroup
  const int split = (int)(blockIdx.x / ntile);
  const int64_t tile = (int64_t)(blockIdx.x % ntile) * TW;
  if (tile >= count) return;
  const int gbeg = (int)((int64_t)split * ngroups / nsplit);
  const int gend = (int)((int64_t)(split + 1) * ngroups / nsplit);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int64_t slot = tile + wave * 16 + (lane & 15);
  const bool valid = slot < count;
  const int64_t cell = valid ? (list ? (int64_t)list[slot] : slot) : 0;

  // exponent B operand (beta, lane l holding k = 4j + l/16), kept in LDS to
  // leave the registers to the 160 accumulators
  __shared__ float sBt[NJ * 64 * AW];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = 4 * j + kq;
    sBt[j * 64 * AW + threadIdx.x] =
        k == 0 ? 1.f : ((valid && k < K3) ? beta[cell * K3 + k] : 0.f);
  }
  const float lz = valid ? logZ[cell] : 0.f;

  constexpr int NB = 4 * NB4;       // accumulator tiles
  constexpr int WIDTH = 16 * NB;    // output row width
  f4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = (f4){0.f, 0.f, 0.f, 0.f};

  // Half-group ping-pong: half h of the node range holds Psi rows 2(h%2),
  // 2(h%2)+1 (20 KB) of group h/2 and lives in buffer h%2; the exponent table
  // of a group travels with its first half.  Halves move global -> LDS with
  // direct (register-free) loads: half h+1 is issued right after the barrier
  // that opens half h and waited for at the next barrier, so its latency runs
  // under the MFMAs of half h.
  __shared__ f4 sB0[2 * NB4 * 64];  // 20 KB each for S
  __shared__ f4 sB1[2 * NB4 * 64];
  __shared__ f4 sA4[NJ * 16];      // exponent operand of one node group
  const float* sA = reinterpret_cast<const float*>(sA4);
  // buffer resources (bounds = the tables); lane l of wave w moves the 16 bytes
  // at offset 16 (64 w + l) + 1024 AW i of a half into LDS element
  // 64 w + 64 AW i + l (a half is 128 NB4 elements; with AW = 8 the last
  // round covers only its first waves, a wave-uniform test)
  const __amdgpu_buffer_rsrc_t rB =
      __builtin_amdgcn_make_buffer_rsrc((void*)psi, (short)0, ngroups * (4 * NB4 * 64 * 16), BUF_DW3);
  const __amdgpu_buffer_rsrc_t rA =
      __builtin_amdgcn_make_buffer_rsrc((void*)phiA, (short)0, ngroups * (NJ * 64 * 4), BUF_DW3);
  const int voff = (int)threadIdx.x * 16;
  const int hend = 2 * gend;
  constexpr int HALF = 2 * NB4 * 64;              // elements of a half
  constexpr int ROUNDS = (HALF + 64 * AW - 1) / (64 * AW);
  auto fetch = [&](f4* dst, int h, bool first) {
#pragma unroll
    for (int i = 0; i < ROUNDS; ++i)
      if (HALF % (64 * AW) == 0 || 64 * wave + 64 * AW * i < HALF)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rB, lds_ptr(dst + 64 * wave + 64 * AW * i), 16,
                                                 voff, h * (HALF * 16) + 1024 * AW * i, 0, 0);
    if (first && threadIdx.x < NJ * 16)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rA, lds_ptr(sA4 + 64 * wave), 16, voff,
                                               (h >> 1) * (NJ * 64 * 4), 0, 0);
    __builtin_amdgcn_sched_barrier(0);  // issue here, ahead of the MFMAs it hides under
  };
  auto half = [&](const f4* buf, float s0, float s1) {
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const float sgr = rr ? s1 : s0;
#pragma unroll
      for (int b4 = 0; b4 < NB4; ++b4) {
        const f4 bv = buf[(rr * NB4 + b4) * 64 + lane];
        acc[4 * b4 + 0] = mfma4(sgr, bv[0], acc[4 * b4 + 0]);
        acc[4 * b4 + 1] = mfma4(sgr, bv[1], acc[4 * b4 + 1]);
        acc[4 * b4 + 2] = mfma4(sgr, bv[2], acc[4 * b4 + 2]);
        acc[4 * b4 + 3] = mfma4(sgr, bv[3], acc[4 * b4 + 3]);
      }
    }
  };
  fetch(sB0, 2 * gbeg, true);
  for (int g = gbeg; g < gend; ++g) {
    const int h = 2 * g;
    // this wave's direct loads have landed before the barrier lets the other
    // waves read them (the barrier alone does not order them)
    vm_wait_all();
    __syncthreads();  // half h is in LDS; every wave is done with buffer 1
    fetch(sB1, h + 1, false);
    f4 e = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NJ; ++j) e = mfma4(sA[j * 64 + lane], sBt[j * 64 * AW + threadIdx.x], e);
    float sg[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) sg[r] = valid ? __expf(e[r] - lz) : 0.f;
    half(sB0, sg[0], sg[1]);
    vm_wait_all();
    __syncthreads();  // half h+1 is in LDS; every wave is done with buffer 0 and sA
    // the last group re-fetches its own first half (never read again), which
    // keeps the loop free of a conditional load
    fetch(sB0, min(h + 2, hend - 2), true);
    half(sB1, sg[2], sg[3]);
  }
  vm_wait_all();  // no direct load may still target LDS when the workgroup ends
  // D layout: lane l, register q -> row 4(l/16) + q of the wave's 16 cells, column l%16
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t sl = tile + wave * 16 + 4 * kq + q;
    if (sl < count) {
      float* dst;
      if (nsplit > 1) {
        dst = Sp + ((size_t)split * ntile * TW + sl) * WIDTH + (lane & 15);
      } else {
        const int64_t cw = list ? (int64_t)list[sl] : sl;
        dst = S + cw * WIDTH + (lane & 15);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) dst[16 * b] = acc[b][q];
    }
  }
}

// S[cell] = sum over splits of Sp[split][slot] (fixed order: deterministic);
// rows of W floats.
template <int W>
__global__ void k_sum_splits(const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
                             int64_t n, int64_t rows, int nsplit, const float* __restrict__ Sp,
                             float* __restrict__ S) {
  const int64_t count = ctr ? (int64_t)(*ctr) : n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slot = t / (W / 4);
  const int q = (int)(t % (W / 4));
  if (slot >= count) return;
  const int64_t cell = list ? (int64_t)list[slot] : slot;
  const size_t stride = (size_t)rows * W;  // rows = tiles x cells per tile
  const f4* src = reinterpret_cast<const f4*>(Sp + (size_t)slot * W) + q;
  f4 acc = src[0];
  for (int k = 1; k < nsplit; ++k) {
    const f4 v = *reinterpret_cast<const f4*>(Sp + k * stride + (size_t)slot * W + 4 * q);
    acc += v;
  }
  reinterpret_cast<f4*>(S + cell * W)[q] = acc;
}

// --------------------------------------------------------------------------
// Newton direction (FP32) with the lambda*I shift of Alg. 1
// --------------------------------------------------------------------------

struct DirOut {
  int32_t* next_list; int32_t* next_ctr;
  int32_t* iters_out; float* resid_out; uint32_t* status_out;
  int32_t* done_list; int32_t* done_ctr;  // converged cells (for refinement), may be null
};

// Stopping tests of Alg. 1 (residual sign read as 1/2 G^T (H + lambda I)^-1 G)
// and the book-keeping shared by the FP32 and FP64 direction kernels, plus
// three exits the paper does not need in FP64:
//  * a dual value below min_p log w~_p certifies that no minimiser exists (the
//    targets lie outside the moment set of distributions on the nodes);
//  * stall: the FP32 residual has not halved for STALL_WINDOW iterations (its
//    rounding floor); with refinement on, such a cell -- like a converged one
//    -- is handed to the compensated refinement, which decides the status;
//  * no progress: a residual above STALL_GATE that has not halved for
//    NOPROGRESS_WINDOW iterations ends the cell as stagnated (iterates that
//    drift along a ray of the dual without reducing the residual).
// Returns 1 when the cell stays live, 2 when it goes to refinement, 0 otherwise.
constexpr int STALL_WINDOW = 6;
constexpr float STALL_GATE = 1e-3f;
constexpr int NOPROGRESS_WINDOW = 30;  // residual above the gate not halved: give up

// Per-cell Newton state, read at kernel entry so that its latency hides
// behind the factorisation.  bmax = max_{i>=1} |beta_i| (wave reduction).
struct CellState {
  int it, itbest;
  uint32_t st;
  float rbest, alpha, L, bmax;
};

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

__device__ __forceinline__ CellState load_state(int64_t cell, int lane, const int32_t* iters_w,
                                                const uint32_t* status_w, const float* rbest_w,
                                                const int32_t* itbest_w, const float* alpha_w,
                                                const float* Lval, const float* beta) {
  // wave-uniform values: keep them in scalar registers
  auto ui = [](int v) { return __builtin_amdgcn_readfirstlane(v); };
  auto uf = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
  CellState cs;
  cs.it = ui(iters_w[cell]);
  cs.itbest = ui(itbest_w[cell]);
  cs.st = (uint32_t)ui((int)status_w[cell]);
  cs.rbest = uf(rbest_w[cell]);
  cs.alpha = uf(alpha_w[cell]);
  cs.L = uf(Lval[cell]);
  cs.bmax = uf(wave_max(lane >= 1 && lane < K3 ? fabsf(beta[cell * K3 + lane]) : 0.f));
  return cs;
}

__device__ __forceinline__ int finish_cell(int64_t cell, float r, float res, bool dir_ok,
                                           uint32_t extra, const SolveParams& p,
                                           const CellState& cs, float* gdot, int32_t* iters_w,
                                           uint32_t* status_w, float* resid_w, float* rbest_w,
                                           int32_t* itbest_w, const DirOut& o) {
  const int it = cs.it + 1;
  iters_w[cell] = it;
  uint32_t st = cs.st | extra;
  resid_w[cell] = r;
  int itbest = cs.itbest;
  if (r < 0.5f * cs.rbest) { rbest_w[cell] = r; itbest_w[cell] = it; itbest = it; }
  const bool conv = (r <= p.tol_grad) || (res <= p.tol_dec && r <= p.tol_loose);
  const bool near = r <= STALL_GATE && p.refine > 0;
  const bool stall = near && (it - itbest >= STALL_WINDOW || cs.alpha <= p.alpha_min ||
                              it >= p.max_iter);
  bool done = true, cand = false;
  if (conv || stall) { st |= MEM_ST_CONVERGED; cand = p.refine > 0; }
  else if (cs.L < p.lmin || (p.beta_max > 0.f && cs.bmax > p.beta_max))
    st |= MEM_ST_NONREALIZABLE;
  else if (!isfinite(r) || !dir_ok) st |= MEM_ST_NONFINITE;
  else if (cs.alpha <= p.alpha_min || it - itbest >= NOPROGRESS_WINDOW)
    st |= MEM_ST_STAGNATED;
  else if (it >= p.max_iter) st |= MEM_ST_MAXITER;
  else done = false;
  status_w[cell] = st;
  if (done) {
    if (o.iters_out) o.iters_out[cell] = it;
    if (o.resid_out) o.resid_out[cell] = r;
    if (o.status_out) o.status_out[cell] = st;
    return cand ? 2 : 0;
  }
  gdot[cell] = -2.f * res;  // G . dbeta = -G^T (H + lambda I)^-1 G
  return 1;
}

// Wave-cooperative Cholesky for one cell per wave.  Lane j < 34 holds column
// j of the SPD matrix in registers (a[i] = A[i][j]); step k shares column k of
// the current matrix (pivot included) through LDS, updates the trailing
// columns and stores column k of L in the same row.  On return lane i holds
// 1 / L[i][i] in dinv; for i > j, lane j's a[i] equals L[i][j] * L[j][j].
__device__ __forceinline__ float rl(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double rl(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// Lm: this wave's LDS copy of L, row k = column k of L ([NH][LST]).  At step k
// every lane publishes its L[lane][k] with one LDS write and reads column k
// back with broadcast reads (all lanes read the same addresses): a step costs
// one write, a few 16-byte reads and the trailing FMAs.
constexpr int LST = NH + 2;  // row stride of Lm (16-byte aligned rows)

// An empty asm that reads and writes every entry of a 34-value column, so that
// the values exist in registers at this point (keeps the factorisation
// right-looking; see wave_chol).
template <typename T>
__device__ __forceinline__ void keep_col(T (&v)[NH]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
               "+v"(v[6]), "+v"(v[7]), "+v"(v[8]));
  asm volatile("" : "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
               "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]));
  asm volatile("" : "+v"(v[18]), "+v"(v[19]), "+v"(v[20]), "+v"(v[21]), "+v"(v[22]),
               "+v"(v[23]), "+v"(v[24]), "+v"(v[25]));
  asm volatile("" : "+v"(v[26]), "+v"(v[27]), "+v"(v[28]), "+v"(v[29]), "+v"(v[30]),
               "+v"(v[31]), "+v"(v[32]), "+v"(v[33]));
}

template <typename T>
__device__ __forceinline__ bool wave_chol(T (&a)[NH], T& dinv, int lane, T& dmin, T& dmax, T* Lm) {
  bool ok = true;
  dmin = (T)FLT_MAX; dmax = 0;
  dinv = 1;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    // column k of the current matrix, pivot included, through row k of Lm
    T* row = Lm + k * LST;
    if (lane < NH) row[lane] = a[k];
    __builtin_amdgcn_wave_barrier();
    T u[NH];
#pragma unroll
    for (int i = k; i < NH; ++i) u[i] = row[i];
    const T d = u[k];
    ok = ok && (d > (T)0) && isfinite(d);
    // the pivot is the same on every lane (read back from LDS): a failed
    // factorisation stops here, uniformly, instead of finishing the sweep
    if (!ok) return false;
    dmin = d < dmin ? d : dmin;
    dmax = d > dmax ? d : dmax;
    const T inv = rsq(d);
    if (lane == k) dinv = inv;
    // A[i][j] -= A[i][k] A[k][j] / d for j > k (multiplier 0 on lanes <= k)
    const T cj = lane > k ? a[k] * (inv * inv) : (T)0;
#pragma unroll
    for (int i = k + 1; i < NH; ++i) a[i] = fma(-u[i], cj, a[i]);
    __builtin_amdgcn_wave_barrier();
    if (lane < NH) row[lane] = lane >= k ? a[k] * inv : (T)0;  // L[lane][k]
    keep_col(a);
    __builtin_amdgcn_wave_barrier();
  }
  return ok;
}

// Forward L w = b, backward L^T d = w; lane i holds b_i and gets w_i, d_i.
// The forward sweep reads L[lane][k] from Lm; the backward sweep uses lane j's
// a[i] = L[i][j] L[j][j] (i > j) left by wave_chol.
template <typename T>
__device__ __forceinline__ void wave_solve(const T (&a)[NH], const T* Lm, T dinv, int lane, T b,
                                           T& w, T& d) {
  const T inv = dinv;
  T acc = b;
  w = 0;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const T wk = rl(acc * inv, k);
    if (lane == k) w = wk;
    if (lane > k && lane < NH) acc = fma(-Lm[k * LST + lane], wk, acc);
  }
  T acc2 = w;
  d = 0;
#pragma unroll
  for (int i = NH - 1; i >= 0; --i) {
    const T di = rl(acc2 * inv, i);
    if (lane == i) d = di;
    if (lane < i) acc2 = fma(-a[i] * inv, di, acc2);
  }
}

// Column `lane` of H = S/s00 - E E^T (i, j >= 1), plus lam on the diagonal.
template <typename T>
__device__ __forceinline__ void load_hcol(const float* Sc, T inv0, const T* E, int lane, T lam,
                                          T (&a)[NH]) {
  const int j = lane < NH ? lane : 0;
  const T ej = E[j + 1];
  // column pair_col(min + 1, max + 1) of S: row i + 1 of the pair triangle at
  // column j + 1 for i < j, row j + 1 at column i + 1 for i >= j; both are a
  // row's diagonal entry plus an offset, so the index is one add and a select
  const int dj = pair_col(j + 1, j + 1) - j;
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int col = i < j ? pair_col(i + 1, i + 1) - i + j : dj + i;
    a[i] = (T)Sc[col] * inv0 - E[i + 1] * ej;
  }
  if (lam != (T)0) {  // uniform: only the shifted retries of Alg. 1
#pragma unroll
    for (int i = 0; i < NH; ++i) a[i] += i == j ? lam : (T)0;
  }
}

constexpr int DIR_WAVES = 4;  // cells (waves) per workgroup of the wave-per-cell kernels

// Newton direction, two cells per wavefront: lanes 32h .. 32h + 31 serve cell
// h of the pair.  Lane j holds column j < 32 of the 34 x 34 matrix over all
// 34 rows, and the right-hand side as row 34; the block of columns 32, 33 that
// no lane holds is tracked as three scalars (its off-diagonal rows are rows
// 32, 33 of the lanes' columns).  The factorisation is H = L D L^T,
// right-looking and free of square roots: step k writes column k of the
// current matrix, pivot d_k included, to LDS; the lanes read it back with
// broadcast reads and subtract A[i][k] A[j][k] / d_k from their columns.
// Eliminating the right-hand-side row is the forward substitution L z = b,
// so afterwards lane j holds z_j and the Newton decrement is
// 1/2 sum z_k^2 / d_k; the backward sweep L^T delta = D^-1 z uses each lane's
// own frozen column entries A[m][j] (m > j).
constexpr int HROWS = 32;  // columns held by lanes
constexpr int HST = 36;    // LDS row stride (16-byte rows): entries 0..31, 32, 33, rhs 34

__device__ __forceinline__ float half_max(float v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <int DW>  // wavefronts per workgroup (2 DW cells)
__global__ __launch_bounds__(64 * DW) void k_direction3(
    const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
    const float* __restrict__ S, const float* __restrict__ M, float* __restrict__ dbeta,
    float* __restrict__ gdot, float* __restrict__ alpha_w, int32_t* __restrict__ iters_w,
    uint32_t* __restrict__ status_w, float* __restrict__ resid_w,
    const float* __restrict__ Lval, float* __restrict__ rbest_w, int32_t* __restrict__ itbest_w,
    const float* __restrict__ beta, SolveParams p, int8_t* __restrict__ codes, DirOut o) {
  const int64_t count = *ctr;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int hf = lane >> 5, j = lane & 31;
  const int64_t slot0 = ((int64_t)blockIdx.x * DW + wv) * 2;
  if (slot0 >= count) return;  // whole wave
  const int64_t slot = slot0 + hf;
  const bool live = slot < count;  // an odd count leaves the second half a read-only copy
  const int64_t cell = list[live ? slot : slot0];
  // per cell: the S row, later the rows of the factor (union), plus 4 floats
  // that take the discarded extras write of the last row
  constexpr int CW = HROWS * HST + 4;
  static_assert(CW >= NCOL, "factor rows must cover the S row");
  __shared__ __align__(16) float sW[DW][2][CW];
  __shared__ float sE[DW][2][K3 + 1];
  float* W = sW[wv][hf];
  float* E = sE[wv][hf];
  auto stage_S = [&]() {
    const f4* src = reinterpret_cast<const f4*>(S + cell * NCOL);
    f4* dst = reinterpret_cast<f4*>(W);
#pragma unroll
    for (int i = 0; i < NCOL / 4 / 32; ++i) dst[j + 32 * i] = src[j + 32 * i];
  };
  stage_S();
  const float* Mc = M + cell * K3;
  const float nn = Mc[0];
  const float mj = Mc[j + 1], m32 = Mc[33], m33 = Mc[34];
  CellState cs;
  cs.it = iters_w[cell];
  cs.itbest = itbest_w[cell];
  cs.st = status_w[cell];
  cs.rbest = rbest_w[cell];
  cs.alpha = alpha_w[cell];
  cs.L = Lval[cell];
  {
    const float* bc = beta + cell * K3;
    const float bm = fmaxf(fabsf(bc[j + 1]), j < 2 ? fabsf(bc[33 + j]) : 0.f);
    cs.bmax = half_max(bm);
  }
  __builtin_amdgcn_wave_barrier();
  const float s00 = W[0];
  const float inv0 = 1.f / s00;
  E[j] = j == 0 ? 1.f : W[j] * inv0;
  if (j < 3) E[32 + j] = W[32 + j] * inv0;
  __builtin_amdgcn_wave_barrier();
  const float e33 = E[33], e34 = E[34];
  const float g = E[j + 1] - mj / nn;
  const float g32 = e33 - m32 / nn, g33 = e34 - m33 / nn;
  float r = half_max(fmaxf(fabsf(g), fmaxf(fabsf(g32), fabsf(g33))));
  if (!isfinite(s00) || !(s00 > 0.f)) r = NAN;

  float a[NH + 1];  // column j, rows 0..33; a[NH] = right-hand side
  float t00, t10, t11, b32, b33;
  auto load_h = [&](float lam) {
    // the column index and E's offset pass through an empty asm so that the
    // addresses and E values are not hoisted out of the retry loop below
    // (they would stay live across the whole factorisation)
    int jj = j, eo = 0;
    asm volatile("" : "+v"(jj), "+v"(eo));
    const float ej = E[eo + jj + 1];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
      const int lo = i < jj ? i : jj, hi = i < jj ? jj : i;
      a[i] = W[pair_col(lo + 1, hi + 1)] * inv0 - E[eo + i + 1] * ej + (i == jj ? lam : 0.f);
    }
    a[NH] = -g;
    t00 = W[pair_col(33, 33)] * inv0 - e33 * e33 + lam;
    t10 = W[pair_col(33, 34)] * inv0 - e33 * e34;
    t11 = W[pair_col(34, 34)] * inv0 - e34 * e34 + lam;
    b32 = -g32;
    b33 = -g33;
  };
  bool ok;
  float dmin, dmax, dj = 1.f;
  auto factor = [&]() {
    __builtin_amdgcn_wave_barrier();  // the S row is dead: its space takes the factor
    int jf = j;  // per-step lane tests stay inside the retry loop (see load_h)
    asm volatile("" : "+v"(jf));
    ok = true;
    dmin = FLT_MAX;
    dmax = 0.f;
#pragma unroll
    for (int k = 0; k < HROWS; ++k) {
      float* row = W + k * HST;
      row[jf] = a[k];
      // rows 32, 33 and the right-hand side of column k come from lane k; the
      // other lanes write theirs to entries 35..37 (row padding and the first
      // entries of row k + 1, which step k + 1 overwrites): no branch, so the
      // compiler keeps the update right-looking
      {
        float* dst = row + (jf == k ? 32 : 35);
        dst[0] = a[32];
        dst[1] = a[33];
        dst[2] = a[NH];
      }
      __builtin_amdgcn_wave_barrier();
      float u[HST];
      const f4* r4 = reinterpret_cast<const f4*>(row);
#pragma unroll
      for (int q = k / 4; q < HST / 4; ++q) {
        const f4 v = r4[q];
        u[4 * q] = v[0]; u[4 * q + 1] = v[1]; u[4 * q + 2] = v[2]; u[4 * q + 3] = v[3];
      }
      const float d = u[k];
      ok = ok && (d > 0.f) && isfinite(d);
      dmin = fminf(dmin, d);
      dmax = fmaxf(dmax, d);
      const float rd = __builtin_amdgcn_rcpf(d);
      if (jf == k) dj = d;
      const float cj = jf > k ? a[k] * rd : 0.f;
#pragma unroll
      for (int i = k + 1; i <= NH; ++i) a[i] = fmaf(-u[i], cj, a[i]);
      const float c32 = u[32] * rd, c33 = u[33] * rd;
      t00 = fmaf(-u[32], c32, t00);
      t10 = fmaf(-u[33], c32, t10);
      t11 = fmaf(-u[33], c33, t11);
      b32 = fmaf(-u[NH], c32, b32);
      b33 = fmaf(-u[NH], c33, b33);
      // materialise the running block here: left to itself the compiler defers
      // these short chains to their use and keeps every step's row alive
      asm volatile("" : "+v"(t00), "+v"(t10), "+v"(t11), "+v"(b32), "+v"(b33), "+v"(dj),
                   "+v"(dmin), "+v"(dmax));
      __builtin_amdgcn_wave_barrier();
    }
    // the last two pivots
    const float d33 = fmaf(-t10 / t00, t10, t11);
    ok = ok && (t00 > 0.f) && isfinite(t00) && (d33 > 0.f) && isfinite(d33);
    dmin = fminf(dmin, fminf(t00, d33));
    dmax = fmaxf(dmax, fmaxf(t00, d33));
  };
  // One copy of the factorisation: a cell whose factorisation fails (and that
  // does not go to the FP64 kernel) goes round again with H + lambda I (Alg. 1),
  // lambda = lambda0 lambda_mul^t for up to 40 retries.
  bool to_fp64 = false;
  uint32_t extra = 0;
  float lam = 0.f;
  for (int tries = 0;; ++tries) {
    load_h(lam);
    factor();
    if (tries == 0 && p.fp64_ratio > 0.f && (!ok || dmin < p.fp64_ratio * dmax)) {
      to_fp64 = isfinite(r);
      break;
    }
    if (ok || !isfinite(r) || tries >= 40) break;
    lam = tries == 0 ? p.lambda0 : lam * p.lambda_mul;
    extra |= MEM_ST_SHIFTED;
    stage_S();  // the factor overwrote the S row
    __builtin_amdgcn_wave_barrier();
  }
  // forward results: z_j on lane j, z_32, z_33; pivots dj, t00, d33
  const float l3332 = t10 / t00;
  const float d33 = fmaf(-l3332, t10, t11);
  const float z32 = b32, z33 = fmaf(-l3332, z32, b33);
  const float zj = a[NH];
  const float res = (ok && !to_fp64)
                        ? 0.5f * (half_sum(zj * zj / dj) + z32 * z32 / t00 + z33 * z33 / d33)
                        : 0.f;
  // backward: delta_m = (z_m - sum_{m' > m} A[m'][m] delta_m') / d_m, lane m's column
  const float dl33 = z33 / d33;
  const float dl32 = (z32 - t10 * dl33) / t00;
  float sacc = fmaf(a[32], dl32, a[33] * dl33);
  const float rdj = __builtin_amdgcn_rcpf(dj);
  float dout = 0.f;
#pragma unroll
  for (int m = HROWS - 1; m >= 0; --m) {
    const float v = (zj - sacc) * rdj;
    const float dA = rl(v, m), dB = rl(v, 32 + m);
    const float dm = hf ? dB : dA;
    if (j == m) dout = dm;
    sacc = fmaf(a[m], dm, sacc);
  }
  const unsigned long long bad = __ballot(!isfinite(dout));
  const bool dfin = ok && ((bad >> (32 * hf)) & 0xffffffffull) == 0ull && isfinite(dl32) &&
                    isfinite(dl33);
  // outcome of the slot, compacted into the lists by k_compact3
  int code = 0;
  if (j == 0 && live) {
    code = to_fp64 ? 3
                   : finish_cell(cell, r, res, dfin, extra, p, cs, gdot, iters_w, status_w,
                                 resid_w, rbest_w, itbest_w, o);
    codes[slot] = (int8_t)code;
  }
  code = __shfl(code, lane & 32);
  if (code == 1 && live) {
    float* db = dbeta + cell * 36;
    db[1 + j] = dout;
    if (j == 0) { db[0] = 0.f; db[33] = dl32; db[34] = dl33; }
  }
}

// First Newton pass in closed form for a cell whose beta is exactly the
// Maxwellian of its gauge (beta_(200) = beta_(020) = beta_(002) = -1/sqrt(2),
// every other beta_i, i >= 1, zero).  Then sigma_p = w_p: the expectations are
// Gauss--Hermite sums of polynomials of degree <= 8, exact for >= 5 points per
// axis, so E[phi_i] = delta_i0 and H = I (orthonormal statistics).  Hence
// G_i = -M_i/n, the Newton direction is dbeta_i = M_i/n and the decrement is
// 1/2 |G|^2.  The outcome goes through the bookkeeping of every other
// direction; cells of any other beta get code 3 (ordinary first assembly).
__global__ __launch_bounds__(256) void k_start3(
    const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
    const float* __restrict__ M, const float* __restrict__ beta, float* __restrict__ dbeta,
    float* __restrict__ gdot, const float* __restrict__ alpha_w, int32_t* __restrict__ iters_w,
    uint32_t* __restrict__ status_w, float* __restrict__ resid_w, const float* __restrict__ Lval,
    float* __restrict__ rbest_w, int32_t* __restrict__ itbest_w, SolveParams p,
    int8_t* __restrict__ codes, float* __restrict__ S, DirOut o) {
  const int64_t count = *ctr;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= count) return;
  const int64_t cell = list[slot];
  const float* b = beta + cell * K3;
  const float sq = -0.70710678118654752f;
  bool maxw = true;
#pragma unroll
  for (int k = 1; k < K3; ++k) {
    const bool square = k == bidx3(2, 0, 0) || k == bidx3(0, 2, 0) || k == bidx3(0, 0, 2);
    maxw = maxw && (b[k] == (square ? sq : 0.f));
  }
  if (!maxw) { codes[slot] = 3; return; }
  const float* Mc = M + cell * K3;
  const float nn = Mc[0];
  float r = 0.f, res = 0.f;
#pragma unroll
  for (int k = 1; k < K3; ++k) {
    const float gk = -(Mc[k] / nn);
    r = fmaxf(r, fabsf(gk));
    res = fmaf(gk, gk, res);
  }
  res *= 0.5f;
  if (!(nn > 0.f) || !isfinite(res)) r = NAN;
  CellState cs;
  cs.it = iters_w[cell];
  cs.itbest = itbest_w[cell];
  cs.st = status_w[cell];
  cs.rbest = rbest_w[cell];
  cs.alpha = alpha_w[cell];
  cs.L = Lval[cell];
  cs.bmax = 0.70710678118654752f;
  const int code = finish_cell(cell, r, res, true, 0u, p, cs, gdot, iters_w, status_w, resid_w,
                               rbest_w, itbest_w, o);
  if (code == 1) {
    float* db = dbeta + cell * 36;
    db[0] = 0.f;
#pragma unroll
    for (int k = 1; k < K3; ++k) db[k] = Mc[k] / nn;
  } else if (code == 2) {
    // a refinement candidate: the refinement's Newton correction reads the
    // cell's S row, here E[phi_i phi_j] = delta_ij exactly (the cell was never
    // assembled in this solve)
    float* Sc = S + cell * NCOL;
    for (int col = 0; col < NCOL; ++col) Sc[col] = 0.f;
    for (int k = 0; k < K3; ++k) Sc[pair_col(k, k)] = 1.f;
  }
  codes[slot] = (int8_t)code;
}

// Stream compaction of the per-slot outcomes of k_direction3 (0 finished,
// 1 live, 2 refinement candidate, 3 FP64 direction) into three cell lists,
// with one atomic per list and workgroup instead of one per cell.
__global__ __launch_bounds__(256) void k_compact3(
    const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
    const int8_t* __restrict__ codes, int32_t* l1, int32_t* c1, int32_t* l2, int32_t* c2,
    int32_t* l3, int32_t* c3) {
  const int64_t count = *ctr;
  if ((int64_t)blockIdx.x * 256 >= count) return;  // whole workgroup
  const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int code = slot < count ? (int)codes[slot] : 0;
  const int cell = slot < count ? list[slot] : 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ int cnt[3][4], base[3][4];
  unsigned long long m[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    m[q] = __ballot(code == q + 1);
    if (lane == 0) cnt[q][wv] = __popcll(m[q]);
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    int32_t* cq = q == 0 ? c1 : (q == 1 ? c2 : c3);
    int tot = 0, off[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) { off[w] = tot; tot += cnt[q][w]; }
    const int b = (tot > 0 && cq) ? atomicAdd(cq, tot) : 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) base[q][w] = b + off[w];
  }
  __syncthreads();
  if (code >= 1 && code <= 3) {
    const int q = code - 1;
    int32_t* lq = q == 0 ? l1 : (q == 1 ? l2 : l3);
    if (lq) {
      const unsigned long long below = lane ? (m[q] & ((1ull << lane) - 1ull)) : 0ull;
      lq[base[q][wv] + __popcll(below)] = cell;
    }
  }
}

// --------------------------------------------------------------------------
// Newton direction in FP64 for cells with a small FP32 pivot ratio
// --------------------------------------------------------------------------
// Same wave-per-cell scheme as k_direction3 with the Hessian formed and
// factorised in double precision (lambda*I shift of Alg. 1 if it still fails).
__global__ __launch_bounds__(256) void k_fallback3(
    const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
    const float* __restrict__ S, const float* __restrict__ M, float* __restrict__ dbeta,
    float* __restrict__ gdot, float* __restrict__ alpha_w, int32_t* __restrict__ iters_w,
    uint32_t* __restrict__ status_w, float* __restrict__ resid_w,
    const float* __restrict__ Lval, float* __restrict__ rbest_w, int32_t* __restrict__ itbest_w,
    const float* __restrict__ beta, SolveParams p, DirOut o) {
  const int64_t count = *ctr;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  __shared__ double sE[DIR_WAVES][K3 + 1];
  __shared__ __align__(16) double sL[DIR_WAVES][NH * LST];
  // persistent: few cells take this path, so a small grid strides over them
  for (int64_t slot = (int64_t)blockIdx.x * DIR_WAVES + wv; slot < count;
       slot += (int64_t)gridDim.x * DIR_WAVES) {
  const int64_t cell = list[slot];
  const float* Sc = S + cell * NCOL;
  const double inv0 = 1.0 / (double)Sc[0];
  double* E = sE[wv];
  if (lane < K3) E[lane] = lane == 0 ? 1.0 : (double)Sc[lane] * inv0;
  __builtin_amdgcn_wave_barrier();
  const float* Mc = M + cell * K3;
  const double nn = Mc[0];
  const double g = lane < NH ? E[lane + 1] - (double)Mc[lane + 1] / nn : 0.0;
  const CellState cs = load_state(cell, lane, iters_w, status_w, rbest_w, itbest_w, alpha_w, Lval,
                                  beta);
  const float r = wave_max((float)fabs(g));
  double a[NH], dinv, dmin, dmax;
  uint32_t extra = MEM_ST_FP64;
  double lam = 0.0;
  bool ok = false;
  for (int tries = 0; tries < 41 && !ok; ++tries) {
    // the lane index passes through an empty asm so that the gathers and lane
    // tests of the (rarely repeated) factorisation are not hoisted out of the
    // retry loop, where they would stay live across it
    int ln = lane;
    asm volatile("" : "+v"(ln));
    load_hcol(Sc, inv0, E, ln, lam, a);
    ok = wave_chol(a, dinv, ln, dmin, dmax, sL[wv]);
    if (!ok) {
      lam = tries == 0 ? (double)p.lambda0 : lam * (double)p.lambda_mul;
      extra |= MEM_ST_SHIFTED;
    }
  }
  double w = 0.0, d = 0.0;
  if (ok) wave_solve(a, sL[wv], dinv, lane, -g, w, d);
  const float res = (float)(0.5 * wave_sum(lane < NH ? w * w : 0.0));
  const bool dfin = ok && __all(lane >= NH || isfinite(d));
  int code = 0;
  if (lane == 0) {
    code = finish_cell(cell, r, res, dfin, extra, p, cs, gdot, iters_w, status_w, resid_w,
                       rbest_w, itbest_w, o);
    if (code == 1) o.next_list[atomicAdd(o.next_ctr, 1)] = (int)cell;
    if (code == 2 && o.done_list) o.done_list[atomicAdd(o.done_ctr, 1)] = (int)cell;
  }
  code = __shfl(code, 0);
  if (code == 1 && lane == 0) dbeta[cell * 36] = 0.f;
  if (code == 1 && lane < NH) dbeta[cell * 36 + 1 + lane] = (float)d;
  __builtin_amdgcn_wave_barrier();  // sE / sL are reused by the next cell
  }
}

// --------------------------------------------------------------------------
// Residual refinement in compensated FP32 arithmetic
// --------------------------------------------------------------------------
// FP32 rounding of the exponent e_p = log w~_p + sum_k beta_k phi_k(p) (terms
// that reach a few hundred and cancel) limits the moment residual the FP32
// Newton iteration can certify to ~1e-5.  For converged cells the residual is
// re-evaluated in double-float arithmetic: every product by TwoProduct (FMA),
// every sum by TwoSum, the accumulated errors carried in a second FP32 word
// (the compensated dot product "Dot2" of Ogita, Rump and Oishi); then one
// Newton correction uses the Hessian already assembled for the cell --
// classical iterative refinement, with FP32 operations only.
//
// The nodes are a tensor grid (x_i, x_j, x_l) and phi_(a,b,c) = h_a h_b h_c
// with h_a = He_a / sqrt(a!), so both the exponent and the moments factor axis
// by axis (sum factorisation):
//   U[i][b,c] = sum_a beta_abc h_a(x_i),  V[i][j][c] = sum_b U[i][b,c] h_b(x_j),
//   e(i,j,l)  = sum_c V[i][j][c] h_c(x_l) + lw_i + lw_j + lw_l - log Z,
//   P[i][j][c] = sum_l sigma(i,j,l) h_c(x_l),  R[i][b,c] = sum_j P[i][j][c] h_b(x_j),
//   E_abc = sum_i R[i][b,c] h_a(x_i),
// where lw is the one-dimensional log w~ (log w~ of a node is the sum over its
// three coordinates).  About 5 terms per node instead of 36 + 35.

// One 64-thread workgroup per cell.  t1 = one-dimensional tables, double-float:
// t1[a * n + k] = h_a(x_k) (a = 0..4), t1[5 * n + k] = lw_k.
// list / ctr may be null (cells 0 .. ncell - 1); racc and out_list may be
// null; G row stride gst (36 for the refinement workspace, K for callers).
// CPB cells per workgroup of NTH threads: (1, 256) for the latency of small
// launches, (1, 64) and (4, 576) for throughput -- four cells on nine waves give
// each of the 4 x 144 node pairs of a 12-point rule its own lane.
template <int CPB, int NTH>
__global__ __launch_bounds__(NTH) void k_accurate3(
    const float2* __restrict__ t1, int n, const int32_t* __restrict__ list,
    const int32_t* __restrict__ ctr, int64_t ncell, const float* __restrict__ M,
    const float* __restrict__ beta, const float* __restrict__ logZ, float* __restrict__ Gacc,
    int gst, float* __restrict__ racc, float tol, int32_t* out_list, int32_t* out_ctr) {
#pragma clang fp contract(off)
  const int64_t count = ctr ? (int64_t)(*ctr) : ncell;
  const int64_t slot0 = (int64_t)blockIdx.x * CPB;
  if (slot0 >= count) return;
  const int nc = (int)(count - slot0 < CPB ? count - slot0 : CPB);  // cells of this workgroup
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  auto sync = [] {
    if constexpr (NTH > 64) __syncthreads();
    else __builtin_amdgcn_wave_barrier();
  };
  __shared__ int64_t scell[CPB];
  if (tid < nc) scell[tid] = list ? (int64_t)list[slot0 + tid] : slot0 + tid;
  extern __shared__ float2 dyn[];
  // per cell: U (later R) [n][15] and V (later P) [n*n][5]; then the 1D tables
  const int per = n * NBC + n * n * 5;
  float2* sT = dyn + CPB * per;  // [6][n]
  auto sU = [&](int q) { return dyn + q * per; };
  auto sV = [&](int q) { return dyn + q * per + n * NBC; };
  for (int t = tid; t < 6 * n; t += NTH) sT[t] = t1[t];
  sync();
  auto H = [&](int a, int k) -> dfl { const float2 v = sT[a * n + k]; return {v.x, v.y}; };

  // U[i][b,c] = sum_a beta_abc h_a(x_i)
  const int nu = n * NBC;
  for (int t = tid; t < nc * nu; t += NTH) {
    const int q = t / nu, tt = t - q * nu;
    const int64_t cell = scell[q];
    const int i = tt / NBC, bc = tt % NBC;
    int m = 0;
    while (tri(m + 1) <= bc) ++m;
    const int c = bc - tri(m), b = m - c;
    dfl u = {0.f, 0.f};
    for (int a = 0; a <= 4 - m; ++a) {
      const int k = bidx3(a, b, c);
      const float bk = k == 0 ? 0.f : beta[cell * K3 + k];  // beta_0 enters as log Z
      df_acc1(u, bk, H(a, i));
    }
    sU(q)[tt] = make_float2(u.h, u.l);
  }
  sync();
  // V[i][j][c] = sum_b U[i][b,c] h_b(x_j)
  const int nv = n * n * 5;
  for (int t = tid; t < nc * nv; t += NTH) {
    const int q = t / nv, tt = t - q * nv;
    const int ij = tt / 5, c = tt % 5, i = ij / n, j = ij % n;
    const float2* U = sU(q);
    dfl v = {0.f, 0.f};
    for (int b = 0; b <= 4 - c; ++b) {
      const float2 u = U[i * NBC + tri(b + c) + c];
      df_acc(v, {u.x, u.y}, H(b, j));
    }
    sV(q)[tt] = make_float2(v.h, v.l);
  }
  sync();
  // exponent, sigma and P[i][j][c] = sum_l sigma h_c(x_l); thread <-> (cell, i, j)
  const int np = n * n;
  for (int t = tid; t < nc * np; t += NTH) {
    const int q = t / np, qq = t - q * np;
    const int i = qq / n, j = qq % n;
    float2* Vq = sV(q);
    const float lz = logZ[scell[q]];
    dfl V[5], P[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const float2 v = Vq[qq * 5 + c];
      V[c] = {v.x, v.y};
      P[c] = {0.f, 0.f};
    }
    dfl base = {-lz, 0.f};
    df_add(base, H(5, i));
    df_add(base, H(5, j));
    for (int l = 0; l < n; ++l) {
      dfl e = base;
      df_add(e, H(5, l));
#pragma unroll
      for (int c = 0; c < 5; ++c) df_acc(e, V[c], H(c, l));
      e = df_norm(e);
      if (e.h < -60.f) continue;  // weight below 1e-26: no measurable moment
      const float ex = expf(e.h);
      const float w = fmaf(ex, e.l, ex);
#pragma unroll
      for (int c = 0; c < 5; ++c) df_acc1(P[c], w, H(c, l));
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) Vq[qq * 5 + c] = make_float2(P[c].h, P[c].l);
  }
  sync();
  // R[i][b,c] = sum_j P[i][j][c] h_b(x_j)
  for (int t = tid; t < nc * nu; t += NTH) {
    const int q = t / nu, tt = t - q * nu;
    const int i = tt / NBC, bc = tt % NBC;
    int m = 0;
    while (tri(m + 1) <= bc) ++m;
    const int c = bc - tri(m), b = m - c;
    const float2* Pq = sV(q);
    dfl r = {0.f, 0.f};
    for (int j = 0; j < n; ++j) {
      const float2 pv = Pq[(i * n + j) * 5 + c];
      df_acc(r, {pv.x, pv.y}, H(b, j));
    }
    sU(q)[tt] = make_float2(r.h, r.l);
  }
  sync();
  // wave q finishes cell q: the quotients and the reduction
  const int q = tid >> 6;
  if (q >= nc) return;
  const int64_t cell = scell[q];
  const float2* R = sU(q);
  // E_abc = sum_i R[i][b,c] h_a(x_i) on lane k = bidx3(a, b, c)
  dfl E = {0.f, 0.f};
  if (lane < K3) {
    int t = 0;
    while ((t + 1) * (t + 2) * (t + 3) / 6 <= lane) ++t;
    const int rr = lane - t * (t + 1) * (t + 2) / 6;
    int m = 0;
    while (tri(m + 1) <= rr) ++m;
    const int c = rr - tri(m), b = m - c, a = t - m;
    for (int i = 0; i < n; ++i) {
      const float2 rv = R[i * NBC + tri(m) + c];
      df_acc(E, {rv.x, rv.y}, H(a, i));
    }
  }
  // G_k = E_k / E_0 - M_k / n without rounding either quotient to FP32 first:
  // each quotient is q1 + q2 with q2 from the exact remainder (fma)
  const float h0 = __shfl(E.h, 0), l0 = __shfl(E.l, 0);
  const float inv0 = 1.f / h0;
  const float nn = M[cell * K3];
  float g = 0.f;
  if (lane >= 1 && lane < K3) {
    const float e1 = E.h * inv0;
    const float e2 = (fmaf(-e1, h0, E.h) + (E.l - e1 * l0)) * inv0;
    const float mi = M[cell * K3 + lane];
    const float m1 = mi / nn;
    const float m2 = fmaf(-m1, nn, mi) / nn;
    g = (e1 - m1) + (e2 - m2);
  }
  if (lane < gst) Gacc[cell * gst + lane] = g;
  const float r = wave_max(fabsf(g));
  if (lane == 0) {
    if (racc) racc[cell] = r;
    if (out_list && !(r <= tol)) out_list[atomicAdd(out_ctr, 1)] = (int)cell;
  }
}

// One Newton correction with the accurate gradient and the FP32 Hessian of
// the cell's last assembly (wave per cell, as k_direction3).
// reset (may be null) is zeroed by the first thread: the counter the next
// residual pass appends to, which this kernel does not read.
__global__ __launch_bounds__(256) void k_refine3(
    const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
    const float* __restrict__ S, const float* __restrict__ Gacc, float* __restrict__ beta,
    int32_t* reset) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && reset) *reset = 0;
  const int64_t count = *ctr;
  const int lane = threadIdx.x & 63;
  const int64_t slot = (int64_t)blockIdx.x * DIR_WAVES + (threadIdx.x >> 6);
  if (slot >= count) return;
  const int64_t cell = list[slot];
  const float* Sc = S + cell * NCOL;
  const float inv0 = 1.f / Sc[0];
  __shared__ float sE[DIR_WAVES][K3 + 1];
  __shared__ __align__(16) float sL[DIR_WAVES][NH * LST];
  float* E = sE[threadIdx.x >> 6];
  if (lane < K3) E[lane] = lane == 0 ? 1.f : Sc[lane] * inv0;
  __builtin_amdgcn_wave_barrier();
  float a[NH], dinv, dmin, dmax;
  load_hcol(Sc, inv0, E, lane, 0.f, a);
  const bool ok = wave_chol(a, dinv, lane, dmin, dmax, sL[threadIdx.x >> 6]);
  if (!ok) return;
  const float g = lane < NH ? Gacc[cell * 36 + 1 + lane] : 0.f;
  float w, d;
  wave_solve(a, sL[threadIdx.x >> 6], dinv, lane, -g, w, d);
  if (__all(lane >= NH || isfinite(d)) && lane < NH) beta[cell * K3 + 1 + lane] += d;
}

// Final status and residual of refined cells.
__global__ void k_refine_final(const int32_t* __restrict__ list, const int32_t* __restrict__ ctr,
                               const float* __restrict__ racc, float tol_loose,
                               uint32_t* __restrict__ status_w, float* resid_out,
                               uint32_t* status_out) {
  const int64_t count = *ctr;
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= count) return;
  const int64_t cell = list[slot];
  const float r = racc[cell];
  uint32_t st = status_w[cell];
  if (!(r <= tol_loose)) st = (st & ~MEM_ST_CONVERGED) | MEM_ST_STAGNATED;
  status_w[cell] = st;
  if (resid_out) resid_out[cell] = r;
  if (status_out) status_out[cell] = st;
}

// --------------------------------------------------------------------------
// E and the covariance block from S (checking entry point)
// --------------------------------------------------------------------------
__global__ void k_unpack3(int64_t n, const float* __restrict__ S, float* E, float* H) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const float* Sc = S + c * NCOL;
  const float inv0 = 1.f / Sc[0];
  if (E)
    for (int k = 0; k < K3; ++k) E[c * K3 + k] = k == 0 ? Sc[0] * inv0 : Sc[k] * inv0;
  if (H)
    for (int i = 0; i < NH; ++i)
      for (int j = 0; j < NH; ++j) {
        const int a = min(i, j), b = max(i, j);
        H[(c * NH + i) * NH + j] = Sc[pair_col(a + 1, b + 1)] * inv0 - Sc[i + 1] * inv0 * Sc[j + 1] * inv0;
      }
}


// --------------------------------------------------------------------------
// Persistent Newton solve: one wavefront runs the whole of Alg. 1 for a cell
// --------------------------------------------------------------------------
// Each wave takes cells from a work queue (one atomic per cell) and iterates
// a cell until a stopping test of Alg. 1 ends it; a converged cell frees its
// wave for the next live one (convergence masking and re-compaction without a
// grid-wide barrier or a launch per Newton pass).  Every step is the one of the
// list-based kernels above: the stopping tests and book-keeping, the
// lambda-shifted Cholesky with the FP64 switch on the pivot ratio, the Armijo
// line search (a full step once full steps are being taken is tested from the
// next pass's own assembly, backtracking on the sum-factorised exponent), the
// closed-form first pass from the gauge Maxwellian.
//
// The Hessian assembly exploits the tensor grid (x_i, x_j, x_l) and the product
// basis phi_(abc) = h_a h_b h_c:
//   E[phi_(abc) phi_(a'b'c')] = sum_{i,j,l} sigma_ijl H_aa'(x_i) H_bb'(x_j) H_cc'(x_l)
// with H_pq = h_p h_q (15 unordered pairs p <= q <= 4), contracted one axis at a
// time (sum factorisation):
//   P1[i][cc'][j] = sum_l sigma_ijl H_cc'(x_l)                (n^3 * 15 FMA)
//   P2[bb'cc'][i] = sum_j P1[i][cc'][j] H_bb'(x_j)            (n^2 * 105 FMA)
//   T[aa'][bb'][cc'] = sum_i H_aa'(x_i) P2[bb'cc'][i]          (n * 484 FMA)
// for the 105 (bb', cc') and 484 (aa', bb', cc') combinations the 630 pair
// columns need: about 47 k FMA per cell and iteration at n = 12, against 1.09 M
// for the dense sigma . Psi product.  The kernel evaluates the last stage once
// per pair column (630 rather than 484 sums, but no gather pass), and lays P1
// and P2 out so that each sum reads contiguous float4 rows of LDS.

// Unordered pair (p, q) of one-dimensional Hermite indices (p, q <= 4): 0..14.
__host__ __device__ constexpr int up_idx(int p, int q) {
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  return lo * 5 - lo * (lo - 1) / 2 + (hi - lo);
}

constexpr int SF_NBC = 105;  // (bb', cc') combinations of the 630 pairs
constexpr int SF_NT = 484;   // (aa', bb', cc') combinations

struct SfTables {
  int8_t bcB[128], bcC[128];  // up-indices of each (bb', cc') combination
  int8_t tA[512];             // aa' of each triple
  int16_t tBC[512];           // its (bb', cc') combination
  int16_t colT[NCOL];         // triple of each pair column (-1: padding column)
  int nbc, nt;
};

// (a, b, c) of basis index k (inverse of bidx3).
__host__ __device__ constexpr void abc_of(int k, int& a, int& b, int& c) {
  int t = 0;
  while ((t + 1) * (t + 2) * (t + 3) / 6 <= k) ++t;
  const int rr = k - t * (t + 1) * (t + 2) / 6;
  int m = 0;
  while ((m + 1) * (m + 2) / 2 <= rr) ++m;
  c = rr - m * (m + 1) / 2;
  b = m - c;
  a = t - m;
}

constexpr SfTables make_sf_tables() {
  SfTables s{};
  int bc_of[225] = {};
  int tri_of[15 * 225] = {};
  for (int q = 0; q < 225; ++q) bc_of[q] = -1;
  for (int q = 0; q < 15 * 225; ++q) tri_of[q] = -1;
  s.nbc = 0;
  s.nt = 0;
  for (int col = 0; col < NCOL; ++col) s.colT[col] = -1;
  for (int i = 0; i < K3; ++i)
    for (int j = i; j < K3; ++j) {
      int a1 = 0, b1 = 0, c1 = 0, a2 = 0, b2 = 0, c2 = 0;
      abc_of(i, a1, b1, c1);
      abc_of(j, a2, b2, c2);
      const int A = up_idx(a1, a2), B = up_idx(b1, b2), C = up_idx(c1, c2);
      if (bc_of[B * 15 + C] < 0) {
        bc_of[B * 15 + C] = s.nbc;
        s.bcB[s.nbc] = (int8_t)B;
        s.bcC[s.nbc] = (int8_t)C;
        ++s.nbc;
      }
      const int q = bc_of[B * 15 + C];
      if (tri_of[A * 225 + B * 15 + C] < 0) {
        tri_of[A * 225 + B * 15 + C] = s.nt;
        s.tA[s.nt] = (int8_t)A;
        s.tBC[s.nt] = (int16_t)q;
        ++s.nt;
      }
      s.colT[pair_col(i, j)] = (int16_t)tri_of[A * 225 + B * 15 + C];
    }
  return s;
}
static_assert(make_sf_tables().nbc == SF_NBC && make_sf_tables().nt == SF_NT,
              "sum-factorisation table sizes");

// The same tables laid out per lane for the persistent kernel at n = 12, which
// runs the three stages on chunks of SF_XC nodes of the first axis; each lane
// reads its whole share with seven coalesced loads:
//   stage 2, element e = lane + 64 r of a chunk (e = bc * SF_XC + x, r < 7):
//     B | C << 4 in byte r & 3 of s2[r >> 2][lane];
//   stage 3, pair column col = lane + 64 r (r < 10): aa' | bc << 4 in half
//     r & 1 of s3[r >> 1][lane], 0xffff for the padding columns.
constexpr int SF_N = 12;
constexpr int SF_XC = 4;                            // first-axis nodes per chunk
constexpr int SF_R2 = (SF_NBC * SF_XC + 63) / 64;  // 7 rounds per chunk
constexpr int SF_R3 = NCOL / 64;                   // 10 rounds
struct SfLane {
  uint32_t s2[(SF_R2 + 3) / 4][64];
  uint32_t s3[(SF_R3 + 1) / 2][64];
};
constexpr SfLane make_sf_lane() {
  const SfTables t = make_sf_tables();
  SfLane s{};
  for (int r = 0; r < SF_R2; ++r)
    for (int ln = 0; ln < 64; ++ln) {
      const int e = ln + 64 * r;
      const uint32_t v = e < SF_NBC * SF_XC
          ? (uint32_t)t.bcB[e / SF_XC] | ((uint32_t)t.bcC[e / SF_XC] << 4) : 0u;
      s.s2[r >> 2][ln] |= v << (8 * (r & 3));
    }
  for (int r = 0; r < SF_R3; ++r)
    for (int ln = 0; ln < 64; ++ln) {
      const int tt = t.colT[ln + 64 * r];
      const uint32_t v = tt >= 0 ? (uint32_t)t.tA[tt] | ((uint32_t)t.tBC[tt] << 4) : 0xffffu;
      s.s3[r >> 1][ln] |= v << (16 * (r & 1));
    }
  return s;
}
__constant__ SfLane c_sfl = make_sf_lane();

// V[q][c] = sum_{a+b+c<=4} b_abc h_a(x_i) h_b(x_j) for every node pair q = (i, j):
// the per-pair coefficients of the sum-factorised exponent (as in k_lse3).
template <int NT>
__device__ __forceinline__ void build_v(const float* sB, const float* sH, float* sV, int lane) {
  float bb[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) bb[k] = sB[k];
#pragma unroll 1
  for (int q = lane; q < NT * NT; q += 64) {
    const int i = q / NT, j = q - (q / NT) * NT;
    float ha[5], hb[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) { ha[a] = sH[a * NT + i]; hb[a] = sH[a * NT + j]; }
    float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 5; ++a) {
#pragma unroll
      for (int b = 0; a + b < 5; ++b) {
        const float pab = ha[a] * hb[b];
#pragma unroll
        for (int c = 0; a + b + c < 5; ++c) v[c] = fmaf(bb[bidx3(a, b, c)], pab, v[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) sV[q * 5 + c] = v[c];
  }
}

// Log-sum-exp of the exponent with coefficients sVb + alpha sVd over all nodes.
template <bool LS, int NT>
__device__ __forceinline__ float wave_lse(int lane, float alpha, const float* sH, const float* sVb,
                                          const float* sVd) {
  float mx = -FLT_MAX, sm = 0.f;
  int z = 0;
  asm volatile("" : "+v"(z));  // keep the table loads inside the pass (see the assembly)
  lse_pairs<LS, NT>(NT, lane, alpha, sH + z, sVb, sVd, mx, sm);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float om = __shfl_xor(mx, off), os = __shfl_xor(sm, off);
    const float nm = fmaxf(mx, om);
    sm = sm * __expf(mx - nm) + os * __expf(om - nm);
    mx = nm;
  }
  return mx + __logf(sm);
}

// Stopping tests and book-keeping of Alg. 1, as finish_cell, on the wave's
// register copy of the cell's state.  Returns 1 (live), 2 (refinement
// candidate) or 0 (finished).
__device__ __forceinline__ int wave_finish(float r, float res, bool dir_ok, uint32_t extra,
                                           const SolveParams& p, CellState& cs) {
  const int it = cs.it + 1;
  cs.it = it;
  uint32_t st = cs.st | extra;
  if (r < 0.5f * cs.rbest) { cs.rbest = r; cs.itbest = it; }
  const bool conv = (r <= p.tol_grad) || (res <= p.tol_dec && r <= p.tol_loose);
  const bool near = r <= STALL_GATE && p.refine > 0;
  const bool stall = near && (it - cs.itbest >= STALL_WINDOW || cs.alpha <= p.alpha_min ||
                              it >= p.max_iter);
  bool done = true, cand = false;
  if (conv || stall) { st |= MEM_ST_CONVERGED; cand = p.refine > 0; }
  else if (cs.L < p.lmin || (p.beta_max > 0.f && cs.bmax > p.beta_max))
    st |= MEM_ST_NONREALIZABLE;
  else if (!isfinite(r) || !dir_ok) st |= MEM_ST_NONFINITE;
  else if (cs.alpha <= p.alpha_min || it - cs.itbest >= NOPROGRESS_WINDOW)
    st |= MEM_ST_STAGNATED;
  else if (it >= p.max_iter) st |= MEM_ST_MAXITER;
  else done = false;
  cs.st = st;
  return done ? (cand ? 2 : 0) : 1;
}

// Wave-uniform copies (scalar registers).  Every value that decides control
// flow in k_newton_wave goes through these: the compiler cannot see that a
// cross-lane broadcast or reduction is equal on all lanes, and a branch on a
// vector register is compiled as divergent; lanes could then run different
// queue iterations, where a broadcast from a masked-off lane is undefined.
__device__ __forceinline__ float uf(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int ui(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Uniform minimum and maximum over the wave (butterfly, then lane 0's value in
// scalar registers).
template <typename T>
__device__ __forceinline__ T wave_min_u(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const T o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return rl(v, 0);
}
template <typename T>
__device__ __forceinline__ T wave_max_u(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const T o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return rl(v, 0);
}

// Right-looking Cholesky (as wave_chol) with the rows in registers only: lane
// i holds row i of A, and step k broadcasts row k from lane k with readlane
// (scalar registers), so no LDS round trip sits in the chain from one pivot to
// the next.  Afterwards lane i keeps a[k] = L[i][k] L[k][k] for k < i (frozen
// at step k) and lane k keeps dinv = 1 / L[k][k].  Each step only parks its
// pivot on lane k: the test of the pivots, their range and the reciprocal
// roots are taken once after the last step, so no branch or bookkeeping sits
// in the chain from one pivot to the next.  A pivot that is not positive and
// finite leaves NaN or infinite values behind it in the registers; the test
// after the last step still finds that pivot on its lane and reports the
// factorisation as failed.
template <typename T>
__device__ __forceinline__ bool wave_chol_rl(T (&a)[NH], T& dinv, int lane, T& dmin, T& dmax) {
  T dk = 1;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const T d = rl(a[k], k);
    if (lane == k) dk = d;
    // the mask is applied to a[k] (ready with the pivot), so only the
    // reciprocal's products sit between one pivot and the next
    const T ak = lane > k ? a[k] : (T)0;
    const T cj = ak * rcp(d);
#pragma unroll
    for (int i = k + 1; i < NH; ++i) a[i] = fma(-rl(a[i], k), cj, a[i]);
  }
  const bool ok = __all(lane >= NH || ((dk > (T)0) && isfinite(dk)));
  dinv = lane < NH ? rsq(dk) : (T)1;
  dmin = ok ? wave_min_u(lane < NH ? dk : (T)FLT_MAX) : (T)0;
  dmax = ok ? wave_max_u(lane < NH ? dk : (T)0) : (T)0;
  return ok;
}

// Forward L w = b and backward L^T d = w on the registers wave_chol_rl leaves:
// lane i holds b_i and gets w_i, d_i.  Lane k's running sum is final once
// step k has read it (later steps update only the lanes below or above it), so
// w and d are scaled on every lane at once after each sweep.
template <typename T>
__device__ __forceinline__ void wave_solve_rl(const T (&a)[NH], T dinv, int lane, T b, T& w,
                                              T& d) {
  // Each step's coefficient carries both reciprocal roots, so the chain from
  // one lane's running sum to the next is a broadcast and one FMA.
  T acc = b;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const T ik = rl(dinv, k);
    const T ck = (lane > k && lane < NH) ? a[k] * (ik * ik) : (T)0;
    acc = fma(-ck, rl(acc, k), acc);
  }
  w = lane < NH ? acc * dinv : (T)0;
  T acc2 = w;
#pragma unroll
  for (int i = NH - 1; i >= 0; --i) {
    const T ii = rl(dinv, i);
    const T ci = lane < i ? a[i] * (dinv * ii) : (T)0;
    acc2 = fma(-ci, rl(acc2, i), acc2);
  }
  d = lane < NH ? acc2 * dinv : (T)0;
}

// LDS of one wave (floats).  W holds one chunk of P1 and of P2 during the
// assembly, then the S row, E in FP32 and, for the FP64 direction, E in FP64.
// sVd holds the line search's direction coefficients.  About 12.5 KB at
// n = 12: three waves per SIMD fit in the 160 KB of a CU.
template <int NT>
struct WaveLds {
  static constexpr int NP = NT * NT;
  static constexpr int W32 = NCOL + 36 + 2 * 36;           // S, E (FP32 and FP64)
  static constexpr int P1C = SF_XC * 15 * NT;               // P1 of a chunk
  static constexpr int WP = P1C + SF_NBC * SF_XC;           // P1 and P2 of a chunk
  static constexpr int WN = WP > W32 ? WP : W32;
  __align__(16) float sH[6 * NT];
  __align__(16) float sHp[15 * NT];
  __align__(16) float sHpT[NT * 16];  // sHp by node: 15 products and a pad per row
  __align__(16) float sHT[NT * 8];     // h_0..h_4 and log w~ by node, two pads per row
  __align__(16) float sB[72];
  __align__(16) float sVb[NP * 5];
  __align__(16) float sVd[NP * 5];
  __align__(16) float W[(WN + 3) / 4 * 4];
};

template <int NT>
__global__ __launch_bounds__(64, 3) void k_newton_wave(
    const float2* __restrict__ t1, int32_t* __restrict__ queue, int64_t ncell,
    const float* __restrict__ M, float* __restrict__ beta, SolveParams p, int closed_start,
    float* __restrict__ S_w, float* __restrict__ logZ_w, int32_t* __restrict__ iters_w,
    uint32_t* __restrict__ status_w, float* __restrict__ resid_w, DirOut o) {
  constexpr int NP = NT * NT;
  static_assert(NT == SF_N, "the per-lane assembly tables are laid out for 12 nodes per axis");
  static_assert(SF_XC == 4 && NT % SF_XC == 0, "chunks of four nodes, read as float4");
  __shared__ WaveLds<NT> L;
  const int lane = threadIdx.x;
  for (int t = lane; t < 6 * NT; t += 64) L.sH[t] = t1[t].x;
  __builtin_amdgcn_wave_barrier();
  for (int t = lane; t < 15 * NT; t += 64) {
    const int pq = t / NT, k = t - (t / NT) * NT;
    int pp = 0;
    while (up_idx(pp, 4) < pq) ++pp;  // pq = up_idx(pp, qq) with qq >= pp
    const int qq = pp + (pq - up_idx(pp, pp));
    L.sHp[t] = L.sH[pp * NT + k] * L.sH[qq * NT + k];
    L.sHpT[k * 16 + pq] = L.sHp[t];
  }
  for (int t = lane; t < NT; t += 64) L.sHpT[t * 16 + 15] = 0.f;
  for (int t = lane; t < NT * 8; t += 64) {
    const int k = t >> 3, c = t & 7;
    L.sHT[t] = c < 6 ? L.sH[c * NT + k] : 0.f;
  }
  __builtin_amdgcn_wave_barrier();
  const float sq = -0.70710678118654752f;

  for (;;) {
    int got = 0;
    if (lane == 0) got = atomicAdd(queue, 1);
    const int slot = __builtin_amdgcn_readlane(got, 0);
    if ((int64_t)slot >= ncell) break;
    // o.next_list, when given, is the order of the cells (a permutation)
    const int64_t cell = o.next_list ? (int64_t)ui(o.next_list[slot]) : (int64_t)slot;
    const float* Mc = M + cell * K3;
    float* bc = beta + cell * K3;
    const bool kin = lane >= 1 && lane < K3;
    const float mraw = lane < K3 ? Mc[lane] : 0.f;
    float bk = kin ? bc[lane] : 0.f;
    const bool fin = lane >= K3 || (isfinite(mraw) && (lane == 0 || isfinite(bk)));
    const float nn = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mraw), 0));
    uint32_t st0 = 0;
    if (__ballot(!fin) != 0ull) st0 = MEM_ST_NONFINITE;
    else if (!(nn > 0.f)) st0 = MEM_ST_NONREALIZABLE;
    st0 = (uint32_t)ui((int)st0);
    // one latch for the queue loop (no continue): a rejected cell skips the
    // solve under a uniform branch and takes its status below
    if (st0 == 0u) {
    if (lane == 0) bc[0] = nn;
    const float mn = kin ? mraw / nn : 0.f;          // M_k / n on lane k
    // cross-lane reads with every lane active: M_{j+1} / n and M_{j+1} on lane j
    const float mnj = __shfl(mn, (lane + 1) & 63);
    const float mrj = __shfl(mraw, (lane + 1) & 63);
    // log Z and the dual value at the starting beta (k_lse3 without search)
    if (lane < 36) L.sB[lane] = bk;
    __builtin_amdgcn_wave_barrier();
    build_v<NT>(L.sB, L.sH, L.sVb, lane);
    __builtin_amdgcn_wave_barrier();
    float lz = uf(wave_lse<false, NT>(lane, 0.f, L.sH, L.sVb, L.sVd));
    CellState cs;
    cs.it = 0; cs.itbest = 0; cs.st = 0; cs.rbest = INFINITY; cs.alpha = 1.f;
    cs.L = uf(lz - wave_sum(bk * mn));
    bool maxw = false;
    if (closed_start) {
      const bool square = lane == bidx3(2, 0, 0) || lane == bidx3(0, 2, 0) || lane == bidx3(0, 0, 2);
      maxw = __ballot(kin && bk != (square ? sq : 0.f)) == 0ull;
    }
    float r = 0.f, res = 0.f;
    int code = 1;
    bool ident_S = false;  // closed-form pass: S is the identity (refinement reads it)
    // The full Newton step is tried by the next pass's own assembly: that
    // pass's sum of sigma gives log Z at the trial point, so accepting the
    // full step under the Armijo test needs no log-sum-exp pass of its own.
    // pending: sB holds the trial point bk + dkp; L0p and gdtp are the dual
    // value and the directional term of the step it was taken from.
    bool pending = false;
    float dkp = 0.f, L0p = 0.f, gdtp = 0.f;
    // backtracking line search of Alg. 1 from alpha = 1 along dv (k_lse3 with
    // the Armijo test); sVb must hold the exponent coefficients at bk
    auto backtrack = [&](float dv, float L0v, float gdtv) {
      if (lane < 36) L.sB[36 + lane] = lane < K3 ? dv : 0.f;
      __builtin_amdgcn_wave_barrier();
      build_v<NT>(L.sB + 36, L.sH, L.sVd, lane);
      __builtin_amdgcn_wave_barrier();
      float alpha = 1.f;
      for (int s = 0;; ++s) {
        const float lzs = uf(wave_lse<true, NT>(lane, alpha, L.sH, L.sVb, L.sVd));
        const float bs = fmaf(alpha, dv, bk);
        const float Ls = uf(lzs - wave_sum(bs * mn));
        const float LD = L0v - Ls;
        const float gradD = -p.c * alpha * gdtv;
        const bool sat = (LD - gradD) >= -(p.atol + p.rtol * fabsf(LD));
        const bool last = sat || s >= p.max_ls;
        bk = (last && kin) ? bs : bk;
        if (last) {
          lz = lzs;
          cs.L = Ls;
          cs.alpha = alpha;
          break;
        }
        alpha *= 0.5f;
      }
    };
    for (;;) {
      float dk = 0.f;  // direction on lane k (beta_k), k >= 1
      uint32_t extra = 0;
      bool dfin = true;
      cs.bmax = uf(wave_max(kin ? fabsf(bk) : 0.f));
      if (cs.it == 0 && maxw) {
        // closed-form first pass from the gauge Maxwellian: H = I, G = -M/n
        const float gk = kin ? -mn : 0.f;
        r = uf(wave_max(fabsf(gk)));
        res = uf(0.5f * wave_sum(gk * gk));
        if (!(nn > 0.f) || !isfinite(res)) r = NAN;
        cs.bmax = 0.70710678118654752f;
        dk = mn;
        ident_S = true;
      } else {
        ident_S = false;
        // the exponent coefficients at the current beta, or at the trial point
        if (!pending && lane < 36) L.sB[lane] = bk;
        __builtin_amdgcn_wave_barrier();
        build_v<NT>(L.sB, L.sH, L.sVb, lane);
        __builtin_amdgcn_wave_barrier();
        // this lane's share of the stage-2 and stage-3 index tables (loaded
        // here, behind an opaque offset, so that they are not held in
        // registers across the direction solve)
        uint32_t s2p[(SF_R2 + 3) / 4], s3p[(SF_R3 + 1) / 2];
        {
          int z = lane;
          asm volatile("" : "+v"(z));
#pragma unroll
          for (int k = 0; k < (SF_R2 + 3) / 4; ++k) s2p[k] = c_sfl.s2[k][z];
#pragma unroll
          for (int k = 0; k < (SF_R3 + 1) / 2; ++k) s3p[k] = c_sfl.s3[k][z];
        }
        // the three stages on chunks of SF_XC first-axis nodes; the pair
        // columns accumulate in registers across the chunks
        float* P1 = L.W;                          // P1[i][pq][j], i in the chunk
        float* P2 = L.W + WaveLds<NT>::P1C;       // P2[bc][i], i in the chunk
        float tcol[SF_R3];
#pragma unroll
        for (int r = 0; r < SF_R3; ++r) tcol[r] = 0.f;
#pragma unroll 1
        for (int x0 = 0; x0 < NT; x0 += SF_XC) {
          // stage 1: sigma and P1[i][pq][j] = sum_l sigma(i, j, l) H_pq(x_l)
          if (lane < SF_XC * NT) {
            // the tables never change, so without an opaque offset the
            // compiler keeps all 252 of them in registers across the kernel
            int z = 0;
            asm volatile("" : "+v"(z));
            const float* sh = L.sH + z;
            const float* sht = L.sHT + z;
            const float* shpt = L.sHpT + z;
            const int il = lane / NT, j = lane - (lane / NT) * NT;
            const int q = (x0 + il) * NT + j;
            const float base = sh[5 * NT + x0 + il] + sh[5 * NT + j];
            float v[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) v[c] = L.sVb[q * 5 + c];
            float acc[15];
#pragma unroll
            for (int t = 0; t < 15; ++t) acc[t] = 0.f;
#pragma unroll
            for (int l = 0; l < NT; ++l) {
              // node l's basis values and log weight as two 16-byte reads
              const float4* hn = reinterpret_cast<const float4*>(sht + l * 8);
              const float4 h03 = hn[0], h47 = hn[1];
              const float hb[6] = {h03.x, h03.y, h03.z, h03.w, h47.x, h47.y};
              float x = base + hb[5];
#pragma unroll
              for (int c = 0; c < 5; ++c) x = fmaf(v[c], hb[c], x);
              const float sg = __expf(x - lz);
              // node l's 15 products as four 16-byte reads
              const float4* hq = reinterpret_cast<const float4*>(shpt + l * 16);
              float hp[16];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const float4 h4 = hq[u];
                hp[4 * u] = h4.x; hp[4 * u + 1] = h4.y; hp[4 * u + 2] = h4.z; hp[4 * u + 3] = h4.w;
              }
#pragma unroll
              for (int t = 0; t < 15; ++t) acc[t] = fmaf(sg, hp[t], acc[t]);
            }
#pragma unroll
            for (int t = 0; t < 15; ++t) P1[(il * 15 + t) * NT + j] = acc[t];
          }
          __builtin_amdgcn_wave_barrier();
          // stage 2: P2[bc][i] = sum_j P1[i][C][j] H_B(x_j)
#pragma unroll
          for (int r = 0; r < SF_R2; ++r) {
            const int e = lane + 64 * r;
            if (r + 1 < SF_R2 || e < SF_NBC * SF_XC) {
              const uint32_t v = (s2p[r >> 2] >> (8 * (r & 3))) & 0xffu;
              const int B = (int)(v & 15u), C = (int)(v >> 4);
              const int il = e & (SF_XC - 1);
              const float4* a4 = reinterpret_cast<const float4*>(P1 + (il * 15 + C) * NT);
              const float4* h4 = reinterpret_cast<const float4*>(L.sHp + B * NT);
              float acc = 0.f;
#pragma unroll
              for (int k = 0; k < NT / 4; ++k) {
                const float4 a = a4[k], h = h4[k];
                acc = fmaf(a.x, h.x, acc);
                acc = fmaf(a.y, h.y, acc);
                acc = fmaf(a.z, h.z, acc);
                acc = fmaf(a.w, h.w, acc);
              }
              P2[e] = acc;
            }
          }
          __builtin_amdgcn_wave_barrier();
          // stage 3: pair column col of triple (aa', bc) gains
          // sum_{i in chunk} H_aa'(x_i) P2[bc][i].  A column that is no pair
          // (entry 0xffff) reads entry 0 and is zeroed after the last chunk, so
          // the loop has no divergent branch and its loads can all be issued
          // ahead of the FMAs.
#pragma unroll
          for (int r = 0; r < SF_R3; ++r) {
            const uint32_t v0 = (s3p[r >> 1] >> (16 * (r & 1))) & 0xffffu;
            const uint32_t v = v0 == 0xffffu ? 0u : v0;
            const int A = (int)(v & 15u), bc = (int)(v >> 4);
            const float4 h = *reinterpret_cast<const float4*>(L.sHp + A * NT + x0);
            const float4 b = *reinterpret_cast<const float4*>(P2 + bc * SF_XC);
            float acc = tcol[r];
            acc = fmaf(h.x, b.x, acc);
            acc = fmaf(h.y, b.y, acc);
            acc = fmaf(h.z, b.z, acc);
            acc = fmaf(h.w, b.w, acc);
            tcol[r] = acc;
          }
          __builtin_amdgcn_wave_barrier();
        }
        // the S row over the dead chunk buffers
        float* Sr = L.W;
#pragma unroll
        for (int r = 0; r < SF_R3; ++r) {
          const uint32_t v0 = (s3p[r >> 1] >> (16 * (r & 1))) & 0xffffu;
          Sr[lane + 64 * r] = v0 == 0xffffu ? 0.f : tcol[r];
        }
        __builtin_amdgcn_wave_barrier();
        // gradient, residual and Newton direction (k_direction3 / k_fallback3)
        const float s00 = uf(Sr[0]);
        if (pending) {
          // Armijo test of the full step from this assembly: the sum of sigma,
          // shifted by the old log Z, is exp of the change of log Z.  Outside a
          // range of e^(+-20) (or if the test fails) the step goes through the
          // backtracking search of Alg. 1 from alpha = 1, and the accepted
          // point is assembled afresh.
          pending = false;
          const float bt = fmaf(1.f, dkp, bk);
          bool accept = false;
          float lzt = 0.f, Lt = 0.f;
          if (isfinite(s00) && s00 > 2e-9f && s00 < 5e8f) {
            lzt = lz + __logf(s00);
            Lt = uf(lzt - wave_sum(bt * mn));
            const float LD = L0p - Lt;
            const float gradD = -p.c * gdtp;
            accept = (LD - gradD) >= -(p.atol + p.rtol * fabsf(LD)) || p.max_ls <= 0;
          }
          if (!accept) {
            if (lane < 36) L.sB[lane] = bk;
            __builtin_amdgcn_wave_barrier();
            build_v<NT>(L.sB, L.sH, L.sVb, lane);
            backtrack(dkp, L0p, gdtp);
            continue;  // assemble at the accepted point
          }
          bk = kin ? bt : bk;
          lz = lzt;
          cs.L = Lt;
          cs.alpha = 1.f;
          cs.bmax = uf(wave_max(kin ? fabsf(bk) : 0.f));
        }
        const float inv0 = 1.f / s00;
        float* E = L.W + NCOL;
        if (lane < K3) E[lane] = lane == 0 ? 1.f : Sr[lane] * inv0;
        __builtin_amdgcn_wave_barrier();
        const float g = lane < NH ? E[lane + 1] - mnj : 0.f;
        r = uf(wave_max(fabsf(g)));
        if (!isfinite(s00) || !(s00 > 0.f)) r = NAN;
        float a[NH], dinv = 1.f, dmin = 0.f, dmax = 0.f;
        bool ok = false, to64 = false;
        float lam = 0.f;
        for (int tries = 0;; ++tries) {
          int ln = lane;
          asm volatile("" : "+v"(ln));
          load_hcol(Sr, inv0, E, ln, lam, a);
          ok = wave_chol_rl(a, dinv, ln, dmin, dmax);
          if (tries == 0 && p.fp64_ratio > 0.f && (!ok || dmin < p.fp64_ratio * dmax)) {
            to64 = isfinite(r);
            break;
          }
          if (ok || !isfinite(r) || tries >= 40) break;
          lam = tries == 0 ? p.lambda0 : lam * p.lambda_mul;
          extra |= MEM_ST_SHIFTED;
        }
        if (!to64) {
          float w = 0.f, d = 0.f;
          if (ok) wave_solve_rl(a, dinv, lane, -g, w, d);
          res = ok ? uf(0.5f * wave_sum(lane < NH ? w * w : 0.f)) : 0.f;
          dfin = ok && __all(lane >= NH || isfinite(d));
          dk = __shfl(d, (lane + 63) & 63);
        } else {
          // FP64 direction: E in double after the FP32 E; the factor stays in
          // registers
          double* Ed = reinterpret_cast<double*>(L.W + NCOL + 36);
          const double inv0d = 1.0 / (double)s00;
          if (lane < K3) Ed[lane] = lane == 0 ? 1.0 : (double)Sr[lane] * inv0d;
          __builtin_amdgcn_wave_barrier();
          const double gd = lane < NH ? Ed[lane + 1] - (double)mrj / (double)nn : 0.0;
          r = uf(wave_max((float)fabs(gd)));
          double ad[NH], dinvd = 1.0, dmind = 0.0, dmaxd = 0.0;
          double lamd = 0.0;
          bool okd = false;
          extra = MEM_ST_FP64;
          for (int tries = 0; tries < 41 && !okd; ++tries) {
            int ln = lane;
            asm volatile("" : "+v"(ln));
            load_hcol(Sr, inv0d, Ed, ln, lamd, ad);
            okd = wave_chol_rl(ad, dinvd, ln, dmind, dmaxd);
            if (!okd) {
              lamd = tries == 0 ? (double)p.lambda0 : lamd * (double)p.lambda_mul;
              extra |= MEM_ST_SHIFTED;
            }
          }
          double w = 0.0, d = 0.0;
          if (okd) wave_solve_rl(ad, dinvd, lane, -gd, w, d);
          res = uf((float)(0.5 * wave_sum(lane < NH ? w * w : 0.0)));
          dfin = okd && __all(lane >= NH || isfinite(d));
          dk = (float)__shfl(d, (lane + 63) & 63);
        }
        dk = kin ? dk : 0.f;
      }
      code = wave_finish(r, res, dfin, extra, p, cs);
      if (code != 1) break;
      if (cs.it >= 2 && cs.alpha == 1.f) {
        // full steps are being taken: try this one by the next pass
        dkp = dk;
        L0p = cs.L;
        gdtp = -2.f * res;
        if (lane < 36) L.sB[lane] = fmaf(1.f, dk, bk);
        pending = true;
      } else {
        backtrack(dk, cs.L, -2.f * res);
      }
    }
    // results of the cell
    if (kin) bc[lane] = bk;
    if (code == 2) {
      float* Sg = S_w + cell * NCOL;
      if (ident_S) {
        // E[phi_i phi_j] = delta_ij: every column written once, by one lane
        for (int col = lane; col < NCOL; col += 64) {
          bool diag = false;
          for (int k = 0; k < K3; ++k) diag = diag || (col == pair_col(k, k));
          Sg[col] = diag ? 1.f : 0.f;
        }
      } else {
        for (int col = lane; col < NCOL; col += 64) Sg[col] = L.W[col];
      }
    }
    if (lane == 0) {
      iters_w[cell] = cs.it;
      status_w[cell] = cs.st;
      resid_w[cell] = r;
      logZ_w[cell] = lz;
      if (o.iters_out) o.iters_out[cell] = cs.it;
      if (o.resid_out) o.resid_out[cell] = r;
      if (o.status_out) o.status_out[cell] = cs.st;
      if (code == 2 && o.done_list) o.done_list[atomicAdd(o.done_ctr, 1)] = (int)cell;
    }
    }  // st0 == 0
    if (st0 != 0u && lane == 0) {
      iters_w[cell] = 0; status_w[cell] = st0; resid_w[cell] = INFINITY;
      if (o.iters_out) o.iters_out[cell] = 0;
      if (o.resid_out) o.resid_out[cell] = INFINITY;
      if (o.status_out) o.status_out[cell] = st0;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_set_ctr(int32_t* ctr, int n, hipStream_t s) {
  k_set_ctr<<<1, 64, 0, s>>>(ctr, n);
  return hipGetLastError();
}

hipError_t launch_init3(mem_ctx_t c, int64_t n, const float* M, float* beta, int32_t* out_list,
                        int32_t* out_ctr, int32_t* iters, float* resid, uint32_t* status,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_init3<<<nblocks(n, 256), 256, 0, s>>>(n, M, beta, c->w_alpha, c->w_iters, c->w_status,
                                           c->w_resid, c->w_rbest, c->w_itbest, out_list, out_ctr,
                                           iters, resid, status);
  return hipGetLastError();
}

hipError_t launch_lse3(mem_ctx_t c, int64_t grid_cells, const int32_t* list, const int32_t* ctr,
                       int64_t n, const float* M, float* beta, bool line_search,
                       const SolveParams& p, int32_t* reset_a, int32_t* reset_b, hipStream_t s) {
  const unsigned nb = (unsigned)(grid_cells > 0 ? grid_cells : 1);
  const int n1 = c->n1d;
  const size_t lds = (size_t)(72 + 6 * n1 + 2 * n1 * n1 * 5) * sizeof(float);
#define MEM_LSE(LS, NT)                                                                         \
  k_lse3<LS, NT><<<nb, 64, lds, s>>>(c->d_t1, n1, list, ctr, n, M, beta, c->w_dbeta, c->w_logZ, \
                                     c->w_L, c->w_alpha, c->w_gdot, p, reset_a, reset_b)
  if (line_search) {
    if (n1 == 12) MEM_LSE(true, 12); else MEM_LSE(true, 0);
  } else {
    if (n1 == 12) MEM_LSE(false, 12); else MEM_LSE(false, 0);
  }
#undef MEM_LSE
  return hipGetLastError();
}

// Node-range splits for a launch of ntile tiles of tw cells: enough
// workgroups to fill the chip when few cells are live, at least 4 node groups
// per split, partial sums within the split buffer.
int assembly_splits(mem_ctx_t c, int ntile, int ngroups, int tw) {
  const int want = c->tune.split_want;  // workgroups
  if (want <= 0 || ntile >= want / 2 || !c->w_Sp) return 1;
  int ns = (want + ntile - 1) / ntile;
  ns = std::min(ns, std::max(1, ngroups / 4));
  while (ns > 1 && (int64_t)ns * ntile * tw > c->sp_rows) --ns;
  return ns;
}

hipError_t launch_sum_splits(mem_ctx_t c, const int32_t* list, const int32_t* ctr, int64_t n,
                             int64_t rows, int nsplit, float* S, hipStream_t s) {
  k_sum_splits<NCOL><<<(unsigned)nblocks(rows * (NCOL / 4), 256), 256, 0, s>>>(
      list, ctr, n, rows, nsplit, c->w_Sp, S);
  return hipGetLastError();
}

hipError_t launch_assemble3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                            const int32_t* ctr, int64_t n, const float* beta, const float* table,
                            float* S, hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  // cells per workgroup: 64 (four waves) or 128 (eight), a tuning parameter
  const int aw = c->tune.asm_waves == 8 ? 8 : 4;
  const int tw = 16 * aw;
  const int ntile = (int)nblocks(grid_cells, tw);
  const int nsplit = assembly_splits(c, ntile, c->ngroups, tw);
  const unsigned grid = (unsigned)(ntile * nsplit);
  if (aw == 8)
    k_assemble3<NBLK / 4, 8><<<grid, 512, 0, s>>>(c->d_phiA, table, c->ngroups, list, ctr, n,
                                                  beta, c->w_logZ, S, ntile, nsplit, c->w_Sp);
  else
    k_assemble3<NBLK / 4, 4><<<grid, 256, 0, s>>>(c->d_phiA, table, c->ngroups, list, ctr, n,
                                                  beta, c->w_logZ, S, ntile, nsplit, c->w_Sp);
  if (nsplit > 1) return launch_sum_splits(c, list, ctr, n, (int64_t)ntile * tw, nsplit, S, s);
  return hipGetLastError();
}

hipError_t launch_assemble5(mem_ctx_t c, int64_t n, const float* beta, const float* table,
                            float* S5, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int ntile = (int)nblocks(n, TILE);
  const int nsplit = assembly_splits(c, ntile, c->ngroups, TILE);
  k_assemble3<NC5 / 64, 4><<<(unsigned)(ntile * nsplit), 256, 0, s>>>(
      c->d_phiA, table, c->ngroups, nullptr, nullptr, n, beta, c->w_logZ, S5, ntile, nsplit,
      c->w_Sp);
  if (nsplit > 1)
    k_sum_splits<NC5><<<(unsigned)nblocks((int64_t)ntile * TILE * (NC5 / 4), 256), 256, 0, s>>>(
        nullptr, nullptr, n, (int64_t)ntile * TILE, nsplit, c->w_Sp, S5);
  return hipGetLastError();
}

hipError_t launch_start3(mem_ctx_t c, int64_t n, const int32_t* list, const int32_t* ctr,
                         const float* M, const float* beta, const SolveParams& p,
                         int32_t* next_list, int32_t* next_ctr, int32_t* asm_list, int32_t* asm_ctr,
                         int32_t* iters, float* resid, uint32_t* status, int32_t* done_list,
                         int32_t* done_ctr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  DirOut o{next_list, next_ctr, iters, resid, status, done_list, done_ctr};
  k_start3<<<nblocks(n, 256), 256, 0, s>>>(list, ctr, M, beta, c->w_dbeta, c->w_gdot, c->w_alpha,
                                           c->w_iters, c->w_status, c->w_resid, c->w_L,
                                           c->w_rbest, c->w_itbest, p, c->w_code, c->w_S, o);
  // 1: live with its direction, 2: converged (refinement), 3: first assembly
  k_compact3<<<nblocks(n, 256), 256, 0, s>>>(list, ctr, c->w_code, next_list, next_ctr, done_list,
                                             done_ctr, asm_list, asm_ctr);
  return hipGetLastError();
}

hipError_t launch_direction3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                             const int32_t* ctr, const float* M, const float* beta,
                             const SolveParams& p,
                             int32_t* next_list, int32_t* next_ctr, int32_t* fb_list,
                             int32_t* fb_ctr, int32_t* iters, float* resid, uint32_t* status,
                             int32_t* done_list, int32_t* done_ctr, hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  DirOut o{next_list, next_ctr, iters, resid, status, done_list, done_ctr};
#define MEM_DIR(DW)                                                                        \
  k_direction3<DW><<<nblocks(grid_cells, 2 * DW), 64 * DW, 0, s>>>(                       \
      list, ctr, c->w_S, M, c->w_dbeta, c->w_gdot, c->w_alpha, c->w_iters, c->w_status,   \
      c->w_resid, c->w_L, c->w_rbest, c->w_itbest, beta, p, c->w_code, o)
  switch (c->tune.dir_waves) {
    case 2: MEM_DIR(2); break;
    case 8: MEM_DIR(8); break;
    default: MEM_DIR(4); break;
  }
#undef MEM_DIR
  k_compact3<<<nblocks(grid_cells, 256), 256, 0, s>>>(list, ctr, c->w_code, next_list, next_ctr,
                                                      done_list, done_ctr, fb_list, fb_ctr);
  return hipGetLastError();
}

hipError_t launch_fallback3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                            const int32_t* ctr, const float* M, const float* beta,
                            const SolveParams& p,
                            int32_t* next_list, int32_t* next_ctr, int32_t* iters, float* resid,
                            uint32_t* status, int32_t* done_list, int32_t* done_ctr,
                            hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  DirOut o{next_list, next_ctr, iters, resid, status, done_list, done_ctr};
  k_fallback3<<<(unsigned)std::min<int64_t>(nblocks(grid_cells, DIR_WAVES), 256), 256, 0, s>>>(list, ctr, c->w_S, M, c->w_dbeta, c->w_gdot,
                                                     c->w_alpha, c->w_iters, c->w_status,
                                                     c->w_resid, c->w_L, c->w_rbest, c->w_itbest,
                                                     beta, p, o);
  return hipGetLastError();
}

// Below this many cells a launch runs four wavefronts per cell (one node pair
// per thread): the grid is too small to fill the chip, so latency decides.
constexpr int64_t ACC_WIDE_BELOW = 16384;

// Variant choice: one cell on four waves for small launches (latency), four
// cells on nine waves for large ones when the rule has 12 points (every lane of
// the exponent phase busy), one cell per wave otherwise.
static hipError_t accurate3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                            const int32_t* ctr, const float* M, const float* beta, float* G,
                            int gst, float* racc, float tol, int32_t* out_list, int32_t* out_ctr,
                            hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  const int n = c->n1d;
  const size_t per = (size_t)(n * NBC + n * n * 5) * sizeof(float2);
  const size_t tab = (size_t)6 * n * sizeof(float2);
  if (grid_cells < ACC_WIDE_BELOW)
    k_accurate3<1, 256><<<(unsigned)grid_cells, 256, per + tab, s>>>(
        c->d_t1, n, list, ctr, grid_cells, M, beta, c->w_logZ, G, gst, racc, tol, out_list, out_ctr);
  else if (n == 12)
    k_accurate3<4, 576><<<(unsigned)nblocks(grid_cells, 4), 576, 4 * per + tab, s>>>(
        c->d_t1, n, list, ctr, grid_cells, M, beta, c->w_logZ, G, gst, racc, tol, out_list, out_ctr);
  else
    k_accurate3<1, 64><<<(unsigned)grid_cells, 64, per + tab, s>>>(
        c->d_t1, n, list, ctr, grid_cells, M, beta, c->w_logZ, G, gst, racc, tol, out_list, out_ctr);
  return hipGetLastError();
}

hipError_t launch_accurate3(mem_ctx_t c, int64_t grid_cells, const int32_t* list, const int32_t* ctr,
                           const float* M, const float* beta, float tol, int32_t* out_list,
                           int32_t* out_ctr, hipStream_t s) {
  return accurate3(c, grid_cells, list, ctr, M, beta, c->w_Gacc, 36, c->w_racc, tol, out_list,
                   out_ctr, s);
}

hipError_t launch_moment_residual3(mem_ctx_t c, int64_t n, const float* M, const float* beta,
                                   float* G, hipStream_t s) {
  return accurate3(c, n, nullptr, nullptr, M, beta, G, K3, nullptr, 0.f, nullptr, nullptr, s);
}

hipError_t launch_refine3(mem_ctx_t c, int64_t grid_cells, const int32_t* list, const int32_t* ctr,
                          const float* M, float* beta, int32_t* reset, hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  k_refine3<<<nblocks(grid_cells, DIR_WAVES), 256, 0, s>>>(list, ctr, c->w_S, c->w_Gacc, beta,
                                                           reset);
  return hipGetLastError();
}

hipError_t launch_refine_final(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                               const int32_t* ctr, float tol_loose, float* resid,
                               uint32_t* status, hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  k_refine_final<<<nblocks(grid_cells, 256), 256, 0, s>>>(list, ctr, c->w_racc, tol_loose,
                                                          c->w_status, resid, status);
  return hipGetLastError();
}

// Persistent Newton solve of cells 0..n-1 (one wave per live cell); ctr[7] is
// the work queue (zeroed by the caller).
// Order in which the persistent kernel takes its cells.  A cell's Newton
// iterations grow with how far its normalised moments lie from the Maxwellian
// it starts from; taking the far ones first leaves short solves for the end
// of the queue, where the grid drains.  Counting sort on max_k |M_k| / M_0
// (k >= 1), two buckets per octave over [2^-8, 2^8), largest first; within a
// bucket the order is arbitrary (each cell's solve does not depend on it).
constexpr int ORD_NB = 32;
constexpr int ORD_TPB = 256;

__device__ __forceinline__ int order_bucket(const float* __restrict__ m) {
  float g = 0.f;
  for (int k = 1; k < K3; ++k) g = fmaxf(g, fabsf(m[k]));
  g = g / m[0];
  const float f = (g > 0.f && isfinite(g))
                      ? fminf(fmaxf(floorf(2.f * log2f(g)) + 16.f, 0.f), (float)(ORD_NB - 1))
                      : 0.f;
  return ORD_NB - 1 - (int)f;
}

__global__ void k_order_zero(int32_t* __restrict__ hist) {
  if (threadIdx.x < ORD_NB) hist[threadIdx.x] = 0;
}

// bucket of every cell, and the buckets' sizes (block histograms in LDS)
__global__ __launch_bounds__(ORD_TPB) void k_order_key(int64_t n, const float* __restrict__ M,
                                                       int32_t* __restrict__ key,
                                                       int32_t* __restrict__ hist) {
  __shared__ int32_t lh[ORD_NB];
  if (threadIdx.x < ORD_NB) lh[threadIdx.x] = 0;
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * ORD_TPB + threadIdx.x;
  if (c < n) {
    const int b = order_bucket(M + c * K3);
    key[c] = b;
    atomicAdd(&lh[b], 1);
  }
  __syncthreads();
  if (threadIdx.x < ORD_NB && lh[threadIdx.x] > 0) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

// bucket sizes -> first position of each bucket (exclusive prefix sum)
__global__ void k_order_scan(int32_t* __restrict__ hist) {
  if (threadIdx.x == 0) {
    int32_t sum = 0;
    for (int b = 0; b < ORD_NB; ++b) {
      const int32_t h = hist[b];
      hist[b] = sum;
      sum += h;
    }
  }
}

// each block reserves its range in every bucket, then writes its cells there
__global__ __launch_bounds__(ORD_TPB) void k_order_scatter(int64_t n,
                                                           const int32_t* __restrict__ key,
                                                           int32_t* __restrict__ cursor,
                                                           int32_t* __restrict__ order) {
  __shared__ int32_t lh[ORD_NB], lb[ORD_NB];
  if (threadIdx.x < ORD_NB) lh[threadIdx.x] = 0;
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * ORD_TPB + threadIdx.x;
  int b = 0, r = 0;
  if (c < n) {
    b = key[c];
    r = atomicAdd(&lh[b], 1);
  }
  __syncthreads();
  if (threadIdx.x < ORD_NB && lh[threadIdx.x] > 0)
    lb[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], lh[threadIdx.x]);
  __syncthreads();
  if (c < n) order[lb[b] + r] = (int32_t)c;
}

hipError_t launch_newton_wave(mem_ctx_t c, int64_t n, const float* M, float* beta,
                              const SolveParams& p, bool closed_start, int32_t* queue,
                              int32_t* iters, float* resid, uint32_t* status, int32_t* done_list,
                              int32_t* done_ctr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (c->n1d != 12) return hipErrorNotSupported;
  const int wpc = c->tune.wave_per_cu > 0 ? c->tune.wave_per_cu : WAVE_SOLVE_PER_CU;
  const int64_t waves = std::min<int64_t>(n, (int64_t)c->n_cu * wpc);
  // with several cells per wave, the cells far from their start go first; the
  // order goes to the kernel as o.next_list (lists 0 to 2 are free while the
  // persistent kernel runs: it keeps no work lists)
  int32_t* order = nullptr;
  if (n >= 4 * waves && n <= INT32_MAX && c->w_list[0] && c->w_list[1] && c->w_list[2]) {
    order = c->w_list[0];
    int32_t* key = c->w_list[1];
    int32_t* hist = c->w_list[2];
    k_order_zero<<<1, 64, 0, s>>>(hist);
    k_order_key<<<nblocks(n, ORD_TPB), ORD_TPB, 0, s>>>(n, M, key, hist);
    k_order_scan<<<1, 64, 0, s>>>(hist);
    k_order_scatter<<<nblocks(n, ORD_TPB), ORD_TPB, 0, s>>>(n, key, hist, order);
  }
  DirOut o{order, nullptr, iters, resid, status, done_list, done_ctr};
  k_newton_wave<12><<<(unsigned)waves, 64, 0, s>>>(c->d_t1, queue, n, M, beta, p,
                                                   closed_start ? 1 : 0, c->w_S, c->w_logZ,
                                                   c->w_iters, c->w_status, c->w_resid, o);
  return hipGetLastError();
}

hipError_t launch_unpack3(mem_ctx_t c, int64_t n, float* E, float* H, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_unpack3<<<nblocks(n, 128), 128, 0, s>>>(n, c->w_S, E, H);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// conditioning monitor of the time step (Sec. 3.5, Sec. 4.6)
// --------------------------------------------------------------------------
// Per cell, a lower bound of cond(H) for the FP32 Hessian at the cell's
// solution, built from the S row the step's flux pass assembled there.  One
// wave per cell; lane j < 34 holds column j of H (= row j).  For unit vectors
// v and u, |H v| <= lambda_max and |H^-1 u| <= 1 / lambda_min, so
// |H v| |H^-1 u| <= cond(H): v and u come from CE3_ITERS steps of power and
// inverse iteration from (1, ..., 1)/sqrt 34, the inverse through the register
// Cholesky.  max(max_j |H e_j|, max_k d_k) / min_k d_k (every LDL^T pivot lies
// between the extreme eigenvalues) is folded in.  +inf where a pivot fails; 0
// for a cell whose S row is not usable.
constexpr int CE3_ITERS = 6;
__global__ __launch_bounds__(64) void k_cond3(int64_t n, const float* __restrict__ S,
                                              float* __restrict__ cond) {
  __shared__ float sS[NCOL + 36];
  const int64_t c = blockIdx.x;
  const int lane = threadIdx.x;
  if (c >= n) return;
  for (int t = lane; t < NCOL; t += 64) sS[t] = S[c * NCOL + t];
  __builtin_amdgcn_wave_barrier();
  const float s00 = uf(sS[0]);
  float* E = sS + NCOL;
  if (lane < K3) E[lane] = lane == 0 ? 1.f : sS[lane] / s00;
  __builtin_amdgcn_wave_barrier();
  if (!(s00 > 0.f) || !isfinite(s00)) {
    if (lane == 0) cond[c] = 0.f;
    return;
  }
  float a[NH];
  load_hcol(sS, 1.f / s00, E, lane, 0.f, a);
  float cs = 0.f;
#pragma unroll
  for (int i = 0; i < NH; ++i) cs = fmaf(a[i], a[i], cs);
  const float hn = uf(sqrtf(wave_max(lane < NH ? cs : 0.f)));
  // power iteration on H (before the factorisation overwrites it)
  const float v0 = lane < NH ? 0.17149858514250882f : 0.f;  // 1 / sqrt 34
  float v = v0, nv = 0.f;
  for (int k = 0; k < CE3_ITERS; ++k) {
    float w = 0.f;
#pragma unroll
    for (int i = 0; i < NH; ++i) w = fmaf(a[i], rl(v, i), w);
    w = lane < NH ? w : 0.f;
    nv = uf(sqrtf(wave_sum(w * w)));
    v = w / nv;
  }
  float dinv = 1.f, dmin = 0.f, dmax = 0.f;
  const bool ok = wave_chol_rl(a, dinv, lane, dmin, dmax);
  float u = v0, nu = 0.f;
  for (int k = 0; ok && k < CE3_ITERS; ++k) {
    float w = 0.f, d = 0.f;
    wave_solve_rl(a, dinv, lane, u, w, d);
    d = lane < NH ? d : 0.f;
    nu = uf(sqrtf(wave_sum(d * d)));
    u = d / nu;
  }
  const float est = nv * nu;
  const float cnd = ok ? fmaxf(isfinite(est) ? est : 0.f, fmaxf(dmax, hn) / dmin)
                       : __builtin_inff();
  if (lane == 0) cond[c] = cnd;
}

hipError_t launch_cond3(mem_ctx_t c, int64_t n, float* cond, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_cond3<<<(unsigned)n, 64, 0, s>>>(n, c->w_S, cond);
  return hipGetLastError();
}

}  // namespace memk
