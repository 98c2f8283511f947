// Mixed-precision moment / Hessian assembly for the 35-moment basis.
//
// S[c][(i,j)] = sum_p sigma_{c,p} phi_i(u_p) phi_j(u_p) (App. C: E[phi] and
// E[phi phi^T] are the columns of one GEMM sigma . Psi because the nodes are
// fixed in gauge coordinates).  The 35 moment columns (0, j) -- which give the
// gradient G = E[phi] - M/n -- are accumulated from FP32 products on the FP32
// matrix cores; the remaining pair columns, which only enter the Hessian, use
// 16-bit matrix cores on hi + lo splits of both operands:
//     sigma Psi ~ sigma_hi Psi_hi + sigma_hi Psi_lo + sigma_lo Psi_hi,
// products exact in FP32, FP32 accumulation.  BF16 keeps 16 significant bits
// per operand pair; FP16 keeps 22 but needs range control: node p carries a
// power-of-two scale 2^k_p (folded into log w~_p of the exponent table and
// divided out of Psi), so sigma' = sigma 2^k_p and Psi' = Psi 2^-k_p stay
// inside the FP16 range.  The Newton iteration keeps using the FP32 gradient,
// so the Hessian's rounding only changes the contraction rate.
//
// Work split (64 cells per workgroup, 4 wavefronts):
//   * wave w computes sigma for cells 16w..16w+15 over a 32-node group with
//     the FP32 exponent MFMA (A = [log w~ | phi] table, B = beta) and shares it
//     through LDS, as FP32 and as 16-bit hi/lo fragments (double-buffered);
//   * wave w then owns column block w (FP32, 16 columns) and 16-bit blocks
//     4 + 9w .. 12 + 9w for all 64 cells, reading its Psi operands straight
//     from global memory one node group ahead (no LDS staging: no two waves
//     of a workgroup share a Psi element).
#include "mem_internal.h"

namespace memk {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int SGN = 32;       // nodes per 16x16x32 k-step
constexpr int MB = 9;         // 16-bit column blocks per wave
constexpr int NFB = 4;        // FP32 column blocks (columns 0..63 hold the moments)

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <bool F16>
struct Half;
template <>
struct Half<false> {
  typedef __bf16 T;
  typedef bf8 V;
  static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Half<true> {
  typedef _Float16 T;
  typedef h8 V;
  static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <typename V>
__device__ __forceinline__ V as_v(uint4 u) {
  return __builtin_bit_cast(V, u);
}

template <bool F16>
__global__ __launch_bounds__(256, 1) void k_assemble3m(
    const float* __restrict__ phiA,   // [2*nsg][NJ][64]   exponent A operand
    const float* __restrict__ psiF,   // [nsg][NFB][64][8] FP32 B operand, blocks 0..3
    const uint4* __restrict__ psiH,   // [nsg][36][64]     16-bit B operand, high part
    const uint4* __restrict__ psiL,   // [nsg][36][64]     16-bit B operand, low part
    int nsg, const int32_t* __restrict__ list, const int32_t* __restrict__ ctr, int64_t n,
    const float* __restrict__ beta, const float* __restrict__ logZ, float* __restrict__ S,
    int ntile, int nsplit, float* __restrict__ Sp) {
  using H = Half<F16>;
  using T = typename H::T;
  using V = typename H::V;
  const int64_t count = ctr ? (int64_t)(*ctr) : n;
  const int split = (int)(blockIdx.x / ntile);
  const int64_t tile0 = (int64_t)(blockIdx.x % ntile) * TILE;
  if (tile0 >= count) return;
  const int sbeg = (int)((int64_t)split * nsg / nsplit);
  const int send = (int)((int64_t)(split + 1) * nsg / nsplit);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int64_t slot = tile0 + wave * 16 + (lane & 15);
  const bool valid = slot < count;
  const int64_t cell = valid ? (list ? (int64_t)list[slot] : slot) : 0;

  float bt[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = 4 * j + kq;
    bt[j] = k == 0 ? 1.f : ((valid && k < K3) ? beta[cell * K3 + k] : 0.f);
  }
  const float lz = valid ? logZ[cell] : 0.f;

  f4 accF[4];
  f4 acc[4][MB];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    accF[t] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < MB; ++b) acc[t][b] = (f4){0.f, 0.f, 0.f, 0.f};
  }

  __shared__ float sF[2][4][8][64];   // sigma (FP32) [buffer][tile][k-step][lane]
  __shared__ uint4 sH[2][4][64];      // 16-bit hi fragments [buffer][tile][lane]
  __shared__ uint4 sL[2][4][64];      // 16-bit lo fragments

  // operands of node group s, loaded one group ahead
  float pa[2 * NJ];
  float4 pf[2];
  uint4 ph[MB], pl[MB];
  auto load = [&](int s) {
#pragma unroll
    for (int j = 0; j < 2 * NJ; ++j) pa[j] = phiA[((size_t)2 * s * NJ + j) * 64 + lane];
    const float4* f = reinterpret_cast<const float4*>(psiF + (((size_t)s * NFB + wave) * 64 + lane) * 8);
    pf[0] = f[0];
    pf[1] = f[1];
    const size_t hb = ((size_t)s * 36 + MB * wave) * 64 + lane;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      ph[b] = psiH[hb + (size_t)b * 64];
      pl[b] = psiL[hb + (size_t)b * 64];
    }
  };
  load(sbeg);

  for (int s = sbeg; s < send; ++s) {
    const int buf = s & 1;
    float ca[2 * NJ];
#pragma unroll
    for (int j = 0; j < 2 * NJ; ++j) ca[j] = pa[j];
    const float cf[8] = {pf[0].x, pf[0].y, pf[0].z, pf[0].w, pf[1].x, pf[1].y, pf[1].z, pf[1].w};
    uint4 ch[MB], cl[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) { ch[b] = ph[b]; cl[b] = pl[b]; }
    if (s + 1 < send) load(s + 1);

    // sigma of this wave's 16 cells at nodes 32s + 16h + 4(l/16) + r
    f4 e0 = {0.f, 0.f, 0.f, 0.f}, e1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      e0 = mfma4(ca[j], bt[j], e0);
      e1 = mfma4(ca[NJ + j], bt[j], e1);
    }
    float sg[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sg[r] = valid ? __expf(e0[r] - lz) : 0.f;
      sg[4 + r] = valid ? __expf(e1[r] - lz) : 0.f;
    }
    V hv, lv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      sF[buf][wave][i][lane] = sg[i];
      const T h = (T)sg[i];
      hv[i] = h;
      lv[i] = (T)(sg[i] - (float)h);
    }
    sH[buf][wave][lane] = __builtin_bit_cast(uint4, hv);
    sL[buf][wave][lane] = __builtin_bit_cast(uint4, lv);
    __syncthreads();

#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int i = 0; i < 8; ++i) accF[t] = mfma4(sF[buf][t][i][lane], cf[i], accF[t]);
      const V ah = as_v<V>(sH[buf][t][lane]);
      const V al = as_v<V>(sL[buf][t][lane]);
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        const V bh = as_v<V>(ch[b]);
        const V bl = as_v<V>(cl[b]);
        acc[t][b] = H::mma(al, bh, acc[t][b]);
        acc[t][b] = H::mma(ah, bl, acc[t][b]);
        acc[t][b] = H::mma(ah, bh, acc[t][b]);
      }
    }
  }

  // D layout: lane l, register q -> row 4(l/16) + q of the tile, column l%16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t sl = tile0 + 16 * t + 4 * kq + q;
      if (sl < count) {
        float* dst;
        if (nsplit > 1) {
          dst = Sp + ((size_t)split * ntile * TILE + sl) * NCOL + (lane & 15);
        } else {
          const int64_t cw = list ? (int64_t)list[sl] : sl;
          dst = S + cw * NCOL + (lane & 15);
        }
        dst[16 * wave] = accF[t][q];
#pragma unroll
        for (int b = 0; b < MB; ++b) dst[16 * (NFB + MB * wave + b)] = acc[t][b][q];
      }
    }
  }
}

int64_t nblocks(int64_t n, int per) { return (n + per - 1) / per; }

}  // namespace

hipError_t launch_assemble3m(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                             const int32_t* ctr, int64_t n, const float* beta, float* S,
                             hipStream_t s) {
  if (grid_cells <= 0) return hipSuccess;
  const int ntile = (int)nblocks(grid_cells, TILE);
  const int nsplit = assembly_splits(c, ntile, 2 * c->nsg_m);
  const unsigned grid = (unsigned)(ntile * nsplit);
  if (c->prec == MEM_PREC_FP16X3)
    k_assemble3m<true><<<grid, 256, 0, s>>>(c->d_phiA_m, c->d_psiF_m,
                                            static_cast<const uint4*>(c->d_psi_hi),
                                            static_cast<const uint4*>(c->d_psi_lo), c->nsg_m,
                                            list, ctr, n, beta, c->w_logZ, S, ntile, nsplit,
                                            c->w_Sp);
  else
    k_assemble3m<false><<<grid, 256, 0, s>>>(c->d_phiA_m, c->d_psiF_m,
                                             static_cast<const uint4*>(c->d_psi_hi),
                                             static_cast<const uint4*>(c->d_psi_lo), c->nsg_m,
                                             list, ctr, n, beta, c->w_logZ, S, ntile, nsplit,
                                             c->w_Sp);
  if (nsplit > 1) return launch_sum_splits(c, list, ctr, n, ntile, nsplit, S, s);
  return hipGetLastError();
}

}  // namespace memk
