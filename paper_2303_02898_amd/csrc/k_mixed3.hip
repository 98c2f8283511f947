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
// Work split (64 cells per workgroup, 8 wavefronts, two per SIMD):
//   * wave w computes sigma for the 16 cells of tile w % 4 over half w / 4 of a
//     32-node group with the FP32 exponent MFMA (A = [log w~ | phi] table,
//     B = beta) and shares it through LDS, as FP32 and as 16-bit hi/lo
//     fragments (double-buffered, one barrier per node group);
//   * the 40 column blocks are split so that each SIMD's pair of waves does
//     the same MFMA work: waves 0..2 own FP32 block w (columns 0..47 hold the
//     35 moment columns) and 16-bit block 3 + w; waves 3..7 own 16-bit blocks
//     6..39 in runs of seven (the last wave six), all four tiles each;
//   * Psi operands go from global memory straight to registers (no two waves
//     of a workgroup share a Psi element); each register is refilled with the
//     next node group right after its last MFMA, and the exponent of the next
//     group is computed among the MFMAs of the current one.
#include "mem_internal.h"

namespace memk {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int MW = 8;                // wavefronts per workgroup
constexpr int MAXB = 7;              // most 16-bit column blocks owned by one wave
constexpr int NHB = NBLK - MIX_FB;   // 16-bit column blocks (37)

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
__global__ __launch_bounds__(64 * MW) void k_assemble3m(
    const float* __restrict__ phiA,   // [2*nsg][NJ][64]       exponent A operand
    const float* __restrict__ psiF,   // [nsg][MIX_FB][64][8]  FP32 B operand, blocks 0..2
    const uint4* __restrict__ psiH,   // [nsg][NHB][64]        16-bit B operand, high part
    const uint4* __restrict__ psiL,   // [nsg][NHB][64]        16-bit B operand, low part
    int nsg, const int32_t* __restrict__ list, const int32_t* __restrict__ ctr, int64_t n,
    const float* __restrict__ beta, const float* __restrict__ logZ, float* __restrict__ S,
    int ntile, int nsplit, float* __restrict__ Sp) {
  using H = Half<F16>;
  using T = typename H::T;
  using V = typename H::V;
  typedef T T4 __attribute__((ext_vector_type(4)));
  const int64_t count = ctr ? (int64_t)(*ctr) : n;
  const int split = (int)(blockIdx.x / ntile);
  const int64_t tile0 = (int64_t)(blockIdx.x % ntile) * TILE;
  if (tile0 >= count) return;
  const int sbeg = (int)((int64_t)split * nsg / nsplit);
  const int send = (int)((int64_t)(split + 1) * nsg / nsplit);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  // sigma duty: tile ts, node half hs
  const int ts = wave & 3, hs = wave >> 2;
  const int64_t slot = tile0 + 16 * ts + (lane & 15);
  const bool valid = slot < count;
  const int64_t cell = valid ? (list ? (int64_t)list[slot] : slot) : 0;
  // column duty
  const bool has_f = wave < MIX_FB;
  const int hb0 = wave < MIX_FB ? wave : 3 + 7 * (wave - MIX_FB);  // first 16-bit block (0-based)
  const int nb = wave < MIX_FB ? 1 : (wave == MW - 1 ? 6 : 7);

  float bt[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = 4 * j + kq;
    bt[j] = k == 0 ? 1.f : ((valid && k < K3) ? beta[cell * K3 + k] : 0.f);
  }
  const float lz = valid ? logZ[cell] : 0.f;

  f4 accF[4];
  f4 acc[4][MAXB];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    accF[t] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < MAXB; ++b) acc[t][b] = (f4){0.f, 0.f, 0.f, 0.f};
  }

  __shared__ float sF[2][4][8][64];   // sigma (FP32) [buffer][tile][k-step][lane]
  __shared__ uint4 sH[2][4][64];      // 16-bit hi fragments [buffer][tile][lane]
  __shared__ uint4 sL[2][4][64];      // 16-bit lo fragments

  // Psi operands of one node group (registers; refilled block by block)
  float cf[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  uint4 ph[MAXB], pl[MAXB];
  auto loadF = [&](int s) {
    if (has_f) {
      const float4* f = reinterpret_cast<const float4*>(psiF + (((size_t)s * MIX_FB + wave) * 64 + lane) * 8);
      const float4 f0 = f[0], f1 = f[1];
      cf[0] = f0.x; cf[1] = f0.y; cf[2] = f0.z; cf[3] = f0.w;
      cf[4] = f1.x; cf[5] = f1.y; cf[6] = f1.z; cf[7] = f1.w;
    }
  };
  auto loadH = [&](int s, int b) {
    const size_t hb = ((size_t)s * NHB + hb0 + b) * 64 + lane;
    ph[b] = psiH[hb];
    pl[b] = psiL[hb];
  };
  // sigma of tile ts at nodes 32s + 16hs + 4(l/16) + r, into LDS buffer buf
  auto sigma = [&](int s, int buf) {
    f4 e = {0.f, 0.f, 0.f, 0.f};
    const float* pa = phiA + ((size_t)(2 * s + hs) * NJ) * 64 + lane;
#pragma unroll
    for (int j = 0; j < NJ; ++j) e = mfma4(pa[j * 64], bt[j], e);
    T4 hv, lv;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float sg = valid ? __expf(e[r] - lz) : 0.f;
      sF[buf][ts][4 * hs + r][lane] = sg;
      const T h = (T)sg;
      hv[r] = h;
      lv[r] = (T)(sg - (float)h);
    }
    reinterpret_cast<uint2*>(&sH[buf][ts][lane])[hs] = __builtin_bit_cast(uint2, hv);
    reinterpret_cast<uint2*>(&sL[buf][ts][lane])[hs] = __builtin_bit_cast(uint2, lv);
  };

  // prologue: operands and sigma of the first group
  loadF(sbeg);
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    if (b < nb) loadH(sbeg, b);
    else { ph[b] = make_uint4(0, 0, 0, 0); pl[b] = make_uint4(0, 0, 0, 0); }
  }
  sigma(sbeg, 0);
  __syncthreads();

  // iteration s: sigma of group s + 1 into the other buffer, the MFMAs of group
  // s from LDS buffer (s - sbeg) & 1, and each Psi register refilled with group
  // s + 1 right after its last use
  for (int s = sbeg; s < send; ++s) {
    const int buf = (s - sbeg) & 1;
    const bool more = s + 1 < send;
    if (more) sigma(s + 1, buf ^ 1);

    if (has_f) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int t = 0; t < 4; ++t) accF[t] = mfma4(sF[buf][t][i][lane], cf[i], accF[t]);
      }
      if (more) loadF(s + 1);
    }
    V ah[4], al[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ah[t] = as_v<V>(sH[buf][t][lane]);
      al[t] = as_v<V>(sL[buf][t][lane]);
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      if (b < nb) {
        const V bh = as_v<V>(ph[b]), bl = as_v<V>(pl[b]);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t][b] = H::mma(al[t], bh, acc[t][b]);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t][b] = H::mma(ah[t], bl, acc[t][b]);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t][b] = H::mma(ah[t], bh, acc[t][b]);
        if (more) loadH(s + 1, b);
      }
    }
    __syncthreads();
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
        if (has_f) dst[16 * wave] = accF[t][q];
#pragma unroll
        for (int b = 0; b < MAXB; ++b)
          if (b < nb) dst[16 * (MIX_FB + hb0 + b)] = acc[t][b][q];
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
  const int nsplit = assembly_splits(c, ntile, 2 * c->nsg_m, TILE);
  const unsigned grid = (unsigned)(ntile * nsplit);
  if (c->prec == MEM_PREC_FP16X3)
    k_assemble3m<true><<<grid, 64 * MW, 0, s>>>(c->d_phiA_m, c->d_psiF_m,
                                            static_cast<const uint4*>(c->d_psi_hi),
                                            static_cast<const uint4*>(c->d_psi_lo), c->nsg_m,
                                            list, ctr, n, beta, c->w_logZ, S, ntile, nsplit,
                                            c->w_Sp);
  else
    k_assemble3m<false><<<grid, 64 * MW, 0, s>>>(c->d_phiA_m, c->d_psiF_m,
                                             static_cast<const uint4*>(c->d_psi_hi),
                                             static_cast<const uint4*>(c->d_psi_lo), c->nsg_m,
                                             list, ctr, n, beta, c->w_logZ, S, ntile, nsplit,
                                             c->w_Sp);
  if (nsplit > 1) return launch_sum_splits(c, list, ctr, n, (int64_t)ntile * TILE, nsplit, S, s);
  return hipGetLastError();
}

}  // namespace memk
