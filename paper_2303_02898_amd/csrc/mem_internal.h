// Internal declarations shared by the host API and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mem.h"

namespace memk {

// ---- 3D, 35-moment layout constants -----------------------------------------
constexpr int K3 = 35;        // basis size (total degree <= 4 in 3 variables)
constexpr int NH = 34;        // Newton unknowns beta_1..beta_34
constexpr int NPAIR = 630;    // pairs (i <= j) of basis functions
constexpr int NCOL = 640;     // pair columns padded to 40 MFMA blocks of 16
constexpr int NBLK = 40;      // 16-column blocks of the assembly GEMM
constexpr int GRP = 16;       // quadrature nodes per MFMA node group
constexpr int NJ = 9;         // 4-wide k-chunks of the exponent GEMM (36 = 9*4)
constexpr int HPACK = 595;    // packed upper triangle of the 34x34 Hessian
constexpr int TILE = 64;      // cells per assembly / line-search workgroup
constexpr int ND4 = 15;       // basis functions of total degree 4 (indices 20..34)
constexpr int NP5 = 120;      // pairs (i <= j) of degree-4 functions
constexpr int NC5 = 128;      // their columns padded to 8 MFMA blocks
constexpr int MIX_FB = 3;     // FP32 column blocks of the mixed assembly (columns 0..47)
constexpr float NEG_BIG = -1.0e30f;  // log weight of padding nodes (exp -> 0)

// Column of the pair (i, j), i <= j, in the row-major upper-triangle order.
__host__ __device__ constexpr int pair_col(int i, int j) {
  return i * K3 - (i * (i - 1)) / 2 + (j - i);
}

// ---- 1D, 5-moment layout ---------------------------------------------------
constexpr int K1 = 5;
constexpr int Q1MAX = 64;

// Per-call options as seen by kernels (plain floats, no host structs).
struct SolveParams {
  float tol_grad, tol_dec, tol_loose;
  int max_iter, max_ls;
  float c, atol, rtol;
  float lambda0, lambda_mul, alpha_min;
  float fp64_ratio;
  float lmin;  // min_p log w~_p: a dual value below it certifies non-realizability
  int refine;  // > 0: converged and stalled cells go on to compensated refinement
  float beta_max;  // |beta|_inf beyond this ends a cell as non-realizable (0 = off)
  int stall_window;  // nine-statistic solve: iterations without halving below the
                     // stall gate before a cell stops as stagnated (0 = default 20)
};

}  // namespace memk

// ---- context -----------------------------------------------------------------
// Everything a captured time step depends on (compared bytewise).
struct StepKey {
  mem_batch_t b;
  float *M, *beta, *g, *t, *dt;
  uint32_t* status;
  memk::SolveParams p;
  int refine;
  uint64_t gen;  // workspace and tuning generation (see mem_ctx_s::ws_gen)
};

// default launch parameters (field order of mem_tuning_t)
constexpr mem_tuning_t TUNE_DEFAULT{4, 512, 0.0, 1, 0, 12, 4, 0};

struct mem_ctx_s {
  int dim = 3, n1d = 12, K = 35, Q = 0, Qpad = 0, ngroups = 0, prec = 0;
  mem_tuning_t tune = TUNE_DEFAULT;  // launch parameters (mem_autotune / mem_set_tuning)
  int device = 0;
  int n_cu = 256;  // compute units of the device (grid of the persistent solve)
  std::string arch;  // gcnArchName of the device (key of the tuning cache)
  // host FP64 tables (checked against the oracle by the tests)
  std::vector<double> h_nodes, h_w, h_phi, h_logw;
  // device tables, 3D
  float* d_phiA = nullptr;   // exponent A operand  [ngroups][NJ][64]
  float* d_psi = nullptr;    // assembly B operand  [ngroups][4][10][64][4]
  // speeds: B operand of the degree-5 products phi_{i+e_x} phi_j (i <= j both of
  // degree 4) [ngroups][4][2][64][4], and for each pair column of
  // C = E[u_x phi phi^T] two sources and weights: src < 1024 is a column of S,
  // src >= 1024 column src - 1024 of S5 (ux_src packs src1 | src2 << 16)
  float* d_psi5 = nullptr;
  float* d_psiF = nullptr;      // flux-only operand: phi_i (columns 0..34), u_x phi_i (35..69)
  int32_t* d_ux_src = nullptr;  // [NPAIR]
  float2* d_ux_w = nullptr;     // [NPAIR]
  // mixed precision (BF16 / FP16 hi + lo) assembly operands, 32-node groups
  int nsg_m = 0;              // node groups of 32 (nodes padded with zero weight)
  float* d_phiA_m = nullptr;  // exponent A operand [2*nsg_m][NJ][64] (FP16: log w~ + k_p ln 2)
  float* d_psiF_m = nullptr;  // FP32 B operand of the moment blocks [nsg_m][MIX_FB][64][8]
  void* d_psi_hi = nullptr;   // 16-bit B operand, high part [nsg_m][NBLK-MIX_FB][64][8]
  void* d_psi_lo = nullptr;   // 16-bit B operand, low part
  float2* d_t1 = nullptr;    // 1D tables (hi, lo): h_a(x_k) at [a*n + k], a <= 4; lw_k at [5n + k]
  // device tables, 1D
  float* d_tab1 = nullptr;   // [Q][8]: phi_0..phi_4, log w~, 0, 0
  // workspace (per cell unless stated)
  int64_t cap_cells = 0;
  int32_t cap_problems = 0;
  float* w_S = nullptr;       // [cap][NCOL]
  float* w_S5 = nullptr;      // [cap][NC5] degree-5 columns (characteristic speeds)
  float* w_dbeta = nullptr;   // [cap][36]
  float* w_logZ = nullptr;    // [cap]
  float* w_L = nullptr;
  float* w_alpha = nullptr;
  float* w_gdot = nullptr;
  float* w_resid = nullptr;
  int32_t* w_iters = nullptr;
  uint32_t* w_status = nullptr;
  int32_t* w_list[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t* w_ctr = nullptr;   // [8] list counters
  int8_t* w_code = nullptr;   // [cap] per-slot outcome of the direction kernel
  float* w_Sp = nullptr;      // [sp_rows][NCOL] partial sums of node-range splits
  int64_t sp_rows = 0;
  float* w_Gacc = nullptr;    // [cap][36] compensated gradient E[phi_i] - M_i/n
  float* w_racc = nullptr;    // [cap] compensated residual
  float* w_rbest = nullptr;   // [cap] best FP32 residual so far (stall test)
  int32_t* w_itbest = nullptr;// [cap] iteration of the last halving of the residual
  int32_t* h_ctr = nullptr;   // pinned host mirror for polling
  unsigned char* scratch = nullptr;  // this device's static scratch (mem_maxent_solve_noalloc)
  // time stepping
  float* w_Mnew = nullptr;    // [cap][K]
  float* w_F = nullptr;       // [cap][K]
  float* w_rho = nullptr;     // [cap]
  float* w_cond = nullptr;    // [cap] lower bound of cond(H) per cell (the step's monitor)
  // second-order interface fluxes: one row per interface (cells + problems <= cap)
  float* w_hM = nullptr;      // Lax--Wendroff half-step moments [cap][K]
  float* w_hB = nullptr;      // their beta [cap][K]
  float* w_hG = nullptr;      // interface gauge (right element's) [cap][3]
  float* w_hF = nullptr;      // Lax--Wendroff flux [cap][K]
  float* w_hLF = nullptr;     // LLF flux [cap][K]
  float* w_hPhi = nullptr;    // FLIC limiter per moment [cap][K]
  int32_t* w_prob = nullptr;  // [cap] problem of each cell
  float* w_gM = nullptr;      // ghost moments   [2*P][K]
  float* w_gB = nullptr;      // ghost beta      [2*P][K]
  float* w_gG = nullptr;      // ghost gauge     [2*P][3]
  float* w_gF = nullptr;      // ghost fluxes    [2*P][K]
  float* w_gR = nullptr;      // ghost radius    [2*P]
  uint32_t* w_rmax = nullptr; // per-problem max radius (float bits) [P]
  // bumped by every reallocation of the workspace and every change of the
  // launch parameters: a captured step holds the old pointers and grid shapes
  uint64_t ws_gen = 0;
  // captured time step of mem_step (use_graph)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t step_exec = nullptr;
  StepKey step_key{};
  // kernel timing (mem_profile_enable / mem_profile_read)
  bool prof = false;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_marks;
  std::string err;
};

// ---- kernel launchers (defined in the .hip files) ------------------------------
namespace memk {

hipError_t launch_solve1(mem_ctx_t c, int64_t n, const float* M, float* beta,
                         const SolveParams& p, int32_t* iters, float* resid,
                         uint32_t* status, hipStream_t s);
hipError_t launch_gauge1(mem_ctx_t c, int64_t n, float* M, float* beta, float* g,
                         hipStream_t s);
// cond (nullable): per cell, a lower bound of cond(H) of the FP32 Hessian at the
// solve's last iterate (+inf where its Cholesky fails; 0 if none assembled)
hipError_t launch_axi_solve(int64_t n, int P, const float4* tab, const float* M, const float* g,
                            float* beta, const SolveParams& p, int32_t* iters, float* resid,
                            uint32_t* status, hipStream_t s, float* cond = nullptr);
hipError_t launch_axi_speeds(int64_t n, int P, const float4* tab, const float* beta, const float* g,
                             float ux_min, float ux_max, float* lam, hipStream_t s);
// A batch of nine-statistic shock problems as the step kernels see it: n
// cells in P problems, problem p owning cells [off[p], off[p+1]); pid[n] and
// pidI[n + P] give the problem of each cell and each interface row; dx[P].
struct AxBatch {
  int64_t n;
  int P;
  const int64_t* off;
  const int32_t* pid;
  const int32_t* pidI;
  const float* dx;
};
// pid, pidI and the ghost multipliers and gauges (rows 2p, 2p + 1) from the
// batch and its ghost states gs[P][6]
hipError_t launch_axi_prologue(const AxBatch& b, const float* gs, int32_t* pid, int32_t* pidI,
                               float* gB, float* gG, hipStream_t s);
// one problem's descriptors: off = {0, n}, dx, gs = left (n, v, T), right (n, v, T)
hipError_t launch_axi_single(int64_t n, float dx, const float* left, const float* right,
                             int64_t* off, float* dxo, float* gs, hipStream_t s);
hipError_t launch_axi_collide(const AxBatch& b, float* M, const float* g, const float* dtp,
                              int stride, float f, float prandtl, float mu_ref, hipStream_t s);
hipError_t launch_axi_fix(int64_t n, const float* M, float* beta, const uint32_t* st, hipStream_t s);
hipError_t launch_axi_dt(const AxBatch& b, const float* lam, const float* glam, float cfl,
                         float* dt, float* scal, int init, hipStream_t s);
hipError_t launch_axi_fv(const AxBatch& b, const float* M, const float* F, const float* lam,
                         const float* g, const float* gM, const float* gF, const float* glam,
                         const float* gG, const float* scal, float* Mout, hipStream_t s);
hipError_t launch_axi_iface(const AxBatch& b, const float* M, const float* F, const float* lam,
                            const float* g, const float* beta, const float* gM, const float* gF,
                            const float* glam, const float* gG, const float* gB,
                            const float* scal, int flic, float* fLF, float* Mh, float* gI,
                            float* bI, float* phi, hipStream_t s);
hipError_t launch_axi_fv2(const AxBatch& b, const float* M, const float* g, const float* gG,
                          const float* fLF, const float* fLW, const float* phi,
                          const uint32_t* stI, const float* scal, float* Mout, hipStream_t s);
hipError_t launch_axi_finish(int P, float* t, float* dt, const float* scal, hipStream_t s);
// cond_max[p] = max(cond_max[p], max of cond over problem p's cells)
hipError_t launch_axi_cond_max(const AxBatch& b, const float* cond, float* cond_max,
                               hipStream_t s);
hipError_t launch_axi_moments_nc(int64_t n, int P, const float4* tab, const float* alpha,
                                 const float* g, float* M, hipStream_t s);
hipError_t launch_axi_gauge(int64_t n, float* M, float* beta, float* g, hipStream_t s);
hipError_t launch_axi_moments(int64_t n, int P, const float4* tab, const float* beta,
                              const float* g, float* M, float* F, hipStream_t s);
hipError_t launch_gauge3(mem_ctx_t c, int64_t n, float* M, float* beta, float* g,
                         hipStream_t s);

// 3D Newton pieces.  Lists are arrays of cell ids with a device counter; a
// null list means "cells 0..n-1".
hipError_t launch_init3(mem_ctx_t c, int64_t n, const float* M, float* beta,
                        int32_t* out_list, int32_t* out_ctr, int32_t* iters, float* resid,
                        uint32_t* status, hipStream_t s);
hipError_t launch_lse3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                       const int32_t* ctr, int64_t n, const float* M, float* beta,
                       bool line_search, const SolveParams& p, int32_t* reset_a,
                       int32_t* reset_b, hipStream_t s);
// 128-column assembly (k_assemble3<2>) with the table d_psi5 or d_psiF
hipError_t launch_assemble5(mem_ctx_t c, int64_t n, const float* beta, const float* table,
                            float* S5, hipStream_t s);
hipError_t launch_assemble3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                            const int32_t* ctr, int64_t n, const float* beta,
                            const float* table, float* S, hipStream_t s);
// Mixed-precision variant of launch_assemble3 (the context's precision
// selects BF16 or FP16); always the plain pair table Psi.
hipError_t launch_assemble3m(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                             const int32_t* ctr, int64_t n, const float* beta, float* S,
                             hipStream_t s);
// Splits of the node range for small launches (1 = none) and their sum.
int assembly_splits(mem_ctx_t c, int ntile, int ngroups, int tw);
hipError_t launch_sum_splits(mem_ctx_t c, const int32_t* list, const int32_t* ctr, int64_t n,
                             int64_t rows, int nsplit, float* S, hipStream_t s);
// First Newton pass of the cells whose beta is exactly the Maxwellian of their
// gauge (closed form: H = I, E = e_0); the others go to asm_list/asm_ctr for
// the ordinary first assembly.
hipError_t launch_start3(mem_ctx_t c, int64_t n, const int32_t* list, const int32_t* ctr,
                         const float* M, const float* beta, const SolveParams& p,
                         int32_t* next_list, int32_t* next_ctr, int32_t* asm_list, int32_t* asm_ctr,
                         int32_t* iters, float* resid, uint32_t* status, int32_t* done_list,
                         int32_t* done_ctr, hipStream_t s);
hipError_t launch_direction3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                             const int32_t* ctr, const float* M, const float* beta,
                             const SolveParams& p,
                             int32_t* next_list, int32_t* next_ctr, int32_t* fb_list,
                             int32_t* fb_ctr, int32_t* iters, float* resid,
                             uint32_t* status, int32_t* done_list, int32_t* done_ctr,
                             hipStream_t s);
hipError_t launch_fallback3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                            const int32_t* ctr, const float* M, const float* beta,
                            const SolveParams& p,
                            int32_t* next_list, int32_t* next_ctr, int32_t* iters,
                            float* resid, uint32_t* status, int32_t* done_list,
                            int32_t* done_ctr, hipStream_t s);
hipError_t launch_accurate3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                            const int32_t* ctr, const float* M, const float* beta, float tol,
                            int32_t* out_list, int32_t* out_ctr, hipStream_t s);
hipError_t launch_moment_residual3(mem_ctx_t c, int64_t n, const float* M, const float* beta,
                                   float* G, hipStream_t s);
hipError_t launch_refine3(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                          const int32_t* ctr, const float* M, float* beta, int32_t* reset, hipStream_t s);
hipError_t launch_refine_final(mem_ctx_t c, int64_t grid_cells, const int32_t* list,
                               const int32_t* ctr, float tol_loose, float* resid,
                               uint32_t* status, hipStream_t s);
hipError_t launch_set_ctr(int32_t* ctr, int n, hipStream_t s);
// Persistent Newton solve of cells 0..n-1: one wavefront per live cell from
// the work queue `queue` (zeroed by the caller); converged cells are appended
// to done_list for the refinement kernels.
constexpr int WAVE_SOLVE_PER_CU = 12;  // default and most: 3 waves per SIMD
hipError_t launch_newton_wave(mem_ctx_t c, int64_t n, const float* M, float* beta,
                              const SolveParams& p, bool closed_start, int32_t* queue,
                              int32_t* iters, float* resid, uint32_t* status, int32_t* done_list,
                              int32_t* done_ctr, hipStream_t s);
hipError_t launch_unpack3(mem_ctx_t c, int64_t n, float* E, float* H, hipStream_t s);
hipError_t launch_flux3(mem_ctx_t c, int64_t n, const float* beta, const float* g,
                        float* F, float* rho_or_lam, bool want_lam, bool radius_only,
                        uint32_t* status, hipStream_t s);

// time stepping
hipError_t launch_collide3(mem_ctx_t c, int64_t n, float* M, const float* g,
                           float h_scalar, const float* dt_prob, const int32_t* prob,
                           float prandtl, float mu_ref, hipStream_t s);
hipError_t launch_fv3(mem_ctx_t c, int64_t n, const float* M, const float* F,
                      const float* rho, const float* g, const int32_t* prob,
                      const int64_t* offsets, const float* dx, const float* dt,
                      float* Mnew, int P, hipStream_t s);
hipError_t launch_prob_map(mem_ctx_t c, const int64_t* offsets, int P, int32_t* prob,
                           hipStream_t s);
hipError_t launch_ghost_pack(mem_ctx_t c, const mem_batch_t* b, hipStream_t s);
hipError_t launch_rho_max(mem_ctx_t c, int64_t n, const float* rho, const int32_t* prob,
                          int P, hipStream_t s);
hipError_t launch_iface3(mem_ctx_t c, int64_t n, int P, const float* M, const float* F,
                        const float* beta, const float* rho, const float* g, const int32_t* prob,
                        const int64_t* offsets, const float* dx, const float* dt, bool flic,
                        hipStream_t s);
hipError_t launch_fv3i(mem_ctx_t c, int64_t n, const float* M, const float* g, const int32_t* prob,
                       const int64_t* offsets, const float* dx, const float* dt, bool flic,
                       float* Mnew, hipStream_t s);
hipError_t launch_zero(int64_t n, float* x, hipStream_t s);
// per cell, a lower bound of cond(H) at the Hessian of the S rows in w_S (the
// step's flux pass): power and inverse iterations, see k_cond3
hipError_t launch_cond3(mem_ctx_t c, int64_t n, float* cond, hipStream_t s);
hipError_t launch_cond_max(int64_t n, const float* cond, const int32_t* prob, float* out,
                           hipStream_t s);
hipError_t launch_dt_cap(mem_ctx_t c, int P, const float* dx, float cfl, float* dt,
                         hipStream_t s);
hipError_t launch_dt_update(mem_ctx_t c, int P, const float* dx, float cfl, float* t,
                            float* dt, bool advance_t, hipStream_t s);
hipError_t launch_status_or(int64_t n, const uint32_t* src, uint32_t* dst, hipStream_t s);
hipError_t launch_maxwell_fallback(mem_ctx_t c, int64_t n, const float* M, float* beta,
                                   hipStream_t s);
hipError_t launch_iter_hist(int64_t n, const int32_t* iters, int nbins, int64_t* hist,
                            hipStream_t s);
hipError_t launch_status_count(int64_t n, const uint32_t* st, int64_t* counts, hipStream_t s);
hipError_t launch_rmax_init(mem_ctx_t c, int P, hipStream_t s);
hipError_t launch_copy(int64_t n, const float* src, float* dst, hipStream_t s);
hipError_t launch_conserved(mem_ctx_t c, const mem_batch_t* b, const float* M,
                            const float* g, double* out, hipStream_t s);

}  // namespace memk

// host table builder (tables.cpp)
namespace memt {
void gauss_hermite(int n, std::vector<double>& x, std::vector<double>& w);
void build_host(int dim, int n, std::vector<double>& nodes, std::vector<double>& wts,
                std::vector<double>& logw, std::vector<double>& phi, int& K, int& Q);
void build_tables(mem_ctx_t c);   // fills host tables and uploads device layouts
}
