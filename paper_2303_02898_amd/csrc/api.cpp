// C ABI of the MEM library: context, argument checks, workspace and the launch
// sequences of the entry points declared in include/mem.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>

#include "mem_internal.h"

using namespace memk;

namespace {

// ---- device scratch of mem_maxent_solve_noalloc --------------------------------
// The Newton workspace of up to NOALLOC_MAX_CELLS cells plus a node-range split
// buffer, carved in a fixed order from one file-scope device array.  Every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never takes the array's address directly: mem_create resolves its device
// address once per device with hipGetSymbolAddress (the device current) and
// every host use goes through that pointer.
constexpr int64_t NOALLOC_MAX_CELLS = 8192;
constexpr int64_t NOALLOC_SPLIT_ROWS = 1024;
constexpr size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of the carved regions (n = NOALLOC_MAX_CELLS rows each).
struct NoallocLayout {
  size_t S, dbeta, logZ, L, alpha, gdot, resid, iters, status, list[5], ctr, code, Sp, Gacc,
      racc, rbest, itbest, total;
};
constexpr NoallocLayout noalloc_layout() {
  NoallocLayout l{};
  const size_t n = (size_t)NOALLOC_MAX_CELLS;
  size_t o = 0;
  auto take = [&o](size_t bytes) { const size_t at = o; o += al256(bytes); return at; };
  l.S = take(n * NCOL * 4);
  l.dbeta = take(n * 36 * 4);
  l.logZ = take(n * 4);
  l.L = take(n * 4);
  l.alpha = take(n * 4);
  l.gdot = take(n * 4);
  l.resid = take(n * 4);
  l.iters = take(n * 4);
  l.status = take(n * 4);
  for (int k = 0; k < 5; ++k) l.list[k] = take(n * 4);
  l.ctr = take(8 * 4);
  l.code = take(n);
  l.Sp = take((size_t)NOALLOC_SPLIT_ROWS * NCOL * 4);
  l.Gacc = take(n * 36 * 4);
  l.racc = take(n * 4);
  l.rbest = take(n * 4);
  l.itbest = take(n * 4);
  l.total = o;
  return l;
}
constexpr NoallocLayout NOALLOC = noalloc_layout();

__device__ __align__(256) unsigned char scratch[NOALLOC.total];

// The context fields the Newton loop (newton3) reads as its workspace.
struct NewtonWorkspace {
  float *S, *dbeta, *logZ, *L, *alpha, *gdot, *resid;
  int32_t* iters;
  uint32_t* status;
  int32_t* list[5];
  int32_t* ctr;
  int8_t* code;
  float* Sp;
  int64_t sp_rows;
  float *Gacc, *racc, *rbest;
  int32_t* itbest;
  bool prof;
  static NewtonWorkspace of(const mem_ctx_s* c) {
    NewtonWorkspace w;
    w.S = c->w_S; w.dbeta = c->w_dbeta; w.logZ = c->w_logZ; w.L = c->w_L;
    w.alpha = c->w_alpha; w.gdot = c->w_gdot; w.resid = c->w_resid; w.iters = c->w_iters;
    w.status = c->w_status;
    for (int k = 0; k < 5; ++k) w.list[k] = c->w_list[k];
    w.ctr = c->w_ctr; w.code = c->w_code; w.Sp = c->w_Sp; w.sp_rows = c->sp_rows;
    w.Gacc = c->w_Gacc; w.racc = c->w_racc; w.rbest = c->w_rbest; w.itbest = c->w_itbest;
    w.prof = c->prof;
    return w;
  }
  void install(mem_ctx_s* c) const {
    c->w_S = S; c->w_dbeta = dbeta; c->w_logZ = logZ; c->w_L = L; c->w_alpha = alpha;
    c->w_gdot = gdot; c->w_resid = resid; c->w_iters = iters; c->w_status = status;
    for (int k = 0; k < 5; ++k) c->w_list[k] = list[k];
    c->w_ctr = ctr; c->w_code = code; c->w_Sp = Sp; c->sp_rows = sp_rows; c->w_Gacc = Gacc;
    c->w_racc = racc; c->w_rbest = rbest; c->w_itbest = itbest; c->prof = prof;
  }
};

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (resolved once per device).
hipError_t resolve_scratch(int device, unsigned char** out) {
  *out = nullptr;
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

mem_err_t fail(mem_ctx_t c, mem_err_t e, const std::string& msg) {
  if (c) c->err = msg;
  return e;
}

#define MEM_HIP(c, x)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail((c), MEM_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// rows of the node-range split buffer (42 MB): splits are used for launches of
// at most a few thousand live cells
constexpr int64_t SP_ROWS = 16384;

template <typename T>
bool dalloc(T*& p, size_t count) {
  dfree(p);
  return hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)) == hipSuccess;
}

// A captured mem_step graph holds workspace pointers: drop it with the workspace.
void drop_step_graph(mem_ctx_t c) {
  ++c->ws_gen;
  if (c->step_exec) { (void)hipGraphExecDestroy(c->step_exec); c->step_exec = nullptr; }
}

void free_workspace(mem_ctx_t c) {
  drop_step_graph(c);
  dfree(c->w_S); dfree(c->w_S5); dfree(c->w_dbeta); dfree(c->w_logZ); dfree(c->w_L);
  dfree(c->w_alpha); dfree(c->w_gdot); dfree(c->w_resid); dfree(c->w_iters);
  dfree(c->w_status);
  for (auto& l : c->w_list) dfree(l);
  dfree(c->w_Gacc); dfree(c->w_racc); dfree(c->w_rbest); dfree(c->w_itbest);
  dfree(c->w_Mnew); dfree(c->w_F); dfree(c->w_rho); dfree(c->w_prob); dfree(c->w_code); dfree(c->w_Sp);
  dfree(c->w_cond);
  dfree(c->w_hM); dfree(c->w_hB); dfree(c->w_hG); dfree(c->w_hF); dfree(c->w_hLF); dfree(c->w_hPhi);
  c->sp_rows = 0;
  c->cap_cells = 0;
}

void free_problems(mem_ctx_t c) {
  drop_step_graph(c);
  dfree(c->w_gM); dfree(c->w_gB); dfree(c->w_gG); dfree(c->w_gF); dfree(c->w_gR);
  dfree(c->w_rmax);
  c->cap_problems = 0;
}

SolveParams params_from(const mem_solve_opts_t* o) {
  mem_solve_opts_t d;
  mem_solve_opts_default(&d);
  if (!o) o = &d;
  SolveParams p;
  p.tol_grad = o->tol_grad; p.tol_dec = o->tol_dec; p.tol_loose = o->tol_grad_loose;
  p.max_iter = o->max_iter; p.max_ls = o->max_ls;
  p.c = o->armijo_c; p.atol = o->atol; p.rtol = o->rtol;
  p.lambda0 = o->lambda0; p.lambda_mul = o->lambda_mul; p.alpha_min = o->alpha_min;
  p.fp64_ratio = o->fp64_pivot_ratio;
  p.beta_max = o->beta_max;
  p.lmin = -3.0e38f;
  p.refine = 0;
  p.stall_window = 0;
  return p;
}

// Lower bound of the dual value at any minimiser: min_p log w~_p (small margin
// for FP32 evaluation of the value).
float dual_floor(mem_ctx_t c) {
  double m = 1e300;
  for (double v : c->h_logw) m = std::min(m, v);
  return (float)(m - 1e-3 * (1.0 + std::fabs(m)));
}

bool opts_ok(const mem_solve_opts_t* o) {
  if (!o) return true;
  return o->max_iter >= 1 && o->max_iter <= 100000 && o->max_ls >= 0 && o->max_ls <= 60 &&
         o->lambda0 > 0.f && o->lambda_mul > 1.f && o->check_every >= 0 &&
         o->fp64_pivot_ratio >= 0.f && o->fp64_pivot_ratio < 1.f && std::isfinite(o->tol_grad) &&
         o->refine >= 0 && o->refine <= 8 && o->beta_max >= 0.f;
}

mem_err_t ensure_cells(mem_ctx_t c, int64_t n) {
  if (n <= c->cap_cells) return MEM_OK;
  return mem_reserve(c, n, c->cap_problems);
}

// Optional event pair around a launch (kernel timing for measurement).
struct ProfScope {
  mem_ctx_t c; int k; hipStream_t s; hipEvent_t b = nullptr, e = nullptr;
  ProfScope(mem_ctx_t c_, int k_, hipStream_t s_) : c(c_), k(k_), s(s_) {
    if (c->prof && c->prof_used + 2 <= c->prof_pool.size()) {
      b = c->prof_pool[c->prof_used++];
      e = c->prof_pool[c->prof_used++];
      (void)hipEventRecord(b, s);
    }
  }
  ~ProfScope() {
    if (b) {
      (void)hipEventRecord(e, s);
      c->prof_marks.push_back({k, {b, e}});
    }
  }
};

// The persistent one-wave-per-cell Newton kernel serves this launch.
bool wave_solver(mem_ctx_t c, int64_t n) {
  return c->tune.solver == 1 && c->prec == MEM_PREC_FP32 && c->n1d == 12 &&
         (c->tune.wave_max_cells <= 0 || n <= c->tune.wave_max_cells);
}

// Newton iterations of Alg. 1 over the live work-list.  With poll > 0 the
// stream is synchronised every `poll` iterations to stop once no cell is live.
// Counters: 0/1 live lists (alternating), 2 FP64 list, 3 converged list,
// 4/5 refinement lists.
mem_err_t newton3(mem_ctx_t c, int64_t n, const float* M, float* beta, const SolveParams& p,
                  int max_iter, int poll, int refine, int32_t* iters, float* resid,
                  uint32_t* status, hipStream_t s, bool try_closed_start = false) {
  int32_t* ctr = c->w_ctr;
  int32_t* done = refine > 0 ? c->w_list[3] : nullptr;
  MEM_HIP(c, launch_set_ctr(ctr, 8, s));
  if (wave_solver(c, n)) {
    // one persistent kernel for the whole Newton loop (counter 7: work queue)
    ProfScope ps(c, 3, s);
    MEM_HIP(c, launch_newton_wave(c, n, M, beta, p, try_closed_start && c->n1d >= 5, &ctr[7],
                                  iters, resid, status, done, &ctr[3], s));
  } else {
  MEM_HIP(c, launch_init3(c, n, M, beta, c->w_list[0], &ctr[0], iters, resid, status, s));
  {
    ProfScope ps(c, 2, s);
    MEM_HIP(c, launch_lse3(c, n, c->w_list[0], &ctr[0], n, M, beta, false, p, nullptr, nullptr, s));
  }
  int cur = 0;
  int64_t grid = n;  // live cells never increase: the last polled count bounds the grids
  // Cells that start at the Maxwellian of their gauge take their first direction
  // in closed form: there sigma_p = w_p, and a rule of >= 5 points per axis
  // integrates the degree <= 8 products exactly, so E[phi] = e_0 and H = I.  The
  // first pass then assembles only the other cells (list 4, counter 6).
  const bool closed_start = try_closed_start && c->n1d >= 5;
  if (closed_start)
    MEM_HIP(c, launch_start3(c, n, c->w_list[0], &ctr[0], M, beta, p, c->w_list[1], &ctr[1],
                             c->w_list[4], &ctr[6], iters, resid, status, done, &ctr[3], s));
  // every live cell takes one direction per pass and ends, at the latest, as
  // MAXITER at its max_iter-th: max_iter passes leave no live cell
  for (int it = 0; it < max_iter; ++it) {
    const int nxt = 1 - cur;
    // this pass's assembly list: list 4 after a closed-form start, else the live list
    int32_t* la = (it == 0 && closed_start) ? c->w_list[4] : c->w_list[cur];
    int32_t* ca = (it == 0 && closed_start) ? &ctr[6] : &ctr[cur];
    {
      ProfScope ps(c, 0, s);
      if (c->prec == MEM_PREC_FP32)
        MEM_HIP(c, launch_assemble3(c, grid, la, ca, n, beta, c->d_psi, c->w_S, s));
      else
        MEM_HIP(c, launch_assemble3m(c, grid, la, ca, n, beta, c->w_S, s));
    }
    {
      ProfScope ps(c, 1, s);
      MEM_HIP(c, launch_direction3(c, grid, la, ca, M, beta, p, c->w_list[nxt], &ctr[nxt],
                                   c->w_list[2], &ctr[2], iters, resid, status, done, &ctr[3], s));
    }
    MEM_HIP(c, launch_fallback3(c, grid, c->w_list[2], &ctr[2], M, beta, p, c->w_list[nxt], &ctr[nxt],
                                iters, resid, status, done, &ctr[3], s));
    {
      ProfScope ps(c, 2, s);
      MEM_HIP(c, launch_lse3(c, grid, c->w_list[nxt], &ctr[nxt], n, M, beta, true, p, &ctr[cur],
                             &ctr[2], s));
    }
    cur = nxt;
    if (poll > 0 && (it + 1) % poll == 0) {
      MEM_HIP(c, hipMemcpyAsync(c->h_ctr, &ctr[cur], sizeof(int32_t), hipMemcpyDeviceToHost, s));
      MEM_HIP(c, hipStreamSynchronize(s));
      if (*c->h_ctr == 0) break;
      grid = *c->h_ctr;
    }
  }
  }
  if (refine > 0) {
    // compensated residual of the converged cells; those above tol_grad get a
    // Newton correction and are evaluated again
    int32_t* la = c->w_list[0];
    int32_t* lb = c->w_list[1];
    // ctr[4] is still zero from the reset above; each refinement pass zeroes the
    // counter the following residual pass appends to
    MEM_HIP(c, launch_accurate3(c, n, c->w_list[3], &ctr[3], M, beta, p.tol_grad, la, &ctr[4], s));
    int ca = 4, cb = 5;
    for (int pass = 0; pass < refine; ++pass) {
      MEM_HIP(c, launch_refine3(c, n, la, &ctr[ca], M, beta, &ctr[cb], s));
      MEM_HIP(c, launch_accurate3(c, n, la, &ctr[ca], M, beta, p.tol_grad, lb, &ctr[cb], s));
      std::swap(la, lb);
      std::swap(ca, cb);
    }
    MEM_HIP(c, launch_refine_final(c, n, c->w_list[3], &ctr[3], p.tol_loose, resid, status, s));
  }
  return MEM_OK;
}


// Process-wide tuning results: key = (device architecture, dimension, nodes per
// axis, moments, precision, bit length of the cell count).  Contexts of the
// same kind on the same kind of device reuse a result instead of timing again.
struct TuneKey {
  std::string arch;
  int dim, n1d, K, prec, bits;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, dim, n1d, K, prec, bits) <
           std::tie(o.arch, o.dim, o.n1d, o.K, o.prec, o.bits);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, mem_tuning_t>& tune_cache() {
  static std::map<TuneKey, mem_tuning_t> m;
  return m;
}
TuneKey tune_key(mem_ctx_t c, int64_t n) {
  int bits = 0;
  while (bits < 63 && (int64_t(1) << bits) <= n) ++bits;
  return TuneKey{c->arch, c->dim, c->n1d, c->K, c->prec, bits};
}
}  // namespace

extern "C" {

const char* mem_strerror(mem_err_t e) {
  switch (e) {
    case MEM_OK: return "ok";
    case MEM_ERR_INVALID_ARG: return "invalid argument";
    case MEM_ERR_HIP: return "HIP runtime error";
    case MEM_ERR_NOMEM: return "device allocation failed";
    case MEM_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown error";
}

const char* mem_last_error(mem_ctx_t c) { return c ? c->err.c_str() : "null context"; }

void mem_solve_opts_default(mem_solve_opts_t* o) {
  if (!o) return;
  o->tol_grad = 2e-6f;
  o->tol_dec = 1e-8f;        // Alg. 1: tol
  o->tol_grad_loose = 1e-5f;
  o->max_iter = 400;         // Alg. 1: maxI
  o->max_ls = 25;            // Alg. 1: maxT
  o->armijo_c = 5e-4f;       // Alg. 1: ArmijoCondition
  o->atol = 5e-6f;
  o->rtol = 5e-5f;
  o->lambda0 = 1e-3f;        // Alg. 1: lambda
  o->lambda_mul = 10.f;
  o->alpha_min = 1e-6f;      // Alg. 1: convergence on the step size
  o->fp64_pivot_ratio = 1e-6f;
  o->check_every = 2;
  o->refine = 3;
  o->beta_max = 25.f;
}

mem_err_t mem_create(const mem_config_t* cfg, mem_ctx_t* out) {
  if (!cfg || !out) return MEM_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->reserved != 0) return MEM_ERR_INVALID_ARG;
  if (cfg->dim != 1 && cfg->dim != 3) return MEM_ERR_UNSUPPORTED;
  if (cfg->n_nodes_1d < 2 || cfg->n_nodes_1d > (cfg->dim == 1 ? Q1MAX : 32)) return MEM_ERR_UNSUPPORTED;
  if (cfg->prec < MEM_PREC_FP32 || cfg->prec > MEM_PREC_FP16X3) return MEM_ERR_UNSUPPORTED;
  if (cfg->dim == 1 && cfg->prec != MEM_PREC_FP32) return MEM_ERR_UNSUPPORTED;
  mem_ctx_t c = new (std::nothrow) mem_ctx_s;
  if (!c) return MEM_ERR_NOMEM;
  c->dim = cfg->dim;
  c->n1d = cfg->n_nodes_1d;
  c->prec = cfg->prec;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return MEM_ERR_HIP; }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) !=
          hipSuccess || c->n_cu <= 0)
    c->n_cu = 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->arch = prop.gcnArchName;
  }
  try {
    memt::build_tables(c);
  } catch (...) {
    mem_destroy(c);
    return MEM_ERR_NOMEM;
  }
  if (hipMalloc((void**)&c->w_ctr, 8 * sizeof(int32_t)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_ctr, sizeof(int32_t)) != hipSuccess) {
    mem_destroy(c);
    return MEM_ERR_NOMEM;
  }
  if (resolve_scratch(c->device, &c->scratch) != hipSuccess) {
    mem_destroy(c);
    return MEM_ERR_HIP;
  }
  *out = c;
  return MEM_OK;
}

mem_err_t mem_destroy(mem_ctx_t c) {
  if (!c) return MEM_ERR_INVALID_ARG;
  (void)hipDeviceSynchronize();
  free_workspace(c);
  free_problems(c);
  dfree(c->d_phiA); dfree(c->d_psi); dfree(c->d_psi5); dfree(c->d_psiF); dfree(c->d_ux_src);
  dfree(c->d_ux_w);
  dfree(c->d_tab1);
  dfree(c->d_t1);
  dfree(c->d_psi_hi); dfree(c->d_psi_lo); dfree(c->d_phiA_m); dfree(c->d_psiF_m);
  dfree(c->w_ctr);
  if (c->h_ctr) (void)hipHostFree(c->h_ctr);
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& ev : c->prof_pool) (void)hipEventDestroy(ev);
  delete c;
  return MEM_OK;
}

mem_err_t mem_reserve(mem_ctx_t c, int64_t max_cells, int32_t max_problems) {
  if (!c || max_cells < 0 || max_problems < 0) return MEM_ERR_INVALID_ARG;
  if (max_cells > (int64_t)INT32_MAX - 64) return fail(c, MEM_ERR_INVALID_ARG, "too many cells");
  if (c->dim == 1) return MEM_OK;
  (void)hipDeviceSynchronize();
  if (max_cells > c->cap_cells) {
    const size_t n = (size_t)max_cells;
    free_workspace(c);
    bool ok = dalloc(c->w_S, n * NCOL) && dalloc(c->w_S5, n * NC5) && dalloc(c->w_dbeta, n * 36) &&
              dalloc(c->w_logZ, n) && dalloc(c->w_L, n) && dalloc(c->w_alpha, n) &&
              dalloc(c->w_gdot, n) && dalloc(c->w_resid, n) && dalloc(c->w_iters, n) &&
              dalloc(c->w_status, n) && dalloc(c->w_list[0], n) && dalloc(c->w_list[1], n) &&
              dalloc(c->w_list[2], n) && dalloc(c->w_list[3], n) && dalloc(c->w_list[4], n) &&
              dalloc(c->w_Gacc, n * 36) &&
              dalloc(c->w_racc, n) && dalloc(c->w_rbest, n) && dalloc(c->w_itbest, n) &&
              dalloc(c->w_Mnew, n * K3) && dalloc(c->w_F, n * K3) &&
              dalloc(c->w_rho, n) && dalloc(c->w_prob, n) && dalloc(c->w_code, n) &&
              dalloc(c->w_Sp, (size_t)SP_ROWS * NCOL) && dalloc(c->w_hM, n * K3) &&
              dalloc(c->w_hB, n * K3) && dalloc(c->w_hG, n * 3) && dalloc(c->w_hF, n * K3) &&
              dalloc(c->w_hLF, n * K3) && dalloc(c->w_hPhi, n * K3) && dalloc(c->w_cond, n);
    if (!ok) { free_workspace(c); return fail(c, MEM_ERR_NOMEM, "workspace allocation"); }
    c->cap_cells = max_cells;
    c->sp_rows = SP_ROWS;
  }
  if (max_problems > c->cap_problems) {
    const size_t P = (size_t)max_problems;
    free_problems(c);
    bool ok = dalloc(c->w_gM, 2 * P * K3) && dalloc(c->w_gB, 2 * P * K3) && dalloc(c->w_gG, 2 * P * 3) &&
              dalloc(c->w_gF, 2 * P * K3) && dalloc(c->w_gR, 2 * P) && dalloc(c->w_rmax, P);
    if (!ok) { free_problems(c); return fail(c, MEM_ERR_NOMEM, "problem workspace allocation"); }
    c->cap_problems = max_problems;
  }
  return MEM_OK;
}

int32_t mem_n_basis(mem_ctx_t c) { return c ? c->K : -1; }
int32_t mem_n_nodes(mem_ctx_t c) { return c ? c->Q : -1; }

mem_err_t mem_copy_table(mem_ctx_t c, int32_t which, double* host_out, int64_t n_values,
                         int64_t* n_total) {
  if (!c) return MEM_ERR_INVALID_ARG;
  const std::vector<double>* v = which == 0 ? &c->h_nodes : which == 1 ? &c->h_w
                               : which == 2 ? &c->h_phi : nullptr;
  if (!v) return fail(c, MEM_ERR_INVALID_ARG, "table id");
  if (n_total) *n_total = (int64_t)v->size();
  if (host_out && n_values > 0)
    std::memcpy(host_out, v->data(), sizeof(double) * (size_t)std::min<int64_t>(n_values, v->size()));
  return MEM_OK;
}

mem_err_t mem_host_table(int32_t dim, int32_t n1d, int32_t which, double* host_out,
                         int64_t n_values, int64_t* n_total) {
  if ((dim != 1 && dim != 3) || n1d < 2 || n1d > (dim == 1 ? Q1MAX : 32) || which < 0 || which > 3)
    return MEM_ERR_INVALID_ARG;
  std::vector<double> nodes, w, logw, phi;
  int K = 0, Q = 0;
  memt::build_host(dim, n1d, nodes, w, logw, phi, K, Q);
  const std::vector<double>& v = which == 0 ? nodes : which == 1 ? w : which == 2 ? phi : logw;
  if (n_total) *n_total = (int64_t)v.size();
  if (host_out && n_values > 0)
    std::memcpy(host_out, v.data(), sizeof(double) * (size_t)std::min<int64_t>(n_values, v.size()));
  return MEM_OK;
}

mem_err_t mem_gauge(mem_ctx_t c, int64_t n, float* M, float* beta, float* g, hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (n < 0 || (n > 0 && (!M || !g))) return fail(c, MEM_ERR_INVALID_ARG, "mem_gauge: arguments");
  if (n == 0) return MEM_OK;
  MEM_HIP(c, c->dim == 1 ? launch_gauge1(c, n, M, beta, g, s) : launch_gauge3(c, n, M, beta, g, s));
  return MEM_OK;
}

mem_err_t mem_maxent_solve(mem_ctx_t c, int64_t n, const float* M, float* beta,
                           const mem_solve_opts_t* opts, int32_t* iters, float* resid,
                           uint32_t* status, hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (n < 0 || (n > 0 && (!M || !beta))) return fail(c, MEM_ERR_INVALID_ARG, "mem_maxent_solve: arguments");
  if (!opts_ok(opts)) return fail(c, MEM_ERR_INVALID_ARG, "mem_maxent_solve: options");
  if (n == 0) return MEM_OK;
  SolveParams p = params_from(opts);
  p.lmin = dual_floor(c);
  if (c->dim == 1) {
    p.refine = 0;
    MEM_HIP(c, launch_solve1(c, n, M, beta, p, iters, resid, status, s));
    return MEM_OK;
  }
  mem_err_t e = ensure_cells(c, n);
  if (e != MEM_OK) return e;
  mem_solve_opts_t d;
  mem_solve_opts_default(&d);
  const int poll = opts ? opts->check_every : d.check_every;
  const int refine = opts ? opts->refine : d.refine;
  p.refine = refine;
  return newton3(c, n, M, beta, p, p.max_iter, poll, refine, iters, resid, status, s, true);
}

mem_err_t mem_maxent_solve_noalloc(mem_ctx_t c, int64_t n, const float* M, float* beta,
                                   const mem_solve_opts_t* opts, int32_t* iters, float* resid,
                                   uint32_t* status, hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (n < 0 || (n > 0 && (!M || !beta)))
    return fail(c, MEM_ERR_INVALID_ARG, "mem_maxent_solve_noalloc: arguments");
  if (n > NOALLOC_MAX_CELLS)
    return fail(c, MEM_ERR_INVALID_ARG,
                "mem_maxent_solve_noalloc: at most " + std::to_string(NOALLOC_MAX_CELLS) +
                    " cells per call (static device scratch)");
  if (!opts_ok(opts)) return fail(c, MEM_ERR_INVALID_ARG, "mem_maxent_solve_noalloc: options");
  if (n == 0) return MEM_OK;
  SolveParams p = params_from(opts);
  p.lmin = dual_floor(c);
  if (c->dim == 1) {  // the 1D solve keeps its whole state in registers
    p.refine = 0;
    MEM_HIP(c, launch_solve1(c, n, M, beta, p, iters, resid, status, s));
    return MEM_OK;
  }
  if (!c->scratch) return fail(c, MEM_ERR_HIP, "mem_maxent_solve_noalloc: no device scratch");
  mem_solve_opts_t d;
  mem_solve_opts_default(&d);
  const int poll = opts ? opts->check_every : d.check_every;
  const int refine = opts ? opts->refine : d.refine;
  p.refine = refine;
  // point the Newton workspace at the scratch for this call, then put the
  // context's own workspace back (the kernels are those of mem_maxent_solve)
  NewtonWorkspace own = NewtonWorkspace::of(c);
  unsigned char* b = c->scratch;
  NewtonWorkspace w;
  w.S = reinterpret_cast<float*>(b + NOALLOC.S);
  w.dbeta = reinterpret_cast<float*>(b + NOALLOC.dbeta);
  w.logZ = reinterpret_cast<float*>(b + NOALLOC.logZ);
  w.L = reinterpret_cast<float*>(b + NOALLOC.L);
  w.alpha = reinterpret_cast<float*>(b + NOALLOC.alpha);
  w.gdot = reinterpret_cast<float*>(b + NOALLOC.gdot);
  w.resid = reinterpret_cast<float*>(b + NOALLOC.resid);
  w.iters = reinterpret_cast<int32_t*>(b + NOALLOC.iters);
  w.status = reinterpret_cast<uint32_t*>(b + NOALLOC.status);
  for (int k = 0; k < 5; ++k) w.list[k] = reinterpret_cast<int32_t*>(b + NOALLOC.list[k]);
  w.ctr = reinterpret_cast<int32_t*>(b + NOALLOC.ctr);
  w.code = reinterpret_cast<int8_t*>(b + NOALLOC.code);
  w.Sp = reinterpret_cast<float*>(b + NOALLOC.Sp);
  w.sp_rows = NOALLOC_SPLIT_ROWS;
  w.Gacc = reinterpret_cast<float*>(b + NOALLOC.Gacc);
  w.racc = reinterpret_cast<float*>(b + NOALLOC.racc);
  w.rbest = reinterpret_cast<float*>(b + NOALLOC.rbest);
  w.itbest = reinterpret_cast<int32_t*>(b + NOALLOC.itbest);
  w.prof = false;  // no host-side event bookkeeping
  w.install(c);
  const mem_err_t e = newton3(c, n, M, beta, p, p.max_iter, poll, refine, iters, resid, status,
                              s, true);
  own.install(c);
  return e;
}

mem_err_t mem_dual(mem_ctx_t c, int64_t n, const float* beta, float* logZ, float* E, float* H,
                   hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (c->dim != 3) return fail(c, MEM_ERR_UNSUPPORTED, "mem_dual: dim 3 only");
  if (n < 0 || (n > 0 && !beta)) return fail(c, MEM_ERR_INVALID_ARG, "mem_dual: arguments");
  if (n == 0) return MEM_OK;
  mem_err_t e = ensure_cells(c, n);
  if (e != MEM_OK) return e;
  SolveParams p = params_from(nullptr);
  float* b = const_cast<float*>(beta);
  MEM_HIP(c, launch_lse3(c, n, nullptr, nullptr, n, nullptr, b, false, p, nullptr, nullptr, s));
  if (c->prec == MEM_PREC_FP32)
    MEM_HIP(c, launch_assemble3(c, n, nullptr, nullptr, n, beta, c->d_psi, c->w_S, s));
  else
    MEM_HIP(c, launch_assemble3m(c, n, nullptr, nullptr, n, beta, c->w_S, s));
  if (logZ) MEM_HIP(c, launch_copy(n, c->w_logZ, logZ, s));
  if (E || H) MEM_HIP(c, launch_unpack3(c, n, E, H, s));
  return MEM_OK;
}

mem_err_t mem_moment_residual(mem_ctx_t c, int64_t n, const float* M, const float* beta,
                              float* G, hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (c->dim != 3) return fail(c, MEM_ERR_UNSUPPORTED, "mem_moment_residual: dim 3 only");
  if (n < 0 || (n > 0 && (!M || !beta || !G)))
    return fail(c, MEM_ERR_INVALID_ARG, "mem_moment_residual: arguments");
  if (n == 0) return MEM_OK;
  mem_err_t e = ensure_cells(c, n);
  if (e != MEM_OK) return e;
  SolveParams p = params_from(nullptr);
  // log Z in FP32 only shifts the exponent: the quotients E_k / E_0 cancel it
  MEM_HIP(c, launch_lse3(c, n, nullptr, nullptr, n, nullptr, const_cast<float*>(beta), false, p,
                         nullptr, nullptr, s));
  MEM_HIP(c, launch_moment_residual3(c, n, M, beta, G, s));
  return MEM_OK;
}

mem_err_t mem_flux(mem_ctx_t c, int64_t n, const float* beta, const float* g, float* F, float* lam,
                   hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (c->dim != 3) return fail(c, MEM_ERR_UNSUPPORTED, "mem_flux: dim 3 only");
  if (n < 0 || (n > 0 && (!beta || !g || (!F && !lam))))
    return fail(c, MEM_ERR_INVALID_ARG, "mem_flux: arguments");
  if (n == 0) return MEM_OK;
  mem_err_t e = ensure_cells(c, n);
  if (e != MEM_OK) return e;
  MEM_HIP(c, launch_flux3(c, n, beta, g, F, lam, lam != nullptr, false, nullptr, s));
  return MEM_OK;
}

mem_err_t mem_collide(mem_ctx_t c, int64_t n, float* M, const float* g, float h, float prandtl,
                      float mu_ref, hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (c->dim != 3) return fail(c, MEM_ERR_UNSUPPORTED, "mem_collide: dim 3 only");
  if (n < 0 || (n > 0 && (!M || !g)) || !(prandtl > 0.5f) || !(mu_ref > 0.f) || !(h >= 0.f))
    return fail(c, MEM_ERR_INVALID_ARG, "mem_collide: arguments");
  if (n == 0) return MEM_OK;
  MEM_HIP(c, launch_collide3(c, n, M, g, h, nullptr, nullptr, prandtl, mu_ref, s));
  return MEM_OK;
}

// Validates the host fields and the device cell offsets (copied to the host:
// every kernel indexes neighbours and problems through them).
// Field and offset checks on every call: the step kernels index neighbours
// through the offsets, so they are read back (ordered on the caller's stream)
// each time rather than trusted from an earlier call with the same pointer.
static mem_err_t check_batch(mem_ctx_t c, const mem_batch_t* b, hipStream_t s) {
  if (!b || b->n_problems <= 0 || b->n_cells < b->n_problems || !b->cell_offsets || !b->dx ||
      !b->M_left || !b->M_right || !b->g_left || !b->g_right || !(b->cfl > 0.f) ||
      !(b->prandtl > 0.5f) || !(b->mu_ref > 0.f) || b->newton_per_step < 1 ||
      b->newton_per_step > 1000 || (b->collision != 0 && b->collision != 1) ||
      (b->use_graph != 0 && b->use_graph != 1) || b->flux_scheme < MEM_FLUX_LLF ||
      b->flux_scheme > MEM_FLUX_FLIC)
    return fail(c, MEM_ERR_INVALID_ARG, "mem_batch_t");
  std::vector<int64_t> off((size_t)b->n_problems + 1);
  MEM_HIP(c, hipMemcpyAsync(off.data(), b->cell_offsets, off.size() * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
  MEM_HIP(c, hipStreamSynchronize(s));
  if (off[0] != 0 || off.back() != b->n_cells)
    return fail(c, MEM_ERR_INVALID_ARG, "cell_offsets must start at 0 and end at n_cells");
  for (size_t p = 0; p + 1 < off.size(); ++p)
    if (off[p + 1] <= off[p]) return fail(c, MEM_ERR_INVALID_ARG, "every problem needs >= 1 cell");
  return MEM_OK;
}

mem_err_t mem_step(mem_ctx_t c, const mem_batch_t* b, float* M, float* beta, float* g, float* t,
                   float* dt, int32_t n_steps, const mem_solve_opts_t* opts, uint32_t* status,
                   hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (c->dim != 3) return fail(c, MEM_ERR_UNSUPPORTED, "mem_step: dim 3 only");
  mem_err_t e = check_batch(c, b, s);
  if (e != MEM_OK) return e;
  if (!M || !beta || !g || !t || !dt || n_steps < 0 || !opts_ok(opts))
    return fail(c, MEM_ERR_INVALID_ARG, "mem_step: arguments");
  const int64_t n = b->n_cells;
  const int P = b->n_problems;
  // rows for the cells, the 2P ghosts and the n + P interfaces (n >= P)
  if (n + P > c->cap_cells || P > c->cap_problems) {
    e = mem_reserve(c, std::max<int64_t>(n + P, c->cap_cells), std::max(P, c->cap_problems));
    if (e != MEM_OK) return e;
  }
  SolveParams p = params_from(opts);
  p.lmin = dual_floor(c);
  const int budget = b->newton_per_step;
  p.max_iter = budget;
  const float Pr = b->collision == 1 ? b->prandtl : 1.f;
  // batch set-up: cell -> problem map, ghost states (solved once), running max
  MEM_HIP(c, launch_prob_map(c, b->cell_offsets, P, c->w_prob, s));
  MEM_HIP(c, launch_ghost_pack(c, b, s));
  mem_solve_opts_t dflt;
  mem_solve_opts_default(&dflt);
  const int refine = opts ? opts->refine : dflt.refine;
  p.refine = refine;
  e = newton3(c, 2 * (int64_t)P, c->w_gM, c->w_gB, p, budget, 0, refine, nullptr, nullptr, nullptr, s,
              true);
  if (e != MEM_OK) return e;
  MEM_HIP(c, launch_flux3(c, 2 * (int64_t)P, c->w_gB, c->w_gG, c->w_gF, c->w_gR, true, true, nullptr, s));
  MEM_HIP(c, launch_rmax_init(c, P, s));
  // solve the current state; set dt where the caller asked for one
  e = newton3(c, n, M, beta, p, budget, 0, refine, nullptr, nullptr, nullptr, s, true);
  if (e != MEM_OK) return e;
  MEM_HIP(c, launch_maxwell_fallback(c, n, M, beta, s));
  MEM_HIP(c, launch_flux3(c, n, beta, g, nullptr, c->w_rho, true, true, status, s));
  MEM_HIP(c, launch_rho_max(c, n, c->w_rho, c->w_prob, P, s));
  MEM_HIP(c, launch_dt_update(c, P, b->dx, b->cfl, t, dt, false, s));
  // one step of Alg. 2 on stream st (no host synchronisation inside)
  auto step_once = [&](hipStream_t st) -> mem_err_t {
    MEM_HIP(c, launch_collide3(c, n, M, g, 0.f, dt, c->w_prob, Pr, b->mu_ref, st));
    mem_err_t er = newton3(c, n, M, beta, p, budget, 0, refine, nullptr, nullptr, nullptr, st);
    if (er != MEM_OK) return er;
    MEM_HIP(c, launch_maxwell_fallback(c, n, M, beta, st));
    if (status) MEM_HIP(c, launch_status_or(n, c->w_status, status, st));
    if (b->iter_hist) MEM_HIP(c, launch_iter_hist(n, c->w_iters, budget + 1, b->iter_hist, st));
    if (b->status_counts) MEM_HIP(c, launch_status_count(n, c->w_status, b->status_counts, st));
    MEM_HIP(c, launch_flux3(c, n, beta, g, c->w_F, c->w_rho, true, true, status, st));
    if (b->cond_max) {  // the monitor, on the S rows the flux pass left at the solutions
      MEM_HIP(c, launch_cond3(c, n, c->w_cond, st));
      MEM_HIP(c, launch_cond_max(n, c->w_cond, c->w_prob, b->cond_max, st));
    }
    MEM_HIP(c, launch_rho_max(c, n, c->w_rho, c->w_prob, P, st));
    // the transport step never exceeds the CFL limit of its own speeds
    MEM_HIP(c, launch_dt_cap(c, P, b->dx, b->cfl, dt, st));
    if (b->flux_scheme == MEM_FLUX_LLF) {
      MEM_HIP(c, launch_fv3(c, n, M, c->w_F, c->w_rho, g, c->w_prob, b->cell_offsets, b->dx, dt,
                            c->w_Mnew, P, st));
    } else {
      // second order: half-step interface states, their MaxEnt solve (from the
      // right element's beta), the flux of that solution, then the update
      const bool flic = b->flux_scheme == MEM_FLUX_FLIC;
      const int64_t ni = n + P;
      MEM_HIP(c, launch_iface3(c, n, P, M, c->w_F, beta, c->w_rho, g, c->w_prob, b->cell_offsets,
                               b->dx, dt, flic, st));
      er = newton3(c, ni, c->w_hM, c->w_hB, p, budget, 0, refine, nullptr, nullptr, nullptr, st);
      if (er != MEM_OK) return er;
      MEM_HIP(c, launch_flux3(c, ni, c->w_hB, c->w_hG, c->w_hF, nullptr, false, false, nullptr, st));
      MEM_HIP(c, launch_fv3i(c, n, M, g, c->w_prob, b->cell_offsets, b->dx, dt, flic, c->w_Mnew,
                             st));
    }
    MEM_HIP(c, launch_collide3(c, n, c->w_Mnew, g, 0.f, dt, c->w_prob, Pr, b->mu_ref, st));
    MEM_HIP(c, launch_gauge3(c, n, c->w_Mnew, beta, g, st));
    MEM_HIP(c, launch_copy(n * K3, c->w_Mnew, M, st));
    MEM_HIP(c, launch_dt_update(c, P, b->dx, b->cfl, t, dt, true, st));
    return MEM_OK;
  };
  if (!b->use_graph || n_steps == 0) {
    for (int step = 0; step < n_steps; ++step) {
      e = step_once(s);
      if (e != MEM_OK) return e;
    }
    return MEM_OK;
  }
  // graph path: capture one step on the private stream (kernels only: no
  // memset or copy nodes), keep it while every pointer and option is the same
  StepKey key{};
  key.b = *b;
  key.M = M; key.beta = beta; key.g = g; key.t = t; key.dt = dt; key.status = status;
  key.p = p; key.refine = refine;
  key.gen = c->ws_gen;
  if (!c->step_exec || std::memcmp(&key, &c->step_key, sizeof(key)) != 0) {
    if (c->step_exec) { (void)hipGraphExecDestroy(c->step_exec); c->step_exec = nullptr; }
    if (!c->cap_stream) MEM_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const bool prof = c->prof;
    c->prof = false;  // no event nodes in the graph
    MEM_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    e = step_once(c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t he = hipStreamEndCapture(c->cap_stream, &graph);
    c->prof = prof;
    if (e != MEM_OK) { if (graph) (void)hipGraphDestroy(graph); return e; }
    if (he != hipSuccess) return fail(c, MEM_ERR_HIP, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&c->step_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) { c->step_exec = nullptr; return fail(c, MEM_ERR_HIP, "hipGraphInstantiate"); }
    c->step_key = key;
  }
  for (int step = 0; step < n_steps; ++step) MEM_HIP(c, hipGraphLaunch(c->step_exec, s));
  return MEM_OK;
}

mem_err_t mem_conserved(mem_ctx_t c, const mem_batch_t* b, const float* M, const float* g,
                        double* out, hipStream_t s) {
  if (!c) return MEM_ERR_INVALID_ARG;
  if (c->dim != 3) return fail(c, MEM_ERR_UNSUPPORTED, "mem_conserved: dim 3 only");
  mem_err_t e = check_batch(c, b, s);
  if (e != MEM_OK) return e;
  if (!M || !g || !out) return fail(c, MEM_ERR_INVALID_ARG, "mem_conserved: arguments");
  MEM_HIP(c, launch_conserved(c, b, M, g, out, s));
  return MEM_OK;
}

mem_err_t mem_get_tuning(mem_ctx_t c, mem_tuning_t* out) {
  if (!c || !out) return MEM_ERR_INVALID_ARG;
  *out = c->tune;
  return MEM_OK;
}

mem_err_t mem_set_tuning(mem_ctx_t c, const mem_tuning_t* in) {
  if (!c || !in) return MEM_ERR_INVALID_ARG;
  const int wpc = in->wave_per_cu, aw = in->asm_waves;
  if ((in->dir_waves != 2 && in->dir_waves != 4 && in->dir_waves != 8) || in->split_want < 0 ||
      in->split_want > 65536 || (in->solver != 0 && in->solver != 1) || in->wave_max_cells < 0 ||
      (wpc != 0 && wpc != 4 && wpc != 8 && wpc != 12) || (aw != 0 && aw != 4 && aw != 8))
    return fail(c, MEM_ERR_INVALID_ARG,
                "mem_set_tuning: dir_waves in {2,4,8}, split_want in [0, 65536], solver 0 or 1, "
                "wave_max_cells >= 0, wave_per_cu in {0,4,8,12}, asm_waves in {0,4,8}");
  c->tune = *in;
  if (c->tune.wave_per_cu == 0) c->tune.wave_per_cu = WAVE_SOLVE_PER_CU;
  if (c->tune.asm_waves == 0) c->tune.asm_waves = 4;
  c->tune.cached = 0;
  ++c->ws_gen;
  return MEM_OK;
}

void mem_tuning_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache().clear();
}

mem_err_t mem_autotune(mem_ctx_t c, int64_t n, const float* M, const float* beta_init,
                       float* beta_work, const mem_solve_opts_t* opts, mem_tuning_t* out,
                       hipStream_t s) {
  if (!c || n <= 0 || !M || !beta_init || !beta_work) return MEM_ERR_INVALID_ARG;
  if (!opts_ok(opts)) return fail(c, MEM_ERR_INVALID_ARG, "mem_autotune: options");
  if (c->dim != 3) {  // the 1D solver has no launch parameters
    if (out) *out = c->tune;
    return MEM_OK;
  }
  const TuneKey key = tune_key(c, n);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      c->tune = it->second;
      c->tune.cached = 1;
      ++c->ws_gen;
      if (out) *out = c->tune;
      return MEM_OK;
    }
  }
  mem_err_t e = ensure_cells(c, n);
  if (e != MEM_OK) return e;
  hipEvent_t ev[2] = {nullptr, nullptr};
  MEM_HIP(c, hipEventCreate(&ev[0]));
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(c, MEM_ERR_HIP, "hipEventCreate");
  }
  const size_t bytes = (size_t)n * K3 * sizeof(float);
  // one warm run, then the faster of two timed runs
  auto trial = [&](const mem_tuning_t& t, double& ms) -> mem_err_t {
    c->tune = t;
    ms = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      MEM_HIP(c, hipMemcpyAsync(beta_work, beta_init, bytes, hipMemcpyDeviceToDevice, s));
      MEM_HIP(c, hipEventRecord(ev[0], s));
      mem_err_t r = mem_maxent_solve(c, n, M, beta_work, opts, nullptr, nullptr, nullptr, s);
      if (r != MEM_OK) return r;
      MEM_HIP(c, hipEventRecord(ev[1], s));
      MEM_HIP(c, hipEventSynchronize(ev[1]));
      float x = 0.f;
      MEM_HIP(c, hipEventElapsedTime(&x, ev[0], ev[1]));
      if (rep > 0) ms = std::min(ms, (double)x);
    }
    return MEM_OK;
  };
  // the search starts from the defaults, so a result does not depend on what
  // the context held before
  mem_tuning_t best = TUNE_DEFAULT;
  double best_ms = 1e30;
  // one coordinate at a time: each candidate value of the field, the others
  // at the best so far
  auto sweep = [&](std::initializer_list<int> vals, int32_t mem_tuning_t::*field) {
    for (int v : vals) {
      if (e != MEM_OK) return;
      mem_tuning_t t = best;
      t.*field = v;
      double ms = 0.0;
      if ((e = trial(t, ms)) != MEM_OK) return;
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
  };
  // the Newton loop first: the persistent kernel (when it applies) or the
  // list-compacted passes, whose launch shapes are tuned next
  best.wave_max_cells = 0;
  if (c->prec == MEM_PREC_FP32 && c->n1d == 12)
    sweep({1, 0}, &mem_tuning_t::solver);
  else
    best.solver = 0;
  if (best.solver == 1) {
    sweep({12, 8, 4}, &mem_tuning_t::wave_per_cu);
  } else {
    sweep({2, 4, 8}, &mem_tuning_t::dir_waves);
    if (c->prec == MEM_PREC_FP32) sweep({4, 8}, &mem_tuning_t::asm_waves);
    sweep({0, 256, 512, 1024, 2048}, &mem_tuning_t::split_want);
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  best.tuned_ms = best_ms;
  c->tune = best;
  ++c->ws_gen;
  if (e == MEM_OK) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache()[key] = best;
  }
  if (out) *out = best;
  return e;
}

mem_err_t mem_profile_enable(mem_ctx_t c, int32_t enable) {
  if (!c) return MEM_ERR_INVALID_ARG;
  c->prof = enable != 0;
  if (c->prof) {
    if (c->prof_pool.empty()) {
      c->prof_pool.resize(8192);
      for (auto& ev : c->prof_pool)
        if (hipEventCreate(&ev) != hipSuccess) return fail(c, MEM_ERR_HIP, "hipEventCreate");
    }
    MEM_HIP(c, hipDeviceSynchronize());
    c->prof_used = 0;
    c->prof_marks.clear();
  }
  return MEM_OK;
}

mem_err_t mem_profile_read(mem_ctx_t c, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!c) return MEM_ERR_INVALID_ARG;
  double ms = 0.0;
  int64_t cnt = 0;
  for (auto& m : c->prof_marks) {
    if (m.first != kernel) continue;
    MEM_HIP(c, hipEventSynchronize(m.second.second));
    float x = 0.f;
    MEM_HIP(c, hipEventElapsedTime(&x, m.second.first, m.second.second));
    ms += x;
    ++cnt;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = cnt;
  return MEM_OK;
}

}  // extern "C"
