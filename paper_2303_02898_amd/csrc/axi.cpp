// C ABI of the nine-statistic discretisation: block-wise Gauss--Legendre rule
// on a box fixed in physical velocity (end of Sec. 3.1), the integration-domain
// formula of the normal-shock set-up, and the solve / moment entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "mem_internal.h"

using namespace memk;

struct mem_axi_s {
  mem_axi_rule_t rule;
  int64_t P = 0;
  std::vector<double> ux, ur, logw;
  float4* d_tab = nullptr;  // (u_x, u_r, log w, u_x - fl(u_x)) per node, then lo parts
  float lmin = 0.f;
  float ux_min = 0.f, ux_max = 0.f;  // node span in u_x
  // time-step workspace (mem_axi_step, mem_axi_step_batch) for up to cap cells
  // in up to cap_p problems, grown on demand
  int64_t cap = 0;
  int32_t cap_p = 0;
  float *w_F = nullptr, *w_lam = nullptr, *w_Mn = nullptr, *w_gh = nullptr, *w_scal = nullptr;
  uint32_t* w_st = nullptr;
  // interface rows (n + P): F_LF, half-step state, gauge, multipliers, limiter,
  // F_LW, status
  float *w_fLF = nullptr, *w_Mh = nullptr, *w_gI = nullptr, *w_bI = nullptr, *w_phi = nullptr,
        *w_fLW = nullptr;
  uint32_t* w_stI = nullptr;
  int32_t *w_pid = nullptr, *w_pidI = nullptr;  // problem of each cell / interface row
  float* w_cond = nullptr;  // per-cell pivot ratios of the last solve (monitor)
  // descriptors of a single problem (mem_axi_step): offsets {0, n}, dx, ghosts
  int64_t* w_off1 = nullptr;
  float *w_dx1 = nullptr, *w_gs1 = nullptr;
  // the last batch whose offsets were read back and checked
  const int64_t* v_off = nullptr;
  int64_t v_n = -1;
  int32_t v_P = -1;
  // captured step (use_graph): valid while the key matches
  struct StepKey {
    mem_axi_batch_t b;
    float *M, *beta, *g, *t, *dt;
    uint32_t* status;
    memk::SolveParams p;
    uint64_t gen;
  };
  uint64_t gen = 0;  // bumped whenever the workspace is reallocated
  StepKey key{};
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
};

namespace {

// Gauss--Legendre nodes and weights on [-1, 1]: Newton's method on P_n from
// the Chebyshev-like start cos(pi (i + 3/4) / (n + 1/2)), with P_n and P_n'
// from the three-term recurrence (n + 1) P_{n+1} = (2n + 1) x P_n - n P_{n-1};
// w_i = 2 / ((1 - x_i^2) P_n'(x_i)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int iter = 0; iter < 100; ++iter) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {  // derivative at the converged node
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = wi;
    w[n - 1 - i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

bool rule_ok(const mem_axi_rule_t* r) {
  return r && std::isfinite(r->ux_lo) && std::isfinite(r->ux_hi) && std::isfinite(r->ur_hi) &&
         r->ux_hi > r->ux_lo && r->ur_hi > 0.0 && r->blocks_x >= 1 && r->blocks_x <= 256 &&
         r->blocks_r >= 1 && r->blocks_r <= 256 && r->order >= 1 && r->order <= 32 &&
         r->reserved == 0 &&
         (int64_t)r->blocks_x * r->blocks_r * r->order * r->order <= (int64_t)1 << 22;
}

// nodes: blocks in x (outer), blocks in r, Gauss--Legendre points in x, in r;
// weight 2 pi u_r hx hr wx wr (the angle integrated exactly)
void build_rule(const mem_axi_rule_t& r, std::vector<double>& ux, std::vector<double>& ur,
                std::vector<double>& logw) {
  std::vector<double> gx, gw;
  gauss_legendre(r.order, gx, gw);
  const double hx = 0.5 * (r.ux_hi - r.ux_lo) / r.blocks_x;
  const double hr = 0.5 * r.ur_hi / r.blocks_r;
  const double two_pi = 6.28318530717958647692;
  ux.clear(); ur.clear(); logw.clear();
  for (int bx = 0; bx < r.blocks_x; ++bx) {
    const double cx = r.ux_lo + (2 * bx + 1) * hx;
    for (int br = 0; br < r.blocks_r; ++br) {
      const double cr = (2 * br + 1) * hr;
      for (int i = 0; i < r.order; ++i)
        for (int j = 0; j < r.order; ++j) {
          const double vr = cr + hr * gx[j];
          ux.push_back(cx + hx * gx[i]);
          ur.push_back(vr);
          logw.push_back(std::log(two_pi * vr * hx * hr * gw[i] * gw[j]));
        }
    }
  }
}

mem_err_t params_axi(const mem_axi_s* h, const mem_solve_opts_t* o, SolveParams& p) {
  mem_solve_opts_t d;
  mem_solve_opts_default(&d);
  if (!o) o = &d;
  if (o->max_iter < 1 || o->max_iter > 100000 || o->max_ls < 0 || o->max_ls > 60 ||
      !(o->lambda0 > 0.f) || !(o->lambda_mul > 1.f) || !(o->fp64_pivot_ratio >= 0.f) ||
      !(o->fp64_pivot_ratio < 1.f) || !std::isfinite(o->tol_grad) || !(o->beta_max >= 0.f) ||
      o->refine < 0 || o->refine > 8)
    return MEM_ERR_INVALID_ARG;
  p.tol_grad = o->tol_grad; p.tol_dec = o->tol_dec; p.tol_loose = o->tol_grad_loose;
  p.max_iter = o->max_iter; p.max_ls = o->max_ls;
  p.c = o->armijo_c; p.atol = o->atol; p.rtol = o->rtol;
  p.lambda0 = o->lambda0; p.lambda_mul = o->lambda_mul; p.alpha_min = o->alpha_min;
  p.fp64_ratio = o->fp64_pivot_ratio;
  p.beta_max = o->beta_max;
  p.lmin = h->lmin;
  p.refine = o->refine;
  p.stall_window = 0;
  return MEM_OK;
}

}  // namespace

extern "C" {

mem_err_t mem_axi_domain(double v_minus, double T_minus, double v_plus, double T_plus,
                         int32_t n_a, int32_t n_b, int32_t n_r, double* box) {
  if (!box || !(T_minus > 0.0) || !(T_plus > 0.0) || !std::isfinite(v_minus) ||
      !std::isfinite(v_plus) || !std::isfinite(T_minus) || !std::isfinite(T_plus) || n_a < 0 ||
      n_b < 0 || n_r < 1)
    return MEM_ERR_INVALID_ARG;
  const double sm = std::sqrt(T_minus), sp = std::sqrt(T_plus);
  box[0] = std::min(v_plus - n_a * sp, v_minus - n_a * sm);
  box[1] = std::max(v_minus + n_b * sm, v_plus + n_b * sp);
  box[2] = std::max(n_r * sm, n_r * sp);
  return MEM_OK;
}

int64_t mem_axi_rule_nodes(const mem_axi_rule_t* rule) {
  if (!rule_ok(rule)) return -1;
  return (int64_t)rule->blocks_x * rule->blocks_r * rule->order * rule->order;
}

mem_err_t mem_axi_host_rule(const mem_axi_rule_t* rule, double* ux, double* ur, double* logw,
                            int64_t n_nodes) {
  if (!rule_ok(rule)) return MEM_ERR_INVALID_ARG;
  if (n_nodes != mem_axi_rule_nodes(rule)) return MEM_ERR_INVALID_ARG;
  std::vector<double> a, b, c;
  build_rule(*rule, a, b, c);
  if (ux) std::copy(a.begin(), a.end(), ux);
  if (ur) std::copy(b.begin(), b.end(), ur);
  if (logw) std::copy(c.begin(), c.end(), logw);
  return MEM_OK;
}

mem_err_t mem_axi_create(const mem_axi_rule_t* rule, mem_axi_t* out) {
  if (!out) return MEM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!rule_ok(rule)) return MEM_ERR_INVALID_ARG;
  mem_axi_s* h = new (std::nothrow) mem_axi_s;
  if (!h) return MEM_ERR_NOMEM;
  h->rule = *rule;
  try {
    build_rule(*rule, h->ux, h->ur, h->logw);
  } catch (...) {
    delete h;
    return MEM_ERR_NOMEM;
  }
  h->P = (int64_t)h->ux.size();
  // P entries (u_x, u_r, log w, u_x - fl(u_x)), then P / 2 float4 holding the
  // pairs (u_r - fl(u_r), log w - fl(log w)) of the compensated residual pass
  std::vector<float4> tab(h->P + (h->P + 1) / 2, make_float4(0.f, 0.f, 0.f, 0.f));
  float* lo = reinterpret_cast<float*>(tab.data() + h->P);
  double mn = 1e300;
  for (int64_t q = 0; q < h->P; ++q) {
    const float hi = (float)h->ux[q];
    const float ur = (float)h->ur[q], lw = (float)h->logw[q];
    tab[q] = make_float4(hi, ur, lw, (float)(h->ux[q] - (double)hi));
    lo[2 * q] = (float)(h->ur[q] - (double)ur);
    lo[2 * q + 1] = (float)(h->logw[q] - (double)lw);
    mn = std::min(mn, h->logw[q]);
  }
  h->ux_min = (float)*std::min_element(h->ux.begin(), h->ux.end());
  h->ux_max = (float)*std::max_element(h->ux.begin(), h->ux.end());
  // a dual value below min_p log w_p certifies that no minimiser exists
  h->lmin = (float)(mn - 1e-3 * (1.0 + std::fabs(mn)));
  if (hipMalloc((void**)&h->d_tab, tab.size() * sizeof(float4)) != hipSuccess) {
    delete h;
    return MEM_ERR_NOMEM;
  }
  if (hipMemcpy(h->d_tab, tab.data(), tab.size() * sizeof(float4), hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(h->d_tab);
    delete h;
    return MEM_ERR_HIP;
  }
  *out = h;
  return MEM_OK;
}

void free_step(mem_axi_s* h) {
  if (h->exec) { (void)hipGraphExecDestroy(h->exec); h->exec = nullptr; }
  ++h->gen;
  for (float** p : {&h->w_F, &h->w_lam, &h->w_Mn, &h->w_gh, &h->w_scal, &h->w_fLF, &h->w_Mh,
                    &h->w_gI, &h->w_bI, &h->w_phi, &h->w_fLW, &h->w_dx1, &h->w_gs1, &h->w_cond})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  for (uint32_t** p : {&h->w_st, &h->w_stI})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  for (int32_t** p : {&h->w_pid, &h->w_pidI})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  if (h->w_off1) { (void)hipFree(h->w_off1); h->w_off1 = nullptr; }
  h->cap = 0;
  h->cap_p = 0;
}

mem_err_t mem_axi_destroy(mem_axi_t h) {
  if (!h) return MEM_ERR_INVALID_ARG;
  (void)hipDeviceSynchronize();
  free_step(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->d_tab) (void)hipFree(h->d_tab);
  delete h;
  return MEM_OK;
}

mem_err_t mem_axi_reserve_batch(mem_axi_t h, int64_t n, int32_t np) {
  if (!h || n < 1 || n > (int64_t)1 << 24 || np < 1 || np > n) return MEM_ERR_INVALID_ARG;
  if (n <= h->cap && np <= h->cap_p) return MEM_OK;
  n = std::max(n, h->cap);
  np = std::max(np, h->cap_p);
  if (hipDeviceSynchronize() != hipSuccess) return MEM_ERR_HIP;
  free_step(h);
  const int64_t ni = n + np;  // interface rows
  auto fl = [](float*& p, int64_t count) {
    return hipMalloc((void**)&p, (size_t)count * sizeof(float)) == hipSuccess;
  };
  auto u32 = [](uint32_t*& p, int64_t count) {
    return hipMalloc((void**)&p, (size_t)count * sizeof(uint32_t)) == hipSuccess;
  };
  auto i32 = [](int32_t*& p, int64_t count) {
    return hipMalloc((void**)&p, (size_t)count * sizeof(int32_t)) == hipSuccess;
  };
  if (!fl(h->w_F, n * 9) || !fl(h->w_lam, n * 2) || !fl(h->w_Mn, n * 9) ||
      !fl(h->w_gh, 64 * (int64_t)np) || !fl(h->w_scal, 2 * (int64_t)np) || !u32(h->w_st, n) ||
      !fl(h->w_fLF, ni * 9) || !fl(h->w_Mh, ni * 9) || !fl(h->w_gI, ni * 3) ||
      !fl(h->w_bI, ni * 9) || !fl(h->w_phi, ni * 9) || !fl(h->w_fLW, ni * 9) ||
      !u32(h->w_stI, ni) || !i32(h->w_pid, n) || !i32(h->w_pidI, ni) || !fl(h->w_dx1, 1) ||
      !fl(h->w_cond, n) ||
      !fl(h->w_gs1, 6) ||
      hipMalloc((void**)&h->w_off1, 2 * sizeof(int64_t)) != hipSuccess) {
    free_step(h);
    return MEM_ERR_NOMEM;
  }
  h->cap = n;
  h->cap_p = np;
  return MEM_OK;
}

mem_err_t mem_axi_reserve(mem_axi_t h, int64_t n) { return mem_axi_reserve_batch(h, n, 1); }

int64_t mem_axi_n_nodes(mem_axi_t h) { return h ? h->P : -1; }

mem_err_t mem_axi_solve(mem_axi_t h, int64_t n, const float* M, const float* g, float* beta,
                        const mem_solve_opts_t* opts, int32_t* iters, float* resid,
                        uint32_t* status, hipStream_t s) {
  if (!h || n < 0 || n > (int64_t)INT32_MAX - 4) return MEM_ERR_INVALID_ARG;
  if (n == 0) return MEM_OK;
  if (!M || !g || !beta) return MEM_ERR_INVALID_ARG;
  SolveParams p;
  if (params_axi(h, opts, p) != MEM_OK) return MEM_ERR_INVALID_ARG;
  if (launch_axi_solve(n, (int)h->P, h->d_tab, M, g, beta, p, iters, resid, status, s) !=
      hipSuccess)
    return MEM_ERR_HIP;
  return MEM_OK;
}

mem_err_t mem_axi_speeds(mem_axi_t h, int64_t n, const float* beta, const float* g, float* lam,
                         hipStream_t s) {
  if (!h || n < 0 || n > (int64_t)INT32_MAX - 4) return MEM_ERR_INVALID_ARG;
  if (n == 0) return MEM_OK;
  if (!beta || !g || !lam) return MEM_ERR_INVALID_ARG;
  return launch_axi_speeds(n, (int)h->P, h->d_tab, beta, g, h->ux_min, h->ux_max, lam, s) ==
                 hipSuccess
             ? MEM_OK
             : MEM_ERR_HIP;
}

#define AXI_HIP(x)                                     \
  do {                                                 \
    if ((x) != hipSuccess) return MEM_ERR_HIP;         \
  } while (0)

}  // extern "C"

namespace {

// Alg. 2 on the nine statistics for a batch of normal-shock problems whose
// descriptors are on the device (see mem.h).  bd: the batch as the caller
// gave it (or the single problem's descriptors); gs: its ghost states.
// Ghost rows: gh = [M 2Px9 | beta 2Px9 | g 2Px3 | F 2Px9 | lam 2Px2].
mem_err_t axi_steps(mem_axi_t h, const mem_axi_batch_t& bd, float* M, float* beta, float* g,
                    float* t, float* dt, int32_t n_steps, const SolveParams& p, uint32_t* status,
                    hipStream_t s) {
  const int64_t n = bd.n_cells;
  const int np = bd.n_problems;
  float* gM = h->w_gh;
  float* gB = gM + 18 * np;
  float* gG = gB + 18 * np;
  float* gF = gG + 6 * np;
  float* gL = gF + 18 * np;
  const AxBatch b{n, np, bd.cell_offsets, h->w_pid, h->w_pidI, bd.dx};
  // problem maps, and the ghost Maxwellians in their own Hermite gauges: the
  // discrete moments, fluxes and speeds of beta = (n, 0, -1/sqrt2, -1, 0, ...)
  AXI_HIP(launch_axi_prologue(b, bd.ghosts, h->w_pid, h->w_pidI, gB, gG, s));
  AXI_HIP(launch_axi_moments(2 * np, (int)h->P, h->d_tab, gB, gG, gM, gF, s));
  AXI_HIP(launch_axi_speeds(2 * np, (int)h->P, h->d_tab, gB, gG, h->ux_min, h->ux_max, gL, s));
  uint32_t* st = status ? status : h->w_st;
  const int tpb = (int)h->P;
  // the per-step solves start from the previous step's multipliers: a cell
  // that does not halve its residual below the stall gate within 6 iterations
  // sits at its FP32 floor (the set-up solve keeps the longer default window)
  SolveParams pw = p;
  pw.stall_window = 6;
  if (n_steps == 0) {  // set-up: the solve of the initial state and its dt
    AXI_HIP(launch_axi_solve(n, tpb, h->d_tab, M, g, beta, p, nullptr, nullptr, st, s));
    AXI_HIP(launch_axi_fix(n, M, beta, st, s));
    AXI_HIP(launch_axi_speeds(n, tpb, h->d_tab, beta, g, h->ux_min, h->ux_max, h->w_lam, s));
    AXI_HIP(launch_axi_dt(b, h->w_lam, gL, bd.cfl, dt, h->w_scal, 1, s));
    return MEM_OK;
  }
  // one step of Alg. 2 on stream q (kernels only: it may be captured)
  auto step_once = [&](hipStream_t q) -> mem_err_t {
    AXI_HIP(launch_axi_collide(b, M, g, dt, 1, 0.5f, bd.prandtl, bd.mu_ref, q));
    AXI_HIP(launch_axi_solve(n, tpb, h->d_tab, M, g, beta, pw, nullptr, nullptr, st, q,
                             bd.cond_max ? h->w_cond : nullptr));
    if (bd.cond_max) AXI_HIP(launch_axi_cond_max(b, h->w_cond, bd.cond_max, q));
    AXI_HIP(launch_axi_fix(n, M, beta, st, q));
    AXI_HIP(launch_axi_moments(n, tpb, h->d_tab, beta, g, nullptr, h->w_F, q));
    AXI_HIP(launch_axi_speeds(n, tpb, h->d_tab, beta, g, h->ux_min, h->ux_max, h->w_lam, q));
    AXI_HIP(launch_axi_dt(b, h->w_lam, gL, bd.cfl, dt, h->w_scal, 0, q));
    if (bd.scheme == MEM_FLUX_LLF) {
      AXI_HIP(launch_axi_fv(b, M, h->w_F, h->w_lam, g, gM, gF, gL, gG, h->w_scal, h->w_Mn, q));
    } else {  // one MaxEnt solve per interface, in the right element's gauge
      AXI_HIP(launch_axi_iface(b, M, h->w_F, h->w_lam, g, beta, gM, gF, gL, gG, gB, h->w_scal,
                               bd.scheme == MEM_FLUX_FLIC, h->w_fLF, h->w_Mh, h->w_gI, h->w_bI,
                               h->w_phi, q));
      AXI_HIP(launch_axi_solve(n + np, tpb, h->d_tab, h->w_Mh, h->w_gI, h->w_bI, pw, nullptr,
                               nullptr, h->w_stI, q));
      AXI_HIP(launch_axi_moments(n + np, tpb, h->d_tab, h->w_bI, h->w_gI, nullptr, h->w_fLW, q));
      AXI_HIP(launch_axi_fv2(b, M, g, gG, h->w_fLF, h->w_fLW, h->w_phi, h->w_stI, h->w_scal,
                             h->w_Mn, q));
    }
    AXI_HIP(launch_copy(n * 9, h->w_Mn, M, q));
    AXI_HIP(launch_axi_collide(b, M, g, h->w_scal, 2, 0.5f, bd.prandtl, bd.mu_ref, q));
    AXI_HIP(launch_axi_gauge(n, M, beta, g, q));
    AXI_HIP(launch_axi_finish(np, t, dt, h->w_scal, q));
    return MEM_OK;
  };
  if (!bd.use_graph) {
    for (int k = 0; k < n_steps; ++k) {
      const mem_err_t e = step_once(s);
      if (e != MEM_OK) return e;
    }
    return MEM_OK;
  }
  mem_axi_s::StepKey key;
  std::memset(&key, 0, sizeof(key));
  key.b = bd;
  key.M = M; key.beta = beta; key.g = g; key.t = t; key.dt = dt; key.status = status;
  key.p = pw;
  key.gen = h->gen;
  if (!h->exec || std::memcmp(&key, &h->key, sizeof(key)) != 0) {
    if (h->exec) { (void)hipGraphExecDestroy(h->exec); h->exec = nullptr; }
    if (!h->cap_stream) AXI_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    AXI_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    const mem_err_t e = step_once(h->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t he = hipStreamEndCapture(h->cap_stream, &graph);
    if (e != MEM_OK || he != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return e != MEM_OK ? e : MEM_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&h->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) { h->exec = nullptr; return MEM_ERR_HIP; }
    h->key = key;
  }
  for (int k = 0; k < n_steps; ++k) AXI_HIP(hipGraphLaunch(h->exec, s));
  return MEM_OK;
}

bool scheme_ok(int32_t sc) { return sc >= MEM_FLUX_LLF && sc <= MEM_FLUX_FLIC; }

}  // namespace

extern "C" {

// One normal-shock problem (see mem.h): its descriptors go to the device and
// the batch driver runs it as a batch of one.
mem_err_t mem_axi_step(mem_axi_t h, const mem_axi_shock_t* pb, float* M, float* beta, float* g,
                       float* t, float* dt, int32_t n_steps, const mem_solve_opts_t* opts,
                       uint32_t* status, hipStream_t s) {
  if (!h || !pb || !M || !beta || !g || !t || !dt || n_steps < 0) return MEM_ERR_INVALID_ARG;
  const int64_t n = pb->n_cells;
  if (n < 1 || n > (int64_t)1 << 24 || !(pb->dx > 0.f) || !(pb->cfl > 0.f) || !(pb->cfl <= 1.f) ||
      !(pb->prandtl > 0.f) || !(pb->mu_ref > 0.f) || !scheme_ok(pb->scheme))
    return MEM_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(pb->ghost_left[k]) || !std::isfinite(pb->ghost_right[k]))
      return MEM_ERR_INVALID_ARG;
  if (!(pb->ghost_left[0] > 0.f) || !(pb->ghost_left[2] > 0.f) || !(pb->ghost_right[0] > 0.f) ||
      !(pb->ghost_right[2] > 0.f))
    return MEM_ERR_INVALID_ARG;
  SolveParams p;
  if (params_axi(h, opts, p) != MEM_OK) return MEM_ERR_INVALID_ARG;
  if (n > h->cap || h->cap_p < 1) {
    const mem_err_t e = mem_axi_reserve_batch(h, n, 1);
    if (e != MEM_OK) return e;
  }
  AXI_HIP(launch_axi_single(n, pb->dx, pb->ghost_left, pb->ghost_right, h->w_off1, h->w_dx1,
                            h->w_gs1, s));
  mem_axi_batch_t bd;
  std::memset(&bd, 0, sizeof(bd));
  bd.n_cells = n;
  bd.n_problems = 1;
  bd.scheme = pb->scheme;
  bd.cell_offsets = h->w_off1;
  bd.dx = h->w_dx1;
  bd.ghosts = h->w_gs1;
  bd.cfl = pb->cfl;
  bd.prandtl = pb->prandtl;
  bd.mu_ref = pb->mu_ref;
  bd.use_graph = pb->use_graph;
  bd.cond_max = pb->cond_max;
  return axi_steps(h, bd, M, beta, g, t, dt, n_steps, p, status, s);
}

mem_err_t mem_axi_step_batch(mem_axi_t h, const mem_axi_batch_t* b, float* M, float* beta,
                             float* g, float* t, float* dt, int32_t n_steps,
                             const mem_solve_opts_t* opts, uint32_t* status, hipStream_t s) {
  if (!h || !b || !M || !beta || !g || !t || !dt || n_steps < 0) return MEM_ERR_INVALID_ARG;
  const int64_t n = b->n_cells;
  const int32_t np = b->n_problems;
  if (np < 1 || n < np || n > (int64_t)1 << 24 || !b->cell_offsets || !b->dx || !b->ghosts ||
      !(b->cfl > 0.f) || !(b->cfl <= 1.f) || !(b->prandtl > 0.f) || !(b->mu_ref > 0.f) ||
      !scheme_ok(b->scheme))
    return MEM_ERR_INVALID_ARG;
  SolveParams p;
  if (params_axi(h, opts, p) != MEM_OK) return MEM_ERR_INVALID_ARG;
  if (n > h->cap || np > h->cap_p) {
    const mem_err_t e = mem_axi_reserve_batch(h, n, np);
    if (e != MEM_OK) return e;
  }
  // offsets are read back and checked once per (pointer, n_cells, n_problems)
  if (b->cell_offsets != h->v_off || n != h->v_n || np != h->v_P) {
    std::vector<int64_t> off((size_t)np + 1);
    AXI_HIP(hipMemcpyAsync(off.data(), b->cell_offsets, off.size() * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
    AXI_HIP(hipStreamSynchronize(s));
    if (off[0] != 0 || off[np] != n) return MEM_ERR_INVALID_ARG;
    for (int32_t q = 0; q < np; ++q)
      if (off[q + 1] <= off[q]) return MEM_ERR_INVALID_ARG;
    h->v_off = b->cell_offsets;
    h->v_n = n;
    h->v_P = np;
  }
  return axi_steps(h, *b, M, beta, g, t, dt, n_steps, p, status, s);
}

mem_err_t mem_axi_gauge(int64_t n, float* M, float* beta, float* g, hipStream_t s) {
  if (n < 0 || n > (int64_t)INT32_MAX - 256) return MEM_ERR_INVALID_ARG;
  if (n == 0) return MEM_OK;
  if (!M || !g) return MEM_ERR_INVALID_ARG;
  return launch_axi_gauge(n, M, beta, g, s) == hipSuccess ? MEM_OK : MEM_ERR_HIP;
}

mem_err_t mem_axi_moments_noncanonical(mem_axi_t h, int64_t n, const float* alpha, const float* g,
                                       float* M, hipStream_t s) {
  if (!h || n < 0 || n > (int64_t)INT32_MAX - 4) return MEM_ERR_INVALID_ARG;
  if (n == 0) return MEM_OK;
  if (!alpha || !g || !M) return MEM_ERR_INVALID_ARG;
  return launch_axi_moments_nc(n, (int)h->P, h->d_tab, alpha, g, M, s) == hipSuccess ? MEM_OK
                                                                                     : MEM_ERR_HIP;
}

mem_err_t mem_axi_moments(mem_axi_t h, int64_t n, const float* beta, const float* g, float* M,
                          float* F, hipStream_t s) {
  if (!h || n < 0 || n > (int64_t)INT32_MAX - 4) return MEM_ERR_INVALID_ARG;
  if (n == 0) return MEM_OK;
  if (!beta || !g) return MEM_ERR_INVALID_ARG;
  if (launch_axi_moments(n, (int)h->P, h->d_tab, beta, g, M, F, s) != hipSuccess)
    return MEM_ERR_HIP;
  return MEM_OK;
}

}  // extern "C"
