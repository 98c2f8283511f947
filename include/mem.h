/*
 * mem.h -- C ABI of the MI355X (gfx950) maximal-entropy moment method library.
 *
 * The library implements, as HIP kernels, the per-cell maximal-entropy dual
 * problem of the canonical-form exponential family and the finite-volume step
 * around it, following "Stabilizing the Maximal Entropy Moment Method for
 * Rarefied Gas Dynamics at Single-Precision" (Zheng, Wang, Chen):
 *
 *   canonical form f = n exp(beta_i phi_i(u_bar) - log Z(beta)),  i >= 1
 *       (Sec. 2.2, eq. "exp family"; beta_0 = n is the number density);
 *   log Z by log-sum-exp over fixed quadrature nodes (Sec. 3.1);
 *   dual objective, gradient and Hessian (App. C);
 *   modified Newton with lambda*I shift and Armijo backtracking (Alg. 1);
 *   gauge u_bar = ((u_x - w_x)/s_x, u_y/s_r, u_z/s_r), Hermite gauge and the
 *       change of gauge T(g', g) (Sec. 3.3);
 *   moment fluxes, local Lax--Friedrichs in local gauges, ES-BGK source
 *       splitting and the time step of Alg. 2 (Sec. 3.4, App. A).
 *
 * Discretisation: tensor Gauss--Hermite nodes fixed in gauge coordinates
 * (n_nodes_1d per axis), basis = orthonormal Hermite products of total degree
 * <= 4: phi_(a,b,c) = He_a(x) He_b(y) He_c(z) / sqrt(a! b! c!), K = 35 in 3D
 * (K = 5 in 1D, phi_k = He_k/sqrt(k!)).  Basis order: by total degree, then
 * lexicographically descending in (a,b,c); index 0 = 1, 1..3 = x, y, z.
 *
 * Conventions for every entry point
 *   - Arrays named M, beta, F, g, lam, iters, resid, status, t, dt are DEVICE
 *     pointers owned by the caller (for example PyTorch tensors), row-major:
 *     M[n][K], beta[n][K], F[n][K], g[n][G] with G = 2 (1D: w, s) or
 *     G = 3 (3D: w_x, s_x, s_r).  Struct arguments (mem_config_t,
 *     mem_solve_opts_t, mem_batch_t) are HOST memory; the pointers inside
 *     mem_batch_t are device pointers.
 *   - Every call is asynchronous on `stream` (NULL = default stream) except
 *     where stated.  A context is used by one stream at a time.
 *   - Return codes report API misuse and HIP failures only.  Numerical
 *     failure of a cell never returns an error: it sets that cell's status
 *     bits (MEM_ST_*) and leaves the rest of the batch untouched.
 *   - Only mem_create and mem_reserve allocate device memory.  Entry points
 *     that need workspace grow it through mem_reserve when it is too small;
 *     reserve first to keep allocation out of timed or captured regions.
 */
#ifndef MEM_H
#define MEM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MEM_API __attribute__((visibility("default")))

typedef struct mem_ctx_s* mem_ctx_t;

typedef enum {
  MEM_OK = 0,
  MEM_ERR_INVALID_ARG = 1,   /* null pointer, negative size, bad option      */
  MEM_ERR_HIP = 2,           /* a HIP runtime call or kernel launch failed   */
  MEM_ERR_NOMEM = 3,         /* device allocation failed                     */
  MEM_ERR_UNSUPPORTED = 4    /* configuration the library does not implement */
} mem_err_t;

/* Arithmetic of the moment/Hessian assembly GEMM. */
typedef enum {
  MEM_PREC_FP32 = 0,         /* FP32 MFMA (v_mfma_f32_16x16x4_f32)           */
  MEM_PREC_BF16X3 = 1,       /* hi+lo BF16 split, 3 products, FP32 accumulate */
  MEM_PREC_FP16X3 = 2        /* hi+lo FP16 split, 3 products, FP32 accumulate */
} mem_prec_t;

/* Per-cell status bits (written by mem_maxent_solve and mem_step). */
#define MEM_ST_CONVERGED     0x01u  /* max_i |G_i| <= tol_grad, or decrement <= tol_dec with max|G| <= tol_grad_loose */
#define MEM_ST_MAXITER       0x02u  /* iteration budget exhausted                                  */
#define MEM_ST_STAGNATED     0x04u  /* line-search step alpha <= alpha_min (Alg. 1 exit test)      */
#define MEM_ST_SHIFTED       0x08u  /* Cholesky needed H + lambda I at least once (Alg. 1)         */
#define MEM_ST_FP64          0x10u  /* FP32 pivot ratio below threshold: direction solved in FP64  */
#define MEM_ST_NONFINITE     0x20u  /* non-finite input or iterate                                 */
#define MEM_ST_NONREALIZABLE 0x40u  /* n <= 0, or the dual value fell below min_p log w~_p, which
                                       certifies that no minimiser exists on the node set, or
                                       |beta| exceeded beta_max                                */
#define MEM_ST_LAMBDA_FAIL   0x80u  /* characteristic speeds could not be computed                 */
#define MEM_ST_MAXWELL_FLUX  0x100u /* mem_step: the solve ended NONREALIZABLE or NONFINITE, so the
                                       cell's fluxes, speeds and next warm start use the Maxwellian
                                       of its gauge instead                                       */

typedef struct {
  int32_t dim;          /* 1 or 3                                                      */
  int32_t n_nodes_1d;   /* Gauss--Hermite nodes per velocity axis (2..64 in 1D, 2..32 in 3D) */
  int32_t prec;         /* mem_prec_t used by the Newton Hessian assembly              */
  int32_t reserved;     /* must be 0                                                   */
} mem_config_t;

/* Options of Alg. 1.  Defaults (mem_solve_opts_default) are the paper's
 * constants where it gives them: tol 1e-8 on the Newton decrement, maxI 400,
 * maxT 25 (26 trials alpha = 1 .. 2^-25), Armijo c = 5e-4, atol = 5e-6,
 * rtol = 5e-5, lambda = 1e-3 growing x10, exit when alpha <= 1e-6. */
typedef struct {
  float   tol_grad;         /* stop when max_{i>=1} |E[phi_i] - M_i/n| <= tol_grad (2e-6)  */
  float   tol_dec;          /* or when 1/2 G^T (H+lambda I)^-1 G <= tol_dec (1e-8) ...      */
  float   tol_grad_loose;   /* ... and max|G| <= tol_grad_loose (1e-5)                       */
  int32_t max_iter;         /* Newton iterations per solve (400)                             */
  int32_t max_ls;           /* line-search halvings (25)                                     */
  float   armijo_c;         /* 5e-4                                                          */
  float   atol;             /* 5e-6                                                          */
  float   rtol;             /* 5e-5                                                          */
  float   lambda0;          /* first Hessian shift (1e-3)                                    */
  float   lambda_mul;       /* shift growth factor (10)                                      */
  float   alpha_min;        /* alpha <= alpha_min ends the solve as stagnated (1e-6)         */
  float   fp64_pivot_ratio; /* min/max Cholesky pivot below this -> FP64 direction (1e-6);
                               0 disables the FP64 path (pure FP32 Alg. 1)                   */
  int32_t check_every;      /* list-compacted Newton loop only (tuning solver 0): poll the
                               live-cell count every this many passes (2), a stream
                               synchronisation each; 0 = never poll (max_iter passes).
                               The persistent solver (solver 1, the default for FP32 on
                               12-point rules) never synchronises and ignores it.         */
  int32_t refine;           /* residual refinement passes (3): cells that converge, or
                               whose FP32 residual (<= 1e-3) stops halving for 6
                               iterations, get their residual re-evaluated with a
                               compensated FP32 exponent and moment sum (double-float
                               arithmetic) and, while above tol_grad, a Newton correction
                               with their FP32 Hessian; the reported resid is this
                               compensated residual and a cell is CONVERGED only if it is
                               <= tol_grad_loose (else STAGNATED).  0 = off.               */
  float   beta_max;         /* |beta_i|, i >= 1, above this ends the cell as NONREALIZABLE
                               (25; 0 = off).  In the Hermite gauge solvable targets have
                               |beta| of order 1-10 (Mott-Smith mixtures up to Mach 10:
                               below 6); iterates that run away along a ray of the dual
                               (targets outside the nodes' moment set) are stopped here
                               long before the dual-value certificate fires.  Independent
                               of it, a residual above 1e-3 that has not halved for 30
                               iterations ends a cell as STAGNATED.                        */
} mem_solve_opts_t;

/* A ragged batch of independent 1D normal-shock problems (dim must be 3).
 * Cells of problem p are cell_offsets[p] .. cell_offsets[p+1]-1 of the flat
 * M/beta/g arrays, ordered left to right.  Boundary (ghost) states are
 * Maxwellian moments M_left/M_right in their own gauges g_left/g_right. */
#define MEM_FLUX_LLF  0  /* local Lax--Friedrichs (first order, eq. "The lax F")             */
#define MEM_FLUX_LW   1  /* two-step Lax--Wendroff (eq. "The lax W")                         */
#define MEM_FLUX_FLIC 2  /* LLF + van Leer-limited Lax--Wendroff correction (eq. "The FLIC") */
typedef struct {
  int64_t        n_cells;        /* host copy of cell_offsets[n_problems]                   */
  int32_t        n_problems;
  int32_t        collision;      /* 0 = BGK (Pr forced to 1), 1 = ES-BGK                   */
  const int64_t* cell_offsets;   /* device [n_problems + 1]                                 */
  const float*   dx;             /* device [n_problems]                                     */
  const float*   M_left;         /* device [n_problems][K]                                  */
  const float*   M_right;        /* device [n_problems][K]                                  */
  const float*   g_left;         /* device [n_problems][3]                                  */
  const float*   g_right;        /* device [n_problems][3]                                  */
  float          cfl;            /* dt = cfl * dx / max spectral radius (0.5)               */
  float          prandtl;        /* 2/3 for monatomic gas (App. A)                          */
  float          mu_ref;         /* viscosity at T = 1; tau = mu_ref / (Pr n)  (sqrt(2/pi)) */
  int32_t        newton_per_step;/* Newton iteration budget per time step (8)               */
  int32_t        use_graph;      /* 1: the first call captures one time step into a hipGraph
                                    (on a private stream of default priority) and every
                                    step replays it with hipGraphLaunch on `stream`; the
                                    graph is kept while the batch, state pointers and
                                    options stay the same.  0: plain launches.  Results
                                    are identical either way.                              */
  int64_t*       iter_hist;      /* device [newton_per_step + 1] or NULL: after each step's
                                    MaxEnt solve, bin k is incremented by the number of
                                    cells whose solve took k Newton iterations (Alg. 1
                                    directions).  Accumulates over calls; never cleared. */
  int32_t        flux_scheme;    /* MEM_FLUX_LLF, MEM_FLUX_LW or MEM_FLUX_FLIC (Sec. 3.4)  */
  float*         cond_max;       /* device [n_problems] or NULL: running maximum, over the
                                    steps and the problem's cells, of a lower bound of
                                    cond(H) for the FP32 Hessian at each cell's solution
                                    (from the S row the step's flux pass assembles there):
                                    |H v| |H^-1 u| for the unit vectors of six power and
                                    inverse iterations from (1, ..., 1)/sqrt 34, or
                                    max(max_j |H e_j|, max_k d_k) / min_k d_k over the LDL^T
                                    pivots d_k if larger; +inf where the FP32 Cholesky of
                                    that Hessian fails.  The conditioning monitor of the
                                    paper's cell-count study (Sec. 3.5, Sec. 4.6).  Costs one
                                    extra kernel per step when set.  Accumulates over calls;
                                    never cleared.                                          */
  int64_t*       status_counts;  /* device [9] or NULL: after each step's MaxEnt solve of the
                                    cells (and the Maxwellian substitution), entry k is
                                    incremented by the number of cells whose status has bit
                                    1 << k (MEM_ST_*; 8 = MEM_ST_MAXWELL_FLUX): cell-steps by
                                    outcome.  Accumulates over calls; never cleared.        */
} mem_batch_t;

/* ---- context -------------------------------------------------------------- */

/* Build the quadrature and basis tables in FP64 on the host, convert them to
 * the device layouts and upload them to the current device.  Allocates. */
MEM_API mem_err_t mem_create(const mem_config_t* cfg, mem_ctx_t* out);
MEM_API mem_err_t mem_destroy(mem_ctx_t ctx);
/* Pre-size the per-cell workspace for up to max_cells cells and max_problems
 * problems (graph- and timing-safe calls afterwards).  mem_step needs rows for
 * n_cells + n_problems (the cells and every interface) and grows the workspace
 * itself, before any capture, when they are missing.  Allocates. */
MEM_API mem_err_t mem_reserve(mem_ctx_t ctx, int64_t max_cells, int32_t max_problems);
MEM_API const char* mem_strerror(mem_err_t err);
/* Detail of the last error on this context (host string, valid until the next call). */
MEM_API const char* mem_last_error(mem_ctx_t ctx);
MEM_API void mem_solve_opts_default(mem_solve_opts_t* opts);
MEM_API int32_t mem_n_basis(mem_ctx_t ctx);   /* K */
MEM_API int32_t mem_n_nodes(mem_ctx_t ctx);   /* Q = n_nodes_1d^dim */
/* Copy a host-side FP64 table built by mem_create (for checking).  which:
 * 0 = nodes [Q][dim], 1 = weights [Q] (sum 1), 2 = Phi [Q][K].  Writes at most
 * n_values doubles to host_out; returns the table size through n_total. */
MEM_API mem_err_t mem_copy_table(mem_ctx_t ctx, int32_t which, double* host_out,
                                 int64_t n_values, int64_t* n_total);

/* Host-only variant of mem_copy_table that needs no device: builds the FP64
 * tables of (dim, n_nodes_1d) on the host and copies table `which` (as above,
 * plus 3 = Lebesgue log weights [Q]). */
MEM_API mem_err_t mem_host_table(int32_t dim, int32_t n_nodes_1d, int32_t which,
                                 double* host_out, int64_t n_values, int64_t* n_total);

/* ---- hot path --------------------------------------------------------------- */

/* Hermite gauge (Sec. 3.3, eqs. "Hermite parameters", "Change gauge M F";
 * Alg. 2 ComputeGaugeParameters + GaugeTransformation).  In place for n_cells
 * cells: reads M and g, computes the Hermite gauge g_H from the moments,
 * writes M <- T(g_H, g) M, beta_{i>=1} <- (T(g, g_H)^T alpha)_{i>=1} (beta may
 * be NULL; beta_0 is left as n) and g <- g_H.  Cells with n <= 0 or a
 * non-positive variance are left unchanged. */
MEM_API mem_err_t mem_gauge(mem_ctx_t ctx, int64_t n_cells, float* M, float* beta,
                            float* g, hipStream_t stream);

/* Alg. 1 for every cell: find beta minimising the dual objective for target
 * moments M (in each cell's gauge, M[:,0] = n > 0).  beta: in = initial guess
 * (beta[:,0] ignored), out = solution with beta[:,0] = n.  iters, resid
 * (max_{i>=1}|G_i| at the returned beta, FP32) and status are per-cell
 * outputs, each may be NULL.  With the persistent solver (mem_tuning_t solver
 * 1) the whole Newton loop is one kernel and the call is fully asynchronous;
 * with the list-compacted loop (solver 0, or the 16-bit precisions) it
 * synchronises `stream` every opts->check_every passes to poll the number of
 * live cells (0 = never). */
MEM_API mem_err_t mem_maxent_solve(mem_ctx_t ctx, int64_t n_cells, const float* M,
                                   float* beta, const mem_solve_opts_t* opts,
                                   int32_t* iters, float* resid, uint32_t* status,
                                   hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): mem_maxent_solve
 * with the Newton workspace taken from a static device array of about 25 MiB
 * that the library holds on every GPU it runs on until the process ends.
 * Same arguments, kernels and results as mem_maxent_solve; at most 8192 cells
 * per call (more returns MEM_ERR_INVALID_ARG and launches nothing).  The call
 * allocates nothing and calls no allocating library routine; with
 * opts->check_every = 0 it never synchronises the stream (each of the
 * max_iter Newton passes is launched; passes with no live cell end at once),
 * so it can be captured.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two streams, or two contexts on the same
 * device) race and give wrong results.  dim 1 contexts need no workspace and
 * run the 1D solve. */
MEM_API mem_err_t mem_maxent_solve_noalloc(mem_ctx_t ctx, int64_t n_cells, const float* M,
                                           float* beta, const mem_solve_opts_t* opts,
                                           int32_t* iters, float* resid, uint32_t* status,
                                           hipStream_t stream);

/* Dual evaluation at given beta (Sec. 3.1 and App. C), for checking the
 * kernels: logZ[n] (log partition function with Lebesgue weights), E[n][K] =
 * E_sigma[phi], H[n][K-1][K-1] = covariance block of the Hessian (i,j >= 1).
 * Any output may be NULL.  dim must be 3. */
MEM_API mem_err_t mem_dual(mem_ctx_t ctx, int64_t n_cells, const float* beta,
                           float* logZ, float* E, float* H, hipStream_t stream);

/* Per-moment residual of a solution: G[n][K] with G[:,0] = 0 and, for k >= 1,
 * G_k = E_sigma[phi_k] / E_sigma[phi_0] - M_k / M_0, the gradient of the dual
 * objective whose size is the stopping quantity of Alg. 1 (max_k |G_k| is
 * what mem_maxent_solve returns as resid).  Evaluated at the context's nodes
 * in compensated FP32 arithmetic (double-float exponent and sums, Ogita-Rump-
 * Oishi Dot2), which agrees with an FP64 evaluation to a few 1e-8 near a
 * solution.  Cells with M_0 <= 0 or non-finite inputs give non-finite G.
 * M, beta, G: device [n_cells][K].  dim must be 3. */
MEM_API mem_err_t mem_moment_residual(mem_ctx_t ctx, int64_t n_cells, const float* M,
                                      const float* beta, float* G, hipStream_t stream);

/* Moment fluxes (eq. "The ME equation", flux line; Alg. 2 ComputeFluxes):
 * F[n][K] = int u_x phi_i(u_bar) f du in each cell's gauge, from beta
 * (beta[:,0] = n) and g.  lam[n][2] (may be NULL) = (min, max) eigenvalue of
 * dF/dM in physical units (local Lax--Friedrichs speeds, Sec. 3.4); each
 * gauge-frame eigenvalue is clamped to the node span [-max|u_x|, max|u_x|],
 * where every eigenvalue of the quadrature pencil lies exactly. */
MEM_API mem_err_t mem_flux(mem_ctx_t ctx, int64_t n_cells, const float* beta,
                           const float* g, float* F, float* lam, hipStream_t stream);

/* ES-BGK source term by operator splitting (eq. "source update", App. A):
 * M <- (1 - h/tau) M + (h/tau) M~(g), tau = mu_ref/(Pr n), in place.  The
 * target M~ is the axisymmetric Gaussian with Sigma = T/Pr I + (1-1/Pr) P/n.
 * dim must be 3. */
MEM_API mem_err_t mem_collide(mem_ctx_t ctx, int64_t n_cells, float* M, const float* g,
                              float h, float prandtl, float mu_ref, hipStream_t stream);

/* Alg. 2 Step, n_steps times, for a ragged batch: Collision(dt/2),
 * Transport(dt) = MaxEnt solve (warm start from beta, at most
 * newton_per_step iterations) + fluxes + characteristic speeds + local
 * Lax--Friedrichs update with neighbours moved into each cell's gauge,
 * Collision(dt/2), Hermite-gauge update.  M, beta, g: device [n_cells][K|3],
 * in/out.  t: device [n_problems], advanced.  dt: device [n_problems], in =
 * step for the first step (a value <= 0 requests one from a solve of the
 * current state), out = step for the next call (CFL rule from the last
 * transport's speeds).  Within a step the transport and the second collision
 * half use min(dt, CFL dx / max speed of that step), so a rise of the speeds
 * never breaks the CFL limit.  status (may be NULL): device [n_cells], OR of the
 * cells' solve status over the steps.  A cell whose moments the nodes cannot
 * represent (solve ends NONREALIZABLE or NONFINITE with finite moments, n > 0)
 * takes beta of the Maxwellian of its gauge (beta_0 = n, -1/sqrt(2) on the
 * pure second-degree statistics) for that step's fluxes and speeds and as the
 * next warm start, and gets MEM_ST_MAXWELL_FLUX: the update stays conservative
 * and finite while the closure there drops to the Maxwellian.
 * flux_scheme LW / FLIC (Sec. 3.4): every interface (n_cells + n_problems of
 * them, boundaries included) is evaluated once, in the gauge of the element
 * to its right, from its neighbours moved into that gauge: the half-step
 * moments (M_l + M_r)/2 + dt/(2 dx) (F_l - F_r) are solved (warm start from
 * the right element's beta, same iteration budget) and their flux is the
 * Lax--Wendroff flux; FLIC adds it to the LLF flux with the van Leer limiter
 * of r = (M_l - M_ll)/(M_r - M_l) per moment (ghosts extend beyond the
 * boundary).  An interface whose half-step state the nodes cannot represent
 * keeps the LLF flux.  The cell to an interface's left takes the same flux
 * moved into its own gauge, so the update stays conservative.  The batch's
 * cell_offsets are read back on `stream` and checked on every call (start 0,
 * end n_cells, every problem at least one cell; else MEM_ERR_INVALID_ARG and
 * nothing launched): one synchronisation of `stream` per call, before any
 * launch; the n_steps steps then run without host synchronisation
 * (mem_conserved makes the same check). */
MEM_API mem_err_t mem_step(mem_ctx_t ctx, const mem_batch_t* batch, float* M, float* beta,
                           float* g, float* t, float* dt, int32_t n_steps,
                           const mem_solve_opts_t* opts, uint32_t* status,
                           hipStream_t stream);

/* Conserved totals per problem in FP64 (check of mem_step):
 * out[p][3] = dx * sum over the problem's cells of (n, n v_x, n (v^2/2 + 3T/2))
 * computed in double precision from M and g.  out is a device double array. */
MEM_API mem_err_t mem_conserved(mem_ctx_t ctx, const mem_batch_t* batch, const float* M,
                                const float* g, double* out, hipStream_t stream);

/* ---- launch tuning ------------------------------------------------------------- */

/* Launch parameters of the 3D Newton kernels (per context).  They change how
 * work is mapped to workgroups, never what is computed; results differ only by
 * the order of floating-point sums. */
typedef struct {
  int32_t dir_waves;   /* cells (wavefronts) per workgroup of the Newton-direction
                          kernel: 2, 4 or 8 (default 4)                            */
  int32_t split_want;  /* workgroups a small assembly launch is spread over by
                          splitting the quadrature nodes into ranges (the node tile
                          of a workgroup is Q / splits); 0 = never split (512)     */
  double  tuned_ms;    /* time of the best trial in mem_autotune (0 = not tuned)   */
  int32_t solver;      /* Newton loop of the 3D FP32 solve: 0 = list-compacted
                          launches per pass with the MFMA assembly (sigma . Psi);
                          1 = one persistent kernel, a wavefront per live cell
                          taken from a work queue, the assembly sum-factorised on
                          the tensor grid (12-point rules only; other rules and the
                          mixed precisions use 0) (default 1)                       */
  int32_t wave_max_cells; /* with solver 1: launches of more cells use solver 0;
                          0 = no limit (default 0)                                   */
  int32_t wave_per_cu; /* with solver 1: wavefronts (cells in flight) per compute
                          unit in the persistent kernel's grid: 4, 8 or 12;
                          0 = 12 (default 12)                                       */
  int32_t asm_waves;   /* with solver 0 in FP32: wavefronts of 16 cells per workgroup
                          of the MFMA assembly, 4 or 8 (64 or 128 cells sharing each
                          node tile staged in LDS); 0 = 4 (default 4)               */
  int32_t cached;      /* set by mem_autotune: 1 when the result came from the
                          process-wide cache instead of timed trials                */
} mem_tuning_t;

/* Time full solves of this batch with every candidate, one coordinate at a
 * time, each trial warm and timed with HIP events on `stream`: the Newton
 * loop (solver in {1, 0}, where the persistent kernel applies); then for
 * solver 1 wave_per_cu in {12, 8, 4}; for solver 0 dir_waves in {2, 4, 8},
 * asm_waves in {4, 8} (FP32) and split_want in {0, 256, 512, 1024, 2048}.
 * Keep the fastest in the context and return it in *out (nullable).  The
 * result is also kept in a process-wide cache keyed by (device architecture,
 * dim, n_nodes_1d, moments, precision, bit length of n_cells): a later call
 * with the same key, from any context, takes the cached result without
 * timing (out->cached = 1).  The same parameters serve mem_step's solves.
 * beta_init is not modified; the trials run in beta_work [n_cells][35]
 * (device, caller-owned).  Synchronous. */
MEM_API mem_err_t mem_autotune(mem_ctx_t ctx, int64_t n_cells, const float* M,
                               const float* beta_init, float* beta_work,
                               const mem_solve_opts_t* opts, mem_tuning_t* out,
                               hipStream_t stream);
MEM_API mem_err_t mem_get_tuning(mem_ctx_t ctx, mem_tuning_t* out);
/* Forget every cached mem_autotune result (the next call times again). */
MEM_API void mem_tuning_cache_clear(void);
MEM_API mem_err_t mem_set_tuning(mem_ctx_t ctx, const mem_tuning_t* in);

/* ---- the paper's own discretisation: nine statistics on a box ---------------- */

/* For 1D flow with cylindrical symmetry in velocity the paper works with nine
 * statistics of (u_x, u_r), u_r = sqrt(u_y^2 + u_z^2), in the gauge
 * u_bar = ((u_x - w_x)/s_x, u_r/s_r) (Sec. 3.3; orthogonal form of the
 * appendix on the 35-moment system).  With x = u_bar_x, y = u_bar_r^2/2 they
 * are, in this order:
 *   1, x, He_2(x)/sqrt2, y - 1, He_3(x)/sqrt6, He_4(x)/sqrt24,
 *   y^2/2 - 2y + 1, x (y - 1), He_2(x)/sqrt2 (y - 1)
 * (the printed eighth statistic, u_x (u_r^2 - 1)/2, is read as
 * u_x (u_r^2 - 2)/2, which makes the set orthonormal under the standard
 * Maxwellian as the paper states).  Integrals run over the box
 * (u_x, u_r) in [ux_lo, ux_hi] x [0, ur_hi] cut into blocks_x x blocks_r equal
 * blocks, each with the tensor Gauss--Legendre rule of `order` points per axis
 * (end of Sec. 3.1); the node weight is 2 pi u_r times the two scaled
 * Gauss--Legendre weights (axisymmetric measure).  The nodes stay fixed in
 * physical velocity, so each cell evaluates the statistics in its own gauge.
 * Units: m = k_B = 1. */
typedef struct {
  double ux_lo, ux_hi;   /* a_x < b_x */
  double ur_hi;          /* b_r > 0 */
  int32_t blocks_x, blocks_r;  /* 1..256 each */
  int32_t order;         /* Gauss--Legendre points per block and axis, 1..32 */
  int32_t reserved;      /* must be 0 */
} mem_axi_rule_t;

typedef struct mem_axi_s* mem_axi_t;

/* Integration-domain formula of the normal-shock set-up (appendix on the
 * shock problem): box[0] = a_x = min(v+ - n_a sqrt(T+), v- - n_a sqrt(T-)),
 * box[1] = b_x = max(v- + n_b sqrt(T-), v+ + n_b sqrt(T+)),
 * box[2] = b_r = n_r max(sqrt(T-), sqrt(T+)).  Host only. */
MEM_API mem_err_t mem_axi_domain(double v_minus, double T_minus, double v_plus, double T_plus,
                                 int32_t n_a, int32_t n_b, int32_t n_r, double* box);

/* Number of nodes P = blocks_x blocks_r order^2 of a rule, or -1 if the rule
 * is invalid.  Host only. */
MEM_API int64_t mem_axi_rule_nodes(const mem_axi_rule_t* rule);

/* The rule's nodes in FP64 on the host, no device needed: ux[P], ur[P],
 * logw[P] (caller-owned, any may be NULL; n_nodes must equal P).  Node order:
 * blocks in x (outer), blocks in r, Gauss--Legendre points in x, then in r. */
MEM_API mem_err_t mem_axi_host_rule(const mem_axi_rule_t* rule, double* ux, double* ur,
                                    double* logw, int64_t n_nodes);

/* Handle holding the rule's node table (u_x as an FP32 pair hi + lo, u_r, log w, and
 * the lo parts of u_r and log w for the compensated residual) on the current device.
 * MEM_ERR_INVALID_ARG for an invalid rule. */
MEM_API mem_err_t mem_axi_create(const mem_axi_rule_t* rule, mem_axi_t* out);
MEM_API mem_err_t mem_axi_destroy(mem_axi_t h);
MEM_API int64_t mem_axi_n_nodes(mem_axi_t h);

/* Alg. 1 on the nine statistics, one wave per cell (FP32 exponent, statistics
 * and sums; FP64 direction for a small pivot ratio as in mem_maxent_solve).
 * M[n][9] targets and g[n][3] = (w_x, s_x, s_r) per cell; beta[n][9] in: start
 * multipliers (beta[:,0] ignored), out: solution with beta[:,0] = n.  Stopping
 * rules and status bits as mem_maxent_solve, including its compensated
 * refinement (opts->refine passes): a cell that ends converged or at its FP32
 * floor takes Newton corrections with the gradient evaluated in double-float
 * FP32 arithmetic; resid is that compensated max_{i>=1} |G_i|, and the cell is
 * converged when it is at most tol_grad_loose, stagnated otherwise.  iters,
 * resid, status may be NULL.  All arrays are device memory, row-major.
 * Asynchronous on stream. */
MEM_API mem_err_t mem_axi_solve(mem_axi_t h, int64_t n_cells, const float* M, const float* g,
                                float* beta, const mem_solve_opts_t* opts, int32_t* iters,
                                float* resid, uint32_t* status, hipStream_t stream);

/* One normal-shock problem on the nine statistics (Alg. 2, Sec. 3.4): n_cells
 * cells of width dx between two fixed ghost Maxwellians given as (n, v, T);
 * cfl in (0, 1]; ES-BGK source with the Prandtl number and the viscosity
 * coefficient mu_ref of tau = mu_ref/(Pr n) (Maxwell molecules); scheme one of
 * MEM_FLUX_LLF, MEM_FLUX_LW, MEM_FLUX_FLIC; use_graph != 0 replays a captured
 * hipGraph of one step (kept while the problem, the pointers, the options and
 * the workspace stay the same). */
typedef struct {
  int32_t n_cells;
  float dx, cfl, prandtl, mu_ref;
  float ghost_left[3], ghost_right[3];  /* (n, v, T) */
  int32_t scheme;
  int32_t use_graph;
  float* cond_max;  /* device [1] or NULL: conditioning monitor (Sec. 3.5,
                       Sec. 4.6): running maximum, over the steps and the cells,
                       of a lower bound of cond(H) for the FP32 8 x 8 Hessian at
                       the last iterate of each cell's solve: |H v| |H^-1 u| for
                       the unit vectors of six power and inverse iterations from
                       (1, ..., 1)/sqrt 8, or max_i H_ii / min pivot if larger;
                       +inf where that Hessian's Cholesky fails.  Accumulates
                       over calls; never cleared. */
} mem_axi_shock_t;

/* A ragged batch of normal-shock problems on the nine statistics, each as in
 * mem_axi_shock_t, stepped together: problem p owns cells
 * [cell_offsets[p], cell_offsets[p+1]) of the concatenated state arrays and
 * keeps its own dx, ghost states, time and dt.  The scheme, cfl, Prandtl
 * number and mu_ref are common.  dx and ghosts are device memory and are not
 * checked on the host: dx > 0 and ghost n, T > 0 (finite) are the caller's to
 * keep, and values outside that give non-finite states, never an access
 * outside the arrays. */
typedef struct {
  int64_t        n_cells;        /* host copy of cell_offsets[n_problems]              */
  int32_t        n_problems;
  int32_t        scheme;         /* MEM_FLUX_LLF, MEM_FLUX_LW or MEM_FLUX_FLIC         */
  const int64_t* cell_offsets;   /* device [n_problems + 1]: 0, increasing, n_cells    */
  const float*   dx;             /* device [n_problems]                                */
  const float*   ghosts;         /* device [n_problems][6]: left (n, v, T), right (n, v, T) */
  float          cfl, prandtl, mu_ref;
  int32_t        use_graph;      /* as in mem_axi_shock_t                              */
  float*         cond_max;       /* device [n_problems] or NULL: per problem, as in
                                    mem_axi_shock_t                                   */
} mem_axi_batch_t;

/* Sizes the step workspace for up to n_cells cells in up to n_problems problems
 * (device allocations; synchronises the device; never shrinks).  The step
 * entry points grow it themselves when a larger call arrives; a caller that
 * reserves first keeps every step call free of allocation and host
 * synchronisation.  mem_axi_reserve(h, n) is mem_axi_reserve_batch(h, n, 1). */
MEM_API mem_err_t mem_axi_reserve_batch(mem_axi_t h, int64_t n_cells, int32_t n_problems);
MEM_API mem_err_t mem_axi_reserve(mem_axi_t h, int64_t n_cells);

/* Time steps of Alg. 2 on the nine statistics with local Lax--Friedrichs
 * fluxes: per step, ES-BGK relaxation over dt/2, Alg. 1 per cell (warm start
 * from beta; a cell the box cannot represent takes the Maxwellian of its
 * gauge), fluxes and speeds, dt_used = min(dt, cfl dx / max speed over cells
 * and ghosts), the update in local gauges (neighbour moments and fluxes moved
 * into each cell's gauge by T(g_i, g_j); both cells of a face use
 * max(rho_i, rho_j), rho = max |speed|; with MEM_FLUX_LW or MEM_FLUX_FLIC
 * each interface instead blends F_LF with the flux of a MaxEnt solve of the
 * half-step state in the right element's gauge, by 1 (LW) or the per-moment van
 * Leer limiter (FLIC), F_LF where that solve fails, and the left cell receives
 * the interface flux moved into its gauge), ES-BGK over dt_used/2, the Hermite
 * gauge of each cell, then t += dt_used and dt <- cfl dx / max speed.  With
 * n_steps = 0 it only sets up: solves the initial state and writes dt.  M[n][9],
 * beta[n][9], g[n][3], t[1], dt[1]: device, in place; status[n] (may be NULL)
 * gets the last solve's status.  Without a large enough mem_axi_reserve it
 * allocates its workspace first (as mem_axi_reserve); otherwise it only
 * launches kernels (or replays the captured step), asynchronously on stream. */
MEM_API mem_err_t mem_axi_step(mem_axi_t h, const mem_axi_shock_t* problem, float* M,
                               float* beta, float* g, float* t, float* dt, int32_t n_steps,
                               const mem_solve_opts_t* opts, uint32_t* status,
                               hipStream_t stream);

/* mem_axi_step for a batch (Alg. 2 per problem, all problems in the same
 * launches): M[n][9], beta[n][9], g[n][3], status[n] (nullable) over the
 * concatenated cells; t[n_problems] and dt[n_problems] per problem (dt from
 * each problem's own cells and ghosts).  The per-cell arithmetic is that of
 * mem_axi_step, so each problem's result equals a separate mem_axi_step of it.
 * cell_offsets are read back and checked (start 0, end n_cells, every problem
 * at least one cell; else MEM_ERR_INVALID_ARG) on the first call with a given
 * (cell_offsets, n_cells, n_problems), which synchronises once; later calls
 * with the same three trust the contents.  Device memory, asynchronous
 * otherwise. */
MEM_API mem_err_t mem_axi_step_batch(mem_axi_t h, const mem_axi_batch_t* batch, float* M,
                                     float* beta, float* g, float* t, float* dt,
                                     int32_t n_steps, const mem_solve_opts_t* opts,
                                     uint32_t* status, hipStream_t stream);

/* Characteristic speeds (Sec. 3.4, the local Lax--Friedrichs bound):
 * lam[n][2] = (min, max) eigenvalue of dF/dM in physical velocity at beta[n][9]
 * and g[n][3]: the extreme generalised eigenvalues of (E[x phi phi^T],
 * E[phi phi^T]) in gauge coordinates (FP32 throughout: Cholesky reduction of
 * the pencil, Householder tridiagonalisation, Sturm-count multisection of the
 * two extremes), mapped to w_x + s_x lambda and clamped to the node span
 * [min u_x, max u_x], where every eigenvalue of the quadrature pencil lies; a
 * pencil that cannot be reduced gives the node span itself.  One wave per
 * cell.  Device memory, asynchronous. */
MEM_API mem_err_t mem_axi_speeds(mem_axi_t h, int64_t n_cells, const float* beta,
                                 const float* g, float* lam, hipStream_t stream);

/* Change of gauge on the nine statistics (Sec. 3.3, eqs. "Hermite Gauge
 * moments" and "Change gauge M F"): per cell, the Hermite gauge g_H of M
 * (w_H = w + s_x E[x], s_xH^2 = s_x^2 Var(x), s_rH^2 = s_r^2 E[u_bar_r^2]/2),
 * then M <- T(g_H, g) M, beta_i <- sum_j T(g, g_H)_ji beta_j for i >= 1
 * (beta_0 kept; beta may be NULL) and g <- g_H.  T is the closed form: 1D
 * Hermite connection coefficients in x times the Laguerre dilation in
 * y = u_bar_r^2/2, evaluated in FP32.  Cells with M_0 <= 0, a non-positive
 * variance or non-finite values are left unchanged.  M[n][9], beta[n][9],
 * g[n][3]: device, in place.  No handle needed. */
MEM_API mem_err_t mem_axi_gauge(int64_t n_cells, float* M, float* beta, float* g,
                                hipStream_t stream);

/* Moments of the non-canonical form of the family, the form the canonical one
 * replaces (relation alpha_0 = log beta_0 - log Z(beta), alpha_i = beta_i; the
 * comparison of Sec. 4.1, Fig. 1): M[n][9] with M_j = sum_p w_p
 * exp(alpha_0 + alpha_i phi_i(u_bar_p)) phi_j(u_bar_p) for alpha[n][9] and
 * g[n][3], summed in plain FP32 with no shift of the exponent.  Rows whose
 * exponent exceeds log(FLT_MAX) at some node come out non-finite (that is the
 * measured outcome, not an error).  One wave per row; device memory,
 * asynchronous. */
MEM_API mem_err_t mem_axi_moments_noncanonical(mem_axi_t h, int64_t n_rows, const float* alpha,
                                               const float* g, float* M, hipStream_t stream);

/* Parameter-to-moment map (Sec. 3.1) and fluxes: M[n][9] = beta_0
 * E_sigma[phi_i], F[n][9] = beta_0 E_sigma[u_x phi_i] with u_x the physical
 * velocity of the node, at beta[n][9] and g[n][3] (E_sigma normalised by
 * sum_p sigma_p).  M or F may be NULL.  Device memory, asynchronous. */
MEM_API mem_err_t mem_axi_moments(mem_axi_t h, int64_t n_cells, const float* beta,
                                  const float* g, float* M, float* F, hipStream_t stream);

/* ---- measurement -------------------------------------------------------------- */

/* Kernel timing with HIP events recorded on the launch stream around every
 * launch of the selected kernels while enabled (enable != 0 clears the
 * totals).  kernel: 0 = assembly GEMM (k_assemble3), 1 = Newton direction
 * (k_direction3), 2 = log-sum-exp / line search (k_lse3).  mem_profile_read
 * synchronises on the recorded events and returns the summed duration in ms
 * and the number of launches timed. */
MEM_API mem_err_t mem_profile_enable(mem_ctx_t ctx, int32_t enable);
MEM_API mem_err_t mem_profile_read(mem_ctx_t ctx, int32_t kernel, double* total_ms,
                                   int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* MEM_H */
