// Host-side FP64 construction of the quadrature and basis tables, and their
// conversion to the device operand layouts of the kernels.
//
// Quadrature (Sec. 3.1, eq. "Numerical integration"): tensor Gauss--Hermite
// rule of the standard normal, nodes fixed in gauge coordinates.  The 1D rule
// is computed from the Jacobi matrix of the probabilists' Hermite polynomials
// (zero diagonal, off-diagonal sqrt(k)): eigenvalues by Sturm-sequence
// bisection, polished by Newton on the orthonormal polynomial p_n, weights
// w_i = 1 / (n p_{n-1}(x_i)^2) (total mass 1).  Lebesgue log weights:
// log w~ = log w + |x|^2/2 + (d/2) log(2 pi).
//
// Basis (App. B, orthogonal form extended to 3D): phi_(a,b,c) = p_a(x) p_b(y)
// p_c(z) with p_k = He_k / sqrt(k!), total degree <= 4, ordered by degree then
// lexicographically descending.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "mem_internal.h"

namespace memt {

namespace {

// orthonormal Hermite values p_0..p_m at x
void ortho_hermite(int m, double x, double* p) {
  p[0] = 1.0;
  if (m >= 1) p[1] = x;
  for (int k = 1; k < m; ++k)
    p[k + 1] = (x * p[k] - std::sqrt((double)k) * p[k - 1]) / std::sqrt((double)(k + 1));
}

// number of eigenvalues of the n x n Jacobi matrix smaller than x
int sturm_count(int n, double x) {
  int cnt = 0;
  double q = -x;
  if (q == 0.0) q = -1e-300;
  if (q < 0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = -x - (double)i / q;
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

}  // namespace

void gauss_hermite(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double bound = 2.0 * std::sqrt((double)n) + 1.0;
  std::vector<double> p(n + 1);
  for (int k = 0; k < n; ++k) {
    double lo = -bound, hi = bound;  // k-th smallest eigenvalue in (lo, hi)
    for (int it = 0; it < 200 && hi - lo > 1e-15 * (1.0 + std::fabs(lo)); ++it) {
      double mid = 0.5 * (lo + hi);
      if (sturm_count(n, mid) > k) hi = mid; else lo = mid;
    }
    double r = 0.5 * (lo + hi);
    for (int it = 0; it < 3; ++it) {  // Newton polish on p_n
      ortho_hermite(n, r, p.data());
      double d = std::sqrt((double)n) * p[n - 1];
      if (d != 0.0) r -= p[n] / d;
    }
    ortho_hermite(n, r, p.data());
    x[k] = r;
    w[k] = 1.0 / ((double)n * p[n - 1] * p[n - 1]);
  }
  // symmetrise (rule is exactly symmetric) and normalise the mass
  for (int k = 0; k < n / 2; ++k) {
    double a = 0.5 * (x[n - 1 - k] - x[k]);
    x[k] = -a; x[n - 1 - k] = a;
    double b = 0.5 * (w[k] + w[n - 1 - k]);
    w[k] = b; w[n - 1 - k] = b;
  }
  if (n % 2) x[n / 2] = 0.0;
  double s = 0.0;
  for (double v : w) s += v;
  for (double& v : w) v /= s;
}

namespace {

void multi_indices(int dim, std::vector<int>& a, std::vector<int>& b, std::vector<int>& c) {
  a.clear(); b.clear(); c.clear();
  for (int tot = 0; tot <= 4; ++tot) {
    if (dim == 1) { a.push_back(tot); b.push_back(0); c.push_back(0); continue; }
    for (int i = tot; i >= 0; --i)
      for (int j = tot - i; j >= 0; --j) { a.push_back(i); b.push_back(j); c.push_back(tot - i - j); }
  }
}

// bfloat16 = the high 16 bits of an IEEE binary32, rounded to nearest even
// (finite inputs only).
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

template <typename T>
T* upload(const std::vector<T>& h) {
  T* d = nullptr;
  if (hipMalloc(&d, h.size() * sizeof(T)) != hipSuccess) throw std::runtime_error("hipMalloc (tables)");
  if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    throw std::runtime_error("hipMemcpy (tables)");
  return d;
}

}  // namespace

void build_host(int dim, int n, std::vector<double>& nodes, std::vector<double>& wts,
                std::vector<double>& logw, std::vector<double>& phi, int& K, int& Q) {
  std::vector<double> x, w;
  gauss_hermite(n, x, w);
  std::vector<int> ia, ib, ic;
  multi_indices(dim, ia, ib, ic);
  K = (int)ia.size();
  Q = dim == 1 ? n : n * n * n;
  nodes.assign((size_t)Q * dim, 0.0);
  wts.assign(Q, 0.0);
  logw.assign(Q, 0.0);
  phi.assign((size_t)Q * K, 0.0);
  const double half_log_2pi = 0.5 * std::log(2.0 * M_PI);
  std::vector<double> px(5), py(5), pz(5);
  for (int p = 0; p < Q; ++p) {
    int i0 = dim == 1 ? p : p / (n * n), i1 = dim == 1 ? 0 : (p / n) % n, i2 = dim == 1 ? 0 : p % n;
    double ux = x[i0], uy = dim == 1 ? 0.0 : x[i1], uz = dim == 1 ? 0.0 : x[i2];
    double wt = dim == 1 ? w[i0] : w[i0] * w[i1] * w[i2];
    nodes[(size_t)p * dim + 0] = ux;
    if (dim == 3) { nodes[(size_t)p * 3 + 1] = uy; nodes[(size_t)p * 3 + 2] = uz; }
    wts[p] = wt;
    logw[p] = std::log(wt) + 0.5 * (ux * ux + uy * uy + uz * uz) + dim * half_log_2pi;
    ortho_hermite(4, ux, px.data());
    ortho_hermite(4, uy, py.data());
    ortho_hermite(4, uz, pz.data());
    for (int k = 0; k < K; ++k) phi[(size_t)p * K + k] = px[ia[k]] * py[ib[k]] * pz[ic[k]];
  }
}

// Operands of the mixed-precision assembly (k_mixed3.hip) in 32-node groups.
// For node group s, k-slot i (0..7) of lane l stands for node
//   32 s + 16 (i / 4) + 4 (l / 16) + i % 4,
// the order in which the exponent MFMA leaves sigma in a lane's registers.
// FP16 tables carry a per-node power-of-two scale: log w~_p + k_p ln 2 in the
// exponent table and Psi 2^-k_p, with k_p = min(15, floor(-log2 w_p)), so that
// sigma 2^k_p <= 2^15 and the tail nodes' large Psi values shrink.
template <typename PhiE, typename Psi>
void build_mixed(mem_ctx_t ctx, const PhiE& phiE, const Psi& psi) {
  using namespace memk;
  const int Q = ctx->Q;
  const int nsg = (Q + 31) / 32;
  const bool f16 = ctx->prec == MEM_PREC_FP16X3;
  ctx->nsg_m = nsg;
  std::vector<int> ks((size_t)nsg * 32, 0);
  if (f16)
    for (int p = 0; p < Q; ++p) {
      const int k = (int)std::floor(-std::log2(ctx->h_w[p]));
      ks[p] = k < 0 ? 0 : (k > 15 ? 15 : k);
    }
  std::vector<float> A((size_t)2 * nsg * NJ * 64);
  for (int g = 0; g < 2 * nsg; ++g)
    for (int j = 0; j < NJ; ++j)
      for (int l = 0; l < 64; ++l) {
        const int p = GRP * g + (l & 15), k = 4 * j + (l >> 4);
        double v = phiE(p, k);
        if (k == 0 && p < Q) v += ks[p] * std::log(2.0);
        A[((size_t)g * NJ + j) * 64 + l] = (float)v;
      }
  auto node = [](int s, int l, int i) { return 32 * s + 16 * (i >> 2) + 4 * (l >> 4) + (i & 3); };
  // FP32 blocks 0..MIX_FB-1 (the 35 moment columns), 16-bit blocks MIX_FB..NBLK-1
  const int nhb = NBLK - MIX_FB;
  std::vector<float> F((size_t)nsg * MIX_FB * 64 * 8);
  std::vector<uint16_t> Hh((size_t)nsg * nhb * 64 * 8), Hl(Hh.size());
  for (int s = 0; s < nsg; ++s)
    for (int l = 0; l < 64; ++l)
      for (int i = 0; i < 8; ++i) {
        const int p = node(s, l, i);
        const double sc = std::ldexp(1.0, -ks[p]);
        for (int b = 0; b < MIX_FB; ++b)
          F[(((size_t)s * MIX_FB + b) * 64 + l) * 8 + i] = (float)(psi(p, 16 * b + (l & 15), false) * sc);
        for (int b = MIX_FB; b < NBLK; ++b) {
          const double v = psi(p, 16 * b + (l & 15), false) * sc;
          const size_t o = (((size_t)s * nhb + (b - MIX_FB)) * 64 + l) * 8 + i;
          if (f16) {
            const _Float16 h = (_Float16)(float)v;
            const _Float16 lo = (_Float16)(float)(v - (double)(float)h);
            Hh[o] = __builtin_bit_cast(uint16_t, h);
            Hl[o] = __builtin_bit_cast(uint16_t, lo);
          } else {
            const uint16_t h = bf16_bits((float)v);
            const uint16_t lo = bf16_bits((float)(v - (double)bf16_value(h)));
            Hh[o] = h;
            Hl[o] = lo;
          }
        }
      }
  ctx->d_phiA_m = upload(A);
  ctx->d_psiF_m = upload(F);
  ctx->d_psi_hi = upload(Hh);
  ctx->d_psi_lo = upload(Hl);
}

void build_tables(mem_ctx_t ctx) {
  const int dim = ctx->dim;
  int K = 0, Q = 0;
  build_host(dim, ctx->n1d, ctx->h_nodes, ctx->h_w, ctx->h_logw, ctx->h_phi, K, Q);
  ctx->K = K;
  ctx->Q = Q;

  if (dim == 1) {
    std::vector<float> t((size_t)Q * 8, 0.f);
    for (int p = 0; p < Q; ++p) {
      for (int k = 0; k < 5; ++k) t[(size_t)p * 8 + k] = (float)ctx->h_phi[(size_t)p * 5 + k];
      t[(size_t)p * 8 + 5] = (float)ctx->h_logw[p];
    }
    ctx->d_tab1 = upload(t);
    ctx->Qpad = Q;
    ctx->ngroups = 0;
    return;
  }

  using namespace memk;
  const int Qpad = (Q + GRP - 1) / GRP * GRP;
  const int ng = Qpad / GRP;
  ctx->Qpad = Qpad;
  ctx->ngroups = ng;
  // exponent operand: PhiE[p][0] = log w~, PhiE[p][k] = phi_k (k = 1..34), [35] = 0
  auto phiE = [&](int p, int k) -> double {
    if (p >= Q) return k == 0 ? (double)NEG_BIG : 0.0;
    if (k == 0) return ctx->h_logw[p];
    if (k >= K3) return 0.0;
    return ctx->h_phi[(size_t)p * K3 + k];
  };
  std::vector<float> A((size_t)ng * NJ * 64);
  for (int g = 0; g < ng; ++g)
    for (int j = 0; j < NJ; ++j)
      for (int l = 0; l < 64; ++l)
        A[((size_t)g * NJ + j) * 64 + l] = (float)phiE(GRP * g + (l & 15), 4 * j + (l >> 4));
  ctx->d_phiA = upload(A);
  // one-dimensional double-float tables of the compensated residual pass:
  // h_a(x_k) = He_a(x_k) / sqrt(a!) for a <= 4 and lw_k = log w_k + x_k^2 / 2 +
  // log(2 pi) / 2 (the 3D log w~ of a node is the sum over its coordinates)
  {
    const int n = ctx->n1d;
    std::vector<double> x, w;
    gauss_hermite(n, x, w);
    std::vector<float2> T1((size_t)6 * n);
    auto split = [](double v) {
      const float h = (float)v;
      return make_float2(h, (float)(v - (double)h));
    };
    double hp[5];
    for (int k = 0; k < n; ++k) {
      ortho_hermite(4, x[k], hp);
      for (int a = 0; a < 5; ++a) T1[(size_t)a * n + k] = split(hp[a]);
      T1[(size_t)5 * n + k] = split(std::log(w[k]) + 0.5 * x[k] * x[k] + 0.5 * std::log(2.0 * M_PI));
    }
    ctx->d_t1 = upload(T1);
  }
  // pair index of each column
  std::vector<int> ci(NCOL, -1), cj(NCOL, -1);
  for (int i = 0; i < K3; ++i)
    for (int j = i; j < K3; ++j) { ci[pair_col(i, j)] = i; cj[pair_col(i, j)] = j; }
  auto psi = [&](int p, int col, bool withx) -> double {
    if (p >= Q || ci[col] < 0) return 0.0;
    double v = ctx->h_phi[(size_t)p * K3 + ci[col]] * ctx->h_phi[(size_t)p * K3 + cj[col]];
    return withx ? v * ctx->h_nodes[(size_t)p * 3] : v;
  };
  // B operand of v_mfma_f32_16x16x4f32 for k-step r of group g:
  // lane l supplies node 16g + 4(l/16) + r, column 16b + l%16; stored as
  // [g][r][b/4][l][b%4] so each lane reads 4 blocks with one 16-byte load.
  auto operand = [&](int nb4, auto&& value) {
    std::vector<float> B((size_t)ng * 4 * nb4 * 64 * 4);
    for (int g = 0; g < ng; ++g)
      for (int r = 0; r < 4; ++r)
        for (int b4 = 0; b4 < nb4; ++b4)
          for (int l = 0; l < 64; ++l)
            for (int q = 0; q < 4; ++q) {
              size_t o = ((((size_t)g * 4 + r) * nb4 + b4) * 64 + l) * 4 + q;
              B[o] = (float)value(GRP * g + 4 * (l >> 4) + r, 16 * (4 * b4 + q) + (l & 15));
            }
    return B;
  };
  ctx->d_psi = upload(operand(10, [&](int p, int col) { return psi(p, col, false); }));

  // Characteristic speeds need C = E[u_x phi phi^T].  Orthonormal Hermite
  // polynomials satisfy x p_a(x) = sqrt(a+1) p_{a+1}(x) + sqrt(a) p_{a-1}(x) at
  // every point, so u_x phi_i = sqrt(a_i+1) phi_{i+e_x} + sqrt(a_i) phi_{i-e_x}
  // node by node and C_ij is a two-term combination of entries of S, except
  // where i and j both have degree 4: there phi_{i+e_x} has degree 5 and
  // E[phi_{i+e_x} phi_j] comes from 120 extra columns (S5).
  std::vector<int> ea, eb, ec;
  multi_indices(3, ea, eb, ec);
  auto index_of = [&](int a, int b, int c) {
    for (int k = 0; k < K3; ++k)
      if (ea[k] == a && eb[k] == b && ec[k] == c) return k;
    return -1;
  };
  auto deg = [&](int k) { return ea[k] + eb[k] + ec[k]; };
  std::vector<int> d4;
  for (int k = 0; k < K3; ++k)
    if (deg(k) == 4) d4.push_back(k);
  std::vector<int> p5i, p5j;  // S5 column -> (i, j), i <= j
  std::vector<int> col5((size_t)K3 * K3, -1);
  for (size_t x = 0; x < d4.size(); ++x)
    for (size_t y = x; y < d4.size(); ++y) {
      col5[(size_t)d4[x] * K3 + d4[y]] = (int)p5i.size();
      p5i.push_back(d4[x]);
      p5j.push_back(d4[y]);
    }
  if ((int)d4.size() != ND4 || (int)p5i.size() != NP5) throw std::runtime_error("degree-4 set");
  std::vector<double> hx(6), hy(6), hz(6);
  ctx->d_psi5 = upload(operand(NC5 / 64, [&](int p, int col) -> double {
    if (p >= Q || col >= NP5) return 0.0;
    const int i = p5i[col], j = p5j[col];
    ortho_hermite(5, ctx->h_nodes[(size_t)p * 3], hx.data());
    ortho_hermite(5, ctx->h_nodes[(size_t)p * 3 + 1], hy.data());
    ortho_hermite(5, ctx->h_nodes[(size_t)p * 3 + 2], hz.data());
    return hx[ea[i] + 1] * hy[eb[i]] * hz[ec[i]] * ctx->h_phi[(size_t)p * K3 + j];
  }));
  // flux-only operand: the 70 columns a flux needs (phi_(100) = u_x)
  ctx->d_psiF = upload(operand(NC5 / 64, [&](int p, int col) -> double {
    if (p >= Q || col >= 2 * K3) return 0.0;
    const double f = ctx->h_phi[(size_t)p * K3 + (col % K3)];
    return col < K3 ? f : f * ctx->h_nodes[(size_t)p * 3];
  }));
  std::vector<int32_t> src(NPAIR);
  std::vector<float2> wts(NPAIR);
  auto scol = [&](int u, int v) { return pair_col(std::min(u, v), std::max(u, v)); };
  for (int i = 0; i < K3; ++i)
    for (int j = i; j < K3; ++j) {
      // raise the lower-degree index (C is symmetric); both of degree 4: S5
      const int r = deg(i) <= 3 ? i : (deg(j) <= 3 ? j : i);
      const int o = r == i ? j : i;
      const int up = index_of(ea[r] + 1, eb[r], ec[r]);
      const int s1 = up >= 0 ? scol(up, o) : 1024 + col5[(size_t)r * K3 + o];
      const int dn = ea[r] > 0 ? index_of(ea[r] - 1, eb[r], ec[r]) : -1;
      const int s2 = dn >= 0 ? scol(dn, o) : s1;
      src[pair_col(i, j)] = s1 | (s2 << 16);
      wts[pair_col(i, j)] = make_float2((float)std::sqrt((double)(ea[r] + 1)),
                                        dn >= 0 ? (float)std::sqrt((double)ea[r]) : 0.f);
    }
  ctx->d_ux_src = upload(src);
  ctx->d_ux_w = upload(wts);
  if (ctx->prec != MEM_PREC_FP32) build_mixed(ctx, phiE, psi);
}

}  // namespace memt
