// Problem set-up and lifetime: level plans, the device arena, checks, pooled pinned
// blocks and capture streams, the Chebyshev bound and the coarse inverse of the
// Stokes hierarchy, and the C ABI for set-up, destruction and problem queries.
#include "runtime.h"

namespace mfs {
namespace rt {

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  while (e--) r *= b;
  return r;
}

LevelGeom make_geom(int dim, const int n[3], int k, int kp) {
  LevelGeom g{};
  g.dim = dim;
  g.k = k;
  g.kp = kp;
  g.ncells = 1;
  g.Nv = 1;
  g.Np = kp > 0 ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = a < dim ? n[a] : 1;
    g.nv[a] = a < dim ? k * n[a] + 1 : 1;
    g.np[a] = (a < dim && kp > 0) ? kp * n[a] + 1 : 1;
    g.ncells *= g.n[a];
    g.Nv *= g.nv[a];
    if (kp > 0) g.Np *= g.np[a];
  }
  return g;
}

int64_t n_vertices(const LevelGeom &g) {
  int64_t v = 1;
  for (int a = 0; a < g.dim; ++a) v *= g.n[a] + 1;
  return v;
}

// level hierarchy: p-levels then h-levels (Sec. 3)
// equal order (Navier-Stokes, Sec. 5): h-levels first, then p-levels
std::vector<LevelGeom> plan_levels_ns(int dim, const int n[3], int k, const mfs_options &o) {
  std::vector<LevelGeom> out;
  out.push_back(make_geom(dim, n, k, k));
  if (!o.mg_levels) return out;
  int nn[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
  while (true) {
    bool ok = true;
    for (int a = 0; a < dim; ++a) ok = ok && (nn[a] % 2 == 0) && (nn[a] > std::max(1, o.coarse_min_cells));
    if (!ok) break;
    for (int a = 0; a < dim; ++a) nn[a] /= 2;
    out.push_back(make_geom(dim, nn, k, k));
  }
  for (int kk = k - 1; kk >= std::max(1, o.p_min); --kk) out.push_back(make_geom(dim, nn, kk, kk));
  return out;
}

std::vector<LevelGeom> plan_levels(int dim, const int n[3], int k, int kp, const mfs_options &o) {
  if (o.pressure_offset == 0) return plan_levels_ns(dim, n, k, o);
  std::vector<LevelGeom> out;
  out.push_back(make_geom(dim, n, k, kp));
  if (!o.mg_levels) return out;
  int nn[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
  int kk = k;
  const int pmin = std::max(1, o.p_min);
  while (kk > pmin) {
    --kk;
    out.push_back(make_geom(dim, nn, kk, 0));
  }
  while (true) {
    bool ok = true;
    for (int a = 0; a < dim; ++a) ok = ok && (nn[a] % 2 == 0) && (nn[a] > std::max(1, o.coarse_min_cells));
    if (!ok) break;
    for (int a = 0; a < dim; ++a) nn[a] /= 2;
    out.push_back(make_geom(dim, nn, kk, 0));
  }
  return out;
}

template <typename T>
void plan_prec_work(Arena &A, PrecWork<T> &w, const std::vector<LevelGeom> &G, int dim, bool full) {
  const int64_t Np = G[0].Np;
  w.pz = A.take<T>(Np);
  w.pinv = A.take<T>(Np);
  if (!full) return;
  const size_t nl = G.size();
  w.x.assign(nl, nullptr);
  w.b.assign(nl, nullptr);
  w.r.assign(nl, nullptr);
  w.d.assign(nl, nullptr);
  for (size_t l = 0; l < nl; ++l) {
    const int64_t nu = dim * G[l].Nv;
    w.x[l] = A.take<T>(nu);
    w.b[l] = A.take<T>(nu);
    w.r[l] = A.take<T>(nu);
    w.d[l] = A.take<T>(nu);
  }
  const int64_t ntot = dim * G[0].Nv + Np;
  w.t_u = A.take<T>(dim * G[0].Nv);
  w.pres = A.take<T>(Np);
  w.ps = A.take<T>(Np);
  w.pp = A.take<T>(Np);
  w.pq = A.take<T>(Np);
  w.full_in = A.take<T>(ntot);
  w.full_out = A.take<T>(ntot);
}

// Navier-Stokes: level vectors are full equal-order vectors ((dim+1) Nv)
template <typename T>
void plan_ns_work(Arena &A, PrecWork<T> &w, const std::vector<LevelGeom> &G, int dim, bool full) {
  if (!full) return;
  const size_t nl = G.size();
  w.x.assign(nl, nullptr);
  w.b.assign(nl, nullptr);
  w.r.assign(nl, nullptr);
  w.d.assign(nl, nullptr);
  for (size_t l = 0; l < nl; ++l) {
    const int64_t n = (dim + 1) * G[l].Nv;
    w.x[l] = A.take<T>(n);
    w.b[l] = A.take<T>(n);
    w.r[l] = A.take<T>(n);
    w.d[l] = A.take<T>(n);
  }
  w.full_in = A.take<T>((dim + 1) * G[0].Nv);
  w.full_out = A.take<T>((dim + 1) * G[0].Nv);
}

// The whole device footprint, carved from one allocation.
void plan_arena(Arena &A, mfs_problem &P, const std::vector<LevelGeom> &G) {
  P.L.resize(G.size());
  if (P.ns) {
    for (size_t l = 0; l < G.size(); ++l) {
      Level &L = P.L[l];
      L.g = G[l];
      const int64_t nvert = n_vertices(G[l]);
      L.X64 = A.take<double>(nvert * P.dim);
      L.X32 = A.take<float>(nvert * P.dim);
      L.tab64 = A.take<double>(TAB_SIZE);
      L.tab32 = A.take<float>(TAB_SIZE);
      L.u0 = A.take<double>((2 * P.dim + 1) * G[l].Nv);  // state [u0 | p0 | u~]
      L.qd64 = A.take<double>(ns_qd_elems(G[l]));
      L.qd32 = A.take<float>(ns_qd_elems(G[l]));
      L.nsinv64 = A.take<double>((P.dim + 1) * G[l].Nv);
      L.nsinv32 = A.take<float>((P.dim + 1) * G[l].Nv);
      if (P.opts.mg_levels && P.opts.relax_type == MFS_RELAX_ASM && l + 1 < G.size()) {
        const int64_t np = asm_patch_size(G[l]);
        L.asm64 = A.take<double>(asm_patch_count(G[l]) * np * np);
        L.asm32 = A.take<float>(asm_patch_count(G[l]) * np * np);
      }
      // FP32 Jacobian: cell-local outputs and a node gather (3D)
      if (P.dim == 3) {
        const int64_t q = G[l].k + 1;
        L.ev32 = A.take<float>(G[l].ncells * 4 * q * q * q);
        L.ev64 = A.take<double>(G[l].ncells * 4 * q * q * q);
      }
      if (l + 1 < G.size()) {
        L.rs64 = A.take<double>(restrict_work_elems(G[l], G[l + 1], P.dim + 1));
        L.rs32 = A.take<float>(restrict_work_elems(G[l], G[l + 1], P.dim + 1));
      }
    }
    const bool full = P.opts.mg_levels != 0;
    plan_ns_work(A, P.w64, G, P.dim, full);
    plan_ns_work(A, P.w32, G, P.dim, full);
    P.coarse_n = full ? (int)((P.dim + 1) * G.back().Nv) : 0;
    P.coarse_inv = A.take<double>((int64_t)P.coarse_n * P.coarse_n);
    const int64_t ntot = (P.dim + 1) * G[0].Nv;
    P.m1 = A.take<double>(G[0].Nv);
    P.scal = A.take<double>(4 * PCG_MAX + 64);
    P.partials = A.take<double>(32 * DOT_BLOCKS);
    P.flags = A.take<int>(64);
    P.tmp_full = A.take<double>(ntot);
    P.tmp2 = A.take<double>(ntot);
    if (full) {  // the BDF2 / Newton driver: history, residual, correction
      P.nw_uh = A.take<double>(P.dim * G[0].Nv);
      P.nw_F = A.take<double>(ntot);
      P.nw_dx = A.take<double>(ntot);
    }
    Krylov &K = P.kr;
    K.m = std::max(1, std::min(P.opts.restart, 30));
    const int64_t nk = full ? ntot : 0;
    K.ld = kr_ld(nk);
    K.V = A.take<double>((K.m + 1) * (nk ? K.ld : 0));
    K.Z = A.take<double>(K.m * (nk ? K.ld : 0));
    K.w = A.take<double>(nk);
    K.dev = A.take<double>(128);
    K.ydev = A.take<double>(64);
    return;
  }
  for (size_t l = 0; l < G.size(); ++l) {
    Level &L = P.L[l];
    L.g = G[l];
    const int64_t nvert = n_vertices(G[l]);
    L.X64 = A.take<double>(nvert * P.dim);
    L.X32 = A.take<float>(nvert * P.dim);
    L.tab64 = A.take<double>(TAB_SIZE);
    L.tab32 = A.take<float>(TAB_SIZE);
    L.diag = A.take<double>(G[l].Nv);
    L.face64 = A.take<double>(q2_face_elems(G[l]) + q1_face_elems(G[l]));
    L.face32 = A.take<float>(q2_face_elems(G[l]) + q1_face_elems(G[l]));
    L.ev64 = A.take<double>(cell_ev_elems(G[l]));
    L.ev32 = A.take<float>(cell_ev_elems(G[l]));
    L.invdiag64 = A.take<double>(G[l].Nv);
    L.invdiag32 = A.take<float>(G[l].Nv);
    if (l + 1 < G.size()) {
      L.rs64 = A.take<double>(restrict_work_elems(G[l], G[l + 1], P.dim));
      L.rs32 = A.take<float>(restrict_work_elems(G[l], G[l + 1], P.dim));
    }
  }
  const bool full = P.opts.mg_levels != 0;
  plan_prec_work(A, P.w64, G, P.dim, full);
  plan_prec_work(A, P.w32, G, P.dim, full);
  const LevelGeom &c = G.back();
  P.coarse_n = full ? (int)(P.dim * c.Nv) : 0;
  P.coarse_inv = A.take<double>((int64_t)P.coarse_n * P.coarse_n);
  const int64_t ntot = P.dim * G[0].Nv + G[0].Np;
  P.m1 = A.take<double>(std::max<int64_t>(G[0].Np, 1));
  P.scal = A.take<double>(4 * PCG_MAX + 64);
  P.partials = A.take<double>(32 * DOT_BLOCKS);
  P.tmp_full = A.take<double>(ntot);
  Krylov &K = P.kr;
  K.m = std::max(1, std::min(P.opts.restart, 30));
  const int64_t nk = full ? ntot : 0;  // Krylov space only when the solver is available
  K.ld = kr_ld(nk);
  K.V = A.take<double>((K.m + 1) * (nk ? K.ld : 0));
  K.Z = A.take<double>(K.m * (nk ? K.ld : 0));
  K.w = A.take<double>(nk);
  K.dev = A.take<double>(128);
  K.ydev = A.take<double>(64);
}

// every cell an axis-aligned box: coordinate a of a vertex depends on its
// index along a only
bool cartesian_grid(const std::vector<double> &X, const LevelGeom &g) {
  const int d = g.dim;
  const int m0 = g.n[0] + 1, m1 = g.n[1] + 1, m2 = d == 3 ? g.n[2] + 1 : 1;
  for (int z = 0; z < m2; ++z)
    for (int y = 0; y < m1; ++y)
      for (int x = 0; x < m0; ++x) {
        const int64_t v = x + (int64_t)m0 * (y + (int64_t)m1 * z);
        const int idx[3] = {x, y, z};
        for (int a = 0; a < d; ++a) {
          int r[3] = {0, 0, 0};
          r[a] = idx[a];
          const int64_t ref = r[0] + (int64_t)m0 * (r[1] + (int64_t)m1 * r[2]);
          if (X[v * d + a] != X[ref * d + a]) return false;
        }
      }
  return true;
}

void check_options(const mfs_options &o) {
  MFS_REQUIRE(o.cheb_degree >= 1 && o.cheb_degree <= 32, MFS_EINVAL, "cheb_degree %d out of range", o.cheb_degree);
  MFS_REQUIRE(o.cheb_range > 1.0, MFS_EINVAL, "cheb_range must exceed 1");
  MFS_REQUIRE(o.restart >= 1 && o.restart <= 30, MFS_EINVAL, "restart must be in [1, 30]");
  MFS_REQUIRE(o.schur_iterations >= 0 && o.schur_iterations < PCG_MAX, MFS_EINVAL, "schur_iterations out of range");
  MFS_REQUIRE(o.precond_precision == MFS_FP32 || o.precond_precision == MFS_FP64, MFS_EINVAL,
              "precond_precision must be MFS_FP32 or MFS_FP64");
  MFS_REQUIRE(o.relax_steps >= 1 && o.relax_steps <= 64, MFS_EINVAL, "relax_steps out of range");
  MFS_REQUIRE(o.relax_omega > 0 && o.relax_omega < 2, MFS_EINVAL, "relax_omega must be in (0, 2)");
  MFS_REQUIRE(o.relax_type == MFS_RELAX_JACOBI || o.relax_type == MFS_RELAX_ASM, MFS_EINVAL,
              "relax_type must be MFS_RELAX_JACOBI or MFS_RELAX_ASM");
}

void check_mesh(const mfs_mesh *mesh, int k, const mfs_options &o) {
  MFS_REQUIRE(mesh != nullptr, MFS_EINVAL, "mesh is NULL");
  MFS_REQUIRE(mesh->dim == 2 || mesh->dim == 3, MFS_EINVAL, "dim must be 2 or 3 (got %d)", mesh->dim);
  for (int a = 0; a < mesh->dim; ++a) MFS_REQUIRE(mesh->n[a] >= 1, MFS_EINVAL, "n[%d] must be >= 1", a);
  MFS_REQUIRE(k >= 1 && k <= 6, MFS_EINVAL, "degree k=%d out of range [1, 6]", k);
  if (o.pressure_offset == 1) MFS_REQUIRE(k >= 2, MFS_EINVAL, "Taylor-Hood needs k >= 2");
  if (o.pressure_offset == 0) {
    MFS_REQUIRE(k <= 3, MFS_EUNSUPPORTED, "Navier-Stokes operator supports k <= 3 (got %d)", k);
    MFS_REQUIRE(!o.mg_levels || k <= 2, MFS_EUNSUPPORTED,
                "Navier-Stokes multigrid needs nested nodes, k <= 2 (got %d)", k);
  }
  MFS_REQUIRE(o.pressure_offset == 0 || o.pressure_offset == 1, MFS_EINVAL, "pressure_offset must be 0 or 1");
  int64_t nodes = 1;
  for (int a = 0; a < mesh->dim; ++a) nodes *= (int64_t)k * mesh->n[a] + 1;
  MFS_REQUIRE(nodes < (1LL << 31) / mesh->dim, MFS_EINVAL, "mesh too large for 32-bit node grid");
}

// Pinned readback blocks and capture streams are kept in process-wide free
// lists and reused by later problems: freeing pinned memory or destroying a
// stream waits for the whole device, which would stall the other problems
// of a request loop every time one of them completes.
constexpr int PINNED_DOUBLES = 192;  // Krylov readback (128) + coefficients (64)
std::mutex g_pool_mu;
std::vector<double *> g_pinned_free;
std::vector<hipStream_t> g_stream_free;

double *pinned_acquire() {
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (!g_pinned_free.empty()) {
      double *p = g_pinned_free.back();
      g_pinned_free.pop_back();
      return p;
    }
  }
  double *p = nullptr;
  MFS_HIP(hipHostMalloc(&p, PINNED_DOUBLES * sizeof(double)));
  return p;
}

hipStream_t capture_stream_acquire() {
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (!g_stream_free.empty()) {
      hipStream_t st = g_stream_free.back();
      g_stream_free.pop_back();
      return st;
    }
  }
  hipStream_t st = nullptr;
  MFS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  return st;
}

void release(mfs_problem *P) {
  if (!P) return;
  for (int i = 0; i < 2; ++i)
    if (P->prec_graph[i]) (void)hipGraphExecDestroy(P->prec_graph[i]);
  if (P->kr.ev) (void)hipEventDestroy(P->kr.ev);
  if (P->kr.ev_pre) (void)hipEventDestroy(P->kr.ev_pre);
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (P->cap_stream) g_stream_free.push_back(P->cap_stream);
    if (P->kr.host) g_pinned_free.push_back(P->kr.host);
  }
  if (P->arena && P->arena_owned) (void)hipFree(P->arena);
  delete P->hp;
  delete P->amr;
  delete P;
}

// ---------------------------------------------------------------- setup pieces
void sturm_max_eig(const std::vector<double> &d, const std::vector<double> &e, double &lmax) {
  // largest eigenvalue of the symmetric tridiagonal (d, e) by bisection
  const int n = (int)d.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0) + (i < n - 1 ? std::fabs(e[i]) : 0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
      const double qq = q == 0 ? 1e-300 : q;
      q = d[i] - x - e[i - 1] * e[i - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= n)
      hi = mid;
    else
      lo = mid;
  }
  lmax = hi;
}

uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// lambda_max(D^{-1} A) on level l by CG-Lanczos (FP64, host-synchronous)
double estimate_lambda(mfs_problem &P, int l, hipStream_t s) {
  Level &L = P.L[l];
  const int64_t n = P.dim * L.g.Nv;
  double *r = P.w64.x[l], *z = P.w64.b[l], *p = P.w64.r[l], *q = P.w64.d[l];
  std::vector<double> h(n);
  uint64_t st = P.opts.seed * 1000003ULL + (uint64_t)l;
  for (int64_t i = 0; i < n; ++i) h[i] = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  MFS_HIP(hipMemcpyAsync(r, h.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  vec_zero_mask_boundary<double>(L.g, r, s);
  double *dv = P.scal + 4 * PCG_MAX;
  auto dot = [&](const double *a, const double *b) {
    multi_dot<double>(a, 0, 1, b, n, dv, P.partials, s);
    double v;
    MFS_HIP(hipMemcpyAsync(&v, dv, sizeof(double), hipMemcpyDeviceToHost, s));
    MFS_HIP(hipStreamSynchronize(s));
    return v;
  };
  vec_diag_scale<double>(L.g, z, L.invdiag64, r, s);
  vec_copy<double>(p, z, n, s);
  double rz = dot(r, z);
  std::vector<double> alpha, beta;
  const int steps = std::max(2, P.opts.lanczos_steps);
  for (int j = 0; j < steps && rz > 0; ++j) {
    apply_A<double>(P, l, q, p, s);
    vec_zero_mask_boundary<double>(L.g, q, s);
    const double pq = dot(p, q);
    if (!(pq > 0)) break;
    const double a = rz / pq;
    vec_axpby<double>(r, -a, q, 1.0, n, s);
    vec_diag_scale<double>(L.g, z, L.invdiag64, r, s);
    const double rz2 = dot(r, z);
    const double b = rz2 / rz;
    vec_axpby<double>(p, 1.0, z, b, n, s);
    alpha.push_back(a);
    beta.push_back(b);
    rz = rz2;
    if (rz2 <= 1e-30 * rz) break;
  }
  const int m = (int)alpha.size();
  MFS_REQUIRE(m > 0, MFS_EINVAL, "Lanczos estimate failed on level %d", l);
  std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
  for (int j = 0; j < m; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j < m - 1) e[j] = std::sqrt(beta[j]) / alpha[j];
  }
  double lmax;
  sturm_max_eig(d, e, lmax);
  return lmax;
}

void setup_coarse(mfs_problem &P, hipStream_t s) {
  const int l = P.nlev - 1;
  const Level &L = P.L[l];
  const int n = P.coarse_n;
  // columns of the constrained coarse A by applying it to unit vectors
  double *e = P.w64.x[l], *col = P.w64.b[l];
  std::vector<double> A((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    vec_fill<double>(e, 0.0, n, s);
    const double one = 1.0;
    MFS_HIP(hipMemcpyAsync(e + j, &one, sizeof(double), hipMemcpyHostToDevice, s));
    apply_A<double>(P, l, col, e, s);
    MFS_HIP(hipMemcpyAsync(A.data() + (size_t)j * n, col, n * sizeof(double), hipMemcpyDeviceToHost, s));
    MFS_HIP(hipStreamSynchronize(s));
  }
  // symmetrise (equal up to rounding), Cholesky, explicit inverse
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
  std::vector<double> Lc((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double sdiag = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) sdiag -= Lc[(size_t)j * n + k] * Lc[(size_t)j * n + k];
    MFS_REQUIRE(sdiag > 0, MFS_EINVAL, "coarse matrix not positive definite");
    const double ljj = std::sqrt(sdiag);
    Lc[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * n + k] * Lc[(size_t)j * n + k];
      Lc[(size_t)i * n + j] = v / ljj;
    }
  }
  std::vector<double> inv((size_t)n * n, 0.0);
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * n + k] * y[k];
      y[i] = v / Lc[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < n; ++k) v -= Lc[(size_t)k * n + i] * inv[(size_t)c * n + k];
      inv[(size_t)c * n + i] = v / Lc[(size_t)i * n + i];
    }
  }
  MFS_HIP(hipMemcpyAsync(P.coarse_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MFS_HIP(hipStreamSynchronize(s));
}

int guard(const std::function<void()> &f) {
  try {
    f();
    return MFS_OK;
  } catch (const mfs::Error &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return MFS_ENOMEM;
  } catch (...) {
    set_error("unexpected exception");
    return MFS_EINVAL;
  }
}

std::vector<LevelGeom> levels_for(const mfs_mesh *mesh, int k, const mfs_options &o) {
  const int kp = o.pressure_offset == 1 ? k - 1 : k;
  return plan_levels(mesh->dim, mesh->n, k, kp, o);
}

int setup_structured(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *arena, size_t bytes,
                     void *stream, mfs_problem **out) {
  mfs_problem *P = nullptr;
  int rc = guard([&] {
    MFS_REQUIRE(out != nullptr, MFS_EINVAL, "out is NULL");
    *out = nullptr;
    mfs_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_options(&o);
    check_mesh(mesh, k, o);
    check_options(o);
    MFS_REQUIRE(mesh->vertices != nullptr, MFS_EINVAL, "vertices is NULL");
    MFS_REQUIRE(nu > 0, MFS_EINVAL, "nu must be positive");
    P = new mfs_problem();
    P->dim = mesh->dim;
    P->nu = nu;
    P->opts = o;
    P->ns = o.pressure_offset == 0;
    hipStream_t s = S(stream);
    P->stream = s;
    auto G = levels_for(mesh, k, o);
    P->nlev = (int)G.size();
    Arena dry;
    plan_arena(dry, *P, G);
    P->arena_bytes = dry.off;
    if (arena) {
      MFS_REQUIRE(bytes >= P->arena_bytes, MFS_ENOMEM, "arena of %zu bytes, the problem needs %zu (mfs_footprint)",
                  bytes, P->arena_bytes);
      MFS_REQUIRE(reinterpret_cast<uintptr_t>(arena) % 256 == 0, MFS_EINVAL, "arena must be 256-byte aligned");
      P->arena = static_cast<char *>(arena);
      P->arena_owned = false;
    } else {
      MFS_HIP(hipMalloc(&P->arena, P->arena_bytes));
    }
    Arena A;
    A.dry = false;
    A.base = P->arena;
    plan_arena(A, *P, G);
    P->kr.host = pinned_acquire();
    P->kr.yhost = P->kr.host + 128;
    MFS_HIP(hipEventCreateWithFlags(&P->kr.ev, hipEventDisableTiming));
    MFS_HIP(hipEventCreateWithFlags(&P->kr.ev_pre, hipEventDisableTiming));
    // vertices per level: fine vertices at indices divisible by 2^h
    const int dim = mesh->dim;
    int hl = 0;
    for (int l = 0; l < P->nlev; ++l) {
      Level &L = P->L[l];
      if (l > 0 && L.g.n[0] != P->L[l - 1].g.n[0]) ++hl;
      const int st = 1 << hl;
      const int64_t nvert = n_vertices(L.g);
      L.Xhost.resize(nvert * dim);
      const int fn0 = mesh->n[0] + 1, fn1 = mesh->n[1] + 1;
      for (int z = 0; z < (dim == 3 ? L.g.n[2] + 1 : 1); ++z)
        for (int y = 0; y <= L.g.n[1]; ++y)
          for (int x = 0; x <= L.g.n[0]; ++x) {
            const int64_t v = x + (int64_t)(L.g.n[0] + 1) * (y + (int64_t)(L.g.n[1] + 1) * z);
            const int64_t fv = (int64_t)x * st + (int64_t)fn0 * ((int64_t)y * st + (int64_t)fn1 * z * st);
            for (int a = 0; a < dim; ++a) L.Xhost[v * dim + a] = mesh->vertices[fv * dim + a];
          }
      L.g.cart = cartesian_grid(L.Xhost, L.g) ? 1 : 0;
      std::vector<float> X32(L.Xhost.begin(), L.Xhost.end());
      MFS_HIP(hipMemcpyAsync(L.X64, L.Xhost.data(), L.Xhost.size() * sizeof(double), hipMemcpyHostToDevice, s));
      MFS_HIP(hipMemcpyAsync(L.X32, X32.data(), X32.size() * sizeof(float), hipMemcpyHostToDevice, s));
      auto tab = make_tables(L.g.k, L.g.kp);
      L.tabh = tab;
      std::vector<float> tab32(tab.begin(), tab.end());
      MFS_HIP(hipMemcpyAsync(L.tab64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
      MFS_HIP(hipMemcpyAsync(L.tab32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice, s));
      MFS_HIP(hipStreamSynchronize(s));
      if (l + 1 < P->nlev) {
        const LevelGeom &c = G[l + 1];
        L.h_to_coarser = c.n[0] != L.g.n[0];
        L.emb = L.h_to_coarser ? h_embedding(c.k) : p_embedding(L.g.k, c.k);
      }
    }
    // geometry check on the finest level
    {
      Level &L = P->L[0];
      int *bad = reinterpret_cast<int *>(P->scal);
      vec_fill<int>(bad, 0x7fffffff, 1, s);
      launch_check_geometry(L.g, L.X64, L.tab64, bad, s);
      int hb = 0;
      MFS_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
      MFS_HIP(hipStreamSynchronize(s));
      MFS_REQUIRE(hb == 0x7fffffff, MFS_EINVAL, "non-positive Jacobian determinant in cell %d", hb);
    }
    if (P->ns) {
      // everything operator-specific waits for mfs_set_linearization
      vec_fill<double>(P->m1, 1.0, P->L[0].g.Nv, s);
      MFS_HIP(hipStreamSynchronize(s));
      *out = P;
      return;
    }
    // diagonals
    for (int l = 0; l < P->nlev; ++l) {
      Level &L = P->L[l];
      vec_fill<double>(L.diag, 0.0, L.g.Nv, s);
      launch_laplace_diagonal(L.g, L.X64, L.tab64, nu, L.diag, s);
      vec_invert_diag(L.g, L.diag, L.invdiag64, L.invdiag32, s);
    }
    // pressure mass: M_p 1 (for the pressure mean) and 1/diag(M_p) for Jacobi-PCG
    if (P->L[0].g.Np > 0) {
      Level &L = P->L[0];
      const LevelGeom &g = L.g;
      double *ones = P->tmp_full;
      vec_fill<double>(ones, 1.0, g.Np, s);
      apply_op<double>(*P, MFS_OP_MASS_P, 0, P->m1, ones, s);
      double *pd = P->w64.pz;  // scratch: diag(M_p)
      vec_fill<double>(pd, 0.0, g.Np, s);
      launch_mass_diagonal(g, L.X64, L.tab64, pd, s);
      vec_fill<double>(ones, 1.0, g.Np, s);
      launch_reciprocal(P->w64.pinv, P->w32.pinv, pd, g.Np, s);
    }
    // Chebyshev bounds and the coarse inverse
    if (o.mg_levels) {
      for (int l = 0; l + 1 < P->nlev; ++l) P->L[l].lambda = o.cheb_safety * estimate_lambda(*P, l, s);
      setup_coarse(*P, s);
    }
    MFS_HIP(hipStreamSynchronize(s));
    *out = P;
  });
  if (rc != MFS_OK) {
    release(P);
    return rc;
  }
  return MFS_OK;
}

void check_problem(const mfs_problem *p) { MFS_REQUIRE(p != nullptr, MFS_EINVAL, "problem is NULL"); }

void check_level(const mfs_problem *p, int level) {
  check_problem(p);
  MFS_REQUIRE(level >= 0 && level < p->namr + p->nhp + p->nlev, MFS_EINVAL, "level %d out of range [0, %d)", level,
              p->namr + p->nhp + p->nlev);
}

void no_amr(const mfs_problem *p, const char *what) {
  check_problem(p);
  MFS_REQUIRE(!p->amr, MFS_EUNSUPPORTED, "%s is not available on a refined-mesh problem", what);
}

void check_prec(int prec) {
  MFS_REQUIRE(prec == MFS_FP32 || prec == MFS_FP64, MFS_EINVAL, "precision must be MFS_FP32 or MFS_FP64");
}

// instantiations used by the other parts of the runtime
template void plan_prec_work<float>(Arena &A, PrecWork<float> &w, const std::vector<LevelGeom> &G, int dim, bool full);
template void plan_prec_work<double>(Arena &A, PrecWork<double> &w, const std::vector<LevelGeom> &G, int dim, bool full);
template void plan_ns_work<float>(Arena &A, PrecWork<float> &w, const std::vector<LevelGeom> &G, int dim, bool full);
template void plan_ns_work<double>(Arena &A, PrecWork<double> &w, const std::vector<LevelGeom> &G, int dim, bool full);

}  // namespace rt
}  // namespace mfs

extern "C" {

void mfs_default_options(mfs_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->pressure_offset = 1;
  o->mg_levels = 1;
  o->cheb_degree = 5;
  o->cheb_range = 20.0;
  o->cheb_safety = 1.2;
  o->lanczos_steps = 20;
  o->p_min = 1;
  o->coarse_min_cells = 2;
  o->schur_iterations = 10;
  o->restart = 30;
  o->maxit = 200;
  o->rtol = 1e-8;
  o->precond_precision = MFS_FP32;
  o->seed = 0;
  o->relax_steps = 5;
  o->relax_omega = 0.5;
  o->graphs = 1;
  o->relax_type = MFS_RELAX_JACOBI;
}

const char *mfs_last_error(void) { return get_error(); }

int mfs_footprint(const mfs_mesh *mesh, int k, const mfs_options *opts, size_t *bytes) {
  return guard([&] {
    mfs_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_options(&o);
    check_mesh(mesh, k, o);
    check_options(o);
    MFS_REQUIRE(bytes != nullptr, MFS_EINVAL, "bytes is NULL");
    auto G = levels_for(mesh, k, o);
    mfs_problem P;
    P.dim = mesh->dim;
    P.opts = o;
    P.ns = o.pressure_offset == 0;
    Arena A;
    plan_arena(A, P, G);
    *bytes = A.off;
  });
}

int mfs_setup(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *stream, mfs_problem **out) {
  return setup_structured(mesh, k, nu, opts, nullptr, 0, stream, out);
}

int mfs_setup_arena(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *arena, size_t bytes,
                    void *stream, mfs_problem **out) {
  if (arena == nullptr) {
    set_error("arena is NULL");
    return MFS_EINVAL;
  }
  return setup_structured(mesh, k, nu, opts, arena, bytes, stream, out);
}

int mfs_destroy(mfs_problem *p) {
  release(p);
  return MFS_OK;
}

int mfs_n_dofs(const mfs_problem *p, int level, int64_t *n_u, int64_t *n_p) {
  return guard([&] {
    check_level(p, level);
    if (p->amr) {
      if (level < p->namr) {
        if (n_u) *n_u = p->amr->lev[level].N;
        if (n_p) *n_p = p->amr->lev[level].N;
        return;
      }
      level -= p->namr;
    }
    if (level < p->nhp) {
      if (n_u) *n_u = p->hp->lev[level].V.N;
      if (n_p) *n_p = level == 0 ? p->hp->Pr.N : 0;
      return;
    }
    const int l = level - p->nhp;
    if (n_u) *n_u = p->L[l].g.Nv;
    if (n_p) *n_p = p->hp ? 0 : p->L[l].g.Np;
  });
}

int mfs_n_levels(const mfs_problem *p, int *n) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(n != nullptr, MFS_EINVAL, "n is NULL");
    *n = p->namr + p->nhp + p->nlev;
  });
}

int mfs_level_info(const mfs_problem *p, int level, int *k, int *n) {
  return guard([&] {
    check_level(p, level);
    if (p->amr) {
      if (level < p->namr) {
        if (k) *k = p->amr->k;
        if (n)
          for (int a = 0; a < 3; ++a) n[a] = p->amr->n;
        return;
      }
      level -= p->namr;
    }
    if (level < p->nhp) {
      const auto &d = p->hp->lev[level].V.deg;
      if (k) *k = *std::max_element(d.begin(), d.end());
      if (n)
        for (int a = 0; a < 3; ++a) n[a] = p->hp->n[a];
      return;
    }
    const int l = level - p->nhp;
    if (k) *k = p->L[l].g.k;
    if (n)
      for (int a = 0; a < 3; ++a) n[a] = p->L[l].g.n[a];
  });
}

int mfs_support_points(const mfs_problem *p, int deg, double *xyz) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(!p->hp, MFS_EUNSUPPORTED, "support points of hp spaces are not provided");
    MFS_REQUIRE(deg >= 1 && deg <= 7, MFS_EINVAL, "degree out of range");
    MFS_REQUIRE(xyz != nullptr, MFS_EINVAL, "buffer is NULL");
    if (p->amr) {
      const AmrSpaceHost &A = p->amr->lev[0].S;
      MFS_REQUIRE(deg == A.k, MFS_EUNSUPPORTED, "refined meshes provide the points of degree %d", A.k);
      for (int64_t i = 0; i < 3 * A.N; ++i) xyz[i] = (double)A.tpos[i] / (double)A.R;
      return;
    }
    const Level &L = p->L[0];
    const int dim = p->dim;
    const auto nodes = gll_nodes(deg);
    int nn[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) nn[a] = deg * L.g.n[a] + 1;
    for (int z = 0; z < nn[2]; ++z)
      for (int y = 0; y < nn[1]; ++y)
        for (int x = 0; x < nn[0]; ++x) {
          const int g[3] = {x, y, z};
          int c[3] = {0, 0, 0};
          double xi[3] = {0, 0, 0};
          for (int a = 0; a < dim; ++a) {
            c[a] = std::min(g[a] / deg, L.g.n[a] - 1);
            xi[a] = nodes[g[a] - deg * c[a]];
          }
          const int64_t id = x + (int64_t)nn[0] * (y + (int64_t)nn[1] * z);
          for (int a = 0; a < dim; ++a) {
            double v = 0;
            for (int vtx = 0; vtx < (1 << dim); ++vtx) {
              double f = 1;
              int vi[3] = {0, 0, 0};
              for (int b = 0; b < dim; ++b) {
                const int hi = (vtx >> b) & 1;
                f *= hi ? xi[b] : 1.0 - xi[b];
                vi[b] = c[b] + hi;
              }
              const int64_t vid = vi[0] + (int64_t)(L.g.n[0] + 1) * (vi[1] + (int64_t)(L.g.n[1] + 1) * vi[2]);
              v += f * L.Xhost[vid * dim + a];
            }
            xyz[id * dim + a] = v;
          }
        }
  });
}

int mfs_quadrature_points(const mfs_problem *p, double *xyz) {
  return guard([&] {
    no_amr(p, "quadrature points");
    MFS_REQUIRE(xyz != nullptr, MFS_EINVAL, "buffer is NULL");
    const Level &L = p->L[0];
    const int64_t nq = L.g.ncells * ipow(L.g.k + 1, p->dim) * p->dim;
    double *d = nullptr;
    MFS_HIP(hipMalloc(&d, nq * sizeof(double)));
    launch_quadrature_points(L.g, L.X64, L.tab64, d, p->stream);
    hipError_t e = hipMemcpyAsync(xyz, d, nq * sizeof(double), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(d);
    MFS_HIP(e);
  });
}

int mfs_quadrature_points_device(const mfs_problem *p, double *xyz, void *stream) {
  return guard([&] {
    no_amr(p, "quadrature points");
    check_problem(p);
    MFS_REQUIRE(xyz != nullptr, MFS_EINVAL, "buffer is NULL");
    const Level &L = p->L[0];
    launch_quadrature_points(L.g, L.X64, L.tab64, xyz, S(stream));
  });
}

int mfs_get_lambda(const mfs_problem *p, int level, double *lambda) {
  return guard([&] {
    no_amr(p, "mfs_get_lambda");
    check_level(p, level);
    MFS_REQUIRE(lambda != nullptr, MFS_EINVAL, "NULL output");
    *lambda = level < p->nhp ? p->hp->lev[level].lambda : p->L[level - p->nhp].lambda;
  });
}

int mfs_set_lambda(mfs_problem *p, int level, double lambda) {
  return guard([&] {
    no_amr(p, "mfs_set_lambda");
    check_level(p, level);
    MFS_REQUIRE(lambda > 0, MFS_EINVAL, "lambda must be positive");
    if (level < p->nhp)
      p->hp->lev[level].lambda = lambda;
    else
      p->L[level - p->nhp].lambda = lambda;
    drop_prec_graph(*p);
  });
}

}  // extern "C"
