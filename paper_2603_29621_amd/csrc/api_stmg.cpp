// hp space-time multigrid (hp-STMG) for the transient Stokes stage system of
// Sec. 4: FGMRES preconditioned by one V-cycle on the Kronecker operator
// G_Q (x) M + tau I_Q (x) A of eq. (proceedings-kronecker).
//
// Levels, by the two coarsening rules of Sec. 4 (space before time,
// polynomial before geometric) without geometric coarsening in time: the
// spatial degree k -> 2, then h while every n is even and larger than 2,
// both at the temporal degree kt, then kt -> 0 on the coarsest mesh (modes
// smooth in space and of high degree in time then meet a coarse level before
// the temporal degree drops).  Every level is a
// Taylor-Hood space with its own operator-only problem (the spatial
// operators, the velocity mass, the Kronecker operator of api_spacetime.cpp).
// Transfers: per stage the constrained velocity transfer and the same
// transfer unconstrained for the degree-(k-1) pressure (the restriction their
// transpose); in time the coarse DG polynomial at the fine nodes, restricted
// by M_c^{-1} P^T M_f (the stage rows are mass-scaled, so the coarse temporal
// operator is the Galerkin one).  Smoother: additive Schwarz over vertex-star
// patches with the whole slab in time (asm_kernels.hip); its patch matrices
// G (x) M_J + tau I (x) A_J come from probing the spatial Stokes operator and
// velocity mass.  Coarsest level: the dense inverse of the operator with the
// first pressure node of every stage pinned to zero.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "runtime.h"

using namespace mfs;
using namespace mfs::rt;

namespace {

// in-place inverse of the row-major n x n matrix A (partial pivoting); false
// when singular
bool invert_dense(std::vector<double> &A, int n) {
  std::vector<int> perm(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)p * n + k])) p = i;
    perm[k] = p;
    if (!(std::fabs(A[(size_t)p * n + k]) > 0.0)) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
    const double ip = 1.0 / A[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) A[(size_t)k * n + j] *= ip;
    A[(size_t)k * n + k] = ip;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[(size_t)i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      A[(size_t)i * n + k] = -f * ip;
    }
  }
  for (int k = n - 1; k >= 0; --k)
    if (perm[k] != k)
      for (int i = 0; i < n; ++i) std::swap(A[(size_t)i * n + k], A[(size_t)i * n + perm[k]]);
  return true;
}

// DG(kt) temporal matrices on the reference slab [0, 1] with the nodal basis
// on the kt+1 Gauss points: M_Q, and G_Q = M_Q^{-1} A_Q with A_Q the
// derivative plus the upwind jump phi_j(0) phi_i(0) (row-major Q x Q)
void dg_time(int kt, std::vector<double> &G, std::vector<double> &M) {
  const int Q = kt + 1;
  std::vector<double> s, ws, t, w;
  gauss_rule(Q, s, ws);
  gauss_rule(Q + 1, t, w);  // exact for the degree-2kt integrands
  const std::vector<double> V = lagrange_values(s, t), D = lagrange_derivs(s, t);
  const std::vector<double> v0 = lagrange_values(s, std::vector<double>{0.0});
  M.assign((size_t)Q * Q, 0.0);
  std::vector<double> A((size_t)Q * Q, 0.0);
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      double m = 0, a = 0;
      for (size_t p = 0; p < t.size(); ++p) {
        m += w[p] * V[p * Q + i] * V[p * Q + j];
        a += w[p] * V[p * Q + i] * D[p * Q + j];
      }
      M[(size_t)i * Q + j] = m;
      A[(size_t)i * Q + j] = a + v0[j] * v0[i];
    }
  std::vector<double> Mi = M;
  MFS_REQUIRE(invert_dense(Mi, Q), MFS_EINVAL, "singular temporal mass");
  G.assign((size_t)Q * Q, 0.0);
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      for (int l = 0; l < Q; ++l) G[(size_t)i * Q + j] += Mi[(size_t)i * Q + l] * A[(size_t)l * Q + j];
}

// P_tau [Qf][Qc]: the DG(kc) polynomial at the DG(kf) nodes; R_tau [Qc][Qf] =
// M_c^{-1} P_tau^T M_f
void time_transfers(int kf, int kc, StageCoef &P, StageCoef &R) {
  const int Qf = kf + 1, Qc = kc + 1;
  std::vector<double> sf, wf, sc, wc, Gf, Mf, Gc, Mc;
  gauss_rule(Qf, sf, wf);
  gauss_rule(Qc, sc, wc);
  const std::vector<double> Pt = lagrange_values(sc, sf);  // [i fine][j coarse]
  dg_time(kf, Gf, Mf);
  dg_time(kc, Gc, Mc);
  MFS_REQUIRE(invert_dense(Mc, Qc), MFS_EINVAL, "singular temporal mass");
  std::vector<double> PtM((size_t)Qc * Qf, 0.0);  // P^T M_f
  for (int a = 0; a < Qc; ++a)
    for (int b = 0; b < Qf; ++b)
      for (int i = 0; i < Qf; ++i) PtM[(size_t)a * Qf + b] += Pt[(size_t)i * Qc + a] * Mf[(size_t)i * Qf + b];
  P = StageCoef{};
  R = StageCoef{};
  for (int i = 0; i < Qf; ++i)
    for (int j = 0; j < Qc; ++j) P.c[i * MFS_MAX_STAGES + j] = Pt[(size_t)i * Qc + j];
  for (int a = 0; a < Qc; ++a)
    for (int b = 0; b < Qf; ++b) {
      double v = 0;
      for (int l = 0; l < Qc; ++l) v += Mc[(size_t)a * Qc + l] * PtM[(size_t)l * Qf + b];
      R.c[a * MFS_MAX_STAGES + b] = v;
    }
}

// the pressure grid of a Taylor-Hood level as a scalar grid of degree kp
LevelGeom pressure_grid(const LevelGeom &g) {
  LevelGeom p = g;
  p.k = g.kp;
  p.kp = 0;
  for (int a = 0; a < 3; ++a) p.nv[a] = g.np[a];
  p.Nv = g.Np;
  p.Np = 0;
  return p;
}

}  // namespace

// level vectors of one precision
template <typename T>
struct StBuf {
  T *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr, *work = nullptr;
  T *Kinv = nullptr;                   // space-time patch inverses (all levels but the coarsest)
  T *rw_v = nullptr, *rw_p = nullptr;  // scratch of the three-pass restrictions to the next level
};

struct StLevel {
  int sp = 0;       // spatial problem
  int kt = 0, Q = 1;
  int64_t N = 0;    // entries per stage: dim Nv + Np
  std::vector<double> G;
  StBuf<double> d;  // FP64 V-cycle
  StBuf<float> f;   // FP32 V-cycle (inside the FP64 FGMRES)
  int kind = 0;     // transfer to the next level: 1 time, 2 space
  bool h = false;
  std::vector<double> emb_v, emb_p;
  StageCoef Pt{}, Rt{};
};

template <typename T>
StBuf<T> &buf(StLevel &L);
template <>
StBuf<double> &buf<double>(StLevel &L) {
  return L.d;
}
template <>
StBuf<float> &buf<float>(StLevel &L) {
  return L.f;
}

struct mfs_stmg {
  int dim = 2;
  double tau = 0.0, omega = 0.5;
  int steps = 2;
  std::vector<mfs_problem *> sp;
  std::vector<LevelGeom> pg;  // pressure grids of the spatial problems
  std::vector<StLevel> lev;
  double *coarse_inv = nullptr;
  int coarse_n = 0;
  // FGMRES (level 0)
  int m = 30;
  int64_t ld = 0;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *dev = nullptr, *ydev = nullptr, *partials = nullptr;
  hipStream_t s = nullptr;
  std::vector<void *> allocs;
  template <typename T>
  T *alloc(int64_t n) {
    void *p = nullptr;
    MFS_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(T)));
    allocs.push_back(p);
    return static_cast<T *>(p);
  }
  ~mfs_stmg() {
    if (s) (void)hipStreamSynchronize(s);
    for (void *p : allocs) (void)hipFree(p);
    for (mfs_problem *p : sp) mfs_destroy(p);
  }
};

namespace {

const LevelGeom &geom(const mfs_stmg &M, int l) { return M.sp[M.lev[l].sp]->L[0].g; }

template <typename T>
void level_apply(mfs_stmg &M, int l, T *dst, const T *src, hipStream_t s) {
  StLevel &L = M.lev[l];
  st_apply<T>(*M.sp[L.sp], L.Q, L.G.data(), M.tau, dst, src, buf<T>(L).work, s);
}

// additive Schwarz steps x <- x + omega B (b - K x).  zero_start: x holds b
// on the Dirichlet rows and 0 elsewhere, where K x = x exactly (identity rows,
// Dirichlet source values ignored in the others), so the first step copies.
template <typename T>
void relax(mfs_stmg &M, int l, bool zero_start, hipStream_t s) {
  StLevel &L = M.lev[l];
  StBuf<T> &B = buf<T>(L);
  const LevelGeom &g = geom(M, l);
  for (int it = 0; it < M.steps; ++it) {
    if (zero_start && it == 0)
      vec_copy<T>(B.t, B.x, (int64_t)L.Q * L.N, s);
    else
      level_apply<T>(M, l, B.t, B.x, s);
    for (int c = 0; c < asm_colours(g); ++c)
      launch_th_apply<T>(g, L.Q, L.N, B.Kinv, c, B.b, B.t, B.x, (T)M.omega, s);
  }
}

// one V-cycle on level l from buf<T>.b into buf<T>.x
template <typename T>
void vcycle(mfs_stmg &M, int l, hipStream_t s) {
  StLevel &L = M.lev[l];
  StBuf<T> &B = buf<T>(L);
  const int64_t n = (int64_t)L.Q * L.N;
  if (l == (int)M.lev.size() - 1) {
    dense_apply<T>(M.coarse_inv, M.coarse_n, B.b, B.x, s);
    return;
  }
  const LevelGeom &g = geom(M, l);
  vec_fill<T>(B.x, T(0), n, s);
  for (int q = 0; q < L.Q; ++q) vec_copy_boundary<T>(g, B.x + q * L.N, B.b + q * L.N, s);
  relax<T>(M, l, true, s);
  level_apply<T>(M, l, B.t, B.x, s);
  vec_copy<T>(B.r, B.b, n, s);
  vec_axpby<T>(B.r, T(-1), B.t, T(1), n, s);  // r = b - K x
  StLevel &C = M.lev[l + 1];
  StBuf<T> &CB = buf<T>(C);
  if (L.kind == 1) {
    stage_mix<T>(CB.b, C.N, C.Q, B.r, L.N, L.Q, L.Rt, T(0), L.N, L.N, s);
  } else {
    const LevelGeom &gc = geom(M, l + 1);
    const LevelGeom &pf = M.pg[L.sp], &pc = M.pg[C.sp];
    for (int q = 0; q < L.Q; ++q) {
      const T *rf = B.r + q * L.N;
      T *bc = CB.b + q * C.N;
      launch_restrict<T>(g, gc, L.h, L.emb_v.data(), bc, rf, s, 0, B.rw_v);
      launch_restrict<T>(pf, pc, L.h, L.emb_p.data(), bc + g.dim * gc.Nv, rf + g.dim * g.Nv, s, 1, B.rw_p, 0);
    }
  }
  vcycle<T>(M, l + 1, s);
  if (L.kind == 1) {
    stage_mix<T>(B.x, L.N, L.Q, CB.x, C.N, C.Q, L.Pt, T(1), L.N, L.N, s);
  } else {
    const LevelGeom &gc = geom(M, l + 1);
    const LevelGeom &pf = M.pg[L.sp], &pc = M.pg[C.sp];
    for (int q = 0; q < L.Q; ++q) {
      T *xf = B.x + q * L.N;
      const T *xc = CB.x + q * C.N;
      launch_prolongate_add<T>(g, gc, L.h, L.emb_v.data(), xf, xc, s);
      launch_prolongate_add<T>(pf, pc, L.h, L.emb_p.data(), xf + g.dim * g.Nv, xc + g.dim * gc.Nv, s, 1, 0);
    }
  }
  relax<T>(M, l, false, s);
}

// spatial patch matrices of level l by probing, then the space-time inverses
void setup_patches(mfs_stmg &M, int l) {
  StLevel &L = M.lev[l];
  mfs_problem &P = *M.sp[L.sp];
  const LevelGeom &g = P.L[0].g;
  hipStream_t s = M.s;
  const int nps = th_patch_size(g);
  const int64_t np = asm_patch_count(g);
  const int64_t nv = (int64_t)g.dim * g.Nv;
  std::vector<void *> tmp;  // probing scratch, freed at the end
  auto talloc = [&](int64_t n) {
    void *q = nullptr;
    MFS_HIP(hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
    tmp.push_back(q);
    return static_cast<double *>(q);
  };
  struct Free {
    std::vector<void *> &v;
    ~Free() {
      for (void *q : v) (void)hipFree(q);
    }
  } free_tmp{tmp};
  double *As = talloc(np * nps * nps), *Ms = talloc(np * nps * nps);
  double *e = talloc(L.N), *ya = talloc(L.N), *ym = talloc(nv);
  for (int c = 0; c < asm_colours(g); ++c)
    for (int j = 0; j < nps; ++j) {
      vec_fill<double>(e, 0.0, L.N, s);
      launch_th_probe_set(g, e, c, j, s);
      apply_op<double>(P, MFS_OP_STOKES, 0, ya, e, s);
      apply_op<double>(P, MFS_OP_MASS_U, 0, ym, e, s);
      launch_th_probe_extract(g, ya, 0, As, c, j, s);
      launch_th_probe_extract(g, ym, nv, Ms, c, j, s);
    }
  StageCoef G{};
  for (int i = 0; i < L.Q; ++i)
    for (int j = 0; j < L.Q; ++j) G.c[i * MFS_MAX_STAGES + j] = L.G[(size_t)i * L.Q + j];
  const int NP = L.Q * nps;
  L.d.Kinv = M.alloc<double>(np * NP * NP);
  L.f.Kinv = M.alloc<float>(np * NP * NP);
  int *status = M.alloc<int>(1);
  MFS_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
  launch_th_form_invert(g, L.Q, G, M.tau, As, Ms, L.d.Kinv, status, s);
  vec_cast<float, double>(L.f.Kinv, L.d.Kinv, np * NP * NP, s);
  int hst = 0;
  MFS_HIP(hipMemcpyAsync(&hst, status, sizeof(int), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  MFS_REQUIRE(hst == 0, MFS_EINVAL, "singular space-time patch matrix on level %d", l);
}

// dense inverse of the coarsest operator with the first pressure node of
// every stage pinned to zero (its row and column of the inverse zeroed but
// for the diagonal, so that x there is 0 whatever b holds)
void setup_coarse(mfs_stmg &M) {
  const int l = (int)M.lev.size() - 1;
  StLevel &L = M.lev[l];
  const LevelGeom &g = geom(M, l);
  const int64_t n64 = (int64_t)L.Q * L.N;
  MFS_REQUIRE(n64 <= 4096, MFS_EUNSUPPORTED, "coarsest space-time level too large for a dense solve (%lld)",
              (long long)n64);
  const int n = (int)n64;
  double *e = M.alloc<double>(n), *y = M.alloc<double>((int64_t)n * n);
  for (int j = 0; j < n; ++j) {
    vec_fill<double>(e, 0.0, n, M.s);
    const double one = 1.0;
    MFS_HIP(hipMemcpyAsync(e + j, &one, sizeof(double), hipMemcpyHostToDevice, M.s));
    level_apply<double>(M, l, y + (int64_t)j * n, e, M.s);  // column j
    MFS_HIP(hipStreamSynchronize(M.s));
  }
  std::vector<double> colmaj((size_t)n * n), A((size_t)n * n);
  MFS_HIP(hipMemcpy(colmaj.data(), y, colmaj.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = colmaj[(size_t)j * n + i];
  std::vector<int> pinned;
  for (int q = 0; q < L.Q; ++q) pinned.push_back((int)(q * L.N + g.dim * g.Nv));
  for (int i : pinned) {
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = 0.0;
    A[(size_t)i * n + i] = 1.0;
  }
  MFS_REQUIRE(invert_dense(A, n), MFS_EINVAL, "singular coarsest space-time operator");
  for (int i : pinned) A[(size_t)i * n + i] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) colmaj[(size_t)j * n + i] = A[(size_t)i * n + j];
  M.coarse_inv = M.alloc<double>((int64_t)n * n);
  M.coarse_n = n;
  MFS_HIP(hipMemcpy(M.coarse_inv, colmaj.data(), colmaj.size() * sizeof(double), hipMemcpyHostToDevice));
}

void check_stmg(const mfs_stmg *m) { MFS_REQUIRE(m != nullptr, MFS_EINVAL, "null space-time multigrid"); }

int64_t top_len(const mfs_stmg &M) { return (int64_t)M.lev[0].Q * M.lev[0].N; }

}  // namespace

extern "C" {

int mfs_stmg_setup(const mfs_mesh *mesh, int k, int kt, double nu, double tau, int relax_steps, double relax_omega,
                   void *stream, mfs_stmg **out) {
  return guard([&] {
    MFS_REQUIRE(mesh && out && mesh->vertices, MFS_EINVAL, "bad arguments");
    *out = nullptr;
    const int dim = mesh->dim;
    MFS_REQUIRE(dim == 2 || dim == 3, MFS_EINVAL, "dim must be 2 or 3");
    if (dim == 2) {
      MFS_REQUIRE(k == 2 || k == 3, MFS_EUNSUPPORTED, "velocity degree %d: 2 or 3 supported in 2D", k);
    } else {
      MFS_REQUIRE(k == 2, MFS_EUNSUPPORTED, "3D: velocity degree 2 supported (patches of 82 unknowns per stage)");
    }
    MFS_REQUIRE(kt >= 0 && kt <= 2, MFS_EUNSUPPORTED, "temporal degree %d: DG(0) to DG(2) supported", kt);
    MFS_REQUIRE(nu > 0 && std::isfinite(nu) && tau > 0 && std::isfinite(tau), MFS_EINVAL,
                "nu and tau must be positive");
    MFS_REQUIRE(relax_steps >= 0 && relax_steps <= 16 && std::isfinite(relax_omega), MFS_EINVAL,
                "bad relaxation parameters");
    for (int a = 0; a < dim; ++a) MFS_REQUIRE(mesh->n[a] >= 1, MFS_EINVAL, "bad mesh size");
    std::unique_ptr<mfs_stmg> M(new mfs_stmg());
    M->dim = dim;
    M->tau = tau;
    M->omega = relax_omega;
    M->steps = relax_steps;
    M->s = S(stream);
    // level specifications
    struct Spec {
      int n[3], k, kt, hl;
    };
    int nn[3] = {mesh->n[0], mesh->n[1], dim == 3 ? mesh->n[2] : 1};
    std::vector<Spec> specs{{{nn[0], nn[1], nn[2]}, k, kt, 0}};
    int kk = k, tt = kt, hl = 0;
    while (kk > 2) specs.push_back({{nn[0], nn[1], nn[2]}, --kk, tt, hl});
    while (true) {
      bool ok = true;
      for (int a = 0; a < dim; ++a) ok = ok && nn[a] % 2 == 0 && nn[a] > 2;
      if (!ok) break;
      for (int a = 0; a < dim; ++a) nn[a] /= 2;
      ++hl;
      specs.push_back({{nn[0], nn[1], nn[2]}, kk, tt, hl});
    }
    while (tt > 0) specs.push_back({{nn[0], nn[1], nn[2]}, kk, --tt, hl});
    // spatial problems: one per distinct (mesh, degree)
    mfs_options o;
    mfs_default_options(&o);
    o.mg_levels = 0;
    o.pressure_offset = 1;
    const int fx = mesh->n[0] + 1, fy = mesh->n[1] + 1;
    int last_k = -1, last_h = -1;
    for (const Spec &sp : specs) {
      StLevel L;
      if (sp.k != last_k || sp.hl != last_h) {
        const int f = 1 << sp.hl;  // keep the fine vertices of index divisible by 2^hl
        const int cx = sp.n[0] + 1, cy = sp.n[1] + 1, cz = dim == 3 ? sp.n[2] + 1 : 1;
        std::vector<double> Xc((size_t)cx * cy * cz * dim);
        for (int l = 0; l < cz; ++l)
          for (int j = 0; j < cy; ++j)
            for (int i = 0; i < cx; ++i)
              for (int a = 0; a < dim; ++a)
                Xc[(((size_t)l * cy + j) * cx + i) * dim + a] =
                    mesh->vertices[(((size_t)l * f * fy + (size_t)j * f) * fx + (size_t)i * f) * dim + a];
        mfs_mesh mc{};
        mc.dim = dim;
        mc.n[0] = sp.n[0];
        mc.n[1] = sp.n[1];
        mc.n[2] = sp.n[2];
        mc.vertices = Xc.data();
        mfs_problem *p = nullptr;
        const int rc = mfs_setup(&mc, sp.k, nu, &o, stream, &p);
        if (rc != MFS_OK) throw mfs::Error{rc};  // mfs_setup set the message
        M->sp.push_back(p);
        M->pg.push_back(pressure_grid(p->L[0].g));
        last_k = sp.k;
        last_h = sp.hl;
      }
      L.sp = (int)M->sp.size() - 1;
      L.kt = sp.kt;
      L.Q = sp.kt + 1;
      const LevelGeom &g = M->sp[L.sp]->L[0].g;
      L.N = (int64_t)g.dim * g.Nv + g.Np;
      std::vector<double> Mq;
      dg_time(sp.kt, L.G, Mq);
      M->lev.push_back(std::move(L));
    }
    const int nl = (int)M->lev.size();
    for (int l = 0; l < nl; ++l) {
      StLevel &L = M->lev[l];
      const int64_t n = (int64_t)L.Q * L.N, nw = (int64_t)L.Q * dim * M->sp[L.sp]->L[0].g.Nv;
      L.d.x = M->alloc<double>(n);
      L.d.b = M->alloc<double>(n);
      L.d.r = M->alloc<double>(n);
      L.d.t = M->alloc<double>(n);
      L.d.work = M->alloc<double>(nw);
      L.f.x = M->alloc<float>(n);
      L.f.b = M->alloc<float>(n);
      L.f.r = M->alloc<float>(n);
      L.f.t = M->alloc<float>(n);
      L.f.work = M->alloc<float>(nw);
      if (l + 1 < nl) {
        const StLevel &C = M->lev[l + 1];
        const LevelGeom &gf = M->sp[L.sp]->L[0].g, &gc = M->sp[C.sp]->L[0].g;
        if (C.Q != L.Q) {
          L.kind = 1;
          time_transfers(L.kt, C.kt, L.Pt, L.Rt);
        } else {
          L.kind = 2;
          L.h = gc.n[0] != gf.n[0];
          L.emb_v = L.h ? h_embedding(gc.k) : p_embedding(gf.k, gc.k);
          L.emb_p = L.h ? h_embedding(gc.kp) : p_embedding(gf.kp, gc.kp);
          const int64_t wv = restrict_work_elems(gf, gc, dim), wp = restrict_work_elems(M->pg[L.sp], M->pg[C.sp], 1);
          L.d.rw_v = M->alloc<double>(wv);
          L.d.rw_p = M->alloc<double>(wp);
          L.f.rw_v = M->alloc<float>(wv);
          L.f.rw_p = M->alloc<float>(wp);
        }
      }
    }
    for (int l = 0; l + 1 < nl; ++l) setup_patches(*M, l);
    setup_coarse(*M);
    // FGMRES space
    const int64_t n0len = top_len(*M);
    M->ld = kr_ld(n0len);
    M->V = M->alloc<double>((int64_t)(M->m + 1) * M->ld);
    M->Z = M->alloc<double>((int64_t)M->m * M->ld);
    M->w = M->alloc<double>(n0len);
    M->dev = M->alloc<double>(128);
    M->ydev = M->alloc<double>(M->m);
    M->partials = M->alloc<double>(32 * DOT_BLOCKS);
    MFS_HIP(hipStreamSynchronize(M->s));
    *out = M.release();
  });
}

int mfs_stmg_destroy(mfs_stmg *m) {
  delete m;
  return MFS_OK;
}

int mfs_stmg_levels(const mfs_stmg *m, int level, int *n_levels, int *n, int *k, int *Q, int64_t *length) {
  return guard([&] {
    check_stmg(m);
    if (n_levels) *n_levels = (int)m->lev.size();
    MFS_REQUIRE(level >= 0 && level < (int)m->lev.size(), MFS_EINVAL, "level %d outside [0, %d)", level,
                (int)m->lev.size());
    const StLevel &L = m->lev[level];
    const LevelGeom &g = m->sp[L.sp]->L[0].g;
    if (n)
      for (int a = 0; a < g.dim; ++a) n[a] = g.n[a];
    if (k) *k = g.k;
    if (Q) *Q = L.Q;
    if (length) *length = (int64_t)L.Q * L.N;
  });
}

int mfs_stmg_vmult(mfs_stmg *m, int level, double *dst, const double *src, void *stream) {
  return guard([&] {
    check_stmg(m);
    MFS_REQUIRE(level >= 0 && level < (int)m->lev.size(), MFS_EINVAL, "level %d outside [0, %d)", level,
                (int)m->lev.size());
    MFS_REQUIRE(dst && src && dst != src, MFS_EINVAL, "bad arguments");
    level_apply<double>(*m, level, dst, src, S(stream));
  });
}

int mfs_stmg_vcycle(mfs_stmg *m, int prec, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_stmg(m);
    MFS_REQUIRE(prec == MFS_FP64 || prec == MFS_FP32, MFS_EINVAL, "bad precision %d", prec);
    MFS_REQUIRE(dst && src, MFS_EINVAL, "bad arguments");
    hipStream_t s = S(stream);
    StLevel &L = m->lev[0];
    const int64_t n = top_len(*m);
    if (prec == MFS_FP64) {
      vec_copy<double>(L.d.b, (const double *)src, n, s);
      vcycle<double>(*m, 0, s);
      vec_copy<double>((double *)dst, L.d.x, n, s);
    } else {
      vec_copy<float>(L.f.b, (const float *)src, n, s);
      vcycle<float>(*m, 0, s);
      vec_copy<float>((float *)dst, L.f.x, n, s);
    }
  });
}

int mfs_stmg_solve(mfs_stmg *m, const double *b, double *x, double rtol, int maxit, int prec, mfs_solve_info *info) {
  return guard([&] {
    check_stmg(m);
    MFS_REQUIRE(prec == MFS_FP64 || prec == MFS_FP32, MFS_EINVAL, "bad precision %d", prec);
    MFS_REQUIRE(b && x && info, MFS_EINVAL, "bad arguments");
    MFS_REQUIRE(rtol > 0 && maxit >= 1, MFS_EINVAL, "bad tolerance or iteration limit");
    const auto t0 = std::chrono::steady_clock::now();
    mfs_stmg &M = *m;
    hipStream_t s = M.s;
    const int64_t n = top_len(M);
    const int mm = M.m;
    double hst[72];
    auto dot = [&](const double *u, const double *v) {
      multi_dot<double>(u, 0, 1, v, n, M.dev + 100, M.partials, s);
      double r = 0;
      MFS_HIP(hipMemcpyAsync(&r, M.dev + 100, sizeof(double), hipMemcpyDeviceToHost, s));
      MFS_HIP(hipStreamSynchronize(s));
      return r;
    };
    vec_fill<double>(x, 0.0, n, s);
    double bnorm = std::sqrt(dot(b, b));
    if (!(bnorm > 0)) bnorm = 1.0;
    int its = 0;
    // r = b - K x
    double *r0 = M.V;
    level_apply<double>(M, 0, M.w, x, s);
    vec_copy<double>(r0, b, n, s);
    vec_axpby<double>(r0, -1.0, M.w, 1.0, n, s);
    double beta = std::sqrt(dot(r0, r0));
    std::vector<double> H((size_t)(mm + 1) * mm), cs(mm), sn(mm), gv(mm + 1);
    while (beta / bnorm > rtol && its < maxit) {
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(gv.begin(), gv.end(), 0.0);
      gv[0] = beta;
      vec_axpby<double>(M.V, 0.0, M.V, 1.0 / beta, n, s);  // V_0 = r / beta
      int j = 0;
      double hn = 1.0;
      while (j < mm) {
        double *vj = M.V + (int64_t)j * M.ld, *zj = M.Z + (int64_t)j * M.ld;
        if (prec == MFS_FP64) {
          vec_copy<double>(M.lev[0].d.b, vj, n, s);
          vcycle<double>(M, 0, s);
          vec_copy<double>(zj, M.lev[0].d.x, n, s);
        } else {
          vec_cast<float, double>(M.lev[0].f.b, vj, n, s);
          vcycle<float>(M, 0, s);
          vec_cast<double, float>(zj, M.lev[0].f.x, n, s);
        }
        level_apply<double>(M, 0, M.w, zj, s);
        // classical Gram-Schmidt, twice
        multi_dot<double>(M.V, M.ld, j + 1, M.w, n, M.dev, M.partials, s);
        multi_axpy<double>(M.w, M.V, M.ld, j + 1, M.dev, n, s);
        multi_dot<double>(M.V, M.ld, j + 1, M.w, n, M.dev + 32, M.partials, s);
        multi_axpy<double>(M.w, M.V, M.ld, j + 1, M.dev + 32, n, s);
        multi_dot<double>(M.w, 0, 1, M.w, n, M.dev + 64, M.partials, s);
        MFS_HIP(hipMemcpyAsync(hst, M.dev, 65 * sizeof(double), hipMemcpyDeviceToHost, s));
        MFS_HIP(hipStreamSynchronize(s));
        hn = std::sqrt(std::max(hst[64], 0.0));
        double *vn = M.V + (int64_t)(j + 1) * M.ld;
        if (hn > 0)
          vec_axpby<double>(vn, 1.0 / hn, M.w, 0.0, n, s);
        else
          vec_fill<double>(vn, 0.0, n, s);
        std::vector<double> col(j + 2);
        for (int i = 0; i <= j; ++i) col[i] = hst[i] + hst[32 + i];
        col[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
          const double tt = cs[i] * col[i] + sn[i] * col[i + 1];
          col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
          col[i] = tt;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        cs[j] = den > 0 ? col[j] / den : 1.0;
        sn[j] = den > 0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        for (int i = 0; i <= j; ++i) H[(size_t)i * mm + j] = col[i];
        ++j;
        ++its;
        if (std::fabs(gv[j]) / bnorm <= rtol || its >= maxit || hn == 0) break;
      }
      std::vector<double> y(j);
      for (int i = j - 1; i >= 0; --i) {
        double v = gv[i];
        for (int c = i + 1; c < j; ++c) v -= H[(size_t)i * mm + c] * y[c];
        y[i] = v / H[(size_t)i * mm + i];
      }
      MFS_HIP(hipMemcpyAsync(M.ydev, y.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
      multi_combine<double>(x, M.Z, M.ld, j, M.ydev, n, true, s);
      MFS_HIP(hipStreamSynchronize(s));
      level_apply<double>(M, 0, M.w, x, s);
      vec_copy<double>(r0, b, n, s);
      vec_axpby<double>(r0, -1.0, M.w, 1.0, n, s);
      beta = std::sqrt(dot(r0, r0));
    }
    info->iterations = its;
    info->rel_residual = beta / bnorm;
    info->status = beta / bnorm <= rtol ? MFS_OK : MFS_ENOCONV;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info->status != MFS_OK) {
      set_error("space-time FGMRES did not reach rtol %.3e within %d iterations (relative residual %.3e)", rtol,
                maxit, beta / bnorm);
      throw mfs::Error{MFS_ENOCONV};
    }
  });
}

}  // extern "C"
