// Host runtime and C ABI of the mfstokes library: problem setup (levels,
// geometry, tables, diagonals, Chebyshev bounds, coarse inverse), operator
// application, the multigrid V-cycle, the block preconditioner and FGMRES as
// a resumable state machine.
//
// Methods: Sec. 3 eq. (stokes_block) (block-triangular preconditioner with
// S ~ nu^{-1} M_p inverted by Jacobi-PCG, A^{-1} ~ one V-cycle, FGMRES), Sec. 2
// eq. (transfer) and Sec. 3 (p-levels down to p_min, then global-coarsening
// h-levels, Chebyshev around point Jacobi, direct coarse solve); Sec. 5
// (equal-order SUPG/PSPG Navier-Stokes Jacobian, monolithic multigrid with
// h-levels first, damped point-Jacobi relaxation and a direct coarse solve,
// inside FGMRES).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "amr.h"
#include "amr_kernels.h"
#include "hp.h"
#include "internal.h"

using namespace mfs;

namespace {

// ------------------------------------------------------------- arena plan
struct Arena {
  size_t off = 0;
  char *base = nullptr;
  bool dry = true;
  template <typename T>
  T *take(int64_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
    off += (size_t)std::max<int64_t>(n, 0) * sizeof(T);
    return p;
  }
};

template <typename T>
struct PrecWork {
  // multigrid level vectors: x, b, r, d (velocity, dim*Nv each)
  std::vector<T *> x, b, r, d;
  T *invdiag_first = nullptr;
  // block preconditioner / Schur PCG
  T *t_u = nullptr;                                    // velocity temporary
  T *pres = nullptr, *ps = nullptr, *pp = nullptr, *pq = nullptr, *pz = nullptr;  // PCG vectors (Np)
  T *pinv = nullptr;                                   // 1/diag(M_p)
  T *full_in = nullptr, *full_out = nullptr;           // cast buffers for the mixed preconditioner
};

struct Level {
  LevelGeom g{};
  double *X64 = nullptr;
  float *X32 = nullptr;
  double *tab64 = nullptr;
  float *tab32 = nullptr;
  double *diag = nullptr;
  double *face64 = nullptr;  // scratch of the specialised degree-2 kernel
  float *face32 = nullptr;
  double *ev64 = nullptr;  // cell-local outputs of the generic kernel (3D, degree >= 3)
  float *ev32 = nullptr;
  double *invdiag64 = nullptr;
  float *invdiag32 = nullptr;
  double lambda = 0.0;          // upper end of the Chebyshev interval
  bool h_to_coarser = false;    // transfer type to level+1
  std::vector<double> emb;      // 1D embedding to level+1
  std::vector<double> Xhost;    // vertices (host copy)
  std::vector<double> tabh;     // 1D tables (host copy)
  // Navier-Stokes (equal order): linearisation point, per-point data, 1/diag(J)
  double *u0 = nullptr;
  double *qd64 = nullptr;
  float *qd32 = nullptr;
  double *nsinv64 = nullptr;
  float *nsinv32 = nullptr;
  // additive Schwarz relaxation: inverse patch matrices (vertex patches)
  double *asm64 = nullptr;
  float *asm32 = nullptr;
  // scratch of the three-pass restriction to the next coarser level
  double *rs64 = nullptr;
  float *rs32 = nullptr;
};

// Stride of the Krylov basis vectors: the length rounded up to an odd number
// of 256-byte units, so that the up to 31 vectors that the Gram-Schmidt
// kernels stream side by side start at staggered offsets modulo the HBM
// channel interleave (a stride that is a multiple of 4 KB sent all streams
// to the same channels at once).
int64_t kr_ld(int64_t n) {
  int64_t l = (n + 31) / 32 * 32;
  if ((l / 32) % 2 == 0) l += 32;
  return l;
}

struct Krylov {
  int m = 30;
  int64_t ld = 0;  // basis stride (kr_ld of the system length)
  double *V = nullptr, *Z = nullptr, *w = nullptr;
  double *dev = nullptr;     // device scalars: h[32], h2[32], nrm2, misc
  double *host = nullptr;    // pinned readback
  double *ydev = nullptr;    // device copy of the GMRES coefficients
  double *yhost = nullptr;   // pinned
  hipEvent_t ev = nullptr;
  hipEvent_t ev_pre = nullptr;  // end of the preconditioner (grouped steps)
  // state
  int state = 0;  // 0 idle, 1 wait initial residual, 2 wait Arnoldi step, 3 wait final check, 4 done
  int j = 0, iters = 0, maxit = 0, prec = MFS_FP32;
  bool graphs = true;
  double rtol = 1e-8, bnorm = 0, beta = 0;
  std::vector<double> H, cs, sn, gv;
  const double *b = nullptr;
  double *x = nullptr;
  hipStream_t s = nullptr;
  std::chrono::steady_clock::time_point t0;
  mfs_solve_info info{};
  bool final_pending = false;
};

// ------------------------------------------------------------- hp levels
// Device copy of an hp space's maps (velocity: the gather drops Dirichlet
// columns, the transposed map has no Dirichlet rows, owners of Dirichlet
// unknowns are -1; pressure: no Dirichlet unknowns).
struct HpDevSpace {
  int64_t N = 0, nrows = 0;
  HpMaps m;  // rows and transposed lists (plain / weighted)
  uint8_t *dir = nullptr;
  int64_t *owner_ev = nullptr;
  int *owner_nb = nullptr;
  int *colour = nullptr;
  int ncolours = 0;
};

template <typename T>
struct HpVecs {
  T *x = nullptr, *b = nullptr, *r = nullptr, *d = nullptr;  // 3N
  T *ev_in = nullptr, *ev_out = nullptr;                       // velocity E-vectors
  T *invdiag = nullptr;                                        // N
};

struct HpLevel {
  HpSpaceHost V;
  HpDevSpace vd;
  int64_t ev_size = 0;
  int64_t *off_u = nullptr;  // per cell: E-vector offset of the cell's [(k+1)^3][3] block
  int *deg = nullptr;        // per cell degree (device)
  std::vector<int> class_k, class_n;
  std::vector<int *> class_cells;
  double lambda = 0.0;
  double *diag = nullptr;
  HpVecs<double> v64;
  HpVecs<float> v32;
};

struct HpData {
  int n[3] = {0, 0, 0};
  int64_t ncells = 0;
  std::vector<HpLevel> lev;
  // pressure space of the finest level
  HpSpaceHost Pr;
  HpDevSpace pd;
  int64_t evp_size = 0;
  int64_t *off_p = nullptr;
  double *evp_in64 = nullptr, *evp_out64 = nullptr;
  float *evp_in32 = nullptr, *evp_out32 = nullptr;
  // coarse side of the last hp transfer: the uniform degree-2 hp space and
  // the index of each of its unknowns in the structured degree-2 node grid
  HpSpaceHost V2;
  HpDevSpace v2d;
  int64_t ev2_size = 0;
  int64_t *off_u2 = nullptr;
  int *deg2 = nullptr;
  int64_t *perm2 = nullptr;
  double *ev2_64 = nullptr, *tmp2_64 = nullptr;
  float *ev2_32 = nullptr, *tmp2_32 = nullptr;
  double *embed = nullptr;  // [8][8][MAXQ*MAXQ] 1D embeddings [fine][coarse]
  double *tab64[7] = {};
  float *tab32[7] = {};
  // block preconditioner
  double *pdiag = nullptr, *m1 = nullptr, *ones = nullptr;
  double *pinv64 = nullptr;
  float *pinv32 = nullptr;
  double *p64[5] = {};  // pres, ps, pp, pq, pz
  float *p32[5] = {};
  double *tu64 = nullptr;
  float *tu32 = nullptr;
  std::vector<void *> allocs;
  template <typename T>
  T *alloc(int64_t n) {
    void *p = nullptr;
    MFS_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(T)));
    allocs.push_back(p);
    return static_cast<T *>(p);
  }
  template <typename T>
  T *upload(const std::vector<T> &v, hipStream_t s) {
    T *p = alloc<T>((int64_t)v.size());
    if (!v.empty()) MFS_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  ~HpData() {
    for (void *p : allocs) (void)hipFree(p);
  }
};

// ------------------------------------------------------------- refined meshes
// Equal-order Navier-Stokes on a locally refined mesh.  Level j of the
// global coarsening sequence: the unknowns' maps to the cell-local values
// (E-vectors [cell][(k+1)^3][4]: velocity components and pressure of a node
// side by side), the
// per-cell corners, the linearisation data, the Jacobi diagonal, V-cycle
// work vectors, and the cell and unknown relations to level j + 1.
// host form of AmrMaps (built on a worker thread, then uploaded)
struct AmrMapsHost {
  int64_t N = 0, nrows = 0;
  std::vector<int> rcol, hcol, trow, wrow, owner;
  std::vector<int64_t> hptr, tptr, wptr, heavy;
  std::vector<double> hval, wval;
};

struct AmrLevel {
  AmrSpaceHost S;  // host space (row maps released after the upload)
  AmrMapsHost mh;              // host maps and colouring, released after the upload
  std::vector<int> colour_host;
  int ncolour_host = 0;
  LevelGeom g{};   // degree and cell count for the cell kernels
  int64_t N = 0, NQ = 0;
  AmrMaps M;       // unknowns <-> E-vector rows (constraints, Dirichlet mask, owners)
  double *X64 = nullptr;
  float *X32 = nullptr;
  double *qd64 = nullptr;
  float *qd32 = nullptr;
  double *ev64[2] = {};  // in, out
  float *ev32[2] = {};
  double *u0 = nullptr;                        // 7 N: state [u0 | p0 | u~]
  double *diag = nullptr;                      // 4 N, diag(J)
  double *inv64 = nullptr;                     // 4 N, 1 / diag(J)
  float *inv32 = nullptr;
  double *w64[4] = {};                         // x, b, r, d (4 N each)
  float *w32[4] = {};
  int *colour = nullptr;
  int ncolours = 0;
  // relation to level j + 1 (the next coarser)
  int *parent = nullptr;
  uint8_t *octant = nullptr;
  int64_t *cptr = nullptr;  // CSR of the fine cells per coarse cell
  int *child = nullptr;
  int64_t *inject = nullptr;  // coarse unknown -> fine unknown
};

struct AmrData {
  HpData H;  // device allocations and uploads
  int n = 0, k = 0, L = 0;
  bool mg = false;  // GC levels + structured hierarchy of the base mesh
  std::vector<AmrLevel> lev;  // finest first; with mg the last is the uniform base mesh
  double *tab64 = nullptr;
  float *tab32 = nullptr;
  AmrEmbed E{};
  double *ones = nullptr, *scratch = nullptr;  // N0 each (pressure mean)
  double *state = nullptr;                      // 4 N0: staging of a linearisation state
  double dt = 0.0;
  int newton = 1;
  bool ready = false;
  bool mg_ready = false;  // multigrid data of the current linearisation
};
}  // namespace

struct mfs_problem {
  int dim = 3;
  double nu = 1.0;
  mfs_options opts{};
  std::vector<Level> L;
  int nlev = 0;
  double *coarse_inv = nullptr;
  int coarse_n = 0;
  PrecWork<double> w64;
  PrecWork<float> w32;
  double *m1 = nullptr;         // M_p 1 (pressure mean)
  int *flags = nullptr;         // device status words (Navier-Stokes set-up)
  double *scal = nullptr;       // device scalars for PCG / means
  double *partials = nullptr;   // reduction scratch
  double *tmp_full = nullptr;   // FP64 full-length temporary
  double *tmp2 = nullptr;       // second one (Navier-Stokes set-up)
  double *nw_uh = nullptr, *nw_F = nullptr, *nw_dx = nullptr;  // BDF2 / Newton driver (level-0 sizes)
  Krylov kr;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  bool arena_owned = true;  // false: the caller's arena (mfs_setup_arena)
  hipStream_t stream = nullptr;
  // Navier-Stokes problem (pressure_offset = 0)
  bool ns = false;
  bool ns_ready = false;
  bool ns_mg_ready = false;  // multigrid data of the current linearisation
  double ns_dt = 0.0;
  int ns_newton = 1;
  // hp problem: hp levels first (global level numbers 0 .. nhp-1), then the
  // structured degree-2 levels in L
  HpData *hp = nullptr;
  int nhp = 0;
  // refined-mesh problem: its levels come first (global numbers 0 .. namr-1)
  AmrData *amr = nullptr;
  int namr = 0;
  // recorded FP32 preconditioner (between w32.full_in and w32.full_out), its
  // capture stream, and whether recording failed once (then launched eagerly)
  hipGraphExec_t prec_graph[2] = {nullptr, nullptr};  // FP32, FP64
  hipStream_t cap_stream = nullptr;
  bool graph_failed = false;
};

namespace {

constexpr int PCG_MAX = 64;  // scalar slots per PCG run (rho[i], pq[i])

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

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

template <typename T>
DevLevel<T> dev(const Level &L);
template <>
DevLevel<double> dev<double>(const Level &L) {
  DevLevel<double> d;
  d.X = L.X64;
  d.tab = L.tab64;
  d.invdiag = L.invdiag64;
  return d;
}
template <>
DevLevel<float> dev<float>(const Level &L) {
  DevLevel<float> d;
  d.X = L.X32;
  d.tab = L.tab32;
  d.invdiag = L.invdiag32;
  return d;
}
template <typename T>
T *face(const Level &L);
template <>
double *face<double>(const Level &L) {
  return L.face64;
}
template <>
float *face<float>(const Level &L) {
  return L.face32;
}
template <typename T>
T *cellev(const Level &L);
template <>
double *cellev<double>(const Level &L) {
  return L.ev64;
}
template <>
float *cellev<float>(const Level &L) {
  return L.ev32;
}
// Generic kernel with cell-local outputs and a node gather instead of global
// atomics, on every 3D level of degree >= 3 (measured at 64^3 against the
// atomics launched one cell colour at a time: Q4/Q3 FP64 1.93 ms against
// 2.21 ms, once the cell-local rows were laid out for the gather).
template <typename T>
bool use_gather(const Level &L) {
  return cell_ev_elems(L.g) > 0;
}
template <typename T>
PrecWork<T> &work(mfs_problem &P);
template <>
PrecWork<double> &work<double>(mfs_problem &P) {
  return P.w64;
}
template <>
PrecWork<float> &work<float>(mfs_problem &P) {
  return P.w32;
}
template <typename T>
T *rwork(const Level &L);
template <>
double *rwork<double>(const Level &L) {
  return L.rs64;
}
template <>
float *rwork<float>(const Level &L) {
  return L.rs32;
}
template <typename T>
const T *invdiag(const Level &L);
template <>
const double *invdiag<double>(const Level &L) {
  return L.invdiag64;
}
template <>
const float *invdiag<float>(const Level &L) {
  return L.invdiag32;
}

// ---------------------------------------------------------------- operators
// velocity-block A on level l: dst = A src (dim*Nv); Dirichlet rows dst = src
bool use_specialised() {
  static const bool off = std::getenv("MFS_GENERIC_KERNELS") != nullptr;
  return !off;
}

template <typename T>
void apply_A(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s) {
  const Level &L = P.L[l];
  if (use_specialised() && q2_face_elems(L.g) > 0 &&
      launch_stokes_q2<T>(L.g, dev<T>(L).X, Q2_A, (T)P.nu, dst, nullptr, src, nullptr, face<T>(L), s))
    return;
  if (use_specialised() && q1_face_elems(L.g) > 0 &&
      launch_laplace_q1<T>(L.g, dev<T>(L).X, (T)P.nu, dst, src, face<T>(L), s))
    return;
  if (use_gather<T>(L)) {
    launch_cell_op_gather<T>(L.g, dev<T>(L), M_LAPLACE, (T)P.nu, dst, nullptr, src, nullptr, src, cellev<T>(L), s);
    return;
  }
  launch_fill_dirichlet<T>(L.g, dst, src, s);
  launch_cell_op<T>(L.g, dev<T>(L), M_LAPLACE, (T)P.nu, dst, nullptr, src, nullptr, s);
}

template <typename T>
const T *ns_qd(const Level &L);
template <>
const double *ns_qd<double>(const Level &L) {
  return L.qd64;
}
template <>
const float *ns_qd<float>(const Level &L) {
  return L.qd32;
}
template <typename T>
const T *ns_invdiag(const Level &L);
template <>
const double *ns_invdiag<double>(const Level &L) {
  return L.nsinv64;
}
template <>
const float *ns_invdiag<float>(const Level &L) {
  return L.nsinv32;
}

// constrained Navier-Stokes Jacobian on level l: identity on the velocity
// Dirichlet rows, cell terms elsewhere (Dirichlet source values ignored)
template <typename T>
void apply_ns(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s) {
  MFS_REQUIRE(P.ns, MFS_EINVAL, "the Navier-Stokes Jacobian needs a problem set up with pressure_offset = 0");
  MFS_REQUIRE(P.ns_ready, MFS_EINVAL, "mfs_set_linearization has not been called");
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  // 3D: cell-local outputs and a deterministic node gather instead of global
  // atomics (at 128^3 Q2Q2 the FP32 atomics cost 45% of the Jacobian; with
  // the cell-local rows laid out for the gather it pays in FP64 too)
  if (g.dim == 3 && cellev<T>(L) != nullptr) {
    T *ev = cellev<T>(L);
    launch_ns<T>(g, dev<T>(L).X, dev<T>(L).tab, 1, (T)P.nu, (T)P.ns_dt, P.ns_newton, src, dst,
                 const_cast<T *>(ns_qd<T>(L)), s, ev);
    const int64_t q = g.k + 1;
    launch_node_gather<T>(g, g.k, g.k, ev, ev + g.ncells * 3 * q * q * q, dst, dst + g.dim * g.Nv, src, s);
    return;
  }
  launch_fill_dirichlet<T>(g, dst, src, s);
  vec_fill<T>(dst + g.dim * g.Nv, T(0), g.Nv, s);
  launch_ns<T>(g, dev<T>(L).X, dev<T>(L).tab, 1, (T)P.nu, (T)P.ns_dt, P.ns_newton, src, dst,
               const_cast<T *>(ns_qd<T>(L)), s);
}

template <typename T>
void apply_op(mfs_problem &P, int op, int l, T *dst, const T *src, hipStream_t s) {
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int64_t nu = g.dim * g.Nv;
  if (op == MFS_OP_NS_JACOBIAN) {
    apply_ns<T>(P, l, dst, src, s);
    return;
  }
  MFS_REQUIRE(!P.ns, MFS_EUNSUPPORTED, "operator %d is not available on an equal-order (Navier-Stokes) problem",
              op);
  switch (op) {
    case MFS_OP_A:
      apply_A<T>(P, l, dst, src, s);
      break;
    case MFS_OP_STOKES:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_specialised() && q2_face_elems(g) > 0 &&
          launch_stokes_q2<T>(g, dev<T>(L).X, Q2_STOKES, (T)P.nu, dst, dst + nu, src, src + nu, face<T>(L), s))
        break;
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_LAPLACE | M_GRADP | M_DIVU, (T)P.nu, dst, dst + nu, src, src + nu,
                                 src, cellev<T>(L), s);
        break;
      }
      launch_fill_dirichlet<T>(g, dst, src, s);
      vec_fill<T>(dst + nu, T(0), g.Np, s);
      launch_cell_op<T>(g, dev<T>(L), M_LAPLACE | M_GRADP | M_DIVU, (T)P.nu, dst, dst + nu, src, src + nu, s);
      break;
    case MFS_OP_B:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_specialised() && q2_face_elems(g) > 0 &&
          launch_stokes_q2<T>(g, dev<T>(L).X, Q2_B, (T)P.nu, dst, nullptr, nullptr, src, face<T>(L), s))
        break;
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_GRADP, (T)P.nu, dst, nullptr, nullptr, src, nullptr, cellev<T>(L), s);
        break;
      }
      launch_fill_dirichlet<T>(g, dst, (const T *)nullptr, s);
      launch_cell_op<T>(g, dev<T>(L), M_GRADP, (T)P.nu, dst, nullptr, nullptr, src, s);
      break;
    case MFS_OP_BT:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_DIVU, (T)P.nu, nullptr, dst, src, nullptr, nullptr, cellev<T>(L), s);
        break;
      }
      vec_fill<T>(dst, T(0), g.Np, s);
      launch_cell_op<T>(g, dev<T>(L), M_DIVU, (T)P.nu, nullptr, dst, src, nullptr, s);
      break;
    case MFS_OP_MASS_U:
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_MASSU, (T)P.nu, dst, nullptr, src, nullptr, src, cellev<T>(L), s);
        break;
      }
      launch_fill_dirichlet<T>(g, dst, src, s);
      launch_cell_op<T>(g, dev<T>(L), M_MASSU, (T)P.nu, dst, nullptr, src, nullptr, s);
      break;
    case MFS_OP_MASS_P:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_specialised() && q2_face_elems(g) > 0 &&
          launch_stokes_q2<T>(g, dev<T>(L).X, Q2_MASSP, (T)P.nu, nullptr, dst, nullptr, src, face<T>(L), s))
        break;
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_MASSP, (T)P.nu, nullptr, dst, nullptr, src, nullptr, cellev<T>(L), s);
        break;
      }
      vec_fill<T>(dst, T(0), g.Np, s);
      launch_cell_op<T>(g, dev<T>(L), M_MASSP, (T)P.nu, nullptr, dst, nullptr, src, s);
      break;
    default:
      MFS_REQUIRE(false, MFS_EUNSUPPORTED, "operator %d not available", op);
  }
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

// ---------------------------------------------------------------- Navier-Stokes set-up
// diag(J) on level l: J applied to the indicator of one node colour and one
// component at a time (colour = node index mod (k+1) per direction, so no two
// nodes of a colour share a cell and each row sees only its own column)
void ns_diagonal(mfs_problem &P, int l, double *diag, hipStream_t s) {
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int q = g.k + 1;
  int ncol = 1;
  for (int a = 0; a < g.dim; ++a) ncol *= q;
  double *e = P.tmp_full, *y = P.tmp2;
  for (int c = 0; c < ncol; ++c)
    for (int comp = 0; comp <= P.dim; ++comp) {
      launch_color_indicator(g, P.dim + 1, q, c, comp, e, s);
      apply_ns<double>(P, l, y, e, s);
      launch_color_extract(g, q, c, comp, y, diag, s);
    }
}

// dense inverse of the coarsest J with pressure node 0 pinned; columns of J
// from colourings with spacing 2k+1 (the stencils of two nodes of a colour
// do not overlap, so every entry of J e_colour belongs to one column)
void ns_setup_coarse(mfs_problem &P, hipStream_t s) {
  const int l = P.nlev - 1;
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int n = P.coarse_n;
  const int64_t Nv = g.Nv;
  const int k = g.k, q = 2 * k + 1;
  int ncol = 1;
  for (int a = 0; a < g.dim; ++a) ncol *= q;
  std::vector<double> A((size_t)n * n, 0.0), y(n);  // row-major
  double *e = P.tmp_full, *yd = P.tmp2;
  auto coord = [&](int64_t i, int c[3]) {
    c[0] = (int)(i % g.nv[0]);
    c[1] = (int)((i / g.nv[0]) % g.nv[1]);
    c[2] = (int)(i / ((int64_t)g.nv[0] * g.nv[1]));
  };
  for (int col = 0; col < ncol; ++col)
    for (int comp = 0; comp <= P.dim; ++comp) {
      launch_color_indicator(g, P.dim + 1, q, col, comp, e, s);
      apply_ns<double>(P, l, yd, e, s);
      MFS_HIP(hipMemcpyAsync(y.data(), yd, n * sizeof(double), hipMemcpyDeviceToHost, s));
      MFS_HIP(hipStreamSynchronize(s));
      for (int64_t j = 0; j < Nv; ++j) {
        int cj[3];
        coord(j, cj);
        if (cj[0] % q + q * (cj[1] % q + q * (cj[2] % q)) != col) continue;
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::max(0, cj[a] - k);
          hi[a] = std::min(g.nv[a] - 1, cj[a] + k);
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
          for (int yy = lo[1]; yy <= hi[1]; ++yy)
            for (int x = lo[0]; x <= hi[0]; ++x) {
              const int64_t i = x + (int64_t)g.nv[0] * (yy + (int64_t)g.nv[1] * z);
              for (int r = 0; r <= P.dim; ++r)
                A[(size_t)(r * Nv + i) * n + comp * Nv + j] = y[r * Nv + i];
            }
      }
    }
  const int pin = (int)(P.dim * Nv);
  for (int i = 0; i < n; ++i) {
    A[(size_t)pin * n + i] = 0.0;
    A[(size_t)i * n + pin] = 0.0;
  }
  A[(size_t)pin * n + pin] = 1.0;
  // LU with partial pivoting (row-major, in place)
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)pr * n + c])) pr = r;
    MFS_REQUIRE(A[(size_t)pr * n + c] != 0.0, MFS_EINVAL, "coarse Navier-Stokes matrix is singular");
    piv[c] = pr;
    if (pr != c)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)pr * n + j]);
    const double inv = 1.0 / A[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      const double f = A[(size_t)r * n + c] * inv;
      A[(size_t)r * n + c] = f;
      if (f != 0.0)
        for (int j = c + 1; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
    }
  }
  // inverse, column-major for dense_apply; the pinned column is dropped
  std::vector<double> inv((size_t)n * n, 0.0), v(n);
  for (int c = 0; c < n; ++c) {
    if (c == pin) continue;
    std::fill(v.begin(), v.end(), 0.0);
    v[c] = 1.0;
    for (int i = 0; i < n; ++i) std::swap(v[i], v[piv[i]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) v[i] -= A[(size_t)i * n + j] * v[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) v[i] -= A[(size_t)i * n + j] * v[j];
      v[i] /= A[(size_t)i * n + i];
    }
    std::copy(v.begin(), v.end(), inv.begin() + (size_t)c * n);
  }
  MFS_HIP(hipMemcpyAsync(P.coarse_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MFS_HIP(hipStreamSynchronize(s));
}

// Additive Schwarz patch inverses of level l at the current linearisation:
// column j of every patch matrix of a colour from one FP64 Jacobian apply to
// the sum of the colour's unit vectors at local index j, then a batched
// inversion; the FP32 copy serves the FP32 multigrid.
void ns_asm_setup(mfs_problem &P, int l, hipStream_t s) {
  Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int64_t n = (P.dim + 1) * g.Nv;
  const int np = asm_patch_size(g);
  double *x = P.w64.b[l], *y = P.w64.r[l];
  vec_fill<double>(x, 0.0, n, s);
  for (int c = 0; c < asm_colours(g); ++c)
    for (int j = 0; j < np; ++j) {
      launch_asm_probe_set(g, x, c, j, 1.0, s);
      apply_ns<double>(P, l, y, x, s);
      launch_asm_probe_extract(g, y, L.asm64, c, j, s);
      launch_asm_probe_set(g, x, c, j, 0.0, s);
    }
  MFS_HIP(hipMemsetAsync(P.flags, 0, sizeof(int), s));
  launch_asm_invert(g, L.asm64, P.flags, s);
  int bad = 0;
  MFS_HIP(hipMemcpyAsync(&bad, P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  MFS_REQUIRE(bad == 0, MFS_EINVAL, "singular additive Schwarz patch matrix on level %d", l);
  vec_cast<float, double>(L.asm32, L.asm64, asm_patch_count(g) * np * np, s);
}

// Jacobi diagonals (or Schwarz patch inverses) and the pinned coarse inverse
// of the current linearisation
void ns_mg_data(mfs_problem &P, hipStream_t s) {
  if (!P.opts.mg_levels) return;
  for (int l = 0; l + 1 < P.nlev; ++l) {
    Level &L = P.L[l];
    const int64_t n = (P.dim + 1) * L.g.Nv;
    double *d = P.w64.x[l];
    ns_diagonal(P, l, d, s);
    launch_reciprocal(L.nsinv64, L.nsinv32, d, n, s);
    if (L.asm64) ns_asm_setup(P, l, s);
  }
  ns_setup_coarse(P, s);
}

// Linearisation at the state x0 = [u0 | p0] ((dim+1) Nv) with the BDF2
// history u~ (dim Nv; NULL: u~ = u0), on every level (the coarse levels take
// the fields at their nodes, which are fine nodes); keep_delta leaves
// delta_1 as the previous linearisation stored it; mg: also the multigrid
// data (diagonals, coarse inverse).  Host-synchronous.
void ns_set_point(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta, bool mg,
                  hipStream_t s) {
  P.ns_ready = false;
  P.ns_mg_ready = false;
  P.ns_dt = dt;
  P.ns_newton = newton ? 1 : 0;
  const int d = P.dim;
  const int64_t Nv = P.L[0].g.Nv;
  double *st = P.L[0].u0;
  MFS_HIP(hipMemcpyAsync(st, x0, (d + 1) * Nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  MFS_HIP(hipMemcpyAsync(st + (d + 1) * Nv, uh ? uh : x0, d * Nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int l = 1; l < P.nlev; ++l) launch_ns_inject(P.L[l - 1].g, P.L[l].g, P.L[l - 1].u0, P.L[l].u0, s, 2 * d + 1);
  NsPoint<double> pt;
  pt.keep_delta = keep_delta;
  for (int l = 0; l < P.nlev; ++l) {
    Level &L = P.L[l];
    launch_ns<double>(L.g, L.X64, L.tab64, 0, P.nu, dt, P.ns_newton, L.u0, nullptr, L.qd64, s, nullptr, nullptr,
                      nullptr, &pt);
    vec_cast<float, double>(L.qd32, L.qd64, ns_qd_elems(L.g), s);
  }
  P.ns_ready = true;
  try {
    if (mg) {
      ns_mg_data(P, s);
      P.ns_mg_ready = true;
    }
    MFS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    P.ns_ready = false;
    throw;
  }
}

// Linearisation point u0 of a Jacobian alone: p0 = 0 and u~ = u0
void ns_set_linearization(mfs_problem &P, const double *u0, double dt, int newton, hipStream_t s) {
  const int64_t nv = P.dim * P.L[0].g.Nv;
  double *x0 = P.tmp2;
  MFS_HIP(hipMemcpyAsync(x0, u0, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  vec_fill<double>(x0 + nv, 0.0, P.L[0].g.Nv, s);
  ns_set_point(P, x0, nullptr, dt, newton, 0, true, s);
}

// F = the nonlinear residual at the level-0 state of the last linearisation;
// Dirichlet velocity rows 0
void ns_residual(mfs_problem &P, double *F, hipStream_t s) {
  MFS_REQUIRE(P.ns_ready, MFS_EINVAL, "no linearisation state: call mfs_set_linearization_point first");
  Level &L = P.L[0];
  const LevelGeom &g = L.g;
  launch_fill_dirichlet<double>(g, F, (const double *)nullptr, s);
  vec_fill<double>(F + g.dim * g.Nv, 0.0, g.Nv, s);
  launch_ns<double>(g, L.X64, L.tab64, 2, P.nu, P.ns_dt, P.ns_newton, nullptr, F, L.qd64, s);
}

// ---------------------------------------------------------------- V-cycle
template <typename T>
void chebyshev(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s) {
  Level &L = P.L[l];
  PrecWork<T> &W = work<T>(P);
  const double lmax = L.lambda, lmin = lmax / P.opts.cheb_range;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho_old = 1.0 / sigma;
  T *Ax = W.r[l], *d = W.d[l];
  // x += d with d from the residual b - A x: fused into the brick kernels
  // where the level has one
  auto step = [&](T c1, T c2, bool first) {
    if (use_specialised() && q2_face_elems(L.g) > 0 &&
        launch_q2_cheb<T>(L.g, dev<T>(L).X, (T)P.nu, x, d, b, invdiag<T>(L), c1, c2, first, face<T>(L), s))
      return;
    if (use_specialised() && q1_face_elems(L.g) > 0 &&
        launch_q1_cheb<T>(L.g, dev<T>(L).X, (T)P.nu, x, d, b, invdiag<T>(L), c1, c2, first, face<T>(L), s))
      return;
    apply_A<T>(P, l, Ax, x, s);
    cheb_update<T>(L.g, x, d, b, Ax, invdiag<T>(L), c1, c2, first, s);
  };
  if (zero_start)  // x on entry is ignored: x = b on the Dirichlet rows, 0 elsewhere, then the first step
    cheb_start<T>(L.g, x, d, b, invdiag<T>(L), (T)(1.0 / theta), s);
  else
    step(T(0), (T)(1.0 / theta), true);
  for (int it = 1; it < P.opts.cheb_degree; ++it) {
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    step((T)(rho * rho_old), (T)(2.0 * rho / delta), false);
    rho_old = rho;
  }
}

template <typename T>
void vcycle_level(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  Level &L = P.L[l];
  if (l == P.nlev - 1) {
    dense_apply<T>(P.coarse_inv, P.coarse_n, b, x, s);
    return;
  }
  const int64_t n = P.dim * L.g.Nv;
  chebyshev<T>(P, l, x, b, true, s);  // from x = b on Dirichlet rows, 0 elsewhere
  T *r = W.r[l];
  apply_A<T>(P, l, r, x, s);
  vec_axpby<T>(r, T(1), b, T(-1), n, s);  // r = b - A x
  Level &C = P.L[l + 1];
  launch_restrict<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), W.b[l + 1], r, s, 0, rwork<T>(L));
  vcycle_level<T>(P, l + 1, W.x[l + 1], W.b[l + 1], s);
  launch_prolongate_add<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), x, W.x[l + 1], s);
  chebyshev<T>(P, l, x, b, false, s);
}

// ---------------------------------------------------------------- Navier-Stokes V-cycle
// One monolithic V-cycle on J (Sec. 5): x = (b on Dirichlet rows, 0 free),
// relax_steps damped Jacobi sweeps, restriction of the residual (pressure
// unconstrained), recursion, prolongation, relax_steps sweeps; on the
// coarsest level x = C b with the pinned dense inverse C.
template <typename T>
void ns_relax(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  const Level &L = P.L[l];
  const int64_t n = (P.dim + 1) * L.g.Nv;
  for (int it = 0; it < P.opts.relax_steps; ++it) {
    apply_ns<T>(P, l, W.d[l], x, s);
    if (L.asm64) {  // additive Schwarz: every colour with the residual b - J x of the sweep's start
      const T *Minv = sizeof(T) == 8 ? (const T *)L.asm64 : (const T *)L.asm32;
      for (int c = 0; c < asm_colours(L.g); ++c)
        launch_asm_apply<T>(L.g, Minv, c, b, W.d[l], x, (T)P.opts.relax_omega, s);
    } else {
      jacobi_relax<T>(x, b, W.d[l], ns_invdiag<T>(L), (T)P.opts.relax_omega, n, s);
    }
  }
}

template <typename T>
void ns_vcycle(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  Level &L = P.L[l];
  if (l == P.nlev - 1) {
    dense_apply<T>(P.coarse_inv, P.coarse_n, b, x, s);
    return;
  }
  const int64_t n = (P.dim + 1) * L.g.Nv;
  launch_fill_dirichlet<T>(L.g, x, b, s);
  vec_fill<T>(x + P.dim * L.g.Nv, T(0), L.g.Nv, s);
  ns_relax<T>(P, l, x, b, s);
  T *r = W.r[l];
  apply_ns<T>(P, l, r, x, s);
  vec_axpby<T>(r, T(1), b, T(-1), n, s);  // r = b - J x
  Level &C = P.L[l + 1];
  launch_restrict<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), W.b[l + 1], r, s, 1, rwork<T>(L));
  ns_vcycle<T>(P, l + 1, W.x[l + 1], W.b[l + 1], s);
  launch_prolongate_add<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), x, W.x[l + 1], s, 1);
  ns_relax<T>(P, l, x, b, s);
}

// ---------------------------------------------------------------- block preconditioner
template <typename T>
void precondition(mfs_problem &P, T *y, const T *r, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  const LevelGeom &g = P.L[0].g;
  const int64_t nu = P.dim * g.Nv, np = g.Np;
  const T *rp = r + nu;
  T *yp = y + nu;
  // Schur: y_p = -nu M_p^{-1} r_p, M_p^{-1} by Jacobi-PCG (z0 = 0)
  double *rho = P.scal, *pqs = P.scal + PCG_MAX;
  vec_fill<T>(W.pz, T(0), np, s);
  vec_copy<T>(W.pres, rp, np, s);
  vec_mul<T>(W.ps, W.pinv, W.pres, np, s);
  vec_copy<T>(W.pp, W.ps, np, s);
  multi_dot<T>(W.pres, 0, 1, W.ps, np, rho, P.partials, s);
  for (int it = 0; it < P.opts.schur_iterations; ++it) {
    apply_op<T>(P, MFS_OP_MASS_P, 0, W.pq, W.pp, s);
    multi_dot<T>(W.pp, 0, 1, W.pq, np, pqs + it, P.partials, s);
    pcg_update1<T>(W.pz, W.pres, W.ps, W.pp, W.pq, W.pinv, np, rho + it, pqs + it, s);
    multi_dot<T>(W.pres, 0, 1, W.ps, np, rho + it + 1, P.partials, s);
    pcg_update2<T>(W.pp, W.ps, np, rho + it + 1, rho + it, s);
  }
  vec_axpby<T>(yp, (T)(-P.nu), W.pz, T(0), np, s);
  // velocity: y_u = Vcycle(r_u - B y_p)
  apply_op<T>(P, MFS_OP_B, 0, W.t_u, yp, s);
  vec_axpby<T>(W.t_u, T(1), r, T(-1), nu, s);
  vcycle_level<T>(P, 0, y, W.t_u, s);
}

// ---------------------------------------------------------------- hp operators
// Cell operators through E-vectors: gather the cells' local values through
// the local->global maps, apply the cell kernels class by class, scatter the
// local results back with the transposed maps (Sec. 3, minimum rule).
template <typename T>
HpVecs<T> &hpv(HpLevel &L);
template <>
HpVecs<double> &hpv<double>(HpLevel &L) {
  return L.v64;
}
template <>
HpVecs<float> &hpv<float>(HpLevel &L) {
  return L.v32;
}
template <typename T>
T *hp_tab(HpData &H, int k);
template <>
double *hp_tab<double>(HpData &H, int k) {
  return H.tab64[k];
}
template <>
float *hp_tab<float>(HpData &H, int k) {
  return H.tab32[k];
}
template <typename T>
T *hp_evp(HpData &H, bool out);
template <>
double *hp_evp<double>(HpData &H, bool out) {
  return out ? H.evp_out64 : H.evp_in64;
}
template <>
float *hp_evp<float>(HpData &H, bool out) {
  return out ? H.evp_out32 : H.evp_in32;
}

template <typename T>
void hp_gather_space(const HpDevSpace &d, int ncomp, const T *x, T *ev, hipStream_t s) {
  hp_gather<T>(d.m, ncomp, x, ev, s);
}
template <typename T>
void hp_scatter_space(const HpDevSpace &d, int ncomp, bool use_dir, const T *ev, const T *src, T *dst, hipStream_t s) {
  hp_scatter<T>(d.m, ncomp, use_dir ? d.dir : nullptr, ev, src, dst, s);
}

// dst = op(src) on hp level l: mode of the cell kernels; velocity output
// Dirichlet rows = src_u (A, Stokes) or 0 (B)
template <typename T>
void hp_apply(mfs_problem &P, int l, int mode, T *dst_u, T *dst_p, const T *src_u, const T *src_p, hipStream_t s) {
  HpData &H = *P.hp;
  HpLevel &L = H.lev[l];
  HpVecs<T> &V = hpv<T>(L);
  const bool need_u = mode & (M_LAPLACE | M_DIVU), need_p = mode & (M_GRADP | M_MASSP);
  const bool out_u = mode & (M_LAPLACE | M_GRADP), out_p = mode & (M_DIVU | M_MASSP);
  if (need_u) hp_gather_space<T>(L.vd, 3, src_u, V.ev_in, s);
  if (need_p) hp_gather_space<T>(H.pd, 1, src_p, hp_evp<T>(H, false), s);
  const Level &S0 = P.L[0];
  EvArgs<T> ev{};
  ev.off_u = L.off_u;
  ev.off_p = H.off_p;
  ev.in_u = V.ev_in;
  ev.out_u = V.ev_out;
  ev.in_p = hp_evp<T>(H, false);
  ev.out_p = hp_evp<T>(H, true);
  for (size_t c = 0; c < L.class_k.size(); ++c) {
    ev.ncells = L.class_n[c];
    ev.cells = L.class_cells[c];
    launch_cell_op_ev<T>(S0.g, L.class_k[c], dev<T>(S0).X, hp_tab<T>(H, L.class_k[c]), mode, (T)P.nu, ev, s);
  }
  if (out_u)
    hp_scatter_space<T>(L.vd, 3, true, V.ev_out, (mode & M_LAPLACE) ? src_u : nullptr, dst_u, s);
  if (out_p) hp_scatter_space<T>(H.pd, 1, false, hp_evp<T>(H, true), nullptr, dst_p, s);
}

template <typename T>
void hp_apply_A(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s) {
  hp_apply<T>(P, l, M_LAPLACE, dst, nullptr, src, nullptr, s);
}

// transfers between hp level l and the next level (hp, or the structured
// degree-2 level 0 for the last hp level): gather coarse local values, embed
// them in the fine cells' degrees, inject into the fine unknowns at their owner
// nodes; restriction is the transposed sequence.
template <typename T>
void hp_prolongate_add(mfs_problem &P, int l, T *xf, const T *xc, hipStream_t s) {
  HpData &H = *P.hp;
  HpLevel &F = H.lev[l];
  T *evf = hpv<T>(F).ev_out;
  if (l + 1 < P.nhp) {
    HpLevel &C = H.lev[l + 1];
    T *evc = hpv<T>(C).ev_in;
    hp_gather_space<T>(C.vd, 3, xc, evc, s);
    hp_embed<T>(H.ncells, 3, F.deg, C.deg, H.embed, F.off_u, C.off_u, evc, evf, false, s);
  } else {
    T *tmp = std::is_same<T, double>::value ? (T *)H.tmp2_64 : (T *)H.tmp2_32;
    T *evc = std::is_same<T, double>::value ? (T *)H.ev2_64 : (T *)H.ev2_32;
    permute<T>(H.v2d.N, 3, H.perm2, xc, P.L[0].g.Nv, tmp, H.v2d.N, false, s);
    hp_gather_space<T>(H.v2d, 3, tmp, evc, s);
    hp_embed<T>(H.ncells, 3, F.deg, H.deg2, H.embed, F.off_u, H.off_u2, evc, evf, false, s);
  }
  hp_inject<T>(F.vd.N, 3, F.vd.owner_ev, F.vd.owner_nb, evf, xf, true, s);
}

template <typename T>
void hp_restrict(mfs_problem &P, int l, T *bc, const T *rf, hipStream_t s) {
  HpData &H = *P.hp;
  HpLevel &F = H.lev[l];
  T *evf = hpv<T>(F).ev_out;
  vec_fill<T>(evf, T(0), F.ev_size, s);
  hp_inject_t<T>(F.vd.N, 3, F.vd.owner_ev, F.vd.owner_nb, rf, evf, s);
  if (l + 1 < P.nhp) {
    HpLevel &C = H.lev[l + 1];
    T *evc = hpv<T>(C).ev_in;
    hp_embed<T>(H.ncells, 3, F.deg, C.deg, H.embed, F.off_u, C.off_u, evf, evc, true, s);
    hp_scatter_space<T>(C.vd, 3, true, evc, nullptr, bc, s);
  } else {
    T *tmp = std::is_same<T, double>::value ? (T *)H.tmp2_64 : (T *)H.tmp2_32;
    T *evc = std::is_same<T, double>::value ? (T *)H.ev2_64 : (T *)H.ev2_32;
    hp_embed<T>(H.ncells, 3, F.deg, H.deg2, H.embed, F.off_u, H.off_u2, evf, evc, true, s);
    hp_scatter_space<T>(H.v2d, 3, true, evc, nullptr, tmp, s);
    permute<T>(H.v2d.N, 3, H.perm2, tmp, H.v2d.N, bc, P.L[0].g.Nv, true, s);
  }
}

template <typename T>
void hp_chebyshev(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s) {
  HpLevel &L = P.hp->lev[l];
  HpVecs<T> &V = hpv<T>(L);
  const double lmax = L.lambda, lmin = lmax / P.opts.cheb_range;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho_old = 1.0 / sigma;
  const int64_t N = L.vd.N;
  if (zero_start) {
    mask_cheb_update<T>(L.vd.dir, N, 3, x, V.d, b, nullptr, V.invdiag, T(0), (T)(1.0 / theta), true, s);
  } else {
    hp_apply_A<T>(P, l, V.r, x, s);
    mask_cheb_update<T>(L.vd.dir, N, 3, x, V.d, b, V.r, V.invdiag, T(0), (T)(1.0 / theta), true, s);
  }
  for (int it = 1; it < P.opts.cheb_degree; ++it) {
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    hp_apply_A<T>(P, l, V.r, x, s);
    mask_cheb_update<T>(L.vd.dir, N, 3, x, V.d, b, V.r, V.invdiag, (T)(rho * rho_old), (T)(2.0 * rho / delta), false,
                        s);
    rho_old = rho;
  }
}

// V-cycle of the velocity block: hp p-levels, then the structured levels
template <typename T>
void hp_vcycle(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  if (l == P.nhp) {
    vcycle_level<T>(P, 0, x, b, s);
    return;
  }
  HpLevel &L = P.hp->lev[l];
  HpVecs<T> &V = hpv<T>(L);
  const int64_t n = 3 * L.vd.N;
  mask_fill_dirichlet<T>(L.vd.dir, L.vd.N, 3, x, b, s);
  hp_chebyshev<T>(P, l, x, b, true, s);
  hp_apply_A<T>(P, l, V.r, x, s);
  vec_axpby<T>(V.r, T(1), b, T(-1), n, s);
  T *bc, *xc;
  if (l + 1 < P.nhp) {
    bc = hpv<T>(P.hp->lev[l + 1]).b;
    xc = hpv<T>(P.hp->lev[l + 1]).x;
  } else {
    bc = work<T>(P).b[0];
    xc = work<T>(P).x[0];
  }
  hp_restrict<T>(P, l, bc, V.r, s);
  hp_vcycle<T>(P, l + 1, xc, bc, s);
  hp_prolongate_add<T>(P, l, x, xc, s);
  hp_chebyshev<T>(P, l, x, b, false, s);
}

template <typename T>
HpVecs<T> &hp0(mfs_problem &P) {
  return hpv<T>(P.hp->lev[0]);
}
template <typename T>
T **hp_pvec(HpData &H);
template <>
double **hp_pvec<double>(HpData &H) {
  return H.p64;
}
template <>
float **hp_pvec<float>(HpData &H) {
  return H.p32;
}

// block preconditioner on the hp system (as precondition())
template <typename T>
void hp_precondition(mfs_problem &P, T *y, const T *r, hipStream_t s) {
  HpData &H = *P.hp;
  const int64_t nu = 3 * H.lev[0].vd.N, np = H.pd.N;
  const T *rp = r + nu;
  T *yp = y + nu;
  T **pv = hp_pvec<T>(H);
  T *pres = pv[0], *ps = pv[1], *pp = pv[2], *pq = pv[3], *pz = pv[4];
  const T *pinv = std::is_same<T, double>::value ? (const T *)H.pinv64 : (const T *)H.pinv32;
  T *tu = std::is_same<T, double>::value ? (T *)H.tu64 : (T *)H.tu32;
  double *rho = P.scal, *pqs = P.scal + PCG_MAX;
  vec_fill<T>(pz, T(0), np, s);
  vec_copy<T>(pres, rp, np, s);
  vec_mul<T>(ps, pinv, pres, np, s);
  vec_copy<T>(pp, ps, np, s);
  multi_dot<T>(pres, 0, 1, ps, np, rho, P.partials, s);
  for (int it = 0; it < P.opts.schur_iterations; ++it) {
    hp_apply<T>(P, 0, M_MASSP, nullptr, pq, nullptr, pp, s);
    multi_dot<T>(pp, 0, 1, pq, np, pqs + it, P.partials, s);
    pcg_update1<T>(pz, pres, ps, pp, pq, pinv, np, rho + it, pqs + it, s);
    multi_dot<T>(pres, 0, 1, ps, np, rho + it + 1, P.partials, s);
    pcg_update2<T>(pp, ps, np, rho + it + 1, rho + it, s);
  }
  vec_axpby<T>(yp, (T)(-P.nu), pz, T(0), np, s);
  hp_apply<T>(P, 0, M_GRADP, tu, nullptr, nullptr, yp, s);
  vec_axpby<T>(tu, T(1), r, T(-1), nu, s);
  hp_vcycle<T>(P, 0, y, tu, s);
}

// the system operator and its preconditioner: Stokes (block preconditioner)
// or Navier-Stokes Jacobian (monolithic V-cycle)
template <typename T>
void amr_apply_ns(mfs_problem &P, int j, T *dst, const T *src, hipStream_t s);
template <typename T>
void amr_vcycle(mfs_problem &P, int j, T *x, const T *b, hipStream_t s);

void apply_system(mfs_problem &P, double *dst, const double *src, hipStream_t s) {
  if (P.amr) {
    amr_apply_ns<double>(P, 0, dst, src, s);
    return;
  }
  if (P.hp) {
    const int64_t nu = 3 * P.hp->lev[0].vd.N;
    hp_apply<double>(P, 0, M_LAPLACE | M_GRADP | M_DIVU, dst, dst + nu, src, src + nu, s);
    return;
  }
  apply_op<double>(P, P.ns ? MFS_OP_NS_JACOBIAN : MFS_OP_STOKES, 0, dst, src, s);
}
// sizes of the system vectors
int64_t sys_vel(const mfs_problem &P) {
  if (P.amr) return 3 * P.amr->lev[0].N;
  return P.hp ? 3 * P.hp->lev[0].vd.N : P.dim * P.L[0].g.Nv;
}
int64_t sys_pres(const mfs_problem &P) {
  if (P.amr) return P.amr->lev[0].N;
  return P.hp ? P.hp->pd.N : P.L[0].g.Np;
}
int64_t sys_n(const mfs_problem &P) { return sys_vel(P) + sys_pres(P); }
template <typename T>
void precondition_any(mfs_problem &P, T *y, const T *r, hipStream_t s) {
  if (P.amr)
    amr_vcycle<T>(P, 0, y, r, s);
  else if (P.hp)
    hp_precondition<T>(P, y, r, s);
  else if (P.ns)
    ns_vcycle<T>(P, 0, y, r, s);
  else
    precondition<T>(P, y, r, s);
}

// The recorded preconditioner holds host values that were current when it
// was recorded (smoother intervals, the linearisation's dt and Newton flag,
// option counts); calls that change them drop the recording.
void drop_prec_graph(mfs_problem &P) {
  for (int i = 0; i < 2; ++i) {
    if (P.prec_graph[i]) (void)hipGraphExecDestroy(P.prec_graph[i]);
    P.prec_graph[i] = nullptr;
  }
}

template <typename T>
PrecWork<T> &prec_work(mfs_problem &P);
template <>
PrecWork<double> &prec_work<double>(mfs_problem &P) {
  return P.w64;
}
template <>
PrecWork<float> &prec_work<float>(mfs_problem &P) {
  return P.w32;
}

// Preconditioner from full_in to full_out of the precision's work vectors on
// stream s.  Its launches (a few hundred small kernels per V-cycle and Schur
// solve, no host synchronisation and no memset) are recorded once on a
// private stream and replayed as one graph launch, so that small problems do
// not pay the host cost of every launch in each FGMRES iteration.  Recording
// that fails (e.g. a runtime without stream capture) falls back to direct
// launches.  The FP64 one is staged through fixed vectors too, since the
// Krylov columns it reads and writes move every iteration.
template <typename T>
void precondition_rec(mfs_problem &P, hipStream_t s) {
  constexpr int w = sizeof(T) == 8 ? 1 : 0;
  T *y = prec_work<T>(P).full_out, *r = prec_work<T>(P).full_in;
  if (!P.kr.graphs || P.graph_failed) {
    precondition_any<T>(P, y, r, s);
    return;
  }
  if (!P.prec_graph[w]) {
    if (!P.cap_stream) P.cap_stream = capture_stream_acquire();
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      P.graph_failed = true;
      precondition_any<T>(P, y, r, s);
      return;
    }
    try {
      precondition_any<T>(P, y, r, P.cap_stream);
    } catch (...) {
      if (hipStreamEndCapture(P.cap_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      throw;
    }
    MFS_HIP(hipStreamEndCapture(P.cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&P.prec_graph[w], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      P.prec_graph[w] = nullptr;
      P.graph_failed = true;
      precondition_any<T>(P, y, r, s);
      return;
    }
  }
  MFS_HIP(hipGraphLaunch(P.prec_graph[w], s));
}

// ---------------------------------------------------------------- FGMRES
void kr_enqueue_residual(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  apply_system(P, K.w, K.x, s);
  vec_axpby<double>(K.w, 1.0, K.b, -1.0, n, s);  // w = b - K x
  multi_dot<double>(K.w, 0, 1, K.w, n, K.dev + 96, P.partials, s);
  MFS_HIP(hipMemcpyAsync(K.host + 96, K.dev + 96, sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipEventRecord(K.ev, s));
}

// one Arnoldi step: z_j = P^{-1} v_j (pre), w = K z_j (the system
// operator), Gram-Schmidt and the readback (post)
void kr_step_pre(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  const int j = K.j;
  double *vj = K.V + (int64_t)j * K.ld, *zj = K.Z + (int64_t)j * K.ld;
  if (K.prec == MFS_FP32) {
    vec_cast<float, double>(P.w32.full_in, vj, n, s);
    precondition_rec<float>(P, s);
    vec_cast<double, float>(zj, P.w32.full_out, n, s);
  } else if (K.graphs && !P.graph_failed) {
    vec_copy<double>(P.w64.full_in, vj, n, s);
    precondition_rec<double>(P, s);
    vec_copy<double>(zj, P.w64.full_out, n, s);
  } else {
    precondition_any<double>(P, zj, vj, s);
  }
}
void kr_step_post(mfs_problem &P, hipStream_t s);
void kr_enqueue_step(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  kr_step_pre(P, s);
  apply_system(P, K.w, K.Z + (int64_t)K.j * K.ld, s);
  kr_step_post(P, s);
}
void kr_step_post(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  const int j = K.j;
  // classical Gram-Schmidt, twice
  // (the second pass's dots and the norm are fused with the updates before them)
  multi_dot<double>(K.V, K.ld, j + 1, K.w, n, K.dev, P.partials, s);
  axpy_dot<double>(K.w, K.V, K.ld, j + 1, K.dev, j + 1, false, n, K.dev + 32, P.partials, s);
  axpy_dot<double>(K.w, K.V, K.ld, j + 1, K.dev + 32, 0, true, n, K.dev + 64, P.partials, s);
  scale_inv_sqrt<double>(K.V + (int64_t)(j + 1) * K.ld, K.w, n, K.dev + 64, s);
  MFS_HIP(hipMemcpyAsync(K.host, K.dev, 65 * sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipEventRecord(K.ev, s));
}

// update x with the current Krylov coefficients (j columns) and enqueue the
// true-residual check
void kr_enqueue_update(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  const int m = K.j;
  if (m > 0) {
    std::vector<double> y(m);
    for (int i = m - 1; i >= 0; --i) {
      double v = K.gv[i];
      for (int c = i + 1; c < m; ++c) v -= K.H[i * K.m + c] * y[c];
      y[i] = v / K.H[i * K.m + i];
    }
    MFS_HIP(hipStreamSynchronize(s));  // previous use of yhost finished
    std::memcpy(K.yhost, y.data(), m * sizeof(double));
    MFS_HIP(hipMemcpyAsync(K.ydev, K.yhost, m * sizeof(double), hipMemcpyHostToDevice, s));
    multi_combine<double>(K.x, K.Z, K.ld, m, K.ydev, n, true, s);
  }
  kr_enqueue_residual(P, s);
}

void kr_finish(mfs_problem &P, double rel, int status) {
  Krylov &K = P.kr;
  hipStream_t s = K.s;
  const int64_t nu = sys_vel(P), np = sys_pres(P);
  const double *m1 = P.amr ? P.amr->ones : P.hp ? P.hp->m1 : P.m1;
  // pressure with zero mass-weighted mean (Navier-Stokes: m1 = 1, nodal mean)
  if (np > 0) {
    double *num = P.scal + 4 * PCG_MAX + 8, *den = num + 1;
    double *ones = P.amr ? P.amr->scratch : P.hp ? P.hp->ones : P.tmp_full;  // scratch of >= np entries
    multi_dot<double>(m1, 0, 1, K.x + nu, np, num, P.partials, s);
    vec_fill<double>(ones, 1.0, np, s);
    multi_dot<double>(m1, 0, 1, ones, np, den, P.partials, s);
    shift_mean(K.x + nu, np, num, den, s);
  }
  MFS_HIP(hipStreamSynchronize(s));
  K.info.iterations = K.iters;
  K.info.status = status;
  K.info.rel_residual = rel;
  K.info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - K.t0).count();
  K.state = 4;
}

// advance the state machine after its event completed; with `defer` an
// Arnoldi step is not enqueued but reported (true) for the caller to enqueue
bool kr_process(mfs_problem &P, bool defer = false) {
  Krylov &K = P.kr;
  hipStream_t s = K.s;
  const int64_t n = sys_n(P);
  if (K.state == 1 || K.state == 3) {
    const double rr = std::sqrt(std::max(K.host[96], 0.0));
    if (K.state == 1 && K.bnorm == 0.0) K.bnorm = rr;  // first call stores ||b - K x0||, replaced below
    const double rel = K.bnorm > 0 ? rr / K.bnorm : 0.0;
    if (rel <= K.rtol || K.iters >= K.maxit) {
      kr_finish(P, rel, rel <= K.rtol ? MFS_OK : MFS_ENOCONV);
      return false;
    }
    // (re)start: V_0 = r / ||r||
    K.beta = rr;
    std::fill(K.H.begin(), K.H.end(), 0.0);
    std::fill(K.gv.begin(), K.gv.end(), 0.0);
    K.gv[0] = rr;
    K.j = 0;
    scale_inv_sqrt<double>(K.V, K.w, n, K.dev + 96, s);
    K.state = 2;
    if (defer) return true;
    kr_enqueue_step(P, s);
    return false;
  }
  if (K.state == 2) {
    const int j = K.j, m = K.m;
    // column j of the Hessenberg matrix
    std::vector<double> h(j + 2);
    for (int i = 0; i <= j; ++i) h[i] = K.host[i] + K.host[32 + i];
    h[j + 1] = std::sqrt(std::max(K.host[64], 0.0));
    for (int i = 0; i < j; ++i) {
      const double t = K.cs[i] * h[i] + K.sn[i] * h[i + 1];
      h[i + 1] = -K.sn[i] * h[i] + K.cs[i] * h[i + 1];
      h[i] = t;
    }
    const double den = std::hypot(h[j], h[j + 1]);
    K.cs[j] = den > 0 ? h[j] / den : 1.0;
    K.sn[j] = den > 0 ? h[j + 1] / den : 0.0;
    h[j] = den;
    K.gv[j + 1] = -K.sn[j] * K.gv[j];
    K.gv[j] = K.cs[j] * K.gv[j];
    for (int i = 0; i <= j; ++i) K.H[i * m + j] = h[i];
    K.j = j + 1;
    K.iters += 1;
    const double est = std::fabs(K.gv[j + 1]) / K.bnorm;
    const bool breakdown = !(h[j] > 0) || K.host[64] <= 0.0;
    if (est <= K.rtol || K.j == m || K.iters >= K.maxit || breakdown) {
      K.state = 3;
      kr_enqueue_update(P, s);
      return false;
    }
    if (defer) return true;
    kr_enqueue_step(P, s);
  }
  return false;
}

}  // namespace

// ====================================================================== C ABI

namespace {
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
}  // namespace

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

namespace {
int setup_structured(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *arena, size_t bytes,
                     void *stream, mfs_problem **out);
}  // namespace

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

}  // extern "C"

namespace {
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
}  // namespace

extern "C" {

int mfs_destroy(mfs_problem *p) {
  release(p);
  return MFS_OK;
}

}  // extern "C"

namespace {
// ---------------------------------------------------------------- hp set-up
// device copy of an hp space's maps; ev_off: per-cell E-vector offset of the
// cell's first component block, ncomp_stride: whether rows carry a component
// stride ((k+1)^3 for the velocity)
// interleave (with vector_comp): the three components of a cell-local node
// are adjacent (slot 3 j + comp) instead of (k+1)^3 apart
// device maps of an hp space: rows cell by cell at the cells' E-vector
// offsets; vector spaces (velocity) keep the three components of a node side
// by side (slot 3 j + comp); constrained spaces drop the Dirichlet columns
// (their values do not enter the cells) and list no rows for Dirichlet
// unknowns (the scatter writes those rows itself)
void hp_upload(HpData &H, const HpSpaceHost &V, bool constrained, const std::vector<int64_t> &ev_off, bool vector_comp,
               HpDevSpace &d, hipStream_t s) {
  const int64_t ncells = (int64_t)V.deg.size();
  d.N = V.N;
  d.nrows = V.row_base[ncells];
  HpMaps &m = d.m;
  m.N = d.N;
  m.nrows = d.nrows;
  m.nb = vector_comp ? 1 : 0;
  const int stride = vector_comp ? 3 : 1;
  std::vector<int> rcol((size_t)d.nrows), rslot((size_t)d.nrows), hcol;
  std::vector<int64_t> hptr(1, 0), tptr((size_t)V.N + 1, 0), wptr((size_t)V.N + 1, 0);
  std::vector<double> hval;
  for (int64_t c = 0; c < ncells; ++c) {
    const int k = V.deg[c], nb = (k + 1) * (k + 1) * (k + 1);
    for (int j = 0; j < nb; ++j) {
      const int64_t r = V.row_base[c] + j;
      MFS_REQUIRE(ev_off[c] + (int64_t)stride * j < (int64_t(1) << 31), MFS_EINVAL, "E-vector too long");
      rslot[r] = (int)(ev_off[c] + (int64_t)stride * j);
      const int64_t b = V.row_ptr[r], e = V.row_ptr[r + 1];
      if (e - b == 1 && V.val[b] == 1.0 && !(constrained && V.dirichlet[V.col[b]])) {
        rcol[r] = V.col[b];
        tptr[V.col[b] + 1] += 1;
        continue;
      }
      rcol[r] = -1 - (int)(hptr.size() - 1);
      for (int64_t q = b; q < e; ++q) {
        const int g = V.col[q];
        if (constrained && V.dirichlet[g]) continue;
        hcol.push_back(g);
        hval.push_back(V.val[q]);
        wptr[g + 1] += 1;
      }
      hptr.push_back((int64_t)hcol.size());
    }
  }
  for (int64_t g = 0; g < V.N; ++g) {
    tptr[g + 1] += tptr[g];
    wptr[g + 1] += wptr[g];
  }
  std::vector<int> tslot((size_t)tptr[V.N]), wslot((size_t)wptr[V.N]);
  std::vector<double> wval((size_t)wptr[V.N]);
  {
    std::vector<int64_t> tf(tptr.begin(), tptr.end() - 1), wf(wptr.begin(), wptr.end() - 1);
    for (int64_t r = 0; r < d.nrows; ++r) {
      if (rcol[r] >= 0) {
        tslot[tf[rcol[r]]++] = rslot[r];
        continue;
      }
      const int64_t h = -1 - (int64_t)rcol[r];
      for (int64_t q = hptr[h]; q < hptr[h + 1]; ++q) {
        const int64_t o = wf[hcol[q]]++;
        wslot[o] = rslot[r];
        wval[o] = hval[q];
      }
    }
  }
  std::vector<int64_t> heavy;
  for (int64_t g = 0; g < V.N; ++g)
    if (!(constrained && V.dirichlet[g]) && (tptr[g + 1] - tptr[g]) + (wptr[g + 1] - wptr[g]) > HP_SCATTER_LIGHT)
      heavy.push_back(g);
  std::vector<int64_t> oev(V.N);
  std::vector<int> onb(V.N);
  for (int64_t g = 0; g < V.N; ++g) {
    const int c = V.owner_cell[g];
    oev[g] = (constrained && V.dirichlet[g]) ? -1 : ev_off[c] + (int64_t)stride * V.owner_local[g];
    onb[g] = vector_comp ? 1 : 0;
  }
  m.rcol = H.upload(rcol, s);
  m.rslot = H.upload(rslot, s);
  m.hptr = H.upload(hptr, s);
  m.hcol = H.upload(hcol, s);
  m.hval = H.upload(hval, s);
  m.tptr = H.upload(tptr, s);
  m.tslot = H.upload(tslot, s);
  m.wptr = H.upload(wptr, s);
  m.wslot = H.upload(wslot, s);
  m.wval = H.upload(wval, s);
  m.nheavy = (int64_t)heavy.size();
  m.heavy = heavy.empty() ? nullptr : H.upload(heavy, s);
  d.owner_ev = H.upload(oev, s);
  d.owner_nb = H.upload(onb, s);
  d.dir = constrained ? H.upload(V.dirichlet, s) : nullptr;
  MFS_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
}

std::vector<int64_t> ev_offsets(const std::vector<int> &deg, int ncomp, int shift, int64_t *total) {
  std::vector<int64_t> off(deg.size());
  int64_t o = 0;
  for (size_t c = 0; c < deg.size(); ++c) {
    off[c] = o;
    const int64_t m = deg[c] + 1 - shift;
    o += ncomp * m * m * m;
  }
  *total = o;
  return off;
}

template <typename T>
void hp_alloc_vecs(HpData &H, HpVecs<T> &v, int64_t N, int64_t ev) {
  v.x = H.alloc<T>(3 * N);
  v.b = H.alloc<T>(3 * N);
  v.r = H.alloc<T>(3 * N);
  v.d = H.alloc<T>(3 * N);
  v.ev_in = H.alloc<T>(ev);
  v.ev_out = H.alloc<T>(ev);
  v.invdiag = H.alloc<T>(N);
}

// lambda_max(D^{-1} A) of hp level l by CG-Lanczos (FP64), as for the
// structured levels
double hp_estimate_lambda(mfs_problem &P, int l, hipStream_t s) {
  HpLevel &L = P.hp->lev[l];
  const int64_t N = L.vd.N, n = 3 * N;
  HpVecs<double> &V = L.v64;
  double *r = V.x, *z = V.b, *p = V.d, *q = V.r;
  std::vector<double> h(n);
  uint64_t st = P.opts.seed * 1000003ULL + (uint64_t)l + 7919ULL;
  for (int64_t i = 0; i < n; ++i) {
    h[i] = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    if (L.V.dirichlet[i % N]) h[i] = 0.0;
  }
  MFS_HIP(hipMemcpyAsync(r, h.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  double *dv = P.scal + 4 * PCG_MAX;
  auto dot = [&](const double *a, const double *b) {
    multi_dot<double>(a, 0, 1, b, n, dv, P.partials, s);
    double v;
    MFS_HIP(hipMemcpyAsync(&v, dv, sizeof(double), hipMemcpyDeviceToHost, s));
    MFS_HIP(hipStreamSynchronize(s));
    return v;
  };
  mask_diag_scale<double>(L.vd.dir, N, 3, z, V.invdiag, r, s);
  vec_copy<double>(p, z, n, s);
  double rz = dot(r, z);
  std::vector<double> alpha, beta;
  const int steps = std::max(2, P.opts.lanczos_steps);
  for (int j = 0; j < steps && rz > 0; ++j) {
    hp_apply_A<double>(P, l, q, p, s);
    const double pq = dot(p, q);
    if (!(pq > 0)) break;
    const double a = rz / pq;
    vec_axpby<double>(r, -a, q, 1.0, n, s);
    mask_diag_scale<double>(L.vd.dir, N, 3, z, V.invdiag, r, s);
    const double rz2 = dot(r, z);
    const double b = rz2 / rz;
    vec_axpby<double>(p, 1.0, z, b, n, s);
    alpha.push_back(a);
    beta.push_back(b);
    rz = rz2;
    if (rz2 <= 1e-30 * rz) break;
  }
  const int m = (int)alpha.size();
  MFS_REQUIRE(m > 0, MFS_EINVAL, "Lanczos estimate failed on hp level %d", l);
  std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
  for (int j = 0; j < m; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j < m - 1) e[j] = std::sqrt(beta[j]) / alpha[j];
  }
  double lmax;
  sturm_max_eig(d, e, lmax);
  return lmax;
}

void hp_build(mfs_problem &P, const std::vector<int> &deg0, hipStream_t s) {
  HpData &H = *P.hp;
  const LevelGeom &g0 = P.L[0].g;
  for (int a = 0; a < 3; ++a) H.n[a] = g0.n[a];
  H.ncells = g0.ncells;
  // degrees per hp level: k <- max(k - 1, 2) until all are 2; that last
  // level is the structured degree-2 level
  std::vector<std::vector<int>> degs{deg0};
  while (P.opts.mg_levels && *std::max_element(degs.back().begin(), degs.back().end()) > 2) {
    std::vector<int> d = degs.back();
    for (int &k : d) k = std::max(k - 1, 2);
    degs.push_back(d);
  }
  if (degs.size() > 1) degs.pop_back();
  H.lev.resize(degs.size());
  P.nhp = (int)degs.size();
  for (size_t l = 0; l < degs.size(); ++l) {
    HpLevel &L = H.lev[l];
    L.V.build(H.n, degs[l]);
    const auto off = ev_offsets(degs[l], 3, 0, &L.ev_size);
    hp_upload(H, L.V, true, off, true, L.vd, s);
    L.off_u = H.upload(off, s);
    L.deg = H.upload(degs[l], s);
    for (int k = 2; k <= 6; ++k) {
      std::vector<int> cells;
      for (int64_t c = 0; c < H.ncells; ++c)
        if (degs[l][c] == k) cells.push_back((int)c);
      if (cells.empty()) continue;
      L.class_k.push_back(k);
      L.class_n.push_back((int)cells.size());
      L.class_cells.push_back(H.upload(cells, s));
    }
    hp_alloc_vecs(H, L.v64, L.V.N, L.ev_size);
    hp_alloc_vecs(H, L.v32, L.V.N, L.ev_size);
    L.diag = H.alloc<double>(L.V.N);
  }
  // pressure space of the finest level (degree k - 1, no Dirichlet unknowns)
  {
    std::vector<int> dp(deg0);
    for (int &k : dp) k -= 1;
    H.Pr.build(H.n, dp);
    const auto off = ev_offsets(deg0, 1, 1, &H.evp_size);
    hp_upload(H, H.Pr, false, off, false, H.pd, s);
    H.off_p = H.upload(off, s);
    H.evp_in64 = H.alloc<double>(H.evp_size);
    H.evp_out64 = H.alloc<double>(H.evp_size);
    H.evp_in32 = H.alloc<float>(H.evp_size);
    H.evp_out32 = H.alloc<float>(H.evp_size);
  }
  // uniform degree 2 and its place in the structured node grid
  {
    std::vector<int> d2(H.ncells, 2);
    H.V2.build(H.n, d2);
    const auto off = ev_offsets(d2, 3, 0, &H.ev2_size);
    hp_upload(H, H.V2, true, off, true, H.v2d, s);
    H.off_u2 = H.upload(off, s);
    H.deg2 = H.upload(d2, s);
    std::vector<int64_t> perm(H.V2.N);
    for (int64_t gi = 0; gi < H.V2.N; ++gi) {
      double p[3];
      H.V2.reference_point(gi, p);
      int64_t idx[3];
      for (int a = 0; a < 3; ++a) idx[a] = (int64_t)std::llround(2.0 * p[a]);
      perm[gi] = idx[0] + (int64_t)g0.nv[0] * (idx[1] + (int64_t)g0.nv[1] * idx[2]);
    }
    H.perm2 = H.upload(perm, s);
    H.ev2_64 = H.alloc<double>(H.ev2_size);
    H.ev2_32 = H.alloc<float>(H.ev2_size);
    H.tmp2_64 = H.alloc<double>(3 * H.V2.N);
    H.tmp2_32 = H.alloc<float>(3 * H.V2.N);
  }
  // 1D embeddings [kf][kc] and per-degree tables
  {
    std::vector<double> E(8 * 8 * MAXQ * MAXQ, 0.0);
    for (int kf = 1; kf <= 7; ++kf)
      for (int kc = 1; kc <= kf; ++kc) {
        double *T = E.data() + ((int64_t)kf * MAXQ + kc) * MAXQ * MAXQ;
        if (kc == kf) {
          for (int i = 0; i <= kf; ++i) T[i * MAXQ + i] = 1.0;
        } else {
          const auto pe = p_embedding(kf, kc);
          for (int i = 0; i <= kf; ++i)
            for (int j = 0; j <= kc; ++j) T[i * MAXQ + j] = pe[i * (kc + 1) + j];
        }
      }
    H.embed = H.upload(E, s);
    for (int k = 2; k <= 6; ++k) {
      const auto t = make_tables(k, k - 1);
      std::vector<float> t32(t.begin(), t.end());
      H.tab64[k] = H.upload(t, s);
      H.tab32[k] = H.upload(t32, s);
    }
  }
  // block preconditioner vectors, Krylov space of the hp system
  const int64_t Nu = H.lev[0].V.N, Np = H.Pr.N, ntot = 3 * Nu + Np;
  for (int i = 0; i < 5; ++i) {
    H.p64[i] = H.alloc<double>(Np);
    H.p32[i] = H.alloc<float>(Np);
  }
  H.tu64 = H.alloc<double>(3 * Nu);
  H.tu32 = H.alloc<float>(3 * Nu);
  H.pdiag = H.alloc<double>(3 * Np);
  H.m1 = H.alloc<double>(Np);
  H.ones = H.alloc<double>(Np);
  H.pinv64 = H.alloc<double>(Np);
  H.pinv32 = H.alloc<float>(Np);
  P.w32.full_in = H.alloc<float>(ntot);
  P.w32.full_out = H.alloc<float>(ntot);
  P.w64.full_in = H.alloc<double>(ntot);
  P.w64.full_out = H.alloc<double>(ntot);
  if (P.opts.mg_levels) {
    Krylov &K = P.kr;
    K.ld = kr_ld(ntot);
    K.V = H.alloc<double>((K.m + 1) * K.ld);
    K.Z = H.alloc<double>(K.m * K.ld);
    K.w = H.alloc<double>(ntot);
  }
  MFS_HIP(hipStreamSynchronize(s));
  // Jacobi diagonals of the velocity block on every hp level: A applied to
  // the indicators of three colours at once (one per component)
  for (int l = 0; l < P.nhp; ++l) {
    HpLevel &L = H.lev[l];
    int ncol = 0;
    const auto col = L.V.colours(&ncol);
    L.vd.colour = H.upload(col, s);
    L.vd.ncolours = ncol;
    double *e = L.v64.x, *y = L.v64.b;
    for (int c = 0; c < ncol; c += 3) {
      const int cols[3] = {c, c + 1 < ncol ? c + 1 : -1, c + 2 < ncol ? c + 2 : -1};
      colour_indicator(L.vd.colour, L.V.N, cols, e, s);
      hp_apply_A<double>(P, l, y, e, s);
      colour_extract(L.vd.colour, L.V.N, cols, y, L.diag, s);
    }
    launch_reciprocal(L.v64.invdiag, L.v32.invdiag, L.diag, L.V.N, s);
  }
  // pressure mass: diagonal (Jacobi-PCG of the Schur complement) and M_p 1
  {
    int ncol = 0;
    const auto col = H.Pr.colours(&ncol);
    H.pd.colour = H.upload(col, s);
    H.pd.ncolours = ncol;
    double *e = H.p64[0], *y = H.p64[1], *ind = H.pdiag;  // pdiag: 3 Np scratch here
    double *diag = H.p64[2];
    for (int c = 0; c < ncol; ++c) {
      const int cols[3] = {c, -1, -1};
      colour_indicator(H.pd.colour, Np, cols, ind, s);
      vec_copy<double>(e, ind, Np, s);
      hp_apply<double>(P, 0, M_MASSP, nullptr, y, nullptr, e, s);
      colour_extract(H.pd.colour, Np, cols, y, diag, s);
    }
    launch_reciprocal(H.pinv64, H.pinv32, diag, Np, s);
    vec_copy<double>(H.pdiag, diag, Np, s);
    vec_fill<double>(H.ones, 1.0, Np, s);
    hp_apply<double>(P, 0, M_MASSP, nullptr, H.m1, nullptr, H.ones, s);
  }
  if (P.opts.mg_levels)
    for (int l = 0; l < P.nhp; ++l) H.lev[l].lambda = P.opts.cheb_safety * hp_estimate_lambda(P, l, s);
  MFS_HIP(hipStreamSynchronize(s));
}
// ---------------------------------------------------------------- refined meshes
template <typename T>
T *amr_ev(AmrLevel &V, int i) {
  if constexpr (sizeof(T) == 8) return V.ev64[i]; else return V.ev32[i];
}
template <typename T>
const T *amr_tab(const AmrData &A) {
  if constexpr (sizeof(T) == 8) return A.tab64; else return A.tab32;
}
template <typename T>
const T *amr_X(const AmrLevel &V) {
  if constexpr (sizeof(T) == 8) return V.X64; else return V.X32;
}
template <typename T>
T *amr_qd(AmrLevel &V) {
  if constexpr (sizeof(T) == 8) return V.qd64; else return V.qd32;
}
template <typename T>
T *amr_w(AmrLevel &V, int i) {
  if constexpr (sizeof(T) == 8) return V.w64[i]; else return V.w32[i];
}
template <typename T>
const T *amr_inv(const AmrLevel &V) {
  if constexpr (sizeof(T) == 8) return V.inv64; else return V.inv32;
}
// levels with their own Jacobian (the uniform base of the multigrid sequence
// belongs to the structured hierarchy)
int amr_nop(const AmrData &A) { return A.mg ? (int)A.lev.size() - 1 : 1; }

// f(0), ..., f(n-1) on n host threads; the first failure is rethrown here
// with its error text (which the worker set in its own thread-local slot)
void parallel_tasks(int n, const std::function<void(int)> &f) {
  std::vector<std::exception_ptr> ex((size_t)std::max(n, 0));
  std::vector<std::string> msg((size_t)std::max(n, 0));
  std::vector<std::thread> th;
  for (int i = 0; i < n; ++i)
    th.emplace_back([&, i] {
      try {
        f(i);
      } catch (...) {
        ex[i] = std::current_exception();
        msg[i] = get_error();
      }
    });
  for (auto &t : th) t.join();
  for (int i = 0; i < n; ++i)
    if (ex[i]) {
      set_error("%s", msg[i].c_str());
      std::rethrow_exception(ex[i]);
    }
}

// device maps of a level: rows are cell-major ((k+1)^3 per cell), so row r's
// E-vector slots are 4r .. 4r+3 and the lists need no slot offsets; rows of
// one unknown with weight 1 store only that unknown
void amr_maps_host(const AmrSpaceHost &S, AmrMapsHost &out) {
  const HpSpaceHost &V = S.V;
  const int64_t nrows = V.row_base[S.ncells], N = S.N;
  out.N = N;
  out.nrows = nrows;
  std::vector<int> &rcol = out.rcol;
  rcol.assign((size_t)nrows, 0);
  std::vector<int64_t> &hptr = out.hptr;
  hptr.assign(1, 0);
  std::vector<int> &hcol = out.hcol;
  std::vector<double> &hval = out.hval;
  std::vector<int64_t> &tptr = out.tptr, &wptr = out.wptr;
  tptr.assign((size_t)N + 1, 0);
  wptr.assign((size_t)N + 1, 0);
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t b = V.row_ptr[r], e = V.row_ptr[r + 1];
    if (e - b == 1 && V.val[b] == 1.0) {
      rcol[r] = V.col[b];
      tptr[V.col[b] + 1] += 1;
      continue;
    }
    rcol[r] = -1 - (int)(hptr.size() - 1);
    for (int64_t q = b; q < e; ++q) {
      hcol.push_back(V.col[q]);
      hval.push_back(V.val[q]);
      wptr[V.col[q] + 1] += 1;
    }
    hptr.push_back((int64_t)hcol.size());
  }
  for (int64_t g = 0; g < N; ++g) {
    tptr[g + 1] += tptr[g];
    wptr[g + 1] += wptr[g];
  }
  std::vector<int> &trow = out.trow, &wrow = out.wrow;
  std::vector<double> &wval = out.wval;
  trow.assign((size_t)tptr[N], 0);
  wrow.assign((size_t)wptr[N], 0);
  wval.assign((size_t)wptr[N], 0.0);
  {
    std::vector<int64_t> tf(tptr.begin(), tptr.end() - 1), wf(wptr.begin(), wptr.end() - 1);
    for (int64_t r = 0; r < nrows; ++r) {
      if (rcol[r] >= 0) {
        trow[tf[rcol[r]]++] = (int)r;
        continue;
      }
      const int64_t h = -1 - (int64_t)rcol[r];
      for (int64_t q = hptr[h]; q < hptr[h + 1]; ++q) {
        const int64_t o = wf[hcol[q]]++;
        wrow[o] = (int)r;
        wval[o] = hval[q];
      }
    }
  }
  std::vector<int64_t> &heavy = out.heavy;
  heavy.clear();
  for (int64_t g = 0; g < N; ++g)
    if ((tptr[g + 1] - tptr[g]) + (wptr[g + 1] - wptr[g]) > AMR_LIGHT) heavy.push_back(g);
  const int64_t nb = V.row_base[1] - V.row_base[0];
  out.owner.resize((size_t)N);
  for (int64_t g = 0; g < N; ++g) out.owner[g] = (int)(V.owner_cell[g] * nb + V.owner_local[g]);
}

void amr_maps_upload(HpData &H, const AmrSpaceHost &S, const AmrMapsHost &h, AmrMaps &M, hipStream_t s) {
  M.N = h.N;
  M.nrows = h.nrows;
  M.rcol = H.upload(h.rcol, s);
  M.hptr = H.upload(h.hptr, s);
  M.hcol = H.upload(h.hcol, s);
  M.hval = H.upload(h.hval, s);
  M.tptr = H.upload(h.tptr, s);
  M.trow = H.upload(h.trow, s);
  M.wptr = H.upload(h.wptr, s);
  M.wrow = H.upload(h.wrow, s);
  M.wval = H.upload(h.wval, s);
  M.dir = H.upload(S.V.dirichlet, s);
  M.owner = H.upload(h.owner, s);
  M.nheavy = (int64_t)h.heavy.size();
  M.heavy = h.heavy.empty() ? nullptr : H.upload(h.heavy, s);
  MFS_HIP(hipStreamSynchronize(s));  // the caller may release the host vectors
}

// device data of a level; `op`: the level applies its own Jacobian
void amr_level_upload(AmrData &A, AmrLevel &V, bool op, bool work, hipStream_t s) {
  AmrSpaceHost &S = V.S;
  const int k = A.k;
  const int64_t nc = S.ncells, NQ = (int64_t)(k + 1) * (k + 1) * (k + 1);
  V.N = S.N;
  V.NQ = NQ;
  LevelGeom &g = V.g;
  g.dim = 3;
  g.k = g.kp = k;
  g.n[0] = g.n[1] = 1;
  g.n[2] = (int)nc;
  g.ncells = nc;
  g.nv[0] = g.nv[1] = k + 1;
  g.nv[2] = (int)(k * nc + 1);
  g.np[0] = g.np[1] = k + 1;
  g.np[2] = g.nv[2];
  g.Nv = g.Np = (int64_t)g.nv[0] * g.nv[1] * g.nv[2];
  g.cart = 1;  // octree leaves of a Cartesian cube
  HpData &H = A.H;
  amr_maps_upload(H, S, V.mh, V.M, s);
  V.mh = AmrMapsHost();
  for (int i = 0; i < 2; ++i) {
    V.ev64[i] = H.alloc<double>(4 * nc * NQ);
    V.ev32[i] = H.alloc<float>(4 * nc * NQ);
  }
  if (op) {
    V.X64 = H.upload(S.Xcell, s);
    std::vector<float> x32(S.Xcell.begin(), S.Xcell.end());
    V.X32 = H.upload(x32, s);
    V.qd64 = H.alloc<double>(nc * NQ * NS_QD);
    V.qd32 = H.alloc<float>(nc * NQ * NS_QD);
    V.u0 = H.alloc<double>(7 * V.N);  // state [u0 (3N) | p0 (N) | u~ (3N)]
    if (A.mg) {
      V.diag = H.alloc<double>(4 * V.N);
      V.inv64 = H.alloc<double>(4 * V.N);
      V.inv32 = H.alloc<float>(4 * V.N);
      MFS_REQUIRE(V.ncolour_host > 0, MFS_EINVAL, "level colouring missing");
      V.colour = H.upload(V.colour_host, s);
      V.ncolours = V.ncolour_host;
      MFS_HIP(hipStreamSynchronize(s));
      std::vector<int>().swap(V.colour_host);
    }
    MFS_HIP(hipStreamSynchronize(s));  // x32 goes out of scope
  }
  if (work)
    for (int i = 0; i < 4; ++i) {
      V.w64[i] = H.alloc<double>(4 * V.N);
      V.w32[i] = H.alloc<float>(4 * V.N);
    }
  MFS_HIP(hipStreamSynchronize(s));
  S.V = HpSpaceHost();  // the row maps and corners live on the device now
  std::vector<double>().swap(S.Xcell);
}

// the levels: the given mesh, and with multigrid its global coarsenings down
// to the uniform base mesh, with their cell and unknown relations
void amr_build(mfs_problem &P, const mfs_refined_mesh &m, int k, bool mg, hipStream_t s) {
  AmrData &A = *P.amr;
  A.n = m.n;
  A.k = k;
  A.L = m.levels;
  A.mg = mg;
  // the meshes of every level: the given one and, with multigrid, its global
  // coarsenings down to the uniform base mesh
  std::vector<std::vector<int>> lv(1), ix(1);
  MFS_REQUIRE(m.ncells >= 1 && m.level && m.idx, MFS_EINVAL, "empty cell list");
  MFS_REQUIRE(m.levels >= 0 && m.levels <= 4, MFS_EINVAL, "refinement levels %d out of range [0, 4]", m.levels);
  lv[0].assign(m.level, m.level + m.ncells);
  ix[0].assign(m.idx, m.idx + 3 * m.ncells);
  if (mg) {
    int top = 0;
    for (int l : lv[0]) top = std::max(top, l);
    MFS_REQUIRE(top >= 1, MFS_EINVAL, "the mesh is not refined: set up the base mesh with mfs_setup");
    MFS_REQUIRE(top <= m.levels, MFS_EINVAL, "cell level %d above the mesh's %d levels", top, m.levels);
    for (int j = 1; j <= top; ++j) {
      lv.emplace_back();
      ix.emplace_back();
      amr_coarsen(m.n, lv[j - 1], ix[j - 1], lv[j], ix[j]);
    }
  }
  const int nlev = (int)lv.size();
  A.lev.resize(nlev);
  const int nop = amr_nop(A);
  // host construction, one thread per level: space, maps, colouring
  parallel_tasks(nlev, [&](int j) {
    AmrLevel &V = A.lev[j];
    V.S.build(m.n, m.levels - j, (int64_t)lv[j].size(), lv[j].data(), ix[j].data(), k);
    amr_maps_host(V.S, V.mh);
    if (mg && j < nop) V.colour_host = V.S.colours(&V.ncolour_host);
  });
  std::vector<AmrTransferHost> T((size_t)nlev - 1);
  std::vector<std::vector<int64_t>> inj((size_t)nlev - 1);
  parallel_tasks(nlev - 1, [&](int j) {
    const AmrLevel &F = A.lev[j], &C = A.lev[j + 1];
    T[j] = amr_transfer(m.n, F.S.level, F.S.idx, C.S.level, C.S.idx);
    inj[j] = amr_injection(F.S, C.S);
  });
  HpData &H = A.H;
  for (int j = 0; j + 1 < nlev; ++j) {
    AmrLevel &F = A.lev[j];
    F.parent = H.upload(T[j].parent, s);
    F.octant = H.upload(T[j].octant, s);
    F.cptr = H.upload(T[j].cptr, s);
    F.child = H.upload(T[j].child, s);
    F.inject = H.upload(inj[j], s);
  }
  MFS_HIP(hipStreamSynchronize(s));  // T and inj go out of scope
  for (size_t j = 0; j < A.lev.size(); ++j) amr_level_upload(A, A.lev[j], (int)j < nop, mg, s);
  const auto tab = make_tables(k, k);
  std::vector<float> tab32(tab.begin(), tab.end());
  A.tab64 = H.upload(tab, s);
  A.tab32 = H.upload(tab32, s);
  A.E.k = k;
  for (int h = 0; h < 2; ++h)
    for (int t = 0; t <= k; ++t)
      for (int q = 0; q <= k; ++q) {
        // coarse basis function q of the k+1 equispaced nodes at fine node t of half h
        const double x = 0.5 * (h + (double)t / k);
        double v = 1.0;
        for (int r = 0; r <= k; ++r)
          if (r != q) v *= (x - (double)r / k) / ((double)(q - r) / k);
        A.E.w[h][t][q] = v;
      }
  const int64_t N0 = A.lev[0].N;
  A.ones = H.alloc<double>(N0);
  A.scratch = H.alloc<double>(N0);
  A.state = H.alloc<double>(4 * N0);
  if (mg) {  // the BDF2 / Newton driver: history, residual, correction
    P.nw_uh = H.alloc<double>(3 * N0);
    P.nw_F = H.alloc<double>(4 * N0);
    P.nw_dx = H.alloc<double>(4 * N0);
  }
  vec_fill<double>(A.ones, 1.0, N0, s);
  MFS_HIP(hipStreamSynchronize(s));
}

// constrained Jacobian on level j: gather with the constraints (the
// velocity's Dirichlet columns dropped), cell kernel on the E-vectors,
// transposed scatter (identity on the velocity Dirichlet rows)
template <typename T>
void amr_apply_ns(mfs_problem &P, int j, T *dst, const T *src, hipStream_t s) {
  AmrData &A = *P.amr;
  MFS_REQUIRE(A.ready, MFS_EINVAL, "mfs_set_linearization has not been called");
  AmrLevel &V = A.lev[j];
  T *evi = amr_ev<T>(V, 0), *evo = amr_ev<T>(V, 1);
  amr_gather<T>(V.M, 4, true, src, evi, s);
  launch_ns<T>(V.g, nullptr, amr_tab<T>(A), 1, (T)P.nu, (T)A.dt, A.newton, nullptr, nullptr, amr_qd<T>(V), s, evo,
               evi, amr_X<T>(V));
  amr_scatter<T>(V.M, evo, src, dst, s);
}

// prolongation from level j+1 to level j (added to xf): gather the coarse
// cells' values through the coarse constraints, embed them in the fine
// cells, take each fine unknown from its owner slot (Dirichlet velocity rows
// and columns zero, pressure unconstrained)
template <typename T>
void amr_prolongate_add(mfs_problem &P, int j, T *xf, const T *xc, hipStream_t s) {
  AmrData &A = *P.amr;
  AmrLevel &F = A.lev[j], &C = A.lev[j + 1];
  T *evc = amr_ev<T>(C, 0), *evf = amr_ev<T>(F, 1);
  amr_gather<T>(C.M, 4, true, xc, evc, s);
  amr_embed<T>(A.E, F.S.ncells, C.S.ncells, F.parent, F.octant, evc, evf, s);
  amr_inject<T>(F.M, evf, xf, true, s);
}

// restriction (the transpose) from level j to level j+1
template <typename T>
void amr_restrict(mfs_problem &P, int j, T *bc, const T *rf, hipStream_t s) {
  AmrData &A = *P.amr;
  AmrLevel &F = A.lev[j], &C = A.lev[j + 1];
  T *evc = amr_ev<T>(C, 0), *evf = amr_ev<T>(F, 1);
  vec_fill<T>(evf, T(0), 4 * F.S.ncells * F.NQ, s);
  amr_inject_t<T>(F.M, rf, evf, s);
  amr_embed_t<T>(A.E, F.S.ncells, C.S.ncells, F.cptr, F.child, F.octant, evf, evc, s);
  amr_scatter<T>(C.M, evc, nullptr, bc, s);
}

template <typename T>
void amr_relax(mfs_problem &P, int j, T *x, const T *b, hipStream_t s) {
  AmrLevel &V = P.amr->lev[j];
  T *d = amr_w<T>(V, 3);
  for (int it = 0; it < P.opts.relax_steps; ++it) {
    amr_apply_ns<T>(P, j, d, x, s);
    jacobi_relax<T>(x, b, d, amr_inv<T>(V), (T)P.opts.relax_omega, 4 * V.N, s);
  }
}

// one V-cycle from level j: as the structured monolithic V-cycle, with the
// GC levels first and the structured hierarchy of the base mesh below them
template <typename T>
void amr_vcycle(mfs_problem &P, int j, T *x, const T *b, hipStream_t s) {
  AmrData &A = *P.amr;
  MFS_REQUIRE(A.mg, MFS_EUNSUPPORTED, "problem was set up without multigrid levels");
  if (j == amr_nop(A)) {
    ns_vcycle<T>(P, 0, x, b, s);
    return;
  }
  AmrLevel &V = A.lev[j], &C = A.lev[j + 1];
  mask_fill_dirichlet<T>(V.M.dir, V.N, 3, x, b, s);  // x = b on Dirichlet rows, 0 elsewhere
  vec_fill<T>(x + 3 * V.N, T(0), V.N, s);
  amr_relax<T>(P, j, x, b, s);
  T *r = amr_w<T>(V, 2);
  amr_apply_ns<T>(P, j, r, x, s);
  vec_axpby<T>(r, T(1), b, T(-1), 4 * V.N, s);  // r = b - J x
  T *xc = amr_w<T>(C, 0), *bc = amr_w<T>(C, 1);
  amr_restrict<T>(P, j, bc, r, s);
  amr_vcycle<T>(P, j + 1, xc, bc, s);
  amr_prolongate_add<T>(P, j, x, xc, s);
  amr_relax<T>(P, j, x, b, s);
}

// Jacobi diagonal of level j by colour probes (FP64): J applied to the
// indicator of one colour in one component gives the diagonal entries of
// that colour (no two unknowns of a colour meet in a cell)
void amr_diagonal(mfs_problem &P, int j, double *diag, hipStream_t s) {
  AmrLevel &V = P.amr->lev[j];
  double *e = V.w64[0], *y = V.w64[1];
  for (int col = 0; col < V.ncolours; ++col)
    for (int comp = 0; comp < 4; ++comp) {
      amr_colour_probe(V.colour, V.N, col, comp, e, s);
      amr_apply_ns<double>(P, j, y, e, s);
      amr_colour_take(V.colour, V.N, col, comp, y, diag, s);
    }
}

// mfs_set_linearization on a refined mesh: u0 at the unknowns of level 0,
// copied at the coarse unknowns level by level; point data per level (u0
// through the unconstrained scalar map into the velocity slots); with
// multigrid the structured base levels and the GC levels' diagonals
// Linearisation at the state x0 = [u0 | p0] (4 N) with the BDF2 history u~
// (3 N; NULL: u~ = u0) on every level (coarse levels take the fields at their
// unknowns, which are fine unknowns), as ns_set_point.
void amr_set_point(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta,
                   bool mg, hipStream_t s) {
  AmrData &A = *P.amr;
  A.ready = false;
  A.mg_ready = false;
  A.dt = dt;
  A.newton = newton ? 1 : 0;
  const int nop = amr_nop(A);
  const int64_t N0 = A.lev[0].N;
  MFS_HIP(hipMemcpyAsync(A.lev[0].u0, x0, 4 * N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  MFS_HIP(hipMemcpyAsync(A.lev[0].u0 + 4 * N0, uh ? uh : x0, 3 * N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int j = 1; j < nop; ++j)
    permute<double>(A.lev[j].N, 7, A.lev[j - 1].inject, A.lev[j - 1].u0, A.lev[j - 1].N, A.lev[j].u0, A.lev[j].N,
                    false, s);
  for (int j = 0; j < nop; ++j) {
    AmrLevel &V = A.lev[j];
    double *ev = V.ev64[0], *evh = V.ev64[1];
    amr_gather<double>(V.M, 4, false, V.u0, ev, s);  // the state keeps its boundary values
    amr_gather<double>(V.M, 3, false, V.u0 + 4 * V.N, evh, s);
    NsPoint<double> pt;
    pt.keep_delta = keep_delta;
    pt.evhist = evh;
    launch_ns<double>(V.g, nullptr, A.tab64, 0, P.nu, dt, A.newton, nullptr, nullptr, V.qd64, s, nullptr, ev, V.X64,
                      &pt);
    vec_cast<float, double>(V.qd32, V.qd64, V.g.ncells * V.NQ * NS_QD, s);
  }
  if (A.mg) {
    AmrLevel &F = A.lev[nop - 1], &B = A.lev[nop];
    MFS_REQUIRE(B.N == P.L[0].g.Nv, MFS_EINVAL, "base level mismatch");
    permute<double>(B.N, 4, F.inject, F.u0, F.N, P.tmp_full, B.N, false, s);
    permute<double>(B.N, 3, F.inject, F.u0 + 4 * F.N, F.N, P.tmp2, B.N, false, s);
    ns_set_point(P, P.tmp_full, P.tmp2, dt, newton, keep_delta, mg, s);  // structured levels; synchronises
    A.ready = true;
    if (!mg) return;
    try {
      for (int j = 0; j < nop; ++j) {
        AmrLevel &V = A.lev[j];
        amr_diagonal(P, j, V.diag, s);
        launch_reciprocal(V.inv64, V.inv32, V.diag, 4 * V.N, s);
      }
      MFS_HIP(hipStreamSynchronize(s));
      A.mg_ready = true;
    } catch (...) {
      A.ready = false;
      throw;
    }
    return;
  }
  MFS_HIP(hipStreamSynchronize(s));
  A.ready = true;
}

// Linearisation point u0 of a Jacobian alone: p0 = 0 and u~ = u0
void amr_set_linearization(mfs_problem &P, const double *u0, double dt, int newton, hipStream_t s) {
  const int64_t N0 = P.amr->lev[0].N;
  double *x0 = P.amr->state;
  MFS_HIP(hipMemcpyAsync(x0, u0, 3 * N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  vec_fill<double>(x0 + 3 * N0, 0.0, N0, s);
  amr_set_point(P, x0, nullptr, dt, newton, 0, true, s);
}

// F = the nonlinear residual at the level-0 state of the last linearisation
// (through the hanging-node maps); Dirichlet velocity rows 0
void amr_residual(mfs_problem &P, double *F, hipStream_t s) {
  AmrData &A = *P.amr;
  MFS_REQUIRE(A.ready, MFS_EINVAL, "no linearisation state: call mfs_set_linearization_point first");
  AmrLevel &V = A.lev[0];
  double *evi = V.ev64[0], *evo = V.ev64[1];
  launch_ns<double>(V.g, nullptr, A.tab64, 2, P.nu, A.dt, A.newton, nullptr, nullptr, V.qd64, s, evo, evi, V.X64);
  amr_scatter<double>(V.M, evo, nullptr, F, s);
}

void amr_vmult(mfs_problem &P, int op, int prec, int level, void *dst, const void *src, hipStream_t s) {
  MFS_REQUIRE(op == MFS_OP_NS_JACOBIAN, MFS_EUNSUPPORTED,
              "refined-mesh problems provide the Navier-Stokes Jacobian (operator %d requested)", op);
  if (prec == MFS_FP64)
    amr_apply_ns<double>(P, level, (double *)dst, (const double *)src, s);
  else
    amr_apply_ns<float>(P, level, (float *)dst, (const float *)src, s);
}

// mfs_vmult on an hp problem: the hp levels (all operators on the finest,
// the velocity block on the others), then the structured levels
void hp_vmult(mfs_problem &P, int op, int prec, int level, void *dst, const void *src, hipStream_t s) {
  if (level >= P.nhp) {
    MFS_REQUIRE(op == MFS_OP_A, MFS_EUNSUPPORTED, "structured levels of an hp problem carry the velocity block only");
    if (prec == MFS_FP64)
      apply_A<double>(P, level - P.nhp, (double *)dst, (const double *)src, s);
    else
      apply_A<float>(P, level - P.nhp, (float *)dst, (const float *)src, s);
    return;
  }
  MFS_REQUIRE(level == 0 || op == MFS_OP_A, MFS_EUNSUPPORTED, "coarser hp levels carry the velocity block only");
  const int64_t nu = 3 * P.hp->lev[level].V.N;
  auto run = [&](auto *d, auto *x) {
    using T = std::remove_pointer_t<decltype(d)>;
    switch (op) {
      case MFS_OP_STOKES: hp_apply<T>(P, level, M_LAPLACE | M_GRADP | M_DIVU, d, d + nu, x, x + nu, s); break;
      case MFS_OP_A: hp_apply<T>(P, level, M_LAPLACE, d, nullptr, x, nullptr, s); break;
      case MFS_OP_B: hp_apply<T>(P, level, M_GRADP, d, nullptr, nullptr, x, s); break;
      case MFS_OP_BT: hp_apply<T>(P, level, M_DIVU, nullptr, d, x, nullptr, s); break;
      case MFS_OP_MASS_P: hp_apply<T>(P, level, M_MASSP, nullptr, d, nullptr, x, s); break;
      default: MFS_REQUIRE(false, MFS_EUNSUPPORTED, "operator %d is not available on hp problems", op);
    }
  };
  if (prec == MFS_FP64)
    run((double *)dst, (const double *)src);
  else
    run((float *)dst, (const float *)src);
}
}  // namespace

extern "C" {

int mfs_setup_hp(const mfs_mesh *mesh, const int *cell_degree, double nu, const mfs_options *opts, void *stream,
                 mfs_problem **out) {
  mfs_problem *P = nullptr;
  int rc = guard([&] {
    MFS_REQUIRE(out != nullptr, MFS_EINVAL, "out is NULL");
    *out = nullptr;
    MFS_REQUIRE(mesh != nullptr && mesh->dim == 3, MFS_EUNSUPPORTED, "hp problems are three-dimensional");
    MFS_REQUIRE(cell_degree != nullptr, MFS_EINVAL, "cell_degree is NULL");
    mfs_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_options(&o);
    MFS_REQUIRE(o.pressure_offset == 1, MFS_EINVAL, "hp problems are Taylor-Hood (pressure_offset = 1)");
    for (int a = 0; a < 3; ++a) MFS_REQUIRE(mesh->n[a] >= 1, MFS_EINVAL, "n[%d] must be >= 1", a);
    const int64_t ncells = (int64_t)mesh->n[0] * mesh->n[1] * mesh->n[2];
    std::vector<int> deg(cell_degree, cell_degree + ncells);
    for (int64_t c = 0; c < ncells; ++c)
      MFS_REQUIRE(deg[c] >= 2 && deg[c] <= 6, MFS_EINVAL, "cell %lld: degree %d out of range [2, 6]", (long long)c,
                  deg[c]);
    mfs_options ob = o;
    ob.p_min = 2;
    const int rcb = mfs_setup(mesh, 2, nu, &ob, stream, &P);
    if (rcb != MFS_OK) throw mfs::Error{rcb};
    P->opts = o;
    P->opts.p_min = 2;
    P->hp = new HpData();
    hp_build(*P, deg, S(stream));
    *out = P;
  });
  if (rc != MFS_OK) {
    release(P);
    return rc;
  }
  return MFS_OK;
}

int mfs_refined_count(const mfs_refined_mesh *mesh, int k, int64_t *n_unknowns, int64_t *n_hanging) {
  return guard([&] {
    MFS_REQUIRE(mesh != nullptr, MFS_EINVAL, "mesh is NULL");
    AmrSpaceHost S;
    S.build(mesh->n, mesh->levels, mesh->ncells, mesh->level, mesh->idx, k);
    if (n_unknowns) *n_unknowns = S.N;
    if (n_hanging) *n_hanging = S.nhanging;
  });
}

int mfs_refined_mg_metrics(const mfs_refined_mesh *mesh, int nprocs, double *eta) {
  return guard([&] {
    MFS_REQUIRE(mesh != nullptr && eta != nullptr, MFS_EINVAL, "NULL argument");
    MFS_REQUIRE(nprocs >= 1, MFS_EINVAL, "nprocs must be >= 1");
    MFS_REQUIRE(mesh->n >= 1 && mesh->n <= 4096 && mesh->levels >= 0 && mesh->levels <= 4 && mesh->ncells >= 1,
                MFS_EINVAL, "bad refined mesh");
    std::vector<int> level(mesh->level, mesh->level + mesh->ncells), idx(mesh->idx, mesh->idx + 3 * mesh->ncells);
    for (int64_t c = 0; c < mesh->ncells; ++c) {
      MFS_REQUIRE(level[c] >= 0 && level[c] <= mesh->levels, MFS_EINVAL, "cell %lld: level out of range",
                  (long long)c);
      for (int a = 0; a < 3; ++a)
        MFS_REQUIRE(idx[3 * c + a] >= 0 && idx[3 * c + a] < (mesh->n << level[c]), MFS_EINVAL,
                    "cell %lld: index out of range", (long long)c);
    }
    amr_mg_metrics(mesh->n, level, idx, nprocs, eta);
  });
}

int mfs_setup_refined(const mfs_refined_mesh *mesh, int k, double nu, const mfs_options *opts, void *stream,
                      mfs_problem **out) {
  mfs_problem *P = nullptr;
  int rc = guard([&] {
    MFS_REQUIRE(out != nullptr, MFS_EINVAL, "out is NULL");
    *out = nullptr;
    MFS_REQUIRE(mesh != nullptr, MFS_EINVAL, "mesh is NULL");
    MFS_REQUIRE(nu > 0 && std::isfinite(nu), MFS_EINVAL, "nu must be positive");
    mfs_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_options(&o);
    MFS_REQUIRE(o.pressure_offset == 0, MFS_EUNSUPPORTED,
                "refined meshes provide the equal-order Navier-Stokes Jacobian (pressure_offset = 0)");
    MFS_REQUIRE(k == 1 || k == 2, MFS_EUNSUPPORTED, "refined meshes support degrees 1 and 2 (got %d)", k);
    MFS_REQUIRE(o.relax_type == MFS_RELAX_JACOBI, MFS_EUNSUPPORTED,
                "refined meshes relax with point Jacobi (additive Schwarz patches need a structured level)");
    MFS_REQUIRE(mesh->n >= 1 && mesh->n <= 4096, MFS_EINVAL, "base cells per direction %d out of range", mesh->n);
    const bool mg = o.mg_levels != 0;
    if (mg) {
      // the structured hierarchy of the uniform base mesh (Cartesian unit cube)
      const int n = mesh->n;
      std::vector<double> X((size_t)3 * (n + 1) * (n + 1) * (n + 1));
      for (int z = 0; z <= n; ++z)
        for (int y = 0; y <= n; ++y)
          for (int x = 0; x <= n; ++x) {
            const size_t v = (size_t)x + (size_t)(n + 1) * (y + (size_t)(n + 1) * z);
            X[3 * v] = (double)x / n;
            X[3 * v + 1] = (double)y / n;
            X[3 * v + 2] = (double)z / n;
          }
      mfs_mesh bm{};
      bm.dim = 3;
      bm.n[0] = bm.n[1] = bm.n[2] = n;
      bm.vertices = X.data();
      const int rcb = mfs_setup(&bm, k, nu, &o, stream, &P);
      if (rcb != MFS_OK) throw mfs::Error{rcb};
    } else {
      P = new mfs_problem();
      P->dim = 3;
      P->nu = nu;
      P->opts = o;
      P->stream = S(stream);
      P->ns = true;
    }
    P->amr = new AmrData();
    amr_build(*P, *mesh, k, mg, S(stream));
    AmrData &A = *P->amr;
    P->namr = amr_nop(A);
    if (mg) {
      // FGMRES and the FP32 staging vectors at the size of the refined system
      const int64_t n0 = 4 * A.lev[0].N;
      Krylov &K = P->kr;
      K.ld = kr_ld(n0);
      K.V = A.H.alloc<double>((K.m + 1) * K.ld);
      K.Z = A.H.alloc<double>(K.m * K.ld);
      K.w = A.H.alloc<double>(n0);
      P->w32.full_in = A.H.alloc<float>(n0);
      P->w32.full_out = A.H.alloc<float>(n0);
      P->w64.full_in = A.H.alloc<double>(n0);
      P->w64.full_out = A.H.alloc<double>(n0);
    }
    *out = P;
  });
  if (rc != MFS_OK) {
    release(P);
    return rc;
  }
  return MFS_OK;
}

}  // extern "C"

namespace {
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

// a structured Taylor-Hood problem whose system operator is the degree-2
// brick kernel (its Arnoldi steps can share one grouped operator launch)
bool q2_groupable(const mfs_problem &P) {
  if (P.hp || P.amr || P.ns || !use_specialised()) return false;
  const LevelGeom &g = P.L[0].g;
  return g.dim == 3 && g.k == 2 && g.kp == 1 && q2_face_elems(g) > 0;
}

void kr_begin(mfs_problem &P, const double *b, double *x, const mfs_options &o, hipStream_t s) {
  Krylov &K = P.kr;
  MFS_REQUIRE(P.opts.mg_levels, MFS_EINVAL, "solve needs the multigrid hierarchy (mg_levels = 1)");
  MFS_REQUIRE(P.hp || P.L[0].g.Np > 0, MFS_EINVAL, "solve needs a pressure space");
  MFS_REQUIRE(!P.ns || (P.ns_ready && P.ns_mg_ready), MFS_EINVAL,
              "mfs_set_linearization has not been called (or the state was set without multigrid data)");
  MFS_REQUIRE(!P.amr || (P.amr->ready && P.amr->mg_ready), MFS_EINVAL,
              "mfs_set_linearization has not been called (or the state was set without multigrid data)");
  const LevelGeom &g = P.L[0].g;
  const int64_t n = sys_n(P);
  K.b = b;
  K.x = x;
  K.s = s;
  K.rtol = o.rtol;
  K.maxit = o.maxit;
  K.prec = o.precond_precision;
  K.graphs = o.graphs != 0;
  K.iters = 0;
  K.j = 0;
  K.H.assign((size_t)(K.m + 1) * K.m, 0.0);
  K.cs.assign(K.m, 0.0);
  K.sn.assign(K.m, 0.0);
  K.gv.assign(K.m + 1, 0.0);
  K.info = mfs_solve_info{};
  K.t0 = std::chrono::steady_clock::now();
  // ||b|| first (state 1 reads it as bnorm), then the residual of x0
  if (P.amr)  // x0: lifting of b's Dirichlet rows
    mask_fill_dirichlet<double>(P.amr->lev[0].M.dir, P.amr->lev[0].N, 3, x, b, s);
  else if (P.hp)
    mask_fill_dirichlet<double>(P.hp->lev[0].vd.dir, P.hp->lev[0].vd.N, 3, x, b, s);
  else
    launch_fill_dirichlet<double>(g, x, b, s);
  vec_fill<double>(x + sys_vel(P), 0.0, sys_pres(P), s);
  multi_dot<double>(b, 0, 1, b, n, K.dev + 100, P.partials, s);
  MFS_HIP(hipMemcpyAsync(K.host + 100, K.dev + 100, sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  K.bnorm = std::sqrt(std::max(K.host[100], 0.0));
  if (K.bnorm == 0.0) K.bnorm = 1.0;
  K.state = 1;
  kr_enqueue_residual(P, s);
}
// Space-time Kronecker operator (Sec. 4 eq. (proceedings-kronecker)) on level
// 0: dst_q = sum_r G[q][r] M_u src_r + tau K src_q on the free rows, dst_q =
// src_q on the velocity Dirichlet rows; stage-major vectors of N entries per
// stage; work holds the Q stage masses (Q dim Nv).
template <typename T>
void st_apply(mfs_problem &P, int Q, const double *G, double tau, T *dst, const T *src, T *work, hipStream_t s) {
  const Level &L = P.L[0];
  const LevelGeom &g = L.g;
  const int64_t nv = P.dim * g.Nv, N = nv + g.Np;
  for (int r = 0; r < Q; ++r) apply_op<T>(P, MFS_OP_MASS_U, 0, work + r * nv, src + r * N, s);
  for (int q = 0; q < Q; ++q) {
    T *dq = dst + q * N;
    apply_op<T>(P, MFS_OP_STOKES, 0, dq, src + q * N, s);
    StageCoef C{};
    for (int r = 0; r < Q; ++r) C.c[r] = G[q * Q + r];
    stage_mix<T>(dq, N, 1, work, nv, Q, C, (T)tau, nv, N, s);
    vec_copy_boundary<T>(g, dq, src + q * N, s);  // identity rows
  }
}

// the state of a Navier-Stokes problem (structured or refined) at x0 = [u0 | p0]
void set_point_any(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta, bool mg,
                   hipStream_t s) {
  if (P.amr)
    amr_set_point(P, x0, uh, dt, newton, keep_delta, mg, s);
  else
    ns_set_point(P, x0, uh, dt, newton, keep_delta, mg, s);
}

// multigrid data (Jacobi diagonals, coarse inverse) of the current state
void point_mg_any(mfs_problem &P, hipStream_t s) {
  ns_mg_data(P, s);
  P.ns_mg_ready = true;
  if (P.amr) {
    AmrData &A = *P.amr;
    for (int j = 0; j < amr_nop(A); ++j) {
      AmrLevel &V = A.lev[j];
      amr_diagonal(P, j, V.diag, s);
      launch_reciprocal(V.inv64, V.inv32, V.diag, 4 * V.N, s);
    }
    A.mg_ready = true;
  }
  MFS_HIP(hipStreamSynchronize(s));
}

double device_norm(mfs_problem &P, const double *v, int64_t n, hipStream_t s) {
  Krylov &K = P.kr;
  multi_dot<double>(v, 0, 1, v, n, K.dev + 110, P.partials, s);
  MFS_HIP(hipMemcpyAsync(K.host + 110, K.dev + 110, sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  return std::sqrt(std::max(K.host[110], 0.0));
}

// One BDF2 step (Sec. 5) by Newton's method: F(x) = 0 with the time
// derivative alpha (u - u~), u~ = (4 u^n - u^{n-1}) / 3, delta_1 frozen at u^n
// for the whole step (so J is the exact derivative of F); each correction
// J dx = -F by FGMRES with the monolithic multigrid preconditioner.  x holds
// the initial guess with the new time level's Dirichlet values on entry.
void bdf2_step(mfs_problem &P, const double *u_n, const double *u_nm1, double *x, double dt,
               const mfs_newton_options &o, mfs_newton_info &info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  info = mfs_newton_info{};
  const int64_t nvel = sys_vel(P), n = sys_n(P);
  // the recorded preconditioner keeps dt and the Newton flag: drop it when they change
  if (P.ns_dt != dt || P.ns_newton != 1) drop_prec_graph(P);
  // u~ and delta_1 at u^n (state [u^n; 0])
  vec_copy<double>(P.nw_uh, u_n, nvel, s);
  vec_axpby<double>(P.nw_uh, -1.0 / 3.0, u_nm1, 4.0 / 3.0, nvel, s);
  double *st = P.nw_dx;
  vec_copy<double>(st, u_n, nvel, s);
  vec_fill<double>(st + nvel, 0.0, n - nvel, s);
  set_point_any(P, st, u_n, dt, 1, 0, false, s);
  mfs_options lo = P.opts;
  lo.rtol = o.linear_rtol;
  lo.maxit = o.linear_maxit;
  lo.precond_precision = o.precond_precision;
  for (int it = 0;; ++it) {
    set_point_any(P, x, P.nw_uh, dt, 1, 1, false, s);
    if (P.amr)
      amr_residual(P, P.nw_F, s);
    else
      ns_residual(P, P.nw_F, s);
    const double r = device_norm(P, P.nw_F, n, s);
    if (it == 0) info.res0 = r;
    info.res = r;
    info.newton_iterations = it;
    if (r <= std::max(o.rtol * info.res0, o.atol) || r == 0.0) {
      info.status = MFS_OK;
      break;
    }
    if (it == o.max_newton) {
      info.status = MFS_ENOCONV;
      break;
    }
    point_mg_any(P, s);
    vec_axpby<double>(P.nw_F, 0.0, P.nw_F, -1.0, n, s);  // b = -F
    // no need to solve beyond a tenth of the Newton target (and rounding
    // would stop FGMRES short of a relative tolerance far below it)
    const double target = std::max(o.rtol * info.res0, o.atol);
    lo.rtol = std::min(0.5, std::max(o.linear_rtol, 0.1 * target / r));
    kr_begin(P, P.nw_F, P.nw_dx, lo, s);
    Krylov &K = P.kr;
    while (K.state != 4) {
      MFS_HIP(hipEventSynchronize(K.ev));
      kr_process(P);
    }
    info.linear_iterations += K.info.iterations;
    if (K.info.status != MFS_OK) info.linear_failures += 1;
    vec_axpby<double>(x, 1.0, P.nw_dx, 1.0, n, s);  // x += dx
  }
  MFS_HIP(hipStreamSynchronize(s));
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}
}  // namespace

extern "C" {

void mfs_default_newton_options(mfs_newton_options *o) {
  if (!o) return;
  o->max_newton = 20;
  o->rtol = 1e-8;
  o->atol = 0.0;
  o->linear_rtol = 1e-6;
  o->linear_maxit = 200;
  o->precond_precision = MFS_FP32;
}

int mfs_st_vmult(mfs_problem *p, int Q, const double *G, double tau, int prec, void *dst, const void *src, void *work,
                 void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(!p->ns && !p->hp && !p->amr && p->L[0].g.Np > 0, MFS_EUNSUPPORTED,
                "the space-time operator needs a structured Taylor-Hood problem");
    MFS_REQUIRE(Q >= 1 && Q <= MFS_MAX_STAGES, MFS_EINVAL, "Q = %d outside [1, %d]", Q, MFS_MAX_STAGES);
    MFS_REQUIRE(G && dst && src && work && dst != src, MFS_EINVAL, "bad arguments");
    MFS_REQUIRE(tau > 0 && std::isfinite(tau), MFS_EINVAL, "tau must be positive");
    if (prec == MFS_FP64)
      st_apply<double>(*p, Q, G, tau, (double *)dst, (const double *)src, (double *)work, S(stream));
    else
      st_apply<float>(*p, Q, G, tau, (float *)dst, (const float *)src, (float *)work, S(stream));
  });
}

int mfs_st_stage_transfer(mfs_problem *p, int q_out, int q_in, const double *C, int prec, void *dst, const void *src,
                          void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(!p->hp && !p->amr, MFS_EUNSUPPORTED, "structured problems only");
    MFS_REQUIRE(q_out >= 1 && q_out <= MFS_MAX_STAGES && q_in >= 1 && q_in <= MFS_MAX_STAGES, MFS_EINVAL,
                "stage counts outside [1, %d]", MFS_MAX_STAGES);
    MFS_REQUIRE(C && dst && src && dst != src, MFS_EINVAL, "bad arguments");
    const LevelGeom &g = p->L[0].g;
    const int64_t N = p->dim * g.Nv + g.Np;
    StageCoef K{};
    for (int i = 0; i < q_out; ++i)
      for (int j = 0; j < q_in; ++j) K.c[i * MFS_MAX_STAGES + j] = C[i * q_in + j];
    if (prec == MFS_FP64)
      stage_mix<double>((double *)dst, N, q_out, (const double *)src, N, q_in, K, 0.0, N, N, S(stream));
    else
      stage_mix<float>((float *)dst, N, q_out, (const float *)src, N, q_in, K, 0.0f, N, N, S(stream));
  });
}

int mfs_set_linearization_point(mfs_problem *p, const double *x0, const double *u_hist, double dt, int newton,
                                int keep_delta, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "linearisation needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(x0 != nullptr, MFS_EINVAL, "x0 is NULL");
    MFS_REQUIRE(dt > 0 && std::isfinite(dt), MFS_EINVAL, "dt must be positive");
    MFS_REQUIRE(!keep_delta || (p->amr ? p->amr->ready : p->ns_ready), MFS_EINVAL,
                "keep_delta needs an earlier linearisation");
    drop_prec_graph(*p);
    set_point_any(*p, x0, u_hist, dt, newton, keep_delta, p->opts.mg_levels != 0, S(stream));
  });
}

int mfs_ns_residual(mfs_problem *p, double *F, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "the residual needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(F != nullptr, MFS_EINVAL, "F is NULL");
    if (p->amr)
      amr_residual(*p, F, S(stream));
    else
      ns_residual(*p, F, S(stream));
  });
}

int mfs_ns_bdf2_step(mfs_problem *p, const double *u_n, const double *u_nm1, double *x, double dt,
                     const mfs_newton_options *opts, mfs_newton_info *info, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "the BDF2 step needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(p->opts.mg_levels, MFS_EINVAL, "the BDF2 step needs the multigrid hierarchy (mg_levels = 1)");
    MFS_REQUIRE(u_n && u_nm1 && x, MFS_EINVAL, "NULL vector");
    MFS_REQUIRE(dt > 0 && std::isfinite(dt), MFS_EINVAL, "dt must be positive");
    mfs_newton_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_newton_options(&o);
    MFS_REQUIRE(o.max_newton >= 0 && o.max_newton <= 1000 && o.rtol >= 0 && o.atol >= 0 && o.linear_rtol > 0 &&
                    o.linear_maxit >= 1,
                MFS_EINVAL, "bad Newton options");
    check_prec(o.precond_precision);
    mfs_newton_info inf{};
    bdf2_step(*p, u_n, u_nm1, x, dt, o, inf, S(stream));
    if (info) *info = inf;
    if (inf.status != MFS_OK) {
      set_error("Newton did not reach rtol %.3e within %d iterations (||F|| %.3e from %.3e)", o.rtol, o.max_newton,
                inf.res, inf.res0);
      throw mfs::Error{MFS_ENOCONV};
    }
  });
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

int mfs_vmult(mfs_problem *p, int op, int prec, int level, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_level(p, level);
    check_prec(prec);
    MFS_REQUIRE(dst && src, MFS_EINVAL, "NULL vector");
    MFS_REQUIRE(dst != src, MFS_EINVAL, "dst and src must not alias");
    if (p->amr) {
      if (level < p->namr) {
        amr_vmult(*p, op, prec, level, dst, src, S(stream));
        return;
      }
      level -= p->namr;
    }
    if (p->hp) {
      hp_vmult(*p, op, prec, level, dst, src, S(stream));
      return;
    }
    if (prec == MFS_FP64)
      apply_op<double>(*p, op, level, (double *)dst, (const double *)src, S(stream));
    else
      apply_op<float>(*p, op, level, (float *)dst, (const float *)src, S(stream));
  });
}

int mfs_diagonal(mfs_problem *p, int level, double *dst, void *stream) {
  return guard([&] {
    check_level(p, level);
    MFS_REQUIRE(dst != nullptr, MFS_EINVAL, "NULL vector");
    hipStream_t s = S(stream);
    if (p->amr) {
      MFS_REQUIRE(p->amr->mg, MFS_EUNSUPPORTED, "problem was set up without multigrid levels");
      MFS_REQUIRE(p->amr->ready, MFS_EINVAL, "mfs_set_linearization has not been called");
      if (level < p->namr) {
        AmrLevel &V = p->amr->lev[level];
        vec_copy<double>(dst, V.diag, 4 * V.N, s);
        return;
      }
      level -= p->namr;
    }
    if (p->hp && level < p->nhp) {
      vec_copy<double>(dst, p->hp->lev[level].diag, p->hp->lev[level].V.N, s);
      return;
    }
    if (p->hp) level -= p->nhp;
    const Level &L = p->L[level];
    if (p->ns) {
      MFS_REQUIRE(p->ns_ready, MFS_EINVAL, "mfs_set_linearization has not been called");
      ns_diagonal(*p, level, dst, s);
      return;
    }
    vec_fill<double>(dst, 0.0, L.g.Nv, s);
    launch_laplace_diagonal(L.g, L.X64, L.tab64, p->nu, dst, s);
    // Dirichlet rows: 1 (identity rows of the constrained operator)
    launch_reciprocal_boundary_one(L.g, dst, s);
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

int mfs_vcycle(mfs_problem *p, int prec, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(p->opts.mg_levels, MFS_EINVAL, "problem was set up without multigrid levels");
    MFS_REQUIRE(dst && src && dst != src, MFS_EINVAL, "bad vectors");
    MFS_REQUIRE(!p->ns || (p->ns_ready && p->ns_mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    MFS_REQUIRE(!p->amr || (p->amr->ready && p->amr->mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    if (p->amr) {
      if (prec == MFS_FP64)
        amr_vcycle<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
      else
        amr_vcycle<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
    } else if (p->hp) {
      if (prec == MFS_FP64)
        hp_vcycle<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
      else
        hp_vcycle<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
    } else if (p->ns) {
      if (prec == MFS_FP64)
        ns_vcycle<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
      else
        ns_vcycle<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
    } else if (prec == MFS_FP64)
      vcycle_level<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
    else
      vcycle_level<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
  });
}

int mfs_prolongate_add(mfs_problem *p, int prec, int fine, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_level(p, fine);
    check_prec(prec);
    MFS_REQUIRE(fine + 1 < p->namr + p->nhp + p->nlev, MFS_EINVAL, "no coarser level below %d", fine);
    if (p->amr) {
      if (fine < p->namr) {
        if (prec == MFS_FP64)
          amr_prolongate_add<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
        else
          amr_prolongate_add<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
        return;
      }
      fine -= p->namr;
    }
    if (fine < p->nhp) {
      if (prec == MFS_FP64)
        hp_prolongate_add<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
      else
        hp_prolongate_add<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
      return;
    }
    fine -= p->nhp;
    const Level &F = p->L[fine], &C = p->L[fine + 1];
    const int ncp = p->ns ? 1 : 0;
    if (prec == MFS_FP64)
      launch_prolongate_add<double>(F.g, C.g, F.h_to_coarser, F.emb.data(), (double *)dst, (const double *)src,
                                    S(stream), ncp);
    else
      launch_prolongate_add<float>(F.g, C.g, F.h_to_coarser, F.emb.data(), (float *)dst, (const float *)src,
                                   S(stream), ncp);
  });
}

int mfs_restrict(mfs_problem *p, int prec, int fine, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_level(p, fine);
    check_prec(prec);
    MFS_REQUIRE(fine + 1 < p->namr + p->nhp + p->nlev, MFS_EINVAL, "no coarser level below %d", fine);
    if (p->amr) {
      if (fine < p->namr) {
        if (prec == MFS_FP64)
          amr_restrict<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
        else
          amr_restrict<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
        return;
      }
      fine -= p->namr;
    }
    if (fine < p->nhp) {
      if (prec == MFS_FP64)
        hp_restrict<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
      else
        hp_restrict<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
      return;
    }
    fine -= p->nhp;
    const Level &F = p->L[fine], &C = p->L[fine + 1];
    const int ncp = p->ns ? 1 : 0;
    if (prec == MFS_FP64)
      launch_restrict<double>(F.g, C.g, F.h_to_coarser, F.emb.data(), (double *)dst, (const double *)src, S(stream),
                              ncp, F.rs64);
    else
      launch_restrict<float>(F.g, C.g, F.h_to_coarser, F.emb.data(), (float *)dst, (const float *)src, S(stream),
                             ncp, F.rs32);
  });
}

int mfs_precondition(mfs_problem *p, int prec, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(p->opts.mg_levels && (p->hp || p->L[0].g.Np > 0), MFS_EINVAL,
                "needs multigrid levels and a pressure space");
    MFS_REQUIRE(dst && src && dst != src, MFS_EINVAL, "bad vectors");
    MFS_REQUIRE(!p->ns || (p->ns_ready && p->ns_mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    MFS_REQUIRE(!p->amr || (p->amr->ready && p->amr->mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    if (prec == MFS_FP64)
      precondition_any<double>(*p, (double *)dst, (const double *)src, S(stream));
    else
      precondition_any<float>(*p, (float *)dst, (const float *)src, S(stream));
  });
}

int mfs_rhs(mfs_problem *p, const double *f_qp, const double *u_dirichlet, double *b, void *stream) {
  return guard([&] {
    no_amr(p, "mfs_rhs");
    check_problem(p);
    MFS_REQUIRE(f_qp && u_dirichlet && b, MFS_EINVAL, "NULL vector");
    MFS_REQUIRE(!p->ns, MFS_EUNSUPPORTED, "mfs_rhs assembles the Stokes right-hand side only");
    MFS_REQUIRE(!p->hp, MFS_EUNSUPPORTED, "mfs_rhs is not provided for hp problems");
    const Level &L = p->L[0];
    const LevelGeom &g = L.g;
    MFS_REQUIRE(g.Np > 0, MFS_EINVAL, "needs a pressure space");
    hipStream_t s = S(stream);
    const int64_t nu = p->dim * g.Nv, n = nu + g.Np;
    double *t = p->tmp_full;
    // t = K_unconstrained * lifting, free velocity rows and all pressure rows
    launch_fill_dirichlet<double>(g, t, (const double *)nullptr, s);
    vec_fill<double>(t + nu, 0.0, g.Np, s);
    launch_cell_op<double>(g, dev<double>(L), M_LAPLACE | M_DIVU, p->nu, t, t + nu, u_dirichlet, nullptr, s, true);
    // b = (f, phi) - t on free rows; u_D on Dirichlet rows; -t on pressure rows
    launch_fill_dirichlet<double>(g, b, u_dirichlet, s);
    vec_fill<double>(b + nu, 0.0, g.Np, s);
    launch_load_vector(g, L.X64, L.tab64, f_qp, b, s);
    vec_axpby<double>(b, -1.0, t, 1.0, n, s);
    (void)n;
  });
}

int mfs_solve_begin(mfs_problem *p, const double *b, double *x, const mfs_options *opts, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(b && x && (const void *)b != (void *)x, MFS_EINVAL, "bad vectors");
    mfs_options o = opts ? *opts : p->opts;
    MFS_REQUIRE(o.rtol > 0 && o.maxit >= 1, MFS_EINVAL, "bad rtol / maxit");
    check_prec(o.precond_precision);
    kr_begin(*p, b, x, o, S(stream));
  });
}

int mfs_solve_advance(mfs_problem *p, int *done, mfs_solve_info *info) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(done != nullptr, MFS_EINVAL, "done is NULL");
    Krylov &K = p->kr;
    *done = 0;
    if (K.state == 4) {
      *done = 1;
      if (info) *info = K.info;
      return;
    }
    MFS_REQUIRE(K.state != 0, MFS_EINVAL, "no solve in progress");
    const hipError_t q = hipEventQuery(K.ev);
    if (q == hipErrorNotReady) return;
    MFS_HIP(q);
    kr_process(*p);
    if (K.state == 4) {
      *done = 1;
      if (info) *info = K.info;
    }
  });
}

int mfs_batch_step(mfs_problem **ps, int n, void *stream, int *done, mfs_solve_info *infos) {
  return guard([&] {
    MFS_REQUIRE(n >= 0 && (n == 0 || (ps != nullptr && done != nullptr)), MFS_EINVAL, "bad problem list");
    for (int i = 0; i < n; ++i) {
      MFS_REQUIRE(ps[i] != nullptr, MFS_EINVAL, "problem %d is NULL", i);
      for (int j = 0; j < i; ++j) MFS_REQUIRE(ps[j] != ps[i], MFS_EINVAL, "problem %d is listed twice", i);
    }
    std::vector<mfs_problem *> group;
    for (int i = 0; i < n; ++i) {
      mfs_problem &P = *ps[i];
      Krylov &K = P.kr;
      done[i] = 0;
      if (K.state != 4) {
        MFS_REQUIRE(K.state != 0, MFS_EINVAL, "problem %d has no solve in progress", i);
        const hipError_t q = hipEventQuery(K.ev);
        if (q == hipErrorNotReady) continue;
        MFS_HIP(q);
        const bool step = kr_process(P, true);
        if (step) {
          if (q2_groupable(P))
            group.push_back(&P);
          else
            kr_enqueue_step(P, K.s);
        }
      }
      if (K.state == 4) {
        done[i] = 1;
        if (infos) infos[i] = K.info;
      }
    }
    if (group.size() == 1) {
      kr_enqueue_step(*group[0], group[0]->kr.s);
      return;
    }
    if (group.empty()) return;
    // preconditioners on the problems' streams, one grouped system operator
    // on `stream`, Gram-Schmidt and readbacks on the problems' streams again
    hipStream_t gs = S(stream);
    std::vector<Q2Problem<double>> q(group.size());
    for (size_t i = 0; i < group.size(); ++i) {
      mfs_problem &P = *group[i];
      Krylov &K = P.kr;
      kr_step_pre(P, K.s);
      MFS_HIP(hipEventRecord(K.ev_pre, K.s));
      MFS_HIP(hipStreamWaitEvent(gs, K.ev_pre, 0));
      const Level &L = P.L[0];
      q[i] = Q2Problem<double>{L.g, L.X64, P.nu, K.w, K.Z + (int64_t)K.j * K.ld, L.face64};
    }
    launch_stokes_q2_group<double>(q.data(), (int)q.size(), gs);
    hipEvent_t e = nullptr;
    MFS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const hipError_t r = hipEventRecord(e, gs);
    if (r == hipSuccess)
      for (mfs_problem *P : group) {
        MFS_HIP(hipStreamWaitEvent(P->kr.s, e, 0));
        kr_step_post(*P, P->kr.s);
      }
    (void)hipEventDestroy(e);
    MFS_HIP(r);
  });
}

int mfs_solve(mfs_problem *p, const double *b, double *x, const mfs_options *opts, mfs_solve_info *info,
              void *stream) {
  int rc = mfs_solve_begin(p, b, x, opts, stream);
  if (rc != MFS_OK) return rc;
  return guard([&] {
    Krylov &K = p->kr;
    while (K.state != 4) {
      MFS_HIP(hipEventSynchronize(K.ev));
      kr_process(*p);
    }
    if (info) *info = K.info;
    if (K.info.status != MFS_OK) {
      set_error("FGMRES did not reach rtol %.3e within %d iterations (relative residual %.3e)", K.rtol, K.maxit,
                K.info.rel_residual);
      throw mfs::Error{MFS_ENOCONV};
    }
  });
}

int mfs_set_linearization(mfs_problem *p, const double *u0, double dt, int newton, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "linearisation needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(u0 != nullptr, MFS_EINVAL, "u0 is NULL");
    MFS_REQUIRE(dt > 0 && std::isfinite(dt), MFS_EINVAL, "dt must be positive");
    drop_prec_graph(*p);
    if (p->amr)
      amr_set_linearization(*p, u0, dt, newton, S(stream));
    else
      ns_set_linearization(*p, u0, dt, newton, S(stream));
  });
}

}  // extern "C"
