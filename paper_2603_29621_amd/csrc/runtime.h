// Host runtime of the mfstokes library, shared by its parts: the problem record
// with its level, Krylov, hp and refined-mesh data, the accessors that pick the
// FP64 or FP32 copy of a level's data, and the functions each part provides to
// the others (one translation unit per part: set-up, Stokes, Navier-Stokes, hp,
// refined meshes, Krylov and space-time).  Internal to the library.
#pragma once

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


namespace mfs {
namespace rt {

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
inline int64_t kr_ld(int64_t n) {
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

}  // namespace rt
}  // namespace mfs

using namespace mfs;
using namespace mfs::rt;

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

namespace mfs {
namespace rt {

constexpr int PCG_MAX = 64;  // scalar slots per PCG run (rho[i], pq[i])

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
DevLevel<T> dev(const Level &L);

template <>
inline DevLevel<double> dev<double>(const Level &L) {
  DevLevel<double> d;
  d.X = L.X64;
  d.tab = L.tab64;
  d.invdiag = L.invdiag64;
  return d;
}

template <>
inline DevLevel<float> dev<float>(const Level &L) {
  DevLevel<float> d;
  d.X = L.X32;
  d.tab = L.tab32;
  d.invdiag = L.invdiag32;
  return d;
}

template <typename T>
T *face(const Level &L);

template <>
inline double *face<double>(const Level &L) {
  return L.face64;
}

template <>
inline float *face<float>(const Level &L) {
  return L.face32;
}

template <typename T>
T *cellev(const Level &L);

template <>
inline double *cellev<double>(const Level &L) {
  return L.ev64;
}

template <>
inline float *cellev<float>(const Level &L) {
  return L.ev32;
}

// Generic kernel with cell-local outputs and a node gather instead of global
// atomics, on every 3D level of degree >= 3 (measured at 64^3 against the
// atomics launched one cell colour at a time: Q4/Q3 FP64 1.93 ms against
// 2.21 ms, once the cell-local rows were laid out for the gather).
template <typename T>
inline bool use_gather(const Level &L) {
  return cell_ev_elems(L.g) > 0;
}

template <typename T>
PrecWork<T> &work(mfs_problem &P);

template <>
inline PrecWork<double> &work<double>(mfs_problem &P) {
  return P.w64;
}

template <>
inline PrecWork<float> &work<float>(mfs_problem &P) {
  return P.w32;
}

template <typename T>
T *rwork(const Level &L);

template <>
inline double *rwork<double>(const Level &L) {
  return L.rs64;
}

template <>
inline float *rwork<float>(const Level &L) {
  return L.rs32;
}

template <typename T>
const T *invdiag(const Level &L);

template <>
inline const double *invdiag<double>(const Level &L) {
  return L.invdiag64;
}

template <>
inline const float *invdiag<float>(const Level &L) {
  return L.invdiag32;
}

// ---------------------------------------------------------------- operators
// velocity-block A on level l: dst = A src (dim*Nv); Dirichlet rows dst = src
inline bool use_specialised() {
  static const bool off = std::getenv("MFS_GENERIC_KERNELS") != nullptr;
  return !off;
}

template <typename T>
const T *ns_qd(const Level &L);

template <>
inline const double *ns_qd<double>(const Level &L) {
  return L.qd64;
}

template <>
inline const float *ns_qd<float>(const Level &L) {
  return L.qd32;
}

template <typename T>
const T *ns_invdiag(const Level &L);

template <>
inline const double *ns_invdiag<double>(const Level &L) {
  return L.nsinv64;
}

template <>
inline const float *ns_invdiag<float>(const Level &L) {
  return L.nsinv32;
}

// ---------------------------------------------------------------- hp operators
// Cell operators through E-vectors: gather the cells' local values through
// the local->global maps, apply the cell kernels class by class, scatter the
// local results back with the transposed maps (Sec. 3, minimum rule).
template <typename T>
HpVecs<T> &hpv(HpLevel &L);

template <>
inline HpVecs<double> &hpv<double>(HpLevel &L) {
  return L.v64;
}

template <>
inline HpVecs<float> &hpv<float>(HpLevel &L) {
  return L.v32;
}

template <typename T>
T *hp_tab(HpData &H, int k);

template <>
inline double *hp_tab<double>(HpData &H, int k) {
  return H.tab64[k];
}

template <>
inline float *hp_tab<float>(HpData &H, int k) {
  return H.tab32[k];
}

template <typename T>
T *hp_evp(HpData &H, bool out);

template <>
inline double *hp_evp<double>(HpData &H, bool out) {
  return out ? H.evp_out64 : H.evp_in64;
}

template <>
inline float *hp_evp<float>(HpData &H, bool out) {
  return out ? H.evp_out32 : H.evp_in32;
}

template <typename T>
HpVecs<T> &hp0(mfs_problem &P) {
  return hpv<T>(P.hp->lev[0]);
}

template <typename T>
T **hp_pvec(HpData &H);

template <>
inline double **hp_pvec<double>(HpData &H) {
  return H.p64;
}

template <>
inline float **hp_pvec<float>(HpData &H) {
  return H.p32;
}

template <typename T>
PrecWork<T> &prec_work(mfs_problem &P);

template <>
inline PrecWork<double> &prec_work<double>(mfs_problem &P) {
  return P.w64;
}

template <>
inline PrecWork<float> &prec_work<float>(mfs_problem &P) {
  return P.w32;
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
inline int amr_nop(const AmrData &A) { return A.mg ? (int)A.lev.size() - 1 : 1; }

// ---------------------------------------------------------------- api_setup.cpp
int64_t ipow(int64_t b, int e);
LevelGeom make_geom(int dim, const int n[3], int k, int kp);
int64_t n_vertices(const LevelGeom &g);
std::vector<LevelGeom> plan_levels_ns(int dim, const int n[3], int k, const mfs_options &o);
std::vector<LevelGeom> plan_levels(int dim, const int n[3], int k, int kp, const mfs_options &o);
template <typename T>
void plan_prec_work(Arena &A, PrecWork<T> &w, const std::vector<LevelGeom> &G, int dim, bool full);
template <typename T>
void plan_ns_work(Arena &A, PrecWork<T> &w, const std::vector<LevelGeom> &G, int dim, bool full);
void plan_arena(Arena &A, mfs_problem &P, const std::vector<LevelGeom> &G);
bool cartesian_grid(const std::vector<double> &X, const LevelGeom &g);
void check_options(const mfs_options &o);
void check_mesh(const mfs_mesh *mesh, int k, const mfs_options &o);
double *pinned_acquire();
hipStream_t capture_stream_acquire();
void release(mfs_problem *P);
void sturm_max_eig(const std::vector<double> &d, const std::vector<double> &e, double &lmax);
uint64_t splitmix64(uint64_t &x);
double estimate_lambda(mfs_problem &P, int l, hipStream_t s);
void setup_coarse(mfs_problem &P, hipStream_t s);
int guard(const std::function<void()> &f);
std::vector<LevelGeom> levels_for(const mfs_mesh *mesh, int k, const mfs_options &o);
int setup_structured(const mfs_mesh *mesh, int k, double nu, const mfs_options *opts, void *arena, size_t bytes,
                     void *stream, mfs_problem **out);
void check_problem(const mfs_problem *p);
void check_level(const mfs_problem *p, int level);
void no_amr(const mfs_problem *p, const char *what);
void check_prec(int prec);

// ---------------------------------------------------------------- api_stokes.cpp
template <typename T>
void apply_A(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s);
template <typename T>
void apply_op(mfs_problem &P, int op, int l, T *dst, const T *src, hipStream_t s);
template <typename T>
void chebyshev(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s);
template <typename T>
void vcycle_level(mfs_problem &P, int l, T *x, const T *b, hipStream_t s);
template <typename T>
void precondition(mfs_problem &P, T *y, const T *r, hipStream_t s);

// ---------------------------------------------------------------- api_ns.cpp
template <typename T>
void apply_ns(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s);
void ns_diagonal(mfs_problem &P, int l, double *diag, hipStream_t s);
void ns_setup_coarse(mfs_problem &P, hipStream_t s);
void ns_asm_setup(mfs_problem &P, int l, hipStream_t s);
void ns_mg_data(mfs_problem &P, hipStream_t s);
void ns_set_point(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta, bool mg,
                  hipStream_t s);
void ns_set_linearization(mfs_problem &P, const double *u0, double dt, int newton, hipStream_t s);
void ns_residual(mfs_problem &P, double *F, hipStream_t s);
template <typename T>
void ns_relax(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s);
template <typename T>
void ns_vcycle(mfs_problem &P, int l, T *x, const T *b, hipStream_t s);
void set_point_any(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta, bool mg,
                   hipStream_t s);
void point_mg_any(mfs_problem &P, hipStream_t s);
double device_norm(mfs_problem &P, const double *v, int64_t n, hipStream_t s);
void bdf2_step(mfs_problem &P, const double *u_n, const double *u_nm1, double *x, double dt,
               const mfs_newton_options &o, mfs_newton_info &info, hipStream_t s);

// ---------------------------------------------------------------- api_hp.cpp
template <typename T>
void hp_gather_space(const HpDevSpace &d, int ncomp, const T *x, T *ev, hipStream_t s);
template <typename T>
void hp_scatter_space(const HpDevSpace &d, int ncomp, bool use_dir, const T *ev, const T *src, T *dst, hipStream_t s);
template <typename T>
void hp_apply(mfs_problem &P, int l, int mode, T *dst_u, T *dst_p, const T *src_u, const T *src_p, hipStream_t s);
template <typename T>
void hp_apply_A(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s);
template <typename T>
void hp_prolongate_add(mfs_problem &P, int l, T *xf, const T *xc, hipStream_t s);
template <typename T>
void hp_restrict(mfs_problem &P, int l, T *bc, const T *rf, hipStream_t s);
template <typename T>
void hp_chebyshev(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s);
template <typename T>
void hp_vcycle(mfs_problem &P, int l, T *x, const T *b, hipStream_t s);
template <typename T>
void hp_precondition(mfs_problem &P, T *y, const T *r, hipStream_t s);
void hp_upload(HpData &H, const HpSpaceHost &V, bool constrained, const std::vector<int64_t> &ev_off, bool vector_comp,
               HpDevSpace &d, hipStream_t s);
std::vector<int64_t> ev_offsets(const std::vector<int> &deg, int ncomp, int shift, int64_t *total);
template <typename T>
void hp_alloc_vecs(HpData &H, HpVecs<T> &v, int64_t N, int64_t ev);
double hp_estimate_lambda(mfs_problem &P, int l, hipStream_t s);
void hp_build(mfs_problem &P, const std::vector<int> &deg0, hipStream_t s);
void hp_vmult(mfs_problem &P, int op, int prec, int level, void *dst, const void *src, hipStream_t s);

// ---------------------------------------------------------------- api_refined.cpp
void parallel_tasks(int n, const std::function<void(int)> &f);
void amr_maps_host(const AmrSpaceHost &S, AmrMapsHost &out);
void amr_maps_upload(HpData &H, const AmrSpaceHost &S, const AmrMapsHost &h, AmrMaps &M, hipStream_t s);
void amr_level_upload(AmrData &A, AmrLevel &V, bool op, bool work, hipStream_t s);
void amr_build(mfs_problem &P, const mfs_refined_mesh &m, int k, bool mg, hipStream_t s);
template <typename T>
void amr_apply_ns(mfs_problem &P, int j, T *dst, const T *src, hipStream_t s);
template <typename T>
void amr_prolongate_add(mfs_problem &P, int j, T *xf, const T *xc, hipStream_t s);
template <typename T>
void amr_restrict(mfs_problem &P, int j, T *bc, const T *rf, hipStream_t s);
template <typename T>
void amr_relax(mfs_problem &P, int j, T *x, const T *b, bool zero_start, hipStream_t s);
template <typename T>
void amr_vcycle(mfs_problem &P, int j, T *x, const T *b, hipStream_t s);
void amr_diagonal(mfs_problem &P, int j, double *diag, hipStream_t s);
void amr_set_point(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta,
                   bool mg, hipStream_t s);
void amr_set_linearization(mfs_problem &P, const double *u0, double dt, int newton, hipStream_t s);
void amr_residual(mfs_problem &P, double *F, hipStream_t s);
void amr_vmult(mfs_problem &P, int op, int prec, int level, void *dst, const void *src, hipStream_t s);

// ---------------------------------------------------------------- api_krylov.cpp
void apply_system(mfs_problem &P, double *dst, const double *src, hipStream_t s);
int64_t sys_vel(const mfs_problem &P);
int64_t sys_pres(const mfs_problem &P);
int64_t sys_n(const mfs_problem &P);
template <typename T>
void precondition_any(mfs_problem &P, T *y, const T *r, hipStream_t s);
void drop_prec_graph(mfs_problem &P);
template <typename T>
void precondition_rec(mfs_problem &P, hipStream_t s);
void kr_enqueue_residual(mfs_problem &P, hipStream_t s);
void kr_step_pre(mfs_problem &P, hipStream_t s);
void kr_enqueue_step(mfs_problem &P, hipStream_t s);
void kr_step_post(mfs_problem &P, hipStream_t s);
void kr_enqueue_update(mfs_problem &P, hipStream_t s);
void kr_finish(mfs_problem &P, double rel, int status);
bool kr_process(mfs_problem &P, bool defer = false);
bool q2_groupable(const mfs_problem &P);
void kr_begin(mfs_problem &P, const double *b, double *x, const mfs_options &o, hipStream_t s);

// ---------------------------------------------------------------- api_spacetime.cpp
template <typename T>
void st_apply(mfs_problem &P, int Q, const double *G, double tau, T *dst, const T *src, T *work, hipStream_t s);

}  // namespace rt
}  // namespace mfs
