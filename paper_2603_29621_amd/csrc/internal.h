// Internal declarations of the mfstokes HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mfstokes.h"

namespace mfs {

// ----------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
const char *get_error();

struct Error {
  int code;
};

#define MFS_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      ::mfs::set_error("HIP error %s at %s:%d: %s", hipGetErrorName(e_), __FILE__, __LINE__, \
                       hipGetErrorString(e_));                                                 \
      throw ::mfs::Error{MFS_EHIP};                                                            \
    }                                                                                          \
  } while (0)

#define MFS_REQUIRE(cond, code, ...)    \
  do {                                  \
    if (!(cond)) {                      \
      ::mfs::set_error(__VA_ARGS__);    \
      throw ::mfs::Error{code};         \
    }                                   \
  } while (0)

// ----------------------------------------------------------------- 1D tables
// Layout of the per-level table array (same layout in FP64 and FP32).
// Every block is MAXQ x MAXQ, row-major [point][node].
constexpr int MAXQ = 8;  // degree <= 7
constexpr int TAB_S = 0;                // velocity basis values at Gauss points  [q][k+1]
constexpr int TAB_D = 1 * MAXQ * MAXQ;  // collocation derivative on Gauss points [q][q]
constexpr int TAB_DS = 2 * MAXQ * MAXQ; // velocity basis derivatives at Gauss points [q][k+1]
constexpr int TAB_SP = 3 * MAXQ * MAXQ; // pressure basis values at Gauss points  [q][kp+1]
constexpr int TAB_DSP = 4 * MAXQ * MAXQ;// pressure basis derivatives at Gauss points [q][kp+1]
constexpr int TAB_W = 5 * MAXQ * MAXQ;  // Gauss weights [q]
constexpr int TAB_X = TAB_W + MAXQ;     // Gauss points [q]
constexpr int TAB_SIZE = TAB_X + MAXQ;

// host computation of the tables (tables.cpp)
std::vector<double> gll_nodes(int k);
void gauss_rule(int q, std::vector<double> &x, std::vector<double> &w);
// V[i*n + j] = phi_j(x_i) for the Lagrange basis of `nodes`
std::vector<double> lagrange_values(const std::vector<double> &nodes, const std::vector<double> &x);
std::vector<double> lagrange_derivs(const std::vector<double> &nodes, const std::vector<double> &x);
std::vector<double> make_tables(int k, int kp);
// 1D prolongation matrix [fine points][coarse nodes]: h-embedding (2k+1 x k+1)
// or p-embedding (kf+1 x kc+1)
std::vector<double> h_embedding(int k);
std::vector<double> p_embedding(int kf, int kc);

// ----------------------------------------------------------------- levels
struct LevelGeom {
  int dim;
  int n[3];        // cells per direction (1 in unused directions)
  int k, kp;       // velocity / pressure degree (kp = 0: no pressure space)
  int nv[3], np[3];
  int64_t Nv, Np, ncells;
  int cart;        // 1: every cell an axis-aligned box (the Navier-Stokes kernels use it)
};

template <typename T>
struct DevLevel {
  const T *X = nullptr;    // vertices [(n0+1)(n1+1)(n2+1)][dim]
  const T *tab = nullptr;  // 1D tables (TAB_*)
  const T *invdiag = nullptr;  // inverse diagonal of A, one component [Nv]
};

// Slot of a cell-local result (3D): node (lx, ly, lz) of component comp of cell
// (cx, cy, cz), q nodes per direction, ncomp components.  For each cell row
// (cy, cz), component and node row (ly, lz) the slots of all cells along x lie
// side by side, q each, so a node gather that reads x-consecutive nodes reads
// consecutive slots, and the cells of a workgroup (consecutive in x) write
// whole lines.
__host__ __device__ __forceinline__ int64_t cell_slot(int n0, int n1, int ncomp, int q, int cx, int cy, int cz,
                                                      int comp, int lx, int ly, int lz) {
  return (((((int64_t)cz * n1 + cy) * ncomp + comp) * q + lz) * q + ly) * ((int64_t)n0 * q) + (int64_t)cx * q + lx;
}

// ----------------------------------------------------------------- kernels
enum CellMode : int {
  M_LAPLACE = 1,  // velocity: nu (grad u, grad v)
  M_GRADP = 2,    // velocity rows: -(p, div v)
  M_DIVU = 4,     // pressure rows: -(div u, q)
  M_MASSP = 8,    // pressure rows: (p, q)
  M_MASSU = 16,   // velocity: (u, v) per component (a mode of its own)
};

template <typename T>
void launch_cell_op(const LevelGeom &g, const DevLevel<T> &d, int mode, T nu, T *dst_u, T *dst_p,
                    const T *src_u, const T *src_p, hipStream_t s, bool src_all = false);  // src_all: lifting (Dirichlet nodes only)
// node gather of cell-local results on a 3D structured grid: velocity
// [cell][3][(k+1)^3] into the degree-k grid (Dirichlet rows = dir_src, 0 when
// null), pressure [cell][(kp+1)^3] into the degree-kp grid; fixed order
template <typename T>
void launch_node_gather(const LevelGeom &g, int k, int kp, T *ev_u, T *ev_p, T *dst_u, T *dst_p, const T *dir_src,
                        hipStream_t s);
// generic cell operator (3D, degree >= 3) with cell-local outputs and a
// deterministic node gather instead of atomic additions: every row of dst_u
// (Dirichlet rows = dir_src, 0 when null) and of dst_p is written; `ev` is a
// scratch buffer of cell_ev_elems(g) elements
int64_t cell_ev_elems(const LevelGeom &g);
// 3D Taylor-Hood Stokes cell work of degree 3 or 4 with one thread per point
// column (modes M_LAPLACE | M_GRADP | M_DIVU, M_LAPLACE (also on levels
// without a pressure space), M_GRADP, M_DIVU, M_MASSP) into the cell-local
// arrays of the node gather; false when the level or mode is not covered (the
// caller uses the generic kernel)
template <typename T>
bool launch_column_cells(const LevelGeom &g, const T *X, int mode, T nu, const T *src_u, const T *src_p, T *ev_u,
                         T *ev_p, hipStream_t s);
template <typename T>
void launch_cell_op_gather(const LevelGeom &g, const DevLevel<T> &d, int mode, T nu, T *dst_u, T *dst_p,
                           const T *src_u, const T *src_p, const T *dir_src, T *ev, hipStream_t s);
// Chebyshev step on a gather level (3D, k >= 3): A x into the cell-local
// arrays, then the node gather fused with the update of the free rows:
// r = inv (b - A x), d = c2 r (first) or c1 d + c2 r, x += d; Dirichlet rows
// of x and d unchanged
template <typename T>
void launch_cell_cheb_gather(const LevelGeom &g, const DevLevel<T> &dv, T nu, T *x, T *d, const T *b, const T *inv,
                             T c1, T c2, bool first, T *ev, hipStream_t s);
// specialised 3D degree-2 kernel, writing every entry of its velocity output
// itself: Q2_STOKES (Stokes Q2/Q1: dst_u = A src_u + B src_p, dst_p = B^T
// src_u; Dirichlet rows dst_u = src_u), Q2_A (dst_u = A src_u, Dirichlet rows
// = src_u), Q2_B (dst_u = B src_p, Dirichlet rows 0; src_u and dst_p unused),
// Q2_MASSP (dst_p = M_p src_p; velocity arguments unused);
// `face` is a scratch buffer of q2_face_elems(g) elements.  Returns false when
// the level does not qualify.
constexpr int Q2_A = 0, Q2_STOKES = 1, Q2_B = 2, Q2_MASSP = 3;
int64_t q2_face_elems(const LevelGeom &g);
template <typename T>
bool launch_stokes_q2(const LevelGeom &g, const T *X, int mode, T nu, T *dst_u, T *dst_p, const T *src_u,
                      const T *src_p, T *face, hipStream_t s);
// One grouped launch (brick kernel, then combine) of the Q2_STOKES operator
// for several problems: dst = K src for each (full vectors).  Up to 16
// problems per launch pair; more are split into further pairs.
template <typename T>
struct Q2Problem {
  LevelGeom g;
  const T *X;
  T nu;
  T *dst;
  const T *src;
  T *face;
};
template <typename T>
void launch_stokes_q2_group(const Q2Problem<T> *probs, int n, hipStream_t s);
// Q2_A with one Chebyshev step fused into its output phase: on every
// non-Dirichlet row, r = inv (b - A x), d = c2 r (first) or c1 d + c2 r,
// x += d; Dirichlet rows of x and d are left alone.  x is updated in place:
// brick-interior nodes by the cell kernel (no other brick reads them, and its
// own brick has them in LDS), brick-face nodes by the combine kernel.  The
// same arithmetic as A followed by cheb_update.
template <typename T>
bool launch_q2_cheb(const LevelGeom &g, const T *X, T nu, T *x, T *d, const T *b, const T *inv, T c1, T c2,
                    bool first, T *face, hipStream_t s);
// specialised 3D degree-1 kernel for the velocity block: dst = A src
// (Dirichlet rows = src); `face` is a scratch buffer of q1_face_elems(g)
// elements.  Returns false when the level does not qualify.
int64_t q1_face_elems(const LevelGeom &g);
template <typename T>
bool launch_laplace_q1(const LevelGeom &g, const T *X, T nu, T *dst, const T *src, T *face, hipStream_t s);
// the same with one Chebyshev step fused into the output (as launch_q2_cheb)
template <typename T>
bool launch_q1_cheb(const LevelGeom &g, const T *X, T nu, T *x, T *d, const T *b, const T *inv, T c1, T c2,
                    bool first, T *face, hipStream_t s);
// diagonal of the scalar Laplacian block (FP64): diag[Nv]
void launch_laplace_diagonal(const LevelGeom &g, const double *X, const double *tab, double nu, double *diag,
                             hipStream_t s);
// diag(M_p) (FP64), pressure degree g.kp in {k-1, k}
void launch_mass_diagonal(const LevelGeom &g, const double *X, const double *tab, double *diag, hipStream_t s);
// r64 = 1/d, r32 = (float)(1/d)
void launch_reciprocal(double *r64, float *r32, const double *d, int64_t n, hipStream_t s);

// additive Schwarz relaxation on the vertex patches of a structured
// equal-order level (degrees 1, 2): patch size, count, colours; column j of
// every patch matrix of a colour by probing (set unit entries, apply J,
// extract, reset); batched in-place inversion (status |= 1 on a zero pivot);
// x += omega W A_P^{-1} (b - t) over the patches of one colour
int asm_patch_size(const LevelGeom &g);
int64_t asm_patch_count(const LevelGeom &g);
int asm_colours(const LevelGeom &g);
void launch_asm_probe_set(const LevelGeom &g, double *x, int colour, int j, double value, hipStream_t s);
void launch_asm_probe_extract(const LevelGeom &g, const double *y, double *M, int colour, int j, hipStream_t s);
void launch_asm_invert(const LevelGeom &g, double *M, int *status, hipStream_t s);
template <typename T>
void launch_asm_apply(const LevelGeom &g, const T *M, int colour, const T *b, const T *t, T *x, T omega,
                      hipStream_t s);
// d[i] = 1 on Dirichlet rows of a scalar velocity-node vector
void launch_reciprocal_boundary_one(const LevelGeom &g, double *d, hipStream_t s);
// det J > 0 check: writes the smallest det J * (cells) and the first bad cell
void launch_check_geometry(const LevelGeom &g, const double *X, const double *tab, int *bad_cell,
                           hipStream_t s);
// Gauss point coordinates [ncells][q^dim][dim]
void launch_quadrature_points(const LevelGeom &g, const double *X, const double *tab, double *out,
                              hipStream_t s);
// load vector (f, phi_i) on velocity rows, f at Gauss points
void launch_load_vector(const LevelGeom &g, const double *X, const double *tab, const double *f_qp,
                        double *b_u, hipStream_t s);

// Dirichlet fill: dst[c*Nv + i] = boundary(i) ? (src ? src[c*Nv+i] : 0) : 0 for c < dim
template <typename T>
void launch_fill_dirichlet(const LevelGeom &g, T *dst_u, const T *src_u, hipStream_t s);

// transfers between a fine level and the next coarser one
// emb_host: host 1D embedding [F+1][kc+1] (h_embedding / p_embedding);
// vectors: `ncu` constrained velocity components (default: dim), then `ncp`
// unconstrained components (1: the equal-order pressure; ncu = 0, ncp = 1 on
// the geometries of a pressure grid: a pressure of its own degree)
template <typename T>
void launch_prolongate_add(const LevelGeom &fine, const LevelGeom &coarse, bool h_transfer, const double *emb_host,
                           T *dst_fine, const T *src_coarse, hipStream_t s, int ncp = 0, int ncu = -1);
// work: scratch of restrict_work_elems(fine, coarse, dim + ncp) elements for
// the three-pass form (nullptr: one-pass gather)
template <typename T>
void launch_restrict(const LevelGeom &fine, const LevelGeom &coarse, bool h_transfer, const double *emb_host,
                     T *dst_coarse, const T *src_fine, hipStream_t s, int ncp = 0, T *work = nullptr, int ncu = -1);
int64_t restrict_work_elems(const LevelGeom &fine, const LevelGeom &coarse, int ncomp);

// ----------------------------------------------------------------- Navier-Stokes (ns_kernels.hip)
// per-quadrature-point linearisation data: u0 (3), grad u0 (9), R(u0, p0) (3),
// delta_1 (1), the residual's Galerkin value term alpha (u0 - u~) + u0.grad u0
// (3) and p0 (1), stored [cell][field][point]
constexpr int NS_QD = 20;
inline int64_t ns_qd_elems(const LevelGeom &g) {
  int64_t nq = 1;
  for (int a = 0; a < g.dim; ++a) nq *= g.k + 1;
  return g.ncells * nq * NS_QD;
}
// A general linearisation state (what = 0): src holds [u0 (dim Nv) | p0 (Nv) |
// u~ (dim Nv)] (structured grid) or evin slot 3 holds p0 and evhist slots
// 0..2 hold u~ (cell-local inputs); keep_delta leaves delta_1 as stored.
template <typename T>
struct NsPoint {
  int keep_delta = 0;
  const T *evhist = nullptr;
};
// what = 0: qd = linearisation data of the nodal velocity src (dim*Nv), or of
// the general state of `pt`;
// what = 2: dst += the nonlinear residual at the stored state (src unused;
// the same outputs as what = 1);
// what = 1: dst += J src on the free velocity rows and all pressure rows
// (src, dst full equal-order vectors; the Dirichlet rows of dst untouched);
// with ev (3D, ncells * 4 * (k+1)^3 elements) the cell results are written
// there instead ([cell][3][(k+1)^3] velocity, then [cell][(k+1)^3] pressure)
// and dst is not touched; with evin (3D) the cell inputs come from there and
// the cell corners from Xcell ([cell][8][3]) instead of src and the node grid
// (refined meshes), and evin and ev hold [cell][(k+1)^3][4] (velocity
// components and pressure of a node side by side)
template <typename T>
void launch_ns(const LevelGeom &g, const T *X, const T *tab, int what, T nu, T dt, int newton, const T *src, T *dst,
               T *qd, hipStream_t s, T *ev = nullptr, const T *evin = nullptr, const T *Xcell = nullptr,
               const NsPoint<T> *pt = nullptr);
// coarse fields = fine fields at the shared nodes (fine index 2 * coarse
// index per direction; h-coarsening at k <= 2 and p-coarsening 2 -> 1), for
// ncomp blocked components (dim when ncomp <= 0)
void launch_ns_inject(const LevelGeom &fine, const LevelGeom &coarse, const double *u_fine, double *u_coarse,
                      hipStream_t s, int ncomp = 0);
// node colouring by (i mod q, j mod q, l mod q): with q = k+1 no two nodes of
// a colour share a cell.  indicator: out = 1 on component `comp` at the nodes
// of `color`, 0 elsewhere (ncomp*Nv entries); extract: diag[comp*Nv + i] =
// y[comp*Nv + i] at those nodes.
void launch_color_indicator(const LevelGeom &g, int ncomp, int q, int color, int comp, double *out, hipStream_t s);
void launch_color_extract(const LevelGeom &g, int q, int color, int comp, const double *y, double *diag,
                          hipStream_t s);
// damped Jacobi sweep: x += omega * invdiag * (b - t)
template <typename T>
void jacobi_relax(T *x, const T *b, const T *t, const T *invdiag, T omega, int64_t n, hipStream_t s);

// vector kernels (vector_kernels.hip)
// stage mixing of stage-major vectors (space-time operators, Sec. 4):
// y_i = a y_i + sum_j C[i][j] x_j over the first ne entries of each stage,
// y_i = a y_i over entries ne .. ny-1 (i < no, j < ni <= MFS_MAX_STAGES;
// a = 0 overwrites y)
constexpr int MFS_MAX_STAGES = 8;
struct StageCoef {
  double c[MFS_MAX_STAGES * MFS_MAX_STAGES];
};
template <typename T>
void stage_mix(T *y, int64_t ldy, int no, const T *x, int64_t ldx, int ni, const StageCoef &C, T a, int64_t ne,
               int64_t ny, hipStream_t s);

// space-time vertex patches of a Taylor-Hood level (asm_kernels.hip): probing
// of the spatial patch matrices (Stokes operator, and the velocity mass with
// nvel = dim Nv rows), the space-time patch inverses G (x) M_s + tau I (x) A_s,
// and the additive update of one colour on stage-major vectors
int th_patch_size(const LevelGeom &g);
void launch_th_probe_set(const LevelGeom &g, double *x, int colour, int j, hipStream_t s);
void launch_th_probe_extract(const LevelGeom &g, const double *y, int64_t nvel, double *M, int colour, int j,
                             hipStream_t s);
void launch_th_form_invert(const LevelGeom &g, int Q, const StageCoef &G, double tau, const double *As,
                           const double *Ms, double *Kinv, int *status, hipStream_t s);
template <typename T>
void launch_th_apply(const LevelGeom &g, int Q, int64_t N, const T *Kinv, int colour, const T *b, const T *t, T *x,
                     T omega, hipStream_t s);
template <typename T>
void vec_fill(T *x, T v, int64_t n, hipStream_t s);
template <typename T>
void vec_copy(T *y, const T *x, int64_t n, hipStream_t s);
template <typename T>
void vec_axpby(T *y, T a, const T *x, T b, int64_t n, hipStream_t s);  // y = a x + b y
template <typename TO, typename TI>
void vec_cast(TO *y, const TI *x, int64_t n, hipStream_t s);
template <typename T>
void vec_zero_mask_boundary(const LevelGeom &g, T *u, hipStream_t s);  // zero Dirichlet rows
template <typename T>
void vec_copy_boundary(const LevelGeom &g, T *u, const T *src, hipStream_t s);  // Dirichlet rows of u = src
// y *= invdiag (per component); Dirichlet rows forced to 0
template <typename T>
void vec_diag_scale(const LevelGeom &g, T *y, const T *invdiag, const T *x, hipStream_t s);
// inverse diagonal with 1 on Dirichlet rows
void vec_invert_diag(const LevelGeom &g, const double *diag, double *invdiag64, float *invdiag32, hipStream_t s);
// Chebyshev step on level vectors (velocity, dim*Nv):
// the first step from x = 0 with the Dirichlet values of b: x = b on the
// Dirichlet rows, d = x = c2 * invdiag * b elsewhere
template <typename T>
void cheb_start(const LevelGeom &g, T *x, T *d, const T *b, const T *invdiag, T c2, hipStream_t s);
//   r = invdiag * (b - Ax) ; d = c1 * d + c2 * r ; x += d   (Dirichlet rows untouched)
template <typename T>
void cheb_update(const LevelGeom &g, T *x, T *d, const T *b, const T *Ax, const T *invdiag, T c1, T c2,
                 bool first, hipStream_t s);
// multiple dot products: out[i] = <V_i, w> for i < m, V_i = V + i*ld (FP64 accumulate)
template <typename T>
void multi_dot(const T *V, int64_t ld, int m, const T *w, int64_t n, double *out, double *partials,
               hipStream_t s);
// w -= sum_i h[i] V_i  (h on device)
template <typename T>
void multi_axpy(T *w, const T *V, int64_t ld, int m, const double *h, int64_t n, hipStream_t s);
// one pass over V: w -= sum_{i<m} h[i] V_i, then out[i] = <V_i, w> for i < md
// (md is 0 or m) and, when norm, out[md] = <w, w>, over the updated w
template <typename T>
void axpy_dot(T *w, const T *V, int64_t ld, int m, const double *h, int md, bool norm, int64_t n, double *out,
              double *partials, hipStream_t s);
// y = sum_i h[i] V_i (+ y if accumulate)
template <typename T>
void multi_combine(T *y, const T *V, int64_t ld, int m, const double *h, int64_t n, bool accumulate,
                   hipStream_t s);
// dense coarse solve: out = Ainv * in (FP64 matrix), with casts
template <typename T>
void dense_apply(const double *Ainv, int n, const T *in, T *out, hipStream_t s);
// PCG steps with device-resident scalars (no host round trip):
//   alpha = rho/pq ; z += alpha p ; res -= alpha q ; s = dinv * res
template <typename T>
void pcg_update1(T *z, T *res, T *sv, const T *p, const T *q, const T *dinv, int64_t n, const double *rho,
                 const double *pq, hipStream_t s);
//   beta = rho_new / rho_old ; p = s + beta p
template <typename T>
void pcg_update2(T *p, const T *sv, int64_t n, const double *rho_new, const double *rho_old, hipStream_t s);
// y = x / sqrt(*nrm2)
template <typename T>
void scale_inv_sqrt(T *y, const T *x, int64_t n, const double *nrm2, hipStream_t s);
// y = a .* x elementwise
template <typename T>
void vec_mul(T *y, const T *a, const T *x, int64_t n, hipStream_t s);
// p -= (*num / *den) * one_vector   (pressure mean shift)
void shift_mean(double *p, int64_t n, const double *num, const double *den, hipStream_t s);

constexpr int DOT_BLOCKS = 2048;

}  // namespace mfs
