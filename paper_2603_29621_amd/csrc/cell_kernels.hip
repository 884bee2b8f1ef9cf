// Generic matrix-free cell kernels: Stokes operator, its blocks, the pressure
// mass, the Laplacian diagonal and setup helpers.
//
// One thread per quadrature point, several cells per workgroup.  Values and
// reference gradients at the (k+1)^dim Gauss points come from 1D
// contractions staged through LDS (sum factorisation): interpolation from the
// GLL nodes to the Gauss points direction by direction, then the collocation
// derivative on the Gauss points.  The transposed sequence integrates the
// test-function coefficients back to the nodes.  Cell contributions are added
// to the output vector with hardware atomics; Dirichlet rows are written by a
// separate fill pass (dst = src there) that also clears the other rows.
//
// Weak forms: Sec. 1 eq. (stokes) and the symmetric block matrix of Sec. 3
// eq. (stokes_block): velocity rows nu (grad u, grad v) - (p, div v),
// pressure rows -(div u, q).
#include "cell_common.h"

namespace mfs {

template <typename T>
struct CellArgs {
  int n0, n1, n2, ncells;
  int nv0, nv1, nv2;
  int np0, np1, np2;
  int64_t Nv, Np;
  const T *X;
  const T *tab;
  const T *src_u;
  const T *src_p;
  T *dst_u;
  T *dst_p;
  T nu;
  int src_all;  // 1: read source values on Dirichlet rows only (the lifting of boundary data)
  // cell-local outputs (velocity [cell][dim][(k+1)^dim], pressure
  // [cell][(kp+1)^dim]) instead of atomic additions into dst, when non-null
  T *ev_u, *ev_p;
  // cells of this launch: all ncells (colour < 0), or the cells whose index
  // parities (x, y, z) are the bits of `colour`, cm0 x cm1 x .. of them
  // (nlaunch in total).  No two cells of one colour share a node, so a node
  // receives at most one atomic addition per launch and the colours, launched
  // in a fixed order on one stream, fix the order of the additions: the
  // result is deterministic.
  int colour, cm0, cm1, nlaunch;
};

template <typename T>
__device__ __forceinline__ int launch_cell(const CellArgs<T> &a, int i) {
  if (a.colour < 0) return i;
  const int x = i % a.cm0, r = i / a.cm0, y = r % a.cm1, z = r / a.cm1;
  return (2 * x + (a.colour & 1)) + a.n0 * ((2 * y + ((a.colour >> 1) & 1)) + a.n1 * (2 * z + (a.colour >> 2)));
}

template <int DIM, int K, int KP, typename T, int MODE>
__global__ void __launch_bounds__((Shape<DIM, K, KP>::BLOCK)) cell_kernel(CellArgs<T> a) {
  using Sh = Shape<DIM, K, KP>;
  constexpr int NQ = Sh::NQ, CPB = Sh::CPB, Q = Sh::Q;
  __shared__ T s_tab[TAB_SIZE];
  constexpr int NBUF = DIM * DIM > 3 ? DIM * DIM : 3;  // batched sweeps of DIM fields
  __shared__ T s_buf[NBUF][CPB * NQ];
  __shared__ T s_X[CPB][Sh::NV * DIM];

  const int tid = threadIdx.x;
  for (int i = tid; i < TAB_SIZE; i += Sh::BLOCK) s_tab[i] = a.tab[i];
  CellCtx<DIM, K, KP, T> c;
  int e;
  Sh::map(tid, e, c.t, c.active);
  const int lin = blockIdx.x * CPB + e;
  c.valid = c.active && lin < a.nlaunch;
  const int cell = c.valid ? launch_cell(a, lin) : 0;
  c.qi = c.t % Q;
  c.qj = (c.t / Q) % Q;
  c.ql = DIM == 3 ? c.t / (Q * Q) : 0;
  c.cx = c.cy = c.cz = 0;
  if (c.valid) {
    c.cx = cell % a.n0;
    const int r = cell / a.n0;
    c.cy = r % a.n1;
    c.cz = DIM == 3 ? r / a.n1 : 0;
  }
  c.b0 = &s_buf[0][e * NQ];
  c.b1 = &s_buf[1][e * NQ];
  c.b2 = &s_buf[2][e * NQ];
  c.bb = &s_buf[0][e * NQ];
  c.bstride = CPB * NQ;
  c.tab = s_tab;
  const bool dir = c.valid ? c.vel_dirichlet(a.nv0, a.nv1, a.nv2) : true;
  const int64_t vnode = c.valid ? c.vel_node(a.nv0, a.nv1) : 0;
  constexpr bool MASSU = (MODE & M_MASSU) != 0;
  static_assert(!MASSU || MODE == M_MASSU, "the velocity mass is a mode of its own");
  constexpr bool NEED_U = (MODE & (M_LAPLACE | M_DIVU)) != 0 || MASSU;
  constexpr bool NEED_P = (MODE & (M_GRADP | M_MASSP)) != 0;
  constexpr bool OUT_U = (MODE & (M_LAPLACE | M_GRADP)) != 0;
  constexpr bool OUT_P = (MODE & (M_DIVU | M_MASSP)) != 0;
  const bool ploc = c.p_local();
  const int64_t pnode = (c.valid && ploc) ? c.p_node(a.np0, a.np1) : 0;
  // the nodal source values of every component are loaded before the vertex
  // loads and the barrier, so their latencies overlap
  T su[3] = {0, 0, 0}, sp = 0;
  if (NEED_U && c.valid && (a.src_all ? dir : !dir)) {
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp) su[comp] = a.src_u[comp * a.Nv + vnode];
  }
  if (NEED_P && c.valid && ploc) sp = a.src_p[pnode];
  if (c.valid)
    for (int idx = c.t; idx < Sh::NV * DIM; idx += NQ) {
      const int v = idx / DIM, comp = idx % DIM;
      const int vx = c.cx + (v & 1), vy = c.cy + ((v >> 1) & 1), vz = c.cz + ((v >> 2) & 1);
      const int64_t vid = vx + (int64_t)(a.n0 + 1) * (vy + (int64_t)(a.n1 + 1) * (DIM == 3 ? vz : 0));
      s_X[e][idx] = a.X[vid * DIM + comp];
    }
  __syncthreads();

  T g[3][3] = {};
  if (NEED_U && !MASSU) {
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
      if (c.active) c.buf(comp)[c.t] = su[comp];
    csync<Sh::WAVE>();
    c.template gradients<DIM>(g);
  }
  T pval = 0;
  if (NEED_P) {
    if (c.active) c.b0[c.t] = sp;
    csync<Sh::WAVE>();
    const T *vals = c.template interpolate<Sh::M, TAB_SP>();
    pval = vals[c.t];
    csync<Sh::WAVE>();
  }

  // geometry at this Gauss point
  T xi[3] = {s_tab[TAB_X + c.qi], s_tab[TAB_X + c.qj], DIM == 3 ? s_tab[TAB_X + c.ql] : T(0)};
  T J[3][3], I[3][3];
  q1_jacobian<DIM>(s_X[e], xi, J);
  const T det = invert<DIM>(J, I);
  T w = s_tab[TAB_W + c.qi] * s_tab[TAB_W + c.qj];
  if (DIM == 3) w *= s_tab[TAB_W + c.ql];
  const T JxW = det * w;

  if constexpr (MASSU) {
    // velocity mass: values at the points, tested with the values
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp) {
      if (c.active) c.b0[c.t] = su[comp];
      csync<Sh::WAVE>();
      const T *vals = c.template interpolate<Sh::N, TAB_S>();
      const T v = vals[c.t];
      csync<Sh::WAVE>();
      if (c.active) c.b0[c.t] = JxW * v;
      csync<Sh::WAVE>();
      const T r = c.template integrate<Sh::N, TAB_S>(c.b0);
      csync<Sh::WAVE>();
      if (a.ev_u) {
        if (c.valid) a.ev_u[cell_slot(a.n0, a.n1, DIM, Q, c.cx, c.cy, c.cz, comp, c.qi, c.qj, c.ql)] = r;
      } else if (c.valid && !dir) {
        atomic_add(a.dst_u + comp * a.Nv + vnode, r);
      }
    }
    return;
  }
  T f[3][3] = {};
  T qv = 0;
  if (MODE & M_LAPLACE) {
    const T s = JxW * a.nu;
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp) {
      T gp[3];
#pragma unroll
      for (int x = 0; x < DIM; ++x) {
        T acc = 0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) acc += I[b][x] * g[comp][b];
        gp[x] = acc * s;
      }
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        T acc = 0;
#pragma unroll
        for (int x = 0; x < DIM; ++x) acc += I[b][x] * gp[x];
        f[comp][b] = acc;
      }
    }
  }
  if (MODE & M_GRADP) {
    const T s = -JxW * pval;
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
#pragma unroll
      for (int b = 0; b < DIM; ++b) f[comp][b] += s * I[b][comp];
  }
  if (MODE & M_DIVU) {
    T div = 0;
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
#pragma unroll
      for (int b = 0; b < DIM; ++b) div += I[b][comp] * g[comp][b];
    qv = -JxW * div;
  }
  if (MODE & M_MASSP) qv += JxW * pval;

  if (OUT_U) {
    T r[3];
    c.template integrate_gradients<DIM>(f, r);
    if (a.ev_u) {
      if (c.valid)
#pragma unroll
        for (int comp = 0; comp < DIM; ++comp)
          a.ev_u[cell_slot(a.n0, a.n1, DIM, Q, c.cx, c.cy, c.cz, comp, c.qi, c.qj, c.ql)] = r[comp];
    } else {
#pragma unroll
      for (int comp = 0; comp < DIM; ++comp)
        if (c.valid && !dir) atomic_add(a.dst_u + comp * a.Nv + vnode, r[comp]);
    }
  }
  if (OUT_P) {
    if (c.active) c.b0[c.t] = qv;
    csync<Sh::WAVE>();
    const T r = c.template integrate<Sh::M, TAB_SP>(c.b0);
    if (a.ev_p) {
      constexpr int M = Sh::M;
      if (c.valid && ploc) a.ev_p[cell_slot(a.n0, a.n1, 1, M, c.cx, c.cy, c.cz, 0, c.qi, c.qj, c.ql)] = r;
    } else if (c.valid && ploc) {
      atomic_add(a.dst_p + pnode, r);
    }
  }
}

// ---------------------------------------------------------------- diagonal
template <int DIM, int K>
__global__ void __launch_bounds__((Shape<DIM, K, 0>::BLOCK)) laplace_diag_kernel(CellArgs<double> a) {
  using Sh = Shape<DIM, K, 0>;
  using T = double;
  constexpr int NQ = Sh::NQ, CPB = Sh::CPB, Q = Sh::Q, NS = DIM == 2 ? 3 : 6;
  __shared__ T s_tab[TAB_SIZE];
  __shared__ T s_G[CPB][NQ * NS];
  __shared__ T s_X[CPB][Sh::NV * DIM];
  const int tid = threadIdx.x;
  for (int i = tid; i < TAB_SIZE; i += Sh::BLOCK) s_tab[i] = a.tab[i];
  int e, t;
  bool active;
  Sh::map(tid, e, t, active);
  const int lin = blockIdx.x * CPB + e;
  const bool valid = active && lin < a.nlaunch;
  const int cell = valid ? launch_cell(a, lin) : 0;
  const int qi = t % Q, qj = (t / Q) % Q, ql = DIM == 3 ? t / (Q * Q) : 0;
  int cx = 0, cy = 0, cz = 0;
  if (valid) {
    cx = cell % a.n0;
    const int r = cell / a.n0;
    cy = r % a.n1;
    cz = DIM == 3 ? r / a.n1 : 0;
  }
  if (valid)
    for (int idx = t; idx < Sh::NV * DIM; idx += NQ) {
      const int v = idx / DIM, comp = idx % DIM;
      const int vx = cx + (v & 1), vy = cy + ((v >> 1) & 1), vz = cz + ((v >> 2) & 1);
      const int64_t vid = vx + (int64_t)(a.n0 + 1) * (vy + (int64_t)(a.n1 + 1) * (DIM == 3 ? vz : 0));
      s_X[e][idx] = a.X[vid * DIM + comp];
    }
  __syncthreads();
  {
    T xi[3] = {s_tab[TAB_X + qi], s_tab[TAB_X + qj], DIM == 3 ? s_tab[TAB_X + ql] : T(0)};
    T J[3][3], I[3][3];
    q1_jacobian<DIM>(s_X[e], xi, J);
    const T det = invert<DIM>(J, I);
    T w = s_tab[TAB_W + qi] * s_tab[TAB_W + qj];
    if (DIM == 3) w *= s_tab[TAB_W + ql];
    const T s = det * w * a.nu;
    // G = s * I I^T (symmetric), stored upper triangle
    int idx = 0;
#pragma unroll
    for (int b = 0; b < DIM; ++b)
#pragma unroll
      for (int b2 = b; b2 < DIM; ++b2) {
        T acc = 0;
#pragma unroll
        for (int x = 0; x < DIM; ++x) acc += I[b][x] * I[b2][x];
        if (active) s_G[e][t * NS + idx] = s * acc;
        ++idx;
      }
  }
  __syncthreads();
  // node (qi, qj, ql): sum over points
  const T *S = s_tab + TAB_S;
  const T *DS = s_tab + TAB_DS;
  T d = 0;
  for (int q = 0; q < NQ; ++q) {
    const int p0 = q % Q, p1 = (q / Q) % Q, p2 = DIM == 3 ? q / (Q * Q) : 0;
    T gphi[3];
    const T v0 = S[p0 * MAXQ + qi], v1 = S[p1 * MAXQ + qj];
    const T d0 = DS[p0 * MAXQ + qi], d1 = DS[p1 * MAXQ + qj];
    if (DIM == 2) {
      gphi[0] = d0 * v1;
      gphi[1] = v0 * d1;
    } else {
      const T v2 = S[p2 * MAXQ + ql], d2 = DS[p2 * MAXQ + ql];
      gphi[0] = d0 * v1 * v2;
      gphi[1] = v0 * d1 * v2;
      gphi[2] = v0 * v1 * d2;
    }
    const T *G = &s_G[e][q * NS];
    int idx = 0;
#pragma unroll
    for (int b = 0; b < DIM; ++b)
#pragma unroll
      for (int b2 = b; b2 < DIM; ++b2) {
        const T term = G[idx++] * gphi[b] * gphi[b2];
        d += b == b2 ? term : 2 * term;
      }
  }
  if (valid) {
    const int gx = cx * K + qi, gy = cy * K + qj, gz = cz * K + ql;
    bool dir = gx == 0 || gx == a.nv0 - 1 || gy == 0 || gy == a.nv1 - 1;
    if (DIM == 3) dir = dir || gz == 0 || gz == a.nv2 - 1;
    if (!dir) {
      const int64_t node = gx + (int64_t)a.nv0 * (gy + (int64_t)a.nv1 * gz);
      atomic_add(a.dst_u + node, d);
    }
  }
}

// diag(M_p)_i = sum_q JxW psi_i(q)^2 (pressure degree KP)
template <int DIM, int K, int KP>
__global__ void __launch_bounds__((Shape<DIM, K, KP>::BLOCK)) mass_diag_kernel(CellArgs<double> a) {
  using Sh = Shape<DIM, K, KP>;
  using T = double;
  constexpr int NQ = Sh::NQ, CPB = Sh::CPB, Q = Sh::Q, M = Sh::M;
  __shared__ T s_tab[TAB_SIZE];
  __shared__ T s_W[CPB][NQ];
  __shared__ T s_X[CPB][Sh::NV * DIM];
  const int tid = threadIdx.x;
  for (int i = tid; i < TAB_SIZE; i += Sh::BLOCK) s_tab[i] = a.tab[i];
  int e, t;
  bool active;
  Sh::map(tid, e, t, active);
  const int lin = blockIdx.x * CPB + e;
  const bool valid = active && lin < a.nlaunch;
  const int cell = valid ? launch_cell(a, lin) : 0;
  const int qi = t % Q, qj = (t / Q) % Q, ql = DIM == 3 ? t / (Q * Q) : 0;
  int cx = 0, cy = 0, cz = 0;
  if (valid) {
    cx = cell % a.n0;
    const int r = cell / a.n0;
    cy = r % a.n1;
    cz = DIM == 3 ? r / a.n1 : 0;
  }
  if (valid)
    for (int idx = t; idx < Sh::NV * DIM; idx += NQ) {
      const int v = idx / DIM, comp = idx % DIM;
      const int vx = cx + (v & 1), vy = cy + ((v >> 1) & 1), vz = cz + ((v >> 2) & 1);
      const int64_t vid = vx + (int64_t)(a.n0 + 1) * (vy + (int64_t)(a.n1 + 1) * (DIM == 3 ? vz : 0));
      s_X[e][idx] = a.X[vid * DIM + comp];
    }
  __syncthreads();
  {
    T xi[3] = {s_tab[TAB_X + qi], s_tab[TAB_X + qj], DIM == 3 ? s_tab[TAB_X + ql] : T(0)};
    T J[3][3], I[3][3];
    q1_jacobian<DIM>(s_X[e], xi, J);
    const T det = invert<DIM>(J, I);
    T w = s_tab[TAB_W + qi] * s_tab[TAB_W + qj];
    if (DIM == 3) w *= s_tab[TAB_W + ql];
    if (active) s_W[e][t] = det * w;
  }
  __syncthreads();
  const bool node = qi < M && qj < M && (DIM == 2 || ql < M);
  if (!valid || !node) return;
  const T *Sp = s_tab + TAB_SP;
  T d = 0;
  for (int q = 0; q < NQ; ++q) {
    const int p0 = q % Q, p1 = (q / Q) % Q, p2 = DIM == 3 ? q / (Q * Q) : 0;
    T v = Sp[p0 * MAXQ + qi] * Sp[p1 * MAXQ + qj];
    if (DIM == 3) v *= Sp[p2 * MAXQ + ql];
    d += s_W[e][q] * v * v;
  }
  const int64_t pn = (cx * KP + qi) + (int64_t)a.np0 * ((cy * KP + qj) + (int64_t)a.np1 * (cz * KP + ql));
  atomic_add(a.dst_p + pn, d);
}

// ---------------------------------------------------------------- setup helpers
// Gauss-point coordinates, det J check, and load vector share this kernel.
template <int DIM, int K>
__global__ void __launch_bounds__((Shape<DIM, K, 0>::BLOCK))
    point_kernel(CellArgs<double> a, int what, double *out, const double *f_qp, int *bad) {
  using Sh = Shape<DIM, K, 0>;
  using T = double;
  constexpr int NQ = Sh::NQ, CPB = Sh::CPB, Q = Sh::Q;
  __shared__ T s_tab[TAB_SIZE];
  __shared__ T s_buf[3][CPB * NQ];
  __shared__ T s_X[CPB][Sh::NV * DIM];
  const int tid = threadIdx.x;
  for (int i = tid; i < TAB_SIZE; i += Sh::BLOCK) s_tab[i] = a.tab[i];
  CellCtx<DIM, K, 0, T> c;
  int e;
  Sh::map(tid, e, c.t, c.active);
  const int lin = blockIdx.x * CPB + e;
  c.valid = c.active && lin < a.nlaunch;
  const int cell = c.valid ? launch_cell(a, lin) : 0;
  c.qi = c.t % Q;
  c.qj = (c.t / Q) % Q;
  c.ql = DIM == 3 ? c.t / (Q * Q) : 0;
  c.cx = c.cy = c.cz = 0;
  if (c.valid) {
    c.cx = cell % a.n0;
    const int r = cell / a.n0;
    c.cy = r % a.n1;
    c.cz = DIM == 3 ? r / a.n1 : 0;
  }
  c.b0 = &s_buf[0][e * NQ];
  c.b1 = &s_buf[1][e * NQ];
  c.b2 = &s_buf[2][e * NQ];
  c.tab = s_tab;
  if (c.valid)
    for (int idx = c.t; idx < Sh::NV * DIM; idx += NQ) {
      const int v = idx / DIM, comp = idx % DIM;
      const int vx = c.cx + (v & 1), vy = c.cy + ((v >> 1) & 1), vz = c.cz + ((v >> 2) & 1);
      const int64_t vid = vx + (int64_t)(a.n0 + 1) * (vy + (int64_t)(a.n1 + 1) * (DIM == 3 ? vz : 0));
      s_X[e][idx] = a.X[vid * DIM + comp];
    }
  __syncthreads();
  T xi[3] = {s_tab[TAB_X + c.qi], s_tab[TAB_X + c.qj], DIM == 3 ? s_tab[TAB_X + c.ql] : T(0)};
  T J[3][3], I[3][3];
  q1_jacobian<DIM>(s_X[e], xi, J);
  const T det = invert<DIM>(J, I);
  const int64_t qid = (int64_t)cell * NQ + c.t;
  if (what == 0) {  // quadrature points
    if (c.valid)
      for (int comp = 0; comp < DIM; ++comp) out[qid * DIM + comp] = q1_point<DIM>(s_X[e], xi, comp);
  } else if (what == 1) {  // geometry check
    if (c.valid && !(det > 0)) atomicMin(bad, cell);
  } else {  // load vector
    T w = s_tab[TAB_W + c.qi] * s_tab[TAB_W + c.qj];
    if (DIM == 3) w *= s_tab[TAB_W + c.ql];
    const bool dir = c.valid ? c.vel_dirichlet(a.nv0, a.nv1, a.nv2) : true;
    const int64_t vnode = c.valid ? c.vel_node(a.nv0, a.nv1) : 0;
    for (int comp = 0; comp < DIM; ++comp) {
      const T fv = c.valid ? f_qp[qid * DIM + comp] * det * w : T(0);
      if (c.active) c.b0[c.t] = fv;
      __syncthreads();
      const T r = c.template integrate<Sh::N, TAB_S>(c.b0);
      __syncthreads();
      if (c.valid && !dir) atomic_add(out + comp * a.Nv + vnode, r);
    }
  }
}

// ---------------------------------------------------------------- dispatch
template <typename T>
static CellArgs<T> make_args(const LevelGeom &g, const T *X, const T *tab) {
  CellArgs<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.ncells = (int)g.ncells;
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.np0 = g.np[0];
  a.np1 = g.np[1];
  a.np2 = g.np[2];
  a.Nv = g.Nv;
  a.Np = g.Np;
  a.X = X;
  a.tab = tab;
  a.colour = -1;
  a.nlaunch = (int)g.ncells;
  return a;
}

// Run `launch(a)` once per cell colour (2^dim colours, fixed order) so that
// atomic accumulation into shared nodes happens in a deterministic order.
template <typename T, typename F>
static void by_colour(CellArgs<T> a, int dim, F launch) {
  for (int col = 0; col < (1 << dim); ++col) {
    const int px = col & 1, py = (col >> 1) & 1, pz = (col >> 2) & 1;
    a.colour = col;
    a.cm0 = (a.n0 - px + 1) / 2;
    a.cm1 = (a.n1 - py + 1) / 2;
    const int cm2 = dim == 3 ? (a.n2 - pz + 1) / 2 : 1;
    a.nlaunch = a.cm0 * a.cm1 * cm2;
    if (a.nlaunch > 0) launch(a);
  }
}

template <int DIM, int K, int KP, typename T, int MODE>
static void go(const CellArgs<T> &a, hipStream_t s) {
  using Sh = Shape<DIM, K, KP>;
  if (a.nlaunch == 0) return;
  const int grid = (a.nlaunch + Sh::CPB - 1) / Sh::CPB;
  hipLaunchKernelGGL((cell_kernel<DIM, K, KP, T, MODE>), dim3(grid), dim3(Sh::BLOCK), 0, s, a);
}

template <int DIM, int K, typename T>
static void dispatch_mode(const CellArgs<T> &a, int mode, int kp, hipStream_t s) {
  if (mode == M_LAPLACE) {
    go<DIM, K, 0, T, M_LAPLACE>(a, s);
    return;
  }
  if (mode == M_MASSU) {
    go<DIM, K, 0, T, M_MASSU>(a, s);
    return;
  }
  if constexpr (K >= 2) {
    if (mode == (M_LAPLACE | M_DIVU)) {  // lifting of Dirichlet data (right-hand side)
      go<DIM, K, K - 1, T, M_LAPLACE | M_DIVU>(a, s);
      return;
    }
    MFS_REQUIRE(kp == K - 1, MFS_EUNSUPPORTED, "cell operator needs pressure degree k-1 (got k=%d kp=%d)", K, kp);
    switch (mode) {
      case M_LAPLACE | M_GRADP | M_DIVU:
        go<DIM, K, K - 1, T, M_LAPLACE | M_GRADP | M_DIVU>(a, s);
        return;
      case M_GRADP:
        go<DIM, K, K - 1, T, M_GRADP>(a, s);
        return;
      case M_DIVU:
        go<DIM, K, K - 1, T, M_DIVU>(a, s);
        return;
      case M_MASSP:
        go<DIM, K, K - 1, T, M_MASSP>(a, s);
        return;
      default:
        break;
    }
  }
  MFS_REQUIRE(false, MFS_EUNSUPPORTED, "unsupported cell operator mode %d for k=%d", mode, K);
}

template <int DIM, typename T>
static void dispatch_k(const CellArgs<T> &a, int k, int kp, int mode, hipStream_t s) {
  switch (k) {
    case 1: dispatch_mode<DIM, 1, T>(a, mode, kp, s); break;
    case 2: dispatch_mode<DIM, 2, T>(a, mode, kp, s); break;
    case 3: dispatch_mode<DIM, 3, T>(a, mode, kp, s); break;
    case 4: dispatch_mode<DIM, 4, T>(a, mode, kp, s); break;
    case 5: dispatch_mode<DIM, 5, T>(a, mode, kp, s); break;
    case 6: dispatch_mode<DIM, 6, T>(a, mode, kp, s); break;
    default: MFS_REQUIRE(false, MFS_EUNSUPPORTED, "degree %d not compiled (1..6)", k);
  }
}

template <typename T>
void launch_cell_op(const LevelGeom &g, const DevLevel<T> &d, int mode, T nu, T *dst_u, T *dst_p,
                    const T *src_u, const T *src_p, hipStream_t s, bool src_all) {
  CellArgs<T> a = make_args<T>(g, d.X, d.tab);
  a.nu = nu;
  a.src_all = src_all ? 1 : 0;
  a.dst_u = dst_u;
  a.dst_p = dst_p;
  a.src_u = src_u;
  a.src_p = src_p;
  // 3D: one launch per cell colour, so that the atomic accumulation is
  // deterministic (2D keeps one launch: it is bound by launch latency)
  if (g.dim == 2)
    dispatch_k<2, T>(a, g.k, g.kp, mode, s);
  else
    by_colour(a, 3, [&](const CellArgs<T> &ac) { dispatch_k<3, T>(ac, g.k, g.kp, mode, s); });
  MFS_HIP(hipGetLastError());
}
template void launch_cell_op<double>(const LevelGeom &, const DevLevel<double> &, int, double, double *, double *,
                                     const double *, const double *, hipStream_t, bool);
template void launch_cell_op<float>(const LevelGeom &, const DevLevel<float> &, int, float, float *, float *,
                                    const float *, const float *, hipStream_t, bool);

template <int DIM, int K>
static void go_diag(const CellArgs<double> &a, hipStream_t s) {
  using Sh = Shape<DIM, K, 0>;
  if (a.nlaunch == 0) return;
  const int grid = (a.nlaunch + Sh::CPB - 1) / Sh::CPB;
  hipLaunchKernelGGL((laplace_diag_kernel<DIM, K>), dim3(grid), dim3(Sh::BLOCK), 0, s, a);
}
template <int DIM, int K>
static void go_point(const CellArgs<double> &a, int what, double *out, const double *f, int *bad, hipStream_t s) {
  using Sh = Shape<DIM, K, 0>;
  if (a.nlaunch == 0) return;
  const int grid = (a.nlaunch + Sh::CPB - 1) / Sh::CPB;
  hipLaunchKernelGGL((point_kernel<DIM, K>), dim3(grid), dim3(Sh::BLOCK), 0, s, a, what, out, f, bad);
}

#define MFS_K_SWITCH(DIM, k, CALL)                                                  \
  switch (k) {                                                                      \
    case 1: CALL(DIM, 1); break;                                                    \
    case 2: CALL(DIM, 2); break;                                                    \
    case 3: CALL(DIM, 3); break;                                                    \
    case 4: CALL(DIM, 4); break;                                                    \
    case 5: CALL(DIM, 5); break;                                                    \
    case 6: CALL(DIM, 6); break;                                                    \
    default: MFS_REQUIRE(false, MFS_EUNSUPPORTED, "degree %d not compiled", (k)); \
  }

void launch_laplace_diagonal(const LevelGeom &g, const double *X, const double *tab, double nu, double *diag,
                             hipStream_t s) {
  CellArgs<double> a = make_args<double>(g, X, tab);
  a.nu = nu;
  a.dst_u = diag;
#define CALL_DIAG(D, K) go_diag<D, K>(ac, s)
  by_colour(a, g.dim, [&](const CellArgs<double> &ac) {
    if (g.dim == 2) {
      MFS_K_SWITCH(2, g.k, CALL_DIAG)
    } else {
      MFS_K_SWITCH(3, g.k, CALL_DIAG)
    }
  });
#undef CALL_DIAG
  MFS_HIP(hipGetLastError());
}

template <int DIM, int K, int KP>
static void go_mass_diag(const CellArgs<double> &a, hipStream_t s) {
  using Sh = Shape<DIM, K, KP>;
  if (a.nlaunch == 0) return;
  const int grid = (a.nlaunch + Sh::CPB - 1) / Sh::CPB;
  hipLaunchKernelGGL((mass_diag_kernel<DIM, K, KP>), dim3(grid), dim3(Sh::BLOCK), 0, s, a);
}
template <int DIM, int K>
static void go_mass_diag_kp(const CellArgs<double> &a, int kp, hipStream_t s) {
  if (kp == K) {
    go_mass_diag<DIM, K, K>(a, s);
    return;
  }
  if constexpr (K >= 2) {
    if (kp == K - 1) {
      go_mass_diag<DIM, K, K - 1>(a, s);
      return;
    }
  }
  MFS_REQUIRE(false, MFS_EUNSUPPORTED, "pressure degree %d with k=%d", kp, K);
}

void launch_mass_diagonal(const LevelGeom &g, const double *X, const double *tab, double *diag, hipStream_t s) {
  CellArgs<double> a = make_args<double>(g, X, tab);
  a.dst_p = diag;
#define CALL_MD(D, K) go_mass_diag_kp<D, K>(ac, g.kp, s)
  by_colour(a, g.dim, [&](const CellArgs<double> &ac) {
    if (g.dim == 2) {
      MFS_K_SWITCH(2, g.k, CALL_MD)
    } else {
      MFS_K_SWITCH(3, g.k, CALL_MD)
    }
  });
#undef CALL_MD
  MFS_HIP(hipGetLastError());
}

static void point_op(const LevelGeom &g, const double *X, const double *tab, int what, double *out,
                     const double *f, int *bad, hipStream_t s) {
  CellArgs<double> a = make_args<double>(g, X, tab);
#define CALL_PT(D, K) go_point<D, K>(ac, what, out, f, bad, s)
  auto run = [&](const CellArgs<double> &ac) {
    if (g.dim == 2) {
      MFS_K_SWITCH(2, g.k, CALL_PT)
    } else {
      MFS_K_SWITCH(3, g.k, CALL_PT)
    }
  };
  if (what == 2)  // the load vector accumulates: by colour (deterministic)
    by_colour(a, g.dim, run);
  else
    run(a);
#undef CALL_PT
  MFS_HIP(hipGetLastError());
}

void launch_quadrature_points(const LevelGeom &g, const double *X, const double *tab, double *out,
                              hipStream_t s) {
  point_op(g, X, tab, 0, out, nullptr, nullptr, s);
}
void launch_check_geometry(const LevelGeom &g, const double *X, const double *tab, int *bad, hipStream_t s) {
  point_op(g, X, tab, 1, nullptr, nullptr, bad, s);
}
void launch_load_vector(const LevelGeom &g, const double *X, const double *tab, const double *f_qp,
                        double *b_u, hipStream_t s) {
  point_op(g, X, tab, 2, b_u, f_qp, nullptr, s);
}

// ---------------------------------------------------------------- Dirichlet fill
// Node gather of cell-local results (3D): every row of dst_u (Dirichlet rows
// = dir_src, or 0) and of dst_p is the sum of the contributions of the cells
// that contain the node, in a fixed order (z, y, x cell index), so the result
// is deterministic.  Along one direction a node at grid index x of a degree-d
// grid lies in cells x/d - 1 (local index d) and x/d (local 0) when d divides
// x, otherwise in cell x/d at local index x % d.
__device__ __forceinline__ int node_cells(int x, int d, int ncell, int cell[2], int loc[2]) {
  const int c = x / d, l = x - c * d;
  int cnt = 0;
  if (l == 0 && c >= 1) {
    cell[cnt] = c - 1;
    loc[cnt++] = d;
  }
  if (c < ncell) {
    cell[cnt] = c;
    loc[cnt++] = l;
  }
  return cnt;
}

template <typename T>
__global__ void __launch_bounds__(256) cell_gather_kernel(CellArgs<T> a, int k, int kp, T *dst_u, T *dst_p,
                                                           const T *dir_src) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int Q = k + 1;
  if (dst_u && i < a.Nv) {
    const int gx = (int)(i % a.nv0);
    const int64_t r = i / a.nv0;
    const int gy = (int)(r % a.nv1), gz = (int)(r / a.nv1);
    if (gx == 0 || gy == 0 || gz == 0 || gx == a.nv0 - 1 || gy == a.nv1 - 1 || gz == a.nv2 - 1) {
      for (int c = 0; c < 3; ++c) dst_u[c * a.Nv + i] = dir_src ? dir_src[c * a.Nv + i] : T(0);
    } else {
      int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
      const int nx = node_cells(gx, k, a.n0, cx, lx), ny = node_cells(gy, k, a.n1, cy, ly),
                nz = node_cells(gz, k, a.n2, cz, lz);
      T acc[3] = {0, 0, 0};
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
          for (int x = 0; x < nx; ++x)
            for (int c = 0; c < 3; ++c)
              acc[c] += a.ev_u[cell_slot(a.n0, a.n1, 3, Q, cx[x], cy[y], cz[z], c, lx[x], ly[y], lz[z])];
      for (int c = 0; c < 3; ++c) dst_u[c * a.Nv + i] = acc[c];
    }
  }
  if (dst_p && i < a.Np) {
    const int M = kp + 1;
    const int px = (int)(i % a.np0);
    const int64_t r = i / a.np0;
    const int py = (int)(r % a.np1), pz = (int)(r / a.np1);
    int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
    const int nx = node_cells(px, kp, a.n0, cx, lx), ny = node_cells(py, kp, a.n1, cy, ly),
              nz = node_cells(pz, kp, a.n2, cz, lz);
    T acc = 0;
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) acc += a.ev_p[cell_slot(a.n0, a.n1, 1, M, cx[x], cy[y], cz[z], 0, lx[x], ly[y], lz[z])];
    dst_p[i] = acc;
  }
}

template <typename T>
void launch_node_gather(const LevelGeom &g, int k, int kp, T *ev_u, T *ev_p, T *dst_u, T *dst_p, const T *dir_src,
                        hipStream_t s) {
  MFS_REQUIRE(g.dim == 3, MFS_EINVAL, "node gather is 3D");
  CellArgs<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.ncells = (int)g.ncells;
  a.nv0 = k * g.n[0] + 1;
  a.nv1 = k * g.n[1] + 1;
  a.nv2 = k * g.n[2] + 1;
  a.np0 = kp * g.n[0] + 1;
  a.np1 = kp * g.n[1] + 1;
  a.np2 = kp * g.n[2] + 1;
  a.Nv = (int64_t)a.nv0 * a.nv1 * a.nv2;
  a.Np = (int64_t)a.np0 * a.np1 * a.np2;
  a.ev_u = ev_u;
  a.ev_p = ev_p;
  const int64_t n = std::max<int64_t>(dst_u ? a.Nv : 0, dst_p ? a.Np : 0);
  if (n > 0)
    hipLaunchKernelGGL((cell_gather_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, k, kp, dst_u,
                       dst_p, dir_src);
  MFS_HIP(hipGetLastError());
}
template void launch_node_gather<double>(const LevelGeom &, int, int, double *, double *, double *, double *,
                                         const double *, hipStream_t);
template void launch_node_gather<float>(const LevelGeom &, int, int, float *, float *, float *, float *, const float *,
                                        hipStream_t);

int64_t cell_ev_elems(const LevelGeom &g) {
  if (g.dim != 3 || g.k < 3) return 0;
  const int64_t q = g.k + 1, m = g.kp > 0 ? g.kp + 1 : 0;
  return g.ncells * (3 * q * q * q + m * m * m);
}

template <typename T>
void launch_cell_op_gather(const LevelGeom &g, const DevLevel<T> &d, int mode, T nu, T *dst_u, T *dst_p,
                           const T *src_u, const T *src_p, const T *dir_src, T *ev, hipStream_t s) {
  MFS_REQUIRE(g.dim == 3 && g.k >= 3 && ev != nullptr, MFS_EINVAL, "cell gather needs a 3D level of degree >= 3");
  CellArgs<T> a = make_args<T>(g, d.X, d.tab);
  a.nu = nu;
  a.src_u = src_u;
  a.src_p = src_p;
  a.ev_u = ev;
  const int64_t q = g.k + 1;
  a.ev_p = ev + g.ncells * 3 * q * q * q;
  if (!launch_column_cells<T>(g, d.X, mode, nu, src_u, src_p, a.ev_u, a.ev_p, s)) dispatch_k<3, T>(a, g.k, g.kp, mode, s);
  const bool out_u = mode & (M_LAPLACE | M_GRADP | M_MASSU), out_p = mode & (M_DIVU | M_MASSP);
  const int64_t n = std::max<int64_t>(out_u ? g.Nv : 0, out_p ? g.Np : 0);
  if (n > 0)
    hipLaunchKernelGGL((cell_gather_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, g.k, g.kp,
                       out_u ? dst_u : (T *)nullptr, out_p ? dst_p : (T *)nullptr, dir_src);
  MFS_HIP(hipGetLastError());
}
template void launch_cell_op_gather<double>(const LevelGeom &, const DevLevel<double> &, int, double, double *,
                                            double *, const double *, const double *, const double *, double *,
                                            hipStream_t);
template void launch_cell_op_gather<float>(const LevelGeom &, const DevLevel<float> &, int, float, float *, float *,
                                           const float *, const float *, const float *, float *, hipStream_t);

// The node gather of the velocity block fused with a Chebyshev step: on every
// free row the contributions of the cells that contain the node are summed in
// the order of cell_gather_kernel into (A x)_j, then r = D^{-1}_j (b_j - (A x)_j),
// d_j = c2 r (first step) or c1 d_j + c2 r, x_j += d_j; Dirichlet rows keep x
// and d.  The same arithmetic as the gather followed by the separate update,
// without writing and re-reading A x.
template <typename T>
__global__ void __launch_bounds__(256) cell_gather_cheb_kernel(CellArgs<T> a, int k, T *x, T *d, const T *b,
                                                                const T *inv, T c1, T c2, int first) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.Nv) return;
  const int Q = k + 1;
  const int gx = (int)(i % a.nv0);
  const int64_t r = i / a.nv0;
  const int gy = (int)(r % a.nv1), gz = (int)(r / a.nv1);
  if (gx == 0 || gy == 0 || gz == 0 || gx == a.nv0 - 1 || gy == a.nv1 - 1 || gz == a.nv2 - 1) return;
  int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
  const int nx = node_cells(gx, k, a.n0, cx, lx), ny = node_cells(gy, k, a.n1, cy, ly),
            nz = node_cells(gz, k, a.n2, cz, lz);
  T acc[3] = {0, 0, 0};
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int xx = 0; xx < nx; ++xx)
        for (int c = 0; c < 3; ++c)
          acc[c] += a.ev_u[cell_slot(a.n0, a.n1, 3, Q, cx[xx], cy[y], cz[z], c, lx[xx], ly[y], lz[z])];
  const T iv = inv[i];
  for (int c = 0; c < 3; ++c) {
    const int64_t j = c * a.Nv + i;
    const T rr = iv * (b[j] - acc[c]);
    const T dn = first ? c2 * rr : c1 * d[j] + c2 * rr;
    d[j] = dn;
    x[j] += dn;
  }
}

template <typename T>
void launch_cell_cheb_gather(const LevelGeom &g, const DevLevel<T> &dv, T nu, T *x, T *d, const T *b, const T *inv,
                             T c1, T c2, bool first, T *ev, hipStream_t s) {
  MFS_REQUIRE(g.dim == 3 && g.k >= 3 && ev != nullptr, MFS_EINVAL, "cell gather needs a 3D level of degree >= 3");
  CellArgs<T> a = make_args<T>(g, dv.X, dv.tab);
  a.nu = nu;
  a.src_u = x;
  a.ev_u = ev;
  const int64_t q = g.k + 1;
  a.ev_p = ev + g.ncells * 3 * q * q * q;
  if (!launch_column_cells<T>(g, dv.X, M_LAPLACE, nu, x, nullptr, a.ev_u, a.ev_p, s))
    dispatch_k<3, T>(a, g.k, g.kp, M_LAPLACE, s);
  hipLaunchKernelGGL((cell_gather_cheb_kernel<T>), dim3((unsigned)((g.Nv + 255) / 256)), dim3(256), 0, s, a, g.k, x,
                     d, b, inv, c1, c2, first ? 1 : 0);
  MFS_HIP(hipGetLastError());
}
template void launch_cell_cheb_gather<double>(const LevelGeom &, const DevLevel<double> &, double, double *, double *,
                                              const double *, const double *, double, double, bool, double *,
                                              hipStream_t);
template void launch_cell_cheb_gather<float>(const LevelGeom &, const DevLevel<float> &, float, float *, float *,
                                             const float *, const float *, float, float, bool, float *, hipStream_t);

template <typename T>
__global__ void fill_dirichlet_kernel(int dim, int nv0, int nv1, int nv2, int64_t Nv, T *dst, const T *src) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nv) return;
  const int gx = (int)(i % nv0);
  const int64_t r = i / nv0;
  const int gy = (int)(r % nv1);
  const int gz = (int)(r / nv1);
  bool d = gx == 0 || gx == nv0 - 1 || gy == 0 || gy == nv1 - 1;
  if (dim == 3) d = d || gz == 0 || gz == nv2 - 1;
  for (int c = 0; c < dim; ++c) dst[c * Nv + i] = (d && src) ? src[c * Nv + i] : T(0);
}

template <typename T>
void launch_fill_dirichlet(const LevelGeom &g, T *dst_u, const T *src_u, hipStream_t s) {
  if (g.Nv == 0) return;
  const int64_t blocks = (g.Nv + 255) / 256;
  hipLaunchKernelGGL((fill_dirichlet_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, g.dim, g.nv[0], g.nv[1],
                     g.nv[2], g.Nv, dst_u, src_u);
  MFS_HIP(hipGetLastError());
}
template void launch_fill_dirichlet<double>(const LevelGeom &, double *, const double *, hipStream_t);
template void launch_fill_dirichlet<float>(const LevelGeom &, float *, const float *, hipStream_t);

}  // namespace mfs
