// SUPG/PSPG-stabilised Navier-Stokes Jacobian (Sec. 5) on equal-order
// Q_k/Q_k elements, matrix-free, one thread per quadrature point.
//
// At the linearisation point (u0, p0 = 0) with BDF2 mass shift
// alpha = 3 / (2 dt), the Jacobian applied to (du, dp) tested with (v, q) is
//   (alpha du + du.grad u0 + u0.grad du, v) + nu (grad du, grad v)
//   - (dp, div v) + (div du, q)
//   + delta_1 (R_lin, u0.grad v) + delta_1 (R(u0), du.grad v) + delta_1 (R_lin, grad q)
// with R_lin = alpha du + du.grad u0 + u0.grad du + grad dp - nu Lap du and
// R(u0) = u0.grad u0 - nu Lap u0; the Oseen variant drops du.grad u0 and the
// R(u0) term.  delta_1 = [(2/dt)^2 + (2|u0|/h_K)^2 + 9 (4 nu / h_K^2)^2]^(-1/2),
// h_K = |K|^(1/d) / k, frozen.  Laplacians are J^{-T} H J^{-1} of the
// reference Hessian (exact on affine cells).
//
// The linearisation kernel stores per quadrature point: u0 (3), grad u0 (9,
// [comp][direction]), R(u0) (3), delta_1 (1), and for the nonlinear residual
// the Galerkin value term alpha (u0 - u~) + u0.grad u0 (3) and p0 (1):
// NS_QD = 20 values, laid out [cell][field][point] so the threads of a cell
// read consecutive words.  At a general state (u0, p0) with the BDF2 history
// u~ = (4 u^n - u^{n-1}) / 3 (time derivative alpha (u - u~)), the strong
// residual is R(u0, p0) = alpha (u0 - u~) + u0.grad u0 + grad p0 - nu Lap u0;
// the linearisation point of a Jacobian alone has p0 = 0 and u~ = u0.
//
// The residual kernel tests F_NS + F_SUPG + F_PSPG at that state from the
// stored data alone: (alpha (u - u~) + u.grad u, v) + (nu grad u - p I
// + delta_1 R (x) u, grad v) + (div u, q) + (delta_1 R, grad q).
#include <algorithm>

#include "cell_common.h"

namespace mfs {

namespace nsk {

// one thread per quadrature point, laid out as the cell kernels' (velocity and
// pressure share the degree here)
template <int DIM, int K>
using Shape = mfs::Shape<DIM, K, K>;

template <typename T>
struct Args {
  int n0, n1, n2, ncells;
  int nv0, nv1, nv2;
  int64_t Nv;
  const T *X, *tab, *src;
  T *dst;
  T *qd;
  T nu, alpha, dt;
  int newton;
  T *ev;  // cell-local outputs instead of atomics when non-null (3D)
  // cell-local inputs (3D): [cell][(k+1)^3][4], the three velocity
  // components and the pressure of a node side by side (the linearisation
  // reads the velocity), and per-cell corner coordinates [cell][8][3]
  // (x fastest) instead of the structured vertex grid; with evin, src, dst
  // and the node grid are unused and ev takes the same layout
  const T *evin;
  const T *Xcell;
  // linearisation at a general state: src = [u0 (DIM Nv) | p0 (Nv) | u~ (DIM
  // Nv)] (with evin: slot 3 = p0, u~ in evhist slots 0..2); 0: src = u0
  // alone, p0 = 0, u~ = u0
  int point;
  int keep_delta;  // leave delta_1 (field 15) as it is
  const T *evhist;
  // cells of this launch: all (colour < 0) or those whose index parities are
  // the bits of `colour` (no two share a node: with one launch per colour in
  // a fixed order, the atomic accumulation is deterministic)
  int colour, cm0, cm1, nlaunch;
};

template <typename T>
__device__ __forceinline__ int launch_cell(const Args<T> &a, int i) {
  if (a.colour < 0) return i;
  const int x = i % a.cm0, r = i / a.cm0, y = r % a.cm1, z = r / a.cm1;
  return (2 * x + (a.colour & 1)) + a.n0 * ((2 * y + ((a.colour >> 1) & 1)) + a.n1 * (2 * z + (a.colour >> 2)));
}

template <int DIM, typename T>
__device__ __forceinline__ T jac_inv(const T *Xc, const T xi[3], T I[3][3]) {
  T J[3][3] = {};
  for (int v = 0; v < (1 << DIM); ++v) {
    T f[3], df[3];
    for (int b = 0; b < DIM; ++b) {
      const bool hi = (v >> b) & 1;
      f[b] = hi ? xi[b] : T(1) - xi[b];
      df[b] = hi ? T(1) : T(-1);
    }
    for (int b = 0; b < DIM; ++b) {
      T d = df[b];
      for (int c = 0; c < DIM; ++c)
        if (c != b) d *= f[c];
      for (int a = 0; a < DIM; ++a) J[a][b] += Xc[v * DIM + a] * d;
    }
  }
  if (DIM == 2) {
    const T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const T r = T(1) / det;
    I[0][0] = J[1][1] * r;
    I[0][1] = -J[0][1] * r;
    I[1][0] = -J[1][0] * r;
    I[1][1] = J[0][0] * r;
    return det;
  }
  const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const T det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const T r = T(1) / det;
  I[0][0] = c00 * r;
  I[1][0] = c01 * r;
  I[2][0] = c02 * r;
  I[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
  I[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
  I[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
  I[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
  I[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
  I[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
  return det;
}

// Per-cell thread context: LDS buffers and sum-factorised evaluation.
template <int DIM, int K, typename T>
struct Ctx {
  static constexpr int Q = K + 1, NQ = Shape<DIM, K>::NQ;
  int t, qi, qj, ql, cx, cy, cz;
  bool valid, active;
  T *b0, *b1, *b2;
  const T *tab;

  __device__ __forceinline__ int64_t node(int nv0, int nv1) const {
    return (int64_t)(cx * K + qi) + (int64_t)nv0 * ((cy * K + qj) + (int64_t)nv1 * (cz * K + ql));
  }
  __device__ __forceinline__ bool dirichlet(int nv0, int nv1, int nv2) const {
    const int gx = cx * K + qi, gy = cy * K + qj, gz = cz * K + ql;
    bool d = gx == 0 || gx == nv0 - 1 || gy == 0 || gy == nv1 - 1;
    if (DIM == 3) d = d || gz == 0 || gz == nv2 - 1;
    return d;
  }
  // nodal value of this thread in b0 on entry: value, reference gradient,
  // and (HESS) reference Hessian (00, 01, 11 | 00, 01, 02, 11, 12, 22) at the point
  // MIXED = false: the mixed second derivatives are not formed (their
  // entries of h are left as they are; Cartesian cells do not need them)
  template <bool HESS, bool MIXED = true>
  __device__ __forceinline__ void evaluate(T &val, T g[3], T h[6]) {
    const T *S = tab + TAB_S;
    T v = sweep<DIM, Q, 0, Q, false>(b0, S, qi, qj, ql);
    if (active) b1[t] = v;
    csync<Shape<DIM, K>::WAVE>();
    v = sweep<DIM, Q, 1, Q, false>(b1, S, qi, qj, ql);
    if (active) b0[t] = v;
    csync<Shape<DIM, K>::WAVE>();
    T *vals = b0;
    if (DIM == 3) {
      v = sweep<DIM, Q, 2, Q, false>(b0, S, qi, qj, ql);
      if (active) b1[t] = v;
      csync<Shape<DIM, K>::WAVE>();
      vals = b1;
    }
    val = vals[t];
    const T *D = tab + TAB_D;
    g[0] = sweep<DIM, Q, 0, Q, false>(vals, D, qi, qj, ql);
    g[1] = sweep<DIM, Q, 1, Q, false>(vals, D, qi, qj, ql);
    g[2] = DIM == 3 ? sweep<DIM, Q, 2, Q, false>(vals, D, qi, qj, ql) : T(0);
    pin(val);
    pin(g[0]);
    pin(g[1]);
    pin(g[2]);
    csync<Shape<DIM, K>::WAVE>();
    if (HESS) {
      if (active) {
        b0[t] = g[0];
        b1[t] = g[1];
        if (DIM == 3) b2[t] = g[2];
      }
      csync<Shape<DIM, K>::WAVE>();
      if (DIM == 2) {
        h[0] = sweep<DIM, Q, 0, Q, false>(b0, D, qi, qj, ql);
        if (MIXED) h[1] = sweep<DIM, Q, 0, Q, false>(b1, D, qi, qj, ql);
        h[2] = sweep<DIM, Q, 1, Q, false>(b1, D, qi, qj, ql);
      } else {
        h[0] = sweep<DIM, Q, 0, Q, false>(b0, D, qi, qj, ql);
        if (MIXED) h[1] = sweep<DIM, Q, 0, Q, false>(b1, D, qi, qj, ql);
        if (MIXED) h[2] = sweep<DIM, Q, 0, Q, false>(b2, D, qi, qj, ql);
        h[3] = sweep<DIM, Q, 1, Q, false>(b1, D, qi, qj, ql);
        if (MIXED) h[4] = sweep<DIM, Q, 1, Q, false>(b2, D, qi, qj, ql);
        h[5] = sweep<DIM, Q, 2, Q, false>(b2, D, qi, qj, ql);
      }
#pragma unroll
      for (int i = 0; i < (DIM == 2 ? 3 : 6); ++i)
        if (MIXED || i == 0 || i == (DIM == 2 ? 2 : 3) || i == 5) pin(h[i]);
      csync<Shape<DIM, K>::WAVE>();
    }
  }
  // test with value and reference-gradient coefficients -> nodal value
  __device__ __forceinline__ T integrate(T val, const T f[3]) {
    if (active) {
      b0[t] = f[0];
      b1[t] = f[1];
      if (DIM == 3) b2[t] = f[2];
    }
    csync<Shape<DIM, K>::WAVE>();
    const T *D = tab + TAB_D;
    T r = val + sweep<DIM, Q, 0, Q, true>(b0, D, qi, qj, ql) + sweep<DIM, Q, 1, Q, true>(b1, D, qi, qj, ql);
    if (DIM == 3) r += sweep<DIM, Q, 2, Q, true>(b2, D, qi, qj, ql);
    csync<Shape<DIM, K>::WAVE>();
    if (active) b0[t] = r;
    csync<Shape<DIM, K>::WAVE>();
    const T *S = tab + TAB_S;
    T out;
    if (DIM == 2) {
      T v = sweep<DIM, Q, 1, Q, true>(b0, S, qi, qj, ql);
      if (active) b1[t] = v;
      csync<Shape<DIM, K>::WAVE>();
      out = sweep<DIM, Q, 0, Q, true>(b1, S, qi, qj, ql);
    } else {
      T v = sweep<DIM, Q, 2, Q, true>(b0, S, qi, qj, ql);
      if (active) b1[t] = v;
      csync<Shape<DIM, K>::WAVE>();
      v = sweep<DIM, Q, 1, Q, true>(b1, S, qi, qj, ql);
      if (active) b0[t] = v;
      csync<Shape<DIM, K>::WAVE>();
      out = sweep<DIM, Q, 0, Q, true>(b0, S, qi, qj, ql);
    }
    csync<Shape<DIM, K>::WAVE>();
    return out;
  }
};

// physical Laplacian of an axis-aligned cell: sum_a I[a][a]^2 H_aa
template <int DIM, typename T>
__device__ __forceinline__ T laplacian_cart(const T h[6], const T I[3][3]) {
  if (DIM == 2) return I[0][0] * I[0][0] * h[0] + I[1][1] * I[1][1] * h[2];
  return I[0][0] * I[0][0] * h[0] + I[1][1] * I[1][1] * h[3] + I[2][2] * I[2][2] * h[5];
}

// physical Laplacian from the reference Hessian: sum_a sum_bc I[b][a] I[c][a] H_bc
template <int DIM, typename T>
__device__ __forceinline__ T laplacian(const T h[6], const T I[3][3]) {
  T H[3][3];
  if (DIM == 2) {
    H[0][0] = h[0];
    H[0][1] = H[1][0] = h[1];
    H[1][1] = h[2];
  } else {
    H[0][0] = h[0];
    H[0][1] = H[1][0] = h[1];
    H[0][2] = H[2][0] = h[2];
    H[1][1] = h[3];
    H[1][2] = H[2][1] = h[4];
    H[2][2] = h[5];
  }
  T s = 0;
  for (int a = 0; a < DIM; ++a)
    for (int b = 0; b < DIM; ++b)
      for (int c = 0; c < DIM; ++c) s += I[b][a] * I[c][a] * H[b][c];
  return s;
}

#define NSK_PROLOGUE                                                                                   \
  using Sh = Shape<DIM, K>;                                                                            \
  constexpr int NQ = Sh::NQ, CPB = Sh::CPB, Q = Sh::Q;                                                 \
  __shared__ T s_tab[TAB_SIZE];                                                                        \
  __shared__ T s_buf[3][CPB * NQ];                                                                     \
  __shared__ T s_X[CPB][Sh::NV * DIM];                                                                 \
  const int tid = threadIdx.x;                                                                         \
  for (int i = tid; i < TAB_SIZE; i += Sh::BLOCK) s_tab[i] = a.tab[i];                                 \
  Ctx<DIM, K, T> c;                                                                                    \
  int e;                                                                                               \
  Sh::map(tid, e, c.t, c.active);                                                                      \
  const int lin_ = blockIdx.x * CPB + e;                                                               \
  c.valid = c.active && lin_ < a.nlaunch;                                                              \
  const int cell = c.valid ? launch_cell(a, lin_) : 0;                                                 \
  c.qi = c.t % Q;                                                                                      \
  c.qj = (c.t / Q) % Q;                                                                                \
  c.ql = DIM == 3 ? c.t / (Q * Q) : 0;                                                                 \
  c.cx = c.cy = c.cz = 0;                                                                              \
  if (c.valid) {                                                                                       \
    c.cx = cell % a.n0;                                                                                \
    const int r_ = cell / a.n0;                                                                        \
    c.cy = r_ % a.n1;                                                                                  \
    c.cz = DIM == 3 ? r_ / a.n1 : 0;                                                                   \
  }                                                                                                    \
  c.b0 = &s_buf[0][e * NQ];                                                                            \
  c.b1 = &s_buf[1][e * NQ];                                                                            \
  c.b2 = &s_buf[2][e * NQ];                                                                            \
  c.tab = s_tab;                                                                                       \
  const int64_t nd = c.valid ? c.node(a.nv0, a.nv1) : 0;                                               \
  const bool dir = c.valid ? c.dirichlet(a.nv0, a.nv1, a.nv2) : true;                                  \
  T *qd = a.qd + ((int64_t)(c.valid ? cell : 0) * NS_QD) * NQ + c.t;

// second half of the prologue: vertices to LDS, barrier, geometry at the
// point (global loads a kernel issues between the two halves overlap the
// vertex loads and the barrier)
#define NSK_PROLOGUE_B                                                                                 \
  if (c.valid && a.Xcell)                                                                              \
    for (int idx = c.t; idx < Sh::NV * DIM; idx += NQ) s_X[e][idx] = a.Xcell[(int64_t)cell * Sh::NV * DIM + idx]; \
  else if (c.valid)                                                                                    \
    for (int idx = c.t; idx < Sh::NV * DIM; idx += NQ) {                                               \
      const int v_ = idx / DIM, comp_ = idx % DIM;                                                     \
      const int vx = c.cx + (v_ & 1), vy = c.cy + ((v_ >> 1) & 1), vz = c.cz + ((v_ >> 2) & 1);        \
      const int64_t vid = vx + (int64_t)(a.n0 + 1) * (vy + (int64_t)(a.n1 + 1) * (DIM == 3 ? vz : 0)); \
      s_X[e][idx] = a.X[vid * DIM + comp_];                                                            \
    }                                                                                                  \
  __syncthreads();                                                                                     \
  T xi[3] = {s_tab[TAB_X + c.qi], s_tab[TAB_X + c.qj], DIM == 3 ? s_tab[TAB_X + c.ql] : T(0)};         \
  T I[3][3] = {};                                                                                      \
  T det_ = T(1);                                                                                       \
  if constexpr (CART) {                                                                                \
    /* axis-aligned box: J = diag(h), the off-diagonals of I stay zero */                              \
    const T hx = s_X[e][DIM] - s_X[e][0], hy = s_X[e][2 * DIM + 1] - s_X[e][1];                        \
    I[0][0] = T(1) / hx;                                                                               \
    I[1][1] = T(1) / hy;                                                                               \
    det_ = hx * hy;                                                                                    \
    if (DIM == 3) {                                                                                    \
      const T hz = s_X[e][4 * DIM + 2] - s_X[e][2];                                                    \
      I[2][2] = T(1) / hz;                                                                             \
      det_ *= hz;                                                                                      \
    }                                                                                                  \
  } else {                                                                                             \
    det_ = jac_inv<DIM>(s_X[e], xi, I);                                                                \
  }                                                                                                    \
  const T det = det_;                                                                                  \
  T wq = s_tab[TAB_W + c.qi] * s_tab[TAB_W + c.qj];                                                    \
  if (DIM == 3) wq *= s_tab[TAB_W + c.ql];                                                             \
  const T JxW = det * wq;

// linearisation data at the quadrature points from the nodal velocity u0
// (CART: every cell an axis-aligned box)
template <int DIM, int K, typename T, bool CART>
__global__ void __launch_bounds__((Shape<DIM, K>::BLOCK)) ns_linearize_kernel(Args<T> a) {
  NSK_PROLOGUE
  NSK_PROLOGUE_B
  T u[3] = {}, U[3][3] = {}, lap[3] = {};
  for (int comp = 0; comp < DIM; ++comp) {
    T v0 = T(0);
    if (c.valid) v0 = a.evin ? a.evin[((int64_t)cell * NQ + c.t) * 4 + comp] : a.src[comp * a.Nv + nd];
    if (c.active) c.b0[c.t] = v0;
    csync<Sh::WAVE>();
    T val, g[3], h[6];
    c.template evaluate<true, !CART>(val, g, h);
    u[comp] = val;
    for (int x = 0; x < DIM; ++x) {
      T s = 0;
      for (int b = 0; b < DIM; ++b) s += I[b][x] * g[b];
      U[comp][x] = s;
    }
    lap[comp] = CART ? laplacian_cart<DIM>(h, I) : laplacian<DIM>(h, I);
  }
  // the state's pressure and the BDF2 history (u~ = u0 and p0 = 0 otherwise)
  T p0 = 0, gp0[3] = {}, uh[3] = {u[0], u[1], u[2]};
  if (a.point) {
    T v0 = T(0);
    if (c.valid) v0 = a.evin ? a.evin[((int64_t)cell * NQ + c.t) * 4 + 3] : a.src[DIM * a.Nv + nd];
    if (c.active) c.b0[c.t] = v0;
    csync<Sh::WAVE>();
    T g[3], h[6];
    c.template evaluate<false>(p0, g, h);
    for (int x = 0; x < DIM; ++x) {
      T s = 0;
      for (int b = 0; b < DIM; ++b) s += I[b][x] * g[b];
      gp0[x] = s;
    }
    for (int comp = 0; comp < DIM; ++comp) {
      v0 = T(0);
      if (c.valid)
        v0 = a.evhist ? a.evhist[((int64_t)cell * NQ + c.t) * 4 + comp] : a.src[(DIM + 1 + comp) * a.Nv + nd];
      if (c.active) c.b0[c.t] = v0;
      csync<Sh::WAVE>();
      c.template evaluate<false>(uh[comp], g, h);
    }
  }
  // cell volume: every thread sums the JxW of its cell's points in a fixed order
  if (c.active) c.b0[c.t] = c.valid ? JxW : T(0);
  csync<Sh::WAVE>();
  T vol = 0;
  for (int q = 0; q < NQ; ++q) vol += c.b0[q];
  csync<Sh::WAVE>();
  const T hK = pow(vol, T(1) / T(DIM)) / T(K);
  T speed2 = 0, R0[3], gal[3];
  for (int comp = 0; comp < DIM; ++comp) {
    speed2 += u[comp] * u[comp];
    T s = 0;
    for (int x = 0; x < DIM; ++x) s += u[x] * U[comp][x];
    gal[comp] = a.alpha * (u[comp] - uh[comp]) + s;
    R0[comp] = gal[comp] + gp0[comp] - a.nu * lap[comp];
  }
  const T t1 = T(2) / a.dt, t2 = T(2) * sqrt(speed2) / hK, t3 = T(4) * a.nu / (hK * hK);
  const T delta = T(1) / sqrt(t1 * t1 + t2 * t2 + T(9) * t3 * t3);
  if (c.valid) {
    for (int f = 0; f < NS_QD; ++f) {
      T v = 0;
      if (f < 3) v = f < DIM ? u[f] : T(0);
      else if (f < 12) v = ((f - 3) / 3 < DIM && (f - 3) % 3 < DIM) ? U[(f - 3) / 3][(f - 3) % 3] : T(0);
      else if (f < 15) v = f - 12 < DIM ? R0[f - 12] : T(0);
      else if (f == 15) {
        if (a.keep_delta) continue;
        v = delta;
      } else if (f < 19) v = f - 16 < DIM ? gal[f - 16] : T(0);
      else v = p0;
      qd[f * NQ] = v;
    }
  }
}

// Jacobian application (CART: every cell an axis-aligned box)
// RES: the nonlinear residual at the stored state instead (no source vector)
template <int DIM, int K, typename T, bool CART, bool RES>
__global__ void __launch_bounds__((Shape<DIM, K>::BLOCK)) ns_jacobian_kernel(Args<T> a) {
  NSK_PROLOGUE
  // every global load of the point (nodal source values of the 4 fields,
  // linearisation data) is issued before the vertex loads and the barrier
  T sv[4] = {0, 0, 0, 0};
  T u0[3] = {}, U[3][3] = {}, R0[3] = {}, dl = 0;
  T gal[3] = {}, p0 = 0;
  if (RES) {
    if (c.valid) {
      for (int x = 0; x < DIM; ++x) gal[x] = qd[(16 + x) * NQ];
      p0 = qd[19 * NQ];
    }
  } else if (c.valid && a.evin) {
    for (int comp = 0; comp <= DIM; ++comp) sv[comp] = a.evin[((int64_t)cell * NQ + c.t) * 4 + comp];
  } else if (c.valid) {
    for (int comp = 0; comp < DIM; ++comp) sv[comp] = dir ? T(0) : a.src[comp * a.Nv + nd];
    sv[DIM] = a.src[DIM * a.Nv + nd];
  }
  if (c.valid) {
    for (int x = 0; x < DIM; ++x) u0[x] = qd[x * NQ];
    for (int cc = 0; cc < DIM; ++cc)
      for (int x = 0; x < DIM; ++x) U[cc][x] = qd[(3 + 3 * cc + x) * NQ];
    for (int x = 0; x < DIM; ++x) R0[x] = qd[(12 + x) * NQ];
    dl = qd[15 * NQ];
  }
  NSK_PROLOGUE_B
  T val_u[3], grad_u[3][3], Rl[3];
  T div = 0;
  if constexpr (RES) {
    for (int cc = 0; cc < DIM; ++cc) {
      val_u[cc] = gal[cc];
      Rl[cc] = R0[cc];
      div += U[cc][cc];
      for (int x = 0; x < DIM; ++x) grad_u[cc][x] = a.nu * U[cc][x] + dl * R0[cc] * u0[x] - (x == cc ? p0 : T(0));
    }
  } else {
  // trial fields
  T w[3] = {}, G[3][3] = {}, L[3] = {};
  for (int comp = 0; comp < DIM; ++comp) {
    if (c.active) c.b0[c.t] = sv[comp];
    csync<Sh::WAVE>();
    T val, g[3], h[6];
    c.template evaluate<true, !CART>(val, g, h);
    w[comp] = val;
    for (int x = 0; x < DIM; ++x) {
      T s = 0;
      for (int b = 0; b < DIM; ++b) s += I[b][x] * g[b];
      G[comp][x] = s;
    }
    L[comp] = CART ? laplacian_cart<DIM>(h, I) : laplacian<DIM>(h, I);
  }
  T P, gP[3] = {};
  {
    if (c.active) c.b0[c.t] = sv[DIM];
    csync<Sh::WAVE>();
    T g[3], h[6];
    c.template evaluate<false>(P, g, h);
    for (int x = 0; x < DIM; ++x) {
      T s = 0;
      for (int b = 0; b < DIM; ++b) s += I[b][x] * g[b];
      gP[x] = s;
    }
  }
  // point physics
  for (int cc = 0; cc < DIM; ++cc) {
    T conv = 0, newt = 0;
    for (int x = 0; x < DIM; ++x) {
      conv += u0[x] * G[cc][x];
      newt += w[x] * U[cc][x];
    }
    if (!a.newton) newt = 0;
    val_u[cc] = a.alpha * w[cc] + newt + conv;
    Rl[cc] = val_u[cc] + gP[cc] - a.nu * L[cc];
  }
  for (int cc = 0; cc < DIM; ++cc) {
    div += G[cc][cc];
    for (int x = 0; x < DIM; ++x) {
      T v = a.nu * G[cc][x] + dl * Rl[cc] * u0[x];
      if (a.newton) v += dl * R0[cc] * w[x];
      if (x == cc) v -= P;
      grad_u[cc][x] = v;
    }
  }
  }
  // test: physical gradient coefficients -> reference (I f), times JxW
  for (int comp = 0; comp < DIM; ++comp) {
    T f[3] = {};
    for (int b = 0; b < DIM; ++b) {
      T s = 0;
      for (int x = 0; x < DIM; ++x) s += I[b][x] * grad_u[comp][x];
      f[b] = JxW * s;
    }
    const T r = c.integrate(JxW * val_u[comp], f);
    if (a.ev) {
      if (c.valid)
        a.ev[a.evin ? ((int64_t)cell * NQ + c.t) * 4 + comp
                    : cell_slot(a.n0, a.n1, 3, Q, c.cx, c.cy, c.cz, comp, c.qi, c.qj, c.ql)] = r;
    } else if (c.valid && !dir) {
      atomicAdd(a.dst + comp * a.Nv + nd, r);
    }
  }
  {
    T f[3] = {};
    for (int b = 0; b < DIM; ++b) {
      T s = 0;
      for (int x = 0; x < DIM; ++x) s += I[b][x] * dl * Rl[x];
      f[b] = JxW * s;
    }
    const T r = c.integrate(JxW * div, f);
    if (a.ev) {
      if (c.valid)
        a.ev[a.evin ? ((int64_t)cell * NQ + c.t) * 4 + 3
                    : (int64_t)a.ncells * 3 * NQ + cell_slot(a.n0, a.n1, 1, Q, c.cx, c.cy, c.cz, 0, c.qi, c.qj, c.ql)] = r;
    } else if (c.valid) {
      atomicAdd(a.dst + DIM * a.Nv + nd, r);
    }
  }
}

#undef NSK_PROLOGUE
#undef NSK_PROLOGUE_B

}  // namespace nsk

template <typename T>
void launch_ns(const LevelGeom &g, const T *X, const T *tab, int what, T nu, T dt, int newton, const T *src, T *dst,
               T *qd, hipStream_t s, T *ev, const T *evin, const T *Xcell, const NsPoint<T> *pt) {
  MFS_REQUIRE(g.kp == g.k, MFS_EUNSUPPORTED, "Navier-Stokes operator needs equal-order elements");
  nsk::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.ncells = (int)g.ncells;
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.Nv = g.Nv;
  a.X = X;
  a.tab = tab;
  a.src = src;
  a.dst = dst;
  a.qd = qd;
  a.nu = nu;
  a.dt = dt;
  a.alpha = T(1.5) / dt;
  a.newton = newton;
  MFS_REQUIRE(ev == nullptr || g.dim == 3, MFS_EINVAL, "cell-local Navier-Stokes outputs are 3D");
  a.ev = ev;
  MFS_REQUIRE(evin == nullptr || (g.dim == 3 && Xcell != nullptr && (what == 0 || ev != nullptr)), MFS_EINVAL,
              "cell-local Navier-Stokes inputs need 3D, corner coordinates and cell-local outputs");
  a.evin = evin;
  a.Xcell = Xcell;
  MFS_REQUIRE(what >= 0 && what <= 2, MFS_EINVAL, "launch_ns: what = %d", what);
  if (pt) {
    MFS_REQUIRE(what == 0 && (evin == nullptr || pt->evhist != nullptr), MFS_EINVAL,
                "a general linearisation state needs the history (cell-local with evin)");
    a.point = 1;
    a.keep_delta = pt->keep_delta;
    a.evhist = pt->evhist;
  }
  a.colour = -1;
  a.nlaunch = (int)g.ncells;
  auto go = [&](const nsk::Args<T> &aa) {
#define NS_GO2(D, KK, C)                                                                                         \
  {                                                                                                              \
    using Sh = nsk::Shape<D, KK>;                                                                                \
    const int grid = (aa.nlaunch + Sh::CPB - 1) / Sh::CPB;                                                       \
    if (what == 0)                                                                                               \
      hipLaunchKernelGGL((nsk::ns_linearize_kernel<D, KK, T, C>), dim3(grid), dim3(Sh::BLOCK), 0, s, aa);        \
    else if (what == 1)                                                                                          \
      hipLaunchKernelGGL((nsk::ns_jacobian_kernel<D, KK, T, C, false>), dim3(grid), dim3(Sh::BLOCK), 0, s, aa);  \
    else                                                                                                         \
      hipLaunchKernelGGL((nsk::ns_jacobian_kernel<D, KK, T, C, true>), dim3(grid), dim3(Sh::BLOCK), 0, s, aa);   \
  }
#define NS_GO(D, KK)        \
  {                         \
    if (g.cart)             \
      NS_GO2(D, KK, true)   \
    else                    \
      NS_GO2(D, KK, false)  \
  }
    if (aa.nlaunch == 0) return;
    if (g.dim == 2) {
      if (g.k == 1) NS_GO(2, 1) else if (g.k == 2) NS_GO(2, 2) else if (g.k == 3) NS_GO(2, 3)
      else MFS_REQUIRE(false, MFS_EUNSUPPORTED, "Navier-Stokes degree %d", g.k);
    } else {
      if (g.k == 1) NS_GO(3, 1) else if (g.k == 2) NS_GO(3, 2) else if (g.k == 3) NS_GO(3, 3)
      else MFS_REQUIRE(false, MFS_EUNSUPPORTED, "Navier-Stokes degree %d", g.k);
    }
#undef NS_GO
#undef NS_GO2
  };
  if (what != 0 && ev == nullptr && g.dim == 3) {
    // atomic accumulation into the node grid (3D): one launch per cell
    // colour, in a fixed order, so that the result is deterministic
    for (int col = 0; col < 8; ++col) {
      nsk::Args<T> ac = a;
      const int px = col & 1, py = (col >> 1) & 1, pz = col >> 2;
      ac.colour = col;
      ac.cm0 = (g.n[0] - px + 1) / 2;
      ac.cm1 = (g.n[1] - py + 1) / 2;
      ac.nlaunch = ac.cm0 * ac.cm1 * ((g.n[2] - pz + 1) / 2);
      go(ac);
    }
  } else {
    go(a);
  }
  MFS_HIP(hipGetLastError());
}

template void launch_ns<double>(const LevelGeom &, const double *, const double *, int, double, double, int,
                                const double *, double *, double *, hipStream_t, double *, const double *,
                                const double *, const NsPoint<double> *);
template void launch_ns<float>(const LevelGeom &, const float *, const float *, int, float, float, int, const float *,
                               float *, float *, hipStream_t, float *, const float *, const float *,
                               const NsPoint<float> *);

namespace {

__global__ void k_ns_inject(int ncomp, int nf0, int nf1, int64_t Nf, int nc0, int nc1, int64_t Nc, const double *uf,
                            double *uc) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int64_t i = c % nc0, j = (c / nc0) % nc1, l = c / ((int64_t)nc0 * nc1);
  const int64_t f = 2 * i + (int64_t)nf0 * (2 * j + (int64_t)nf1 * 2 * l);
  for (int comp = 0; comp < ncomp; ++comp) uc[comp * Nc + c] = uf[comp * Nf + f];
}

__device__ __forceinline__ int node_color(const LevelGeom &g, int q, int64_t i) {
  const int64_t x = i % g.nv[0], y = (i / g.nv[0]) % g.nv[1], z = i / ((int64_t)g.nv[0] * g.nv[1]);
  return (int)(x % q) + q * ((int)(y % q) + q * (int)(z % q));
}

__global__ void k_color_indicator(LevelGeom g, int ncomp, int q, int color, int comp, double *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.Nv) return;
  const bool on = node_color(g, q, i) == color;
  for (int c = 0; c < ncomp; ++c) out[c * g.Nv + i] = (on && c == comp) ? 1.0 : 0.0;
}

__global__ void k_color_extract(LevelGeom g, int q, int color, int comp, const double *y, double *diag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.Nv) return;
  if (node_color(g, q, i) == color) diag[comp * g.Nv + i] = y[comp * g.Nv + i];
}

template <typename T>
__global__ void k_jacobi_relax(T *x, const T *b, const T *t, const T *invdiag, T omega, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += omega * invdiag[i] * (b[i] - t[i]);
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

}  // namespace

void launch_ns_inject(const LevelGeom &fine, const LevelGeom &coarse, const double *u_fine, double *u_coarse,
                      hipStream_t s, int ncomp) {
  for (int a = 0; a < fine.dim; ++a)
    MFS_REQUIRE(fine.nv[a] == 2 * coarse.nv[a] - 1, MFS_EUNSUPPORTED,
                "coarse nodes are not every second fine node (degree > 2)");
  if (ncomp <= 0) ncomp = fine.dim;
  hipLaunchKernelGGL(k_ns_inject, dim3((unsigned)((coarse.Nv + 255) / 256)), dim3(256), 0, s, ncomp, fine.nv[0],
                     fine.nv[1], fine.Nv, coarse.nv[0], coarse.nv[1], coarse.Nv, u_fine, u_coarse);
  MFS_HIP(hipGetLastError());
}

void launch_color_indicator(const LevelGeom &g, int ncomp, int q, int color, int comp, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_color_indicator, dim3((unsigned)((g.Nv + 255) / 256)), dim3(256), 0, s, g, ncomp, q, color,
                     comp, out);
  MFS_HIP(hipGetLastError());
}

void launch_color_extract(const LevelGeom &g, int q, int color, int comp, const double *y, double *diag,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_color_extract, dim3((unsigned)((g.Nv + 255) / 256)), dim3(256), 0, s, g, q, color, comp, y,
                     diag);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void jacobi_relax(T *x, const T *b, const T *t, const T *invdiag, T omega, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_jacobi_relax<T>, dim3(blocks_for(n)), dim3(256), 0, s, x, b, t, invdiag, omega, n);
  MFS_HIP(hipGetLastError());
}
template void jacobi_relax<double>(double *, const double *, const double *, const double *, double, int64_t,
                                   hipStream_t);
template void jacobi_relax<float>(float *, const float *, const float *, const float *, float, int64_t, hipStream_t);

}  // namespace mfs
