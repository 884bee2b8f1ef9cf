// Device helpers shared by the cell kernels (sum-factorisation sweeps through
// LDS, Q1 geometry, per-cell thread context).  Internal to the library.
#pragma once

#include "internal.h"

namespace mfs {

// Thread layout: one thread per quadrature point.  When a cell's points fit
// in a wavefront (NQ <= 64) the cells are packed per wavefront (64 / NQ of
// them, the remaining lanes idle) and the LDS sweeps of a cell synchronise
// at wavefront scope only; larger cells span several wavefronts and use
// workgroup barriers.
template <int DIM, int K, int KP>
struct Shape {
  static constexpr int Q = K + 1;
  static constexpr int N = K + 1;
  static constexpr int M = KP + 1;
  static constexpr int NQ = DIM == 2 ? Q * Q : Q * Q * Q;
  static constexpr bool WAVE = NQ <= 64;
  static constexpr int CPW = WAVE ? 64 / NQ : 0;  // cells per wavefront
  static constexpr int CPB = WAVE ? 4 * CPW : (NQ >= 256 ? 1 : 256 / NQ);
  static constexpr int NT = WAVE ? 256 : CPB * NQ;
  static constexpr int BLOCK = WAVE ? 256 : (NT + 63) / 64 * 64;
  static constexpr int NV = 1 << DIM;
  // thread -> (cell e of the block, point t); inactive threads get a valid e
  __device__ static void map(int tid, int &e, int &t, bool &active) {
    if (WAVE) {
      const int w = tid >> 6, l = tid & 63, sl = l / NQ;
      active = sl < CPW;
      e = w * CPW + (active ? sl : 0);
      t = active ? l - sl * NQ : 0;
    } else {
      active = tid < NT;
      e = active ? tid / NQ : CPB - 1;
      t = active ? tid - e * NQ : 0;
    }
  }
};

// synchronisation of the threads of one cell between LDS sweeps
template <bool WAVE>
__device__ __forceinline__ void csync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Materialise a value in a register at this point of the program.  Values
// swept out of LDS are needed only after later sweeps; without this the
// compiler keeps the loaded operands live until the use instead of the one
// result (tens of extra registers per sweep, lower occupancy).
template <typename T>
__device__ __forceinline__ void pin(T &v) {
  asm volatile("" : "+v"(v));
}

// out = sum_m mat(r, m) in[.. m ..] along direction DIR; TR reads mat(m, r).
template <int DIM, int Q, int DIR, int C, bool TR, typename T>
__device__ __forceinline__ T sweep(const T *in, const T *mat, int qi, int qj, int ql) {
  const int r = DIR == 0 ? qi : (DIR == 1 ? qj : ql);
  const int base = DIR == 0 ? Q * (qj + Q * ql) : (DIR == 1 ? qi + Q * Q * ql : qi + Q * qj);
  constexpr int stride = DIR == 0 ? 1 : (DIR == 1 ? Q : Q * Q);
  T s = 0;
#pragma unroll
  for (int m = 0; m < C; ++m) {
    const T c = TR ? mat[m * MAXQ + r] : mat[r * MAXQ + m];
    s += c * in[base + m * stride];
  }
  return s;
}

// Q1 map: Jacobian J[a][b] = dx_a / dxi_b at reference point xi.
template <int DIM, typename T>
__device__ __forceinline__ void q1_jacobian(const T *Xc, const T xi[3], T J[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = 0;
#pragma unroll
  for (int v = 0; v < (1 << DIM); ++v) {
    T f[3], df[3];
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      const bool hi = (v >> b) & 1;
      f[b] = hi ? xi[b] : T(1) - xi[b];
      df[b] = hi ? T(1) : T(-1);
    }
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      T d = df[b];
#pragma unroll
      for (int c = 0; c < DIM; ++c)
        if (c != b) d *= f[c];
#pragma unroll
      for (int a = 0; a < DIM; ++a) J[a][b] += Xc[v * DIM + a] * d;
    }
  }
}

template <int DIM, typename T>
__device__ __forceinline__ T q1_point(const T *Xc, const T xi[3], int a) {
  T s = 0;
#pragma unroll
  for (int v = 0; v < (1 << DIM); ++v) {
    T f = 1;
#pragma unroll
    for (int b = 0; b < DIM; ++b) f *= ((v >> b) & 1) ? xi[b] : T(1) - xi[b];
    s += Xc[v * DIM + a] * f;
  }
  return s;
}

// inverse and determinant
template <int DIM, typename T>
__device__ __forceinline__ T invert(const T J[3][3], T I[3][3]) {
  if (DIM == 2) {
    const T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const T r = T(1) / det;
    I[0][0] = J[1][1] * r;
    I[0][1] = -J[0][1] * r;
    I[1][0] = -J[1][0] * r;
    I[1][1] = J[0][0] * r;
    return det;
  } else {
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
}

template <typename T>
__device__ __forceinline__ void atomic_add(T *p, T v) {
  unsafeAtomicAdd(p, v);
}

// Per-cell context shared by the kernels below.
template <int DIM, int K, int KP, typename T>
struct CellCtx {
  using Sh = Shape<DIM, K, KP>;
  static constexpr int Q = Sh::Q, N = Sh::N, M = Sh::M, NQ = Sh::NQ;
  int t, qi, qj, ql;
  int cx, cy, cz;
  bool valid, active;
  T *b0, *b1, *b2;
  const T *tab;
  // buffer i of this cell = bb + i * bstride (the batched sweeps below use
  // up to max(2, DIM) * NC of them; b0, b1, b2 are buffers 0, 1, 2)
  T *bb = nullptr;
  int bstride = 0;
  __device__ __forceinline__ T *buf(int i) const { return bb + i * bstride; }

  __device__ __forceinline__ bool vel_dirichlet(int nv0, int nv1, int nv2) const {
    const int gx = cx * K + qi, gy = cy * K + qj, gz = cz * K + ql;
    bool d = gx == 0 || gx == nv0 - 1 || gy == 0 || gy == nv1 - 1;
    if (DIM == 3) d = d || gz == 0 || gz == nv2 - 1;
    return d;
  }
  __device__ __forceinline__ int64_t vel_node(int nv0, int nv1) const {
    return (int64_t)(cx * K + qi) + (int64_t)nv0 * ((cy * K + qj) + (int64_t)nv1 * (cz * K + ql));
  }
  __device__ __forceinline__ bool p_local() const { return qi < M && qj < M && (DIM == 2 || ql < M); }
  __device__ __forceinline__ int64_t p_node(int np0, int np1) const {
    return (int64_t)(cx * KP + qi) + (int64_t)np0 * ((cy * KP + qj) + (int64_t)np1 * (cz * KP + ql));
  }

  // values at the Gauss points from nodal values in b0 (extent C per direction);
  // result returned and left in the returned buffer
  template <int C, int OFF>
  __device__ __forceinline__ const T *interpolate() {
    const T *S = tab + OFF;
    if (DIM == 2) {
      T v = sweep<DIM, Q, 0, C, false>(b0, S, qi, qj, ql);
      if (active) b1[t] = v;
      csync<Sh::WAVE>();
      v = sweep<DIM, Q, 1, C, false>(b1, S, qi, qj, ql);
      if (active) b0[t] = v;
      csync<Sh::WAVE>();
      return b0;
    } else {
      T v = sweep<DIM, Q, 0, C, false>(b0, S, qi, qj, ql);
      if (active) b1[t] = v;
      csync<Sh::WAVE>();
      v = sweep<DIM, Q, 1, C, false>(b1, S, qi, qj, ql);
      if (active) b0[t] = v;
      csync<Sh::WAVE>();
      v = sweep<DIM, Q, 2, C, false>(b0, S, qi, qj, ql);
      if (active) b1[t] = v;
      csync<Sh::WAVE>();
      return b1;
    }
  }
  // transposed interpolation of the point values in `in`; returns the nodal
  // value of this thread (meaningful when its indices are < C)
  template <int C, int OFF>
  __device__ __forceinline__ T integrate(T *in) {
    const T *S = tab + OFF;
    T *o = in == b0 ? b1 : b0;
    if (DIM == 2) {
      T v = sweep<DIM, Q, 1, Q, true>(in, S, qi, qj, ql);
      if (active) o[t] = v;
      csync<Sh::WAVE>();
      return sweep<DIM, Q, 0, Q, true>(o, S, qi, qj, ql);
    } else {
      T v = sweep<DIM, Q, 2, Q, true>(in, S, qi, qj, ql);
      if (active) o[t] = v;
      csync<Sh::WAVE>();
      v = sweep<DIM, Q, 1, Q, true>(o, S, qi, qj, ql);
      if (active) in[t] = v;
      csync<Sh::WAVE>();
      return sweep<DIM, Q, 0, Q, true>(in, S, qi, qj, ql);
    }
  }

  // reference gradient of component values (nodal, already in b0) at point t
  __device__ __forceinline__ void gradient(T g[3]) {
    const T *vals = interpolate<N, TAB_S>();
    const T *D = tab + TAB_D;
    g[0] = sweep<DIM, Q, 0, Q, false>(vals, D, qi, qj, ql);
    g[1] = sweep<DIM, Q, 1, Q, false>(vals, D, qi, qj, ql);
    if (DIM == 3) g[2] = sweep<DIM, Q, 2, Q, false>(vals, D, qi, qj, ql);
    pin(g[0]);
    pin(g[1]);
    if (DIM == 3) pin(g[2]);
    csync<Sh::WAVE>();
  }

  // Reference gradients of NC fields at point t.  On entry buffer i (i < NC)
  // holds the nodal values of field i and the caller has synchronised; the
  // fields pass through every sweep together, one synchronisation per pass.
  template <int NC>
  __device__ __forceinline__ void gradients(T g[][3]) {
    const T *S = tab + TAB_S, *D = tab + TAB_D;
    T v[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) v[i] = sweep<DIM, Q, 0, N, false>(buf(i), S, qi, qj, ql);
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (active) buf(NC + i)[t] = v[i];
    csync<Sh::WAVE>();
#pragma unroll
    for (int i = 0; i < NC; ++i) v[i] = sweep<DIM, Q, 1, N, false>(buf(NC + i), S, qi, qj, ql);
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (active) buf(i)[t] = v[i];
    csync<Sh::WAVE>();
    int vb = 0;  // buffer offset of the point values
    if (DIM == 3) {
#pragma unroll
      for (int i = 0; i < NC; ++i) v[i] = sweep<DIM, Q, 2, N, false>(buf(i), S, qi, qj, ql);
#pragma unroll
      for (int i = 0; i < NC; ++i)
        if (active) buf(NC + i)[t] = v[i];
      csync<Sh::WAVE>();
      vb = NC;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      g[i][0] = sweep<DIM, Q, 0, Q, false>(buf(vb + i), D, qi, qj, ql);
      g[i][1] = sweep<DIM, Q, 1, Q, false>(buf(vb + i), D, qi, qj, ql);
      if (DIM == 3) g[i][2] = sweep<DIM, Q, 2, Q, false>(buf(vb + i), D, qi, qj, ql);
      pin(g[i][0]);
      pin(g[i][1]);
      if (DIM == 3) pin(g[i][2]);
    }
    csync<Sh::WAVE>();
  }

  // Transposed: nodal results r[i] = sum_q f_i,b(q) d_b phi(q) of NC fields,
  // all fields per pass (buffers 0 .. DIM*NC-1)
  template <int NC>
  __device__ __forceinline__ void integrate_gradients(const T f[][3], T r[]) {
    const T *S = tab + TAB_S, *D = tab + TAB_D;
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
      for (int b = 0; b < DIM; ++b)
        if (active) buf(DIM * i + b)[t] = f[i][b];
    csync<Sh::WAVE>();
    T v[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      v[i] = sweep<DIM, Q, 0, Q, true>(buf(DIM * i), D, qi, qj, ql) +
             sweep<DIM, Q, 1, Q, true>(buf(DIM * i + 1), D, qi, qj, ql);
      if (DIM == 3) v[i] += sweep<DIM, Q, 2, Q, true>(buf(DIM * i + 2), D, qi, qj, ql);
      pin(v[i]);
    }
    csync<Sh::WAVE>();
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (active) buf(i)[t] = v[i];
    csync<Sh::WAVE>();
    int src = 0;
    if (DIM == 3) {
#pragma unroll
      for (int i = 0; i < NC; ++i) v[i] = sweep<DIM, Q, 2, Q, true>(buf(i), S, qi, qj, ql);
#pragma unroll
      for (int i = 0; i < NC; ++i)
        if (active) buf(NC + i)[t] = v[i];
      csync<Sh::WAVE>();
      src = NC;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) v[i] = sweep<DIM, Q, 1, Q, true>(buf(src + i), S, qi, qj, ql);
    const int dstb = src == 0 ? NC : 0;
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (active) buf(dstb + i)[t] = v[i];
    csync<Sh::WAVE>();
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      r[i] = sweep<DIM, Q, 0, Q, true>(buf(dstb + i), S, qi, qj, ql);
      pin(r[i]);
    }
    csync<Sh::WAVE>();
  }

  // test with reference gradients: sum_q f_b(q) d_b phi_i(q) -> nodal value
  __device__ __forceinline__ T integrate_gradient(const T f[3]) {
    if (active) {
      b0[t] = f[0];
      b1[t] = f[1];
      if (DIM == 3) b2[t] = f[2];
    }
    csync<Sh::WAVE>();
    const T *D = tab + TAB_D;
    T r = sweep<DIM, Q, 0, Q, true>(b0, D, qi, qj, ql) + sweep<DIM, Q, 1, Q, true>(b1, D, qi, qj, ql);
    if (DIM == 3) r += sweep<DIM, Q, 2, Q, true>(b2, D, qi, qj, ql);
    csync<Sh::WAVE>();
    if (active) b0[t] = r;
    csync<Sh::WAVE>();
    T v = integrate<N, TAB_S>(b0);
    csync<Sh::WAVE>();
    return v;
  }
};

}  // namespace mfs
