// 3D Taylor-Hood Stokes cell kernel for degrees k = 3, 4 with one thread per
// column of quadrature points.
//
// Weak form: Sec. 1 eq. (stokes) in the symmetric block form of Sec. 3
// eq. (stokes_block): velocity rows nu (grad u, grad v) - (p, div v),
// pressure rows -(div u, q), and the pressure mass (p, q) of the Schur
// complement approximation; Gauss quadrature with k+1 points per direction,
// velocity on the GLL nodes of degree k, pressure on those of degree k-1.
// Modes: the Stokes operator, the velocity block A (also on the p-levels of
// the velocity multigrid, which carry no pressure space), B, B^T and the
// pressure mass.
//
// Work decomposition
//  * Thread (cell, i, j), i, j < k+1: one column of points (or nodes) along
//    z.  Cells are packed per wavefront (sweeps synchronised at wavefront
//    scope) or, where that leaves many lanes idle, across the workgroup.
//  * Sum factorisation: the x and y contractions go through LDS (a thread
//    reads one row of k+1 values per output); the z contraction of a column
//    stays in registers.  Values, x- and y-derivatives come straight from the
//    nodal values (basis S, derivative DS at the Gauss points).
//  * Geometry once per point for all three velocity components: along a
//    column the z-column of the trilinear Jacobian is constant and the other
//    two are linear in z.
//  * The transposed sequence integrates; every thread writes its column of
//    nodal results into the cell-local arrays (cell_slot layout) that the
//    node gather sums in a fixed order (deterministic, no atomics).
#include "hp.h"
#include "internal.h"
#include <type_traits>

namespace mfs {
namespace col {

// ---- compile-time 1D tables on [0, 1]

// Legendre polynomial P_n and its derivative at t (three-term recurrence)
constexpr void legendre(int n, double t, double &p, double &dp) {
  double p0 = 1.0, p1 = t;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int m = 2; m <= n; ++m) {
    const double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (t * p1 - p0) / (t * t - 1.0);
}
// cos by its Taylor series after reduction to [-pi, pi] (initial guesses only)
constexpr double ccos(double x) {
  constexpr double pi = 3.14159265358979323846;
  while (x > pi) x -= 2 * pi;
  while (x < -pi) x += 2 * pi;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

template <int K>
struct Tab1 {
  static constexpr int Q = K + 1, M = K;
  double x[Q], w[Q];         // Gauss points and weights
  double S[Q][Q], DS[Q][Q];  // velocity basis (GLL nodes of degree K) and its derivative at the points
  double Sp[Q][M];           // pressure basis (GLL nodes of degree K-1) at the points
  constexpr Tab1() : x{}, w{}, S{}, DS{}, Sp{} {
    constexpr double pi = 3.14159265358979323846;
    // Gauss-Legendre rule on [-1, 1]: the roots of P_Q by Newton's method from
    // the usual cosine guesses; weights 2 / ((1 - t^2) P_Q'(t)^2)
    double gx[Q] = {}, gw[Q] = {};
    for (int i = 0; i < Q; ++i) {
      double t = -ccos(pi * (i + 0.75) / (Q + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p = 0, dp = 0;
        legendre(Q, t, p, dp);
        t -= p / dp;
      }
      double p = 0, dp = 0;
      legendre(Q, t, p, dp);
      gx[i] = t;
      gw[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    for (int q = 0; q < Q; ++q) {
      x[q] = 0.5 * (gx[q] + 1.0);
      w[q] = 0.5 * gw[q];
    }
    // GLL nodes of degree deg on [0, 1]: the end points and the roots of
    // P_deg' (Newton's method on P_deg' from the Chebyshev-Gauss-Lobatto
    // guesses, with P_deg'' from the Legendre equation)
    double nv[Q] = {}, np[M] = {};
    auto gll = [](int deg, double *out) {
      out[0] = 0.0;
      out[deg] = 1.0;
      for (int i = 1; i < deg; ++i) {
        double t = -ccos(pi * i / deg);
        for (int it = 0; it < 100; ++it) {
          double p = 0, dp = 0;
          legendre(deg, t, p, dp);
          const double d2p = (2.0 * t * dp - deg * (deg + 1) * p) / (1.0 - t * t);
          t -= dp / d2p;
        }
        out[i] = 0.5 * (t + 1.0);
      }
    };
    gll(K, nv);
    gll(K - 1, np);
    for (int q = 0; q < Q; ++q) {
      for (int n = 0; n < Q; ++n) {
        double v = 1.0, d = 0.0;
        for (int l = 0; l < Q; ++l) {
          if (l == n) continue;
          double term = 1.0 / (nv[n] - nv[l]);
          for (int m = 0; m < Q; ++m)
            if (m != n && m != l) term *= (x[q] - nv[m]) / (nv[n] - nv[m]);
          d += term;
          v *= (x[q] - nv[l]) / (nv[n] - nv[l]);
        }
        S[q][n] = v;
        DS[q][n] = d;
      }
      for (int m = 0; m < M; ++m) {
        double v = 1.0;
        for (int l = 0; l < M; ++l)
          if (l != m) v *= (x[q] - np[l]) / (np[m] - np[l]);
        Sp[q][m] = v;
      }
    }
  }
};

template <int K>
struct C {
  static constexpr Tab1<K> t{};
};

template <typename T>
struct Args {
  int n0, n1, n2, ncells;
  int nv0, nv1, nv2, np0, np1;
  int64_t Nv;
  const T *X, *src_u, *src_p;
  T *ev_u, *ev_p;
  T nu;
  // cell-local (E-vector) inputs and outputs of the cells of one degree class
  // of an hp space (EV kernels): node (i, j, l) of a cell at i + Q j + Q^2 l,
  // the three velocity components side by side
  const int *cells;
  const int64_t *off_u, *off_p;
  const T *in_u, *in_p;
  T *out_u, *out_p;
};

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/d: hardware reciprocal refined by Newton steps
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  float e = __builtin_fmaf(-d, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// Cells of a workgroup of 256 threads: packed per wavefront (a cell's
// (k+1)^2 columns never straddle two wavefronts, and the sweeps synchronise at
// wavefront scope), or packed across the workgroup with workgroup barriers
// where that keeps more lanes busy per CU within the LDS: k = 5 (7 cells in
// 252 lanes against 1 cell in 36 of every 64), and in FP32 k = 4 (10 cells in
// 250 lanes against 8 in 200) and k = 6 (5 in 245 against 4 in 196); in FP64
// the packed k = 4 and k = 6 cells' LDS would allow too few workgroups per CU.
template <int K, typename T>
struct Layout {
  static constexpr int Q2 = (K + 1) * (K + 1);
  static constexpr bool WAVE = !(K == 5 || (sizeof(T) == 4 && (K == 4 || K == 6)));
  static constexpr int CPW = 64 / Q2;
  static constexpr int CPB = WAVE ? 4 * CPW : 256 / Q2;
};

template <bool WAVE>
__device__ __forceinline__ void csync() {
  if constexpr (WAVE)
    wsync();
  else
    __syncthreads();
}

// Materialise a value in a register here: without it the compiler sinks a
// sweep's arithmetic to the distant use and keeps the loaded LDS operands
// live instead of the one result
template <typename T>
__device__ __forceinline__ void pin(T &v) {
  asm volatile("" : "+v"(v));
}

// LDS table layout (per-lane rows and columns are read from here)
constexpr int LT_S = 0, LT_DS = 64, LT_SP = 128, LT_X = 192, LT_W = 200, LT_SIZE = 208;  // [q * 8 + n]

// Per-cell LDS stride for n elements of T.  FP32: the smallest stride >= n
// that is 8 words past a multiple of 32 words, so that the (cell, j, i)
// stores and the (cell, i) row reads of a sweep spread evenly over the banks
// (k = 3 cell kernel 323 -> 281 us at 64^3).  FP64: one element of padding,
// which measured fewer conflicts for the 64-bit accesses than the FP32 rule
// (k = 4: 71 M against 155 M conflict cycles per dispatch).
template <typename T>
constexpr int pad_stride(int n) {
  if (sizeof(T) == 8) return n + 1;
  int s = n;
  while (s % 32 != 8) ++s;
  return s;
}

// occupancy target (waves per SIMD): FP64 3 (<= 168 registers), FP32 4
template <typename T, int K>
constexpr int waves_target() {
  return sizeof(T) == 8 ? (K <= 4 ? 3 : 2) : (K <= 4 ? 4 : 3);
}

// EV: cells of one hp degree class, E-vector inputs and outputs
template <int K, typename T, int MODE, bool EV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_target<T, K>()))) column_kernel(Args<T> a) {
  constexpr int Q = K + 1, M = K, Q2 = Q * Q, Q3 = Q2 * Q;
  using LY = Layout<K, T>;
  constexpr int CPB = LY::CPB;
  constexpr bool LAP = (MODE & M_LAPLACE) != 0, GRADP = (MODE & M_GRADP) != 0, DIVU = (MODE & M_DIVU) != 0;
  constexpr bool MASSP = (MODE & M_MASSP) != 0;
  constexpr bool NEED_U = LAP || DIVU, OUT_U = LAP || GRADP, NEED_P = GRADP || MASSP, OUT_P = DIVU || MASSP;
  constexpr const Tab1<K> &TB = C<K>::t;
  static_assert(Q2 <= 64, "a cell's columns fit in one wavefront");
  // per-cell arrays padded so that the cells of a wavefront start on
  // different LDS banks
  // (the pressure mass alone needs no velocity arrays and pressure-sized sweep results)
  constexpr bool VEL = NEED_U || OUT_U;
  constexpr int SU = pad_stride<T>(VEL ? 3 * Q3 : 1), SW = pad_stride<T>(VEL ? 2 * Q3 : M * Q2),
                SP = pad_stride<T>(M * Q2);
  __shared__ T s_tab[LT_SIZE];
  __shared__ T s_u[CPB][SU];  // nodal velocity; later the z-integrated test coefficients
  __shared__ T s_w[CPB][SW];  // results of an x or y sweep
  __shared__ T s_p[CPB][SP];  // nodal pressure; later pressure sweep results
  __shared__ T s_X[CPB][24];  // vertices

  const int tid = threadIdx.x;
  for (int i = tid; i < LT_SIZE; i += 256) {
    const int blk = i >> 6, r = (i >> 3) & 7, cc = i & 7;
    T v = 0;
    if (blk == 0 && r < Q && cc < Q) v = (T)TB.S[r][cc];
    if (blk == 1 && r < Q && cc < Q) v = (T)TB.DS[r][cc];
    if (blk == 2 && r < Q && cc < M) v = (T)TB.Sp[r][cc];
    if (i >= LT_X && i < LT_X + Q) v = (T)TB.x[i - LT_X];
    if (i >= LT_W && i < LT_W + Q) v = (T)TB.w[i - LT_W];
    s_tab[i] = v;
  }
  int e, t;
  bool active;
  if constexpr (LY::WAVE) {
    const int wv = tid >> 6, ln = tid & 63, sl = ln / Q2;
    active = sl < LY::CPW;
    e = wv * LY::CPW + (active ? sl : 0);
    t = active ? ln - sl * Q2 : 0;
  } else {
    active = tid < CPB * Q2;
    e = active ? tid / Q2 : CPB - 1;
    t = active ? tid - e * Q2 : 0;
  }
  const int ti = t % Q, tj = t / Q;
  const int lin = blockIdx.x * CPB + e;
  const bool valid = active && lin < a.ncells;
  const int cell = EV ? (valid ? a.cells[lin] : 0) : lin;
  int cx = 0, cy = 0, cz = 0;
  if (valid) {
    cx = cell % a.n0;
    const int r = cell / a.n0;
    cy = r % a.n1;
    cz = r / a.n1;
  }
  const int64_t ou = (EV && valid) ? a.off_u[cell] : 0, op = (EV && valid) ? a.off_p[cell] : 0;

  // ---- load: this thread's velocity column (zero on Dirichlet nodes),
  // pressure column, and a share of the cell's vertices
  const int gx = cx * K + ti, gy = cy * K + tj;
  const bool xy_dir = gx == 0 || gy == 0 || gx == a.nv0 - 1 || gy == a.nv1 - 1;
  const int64_t xy_off = gx + (int64_t)a.nv0 * gy, zstride = (int64_t)a.nv0 * a.nv1;
  T uv[3][Q];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const int gz = cz * K + l;
      T v = 0;
      if (EV) {
        if (NEED_U && valid) v = a.in_u[ou + 3 * (ti + Q * tj + Q2 * l) + c];
      } else if (NEED_U && valid && !xy_dir && gz > 0 && gz < a.nv2 - 1) {
        v = a.src_u[c * a.Nv + zstride * gz + xy_off];
      }
      uv[c][l] = v;
    }
  const bool pcol = ti < M && tj < M;
  T pv[M];
#pragma unroll
  for (int l = 0; l < M; ++l) {
    T v = 0;
    if (NEED_P && valid && pcol)
      v = EV ? a.in_p[op + ti + M * tj + M * M * l]
             : a.src_p[(cx * (K - 1) + ti) + (int64_t)a.np0 * ((cy * (K - 1) + tj) + (int64_t)a.np1 * (cz * (K - 1) + l))];
    pv[l] = v;
  }
  if (valid)
    for (int idx = t; idx < 24; idx += Q2) {
      const int v = idx / 3, comp = idx % 3;
      const int64_t vid = (cx + (v & 1)) + (int64_t)(a.n0 + 1) * ((cy + ((v >> 1) & 1)) + (int64_t)(a.n1 + 1) * (cz + (v >> 2)));
      s_X[e][idx] = a.X[3 * vid + comp];
    }
  if (active) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int l = 0; l < Q; ++l) s_u[e][c * Q3 + l * Q2 + tj * Q + ti] = uv[c][l];
    if (NEED_P && pcol)
#pragma unroll
      for (int l = 0; l < M; ++l) s_p[e][l * M * M + tj * M + ti] = pv[l];
  }
  __syncthreads();

  // per-lane 1D coefficients: rows (value / derivative at this thread's point
  // i or j) and columns (the basis function of node i or j at every point)
  const T *tS = s_tab + LT_S, *tD = s_tab + LT_DS, *tP = s_tab + LT_SP;

  // ---- forward: reference gradients of the 3 components along the column
  T g[3][3][Q];
  if (NEED_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      asm volatile("" ::: "memory");
      const T *uc = &s_u[e][c * Q3];
      T *wa = &s_w[e][0], *wb = &s_w[e][Q3];
      // x: values and x-derivatives at point i of node row (j, l)
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int n = 0; n < Q; ++n) {
          const T u = uc[l * Q2 + tj * Q + n];
          s0 += tS[ti * 8 + n] * u;
          s1 += tD[ti * 8 + n] * u;
        }
        if (active) {
          wa[l * Q2 + tj * Q + ti] = s0;
          wb[l * Q2 + tj * Q + ti] = s1;
        }
      }
      csync<LY::WAVE>();
      // y: at point (i, j) of node layer l: value, x-derivative, y-derivative
      T V[Q], Dx[Q], Dy[Q];
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        T v = 0, dx = 0, dy = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) {
          const T ta = wa[l * Q2 + m * Q + ti], tb = wb[l * Q2 + m * Q + ti];
          const T sy = tS[tj * 8 + m];
          v += sy * ta;
          dx += sy * tb;
          dy += tD[tj * 8 + m] * ta;
        }
        V[l] = v;
        Dx[l] = dx;
        Dy[l] = dy;
        pin(V[l]);
        pin(Dx[l]);
        pin(Dy[l]);
      }
      csync<LY::WAVE>();
      // z in registers
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int l = 0; l < Q; ++l) {
          const T sz = tS[qz * 8 + l];
          a0 += sz * Dx[l];
          a1 += sz * Dy[l];
          a2 += tD[qz * 8 + l] * V[l];
        }
        g[c][0][qz] = a0;
        g[c][1][qz] = a1;
        g[c][2][qz] = a2;
        pin(g[c][0][qz]);
        pin(g[c][1][qz]);
        pin(g[c][2][qz]);
      }
    }
  }
  // pressure values along the column
  T pq[Q];
  if (NEED_P) {
    // x: thread (i, j < M): point i of pressure node row (j, l)
    T *pw = &s_w[e][0];
    if (active && tj < M)
#pragma unroll
      for (int l = 0; l < M; ++l) {
        T s0 = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) s0 += tP[ti * 8 + m] * s_p[e][l * M * M + tj * M + m];
        pw[l * Q * M + tj * Q + ti] = s0;
      }
    csync<LY::WAVE>();
    T PV[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
      T s0 = 0;
#pragma unroll
      for (int m = 0; m < M; ++m) s0 += tP[tj * 8 + m] * pw[l * Q * M + m * Q + ti];
      PV[l] = s0;
      pin(PV[l]);
    }
    csync<LY::WAVE>();
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      T s0 = 0;
#pragma unroll
      for (int l = 0; l < M; ++l) s0 += tP[qz * 8 + l] * PV[l];
      pq[qz] = s0;
      pin(pq[qz]);
    }
  }

  // ---- points of the column: geometry once for all components
  T qv[Q];
  {
    const T x0 = s_tab[LT_X + ti], x1 = s_tab[LT_X + tj];
    const T wij = s_tab[LT_W + ti] * s_tab[LT_W + tj];
    auto V = [&](int vx, int vy, int vz, int comp) -> T { return s_X[e][3 * (vx + 2 * vy + 4 * vz) + comp]; };
    // d x / d xi0 = a0 + xi2 da (at xi1), d x / d xi1 = b0 + xi2 db (at xi0),
    // d x / d xi2 = J2 (bilinear in xi0, xi1, constant along the column)
    T a0[3], da[3], b0[3], db[3], J2[3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const T e00 = (T(1) - x1) * (V(1, 0, 0, comp) - V(0, 0, 0, comp)) + x1 * (V(1, 1, 0, comp) - V(0, 1, 0, comp));
      const T e01 = (T(1) - x1) * (V(1, 0, 1, comp) - V(0, 0, 1, comp)) + x1 * (V(1, 1, 1, comp) - V(0, 1, 1, comp));
      a0[comp] = e00;
      da[comp] = e01 - e00;
      const T f00 = (T(1) - x0) * (V(0, 1, 0, comp) - V(0, 0, 0, comp)) + x0 * (V(1, 1, 0, comp) - V(1, 0, 0, comp));
      const T f01 = (T(1) - x0) * (V(0, 1, 1, comp) - V(0, 0, 1, comp)) + x0 * (V(1, 1, 1, comp) - V(1, 0, 1, comp));
      b0[comp] = f00;
      db[comp] = f01 - f00;
      const T lo = (T(1) - x0) * (V(0, 0, 1, comp) - V(0, 0, 0, comp)) + x0 * (V(1, 0, 1, comp) - V(1, 0, 0, comp));
      const T hi = (T(1) - x0) * (V(0, 1, 1, comp) - V(0, 1, 0, comp)) + x0 * (V(1, 1, 1, comp) - V(1, 1, 0, comp));
      J2[comp] = lo + x1 * (hi - lo);
    }
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      asm volatile("" ::: "memory");
      const T x2 = s_tab[LT_X + qz];
      T J0[3], J1[3];
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        J0[comp] = a0[comp] + x2 * da[comp];
        J1[comp] = b0[comp] + x2 * db[comp];
      }
      // rows of adj(J) = det J * J^{-1}: J1 x J2, J2 x J0, J0 x J1
      T A[3][3];
      A[0][0] = J1[1] * J2[2] - J1[2] * J2[1];
      A[0][1] = J1[2] * J2[0] - J1[0] * J2[2];
      A[0][2] = J1[0] * J2[1] - J1[1] * J2[0];
      A[1][0] = J2[1] * J0[2] - J2[2] * J0[1];
      A[1][1] = J2[2] * J0[0] - J2[0] * J0[2];
      A[1][2] = J2[0] * J0[1] - J2[1] * J0[0];
      A[2][0] = J0[1] * J1[2] - J0[2] * J1[1];
      A[2][1] = J0[2] * J1[0] - J0[0] * J1[2];
      A[2][2] = J0[0] * J1[1] - J0[1] * J1[0];
      const T det = J0[0] * A[0][0] + J0[1] * A[0][1] + J0[2] * A[0][2];
      const T w = wij * s_tab[LT_W + qz];
      const T wnd = w * a.nu * recip(det);
      T div = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // z = adj^T ghat = det * physical gradient of component c
        T z[3] = {0, 0, 0};
        if (NEED_U) {
#pragma unroll
          for (int x = 0; x < 3; ++x) z[x] = A[0][x] * g[c][0][qz] + A[1][x] * g[c][1][qz] + A[2][x] * g[c][2][qz];
          div += z[c];
        }
        if (OUT_U) {
          T v[3];
#pragma unroll
          for (int x = 0; x < 3; ++x) v[x] = LAP ? wnd * z[x] : T(0);
          if (GRADP) v[c] -= w * pq[qz];
          // test-gradient coefficients adj * v
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            g[c][b][qz] = A[b][0] * v[0] + A[b][1] * v[1] + A[b][2] * v[2];
            pin(g[c][b][qz]);
          }
        }
      }
      qv[qz] = (DIVU ? -w * div : T(0)) + (MASSP ? w * det * pq[qz] : T(0));
      pin(qv[qz]);
    }
  }

  // ---- backward: integrate against the test functions, column by column
  // output slot of node (i, j, 0), component 0, and the strides to the next
  // component and node layer
  const int64_t row0 = EV ? ou + 3 * (ti + Q * tj) : cell_slot(a.n0, a.n1, 3, Q, cx, cy, cz, 0, ti, tj, 0);
  const int64_t cstride = EV ? 1 : cell_slot(a.n0, a.n1, 3, Q, cx, cy, cz, 1, ti, tj, 0) - row0;
  const int64_t lstride = EV ? 3 * Q2 : cell_slot(a.n0, a.n1, 3, Q, cx, cy, cz, 0, ti, tj, 1) - row0;
  T *const outu = EV ? a.out_u : a.ev_u;
  if (OUT_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      asm volatile("" ::: "memory");
      // z: test coefficients of x-derivative (S), y-derivative (S) and
      // z-derivative (DS) tests at node layer l
      T *z0 = &s_u[e][0], *z1 = &s_u[e][Q3], *z2 = &s_u[e][2 * Q3];
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) {
          const T sz = tS[qz * 8 + l];
          s0 += sz * g[c][0][qz];
          s1 += sz * g[c][1][qz];
          s2 += tD[qz * 8 + l] * g[c][2][qz];
        }
        if (active) {
          z0[l * Q2 + tj * Q + ti] = s0;
          z1[l * Q2 + tj * Q + ti] = s1;
          z2[l * Q2 + tj * Q + ti] = s2;
        }
      }
      csync<LY::WAVE>();
      // y transposed: thread (i, j) = (point i, node j)
      T *wx = &s_w[e][0], *ws = &s_w[e][Q3];
      T rx[Q], rs[Q];
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          const T sy = tS[qy * 8 + tj], dy = tD[qy * 8 + tj];
          s0 += sy * z0[l * Q2 + qy * Q + ti];
          s1 += dy * z1[l * Q2 + qy * Q + ti] + sy * z2[l * Q2 + qy * Q + ti];
        }
        rx[l] = s0;
        rs[l] = s1;
        pin(rx[l]);
        pin(rs[l]);
      }
      if (active)
#pragma unroll
        for (int l = 0; l < Q; ++l) {
          wx[l * Q2 + tj * Q + ti] = rx[l];
          ws[l * Q2 + tj * Q + ti] = rs[l];
        }
      csync<LY::WAVE>();
      // x transposed: thread (i, j) = node (i, j)
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        T r = 0;
#pragma unroll
        for (int qx = 0; qx < Q; ++qx)
          r += tD[qx * 8 + ti] * wx[l * Q2 + tj * Q + qx] + tS[qx * 8 + ti] * ws[l * Q2 + tj * Q + qx];
        if (valid) outu[row0 + c * cstride + l * lstride] = r;
      }
      csync<LY::WAVE>();
    }
  }
  if (OUT_P) {
    // pressure tests: z in registers, then y and x through LDS
    T *pz = &s_w[e][0], *py = &s_p[e][0];
    if (active)
#pragma unroll
      for (int l = 0; l < M; ++l) {
        T s0 = 0;
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) s0 += tP[qz * 8 + l] * qv[qz];
        pz[l * Q2 + tj * Q + ti] = s0;
      }
    csync<LY::WAVE>();
    if (active && tj < M)
#pragma unroll
      for (int l = 0; l < M; ++l) {
        T s0 = 0;
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) s0 += tP[qy * 8 + tj] * pz[l * Q2 + qy * Q + ti];
        py[l * Q * M + tj * Q + ti] = s0;
      }
    csync<LY::WAVE>();
    if (valid && pcol) {
      const int64_t p0 = EV ? op + ti + M * tj : cell_slot(a.n0, a.n1, 1, M, cx, cy, cz, 0, ti, tj, 0);
      const int64_t pl = EV ? M * M : cell_slot(a.n0, a.n1, 1, M, cx, cy, cz, 0, ti, tj, 1) - p0;
      T *const outp = EV ? a.out_p : a.ev_p;
#pragma unroll
      for (int l = 0; l < M; ++l) {
        T s0 = 0;
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) s0 += tP[qx * 8 + ti] * py[l * Q * M + tj * Q + qx];
        outp[p0 + l * pl] = s0;
      }
    }
  }
}

template <int K, typename T, int MODE, bool EV>
static void go(const Args<T> &a, hipStream_t s) {
  if (a.ncells == 0) return;
  constexpr int CPB = Layout<K, T>::CPB;
  const int grid = (a.ncells + CPB - 1) / CPB;
  hipLaunchKernelGGL((column_kernel<K, T, MODE, EV>), dim3(grid), dim3(256), 0, s, a);
}

template <int K, typename T, bool EV>
static bool go_mode(const Args<T> &a, int mode, hipStream_t s) {
  switch (mode) {
    case M_LAPLACE | M_GRADP | M_DIVU: go<K, T, M_LAPLACE | M_GRADP | M_DIVU, EV>(a, s); return true;
    case M_LAPLACE: go<K, T, M_LAPLACE, EV>(a, s); return true;
    case M_GRADP: go<K, T, M_GRADP, EV>(a, s); return true;
    case M_DIVU: go<K, T, M_DIVU, EV>(a, s); return true;
    case M_MASSP: go<K, T, M_MASSP, EV>(a, s); return true;
    default: return false;
  }
}

template <typename T, bool EV>
static bool go_k(int k, const Args<T> &a, int mode, hipStream_t s) {
  if constexpr (!EV) {
    if (k == 3) return go_mode<3, T, EV>(a, mode, s);
  }
  if constexpr (!EV || std::is_same_v<T, float>) {
    if (k == 4) return go_mode<4, T, EV>(a, mode, s);
  }
  switch (k) {
    case 5: return go_mode<5, T, EV>(a, mode, s);
    case 6: return go_mode<6, T, EV>(a, mode, s);
    default: return false;
  }
}

}  // namespace col

template <typename T>
bool launch_column_cells(const LevelGeom &g, const T *X, int mode, T nu, const T *src_u, const T *src_p, T *ev_u,
                         T *ev_p, hipStream_t s) {
  // the velocity block alone also on levels without a pressure space
  const bool pres_ok = g.kp == g.k - 1 || (mode == M_LAPLACE && g.kp == 0);
  if (g.dim != 3 || g.k < 3 || g.k > 6 || !pres_ok || g.ncells == 0) return false;
  col::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.ncells = (int)g.ncells;
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.np0 = g.np[0];
  a.np1 = g.np[1];
  a.Nv = g.Nv;
  a.X = X;
  a.src_u = src_u;
  a.src_p = src_p;
  a.ev_u = ev_u;
  a.ev_p = ev_p;
  a.nu = nu;
  const bool ok = col::go_k<T, false>(g.k, a, mode, s);
  if (ok) MFS_HIP(hipGetLastError());
  return ok;
}
template <typename T>
bool launch_column_ev(const LevelGeom &g, int k, const T *X, int mode, T nu, const EvArgs<T> &ev, hipStream_t s) {
  // Degree classes of an hp mesh hold a few thousand cells.  At k = 3 (and
  // k = 4 in FP64) the column kernel then launches fewer waves than the chip
  // has slots (four and two cells per wave), and the generic kernel, one
  // thread per point, is the faster one; FP32 at k = 4 packs ten cells per
  // workgroup and from k = 5 on the column kernel wins at these sizes too.
  const int kmin = std::is_same_v<T, float> ? 4 : 5;
  if (g.dim != 3 || k < kmin || k > 6) return false;
  col::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.ncells = ev.ncells;
  a.X = X;
  a.nu = nu;
  a.cells = ev.cells;
  a.off_u = ev.off_u;
  a.off_p = ev.off_p;
  a.in_u = ev.in_u;
  a.in_p = ev.in_p;
  a.out_u = ev.out_u;
  a.out_p = ev.out_p;
  const bool ok = col::go_k<T, true>(k, a, mode, s);
  if (ok) MFS_HIP(hipGetLastError());
  return ok;
}
template bool launch_column_ev<double>(const LevelGeom &, int, const double *, int, double, const EvArgs<double> &,
                                       hipStream_t);
template bool launch_column_ev<float>(const LevelGeom &, int, const float *, int, float, const EvArgs<float> &,
                                      hipStream_t);
template bool launch_column_cells<double>(const LevelGeom &, const double *, int, double, const double *,
                                          const double *, double *, double *, hipStream_t);
template bool launch_column_cells<float>(const LevelGeom &, const float *, int, float, const float *, const float *,
                                         float *, float *, hipStream_t);

}  // namespace mfs
