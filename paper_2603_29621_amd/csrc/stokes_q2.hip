// 3D degree-2 cell kernel: Stokes operator Q2/Q1 (and the velocity block A
// alone) on trilinear hexahedra, specialised for gfx950.
//
// Weak form: Sec. 1 eq. (stokes) in the symmetric block form of Sec. 3
// eq. (stokes_block): velocity rows nu (grad u, grad v) - (p, div v),
// pressure rows -(div u, q); Gauss quadrature with 3 points per direction.
//
// Work decomposition
//  * A workgroup owns a brick of BX x BY x BZ cells.  Its nodal velocity,
//    pressure and vertex values are loaded once into LDS with coalesced
//    row loads; the same LDS buffer later accumulates the brick's output.
//  * One thread per (cell, velocity component); a wave holds one component
//    of the brick's 64 cells.  The thread walks the three z-slabs of
//    quadrature points; within a slab every 1D contraction runs in
//    registers: z is contracted straight from the nodal values (values with
//    the basis S, z-derivatives with the derivative table DS), x and y by
//    sum factorisation and the collocation derivative on the Gauss points.
//    Only the divergence couples the components; each thread integrates its
//    own share of it against the pressure test functions.
//  * Geometry per point from the cell's 8 vertices: Jacobian columns (each
//    depends on the two other reference coordinates only), cofactor matrix,
//    determinant; no stored metric.
//  * The transposed sequence integrates the test functions; each thread adds
//    its nodal contributions into its component's slice of an LDS output
//    buffer (one wave per slice, lanes never collide within an instruction,
//    so the accumulation order is fixed), then the brick is written out:
//    nodes strictly inside the brick with plain stores, nodes on brick faces
//    into the brick's slot of a face buffer.  A second kernel sums the (at
//    most 8) face-buffer contributions of every brick-face node in a fixed
//    order and writes the Dirichlet rows (dst = src), so no global atomics
//    and no cleared destination are needed and the result is deterministic.
#include <algorithm>

#include "internal.h"

namespace mfs {

namespace q2 {

constexpr int BX = 8, BY = 4, BZ = 2;
constexpr int NCELL = BX * BY * BZ;  // 64
constexpr int NT = 3 * NCELL;        // 192 threads: (cell, slab)
constexpr int VX = 2 * BX + 1, VY = 2 * BY + 1, VZ = 2 * BZ + 1;
// LDS layout of a node row: the BX+1 even-x nodes first, then the BX odd-x
// nodes, so the cells of a wave (x stride 2 nodes) read consecutive slots; a
// row pitch of 20 slots puts the next cell row in y on the other half of the
// banks (conflict-free for 4- and 8-byte elements).
constexpr int RX = 20;
constexpr int RXY = RX * VY;  // 180
constexpr int NVB = RXY * VZ;  // 900 slots per component
__device__ __forceinline__ int xpos(int lx) { return (lx & 1) ? (BX + 1) + (lx >> 1) : (lx >> 1); }
constexpr int XOFF[3] = {0, BX + 1, 1};  // slot offsets of the cell's nodes 0, 1, 2 from its first node
constexpr int PX = BX + 1, PY = BY + 1, PZ = BZ + 1;
constexpr int NPB = PX * PY * PZ;  // pressure (and vertex) nodes per brick
constexpr int NVF = VX * VY * VZ;  // velocity nodes per brick and component (face buffer layout)
constexpr int FACE_PER_BRICK = 3 * NVF + NPB;

// Degree-2 tables as compile-time constants: 3-point Gauss rule on [0, 1],
// Lagrange bases on the GLL nodes {0, 1/2, 1} (velocity) and {0, 1}
// (pressure), and the collocation derivative on the Gauss points.
constexpr double csqrt(double v) {
  double r = v > 1 ? v : 1.0;
  for (int i = 0; i < 64; ++i) r = 0.5 * (r + v / r);
  return r;
}
struct Consts {
  double x[3], w[3];
  double S[3][3], D[3][3], DS[3][3], Sp[3][2];
  constexpr Consts() : x{}, w{}, S{}, D{}, DS{}, Sp{} {
    const double h = 0.5 * csqrt(0.6);
    x[0] = 0.5 - h;
    x[1] = 0.5;
    x[2] = 0.5 + h;
    w[0] = 5.0 / 18.0;
    w[1] = 8.0 / 18.0;
    w[2] = 5.0 / 18.0;
    const double nd[3] = {0.0, 0.5, 1.0};
    for (int q = 0; q < 3; ++q) {
      for (int n = 0; n < 3; ++n) {
        double v = 1.0, d = 0.0;
        for (int l = 0; l < 3; ++l) {
          if (l == n) continue;
          double term = 1.0 / (nd[n] - nd[l]);
          for (int m = 0; m < 3; ++m)
            if (m != n && m != l) term *= (x[q] - nd[m]) / (nd[n] - nd[m]);
          d += term;
          v *= (x[q] - nd[l]) / (nd[n] - nd[l]);
        }
        S[q][n] = v;
        DS[q][n] = d;
      }
      for (int p = 0; p < 3; ++p) {
        double d = 0.0;
        for (int l = 0; l < 3; ++l) {
          if (l == p) continue;
          double term = 1.0 / (x[p] - x[l]);
          for (int m = 0; m < 3; ++m)
            if (m != p && m != l) term *= (x[q] - x[m]) / (x[p] - x[m]);
          d += term;
        }
        D[q][p] = d;
      }
      Sp[q][0] = 1.0 - x[q];
      Sp[q][1] = x[q];
    }
  }
};
constexpr Consts KC{};

// typed access to the constants (folded at compile time)
template <typename T>
struct Tab {
  static constexpr T S(int q, int n) { return (T)KC.S[q][n]; }
  static constexpr T D(int q, int p) { return (T)KC.D[q][p]; }
  static constexpr T DS(int q, int n) { return (T)KC.DS[q][n]; }
  static constexpr T Sp(int q, int m) { return (T)KC.Sp[q][m]; }
  static constexpr T w(int q) { return (T)KC.w[q]; }
  static constexpr T x(int q) { return (T)KC.x[q]; }
};

template <typename T>
struct Args {
  int n0, n1, n2;
  int nv0, nv1, nv2;
  int np0, np1;
  int nbx, nby, nbz, nblocks;
  int64_t Nv;
  const T *X, *src_u, *src_p;
  T *dst_u, *dst_p;
  T *face;  // per brick: 3 x VX*VY*VZ velocity + PX*PY*PZ pressure partial sums (face nodes only)
  T nu;
  // fused Chebyshev step (Q2_CHEB): dst_u is the iterate x (== src_u)
  const T *cb, *cinv;
  T *cd;
  T c1, c2;
  int cfirst;
};

// Q2_A with the Chebyshev step in the output phase (library-internal mode)
constexpr int Q2_CHEB = 4;

// the Chebyshev step of one row: v = (A x)_j, xo = x_j
template <typename T>
__device__ __forceinline__ void cheb_row(const Args<T> &a, int64_t j, int64_t node, T v, T xo) {
  const T r = a.cinv[node] * (a.cb[j] - v);
  const T dn = a.cfirst ? a.c2 * r : a.c1 * a.cd[j] + a.c2 * r;
  a.cd[j] = dn;
  a.dst_u[j] = xo + dn;
}

// Accumulation into the LDS output slices.  Each slice belongs to one wave.
// FP64 uses the LDS atomic add.  FP32 uses plain read-modify-writes (the FP32
// LDS atomic is several times slower on gfx950), ordered so that no two lanes
// of the wave can touch the same node between two compiler barriers: the
// cells of a wave are 2 nodes apart per direction, so node offsets that agree
// on which coordinates equal 2 never collide across lanes.
template <typename T>
__device__ __forceinline__ void lds_acc(T *p, T v) {
  if constexpr (sizeof(T) == 8)
    atomicAdd(p, v);
  else
    *p += v;
}
template <typename T>
__device__ __forceinline__ void lds_batch_end() {
  if constexpr (sizeof(T) == 4) asm volatile("" ::: "memory");
}

// 1/d: hardware reciprocal refined by two Newton steps
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

// KM: Q2_STOKES (velocity rows A u + B p, pressure rows B^T u), Q2_A (A u),
// Q2_B (B p alone: no velocity input, no pressure output), Q2_MASSP (pressure
// mass matrix alone; wave c integrates z-slab c of every cell and the three
// partial sums meet in the pressure output)
// the work of brick b of a problem
template <typename T, int KM>
__device__ __forceinline__ void q2_brick(const Args<T> &a, const int b) {
  constexpr bool MASS = KM == Q2_MASSP;
  constexpr bool CHEB = KM == Q2_CHEB;
  constexpr bool PRES = KM != Q2_A && !CHEB;                     // pressure input
  constexpr bool VIN = KM == Q2_STOKES || KM == Q2_A || CHEB;    // velocity input
  constexpr bool POUT = KM == Q2_STOKES || MASS;         // pressure output
  constexpr bool VOUT = !MASS;                           // velocity output
  __shared__ T sU[3 * NVB];  // input velocity of the brick
  __shared__ T sO[3 * NVB];  // output velocity, one slice per component wave
  __shared__ T sP[NPB];      // input pressure
  __shared__ T sQ[3 * NPB];  // output pressure partials, one slice per component wave
  __shared__ T sX[3 * NPB];  // vertices

  // brick index; consecutive bricks share an XCD (round-robin dispatch over 8)
  const int bx = b % a.nbx, by = (b / a.nbx) % a.nby, bz = b / (a.nbx * a.nby);
  const int gx0 = 2 * BX * bx, gy0 = 2 * BY * by, gz0 = 2 * BZ * bz;
  const int tid = threadIdx.x;

  // ---- load the brick (velocity nodal values, pressure, vertices); clear outputs
  // Thread -> node (lx, ly) of a z-plane of the brick, planes (c, lz) in turn:
  // the node offsets are per-thread constants and the plane offsets uniform,
  // and every global load is issued before the first LDS store.
  constexpr int PLANE = VX * VY;  // 153 <= NT
  const bool pl_on = tid < PLANE;
  const int plx = tid % VX, ply = tid / VX;
  const int pgx = gx0 + plx, pgy = gy0 + ply;
  const bool xy_in = pl_on && pgx < a.nv0 && pgy < a.nv1;
  const bool xy_dir = pgx == 0 || pgy == 0 || pgx == a.nv0 - 1 || pgy == a.nv1 - 1;
  const int64_t xy_off = pgx + (int64_t)a.nv0 * pgy;
  const int lds_xy = xpos(plx) + RX * ply;
  const int64_t zstride = (int64_t)a.nv0 * a.nv1;
  {
    T vv[3 * VZ];
#pragma unroll
    for (int pl = 0; pl < 3 * VZ; ++pl) {
      const int c = pl / VZ, lz = pl % VZ;
      const int gz = gz0 + lz;
      T v = 0;
      if (VIN && xy_in && !xy_dir && gz > 0 && gz < a.nv2 - 1) v = a.src_u[c * a.Nv + zstride * gz + xy_off];
      vv[pl] = v;
    }
#pragma unroll
    for (int pl = 0; pl < 3 * VZ; ++pl) {
      const int c = pl / VZ, lz = pl % VZ;
      if (pl_on) {
        if (VIN) sU[c * NVB + RXY * lz + lds_xy] = vv[pl];
        if (VOUT) sO[c * NVB + RXY * lz + lds_xy] = 0;
      }
    }
  }
  for (int idx = tid; idx < NPB; idx += NT) {
    const int lx = idx % PX, ly = (idx / PX) % PY, lz = idx / (PX * PY);
    const int px = BX * bx + lx, py = BY * by + ly, pz = BZ * bz + lz;
    const bool in = px <= a.n0 && py <= a.n1 && pz <= a.n2;
    T pv = 0;
    if (PRES && in) pv = a.src_p[px + (int64_t)a.np0 * (py + (int64_t)a.np1 * pz)];
    sP[idx] = pv;
    sQ[idx] = 0;
    sQ[NPB + idx] = 0;
    sQ[2 * NPB + idx] = 0;
    for (int c = 0; c < 3; ++c)
      sX[3 * idx + c] = in ? a.X[3 * (px + (int64_t)(a.n0 + 1) * (py + (int64_t)(a.n1 + 1) * pz)) + c] : T(0);
  }
  __syncthreads();

  // ---- thread -> (component = wave, cell in brick = lane)
  const int c = __builtin_amdgcn_readfirstlane(tid / NCELL);
  const int e = tid % NCELL;
  const int ex = e % BX, ey = (e / BX) % BY, ez = e / (BX * BY);
  const int cx = BX * bx + ex, cy = BY * by + ey, cz = BZ * bz + ez;
  const bool valid = cx < a.n0 && cy < a.n1 && cz < a.n2;
  auto V = [&](int vx, int vy, int vz, int comp) -> T {
    return sX[3 * ((ex + vx) + PX * ((ey + vy) + PY * (ez + vz))) + comp];
  };
  // one-hot of the component (selects without branches)
  const T oh[3] = {T(c == 0), T(c == 1), T(c == 2)};
  const T *uc = &sU[c * NVB + ex + RX * 2 * ey + RXY * 2 * ez];
  T *oc = &sO[c * NVB + ex + RX * 2 * ey + RXY * 2 * ez];

#pragma unroll 1
  for (int sl = MASS ? c : 0; sl < (MASS ? c + 1 : 3); ++sl) {
    // re-read the nodal values from LDS in every slab instead of keeping all
    // 27 in registers across the loop (register budget: occupancy)
    asm volatile("" ::: "memory");
    // forward: reference gradient of component c at the 9 points of slab sl
    T g[3][9];
    if (VIN) {
      T za[9], zb[9];  // z-contracted nodal planes: values (S) and z-derivative (DS)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const T *col = uc + XOFF[i] + RX * j;
          const T u0 = col[0], u1 = col[RXY], u2 = col[2 * RXY];
          za[i + 3 * j] = Tab<T>::S(sl, 0) * u0 + Tab<T>::S(sl, 1) * u1 + Tab<T>::S(sl, 2) * u2;
          zb[i + 3 * j] = Tab<T>::DS(sl, 0) * u0 + Tab<T>::DS(sl, 1) * u1 + Tab<T>::DS(sl, 2) * u2;
        }
      T ya[9], yb[9];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          ya[i + 3 * q] = Tab<T>::S(q, 0) * za[i] + Tab<T>::S(q, 1) * za[i + 3] + Tab<T>::S(q, 2) * za[i + 6];
          yb[i + 3 * q] = Tab<T>::S(q, 0) * zb[i] + Tab<T>::S(q, 1) * zb[i + 3] + Tab<T>::S(q, 2) * zb[i + 6];
        }
      T uq[9];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          uq[q + 3 * j] = Tab<T>::S(q, 0) * ya[3 * j] + Tab<T>::S(q, 1) * ya[3 * j + 1] + Tab<T>::S(q, 2) * ya[3 * j + 2];
          g[2][q + 3 * j] = Tab<T>::S(q, 0) * yb[3 * j] + Tab<T>::S(q, 1) * yb[3 * j + 1] + Tab<T>::S(q, 2) * yb[3 * j + 2];
        }
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          g[0][i + 3 * j] = Tab<T>::D(i, 0) * uq[3 * j] + Tab<T>::D(i, 1) * uq[3 * j + 1] + Tab<T>::D(i, 2) * uq[3 * j + 2];
          g[1][i + 3 * j] = Tab<T>::D(j, 0) * uq[i] + Tab<T>::D(j, 1) * uq[i + 3] + Tab<T>::D(j, 2) * uq[i + 6];
        }
    }
    // pressure: z-contracted nodal plane of the slab (interpolated in x, y per point)
    T pz[4];
    if (PRES) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const T *col = &sP[(ex + i) + PX * ((ey + j) + PY * ez)];
          pz[i + 2 * j] = Tab<T>::Sp(sl, 0) * col[0] + Tab<T>::Sp(sl, 1) * col[PX * PY];
        }
    }

    // geometry: Jacobian columns d/dxi0 (depends on xi1), d/dxi1 (on xi0) at this
    // slab, d/dxi2 bilinear in (xi0, xi1)
    T a0[3], da[3], b0[3], db[3], c2[2][2][3];
    {
      const T s2 = Tab<T>::x(sl), m2 = T(1) - s2;
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        a0[comp] = m2 * (V(1, 0, 0, comp) - V(0, 0, 0, comp)) + s2 * (V(1, 0, 1, comp) - V(0, 0, 1, comp));
        da[comp] = m2 * (V(1, 1, 0, comp) - V(0, 1, 0, comp)) + s2 * (V(1, 1, 1, comp) - V(0, 1, 1, comp)) - a0[comp];
        b0[comp] = m2 * (V(0, 1, 0, comp) - V(0, 0, 0, comp)) + s2 * (V(0, 1, 1, comp) - V(0, 0, 1, comp));
        db[comp] = m2 * (V(1, 1, 0, comp) - V(1, 0, 0, comp)) + s2 * (V(1, 1, 1, comp) - V(1, 0, 1, comp)) - b0[comp];
#pragma unroll
        for (int vy = 0; vy < 2; ++vy)
#pragma unroll
          for (int vx = 0; vx < 2; ++vx) c2[vy][vx][comp] = V(vx, vy, 1, comp) - V(vx, vy, 0, comp);
      }
    }
    const T ws = Tab<T>::w(sl);
    // this component's share of the pressure test integrals -(div u, q):
    // accumulated per point into the 2x2 nodal plane of the slab
    T pacc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int q = i + 3 * j;
        const T s0 = Tab<T>::x(i), s1 = Tab<T>::x(j);
        T J0[3], J1[3], J2[3];
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
          J0[comp] = a0[comp] + s1 * da[comp];  // d x / d xi0 at xi1
          J1[comp] = b0[comp] + s0 * db[comp];  // d x / d xi1 at xi0
          const T lo = c2[0][0][comp] + s0 * (c2[0][1][comp] - c2[0][0][comp]);
          const T hi = c2[1][0][comp] + s0 * (c2[1][1][comp] - c2[1][0][comp]);
          J2[comp] = lo + s1 * (hi - lo);
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
        const T w = ws * Tab<T>::w(i) * Tab<T>::w(j);
        // z = adj^T ghat (= det * physical gradient of component c)
        T z[3] = {0, 0, 0};
        if (VIN) {
#pragma unroll
          for (int x = 0; x < 3; ++x) z[x] = A[0][x] * g[0][q] + A[1][x] * g[1][q] + A[2][x] * g[2][q];
        }
        T p = 0;
        if (PRES)
          p = Tab<T>::Sp(i, 0) * (Tab<T>::Sp(j, 0) * pz[0] + Tab<T>::Sp(j, 1) * pz[2]) +
              Tab<T>::Sp(i, 1) * (Tab<T>::Sp(j, 0) * pz[1] + Tab<T>::Sp(j, 1) * pz[3]);
        if (POUT) {
          // pressure test integrand: mass (p q det w) or this component's share of -(div u) q
          const T qa = MASS ? w * det * p : -w * (oh[0] * z[0] + oh[1] * z[1] + oh[2] * z[2]);
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) pacc[n + 2 * m] += (Tab<T>::Sp(i, n) * Tab<T>::Sp(j, m)) * qa;
        }
        if (VOUT) {
          T v[3] = {0, 0, 0};
          if (VIN) {
            const T nd = a.nu * recip(det);
#pragma unroll
            for (int x = 0; x < 3; ++x) v[x] = nd * z[x];
          }
          if (PRES) {
#pragma unroll
            for (int x = 0; x < 3; ++x) v[x] -= oh[x] * p;
          }
          // test-gradient coefficients: w * adj * v
#pragma unroll
          for (int bb = 0; bb < 3; ++bb) g[bb][q] = w * (A[bb][0] * v[0] + A[bb][1] * v[1] + A[bb][2] * v[2]);
        }
      }

    // backward: integrate against the test functions, add into the brick slice
    if (valid) {
      if (POUT) {
        // pressure cells are 1 node apart: one node offset per batch
#pragma unroll
        for (int lz = 0; lz < 2; ++lz)
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n) {
              lds_acc(&sQ[c * NPB + (ex + n) + PX * ((ey + m) + PY * (ez + lz))], Tab<T>::Sp(sl, lz) * pacc[n + 2 * m]);
              lds_batch_end<T>();
            }
      }
      if (!VOUT) continue;
      T r[9];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          r[i + 3 * j] = Tab<T>::D(0, i) * g[0][3 * j] + Tab<T>::D(1, i) * g[0][3 * j + 1] + Tab<T>::D(2, i) * g[0][3 * j + 2] +
                         Tab<T>::D(0, j) * g[1][i] + Tab<T>::D(1, j) * g[1][i + 3] + Tab<T>::D(2, j) * g[1][i + 6];
      T ra[9], rb[9];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          ra[n + 3 * j] = Tab<T>::S(0, n) * r[3 * j] + Tab<T>::S(1, n) * r[3 * j + 1] + Tab<T>::S(2, n) * r[3 * j + 2];
          rb[n + 3 * j] = Tab<T>::S(0, n) * g[2][3 * j] + Tab<T>::S(1, n) * g[2][3 * j + 1] + Tab<T>::S(2, n) * g[2][3 * j + 2];
        }
      T na[9], nb[9];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          na[n + 3 * m] = Tab<T>::S(0, m) * ra[n] + Tab<T>::S(1, m) * ra[n + 3] + Tab<T>::S(2, m) * ra[n + 6];
          nb[n + 3 * m] = Tab<T>::S(0, m) * rb[n] + Tab<T>::S(1, m) * rb[n + 3] + Tab<T>::S(2, m) * rb[n + 6];
        }
      T outv[27];
#pragma unroll
      for (int lz = 0; lz < 3; ++lz) {
        const T fa = Tab<T>::S(sl, lz), fb = Tab<T>::DS(sl, lz);
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
          for (int n = 0; n < 3; ++n) outv[n + 3 * m + 9 * lz] = fa * na[n + 3 * m] + fb * nb[n + 3 * m];
      }
      // batch by the set of coordinates equal to 2
#pragma unroll
      for (int bs = 0; bs < 8; ++bs) {
#pragma unroll
        for (int lz = 0; lz < 3; ++lz)
#pragma unroll
          for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int n = 0; n < 3; ++n)
              if (((n == 2) | ((m == 2) << 1) | ((lz == 2) << 2)) == bs)
                lds_acc(oc + XOFF[n] + RX * m + RXY * lz, outv[n + 3 * m + 9 * lz]);
        lds_batch_end<T>();
      }
    }
  }
  __syncthreads();

  // ---- write the brick: interior nodes to dst, face-node partial sums to the
  // brick's slot of the face buffer (summed by the combine kernel)
  T *fb = a.face + (int64_t)b * FACE_PER_BRICK;
  if (VOUT) {
    // same plane mapping as the load; Dirichlet rows and nodes outside the
    // mesh are left to the combine kernel
    const bool st_ok = pl_on && pgx > 0 && pgx < a.nv0 - 1 && pgy > 0 && pgy < a.nv1 - 1;
    const bool xy_int = plx > 0 && plx < VX - 1 && ply > 0 && ply < VY - 1;
#pragma unroll
    for (int pl = 0; pl < 3 * VZ; ++pl) {
      const int c = pl / VZ, lz = pl % VZ;
      const int gz = gz0 + lz;
      if (!st_ok || gz == 0 || gz >= a.nv2 - 1) continue;
      const T v = sO[c * NVB + RXY * lz + lds_xy];
      if (xy_int && lz > 0 && lz < VZ - 1) {
        const int64_t node = zstride * gz + xy_off;
        if (CHEB)
          cheb_row(a, c * a.Nv + node, node, v, sU[c * NVB + RXY * lz + lds_xy]);
        else
          a.dst_u[c * a.Nv + node] = v;
      } else
        fb[c * NVF + PLANE * lz + tid] = v;
    }
  }
  if (POUT)
    for (int idx = tid; idx < NPB; idx += NT) {
      const int lx = idx % PX, ly = (idx / PX) % PY, lz = idx / (PX * PY);
      const int px = BX * bx + lx, py = BY * by + ly, pz = BZ * bz + lz;
      if (px > a.n0 || py > a.n1 || pz > a.n2) continue;
      const T v = sQ[idx] + sQ[NPB + idx] + sQ[2 * NPB + idx];
      const bool inner = lx > 0 && lx < PX - 1 && ly > 0 && ly < PY - 1 && lz > 0 && lz < PZ - 1;
      if (inner)
        a.dst_p[px + (int64_t)a.np0 * (py + (int64_t)a.np1 * pz)] = v;
      else
        fb[3 * NVF + idx] = v;
    }
}

template <typename T, int KM>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) stokes_q2_kernel(Args<T> a) {
  // brick index; consecutive bricks share an XCD (round-robin dispatch over 8)
  int b = blockIdx.x;
  if (a.nblocks % 8 == 0) b = (b % 8) * (a.nblocks / 8) + b / 8;  // a bijection when 8 | nblocks
  q2_brick<T, KM>(a, b);
}

// Grouped launch over several problems (the brick kernel or the combine of
// each): block ranges [start[g], start[g+1]) belong to problem g
constexpr int MAXG = 16;
template <typename T>
struct Group {
  Args<T> a[MAXG];
  int start[MAXG + 1];
  int n;
};
__device__ __forceinline__ int group_of(const int *start, int n, int blk) {
  int g = 0;
  while (g + 1 < n && blk >= start[g + 1]) ++g;
  return g;
}

template <typename T, int KM>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) stokes_q2_group_kernel(Group<T> G) {
  const int g = group_of(G.start, G.n, blockIdx.x);
  q2_brick<T, KM>(G.a[g], blockIdx.x - G.start[g]);
}

// Face nodes: sum the partials of every brick containing the node, in a fixed
// order (z, y, x brick index); Dirichlet rows: dst = src.
template <typename T, int KM>
__device__ __forceinline__ void q2_combine(const Args<T> &a, int64_t i) {
  constexpr bool POUT = KM == Q2_STOKES || KM == Q2_MASSP;
  if (KM != Q2_MASSP && i < a.Nv) {
    const int gx = (int)(i % a.nv0);
    const int64_t r = i / a.nv0;
    const int gy = (int)(r % a.nv1), gz = (int)(r / a.nv1);
    const bool dir = gx == 0 || gy == 0 || gz == 0 || gx == a.nv0 - 1 || gy == a.nv1 - 1 || gz == a.nv2 - 1;
    if (dir) {
      if (KM != Q2_CHEB)
#pragma unroll
        for (int c = 0; c < 3; ++c) a.dst_u[c * a.Nv + i] = KM != Q2_B ? a.src_u[c * a.Nv + i] : T(0);
    } else if (gx % (2 * BX) == 0 || gy % (2 * BY) == 0 || gz % (2 * BZ) == 0) {
      int bxs[2], bys[2], bzs[2], nxs = 0, nys = 0, nzs = 0;
      auto bricks = [](int g, int B2, int nb, int *out, int &cnt) {
        const int b0 = g / B2;
        if (g % B2 == 0 && b0 >= 1) out[cnt++] = b0 - 1;
        if (b0 < nb) out[cnt++] = b0;
      };
      bricks(gz, 2 * BZ, a.nbz, bzs, nzs);
      bricks(gy, 2 * BY, a.nby, bys, nys);
      bricks(gx, 2 * BX, a.nbx, bxs, nxs);
      T acc[3] = {0, 0, 0};
      for (int z = 0; z < nzs; ++z)
        for (int y = 0; y < nys; ++y)
          for (int x = 0; x < nxs; ++x) {
            const int lb = bxs[x] + a.nbx * (bys[y] + a.nby * bzs[z]);
            const T *fb = a.face + (int64_t)lb * FACE_PER_BRICK;
            const int l = (gx - 2 * BX * bxs[x]) + VX * ((gy - 2 * BY * bys[y]) + VY * (gz - 2 * BZ * bzs[z]));
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += fb[c * NVF + l];
          }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (KM == Q2_CHEB)
          cheb_row(a, c * a.Nv + i, i, acc[c], a.src_u[c * a.Nv + i]);
        else
          a.dst_u[c * a.Nv + i] = acc[c];
      }
    }
  }
  if (POUT) {
    const int64_t Np = (int64_t)a.np0 * a.np1 * (a.n2 + 1);
    if (i < Np) {
      const int px = (int)(i % a.np0);
      const int64_t r = i / a.np0;
      const int py = (int)(r % a.np1), pz = (int)(r / a.np1);
      if (px % BX == 0 || py % BY == 0 || pz % BZ == 0) {
        int bxs[2], bys[2], bzs[2], nxs = 0, nys = 0, nzs = 0;
        auto bricks = [](int g, int B, int nb, int *out, int &cnt) {
          const int b0 = g / B;
          if (g % B == 0 && b0 >= 1) out[cnt++] = b0 - 1;
          if (b0 < nb) out[cnt++] = b0;
        };
        bricks(pz, BZ, a.nbz, bzs, nzs);
        bricks(py, BY, a.nby, bys, nys);
        bricks(px, BX, a.nbx, bxs, nxs);
        T acc = 0;
        for (int z = 0; z < nzs; ++z)
          for (int y = 0; y < nys; ++y)
            for (int x = 0; x < nxs; ++x) {
              const int lb = bxs[x] + a.nbx * (bys[y] + a.nby * bzs[z]);
              const T *fb = a.face + (int64_t)lb * FACE_PER_BRICK + 3 * NVF;
              acc += fb[(px - BX * bxs[x]) + PX * ((py - BY * bys[y]) + PY * (pz - BZ * bzs[z]))];
            }
        a.dst_p[i] = acc;
      }
    }
  }
}

template <typename T, int KM>
__global__ void __launch_bounds__(256) q2_combine_kernel(Args<T> a) {
  q2_combine<T, KM>(a, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

template <typename T, int KM>
__global__ void __launch_bounds__(256) q2_combine_group_kernel(Group<T> G) {
  const int g = group_of(G.start, G.n, blockIdx.x);
  q2_combine<T, KM>(G.a[g], (blockIdx.x - G.start[g]) * (int64_t)blockDim.x + threadIdx.x);
}

}  // namespace q2

int64_t q2_face_elems(const LevelGeom &g) {
  if (g.dim != 3 || g.k != 2) return 0;
  const int64_t nb = (int64_t)((g.n[0] + q2::BX - 1) / q2::BX) * ((g.n[1] + q2::BY - 1) / q2::BY) *
                     ((g.n[2] + q2::BZ - 1) / q2::BZ);
  return nb * q2::FACE_PER_BRICK;
}

namespace {
template <typename T>
q2::Args<T> q2_args(const LevelGeom &g, const T *X, T nu, T *dst_u, T *dst_p, const T *src_u, const T *src_p,
                    T *face) {
  q2::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.np0 = g.n[0] + 1;
  a.np1 = g.n[1] + 1;
  a.nbx = (g.n[0] + q2::BX - 1) / q2::BX;
  a.nby = (g.n[1] + q2::BY - 1) / q2::BY;
  a.nbz = (g.n[2] + q2::BZ - 1) / q2::BZ;
  a.nblocks = a.nbx * a.nby * a.nbz;
  a.Nv = g.Nv;
  a.X = X;
  a.src_u = src_u;
  a.src_p = src_p;
  a.dst_u = dst_u;
  a.dst_p = dst_p;
  a.face = face;
  a.nu = nu;
  return a;
}
}  // namespace

template <typename T>
void launch_stokes_q2_group(const Q2Problem<T> *probs, int n, hipStream_t s) {
  for (int first = 0; first < n; first += q2::MAXG) {
    const int cnt = std::min(q2::MAXG, n - first);
    q2::Group<T> G{};
    q2::Group<T> C{};
    G.n = C.n = cnt;
    int nb = 0, nc = 0;
    for (int j = 0; j < cnt; ++j) {
      const Q2Problem<T> &p = probs[first + j];
      MFS_REQUIRE(p.g.dim == 3 && p.g.k == 2 && p.g.kp == 1 && p.face != nullptr, MFS_EINVAL,
                  "grouped Q2/Q1 Stokes launch needs 3D degree-2 Taylor-Hood levels");
      G.a[j] = C.a[j] = q2_args<T>(p.g, p.X, p.nu, p.dst, p.dst + 3 * p.g.Nv, p.src, p.src + 3 * p.g.Nv, p.face);
      G.start[j] = nb;
      C.start[j] = nc;
      nb += G.a[j].nblocks;
      nc += (int)((std::max<int64_t>(p.g.Nv, p.g.Np) + 255) / 256);
    }
    G.start[cnt] = nb;
    C.start[cnt] = nc;
    hipLaunchKernelGGL((q2::stokes_q2_group_kernel<T, Q2_STOKES>), dim3(nb), dim3(q2::NT), 0, s, G);
    hipLaunchKernelGGL((q2::q2_combine_group_kernel<T, Q2_STOKES>), dim3(nc), dim3(256), 0, s, C);
    MFS_HIP(hipGetLastError());
  }
}
template void launch_stokes_q2_group<double>(const Q2Problem<double> *, int, hipStream_t);
template void launch_stokes_q2_group<float>(const Q2Problem<float> *, int, hipStream_t);

template <typename T>
bool launch_stokes_q2(const LevelGeom &g, const T *X, int mode, T nu, T *dst_u, T *dst_p, const T *src_u,
                      const T *src_p, T *face, hipStream_t s) {
  if (g.dim != 3 || g.k != 2 || face == nullptr) return false;
  if (mode != Q2_A && g.kp != 1) return false;
  q2::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.np0 = g.n[0] + 1;
  a.np1 = g.n[1] + 1;
  a.nbx = (g.n[0] + q2::BX - 1) / q2::BX;
  a.nby = (g.n[1] + q2::BY - 1) / q2::BY;
  a.nbz = (g.n[2] + q2::BZ - 1) / q2::BZ;
  a.nblocks = a.nbx * a.nby * a.nbz;
  a.Nv = g.Nv;
  a.X = X;
  a.src_u = src_u;
  a.src_p = src_p;
  a.dst_u = dst_u;
  a.dst_p = dst_p;
  a.face = face;
  a.nu = nu;
  const int64_t nthreads = mode == Q2_STOKES ? std::max<int64_t>(g.Nv, g.Np) : (mode == Q2_MASSP ? g.Np : g.Nv);
  const unsigned cgrid = (unsigned)((nthreads + 255) / 256);
#define Q2_GO(KM)                                                                                       \
  hipLaunchKernelGGL((q2::stokes_q2_kernel<T, KM>), dim3(a.nblocks), dim3(q2::NT), 0, s, a);            \
  hipLaunchKernelGGL((q2::q2_combine_kernel<T, KM>), dim3(cgrid), dim3(256), 0, s, a);
  if (mode == Q2_STOKES) {
    Q2_GO(Q2_STOKES)
  } else if (mode == Q2_MASSP) {
    Q2_GO(Q2_MASSP)
  } else if (mode == Q2_B) {
    Q2_GO(Q2_B)
  } else {
    Q2_GO(Q2_A)
  }
#undef Q2_GO
  MFS_HIP(hipGetLastError());
  return true;
}

template <typename T>
bool launch_q2_cheb(const LevelGeom &g, const T *X, T nu, T *x, T *d, const T *b, const T *inv, T c1, T c2,
                    bool first, T *face, hipStream_t s) {
  if (g.dim != 3 || g.k != 2 || face == nullptr) return false;
  q2::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.np0 = g.n[0] + 1;
  a.np1 = g.n[1] + 1;
  a.nbx = (g.n[0] + q2::BX - 1) / q2::BX;
  a.nby = (g.n[1] + q2::BY - 1) / q2::BY;
  a.nbz = (g.n[2] + q2::BZ - 1) / q2::BZ;
  a.nblocks = a.nbx * a.nby * a.nbz;
  a.Nv = g.Nv;
  a.X = X;
  a.src_u = x;
  a.dst_u = x;
  a.face = face;
  a.nu = nu;
  a.cb = b;
  a.cinv = inv;
  a.cd = d;
  a.c1 = c1;
  a.c2 = c2;
  a.cfirst = first ? 1 : 0;
  const unsigned cgrid = (unsigned)((g.Nv + 255) / 256);
  hipLaunchKernelGGL((q2::stokes_q2_kernel<T, q2::Q2_CHEB>), dim3(a.nblocks), dim3(q2::NT), 0, s, a);
  hipLaunchKernelGGL((q2::q2_combine_kernel<T, q2::Q2_CHEB>), dim3(cgrid), dim3(256), 0, s, a);
  MFS_HIP(hipGetLastError());
  return true;
}

template bool launch_q2_cheb<double>(const LevelGeom &, const double *, double, double *, double *, const double *,
                                     const double *, double, double, bool, double *, hipStream_t);
template bool launch_q2_cheb<float>(const LevelGeom &, const float *, float, float *, float *, const float *,
                                    const float *, float, float, bool, float *, hipStream_t);

template bool launch_stokes_q2<double>(const LevelGeom &, const double *, int, double, double *, double *,
                                       const double *, const double *, double *, hipStream_t);
template bool launch_stokes_q2<float>(const LevelGeom &, const float *, int, float, float *, float *, const float *,
                                      const float *, float *, hipStream_t);

}  // namespace mfs
