// 3D degree-1 cell kernel: the velocity block A = nu (grad u, grad v) of the
// Stokes operator (Sec. 1 eq. (stokes), velocity rows of Sec. 3
// eq. (stokes_block)) on trilinear hexahedra with the 2-point Gauss rule, for
// the degree-1 levels of the Stokes multigrid hierarchy.
//
// Work decomposition (the brick scheme of the degree-2 kernel):
//  * A workgroup owns a brick of 8 x 4 x 2 cells and 192 threads, one per
//    (cell, velocity component); wave c holds component c of the 64 cells.
//  * The brick's nodal velocity and vertex coordinates (the nodes of a
//    degree-1 level are the mesh vertices) are loaded into LDS by z-planes.
//    A row pitch of 40 slots puts the 8 x 4 cells of a half-wave on distinct
//    bank pairs.
//  * Each thread forms the edge differences of its cell's 8 nodal values and
//    vertex coordinates; at every Gauss point the reference gradient and the
//    Jacobian columns are bilinear interpolants of those differences.  The
//    cofactor matrix and determinant give w nu det J^{-1} J^{-T} grad u, which
//    is integrated against the test gradients in the same difference form.
//  * Accumulation into the wave's own component slice of an LDS output
//    buffer in 8 batches, one per local node offset (cells of a wave are one
//    node apart, so within a batch no two lanes touch the same node).
//  * Brick-interior nodes are stored directly, brick-face nodes go to the
//    brick's slot of a face buffer, and a second kernel sums the at most 8
//    contributions of each face node in a fixed order and writes the
//    Dirichlet rows (dst = src): deterministic, no global atomics.
#include <algorithm>

#include "internal.h"

namespace mfs {

namespace q1 {

constexpr int BX = 8, BY = 4, BZ = 2;
constexpr int NCELL = BX * BY * BZ;  // 64
constexpr int NT = 3 * NCELL;        // 192
constexpr int VX = BX + 1, VY = BY + 1, VZ = BZ + 1;
constexpr int RX = 40, RXY = RX * VY, NVB = RXY * VZ;  // LDS slots per component
constexpr int PLANE = VX * VY;                         // nodes of a z-plane of the brick
constexpr int NVF = PLANE * VZ;                        // nodes of the brick per component
constexpr int FACE_PER_BRICK = 3 * NVF;

template <typename T>
struct Args {
  int n0, n1, n2;
  int nv0, nv1, nv2;
  int nbx, nby, nbz, nblocks;
  int64_t Nv;
  const T *X, *src;
  T *dst, *face;
  T nu;
  // fused Chebyshev step (CHEB kernels): dst is the iterate x (== src)
  const T *cb, *cinv;
  T *cd;
  T c1, c2;
  int cfirst;
};

// the Chebyshev step of one row: v = (A x)_j, xo = x_j
template <typename T>
__device__ __forceinline__ void cheb_row(const Args<T> &a, int64_t j, int64_t node, T v, T xo) {
  const T r = a.cinv[node] * (a.cb[j] - v);
  const T dn = a.cfirst ? a.c2 * r : a.c1 * a.cd[j] + a.c2 * r;
  a.cd[j] = dn;
  a.dst[j] = xo + dn;
}

// 2-point Gauss rule on [0, 1]: 1/2 -+ 1/(2 sqrt 3), weights 1/2
template <typename T>
struct G2 {
  static constexpr T x(int q) { return q == 0 ? T(0.21132486540518711775) : T(0.78867513459481288225); }
  // linear Lagrange basis on {0, 1} at Gauss point q: node 0 -> 1 - x, node 1 -> x
  static constexpr T phi(int q, int n) { return n == 0 ? T(1) - x(q) : x(q); }
};

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

// CHEB: A followed by one Chebyshev step (see launch_q1_cheb)
template <typename T, bool CHEB>
__global__ void __launch_bounds__(NT) laplace_q1_kernel(Args<T> a) {
  __shared__ T sU[3 * NVB];  // input velocity
  __shared__ T sO[3 * NVB];  // output velocity, one slice per component wave
  __shared__ T sX[3 * NVB];  // vertex coordinates, same layout

  int b = blockIdx.x;
  if (a.nblocks % 8 == 0) b = (b % 8) * (a.nblocks / 8) + b / 8;  // XCD-contiguous bricks
  const int bx = b % a.nbx, by = (b / a.nbx) % a.nby, bz = b / (a.nbx * a.nby);
  const int gx0 = BX * bx, gy0 = BY * by, gz0 = BZ * bz;
  const int tid = threadIdx.x;

  // ---- load by z-planes: thread -> node (x, y), planes (component, z)
  const bool pl_on = tid < PLANE;
  const int plx = tid % VX, ply = tid / VX;
  const int pgx = gx0 + plx, pgy = gy0 + ply;
  const bool xy_in = pl_on && pgx < a.nv0 && pgy < a.nv1;
  const bool xy_dir = pgx == 0 || pgy == 0 || pgx == a.nv0 - 1 || pgy == a.nv1 - 1;
  const int64_t xy_off = pgx + (int64_t)a.nv0 * pgy;
  const int lds_xy = plx + RX * ply;
  const int64_t zstride = (int64_t)a.nv0 * a.nv1;
  {
    T vv[3 * VZ], xv[3 * VZ];
#pragma unroll
    for (int pl = 0; pl < 3 * VZ; ++pl) {
      const int c = pl / VZ, lz = pl % VZ;
      const int gz = gz0 + lz;
      T v = 0, x = 0;
      if (xy_in && gz < a.nv2) {
        if (!xy_dir && gz > 0 && gz < a.nv2 - 1) v = a.src[c * a.Nv + zstride * gz + xy_off];
        x = a.X[3 * (zstride * gz + xy_off) + c];
      }
      vv[pl] = v;
      xv[pl] = x;
    }
#pragma unroll
    for (int pl = 0; pl < 3 * VZ; ++pl) {
      const int c = pl / VZ, lz = pl % VZ;
      if (pl_on) {
        sU[c * NVB + RXY * lz + lds_xy] = vv[pl];
        sO[c * NVB + RXY * lz + lds_xy] = 0;
        sX[c * NVB + RXY * lz + lds_xy] = xv[pl];
      }
    }
  }
  __syncthreads();

  // ---- thread -> (component = wave, cell = lane)
  const int c = __builtin_amdgcn_readfirstlane(tid / NCELL);
  const int e = tid % NCELL;
  const int ex = e % BX, ey = (e / BX) % BY, ez = e / (BX * BY);
  const bool valid = gx0 + ex < a.n0 && gy0 + ey < a.n1 && gz0 + ez < a.n2;
  const int base = ex + RX * ey + RXY * ez;
  if (valid) {
    // edge differences of the nodal values (d/dxi_0 along x-edges (j, l), ...)
    T ux[4], uy[4], uz[4];
    T Xx[3][4], Xy[3][4], Xz[3][4];
    {
      const T *u = &sU[c * NVB + base];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          ux[p + 2 * q] = u[1 + RX * p + RXY * q] - u[RX * p + RXY * q];
          uy[p + 2 * q] = u[p + RX + RXY * q] - u[p + RXY * q];
          uz[p + 2 * q] = u[p + RX * q + RXY] - u[p + RX * q];
        }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T *x = &sX[d * NVB + base];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            Xx[d][p + 2 * q] = x[1 + RX * p + RXY * q] - x[RX * p + RXY * q];
            Xy[d][p + 2 * q] = x[p + RX + RXY * q] - x[p + RXY * q];
            Xz[d][p + 2 * q] = x[p + RX * q + RXY] - x[p + RX * q];
          }
      }
    }
    // test-gradient integrals in difference form
    T A0[4] = {0, 0, 0, 0}, A1[4] = {0, 0, 0, 0}, A2[4] = {0, 0, 0, 0};
    const T wnu = T(0.125) * a.nu;
#pragma unroll
    for (int ql = 0; ql < 2; ++ql)
#pragma unroll
      for (int qj = 0; qj < 2; ++qj)
#pragma unroll
        for (int qi = 0; qi < 2; ++qi) {
          // bilinear weights of the edge differences at this point
          T wyz[4], wxz[4], wxy[4];
#pragma unroll
          for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              wyz[p + 2 * q] = G2<T>::phi(qj, p) * G2<T>::phi(ql, q);
              wxz[p + 2 * q] = G2<T>::phi(qi, p) * G2<T>::phi(ql, q);
              wxy[p + 2 * q] = G2<T>::phi(qi, p) * G2<T>::phi(qj, q);
            }
          T g[3] = {0, 0, 0}, J0[3] = {0, 0, 0}, J1[3] = {0, 0, 0}, J2[3] = {0, 0, 0};
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            g[0] += wyz[r] * ux[r];
            g[1] += wxz[r] * uy[r];
            g[2] += wxy[r] * uz[r];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              J0[d] += wyz[r] * Xx[d][r];
              J1[d] += wxz[r] * Xy[d][r];
              J2[d] += wxy[r] * Xz[d][r];
            }
          }
          // rows of adj(J) = det J * J^{-1}
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
          const T nd = wnu * recip(det);
          T v[3];
#pragma unroll
          for (int x = 0; x < 3; ++x) v[x] = nd * (A[0][x] * g[0] + A[1][x] * g[1] + A[2][x] * g[2]);
          T f[3];
#pragma unroll
          for (int bb = 0; bb < 3; ++bb) f[bb] = A[bb][0] * v[0] + A[bb][1] * v[1] + A[bb][2] * v[2];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            A0[r] += wyz[r] * f[0];
            A1[r] += wxz[r] * f[1];
            A2[r] += wxy[r] * f[2];
          }
        }
    // node (i, j, l): d phi / d xi_0 = (2i - 1) phi_j phi_l, ...
    T *o = &sO[c * NVB + base];
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const T r = (i ? A0[j + 2 * l] : -A0[j + 2 * l]) + (j ? A1[i + 2 * l] : -A1[i + 2 * l]) +
                      (l ? A2[i + 2 * j] : -A2[i + 2 * j]);
          lds_acc(o + i + RX * j + RXY * l, r);
          lds_batch_end<T>();
        }
  }
  __syncthreads();

  // ---- store: interior nodes to dst, brick-face partial sums to the face buffer
  T *fb = a.face + (int64_t)b * FACE_PER_BRICK;
  const bool st_ok = pl_on && pgx > 0 && pgx < a.nv0 - 1 && pgy > 0 && pgy < a.nv1 - 1;
  const bool xy_int = plx > 0 && plx < VX - 1 && ply > 0 && ply < VY - 1;
#pragma unroll
  for (int pl = 0; pl < 3 * VZ; ++pl) {
    const int cc = pl / VZ, lz = pl % VZ;
    const int gz = gz0 + lz;
    if (!st_ok || gz == 0 || gz >= a.nv2 - 1) continue;
    const T v = sO[cc * NVB + RXY * lz + lds_xy];
    if (xy_int && lz > 0 && lz < VZ - 1) {
      const int64_t node = zstride * gz + xy_off;
      if (CHEB)
        cheb_row(a, cc * a.Nv + node, node, v, sU[cc * NVB + RXY * lz + lds_xy]);
      else
        a.dst[cc * a.Nv + node] = v;
    } else
      fb[cc * NVF + PLANE * lz + tid] = v;
  }
}

// Face nodes and Dirichlet rows, one workgroup per brick: a brick owns its
// nodes below its far faces (the last brick in a direction also its far
// face); an owned brick-face node sums the partials of every brick that
// contains it in a fixed order (z, y, x brick index); Dirichlet rows get
// dst = src.
template <typename T, bool CHEB>
__global__ void __launch_bounds__(256) q1_combine_kernel(Args<T> a) {
  const int b = blockIdx.x;
  const int bx = b % a.nbx, by = (b / a.nbx) % a.nby, bz = b / (a.nbx * a.nby);
  const bool lastx = bx == a.nbx - 1, lasty = by == a.nby - 1, lastz = bz == a.nbz - 1;
  for (int t = threadIdx.x; t < NVF; t += blockDim.x) {
    const int lx = t % VX, ly = (t / VX) % VY, lz = t / PLANE;
    if ((lx == VX - 1 && !lastx) || (ly == VY - 1 && !lasty) || (lz == VZ - 1 && !lastz)) continue;
    const int gx = BX * bx + lx, gy = BY * by + ly, gz = BZ * bz + lz;
    if (gx >= a.nv0 || gy >= a.nv1 || gz >= a.nv2) continue;
    const int64_t i = gx + (int64_t)a.nv0 * (gy + (int64_t)a.nv1 * gz);
    if (gx == 0 || gy == 0 || gz == 0 || gx == a.nv0 - 1 || gy == a.nv1 - 1 || gz == a.nv2 - 1) {
      if (!CHEB)
#pragma unroll
        for (int c = 0; c < 3; ++c) a.dst[c * a.Nv + i] = a.src[c * a.Nv + i];
      continue;
    }
    if (lx != 0 && ly != 0 && lz != 0) continue;  // brick interior: written by the cell kernel
    const int dz0 = (lz == 0) ? -1 : 0, dy0 = (ly == 0) ? -1 : 0, dx0 = (lx == 0) ? -1 : 0;
    T acc[3] = {0, 0, 0};
    for (int dz = dz0; dz <= 0; ++dz)
      for (int dy = dy0; dy <= 0; ++dy)
        for (int dx = dx0; dx <= 0; ++dx) {
          const int lb = (bx + dx) + a.nbx * ((by + dy) + a.nby * (bz + dz));
          const int l = (lx - dx * (VX - 1)) + VX * ((ly - dy * (VY - 1)) + VY * (lz - dz * (VZ - 1)));
          const T *fb = a.face + (int64_t)lb * FACE_PER_BRICK;
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[c] += fb[c * NVF + l];
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (CHEB)
        cheb_row(a, c * a.Nv + i, i, acc[c], a.src[c * a.Nv + i]);
      else
        a.dst[c * a.Nv + i] = acc[c];
    }
  }
}

}  // namespace q1

int64_t q1_face_elems(const LevelGeom &g) {
  if (g.dim != 3 || g.k != 1) return 0;
  const int64_t nb = (int64_t)((g.n[0] + q1::BX - 1) / q1::BX) * ((g.n[1] + q1::BY - 1) / q1::BY) *
                     ((g.n[2] + q1::BZ - 1) / q1::BZ);
  return nb * q1::FACE_PER_BRICK;
}

namespace {
template <typename T>
q1::Args<T> q1_args(const LevelGeom &g, const T *X, T nu, T *dst, const T *src, T *face) {
  q1::Args<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.n2 = g.n[2];
  a.nv0 = g.nv[0];
  a.nv1 = g.nv[1];
  a.nv2 = g.nv[2];
  a.nbx = (g.n[0] + q1::BX - 1) / q1::BX;
  a.nby = (g.n[1] + q1::BY - 1) / q1::BY;
  a.nbz = (g.n[2] + q1::BZ - 1) / q1::BZ;
  a.nblocks = a.nbx * a.nby * a.nbz;
  a.Nv = g.Nv;
  a.X = X;
  a.src = src;
  a.dst = dst;
  a.face = face;
  a.nu = nu;
  return a;
}
}  // namespace

template <typename T>
bool launch_laplace_q1(const LevelGeom &g, const T *X, T nu, T *dst, const T *src, T *face, hipStream_t s) {
  if (g.dim != 3 || g.k != 1 || face == nullptr) return false;
  const q1::Args<T> a = q1_args<T>(g, X, nu, dst, src, face);
  hipLaunchKernelGGL((q1::laplace_q1_kernel<T, false>), dim3(a.nblocks), dim3(q1::NT), 0, s, a);
  hipLaunchKernelGGL((q1::q1_combine_kernel<T, false>), dim3(a.nblocks), dim3(256), 0, s, a);
  MFS_HIP(hipGetLastError());
  return true;
}

template <typename T>
bool launch_q1_cheb(const LevelGeom &g, const T *X, T nu, T *x, T *d, const T *b, const T *inv, T c1, T c2,
                    bool first, T *face, hipStream_t s) {
  if (g.dim != 3 || g.k != 1 || face == nullptr) return false;
  q1::Args<T> a = q1_args<T>(g, X, nu, x, x, face);
  a.cb = b;
  a.cinv = inv;
  a.cd = d;
  a.c1 = c1;
  a.c2 = c2;
  a.cfirst = first ? 1 : 0;
  hipLaunchKernelGGL((q1::laplace_q1_kernel<T, true>), dim3(a.nblocks), dim3(q1::NT), 0, s, a);
  hipLaunchKernelGGL((q1::q1_combine_kernel<T, true>), dim3(a.nblocks), dim3(256), 0, s, a);
  MFS_HIP(hipGetLastError());
  return true;
}

template bool launch_q1_cheb<double>(const LevelGeom &, const double *, double, double *, double *, const double *,
                                     const double *, double, double, bool, double *, hipStream_t);
template bool launch_q1_cheb<float>(const LevelGeom &, const float *, float, float *, float *, const float *,
                                    const float *, float, float, bool, float *, hipStream_t);

template bool launch_laplace_q1<double>(const LevelGeom &, const double *, double, double *, const double *, double *,
                                        hipStream_t);
template bool launch_laplace_q1<float>(const LevelGeom &, const float *, float, float *, const float *, float *,
                                       hipStream_t);

}  // namespace mfs
