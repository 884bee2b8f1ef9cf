// Vector kernels: fills, casts, axpy, Jacobi scaling, the Chebyshev update,
// deterministic multi-vector dot products (fixed two-stage reduction order),
// multi-vector updates for Gram-Schmidt, the dense coarse-level solve and the
// device-resident scalar updates of the Schur PCG.
#include "internal.h"

namespace mfs {

namespace {
constexpr int VB = 256;
inline unsigned nblocks(int64_t n, int per = VB) {
  int64_t b = (n + per - 1) / per;
  if (b > 65535LL * 16) b = 65535LL * 16;
  return (unsigned)(b < 1 ? 1 : b);
}

__device__ __forceinline__ bool on_boundary(int dim, int nv0, int nv1, int nv2, int64_t i) {
  const int gx = (int)(i % nv0);
  const int64_t r = i / nv0;
  const int gy = (int)(r % nv1);
  const int gz = (int)(r / nv1);
  bool d = gx == 0 || gx == nv0 - 1 || gy == 0 || gy == nv1 - 1;
  if (dim == 3) d = d || gz == 0 || gz == nv2 - 1;
  return d;
}
}  // namespace

template <typename T>
__global__ void k_fill(T *x, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
template <typename T>
__global__ void k_copy(T *y, const T *x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}
template <typename T>
__global__ void k_axpby(T *y, T a, const T *x, T b, int64_t n) {
  // b == 0 never reads y (it may hold uninitialised memory)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b == T(0) ? a * x[i] : a * x[i] + b * y[i];
}
template <typename TO, typename TI>
__global__ void k_cast(TO *y, const TI *x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (TO)x[i];
}

template <typename T>
void vec_fill(T *x, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(nblocks(n)), dim3(VB), 0, s, x, v, n);
}
template <typename T>
void vec_copy(T *y, const T *x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3(nblocks(n)), dim3(VB), 0, s, y, x, n);
}
template <typename T>
void vec_axpby(T *y, T a, const T *x, T b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby<T>, dim3(nblocks(n)), dim3(VB), 0, s, y, a, x, b, n);
}
template <typename TO, typename TI>
void vec_cast(TO *y, const TI *x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_cast<TO, TI>), dim3(nblocks(n)), dim3(VB), 0, s, y, x, n);
}

// stage mixing of stage-major vectors (space-time operators, Sec. 4):
// y_i[e] = a y_i[e] + sum_j C[i][j] x_j[e] for e < ne (ldx, ldy: stage
// strides), and y_i[e] *= a for ne <= e < ny (the rows without a mixed term)
template <typename T>
__global__ void k_stage_mix(T *y, int64_t ldy, int no, const T *x, int64_t ldx, int ni, StageCoef C, T a, int64_t ne,
                            int64_t ny) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ny; e += (int64_t)gridDim.x * blockDim.x) {
    T xv[MFS_MAX_STAGES];
    if (e < ne)
      for (int j = 0; j < ni; ++j) xv[j] = x[j * ldx + e];
    for (int i = 0; i < no; ++i) {
      T v = a == T(0) ? T(0) : a * y[i * ldy + e];
      if (e < ne)
        for (int j = 0; j < ni; ++j) v += (T)C.c[i * MFS_MAX_STAGES + j] * xv[j];
      y[i * ldy + e] = v;
    }
  }
}
template <typename T>
void stage_mix(T *y, int64_t ldy, int no, const T *x, int64_t ldx, int ni, const StageCoef &C, T a, int64_t ne,
               int64_t ny, hipStream_t s) {
  if (ny <= 0) return;
  hipLaunchKernelGGL(k_stage_mix<T>, dim3(nblocks(ny)), dim3(VB), 0, s, y, ldy, no, x, ldx, ni, C, a, ne, ny);
}
template void stage_mix<double>(double *, int64_t, int, const double *, int64_t, int, const StageCoef &, double,
                                int64_t, int64_t, hipStream_t);
template void stage_mix<float>(float *, int64_t, int, const float *, int64_t, int, const StageCoef &, float, int64_t,
                               int64_t, hipStream_t);

template <typename T>
__global__ void k_zero_boundary(int dim, int nv0, int nv1, int nv2, int64_t Nv, T *u) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Nv || !on_boundary(dim, nv0, nv1, nv2, i)) return;
  for (int c = 0; c < dim; ++c) u[c * Nv + i] = 0;
}
template <typename T>
void vec_zero_mask_boundary(const LevelGeom &g, T *u, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_boundary<T>, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv,
                     u);
}

template <typename T>
__global__ void k_copy_boundary(int dim, int nv0, int nv1, int nv2, int64_t Nv, T *u, const T *src) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Nv || !on_boundary(dim, nv0, nv1, nv2, i)) return;
  for (int c = 0; c < dim; ++c) u[c * Nv + i] = src[c * Nv + i];
}
template <typename T>
void vec_copy_boundary(const LevelGeom &g, T *u, const T *src, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_boundary<T>, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv,
                     u, src);
}

template <typename T>
__global__ void k_diag_scale(int dim, int nv0, int nv1, int nv2, int64_t Nv, T *y, const T *inv, const T *x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Nv) return;
  const bool d = on_boundary(dim, nv0, nv1, nv2, i);
  for (int c = 0; c < dim; ++c) y[c * Nv + i] = d ? T(0) : inv[i] * x[c * Nv + i];
}
template <typename T>
void vec_diag_scale(const LevelGeom &g, T *y, const T *invdiag, const T *x, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_scale<T>, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv, y,
                     invdiag, x);
}

__global__ void k_invert_diag(int dim, int nv0, int nv1, int nv2, int64_t Nv, const double *d, double *i64,
                              float *i32) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Nv) return;
  const double v = on_boundary(dim, nv0, nv1, nv2, i) ? 1.0 : 1.0 / d[i];
  i64[i] = v;
  i32[i] = (float)v;
}
void vec_invert_diag(const LevelGeom &g, const double *diag, double *i64, float *i32, hipStream_t s) {
  hipLaunchKernelGGL(k_invert_diag, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv, diag,
                     i64, i32);
}

// Chebyshev step.  Free rows: r = invdiag (b - Ax) (Ax = 0 when null),
// d = c1 d + c2 r (d = c2 r on the first step), x += d.  Dirichlet rows keep x.
template <typename T>
__global__ void k_cheb(int dim, int nv0, int nv1, int nv2, int64_t Nv, T *x, T *d, const T *b, const T *Ax,
                       const T *inv, T c1, T c2, int first) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Nv || on_boundary(dim, nv0, nv1, nv2, i)) return;
  const T iv = inv[i];
  for (int c = 0; c < dim; ++c) {
    const int64_t j = c * Nv + i;
    const T r = iv * (b[j] - (Ax ? Ax[j] : T(0)));
    const T dn = first ? c2 * r : c1 * d[j] + c2 * r;
    d[j] = dn;
    x[j] += dn;
  }
}
// first step from x = 0: Dirichlet rows x = b; free rows d = c2 D^{-1} b, x = d
// (the operator vanishes there on x = 0 plus Dirichlet values, whose columns
// the constrained operator drops)
template <typename T>
__global__ void k_cheb_start(int dim, int nv0, int nv1, int nv2, int64_t Nv, T *x, T *d, const T *b, const T *inv,
                             T c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Nv) return;
  if (on_boundary(dim, nv0, nv1, nv2, i)) {
    for (int c = 0; c < dim; ++c) x[c * Nv + i] = b[c * Nv + i];
    return;
  }
  const T iv = inv[i];
  for (int c = 0; c < dim; ++c) {
    const int64_t j = c * Nv + i;
    const T dn = c2 * (iv * b[j]);
    d[j] = dn;
    x[j] = dn;
  }
}
template <typename T>
void cheb_start(const LevelGeom &g, T *x, T *d, const T *b, const T *invdiag, T c2, hipStream_t s) {
  hipLaunchKernelGGL(k_cheb_start<T>, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv, x, d,
                     b, invdiag, c2);
}
template void cheb_start<double>(const LevelGeom &, double *, double *, const double *, const double *, double,
                                 hipStream_t);
template void cheb_start<float>(const LevelGeom &, float *, float *, const float *, const float *, float, hipStream_t);

template <typename T>
void cheb_update(const LevelGeom &g, T *x, T *d, const T *b, const T *Ax, const T *invdiag, T c1, T c2, bool first,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_cheb<T>, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv, x, d, b,
                     Ax, invdiag, c1, c2, first ? 1 : 0);
}

// ------------------------------------------------------------ reductions
// Multi-vector kernels over the Krylov basis.  Every thread reads the same
// element of up to MM columns; the loads are unconditional (columns beyond m
// re-read column m - 1 and get coefficient 0), so all of them are in flight
// at once instead of one guarded load, and one wait, per column.
constexpr int MAXM = 32;

template <typename T, int MM>
__device__ __forceinline__ void load_cols(const T *V, int64_t ld, int m, int64_t j, double v[MM]) {
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    const int ii = i < m ? i : m - 1;
    v[i] = (double)V[ii * ld + j];
  }
}

// m coefficients from device memory into LDS, zero-padded to MAXM
__device__ __forceinline__ void load_coefs(double *sh, const double *h, int m) {
  if ((int)threadIdx.x < MAXM) sh[threadIdx.x] = (int)threadIdx.x < m ? h[threadIdx.x] : 0.0;
  __syncthreads();
}

// block tree reduction of per-thread values, written to partials[k * DOT_BLOCKS + block]
__device__ __forceinline__ void block_partial(double a, int k, double *partials, double *red) {
  red[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[k * DOT_BLOCKS + blockIdx.x] = red[0];
  __syncthreads();
}

template <typename T, int MM>
__global__ void __launch_bounds__(256) k_multi_dot_partial(const T *V, int64_t ld, int m, const T *w, int64_t n,
                                                           double *partials) {
  double acc[MM];
#pragma unroll
  for (int i = 0; i < MM; ++i) acc[i] = 0.0;
  // contiguous chunk per block: fixed summation order
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t beg = blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
    double v[MM];
    load_cols<T, MM>(V, ld, m, j, v);
    const double wj = (double)w[j];
#pragma unroll
    for (int i = 0; i < MM; ++i) acc[i] += v[i] * wj;
  }
  __shared__ double red[256];
#pragma unroll
  for (int i = 0; i < MM; ++i)
    if (i < m) block_partial(acc[i], i, partials, red);
}

__global__ void __launch_bounds__(256) k_multi_dot_final(const double *partials, int nb, double *out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double a = 0;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) a += partials[i * DOT_BLOCKS + j];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// column-group sizes the multi-vector kernels are instantiated for
#define MFS_MM_DISPATCH(m, KERNEL_LAUNCH) \
  do {                                    \
    if ((m) <= 1) {                       \
      constexpr int MM = 1;               \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 2) {                \
      constexpr int MM = 2;               \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 4) {                \
      constexpr int MM = 4;               \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 8) {                \
      constexpr int MM = 8;               \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 12) {               \
      constexpr int MM = 12;              \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 16) {               \
      constexpr int MM = 16;              \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 20) {               \
      constexpr int MM = 20;              \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 24) {               \
      constexpr int MM = 24;              \
      KERNEL_LAUNCH;                      \
    } else if ((m) <= 28) {               \
      constexpr int MM = 28;              \
      KERNEL_LAUNCH;                      \
    } else {                              \
      constexpr int MM = 32;              \
      KERNEL_LAUNCH;                      \
    }                                     \
  } while (0)

int dot_blocks(int64_t n) {
  int nb = (int)((n + 2047) / 2048);
  return nb < 1 ? 1 : (nb > DOT_BLOCKS ? DOT_BLOCKS : nb);
}

template <typename T>
void multi_dot(const T *V, int64_t ld, int m, const T *w, int64_t n, double *out, double *partials, hipStream_t s) {
  MFS_REQUIRE(m >= 1 && m <= MAXM, MFS_EINVAL, "multi_dot: m=%d out of range", m);
  const int nb = dot_blocks(n);
  MFS_MM_DISPATCH(m, hipLaunchKernelGGL((k_multi_dot_partial<T, MM>), dim3(nb), dim3(256), 0, s, V, ld, m, w, n,
                                        partials));
  hipLaunchKernelGGL(k_multi_dot_final, dim3(m), dim3(256), 0, s, partials, nb, out);
}

template <typename T, int MM>
__global__ void __launch_bounds__(VB) k_multi_axpy(T *w, const T *V, int64_t ld, int m, const double *h, int64_t n) {
  __shared__ double sh[MAXM];
  load_coefs(sh, h, m);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double v[MM];
    load_cols<T, MM>(V, ld, m, j, v);
    double acc = (double)w[j];
#pragma unroll
    for (int i = 0; i < MM; ++i) acc -= sh[i] * v[i];
    w[j] = (T)acc;
  }
}
template <typename T>
void multi_axpy(T *w, const T *V, int64_t ld, int m, const double *h, int64_t n, hipStream_t s) {
  MFS_REQUIRE(m >= 1 && m <= MAXM, MFS_EINVAL, "multi_axpy: m=%d out of range", m);
  MFS_MM_DISPATCH(m, hipLaunchKernelGGL((k_multi_axpy<T, MM>), dim3(nblocks(n)), dim3(VB), 0, s, w, V, ld, m, h, n));
}

// fused update and dot products (see axpy_dot); the same chunking and
// reduction order as k_multi_dot_partial
template <typename T, int MM>
__global__ void __launch_bounds__(256) k_axpy_dot_partial(T *w, const T *V, int64_t ld, int m, const double *h,
                                                          int md, int norm, int64_t n, double *partials) {
  __shared__ double sh[MAXM];
  load_coefs(sh, h, m);
  double acc[MM + 1];
#pragma unroll
  for (int i = 0; i <= MM; ++i) acc[i] = 0.0;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t beg = blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
    double v[MM];
    load_cols<T, MM>(V, ld, m, j, v);
    double wj = (double)w[j];
#pragma unroll
    for (int i = 0; i < MM; ++i) wj -= sh[i] * v[i];
    const T wt = (T)wj;
    w[j] = wt;
    const double wd = (double)wt;
#pragma unroll
    for (int i = 0; i < MM; ++i) acc[i] += v[i] * wd;
    acc[MM] += wd * wd;
  }
  __shared__ double red[256];
#pragma unroll
  for (int i = 0; i < MM; ++i)
    if (i < md) block_partial(acc[i], i, partials, red);
  if (norm) block_partial(acc[MM], md, partials, red);
}
template <typename T>
void axpy_dot(T *w, const T *V, int64_t ld, int m, const double *h, int md, bool norm, int64_t n, double *out,
              double *partials, hipStream_t s) {
  MFS_REQUIRE(m >= 1 && m <= MAXM - 1 && (md == 0 || md == m), MFS_EINVAL, "axpy_dot: m=%d md=%d", m, md);
  const int nb = dot_blocks(n);
  const int nf = norm ? 1 : 0;
  MFS_MM_DISPATCH(m, hipLaunchKernelGGL((k_axpy_dot_partial<T, MM>), dim3(nb), dim3(256), 0, s, w, V, ld, m, h, md,
                                        nf, n, partials));
  if (md + nf > 0) hipLaunchKernelGGL(k_multi_dot_final, dim3(md + nf), dim3(256), 0, s, partials, nb, out);
}

template <typename T, int MM>
__global__ void __launch_bounds__(VB) k_multi_combine(T *y, const T *V, int64_t ld, int m, const double *h, int64_t n,
                                                      int acc_in) {
  __shared__ double sh[MAXM];
  load_coefs(sh, h, m);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double v[MM];
    load_cols<T, MM>(V, ld, m, j, v);
    double acc = acc_in ? (double)y[j] : 0.0;
#pragma unroll
    for (int i = 0; i < MM; ++i) acc += sh[i] * v[i];
    y[j] = (T)acc;
  }
}
template <typename T>
void multi_combine(T *y, const T *V, int64_t ld, int m, const double *h, int64_t n, bool accumulate, hipStream_t s) {
  MFS_REQUIRE(m >= 1 && m <= MAXM, MFS_EINVAL, "multi_combine: m=%d out of range", m);
  MFS_MM_DISPATCH(m, hipLaunchKernelGGL((k_multi_combine<T, MM>), dim3(nblocks(n)), dim3(VB), 0, s, y, V, ld, m, h,
                                        n, accumulate ? 1 : 0));
}

// out = Ainv in, Ainv symmetric n x n FP64 (column-major = row-major)
template <typename T>
__global__ void k_dense_apply(const double *A, int n, const T *in, T *out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0;
  for (int c = 0; c < n; ++c) acc += A[(int64_t)c * n + r] * (double)in[c];
  out[r] = (T)acc;
}
template <typename T>
void dense_apply(const double *Ainv, int n, const T *in, T *out, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_apply<T>, dim3((n + 127) / 128), dim3(128), 0, s, Ainv, n, in, out);
}

template <typename T>
__global__ void k_pcg1(T *z, T *res, T *sv, const T *p, const T *q, const T *dinv, int64_t n, const double *rho,
                       const double *pq) {
  const double den = *pq;
  const T alpha = den != 0.0 ? (T)(*rho / den) : T(0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    z[i] += alpha * p[i];
    const T r = res[i] - alpha * q[i];
    res[i] = r;
    sv[i] = dinv[i] * r;
  }
}
template <typename T>
void pcg_update1(T *z, T *res, T *sv, const T *p, const T *q, const T *dinv, int64_t n, const double *rho,
                 const double *pq, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg1<T>, dim3(nblocks(n)), dim3(VB), 0, s, z, res, sv, p, q, dinv, n, rho, pq);
}
template <typename T>
__global__ void k_pcg2(T *p, const T *sv, int64_t n, const double *rn, const double *ro) {
  const double den = *ro;
  const T beta = den != 0.0 ? (T)(*rn / den) : T(0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = sv[i] + beta * p[i];
}
template <typename T>
void pcg_update2(T *p, const T *sv, int64_t n, const double *rho_new, const double *rho_old, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg2<T>, dim3(nblocks(n)), dim3(VB), 0, s, p, sv, n, rho_new, rho_old);
}
template <typename T>
__global__ void k_scale_inv_sqrt(T *y, const T *x, int64_t n, const double *nrm2) {
  const double v = *nrm2;
  const T f = v > 0.0 ? (T)(1.0 / sqrt(v)) : T(0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * f;
}
template <typename T>
void scale_inv_sqrt(T *y, const T *x, int64_t n, const double *nrm2, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inv_sqrt<T>, dim3(nblocks(n)), dim3(VB), 0, s, y, x, n, nrm2);
}
template <typename T>
__global__ void k_vec_mul(T *y, const T *a, const T *x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] * x[i];
}
template <typename T>
void vec_mul(T *y, const T *a, const T *x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_mul<T>, dim3(nblocks(n)), dim3(VB), 0, s, y, a, x, n);
}
__global__ void k_shift_mean(double *p, int64_t n, const double *num, const double *den) {
  const double c = *num / *den;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] -= c;
}
void shift_mean(double *p, int64_t n, const double *num, const double *den, hipStream_t s) {
  hipLaunchKernelGGL(k_shift_mean, dim3(nblocks(n)), dim3(VB), 0, s, p, n, num, den);
}

__global__ void k_reciprocal(double *r64, float *r32, const double *d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = 1.0 / d[i];
    r64[i] = v;
    r32[i] = (float)v;
  }
}
void launch_reciprocal(double *r64, float *r32, const double *d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_reciprocal, dim3(nblocks(n)), dim3(VB), 0, s, r64, r32, d, n);
}

__global__ void k_boundary_one(int dim, int nv0, int nv1, int nv2, int64_t Nv, double *d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < Nv && on_boundary(dim, nv0, nv1, nv2, i)) d[i] = 1.0;
}
void launch_reciprocal_boundary_one(const LevelGeom &g, double *d, hipStream_t s) {
  hipLaunchKernelGGL(k_boundary_one, dim3(nblocks(g.Nv)), dim3(VB), 0, s, g.dim, g.nv[0], g.nv[1], g.nv[2], g.Nv, d);
}

#define INST(T)                                                                                   \
  template void vec_fill<T>(T *, T, int64_t, hipStream_t);                                        \
  template void vec_copy<T>(T *, const T *, int64_t, hipStream_t);                                \
  template void vec_axpby<T>(T *, T, const T *, T, int64_t, hipStream_t);                         \
  template void vec_zero_mask_boundary<T>(const LevelGeom &, T *, hipStream_t);                   \
  template void vec_copy_boundary<T>(const LevelGeom &, T *, const T *, hipStream_t);             \
  template void vec_diag_scale<T>(const LevelGeom &, T *, const T *, const T *, hipStream_t);     \
  template void cheb_update<T>(const LevelGeom &, T *, T *, const T *, const T *, const T *, T, T, \
                               bool, hipStream_t);                                                \
  template void multi_dot<T>(const T *, int64_t, int, const T *, int64_t, double *, double *,     \
                             hipStream_t);                                                        \
  template void multi_axpy<T>(T *, const T *, int64_t, int, const double *, int64_t, hipStream_t); \
  template void axpy_dot<T>(T *, const T *, int64_t, int, const double *, int, bool, int64_t, double *, \
                            double *, hipStream_t);                                               \
  template void multi_combine<T>(T *, const T *, int64_t, int, const double *, int64_t, bool,     \
                                 hipStream_t);                                                    \
  template void dense_apply<T>(const double *, int, const T *, T *, hipStream_t);                 \
  template void pcg_update1<T>(T *, T *, T *, const T *, const T *, const T *, int64_t, const double *, \
                               const double *, hipStream_t);                                      \
  template void pcg_update2<T>(T *, const T *, int64_t, const double *, const double *, hipStream_t); \
  template void scale_inv_sqrt<T>(T *, const T *, int64_t, const double *, hipStream_t);         \
  template void vec_mul<T>(T *, const T *, const T *, int64_t, hipStream_t);
INST(double)
INST(float)
#undef INST
template void vec_cast<float, double>(float *, const double *, int64_t, hipStream_t);
template void vec_cast<double, float>(double *, const float *, int64_t, hipStream_t);
template void vec_fill<int>(int *, int, int64_t, hipStream_t);

}  // namespace mfs
