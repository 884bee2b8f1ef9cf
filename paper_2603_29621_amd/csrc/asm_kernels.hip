// Additive Schwarz relaxation on vertex patches of a structured equal-order
// Navier-Stokes level (Sec. 2: ASM as the ingredient of a relaxation
// smoother; Sec. 5, Exp. 4: two relaxation steps around ASM).
//
// Patch of vertex v: every unknown (d velocity components, pressure) at the
// nodes whose lattice index i satisfies |i_a - k v_a| < k along every axis,
// Dirichlet unknowns left out: the nodes inside the vertex star, plus the
// star's nodes on the domain boundary.  Local index li = field * B + node,
// node = a_0 + W (a_1 + W a_2) with W = 2k - 1, i_a = k v_a - (k - 1) + a_a;
// absent entries (outside the lattice, Dirichlet) carry identity rows and
// columns, so every patch matrix has the fixed size NP = B (d + 1).
//
// Patches of one colour (vertex index parity per axis) share no cell, so
//  * probing: one unit vector per patch of a colour at local index j gives
//    column j of every patch matrix of that colour from one Jacobian apply;
//  * apply: the patches of a colour touch disjoint unknowns, so their
//    updates are plain read-modify-writes; colours run one after the other,
//    all with the residual of the sweep's start (additive), in a fixed order.
//
// Storage: the inverse of patch p (vertex-lexicographic id) at M + p NP^2,
// column-major (column j contiguous over the rows), so the NP threads of a
// patch read one column per step with a coalesced load.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace mfs {

namespace {

template <int DIM, int K>
struct Pt {
  static constexpr int W = 2 * K - 1;
  static constexpr int B = DIM == 3 ? W * W * W : W * W;
  static constexpr int NP = B * (DIM + 1);
  // threads per patch in the apply kernel (a power of two >= NP)
  static constexpr int NPP = NP <= 4 ? 4 : NP <= 32 ? 32 : NP <= 64 ? 64 : 128;
};

struct Colour {
  int c[3];
  int nvc[3];
  int64_t count;
};

inline Colour colour_of(const LevelGeom &g, int colour) {
  Colour C{};
  C.count = 1;
  for (int a = 0; a < 3; ++a) {
    C.c[a] = a < g.dim ? (colour >> a) & 1 : 0;
    C.nvc[a] = a < g.dim ? (g.n[a] + 2 - C.c[a]) / 2 : 1;
    C.count *= C.nvc[a];
  }
  return C;
}

// vertex of patch number q within colour C; patch id (vertex-lexicographic)
__device__ __forceinline__ void patch_vertex(const LevelGeom &g, const Colour &C, int64_t q, int v[3], int64_t *pid) {
  const int t0 = (int)(q % C.nvc[0]);
  const int64_t r = q / C.nvc[0];
  const int t1 = (int)(r % C.nvc[1]);
  const int t2 = (int)(r / C.nvc[1]);
  v[0] = 2 * t0 + C.c[0];
  v[1] = 2 * t1 + C.c[1];
  v[2] = 2 * t2 + C.c[2];
  *pid = v[0] + (int64_t)(g.n[0] + 1) * (v[1] + (int64_t)(g.n[1] + 1) * v[2]);
}

// global unknown of local index li of the patch at vertex v (-1: absent);
// *w = 1 / (number of patches holding it)
template <int DIM, int K>
__device__ __forceinline__ int64_t patch_dof(const LevelGeom &g, const int v[3], int li, double *w) {
  using P = Pt<DIM, K>;
  const int f = li / P::B;
  int nd = li % P::B;
  int64_t idx = 0, stride = 1;
  bool bnd = false;
  double wt = 1.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int i = K * v[a] - (K - 1) + nd % P::W;
    nd /= P::W;
    const int last = K * g.n[a];
    if (i < 0 || i > last) return -1;
    bnd = bnd || i == 0 || i == last;
    if (i % K) wt *= 0.5;
    idx += stride * i;
    stride *= last + 1;
  }
  if (f < DIM && bnd) return -1;
  *w = wt;
  return f * g.Nv + idx;
}

template <int DIM, int K>
__global__ void k_probe_set(LevelGeom g, Colour C, double *x, int j, double value) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= C.count) return;
  int v[3];
  int64_t pid;
  patch_vertex(g, C, q, v, &pid);
  double w;
  const int64_t gi = patch_dof<DIM, K>(g, v, j, &w);
  if (gi >= 0) x[gi] = value;
}

template <int DIM, int K>
__global__ void k_probe_extract(LevelGeom g, Colour C, const double *y, double *M, int j) {
  constexpr int NP = Pt<DIM, K>::NP;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= C.count * NP) return;
  const int64_t q = t / NP;
  const int i = (int)(t % NP);
  int v[3];
  int64_t pid;
  patch_vertex(g, C, q, v, &pid);
  double w;
  const int64_t gi = patch_dof<DIM, K>(g, v, i, &w);
  M[pid * NP * NP + (int64_t)j * NP + i] = gi >= 0 ? y[gi] : (i == j ? 1.0 : 0.0);
}

// In-place Gauss-Jordan inversion with partial (row) pivoting of the NP x NP
// matrix a (column-major; in LDS, or in global memory when it does not fit),
// by the INV_T threads of a workgroup.  Row
// interchanges are recorded and undone as column interchanges at the end.  A
// zero or non-finite pivot sets *status.
constexpr int INV_T = 256;
template <int NP>
__device__ void gj_invert_lds(double *a, double *fcol, double *rrow, int *perm, int *sp, double *spiv, int *status) {
  constexpr int RP = NP <= 64 ? 64 : NP <= 128 ? 128 : 256;  // rows per column group (whole waves)
  constexpr int CG = INV_T / RP;                             // column groups
  static_assert(NP <= 256, "patch too large for the row groups");
  const int tid = threadIdx.x;
  for (int k = 0; k < NP; ++k) {
    if (tid < 64) {  // pivot: largest |a[i][k]|, i >= k, first index on ties
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < NP; i += 64) {
        const double m = fabs(a[k * NP + i]);
        if (m > best) {
          best = m;
          bi = i;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        *sp = bi;
        perm[k] = bi;
      }
    }
    __syncthreads();
    const int p = *sp;
    if (p != k)
      for (int j = tid; j < NP; j += INV_T) {
        const double t = a[j * NP + k];
        a[j * NP + k] = a[j * NP + p];
        a[j * NP + p] = t;
      }
    __syncthreads();
    if (tid == 0) {
      const double piv = a[k * NP + k];
      if (!(piv != 0.0) || !isfinite(piv)) atomicOr(status, 1);
      *spiv = 1.0 / piv;
    }
    __syncthreads();
    const double ip = *spiv;
    for (int e = tid; e < NP; e += INV_T) {
      fcol[e] = e == k ? 0.0 : a[k * NP + e];           // factors of the other rows
      rrow[e] = e == k ? ip : a[e * NP + k] * ip;       // the scaled pivot row
    }
    __syncthreads();
    // thread (row i, column group h): lanes run over rows, so a column's
    // entries are consecutive words and the pivot row value is a broadcast
    for (int t = tid; t < RP * CG; t += INV_T) {
      const int i = t % RP, h = t / RP;
      if (i >= NP) continue;
      const double f = fcol[i];
#pragma unroll 6
      for (int j = h; j < NP; j += CG) {
        const double r = rrow[j];
        double &x = a[j * NP + i];
        x = i == k ? r : (j == k ? 0.0 : x) - f * r;
      }
    }
    __syncthreads();
  }
  for (int k = NP - 1; k >= 0; --k) {  // undo the row interchanges as column interchanges
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < NP; i += INV_T) {
        const double t = a[k * NP + i];
        a[k * NP + i] = a[p * NP + i];
        a[p * NP + i] = t;
      }
    __syncthreads();
  }
}

// one workgroup per patch, the matrix in LDS (column-major like the storage)
template <int NP>
__global__ void __launch_bounds__(INV_T) k_invert(double *M, int *status) {
  __shared__ double a[NP * NP];
  __shared__ double fcol[NP], rrow[NP];
  __shared__ int perm[NP];
  __shared__ int sp;
  __shared__ double spiv;
  double *Mp = M + (int64_t)blockIdx.x * NP * NP;
  const int tid = threadIdx.x;
  for (int e = tid; e < NP * NP; e += INV_T) a[e] = Mp[e];
  __syncthreads();
  gj_invert_lds<NP>(a, fcol, rrow, perm, &sp, &spiv, status);
  for (int e = tid; e < NP * NP; e += INV_T) Mp[e] = a[e];
}

// x += omega W A_P^{-1} (b - t) on the patches of one colour; NPP threads per
// patch, thread i owns row i
constexpr int APPLY_T = 256;
template <typename T, int DIM, int K>
__global__ void __launch_bounds__(APPLY_T) k_asm_apply(LevelGeom g, Colour C, const T *__restrict__ M,
                                                        const T *__restrict__ b, const T *__restrict__ t,
                                                        T *__restrict__ x, T omega) {
  using P = Pt<DIM, K>;
  constexpr int NP = P::NP, NPP = P::NPP, PPB = APPLY_T / NPP;
  __shared__ T sr[PPB][NPP];
  const int lp = threadIdx.x / NPP, i = threadIdx.x % NPP;
  const int64_t q = blockIdx.x * (int64_t)PPB + lp;
  const bool on = q < C.count;
  int v[3] = {0, 0, 0};
  int64_t pid = 0, gi = -1;
  double w = 0.0;
  if (on) {
    patch_vertex(g, C, q, v, &pid);
    if (i < NP) gi = patch_dof<DIM, K>(g, v, i, &w);
  }
  sr[lp][i] = gi >= 0 ? b[gi] - t[gi] : T(0);
  __syncthreads();
  if (!on || i >= NP) return;
  const T *Mp = M + pid * NP * NP + i;
  // four partial sums, so that a thread keeps several column loads in flight
  T y[4] = {0, 0, 0, 0};
#pragma unroll 8
  for (int j = 0; j < NP; ++j) y[j & 3] += Mp[(int64_t)j * NP] * sr[lp][j];
  if (gi >= 0) x[gi] += omega * (T)w * ((y[0] + y[1]) + (y[2] + y[3]));
}

template <int DIM, int K, typename F>
void by_degree(const LevelGeom &g, F &&f) {
  (void)g;
  f(std::integral_constant<int, DIM>{}, std::integral_constant<int, K>{});
}

template <typename F>
void dispatch(const LevelGeom &g, F &&f) {
  MFS_REQUIRE(g.k == 1 || g.k == 2, MFS_EUNSUPPORTED, "additive Schwarz patches support degrees 1 and 2 (got %d)",
              g.k);
  if (g.dim == 2 && g.k == 1) return by_degree<2, 1>(g, f);
  if (g.dim == 2 && g.k == 2) return by_degree<2, 2>(g, f);
  if (g.dim == 3 && g.k == 1) return by_degree<3, 1>(g, f);
  return by_degree<3, 2>(g, f);
}

inline unsigned grid_of(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// ------------------------------------------------------------------------
// Space-time patches of a Taylor-Hood level (Sec. 4: the space-time ASM
// smoother; the vertex-star patch with the whole slab in time).  Patch of
// vertex v, per stage: the velocity components at the velocity nodes i with
// |i_a - K v_a| < K and the pressure at the pressure nodes j with
// |j_a - (K-1) v_a| < K-1; spatial slot li = field * BV + node for the
// velocity, DIM BV + node for the pressure; absent slots (outside the
// lattice, velocity Dirichlet) carry identity rows and columns.  The
// space-time slot is q NPS + li (stage-major).  Same colours as above.
template <int DIM, int K>
struct Th {
  static constexpr int W = 2 * K - 1, WP = 2 * K - 3;
  static constexpr int BV = DIM == 3 ? W * W * W : W * W;
  static constexpr int BP = DIM == 3 ? WP * WP * WP : WP * WP;
  static constexpr int NPS = DIM * BV + BP;
};

// spatial unknown of slot li of the patch at vertex v (-1: absent); *w = 1 /
// (number of patches holding it)
template <int DIM, int K>
__device__ __forceinline__ int64_t th_slot(const LevelGeom &g, const int v[3], int li, double *w) {
  using P = Th<DIM, K>;
  const bool vel = li < DIM * P::BV;
  const int f = vel ? li / P::BV : DIM;
  int nd = vel ? li % P::BV : li - DIM * P::BV;
  const int deg = vel ? K : K - 1, wid = vel ? P::W : P::WP;
  int64_t idx = 0, stride = 1;
  bool bnd = false;
  double wt = 1.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int i = deg * v[a] - (deg - 1) + nd % wid;
    nd /= wid;
    const int last = deg * g.n[a];
    if (i < 0 || i > last) return -1;
    bnd = bnd || i == 0 || i == last;
    if (i % deg) wt *= 0.5;
    idx += stride * i;
    stride *= last + 1;
  }
  if (vel && bnd) return -1;
  *w = wt;
  return vel ? f * g.Nv + idx : DIM * g.Nv + idx;
}

__device__ __forceinline__ void vertex_of(const LevelGeom &g, int64_t pid, int v[3]) {
  v[0] = (int)(pid % (g.n[0] + 1));
  const int64_t r = pid / (g.n[0] + 1);
  v[1] = (int)(r % (g.n[1] + 1));
  v[2] = (int)(r / (g.n[1] + 1));
}

template <int DIM, int K>
__global__ void k_th_probe_set(LevelGeom g, Colour C, double *x, int j) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= C.count) return;
  int v[3];
  int64_t pid;
  patch_vertex(g, C, q, v, &pid);
  double w;
  const int64_t gi = th_slot<DIM, K>(g, v, j, &w);
  if (gi >= 0) x[gi] = 1.0;
}

// column j of the spatial patch matrices of one colour from y = A e_j; with
// nvel > 0, y holds only the first nvel rows (the velocity mass) and the
// pressure rows are 0
template <int DIM, int K>
__global__ void k_th_probe_extract(LevelGeom g, Colour C, const double *y, int64_t nvel, double *M, int j) {
  constexpr int NPS = Th<DIM, K>::NPS;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= C.count * NPS) return;
  const int64_t q = t / NPS;
  const int i = (int)(t % NPS);
  int v[3];
  int64_t pid;
  patch_vertex(g, C, q, v, &pid);
  double w;
  const int64_t gi = th_slot<DIM, K>(g, v, i, &w);
  double val = 0.0;
  if (gi >= 0 && (nvel == 0 || gi < nvel)) val = y[gi];
  M[pid * NPS * NPS + (int64_t)j * NPS + i] = val;
}

// space-time patch matrix G (x) M_s + tau I (x) A_s (identity on absent
// slots), inverted in LDS; one workgroup per patch
template <int DIM, int K, int Q>
__global__ void __launch_bounds__(INV_T) k_th_form_invert(LevelGeom g, StageCoef G, double tau,
                                                          const double *__restrict__ As,
                                                          const double *__restrict__ Ms, double *Kinv,
                                                          int *status) {
  constexpr int NPS = Th<DIM, K>::NPS, NP = Q * NPS;
  constexpr bool IN_LDS = NP <= 128;  // 128 KB; larger patches are inverted in place in global memory
  __shared__ double lds[IN_LDS ? NP * NP : 1];
  __shared__ double fcol[NP], rrow[NP];
  __shared__ int perm[NP];
  __shared__ int present[NPS];
  __shared__ int sp;
  __shared__ double spiv;
  const int64_t pid = blockIdx.x;
  const int tid = threadIdx.x;
  int v[3];
  vertex_of(g, pid, v);
  for (int i = tid; i < NPS; i += INV_T) {
    double w;
    present[i] = th_slot<DIM, K>(g, v, i, &w) >= 0;
  }
  __syncthreads();
  const double *Ap = As + pid * NPS * NPS, *Mp = Ms + pid * NPS * NPS;
  double *Kp = Kinv + pid * NP * NP;
  double *a = IN_LDS ? lds : Kp;
  for (int e = tid; e < NP * NP; e += INV_T) {
    const int c = e / NP, r = e % NP;  // column-major: a[c * NP + r]
    const int qc = c / NPS, jc = c % NPS, qr = r / NPS, ir = r % NPS;
    double val;
    if (!present[jc] || !present[ir])
      val = r == c ? 1.0 : 0.0;
    else
      val = G.c[qr * MFS_MAX_STAGES + qc] * Mp[jc * NPS + ir] + (qr == qc ? tau * Ap[jc * NPS + ir] : 0.0);
    a[e] = val;
  }
  __syncthreads();
  gj_invert_lds<NP>(a, fcol, rrow, perm, &sp, &spiv, status);
  if constexpr (IN_LDS)
    for (int e = tid; e < NP * NP; e += INV_T) Kp[e] = a[e];
}

// x += omega W Kp^{-1} (b - t) on the space-time patches of one colour;
// stage-major vectors of Q stages of N entries; NPP threads per patch
template <typename T, int DIM, int K, int Q>
__global__ void __launch_bounds__(APPLY_T) k_th_apply(LevelGeom g, Colour C, int64_t N,
                                                      const T *__restrict__ Kinv, const T *__restrict__ b,
                                                      const T *__restrict__ t, T *__restrict__ x, T omega) {
  constexpr int NPS = Th<DIM, K>::NPS, NP = Q * NPS;
  constexpr int NPP = NP <= 32 ? 32 : NP <= 64 ? 64 : NP <= 128 ? 128 : 256, PPB = APPLY_T / NPP;
  __shared__ T sr[PPB][NPP];
  const int lp = threadIdx.x / NPP, i = threadIdx.x % NPP;
  const int64_t q = blockIdx.x * (int64_t)PPB + lp;
  const bool on = q < C.count;
  int v[3] = {0, 0, 0};
  int64_t pid = 0, gi = -1;
  double w = 0.0;
  if (on && i < NP) {
    patch_vertex(g, C, q, v, &pid);
    const int64_t gs = th_slot<DIM, K>(g, v, i % NPS, &w);
    if (gs >= 0) gi = (i / NPS) * N + gs;
  }
  sr[lp][i] = gi >= 0 ? b[gi] - t[gi] : T(0);
  __syncthreads();
  if (!on || i >= NP) return;
  const T *Kp = Kinv + pid * NP * NP + i;
  // four partial sums, so that a thread keeps several column loads in flight
  T y[4] = {0, 0, 0, 0};
#pragma unroll 8
  for (int j = 0; j < NP; ++j) y[j & 3] += Kp[(int64_t)j * NP] * sr[lp][j];
  if (gi >= 0) x[gi] += omega * (T)w * ((y[0] + y[1]) + (y[2] + y[3]));
}

// (DIM, K, Q) of the supported space-time patches: 2D with K = 2, 3 and
// Q <= 3 (at most 177 unknowns), 3D with K = 2 and Q <= 3 (82, 164, 246);
// patches of more than 128 unknowns are inverted in global memory
template <typename F>
void th_dispatch(const LevelGeom &g, int Q, F &&f) {
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I1 = std::integral_constant<int, 1>;
  if (g.dim == 2) {
    if (g.k == 2 && Q == 1) return f(I2{}, I2{}, I1{});
    if (g.k == 2 && Q == 2) return f(I2{}, I2{}, I2{});
    if (g.k == 2 && Q == 3) return f(I2{}, I2{}, I3{});
    if (g.k == 3 && Q == 1) return f(I2{}, I3{}, I1{});
    if (g.k == 3 && Q == 2) return f(I2{}, I3{}, I2{});
    if (g.k == 3 && Q == 3) return f(I2{}, I3{}, I3{});
  } else {
    if (g.k == 2 && Q == 1) return f(I3{}, I2{}, I1{});
    if (g.k == 2 && Q == 2) return f(I3{}, I2{}, I2{});
    if (g.k == 2 && Q == 3) return f(I3{}, I2{}, I3{});
  }
  MFS_REQUIRE(false, MFS_EUNSUPPORTED, "space-time patches: dim %d, k = %d with %d stages not supported", g.dim,
              g.k, Q);
}

}  // namespace

int asm_patch_size(const LevelGeom &g) {
  const int w = 2 * g.k - 1;
  return (g.dim == 3 ? w * w * w : w * w) * (g.dim + 1);
}

int64_t asm_patch_count(const LevelGeom &g) {
  int64_t c = 1;
  for (int a = 0; a < g.dim; ++a) c *= g.n[a] + 1;
  return c;
}

int asm_colours(const LevelGeom &g) { return 1 << g.dim; }

void launch_asm_probe_set(const LevelGeom &g, double *x, int colour, int j, double value, hipStream_t s) {
  const Colour C = colour_of(g, colour);
  dispatch(g, [&](auto D, auto Kc) {
    hipLaunchKernelGGL((k_probe_set<decltype(D)::value, decltype(Kc)::value>), dim3(grid_of(C.count, 256)), dim3(256),
                       0, s, g, C, x, j, value);
  });
  MFS_HIP(hipGetLastError());
}

void launch_asm_probe_extract(const LevelGeom &g, const double *y, double *M, int colour, int j, hipStream_t s) {
  const Colour C = colour_of(g, colour);
  const int64_t n = C.count * asm_patch_size(g);
  dispatch(g, [&](auto D, auto Kc) {
    hipLaunchKernelGGL((k_probe_extract<decltype(D)::value, decltype(Kc)::value>), dim3(grid_of(n, 256)), dim3(256), 0,
                       s, g, C, y, M, j);
  });
  MFS_HIP(hipGetLastError());
}

void launch_asm_invert(const LevelGeom &g, double *M, int *status, hipStream_t s) {
  const int64_t np = asm_patch_count(g);
  MFS_REQUIRE(np <= 0x7fffffff, MFS_EINVAL, "too many patches");
  dispatch(g, [&](auto D, auto Kc) {
    constexpr int NP = Pt<decltype(D)::value, decltype(Kc)::value>::NP;
    hipLaunchKernelGGL((k_invert<NP>), dim3((unsigned)np), dim3(INV_T), 0, s, M, status);
  });
  MFS_HIP(hipGetLastError());
}

template <typename T>
void launch_asm_apply(const LevelGeom &g, const T *M, int colour, const T *b, const T *t, T *x, T omega,
                      hipStream_t s) {
  const Colour C = colour_of(g, colour);
  dispatch(g, [&](auto D, auto Kc) {
    constexpr int DD = decltype(D)::value, KK = decltype(Kc)::value;
    constexpr int PPB = APPLY_T / Pt<DD, KK>::NPP;
    hipLaunchKernelGGL((k_asm_apply<T, DD, KK>), dim3(grid_of(C.count, PPB)), dim3(APPLY_T), 0, s, g, C, M, b, t, x,
                       omega);
  });
  MFS_HIP(hipGetLastError());
}

template void launch_asm_apply<double>(const LevelGeom &, const double *, int, const double *, const double *,
                                       double *, double, hipStream_t);
template void launch_asm_apply<float>(const LevelGeom &, const float *, int, const float *, const float *, float *,
                                      float, hipStream_t);

int th_patch_size(const LevelGeom &g) {
  const int w = 2 * g.k - 1, wp = 2 * g.k - 3;
  return g.dim * (g.dim == 3 ? w * w * w : w * w) + (g.dim == 3 ? wp * wp * wp : wp * wp);
}

void launch_th_probe_set(const LevelGeom &g, double *x, int colour, int j, hipStream_t s) {
  const Colour C = colour_of(g, colour);
  th_dispatch(g, 1, [&](auto D, auto Kc, auto) {
    hipLaunchKernelGGL((k_th_probe_set<decltype(D)::value, decltype(Kc)::value>), dim3(grid_of(C.count, 256)),
                       dim3(256), 0, s, g, C, x, j);
  });
  MFS_HIP(hipGetLastError());
}

void launch_th_probe_extract(const LevelGeom &g, const double *y, int64_t nvel, double *M, int colour, int j,
                             hipStream_t s) {
  const Colour C = colour_of(g, colour);
  const int64_t n = C.count * th_patch_size(g);
  th_dispatch(g, 1, [&](auto D, auto Kc, auto) {
    hipLaunchKernelGGL((k_th_probe_extract<decltype(D)::value, decltype(Kc)::value>), dim3(grid_of(n, 256)),
                       dim3(256), 0, s, g, C, y, nvel, M, j);
  });
  MFS_HIP(hipGetLastError());
}

void launch_th_form_invert(const LevelGeom &g, int Q, const StageCoef &G, double tau, const double *As,
                           const double *Ms, double *Kinv, int *status, hipStream_t s) {
  const int64_t np = asm_patch_count(g);
  MFS_REQUIRE(np <= 0x7fffffff, MFS_EINVAL, "too many patches");
  th_dispatch(g, Q, [&](auto D, auto Kc, auto Qc) {
    hipLaunchKernelGGL((k_th_form_invert<decltype(D)::value, decltype(Kc)::value, decltype(Qc)::value>),
                       dim3((unsigned)np), dim3(INV_T), 0, s, g, G, tau, As, Ms, Kinv, status);
  });
  MFS_HIP(hipGetLastError());
}

template <typename T>
void launch_th_apply(const LevelGeom &g, int Q, int64_t N, const T *Kinv, int colour, const T *b, const T *t, T *x,
                     T omega, hipStream_t s) {
  const Colour C = colour_of(g, colour);
  th_dispatch(g, Q, [&](auto D, auto Kc, auto Qc) {
    constexpr int DD = decltype(D)::value, KK = decltype(Kc)::value, QQ = decltype(Qc)::value;
    constexpr int NP = QQ * Th<DD, KK>::NPS;
    constexpr int PPB = APPLY_T / (NP <= 32 ? 32 : NP <= 64 ? 64 : NP <= 128 ? 128 : 256);
    hipLaunchKernelGGL((k_th_apply<T, DD, KK, QQ>), dim3(grid_of(C.count, PPB)), dim3(APPLY_T), 0, s, g, C, N, Kinv,
                       b, t, x, omega);
  });
  MFS_HIP(hipGetLastError());
}
template void launch_th_apply<double>(const LevelGeom &, int, int64_t, const double *, int, const double *,
                                      const double *, double *, double, hipStream_t);
template void launch_th_apply<float>(const LevelGeom &, int, int64_t, const float *, int, const float *,
                                     const float *, float *, float, hipStream_t);

}  // namespace mfs
