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

// In-place Gauss-Jordan inversion with partial (row) pivoting, one
// workgroup per patch, the matrix in LDS (column-major like the storage).
// Row interchanges are recorded and undone as column interchanges at the
// end.  A zero or non-finite pivot sets *status.
constexpr int INV_T = 256;
template <int NP>
__global__ void __launch_bounds__(INV_T) k_invert(double *M, int *status) {
  constexpr int RP = NP <= 64 ? 64 : 128;  // rows per column group (whole waves)
  constexpr int CG = INV_T / RP;           // column groups
  __shared__ double a[NP * NP];
  __shared__ double fcol[NP], rrow[NP];
  __shared__ int perm[NP];
  __shared__ int sp;
  __shared__ double spiv;
  double *Mp = M + (int64_t)blockIdx.x * NP * NP;
  const int tid = threadIdx.x;
  for (int e = tid; e < NP * NP; e += INV_T) a[e] = Mp[e];
  __syncthreads();
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
        sp = bi;
        perm[k] = bi;
      }
    }
    __syncthreads();
    const int p = sp;
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
      spiv = 1.0 / piv;
    }
    __syncthreads();
    const double ip = spiv;
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
  T y = 0;
#pragma unroll 4
  for (int j = 0; j < NP; ++j) y += Mp[(int64_t)j * NP] * sr[lp][j];
  if (gi >= 0) x[gi] += omega * (T)w * y;
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

}  // namespace mfs
