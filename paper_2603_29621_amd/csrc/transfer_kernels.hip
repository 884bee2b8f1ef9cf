// Multigrid transfer between a fine level and the next coarser one, Sec. 2
// eq. (transfer): prolongation x_f = sum_e S_e W_e P_e C_e G_e x_c cell by
// coarse cell, restriction its transpose.
//
// On the structured grid the cell-local embedding P_e is the tensor product
// of one 1D matrix E (h: the coarse Q_k basis at the 2k+1 nodes of the two
// children; p: the Q_kc basis at the Q_kf nodes), the weight W = 1/m (m = the
// number of coarse cells containing a fine node) and the Dirichlet constraint
// masks are separable per direction.  Both kernels therefore work per global
// node with no atomics:
//  * prolongation: thread per fine node, value interpolated from its owning
//    coarse cell (every coarse cell containing the node yields the same value
//    because the coarse function is continuous, so the weighted sum over the m
//    cells equals this single evaluation);
//  * restriction: the transpose, applied direction by direction in three
//    passes (x, then y, then z), each a banded 1D operator: a coarse node
//    gathers the fine nodes of the (one or two) coarse cells that contain it.
//    Because the coarse basis functions are continuous, the averaged weights
//    W = 1/m of eq. (transfer) equal evaluation in one owner cell per fine node
//    (the lower cell, the last one at the end), which is what the passes use.
// Vectors hold `ncu` components carrying the Dirichlet constraints (the
// velocity) followed by `ncp` unconstrained ones (the equal-order pressure of
// the monolithic Navier-Stokes hierarchy), each of one scalar node grid.
#include "internal.h"

namespace mfs {

struct TransferArgs {
  int dim;
  int ncu, ncp;  // constrained / unconstrained components
  int F;    // fine nodes per coarse cell edge minus one (h: 2k, p: kf)
  int kc;   // coarse degree
  int nc[3];          // coarse cells per direction
  int nf[3], ncn[3];  // fine / coarse node counts per direction
  int64_t Nf, Nc;
  double E[MAXQ * 2 * MAXQ];  // [F+1][kc+1], row-major with row stride MAXQ
};

template <typename T>
__global__ void k_prolongate_add(TransferArgs a, T *dst, const T *src) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= a.Nf) return;
  int g[3] = {(int)(f % a.nf[0]), (int)((f / a.nf[0]) % a.nf[1]), 0};
  if (a.dim == 3) g[2] = (int)(f / ((int64_t)a.nf[0] * a.nf[1]));
  int C[3] = {0, 0, 0}, i[3] = {0, 0, 0};
  bool fine_bnd = false;
  for (int d = 0; d < a.dim; ++d) {
    fine_bnd = fine_bnd || g[d] == 0 || g[d] == a.nf[d] - 1;  // fine Dirichlet row of P is zero
    C[d] = g[d] / a.F;
    if (C[d] >= a.nc[d]) C[d] = a.nc[d] - 1;
    i[d] = g[d] - a.F * C[d];
  }
  const int n1 = a.kc + 1;
  const int nz = a.dim == 3 ? n1 : 1;
  for (int comp = 0; comp < a.ncu + a.ncp; ++comp) {
    const bool con = comp < a.ncu;
    if (con && fine_bnd) continue;
    double acc = 0;
    for (int j2 = 0; j2 < nz; ++j2) {
      const int c2 = a.dim == 3 ? C[2] * a.kc + j2 : 0;
      if (con && a.dim == 3 && (c2 == 0 || c2 == a.ncn[2] - 1)) continue;
      const double e2 = a.dim == 3 ? a.E[i[2] * MAXQ + j2] : 1.0;
      for (int j1 = 0; j1 < n1; ++j1) {
        const int c1 = C[1] * a.kc + j1;
        if (con && (c1 == 0 || c1 == a.ncn[1] - 1)) continue;
        const double e21 = e2 * a.E[i[1] * MAXQ + j1];
        for (int j0 = 0; j0 < n1; ++j0) {
          const int c0 = C[0] * a.kc + j0;
          if (con && (c0 == 0 || c0 == a.ncn[0] - 1)) continue;
          const int64_t cn = c0 + (int64_t)a.ncn[0] * (c1 + (int64_t)a.ncn[1] * c2);
          acc += e21 * a.E[i[0] * MAXQ + j0] * (double)src[comp * a.Nc + cn];
        }
      }
    }
    dst[comp * a.Nf + f] += (T)acc;
  }
}

// 3D fast path of the prolongation for a compile-time coarse degree KC and
// fine span F: the 1D weights of the thread's node are picked out of the
// embedding table by uniform (scalar) loads and per-lane selects, and the
// (KC+1)^3 coarse values are gathered with no branches (weights of the
// constrained coarse boundary nodes are zero; every index stays in the coarse
// grid).  FP32 vectors are interpolated in FP32.
template <typename T, int KC, int F>
__global__ void __launch_bounds__(256) k_prolongate_add3(TransferArgs a, T *dst, const T *src) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= a.Nf) return;
  const int g[3] = {(int)(f % a.nf[0]), (int)((f / a.nf[0]) % a.nf[1]), (int)(f / ((int64_t)a.nf[0] * a.nf[1]))};
  bool fine_bnd = false;
  int C[3];
  T w[3][KC + 1], wm[3][KC + 1];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    fine_bnd = fine_bnd || g[d] == 0 || g[d] == a.nf[d] - 1;
    C[d] = g[d] / F;
    if (C[d] >= a.nc[d]) C[d] = a.nc[d] - 1;
    const int i = g[d] - F * C[d];
#pragma unroll
    for (int j = 0; j <= KC; ++j) {
      T e = 0;
#pragma unroll
      for (int ii = 0; ii <= F; ++ii) e = ii == i ? (T)a.E[ii * MAXQ + j] : e;
      const int cn = C[d] * KC + j;
      w[d][j] = e;
      wm[d][j] = (cn == 0 || cn == a.ncn[d] - 1) ? T(0) : e;
    }
  }
  const int64_t sy = a.ncn[0], sz = (int64_t)a.ncn[0] * a.ncn[1];
  const int64_t cbase = (int64_t)C[0] * KC + sy * C[1] * KC + sz * C[2] * KC;
  for (int comp = 0; comp < a.ncu + a.ncp; ++comp) {
    const bool con = comp < a.ncu;
    if (con && fine_bnd) continue;
    const T *s = src + comp * a.Nc + cbase;
    T acc = 0;
#pragma unroll
    for (int j2 = 0; j2 <= KC; ++j2)
#pragma unroll
      for (int j1 = 0; j1 <= KC; ++j1) {
        const T w21 = con ? wm[2][j2] * wm[1][j1] : w[2][j2] * w[1][j1];
#pragma unroll
        for (int j0 = 0; j0 <= KC; ++j0) acc += w21 * (con ? wm[0][j0] : w[0][j0]) * s[j0 + sy * j1 + sz * j2];
      }
    dst[comp * a.Nf + f] += acc;
  }
}

// per direction: list of (fine index, coefficient) contributing to coarse node gc
// (con: skip the fine Dirichlet nodes, whose rows of P are zero)
__device__ __forceinline__ int restrict_list(const TransferArgs &a, int d, int gc, bool con, int *fi, double *cf) {
  int cnt = 0;
  const int nc = a.nc[d];
  int cells[2], nce = 0;
  int C0 = gc / a.kc;
  if (C0 < nc) cells[nce++] = C0;
  if (gc % a.kc == 0 && C0 - 1 >= 0) cells[nce++] = C0 - 1;
  for (int e = 0; e < nce; ++e) {
    const int C = cells[e];
    const int j = gc - a.kc * C;
    for (int i = 0; i <= a.F; ++i) {
      const int gf = a.F * C + i;
      const bool edge = gf == 0 || gf == a.nf[d] - 1;
      if (con && edge) continue;
      const double m = (gf % a.F == 0 && !edge) ? 2.0 : 1.0;  // interior node shared by two coarse cells
      const double v = a.E[i * MAXQ + j] / m;
      int found = -1;
      for (int q = 0; q < cnt; ++q)
        if (fi[q] == gf) found = q;
      if (found >= 0)
        cf[found] += v;
      else {
        fi[cnt] = gf;
        cf[cnt] = v;
        ++cnt;
      }
    }
  }
  return cnt;
}

template <typename T>
__global__ void k_restrict(TransferArgs a, T *dst, const T *src) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= a.Nc) return;
  int g[3] = {(int)(c % a.ncn[0]), (int)((c / a.ncn[0]) % a.ncn[1]), 0};
  if (a.dim == 3) g[2] = (int)(c / ((int64_t)a.ncn[0] * a.ncn[1]));
  bool dir = false;
  for (int d = 0; d < a.dim; ++d) dir = dir || g[d] == 0 || g[d] == a.ncn[d] - 1;
  int fi[3][2 * 2 * MAXQ];
  double cf[3][2 * 2 * MAXQ];
  for (int pass = 0; pass < 2; ++pass) {
    const bool con = pass == 0;
    const int c0 = con ? 0 : a.ncu, c1 = con ? a.ncu : a.ncu + a.ncp;
    if (c0 == c1) continue;
    if (con && dir) {
      for (int comp = c0; comp < c1; ++comp) dst[comp * a.Nc + c] = 0;
      continue;
    }
    int cnt[3] = {1, 1, 1};
    fi[2][0] = 0;
    cf[2][0] = 1.0;
    for (int d = 0; d < a.dim; ++d) cnt[d] = restrict_list(a, d, g[d], con, fi[d], cf[d]);
    for (int comp = c0; comp < c1; ++comp) {
      double acc = 0;
      for (int z = 0; z < cnt[2]; ++z)
        for (int y = 0; y < cnt[1]; ++y) {
          const double cyz = cf[2][z] * cf[1][y];
          const int64_t row = (int64_t)a.nf[0] * (fi[1][y] + (int64_t)a.nf[1] * fi[2][z]);
          for (int x = 0; x < cnt[0]; ++x) acc += cyz * cf[0][x] * (double)src[comp * a.Nf + row + fi[0][x]];
        }
      dst[comp * a.Nc + c] = (T)acc;
    }
  }
}

// one separable restriction pass along direction d: out has the coarse node
// count along d and the input extents elsewhere; components < ncu carry the
// Dirichlet masks (fine and coarse boundary nodes along d are dropped)
template <typename T>
__global__ void k_restrict_pass(TransferArgs a, int d, int ni0, int ni1, int ni2, int no0, int no1, int no2,
                                int ncomp, int64_t in_stride, int64_t out_stride, const T *in, T *out) {
  const int64_t nout = (int64_t)no0 * no1 * no2;
  const int F = a.F, kc = a.kc, nc = a.nc[d], nf = a.nf[d], ncn = a.ncn[d];
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < nout; o += (int64_t)gridDim.x * blockDim.x) {
    const int o0 = (int)(o % no0), o1 = (int)((o / no0) % no1), o2 = (int)(o / ((int64_t)no0 * no1));
    const int j = d == 0 ? o0 : (d == 1 ? o1 : o2);
    const int64_t sd = d == 0 ? 1 : (d == 1 ? (int64_t)ni0 : (int64_t)ni0 * ni1);
    const int64_t base = (d == 0 ? 0 : o0) + (int64_t)ni0 * ((d == 1 ? 0 : o1) + (int64_t)ni1 * (d == 2 ? 0 : o2));
    const bool cbnd = j == 0 || j == ncn - 1;
    // fine range of the coarse cells containing j
    const int C0 = (j % kc == 0 && j > 0) ? j / kc - 1 : j / kc;
    const int C1 = j / kc < nc ? j / kc : nc - 1;
    const int f0 = F * C0, f1 = F * (C1 + 1);
    for (int comp = 0; comp < ncomp; ++comp) {
      const bool con = comp < a.ncu;
      double acc = 0;
      if (!(con && cbnd)) {
        for (int f = f0; f <= f1; ++f) {
          if (con && (f == 0 || f == nf - 1)) continue;
          const int own = f / F < nc ? f / F : nc - 1;
          const int jl = j - kc * own;
          if (jl < 0 || jl > kc) continue;
          acc += a.E[(f - F * own) * MAXQ + jl] * (double)in[comp * in_stride + base + sd * f];
        }
      }
      out[comp * out_stride + o] = (T)acc;
    }
  }
}

// the same pass for a compile-time coarse degree KC and fine span F: the at
// most 2F+1 fine nodes of the (one or two) coarse cells containing the
// output node, with their weights picked out of the embedding table once per
// thread by uniform loads and per-lane selects
template <typename T, int KC, int F>
__global__ void __launch_bounds__(256) k_restrict_pass3(TransferArgs a, int d, int ni0, int ni1, int ni2, int no0,
                                                        int no1, int no2, int ncomp, int64_t in_stride,
                                                        int64_t out_stride, const T *in, T *out) {
  const int64_t nout = (int64_t)no0 * no1 * no2;
  const int nc = a.nc[d], nf = a.nf[d], ncn = a.ncn[d];
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < nout; o += (int64_t)gridDim.x * blockDim.x) {
    const int o0 = (int)(o % no0), o1 = (int)((o / no0) % no1), o2 = (int)(o / ((int64_t)no0 * no1));
    const int j = d == 0 ? o0 : (d == 1 ? o1 : o2);
    const int64_t sd = d == 0 ? 1 : (d == 1 ? (int64_t)ni0 : (int64_t)ni0 * ni1);
    const int64_t base = (d == 0 ? 0 : o0) + (int64_t)ni0 * ((d == 1 ? 0 : o1) + (int64_t)ni1 * (d == 2 ? 0 : o2));
    const bool cbnd = j == 0 || j == ncn - 1;
    const int C0 = (j % KC == 0 && j > 0) ? j / KC - 1 : j / KC;
    const int C1 = j / KC < nc ? j / KC : nc - 1;
    const int f0 = F * C0, f1 = F * (C1 + 1);
    T w[2 * F + 1], wm[2 * F + 1];
#pragma unroll
    for (int t = 0; t <= 2 * F; ++t) {
      const int f = f0 + t;
      const int own = f / F < nc ? f / F : nc - 1;
      const int jl = j - KC * own, il = f - F * own;
      T e = 0;
#pragma unroll
      for (int ii = 0; ii <= F; ++ii)
#pragma unroll
        for (int jj = 0; jj <= KC; ++jj) e = (ii == il && jj == jl) ? (T)a.E[ii * MAXQ + jj] : e;
      const bool in_range = f <= f1;
      w[t] = in_range ? e : T(0);
      wm[t] = (in_range && !cbnd && f != 0 && f != nf - 1) ? e : T(0);
    }
    const int nt = f1 - f0;  // < 2F + 1
    for (int comp = 0; comp < ncomp; ++comp) {
      const bool con = comp < a.ncu;
      const T *s = in + comp * in_stride + base + sd * f0;
      T acc = 0;
#pragma unroll
      for (int t = 0; t <= 2 * F; ++t)
        if (t <= nt) acc += (con ? wm[t] : w[t]) * s[sd * t];
      out[comp * out_stride + o] = acc;
    }
  }
}

static TransferArgs make_targs(const LevelGeom &fine, const LevelGeom &coarse, bool h, const double *emb_host,
                               int ncp, int ncu) {
  TransferArgs a{};
  a.dim = fine.dim;
  a.ncu = ncu < 0 ? fine.dim : ncu;
  a.ncp = ncp;
  a.kc = coarse.k;
  a.F = h ? 2 * coarse.k : fine.k;
  for (int d = 0; d < 3; ++d) {
    a.nc[d] = coarse.n[d];
    a.nf[d] = fine.nv[d];
    a.ncn[d] = coarse.nv[d];
  }
  a.Nf = fine.Nv;
  a.Nc = coarse.Nv;
  for (int i = 0; i <= a.F; ++i)
    for (int j = 0; j <= a.kc; ++j) a.E[i * MAXQ + j] = emb_host[i * (a.kc + 1) + j];
  return a;
}

template <typename T>
void launch_prolongate_add(const LevelGeom &fine, const LevelGeom &coarse, bool h, const double *emb, T *dst_fine,
                           const T *src_coarse, hipStream_t s, int ncp, int ncu) {
  const TransferArgs a = make_targs(fine, coarse, h, emb, ncp, ncu);
  const dim3 grid((unsigned)((fine.Nv + 255) / 256)), block(256);
  if (fine.dim == 3 && a.kc == 1 && a.F == 2)
    hipLaunchKernelGGL((k_prolongate_add3<T, 1, 2>), grid, block, 0, s, a, dst_fine, src_coarse);
  else if (fine.dim == 3 && a.kc == 2 && a.F == 4)
    hipLaunchKernelGGL((k_prolongate_add3<T, 2, 4>), grid, block, 0, s, a, dst_fine, src_coarse);
  else if (fine.dim == 3 && a.kc == 2 && a.F == 3)
    hipLaunchKernelGGL((k_prolongate_add3<T, 2, 3>), grid, block, 0, s, a, dst_fine, src_coarse);
  else if (fine.dim == 3 && a.kc == 3 && a.F == 4)
    hipLaunchKernelGGL((k_prolongate_add3<T, 3, 4>), grid, block, 0, s, a, dst_fine, src_coarse);
  else
    hipLaunchKernelGGL(k_prolongate_add<T>, grid, block, 0, s, a, dst_fine, src_coarse);
  MFS_HIP(hipGetLastError());
}
template <typename T>
void launch_restrict(const LevelGeom &fine, const LevelGeom &coarse, bool h, const double *emb, T *dst_coarse,
                     const T *src_fine, hipStream_t s, int ncp, T *work, int ncu) {
  const TransferArgs a = make_targs(fine, coarse, h, emb, ncp, ncu);
  if (work == nullptr) {  // single-pass gather (no scratch available)
    hipLaunchKernelGGL(k_restrict<T>, dim3((unsigned)((coarse.Nv + 255) / 256)), dim3(256), 0, s, a, dst_coarse,
                       src_fine);
    MFS_HIP(hipGetLastError());
    return;
  }
  const int ncomp = a.ncu + a.ncp;
  int ext[3] = {fine.nv[0], fine.nv[1], fine.nv[2]};
  const T *in = src_fine;
  int64_t in_stride = fine.Nv;
  T *bufs[2] = {work, work + (int64_t)ncomp * restrict_work_elems(fine, coarse, 1) / 2};
  for (int d = 0; d < fine.dim; ++d) {
    int oext[3] = {ext[0], ext[1], ext[2]};
    oext[d] = coarse.nv[d];
    const int64_t nout = (int64_t)oext[0] * oext[1] * oext[2];
    const bool last = d == fine.dim - 1;
    T *out = last ? dst_coarse : bufs[d & 1];
    const int64_t out_stride = last ? coarse.Nv : nout;
    const unsigned grid = (unsigned)std::min<int64_t>((nout + 255) / 256, 65535);
#define RP_ARGS a, d, ext[0], ext[1], ext[2], oext[0], oext[1], oext[2], ncomp, in_stride, out_stride, in, out
    if (fine.dim == 3 && a.kc == 1 && a.F == 2)
      hipLaunchKernelGGL((k_restrict_pass3<T, 1, 2>), dim3(grid), dim3(256), 0, s, RP_ARGS);
    else if (fine.dim == 3 && a.kc == 2 && a.F == 4)
      hipLaunchKernelGGL((k_restrict_pass3<T, 2, 4>), dim3(grid), dim3(256), 0, s, RP_ARGS);
    else if (fine.dim == 3 && a.kc == 2 && a.F == 3)
      hipLaunchKernelGGL((k_restrict_pass3<T, 2, 3>), dim3(grid), dim3(256), 0, s, RP_ARGS);
    else if (fine.dim == 3 && a.kc == 3 && a.F == 4)
      hipLaunchKernelGGL((k_restrict_pass3<T, 3, 4>), dim3(grid), dim3(256), 0, s, RP_ARGS);
    else
      hipLaunchKernelGGL(k_restrict_pass<T>, dim3(grid), dim3(256), 0, s, RP_ARGS);
#undef RP_ARGS
    MFS_HIP(hipGetLastError());
    in = out;
    in_stride = nout;
    for (int b = 0; b < 3; ++b) ext[b] = oext[b];
  }
}

// scratch (elements) of the three-pass restriction for ncomp components: the
// two intermediate arrays after the x and y passes
int64_t restrict_work_elems(const LevelGeom &fine, const LevelGeom &coarse, int ncomp) {
  const int64_t a1 = (int64_t)coarse.nv[0] * fine.nv[1] * fine.nv[2];
  const int64_t a2 = (int64_t)coarse.nv[0] * coarse.nv[1] * fine.nv[2];
  return 2 * ncomp * std::max(a1, a2);
}
template void launch_prolongate_add<double>(const LevelGeom &, const LevelGeom &, bool, const double *, double *,
                                            const double *, hipStream_t, int, int);
template void launch_prolongate_add<float>(const LevelGeom &, const LevelGeom &, bool, const double *, float *,
                                           const float *, hipStream_t, int, int);
template void launch_restrict<double>(const LevelGeom &, const LevelGeom &, bool, const double *, double *,
                                      const double *, hipStream_t, int, double *, int);
template void launch_restrict<float>(const LevelGeom &, const LevelGeom &, bool, const double *, float *,
                                     const float *, hipStream_t, int, float *, int);

}  // namespace mfs
