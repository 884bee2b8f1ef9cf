// Device kernels of the refined-mesh multigrid (Sec. 5 on locally refined
// meshes; eq. (transfer)): the cell-wise embedding between a mesh and its
// global coarsening on E-vectors, and the colour probes of the Jacobi
// diagonal.
//
// E-vector layout of a level with nc cells and nq = (k+1)^3 nodes per cell:
// component c of node t of cell e at (e*nq + t)*4 + c.
#include <algorithm>

#include "amr_kernels.h"

namespace mfs {

namespace {

// first slot of component comp of cell e, and the stride between its nodes
__device__ __forceinline__ int64_t ev_at(int64_t nc, int nq, int64_t e, int comp) {
  (void)nc;
  return e * nq * 4 + comp;
}
__device__ __forceinline__ int ev_step(int comp) {
  (void)comp;
  return 4;
}

constexpr int AB = 256;
unsigned agrid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + AB - 1) / AB, 65535 * 8)); }

template <typename T, int NC, bool MASK>
__global__ void k_amr_gather(AmrMaps M, const T *x, T *ev) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < M.nrows; r += (int64_t)gridDim.x * blockDim.x) {
    const int c0 = M.rcol[r];
    T out[NC];
    if (c0 >= 0) {  // plain row
      const bool d = MASK && M.dir[c0];
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) out[comp] = (d && comp < 3) ? T(0) : x[comp * M.N + c0];
    } else {
      const int64_t h = -1 - (int64_t)c0;
      double s[NC] = {};
      for (int64_t j = M.hptr[h]; j < M.hptr[h + 1]; ++j) {
        const int64_t c = M.hcol[j];
        const double w = M.hval[j];
        const bool d = MASK && M.dir[c];
#pragma unroll
        for (int comp = 0; comp < NC; ++comp)
          if (!(d && comp < 3)) s[comp] += w * (double)x[comp * M.N + c];
      }
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) out[comp] = (T)s[comp];
    }
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) ev[4 * r + comp] = out[comp];
  }
}

// one thread per unknown with at most AMR_LIGHT rows in all, four components
// read together from each row: plain rows first, then the weighted ones
template <typename T>
__global__ void k_amr_scatter(AmrMaps M, const T *ev, const T *src, T *dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M.N; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = M.tptr[i], e = M.tptr[i + 1], wb = M.wptr[i], we = M.wptr[i + 1];
    if ((e - b) + (we - wb) > AMR_LIGHT) continue;  // summed by k_amr_scatter_heavy
    double s[4] = {0, 0, 0, 0};
    for (int64_t j = b; j < e; ++j) {
      const T *v = ev + 4 * (int64_t)M.trow[j];
#pragma unroll
      for (int comp = 0; comp < 4; ++comp) s[comp] += (double)v[comp];
    }
    for (int64_t j = wb; j < we; ++j) {
      const double w = M.wval[j];
      const T *v = ev + 4 * (int64_t)M.wrow[j];
#pragma unroll
      for (int comp = 0; comp < 4; ++comp) s[comp] += w * (double)v[comp];
    }
    const bool d = M.dir[i];
#pragma unroll
    for (int comp = 0; comp < 4; ++comp)
      dst[comp * M.N + i] = (d && comp < 3) ? (src ? src[comp * M.N + i] : T(0)) : (T)s[comp];
  }
}

// one wave per long list: strided partial sums over the plain then the
// weighted rows, then a butterfly (the same order on every call)
template <typename T>
__global__ void __launch_bounds__(AB) k_amr_scatter_heavy(AmrMaps M, const T *ev, const T *src, T *dst) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t hh = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; hh < M.nheavy; hh += waves) {
    const int64_t i = M.heavy[hh];
    const int64_t b = M.tptr[i], nu = M.tptr[i + 1] - b, wb = M.wptr[i], nw = M.wptr[i + 1] - wb;
    double s[4] = {0, 0, 0, 0};
    for (int64_t j = lane; j < nu + nw; j += 64) {
      const double w = j < nu ? 1.0 : M.wval[wb + j - nu];
      const T *v = ev + 4 * (int64_t)(j < nu ? M.trow[b + j] : M.wrow[wb + j - nu]);
#pragma unroll
      for (int comp = 0; comp < 4; ++comp) s[comp] += w * (double)v[comp];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int comp = 0; comp < 4; ++comp) s[comp] += __shfl_xor(s[comp], off, 64);
    if (lane == 0) {
      const bool d = M.dir[i];
#pragma unroll
      for (int comp = 0; comp < 4; ++comp)
        dst[comp * M.N + i] = (d && comp < 3) ? (src ? src[comp * M.N + i] : T(0)) : (T)s[comp];
    }
  }
}

template <typename T>
__global__ void k_amr_inject(AmrMaps M, const T *ev, T *x, int add) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < M.N; g += (int64_t)gridDim.x * blockDim.x) {
    const T *v = ev + 4 * (int64_t)M.owner[g];
    const int c0 = M.dir[g] ? 3 : 0;
    for (int comp = c0; comp < 4; ++comp) {
      if (add)
        x[comp * M.N + g] += v[comp];
      else
        x[comp * M.N + g] = v[comp];
    }
  }
}

template <typename T>
__global__ void k_amr_inject_t(AmrMaps M, const T *x, T *ev) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < M.N; g += (int64_t)gridDim.x * blockDim.x) {
    T *v = ev + 4 * (int64_t)M.owner[g];
    const int c0 = M.dir[g] ? 3 : 0;
    for (int comp = c0; comp < 4; ++comp) v[comp] = x[comp * M.N + g];
  }
}

// fine[f][comp][t] = sum_s W(oct[f])[t][s] coarse[parent[f]][comp][s]:
// unchanged cells (octant 8) copy, split cells apply the tensor product of
// the three half-cell 1D embeddings
template <typename T>
__global__ void k_embed(AmrEmbed E, int64_t ncf, int64_t ncc, const int *parent, const uint8_t *oct, const T *evc,
                        T *evf) {
  const int q = E.k + 1, nq = q * q * q;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ncf * 4 * nq) return;
  const int t = (int)(i % nq);
  const int comp = (int)((i / nq) % 4);
  const int64_t f = i / (4 * nq);
  const int64_t c = parent[f];
  const int o = oct[f];
  const T *src = evc + ev_at(ncc, nq, c, comp);
  const int st = ev_step(comp);
  T out;
  if (o == 8) {
    out = src[t * st];
  } else {
    const int tx = t % q, ty = (t / q) % q, tz = t / (q * q);
    const double *wx = E.w[o & 1][tx], *wy = E.w[(o >> 1) & 1][ty], *wz = E.w[(o >> 2) & 1][tz];
    double acc = 0.0;
    for (int sz = 0; sz < q; ++sz)
      for (int sy = 0; sy < q; ++sy) {
        const double wyz = wy[sy] * wz[sz];
        for (int sx = 0; sx < q; ++sx) acc += wx[sx] * wyz * (double)src[(sx + q * (sy + q * sz)) * st];
      }
    out = (T)acc;
  }
  evf[ev_at(ncf, nq, f, comp) + t * st] = out;
}

// coarse[c][comp][s] = sum over the children f of c, sum_t W(oct[f])[t][s] fine[f][comp][t]
template <typename T>
__global__ void k_embed_t(AmrEmbed E, int64_t ncf, int64_t ncc, const int64_t *cptr, const int *child,
                          const uint8_t *oct, const T *evf, T *evc) {
  const int q = E.k + 1, nq = q * q * q;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ncc * 4 * nq) return;
  const int s = (int)(i % nq);
  const int comp = (int)((i / nq) % 4);
  const int64_t c = i / (4 * nq);
  const int sx = s % q, sy = (s / q) % q, sz = s / (q * q);
  const int st = ev_step(comp);
  double acc = 0.0;
  for (int64_t e = cptr[c]; e < cptr[c + 1]; ++e) {
    const int64_t f = child[e];
    const int o = oct[f];
    const T *src = evf + ev_at(ncf, nq, f, comp);
    if (o == 8) {
      acc += (double)src[s * st];
      continue;
    }
    const int hx = o & 1, hy = (o >> 1) & 1, hz = (o >> 2) & 1;
    for (int tz = 0; tz < q; ++tz)
      for (int ty = 0; ty < q; ++ty) {
        const double wyz = E.w[hy][ty][sy] * E.w[hz][tz][sz];
        for (int tx = 0; tx < q; ++tx) acc += E.w[hx][tx][sx] * wyz * (double)src[(tx + q * (ty + q * tz)) * st];
      }
  }
  evc[ev_at(ncc, nq, c, comp) + s * st] = (T)acc;
}

__global__ void k_colour_probe(const int *colour, int64_t N, int col, int comp, double *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const bool on = colour[i] == col;
  for (int c = 0; c < 4; ++c) out[c * N + i] = (on && c == comp) ? 1.0 : 0.0;
}

__global__ void k_colour_take(const int *colour, int64_t N, int col, int comp, const double *y, double *diag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (colour[i] == col) diag[comp * N + i] = y[comp * N + i];
}

unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
void amr_gather(const AmrMaps &M, int ncomp, bool mask, const T *x, T *ev, hipStream_t s) {
  const dim3 g(agrid(M.nrows)), b(AB);
  if (ncomp == 4 && mask)
    hipLaunchKernelGGL((k_amr_gather<T, 4, true>), g, b, 0, s, M, x, ev);
  else if (ncomp == 4)
    hipLaunchKernelGGL((k_amr_gather<T, 4, false>), g, b, 0, s, M, x, ev);
  else if (ncomp == 3 && !mask)
    hipLaunchKernelGGL((k_amr_gather<T, 3, false>), g, b, 0, s, M, x, ev);
  else
    MFS_REQUIRE(false, MFS_EINVAL, "amr_gather: unsupported component count");
  MFS_HIP(hipGetLastError());
}

template <typename T>
void amr_scatter(const AmrMaps &M, const T *ev, const T *src, T *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_scatter<T>, dim3(agrid(M.N)), dim3(AB), 0, s, M, ev, src, dst);
  if (M.nheavy > 0)
    hipLaunchKernelGGL(k_amr_scatter_heavy<T>, dim3(agrid(M.nheavy * 64)), dim3(AB), 0, s, M, ev, src, dst);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void amr_inject(const AmrMaps &M, const T *ev, T *x, bool add, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_inject<T>, dim3(agrid(M.N)), dim3(AB), 0, s, M, ev, x, add ? 1 : 0);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void amr_inject_t(const AmrMaps &M, const T *x, T *ev, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_inject_t<T>, dim3(agrid(M.N)), dim3(AB), 0, s, M, x, ev);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void amr_embed(const AmrEmbed &E, int64_t ncf, int64_t ncc, const int *parent, const uint8_t *oct, const T *evc,
               T *evf, hipStream_t s) {
  const int nq = (E.k + 1) * (E.k + 1) * (E.k + 1);
  hipLaunchKernelGGL(k_embed<T>, dim3(nblocks(ncf * 4 * nq)), dim3(256), 0, s, E, ncf, ncc, parent, oct, evc, evf);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void amr_embed_t(const AmrEmbed &E, int64_t ncf, int64_t ncc, const int64_t *cptr, const int *child,
                 const uint8_t *oct, const T *evf, T *evc, hipStream_t s) {
  const int nq = (E.k + 1) * (E.k + 1) * (E.k + 1);
  hipLaunchKernelGGL(k_embed_t<T>, dim3(nblocks(ncc * 4 * nq)), dim3(256), 0, s, E, ncf, ncc, cptr, child, oct, evf,
                     evc);
  MFS_HIP(hipGetLastError());
}

void amr_colour_probe(const int *colour, int64_t N, int col, int comp, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_colour_probe, dim3(nblocks(N)), dim3(256), 0, s, colour, N, col, comp, out);
  MFS_HIP(hipGetLastError());
}

void amr_colour_take(const int *colour, int64_t N, int col, int comp, const double *y, double *diag, hipStream_t s) {
  hipLaunchKernelGGL(k_colour_take, dim3(nblocks(N)), dim3(256), 0, s, colour, N, col, comp, y, diag);
  MFS_HIP(hipGetLastError());
}

#define AMR_INST(T)                                                                                    \
  template void amr_gather<T>(const AmrMaps &, int, bool, const T *, T *, hipStream_t);                 \
  template void amr_scatter<T>(const AmrMaps &, const T *, const T *, T *, hipStream_t);                \
  template void amr_inject<T>(const AmrMaps &, const T *, T *, bool, hipStream_t);                      \
  template void amr_inject_t<T>(const AmrMaps &, const T *, T *, hipStream_t);
AMR_INST(double)
AMR_INST(float)
#undef AMR_INST

template void amr_embed<double>(const AmrEmbed &, int64_t, int64_t, const int *, const uint8_t *, const double *,
                                double *, hipStream_t);
template void amr_embed<float>(const AmrEmbed &, int64_t, int64_t, const int *, const uint8_t *, const float *,
                               float *, hipStream_t);
template void amr_embed_t<double>(const AmrEmbed &, int64_t, int64_t, const int64_t *, const int *, const uint8_t *,
                                  const double *, double *, hipStream_t);
template void amr_embed_t<float>(const AmrEmbed &, int64_t, int64_t, const int64_t *, const int *, const uint8_t *,
                                 const float *, float *, hipStream_t);

}  // namespace mfs
