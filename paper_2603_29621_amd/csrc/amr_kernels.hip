// Device kernels of the refined-mesh multigrid (Sec. 5 on locally refined
// meshes; eq. (transfer)): the cell-wise embedding between a mesh and its
// global coarsening on E-vectors, and the colour probes of the Jacobi
// diagonal.
//
// E-vector layout of a level with nc cells and nq = (k+1)^3 nodes per cell:
// component c < 3 of node t of cell e at (e*nq + t)*3 + c, the fourth
// (pressure) at 3*nc*nq + e*nq + t.
#include "amr_kernels.h"

namespace mfs {

namespace {

// first slot of component comp of cell e, and the stride between its nodes
__device__ __forceinline__ int64_t ev_at(int64_t nc, int nq, int64_t e, int comp) {
  return comp < 3 ? e * nq * 3 + comp : 3 * nc * nq + e * nq;
}
__device__ __forceinline__ int ev_step(int comp) { return comp < 3 ? 3 : 1; }

// weight of coarse node s for fine node t of a child in octant o (8: the
// same cell, identity)
__device__ __forceinline__ double embed_weight(const AmrEmbed &E, int oct, int t, int s) {
  const int q = E.k + 1;
  double w = 1.0;
  for (int a = 0; a < 3; ++a) {
    int ta = t, sa = s;
    for (int b = 0; b < a; ++b) {
      ta /= q;
      sa /= q;
    }
    ta %= q;
    sa %= q;
    if (oct == 8)
      w *= (ta == sa) ? 1.0 : 0.0;
    else
      w *= E.w[(oct >> a) & 1][ta][sa];
  }
  return w;
}

// fine[f][comp][t] = sum_s W(oct[f])[t][s] coarse[parent[f]][comp][s]
template <typename T>
__global__ void k_embed(AmrEmbed E, int64_t ncf, int64_t ncc, const int *parent, const uint8_t *oct, const T *evc,
                        T *evf) {
  const int nq = (E.k + 1) * (E.k + 1) * (E.k + 1);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ncf * 4 * nq) return;
  const int t = (int)(i % nq);
  const int comp = (int)((i / nq) % 4);
  const int64_t f = i / (4 * nq);
  const int64_t c = parent[f];
  const int o = oct[f];
  const T *src = evc + ev_at(ncc, nq, c, comp);
  const int st = ev_step(comp);
  double acc = 0.0;
  for (int s = 0; s < nq; ++s) {
    const double w = embed_weight(E, o, t, s);
    if (w != 0.0) acc += w * (double)src[s * st];
  }
  evf[ev_at(ncf, nq, f, comp) + t * st] = (T)acc;
}

// coarse[c][comp][s] = sum over the children f of c, sum_t W(oct[f])[t][s] fine[f][comp][t]
template <typename T>
__global__ void k_embed_t(AmrEmbed E, int64_t ncf, int64_t ncc, const int64_t *cptr, const int *child,
                          const uint8_t *oct, const T *evf, T *evc) {
  const int nq = (E.k + 1) * (E.k + 1) * (E.k + 1);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ncc * 4 * nq) return;
  const int s = (int)(i % nq);
  const int comp = (int)((i / nq) % 4);
  const int64_t c = i / (4 * nq);
  double acc = 0.0;
  for (int64_t e = cptr[c]; e < cptr[c + 1]; ++e) {
    const int64_t f = child[e];
    const int o = oct[f];
    const T *src = evf + ev_at(ncf, nq, f, comp);
    const int st = ev_step(comp);
    for (int t = 0; t < nq; ++t) {
      const double w = embed_weight(E, o, t, s);
      if (w != 0.0) acc += w * (double)src[t * st];
    }
  }
  evc[ev_at(ncc, nq, c, comp) + s * ev_step(comp)] = (T)acc;
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

template void amr_embed<double>(const AmrEmbed &, int64_t, int64_t, const int *, const uint8_t *, const double *,
                                double *, hipStream_t);
template void amr_embed<float>(const AmrEmbed &, int64_t, int64_t, const int *, const uint8_t *, const float *,
                               float *, hipStream_t);
template void amr_embed_t<double>(const AmrEmbed &, int64_t, int64_t, const int64_t *, const int *, const uint8_t *,
                                  const double *, double *, hipStream_t);
template void amr_embed_t<float>(const AmrEmbed &, int64_t, int64_t, const int64_t *, const int *, const uint8_t *,
                                 const float *, float *, hipStream_t);

}  // namespace mfs
