// Device kernels of the hp spaces (Sec. 3, minimum rule): gather of
// cell-local values through the sparse local->global map, its transpose
// (scatter, deterministic: one thread per global unknown), the per-cell tensor
// embedding between degrees used by the p-transfers, owner injection,
// permutations, masked smoother updates and colour probes for diagonals.
#include "hp.h"

namespace mfs {

namespace {

constexpr int HB = 256;
unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + HB - 1) / HB, 65535 * 8)); }

// NC components at once: the map entries are read once
template <typename T, int NC>
__global__ void k_gather(HpMaps M, const T *x, T *ev) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < M.nrows; r += (int64_t)gridDim.x * blockDim.x) {
    const int c0 = M.rcol[r];
    T out[NC];
    if (c0 >= 0) {  // plain row
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) out[comp] = x[comp * M.N + c0];
    } else {
      const int64_t h = -1 - (int64_t)c0;
      double s[NC] = {};
      for (int64_t j = M.hptr[h]; j < M.hptr[h + 1]; ++j) {
        const double w = M.hval[j];
        const int64_t c = M.hcol[j];
#pragma unroll
        for (int comp = 0; comp < NC; ++comp) s[comp] += w * (double)x[comp * M.N + c];
      }
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) out[comp] = (T)s[comp];
    }
    const int64_t base = M.rslot[r];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) ev[base + (int64_t)comp * M.nb] = out[comp];
  }
}

template <typename T, int NC>
__global__ void k_scatter(HpMaps M, const uint8_t *dir, const T *ev, const T *src, T *dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M.N; i += (int64_t)gridDim.x * blockDim.x) {
    if (dir != nullptr && dir[i]) {
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) dst[comp * M.N + i] = src ? src[comp * M.N + i] : T(0);
      continue;
    }
    const int64_t b = M.tptr[i], e = M.tptr[i + 1], wb = M.wptr[i], we = M.wptr[i + 1];
    if ((e - b) + (we - wb) > HP_SCATTER_LIGHT) continue;  // summed by k_scatter_heavy
    double s[NC] = {};
    for (int64_t j = b; j < e; ++j) {
      const int64_t o = M.tslot[j];
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) s[comp] += (double)ev[o + comp * M.nb];
    }
    for (int64_t j = wb; j < we; ++j) {
      const double w = M.wval[j];
      const int64_t o = M.wslot[j];
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) s[comp] += w * (double)ev[o + comp * M.nb];
    }
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) dst[comp * M.N + i] = (T)s[comp];
  }
}

// one wave per long list: strided partial sums over the lanes (plain rows,
// then weighted rows), then a butterfly over the wave (the same order on
// every call)
template <typename T, int NC>
__global__ void __launch_bounds__(HB) k_scatter_heavy(HpMaps M, const T *ev, T *dst) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t h = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; h < M.nheavy; h += waves) {
    const int64_t i = M.heavy[h];
    const int64_t b = M.tptr[i], nu = M.tptr[i + 1] - b, wb = M.wptr[i], nw = M.wptr[i + 1] - wb;
    double s[NC] = {};
    for (int64_t j = lane; j < nu + nw; j += 64) {
      const double w = j < nu ? 1.0 : M.wval[wb + j - nu];
      const int64_t o = j < nu ? M.tslot[b + j] : M.wslot[wb + j - nu];
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) s[comp] += w * (double)ev[o + comp * M.nb];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) s[comp] += __shfl_xor(s[comp], off, 64);
    if (lane == 0)
#pragma unroll
      for (int comp = 0; comp < NC; ++comp) dst[comp * M.N + i] = (T)s[comp];
  }
}

// one workgroup per cell; three 1D passes through LDS
template <typename T>
__global__ void __launch_bounds__(256) k_embed(int64_t ncells, int ncomp, const int *kf, const int *kc,
                                               const double *tables, const int64_t *off_f, const int64_t *off_c,
                                               const T *in, T *out, int transpose) {
  __shared__ double s_a[MAXQ * MAXQ * MAXQ];
  __shared__ double s_b[MAXQ * MAXQ * MAXQ];
  __shared__ double s_E[MAXQ * MAXQ];
  const int64_t c = blockIdx.x;
  if (c >= ncells) return;
  const int f1 = kf[c] + 1, c1 = kc[c] + 1;
  const double *E = tables + ((int64_t)kf[c] * MAXQ + kc[c]) * MAXQ * MAXQ;  // [fine][coarse]
  for (int i = threadIdx.x; i < MAXQ * MAXQ; i += blockDim.x) s_E[i] = E[i];
  // input extent ni per direction, output extent no
  const int ni = transpose ? f1 : c1, no = transpose ? c1 : f1;
  const int64_t oi = transpose ? off_f[c] : off_c[c], oo = transpose ? off_c[c] : off_f[c];
  const int sin3 = ni * ni * ni, sout3 = no * no * no;
  for (int comp = 0; comp < ncomp; ++comp) {
    __syncthreads();
    for (int i = threadIdx.x; i < sin3; i += blockDim.x) s_a[i] = (double)in[oi + (int64_t)i * ncomp + comp];
    __syncthreads();
    // x: [l][j][i_in] -> [l][j][i_out]
    for (int t = threadIdx.x; t < no * ni * ni; t += blockDim.x) {
      const int io = t % no, j = (t / no) % ni, l = t / (no * ni);
      double s = 0;
      for (int m = 0; m < ni; ++m) s += (transpose ? s_E[m * MAXQ + io] : s_E[io * MAXQ + m]) * s_a[m + ni * (j + ni * l)];
      s_b[io + no * (j + ni * l)] = s;
    }
    __syncthreads();
    // y
    for (int t = threadIdx.x; t < no * no * ni; t += blockDim.x) {
      const int i = t % no, jo = (t / no) % no, l = t / (no * no);
      double s = 0;
      for (int m = 0; m < ni; ++m) s += (transpose ? s_E[m * MAXQ + jo] : s_E[jo * MAXQ + m]) * s_b[i + no * (m + ni * l)];
      s_a[i + no * (jo + no * l)] = s;
    }
    __syncthreads();
    // z
    for (int t = threadIdx.x; t < sout3; t += blockDim.x) {
      const int i = t % no, j = (t / no) % no, lo = t / (no * no);
      double s = 0;
      for (int m = 0; m < ni; ++m) s += (transpose ? s_E[m * MAXQ + lo] : s_E[lo * MAXQ + m]) * s_a[i + no * (j + no * m)];
      out[oo + (int64_t)t * ncomp + comp] = (T)s;
    }
  }
}

template <typename T>
__global__ void k_inject(int64_t N, int ncomp, const int64_t *owner_ev, const int *owner_nb, const T *ev, T *x,
                         int add) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = owner_ev[g];
    if (o < 0) continue;
    for (int comp = 0; comp < ncomp; ++comp) {
      const T v = ev[o + (int64_t)comp * owner_nb[g]];
      if (add)
        x[comp * N + g] += v;
      else
        x[comp * N + g] = v;
    }
  }
}

template <typename T>
__global__ void k_inject_t(int64_t N, int ncomp, const int64_t *owner_ev, const int *owner_nb, const T *x, T *ev) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = owner_ev[g];
    if (o < 0) continue;
    for (int comp = 0; comp < ncomp; ++comp) ev[o + (int64_t)comp * owner_nb[g]] = x[comp * N + g];
  }
}

template <typename T>
__global__ void k_permute(int64_t n, int ncomp, const int64_t *perm, const T *x, int64_t Nx, T *y, int64_t Ny,
                          int scatter) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int comp = 0; comp < ncomp; ++comp) {
      if (scatter)
        y[comp * Ny + perm[i]] = x[comp * Nx + i];
      else
        y[comp * Ny + i] = x[comp * Nx + perm[i]];
    }
}

template <typename T>
__global__ void k_mask_fill(const uint8_t *mask, int64_t N, int ncomp, T *x, const T *src) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    for (int comp = 0; comp < ncomp; ++comp) x[comp * N + i] = (mask[i] && src) ? src[comp * N + i] : T(0);
}

template <typename T>
__global__ void k_mask_diag_scale(const uint8_t *mask, int64_t N, int ncomp, T *y, const T *invdiag, const T *x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    for (int comp = 0; comp < ncomp; ++comp) y[comp * N + i] = mask[i] ? T(0) : invdiag[i] * x[comp * N + i];
}

template <typename T>
__global__ void k_mask_cheb(const uint8_t *mask, int64_t N, int ncomp, T *x, T *d, const T *b, const T *Ax,
                            const T *invdiag, T c1, T c2, int first) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    if (mask[i]) continue;
    for (int comp = 0; comp < ncomp; ++comp) {
      const int64_t k = comp * N + i;
      const T r = invdiag[i] * (b[k] - (Ax ? Ax[k] : T(0)));
      const T dn = first ? c2 * r : c1 * d[k] + c2 * r;
      d[k] = dn;
      x[k] += dn;
    }
  }
}

__global__ void k_colour_ind(const int *colour, int64_t N, int c0, int c1, int c2, double *out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = colour[i];
    out[i] = c == c0 ? 1.0 : 0.0;
    out[N + i] = c == c1 ? 1.0 : 0.0;
    out[2 * N + i] = c == c2 ? 1.0 : 0.0;
  }
}

__global__ void k_colour_ext(const int *colour, int64_t N, int c0, int c1, int c2, const double *y, double *diag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = colour[i];
    if (c == c0) diag[i] = y[i];
    if (c == c1) diag[i] = y[N + i];
    if (c == c2) diag[i] = y[2 * N + i];
  }
}

}  // namespace

template <typename T>
void hp_gather(const HpMaps &M, int ncomp, const T *x, T *ev, hipStream_t s) {
  if (M.nrows == 0) return;
  if (ncomp == 3)
    hipLaunchKernelGGL((k_gather<T, 3>), dim3(grid_for(M.nrows)), dim3(HB), 0, s, M, x, ev);
  else
    hipLaunchKernelGGL((k_gather<T, 1>), dim3(grid_for(M.nrows)), dim3(HB), 0, s, M, x, ev);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void hp_scatter(const HpMaps &M, int ncomp, const uint8_t *dirichlet, const T *ev, const T *src, T *dst,
                hipStream_t s) {
  if (M.N == 0) return;
  const unsigned hgrid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>((M.nheavy + HB / 64 - 1) / (HB / 64), 65535 * 8));
  if (ncomp == 3) {
    hipLaunchKernelGGL((k_scatter<T, 3>), dim3(grid_for(M.N)), dim3(HB), 0, s, M, dirichlet, ev, src, dst);
    if (M.nheavy > 0) hipLaunchKernelGGL((k_scatter_heavy<T, 3>), dim3(hgrid), dim3(HB), 0, s, M, ev, dst);
  } else {
    hipLaunchKernelGGL((k_scatter<T, 1>), dim3(grid_for(M.N)), dim3(HB), 0, s, M, dirichlet, ev, src, dst);
    if (M.nheavy > 0) hipLaunchKernelGGL((k_scatter_heavy<T, 1>), dim3(hgrid), dim3(HB), 0, s, M, ev, dst);
  }
  MFS_HIP(hipGetLastError());
}

template <typename T>
void hp_embed(int64_t ncells, int ncomp, const int *kf, const int *kc, const double *tables, const int64_t *off_f,
              const int64_t *off_c, const T *in, T *out, bool transpose, hipStream_t s) {
  if (ncells == 0) return;
  hipLaunchKernelGGL(k_embed<T>, dim3((unsigned)ncells), dim3(256), 0, s, ncells, ncomp, kf, kc, tables, off_f,
                     off_c, in, out, transpose ? 1 : 0);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void hp_inject(int64_t N, int ncomp, const int64_t *owner_ev, const int *owner_nb, const T *ev, T *x, bool add,
               hipStream_t s) {
  hipLaunchKernelGGL(k_inject<T>, dim3(grid_for(N)), dim3(HB), 0, s, N, ncomp, owner_ev, owner_nb, ev, x,
                     add ? 1 : 0);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void hp_inject_t(int64_t N, int ncomp, const int64_t *owner_ev, const int *owner_nb, const T *x, T *ev,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_inject_t<T>, dim3(grid_for(N)), dim3(HB), 0, s, N, ncomp, owner_ev, owner_nb, x, ev);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void permute(int64_t n, int ncomp, const int64_t *perm, const T *x, int64_t Nx, T *y, int64_t Ny, bool scatter,
             hipStream_t s) {
  hipLaunchKernelGGL(k_permute<T>, dim3(grid_for(n)), dim3(HB), 0, s, n, ncomp, perm, x, Nx, y, Ny, scatter ? 1 : 0);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void mask_fill_dirichlet(const uint8_t *mask, int64_t N, int ncomp, T *x, const T *src, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_fill<T>, dim3(grid_for(N)), dim3(HB), 0, s, mask, N, ncomp, x, src);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void mask_diag_scale(const uint8_t *mask, int64_t N, int ncomp, T *y, const T *invdiag, const T *x, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_diag_scale<T>, dim3(grid_for(N)), dim3(HB), 0, s, mask, N, ncomp, y, invdiag, x);
  MFS_HIP(hipGetLastError());
}

template <typename T>
void mask_cheb_update(const uint8_t *mask, int64_t N, int ncomp, T *x, T *d, const T *b, const T *Ax,
                      const T *invdiag, T c1, T c2, bool first, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_cheb<T>, dim3(grid_for(N)), dim3(HB), 0, s, mask, N, ncomp, x, d, b, Ax, invdiag, c1, c2,
                     first ? 1 : 0);
  MFS_HIP(hipGetLastError());
}

void colour_indicator(const int *colour, int64_t N, const int cols[3], double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_colour_ind, dim3(grid_for(N)), dim3(HB), 0, s, colour, N, cols[0], cols[1], cols[2], out);
  MFS_HIP(hipGetLastError());
}

void colour_extract(const int *colour, int64_t N, const int cols[3], const double *y, double *diag, hipStream_t s) {
  hipLaunchKernelGGL(k_colour_ext, dim3(grid_for(N)), dim3(HB), 0, s, colour, N, cols[0], cols[1], cols[2], y, diag);
  MFS_HIP(hipGetLastError());
}

#define HP_INST(T)                                                                                                   \
  template void hp_gather<T>(const HpMaps &, int, const T *, T *, hipStream_t);                                     \
  template void hp_scatter<T>(const HpMaps &, int, const uint8_t *, const T *, const T *, T *, hipStream_t);         \
  template void hp_embed<T>(int64_t, int, const int *, const int *, const double *, const int64_t *,                \
                            const int64_t *, const T *, T *, bool, hipStream_t);                                     \
  template void hp_inject<T>(int64_t, int, const int64_t *, const int *, const T *, T *, bool, hipStream_t);        \
  template void hp_inject_t<T>(int64_t, int, const int64_t *, const int *, const T *, T *, hipStream_t);            \
  template void permute<T>(int64_t, int, const int64_t *, const T *, int64_t, T *, int64_t, bool, hipStream_t);     \
  template void mask_fill_dirichlet<T>(const uint8_t *, int64_t, int, T *, const T *, hipStream_t);                 \
  template void mask_diag_scale<T>(const uint8_t *, int64_t, int, T *, const T *, const T *, hipStream_t);          \
  template void mask_cheb_update<T>(const uint8_t *, int64_t, int, T *, T *, const T *, const T *, const T *, T, T, \
                                    bool, hipStream_t);
HP_INST(double)
HP_INST(float)
#undef HP_INST

}  // namespace mfs
