// Q2/Q1 Stokes operator application that allocates nothing, for callers that
// cannot allocate device memory.  The degree-2 brick kernel and its face-node
// combine are the ones mfs_vmult runs (operator of Sec. 1 eq. (stokes) in the
// symmetric block form of Sec. 3 eq. (stokes_block)); only their scratch (the
// per-brick face partial sums) lives in a static device array instead of a
// problem's allocation.
//
// The array's host-side name is not a device address: kernels get the
// address that hipGetSymbolAddress returns for the current device, taken once
// per device and kept.  Every call on a device shares that device's array, so
// calls that overlap on one GPU (different streams, or different host
// threads) race on it; calls in one stream are ordered and safe.  Each call
// writes every scratch slot it reads before reading it, so nothing has to be
// cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace mfs {
namespace {

constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[MFS_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};

void *scratch_on_current_device() {
  int dev = -1;
  MFS_HIP(hipGetDevice(&dev));
  MFS_REQUIRE(dev >= 0 && dev < MAX_DEVICES, MFS_EUNSUPPORTED, "device %d outside the supported range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void *p = nullptr;
    MFS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MFS_REQUIRE(p != nullptr, MFS_EHIP, "no device address for the static scratch");
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

LevelGeom q2q1_geom(const int n[3]) {
  LevelGeom g{};
  g.dim = 3;
  g.k = 2;
  g.kp = 1;
  g.ncells = 1;
  g.Nv = 1;
  g.Np = 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = n[a];
    g.nv[a] = 2 * n[a] + 1;
    g.np[a] = n[a] + 1;
    g.ncells *= n[a];
    g.Nv *= g.nv[a];
    g.Np *= g.np[a];
  }
  return g;
}

template <typename T>
void apply(const int n[3], const void *X, double nu, void *dst, const void *src, hipStream_t s) {
  const LevelGeom g = q2q1_geom(n);
  const int64_t need = q2_face_elems(g) * (int64_t)sizeof(T);
  MFS_REQUIRE(need <= (int64_t)MFS_NOALLOC_SCRATCH_BYTES, MFS_EINVAL,
              "mesh %dx%dx%d needs %lld scratch bytes, the static scratch holds %lld", n[0], n[1], n[2],
              (long long)need, (long long)MFS_NOALLOC_SCRATCH_BYTES);
  T *face = static_cast<T *>(scratch_on_current_device());
  T *du = static_cast<T *>(dst);
  const T *su = static_cast<const T *>(src);
  const bool ok = launch_stokes_q2<T>(g, static_cast<const T *>(X), Q2_STOKES, (T)nu, du, du + 3 * g.Nv, su,
                                      su + 3 * g.Nv, face, s);
  MFS_REQUIRE(ok, MFS_EUNSUPPORTED, "the degree-2 brick kernel does not take this mesh");
}

}  // namespace
}  // namespace mfs

extern "C" int mfs_stokes_vmult_noalloc(const int n[3], const void *vertices, double nu, int prec, void *dst,
                                        const void *src, void *stream) {
  using namespace mfs;
  try {
    MFS_REQUIRE(n != nullptr && vertices != nullptr && dst != nullptr && src != nullptr, MFS_EINVAL,
                "NULL argument");
    MFS_REQUIRE(dst != src, MFS_EINVAL, "dst and src must not alias");
    MFS_REQUIRE(prec == MFS_FP64 || prec == MFS_FP32, MFS_EINVAL, "precision must be MFS_FP64 or MFS_FP32");
    for (int a = 0; a < 3; ++a)
      MFS_REQUIRE(n[a] >= 1 && n[a] <= 4096, MFS_EINVAL, "cells per direction must be in [1, 4096]");
    MFS_REQUIRE(nu > 0, MFS_EINVAL, "nu must be positive");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (prec == MFS_FP64)
      apply<double>(n, vertices, nu, dst, src, s);
    else
      apply<float>(n, vertices, nu, dst, src, s);
    return MFS_OK;
  } catch (const mfs::Error &e) {
    return e.code;
  } catch (...) {
    set_error("unexpected exception");
    return MFS_EINVAL;
  }
}
