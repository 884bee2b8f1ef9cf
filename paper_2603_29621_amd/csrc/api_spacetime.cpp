// Space-time Kronecker operator G_Q (x) M + tau I_Q (x) A on stage-major vectors and
// the temporal stage transfers (Sec. 4 eq. (proceedings-kronecker)), with their C ABI.
#include "runtime.h"

namespace mfs {
namespace rt {

// Space-time Kronecker operator (Sec. 4 eq. (proceedings-kronecker)) on level
// 0: dst_q = sum_r G[q][r] M_u src_r + tau K src_q on the free rows, dst_q =
// src_q on the velocity Dirichlet rows; stage-major vectors of N entries per
// stage; work holds the Q stage masses (Q dim Nv).
template <typename T>
void st_apply(mfs_problem &P, int Q, const double *G, double tau, T *dst, const T *src, T *work, hipStream_t s) {
  const Level &L = P.L[0];
  const LevelGeom &g = L.g;
  const int64_t nv = P.dim * g.Nv, N = nv + g.Np;
  for (int r = 0; r < Q; ++r) apply_op<T>(P, MFS_OP_MASS_U, 0, work + r * nv, src + r * N, s);
  for (int q = 0; q < Q; ++q) {
    T *dq = dst + q * N;
    apply_op<T>(P, MFS_OP_STOKES, 0, dq, src + q * N, s);
    StageCoef C{};
    for (int r = 0; r < Q; ++r) C.c[r] = G[q * Q + r];
    stage_mix<T>(dq, N, 1, work, nv, Q, C, (T)tau, nv, N, s);
    vec_copy_boundary<T>(g, dq, src + q * N, s);  // identity rows
  }
}

// instantiations used by the other parts of the runtime
template void st_apply<float>(mfs_problem &P, int Q, const double *G, double tau, float *dst, const float *src, float *work, hipStream_t s);
template void st_apply<double>(mfs_problem &P, int Q, const double *G, double tau, double *dst, const double *src, double *work, hipStream_t s);

}  // namespace rt
}  // namespace mfs

extern "C" {

int mfs_st_vmult(mfs_problem *p, int Q, const double *G, double tau, int prec, void *dst, const void *src, void *work,
                 void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(!p->ns && !p->hp && !p->amr && p->L[0].g.Np > 0, MFS_EUNSUPPORTED,
                "the space-time operator needs a structured Taylor-Hood problem");
    MFS_REQUIRE(Q >= 1 && Q <= MFS_MAX_STAGES, MFS_EINVAL, "Q = %d outside [1, %d]", Q, MFS_MAX_STAGES);
    MFS_REQUIRE(G && dst && src && work && dst != src, MFS_EINVAL, "bad arguments");
    MFS_REQUIRE(tau > 0 && std::isfinite(tau), MFS_EINVAL, "tau must be positive");
    if (prec == MFS_FP64)
      st_apply<double>(*p, Q, G, tau, (double *)dst, (const double *)src, (double *)work, S(stream));
    else
      st_apply<float>(*p, Q, G, tau, (float *)dst, (const float *)src, (float *)work, S(stream));
  });
}

int mfs_st_stage_transfer(mfs_problem *p, int q_out, int q_in, const double *C, int prec, void *dst, const void *src,
                          void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(!p->hp && !p->amr, MFS_EUNSUPPORTED, "structured problems only");
    MFS_REQUIRE(q_out >= 1 && q_out <= MFS_MAX_STAGES && q_in >= 1 && q_in <= MFS_MAX_STAGES, MFS_EINVAL,
                "stage counts outside [1, %d]", MFS_MAX_STAGES);
    MFS_REQUIRE(C && dst && src && dst != src, MFS_EINVAL, "bad arguments");
    const LevelGeom &g = p->L[0].g;
    const int64_t N = p->dim * g.Nv + g.Np;
    StageCoef K{};
    for (int i = 0; i < q_out; ++i)
      for (int j = 0; j < q_in; ++j) K.c[i * MFS_MAX_STAGES + j] = C[i * q_in + j];
    if (prec == MFS_FP64)
      stage_mix<double>((double *)dst, N, q_out, (const double *)src, N, q_in, K, 0.0, N, N, S(stream));
    else
      stage_mix<float>((float *)dst, N, q_out, (const float *)src, N, q_in, K, 0.0f, N, N, S(stream));
  });
}

}  // extern "C"
