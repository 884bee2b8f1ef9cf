// Stokes operators (Sec. 1 eq. (stokes), Sec. 3 eq. (stokes_block)) on every level, the
// Chebyshev-smoothed V-cycle (Sec. 2, Sec. 3), the block-triangular preconditioner,
// and their C ABI (vmult, diagonal, V-cycle, transfers, preconditioner, right-hand side).
#include "runtime.h"

namespace mfs {
namespace rt {

template <typename T>
void apply_A(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s) {
  const Level &L = P.L[l];
  if (use_specialised() && q2_face_elems(L.g) > 0 &&
      launch_stokes_q2<T>(L.g, dev<T>(L).X, Q2_A, (T)P.nu, dst, nullptr, src, nullptr, face<T>(L), s))
    return;
  if (use_specialised() && q1_face_elems(L.g) > 0 &&
      launch_laplace_q1<T>(L.g, dev<T>(L).X, (T)P.nu, dst, src, face<T>(L), s))
    return;
  if (use_gather<T>(L)) {
    launch_cell_op_gather<T>(L.g, dev<T>(L), M_LAPLACE, (T)P.nu, dst, nullptr, src, nullptr, src, cellev<T>(L), s);
    return;
  }
  launch_fill_dirichlet<T>(L.g, dst, src, s);
  launch_cell_op<T>(L.g, dev<T>(L), M_LAPLACE, (T)P.nu, dst, nullptr, src, nullptr, s);
}

template <typename T>
void apply_op(mfs_problem &P, int op, int l, T *dst, const T *src, hipStream_t s) {
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int64_t nu = g.dim * g.Nv;
  if (op == MFS_OP_NS_JACOBIAN) {
    apply_ns<T>(P, l, dst, src, s);
    return;
  }
  MFS_REQUIRE(!P.ns, MFS_EUNSUPPORTED, "operator %d is not available on an equal-order (Navier-Stokes) problem",
              op);
  switch (op) {
    case MFS_OP_A:
      apply_A<T>(P, l, dst, src, s);
      break;
    case MFS_OP_STOKES:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_specialised() && q2_face_elems(g) > 0 &&
          launch_stokes_q2<T>(g, dev<T>(L).X, Q2_STOKES, (T)P.nu, dst, dst + nu, src, src + nu, face<T>(L), s))
        break;
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_LAPLACE | M_GRADP | M_DIVU, (T)P.nu, dst, dst + nu, src, src + nu,
                                 src, cellev<T>(L), s);
        break;
      }
      launch_fill_dirichlet<T>(g, dst, src, s);
      vec_fill<T>(dst + nu, T(0), g.Np, s);
      launch_cell_op<T>(g, dev<T>(L), M_LAPLACE | M_GRADP | M_DIVU, (T)P.nu, dst, dst + nu, src, src + nu, s);
      break;
    case MFS_OP_B:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_specialised() && q2_face_elems(g) > 0 &&
          launch_stokes_q2<T>(g, dev<T>(L).X, Q2_B, (T)P.nu, dst, nullptr, nullptr, src, face<T>(L), s))
        break;
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_GRADP, (T)P.nu, dst, nullptr, nullptr, src, nullptr, cellev<T>(L), s);
        break;
      }
      launch_fill_dirichlet<T>(g, dst, (const T *)nullptr, s);
      launch_cell_op<T>(g, dev<T>(L), M_GRADP, (T)P.nu, dst, nullptr, nullptr, src, s);
      break;
    case MFS_OP_BT:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_DIVU, (T)P.nu, nullptr, dst, src, nullptr, nullptr, cellev<T>(L), s);
        break;
      }
      vec_fill<T>(dst, T(0), g.Np, s);
      launch_cell_op<T>(g, dev<T>(L), M_DIVU, (T)P.nu, nullptr, dst, src, nullptr, s);
      break;
    case MFS_OP_MASS_U:
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_MASSU, (T)P.nu, dst, nullptr, src, nullptr, src, cellev<T>(L), s);
        break;
      }
      launch_fill_dirichlet<T>(g, dst, src, s);
      launch_cell_op<T>(g, dev<T>(L), M_MASSU, (T)P.nu, dst, nullptr, src, nullptr, s);
      break;
    case MFS_OP_MASS_P:
      MFS_REQUIRE(g.kp > 0, MFS_EINVAL, "level %d has no pressure space", l);
      if (use_specialised() && q2_face_elems(g) > 0 &&
          launch_stokes_q2<T>(g, dev<T>(L).X, Q2_MASSP, (T)P.nu, nullptr, dst, nullptr, src, face<T>(L), s))
        break;
      if (use_gather<T>(L)) {
        launch_cell_op_gather<T>(g, dev<T>(L), M_MASSP, (T)P.nu, nullptr, dst, nullptr, src, nullptr, cellev<T>(L), s);
        break;
      }
      vec_fill<T>(dst, T(0), g.Np, s);
      launch_cell_op<T>(g, dev<T>(L), M_MASSP, (T)P.nu, nullptr, dst, nullptr, src, s);
      break;
    default:
      MFS_REQUIRE(false, MFS_EUNSUPPORTED, "operator %d not available", op);
  }
}

// ---------------------------------------------------------------- V-cycle
template <typename T>
void chebyshev(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s) {
  Level &L = P.L[l];
  PrecWork<T> &W = work<T>(P);
  const double lmax = L.lambda, lmin = lmax / P.opts.cheb_range;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho_old = 1.0 / sigma;
  T *Ax = W.r[l], *d = W.d[l];
  // x += d with d from the residual b - A x: fused into the brick kernels
  // where the level has one, and into the node gather on the levels that sum
  // cell-local results
  auto step = [&](T c1, T c2, bool first) {
    if (use_specialised() && q2_face_elems(L.g) > 0 &&
        launch_q2_cheb<T>(L.g, dev<T>(L).X, (T)P.nu, x, d, b, invdiag<T>(L), c1, c2, first, face<T>(L), s))
      return;
    if (use_specialised() && q1_face_elems(L.g) > 0 &&
        launch_q1_cheb<T>(L.g, dev<T>(L).X, (T)P.nu, x, d, b, invdiag<T>(L), c1, c2, first, face<T>(L), s))
      return;
    if (use_gather<T>(L) && L.g.dim == 3 && L.g.k >= 3) {
      launch_cell_cheb_gather<T>(L.g, dev<T>(L), (T)P.nu, x, d, b, invdiag<T>(L), c1, c2, first, cellev<T>(L), s);
      return;
    }
    apply_A<T>(P, l, Ax, x, s);
    cheb_update<T>(L.g, x, d, b, Ax, invdiag<T>(L), c1, c2, first, s);
  };
  if (zero_start)  // x on entry is ignored: x = b on the Dirichlet rows, 0 elsewhere, then the first step
    cheb_start<T>(L.g, x, d, b, invdiag<T>(L), (T)(1.0 / theta), s);
  else
    step(T(0), (T)(1.0 / theta), true);
  for (int it = 1; it < P.opts.cheb_degree; ++it) {
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    step((T)(rho * rho_old), (T)(2.0 * rho / delta), false);
    rho_old = rho;
  }
}

template <typename T>
void vcycle_level(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  Level &L = P.L[l];
  if (l == P.nlev - 1) {
    dense_apply<T>(P.coarse_inv, P.coarse_n, b, x, s);
    return;
  }
  const int64_t n = P.dim * L.g.Nv;
  chebyshev<T>(P, l, x, b, true, s);  // from x = b on Dirichlet rows, 0 elsewhere
  T *r = W.r[l];
  apply_A<T>(P, l, r, x, s);
  vec_axpby<T>(r, T(1), b, T(-1), n, s);  // r = b - A x
  Level &C = P.L[l + 1];
  launch_restrict<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), W.b[l + 1], r, s, 0, rwork<T>(L));
  vcycle_level<T>(P, l + 1, W.x[l + 1], W.b[l + 1], s);
  launch_prolongate_add<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), x, W.x[l + 1], s);
  chebyshev<T>(P, l, x, b, false, s);
}

// ---------------------------------------------------------------- block preconditioner
template <typename T>
void precondition(mfs_problem &P, T *y, const T *r, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  const LevelGeom &g = P.L[0].g;
  const int64_t nu = P.dim * g.Nv, np = g.Np;
  const T *rp = r + nu;
  T *yp = y + nu;
  // Schur: y_p = -nu M_p^{-1} r_p, M_p^{-1} by Jacobi-PCG (z0 = 0)
  double *rho = P.scal, *pqs = P.scal + PCG_MAX;
  vec_fill<T>(W.pz, T(0), np, s);
  vec_copy<T>(W.pres, rp, np, s);
  vec_mul<T>(W.ps, W.pinv, W.pres, np, s);
  vec_copy<T>(W.pp, W.ps, np, s);
  multi_dot<T>(W.pres, 0, 1, W.ps, np, rho, P.partials, s);
  for (int it = 0; it < P.opts.schur_iterations; ++it) {
    apply_op<T>(P, MFS_OP_MASS_P, 0, W.pq, W.pp, s);
    multi_dot<T>(W.pp, 0, 1, W.pq, np, pqs + it, P.partials, s);
    pcg_update1<T>(W.pz, W.pres, W.ps, W.pp, W.pq, W.pinv, np, rho + it, pqs + it, s);
    multi_dot<T>(W.pres, 0, 1, W.ps, np, rho + it + 1, P.partials, s);
    pcg_update2<T>(W.pp, W.ps, np, rho + it + 1, rho + it, s);
  }
  vec_axpby<T>(yp, (T)(-P.nu), W.pz, T(0), np, s);
  // velocity: y_u = Vcycle(r_u - B y_p)
  apply_op<T>(P, MFS_OP_B, 0, W.t_u, yp, s);
  vec_axpby<T>(W.t_u, T(1), r, T(-1), nu, s);
  vcycle_level<T>(P, 0, y, W.t_u, s);
}

// instantiations used by the other parts of the runtime
template void apply_A<float>(mfs_problem &P, int l, float *dst, const float *src, hipStream_t s);
template void apply_A<double>(mfs_problem &P, int l, double *dst, const double *src, hipStream_t s);
template void apply_op<float>(mfs_problem &P, int op, int l, float *dst, const float *src, hipStream_t s);
template void apply_op<double>(mfs_problem &P, int op, int l, double *dst, const double *src, hipStream_t s);
template void chebyshev<float>(mfs_problem &P, int l, float *x, const float *b, bool zero_start, hipStream_t s);
template void chebyshev<double>(mfs_problem &P, int l, double *x, const double *b, bool zero_start, hipStream_t s);
template void vcycle_level<float>(mfs_problem &P, int l, float *x, const float *b, hipStream_t s);
template void vcycle_level<double>(mfs_problem &P, int l, double *x, const double *b, hipStream_t s);
template void precondition<float>(mfs_problem &P, float *y, const float *r, hipStream_t s);
template void precondition<double>(mfs_problem &P, double *y, const double *r, hipStream_t s);

}  // namespace rt
}  // namespace mfs

extern "C" {

int mfs_vmult(mfs_problem *p, int op, int prec, int level, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_level(p, level);
    check_prec(prec);
    MFS_REQUIRE(dst && src, MFS_EINVAL, "NULL vector");
    MFS_REQUIRE(dst != src, MFS_EINVAL, "dst and src must not alias");
    if (p->amr) {
      if (level < p->namr) {
        amr_vmult(*p, op, prec, level, dst, src, S(stream));
        return;
      }
      level -= p->namr;
    }
    if (p->hp) {
      hp_vmult(*p, op, prec, level, dst, src, S(stream));
      return;
    }
    if (prec == MFS_FP64)
      apply_op<double>(*p, op, level, (double *)dst, (const double *)src, S(stream));
    else
      apply_op<float>(*p, op, level, (float *)dst, (const float *)src, S(stream));
  });
}

int mfs_diagonal(mfs_problem *p, int level, double *dst, void *stream) {
  return guard([&] {
    check_level(p, level);
    MFS_REQUIRE(dst != nullptr, MFS_EINVAL, "NULL vector");
    hipStream_t s = S(stream);
    if (p->amr) {
      MFS_REQUIRE(p->amr->mg, MFS_EUNSUPPORTED, "problem was set up without multigrid levels");
      MFS_REQUIRE(p->amr->ready, MFS_EINVAL, "mfs_set_linearization has not been called");
      if (level < p->namr) {
        AmrLevel &V = p->amr->lev[level];
        vec_copy<double>(dst, V.diag, 4 * V.N, s);
        return;
      }
      level -= p->namr;
    }
    if (p->hp && level < p->nhp) {
      vec_copy<double>(dst, p->hp->lev[level].diag, p->hp->lev[level].V.N, s);
      return;
    }
    if (p->hp) level -= p->nhp;
    const Level &L = p->L[level];
    if (p->ns) {
      MFS_REQUIRE(p->ns_ready, MFS_EINVAL, "mfs_set_linearization has not been called");
      ns_diagonal(*p, level, dst, s);
      return;
    }
    vec_fill<double>(dst, 0.0, L.g.Nv, s);
    launch_laplace_diagonal(L.g, L.X64, L.tab64, p->nu, dst, s);
    // Dirichlet rows: 1 (identity rows of the constrained operator)
    launch_reciprocal_boundary_one(L.g, dst, s);
  });
}

int mfs_vcycle(mfs_problem *p, int prec, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(p->opts.mg_levels, MFS_EINVAL, "problem was set up without multigrid levels");
    MFS_REQUIRE(dst && src && dst != src, MFS_EINVAL, "bad vectors");
    MFS_REQUIRE(!p->ns || (p->ns_ready && p->ns_mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    MFS_REQUIRE(!p->amr || (p->amr->ready && p->amr->mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    if (p->amr) {
      if (prec == MFS_FP64)
        amr_vcycle<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
      else
        amr_vcycle<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
    } else if (p->hp) {
      if (prec == MFS_FP64)
        hp_vcycle<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
      else
        hp_vcycle<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
    } else if (p->ns) {
      if (prec == MFS_FP64)
        ns_vcycle<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
      else
        ns_vcycle<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
    } else if (prec == MFS_FP64)
      vcycle_level<double>(*p, 0, (double *)dst, (const double *)src, S(stream));
    else
      vcycle_level<float>(*p, 0, (float *)dst, (const float *)src, S(stream));
  });
}

int mfs_prolongate_add(mfs_problem *p, int prec, int fine, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_level(p, fine);
    check_prec(prec);
    MFS_REQUIRE(fine + 1 < p->namr + p->nhp + p->nlev, MFS_EINVAL, "no coarser level below %d", fine);
    if (p->amr) {
      if (fine < p->namr) {
        if (prec == MFS_FP64)
          amr_prolongate_add<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
        else
          amr_prolongate_add<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
        return;
      }
      fine -= p->namr;
    }
    if (fine < p->nhp) {
      if (prec == MFS_FP64)
        hp_prolongate_add<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
      else
        hp_prolongate_add<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
      return;
    }
    fine -= p->nhp;
    const Level &F = p->L[fine], &C = p->L[fine + 1];
    const int ncp = p->ns ? 1 : 0;
    if (prec == MFS_FP64)
      launch_prolongate_add<double>(F.g, C.g, F.h_to_coarser, F.emb.data(), (double *)dst, (const double *)src,
                                    S(stream), ncp);
    else
      launch_prolongate_add<float>(F.g, C.g, F.h_to_coarser, F.emb.data(), (float *)dst, (const float *)src,
                                   S(stream), ncp);
  });
}

int mfs_restrict(mfs_problem *p, int prec, int fine, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_level(p, fine);
    check_prec(prec);
    MFS_REQUIRE(fine + 1 < p->namr + p->nhp + p->nlev, MFS_EINVAL, "no coarser level below %d", fine);
    if (p->amr) {
      if (fine < p->namr) {
        if (prec == MFS_FP64)
          amr_restrict<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
        else
          amr_restrict<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
        return;
      }
      fine -= p->namr;
    }
    if (fine < p->nhp) {
      if (prec == MFS_FP64)
        hp_restrict<double>(*p, fine, (double *)dst, (const double *)src, S(stream));
      else
        hp_restrict<float>(*p, fine, (float *)dst, (const float *)src, S(stream));
      return;
    }
    fine -= p->nhp;
    const Level &F = p->L[fine], &C = p->L[fine + 1];
    const int ncp = p->ns ? 1 : 0;
    if (prec == MFS_FP64)
      launch_restrict<double>(F.g, C.g, F.h_to_coarser, F.emb.data(), (double *)dst, (const double *)src, S(stream),
                              ncp, F.rs64);
    else
      launch_restrict<float>(F.g, C.g, F.h_to_coarser, F.emb.data(), (float *)dst, (const float *)src, S(stream),
                             ncp, F.rs32);
  });
}

int mfs_precondition(mfs_problem *p, int prec, void *dst, const void *src, void *stream) {
  return guard([&] {
    check_problem(p);
    check_prec(prec);
    MFS_REQUIRE(p->opts.mg_levels && (p->hp || p->L[0].g.Np > 0), MFS_EINVAL,
                "needs multigrid levels and a pressure space");
    MFS_REQUIRE(dst && src && dst != src, MFS_EINVAL, "bad vectors");
    MFS_REQUIRE(!p->ns || (p->ns_ready && p->ns_mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    MFS_REQUIRE(!p->amr || (p->amr->ready && p->amr->mg_ready), MFS_EINVAL,
                "mfs_set_linearization has not been called (or the state was set without multigrid data)");
    if (prec == MFS_FP64)
      precondition_any<double>(*p, (double *)dst, (const double *)src, S(stream));
    else
      precondition_any<float>(*p, (float *)dst, (const float *)src, S(stream));
  });
}

int mfs_rhs(mfs_problem *p, const double *f_qp, const double *u_dirichlet, double *b, void *stream) {
  return guard([&] {
    no_amr(p, "mfs_rhs");
    check_problem(p);
    MFS_REQUIRE(f_qp && u_dirichlet && b, MFS_EINVAL, "NULL vector");
    MFS_REQUIRE(!p->ns, MFS_EUNSUPPORTED, "mfs_rhs assembles the Stokes right-hand side only");
    MFS_REQUIRE(!p->hp, MFS_EUNSUPPORTED, "mfs_rhs is not provided for hp problems");
    const Level &L = p->L[0];
    const LevelGeom &g = L.g;
    MFS_REQUIRE(g.Np > 0, MFS_EINVAL, "needs a pressure space");
    hipStream_t s = S(stream);
    const int64_t nu = p->dim * g.Nv, n = nu + g.Np;
    double *t = p->tmp_full;
    // t = K_unconstrained * lifting, free velocity rows and all pressure rows
    launch_fill_dirichlet<double>(g, t, (const double *)nullptr, s);
    vec_fill<double>(t + nu, 0.0, g.Np, s);
    launch_cell_op<double>(g, dev<double>(L), M_LAPLACE | M_DIVU, p->nu, t, t + nu, u_dirichlet, nullptr, s, true);
    // b = (f, phi) - t on free rows; u_D on Dirichlet rows; -t on pressure rows
    launch_fill_dirichlet<double>(g, b, u_dirichlet, s);
    vec_fill<double>(b + nu, 0.0, g.Np, s);
    launch_load_vector(g, L.X64, L.tab64, f_qp, b, s);
    vec_axpby<double>(b, -1.0, t, 1.0, n, s);
    (void)n;
  });
}

}  // extern "C"
