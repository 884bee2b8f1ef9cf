// Equal-order SUPG/PSPG Navier-Stokes on structured meshes (Sec. 5): the Jacobian, its
// linearisation at a general state, the residual, the monolithic multigrid data
// (Jacobi diagonals, additive Schwarz patch inverses, pinned coarse inverse), the
// relaxation and V-cycle, and the BDF2 / Newton-Krylov step, with their C ABI.
#include "runtime.h"

namespace mfs {
namespace rt {

// constrained Navier-Stokes Jacobian on level l: identity on the velocity
// Dirichlet rows, cell terms elsewhere (Dirichlet source values ignored)
template <typename T>
void apply_ns(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s) {
  MFS_REQUIRE(P.ns, MFS_EINVAL, "the Navier-Stokes Jacobian needs a problem set up with pressure_offset = 0");
  MFS_REQUIRE(P.ns_ready, MFS_EINVAL, "mfs_set_linearization has not been called");
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  // 3D: cell-local outputs and a deterministic node gather instead of global
  // atomics (at 128^3 Q2Q2 the FP32 atomics cost 45% of the Jacobian; with
  // the cell-local rows laid out for the gather it pays in FP64 too)
  if (g.dim == 3 && cellev<T>(L) != nullptr) {
    T *ev = cellev<T>(L);
    launch_ns<T>(g, dev<T>(L).X, dev<T>(L).tab, 1, (T)P.nu, (T)P.ns_dt, P.ns_newton, src, dst,
                 const_cast<T *>(ns_qd<T>(L)), s, ev);
    const int64_t q = g.k + 1;
    launch_node_gather<T>(g, g.k, g.k, ev, ev + g.ncells * 3 * q * q * q, dst, dst + g.dim * g.Nv, src, s);
    return;
  }
  launch_fill_dirichlet<T>(g, dst, src, s);
  vec_fill<T>(dst + g.dim * g.Nv, T(0), g.Nv, s);
  launch_ns<T>(g, dev<T>(L).X, dev<T>(L).tab, 1, (T)P.nu, (T)P.ns_dt, P.ns_newton, src, dst,
               const_cast<T *>(ns_qd<T>(L)), s);
}

// ---------------------------------------------------------------- Navier-Stokes set-up
// diag(J) on level l: J applied to the indicator of one node colour and one
// component at a time (colour = node index mod (k+1) per direction, so no two
// nodes of a colour share a cell and each row sees only its own column)
void ns_diagonal(mfs_problem &P, int l, double *diag, hipStream_t s) {
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int q = g.k + 1;
  int ncol = 1;
  for (int a = 0; a < g.dim; ++a) ncol *= q;
  double *e = P.tmp_full, *y = P.tmp2;
  for (int c = 0; c < ncol; ++c)
    for (int comp = 0; comp <= P.dim; ++comp) {
      launch_color_indicator(g, P.dim + 1, q, c, comp, e, s);
      apply_ns<double>(P, l, y, e, s);
      launch_color_extract(g, q, c, comp, y, diag, s);
    }
}

// dense inverse of the coarsest J with pressure node 0 pinned; columns of J
// from colourings with spacing 2k+1 (the stencils of two nodes of a colour
// do not overlap, so every entry of J e_colour belongs to one column)
void ns_setup_coarse(mfs_problem &P, hipStream_t s) {
  const int l = P.nlev - 1;
  const Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int n = P.coarse_n;
  const int64_t Nv = g.Nv;
  const int k = g.k, q = 2 * k + 1;
  int ncol = 1;
  for (int a = 0; a < g.dim; ++a) ncol *= q;
  std::vector<double> A((size_t)n * n, 0.0), y(n);  // row-major
  double *e = P.tmp_full, *yd = P.tmp2;
  auto coord = [&](int64_t i, int c[3]) {
    c[0] = (int)(i % g.nv[0]);
    c[1] = (int)((i / g.nv[0]) % g.nv[1]);
    c[2] = (int)(i / ((int64_t)g.nv[0] * g.nv[1]));
  };
  for (int col = 0; col < ncol; ++col)
    for (int comp = 0; comp <= P.dim; ++comp) {
      launch_color_indicator(g, P.dim + 1, q, col, comp, e, s);
      apply_ns<double>(P, l, yd, e, s);
      MFS_HIP(hipMemcpyAsync(y.data(), yd, n * sizeof(double), hipMemcpyDeviceToHost, s));
      MFS_HIP(hipStreamSynchronize(s));
      for (int64_t j = 0; j < Nv; ++j) {
        int cj[3];
        coord(j, cj);
        if (cj[0] % q + q * (cj[1] % q + q * (cj[2] % q)) != col) continue;
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::max(0, cj[a] - k);
          hi[a] = std::min(g.nv[a] - 1, cj[a] + k);
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
          for (int yy = lo[1]; yy <= hi[1]; ++yy)
            for (int x = lo[0]; x <= hi[0]; ++x) {
              const int64_t i = x + (int64_t)g.nv[0] * (yy + (int64_t)g.nv[1] * z);
              for (int r = 0; r <= P.dim; ++r)
                A[(size_t)(r * Nv + i) * n + comp * Nv + j] = y[r * Nv + i];
            }
      }
    }
  const int pin = (int)(P.dim * Nv);
  for (int i = 0; i < n; ++i) {
    A[(size_t)pin * n + i] = 0.0;
    A[(size_t)i * n + pin] = 0.0;
  }
  A[(size_t)pin * n + pin] = 1.0;
  // LU with partial pivoting (row-major, in place)
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)pr * n + c])) pr = r;
    MFS_REQUIRE(A[(size_t)pr * n + c] != 0.0, MFS_EINVAL, "coarse Navier-Stokes matrix is singular");
    piv[c] = pr;
    if (pr != c)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)pr * n + j]);
    const double inv = 1.0 / A[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      const double f = A[(size_t)r * n + c] * inv;
      A[(size_t)r * n + c] = f;
      if (f != 0.0)
        for (int j = c + 1; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
    }
  }
  // inverse, column-major for dense_apply; the pinned column is dropped
  std::vector<double> inv((size_t)n * n, 0.0), v(n);
  for (int c = 0; c < n; ++c) {
    if (c == pin) continue;
    std::fill(v.begin(), v.end(), 0.0);
    v[c] = 1.0;
    for (int i = 0; i < n; ++i) std::swap(v[i], v[piv[i]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) v[i] -= A[(size_t)i * n + j] * v[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) v[i] -= A[(size_t)i * n + j] * v[j];
      v[i] /= A[(size_t)i * n + i];
    }
    std::copy(v.begin(), v.end(), inv.begin() + (size_t)c * n);
  }
  MFS_HIP(hipMemcpyAsync(P.coarse_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MFS_HIP(hipStreamSynchronize(s));
}

// Additive Schwarz patch inverses of level l at the current linearisation:
// column j of every patch matrix of a colour from one FP64 Jacobian apply to
// the sum of the colour's unit vectors at local index j, then a batched
// inversion; the FP32 copy serves the FP32 multigrid.
void ns_asm_setup(mfs_problem &P, int l, hipStream_t s) {
  Level &L = P.L[l];
  const LevelGeom &g = L.g;
  const int64_t n = (P.dim + 1) * g.Nv;
  const int np = asm_patch_size(g);
  double *x = P.w64.b[l], *y = P.w64.r[l];
  vec_fill<double>(x, 0.0, n, s);
  for (int c = 0; c < asm_colours(g); ++c)
    for (int j = 0; j < np; ++j) {
      launch_asm_probe_set(g, x, c, j, 1.0, s);
      apply_ns<double>(P, l, y, x, s);
      launch_asm_probe_extract(g, y, L.asm64, c, j, s);
      launch_asm_probe_set(g, x, c, j, 0.0, s);
    }
  MFS_HIP(hipMemsetAsync(P.flags, 0, sizeof(int), s));
  launch_asm_invert(g, L.asm64, P.flags, s);
  int bad = 0;
  MFS_HIP(hipMemcpyAsync(&bad, P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  MFS_REQUIRE(bad == 0, MFS_EINVAL, "singular additive Schwarz patch matrix on level %d", l);
  vec_cast<float, double>(L.asm32, L.asm64, asm_patch_count(g) * np * np, s);
}

// Jacobi diagonals (or Schwarz patch inverses) and the pinned coarse inverse
// of the current linearisation
void ns_mg_data(mfs_problem &P, hipStream_t s) {
  if (!P.opts.mg_levels) return;
  for (int l = 0; l + 1 < P.nlev; ++l) {
    Level &L = P.L[l];
    const int64_t n = (P.dim + 1) * L.g.Nv;
    double *d = P.w64.x[l];
    ns_diagonal(P, l, d, s);
    launch_reciprocal(L.nsinv64, L.nsinv32, d, n, s);
    if (L.asm64) ns_asm_setup(P, l, s);
  }
  ns_setup_coarse(P, s);
}

// Linearisation at the state x0 = [u0 | p0] ((dim+1) Nv) with the BDF2
// history u~ (dim Nv; NULL: u~ = u0), on every level (the coarse levels take
// the fields at their nodes, which are fine nodes); keep_delta leaves
// delta_1 as the previous linearisation stored it; mg: also the multigrid
// data (diagonals, coarse inverse).  Host-synchronous.
void ns_set_point(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta, bool mg,
                  hipStream_t s) {
  P.ns_ready = false;
  P.ns_mg_ready = false;
  P.ns_dt = dt;
  P.ns_newton = newton ? 1 : 0;
  const int d = P.dim;
  const int64_t Nv = P.L[0].g.Nv;
  double *st = P.L[0].u0;
  MFS_HIP(hipMemcpyAsync(st, x0, (d + 1) * Nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  MFS_HIP(hipMemcpyAsync(st + (d + 1) * Nv, uh ? uh : x0, d * Nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int l = 1; l < P.nlev; ++l) launch_ns_inject(P.L[l - 1].g, P.L[l].g, P.L[l - 1].u0, P.L[l].u0, s, 2 * d + 1);
  NsPoint<double> pt;
  pt.keep_delta = keep_delta;
  for (int l = 0; l < P.nlev; ++l) {
    Level &L = P.L[l];
    launch_ns<double>(L.g, L.X64, L.tab64, 0, P.nu, dt, P.ns_newton, L.u0, nullptr, L.qd64, s, nullptr, nullptr,
                      nullptr, &pt);
    vec_cast<float, double>(L.qd32, L.qd64, ns_qd_elems(L.g), s);
  }
  P.ns_ready = true;
  try {
    if (mg) {
      ns_mg_data(P, s);
      P.ns_mg_ready = true;
    }
    MFS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    P.ns_ready = false;
    throw;
  }
}

// Linearisation point u0 of a Jacobian alone: p0 = 0 and u~ = u0
void ns_set_linearization(mfs_problem &P, const double *u0, double dt, int newton, hipStream_t s) {
  const int64_t nv = P.dim * P.L[0].g.Nv;
  double *x0 = P.tmp2;
  MFS_HIP(hipMemcpyAsync(x0, u0, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  vec_fill<double>(x0 + nv, 0.0, P.L[0].g.Nv, s);
  ns_set_point(P, x0, nullptr, dt, newton, 0, true, s);
}

// F = the nonlinear residual at the level-0 state of the last linearisation;
// Dirichlet velocity rows 0
void ns_residual(mfs_problem &P, double *F, hipStream_t s) {
  MFS_REQUIRE(P.ns_ready, MFS_EINVAL, "no linearisation state: call mfs_set_linearization_point first");
  Level &L = P.L[0];
  const LevelGeom &g = L.g;
  launch_fill_dirichlet<double>(g, F, (const double *)nullptr, s);
  vec_fill<double>(F + g.dim * g.Nv, 0.0, g.Nv, s);
  launch_ns<double>(g, L.X64, L.tab64, 2, P.nu, P.ns_dt, P.ns_newton, nullptr, F, L.qd64, s);
}

// ---------------------------------------------------------------- Navier-Stokes V-cycle
// One monolithic V-cycle on J (Sec. 5): x = (b on Dirichlet rows, 0 free),
// relax_steps damped Jacobi sweeps, restriction of the residual (pressure
// unconstrained), recursion, prolongation, relax_steps sweeps; on the
// coarsest level x = C b with the pinned dense inverse C.
template <typename T>
void ns_relax(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  const Level &L = P.L[l];
  const int64_t n = (P.dim + 1) * L.g.Nv;
  for (int it = 0; it < P.opts.relax_steps; ++it) {
    // from the zero start (x = b on the Dirichlet rows, 0 elsewhere) J x = x
    // exactly: identity rows, Dirichlet source values ignored in the others
    if (zero_start && it == 0)
      vec_copy<T>(W.d[l], x, n, s);
    else
      apply_ns<T>(P, l, W.d[l], x, s);
    if (L.asm64) {  // additive Schwarz: every colour with the residual b - J x of the sweep's start
      const T *Minv = sizeof(T) == 8 ? (const T *)L.asm64 : (const T *)L.asm32;
      for (int c = 0; c < asm_colours(L.g); ++c)
        launch_asm_apply<T>(L.g, Minv, c, b, W.d[l], x, (T)P.opts.relax_omega, s);
    } else {
      jacobi_relax<T>(x, b, W.d[l], ns_invdiag<T>(L), (T)P.opts.relax_omega, n, s);
    }
  }
}

template <typename T>
void ns_vcycle(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  PrecWork<T> &W = work<T>(P);
  Level &L = P.L[l];
  if (l == P.nlev - 1) {
    dense_apply<T>(P.coarse_inv, P.coarse_n, b, x, s);
    return;
  }
  const int64_t n = (P.dim + 1) * L.g.Nv;
  launch_fill_dirichlet<T>(L.g, x, b, s);
  vec_fill<T>(x + P.dim * L.g.Nv, T(0), L.g.Nv, s);
  ns_relax<T>(P, l, x, b, true, s);
  T *r = W.r[l];
  apply_ns<T>(P, l, r, x, s);
  vec_axpby<T>(r, T(1), b, T(-1), n, s);  // r = b - J x
  Level &C = P.L[l + 1];
  launch_restrict<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), W.b[l + 1], r, s, 1, rwork<T>(L));
  ns_vcycle<T>(P, l + 1, W.x[l + 1], W.b[l + 1], s);
  launch_prolongate_add<T>(L.g, C.g, L.h_to_coarser, L.emb.data(), x, W.x[l + 1], s, 1);
  ns_relax<T>(P, l, x, b, false, s);
}

// the state of a Navier-Stokes problem (structured or refined) at x0 = [u0 | p0]
void set_point_any(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta, bool mg,
                   hipStream_t s) {
  if (P.amr)
    amr_set_point(P, x0, uh, dt, newton, keep_delta, mg, s);
  else
    ns_set_point(P, x0, uh, dt, newton, keep_delta, mg, s);
}

// multigrid data (Jacobi diagonals, coarse inverse) of the current state
void point_mg_any(mfs_problem &P, hipStream_t s) {
  ns_mg_data(P, s);
  P.ns_mg_ready = true;
  if (P.amr) {
    AmrData &A = *P.amr;
    for (int j = 0; j < amr_nop(A); ++j) {
      AmrLevel &V = A.lev[j];
      amr_diagonal(P, j, V.diag, s);
      launch_reciprocal(V.inv64, V.inv32, V.diag, 4 * V.N, s);
    }
    A.mg_ready = true;
  }
  MFS_HIP(hipStreamSynchronize(s));
}

double device_norm(mfs_problem &P, const double *v, int64_t n, hipStream_t s) {
  Krylov &K = P.kr;
  multi_dot<double>(v, 0, 1, v, n, K.dev + 110, P.partials, s);
  MFS_HIP(hipMemcpyAsync(K.host + 110, K.dev + 110, sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  return std::sqrt(std::max(K.host[110], 0.0));
}

// One BDF2 step (Sec. 5) by Newton's method: F(x) = 0 with the time
// derivative alpha (u - u~), u~ = (4 u^n - u^{n-1}) / 3, delta_1 frozen at u^n
// for the whole step (so J is the exact derivative of F); each correction
// J dx = -F by FGMRES with the monolithic multigrid preconditioner.  x holds
// the initial guess with the new time level's Dirichlet values on entry.
void bdf2_step(mfs_problem &P, const double *u_n, const double *u_nm1, double *x, double dt,
               const mfs_newton_options &o, mfs_newton_info &info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  info = mfs_newton_info{};
  const int64_t nvel = sys_vel(P), n = sys_n(P);
  // the recorded preconditioner keeps dt and the Newton flag: drop it when they change
  if (P.ns_dt != dt || P.ns_newton != 1) drop_prec_graph(P);
  // u~ and delta_1 at u^n (state [u^n; 0])
  vec_copy<double>(P.nw_uh, u_n, nvel, s);
  vec_axpby<double>(P.nw_uh, -1.0 / 3.0, u_nm1, 4.0 / 3.0, nvel, s);
  double *st = P.nw_dx;
  vec_copy<double>(st, u_n, nvel, s);
  vec_fill<double>(st + nvel, 0.0, n - nvel, s);
  set_point_any(P, st, u_n, dt, 1, 0, false, s);
  mfs_options lo = P.opts;
  lo.rtol = o.linear_rtol;
  lo.maxit = o.linear_maxit;
  lo.precond_precision = o.precond_precision;
  for (int it = 0;; ++it) {
    set_point_any(P, x, P.nw_uh, dt, 1, 1, false, s);
    if (P.amr)
      amr_residual(P, P.nw_F, s);
    else
      ns_residual(P, P.nw_F, s);
    const double r = device_norm(P, P.nw_F, n, s);
    if (it == 0) info.res0 = r;
    info.res = r;
    info.newton_iterations = it;
    if (r <= std::max(o.rtol * info.res0, o.atol) || r == 0.0) {
      info.status = MFS_OK;
      break;
    }
    if (it == o.max_newton) {
      info.status = MFS_ENOCONV;
      break;
    }
    point_mg_any(P, s);
    vec_axpby<double>(P.nw_F, 0.0, P.nw_F, -1.0, n, s);  // b = -F
    // no need to solve beyond a tenth of the Newton target (and rounding
    // would stop FGMRES short of a relative tolerance far below it)
    const double target = std::max(o.rtol * info.res0, o.atol);
    lo.rtol = std::min(0.5, std::max(o.linear_rtol, 0.1 * target / r));
    kr_begin(P, P.nw_F, P.nw_dx, lo, s);
    Krylov &K = P.kr;
    while (K.state != 4) {
      MFS_HIP(hipEventSynchronize(K.ev));
      kr_process(P);
    }
    info.linear_iterations += K.info.iterations;
    if (K.info.status != MFS_OK) info.linear_failures += 1;
    vec_axpby<double>(x, 1.0, P.nw_dx, 1.0, n, s);  // x += dx
  }
  MFS_HIP(hipStreamSynchronize(s));
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// instantiations used by the other parts of the runtime
template void apply_ns<float>(mfs_problem &P, int l, float *dst, const float *src, hipStream_t s);
template void apply_ns<double>(mfs_problem &P, int l, double *dst, const double *src, hipStream_t s);
template void ns_relax<float>(mfs_problem &P, int l, float *x, const float *b, bool zero_start, hipStream_t s);
template void ns_relax<double>(mfs_problem &P, int l, double *x, const double *b, bool zero_start, hipStream_t s);
template void ns_vcycle<float>(mfs_problem &P, int l, float *x, const float *b, hipStream_t s);
template void ns_vcycle<double>(mfs_problem &P, int l, double *x, const double *b, hipStream_t s);

}  // namespace rt
}  // namespace mfs

extern "C" {

void mfs_default_newton_options(mfs_newton_options *o) {
  if (!o) return;
  o->max_newton = 20;
  o->rtol = 1e-8;
  o->atol = 0.0;
  o->linear_rtol = 1e-6;
  o->linear_maxit = 200;
  o->precond_precision = MFS_FP32;
}

int mfs_set_linearization_point(mfs_problem *p, const double *x0, const double *u_hist, double dt, int newton,
                                int keep_delta, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "linearisation needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(x0 != nullptr, MFS_EINVAL, "x0 is NULL");
    MFS_REQUIRE(dt > 0 && std::isfinite(dt), MFS_EINVAL, "dt must be positive");
    MFS_REQUIRE(!keep_delta || (p->amr ? p->amr->ready : p->ns_ready), MFS_EINVAL,
                "keep_delta needs an earlier linearisation");
    drop_prec_graph(*p);
    set_point_any(*p, x0, u_hist, dt, newton, keep_delta, p->opts.mg_levels != 0, S(stream));
  });
}

int mfs_ns_residual(mfs_problem *p, double *F, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "the residual needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(F != nullptr, MFS_EINVAL, "F is NULL");
    if (p->amr)
      amr_residual(*p, F, S(stream));
    else
      ns_residual(*p, F, S(stream));
  });
}

int mfs_ns_bdf2_step(mfs_problem *p, const double *u_n, const double *u_nm1, double *x, double dt,
                     const mfs_newton_options *opts, mfs_newton_info *info, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "the BDF2 step needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(p->opts.mg_levels, MFS_EINVAL, "the BDF2 step needs the multigrid hierarchy (mg_levels = 1)");
    MFS_REQUIRE(u_n && u_nm1 && x, MFS_EINVAL, "NULL vector");
    MFS_REQUIRE(dt > 0 && std::isfinite(dt), MFS_EINVAL, "dt must be positive");
    mfs_newton_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_newton_options(&o);
    MFS_REQUIRE(o.max_newton >= 0 && o.max_newton <= 1000 && o.rtol >= 0 && o.atol >= 0 && o.linear_rtol > 0 &&
                    o.linear_maxit >= 1,
                MFS_EINVAL, "bad Newton options");
    check_prec(o.precond_precision);
    mfs_newton_info inf{};
    bdf2_step(*p, u_n, u_nm1, x, dt, o, inf, S(stream));
    if (info) *info = inf;
    if (inf.status != MFS_OK) {
      set_error("Newton did not reach rtol %.3e within %d iterations (||F|| %.3e from %.3e)", o.rtol, o.max_newton,
                inf.res, inf.res0);
      throw mfs::Error{MFS_ENOCONV};
    }
  });
}

int mfs_set_linearization(mfs_problem *p, const double *u0, double dt, int newton, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(p->ns, MFS_EINVAL, "linearisation needs a problem set up with pressure_offset = 0");
    MFS_REQUIRE(u0 != nullptr, MFS_EINVAL, "u0 is NULL");
    MFS_REQUIRE(dt > 0 && std::isfinite(dt), MFS_EINVAL, "dt must be positive");
    drop_prec_graph(*p);
    if (p->amr)
      amr_set_linearization(*p, u0, dt, newton, S(stream));
    else
      ns_set_linearization(*p, u0, dt, newton, S(stream));
  });
}

}  // extern "C"
