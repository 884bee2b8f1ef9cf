// FGMRES with an FP64 outer iteration and an FP32 or FP64 preconditioner (Sec. 3): the
// system and preconditioner dispatch over problem kinds, the recorded preconditioner
// graphs, the resumable iteration state machine, and the C ABI for solves and grouped
// serving steps.
#include "runtime.h"

namespace mfs {
namespace rt {

void apply_system(mfs_problem &P, double *dst, const double *src, hipStream_t s) {
  if (P.amr) {
    amr_apply_ns<double>(P, 0, dst, src, s);
    return;
  }
  if (P.hp) {
    const int64_t nu = 3 * P.hp->lev[0].vd.N;
    hp_apply<double>(P, 0, M_LAPLACE | M_GRADP | M_DIVU, dst, dst + nu, src, src + nu, s);
    return;
  }
  apply_op<double>(P, P.ns ? MFS_OP_NS_JACOBIAN : MFS_OP_STOKES, 0, dst, src, s);
}

// sizes of the system vectors
int64_t sys_vel(const mfs_problem &P) {
  if (P.amr) return 3 * P.amr->lev[0].N;
  return P.hp ? 3 * P.hp->lev[0].vd.N : P.dim * P.L[0].g.Nv;
}

int64_t sys_pres(const mfs_problem &P) {
  if (P.amr) return P.amr->lev[0].N;
  return P.hp ? P.hp->pd.N : P.L[0].g.Np;
}

int64_t sys_n(const mfs_problem &P) { return sys_vel(P) + sys_pres(P); }

template <typename T>
void precondition_any(mfs_problem &P, T *y, const T *r, hipStream_t s) {
  if (P.amr)
    amr_vcycle<T>(P, 0, y, r, s);
  else if (P.hp)
    hp_precondition<T>(P, y, r, s);
  else if (P.ns)
    ns_vcycle<T>(P, 0, y, r, s);
  else
    precondition<T>(P, y, r, s);
}

// The recorded preconditioner holds host values that were current when it
// was recorded (smoother intervals, the linearisation's dt and Newton flag,
// option counts); calls that change them drop the recording.
void drop_prec_graph(mfs_problem &P) {
  for (int i = 0; i < 2; ++i) {
    if (P.prec_graph[i]) (void)hipGraphExecDestroy(P.prec_graph[i]);
    P.prec_graph[i] = nullptr;
  }
}

// Preconditioner from full_in to full_out of the precision's work vectors on
// stream s.  Its launches (a few hundred small kernels per V-cycle and Schur
// solve, no host synchronisation and no memset) are recorded once on a
// private stream and replayed as one graph launch, so that small problems do
// not pay the host cost of every launch in each FGMRES iteration.  Recording
// that fails (e.g. a runtime without stream capture) falls back to direct
// launches.  The FP64 one is staged through fixed vectors too, since the
// Krylov columns it reads and writes move every iteration.
template <typename T>
void precondition_rec(mfs_problem &P, hipStream_t s) {
  constexpr int w = sizeof(T) == 8 ? 1 : 0;
  T *y = prec_work<T>(P).full_out, *r = prec_work<T>(P).full_in;
  if (!P.kr.graphs || P.graph_failed) {
    precondition_any<T>(P, y, r, s);
    return;
  }
  if (!P.prec_graph[w]) {
    if (!P.cap_stream) P.cap_stream = capture_stream_acquire();
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      P.graph_failed = true;
      precondition_any<T>(P, y, r, s);
      return;
    }
    try {
      precondition_any<T>(P, y, r, P.cap_stream);
    } catch (...) {
      if (hipStreamEndCapture(P.cap_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      throw;
    }
    MFS_HIP(hipStreamEndCapture(P.cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&P.prec_graph[w], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      P.prec_graph[w] = nullptr;
      P.graph_failed = true;
      precondition_any<T>(P, y, r, s);
      return;
    }
  }
  MFS_HIP(hipGraphLaunch(P.prec_graph[w], s));
}

// ---------------------------------------------------------------- FGMRES
void kr_enqueue_residual(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  apply_system(P, K.w, K.x, s);
  vec_axpby<double>(K.w, 1.0, K.b, -1.0, n, s);  // w = b - K x
  multi_dot<double>(K.w, 0, 1, K.w, n, K.dev + 96, P.partials, s);
  MFS_HIP(hipMemcpyAsync(K.host + 96, K.dev + 96, sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipEventRecord(K.ev, s));
}

// one Arnoldi step: z_j = P^{-1} v_j (pre), w = K z_j (the system
// operator), Gram-Schmidt and the readback (post)
void kr_step_pre(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  const int j = K.j;
  double *vj = K.V + (int64_t)j * K.ld, *zj = K.Z + (int64_t)j * K.ld;
  if (K.prec == MFS_FP32) {
    vec_cast<float, double>(P.w32.full_in, vj, n, s);
    precondition_rec<float>(P, s);
    vec_cast<double, float>(zj, P.w32.full_out, n, s);
  } else if (K.graphs && !P.graph_failed) {
    vec_copy<double>(P.w64.full_in, vj, n, s);
    precondition_rec<double>(P, s);
    vec_copy<double>(zj, P.w64.full_out, n, s);
  } else {
    precondition_any<double>(P, zj, vj, s);
  }
}

void kr_enqueue_step(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  kr_step_pre(P, s);
  apply_system(P, K.w, K.Z + (int64_t)K.j * K.ld, s);
  kr_step_post(P, s);
}

void kr_step_post(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  const int j = K.j;
  // classical Gram-Schmidt, twice
  // (the second pass's dots and the norm are fused with the updates before them)
  multi_dot<double>(K.V, K.ld, j + 1, K.w, n, K.dev, P.partials, s);
  axpy_dot<double>(K.w, K.V, K.ld, j + 1, K.dev, j + 1, false, n, K.dev + 32, P.partials, s);
  axpy_dot<double>(K.w, K.V, K.ld, j + 1, K.dev + 32, 0, true, n, K.dev + 64, P.partials, s);
  scale_inv_sqrt<double>(K.V + (int64_t)(j + 1) * K.ld, K.w, n, K.dev + 64, s);
  MFS_HIP(hipMemcpyAsync(K.host, K.dev, 65 * sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipEventRecord(K.ev, s));
}

// update x with the current Krylov coefficients (j columns) and enqueue the
// true-residual check
void kr_enqueue_update(mfs_problem &P, hipStream_t s) {
  Krylov &K = P.kr;
  const int64_t n = sys_n(P);
  const int m = K.j;
  if (m > 0) {
    std::vector<double> y(m);
    for (int i = m - 1; i >= 0; --i) {
      double v = K.gv[i];
      for (int c = i + 1; c < m; ++c) v -= K.H[i * K.m + c] * y[c];
      y[i] = v / K.H[i * K.m + i];
    }
    MFS_HIP(hipStreamSynchronize(s));  // previous use of yhost finished
    std::memcpy(K.yhost, y.data(), m * sizeof(double));
    MFS_HIP(hipMemcpyAsync(K.ydev, K.yhost, m * sizeof(double), hipMemcpyHostToDevice, s));
    multi_combine<double>(K.x, K.Z, K.ld, m, K.ydev, n, true, s);
  }
  kr_enqueue_residual(P, s);
}

void kr_finish(mfs_problem &P, double rel, int status) {
  Krylov &K = P.kr;
  hipStream_t s = K.s;
  const int64_t nu = sys_vel(P), np = sys_pres(P);
  const double *m1 = P.amr ? P.amr->ones : P.hp ? P.hp->m1 : P.m1;
  // pressure with zero mass-weighted mean (Navier-Stokes: m1 = 1, nodal mean)
  if (np > 0) {
    double *num = P.scal + 4 * PCG_MAX + 8, *den = num + 1;
    double *ones = P.amr ? P.amr->scratch : P.hp ? P.hp->ones : P.tmp_full;  // scratch of >= np entries
    multi_dot<double>(m1, 0, 1, K.x + nu, np, num, P.partials, s);
    vec_fill<double>(ones, 1.0, np, s);
    multi_dot<double>(m1, 0, 1, ones, np, den, P.partials, s);
    shift_mean(K.x + nu, np, num, den, s);
  }
  MFS_HIP(hipStreamSynchronize(s));
  K.info.iterations = K.iters;
  K.info.status = status;
  K.info.rel_residual = rel;
  K.info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - K.t0).count();
  K.state = 4;
}

// advance the state machine after its event completed; with `defer` an
// Arnoldi step is not enqueued but reported (true) for the caller to enqueue
bool kr_process(mfs_problem &P, bool defer) {
  Krylov &K = P.kr;
  hipStream_t s = K.s;
  const int64_t n = sys_n(P);
  if (K.state == 1 || K.state == 3) {
    const double rr = std::sqrt(std::max(K.host[96], 0.0));
    const double rel = rr / K.bnorm;  // kr_begin set bnorm = ||b||, or 1 for b = 0
    if (rel <= K.rtol || K.iters >= K.maxit) {
      kr_finish(P, rel, rel <= K.rtol ? MFS_OK : MFS_ENOCONV);
      return false;
    }
    // (re)start: V_0 = r / ||r||
    K.beta = rr;
    std::fill(K.H.begin(), K.H.end(), 0.0);
    std::fill(K.gv.begin(), K.gv.end(), 0.0);
    K.gv[0] = rr;
    K.j = 0;
    scale_inv_sqrt<double>(K.V, K.w, n, K.dev + 96, s);
    K.state = 2;
    if (defer) return true;
    kr_enqueue_step(P, s);
    return false;
  }
  if (K.state == 2) {
    const int j = K.j, m = K.m;
    // column j of the Hessenberg matrix
    std::vector<double> h(j + 2);
    for (int i = 0; i <= j; ++i) h[i] = K.host[i] + K.host[32 + i];
    h[j + 1] = std::sqrt(std::max(K.host[64], 0.0));
    for (int i = 0; i < j; ++i) {
      const double t = K.cs[i] * h[i] + K.sn[i] * h[i + 1];
      h[i + 1] = -K.sn[i] * h[i] + K.cs[i] * h[i + 1];
      h[i] = t;
    }
    const double den = std::hypot(h[j], h[j + 1]);
    K.cs[j] = den > 0 ? h[j] / den : 1.0;
    K.sn[j] = den > 0 ? h[j + 1] / den : 0.0;
    h[j] = den;
    K.gv[j + 1] = -K.sn[j] * K.gv[j];
    K.gv[j] = K.cs[j] * K.gv[j];
    for (int i = 0; i <= j; ++i) K.H[i * m + j] = h[i];
    K.j = j + 1;
    K.iters += 1;
    const double est = std::fabs(K.gv[j + 1]) / K.bnorm;
    const bool breakdown = !(h[j] > 0) || K.host[64] <= 0.0;
    if (est <= K.rtol || K.j == m || K.iters >= K.maxit || breakdown) {
      K.state = 3;
      kr_enqueue_update(P, s);
      return false;
    }
    if (defer) return true;
    kr_enqueue_step(P, s);
  }
  return false;
}

// a structured Taylor-Hood problem whose system operator is the degree-2
// brick kernel (its Arnoldi steps can share one grouped operator launch)
bool q2_groupable(const mfs_problem &P) {
  if (P.hp || P.amr || P.ns || !use_specialised()) return false;
  const LevelGeom &g = P.L[0].g;
  return g.dim == 3 && g.k == 2 && g.kp == 1 && q2_face_elems(g) > 0;
}

void kr_begin(mfs_problem &P, const double *b, double *x, const mfs_options &o, hipStream_t s) {
  Krylov &K = P.kr;
  MFS_REQUIRE(P.opts.mg_levels, MFS_EINVAL, "solve needs the multigrid hierarchy (mg_levels = 1)");
  MFS_REQUIRE(P.hp || P.L[0].g.Np > 0, MFS_EINVAL, "solve needs a pressure space");
  MFS_REQUIRE(!P.ns || (P.ns_ready && P.ns_mg_ready), MFS_EINVAL,
              "mfs_set_linearization has not been called (or the state was set without multigrid data)");
  MFS_REQUIRE(!P.amr || (P.amr->ready && P.amr->mg_ready), MFS_EINVAL,
              "mfs_set_linearization has not been called (or the state was set without multigrid data)");
  const LevelGeom &g = P.L[0].g;
  const int64_t n = sys_n(P);
  K.b = b;
  K.x = x;
  K.s = s;
  K.rtol = o.rtol;
  K.maxit = o.maxit;
  K.prec = o.precond_precision;
  K.graphs = o.graphs != 0;
  K.iters = 0;
  K.j = 0;
  K.H.assign((size_t)(K.m + 1) * K.m, 0.0);
  K.cs.assign(K.m, 0.0);
  K.sn.assign(K.m, 0.0);
  K.gv.assign(K.m + 1, 0.0);
  K.info = mfs_solve_info{};
  K.t0 = std::chrono::steady_clock::now();
  // ||b|| first (state 1 reads it as bnorm), then the residual of x0
  if (P.amr)  // x0: lifting of b's Dirichlet rows
    mask_fill_dirichlet<double>(P.amr->lev[0].M.dir, P.amr->lev[0].N, 3, x, b, s);
  else if (P.hp)
    mask_fill_dirichlet<double>(P.hp->lev[0].vd.dir, P.hp->lev[0].vd.N, 3, x, b, s);
  else
    launch_fill_dirichlet<double>(g, x, b, s);
  vec_fill<double>(x + sys_vel(P), 0.0, sys_pres(P), s);
  multi_dot<double>(b, 0, 1, b, n, K.dev + 100, P.partials, s);
  MFS_HIP(hipMemcpyAsync(K.host + 100, K.dev + 100, sizeof(double), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  K.bnorm = std::sqrt(std::max(K.host[100], 0.0));
  if (K.bnorm == 0.0) K.bnorm = 1.0;
  K.state = 1;
  kr_enqueue_residual(P, s);
}

// instantiations used by the other parts of the runtime
template void precondition_any<float>(mfs_problem &P, float *y, const float *r, hipStream_t s);
template void precondition_any<double>(mfs_problem &P, double *y, const double *r, hipStream_t s);
template void precondition_rec<float>(mfs_problem &P, hipStream_t s);
template void precondition_rec<double>(mfs_problem &P, hipStream_t s);

}  // namespace rt
}  // namespace mfs

extern "C" {

int mfs_solve_begin(mfs_problem *p, const double *b, double *x, const mfs_options *opts, void *stream) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(b && x && (const void *)b != (void *)x, MFS_EINVAL, "bad vectors");
    mfs_options o = opts ? *opts : p->opts;
    MFS_REQUIRE(o.rtol > 0 && o.maxit >= 1, MFS_EINVAL, "bad rtol / maxit");
    check_prec(o.precond_precision);
    kr_begin(*p, b, x, o, S(stream));
  });
}

int mfs_solve_advance(mfs_problem *p, int *done, mfs_solve_info *info) {
  return guard([&] {
    check_problem(p);
    MFS_REQUIRE(done != nullptr, MFS_EINVAL, "done is NULL");
    Krylov &K = p->kr;
    *done = 0;
    if (K.state == 4) {
      *done = 1;
      if (info) *info = K.info;
      return;
    }
    MFS_REQUIRE(K.state != 0, MFS_EINVAL, "no solve in progress");
    const hipError_t q = hipEventQuery(K.ev);
    if (q == hipErrorNotReady) return;
    MFS_HIP(q);
    kr_process(*p);
    if (K.state == 4) {
      *done = 1;
      if (info) *info = K.info;
    }
  });
}

int mfs_batch_step(mfs_problem **ps, int n, void *stream, int *done, mfs_solve_info *infos) {
  return guard([&] {
    MFS_REQUIRE(n >= 0 && (n == 0 || (ps != nullptr && done != nullptr)), MFS_EINVAL, "bad problem list");
    for (int i = 0; i < n; ++i) {
      MFS_REQUIRE(ps[i] != nullptr, MFS_EINVAL, "problem %d is NULL", i);
      for (int j = 0; j < i; ++j) MFS_REQUIRE(ps[j] != ps[i], MFS_EINVAL, "problem %d is listed twice", i);
    }
    std::vector<mfs_problem *> group;
    for (int i = 0; i < n; ++i) {
      mfs_problem &P = *ps[i];
      Krylov &K = P.kr;
      done[i] = 0;
      if (K.state != 4) {
        MFS_REQUIRE(K.state != 0, MFS_EINVAL, "problem %d has no solve in progress", i);
        const hipError_t q = hipEventQuery(K.ev);
        if (q == hipErrorNotReady) continue;
        MFS_HIP(q);
        const bool step = kr_process(P, true);
        if (step) {
          if (q2_groupable(P))
            group.push_back(&P);
          else
            kr_enqueue_step(P, K.s);
        }
      }
      if (K.state == 4) {
        done[i] = 1;
        if (infos) infos[i] = K.info;
      }
    }
    if (group.size() == 1) {
      kr_enqueue_step(*group[0], group[0]->kr.s);
      return;
    }
    if (group.empty()) return;
    // preconditioners on the problems' streams, one grouped system operator
    // on `stream`, Gram-Schmidt and readbacks on the problems' streams again
    hipStream_t gs = S(stream);
    std::vector<Q2Problem<double>> q(group.size());
    for (size_t i = 0; i < group.size(); ++i) {
      mfs_problem &P = *group[i];
      Krylov &K = P.kr;
      kr_step_pre(P, K.s);
      MFS_HIP(hipEventRecord(K.ev_pre, K.s));
      MFS_HIP(hipStreamWaitEvent(gs, K.ev_pre, 0));
      const Level &L = P.L[0];
      q[i] = Q2Problem<double>{L.g, L.X64, P.nu, K.w, K.Z + (int64_t)K.j * K.ld, L.face64};
    }
    launch_stokes_q2_group<double>(q.data(), (int)q.size(), gs);
    hipEvent_t e = nullptr;
    MFS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const hipError_t r = hipEventRecord(e, gs);
    if (r == hipSuccess)
      for (mfs_problem *P : group) {
        MFS_HIP(hipStreamWaitEvent(P->kr.s, e, 0));
        kr_step_post(*P, P->kr.s);
      }
    (void)hipEventDestroy(e);
    MFS_HIP(r);
  });
}

int mfs_solve(mfs_problem *p, const double *b, double *x, const mfs_options *opts, mfs_solve_info *info,
              void *stream) {
  int rc = mfs_solve_begin(p, b, x, opts, stream);
  if (rc != MFS_OK) return rc;
  return guard([&] {
    Krylov &K = p->kr;
    while (K.state != 4) {
      MFS_HIP(hipEventSynchronize(K.ev));
      kr_process(*p);
    }
    if (info) *info = K.info;
    if (K.info.status != MFS_OK) {
      set_error("FGMRES did not reach rtol %.3e within %d iterations (relative residual %.3e)", K.rtol, K.maxit,
                K.info.rel_residual);
      throw mfs::Error{MFS_ENOCONV};
    }
  });
}

}  // extern "C"
