// Equal-order Navier-Stokes on locally refined meshes (Sec. 5): host maps with hanging
// nodes, their upload, the global-coarsening levels, the Jacobian through E-vectors,
// transfers, relaxation and V-cycle, the linearisation and residual, and the C ABI for
// refined meshes (counts, partition metrics, set-up).
#include "runtime.h"

namespace mfs {
namespace rt {

// f(0), ..., f(n-1) on n host threads; the first failure is rethrown here
// with its error text (which the worker set in its own thread-local slot)
void parallel_tasks(int n, const std::function<void(int)> &f) {
  std::vector<std::exception_ptr> ex((size_t)std::max(n, 0));
  std::vector<std::string> msg((size_t)std::max(n, 0));
  std::vector<std::thread> th;
  for (int i = 0; i < n; ++i)
    th.emplace_back([&, i] {
      try {
        f(i);
      } catch (...) {
        ex[i] = std::current_exception();
        msg[i] = get_error();
      }
    });
  for (auto &t : th) t.join();
  for (int i = 0; i < n; ++i)
    if (ex[i]) {
      set_error("%s", msg[i].c_str());
      std::rethrow_exception(ex[i]);
    }
}

// device maps of a level: rows are cell-major ((k+1)^3 per cell), so row r's
// E-vector slots are 4r .. 4r+3 and the lists need no slot offsets; rows of
// one unknown with weight 1 store only that unknown
void amr_maps_host(const AmrSpaceHost &S, AmrMapsHost &out) {
  const HpSpaceHost &V = S.V;
  const int64_t nrows = V.row_base[S.ncells], N = S.N;
  out.N = N;
  out.nrows = nrows;
  std::vector<int> &rcol = out.rcol;
  rcol.assign((size_t)nrows, 0);
  std::vector<int64_t> &hptr = out.hptr;
  hptr.assign(1, 0);
  std::vector<int> &hcol = out.hcol;
  std::vector<double> &hval = out.hval;
  std::vector<int64_t> &tptr = out.tptr, &wptr = out.wptr;
  tptr.assign((size_t)N + 1, 0);
  wptr.assign((size_t)N + 1, 0);
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t b = V.row_ptr[r], e = V.row_ptr[r + 1];
    if (e - b == 1 && V.val[b] == 1.0) {
      rcol[r] = V.col[b];
      tptr[V.col[b] + 1] += 1;
      continue;
    }
    rcol[r] = -1 - (int)(hptr.size() - 1);
    for (int64_t q = b; q < e; ++q) {
      hcol.push_back(V.col[q]);
      hval.push_back(V.val[q]);
      wptr[V.col[q] + 1] += 1;
    }
    hptr.push_back((int64_t)hcol.size());
  }
  for (int64_t g = 0; g < N; ++g) {
    tptr[g + 1] += tptr[g];
    wptr[g + 1] += wptr[g];
  }
  std::vector<int> &trow = out.trow, &wrow = out.wrow;
  std::vector<double> &wval = out.wval;
  trow.assign((size_t)tptr[N], 0);
  wrow.assign((size_t)wptr[N], 0);
  wval.assign((size_t)wptr[N], 0.0);
  {
    std::vector<int64_t> tf(tptr.begin(), tptr.end() - 1), wf(wptr.begin(), wptr.end() - 1);
    for (int64_t r = 0; r < nrows; ++r) {
      if (rcol[r] >= 0) {
        trow[tf[rcol[r]]++] = (int)r;
        continue;
      }
      const int64_t h = -1 - (int64_t)rcol[r];
      for (int64_t q = hptr[h]; q < hptr[h + 1]; ++q) {
        const int64_t o = wf[hcol[q]]++;
        wrow[o] = (int)r;
        wval[o] = hval[q];
      }
    }
  }
  std::vector<int64_t> &heavy = out.heavy;
  heavy.clear();
  for (int64_t g = 0; g < N; ++g)
    if ((tptr[g + 1] - tptr[g]) + (wptr[g + 1] - wptr[g]) > AMR_LIGHT) heavy.push_back(g);
  const int64_t nb = V.row_base[1] - V.row_base[0];
  out.owner.resize((size_t)N);
  for (int64_t g = 0; g < N; ++g) out.owner[g] = (int)(V.owner_cell[g] * nb + V.owner_local[g]);
}

void amr_maps_upload(HpData &H, const AmrSpaceHost &S, const AmrMapsHost &h, AmrMaps &M, hipStream_t s) {
  M.N = h.N;
  M.nrows = h.nrows;
  M.rcol = H.upload(h.rcol, s);
  M.hptr = H.upload(h.hptr, s);
  M.hcol = H.upload(h.hcol, s);
  M.hval = H.upload(h.hval, s);
  M.tptr = H.upload(h.tptr, s);
  M.trow = H.upload(h.trow, s);
  M.wptr = H.upload(h.wptr, s);
  M.wrow = H.upload(h.wrow, s);
  M.wval = H.upload(h.wval, s);
  M.dir = H.upload(S.V.dirichlet, s);
  M.owner = H.upload(h.owner, s);
  M.nheavy = (int64_t)h.heavy.size();
  M.heavy = h.heavy.empty() ? nullptr : H.upload(h.heavy, s);
  MFS_HIP(hipStreamSynchronize(s));  // the caller may release the host vectors
}

// device data of a level; `op`: the level applies its own Jacobian
void amr_level_upload(AmrData &A, AmrLevel &V, bool op, bool work, hipStream_t s) {
  AmrSpaceHost &S = V.S;
  const int k = A.k;
  const int64_t nc = S.ncells, NQ = (int64_t)(k + 1) * (k + 1) * (k + 1);
  V.N = S.N;
  V.NQ = NQ;
  LevelGeom &g = V.g;
  g.dim = 3;
  g.k = g.kp = k;
  g.n[0] = g.n[1] = 1;
  g.n[2] = (int)nc;
  g.ncells = nc;
  g.nv[0] = g.nv[1] = k + 1;
  g.nv[2] = (int)(k * nc + 1);
  g.np[0] = g.np[1] = k + 1;
  g.np[2] = g.nv[2];
  g.Nv = g.Np = (int64_t)g.nv[0] * g.nv[1] * g.nv[2];
  g.cart = 1;  // octree leaves of a Cartesian cube
  HpData &H = A.H;
  amr_maps_upload(H, S, V.mh, V.M, s);
  V.mh = AmrMapsHost();
  for (int i = 0; i < 2; ++i) {
    V.ev64[i] = H.alloc<double>(4 * nc * NQ);
    V.ev32[i] = H.alloc<float>(4 * nc * NQ);
  }
  if (op) {
    V.X64 = H.upload(S.Xcell, s);
    std::vector<float> x32(S.Xcell.begin(), S.Xcell.end());
    V.X32 = H.upload(x32, s);
    V.qd64 = H.alloc<double>(nc * NQ * NS_QD);
    V.qd32 = H.alloc<float>(nc * NQ * NS_QD);
    V.u0 = H.alloc<double>(7 * V.N);  // state [u0 (3N) | p0 (N) | u~ (3N)]
    if (A.mg) {
      V.diag = H.alloc<double>(4 * V.N);
      V.inv64 = H.alloc<double>(4 * V.N);
      V.inv32 = H.alloc<float>(4 * V.N);
      MFS_REQUIRE(V.ncolour_host > 0, MFS_EINVAL, "level colouring missing");
      V.colour = H.upload(V.colour_host, s);
      V.ncolours = V.ncolour_host;
      MFS_HIP(hipStreamSynchronize(s));
      std::vector<int>().swap(V.colour_host);
    }
    MFS_HIP(hipStreamSynchronize(s));  // x32 goes out of scope
  }
  if (work)
    for (int i = 0; i < 4; ++i) {
      V.w64[i] = H.alloc<double>(4 * V.N);
      V.w32[i] = H.alloc<float>(4 * V.N);
    }
  MFS_HIP(hipStreamSynchronize(s));
  S.V = HpSpaceHost();  // the row maps and corners live on the device now
  std::vector<double>().swap(S.Xcell);
}

// the levels: the given mesh, and with multigrid its global coarsenings down
// to the uniform base mesh, with their cell and unknown relations
void amr_build(mfs_problem &P, const mfs_refined_mesh &m, int k, bool mg, hipStream_t s) {
  AmrData &A = *P.amr;
  A.n = m.n;
  A.k = k;
  A.L = m.levels;
  A.mg = mg;
  // the meshes of every level: the given one and, with multigrid, its global
  // coarsenings down to the uniform base mesh
  std::vector<std::vector<int>> lv(1), ix(1);
  MFS_REQUIRE(m.ncells >= 1 && m.level && m.idx, MFS_EINVAL, "empty cell list");
  MFS_REQUIRE(m.levels >= 0 && m.levels <= 4, MFS_EINVAL, "refinement levels %d out of range [0, 4]", m.levels);
  lv[0].assign(m.level, m.level + m.ncells);
  ix[0].assign(m.idx, m.idx + 3 * m.ncells);
  if (mg) {
    int top = 0;
    for (int l : lv[0]) top = std::max(top, l);
    MFS_REQUIRE(top >= 1, MFS_EINVAL, "the mesh is not refined: set up the base mesh with mfs_setup");
    MFS_REQUIRE(top <= m.levels, MFS_EINVAL, "cell level %d above the mesh's %d levels", top, m.levels);
    for (int j = 1; j <= top; ++j) {
      lv.emplace_back();
      ix.emplace_back();
      amr_coarsen(m.n, lv[j - 1], ix[j - 1], lv[j], ix[j]);
    }
  }
  const int nlev = (int)lv.size();
  A.lev.resize(nlev);
  const int nop = amr_nop(A);
  // host construction, one thread per level: space, maps, colouring
  parallel_tasks(nlev, [&](int j) {
    AmrLevel &V = A.lev[j];
    V.S.build(m.n, m.levels - j, (int64_t)lv[j].size(), lv[j].data(), ix[j].data(), k);
    amr_maps_host(V.S, V.mh);
    if (mg && j < nop) V.colour_host = V.S.colours(&V.ncolour_host);
  });
  std::vector<AmrTransferHost> T((size_t)nlev - 1);
  std::vector<std::vector<int64_t>> inj((size_t)nlev - 1);
  parallel_tasks(nlev - 1, [&](int j) {
    const AmrLevel &F = A.lev[j], &C = A.lev[j + 1];
    T[j] = amr_transfer(m.n, F.S.level, F.S.idx, C.S.level, C.S.idx);
    inj[j] = amr_injection(F.S, C.S);
  });
  HpData &H = A.H;
  for (int j = 0; j + 1 < nlev; ++j) {
    AmrLevel &F = A.lev[j];
    F.parent = H.upload(T[j].parent, s);
    F.octant = H.upload(T[j].octant, s);
    F.cptr = H.upload(T[j].cptr, s);
    F.child = H.upload(T[j].child, s);
    F.inject = H.upload(inj[j], s);
  }
  MFS_HIP(hipStreamSynchronize(s));  // T and inj go out of scope
  for (size_t j = 0; j < A.lev.size(); ++j) amr_level_upload(A, A.lev[j], (int)j < nop, mg, s);
  const auto tab = make_tables(k, k);
  std::vector<float> tab32(tab.begin(), tab.end());
  A.tab64 = H.upload(tab, s);
  A.tab32 = H.upload(tab32, s);
  A.E.k = k;
  for (int h = 0; h < 2; ++h)
    for (int t = 0; t <= k; ++t)
      for (int q = 0; q <= k; ++q) {
        // coarse basis function q of the k+1 equispaced nodes at fine node t of half h
        const double x = 0.5 * (h + (double)t / k);
        double v = 1.0;
        for (int r = 0; r <= k; ++r)
          if (r != q) v *= (x - (double)r / k) / ((double)(q - r) / k);
        A.E.w[h][t][q] = v;
      }
  const int64_t N0 = A.lev[0].N;
  A.ones = H.alloc<double>(N0);
  A.scratch = H.alloc<double>(N0);
  A.state = H.alloc<double>(4 * N0);
  if (mg) {  // the BDF2 / Newton driver: history, residual, correction
    P.nw_uh = H.alloc<double>(3 * N0);
    P.nw_F = H.alloc<double>(4 * N0);
    P.nw_dx = H.alloc<double>(4 * N0);
  }
  vec_fill<double>(A.ones, 1.0, N0, s);
  MFS_HIP(hipStreamSynchronize(s));
}

// constrained Jacobian on level j: gather with the constraints (the
// velocity's Dirichlet columns dropped), cell kernel on the E-vectors,
// transposed scatter (identity on the velocity Dirichlet rows)
template <typename T>
void amr_apply_ns(mfs_problem &P, int j, T *dst, const T *src, hipStream_t s) {
  AmrData &A = *P.amr;
  MFS_REQUIRE(A.ready, MFS_EINVAL, "mfs_set_linearization has not been called");
  AmrLevel &V = A.lev[j];
  T *evi = amr_ev<T>(V, 0), *evo = amr_ev<T>(V, 1);
  amr_gather<T>(V.M, 4, true, src, evi, s);
  launch_ns<T>(V.g, nullptr, amr_tab<T>(A), 1, (T)P.nu, (T)A.dt, A.newton, nullptr, nullptr, amr_qd<T>(V), s, evo,
               evi, amr_X<T>(V));
  amr_scatter<T>(V.M, evo, src, dst, s);
}

// prolongation from level j+1 to level j (added to xf): gather the coarse
// cells' values through the coarse constraints, embed them in the fine
// cells, take each fine unknown from its owner slot (Dirichlet velocity rows
// and columns zero, pressure unconstrained)
template <typename T>
void amr_prolongate_add(mfs_problem &P, int j, T *xf, const T *xc, hipStream_t s) {
  AmrData &A = *P.amr;
  AmrLevel &F = A.lev[j], &C = A.lev[j + 1];
  T *evc = amr_ev<T>(C, 0), *evf = amr_ev<T>(F, 1);
  amr_gather<T>(C.M, 4, true, xc, evc, s);
  amr_embed<T>(A.E, F.S.ncells, C.S.ncells, F.parent, F.octant, evc, evf, s);
  amr_inject<T>(F.M, evf, xf, true, s);
}

// restriction (the transpose) from level j to level j+1
template <typename T>
void amr_restrict(mfs_problem &P, int j, T *bc, const T *rf, hipStream_t s) {
  AmrData &A = *P.amr;
  AmrLevel &F = A.lev[j], &C = A.lev[j + 1];
  T *evc = amr_ev<T>(C, 0), *evf = amr_ev<T>(F, 1);
  vec_fill<T>(evf, T(0), 4 * F.S.ncells * F.NQ, s);
  amr_inject_t<T>(F.M, rf, evf, s);
  amr_embed_t<T>(A.E, F.S.ncells, C.S.ncells, F.cptr, F.child, F.octant, evf, evc, s);
  amr_scatter<T>(C.M, evc, nullptr, bc, s);
}

template <typename T>
void amr_relax(mfs_problem &P, int j, T *x, const T *b, bool zero_start, hipStream_t s) {
  AmrLevel &V = P.amr->lev[j];
  T *d = amr_w<T>(V, 3);
  for (int it = 0; it < P.opts.relax_steps; ++it) {
    // from the zero start (x = b on the Dirichlet rows, 0 elsewhere) J x = x
    // exactly: identity rows, Dirichlet source values ignored in the others
    if (zero_start && it == 0)
      vec_copy<T>(d, x, 4 * V.N, s);
    else
      amr_apply_ns<T>(P, j, d, x, s);
    jacobi_relax<T>(x, b, d, amr_inv<T>(V), (T)P.opts.relax_omega, 4 * V.N, s);
  }
}

// one V-cycle from level j: as the structured monolithic V-cycle, with the
// GC levels first and the structured hierarchy of the base mesh below them
template <typename T>
void amr_vcycle(mfs_problem &P, int j, T *x, const T *b, hipStream_t s) {
  AmrData &A = *P.amr;
  MFS_REQUIRE(A.mg, MFS_EUNSUPPORTED, "problem was set up without multigrid levels");
  if (j == amr_nop(A)) {
    ns_vcycle<T>(P, 0, x, b, s);
    return;
  }
  AmrLevel &V = A.lev[j], &C = A.lev[j + 1];
  mask_fill_dirichlet<T>(V.M.dir, V.N, 3, x, b, s);  // x = b on Dirichlet rows, 0 elsewhere
  vec_fill<T>(x + 3 * V.N, T(0), V.N, s);
  amr_relax<T>(P, j, x, b, true, s);
  T *r = amr_w<T>(V, 2);
  amr_apply_ns<T>(P, j, r, x, s);
  vec_axpby<T>(r, T(1), b, T(-1), 4 * V.N, s);  // r = b - J x
  T *xc = amr_w<T>(C, 0), *bc = amr_w<T>(C, 1);
  amr_restrict<T>(P, j, bc, r, s);
  amr_vcycle<T>(P, j + 1, xc, bc, s);
  amr_prolongate_add<T>(P, j, x, xc, s);
  amr_relax<T>(P, j, x, b, false, s);
}

// Jacobi diagonal of level j by colour probes (FP64): J applied to the
// indicator of one colour in one component gives the diagonal entries of
// that colour (no two unknowns of a colour meet in a cell)
void amr_diagonal(mfs_problem &P, int j, double *diag, hipStream_t s) {
  AmrLevel &V = P.amr->lev[j];
  double *e = V.w64[0], *y = V.w64[1];
  for (int col = 0; col < V.ncolours; ++col)
    for (int comp = 0; comp < 4; ++comp) {
      amr_colour_probe(V.colour, V.N, col, comp, e, s);
      amr_apply_ns<double>(P, j, y, e, s);
      amr_colour_take(V.colour, V.N, col, comp, y, diag, s);
    }
}

// mfs_set_linearization on a refined mesh: u0 at the unknowns of level 0,
// copied at the coarse unknowns level by level; point data per level (u0
// through the unconstrained scalar map into the velocity slots); with
// multigrid the structured base levels and the GC levels' diagonals
// Linearisation at the state x0 = [u0 | p0] (4 N) with the BDF2 history u~
// (3 N; NULL: u~ = u0) on every level (coarse levels take the fields at their
// unknowns, which are fine unknowns), as ns_set_point.
void amr_set_point(mfs_problem &P, const double *x0, const double *uh, double dt, int newton, int keep_delta,
                   bool mg, hipStream_t s) {
  AmrData &A = *P.amr;
  A.ready = false;
  A.mg_ready = false;
  A.dt = dt;
  A.newton = newton ? 1 : 0;
  const int nop = amr_nop(A);
  const int64_t N0 = A.lev[0].N;
  MFS_HIP(hipMemcpyAsync(A.lev[0].u0, x0, 4 * N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  MFS_HIP(hipMemcpyAsync(A.lev[0].u0 + 4 * N0, uh ? uh : x0, 3 * N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int j = 1; j < nop; ++j)
    permute<double>(A.lev[j].N, 7, A.lev[j - 1].inject, A.lev[j - 1].u0, A.lev[j - 1].N, A.lev[j].u0, A.lev[j].N,
                    false, s);
  for (int j = 0; j < nop; ++j) {
    AmrLevel &V = A.lev[j];
    double *ev = V.ev64[0], *evh = V.ev64[1];
    amr_gather<double>(V.M, 4, false, V.u0, ev, s);  // the state keeps its boundary values
    amr_gather<double>(V.M, 3, false, V.u0 + 4 * V.N, evh, s);
    NsPoint<double> pt;
    pt.keep_delta = keep_delta;
    pt.evhist = evh;
    launch_ns<double>(V.g, nullptr, A.tab64, 0, P.nu, dt, A.newton, nullptr, nullptr, V.qd64, s, nullptr, ev, V.X64,
                      &pt);
    vec_cast<float, double>(V.qd32, V.qd64, V.g.ncells * V.NQ * NS_QD, s);
  }
  if (A.mg) {
    AmrLevel &F = A.lev[nop - 1], &B = A.lev[nop];
    MFS_REQUIRE(B.N == P.L[0].g.Nv, MFS_EINVAL, "base level mismatch");
    permute<double>(B.N, 4, F.inject, F.u0, F.N, P.tmp_full, B.N, false, s);
    permute<double>(B.N, 3, F.inject, F.u0 + 4 * F.N, F.N, P.tmp2, B.N, false, s);
    ns_set_point(P, P.tmp_full, P.tmp2, dt, newton, keep_delta, mg, s);  // structured levels; synchronises
    A.ready = true;
    if (!mg) return;
    try {
      for (int j = 0; j < nop; ++j) {
        AmrLevel &V = A.lev[j];
        amr_diagonal(P, j, V.diag, s);
        launch_reciprocal(V.inv64, V.inv32, V.diag, 4 * V.N, s);
      }
      MFS_HIP(hipStreamSynchronize(s));
      A.mg_ready = true;
    } catch (...) {
      A.ready = false;
      throw;
    }
    return;
  }
  MFS_HIP(hipStreamSynchronize(s));
  A.ready = true;
}

// Linearisation point u0 of a Jacobian alone: p0 = 0 and u~ = u0
void amr_set_linearization(mfs_problem &P, const double *u0, double dt, int newton, hipStream_t s) {
  const int64_t N0 = P.amr->lev[0].N;
  double *x0 = P.amr->state;
  MFS_HIP(hipMemcpyAsync(x0, u0, 3 * N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  vec_fill<double>(x0 + 3 * N0, 0.0, N0, s);
  amr_set_point(P, x0, nullptr, dt, newton, 0, true, s);
}

// F = the nonlinear residual at the level-0 state of the last linearisation
// (through the hanging-node maps); Dirichlet velocity rows 0
void amr_residual(mfs_problem &P, double *F, hipStream_t s) {
  AmrData &A = *P.amr;
  MFS_REQUIRE(A.ready, MFS_EINVAL, "no linearisation state: call mfs_set_linearization_point first");
  AmrLevel &V = A.lev[0];
  double *evi = V.ev64[0], *evo = V.ev64[1];
  launch_ns<double>(V.g, nullptr, A.tab64, 2, P.nu, A.dt, A.newton, nullptr, nullptr, V.qd64, s, evo, evi, V.X64);
  amr_scatter<double>(V.M, evo, nullptr, F, s);
}

void amr_vmult(mfs_problem &P, int op, int prec, int level, void *dst, const void *src, hipStream_t s) {
  MFS_REQUIRE(op == MFS_OP_NS_JACOBIAN, MFS_EUNSUPPORTED,
              "refined-mesh problems provide the Navier-Stokes Jacobian (operator %d requested)", op);
  if (prec == MFS_FP64)
    amr_apply_ns<double>(P, level, (double *)dst, (const double *)src, s);
  else
    amr_apply_ns<float>(P, level, (float *)dst, (const float *)src, s);
}

// instantiations used by the other parts of the runtime
template void amr_apply_ns<float>(mfs_problem &P, int j, float *dst, const float *src, hipStream_t s);
template void amr_apply_ns<double>(mfs_problem &P, int j, double *dst, const double *src, hipStream_t s);
template void amr_prolongate_add<float>(mfs_problem &P, int j, float *xf, const float *xc, hipStream_t s);
template void amr_prolongate_add<double>(mfs_problem &P, int j, double *xf, const double *xc, hipStream_t s);
template void amr_restrict<float>(mfs_problem &P, int j, float *bc, const float *rf, hipStream_t s);
template void amr_restrict<double>(mfs_problem &P, int j, double *bc, const double *rf, hipStream_t s);
template void amr_relax<float>(mfs_problem &P, int j, float *x, const float *b, bool zero_start, hipStream_t s);
template void amr_relax<double>(mfs_problem &P, int j, double *x, const double *b, bool zero_start, hipStream_t s);
template void amr_vcycle<float>(mfs_problem &P, int j, float *x, const float *b, hipStream_t s);
template void amr_vcycle<double>(mfs_problem &P, int j, double *x, const double *b, hipStream_t s);

}  // namespace rt
}  // namespace mfs

extern "C" {

int mfs_refined_count(const mfs_refined_mesh *mesh, int k, int64_t *n_unknowns, int64_t *n_hanging) {
  return guard([&] {
    MFS_REQUIRE(mesh != nullptr, MFS_EINVAL, "mesh is NULL");
    AmrSpaceHost S;
    S.build(mesh->n, mesh->levels, mesh->ncells, mesh->level, mesh->idx, k);
    if (n_unknowns) *n_unknowns = S.N;
    if (n_hanging) *n_hanging = S.nhanging;
  });
}

int mfs_refined_mg_metrics(const mfs_refined_mesh *mesh, int nprocs, double *eta) {
  return guard([&] {
    MFS_REQUIRE(mesh != nullptr && eta != nullptr, MFS_EINVAL, "NULL argument");
    MFS_REQUIRE(nprocs >= 1, MFS_EINVAL, "nprocs must be >= 1");
    MFS_REQUIRE(mesh->n >= 1 && mesh->n <= 4096 && mesh->levels >= 0 && mesh->levels <= 4 && mesh->ncells >= 1,
                MFS_EINVAL, "bad refined mesh");
    std::vector<int> level(mesh->level, mesh->level + mesh->ncells), idx(mesh->idx, mesh->idx + 3 * mesh->ncells);
    for (int64_t c = 0; c < mesh->ncells; ++c) {
      MFS_REQUIRE(level[c] >= 0 && level[c] <= mesh->levels, MFS_EINVAL, "cell %lld: level out of range",
                  (long long)c);
      for (int a = 0; a < 3; ++a)
        MFS_REQUIRE(idx[3 * c + a] >= 0 && idx[3 * c + a] < (mesh->n << level[c]), MFS_EINVAL,
                    "cell %lld: index out of range", (long long)c);
    }
    amr_mg_metrics(mesh->n, level, idx, nprocs, eta);
  });
}

int mfs_setup_refined(const mfs_refined_mesh *mesh, int k, double nu, const mfs_options *opts, void *stream,
                      mfs_problem **out) {
  mfs_problem *P = nullptr;
  int rc = guard([&] {
    MFS_REQUIRE(out != nullptr, MFS_EINVAL, "out is NULL");
    *out = nullptr;
    MFS_REQUIRE(mesh != nullptr, MFS_EINVAL, "mesh is NULL");
    MFS_REQUIRE(nu > 0 && std::isfinite(nu), MFS_EINVAL, "nu must be positive");
    mfs_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_options(&o);
    MFS_REQUIRE(o.pressure_offset == 0, MFS_EUNSUPPORTED,
                "refined meshes provide the equal-order Navier-Stokes Jacobian (pressure_offset = 0)");
    MFS_REQUIRE(k == 1 || k == 2, MFS_EUNSUPPORTED, "refined meshes support degrees 1 and 2 (got %d)", k);
    MFS_REQUIRE(o.relax_type == MFS_RELAX_JACOBI, MFS_EUNSUPPORTED,
                "refined meshes relax with point Jacobi (additive Schwarz patches need a structured level)");
    MFS_REQUIRE(mesh->n >= 1 && mesh->n <= 4096, MFS_EINVAL, "base cells per direction %d out of range", mesh->n);
    const bool mg = o.mg_levels != 0;
    if (mg) {
      // the structured hierarchy of the uniform base mesh (Cartesian unit cube)
      const int n = mesh->n;
      std::vector<double> X((size_t)3 * (n + 1) * (n + 1) * (n + 1));
      for (int z = 0; z <= n; ++z)
        for (int y = 0; y <= n; ++y)
          for (int x = 0; x <= n; ++x) {
            const size_t v = (size_t)x + (size_t)(n + 1) * (y + (size_t)(n + 1) * z);
            X[3 * v] = (double)x / n;
            X[3 * v + 1] = (double)y / n;
            X[3 * v + 2] = (double)z / n;
          }
      mfs_mesh bm{};
      bm.dim = 3;
      bm.n[0] = bm.n[1] = bm.n[2] = n;
      bm.vertices = X.data();
      const int rcb = mfs_setup(&bm, k, nu, &o, stream, &P);
      if (rcb != MFS_OK) throw mfs::Error{rcb};
    } else {
      P = new mfs_problem();
      P->dim = 3;
      P->nu = nu;
      P->opts = o;
      P->stream = S(stream);
      P->ns = true;
    }
    P->amr = new AmrData();
    amr_build(*P, *mesh, k, mg, S(stream));
    AmrData &A = *P->amr;
    P->namr = amr_nop(A);
    if (mg) {
      // FGMRES and the FP32 staging vectors at the size of the refined system
      const int64_t n0 = 4 * A.lev[0].N;
      Krylov &K = P->kr;
      K.ld = kr_ld(n0);
      K.V = A.H.alloc<double>((K.m + 1) * K.ld);
      K.Z = A.H.alloc<double>(K.m * K.ld);
      K.w = A.H.alloc<double>(n0);
      P->w32.full_in = A.H.alloc<float>(n0);
      P->w32.full_out = A.H.alloc<float>(n0);
      P->w64.full_in = A.H.alloc<double>(n0);
      P->w64.full_out = A.H.alloc<double>(n0);
    }
    *out = P;
  });
  if (rc != MFS_OK) {
    release(P);
    return rc;
  }
  return MFS_OK;
}

}  // extern "C"
