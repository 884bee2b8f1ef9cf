// hp Stokes (Sec. 3, minimum rule): device maps of the hp spaces, the class-wise
// operators on E-vectors, p-transfers, the hp V-cycle and block preconditioner, the
// hp set-up and its C ABI.
#include "runtime.h"

namespace mfs {
namespace rt {

template <typename T>
void hp_gather_space(const HpDevSpace &d, int ncomp, const T *x, T *ev, hipStream_t s) {
  hp_gather<T>(d.m, ncomp, x, ev, s);
}

template <typename T>
void hp_scatter_space(const HpDevSpace &d, int ncomp, bool use_dir, const T *ev, const T *src, T *dst, hipStream_t s) {
  hp_scatter<T>(d.m, ncomp, use_dir ? d.dir : nullptr, ev, src, dst, s);
}

// dst = op(src) on hp level l: mode of the cell kernels; velocity output
// Dirichlet rows = src_u (A, Stokes) or 0 (B)
template <typename T>
void hp_apply(mfs_problem &P, int l, int mode, T *dst_u, T *dst_p, const T *src_u, const T *src_p, hipStream_t s) {
  HpData &H = *P.hp;
  HpLevel &L = H.lev[l];
  HpVecs<T> &V = hpv<T>(L);
  const bool need_u = mode & (M_LAPLACE | M_DIVU), need_p = mode & (M_GRADP | M_MASSP);
  const bool out_u = mode & (M_LAPLACE | M_GRADP), out_p = mode & (M_DIVU | M_MASSP);
  if (need_u) hp_gather_space<T>(L.vd, 3, src_u, V.ev_in, s);
  if (need_p) hp_gather_space<T>(H.pd, 1, src_p, hp_evp<T>(H, false), s);
  const Level &S0 = P.L[0];
  EvArgs<T> ev{};
  ev.off_u = L.off_u;
  ev.off_p = H.off_p;
  ev.in_u = V.ev_in;
  ev.out_u = V.ev_out;
  ev.in_p = hp_evp<T>(H, false);
  ev.out_p = hp_evp<T>(H, true);
  for (size_t c = 0; c < L.class_k.size(); ++c) {
    ev.ncells = L.class_n[c];
    ev.cells = L.class_cells[c];
    launch_cell_op_ev<T>(S0.g, L.class_k[c], dev<T>(S0).X, hp_tab<T>(H, L.class_k[c]), mode, (T)P.nu, ev, s);
  }
  if (out_u)
    hp_scatter_space<T>(L.vd, 3, true, V.ev_out, (mode & M_LAPLACE) ? src_u : nullptr, dst_u, s);
  if (out_p) hp_scatter_space<T>(H.pd, 1, false, hp_evp<T>(H, true), nullptr, dst_p, s);
}

template <typename T>
void hp_apply_A(mfs_problem &P, int l, T *dst, const T *src, hipStream_t s) {
  hp_apply<T>(P, l, M_LAPLACE, dst, nullptr, src, nullptr, s);
}

// transfers between hp level l and the next level (hp, or the structured
// degree-2 level 0 for the last hp level): gather coarse local values, embed
// them in the fine cells' degrees, inject into the fine unknowns at their owner
// nodes; restriction is the transposed sequence.
template <typename T>
void hp_prolongate_add(mfs_problem &P, int l, T *xf, const T *xc, hipStream_t s) {
  HpData &H = *P.hp;
  HpLevel &F = H.lev[l];
  T *evf = hpv<T>(F).ev_out;
  if (l + 1 < P.nhp) {
    HpLevel &C = H.lev[l + 1];
    T *evc = hpv<T>(C).ev_in;
    hp_gather_space<T>(C.vd, 3, xc, evc, s);
    hp_embed<T>(H.ncells, 3, F.deg, C.deg, H.embed, F.off_u, C.off_u, evc, evf, false, s);
  } else {
    T *tmp = std::is_same<T, double>::value ? (T *)H.tmp2_64 : (T *)H.tmp2_32;
    T *evc = std::is_same<T, double>::value ? (T *)H.ev2_64 : (T *)H.ev2_32;
    permute<T>(H.v2d.N, 3, H.perm2, xc, P.L[0].g.Nv, tmp, H.v2d.N, false, s);
    hp_gather_space<T>(H.v2d, 3, tmp, evc, s);
    hp_embed<T>(H.ncells, 3, F.deg, H.deg2, H.embed, F.off_u, H.off_u2, evc, evf, false, s);
  }
  hp_inject<T>(F.vd.N, 3, F.vd.owner_ev, F.vd.owner_nb, evf, xf, true, s);
}

template <typename T>
void hp_restrict(mfs_problem &P, int l, T *bc, const T *rf, hipStream_t s) {
  HpData &H = *P.hp;
  HpLevel &F = H.lev[l];
  T *evf = hpv<T>(F).ev_out;
  vec_fill<T>(evf, T(0), F.ev_size, s);
  hp_inject_t<T>(F.vd.N, 3, F.vd.owner_ev, F.vd.owner_nb, rf, evf, s);
  if (l + 1 < P.nhp) {
    HpLevel &C = H.lev[l + 1];
    T *evc = hpv<T>(C).ev_in;
    hp_embed<T>(H.ncells, 3, F.deg, C.deg, H.embed, F.off_u, C.off_u, evf, evc, true, s);
    hp_scatter_space<T>(C.vd, 3, true, evc, nullptr, bc, s);
  } else {
    T *tmp = std::is_same<T, double>::value ? (T *)H.tmp2_64 : (T *)H.tmp2_32;
    T *evc = std::is_same<T, double>::value ? (T *)H.ev2_64 : (T *)H.ev2_32;
    hp_embed<T>(H.ncells, 3, F.deg, H.deg2, H.embed, F.off_u, H.off_u2, evf, evc, true, s);
    hp_scatter_space<T>(H.v2d, 3, true, evc, nullptr, tmp, s);
    permute<T>(H.v2d.N, 3, H.perm2, tmp, H.v2d.N, bc, P.L[0].g.Nv, true, s);
  }
}

template <typename T>
void hp_chebyshev(mfs_problem &P, int l, T *x, const T *b, bool zero_start, hipStream_t s) {
  HpLevel &L = P.hp->lev[l];
  HpVecs<T> &V = hpv<T>(L);
  const double lmax = L.lambda, lmin = lmax / P.opts.cheb_range;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho_old = 1.0 / sigma;
  const int64_t N = L.vd.N;
  if (zero_start) {
    mask_cheb_update<T>(L.vd.dir, N, 3, x, V.d, b, nullptr, V.invdiag, T(0), (T)(1.0 / theta), true, s);
  } else {
    hp_apply_A<T>(P, l, V.r, x, s);
    mask_cheb_update<T>(L.vd.dir, N, 3, x, V.d, b, V.r, V.invdiag, T(0), (T)(1.0 / theta), true, s);
  }
  for (int it = 1; it < P.opts.cheb_degree; ++it) {
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    hp_apply_A<T>(P, l, V.r, x, s);
    mask_cheb_update<T>(L.vd.dir, N, 3, x, V.d, b, V.r, V.invdiag, (T)(rho * rho_old), (T)(2.0 * rho / delta), false,
                        s);
    rho_old = rho;
  }
}

// V-cycle of the velocity block: hp p-levels, then the structured levels
template <typename T>
void hp_vcycle(mfs_problem &P, int l, T *x, const T *b, hipStream_t s) {
  if (l == P.nhp) {
    vcycle_level<T>(P, 0, x, b, s);
    return;
  }
  HpLevel &L = P.hp->lev[l];
  HpVecs<T> &V = hpv<T>(L);
  const int64_t n = 3 * L.vd.N;
  mask_fill_dirichlet<T>(L.vd.dir, L.vd.N, 3, x, b, s);
  hp_chebyshev<T>(P, l, x, b, true, s);
  hp_apply_A<T>(P, l, V.r, x, s);
  vec_axpby<T>(V.r, T(1), b, T(-1), n, s);
  T *bc, *xc;
  if (l + 1 < P.nhp) {
    bc = hpv<T>(P.hp->lev[l + 1]).b;
    xc = hpv<T>(P.hp->lev[l + 1]).x;
  } else {
    bc = work<T>(P).b[0];
    xc = work<T>(P).x[0];
  }
  hp_restrict<T>(P, l, bc, V.r, s);
  hp_vcycle<T>(P, l + 1, xc, bc, s);
  hp_prolongate_add<T>(P, l, x, xc, s);
  hp_chebyshev<T>(P, l, x, b, false, s);
}

// block preconditioner on the hp system (as precondition())
template <typename T>
void hp_precondition(mfs_problem &P, T *y, const T *r, hipStream_t s) {
  HpData &H = *P.hp;
  const int64_t nu = 3 * H.lev[0].vd.N, np = H.pd.N;
  const T *rp = r + nu;
  T *yp = y + nu;
  T **pv = hp_pvec<T>(H);
  T *pres = pv[0], *ps = pv[1], *pp = pv[2], *pq = pv[3], *pz = pv[4];
  const T *pinv = std::is_same<T, double>::value ? (const T *)H.pinv64 : (const T *)H.pinv32;
  T *tu = std::is_same<T, double>::value ? (T *)H.tu64 : (T *)H.tu32;
  double *rho = P.scal, *pqs = P.scal + PCG_MAX;
  vec_fill<T>(pz, T(0), np, s);
  vec_copy<T>(pres, rp, np, s);
  vec_mul<T>(ps, pinv, pres, np, s);
  vec_copy<T>(pp, ps, np, s);
  multi_dot<T>(pres, 0, 1, ps, np, rho, P.partials, s);
  for (int it = 0; it < P.opts.schur_iterations; ++it) {
    hp_apply<T>(P, 0, M_MASSP, nullptr, pq, nullptr, pp, s);
    multi_dot<T>(pp, 0, 1, pq, np, pqs + it, P.partials, s);
    pcg_update1<T>(pz, pres, ps, pp, pq, pinv, np, rho + it, pqs + it, s);
    multi_dot<T>(pres, 0, 1, ps, np, rho + it + 1, P.partials, s);
    pcg_update2<T>(pp, ps, np, rho + it + 1, rho + it, s);
  }
  vec_axpby<T>(yp, (T)(-P.nu), pz, T(0), np, s);
  hp_apply<T>(P, 0, M_GRADP, tu, nullptr, nullptr, yp, s);
  vec_axpby<T>(tu, T(1), r, T(-1), nu, s);
  hp_vcycle<T>(P, 0, y, tu, s);
}

// ---------------------------------------------------------------- hp set-up
// device copy of an hp space's maps; ev_off: per-cell E-vector offset of the
// cell's first component block, ncomp_stride: whether rows carry a component
// stride ((k+1)^3 for the velocity)
// interleave (with vector_comp): the three components of a cell-local node
// are adjacent (slot 3 j + comp) instead of (k+1)^3 apart
// device maps of an hp space: rows cell by cell at the cells' E-vector
// offsets; vector spaces (velocity) keep the three components of a node side
// by side (slot 3 j + comp); constrained spaces drop the Dirichlet columns
// (their values do not enter the cells) and list no rows for Dirichlet
// unknowns (the scatter writes those rows itself)
void hp_upload(HpData &H, const HpSpaceHost &V, bool constrained, const std::vector<int64_t> &ev_off, bool vector_comp,
               HpDevSpace &d, hipStream_t s) {
  const int64_t ncells = (int64_t)V.deg.size();
  d.N = V.N;
  d.nrows = V.row_base[ncells];
  HpMaps &m = d.m;
  m.N = d.N;
  m.nrows = d.nrows;
  m.nb = vector_comp ? 1 : 0;
  const int stride = vector_comp ? 3 : 1;
  std::vector<int> rcol((size_t)d.nrows), rslot((size_t)d.nrows), hcol;
  std::vector<int64_t> hptr(1, 0), tptr((size_t)V.N + 1, 0), wptr((size_t)V.N + 1, 0);
  std::vector<double> hval;
  for (int64_t c = 0; c < ncells; ++c) {
    const int k = V.deg[c], nb = (k + 1) * (k + 1) * (k + 1);
    for (int j = 0; j < nb; ++j) {
      const int64_t r = V.row_base[c] + j;
      MFS_REQUIRE(ev_off[c] + (int64_t)stride * j < (int64_t(1) << 31), MFS_EINVAL, "E-vector too long");
      rslot[r] = (int)(ev_off[c] + (int64_t)stride * j);
      const int64_t b = V.row_ptr[r], e = V.row_ptr[r + 1];
      if (e - b == 1 && V.val[b] == 1.0 && !(constrained && V.dirichlet[V.col[b]])) {
        rcol[r] = V.col[b];
        tptr[V.col[b] + 1] += 1;
        continue;
      }
      rcol[r] = -1 - (int)(hptr.size() - 1);
      for (int64_t q = b; q < e; ++q) {
        const int g = V.col[q];
        if (constrained && V.dirichlet[g]) continue;
        hcol.push_back(g);
        hval.push_back(V.val[q]);
        wptr[g + 1] += 1;
      }
      hptr.push_back((int64_t)hcol.size());
    }
  }
  for (int64_t g = 0; g < V.N; ++g) {
    tptr[g + 1] += tptr[g];
    wptr[g + 1] += wptr[g];
  }
  std::vector<int> tslot((size_t)tptr[V.N]), wslot((size_t)wptr[V.N]);
  std::vector<double> wval((size_t)wptr[V.N]);
  {
    std::vector<int64_t> tf(tptr.begin(), tptr.end() - 1), wf(wptr.begin(), wptr.end() - 1);
    for (int64_t r = 0; r < d.nrows; ++r) {
      if (rcol[r] >= 0) {
        tslot[tf[rcol[r]]++] = rslot[r];
        continue;
      }
      const int64_t h = -1 - (int64_t)rcol[r];
      for (int64_t q = hptr[h]; q < hptr[h + 1]; ++q) {
        const int64_t o = wf[hcol[q]]++;
        wslot[o] = rslot[r];
        wval[o] = hval[q];
      }
    }
  }
  std::vector<int64_t> heavy;
  for (int64_t g = 0; g < V.N; ++g)
    if (!(constrained && V.dirichlet[g]) && (tptr[g + 1] - tptr[g]) + (wptr[g + 1] - wptr[g]) > HP_SCATTER_LIGHT)
      heavy.push_back(g);
  std::vector<int64_t> oev(V.N);
  std::vector<int> onb(V.N);
  for (int64_t g = 0; g < V.N; ++g) {
    const int c = V.owner_cell[g];
    oev[g] = (constrained && V.dirichlet[g]) ? -1 : ev_off[c] + (int64_t)stride * V.owner_local[g];
    onb[g] = vector_comp ? 1 : 0;
  }
  m.rcol = H.upload(rcol, s);
  m.rslot = H.upload(rslot, s);
  m.hptr = H.upload(hptr, s);
  m.hcol = H.upload(hcol, s);
  m.hval = H.upload(hval, s);
  m.tptr = H.upload(tptr, s);
  m.tslot = H.upload(tslot, s);
  m.wptr = H.upload(wptr, s);
  m.wslot = H.upload(wslot, s);
  m.wval = H.upload(wval, s);
  m.nheavy = (int64_t)heavy.size();
  m.heavy = heavy.empty() ? nullptr : H.upload(heavy, s);
  d.owner_ev = H.upload(oev, s);
  d.owner_nb = H.upload(onb, s);
  d.dir = constrained ? H.upload(V.dirichlet, s) : nullptr;
  MFS_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
}

std::vector<int64_t> ev_offsets(const std::vector<int> &deg, int ncomp, int shift, int64_t *total) {
  std::vector<int64_t> off(deg.size());
  int64_t o = 0;
  for (size_t c = 0; c < deg.size(); ++c) {
    off[c] = o;
    const int64_t m = deg[c] + 1 - shift;
    o += ncomp * m * m * m;
  }
  *total = o;
  return off;
}

template <typename T>
void hp_alloc_vecs(HpData &H, HpVecs<T> &v, int64_t N, int64_t ev) {
  v.x = H.alloc<T>(3 * N);
  v.b = H.alloc<T>(3 * N);
  v.r = H.alloc<T>(3 * N);
  v.d = H.alloc<T>(3 * N);
  v.ev_in = H.alloc<T>(ev);
  v.ev_out = H.alloc<T>(ev);
  v.invdiag = H.alloc<T>(N);
}

// lambda_max(D^{-1} A) of hp level l by CG-Lanczos (FP64), as for the
// structured levels
double hp_estimate_lambda(mfs_problem &P, int l, hipStream_t s) {
  HpLevel &L = P.hp->lev[l];
  const int64_t N = L.vd.N, n = 3 * N;
  HpVecs<double> &V = L.v64;
  double *r = V.x, *z = V.b, *p = V.d, *q = V.r;
  std::vector<double> h(n);
  uint64_t st = P.opts.seed * 1000003ULL + (uint64_t)l + 7919ULL;
  for (int64_t i = 0; i < n; ++i) {
    h[i] = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    if (L.V.dirichlet[i % N]) h[i] = 0.0;
  }
  MFS_HIP(hipMemcpyAsync(r, h.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  double *dv = P.scal + 4 * PCG_MAX;
  auto dot = [&](const double *a, const double *b) {
    multi_dot<double>(a, 0, 1, b, n, dv, P.partials, s);
    double v;
    MFS_HIP(hipMemcpyAsync(&v, dv, sizeof(double), hipMemcpyDeviceToHost, s));
    MFS_HIP(hipStreamSynchronize(s));
    return v;
  };
  mask_diag_scale<double>(L.vd.dir, N, 3, z, V.invdiag, r, s);
  vec_copy<double>(p, z, n, s);
  double rz = dot(r, z);
  std::vector<double> alpha, beta;
  const int steps = std::max(2, P.opts.lanczos_steps);
  for (int j = 0; j < steps && rz > 0; ++j) {
    hp_apply_A<double>(P, l, q, p, s);
    const double pq = dot(p, q);
    if (!(pq > 0)) break;
    const double a = rz / pq;
    vec_axpby<double>(r, -a, q, 1.0, n, s);
    mask_diag_scale<double>(L.vd.dir, N, 3, z, V.invdiag, r, s);
    const double rz2 = dot(r, z);
    const double b = rz2 / rz;
    vec_axpby<double>(p, 1.0, z, b, n, s);
    alpha.push_back(a);
    beta.push_back(b);
    rz = rz2;
    if (rz2 <= 1e-30 * rz) break;
  }
  const int m = (int)alpha.size();
  MFS_REQUIRE(m > 0, MFS_EINVAL, "Lanczos estimate failed on hp level %d", l);
  std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
  for (int j = 0; j < m; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j < m - 1) e[j] = std::sqrt(beta[j]) / alpha[j];
  }
  double lmax;
  sturm_max_eig(d, e, lmax);
  return lmax;
}

void hp_build(mfs_problem &P, const std::vector<int> &deg0, hipStream_t s) {
  HpData &H = *P.hp;
  const LevelGeom &g0 = P.L[0].g;
  for (int a = 0; a < 3; ++a) H.n[a] = g0.n[a];
  H.ncells = g0.ncells;
  // degrees per hp level: k <- max(k - 1, 2) until all are 2; that last
  // level is the structured degree-2 level
  std::vector<std::vector<int>> degs{deg0};
  while (P.opts.mg_levels && *std::max_element(degs.back().begin(), degs.back().end()) > 2) {
    std::vector<int> d = degs.back();
    for (int &k : d) k = std::max(k - 1, 2);
    degs.push_back(d);
  }
  if (degs.size() > 1) degs.pop_back();
  H.lev.resize(degs.size());
  P.nhp = (int)degs.size();
  for (size_t l = 0; l < degs.size(); ++l) {
    HpLevel &L = H.lev[l];
    L.V.build(H.n, degs[l]);
    const auto off = ev_offsets(degs[l], 3, 0, &L.ev_size);
    hp_upload(H, L.V, true, off, true, L.vd, s);
    L.off_u = H.upload(off, s);
    L.deg = H.upload(degs[l], s);
    for (int k = 2; k <= 6; ++k) {
      std::vector<int> cells;
      for (int64_t c = 0; c < H.ncells; ++c)
        if (degs[l][c] == k) cells.push_back((int)c);
      if (cells.empty()) continue;
      L.class_k.push_back(k);
      L.class_n.push_back((int)cells.size());
      L.class_cells.push_back(H.upload(cells, s));
    }
    hp_alloc_vecs(H, L.v64, L.V.N, L.ev_size);
    hp_alloc_vecs(H, L.v32, L.V.N, L.ev_size);
    L.diag = H.alloc<double>(L.V.N);
  }
  // pressure space of the finest level (degree k - 1, no Dirichlet unknowns)
  {
    std::vector<int> dp(deg0);
    for (int &k : dp) k -= 1;
    H.Pr.build(H.n, dp);
    const auto off = ev_offsets(deg0, 1, 1, &H.evp_size);
    hp_upload(H, H.Pr, false, off, false, H.pd, s);
    H.off_p = H.upload(off, s);
    H.evp_in64 = H.alloc<double>(H.evp_size);
    H.evp_out64 = H.alloc<double>(H.evp_size);
    H.evp_in32 = H.alloc<float>(H.evp_size);
    H.evp_out32 = H.alloc<float>(H.evp_size);
  }
  // uniform degree 2 and its place in the structured node grid
  {
    std::vector<int> d2(H.ncells, 2);
    H.V2.build(H.n, d2);
    const auto off = ev_offsets(d2, 3, 0, &H.ev2_size);
    hp_upload(H, H.V2, true, off, true, H.v2d, s);
    H.off_u2 = H.upload(off, s);
    H.deg2 = H.upload(d2, s);
    std::vector<int64_t> perm(H.V2.N);
    for (int64_t gi = 0; gi < H.V2.N; ++gi) {
      double p[3];
      H.V2.reference_point(gi, p);
      int64_t idx[3];
      for (int a = 0; a < 3; ++a) idx[a] = (int64_t)std::llround(2.0 * p[a]);
      perm[gi] = idx[0] + (int64_t)g0.nv[0] * (idx[1] + (int64_t)g0.nv[1] * idx[2]);
    }
    H.perm2 = H.upload(perm, s);
    H.ev2_64 = H.alloc<double>(H.ev2_size);
    H.ev2_32 = H.alloc<float>(H.ev2_size);
    H.tmp2_64 = H.alloc<double>(3 * H.V2.N);
    H.tmp2_32 = H.alloc<float>(3 * H.V2.N);
  }
  // 1D embeddings [kf][kc] and per-degree tables
  {
    std::vector<double> E(8 * 8 * MAXQ * MAXQ, 0.0);
    for (int kf = 1; kf <= 7; ++kf)
      for (int kc = 1; kc <= kf; ++kc) {
        double *T = E.data() + ((int64_t)kf * MAXQ + kc) * MAXQ * MAXQ;
        if (kc == kf) {
          for (int i = 0; i <= kf; ++i) T[i * MAXQ + i] = 1.0;
        } else {
          const auto pe = p_embedding(kf, kc);
          for (int i = 0; i <= kf; ++i)
            for (int j = 0; j <= kc; ++j) T[i * MAXQ + j] = pe[i * (kc + 1) + j];
        }
      }
    H.embed = H.upload(E, s);
    for (int k = 2; k <= 6; ++k) {
      const auto t = make_tables(k, k - 1);
      std::vector<float> t32(t.begin(), t.end());
      H.tab64[k] = H.upload(t, s);
      H.tab32[k] = H.upload(t32, s);
    }
  }
  // block preconditioner vectors, Krylov space of the hp system
  const int64_t Nu = H.lev[0].V.N, Np = H.Pr.N, ntot = 3 * Nu + Np;
  for (int i = 0; i < 5; ++i) {
    H.p64[i] = H.alloc<double>(Np);
    H.p32[i] = H.alloc<float>(Np);
  }
  H.tu64 = H.alloc<double>(3 * Nu);
  H.tu32 = H.alloc<float>(3 * Nu);
  H.pdiag = H.alloc<double>(3 * Np);
  H.m1 = H.alloc<double>(Np);
  H.ones = H.alloc<double>(Np);
  H.pinv64 = H.alloc<double>(Np);
  H.pinv32 = H.alloc<float>(Np);
  P.w32.full_in = H.alloc<float>(ntot);
  P.w32.full_out = H.alloc<float>(ntot);
  P.w64.full_in = H.alloc<double>(ntot);
  P.w64.full_out = H.alloc<double>(ntot);
  if (P.opts.mg_levels) {
    Krylov &K = P.kr;
    K.ld = kr_ld(ntot);
    K.V = H.alloc<double>((K.m + 1) * K.ld);
    K.Z = H.alloc<double>(K.m * K.ld);
    K.w = H.alloc<double>(ntot);
  }
  MFS_HIP(hipStreamSynchronize(s));
  // Jacobi diagonals of the velocity block on every hp level: A applied to
  // the indicators of three colours at once (one per component)
  for (int l = 0; l < P.nhp; ++l) {
    HpLevel &L = H.lev[l];
    int ncol = 0;
    const auto col = L.V.colours(&ncol);
    L.vd.colour = H.upload(col, s);
    L.vd.ncolours = ncol;
    double *e = L.v64.x, *y = L.v64.b;
    for (int c = 0; c < ncol; c += 3) {
      const int cols[3] = {c, c + 1 < ncol ? c + 1 : -1, c + 2 < ncol ? c + 2 : -1};
      colour_indicator(L.vd.colour, L.V.N, cols, e, s);
      hp_apply_A<double>(P, l, y, e, s);
      colour_extract(L.vd.colour, L.V.N, cols, y, L.diag, s);
    }
    launch_reciprocal(L.v64.invdiag, L.v32.invdiag, L.diag, L.V.N, s);
  }
  // pressure mass: diagonal (Jacobi-PCG of the Schur complement) and M_p 1
  {
    int ncol = 0;
    const auto col = H.Pr.colours(&ncol);
    H.pd.colour = H.upload(col, s);
    H.pd.ncolours = ncol;
    double *e = H.p64[0], *y = H.p64[1], *ind = H.pdiag;  // pdiag: 3 Np scratch here
    double *diag = H.p64[2];
    for (int c = 0; c < ncol; ++c) {
      const int cols[3] = {c, -1, -1};
      colour_indicator(H.pd.colour, Np, cols, ind, s);
      vec_copy<double>(e, ind, Np, s);
      hp_apply<double>(P, 0, M_MASSP, nullptr, y, nullptr, e, s);
      colour_extract(H.pd.colour, Np, cols, y, diag, s);
    }
    launch_reciprocal(H.pinv64, H.pinv32, diag, Np, s);
    vec_copy<double>(H.pdiag, diag, Np, s);
    vec_fill<double>(H.ones, 1.0, Np, s);
    hp_apply<double>(P, 0, M_MASSP, nullptr, H.m1, nullptr, H.ones, s);
  }
  if (P.opts.mg_levels)
    for (int l = 0; l < P.nhp; ++l) H.lev[l].lambda = P.opts.cheb_safety * hp_estimate_lambda(P, l, s);
  MFS_HIP(hipStreamSynchronize(s));
}

// mfs_vmult on an hp problem: the hp levels (all operators on the finest,
// the velocity block on the others), then the structured levels
void hp_vmult(mfs_problem &P, int op, int prec, int level, void *dst, const void *src, hipStream_t s) {
  if (level >= P.nhp) {
    MFS_REQUIRE(op == MFS_OP_A, MFS_EUNSUPPORTED, "structured levels of an hp problem carry the velocity block only");
    if (prec == MFS_FP64)
      apply_A<double>(P, level - P.nhp, (double *)dst, (const double *)src, s);
    else
      apply_A<float>(P, level - P.nhp, (float *)dst, (const float *)src, s);
    return;
  }
  MFS_REQUIRE(level == 0 || op == MFS_OP_A, MFS_EUNSUPPORTED, "coarser hp levels carry the velocity block only");
  const int64_t nu = 3 * P.hp->lev[level].V.N;
  auto run = [&](auto *d, auto *x) {
    using T = std::remove_pointer_t<decltype(d)>;
    switch (op) {
      case MFS_OP_STOKES: hp_apply<T>(P, level, M_LAPLACE | M_GRADP | M_DIVU, d, d + nu, x, x + nu, s); break;
      case MFS_OP_A: hp_apply<T>(P, level, M_LAPLACE, d, nullptr, x, nullptr, s); break;
      case MFS_OP_B: hp_apply<T>(P, level, M_GRADP, d, nullptr, nullptr, x, s); break;
      case MFS_OP_BT: hp_apply<T>(P, level, M_DIVU, nullptr, d, x, nullptr, s); break;
      case MFS_OP_MASS_P: hp_apply<T>(P, level, M_MASSP, nullptr, d, nullptr, x, s); break;
      default: MFS_REQUIRE(false, MFS_EUNSUPPORTED, "operator %d is not available on hp problems", op);
    }
  };
  if (prec == MFS_FP64)
    run((double *)dst, (const double *)src);
  else
    run((float *)dst, (const float *)src);
}

// instantiations used by the other parts of the runtime
template void hp_gather_space<float>(const HpDevSpace &d, int ncomp, const float *x, float *ev, hipStream_t s);
template void hp_gather_space<double>(const HpDevSpace &d, int ncomp, const double *x, double *ev, hipStream_t s);
template void hp_scatter_space<float>(const HpDevSpace &d, int ncomp, bool use_dir, const float *ev, const float *src, float *dst, hipStream_t s);
template void hp_scatter_space<double>(const HpDevSpace &d, int ncomp, bool use_dir, const double *ev, const double *src, double *dst, hipStream_t s);
template void hp_apply<float>(mfs_problem &P, int l, int mode, float *dst_u, float *dst_p, const float *src_u, const float *src_p, hipStream_t s);
template void hp_apply<double>(mfs_problem &P, int l, int mode, double *dst_u, double *dst_p, const double *src_u, const double *src_p, hipStream_t s);
template void hp_apply_A<float>(mfs_problem &P, int l, float *dst, const float *src, hipStream_t s);
template void hp_apply_A<double>(mfs_problem &P, int l, double *dst, const double *src, hipStream_t s);
template void hp_prolongate_add<float>(mfs_problem &P, int l, float *xf, const float *xc, hipStream_t s);
template void hp_prolongate_add<double>(mfs_problem &P, int l, double *xf, const double *xc, hipStream_t s);
template void hp_restrict<float>(mfs_problem &P, int l, float *bc, const float *rf, hipStream_t s);
template void hp_restrict<double>(mfs_problem &P, int l, double *bc, const double *rf, hipStream_t s);
template void hp_chebyshev<float>(mfs_problem &P, int l, float *x, const float *b, bool zero_start, hipStream_t s);
template void hp_chebyshev<double>(mfs_problem &P, int l, double *x, const double *b, bool zero_start, hipStream_t s);
template void hp_vcycle<float>(mfs_problem &P, int l, float *x, const float *b, hipStream_t s);
template void hp_vcycle<double>(mfs_problem &P, int l, double *x, const double *b, hipStream_t s);
template void hp_precondition<float>(mfs_problem &P, float *y, const float *r, hipStream_t s);
template void hp_precondition<double>(mfs_problem &P, double *y, const double *r, hipStream_t s);
template void hp_alloc_vecs<float>(HpData &H, HpVecs<float> &v, int64_t N, int64_t ev);
template void hp_alloc_vecs<double>(HpData &H, HpVecs<double> &v, int64_t N, int64_t ev);

}  // namespace rt
}  // namespace mfs

extern "C" {

int mfs_setup_hp(const mfs_mesh *mesh, const int *cell_degree, double nu, const mfs_options *opts, void *stream,
                 mfs_problem **out) {
  mfs_problem *P = nullptr;
  int rc = guard([&] {
    MFS_REQUIRE(out != nullptr, MFS_EINVAL, "out is NULL");
    *out = nullptr;
    MFS_REQUIRE(mesh != nullptr && mesh->dim == 3, MFS_EUNSUPPORTED, "hp problems are three-dimensional");
    MFS_REQUIRE(cell_degree != nullptr, MFS_EINVAL, "cell_degree is NULL");
    mfs_options o;
    if (opts)
      o = *opts;
    else
      mfs_default_options(&o);
    MFS_REQUIRE(o.pressure_offset == 1, MFS_EINVAL, "hp problems are Taylor-Hood (pressure_offset = 1)");
    for (int a = 0; a < 3; ++a) MFS_REQUIRE(mesh->n[a] >= 1, MFS_EINVAL, "n[%d] must be >= 1", a);
    const int64_t ncells = (int64_t)mesh->n[0] * mesh->n[1] * mesh->n[2];
    std::vector<int> deg(cell_degree, cell_degree + ncells);
    for (int64_t c = 0; c < ncells; ++c)
      MFS_REQUIRE(deg[c] >= 2 && deg[c] <= 6, MFS_EINVAL, "cell %lld: degree %d out of range [2, 6]", (long long)c,
                  deg[c]);
    mfs_options ob = o;
    ob.p_min = 2;
    const int rcb = mfs_setup(mesh, 2, nu, &ob, stream, &P);
    if (rcb != MFS_OK) throw mfs::Error{rcb};
    P->opts = o;
    P->opts.p_min = 2;
    P->hp = new HpData();
    hp_build(*P, deg, S(stream));
    *out = P;
  });
  if (rc != MFS_OK) {
    release(P);
    return rc;
  }
  return MFS_OK;
}

}  // extern "C"
