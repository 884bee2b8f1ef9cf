// Cell kernels on cell-local value arrays (E-vectors) for hp spaces (Sec. 3):
// the same weak forms and sum-factorised evaluation as the structured cell
// kernels, for the cells of one degree class.  Inputs are the cells' local
// nodal values (gathered through the hp local->global map), outputs their
// local results (scattered back by the transposed map), so every local node is
// written by exactly one thread and no atomics are needed.
#include "cell_common.h"
#include "hp.h"

namespace mfs {

namespace {

template <typename T>
struct EvKArgs {
  int n0, n1, ncells;
  const T *X, *tab;
  T nu;
  EvArgs<T> ev;
};

template <int K, typename T, int MODE>
__global__ void __launch_bounds__((Shape<3, K, K - 1>::BLOCK)) cell_kernel_ev(EvKArgs<T> a) {
  constexpr int DIM = 3;
  using Sh = Shape<DIM, K, K - 1>;
  constexpr int NQ = Sh::NQ, CPB = Sh::CPB, Q = Sh::Q, M = Sh::M;
  __shared__ T s_tab[TAB_SIZE];
  constexpr int NBUF = DIM * DIM > 3 ? DIM * DIM : 3;  // batched sweeps of DIM fields
  __shared__ T s_buf[NBUF][CPB * NQ];
  __shared__ T s_X[CPB][Sh::NV * DIM];

  const int tid = threadIdx.x;
  for (int i = tid; i < TAB_SIZE; i += Sh::BLOCK) s_tab[i] = a.tab[i];
  CellCtx<DIM, K, K - 1, T> c;
  int e;
  Sh::map(tid, e, c.t, c.active);
  const int slot = blockIdx.x * CPB + e;
  c.valid = c.active && slot < a.ncells;
  const int cell = c.valid ? a.ev.cells[slot] : 0;
  c.qi = c.t % Q;
  c.qj = (c.t / Q) % Q;
  c.ql = c.t / (Q * Q);
  c.cx = cell % a.n0;
  c.cy = (cell / a.n0) % a.n1;
  c.cz = cell / (a.n0 * a.n1);
  c.b0 = &s_buf[0][e * NQ];
  c.b1 = &s_buf[1][e * NQ];
  c.b2 = &s_buf[2][e * NQ];
  c.bb = &s_buf[0][e * NQ];
  c.bstride = CPB * NQ;
  c.tab = s_tab;
  constexpr bool NEED_U = (MODE & (M_LAPLACE | M_DIVU)) != 0;
  constexpr bool NEED_P = (MODE & (M_GRADP | M_MASSP)) != 0;
  constexpr bool OUT_U = (MODE & (M_LAPLACE | M_GRADP)) != 0;
  constexpr bool OUT_P = (MODE & (M_DIVU | M_MASSP)) != 0;
  const int64_t ou = c.valid ? a.ev.off_u[cell] : 0;
  const int64_t op = c.valid ? a.ev.off_p[cell] : 0;
  const bool ploc = c.p_local();
  const int jp = c.qi + M * (c.qj + M * c.ql);
  // source values of every component loaded before the vertex loads and the barrier
  T su[3] = {0, 0, 0}, sp = 0;
  if (NEED_U && c.valid) {
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp) su[comp] = a.ev.in_u[ou + 3 * c.t + comp];
  }
  if (NEED_P && c.valid && ploc) sp = a.ev.in_p[op + jp];
  if (c.valid)
    for (int idx = c.t; idx < Sh::NV * DIM; idx += NQ) {
      const int v = idx / DIM, comp = idx % DIM;
      const int vx = c.cx + (v & 1), vy = c.cy + ((v >> 1) & 1), vz = c.cz + ((v >> 2) & 1);
      const int64_t vid = vx + (int64_t)(a.n0 + 1) * (vy + (int64_t)(a.n1 + 1) * vz);
      s_X[e][idx] = a.X[vid * DIM + comp];
    }
  __syncthreads();

  T g[3][3] = {};
  if (NEED_U) {
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
      if (c.active) c.buf(comp)[c.t] = su[comp];
    csync<Sh::WAVE>();
    c.template gradients<DIM>(g);
  }
  T pval = 0;
  if (NEED_P) {
    if (c.active) c.b0[c.t] = sp;
    csync<Sh::WAVE>();
    const T *vals = c.template interpolate<M, TAB_SP>();
    pval = vals[c.t];
    csync<Sh::WAVE>();
  }

  T xi[3] = {s_tab[TAB_X + c.qi], s_tab[TAB_X + c.qj], s_tab[TAB_X + c.ql]};
  T J[3][3], I[3][3];
  q1_jacobian<DIM>(s_X[e], xi, J);
  const T det = invert<DIM>(J, I);
  const T JxW = det * s_tab[TAB_W + c.qi] * s_tab[TAB_W + c.qj] * s_tab[TAB_W + c.ql];

  T f[3][3] = {};
  T qv = 0;
  if (MODE & M_LAPLACE) {
    const T s = JxW * a.nu;
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp) {
      T gp[3];
#pragma unroll
      for (int x = 0; x < DIM; ++x) {
        T acc = 0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) acc += I[b][x] * g[comp][b];
        gp[x] = acc * s;
      }
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        T acc = 0;
#pragma unroll
        for (int x = 0; x < DIM; ++x) acc += I[b][x] * gp[x];
        f[comp][b] = acc;
      }
    }
  }
  if (MODE & M_GRADP) {
    const T s = -JxW * pval;
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
#pragma unroll
      for (int b = 0; b < DIM; ++b) f[comp][b] += s * I[b][comp];
  }
  if (MODE & M_DIVU) {
    T div = 0;
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
#pragma unroll
      for (int b = 0; b < DIM; ++b) div += I[b][comp] * g[comp][b];
    qv = -JxW * div;
  }
  if (MODE & M_MASSP) qv += JxW * pval;

  if (OUT_U) {
    T r[3];
    c.template integrate_gradients<DIM>(f, r);
#pragma unroll
    for (int comp = 0; comp < DIM; ++comp)
      if (c.valid) a.ev.out_u[ou + 3 * c.t + comp] = r[comp];
  }
  if (OUT_P) {
    if (c.active) c.b0[c.t] = qv;
    csync<Sh::WAVE>();
    const T r = c.template integrate<M, TAB_SP>(c.b0);
    if (c.valid && ploc) a.ev.out_p[op + jp] = r;
  }
}

template <int K, typename T, int MODE>
void go_ev(const EvKArgs<T> &a, hipStream_t s) {
  using Sh = Shape<3, K, K - 1>;
  if (a.ncells == 0) return;
  const int grid = (a.ncells + Sh::CPB - 1) / Sh::CPB;
  hipLaunchKernelGGL((cell_kernel_ev<K, T, MODE>), dim3(grid), dim3(Sh::BLOCK), 0, s, a);
}

template <int K, typename T>
void ev_mode(const EvKArgs<T> &a, int mode, hipStream_t s) {
  switch (mode) {
    case M_LAPLACE: go_ev<K, T, M_LAPLACE>(a, s); return;
    case M_LAPLACE | M_GRADP | M_DIVU: go_ev<K, T, M_LAPLACE | M_GRADP | M_DIVU>(a, s); return;
    case M_GRADP: go_ev<K, T, M_GRADP>(a, s); return;
    case M_DIVU: go_ev<K, T, M_DIVU>(a, s); return;
    case M_MASSP: go_ev<K, T, M_MASSP>(a, s); return;
    default: MFS_REQUIRE(false, MFS_EUNSUPPORTED, "unsupported hp cell operator mode %d", mode);
  }
}

}  // namespace

template <typename T>
void launch_cell_op_ev(const LevelGeom &g, int k, const T *X, const T *tab, int mode, T nu, const EvArgs<T> &ev,
                       hipStream_t s) {
  if (ev.ncells > 0 && launch_column_ev<T>(g, k, X, mode, nu, ev, s)) return;
  EvKArgs<T> a{};
  a.n0 = g.n[0];
  a.n1 = g.n[1];
  a.ncells = ev.ncells;
  a.X = X;
  a.tab = tab;
  a.nu = nu;
  a.ev = ev;
  switch (k) {
    case 2: ev_mode<2, T>(a, mode, s); break;
    case 3: ev_mode<3, T>(a, mode, s); break;
    case 4: ev_mode<4, T>(a, mode, s); break;
    case 5: ev_mode<5, T>(a, mode, s); break;
    case 6: ev_mode<6, T>(a, mode, s); break;
    default: MFS_REQUIRE(false, MFS_EUNSUPPORTED, "hp degree %d not compiled (2..6)", k);
  }
  MFS_HIP(hipGetLastError());
}
template void launch_cell_op_ev<double>(const LevelGeom &, int, const double *, const double *, int, double,
                                        const EvArgs<double> &, hipStream_t);
template void launch_cell_op_ev<float>(const LevelGeom &, int, const float *, const float *, int, float,
                                       const EvArgs<float> &, hipStream_t);

}  // namespace mfs
