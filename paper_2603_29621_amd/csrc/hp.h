// hp spaces (per-cell degree, minimum rule, Sec. 3) on structured 3D meshes:
// host construction of the entity numbering and of the sparse maps between
// global unknowns and cell-local nodal values, and the device kernels that use
// them.  Internal to the library.
//
// Global unknowns, by mesh entity: vertices (lexicographic, x fastest); edges
// along x, y, z (lexicographic over their index boxes, m_e - 1 unknowns at the
// interior degree-m_e GLL points, m_e = lowest degree of the cells around the
// edge); faces normal to x, y, z ((m_f - 1)^2 unknowns at the interior tensor
// GLL points, lower free axis fastest, m_f = lowest degree of the cells on
// either side); cell interiors ((k - 1)^3, x fastest).  A cell's nodal values
// on an edge or face of lower degree are the entity's polynomial evaluated at
// the cell's GLL nodes (the face polynomial interpolates its edges at its own
// GLL points), which is what continuity across cells of different degree
// leaves of the space.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace mfs {

struct HpSpaceHost {
  int n[3] = {0, 0, 0};
  std::vector<int> deg;  // per cell (lexicographic)
  int64_t nvert = 0, N = 0;
  int ebox[3][3], fbox[3][3];
  std::vector<int> edeg[3], fdeg[3];
  std::vector<int64_t> eoff[3], foff[3], coff;
  std::vector<uint8_t> dirichlet;  // per unknown
  // cell-local rows: cell c owns rows row_base[c] .. row_base[c] + (k+1)^3
  std::vector<int64_t> row_base;
  std::vector<int64_t> row_ptr;
  std::vector<int> col;
  std::vector<double> val;
  // a cell with a local node exactly at the unknown's point, and that node
  std::vector<int> owner_cell, owner_local;

  void build(const int n_[3], const std::vector<int> &degrees);
  int cell_degree(int64_t c) const { return deg[c]; }
  // global reference coordinates ([0, n_a]) of unknown g
  void reference_point(int64_t g, double p[3]) const;
  // colour of each unknown: no two unknowns of a colour lie in a common cell
  std::vector<int> colours(int *ncolours) const;

 private:
  int64_t vertex(int x, int y, int z) const { return x + (int64_t)(n[0] + 1) * (y + (int64_t)(n[1] + 1) * z); }
  int64_t eidx(int a, const int e[3]) const { return e[0] + (int64_t)ebox[a][0] * (e[1] + (int64_t)ebox[a][1] * e[2]); }
  int64_t fidx(int a, const int f[3]) const { return f[0] + (int64_t)fbox[a][0] * (f[1] + (int64_t)fbox[a][1] * f[2]); }
  void edge_weights(int a, const int e[3], double t, double scale, std::vector<std::pair<int64_t, double>> &out) const;
  void face_weights(int a, const int f[3], double s, double t, std::vector<std::pair<int64_t, double>> &out) const;
};

// Transposed map: for every unknown, the cell-local slots it feeds, as
// (E-vector index of the slot for component 0, component stride, weight).
struct HpTransposed {
  std::vector<int64_t> ptr, ev;
  std::vector<int> nb;
  std::vector<double> val;
};

// ---------------------------------------------------------------- device kernels (hp_kernels.hip)
// Device map between the unknowns (ncomp blocks of N) and the cell-local
// rows of an E-vector.  A plain row (one unknown, weight 1) stores only its
// unknown; weighted rows (interpolated nodes at degree jumps) have a CSR of
// their own (-1 - h in rcol).  Row r's slots start at rslot[r], components nb
// apart.  Per unknown the transposed lists name the slots of its plain rows,
// then the slots of its weighted rows with the weights.
struct HpMaps {
  int64_t N = 0, nrows = 0;
  int nb = 0;
  const int *rcol = nullptr, *rslot = nullptr;
  const int64_t *hptr = nullptr;
  const int *hcol = nullptr;
  const double *hval = nullptr;
  const int64_t *tptr = nullptr;
  const int *tslot = nullptr;
  const int64_t *wptr = nullptr;
  const int *wslot = nullptr;
  const double *wval = nullptr;
  int64_t nheavy = 0;  // unknowns with more than HP_SCATTER_LIGHT rows in all (no Dirichlet flag)
  const int64_t *heavy = nullptr;
};
// dst[comp*N + i] = dirichlet[i] ? (src ? src[..] : 0) : sum over i's rows of w ev[slot + comp*nb]
// Lists of up to HP_SCATTER_LIGHT rows are summed by one thread each, the
// heavy unknowns by one wave each, in a fixed order.
constexpr int HP_SCATTER_LIGHT = 16;
template <typename T>
void hp_scatter(const HpMaps &M, int ncomp, const uint8_t *dirichlet, const T *ev, const T *src, T *dst,
                hipStream_t s);
// E-vector gather: ev[rslot[r] + comp*nb] = sum over row r of w x[comp*N + col], comp < ncomp
template <typename T>
void hp_gather(const HpMaps &M, int ncomp, const T *x, T *ev, hipStream_t s);
// per cell c of the list: ev_f = (E (x) E (x) E) ev_c (transpose: ev_c = (E^T..) ev_f)
// with E the 1D embedding from the coarse degree kc[c] to the fine degree
// kf[c] (tables[kf][kc], MAXQ x MAXQ row-major [fine node][coarse node]),
// ncomp components of a node side by side
template <typename T>
void hp_embed(int64_t ncells, int ncomp, const int *kf, const int *kc, const double *tables,
              const int64_t *off_f, const int64_t *off_c, const T *in, T *out, bool transpose, hipStream_t s);
// owner slots: x[comp*N + g] (+)= ev[owner_ev[g] + comp*owner_nb[g]] (owner_ev < 0: skipped);
// transpose: ev[owner_ev[g] + ..] = x[comp*N + g] (ev cleared beforehand)
template <typename T>
void hp_inject(int64_t N, int ncomp, const int64_t *owner_ev, const int *owner_nb, const T *ev, T *x, bool add,
               hipStream_t s);
template <typename T>
void hp_inject_t(int64_t N, int ncomp, const int64_t *owner_ev, const int *owner_nb, const T *x, T *ev,
                 hipStream_t s);
// y[comp*Ny + perm[i]] = x[comp*Nx + i] (scatter) or y[comp*Ny + i] = x[comp*Nx + perm[i]] (gather)
template <typename T>
void permute(int64_t n, int ncomp, const int64_t *perm, const T *x, int64_t Nx, T *y, int64_t Ny, bool scatter,
             hipStream_t s);
// masked vector operations on ncomp blocks of N unknowns with one scalar
// inverse diagonal shared by the blocks
template <typename T>
void mask_fill_dirichlet(const uint8_t *mask, int64_t N, int ncomp, T *x, const T *src, hipStream_t s);
template <typename T>
void mask_diag_scale(const uint8_t *mask, int64_t N, int ncomp, T *y, const T *invdiag, const T *x, hipStream_t s);
template <typename T>
void mask_cheb_update(const uint8_t *mask, int64_t N, int ncomp, T *x, T *d, const T *b, const T *Ax,
                      const T *invdiag, T c1, T c2, bool first, hipStream_t s);
// out[comp*N + i] = (colour[i] == cols[comp]) ? 1 : 0, for comp < 3
// (cols[comp] < 0: the component is 0)
void colour_indicator(const int *colour, int64_t N, const int cols[3], double *out, hipStream_t s);
// diag[i] = y[comp*N + i] where colour[i] == cols[comp]
void colour_extract(const int *colour, int64_t N, const int cols[3], const double *y, double *diag, hipStream_t s);

// cell kernels on E-vectors (cell_kernels.hip): one degree class of cells,
// local values in, local results out (velocity [(k+1)^3][3], components of a
// node side by side, pressure [k^3]
// per cell at the per-cell offsets)
template <typename T>
struct EvArgs {
  int ncells;        // cells in the class
  const int *cells;  // their ids
  const int64_t *off_u, *off_p;  // per cell id
  const T *in_u, *in_p;
  T *out_u, *out_p;
};
template <typename T>
void launch_cell_op_ev(const LevelGeom &g, int k, const T *X, const T *tab, int mode, T nu, const EvArgs<T> &ev,
                       hipStream_t s);
// the same work by the column kernel (degrees 5, 6; FP32 also 4); false when not covered
template <typename T>
bool launch_column_ev(const LevelGeom &g, int k, const T *X, int mode, T nu, const EvArgs<T> &ev, hipStream_t s);

}  // namespace mfs
