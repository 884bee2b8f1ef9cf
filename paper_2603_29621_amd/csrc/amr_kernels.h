// Refined-mesh multigrid kernels (amr_kernels.hip).  Internal to the library.
#pragma once

#include <cstdint>

#include "internal.h"

namespace mfs {

// 1D embeddings of the k+1 equispaced nodes of a cell into its lower (0) and
// upper (1) half: w[h][t][s] = value of the coarse basis function s at fine
// node t of half h
struct AmrEmbed {
  int k;
  double w[2][3][3];
};

// E-vectors of a level: [cell][(k+1)^3][4], the three velocity components and
// the pressure of a cell-local node side by side (row r = cell*(k+1)^3 + node
// holds slots 4r .. 4r+3).

// Maps between the unknowns (4 blocks of N) and the E-vector rows.  Almost
// every row is one unknown with weight 1 (a plain row); the rows of hanging
// nodes combine several unknowns (weighted rows), kept in a CSR of their own.
// The transposed lists split the same way.
struct AmrMaps {
  int64_t N = 0, nrows = 0;
  const int *rcol = nullptr;      // per row: its unknown, or -1 - h for weighted row h
  const int64_t *hptr = nullptr;  // weighted rows: unknown, weight
  const int *hcol = nullptr;
  const double *hval = nullptr;
  const int64_t *tptr = nullptr;  // per unknown: the plain rows holding it
  const int *trow = nullptr;
  const int64_t *wptr = nullptr;  // per unknown: the weighted rows using it, with the weight
  const int *wrow = nullptr;
  const double *wval = nullptr;
  const uint8_t *dir = nullptr;   // velocity Dirichlet unknowns
  const int *owner = nullptr;     // a row holding the unknown's own node
  int64_t nheavy = 0;             // unknowns with more than AMR_LIGHT rows in all
  const int64_t *heavy = nullptr;
};
constexpr int AMR_LIGHT = 16;

// ev rows = C x: components 0 .. ncomp-1 of the 4 blocks of x; with mask the
// velocity values of Dirichlet unknowns are taken as 0 (the constrained
// operator ignores them)
template <typename T>
void amr_gather(const AmrMaps &M, int ncomp, bool mask, const T *x, T *ev, hipStream_t s);
// dst = C^T ev (all 4 components); velocity rows of Dirichlet unknowns are
// src (or 0 without src) instead
template <typename T>
void amr_scatter(const AmrMaps &M, const T *ev, const T *src, T *dst, hipStream_t s);
// x (+)= the value at each unknown's owner row (velocity of Dirichlet
// unknowns skipped); transpose: ev owner rows = x (ev cleared beforehand)
template <typename T>
void amr_inject(const AmrMaps &M, const T *ev, T *x, bool add, hipStream_t s);
template <typename T>
void amr_inject_t(const AmrMaps &M, const T *x, T *ev, hipStream_t s);

// fine E-vector (ncf cells, 4 components) from the coarse one (ncc cells):
// each fine cell takes its parent's values through the embedding of its
// octant (octant 8: the same cell, copied)
template <typename T>
void amr_embed(const AmrEmbed &E, int64_t ncf, int64_t ncc, const int *parent, const uint8_t *oct, const T *evc,
               T *evf, hipStream_t s);
// transpose: every coarse cell sums the transposed embeddings of its fine
// cells (cptr/child: CSR list of the fine cells of each coarse cell)
template <typename T>
void amr_embed_t(const AmrEmbed &E, int64_t ncf, int64_t ncc, const int64_t *cptr, const int *child,
                 const uint8_t *oct, const T *evf, T *evc, hipStream_t s);
// out (4 blocks of N) = indicator of the unknowns of colour col in component comp
void amr_colour_probe(const int *colour, int64_t N, int col, int comp, double *out, hipStream_t s);
// diag[comp*N + i] = y[comp*N + i] for the unknowns of colour col
void amr_colour_take(const int *colour, int64_t N, int col, int comp, const double *y, double *diag, hipStream_t s);

}  // namespace mfs
