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

// E-vectors: velocity [cell][(k+1)^3][3], then pressure [cell][(k+1)^3].
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
