// Host-side building blocks of the typed-ELL multigrid hierarchies (the H(div) problem and the
// Stokes velocity block of the Darcy-Stokes problem): matrices under assembly, their typed ELL
// form, dense SPD inverses and the vertex-patch tables of the additive Schwarz smoother.
#pragma once

#include <functional>
#include <vector>

#include "hdiv_internal.h"

namespace fdd {

// Rows of a matrix under assembly: at most `cap` (column, value) pairs per row.
struct RowBuilder {
  int rows, cap;
  std::vector<int> cnt, col;
  std::vector<double> val;
  bool overflow = false;
  RowBuilder(int r, int c) : rows(r), cap(c), cnt(r, 0), col((size_t)r * c), val((size_t)r * c) {}
  // adds v to entry (i, j); false (and the overflow flag) when row i is full
  bool add(int i, int j, double v);
  // ELL form, columns ascending within a row, rows typed by their value sequence
  void to_ell(HdMat* M, int ncols) const;
};

// Entry (i, j) of an ELL matrix (0 if absent).
double ell_entry(const HdMat& M, int i, int j);

// R = P^T for an ELL matrix P with `cols` columns.
void ell_transpose(const HdMat& P, int cols, HdMat* R);

// SPD inverse by Cholesky (row-major, in place); false if not positive definite.
bool spd_inverse(std::vector<double>& A, int m);

// Vertex-patch tables of level L (its matrix L->A set) with patch stride pw (1, 8 or kHdPatch):
// `list(v, dofs)` writes the dofs of patch v (at most pw) and returns their count (0: no patch).
// Every dof may lie in at most two patches.  Patch matrices are deduplicated into types
// (congruent patches are bit-identical) and inverted.  Returns nullptr or a message.
const char* build_patch_tables(HdLevel* L, int nvert, int pw,
                               const std::function<int(int, int*)>& list);

}  // namespace fdd
