// Exact inverse of a sparse symmetric positive definite matrix, prepared on the
// host for level-scheduled application inside a workgroup.
//
// The preconditioner of eq. (7) needs (B' + eps I)^-1 and (B'' + eps I)^-1,
// which the paper precomputes once (Sec. II-A).  Here they are represented as
// a Cholesky factor under a minimum-degree ordering, split into
//   * a sparse prefix (the first c pivots), whose triangular solves take only
//     a few dependency levels, and
//   * a dense trailing core of k = N - c pivots, kept as the explicit inverse of
//     its Schur complement S = A22 - L21 L21^T.
// Solving A x = b then is: forward levels over the prefix, t = b2 - L21 y1,
// x2 = S^-1 t, backward levels over the prefix with x2 known.
#pragma once

#include <vector>

namespace pfx {

// Symmetric matrix in CSR with both triangles stored, columns sorted.
struct SparseSym {
  int n = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

struct HybridFactor {
  int N = 0, c = 0, k = 0;
  std::vector<int> perm;   // perm[p] = matrix row at factor position p
  std::vector<int> pinv;   // pinv[row] = factor position
  // forward solve: prefix rows grouped by level
  std::vector<int> f_lev, f_rows;
  // strictly lower rows of L restricted to prefix columns, for all N positions
  std::vector<int> L_ptr, L_col;
  std::vector<double> L_val;
  std::vector<double> dinv;  // 1 / L[j][j], j < c
  // backward solve: prefix rows grouped by reverse level; row j lists (i, L[i][j]), i > j
  std::vector<int> b_lev, b_rows;
  std::vector<int> T_ptr, T_col;
  std::vector<double> T_val;
  std::vector<double> Sinv;  // k x k, symmetric
  int factor_nnz = 0;        // nonzeros of the full Cholesky factor
  int n_fwd_levels() const { return (int)f_lev.size() - 1; }
  int n_bwd_levels() const { return (int)b_lev.size() - 1; }
};

// Minimum-degree elimination order of the graph of A (lowest index on ties).
std::vector<int> min_degree_order(const SparseSym& A);

// Keep only the entries whose rows and columns fall in the same block of
// `block` consecutive positions of a breadth-first order of A's graph.
SparseSym block_diagonal_part(const SparseSym& A, int block);

// Factorise A (which must already hold any regularisation).  Throws
// PfError(PF_SINGULAR_SETUP) if a pivot is not positive.
HybridFactor hybrid_factor(const SparseSym& A, int max_levels, int max_core);

// Reference application of the hybrid factor (host, FP64), used by the
// library's own set-up self-check: returns x with A x = b.
std::vector<double> hybrid_solve(const HybridFactor& F, const std::vector<double>& b);

}  // namespace pfx
