// Exact inverse of a sparse symmetric matrix (positive definite or not),
// prepared on the host for application inside a workgroup.
//
// The preconditioner of eq. (7) needs (B' + eps I)^-1 and (B'' + eps I)^-1,
// which the paper precomputes once (Sec. II-A).  Here they are represented as
// an L D L^T factor (unit lower L) under a minimum-degree ordering, split into
//   * a sparse prefix (the first c pivots), whose triangular solves take only
//     a few dependency levels, and
//   * a dense trailing core of k = N - c pivots, kept as the explicit inverse of
//     its Schur complement S = A22 - L21 D1 L21^T (Gauss-Jordan with pivoting).
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
// PfError(PF_SINGULAR_SETUP) on a zero pivot or a singular core.
HybridFactor hybrid_factor(const SparseSym& A, int max_levels, int max_core);

// Reference application of the hybrid factor (host, FP64), used by the
// library's own set-up self-check: returns x with A x = b.
std::vector<double> hybrid_solve(const HybridFactor& F, const std::vector<double>& b);

// Explicit application form of a hybrid factor.  With the unit lower factor
// L = [L11 0; L21 I] and the block diagonal Dt = diag(D, S), A = L Dt L^T, so
//   A^-1 b = L^-T Dt^-1 L^-1 b.
// L^-1 is formed explicitly: column j (j < c) is the sparse solution of
// L y = e_j, whose nonzeros are the positions reachable from j in the graph of
// L (a few per column when the prefix has few levels); columns j >= c are unit
// vectors.  The application then takes three passes with no dependency chain
// inside any of them:
//   E1:  u = Dt'^-1 L^-1 b, one sparse row per position: rows r < c give
//        y_r = D_r^-1 (L^-1 b)_r, rows r >= c give t = (L^-1 b)_r (the right-
//        hand side of the dense core);
//   E2:  x2 = S^-1 t (dense k x k);
//   E3:  x = L^-T [y ; x2], row p being column p of L^-1.
// Rows list (position, value) pairs over factor positions.
struct ExplicitFactor {
  int N = 0, c = 0, k = 0;
  std::vector<std::vector<std::pair<int, double>>> e1;  // N rows
  std::vector<std::vector<std::pair<int, double>>> e3;  // N rows
  std::vector<double> Sinv;                             // k x k
  std::vector<int> perm, pinv;                          // as in HybridFactor
  long entries() const;
};

ExplicitFactor explicit_form(const HybridFactor& F);

// x = A^-1 b through the explicit form (host, FP64; b and x in matrix order).
std::vector<double> explicit_solve(const ExplicitFactor& E, const std::vector<double>& b);

// Factor A for explicit application, choosing the number of prefix levels
// (1..max_levels, dense core at most max_core) that minimises the per-thread
// work of one application on `block` threads: padded sparse entries / block
// plus the core size.
ExplicitFactor explicit_factor(const SparseSym& A, int max_levels, int max_core, int block);

}  // namespace pfx
