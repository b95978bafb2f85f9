// Sparse complex-symmetric L D L^T factor of a feeder's Y_NN, for applying
// Z = Y_NN^-1 by triangular solves instead of a dense product (the sparse
// Z-bus variant the paper leaves as future work, Sec. II-B).
//
// Y_NN of a radial feeder is complex symmetric (not Hermitian) with a
// positive definite real part when every segment has resistance, so the
// factorisation runs without pivoting.  Under a minimum-degree order the
// radial structure gives almost no fill.  The solves run level by level: a
// row's forward (backward) level is one more than the deepest row it reads.
#pragma once

#include <complex>
#include <vector>

namespace pfx {

struct ComplexLdl {
  using cplx = std::complex<double>;
  int n = 0;
  std::vector<int> perm;   // perm[p] = matrix row at factor position p
  // strictly lower L by rows (factor positions)
  std::vector<int> L_ptr, L_col;
  std::vector<cplx> L_val;
  std::vector<cplx> dinv;  // 1 / D
  // strictly upper L^T by rows: row j lists (i, L[i][j]) for i > j
  std::vector<int> T_ptr, T_col;
  std::vector<cplx> T_val;
  // forward and backward levels: rows of level l are rows[lev[l] .. lev[l + 1])
  std::vector<int> f_lev, f_rows, b_lev, b_rows;
};

// Factorise the n x n matrix given in CSR (both triangles, complex values).
// Throws PfError(PF_SINGULAR_SETUP) on a zero pivot.
ComplexLdl complex_ldl(int n, const std::vector<int>& ptr, const std::vector<int>& col,
                       const std::vector<std::complex<double>>& val);

// Host application of the factor: x with A x = b (matrix order).
std::vector<std::complex<double>> complex_ldl_solve(const ComplexLdl& F,
                                                    const std::vector<std::complex<double>>& b);

}  // namespace pfx
