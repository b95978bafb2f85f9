// Sparse complex-symmetric L D L^T of Y_NN with level schedules for the
// triangular solves.
#include "zfactor.hpp"

#include <algorithm>
#include <map>
#include <string>

#include "common.hpp"
#include "factor.hpp"

namespace pfx {

ComplexLdl complex_ldl(int n, const std::vector<int>& ptr, const std::vector<int>& col,
                       const std::vector<std::complex<double>>& val) {
  using cplx = std::complex<double>;
  ComplexLdl F;
  F.n = n;
  // Minimum-degree order of the sparsity graph (values do not matter for it).
  SparseSym pattern;
  pattern.n = n;
  pattern.ptr = ptr;
  pattern.col = col;
  pattern.val.assign(col.size(), 1.0);
  F.perm = min_degree_order(pattern);
  std::vector<int> pinv(n);
  for (int p = 0; p < n; ++p) pinv[F.perm[p]] = p;
  // Rows of the permuted matrix as ordered maps; elimination fills them in.
  std::vector<std::map<int, cplx>> a(n);
  for (int i = 0; i < n; ++i)
    for (int q = ptr[i]; q < ptr[i + 1]; ++q) a[pinv[i]][pinv[col[q]]] += val[q];
  std::vector<std::map<int, cplx>> lrows(n);   // strictly lower L by rows
  F.dinv.assign(n, cplx(0.0));
  for (int k = 0; k < n; ++k) {
    const cplx d = a[k][k];
    if (!(std::abs(d) > 0)) fail(PF_SINGULAR_SETUP, "zero pivot in the sparse Y_NN factor at " + std::to_string(k));
    F.dinv[k] = 1.0 / d;
    // Column k below the diagonal equals row k right of it (symmetry).  Only
    // the upper parts (diagonal included) of the trailing rows are read and
    // updated, so they carry the whole trailing matrix.
    std::vector<std::pair<int, cplx>> below;
    for (auto it = a[k].upper_bound(k); it != a[k].end(); ++it) below.push_back(*it);
    for (auto [i, aik] : below) {
      const cplx l = aik / d;
      lrows[i][k] = l;
      for (auto [j, akj] : below)
        if (j >= i) a[i][j] -= l * akj;
    }
    a[k].clear();
  }
  // CSR of L by rows and of L^T by rows.
  F.L_ptr.assign(n + 1, 0);
  std::vector<std::vector<std::pair<int, cplx>>> trows(n);
  for (int i = 0; i < n; ++i) {
    for (auto [j, l] : lrows[i]) {
      F.L_col.push_back(j);
      F.L_val.push_back(l);
      trows[j].push_back({i, l});
    }
    F.L_ptr[i + 1] = (int)F.L_col.size();
  }
  F.T_ptr.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) {
    for (auto [i, l] : trows[j]) {
      F.T_col.push_back(i);
      F.T_val.push_back(l);
    }
    F.T_ptr[j + 1] = (int)F.T_col.size();
  }
  // Levels: forward, a row after every row it reads; backward, likewise on L^T.
  std::vector<int> fl(n, 0), bl(n, 0);
  int nf = 0, nb = 0;
  for (int i = 0; i < n; ++i) {
    for (int q = F.L_ptr[i]; q < F.L_ptr[i + 1]; ++q) fl[i] = std::max(fl[i], fl[F.L_col[q]] + 1);
    nf = std::max(nf, fl[i] + 1);
  }
  for (int j = n - 1; j >= 0; --j) {
    for (int q = F.T_ptr[j]; q < F.T_ptr[j + 1]; ++q) bl[j] = std::max(bl[j], bl[F.T_col[q]] + 1);
    nb = std::max(nb, bl[j] + 1);
  }
  auto group = [n](const std::vector<int>& lev, int nl, std::vector<int>& starts, std::vector<int>& rows) {
    starts.assign(nl + 1, 0);
    for (int i = 0; i < n; ++i) ++starts[lev[i] + 1];
    for (int l = 0; l < nl; ++l) starts[l + 1] += starts[l];
    rows.assign(n, 0);
    std::vector<int> fill(starts.begin(), starts.end() - 1);
    for (int i = 0; i < n; ++i) rows[fill[lev[i]]++] = i;
  };
  group(fl, nf, F.f_lev, F.f_rows);
  group(bl, nb, F.b_lev, F.b_rows);
  return F;
}

std::vector<std::complex<double>> complex_ldl_solve(const ComplexLdl& F,
                                                    const std::vector<std::complex<double>>& b) {
  using cplx = std::complex<double>;
  const int n = F.n;
  std::vector<cplx> u(n);
  for (int p = 0; p < n; ++p) u[p] = b[F.perm[p]];
  for (int i = 0; i < n; ++i)
    for (int q = F.L_ptr[i]; q < F.L_ptr[i + 1]; ++q) u[i] -= F.L_val[q] * u[F.L_col[q]];
  for (int i = 0; i < n; ++i) u[i] *= F.dinv[i];
  for (int j = n - 1; j >= 0; --j)
    for (int q = F.T_ptr[j]; q < F.T_ptr[j + 1]; ++q) u[j] -= F.T_val[q] * u[F.T_col[q]];
  std::vector<cplx> x(n);
  for (int p = 0; p < n; ++p) x[F.perm[p]] = u[p];
  return x;
}

}  // namespace pfx
