// Transmission network registration: index sets, internal ordering, the
// preconditioner blocks of eq. (7) and their precomputed inverses.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <string>

#include "tx.hpp"

namespace pfx {

namespace {

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

void upload_factor(Context* ctx, SpdBuffers& s) {
  const HybridFactor& F = s.host;
  s.pinv = upload(ctx, F.pinv);
  s.f_lev = upload(ctx, F.f_lev);
  s.f_rows = upload(ctx, F.f_rows);
  s.L_ptr = upload(ctx, F.L_ptr);
  s.L_col = upload(ctx, F.L_col);
  s.b_lev = upload(ctx, F.b_lev);
  s.b_rows = upload(ctx, F.b_rows);
  s.T_ptr = upload(ctx, F.T_ptr);
  s.T_col = upload(ctx, F.T_col);
  s.L_val64 = upload(ctx, F.L_val);
  s.dinv64 = upload(ctx, F.dinv);
  s.T_val64 = upload(ctx, F.T_val);
  s.Sinv64 = upload(ctx, F.Sinv);
  s.L_val32 = upload(ctx, cast_vec<float>(F.L_val));
  s.dinv32 = upload(ctx, cast_vec<float>(F.dinv));
  s.T_val32 = upload(ctx, cast_vec<float>(F.T_val));
  s.Sinv32 = upload(ctx, cast_vec<float>(F.Sinv));
}

// A principal submatrix of -Im(Y) (rows/cols 0..k-1 of the internal order) plus eps I.
SparseSym leading_block(const std::vector<int>& ptr, const std::vector<int>& col,
                        const std::vector<double>& yim, int k, double eps) {
  SparseSym A;
  A.n = k;
  A.ptr.assign(k + 1, 0);
  for (int i = 0; i < k; ++i) {
    bool diag = false;
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
      int j = col[p];
      if (j >= k) continue;
      double v = -yim[p];
      if (j == i) {
        v += eps;
        diag = true;
      }
      A.col.push_back(j);
      A.val.push_back(v);
    }
    if (!diag) {  // keep columns sorted
      auto it = std::lower_bound(A.col.begin() + A.ptr[i], A.col.end(), i);
      size_t pos = it - A.col.begin();
      A.col.insert(A.col.begin() + pos, i);
      A.val.insert(A.val.begin() + pos, eps);
    }
    A.ptr[i + 1] = (int)A.col.size();
  }
  return A;
}

void check_factor(const SparseSym& A, const HybridFactor& F, const char* name) {
  // Set-up self-check: solve against a fixed right-hand side and verify the residual.
  std::vector<double> b(A.n);
  for (int i = 0; i < A.n; ++i) b[i] = 1.0 + 0.25 * std::sin(0.7 * i);
  std::vector<double> x = hybrid_solve(F, b);
  // Backward-error test: |b - A x| against |A| |x| + |b| (the matrix may be indefinite).
  double rmax = 0.0, scale = 0.0;
  for (int i = 0; i < A.n; ++i) {
    double r = b[i], ax = 0.0;
    for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      r -= A.val[p] * x[A.col[p]];
      ax += std::fabs(A.val[p] * x[A.col[p]]);
    }
    rmax = std::max(rmax, std::fabs(r));
    scale = std::max(scale, ax + std::fabs(b[i]));
  }
  if (!(rmax <= 1e-9 * scale))
    fail(PF_SINGULAR_SETUP, std::string(name) + " factor self-check failed, residual " + std::to_string(rmax));
}

}  // namespace

template <typename T>
SpdDev<T> SpdBuffers::view() const {
  constexpr bool f64 = sizeof(T) == 8;
  SpdDev<T> d;
  d.N = host.N;
  d.c = host.c;
  d.k = host.k;
  d.nfl = host.n_fwd_levels();
  d.nbl = host.n_bwd_levels();
  d.pinv = pinv.as<int>();
  d.f_lev = f_lev.as<int>();
  d.f_rows = f_rows.as<int>();
  d.L_ptr = L_ptr.as<int>();
  d.L_col = L_col.as<int>();
  d.L_val = f64 ? L_val64.as<T>() : L_val32.as<T>();
  d.dinv = f64 ? dinv64.as<T>() : dinv32.as<T>();
  d.b_lev = b_lev.as<int>();
  d.b_rows = b_rows.as<int>();
  d.T_ptr = T_ptr.as<int>();
  d.T_col = T_col.as<int>();
  d.T_val = f64 ? T_val64.as<T>() : T_val32.as<T>();
  d.Sinv = f64 ? Sinv64.as<T>() : Sinv32.as<T>();
  return d;
}

template <typename T>
TxDev<T> TxNetwork::view() const {
  constexpr bool f64 = sizeof(T) == 8;
  TxDev<T> d;
  d.n = n;
  d.nth = nth;
  d.npq = npq;
  d.m = m;
  d.y_ptr = y_ptr.as<int>();
  d.y_col = y_col.as<int>();
  d.y_re = y_re.as<double>();
  d.y_im = y_im.as<double>();
  d.int2ext = int2ext_d.as<int>();
  d.bp = bp.view<T>();
  d.bpp = bpp.view<T>();
  d.g_ptr = g_ptr.as<int>();
  d.g_col = g_col.as<int>();
  d.g_val = f64 ? g_val64.as<T>() : g_val32.as<T>();
  d.gt_ptr = gt_ptr.as<int>();
  d.gt_col = gt_col.as<int>();
  d.gt_val = f64 ? gt_val64.as<T>() : gt_val32.as<T>();
  d.n_branch = n_branch;
  d.br_f = br_f.as<int>();
  d.br_t = br_t.as<int>();
  d.br_ys_re = br_ys_re.as<double>();
  d.br_ys_im = br_ys_im.as<double>();
  d.br_b = br_b.as<double>();
  d.yt_ptr = yt_ptr.as<int>();
  d.yt_col = yt_col.as<int>();
  d.yt_re = yt_re.as<double>();
  d.yt_im = yt_im.as<double>();
  return d;
}

template SpdDev<double> SpdBuffers::view<double>() const;
template SpdDev<float> SpdBuffers::view<float>() const;
template TxDev<double> TxNetwork::view<double>() const;
template TxDev<float> TxNetwork::view<float>() const;

TxNetwork* tx_network_create(Context* ctx, int n_bus, int nnz, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* y_re, const double* y_im,
                             const int8_t* bus_type, int n_branch, const int32_t* br_f,
                             const int32_t* br_t, const double* br_r, const double* br_x,
                             const double* br_b, const pf_opts& setup) {
  require(n_bus >= 2, "n_bus must be at least 2");
  require(nnz >= n_bus && row_ptr && col_idx && y_re && y_im && bus_type, "bad Ybus arguments");
  require(row_ptr[0] == 0 && row_ptr[n_bus] == nnz, "row_ptr must start at 0 and end at nnz");
  require(n_branch >= 0, "n_branch must be >= 0");
  if (n_branch > 0) require(br_f && br_t && br_r && br_x && br_b, "null branch array");
  int n_slack = 0;
  std::vector<int> pq, pv;
  int slack = -1;
  for (int i = 0; i < n_bus; ++i) {
    require(bus_type[i] >= 0 && bus_type[i] <= 2, "bus_type must be 0, 1 or 2");
    if (bus_type[i] == 0) pq.push_back(i);
    else if (bus_type[i] == 1) pv.push_back(i);
    else {
      slack = i;
      ++n_slack;
    }
  }
  require(n_slack == 1, "exactly one slack bus is required");
  for (int i = 0; i < n_bus; ++i) {
    require(row_ptr[i + 1] >= row_ptr[i], "row_ptr must be non-decreasing");
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
      require(col_idx[p] >= 0 && col_idx[p] < n_bus, "column index out of range");
  }

  auto net = std::make_unique<TxNetwork>();
  net->ctx = ctx;
  net->setup = setup;
  net->n = n_bus;
  net->nth = n_bus - 1;
  net->npq = (int)pq.size();
  net->m = net->nth + net->npq;
  net->n_branch = n_branch;
  net->int2ext = pq;
  net->int2ext.insert(net->int2ext.end(), pv.begin(), pv.end());
  net->int2ext.push_back(slack);
  net->ext2int.assign(n_bus, 0);
  for (int i = 0; i < n_bus; ++i) net->ext2int[net->int2ext[i]] = i;

  // Ybus in internal order, duplicates summed, columns sorted.
  std::vector<int> ptr(n_bus + 1, 0), col;
  std::vector<double> yre, yim;
  for (int i = 0; i < n_bus; ++i) {
    int e = net->int2ext[i];
    std::map<int, std::complex<double>> row;
    for (int p = row_ptr[e]; p < row_ptr[e + 1]; ++p)
      row[net->ext2int[col_idx[p]]] += std::complex<double>(y_re[p], y_im[p]);
    for (auto& [j, y] : row) {
      col.push_back(j);
      yre.push_back(y.real());
      yim.push_back(y.imag());
    }
    ptr[i + 1] = (int)col.size();
  }
  net->nnz = (int)col.size();

  // B' = -Im(Y)[Theta, Theta] + eps I, B'' = -Im(Y)[Q, Q] + eps I (eqs. (7)-(9)).
  const double eps = setup.eps;
  SparseSym Bp = leading_block(ptr, col, yim, net->nth, eps);
  SparseSym Bpp = leading_block(ptr, col, yim, net->npq, eps);
  if (setup.precond_block > 0) {
    Bp = block_diagonal_part(Bp, setup.precond_block);
    Bpp = block_diagonal_part(Bpp, setup.precond_block);
  }
  net->bp.host = hybrid_factor(Bp, setup.factor_max_levels, setup.factor_max_core);
  check_factor(Bp, net->bp.host, "B'");
  if (net->npq > 0) {
    net->bpp.host = hybrid_factor(Bpp, setup.factor_max_levels, setup.factor_max_core);
    check_factor(Bpp, net->bpp.host, "B''");
  }

  // G = -Re(Y)[Q, Theta] with columns as positions of the B' factor, and G^T
  // with columns as positions of the B'' factor.
  std::vector<int> gptr(net->npq + 1, 0), gcol;
  std::vector<double> gval;
  std::vector<std::vector<std::pair<int, double>>> gt_rows(net->nth);
  for (int q = 0; q < net->npq; ++q) {
    for (int p = ptr[q]; p < ptr[q + 1]; ++p) {
      int j = col[p];
      if (j >= net->nth) continue;
      double g = -yre[p];
      gcol.push_back(net->bp.host.pinv[j]);
      gval.push_back(g);
      gt_rows[j].push_back({net->bpp.host.pinv.empty() ? 0 : net->bpp.host.pinv[q], g});
    }
    gptr[q + 1] = (int)gcol.size();
  }
  std::vector<int> gtptr(net->nth + 1, 0), gtcol;
  std::vector<double> gtval;
  for (int j = 0; j < net->nth; ++j) {
    for (auto [c, v] : gt_rows[j]) {
      gtcol.push_back(c);
      gtval.push_back(v);
    }
    gtptr[j + 1] = (int)gtcol.size();
  }

  net->y_ptr = upload(ctx, ptr);
  net->y_col = upload(ctx, col);
  net->y_re = upload(ctx, yre);
  net->y_im = upload(ctx, yim);
  net->int2ext_d = upload(ctx, net->int2ext);
  {
    std::vector<int> tp(n_bus + 1, 0), tc(col.size());
    std::vector<double> tr(col.size()), ti(col.size());
    for (int j : col) tp[j + 1]++;
    for (int i = 0; i < n_bus; ++i) tp[i + 1] += tp[i];
    std::vector<int> fill(tp.begin(), tp.end() - 1);
    for (int i = 0; i < n_bus; ++i)
      for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
        const int q = fill[col[p]]++;
        tc[q] = i;
        tr[q] = yre[p];
        ti[q] = yim[p];
      }
    net->yt_ptr = upload(ctx, tp);
    net->yt_col = upload(ctx, tc);
    net->yt_re = upload(ctx, tr);
    net->yt_im = upload(ctx, ti);
  }
  upload_factor(ctx, net->bp);
  if (net->npq > 0) upload_factor(ctx, net->bpp);
  net->g_ptr = upload(ctx, gptr);
  net->g_col = upload(ctx, gcol);
  net->g_val64 = upload(ctx, gval);
  net->g_val32 = upload(ctx, cast_vec<float>(gval));
  net->gt_ptr = upload(ctx, gtptr);
  net->gt_col = upload(ctx, gtcol);
  net->gt_val64 = upload(ctx, gtval);
  net->gt_val32 = upload(ctx, cast_vec<float>(gtval));

  std::vector<int> bf(n_branch), bt(n_branch);
  std::vector<double> ysr(n_branch), ysi(n_branch), bb(n_branch);
  for (int k = 0; k < n_branch; ++k) {
    require(br_f[k] >= 0 && br_f[k] < n_bus && br_t[k] >= 0 && br_t[k] < n_bus,
            "branch bus index out of range");
    require(br_f[k] != br_t[k], "a branch must join two different buses");
    bf[k] = net->ext2int[br_f[k]];
    bt[k] = net->ext2int[br_t[k]];
    const std::complex<double> z(br_r[k], br_x[k]);
    require(std::abs(z) > 0, "zero branch impedance");
    const std::complex<double> ys = 1.0 / z;
    ysr[k] = ys.real();
    ysi[k] = ys.imag();
    bb[k] = br_b[k];
  }
  net->br_f = upload(ctx, bf);
  net->br_t = upload(ctx, bt);
  net->br_ys_re = upload(ctx, ysr);
  net->br_ys_im = upload(ctx, ysi);
  net->br_b = upload(ctx, bb);
  std::vector<int> iptr(n_bus + 1, 0), ibr(2 * (size_t)n_branch);
  for (int k = 0; k < n_branch; ++k) {
    iptr[bf[k] + 1]++;
    iptr[bt[k] + 1]++;
  }
  for (int i = 0; i < n_bus; ++i) iptr[i + 1] += iptr[i];
  {
    std::vector<int> fill(iptr.begin(), iptr.end() - 1);
    for (int k = 0; k < n_branch; ++k) {
      ibr[fill[bf[k]]++] = k;
      ibr[fill[bt[k]]++] = k;
    }
  }
  net->inc_ptr = upload(ctx, iptr);
  net->inc_br = upload(ctx, ibr);
  net->desc64 = upload(ctx, std::vector<TxDev<double>>{net->view<double>()});
  net->desc32 = upload(ctx, std::vector<TxDev<float>>{net->view<float>()});
  return net.release();
}

}  // namespace pfx
