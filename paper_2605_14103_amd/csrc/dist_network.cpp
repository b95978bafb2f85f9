// Feeder registration: slack/non-slack split, reduced impedance matrix
// Z = inv(Y_NN) and no-load voltage v0 = -Z Y_NS v_S (Sec. II-B, eq. (10)).
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <string>

#include "dist.hpp"
#include "zfactor.hpp"

namespace pfx {

namespace {

using cplx = std::complex<double>;

// In-place inverse of a dense complex matrix (row-major n x n) by LU with
// partial pivoting.  Throws PF_SINGULAR_SETUP on a zero pivot.
void invert_dense(std::vector<cplx>& A, int n) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(A[(size_t)i * n + k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (!(best > 0)) fail(PF_SINGULAR_SETUP, "Y_NN is singular at column " + std::to_string(k));
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
    const cplx inv = 1.0 / A[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      cplx l = A[(size_t)i * n + k] * inv;
      A[(size_t)i * n + k] = l;
      if (l == cplx(0.0))
        continue;
      cplx* ri = &A[(size_t)i * n];
      const cplx* rk = &A[(size_t)k * n];
      for (int j = k + 1; j < n; ++j) ri[j] -= l * rk[j];
    }
  }
  // Solve for the inverse column by column: A = P^T L U.
  std::vector<cplx> X((size_t)n * n, cplx(0.0));
  std::vector<cplx> col(n);
  for (int c = 0; c < n; ++c) {
    std::fill(col.begin(), col.end(), cplx(0.0));
    col[c] = 1.0;
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(col[k], col[piv[k]]);
    for (int i = 0; i < n; ++i) {
      cplx s = col[i];
      const cplx* ri = &A[(size_t)i * n];
      for (int j = 0; j < i; ++j) s -= ri[j] * col[j];
      col[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      cplx s = col[i];
      const cplx* ri = &A[(size_t)i * n];
      for (int j = i + 1; j < n; ++j) s -= ri[j] * col[j];
      col[i] = s / ri[i];
    }
    for (int i = 0; i < n; ++i) X[(size_t)i * n + c] = col[i];
  }
  A.swap(X);
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

DistDev DistNetwork::view() const {
  DistDev d;
  d.nN = nN;
  d.nNs = round_up(nN, 64);
  d.Kp = Kp;
  d.Np = Np;
  d.y = y.view<double2>();
  d.node = node.as<int4>();
  d.c = c.as<double2>();
  d.v0 = v0.as<double>();
  d.free2ext = free2ext_d.as<int>();
  d.zf_nfq = zf_nfq;
  d.zf_nbq = zf_nbq;
  d.zf_pinv = zf_pinv.as<int>();
  d.zf_fmeta = zf_fmeta.as<int4>();
  d.zf_frow = zf_frow.as<int>();
  d.zf_fcol = zf_fcol.as<int>();
  d.zf_bmeta = zf_bmeta.as<int4>();
  d.zf_brow = zf_brow.as<int>();
  d.zf_bcol = zf_bcol.as<int>();
  d.zf_fval64 = zf_fval64.as<double2>();
  d.zf_bval64 = zf_bval64.as<double2>();
  d.zf_bd64 = zf_bd64.as<double2>();
  d.zf_fval32 = zf_fval32.as<float2>();
  d.zf_bval32 = zf_bval32.as<float2>();
  d.zf_bd32 = zf_bd32.as<float2>();
  return d;
}

DistNetwork* dist_network_create(Context* ctx, int n_node, int nnz, const int32_t* row_ptr,
                                 const int32_t* col_idx, const double* y_re, const double* y_im,
                                 const int32_t* slack_nodes, const double* v_slack, int n_wye,
                                 const int32_t* wye_node, int n_delta, const int32_t* delta_nodes,
                                 const pf_opts& setup) {
  (void)setup;
  require(n_node >= 4, "a feeder needs the three slack phases and at least one free node");
  require(row_ptr && col_idx && y_re && y_im && slack_nodes && v_slack, "null argument");
  require(row_ptr[0] == 0 && row_ptr[n_node] == nnz && nnz >= 0, "bad row_ptr");
  require(n_wye >= 0 && n_delta >= 0, "bad load counts");
  if (n_wye > 0) require(wye_node != nullptr, "null wye_node");
  if (n_delta > 0) require(delta_nodes != nullptr, "null delta_nodes");
  auto net = std::make_unique<DistNetwork>();
  net->ctx = ctx;
  net->n_node = n_node;
  std::vector<int> ext2free(n_node, 0);
  for (int s = 0; s < 3; ++s) {
    require(slack_nodes[s] >= 0 && slack_nodes[s] < n_node, "slack node out of range");
    net->slack[s] = slack_nodes[s];
    ext2free[slack_nodes[s]] = -1;
  }
  require(slack_nodes[0] != slack_nodes[1] && slack_nodes[1] != slack_nodes[2] &&
              slack_nodes[0] != slack_nodes[2],
          "slack nodes must be distinct");
  for (int q = 0; q < 6; ++q) net->v_slack[q] = v_slack[q];
  for (int i = 0; i < n_node; ++i)
    if (ext2free[i] == 0) {
      ext2free[i] = (int)net->free2ext.size();
      net->free2ext.push_back(i);
    }
  const int nN = (int)net->free2ext.size();
  require(nN <= ZB_MAX_FREE, "at most " + std::to_string(ZB_MAX_FREE) + " free nodes are supported");
  require(n_node < (1 << 30), "too many nodes");
  net->nN = nN;
  const int nNs = round_up(nN, 64);
  net->Kp = round_up(2 * nN, ZB_BK);
  net->Np = round_up(2 * nN, ZB_BN);

  // Y_NN (rows over free nodes) and c = Y_NS v_S.
  std::vector<SellRow> rows(nNs);
  std::vector<double> cc(2 * (size_t)nNs, 0.0);
  int nnz_nn = 0;
  std::vector<cplx> Yd((size_t)nN * nN, cplx(0.0));
  for (int fi = 0; fi < nN; ++fi) {
    const int e = net->free2ext[fi];
    require(row_ptr[e + 1] >= row_ptr[e], "row_ptr must be non-decreasing");
    std::map<int, cplx> row;
    cplx acc(0.0);
    for (int p = row_ptr[e]; p < row_ptr[e + 1]; ++p) {
      const int j = col_idx[p];
      require(j >= 0 && j < n_node, "column index out of range");
      const cplx y(y_re[p], y_im[p]);
      if (ext2free[j] >= 0) {
        row[ext2free[j]] += y;
      } else {
        int s = j == slack_nodes[0] ? 0 : (j == slack_nodes[1] ? 1 : 2);
        acc += y * cplx(v_slack[2 * s], v_slack[2 * s + 1]);
      }
    }
    for (auto& [j, y] : row) {
      rows[fi].emplace_back(j, y.real(), y.imag());
      Yd[(size_t)fi * nN + j] = y;
    }
    nnz_nn += (int)row.size();
    cc[2 * fi] = acc.real();
    cc[2 * fi + 1] = acc.imag();
  }
  net->nnz = nnz_nn;

  // Sparse L D L^T of Y_NN for the sparse variant, checked against the dense
  // inverse below.
  std::vector<int> zp(nN + 1, 0), zc;
  std::vector<cplx> zv;
  for (int i = 0; i < nN; ++i) {
    for (auto [j, re, im] : rows[i]) {
      zc.push_back(j);
      zv.push_back(cplx(re, im));
    }
    zp[i + 1] = (int)zc.size();
  }
  const ComplexLdl zf = complex_ldl(nN, zp, zc, zv);
  invert_dense(Yd, nN);  // Yd now holds Z
  {
    std::vector<cplx> b(nN), ref(nN, cplx(0.0));
    for (int i = 0; i < nN; ++i) b[i] = cplx(std::sin(0.37 * i + 0.1), std::cos(0.91 * i));
    for (int i = 0; i < nN; ++i)
      for (int l = 0; l < nN; ++l) ref[i] += Yd[(size_t)i * nN + l] * b[l];
    const std::vector<cplx> x = complex_ldl_solve(zf, b);
    double err = 0.0, mag = 0.0;
    for (int i = 0; i < nN; ++i) {
      err = std::max(err, std::abs(x[i] - ref[i]));
      mag = std::max(mag, std::abs(ref[i]));
    }
    if (!(err <= 1e-8 * mag))
      fail(PF_SINGULAR_SETUP, "sparse factor of Y_NN disagrees with the dense inverse (" + std::to_string(err) + ")");
  }
  std::vector<double> v0(2 * (size_t)nN);
  for (int i = 0; i < nN; ++i) {
    cplx s(0.0);
    for (int l = 0; l < nN; ++l) s += Yd[(size_t)i * nN + l] * cplx(cc[2 * l], cc[2 * l + 1]);
    v0[2 * i] = -s.real();
    v0[2 * i + 1] = -s.imag();
  }
  const int Kp = net->Kp, Np = net->Np;
  // W row-major (Kp x Np; the FP32 copy keeps this layout) ...
  std::vector<double> W((size_t)Kp * Np, 0.0);
  for (int i = 0; i < nN; ++i)
    for (int l = 0; l < nN; ++l) {
      const cplx z = Yd[(size_t)i * nN + l];
      W[(size_t)(2 * l) * Np + 2 * i] = z.real();
      W[(size_t)(2 * l + 1) * Np + 2 * i] = -z.imag();
      W[(size_t)(2 * l) * Np + 2 * i + 1] = z.imag();
      W[(size_t)(2 * l + 1) * Np + 2 * i + 1] = z.real();
    }
  // ... and the FP64 copy in K blocks of ZB_BK: (k, n) at ((k / ZB_BK) Np + n) ZB_BK + k % ZB_BK
  std::vector<double> Wb((size_t)Kp * Np);
  for (int k = 0; k < Kp; ++k)
    for (int n = 0; n < Np; ++n) Wb[((size_t)(k / ZB_BK) * Np + n) * ZB_BK + k % ZB_BK] = W[(size_t)k * Np + n];

  // Load tables.
  std::vector<uint8_t> wye(nN, 0);
  for (int q = 0; q < n_wye; ++q) {
    const int e = wye_node[q];
    require(e >= 0 && e < n_node && ext2free[e] >= 0, "wye load node must be a free node");
    wye[ext2free[e]] = 1;
  }
  std::vector<int> dn(nN, -1), dpv(nN, -1);
  for (int q = 0; q < n_delta; ++q) {
    int f[3];
    for (int p = 0; p < 3; ++p) {
      const int e = delta_nodes[3 * q + p];
      require(e >= 0 && e < n_node && ext2free[e] >= 0, "delta load node must be a free node");
      f[p] = ext2free[e];
      require(dn[f[p]] < 0, "a node belongs to two delta loads");
    }
    require(f[0] != f[1] && f[1] != f[2] && f[0] != f[2], "delta nodes must be distinct");
    for (int p = 0; p < 3; ++p) {
      dn[f[p]] = f[(p + 1) % 3];
      dpv[f[p]] = f[(p + 2) % 3];
    }
  }
  net->n_wye = n_wye;
  net->n_delta = n_delta;

  std::vector<int> nodes(4 * (size_t)nNs, 0);
  for (int i = 0; i < nN; ++i) {
    nodes[4 * i] = net->free2ext[i] | (wye[i] ? 1 << 30 : 0);
    nodes[4 * i + 1] = dn[i];
    nodes[4 * i + 2] = dpv[i];
    nodes[4 * i + 3] = dpv[i] >= 0 ? net->free2ext[dpv[i]] : 0;
  }
  for (int i = nN; i < nNs; ++i) nodes[4 * i + 1] = -1;

  upload_sell(ctx, build_sell(rows, 4), true, net->y);
  {
    // Level slices of the two solves (see DistDev): rows of each level in
    // chunks of 64, entries padded to a multiple of 4.
    struct Slices {
      std::vector<int> meta, row, col;
      std::vector<cplx> val, dinv;
      int count = 0;
    };
    auto slices = [&](const std::vector<int>& lev_start, const std::vector<int>& lev_rows,
                      const std::vector<int>& rptr, const std::vector<int>& rcol, const std::vector<cplx>& rval,
                      bool with_dinv) {
      Slices S;
      const int nl = (int)lev_start.size() - 1;
      for (int l = 0; l < nl; ++l) {
        for (int q0 = lev_start[l]; q0 < lev_start[l + 1]; q0 += 64) {
          const int q1 = std::min(q0 + 64, lev_start[l + 1]);
          int w = 4;
          for (int q = q0; q < q1; ++q) w = std::max(w, rptr[lev_rows[q] + 1] - rptr[lev_rows[q]]);
          w = (w + 3) / 4 * 4;
          const size_t base = S.col.size();
          S.meta.insert(S.meta.end(), {(int)base, w, q1 == lev_start[l + 1] ? 1 : 0, 0});
          ++S.count;
          S.col.resize(base + 64 * (size_t)w, 0);
          S.val.resize(base + 64 * (size_t)w, cplx(0.0));
          for (int lane = 0; lane < 64; ++lane) {
            const int q = q0 + lane;
            const int r = q < q1 ? lev_rows[q] : -1;
            S.row.push_back(r);
            if (with_dinv) S.dinv.push_back(r >= 0 ? zf.dinv[r] : cplx(0.0));
            if (r < 0) continue;
            for (int t = rptr[r], e = 0; t < rptr[r + 1]; ++t, ++e) {
              S.col[base + 64 * (size_t)e + lane] = rcol[t];
              S.val[base + 64 * (size_t)e + lane] = rval[t];
            }
          }
        }
      }
      if (S.count == 0) {  // keep every buffer non-empty
        S.meta = {0, 0, 0, 0};
        S.row = {-1};
        S.col = {0};
        S.val = {cplx(0.0)};
        S.dinv = {cplx(0.0)};
      }
      return S;
    };
    const Slices F = slices(zf.f_lev, zf.f_rows, zf.L_ptr, zf.L_col, zf.L_val, false);
    const Slices Bk = slices(zf.b_lev, zf.b_rows, zf.T_ptr, zf.T_col, zf.T_val, true);
    auto interleave = [](const std::vector<cplx>& v) {
      std::vector<double> d(2 * v.size());
      for (size_t i = 0; i < v.size(); ++i) {
        d[2 * i] = v[i].real();
        d[2 * i + 1] = v[i].imag();
      }
      return d;
    };
    auto up64 = [&](const std::vector<cplx>& v) { return upload(ctx, interleave(v)); };
    auto up32 = [&](const std::vector<cplx>& v) {
      const std::vector<double> d = interleave(v);
      return upload(ctx, std::vector<float>(d.begin(), d.end()));
    };
    std::vector<int> pinv(nN > 0 ? nN : 1, 0);
    for (int p = 0; p < nN; ++p) pinv[zf.perm[p]] = p;
    net->zf_nfq = F.count;
    net->zf_nbq = Bk.count;
    net->zf_pinv = upload(ctx, pinv);
    net->zf_fmeta = upload(ctx, F.meta);
    net->zf_frow = upload(ctx, F.row);
    net->zf_fcol = upload(ctx, F.col);
    net->zf_bmeta = upload(ctx, Bk.meta);
    net->zf_brow = upload(ctx, Bk.row);
    net->zf_bcol = upload(ctx, Bk.col);
    net->zf_fval64 = up64(F.val);
    net->zf_bval64 = up64(Bk.val);
    net->zf_bd64 = up64(Bk.dinv);
    net->zf_fval32 = up32(F.val);
    net->zf_bval32 = up32(Bk.val);
    net->zf_bd32 = up32(Bk.dinv);
  }
  net->node = upload(ctx, nodes);
  net->c = upload(ctx, cc);
  net->v0 = upload(ctx, v0);
  net->free2ext_d = upload(ctx, net->free2ext);
  net->W64 = upload(ctx, Wb);
  net->W32 = upload(ctx, std::vector<float>(W.begin(), W.end()));
  net->slack_d = upload(ctx, std::vector<int>(net->slack, net->slack + 3));
  net->vslack_d = upload(ctx, std::vector<double>(net->v_slack, net->v_slack + 6));
  return net.release();
}

}  // namespace pfx
