// Transmission network registration: index sets, internal ordering, the
// preconditioner blocks of eq. (7) with their precomputed inverses, and the
// sliced layouts the kernels read.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <numeric>
#include <string>
#include <tuple>

#include "direct.hpp"
#include "tx.hpp"

namespace pfx {

namespace {

constexpr int SLICE = 64;

using Row = SellRow;

// Lay out one explicit factor for workgroups of `block` threads with kb bus
// slots each (the factor order has N <= kb * block rows).
void upload_factor(Context* ctx, EfBuffers& f, int block, int kb, int nbp) {
  const ExplicitFactor& E = f.host;
  const int N = E.N, nw = block / SLICE;
  // E1: rows by decreasing length, columns in matrix order.
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return E.e1[a].size() > E.e1[b].size(); });
  const int ns1 = (N + SLICE - 1) / SLICE;
  std::vector<Row> rows1((size_t)ns1 * SLICE);
  std::vector<int> rid((size_t)ns1 * SLICE, -1);
  for (int q = 0; q < N; ++q) {
    const int r = order[q];
    rid[q] = r;
    for (auto [j, v] : E.e1[r]) rows1[q].push_back({E.perm[j], v, 0.0});
  }
  const auto [off1, width1] = upload_psell(ctx, rows1, f.e1);   // widths in groups of four entries
  // Slices to waves: longest first, each to the least loaded wave with room.
  std::vector<int> sl(ns1);
  std::iota(sl.begin(), sl.end(), 0);
  std::stable_sort(sl.begin(), sl.end(), [&](int a, int b) { return width1[a] > width1[b]; });
  // (the slice list is longest first, so the greedy assignment balances the
  // longest slices first; a wave may take any number of slices, so the one
  // with the longest slice takes few others)
  // Per wave, e1_nq entries: (group offset, width, first row of the slice, 0);
  // width 0 past the wave's list.
  std::vector<int> load(nw, 0), cnt(nw, 0), owner(ns1, 0), slot(ns1, 0);
  for (int s : sl) {
    int best = 0;
    for (int w = 1; w < nw; ++w)
      if (load[w] < load[best]) best = w;
    owner[s] = best;
    slot[s] = cnt[best]++;
    load[best] += (width1[s] + 1) / 2 + 1;   // rounds of up to two groups, plus the slice's own overhead
  }
  const int nq1 = std::max(1, *std::max_element(cnt.begin(), cnt.end()));
  std::vector<int> wave_list((size_t)nw * nq1 * 4, 0);
  for (int s = 0; s < ns1; ++s) {
    int* e = &wave_list[((size_t)owner[s] * nq1 + slot[s]) * 4];
    e[0] = off1[s];
    e[1] = width1[s];
    e[2] = s * SLICE;
  }
  f.e1_nq = nq1;
  // E3: one row per matrix row (bus order), padded to nbp rows.
  std::vector<Row> rows3(nbp);
  for (int i = 0; i < N; ++i)
    for (auto [p, v] : E.e3[E.pinv[i]]) rows3[i].push_back({p, v, 0.0});
  upload_psell(ctx, rows3, f.e3);
  {
    // E3 again with its rows sorted by length (the pass that stores its
    // results to LDS rather than to the owning threads' registers): slices of
    // 64 rows, longest first, each to the wave with the fewest rounds so far
    // and a free slot; the slice goes to position slot * nw + wave.
    std::vector<int> ord(N);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      return E.e3[E.pinv[a]].size() > E.e3[E.pinv[b]].size();
    });
    const int ns = (N + SLICE - 1) / SLICE;
    if (ns > nw * kb) fail(PF_INVALID_ARG, "factor does not fit the workgroup layout");
    std::vector<Row> rows3s((size_t)nw * kb * SLICE);
    std::vector<int> rid3((size_t)nw * kb * SLICE, -1), load3(nw, 0), cnt3(nw, 0);
    for (int s = 0; s < ns; ++s) {
      const int w4 = std::max(4, ((int)E.e3[E.pinv[ord[(size_t)s * SLICE]]].size() + 3) / 4 * 4);
      int best = -1;
      for (int w = 0; w < nw; ++w)
        if (cnt3[w] < kb && (best < 0 || load3[w] < load3[best])) best = w;
      const int pos = cnt3[best]++ * nw + best;
      load3[best] += (w4 + 7) / 8;   // rounds of eight entries, then one of four
      for (int l = 0; l < SLICE && s * SLICE + l < N; ++l) {
        const int i = ord[(size_t)s * SLICE + l];
        for (auto [p, v] : E.e3[E.pinv[i]]) rows3s[(size_t)pos * SLICE + l].push_back({p, v, 0.0});
        rid3[(size_t)pos * SLICE + l] = i;
      }
    }
    upload_psell(ctx, rows3s, f.e3s);
    f.e3s_row = upload(ctx, rid3);
  }
  // With no core, A^-1 = E3 E1 (times the permutation) may stay sparse: if its
  // sliced rows are not much longer than E1's and E3's together, it is
  // applied in one pass with no barrier inside.
  f.direct = false;
  if (E.k == 0) {
    std::vector<Row> rowsd(nbp);
    long nnz = 0;
    for (int i = 0; i < N; ++i) {
      std::map<int, double> acc;
      for (auto [p, v3] : E.e3[E.pinv[i]])
        for (auto [j, v1] : E.e1[p]) acc[E.perm[j]] += v3 * v1;
      for (auto [c, v] : acc) rowsd[i].push_back({c, v, 0.0});
      nnz += (long)acc.size();
    }
    // stored entries of a sliced layout: 64 lanes times each slice's longest
    // row rounded up to a group of four
    auto padded = [](const std::vector<Row>& rows) {
      long t = 0;
      for (size_t s = 0; s < rows.size(); s += SLICE) {
        size_t w = 1;
        for (size_t l = s; l < s + SLICE && l < rows.size(); ++l) w = std::max(w, rows[l].size());
        t += SLICE * (long)((w + 3) / 4 * 4);
      }
      return t;
    };
    if (2 * padded(rowsd) <= 3 * (padded(rows1) + padded(rows3))) {
      upload_psell(ctx, rowsd, f.inv);
      f.direct = true;
    }
  }
  f.e1_row = upload(ctx, rid);
  f.e1_wave = upload(ctx, wave_list);
  // S^-1 in packs of P columns per row, [l / P][i][P], zero-padded (P = 2 in
  // FP64, 4 in FP32: one 16-byte load per pack)
  const int k = E.k;
  auto packed = [&](int P) {
    const int kp = (k + P - 1) / P;
    std::vector<double> out((size_t)std::max(1, kp * k * P), 0.0);
    for (int lp = 0; lp < kp; ++lp)
      for (int i = 0; i < k; ++i)
        for (int q = 0; q < P; ++q) {
          const int l = lp * P + q;
          if (l < k) out[((size_t)lp * k + i) * P + q] = E.Sinv[(size_t)l * k + i];
        }
    return out;
  };
  f.sinv64 = upload(ctx, packed(2));
  const std::vector<double> s4 = packed(4);
  f.sinv32 = upload(ctx, std::vector<float>(s4.begin(), s4.end()));
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

void check_factor(const SparseSym& A, const ExplicitFactor& F, const char* name) {
  // Set-up self-check: solve against a fixed right-hand side and verify the residual.
  std::vector<double> b(A.n);
  for (int i = 0; i < A.n; ++i) b[i] = 1.0 + 0.25 * std::sin(0.7 * i);
  std::vector<double> x = explicit_solve(F, b);
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
EfDev<T> EfBuffers::view() const {
  constexpr bool f64 = sizeof(T) == 8;
  EfDev<T> d;
  d.N = host.N;
  d.c = host.c;
  d.k = host.k;
  d.e1 = e1.view<T>();
  d.e1_row = e1_row.as<int>();
  d.e1_wave = e1_wave.as<int>();
  d.e1_nq = e1_nq;
  d.e3 = e3.view<T>();
  d.e3s = e3s.view<T>();
  d.e3s_row = e3s_row.as<int>();
  d.sinv = f64 ? sinv64.as<T>() : sinv32.as<T>();
  d.direct = direct ? 1 : 0;
  d.inv = direct ? inv.view<T>() : PSell<T>{nullptr, nullptr, nullptr, nullptr};
  return d;
}

template <typename T>
TxDev<T> TxNetwork::view() const {
  TxDev<T> d;
  d.n = n;
  d.nth = nth;
  d.npq = npq;
  d.m = m;
  d.kb = kb;
  d.nbp = nbp;
  d.int2ext = int2ext_d.as<int>();
  d.y64 = y.view<double2>();
  d.yT = y.view<typename Vec2<T>::type>();
  d.yt = yt.view<double2>();
  d.g = g.view<T>();
  d.gt = gt.view<double>();
  d.bp = bp.view<T>();
  d.bpp = bpp.view<T>();
  d.n_branch = n_branch;
  d.br_f = br_f.as<int>();
  d.br_t = br_t.as<int>();
  d.br_ys_re = br_ys_re.as<double>();
  d.br_ys_im = br_ys_im.as<double>();
  d.br_b = br_b.as<double>();
  return d;
}

template EfDev<double> EfBuffers::view<double>() const;
template EfDev<float> EfBuffers::view<float>() const;
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
  std::vector<int> degree(n_bus, 0);
  for (int i = 0; i < n_bus; ++i) {
    require(row_ptr[i + 1] >= row_ptr[i], "row_ptr must be non-decreasing");
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
      require(col_idx[p] >= 0 && col_idx[p] < n_bus, "column index out of range");
      if (col_idx[p] != i) ++degree[i];
    }
  }
  auto by_degree = [&](int a, int b) { return degree[a] != degree[b] ? degree[a] > degree[b] : a < b; };
  std::sort(pq.begin(), pq.end(), by_degree);
  std::sort(pv.begin(), pv.end(), by_degree);
  int blk = 0, kbs = 0;
  nr_shape(n_bus, &blk, &kbs);
  {
    // Wave w of a workgroup owns the 64-bus slices k NW + w.  Deal the full
    // 64-bus groups of PQ buses (widest rows first) to the waves in a zigzag
    // (0 .. NW-1, then NW-1 .. 0, ...), so that every wave gets a like share
    // of long rows in each sliced pass.  A last incomplete row of groups keeps
    // the plain order, and buses never leave the PQ range.
    const int nw = blk / 64, full = (int)pq.size() / 64;
    std::vector<int> dealt(pq);
    for (int g = 0; g < full; ++g) {
      const int k = g / nw, r = g % nw;
      const bool whole_row = (k + 1) * nw <= full;
      const int slice = k * nw + ((k % 2 == 1 && whole_row) ? nw - 1 - r : r);
      std::copy(pq.begin() + (size_t)g * 64, pq.begin() + (size_t)g * 64 + 64, dealt.begin() + (size_t)slice * 64);
    }
    pq.swap(dealt);
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
  net->block = blk;
  net->kb = kbs;
  net->nbp = net->block * net->kb;
  const int nbp = net->nbp, nth = net->nth, npq = net->npq;

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
  SparseSym Bp = leading_block(ptr, col, yim, nth, eps);
  SparseSym Bpp = leading_block(ptr, col, yim, npq, eps);
  if (setup.precond_block > 0) {
    Bp = block_diagonal_part(Bp, setup.precond_block);
    Bpp = block_diagonal_part(Bpp, setup.precond_block);
  }
  net->bp.host = explicit_factor(Bp, setup.factor_max_levels, setup.factor_max_core, net->block);
  check_factor(Bp, net->bp.host, "B'");
  upload_factor(ctx, net->bp, net->block, net->kb, nbp);
  if (npq > 0) {
    net->bpp.host = explicit_factor(Bpp, setup.factor_max_levels, setup.factor_max_core, net->block);
    check_factor(Bpp, net->bpp.host, "B''");
    upload_factor(ctx, net->bpp, net->block, net->kb, nbp);
  }

  // Sliced layouts by internal bus: Ybus, Ybus^T, G = -Re(Y)[Q, Theta] and G^T.
  std::vector<Row> yr(nbp), ytr(nbp), gr(nbp), gtr(nbp);
  for (int i = 0; i < n_bus; ++i)
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int j = col[p];
      yr[i].push_back({j, yre[p], yim[p]});
      ytr[j].push_back({i, yre[p], yim[p]});
      if (i < npq && j < nth) {
        gr[i].push_back({j, -yre[p], 0.0});
        gtr[j].push_back({i, -yre[p], 0.0});
      }
    }
  const auto hy = upload_psell(ctx, yr, net->y, true);
  {
    // Layout entry of each caller CSR entry: row i's p-th (sorted) internal
    // entry sits at 4 (off[i / 64] + 64 (p / 4) + i % 64) + p % 4.
    const std::vector<int>& yoff = hy.first;
    auto ypos = [&](int i, int p) {
      return 4 * ((int64_t)yoff[i / 64] + 64 * (int64_t)(p / 4) + i % 64) + p % 4;
    };
    int64_t E = 0;
    for (int w : hy.second) E += 4 * 64 * (int64_t)w;
    std::vector<std::vector<int>> src(E);
    for (int e = 0; e < n_bus; ++e) {
      const int i = net->ext2int[e];
      for (int p = row_ptr[e]; p < row_ptr[e + 1]; ++p) {
        const int j = net->ext2int[col_idx[p]];
        const int* at = std::lower_bound(col.data() + ptr[i], col.data() + ptr[i + 1], j);
        const int64_t q = ypos(i, (int)(at - (col.data() + ptr[i])));
        src[q].push_back(p);
      }
    }
    net->y_ptr = ptr;
    net->y_col = col;
    net->y_pos.assign(col.size(), 0);
    for (int i = 0; i < n_bus; ++i)
      for (int p = ptr[i]; p < ptr[i + 1]; ++p) net->y_pos[p] = (int)ypos(i, p - ptr[i]);
    std::vector<int> sp(E + 1, 0), si;
    for (int64_t q = 0; q < E; ++q) {
      si.insert(si.end(), src[q].begin(), src[q].end());
      sp[q + 1] = (int)si.size();
    }
    if (si.empty()) si.push_back(0);
    net->caller_nnz = nnz;
    net->y_entries = E;
    net->ysrc_ptr = upload(ctx, sp);
    net->ysrc_idx = upload(ctx, si);
  }
  upload_psell(ctx, ytr, net->yt, true);
  upload_psell(ctx, gr, net->g);
  upload_psell(ctx, gtr, net->gt);
  net->int2ext_d = upload(ctx, net->int2ext);

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

namespace pfx {

void ensure_direct(TxNetwork& net) {
  if (net.direct_ready) return;
  const DirectLuHost D = build_direct_lu(net);
  Context* ctx = net.ctx;
  auto up = [&](const std::vector<int>& v) { return upload(ctx, v.empty() ? std::vector<int>{0} : v); };
  net.dl_fpos = up(D.fpos);
  net.dl_soff = up(D.soff);
  net.dl_sidx = up(D.sidx);
  net.dl_fph = up(D.fph);
  net.dl_ftg = up(D.ftg.empty() ? std::vector<int>{0, 0, 0, 0} : D.ftg);
  net.dl_fct = up(D.fct.empty() ? std::vector<int>{0, 0, 0, 0} : D.fct);
  net.dl_bph = up(D.bph);
  net.dl_brow = up(D.brow);
  net.dl_je = up(D.je.empty() ? std::vector<int>{0, 0, 0, 0} : D.je);
  DirectDev& d = net.direct;
  d.m = D.m;
  d.n_s = D.n_s;
  d.n_val = D.n_val;
  d.n_je = (int)D.je.size() / 4;
  d.n_fph = (int)D.fph.size() - 1;
  d.n_bph = (int)D.bph.size() - 1;
  d.n_tg = (int)D.ftg.size() / 4;
  d.n_ct = (int)D.fct.size() / 4;
  d.fpos = net.dl_fpos.as<int>();
  d.soff = net.dl_soff.as<int>();
  d.sidx = net.dl_sidx.as<int>();
  d.fph = net.dl_fph.as<int>();
  d.ftg = net.dl_ftg.as<int4>();
  d.fct = net.dl_fct.as<int4>();
  d.bph = net.dl_bph.as<int>();
  d.brow = net.dl_brow.as<int>();
  d.je = net.dl_je.as<int4>();
  net.direct_nval = D.n_val;
  net.direct_ready = true;
}

}  // namespace pfx
