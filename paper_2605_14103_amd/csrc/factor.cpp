#include "factor.hpp"

#include <algorithm>
#include <cmath>
#include <queue>
#include <set>
#include <string>

#include "common.hpp"

namespace pfx {

std::vector<int> min_degree_order(const SparseSym& A) {
  const int n = A.n;
  std::vector<std::set<int>> adj(n);
  for (int i = 0; i < n; ++i)
    for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
      if (A.col[p] != i) adj[i].insert(A.col[p]);
  std::vector<char> alive(n, 1);
  using Item = std::pair<int, int>;  // (degree, node): smallest degree, then lowest index
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
  for (int i = 0; i < n; ++i) pq.push({(int)adj[i].size(), i});
  std::vector<int> order;
  order.reserve(n);
  while (!pq.empty()) {
    auto [d, v] = pq.top();
    pq.pop();
    if (!alive[v] || d != (int)adj[v].size()) continue;
    alive[v] = 0;
    order.push_back(v);
    std::vector<int> nb(adj[v].begin(), adj[v].end());
    for (int u : nb) {
      adj[u].erase(v);
      for (int w : nb)
        if (w != u) adj[u].insert(w);
    }
    for (int u : nb) pq.push({(int)adj[u].size(), u});
    adj[v].clear();
  }
  return order;
}

SparseSym block_diagonal_part(const SparseSym& A, int block) {
  const int n = A.n;
  std::vector<int> pos(n, -1);
  int next = 0;
  for (int s = 0; s < n; ++s) {  // breadth-first over every component
    if (pos[s] >= 0) continue;
    std::vector<int> queue{s};
    pos[s] = next++;
    for (size_t q = 0; q < queue.size(); ++q) {
      int u = queue[q];
      for (int p = A.ptr[u]; p < A.ptr[u + 1]; ++p) {
        int w = A.col[p];
        if (pos[w] < 0) {
          pos[w] = next++;
          queue.push_back(w);
        }
      }
    }
  }
  SparseSym B;
  B.n = n;
  B.ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int j = A.col[p];
      if (pos[i] / block == pos[j] / block) {
        B.col.push_back(j);
        B.val.push_back(A.val[p]);
      }
    }
    B.ptr[i + 1] = (int)B.col.size();
  }
  return B;
}

HybridFactor hybrid_factor(const SparseSym& A0, int max_levels, int max_core) {
  const int N = A0.n;
  HybridFactor F;
  F.N = N;
  F.perm = min_degree_order(A0);
  F.pinv.assign(N, 0);
  for (int p = 0; p < N; ++p) F.pinv[F.perm[p]] = p;

  // Permuted matrix P A P^T, lower triangle by column.
  std::vector<std::vector<std::pair<int, double>>> acol(N);
  double amax = 0.0;
  for (int i = 0; i < N; ++i)
    for (int p = A0.ptr[i]; p < A0.ptr[i + 1]; ++p) {
      int pi = F.pinv[i], pj = F.pinv[A0.col[p]];
      amax = std::max(amax, std::fabs(A0.val[p]));
      if (pi >= pj) acol[pj].push_back({pi, A0.val[p]});
    }

  // Symbolic elimination: column patterns (rows > j) and row lists.
  std::vector<std::vector<int>> colr(N);
  std::vector<std::vector<std::pair<int, int>>> rowlist(N);  // (column k, index of row in colr[k])
  std::vector<int> mark(N, -1), pattern;
  for (int j = 0; j < N; ++j) {
    pattern.clear();
    for (auto [i, a] : acol[j])
      if (i != j && mark[i] != j) {
        mark[i] = j;
        pattern.push_back(i);
      }
    for (auto [k, idx] : rowlist[j])
      for (size_t q = idx + 1; q < colr[k].size(); ++q) {
        int i = colr[k][q];
        if (mark[i] != j) {
          mark[i] = j;
          pattern.push_back(i);
        }
      }
    std::sort(pattern.begin(), pattern.end());
    colr[j] = pattern;
    for (size_t q = 0; q < pattern.size(); ++q) rowlist[pattern[q]].push_back({j, (int)q});
  }
  int fnnz = N;
  for (int j = 0; j < N; ++j) fnnz += (int)colr[j].size();
  F.factor_nnz = fnnz;

  // Dependency levels and the prefix length.
  std::vector<int> lev(N, 0);
  for (int i = 0; i < N; ++i)
    for (auto [k, idx] : rowlist[i]) lev[i] = std::max(lev[i], lev[k] + 1);
  int c = 0, run_max = -1;
  for (int i = 0; i < N; ++i) {
    run_max = std::max(run_max, lev[i]);
    if (run_max + 1 <= max_levels) c = i + 1;
    else break;
  }
  if (N - c > max_core) c = N - max_core;
  if (c < 0) c = 0;
  F.c = c;
  F.k = N - c;
  const int k = F.k;

  // Numeric left-looking L D L^T over the prefix columns (unit lower L).
  std::vector<std::vector<double>> colv(c);
  std::vector<double> D(c);
  std::vector<double> w(N, 0.0);
  for (int j = 0; j < c; ++j) {
    double wjj = 0.0;
    for (int i : colr[j]) w[i] = 0.0;
    for (auto [i, a] : acol[j]) {
      if (i == j) wjj += a;
      else w[i] += a;
    }
    for (auto [kk, idx] : rowlist[j]) {
      const double ljk = colv[kk][idx], dk = D[kk];
      wjj -= ljk * ljk * dk;
      for (size_t q = idx + 1; q < colr[kk].size(); ++q) w[colr[kk][q]] -= colv[kk][q] * ljk * dk;
    }
    if (!(std::fabs(wjj) > 1e-13 * std::max(amax, 1e-300)) || !std::isfinite(wjj))
      fail(PF_SINGULAR_SETUP, "zero pivot at position " + std::to_string(j));
    D[j] = wjj;
    colv[j].resize(colr[j].size());
    for (size_t q = 0; q < colr[j].size(); ++q) colv[j][q] = w[colr[j][q]] / wjj;
  }

  // Forward level lists over the prefix.
  int nfl = 0;
  for (int i = 0; i < c; ++i) nfl = std::max(nfl, lev[i] + 1);
  F.f_lev.assign(nfl + 1, 0);
  for (int i = 0; i < c; ++i) F.f_lev[lev[i] + 1]++;
  for (int l = 0; l < nfl; ++l) F.f_lev[l + 1] += F.f_lev[l];
  F.f_rows.assign(c, 0);
  {
    std::vector<int> fill(F.f_lev.begin(), F.f_lev.end() - 1);
    for (int i = 0; i < c; ++i) F.f_rows[fill[lev[i]]++] = i;
  }
  // Rows of L restricted to prefix columns, for all N positions.
  F.L_ptr.assign(N + 1, 0);
  for (int i = 0; i < N; ++i) {
    for (auto [kk, idx] : rowlist[i])
      if (kk < c) {
        F.L_col.push_back(kk);
        F.L_val.push_back(colv[kk][idx]);
      }
    F.L_ptr[i + 1] = (int)F.L_col.size();
  }
  F.dinv.resize(c);
  for (int j = 0; j < c; ++j) F.dinv[j] = 1.0 / D[j];

  // Backward levels over the prefix.
  std::vector<int> blev(c, 0);
  for (int j = c - 1; j >= 0; --j)
    for (int i : colr[j])
      if (i < c) blev[j] = std::max(blev[j], blev[i] + 1);
  int nbl = 0;
  for (int j = 0; j < c; ++j) nbl = std::max(nbl, blev[j] + 1);
  F.b_lev.assign(nbl + 1, 0);
  for (int j = 0; j < c; ++j) F.b_lev[blev[j] + 1]++;
  for (int l = 0; l < nbl; ++l) F.b_lev[l + 1] += F.b_lev[l];
  F.b_rows.assign(c, 0);
  {
    std::vector<int> fill(F.b_lev.begin(), F.b_lev.end() - 1);
    for (int j = 0; j < c; ++j) F.b_rows[fill[blev[j]]++] = j;
  }
  F.T_ptr.assign(c + 1, 0);
  for (int j = 0; j < c; ++j) {
    for (size_t q = 0; q < colr[j].size(); ++q) {
      F.T_col.push_back(colr[j][q]);
      F.T_val.push_back(colv[j][q]);
    }
    F.T_ptr[j + 1] = (int)F.T_col.size();
  }

  // Dense core: S = A22 - L21 D11 L21^T, kept as S^-1 (Gauss-Jordan with partial pivoting).
  if (k > 0) {
    std::vector<double> S((size_t)k * k, 0.0);
    for (int j = c; j < N; ++j)
      for (auto [i, a] : acol[j]) {
        S[(size_t)(i - c) * k + (j - c)] += a;
        if (i != j) S[(size_t)(j - c) * k + (i - c)] += a;
      }
    for (int kk = 0; kk < c; ++kk) {
      const auto& rr = colr[kk];
      const auto& vv = colv[kk];
      size_t q0 = std::lower_bound(rr.begin(), rr.end(), c) - rr.begin();
      for (size_t a = q0; a < rr.size(); ++a)
        for (size_t b = q0; b < rr.size(); ++b)
          S[(size_t)(rr[a] - c) * k + (rr[b] - c)] -= vv[a] * D[kk] * vv[b];
    }
    std::vector<double> Inv((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) Inv[(size_t)i * k + i] = 1.0;
    double smax = 0.0;
    for (double v : S) smax = std::max(smax, std::fabs(v));
    for (int col = 0; col < k; ++col) {
      int p = col;
      for (int i = col + 1; i < k; ++i)
        if (std::fabs(S[(size_t)i * k + col]) > std::fabs(S[(size_t)p * k + col])) p = i;
      if (!(std::fabs(S[(size_t)p * k + col]) > 1e-14 * std::max(smax, 1e-300)))
        fail(PF_SINGULAR_SETUP, "singular dense core at column " + std::to_string(col));
      if (p != col)
        for (int q = 0; q < k; ++q) {
          std::swap(S[(size_t)p * k + q], S[(size_t)col * k + q]);
          std::swap(Inv[(size_t)p * k + q], Inv[(size_t)col * k + q]);
        }
      const double piv = 1.0 / S[(size_t)col * k + col];
      for (int q = 0; q < k; ++q) {
        S[(size_t)col * k + q] *= piv;
        Inv[(size_t)col * k + q] *= piv;
      }
      for (int i = 0; i < k; ++i) {
        if (i == col) continue;
        const double f = S[(size_t)i * k + col];
        if (f == 0.0) continue;
        for (int q = 0; q < k; ++q) {
          S[(size_t)i * k + q] -= f * S[(size_t)col * k + q];
          Inv[(size_t)i * k + q] -= f * Inv[(size_t)col * k + q];
        }
      }
    }
    F.Sinv.assign((size_t)k * k, 0.0);
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b)
        F.Sinv[(size_t)a * k + b] = 0.5 * (Inv[(size_t)a * k + b] + Inv[(size_t)b * k + a]);
  }
  return F;
}

std::vector<double> hybrid_solve(const HybridFactor& F, const std::vector<double>& b) {
  std::vector<double> x(F.N);
  for (int r = 0; r < F.N; ++r) x[F.pinv[r]] = b[r];
  for (int l = 0; l + 1 < (int)F.f_lev.size(); ++l)
    for (int q = F.f_lev[l]; q < F.f_lev[l + 1]; ++q) {
      int i = F.f_rows[q];
      double a = x[i];
      for (int p = F.L_ptr[i]; p < F.L_ptr[i + 1]; ++p) a -= F.L_val[p] * x[F.L_col[p]];
      x[i] = a;
    }
  std::vector<double> t(F.k);
  for (int i = F.c; i < F.N; ++i) {
    double a = x[i];
    for (int p = F.L_ptr[i]; p < F.L_ptr[i + 1]; ++p) a -= F.L_val[p] * x[F.L_col[p]];
    t[i - F.c] = a;
  }
  for (int i = 0; i < F.k; ++i) {
    double a = 0.0;
    for (int l = 0; l < F.k; ++l) a += F.Sinv[(size_t)l * F.k + i] * t[l];
    x[F.c + i] = a;
  }
  for (int j = 0; j < F.c; ++j) x[j] *= F.dinv[j];
  for (int l = 0; l + 1 < (int)F.b_lev.size(); ++l)
    for (int q = F.b_lev[l]; q < F.b_lev[l + 1]; ++q) {
      int j = F.b_rows[q];
      double a = x[j];
      for (int p = F.T_ptr[j]; p < F.T_ptr[j + 1]; ++p) a -= F.T_val[p] * x[F.T_col[p]];
      x[j] = a;
    }
  std::vector<double> out(F.N);
  for (int r = 0; r < F.N; ++r) out[r] = x[F.pinv[r]];
  return out;
}

}  // namespace pfx

namespace pfx {

long ExplicitFactor::entries() const {
  long e = 0;
  for (const auto& r : e1) e += (long)r.size();
  for (const auto& r : e3) e += (long)r.size();
  return e;
}

ExplicitFactor explicit_form(const HybridFactor& F) {
  const int N = F.N, c = F.c, k = F.k;
  ExplicitFactor E;
  E.N = N;
  E.c = c;
  E.k = k;
  E.perm = F.perm;
  E.pinv = F.pinv;
  E.Sinv = F.Sinv;
  // Column lists of L over prefix columns: lc[j] = rows i > j with L[i][j] != 0.
  std::vector<std::vector<std::pair<int, double>>> lc(c);
  for (int i = 0; i < N; ++i)
    for (int p = F.L_ptr[i]; p < F.L_ptr[i + 1]; ++p) lc[F.L_col[p]].push_back({i, F.L_val[p]});
  E.e1.assign(N, {});
  E.e3.assign(N, {});
  std::vector<int> mark(N, -1);
  std::vector<double> y(N, 0.0);
  std::vector<int> reach;
  for (int j = 0; j < c; ++j) {
    // nonzero pattern of L^-1 e_j: positions reachable from j through L
    reach.clear();
    reach.push_back(j);
    mark[j] = j;
    for (size_t q = 0; q < reach.size(); ++q) {
      const int u = reach[q];
      if (u >= c) continue;
      for (auto [v, l] : lc[u])
        if (mark[v] != j) {
          mark[v] = j;
          reach.push_back(v);
        }
    }
    std::sort(reach.begin(), reach.end());
    // forward substitution in increasing position order (L is lower triangular)
    y[j] = 1.0;
    for (int u : reach) {
      if (u == j) continue;
      double a = 0.0;
      for (int p = F.L_ptr[u]; p < F.L_ptr[u + 1]; ++p) a -= F.L_val[p] * y[F.L_col[p]];
      y[u] = a;
    }
    for (int u : reach) {
      if (y[u] != 0.0) {
        E.e3[j].push_back({u, y[u]});                                  // column j of L^-1
        E.e1[u].push_back({j, u < c ? F.dinv[u] * y[u] : y[u]});       // row u of Dt'^-1 L^-1
      }
    }
    for (int u : reach) y[u] = 0.0;   // positions outside the next reach must read as zero
  }
  for (int r = c; r < N; ++r) {
    E.e1[r].push_back({r, 1.0});
    E.e3[r].push_back({r, 1.0});
  }
  for (auto& r : E.e1) std::sort(r.begin(), r.end());
  return E;
}

std::vector<double> explicit_solve(const ExplicitFactor& E, const std::vector<double>& b) {
  const int N = E.N, c = E.c, k = E.k;
  std::vector<double> bf(N), u(N), x(N);
  for (int r = 0; r < N; ++r) bf[E.pinv[r]] = b[r];
  for (int r = 0; r < N; ++r) {
    double a = 0.0;
    for (auto [j, v] : E.e1[r]) a += v * bf[j];
    u[r] = a;
  }
  for (int i = 0; i < k; ++i) {
    double a = 0.0;
    for (int l = 0; l < k; ++l) a += E.Sinv[(size_t)l * k + i] * u[c + l];
    x[c + i] = a;
  }
  for (int r = 0; r < c; ++r) x[r] = u[r];
  std::vector<double> out(N);
  for (int p = 0; p < N; ++p) {
    double a = 0.0;
    for (auto [j, v] : E.e3[p]) a += v * x[j];
    out[E.perm[p]] = a;
  }
  return out;
}

ExplicitFactor explicit_factor(const SparseSym& A, int max_levels, int max_core, int block) {
  ExplicitFactor best;
  double best_cost = -1.0;
  std::string last_error;
  for (int lv = 1; lv <= std::max(1, max_levels); ++lv) {
    HybridFactor F;
    try {
      F = hybrid_factor(A, lv, max_core);
    } catch (const PfError& e) {
      last_error = e.what();
      continue;
    }
    ExplicitFactor E = explicit_form(F);
    // Sparse entries padded to slices of 64 rows sorted by length, as laid out on the device.
    auto padded = [](const std::vector<std::vector<std::pair<int, double>>>& rows) {
      std::vector<int> len;
      for (const auto& r : rows) len.push_back((int)r.size());
      std::sort(len.begin(), len.end(), std::greater<int>());
      long pad = 0;
      for (size_t s = 0; s < len.size(); s += 64) pad += 64L * len[s];
      return pad;
    };
    const double cost = (double)(padded(E.e1) + padded(E.e3)) / block + (double)E.k * E.k / std::max(1, std::min(E.k, block));
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = std::move(E);
    }
    if (F.n_fwd_levels() < lv) break;   // more levels would not change the split
  }
  if (best_cost < 0) fail(PF_SINGULAR_SETUP, last_error.empty() ? "factorisation failed" : last_error);
  return best;
}

}  // namespace pfx
