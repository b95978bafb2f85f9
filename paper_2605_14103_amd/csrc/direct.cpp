// Symbolic analysis of the direct Newton step (see direct.hpp).
#include "direct.hpp"

#include <algorithm>
#include <map>
#include <set>
#include <string>

#include "common.hpp"
#include "factor.hpp"
#include "tx.hpp"

namespace pfx {

DirectLuHost build_direct_lu(const TxNetwork& net) {
  DirectLuHost D;
  const int nth = net.nth, npq = net.npq, n = net.n, nbp = net.nbp;
  const int m = nth + npq;
  D.m = m;
  // state s: theta of bus s for s < nth, |V| of bus s - nth otherwise
  auto states_of = [&](int bus, int out[2], int type[2]) {
    int c = 0;
    if (bus < nth) {
      out[c] = bus;
      type[c++] = 0;
    }
    if (bus < npq) {
      out[c] = nth + bus;
      type[c++] = 1;
    }
    return c;
  };
  std::vector<std::set<int>> adj(m);
  for (int i = 0; i < n; ++i)
    for (int p = net.y_ptr[i]; p < net.y_ptr[i + 1]; ++p) {
      int ri[2], rt[2], ck[2], ct[2];
      const int nr = states_of(i, ri, rt), nc = states_of(net.y_col[p], ck, ct);
      for (int x = 0; x < nr; ++x)
        for (int y = 0; y < nc; ++y)
          if (ri[x] != ck[y]) {
            adj[ri[x]].insert(ck[y]);
            adj[ck[y]].insert(ri[x]);
          }
    }
  SparseSym A;
  A.n = m;
  A.ptr.assign(m + 1, 0);
  for (int s = 0; s < m; ++s) {
    A.col.insert(A.col.end(), adj[s].begin(), adj[s].end());
    A.ptr[s + 1] = (int)A.col.size();
  }
  A.val.assign(A.col.size(), 1.0);
  const std::vector<int> perm = min_degree_order(A);
  std::vector<int> pinv(m);
  for (int p = 0; p < m; ++p) pinv[perm[p]] = p;
  // Symbolic elimination in factor order: S(k) = later neighbours; they become a clique.
  std::vector<std::set<int>> g(m);
  for (int s = 0; s < m; ++s)
    for (int t : adj[s]) g[pinv[s]].insert(pinv[t]);
  D.soff.assign(m + 1, 0);
  for (int k = 0; k < m; ++k) {
    std::vector<int> S(g[k].upper_bound(k), g[k].end());
    for (size_t a = 0; a < S.size(); ++a)
      for (size_t b = a + 1; b < S.size(); ++b) {
        g[S[a]].insert(S[b]);
        g[S[b]].insert(S[a]);
      }
    D.sidx.insert(D.sidx.end(), S.begin(), S.end());
    D.soff[k + 1] = (int)D.sidx.size();
  }
  D.n_s = (int)D.sidx.size();
  D.n_val = m + 2 * D.n_s;
  if (D.n_val > DIRECT_MAX_VALUES)
    fail(PF_INVALID_ARG, "the direct Newton step holds at most " + std::to_string(DIRECT_MAX_VALUES) +
                             " factor values per scenario; this network needs " + std::to_string(D.n_val));
  auto pos = [&](int i, int j) {
    if (i == j) return i;
    const int c = std::min(i, j), r = std::max(i, j);
    const int* b = D.sidx.data() + D.soff[c];
    const int* e = D.sidx.data() + D.soff[c + 1];
    const int* at = std::lower_bound(b, e, r);
    if (at == e || *at != r) fail(PF_SINGULAR_SETUP, "entry outside the symbolic pattern of the Jacobian");
    return (i > j ? m : m + D.n_s) + D.soff[c] + (int)(at - b);
  };
  // elimination-tree levels: the parent of k is the first entry of S(k)
  std::vector<int> lf(m, 0), lb(m, 0);
  for (int k = 0; k < m; ++k)
    if (D.soff[k + 1] > D.soff[k]) lf[D.sidx[D.soff[k]]] = std::max(lf[D.sidx[D.soff[k]]], lf[k] + 1);
  for (int k = m - 1; k >= 0; --k)
    for (int q = D.soff[k]; q < D.soff[k + 1]; ++q) lb[k] = std::max(lb[k], lb[D.sidx[q]] + 1);
  const int nf = m ? *std::max_element(lf.begin(), lf.end()) + 1 : 0;
  const int nb = m ? *std::max_element(lb.begin(), lb.end()) + 1 : 0;
  std::vector<std::vector<int>> by_f(nf), by_b(nb);
  for (int k = 0; k < m; ++k) {
    by_f[lf[k]].push_back(k);
    by_b[lb[k]].push_back(k);
  }
  D.fph.assign(1, 0);
  for (int f = 0; f < nf; ++f) {
    // key: value index for matrix targets, -1 - row for right-hand-side targets
    std::map<int, std::vector<int>> contrib;
    for (int k : by_f[f]) {
      const int s0 = D.soff[k], cnt = D.soff[k + 1] - s0;
      for (int x = 0; x < cnt; ++x) {
        for (int y = 0; y < cnt; ++y) {
          auto& c = contrib[pos(D.sidx[s0 + x], D.sidx[s0 + y])];
          c.insert(c.end(), {m + s0 + x, m + D.n_s + s0 + y, k, 0});
        }
        auto& c = contrib[-1 - D.sidx[s0 + x]];
        c.insert(c.end(), {m + s0 + x, k, k, 0});
      }
    }
    for (auto& [key, c] : contrib) {
      const int first = (int)D.fct.size() / 4;
      D.fct.insert(D.fct.end(), c.begin(), c.end());
      D.ftg.insert(D.ftg.end(), {key >= 0 ? key : -1 - key, first, (int)D.fct.size() / 4, key >= 0 ? 0 : 1});
    }
    D.fph.push_back((int)D.ftg.size() / 4);
  }
  D.bph.assign(1, 0);
  for (int l = 0; l < nb; ++l) {
    D.brow.insert(D.brow.end(), by_b[l].begin(), by_b[l].end());
    D.bph.push_back((int)D.brow.size());
  }
  D.fpos.assign(2 * nbp, -1);
  for (int s = 0; s < m; ++s) D.fpos[s < nth ? s : nbp + (s - nth)] = pinv[s];
  for (int i = 0; i < n; ++i)
    for (int p = net.y_ptr[i]; p < net.y_ptr[i + 1]; ++p) {
      const int k = net.y_col[p];
      int ri[2], rt[2], ck[2], ct[2];
      const int nr = states_of(i, ri, rt), nc = states_of(k, ck, ct);
      for (int x = 0; x < nr; ++x)
        for (int y = 0; y < nc; ++y) {
          const int kind = 2 * rt[x] + ct[y];
          D.je.insert(D.je.end(), {pos(pinv[ri[x]], pinv[ck[y]]) | (kind << 28), i, k, net.y_pos[p]});
        }
    }
  return D;
}

}  // namespace pfx
