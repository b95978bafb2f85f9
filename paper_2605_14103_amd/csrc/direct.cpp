// Symbolic analysis of the direct Newton step (see direct.hpp).
#include "direct.hpp"

#include <algorithm>
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
  D.uoff.assign(m + 1, 0);
  for (int k = 0; k < m; ++k) {
    for (int q = D.soff[k]; q < D.soff[k + 1]; ++q)
      for (int r = D.soff[k]; r < D.soff[k + 1]; ++r) D.upd.push_back(pos(D.sidx[q], D.sidx[r]));
    D.uoff[k + 1] = (int)D.upd.size();
  }
  std::vector<std::vector<int>> uc(m);
  for (int i = 0; i < m; ++i)
    for (int q = D.soff[i]; q < D.soff[i + 1]; ++q) uc[D.sidx[q]].push_back(i);
  D.ucp.assign(m + 1, 0);
  for (int k = 0; k < m; ++k) {
    for (int i : uc[k]) {
      D.ucol.push_back(i);
      D.ucol.push_back(pos(i, k));
    }
    D.ucp[k + 1] = (int)D.ucol.size() / 2;
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
