// Shared symbolic analysis for the direct Newton step: the pattern of the
// polar Jacobian of eq. (4) (states theta over Theta, |V| over Q), a
// minimum-degree order of it, its fill under LU without pivoting and the
// static schedule of the numeric factorisation, which then runs per scenario
// (the batched sparse direct solve the paper points to as an outlook, Sec. IV).
//
// J is structurally symmetric (J[a][b] is nonzero where the buses of states a
// and b are equal or joined by a branch), so L and U share one pattern: for
// pivot k, S(k) lists the later positions i with L[i][k] != 0, which are also
// the later positions j with U[k][j] != 0.  Values of one scenario's factor
// are stored as [diagonal U[k][k] (m) | L columns by pivot, unscaled
// (L[i][k] U[k][k]) | U rows by pivot].
#pragma once

#include <vector>

namespace pfx {

struct TxNetwork;

struct DirectLuHost {
  int m = 0, n_s = 0, n_val = 0;
  std::vector<int> fpos;     // [2 nbp]: factor position of theta_i (i) and |V|_i (nbp + i), -1 if none
  std::vector<int> soff;     // [m + 1]: S(k) = sidx[soff[k] .. soff[k + 1])
  std::vector<int> sidx;
  // Factorisation (with the forward solve) by levels of the elimination
  // tree: pivots of one level are never ancestor and descendant, so none
  // changes another's row, column or right-hand-side entry.  Phase f lists
  // its targets ftg[fph[f] .. fph[f + 1]) (4 ints: value or right-hand-side
  // index, first and end contribution, 1 for a right-hand-side target); a
  // target takes all its contributions of the phase, in pivot order, from
  // fct (4 ints: L entry, U entry or right-hand-side index of the pivot, the
  // pivot, 0): target -= L[i][k] x / U[k][k].
  std::vector<int> fph, ftg, fct;
  // Backward solve by levels: phase b computes x_k for the rows
  // brow[bph[b] .. bph[b + 1]), whose U entries reference solved rows only.
  std::vector<int> bph, brow;
  std::vector<int> je;       // J entries, 4 ints each: (value index | kind << 28, bus i, bus k, Ybus layout index)
};

// Factor values per scenario beyond which the direct step is refused (the
// factor lives in LDS when it fits there, else in network-owned device
// memory, DIRECT_MAX_VALUES doubles per scenario of a batch).
constexpr int DIRECT_MAX_VALUES = 1 << 22;

// Builds the analysis for a registered network.  Throws PfError
// (PF_INVALID_ARG) when the factor would exceed DIRECT_MAX_VALUES values.
DirectLuHost build_direct_lu(const TxNetwork& net);

}  // namespace pfx
