// Transmission network: host-side record and the plain device views the
// Newton-Raphson, branch-loss and adjoint kernels take by value.
//
// Internal bus order.  Buses are renumbered so that PQ buses come first, then
// PV buses, then the slack (each group by decreasing degree, so that rows of
// similar length share a slice; the full 64-bus groups of PQ buses are dealt
// to the waves of a workgroup in a zigzag so that each wave gets a like share
// of long rows).  With n buses, nth = n - 1 and npq PQ buses,
// Theta is internal buses 0..nth-1 and Q is 0..npq-1.  The kernels hold the
// Newton state x = [theta over Theta ; |V| over Q] (eq. (1)) bus-major: two
// planes of nbp (padded bus count) entries, angle of bus i at i and magnitude
// of bus i at nbp + i, zero where a bus carries no such state.  A thread owns
// buses t + k block (k < kb) and both of their entries.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"
#include "factor.hpp"
#include "sell.hpp"

namespace pfx {

// Device view of one explicit factor (factor.hpp, ExplicitFactor) laid out for
// one workgroup of `block` threads.
//   E1: rows sorted by length into slices; slice lists per wave (at most kb
//       slices each, resolved to entry offset and width), row ids per lane
//       (factor position, -1 for none); input
//       columns are positions of the matrix order (the permutation is folded in).
//   E3: one row per matrix row i (bus order), slices = consecutive 64 rows;
//       columns are factor positions.
template <typename T>
struct EfDev {
  int N, c, k;
  PSell<T> e1;
  const int* e1_row;     // [n_slices * 64]
  const int* e1_wave;    // [n_waves * e1_nq][4]: group offset, width in groups, first row id index, 0
  int e1_nq;             // entries per wave in e1_wave
  PSell<T> e3;
  // The same E3 rows sorted by length into slices dealt to (slot, wave)
  // positions k NW + w with balanced rounds; e3s_row[slice * 64 + lane] is
  // the row's matrix row (-1 for padding).  Used where the result goes to LDS.
  PSell<T> e3s;
  const int* e3s_row;
  const T* sinv;         // S^-1 (k x k) in packs [l / P][i][P], P = 16 / sizeof(T)
  // With no dense core the inverse itself may be sparse enough to apply in one
  // pass: then `direct` is 1 and `inv` holds A^-1 by rows in bus order, with
  // columns in matrix order (E1, E2 and E3 are not used).
  int direct;
  PSell<T> inv;
};

template <typename T>
struct TxDev {
  int n, nth, npq, m;
  int kb;                // bus slots per thread
  int nbp;               // padded bus count, kb * block
  const int* int2ext;    // internal bus -> caller's bus index
  PSell<double2> y64;    // Ybus rows by internal bus (FP64 values)
  PSell<typename Vec2<T>::type> yT;   // the same entries in T (Jacobian-vector products)
  PSell<double2> yt;     // Ybus^T rows (adjoint)
  PSell<T> g;            // G = -Re(Ybus)[Q, Theta]: rows PQ buses, columns Theta buses
  PSell<double> gt;      // G^T: rows Theta buses, columns PQ buses (adjoint)
  EfDev<T> bp;           // (B' + eps I)^-1 over Theta
  EfDev<T> bpp;          // (B'' + eps I)^-1 over Q
  // branch list (internal bus numbers) for the branch-current loss
  int n_branch;
  const int* br_f;
  const int* br_t;
  const double* br_ys_re;
  const double* br_ys_im;
  const double* br_b;
};

// Device view of the direct Newton step's shared analysis (direct.hpp).
struct DirectDev {
  int m, n_s, n_val, n_je, n_fph, n_bph, n_tg, n_ct;
  const int* fpos;   // [2 nbp]
  const int* soff;   // [m + 1]
  const int* sidx;
  const int* fph;    // [n_fph + 1]
  const int4* ftg;   // (target, first contribution, end, 1 for a right-hand-side target)
  const int4* fct;   // (L entry, U entry or right-hand-side index, pivot, 0)
  const int* bph;    // [n_bph + 1]
  const int* brow;
  const int4* je;    // (value index | kind << 28, bus i, bus k, Ybus layout index)
};

struct EfBuffers {
  ExplicitFactor host;
  bool direct = false;
  PSellBuffers inv;
  PSellBuffers e1, e3, e3s;
  DeviceBuffer e1_row, e1_wave, e3s_row, sinv64, sinv32;
  int e1_nq = 0;
  template <typename T>
  EfDev<T> view() const;
};

struct TxNetwork {
  Context* ctx = nullptr;
  int n = 0, nth = 0, npq = 0, m = 0, nnz = 0, n_branch = 0;
  int block = 0, kb = 0, nbp = 0;   // workgroup shape of the solve kernels
  std::vector<int> int2ext, ext2int;
  pf_opts setup{};
  DeviceBuffer int2ext_d;
  PSellBuffers y, yt;   // values are complex (re, im pairs)
  PSellBuffers g, gt;
  EfBuffers bp, bpp;
  DeviceBuffer br_f, br_t, br_ys_re, br_ys_im, br_b;
  DeviceBuffer inc_ptr, inc_br;   // branches incident to each internal bus
  // Caller CSR entries that sum into each entry of the y64 layout (for
  // per-scenario values): entries src_idx[src_ptr[q] .. src_ptr[q + 1]) of
  // the caller's CSR make layout entry q (none for padding).
  int caller_nnz = 0;
  int64_t y_entries = 0;
  DeviceBuffer ysrc_ptr, ysrc_idx;
  // internal Ybus pattern (rows by internal bus, sorted columns) and the
  // layout entry of each internal entry
  std::vector<int> y_ptr, y_col, y_pos;
  // direct Newton step: analysis built on first use
  bool direct_ready = false;
  int direct_nval = 0;
  DirectDev direct{};
  DeviceBuffer dl_fpos, dl_soff, dl_sidx, dl_fph, dl_ftg, dl_fct, dl_bph, dl_brow, dl_je;
  // solve workspaces (grow-only), shared by the network's calls and ordered by `order`
  DeviceBuffer ws_d, ws_basis, ws_adj, ws_y, ws_dval;
  CallOrder order;
  // the device views themselves, resident in device memory so kernels take one pointer
  DeviceBuffer desc64, desc32;
  template <typename T>
  TxDev<T> view() const;
  template <typename T>
  const TxDev<T>* desc() const {
    return sizeof(T) == 8 ? desc64.as<const TxDev<T>>() : desc32.as<const TxDev<T>>();
  }
};

// Workgroup shape for a network of n buses: block threads, kb bus slots per
// thread (n <= kb * block).
void nr_shape(int n, int* block, int* kb);

// Resumable per-scenario Newton state of the serving engine's step launches:
// phase 0 = not started (the next launch begins from the flat start),
// 1 = between launches (the workspace holds the last iterate, its mismatch F
// and the V and I planes that mismatch formed; fnorm is max |F|, already
// tested), 2 = finished (outputs written).
struct NrSlotState {
  int32_t phase, newton, gtotal, pad;
  double fnorm, work, fprev, eta;
};

// Launchers (nr_kernels.hip).
struct NRLaunch {
  int batch;
  int64_t ld;
  const double* p_inj;
  const double* q_inj;
  const double* vm_set;
  double* v_out;
  int32_t* newton_iters;
  int32_t* gmres_iters;
  uint8_t* converged;
  double* final_mismatch;
  double* work_bytes;
  double tol, diverge, rtol;
  int max_newton, restart, max_restarts;
  // adaptive forcing term (1) or rtol for every Newton step (0); see pf_opts
  int forcing;
  double forcing_max;
  double* ws_d;
  int64_t ws_d_stride;
  void* ws_basis;
  int64_t ws_b_stride;
  // Per-scenario Ybus values in the layout of TxDev::y64 (yv_stride entries
  // per scenario): FP64 for the mismatch and, for an FP32 inner solve, an FP32
  // copy for the Jacobian-vector products (yvT == yv64 in FP64).  Null: the
  // network's own values for every scenario.
  const double2* yv64;
  const void* yvT;
  int64_t yv_stride;
  double yv_nnz;  // entries counted by the byte model (0 with shared values)
  // Scenario of each workgroup: slots[g] (null: scenario g).  Every
  // per-scenario array above is indexed by that scenario.
  const int32_t* slots;
  // Step launches (null: one whole solve per launch): each workgroup resumes
  // its scenario from state[], runs at most step_iters Newton updates and
  // sets step_done[g] to 1 when the scenario finished (outputs written) or
  // to 0 when it saved its state for a later launch.
  NrSlotState* state;
  int step_iters;
  uint8_t* step_done;
  // Direct Newton step whose factor does not fit LDS: each scenario's factor
  // values at ws_dval + b * ws_dval_stride (device memory).
  double* ws_dval;
  int64_t ws_dval_stride;
};

// Gather per-scenario Ybus values given in the caller's CSR entry order
// (complex [batch][ldy]) into the y64 layout, in FP64 and (yv32 not null) FP32;
// padding entries are written as zero.
void launch_y_gather(const TxNetwork& net, int batch, int64_t ldy, const double* y_vals, double2* yv64,
                     float2* yv32, hipStream_t s);

// Doubles of per-scenario FP64 workspace the NR kernel needs, and the padded
// state length (2 nbp: an angle plane and a magnitude plane) of its vectors.
int64_t nr_ws_doubles(const TxNetwork& net);
int64_t nr_padded_rows(const TxNetwork& net);
void launch_nr(const TxNetwork& net, bool mixed, const NRLaunch& a, hipStream_t s);
// Direct Newton step (FP64), after ensure_direct(net).  direct_lds_fits:
// whether the factor values fit the kernel's LDS (otherwise the launch needs
// a.ws_dval with net.direct_nval doubles per scenario).
void ensure_direct(TxNetwork& net);
bool direct_lds_fits(const TxNetwork& net);
void launch_nr_direct(const TxNetwork& net, const NRLaunch& a, hipStream_t s);

struct LossLaunch {
  int batch;
  int64_t ld;
  const double* v;
  double* loss;
  double* dl_dv;
};
void launch_branch_loss(const TxNetwork& net, const LossLaunch& a, hipStream_t s);

struct AdjLaunch {
  int batch;
  int64_t ld;
  const double* v;
  const double* dl_dv;
  double* grad_p;
  double* grad_q;
  int32_t* gmres_iters;
  uint8_t* converged;
  double rtol;
  int restart, max_restarts;
  double* ws_d;
  int64_t ws_d_stride;
  double* ws_basis;
  int64_t ws_b_stride;
};
int64_t adj_ws_doubles(const TxNetwork& net);
void launch_adjoint(const TxNetwork& net, const AdjLaunch& a, hipStream_t s);

TxNetwork* tx_network_create(Context* ctx, int n_bus, int nnz, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* y_re, const double* y_im,
                             const int8_t* bus_type, int n_branch, const int32_t* br_f,
                             const int32_t* br_t, const double* br_r, const double* br_x,
                             const double* br_b, const pf_opts& setup);

}  // namespace pfx
