// Three-phase radial feeder for the Z-bus fixed point (Sec. II-B, eq. (10)).
//
// Free nodes (all phase nodes except the three slack phases) are numbered
// 0..nN-1 in the caller's order.  Per-scenario state is scenario-major with a
// padded row of Kp reals: node i's complex value is at [2i], [2i+1].  The
// product delta = Z r is a real GEMM D = R W over those rows, with W the
// real-block form of Z:
//   W[2l][2i] = Re Z[i][l],  W[2l+1][2i] = -Im Z[i][l],
//   W[2l][2i+1] = Im Z[i][l], W[2l+1][2i+1] = Re Z[i][l],
// zero-padded to Kp x Np (Kp = 2 nN rounded up to the GEMM's K step, Np to
// its N tile).
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"
#include "sell.hpp"

namespace pfx {

// Free nodes are also grouped in slices of 64 (one wavefront) for the
// residual kernel: nNs = nN rounded up to 64, and a thread of the residual's
// workgroup owns nodes t + k * ZB_THREADS.
struct DistDev {
  int nN, nNs, Kp, Np;
  Sell<double2> y;         // Y_NN over free nodes (nNs rows, widths multiples of 4)
  const int4* node;        // [nNs] x: caller's index | (wye load ? 1 << 30 : 0),
                           //       y: next phase of a delta bus (-1 if none),
                           //       z: previous phase, w: caller's index of z
  const double2* c;        // [nNs] Y_NS v_S (zero past nN)
  const double* v0;        // no-load voltage, complex interleaved [nN]
  const int* free2ext;     // free node -> caller's node index
  // Sparse L D L^T of Y_NN (zfactor.hpp) for the sparse variant; free node
  // i sits at factor position pinv[i].  Each solve is a list of slices of
  // 64 rows (one row per lane), level after level: slice q holds row ids
  // row[64 q + lane] (-1 for padding) and entries (value, column) at
  // meta[q].x + 64 e + lane for e < meta[q].y (a multiple of 4, at least 4,
  // padding zero); meta[q].z is 1 on the last slice of a level.  The
  // backward slices also hold each row's 1 / D.  Values complex, in FP64
  // and FP32.
  int zf_nfq, zf_nbq;          // forward / backward slice counts
  const int* zf_pinv;          // [nN]
  const int4* zf_fmeta;
  const int* zf_frow;
  const int* zf_fcol;
  const int4* zf_bmeta;
  const int* zf_brow;
  const int* zf_bcol;
  const double2* zf_fval64;
  const double2* zf_bval64;
  const double2* zf_bd64;      // [64 x backward slices]
  const float2* zf_fval32;
  const float2* zf_bval32;
  const float2* zf_bd32;
};

struct DistNetwork {
  Context* ctx = nullptr;
  int n_node = 0, nN = 0, nnz = 0, Kp = 0, Np = 0, n_wye = 0, n_delta = 0;
  int slack[3] = {0, 1, 2};
  double v_slack[6] = {0, 0, 0, 0, 0, 0};
  std::vector<int> free2ext;
  SellBuffers y;
  DeviceBuffer node, c, v0, free2ext_d;
  int zf_nfq = 0, zf_nbq = 0;
  DeviceBuffer zf_pinv, zf_fmeta, zf_frow, zf_fcol, zf_bmeta, zf_brow, zf_bcol;
  DeviceBuffer zf_fval64, zf_bval64, zf_bd64, zf_fval32, zf_bval32, zf_bd32;
  DeviceBuffer W64, W32;   // Kp x Np real-block Z (Np = 2 nN rounded up to the N tile); W32
                           // row-major, W64 in K blocks of ZB_BK: (k, n) at
                           // ((k / ZB_BK) Np + n) ZB_BK + k % ZB_BK
  DeviceBuffer slack_d;    // 3 slack node indices
  DeviceBuffer vslack_d;   // 6 doubles
  // workspaces (grow-only); calls on one network must not overlap
  DeviceBuffer ws_v, ws_r, ws_s, ws_act, ws_cnt;
  CallOrder order;   // orders the solves that share these workspaces
  int32_t* count_host = nullptr;   // pinned readback of the active counts
  int count_host_len = 0;
  ~DistNetwork();
  DistDev view() const;
};

DistNetwork* dist_network_create(Context* ctx, int n_node, int nnz, const int32_t* row_ptr,
                                 const int32_t* col_idx, const double* y_re, const double* y_im,
                                 const int32_t* slack_nodes, const double* v_slack, int n_wye,
                                 const int32_t* wye_node, int n_delta, const int32_t* delta_nodes,
                                 const pf_opts& setup);

// Residual workgroup size and GEMM tile sizes shared by the host sizing and
// the kernels.
constexpr int ZB_THREADS = 256;
constexpr int ZB_MAX_FREE = 4096;   // free nodes (the residual keeps v in LDS)
constexpr int ZB_BM = 128;   // scenarios per tile
constexpr int ZB_BN = 128;   // output reals per tile
constexpr int ZB_BK = 16;    // K step
// Iteration caps up to this many are enqueued at once in the asynchronous mode.
constexpr int ZB_ASYNC_MAX_ITER = 1000;

struct ZbusLaunch {
  int batch;
  int64_t ld;
  const double* s_wye;
  const double* s_delta;
  double* v_out;
  int32_t* iters;
  uint8_t* converged;
  double* final_mismatch;
  double* sum_abs_change;
  double tol;
  int max_iter;
  int sparse;         // 1: v += Y_NN^-1 r by the sparse factor instead of the dense product
  int async;          // 1: every iteration enqueued at once (kernels exit once count[] shows none active)
  // workspace
  double* v;          // [rows][Kp] FP64 state
  void* r;            // [rows][Kp] residual in the GEMM's type (rows = batch rounded up to ZB_BM)
  double* st;         // [batch][3]: mismatch, sum |v| at the last residual, change of sum |v|
  int32_t* active;    // [rows] 1 while the scenario still iterates
  int32_t* count;     // [max_iter + 1] scenarios still active at each iteration (may be null)
  int32_t* count_host;  // pinned host copy of `count`, read back by the host loop
  // Scenario of residual row / workgroup g: slots[g] (null: scenario g).  The
  // state v, the inputs, outputs, statistics and flags are indexed by the
  // scenario, the residual rows r by g.  With slots set, each scenario's own
  // iteration count stands in for the launch's iteration number, and the
  // residual sets step_done[g] to 1 once the scenario stopped iterating.
  const int32_t* slots;
  uint8_t* step_done;
};

// Runs the whole fixed point on `stream` (host loop over iterations).
void run_zbus(DistNetwork& net, bool mixed, const ZbusLaunch& a, hipStream_t s);

// Serving-engine pieces over the scenarios a.slots[0 .. a.batch): start them
// from v0; run `iters` fixed-point iterations (residual, then the update for
// those still iterating; a.step_done reports the ones that stopped); write
// the outputs (v_out, final_mismatch) of finished ones.
void zbus_init_slots(DistNetwork& net, const ZbusLaunch& a, hipStream_t s);
void zbus_step(DistNetwork& net, bool mixed, const ZbusLaunch& a, int iters, hipStream_t s);
void zbus_finish_slots(DistNetwork& net, const ZbusLaunch& a, hipStream_t s);

}  // namespace pfx
