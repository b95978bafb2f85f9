// Transmission network: host-side record and the plain device views the
// Newton-Raphson, branch-loss and adjoint kernels take by value.
//
// Internal bus order.  Buses are renumbered so that PQ buses come first, then
// PV buses, then the slack.  With n buses, nth = n - 1 and npq PQ buses, the
// Newton state x = [theta over Theta ; |V| over Q] (eq. (1)) then has row r <
// nth for the angle of internal bus r and row nth + q for the magnitude of
// internal bus q < npq: no index maps are needed inside the kernels.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"
#include "factor.hpp"

namespace pfx {

// Device view of one HybridFactor (see factor.hpp), values in T.
template <typename T>
struct SpdDev {
  int N, c, k, nfl, nbl;
  const int* pinv;
  const int* f_lev;
  const int* f_rows;
  const int* L_ptr;
  const int* L_col;
  const T* L_val;
  const T* dinv;
  const int* b_lev;
  const int* b_rows;
  const int* T_ptr;
  const int* T_col;
  const T* T_val;
  const T* Sinv;
};

template <typename T>
struct TxDev {
  int n, nth, npq, m;
  const int* y_ptr;      // Ybus CSR in internal order
  const int* y_col;
  const double* y_re;
  const double* y_im;
  const int* int2ext;    // internal bus -> caller's bus index
  SpdDev<T> bp;          // (B' + eps I)^-1 over Theta
  SpdDev<T> bpp;         // (B'' + eps I)^-1 over Q
  const int* g_ptr;      // G = -Re(Ybus)[Q, Theta]; columns as factor positions of bp
  const int* g_col;
  const T* g_val;
  const int* gt_ptr;     // G^T; rows Theta, columns as factor positions of bpp
  const int* gt_col;
  const T* gt_val;
  const int* yt_ptr;     // Ybus^T CSR (internal order), for the adjoint
  const int* yt_col;
  const double* yt_re;
  const double* yt_im;
  // branch list (internal bus numbers) for the branch-current loss
  int n_branch;
  const int* br_f;
  const int* br_t;
  const double* br_ys_re;
  const double* br_ys_im;
  const double* br_b;
};

// Device copies of one factor: index arrays once, values in FP64 and FP32.
struct SpdBuffers {
  HybridFactor host;
  DeviceBuffer pinv, f_lev, f_rows, L_ptr, L_col, b_lev, b_rows, T_ptr, T_col;
  DeviceBuffer L_val64, dinv64, T_val64, Sinv64;
  DeviceBuffer L_val32, dinv32, T_val32, Sinv32;
  template <typename T>
  SpdDev<T> view() const;
};

struct TxNetwork {
  Context* ctx = nullptr;
  int n = 0, nth = 0, npq = 0, m = 0, nnz = 0, n_branch = 0;
  std::vector<int> int2ext, ext2int;
  pf_opts setup{};
  DeviceBuffer y_ptr, y_col, y_re, y_im, int2ext_d;
  DeviceBuffer yt_ptr, yt_col, yt_re, yt_im;   // Ybus^T (internal order) for the adjoint
  SpdBuffers bp, bpp;
  DeviceBuffer g_ptr, g_col, g_val64, g_val32, gt_ptr, gt_col, gt_val64, gt_val32;
  DeviceBuffer br_f, br_t, br_ys_re, br_ys_im, br_b;
  DeviceBuffer inc_ptr, inc_br;   // branches incident to each internal bus
  // solve workspaces (grow-only); calls on one network must not overlap
  DeviceBuffer ws_d, ws_basis, ws_adj;
  // the device views themselves, resident in device memory so kernels take one pointer
  DeviceBuffer desc64, desc32;
  template <typename T>
  TxDev<T> view() const;
  template <typename T>
  const TxDev<T>* desc() const {
    return sizeof(T) == 8 ? desc64.as<const TxDev<T>>() : desc32.as<const TxDev<T>>();
  }
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
  double* ws_d;
  int64_t ws_d_stride;
  void* ws_basis;
  int64_t ws_b_stride;
};

// Doubles of per-scenario FP64 workspace the NR kernel needs, and the padded
// state length (rows per thread times threads) of its vectors.
int64_t nr_ws_doubles(const TxNetwork& net);
int64_t nr_padded_rows(const TxNetwork& net);
void launch_nr(const TxNetwork& net, bool mixed, const NRLaunch& a, hipStream_t s);

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
