// C ABI: transmission grids (Newton-Raphson, branch loss, adjoint).
#include <cmath>
#include <complex>
#include <map>
#include <string>

#include "common.hpp"
#include "engine.hpp"
#include "tx.hpp"

using namespace pfx;

namespace {

TxNetwork* tx_of(pf_tx_network* h) {
  check_handle(h, "transmission network");
  return reinterpret_cast<TxNetwork*>(h);
}

void check_ld(int32_t batch, int64_t ld, int rows) {
  require(batch >= 0, "batch must be >= 0");
  require(ld >= rows, "ld must be at least the row length (" + std::to_string(rows) + ")");
}

}  // namespace

extern "C" {

pf_status pf_tx_ybus_from_branches(int32_t n_bus, int32_t n_branch, const int32_t* f, const int32_t* t,
                                   const double* r, const double* x, const double* b, int32_t cap,
                                   int32_t* row_ptr, int32_t* col_idx, double* y_re, double* y_im,
                                   int32_t* nnz_out) {
  return guarded([&] {
    require(n_bus >= 1 && n_branch >= 0, "bad sizes");
    if (n_branch > 0) require(f && t && r && x && b, "null branch array");
    std::vector<std::map<int, std::complex<double>>> rows(n_bus);
    for (int i = 0; i < n_bus; ++i) rows[i][i] += 0.0;
    for (int k = 0; k < n_branch; ++k) {
      require(f[k] >= 0 && f[k] < n_bus && t[k] >= 0 && t[k] < n_bus, "branch bus index out of range");
      require(f[k] != t[k], "a branch must join two different buses");
      const std::complex<double> z(r[k], x[k]);
      require(std::abs(z) > 0, "zero branch impedance");
      const std::complex<double> ys = 1.0 / z, ysh(0.0, 0.5 * b[k]);
      rows[f[k]][f[k]] += ys + ysh;
      rows[t[k]][t[k]] += ys + ysh;
      rows[f[k]][t[k]] -= ys;
      rows[t[k]][f[k]] -= ys;
    }
    emit_csr(n_bus, rows, cap, row_ptr, col_idx, y_re, y_im, nnz_out);
  });
}

pf_status pf_tx_network_create(pf_context* c, int32_t n_bus, int32_t nnz, const int32_t* row_ptr,
                               const int32_t* col_idx, const double* y_re, const double* y_im,
                               const int8_t* bus_type, int32_t n_branch, const int32_t* br_f,
                               const int32_t* br_t, const double* br_r, const double* br_x,
                               const double* br_b, const pf_opts* setup_opts, pf_tx_network** out) {
  return guarded([&] {
    require(out != nullptr, "out must not be null");
    *out = nullptr;
    check_handle(c, "context");
    auto* ctx = reinterpret_cast<Context*>(c);
    activate(ctx);
    const pf_opts o = resolve_opts(setup_opts);
    TxNetwork* net = tx_network_create(ctx, n_bus, nnz, row_ptr, col_idx, y_re, y_im, bus_type, n_branch,
                                       br_f, br_t, br_r, br_x, br_b, o);
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->tx_nets.insert(net);
    }
    registry().add(net);
    *out = reinterpret_cast<pf_tx_network*>(net);
  });
}

void pf_tx_network_destroy(pf_tx_network* h) {
  if (!registry().has(h)) return;
  auto* net = reinterpret_cast<TxNetwork*>(h);
  Context* ctx = net->ctx;
  destroy_engines_of(ctx, net);
  registry().remove(net);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tx_nets.erase(net);
  }
  delete net;
}

pf_status pf_tx_network_info(const pf_tx_network* h, int32_t* n_bus, int32_t* n_theta, int32_t* n_q,
                             int32_t* nnz, int32_t* factor_nnz, int32_t* core_bp, int32_t* core_bpp) {
  return guarded([&] {
    const TxNetwork* net = tx_of(const_cast<pf_tx_network*>(h));
    if (n_bus) *n_bus = net->n;
    if (n_theta) *n_theta = net->nth;
    if (n_q) *n_q = net->npq;
    if (nnz) *nnz = net->nnz;
    if (factor_nnz) *factor_nnz = (int32_t)(net->bp.host.entries() + net->bpp.host.entries());
    if (core_bp) *core_bp = net->bp.host.k;
    if (core_bpp) *core_bpp = net->bpp.host.k;
  });
}

}  // extern "C"

namespace {

void tx_solve(pf_tx_network* h, const pf_opts* opts, int32_t batch, int64_t ld, const double* p_inj,
              const double* q_inj, const double* vm_set, int64_t ldy, const double* y_vals, double* v_out,
              int32_t* newton_iters, int32_t* gmres_iters, uint8_t* converged, double* final_mismatch,
              double* work_bytes, pf_stream stream) {
  TxNetwork* net = tx_of(h);
  const pf_opts o = resolve_opts(opts);
  check_ld(batch, ld, net->n);
  if (batch == 0) return;
  require(p_inj && q_inj && vm_set && v_out && newton_iters && converged, "null required pointer");
  activate(net->ctx);
  const hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(net->order.mu);
  const bool direct = o.nr_direct == 1;
  if (direct) {
    net->order.drain();   // the analysis is written into the network once, with no call in flight
    ensure_direct(*net);
  }
  const bool mixed = o.precision == PF_MIXED && !direct;
  const int64_t dstride = nr_ws_doubles(*net);
  const int64_t bstride = (int64_t)(o.gmres_restart + 1) * nr_padded_rows(*net);
  net->order.grow(net->ws_d, net->ctx, (size_t)batch * dstride * sizeof(double));
  const bool dval = direct && !direct_lds_fits(*net);
  if (dval) net->order.grow(net->ws_dval, net->ctx, (size_t)batch * net->direct_nval * sizeof(double));
  if (!direct)
    net->order.grow(net->ws_basis, net->ctx, (size_t)batch * bstride * (mixed ? sizeof(float) : sizeof(double)));
  net->order.begin(hs);
  NRLaunch a{};
  if (y_vals) {
    // FP64 layout copy, then (mixed) the FP32 copy behind it
    const size_t n64 = (size_t)batch * net->y_entries;
    net->order.grow(net->ws_y, net->ctx, n64 * sizeof(double2) + (mixed ? n64 * sizeof(float2) : 0));
    double2* y64 = net->ws_y.as<double2>();
    float2* y32 = mixed ? reinterpret_cast<float2*>(y64 + n64) : nullptr;
    launch_y_gather(*net, batch, ldy, y_vals, y64, y32, hs);
    a.yv64 = y64;
    a.yvT = mixed ? static_cast<const void*>(y32) : static_cast<const void*>(y64);
    a.yv_stride = net->y_entries;
    a.yv_nnz = net->nnz;
  }
  a.batch = batch;
  a.ld = ld;
  a.p_inj = p_inj;
  a.q_inj = q_inj;
  a.vm_set = vm_set;
  a.v_out = v_out;
  a.newton_iters = newton_iters;
  a.gmres_iters = gmres_iters;
  a.converged = converged;
  a.final_mismatch = final_mismatch;
  a.work_bytes = work_bytes;
  a.tol = o.tol;
  a.diverge = o.diverge;
  a.rtol = o.gmres_rtol;
  a.forcing = o.forcing;
  a.forcing_max = o.forcing_max;
  a.max_newton = o.max_newton;
  a.restart = o.gmres_restart;
  a.max_restarts = o.gmres_max_restarts;
  a.ws_d = net->ws_d.as<double>();
  a.ws_d_stride = dstride;
  a.ws_basis = net->ws_basis.as<void>();
  a.ws_b_stride = bstride;
  if (dval) {
    a.ws_dval = net->ws_dval.as<double>();
    a.ws_dval_stride = net->direct_nval;
  }
  if (direct) launch_nr_direct(*net, a, hs);
  else launch_nr(*net, mixed, a, hs);
  net->order.end(hs);
}

}  // namespace

extern "C" {

pf_status pf_tx_solve(pf_tx_network* h, const pf_opts* opts, int32_t batch, int64_t ld,
                      const double* p_inj, const double* q_inj, const double* vm_set, double* v_out,
                      int32_t* newton_iters, int32_t* gmres_iters, uint8_t* converged,
                      double* final_mismatch, double* work_bytes, pf_stream stream) {
  return guarded([&] {
    tx_solve(h, opts, batch, ld, p_inj, q_inj, vm_set, 0, nullptr, v_out, newton_iters, gmres_iters, converged,
             final_mismatch, work_bytes, stream);
  });
}

pf_status pf_tx_solve_yvals(pf_tx_network* h, const pf_opts* opts, int32_t batch, int64_t ld,
                            const double* p_inj, const double* q_inj, const double* vm_set, int64_t ldy,
                            const double* y_vals, double* v_out, int32_t* newton_iters, int32_t* gmres_iters,
                            uint8_t* converged, double* final_mismatch, double* work_bytes, pf_stream stream) {
  return guarded([&] {
    const TxNetwork* net = tx_of(h);
    require(ldy >= net->caller_nnz, "ldy must be at least nnz (" + std::to_string(net->caller_nnz) + ")");
    require(y_vals != nullptr || batch == 0, "y_vals must not be null");
    tx_solve(h, opts, batch, ld, p_inj, q_inj, vm_set, ldy, y_vals, v_out, newton_iters, gmres_iters,
             converged, final_mismatch, work_bytes, stream);
  });
}

pf_status pf_tx_ybus_switch(int32_t n_bus, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                            const double* y_re, const double* y_im, int32_t n_branch, const int32_t* f,
                            const int32_t* t, const double* r, const double* x, const double* b, int32_t batch,
                            const uint8_t* branch_on, int64_t ldy, double* y_vals) {
  return guarded([&] {
    require(n_bus >= 1 && nnz >= 0 && n_branch >= 0 && batch >= 0, "bad sizes");
    require(ldy >= nnz, "ldy must be at least nnz");
    require(row_ptr && (nnz == 0 || (col_idx && y_re && y_im)), "null CSR array");
    if (n_branch > 0) require(f && t && r && x && b, "null branch array");
    if (batch > 0) require(branch_on && y_vals, "null branch_on or y_vals");
    require(row_ptr[0] == 0 && row_ptr[n_bus] == nnz, "row_ptr must run from 0 to nnz");
    auto find = [&](int i, int j) {
      require(i >= 0 && i < n_bus && j >= 0 && j < n_bus, "branch bus index out of range");
      for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
        if (col_idx[p] == j) return p;
      fail(PF_INVALID_ARG, "branch (" + std::to_string(i) + ", " + std::to_string(j) + ") has no entry in the pattern");
      return -1;
    };
    // the four entries each branch stamps and what it adds there
    struct Stamp {
      int ff, tt, ft, tf;
      std::complex<double> diag, off;
    };
    std::vector<Stamp> st(n_branch);
    for (int k = 0; k < n_branch; ++k) {
      require(f[k] != t[k], "a branch must join two different buses");
      const std::complex<double> z(r[k], x[k]);
      require(std::abs(z) > 0, "zero branch impedance");
      const std::complex<double> ys = 1.0 / z;
      st[k] = {find(f[k], f[k]), find(t[k], t[k]), find(f[k], t[k]), find(t[k], f[k]),
               ys + std::complex<double>(0.0, 0.5 * b[k]), -ys};
    }
    for (int s = 0; s < batch; ++s) {
      double* out = y_vals + 2 * ldy * (int64_t)s;
      for (int p = 0; p < nnz; ++p) {
        out[2 * p] = y_re[p];
        out[2 * p + 1] = y_im[p];
      }
      const uint8_t* on = branch_on + (int64_t)n_branch * s;
      for (int k = 0; k < n_branch; ++k) {
        if (on[k]) continue;
        const Stamp& q = st[k];
        for (int p : {q.ff, q.tt}) {
          out[2 * p] -= q.diag.real();
          out[2 * p + 1] -= q.diag.imag();
        }
        for (int p : {q.ft, q.tf}) {
          out[2 * p] -= q.off.real();
          out[2 * p + 1] -= q.off.imag();
        }
      }
    }
  });
}

pf_status pf_tx_branch_loss(pf_tx_network* h, int32_t batch, int64_t ld, const double* v, double* loss,
                            double* dl_dv, pf_stream stream) {
  return guarded([&] {
    TxNetwork* net = tx_of(h);
    check_ld(batch, ld, net->n);
    require(net->n_branch > 0, "the network was registered without a branch list");
    if (batch == 0) return;
    require(v && loss, "null required pointer");
    activate(net->ctx);
    LossLaunch a{batch, ld, v, loss, dl_dv};
    launch_branch_loss(*net, a, reinterpret_cast<hipStream_t>(stream));
  });
}

pf_status pf_tx_adjoint(pf_tx_network* h, const pf_opts* opts, int32_t batch, int64_t ld, const double* v,
                        const double* dl_dv, double* grad_p, double* grad_q, int32_t* gmres_iters,
                        uint8_t* converged, pf_stream stream) {
  return guarded([&] {
    TxNetwork* net = tx_of(h);
    pf_opts o = resolve_opts(opts);
    check_ld(batch, ld, net->n);
    if (batch == 0) return;
    require(v && dl_dv && grad_p && grad_q, "null required pointer");
    activate(net->ctx);
    const double rtol = (opts && opts->gmres_rtol > 0) ? opts->gmres_rtol : 1e-10;
    const int64_t dstride = adj_ws_doubles(*net);
    const int64_t bstride = (int64_t)(o.gmres_restart + 1) * nr_padded_rows(*net);
    const hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(net->order.mu);
    net->order.grow(net->ws_adj, net->ctx, (size_t)batch * (dstride + bstride) * sizeof(double));
    net->order.begin(hs);
    AdjLaunch a{};
    a.batch = batch;
    a.ld = ld;
    a.v = v;
    a.dl_dv = dl_dv;
    a.grad_p = grad_p;
    a.grad_q = grad_q;
    a.gmres_iters = gmres_iters;
    a.converged = converged;
    a.rtol = rtol;
    a.restart = o.gmres_restart;
    a.max_restarts = o.gmres_max_restarts;
    a.ws_d = net->ws_adj.as<double>();
    a.ws_d_stride = dstride;
    a.ws_basis = net->ws_adj.as<double>() + (int64_t)batch * dstride;
    a.ws_b_stride = bstride;
    launch_adjoint(*net, a, hs);
    net->order.end(hs);
  });
}

}  // extern "C"
