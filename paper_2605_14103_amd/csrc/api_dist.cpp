// C ABI: radial three-phase feeders (Z-bus fixed point).
#include <cmath>
#include <complex>
#include <map>
#include <string>

#include "common.hpp"
#include "engine.hpp"
#include "dist.hpp"

using namespace pfx;

namespace pfx {
DistNetwork::~DistNetwork() {
  if (count_host) (void)hipHostFree(count_host);
}
}  // namespace pfx

namespace {

DistNetwork* dist_of(pf_dist_network* h) {
  check_handle(h, "feeder");
  return reinterpret_cast<DistNetwork*>(h);
}

}  // namespace

extern "C" {

pf_status pf_dist_ybus_from_segments(int32_t n_bus, int32_t n_seg, const int32_t* seg_from,
                                     const int32_t* seg_to, const double* z, int32_t cap, int32_t* row_ptr,
                                     int32_t* col_idx, double* y_re, double* y_im, int32_t* nnz_out) {
  return guarded([&] {
    using cplx = std::complex<double>;
    require(n_bus >= 1 && n_seg >= 0, "bad sizes");
    if (n_seg > 0) require(seg_from && seg_to && z, "null segment array");
    const int n = 3 * n_bus;
    std::vector<std::map<int, cplx>> rows(n);
    for (int i = 0; i < n; ++i) rows[i][i] += 0.0;
    for (int s = 0; s < n_seg; ++s) {
      const int a = seg_from[s], c = seg_to[s];
      require(a >= 0 && a < n_bus && c >= 0 && c < n_bus && a != c, "segment bus index out of range");
      // y = inv(z) for the 3x3 complex z (Gauss-Jordan with partial pivoting)
      cplx m[3][6];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          m[i][j] = cplx(z[18 * s + 6 * i + 2 * j], z[18 * s + 6 * i + 2 * j + 1]);
          m[i][3 + j] = i == j ? 1.0 : 0.0;
        }
      for (int k = 0; k < 3; ++k) {
        int p = k;
        for (int i = k + 1; i < 3; ++i)
          if (std::abs(m[i][k]) > std::abs(m[p][k])) p = i;
        if (!(std::abs(m[p][k]) > 0)) fail(PF_SINGULAR_SETUP, "singular segment impedance " + std::to_string(s));
        if (p != k)
          for (int j = 0; j < 6; ++j) std::swap(m[k][j], m[p][j]);
        const cplx inv = 1.0 / m[k][k];
        for (int j = 0; j < 6; ++j) m[k][j] *= inv;
        for (int i = 0; i < 3; ++i)
          if (i != k) {
            const cplx f = m[i][k];
            for (int j = 0; j < 6; ++j) m[i][j] -= f * m[k][j];
          }
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const cplx y = m[i][3 + j];
          rows[3 * a + i][3 * a + j] += y;
          rows[3 * c + i][3 * c + j] += y;
          rows[3 * a + i][3 * c + j] -= y;
          rows[3 * c + i][3 * a + j] -= y;
        }
    }
    emit_csr(n, rows, cap, row_ptr, col_idx, y_re, y_im, nnz_out);
  });
}

pf_status pf_dist_network_create(pf_context* c, int32_t n_node, int32_t nnz, const int32_t* row_ptr,
                                 const int32_t* col_idx, const double* y_re, const double* y_im,
                                 const int32_t* slack_nodes, const double* v_slack, int32_t n_wye,
                                 const int32_t* wye_node, int32_t n_delta, const int32_t* delta_nodes,
                                 const pf_opts* setup_opts, pf_dist_network** out) {
  return guarded([&] {
    require(out != nullptr, "out must not be null");
    *out = nullptr;
    check_handle(c, "context");
    auto* ctx = reinterpret_cast<Context*>(c);
    activate(ctx);
    const pf_opts o = resolve_opts(setup_opts);
    DistNetwork* net = dist_network_create(ctx, n_node, nnz, row_ptr, col_idx, y_re, y_im, slack_nodes,
                                           v_slack, n_wye, wye_node, n_delta, delta_nodes, o);
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->dist_nets.insert(net);
    }
    registry().add(net);
    *out = reinterpret_cast<pf_dist_network*>(net);
  });
}

void pf_dist_network_destroy(pf_dist_network* h) {
  if (!registry().has(h)) return;
  auto* net = reinterpret_cast<DistNetwork*>(h);
  Context* ctx = net->ctx;
  destroy_engines_of(ctx, net);
  registry().remove(net);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->dist_nets.erase(net);
  }
  delete net;
}

pf_status pf_dist_network_info(const pf_dist_network* h, int32_t* n_node, int32_t* n_free, int32_t* n_wye,
                               int32_t* n_delta) {
  return guarded([&] {
    const DistNetwork* net = dist_of(const_cast<pf_dist_network*>(h));
    if (n_node) *n_node = net->n_node;
    if (n_free) *n_free = net->nN;
    if (n_wye) *n_wye = net->n_wye;
    if (n_delta) *n_delta = net->n_delta;
  });
}

pf_status pf_dist_solve(pf_dist_network* h, const pf_opts* opts, int32_t batch, int64_t ld,
                        const double* s_wye, const double* s_delta, double* v_out, int32_t* iters,
                        uint8_t* converged, double* final_mismatch, double* sum_abs_change,
                        pf_stream stream) {
  return guarded([&] {
    DistNetwork* net = dist_of(h);
    const pf_opts o = resolve_opts(opts);
    require(batch >= 0, "batch must be >= 0");
    require(ld >= net->n_node, "ld must be at least n_node");
    if (batch == 0) return;
    require(s_wye && s_delta && v_out && iters && converged, "null required pointer");
    activate(net->ctx);
    const hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(net->order.mu);
    const bool mixed = o.precision == PF_MIXED;
    const int rows = (batch + ZB_BM - 1) / ZB_BM * ZB_BM;
    const size_t tsz = mixed ? sizeof(float) : sizeof(double);
    net->order.grow(net->ws_v, net->ctx, (size_t)batch * net->Kp * sizeof(double));
    const size_t rbytes = (size_t)rows * net->Kp * tsz;
    if (net->ws_r.bytes() < rbytes) {
      net->order.grow(net->ws_r, net->ctx, rbytes);
      // padding rows and columns of R must read as zeros
      PFX_HIP(hipMemset(net->ws_r.as<void>(), 0, net->ws_r.bytes()));
    }
    net->order.grow(net->ws_s, net->ctx, (size_t)batch * 3 * sizeof(double));
    net->order.grow(net->ws_act, net->ctx, (size_t)rows * sizeof(int32_t));
    net->order.grow(net->ws_cnt, net->ctx, (size_t)(o.zbus_max_iter + 1) * sizeof(int32_t));
    if ((!o.zbus_async || o.zbus_max_iter > ZB_ASYNC_MAX_ITER) && net->count_host_len < o.zbus_max_iter + 1) {
      net->order.drain();
      if (net->count_host) PFX_HIP(hipHostFree(net->count_host));
      net->count_host = nullptr;
      PFX_HIP(hipHostMalloc(reinterpret_cast<void**>(&net->count_host),
                            sizeof(int32_t) * (o.zbus_max_iter + 1), hipHostMallocDefault));
      net->count_host_len = o.zbus_max_iter + 1;
    }
    ZbusLaunch a{};
    a.batch = batch;
    a.ld = ld;
    a.s_wye = s_wye;
    a.s_delta = s_delta;
    a.v_out = v_out;
    a.iters = iters;
    a.converged = converged;
    a.final_mismatch = final_mismatch;
    a.sum_abs_change = sum_abs_change;
    a.tol = o.tol;
    a.max_iter = o.zbus_max_iter;
    a.sparse = o.zbus_sparse;
    a.async = o.zbus_async;
    a.v = net->ws_v.as<double>();
    a.r = net->ws_r.as<void>();
    a.st = net->ws_s.as<double>();
    a.active = net->ws_act.as<int32_t>();
    a.count = net->ws_cnt.as<int32_t>();
    a.count_host = net->count_host;
    net->order.begin(hs);
    run_zbus(*net, mixed, a, hs);
    net->order.end(hs);
  });
}

}  // extern "C"
