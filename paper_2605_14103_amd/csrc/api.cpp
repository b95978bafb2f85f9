// C ABI: context, options, last error, device buffers and shared helpers.
#include <cmath>
#include <string>

#include "common.hpp"
#include "dist.hpp"
#include "engine.hpp"
#include "tx.hpp"

namespace pfx {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

Registry& registry() {
  static Registry r;
  return r;
}

void DeviceBuffer::allocate(Context* ctx, size_t bytes) {
  release();
  if (bytes == 0) return;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->budget && ctx->held + bytes > ctx->budget)
      fail(PF_OUT_OF_MEMORY, "context HBM budget exceeded: need " + std::to_string(bytes) +
                                 " more bytes, hold " + std::to_string(ctx->held) + " of " +
                                 std::to_string(ctx->budget));
    ctx->held += bytes;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->held -= bytes;
    fail(PF_OUT_OF_MEMORY, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
  }
  ctx_ = ctx;
  ptr_ = p;
  bytes_ = bytes;
}

void DeviceBuffer::release() {
  if (ptr_) {
    (void)hipFree(ptr_);
    std::lock_guard<std::mutex> lk(ctx_->mu);
    ctx_->held -= bytes_;
  }
  ctx_ = nullptr;
  ptr_ = nullptr;
  bytes_ = 0;
}

pf_opts resolve_opts(const pf_opts* o) {
  pf_opts r;
  pf_opts_default(&r);
  if (o) r = *o;
  require(r.precision == PF_FP64 || r.precision == PF_MIXED, "precision must be PF_FP64 or PF_MIXED");
  require(r.tol > 0 && std::isfinite(r.tol), "tol must be positive");
  require(r.max_newton >= 0 && r.max_newton <= 1000, "max_newton must be 0..1000");
  require(r.gmres_restart >= 1 && r.gmres_restart <= 64, "gmres_restart must be 1..64");
  require(r.gmres_max_restarts >= 1 && r.gmres_max_restarts <= 1000, "gmres_max_restarts must be 1..1000");
  // Inexact Newton: each linear solve only has to cut the preconditioned
  // residual by 1e-3; the FP64 mismatch test decides convergence, so the
  // answer is unchanged while the GMRES steps per Newton step drop.
  if (r.gmres_rtol == 0) r.gmres_rtol = 1e-3;
  require(r.gmres_rtol > 0 && r.gmres_rtol < 1, "gmres_rtol must be in (0, 1)");
  require(r.diverge > 0, "diverge must be positive");
  require(r.zbus_max_iter >= 0 && r.zbus_max_iter <= 100000, "zbus_max_iter must be 0..100000");
  require(r.eps >= 0 && std::isfinite(r.eps), "eps must be >= 0");
  require(r.precond_block >= 0, "precond_block must be >= 0");
  require(r.factor_max_levels >= 1, "factor_max_levels must be >= 1");
  require(r.factor_max_core >= 0 && r.factor_max_core <= 2048, "factor_max_core must be 0..2048");
  require(r.zbus_sparse == 0 || r.zbus_sparse == 1, "zbus_sparse must be 0 or 1");
  require(r.nr_direct == 0 || r.nr_direct == 1, "nr_direct must be 0 or 1");
  require(r.zbus_async == 0 || r.zbus_async == 1, "zbus_async must be 0 or 1");
  require(r.step_iters >= 1 && r.step_iters <= 1000, "step_iters must be 1..1000");
  require(r.forcing == 0 || r.forcing == 1, "forcing must be 0 or 1");
  require(r.forcing_max > 0 && r.forcing_max < 1, "forcing_max must be in (0, 1)");
  return r;
}

void emit_csr(int n, const std::vector<std::map<int, std::complex<double>>>& rows, int cap,
              int32_t* row_ptr, int32_t* col_idx, double* y_re, double* y_im, int32_t* nnz_out) {
  int64_t nnz = 0;
  for (auto& r : rows) nnz += (int64_t)r.size();
  require(nnz < ((int64_t)1 << 31), "too many nonzeros");
  require(nnz_out != nullptr, "nnz_out must not be null");
  *nnz_out = (int32_t)nnz;
  require(nnz <= cap, "output capacity too small: need " + std::to_string(nnz));
  require(row_ptr && col_idx && y_re && y_im, "null output array");
  int p = 0;
  row_ptr[0] = 0;
  for (int i = 0; i < n; ++i) {
    for (auto& [j, y] : rows[i]) {
      col_idx[p] = j;
      y_re[p] = y.real();
      y_im[p] = y.imag();
      ++p;
    }
    row_ptr[i + 1] = p;
  }
}

}  // namespace pfx

using namespace pfx;

extern "C" {

void pf_opts_default(pf_opts* o) {
  if (!o) return;
  o->precision = PF_FP64;
  o->tol = 1e-8;
  o->max_newton = 20;
  o->gmres_restart = 30;
  o->gmres_max_restarts = 10;
  o->gmres_rtol = 0.0;
  o->diverge = 1e6;
  o->zbus_max_iter = 100;
  o->eps = 1e-8;
  o->precond_block = 0;
  o->factor_max_levels = 8;
  o->factor_max_core = 384;
  o->zbus_sparse = 0;
  o->nr_direct = 0;
  o->zbus_async = 0;
  o->step_iters = 1;
  o->forcing = 1;
  o->forcing_max = 0.01;
}

const char* pf_last_error(void) { return g_last_error.c_str(); }

pf_status pf_context_create(int32_t device, uint64_t hbm_budget_bytes, pf_context** out) {
  return guarded([&] {
    require(out != nullptr, "out must not be null");
    *out = nullptr;
    int count = 0;
    PFX_HIP(hipGetDeviceCount(&count));
    require(device >= 0 && device < count, "device index out of range");
    auto ctx = std::make_unique<Context>();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    PFX_HIP(hipSetDevice(device));
    PFX_HIP(hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, device));
    scratch_init(device);
    registry().add(ctx.get());
    *out = reinterpret_cast<pf_context*>(ctx.release());
  });
}

void pf_context_destroy(pf_context* c) {
  auto* ctx = reinterpret_cast<Context*>(c);
  if (!registry().has(ctx)) return;
  (void)hipSetDevice(ctx->device);
  destroy_engines_of(ctx, nullptr);
  (void)hipDeviceSynchronize();
  for (void* t : std::set<void*>(ctx->tx_nets)) {
    registry().remove(t);
    delete static_cast<TxNetwork*>(t);
  }
  for (void* d : std::set<void*>(ctx->dist_nets)) {
    registry().remove(d);
    delete static_cast<DistNetwork*>(d);
  }
  registry().remove(ctx);
  delete ctx;
}

uint64_t pf_context_bytes(const pf_context* c) {
  auto* ctx = reinterpret_cast<Context*>(const_cast<pf_context*>(c));
  if (!registry().has(ctx)) return 0;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return ctx->held;
}

}  // extern "C"
