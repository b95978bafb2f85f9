// Newton-Raphson solves that allocate nothing: pf_tx_solve's kernels with
// their per-scenario workspace (Newton state, GMRES vectors, Krylov basis)
// carved from one fixed device array instead of network-owned buffers.
//
// The array is a file-scope __device__ symbol, so every device the library
// runs on holds its own copy from module load until the process ends.  In
// host code its name is only a host-side stand-in: its device address is
// taken once per device with hipGetSymbolAddress (scratch_init, called by
// pf_context_create with the device current) and only that address is ever
// handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.hpp"
#include "tx.hpp"

namespace pfx {

namespace {

constexpr size_t kScratchBytes = (size_t)PF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the array's device address and the event that orders calls
// sharing it (each call's kernels wait for the previous call's).
struct ScratchDev {
  std::mutex mu;
  void* ptr = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;
};

ScratchDev g_dev[kMaxDevices];

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

void scratch_init(int device) {
  require(device >= 0 && device < kMaxDevices, "device index beyond the no-allocation table");
  ScratchDev& d = g_dev[device];
  std::lock_guard<std::mutex> lk(d.mu);
  if (d.ptr) return;
  void* p = nullptr;
  PFX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  require(p != nullptr, "no device address for the scratch array");
  PFX_HIP(hipEventCreateWithFlags(&d.done, hipEventDisableTiming));
  d.ptr = p;
}

size_t noalloc_tx_bytes(const TxNetwork& net, const pf_opts& o, int batch) {
  const size_t w = o.precision == PF_MIXED ? sizeof(float) : sizeof(double);
  const size_t ws = align256((size_t)batch * nr_ws_doubles(net) * sizeof(double));
  const size_t basis = (size_t)batch * (o.gmres_restart + 1) * nr_padded_rows(net) * w;
  return ws + basis;
}

}  // namespace pfx

using namespace pfx;

extern "C" {

pf_status pf_tx_solve_noalloc(pf_tx_network* h, const pf_opts* opts, int32_t batch, int64_t ld,
                              const double* p_inj, const double* q_inj, const double* vm_set, double* v_out,
                              int32_t* newton_iters, int32_t* gmres_iters, uint8_t* converged,
                              double* final_mismatch, double* work_bytes, pf_stream stream) {
  return guarded([&] {
    check_handle(h, "transmission network");
    TxNetwork* net = reinterpret_cast<TxNetwork*>(h);
    const pf_opts o = resolve_opts(opts);
    require(o.nr_direct == 0, "pf_tx_solve_noalloc runs the GMRES Newton step only (nr_direct must be 0)");
    require(batch >= 0, "batch must be >= 0");
    require(ld >= net->n, "ld must be at least the row length (" + std::to_string(net->n) + ")");
    if (batch == 0) return;
    require(p_inj && q_inj && vm_set && v_out && newton_iters && converged, "null required pointer");
    const size_t need = noalloc_tx_bytes(*net, o, batch);
    if (need > kScratchBytes)
      fail(PF_INVALID_ARG, "batch of " + std::to_string(batch) + " needs " + std::to_string(need) +
                               " bytes of scratch; the fixed array holds " + std::to_string(kScratchBytes));
    const int dev = net->ctx->device;
    activate(net->ctx);
    ScratchDev& d = g_dev[dev];
    std::lock_guard<std::mutex> lk(d.mu);
    require(d.ptr != nullptr, "scratch array not set up on this device");
    const hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
    const bool mixed = o.precision == PF_MIXED;
    NRLaunch a{};
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
    a.ws_d = static_cast<double*>(d.ptr);
    a.ws_d_stride = nr_ws_doubles(*net);
    a.ws_basis = static_cast<unsigned char*>(d.ptr) +
                 align256((size_t)batch * nr_ws_doubles(*net) * sizeof(double));
    a.ws_b_stride = (int64_t)(o.gmres_restart + 1) * nr_padded_rows(*net);
    if (d.pending) PFX_HIP(hipStreamWaitEvent(hs, d.done, 0));
    launch_nr(*net, mixed, a, hs);
    PFX_HIP(hipEventRecord(d.done, hs));
    d.pending = true;
  });
}

}  // extern "C"
