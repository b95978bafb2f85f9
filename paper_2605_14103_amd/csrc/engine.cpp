// Serving engine: continuous batching of power-flow requests on one network.
//
// An engine owns device memory for `max_slots` scenarios (inputs, outputs and
// solver workspace; the slot count follows from an HBM byte budget) and
// `n_streams` HIP streams, each driven by a worker thread.  Requests are
// queued FIFO.  Whenever a worker is idle, the dispatcher packs the longest
// FIFO prefix of waiting requests that fits a contiguous run of free slots
// into one job and hands it to that worker, which stages the inputs, launches
// the batched solve on its stream, copies the results back and frees the
// slots.  Requests that arrive while other jobs run are therefore admitted as
// soon as slots and a stream free up, and their kernels run concurrently with
// the jobs already on the device.  Each scenario is solved by its own
// workgroup(s) with arithmetic that does not depend on the other scenarios of
// the job, so a result is bit-identical alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"
#include "dist.hpp"
#include "engine.hpp"
#include "tx.hpp"

namespace pfx {

namespace {

struct Request {
  int64_t id = 0;
  int n = 0;
  std::vector<double> in[3];
  int first = -1;      // first slot while in flight
  bool done = false;
  std::string error;
  std::vector<double> v;          // complex interleaved, n rows
  std::vector<int32_t> iters;
  std::vector<uint8_t> conv;
  std::vector<double> mismatch;
  double t_submit = 0, t_launch = 0, t_done = 0;   // seconds since the engine was created
};

struct Job {
  int first = 0, n = 0;
  std::vector<int64_t> ids;
};

struct Worker {
  hipStream_t stream = nullptr;
  std::thread th;
  bool busy = false;
  bool has_job = false;
  Job job;
  DeviceBuffer r, count;      // feeder only: residual rows for a whole job, active counts
  int32_t* count_host = nullptr;
};

}  // namespace

struct Engine {
  Context* ctx = nullptr;
  int kind = 0;               // 0 transmission, 1 feeder
  TxNetwork* tx = nullptr;
  DistNetwork* dist = nullptr;
  pf_opts opts{};
  bool mixed = false;
  int row = 0;                // reals per scenario row of an input (n_bus, or 2 n_node for complex)
  int n_in = 0;
  int max_slots = 0;
  uint64_t per_slot = 0;
  // slot-indexed device buffers
  DeviceBuffer in_d[3], v_d, iters_d, conv_d, mis_d, ws_d, ws_b, st_d, act_d;
  int64_t ws_stride = 0, wb_stride = 0;
  // slot-indexed pinned host staging
  double* in_h[3] = {nullptr, nullptr, nullptr};
  double* v_h = nullptr;
  double* mis_h = nullptr;
  int32_t* iters_h = nullptr;
  uint8_t* conv_h = nullptr;
  std::vector<char> used;
  std::vector<Worker> workers;
  std::mutex mu;
  std::condition_variable cv_dispatch, cv_work, cv_done;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  std::deque<int64_t> pending;
  std::map<int64_t, Request> reqs;
  std::deque<int64_t> completed;
  bool stop = false;
  std::thread dispatcher;
  uint64_t n_jobs = 0, n_scen = 0;
  int in_flight = 0;

  ~Engine();
  int find_range(int n) const;
  void dispatch_loop();
  void worker_loop(int w);
  void run_job(Worker& wk, const Job& job);
};

namespace {

template <typename T>
T* host_alloc(size_t count) {
  void* p = nullptr;
  PFX_HIP(hipHostMalloc(&p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault));
  return static_cast<T*>(p);
}

uint64_t tx_slot_bytes(const TxNetwork& net, bool mixed, int R) {
  const uint64_t n = net.n;
  return 8ull * (3 * n + 2 * n)            // p, q, vm in; v out
         + 4 + 1 + 8                       // iterations, flag, mismatch
         + 8ull * nr_ws_doubles(net)       // FP64 workspace
         + (uint64_t)(R + 1) * nr_padded_rows(net) * (mixed ? 4 : 8);  // Krylov basis
}

uint64_t dist_slot_bytes(const DistNetwork& net, bool mixed) {
  const uint64_t nn = net.n_node;
  return 16ull * (3 * nn)                  // s_wye, s_delta in; v out
         + 4 + 1 + 8                       // iterations, flag, mismatch
         + 8ull * net.Kp + 3 * 8 + 4       // state, statistics, active flag
         + (uint64_t)net.Kp * (mixed ? 4 : 8);   // residual row (one per worker, counted per slot)
}

}  // namespace

uint64_t engine_slot_bytes(int kind, void* net, const pf_opts& o) {
  const bool mixed = o.precision == PF_MIXED;
  if (kind == 0) return tx_slot_bytes(*static_cast<TxNetwork*>(net), mixed, o.gmres_restart);
  return dist_slot_bytes(*static_cast<DistNetwork*>(net), mixed);
}

Engine* engine_create(Context* ctx, int kind, void* network, uint64_t hbm_bytes, int n_streams,
                      const pf_opts& o) {
  require(kind == 0 || kind == 1, "kind must be 0 (transmission) or 1 (feeder)");
  require(n_streams >= 1 && n_streams <= 8, "n_streams must be 1..8");
  auto e = std::make_unique<Engine>();
  e->ctx = ctx;
  e->kind = kind;
  e->opts = o;
  e->mixed = o.precision == PF_MIXED;
  e->per_slot = engine_slot_bytes(kind, network, o);
  e->max_slots = (int)std::min<uint64_t>(hbm_bytes / e->per_slot, 1u << 20);
  require(e->max_slots >= 1, "HBM budget below one scenario's footprint (" + std::to_string(e->per_slot) + " bytes)");
  const size_t S = e->max_slots;
  if (kind == 0) {
    e->tx = static_cast<TxNetwork*>(network);
    const TxNetwork& net = *e->tx;
    e->row = net.n;
    e->n_in = 3;
    for (int i = 0; i < 3; ++i) e->in_d[i].allocate(ctx, S * net.n * 8);
    e->v_d.allocate(ctx, S * net.n * 16);
    e->ws_stride = nr_ws_doubles(net);
    e->wb_stride = (int64_t)(o.gmres_restart + 1) * nr_padded_rows(net);
    e->ws_d.allocate(ctx, S * e->ws_stride * 8);
    e->ws_b.allocate(ctx, S * e->wb_stride * (e->mixed ? 4 : 8));
  } else {
    e->dist = static_cast<DistNetwork*>(network);
    const DistNetwork& net = *e->dist;
    e->row = 2 * net.n_node;
    e->n_in = 2;
    for (int i = 0; i < 2; ++i) e->in_d[i].allocate(ctx, S * net.n_node * 16);
    e->v_d.allocate(ctx, S * net.n_node * 16);
    e->ws_d.allocate(ctx, S * net.Kp * 8);
    e->st_d.allocate(ctx, S * 3 * 8);
    e->act_d.allocate(ctx, (S + ZB_BM) * 4);
  }
  e->iters_d.allocate(ctx, S * 4);
  e->conv_d.allocate(ctx, S);
  e->mis_d.allocate(ctx, S * 8);
  const int vrow = kind == 0 ? 2 * e->tx->n : 2 * e->dist->n_node;
  for (int i = 0; i < e->n_in; ++i) e->in_h[i] = host_alloc<double>(S * e->row);
  e->v_h = host_alloc<double>(S * vrow);
  e->mis_h = host_alloc<double>(S);
  e->iters_h = host_alloc<int32_t>(S);
  e->conv_h = host_alloc<uint8_t>(S);
  e->used.assign(S, 0);
  e->workers.resize(n_streams);
  for (auto& w : e->workers) {
    PFX_HIP(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
    if (kind == 1) {
      const size_t rows = (S + ZB_BM - 1) / ZB_BM * ZB_BM;
      w.r.allocate(ctx, rows * e->dist->Kp * (e->mixed ? 4 : 8));
      PFX_HIP(hipMemset(w.r.as<void>(), 0, w.r.bytes()));
      w.count.allocate(ctx, (o.zbus_max_iter + 1) * 4);
      w.count_host = host_alloc<int32_t>(o.zbus_max_iter + 1);
    }
  }
  Engine* raw = e.get();
  for (int i = 0; i < n_streams; ++i) raw->workers[i].th = std::thread([raw, i] { raw->worker_loop(i); });
  raw->dispatcher = std::thread([raw] { raw->dispatch_loop(); });
  return e.release();
}

Engine::~Engine() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_dispatch.notify_all();
  cv_work.notify_all();
  if (dispatcher.joinable()) dispatcher.join();
  for (auto& w : workers)
    if (w.th.joinable()) w.th.join();
  for (auto& w : workers) {
    if (w.stream) (void)hipStreamDestroy(w.stream);
    if (w.count_host) (void)hipHostFree(w.count_host);
  }
  for (auto* p : in_h)
    if (p) (void)hipHostFree(p);
  if (v_h) (void)hipHostFree(v_h);
  if (mis_h) (void)hipHostFree(mis_h);
  if (iters_h) (void)hipHostFree(iters_h);
  if (conv_h) (void)hipHostFree(conv_h);
}

// First run of n consecutive free slots, or -1.
int Engine::find_range(int n) const {
  int run = 0;
  for (int s = 0; s < max_slots; ++s) {
    run = used[s] ? 0 : run + 1;
    if (run == n) return s - n + 1;
  }
  return -1;
}

void Engine::dispatch_loop() {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_dispatch.wait(lk, [&] {
      if (stop) return true;
      if (pending.empty()) return false;
      for (auto& w : workers)
        if (!w.busy) return true;
      return false;
    });
    if (stop) return;
    int wi = -1;
    for (size_t i = 0; i < workers.size(); ++i)
      if (!workers[i].busy) {
        wi = (int)i;
        break;
      }
    // longest FIFO prefix that fits one contiguous free range
    Job job;
    int total = 0;
    size_t take = 0;
    int first = -1;
    for (size_t k = 0; k < pending.size(); ++k) {
      const int n = reqs[pending[k]].n;
      const int f = find_range(total + n);
      if (f < 0) break;
      total += n;
      first = f;
      take = k + 1;
    }
    if (take == 0) {  // nothing fits now; wait for a job to finish
      cv_dispatch.wait(lk, [&] { return stop || in_flight == 0 || find_range(reqs[pending.front()].n) >= 0; });
      continue;
    }
    job.first = first;
    job.n = total;
    int off = first;
    for (size_t k = 0; k < take; ++k) {
      Request& r = reqs[pending.front()];
      pending.pop_front();
      r.first = off;
      r.t_launch = now();
      for (int i = 0; i < n_in; ++i)
        std::memcpy(in_h[i] + (size_t)off * row, r.in[i].data(), sizeof(double) * (size_t)r.n * row);
      for (int q = 0; q < r.n; ++q) used[off + q] = 1;
      job.ids.push_back(r.id);
      off += r.n;
    }
    Worker& w = workers[wi];
    w.busy = true;
    w.has_job = true;
    w.job = std::move(job);
    ++in_flight;
    cv_work.notify_all();
  }
}

void Engine::run_job(Worker& wk, const Job& job) {
  const int first = job.first, n = job.n;
  const hipStream_t s = wk.stream;
  for (int i = 0; i < n_in; ++i)
    PFX_HIP(hipMemcpyAsync(in_d[i].as<double>() + (size_t)first * row, in_h[i] + (size_t)first * row,
                           sizeof(double) * (size_t)n * row, hipMemcpyHostToDevice, s));
  size_t vrow = 0;
  if (kind == 0) {
    const TxNetwork& net = *tx;
    vrow = 2 * net.n;
    NRLaunch a{};
    a.batch = n;
    a.ld = net.n;
    a.p_inj = in_d[0].as<double>() + (size_t)first * net.n;
    a.q_inj = in_d[1].as<double>() + (size_t)first * net.n;
    a.vm_set = in_d[2].as<double>() + (size_t)first * net.n;
    a.v_out = v_d.as<double>() + (size_t)first * vrow;
    a.newton_iters = iters_d.as<int32_t>() + first;
    a.gmres_iters = nullptr;
    a.converged = conv_d.as<uint8_t>() + first;
    a.final_mismatch = mis_d.as<double>() + first;
    a.work_bytes = nullptr;
    a.tol = opts.tol;
    a.diverge = opts.diverge;
    a.rtol = opts.gmres_rtol;
    a.max_newton = opts.max_newton;
    a.restart = opts.gmres_restart;
    a.max_restarts = opts.gmres_max_restarts;
    a.ws_d = ws_d.as<double>() + (size_t)first * ws_stride;
    a.ws_d_stride = ws_stride;
    a.ws_basis = ws_b.as<char>() + (size_t)first * wb_stride * (mixed ? 4 : 8);
    a.ws_b_stride = wb_stride;
    launch_nr(net, mixed, a, s);
  } else {
    DistNetwork& net = *dist;
    vrow = 2 * net.n_node;
    ZbusLaunch a{};
    a.batch = n;
    a.ld = net.n_node;
    a.s_wye = in_d[0].as<double>() + (size_t)first * row;
    a.s_delta = in_d[1].as<double>() + (size_t)first * row;
    a.v_out = v_d.as<double>() + (size_t)first * vrow;
    a.iters = iters_d.as<int32_t>() + first;
    a.converged = conv_d.as<uint8_t>() + first;
    a.final_mismatch = mis_d.as<double>() + first;
    a.sum_abs_change = nullptr;
    a.tol = opts.tol;
    a.max_iter = opts.zbus_max_iter;
    a.sparse = opts.zbus_sparse;
    a.v = ws_d.as<double>() + (size_t)first * net.Kp;
    a.r = wk.r.as<void>();
    a.st = st_d.as<double>() + (size_t)first * 3;
    a.active = act_d.as<int32_t>() + first;
    a.count = wk.count.as<int32_t>();
    a.count_host = wk.count_host;
    run_zbus(net, mixed, a, s);
  }
  PFX_HIP(hipMemcpyAsync(v_h + (size_t)first * vrow, v_d.as<double>() + (size_t)first * vrow,
                         sizeof(double) * (size_t)n * vrow, hipMemcpyDeviceToHost, s));
  PFX_HIP(hipMemcpyAsync(iters_h + first, iters_d.as<int32_t>() + first, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
  PFX_HIP(hipMemcpyAsync(conv_h + first, conv_d.as<uint8_t>() + first, (size_t)n, hipMemcpyDeviceToHost, s));
  PFX_HIP(hipMemcpyAsync(mis_h + first, mis_d.as<double>() + first, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  PFX_HIP(hipStreamSynchronize(s));
}

void Engine::worker_loop(int wi) {
  (void)hipSetDevice(ctx->device);
  Worker& wk = workers[wi];
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || wk.has_job; });
    if (stop) return;
    Job job = wk.job;
    wk.has_job = false;
    lk.unlock();
    std::string err;
    try {
      run_job(wk, job);
    } catch (const std::exception& e) {
      err = e.what();
    }
    lk.lock();
    const size_t vrow = kind == 0 ? 2 * (size_t)tx->n : 2 * (size_t)dist->n_node;
    for (int64_t id : job.ids) {
      Request& r = reqs[id];
      r.error = err;
      const size_t f = r.first;
      r.v.assign(v_h + f * vrow, v_h + (f + r.n) * vrow);
      r.iters.assign(iters_h + f, iters_h + f + r.n);
      r.conv.assign(conv_h + f, conv_h + f + r.n);
      r.mismatch.assign(mis_h + f, mis_h + f + r.n);
      for (int q = 0; q < r.n; ++q) used[f + q] = 0;
      r.done = true;
      r.t_done = now();
      r.first = -1;
      for (auto& in : r.in) std::vector<double>().swap(in);
      completed.push_back(id);
    }
    ++n_jobs;
    n_scen += job.n;
    --in_flight;
    wk.busy = false;
    cv_dispatch.notify_all();
    cv_done.notify_all();
  }
}

void engine_destroy(Engine* e) { delete e; }

void* engine_network(const Engine* e) { return e->kind == 0 ? (void*)e->tx : (void*)e->dist; }

Context* engine_context(const Engine* e) { return e->ctx; }

void engine_submit(Engine* e, int64_t id, int n, const double* in0, const double* in1, const double* in2) {
  require(n >= 1, "a request needs at least one scenario");
  if (n > e->max_slots)
    fail(PF_NOT_ADMITTED, "request of " + std::to_string(n) + " scenarios exceeds the engine's " +
                              std::to_string(e->max_slots) + " slots");
  const double* ins[3] = {in0, in1, in2};
  Request r;
  r.id = id;
  r.n = n;
  r.t_submit = e->now();
  for (int i = 0; i < e->n_in; ++i) {
    require(ins[i] != nullptr, "null input array");
    r.in[i].assign(ins[i], ins[i] + (size_t)n * e->row);
  }
  {
    std::lock_guard<std::mutex> lk(e->mu);
    require(!e->reqs.count(id), "request id already in use");
    e->reqs.emplace(id, std::move(r));
    e->pending.push_back(id);
  }
  e->cv_dispatch.notify_all();
}

int engine_poll(Engine* e, int max, int64_t* ids, double timeout_s) {
  std::unique_lock<std::mutex> lk(e->mu);
  if (timeout_s > 0 && e->completed.empty())
    e->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !e->completed.empty(); });
  int k = 0;
  while (k < max && !e->completed.empty()) {
    ids[k++] = e->completed.front();
    e->completed.pop_front();
  }
  return k;
}

int engine_request_size(Engine* e, int64_t id) {
  std::lock_guard<std::mutex> lk(e->mu);
  auto it = e->reqs.find(id);
  return it == e->reqs.end() ? -1 : it->second.n;
}

void engine_fetch(Engine* e, int64_t id, double* v_out, int32_t* iters, uint8_t* conv, double* mismatch,
                  double* times) {
  std::lock_guard<std::mutex> lk(e->mu);
  auto it = e->reqs.find(id);
  require(it != e->reqs.end(), "unknown request id");
  Request& r = it->second;
  require(r.done, "request not finished");
  if (!r.error.empty()) {
    const std::string msg = r.error;
    e->reqs.erase(it);
    fail(PF_HIP_ERROR, "request failed: " + msg);
  }
  if (v_out) std::memcpy(v_out, r.v.data(), sizeof(double) * r.v.size());
  if (iters) std::memcpy(iters, r.iters.data(), 4 * r.iters.size());
  if (conv) std::memcpy(conv, r.conv.data(), r.conv.size());
  if (mismatch) std::memcpy(mismatch, r.mismatch.data(), 8 * r.mismatch.size());
  if (times) {
    times[0] = r.t_submit;
    times[1] = r.t_launch;
    times[2] = r.t_done;
  }
  e->reqs.erase(it);
}

void engine_info(Engine* e, int32_t* max_slots, uint64_t* slot_bytes, int32_t* queued, int32_t* in_flight,
                 uint64_t* jobs, uint64_t* scenarios) {
  std::lock_guard<std::mutex> lk(e->mu);
  if (max_slots) *max_slots = e->max_slots;
  if (slot_bytes) *slot_bytes = e->per_slot;
  if (queued) *queued = (int32_t)e->pending.size();
  if (in_flight) *in_flight = e->in_flight;
  if (jobs) *jobs = e->n_jobs;
  if (scenarios) *scenarios = e->n_scen;
}

}  // namespace pfx
