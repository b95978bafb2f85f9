// Serving engine: step-level continuous batching of power-flow scenarios on
// one network.
//
// An engine owns device memory for `max_slots` scenarios (inputs, outputs,
// solver state and workspace; the slot count follows from an HBM byte
// budget).  A step advances every scenario in the engine's occupied slots by
// at most a given number of Newton updates (transmission) or fixed-point
// iterations (feeder) in one launch over the list of those slots.  A scenario
// resumes exactly where its previous step left it, since its whole state
// lives in its slot, so its arithmetic, and its result bit for bit, are those
// of one uninterrupted solve, whatever else shares the steps.  Between steps
// the scenarios that finished are harvested (results copied out, slots freed)
// and waiting scenarios are admitted into any free slots.
//
// Two ways to drive an engine:
//  * caller-driven (created with n_streams = 0): pf_engine_admit places
//    scenarios into chosen free slots, pf_engine_step runs one step on the
//    caller's stream and returns the slots that finished, pf_engine_harvest
//    copies their results out and frees them;
//  * request-driven (n_streams >= 1): requests are queued by
//    pf_engine_submit; each of n_streams cohorts (a HIP stream and a host
//    thread) loops over admit -> step -> harvest; all scenarios of a request
//    join one cohort, and the request is reported by pf_engine_poll once its
//    last scenario is harvested.  Admission takes requests in arrival order
//    into any free slots; a request that does not fit yet may be passed by
//    later ones a bounded number of times.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"
#include "dist.hpp"
#include "engine.hpp"
#include "tx.hpp"

namespace pfx {

namespace {

// How many times the oldest waiting request may be passed by later ones
// before admission waits for it.
constexpr int kMaxBypass = 8;

// Recycled host buffers for requests' results.  A large request's first
// touch of fresh pages costs more than copying its data (about 0.5 ms per MB
// against 0.1), and submit runs on the caller's thread, so buffers released
// by fetched requests are kept (up to kPoolBytes) and handed out again, the
// closest capacity that fits (if not over four times the size asked for).
// Inputs are not copied at submission at all: admission reads them from the
// caller's arrays straight into the pinned slot rows.
constexpr size_t kPoolBytes = size_t(2) << 30;

class BufferPool {
 public:
  std::vector<double> get(size_t n) {
    std::vector<double> v;
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = free_.lower_bound(n);
      if (it != free_.end() && it->first <= 4 * n + 65536) {   // a small request leaves big buffers alone
        v = std::move(it->second);
        bytes_ -= it->first * sizeof(double);
        free_.erase(it);
      }
    }
    v.resize(n);  // within the capacity: no new pages (a grown tail is zeroed)
    return v;
  }
  void put(std::vector<double>& v) {
    const size_t cap = v.capacity();
    if (cap == 0) return;
    std::lock_guard<std::mutex> lk(mu_);
    if (bytes_ + cap * sizeof(double) > kPoolBytes) {
      std::vector<double>().swap(v);
      return;
    }
    bytes_ += cap * sizeof(double);
    free_.emplace(cap, std::move(v));
    v = std::vector<double>();
  }

 private:
  std::mutex mu_;
  std::multimap<size_t, std::vector<double>> free_;   // by capacity
  size_t bytes_ = 0;
};

struct Request {
  int64_t id = 0;
  int n = 0;
  const double* in[3] = {nullptr, nullptr, nullptr};   // the caller's inputs, read at admission
  int left = 0;        // scenarios not yet harvested
  int bypassed = 0;
  bool admitted = false;
  bool done = false;
  std::string error;
  std::vector<double> v;          // complex interleaved, n rows
  std::vector<int32_t> iters;
  std::vector<uint8_t> conv;
  std::vector<double> mismatch;
  double t_submit = 0, t_launch = 0, t_done = 0;   // seconds since the engine was created
};

// A stream with the scenarios it steps.  In a caller-driven engine the one
// cohort runs on the stream each call names.
struct Cohort {
  hipStream_t stream = nullptr;
  std::thread th;
  std::vector<int> active;   // occupied slots still iterating, in admission order
  std::vector<int> fresh;    // admitted since the last step
  DeviceBuffer list_d, fresh_d, harv_d, done_d, r;   // r: feeder residual rows
  int32_t* list_h = nullptr;
  int32_t* fresh_h = nullptr;
  int32_t* harv_h = nullptr;
  uint8_t* done_h = nullptr;
};

template <typename T>
T* host_alloc(size_t count) {
  void* p = nullptr;
  PFX_HIP(hipHostMalloc(&p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault));
  std::memset(p, 0, std::max<size_t>(count, 1) * sizeof(T));
  return static_cast<T*>(p);
}

uint64_t tx_slot_bytes(const TxNetwork& net, bool mixed, int R) {
  const uint64_t n = net.n;
  return 8ull * (3 * n + 2 * n)            // p, q, vm in; v out
         + 4 + 1 + 8                       // iterations, flag, mismatch
         + sizeof(NrSlotState)             // resumable Newton state
         + 8ull * nr_ws_doubles(net)       // FP64 workspace
         + (uint64_t)(R + 1) * nr_padded_rows(net) * (mixed ? 4 : 8);  // Krylov basis
}

uint64_t dist_row_bytes(const DistNetwork& net, bool mixed) { return (uint64_t)net.Kp * (mixed ? 4 : 8); }

uint64_t dist_slot_bytes(const DistNetwork& net, bool mixed) {
  const uint64_t nn = net.n_node;
  return 16ull * (3 * nn)                  // s_wye, s_delta in; v out
         + 4 + 1 + 8                       // iterations, flag, mismatch
         + 8ull * net.Kp + 3 * 8 + 4       // state, statistics, active flag
         + dist_row_bytes(net, mixed);     // one cohort's residual row
}

// Calls f(first, count) for each run of consecutive values of sorted `s`,
// all of which must lie in [0, limit).
template <typename F>
void for_runs(const std::vector<int>& s, int limit, F&& f) {
  size_t i = 0;
  while (i < s.size()) {
    size_t j = i + 1;
    while (j < s.size() && s[j] == s[j - 1] + 1) ++j;
    if (s[i] < 0 || s[j - 1] >= limit) fail(PF_INVALID_ARG, "slot outside the engine");
    f(s[i], (int)(j - i));
    i = j;
  }
}

}  // namespace

struct Engine {
  Context* ctx = nullptr;
  int kind = 0;               // 0 transmission, 1 feeder
  TxNetwork* tx = nullptr;
  DistNetwork* dist = nullptr;
  pf_opts opts{};
  bool mixed = false;
  bool driven = false;        // request-driven (own cohorts and threads)
  int row = 0;                // reals per scenario row of an input (n_bus, or 2 n_node for complex)
  int vrow = 0;               // reals per scenario row of the output
  int n_in = 0;
  int max_slots = 0;
  uint64_t per_slot = 0;
  // slot-indexed device buffers
  DeviceBuffer in_d[3], v_d, iters_d, conv_d, mis_d, ws_d, ws_b, state_d, st_d, act_d;
  int64_t ws_stride = 0, wb_stride = 0;
  // slot-indexed pinned host staging
  double* in_h[3] = {nullptr, nullptr, nullptr};
  double* v_h = nullptr;
  double* mis_h = nullptr;
  int32_t* iters_h = nullptr;
  uint8_t* conv_h = nullptr;
  NrSlotState* zero_state_h = nullptr;
  // slot bookkeeping (under mu): 0 free, 1 iterating, 2 finished and not yet harvested
  std::vector<int8_t> slot_st;
  std::vector<int64_t> slot_req;
  std::vector<int> slot_idx;
  std::set<int> free_slots;
  std::vector<Cohort> cohorts;
  std::mutex mu;
  std::mutex drive_mu;         // caller-driven calls, one at a time
  std::condition_variable cv_work, cv_done;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  std::deque<int64_t> pending;
  std::map<int64_t, Request> reqs;
  std::deque<int64_t> completed;
  BufferPool pool;             // request results (own lock)
  bool stop = false;
  uint64_t n_steps = 0, n_scen = 0;

  ~Engine();
  void stage_in(Cohort& c, std::vector<int> slots, hipStream_t s);
  std::vector<int> step(Cohort& c, int iters, hipStream_t s);
  void collect(Cohort& c, std::vector<int> slots, hipStream_t s);
  bool can_admit() const;
  std::vector<int> admit_pending(std::vector<std::pair<const Request*, int>>& copies);
  void stage_rows(const std::vector<int>& slots, const std::vector<std::pair<const Request*, int>>& copies);
  void hand_over(const std::vector<int>& slots);
  void complete(const std::vector<int>& slots, const std::string& err);
  void cohort_loop(int ci);
  int occupied() const { return max_slots - (int)free_slots.size(); }
};

uint64_t engine_slot_bytes(int kind, void* net, const pf_opts& o) {
  const bool mixed = o.precision == PF_MIXED;
  if (kind == 0) return tx_slot_bytes(*static_cast<TxNetwork*>(net), mixed, o.gmres_restart);
  return dist_slot_bytes(*static_cast<DistNetwork*>(net), mixed);
}

Engine* engine_create(Context* ctx, int kind, void* network, uint64_t hbm_bytes, int n_streams,
                      const pf_opts& o) {
  require(kind == 0 || kind == 1, "kind must be 0 (transmission) or 1 (feeder)");
  require(n_streams >= 0 && n_streams <= 8, "n_streams must be 0..8");
  auto e = std::make_unique<Engine>();
  e->ctx = ctx;
  e->kind = kind;
  e->opts = o;
  e->mixed = o.precision == PF_MIXED;
  e->driven = n_streams > 0;
  const int n_cohorts = std::max(1, n_streams);
  e->per_slot = engine_slot_bytes(kind, network, o);
  // every cohort beyond the first needs its own feeder residual row per slot
  const uint64_t extra = kind == 1 ? (uint64_t)(n_cohorts - 1) *
                                         dist_row_bytes(*static_cast<DistNetwork*>(network), e->mixed)
                                   : 0;
  e->max_slots = (int)std::min<uint64_t>(hbm_bytes / (e->per_slot + extra), 1u << 20);
  require(e->max_slots >= 1, "HBM budget below one scenario's footprint (" + std::to_string(e->per_slot) + " bytes)");
  const size_t S = e->max_slots;
  if (kind == 0) {
    e->tx = static_cast<TxNetwork*>(network);
    const TxNetwork& net = *e->tx;
    e->row = net.n;
    e->vrow = 2 * net.n;
    e->n_in = 3;
    for (int i = 0; i < 3; ++i) e->in_d[i].allocate(ctx, S * net.n * 8);
    e->v_d.allocate(ctx, S * net.n * 16);
    e->ws_stride = nr_ws_doubles(net);
    e->wb_stride = (int64_t)(o.gmres_restart + 1) * nr_padded_rows(net);
    e->ws_d.allocate(ctx, S * e->ws_stride * 8);
    e->ws_b.allocate(ctx, S * e->wb_stride * (e->mixed ? 4 : 8));
    e->state_d.allocate(ctx, S * sizeof(NrSlotState));
    e->zero_state_h = host_alloc<NrSlotState>(S);
  } else {
    e->dist = static_cast<DistNetwork*>(network);
    const DistNetwork& net = *e->dist;
    e->row = 2 * net.n_node;
    e->vrow = 2 * net.n_node;
    e->n_in = 2;
    for (int i = 0; i < 2; ++i) e->in_d[i].allocate(ctx, S * net.n_node * 16);
    e->v_d.allocate(ctx, S * net.n_node * 16);
    e->ws_d.allocate(ctx, S * net.Kp * 8);
    e->st_d.allocate(ctx, S * 3 * 8);
    e->act_d.allocate(ctx, S * 4);
  }
  e->iters_d.allocate(ctx, S * 4);
  e->conv_d.allocate(ctx, S);
  e->mis_d.allocate(ctx, S * 8);
  for (int i = 0; i < e->n_in; ++i) e->in_h[i] = host_alloc<double>(S * e->row);
  e->v_h = host_alloc<double>(S * e->vrow);
  e->mis_h = host_alloc<double>(S);
  e->iters_h = host_alloc<int32_t>(S);
  e->conv_h = host_alloc<uint8_t>(S);
  e->slot_st.assign(S, 0);
  e->slot_req.assign(S, -1);
  e->slot_idx.assign(S, 0);
  for (int s = 0; s < (int)S; ++s) e->free_slots.insert(e->free_slots.end(), s);
  e->cohorts.resize(n_cohorts);
  for (auto& c : e->cohorts) {
    if (e->driven) PFX_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    c.list_d.allocate(ctx, S * 4);
    c.fresh_d.allocate(ctx, S * 4);
    c.harv_d.allocate(ctx, S * 4);
    c.done_d.allocate(ctx, S);
    c.list_h = host_alloc<int32_t>(S);
    c.fresh_h = host_alloc<int32_t>(S);
    c.harv_h = host_alloc<int32_t>(S);
    c.done_h = host_alloc<uint8_t>(S);
    if (kind == 1) {
      // rows of the step's residual by list position, padded to the GEMM's
      // row tile; padding columns must read as zeros
      const size_t rows = (S + ZB_BM - 1) / ZB_BM * ZB_BM;
      c.r.allocate(ctx, rows * e->dist->Kp * (e->mixed ? 4 : 8));
      PFX_HIP(hipMemset(c.r.as<void>(), 0, c.r.bytes()));
    }
  }
  Engine* raw = e.get();
  if (raw->driven)
    for (int i = 0; i < n_cohorts; ++i) raw->cohorts[i].th = std::thread([raw, i] { raw->cohort_loop(i); });
  return e.release();
}

Engine::~Engine() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_work.notify_all();
  for (auto& c : cohorts)
    if (c.th.joinable()) c.th.join();
  for (auto& c : cohorts) {
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    if (c.stream) (void)hipStreamDestroy(c.stream);
    for (void* p : {(void*)c.list_h, (void*)c.fresh_h, (void*)c.harv_h, (void*)c.done_h})
      if (p) (void)hipHostFree(p);
  }
  for (auto* p : in_h)
    if (p) (void)hipHostFree(p);
  for (void* p : {(void*)v_h, (void*)mis_h, (void*)iters_h, (void*)conv_h, (void*)zero_state_h})
    if (p) (void)hipHostFree(p);
}

// Copies the inputs of newly occupied slots (already in the pinned staging
// rows) to the device and adds the slots to the cohort.
void Engine::stage_in(Cohort& c, std::vector<int> slots, hipStream_t s) {
  if (slots.empty()) return;
  std::sort(slots.begin(), slots.end());
  for_runs(slots, max_slots, [&](int first, int cnt) {
    for (int i = 0; i < n_in; ++i)
      PFX_HIP(hipMemcpyAsync(in_d[i].as<double>() + (size_t)first * row, in_h[i] + (size_t)first * row,
                             sizeof(double) * (size_t)cnt * row, hipMemcpyHostToDevice, s));
    if (kind == 0)
      PFX_HIP(hipMemcpyAsync(state_d.as<NrSlotState>() + first, zero_state_h + first,
                             sizeof(NrSlotState) * (size_t)cnt, hipMemcpyHostToDevice, s));
  });
  c.active.insert(c.active.end(), slots.begin(), slots.end());
  c.fresh.insert(c.fresh.end(), slots.begin(), slots.end());
}

// One step over the cohort's occupied slots; returns the slots that finished
// (removed from the cohort).  Waits for the stream.
std::vector<int> Engine::step(Cohort& c, int iters, hipStream_t s) {
  const int n = (int)c.active.size();
  if (n == 0) return {};
  std::copy(c.active.begin(), c.active.end(), c.list_h);
  PFX_HIP(hipMemcpyAsync(c.list_d.as<int32_t>(), c.list_h, 4 * (size_t)n, hipMemcpyHostToDevice, s));
  if (kind == 0) {
    const TxNetwork& net = *tx;
    NRLaunch a{};
    a.batch = n;
    a.ld = net.n;
    a.p_inj = in_d[0].as<double>();
    a.q_inj = in_d[1].as<double>();
    a.vm_set = in_d[2].as<double>();
    a.v_out = v_d.as<double>();
    a.newton_iters = iters_d.as<int32_t>();
    a.converged = conv_d.as<uint8_t>();
    a.final_mismatch = mis_d.as<double>();
    a.tol = opts.tol;
    a.diverge = opts.diverge;
    a.rtol = opts.gmres_rtol;
    a.forcing = opts.forcing;
    a.forcing_max = opts.forcing_max;
    a.max_newton = opts.max_newton;
    a.restart = opts.gmres_restart;
    a.max_restarts = opts.gmres_max_restarts;
    a.ws_d = ws_d.as<double>();
    a.ws_d_stride = ws_stride;
    a.ws_basis = ws_b.as<void>();
    a.ws_b_stride = wb_stride;
    a.slots = c.list_d.as<int32_t>();
    a.state = state_d.as<NrSlotState>();
    a.step_iters = iters;
    a.step_done = c.done_d.as<uint8_t>();
    launch_nr(net, mixed, a, s);
  } else {
    DistNetwork& net = *dist;
    ZbusLaunch a{};
    a.ld = net.n_node;
    a.s_wye = in_d[0].as<double>();
    a.s_delta = in_d[1].as<double>();
    a.v_out = v_d.as<double>();
    a.iters = iters_d.as<int32_t>();
    a.converged = conv_d.as<uint8_t>();
    a.final_mismatch = mis_d.as<double>();
    a.tol = opts.tol;
    a.max_iter = opts.zbus_max_iter;
    a.sparse = opts.zbus_sparse;
    a.v = ws_d.as<double>();
    a.r = c.r.as<void>();
    a.st = st_d.as<double>();
    a.active = act_d.as<int32_t>();
    if (!c.fresh.empty()) {
      std::copy(c.fresh.begin(), c.fresh.end(), c.fresh_h);
      PFX_HIP(hipMemcpyAsync(c.fresh_d.as<int32_t>(), c.fresh_h, 4 * c.fresh.size(), hipMemcpyHostToDevice, s));
      a.batch = (int)c.fresh.size();
      a.slots = c.fresh_d.as<int32_t>();
      zbus_init_slots(net, a, s);
    }
    a.batch = n;
    a.slots = c.list_d.as<int32_t>();
    a.step_done = c.done_d.as<uint8_t>();
    zbus_step(net, mixed, a, iters, s);
  }
  c.fresh.clear();
  PFX_HIP(hipMemcpyAsync(c.done_h, c.done_d.as<uint8_t>(), (size_t)n, hipMemcpyDeviceToHost, s));
  PFX_HIP(hipStreamSynchronize(s));
  std::vector<int> done, keep;
  keep.reserve(n);
  for (int g = 0; g < n; ++g) (c.done_h[g] ? done : keep).push_back(c.active[g]);
  c.active.swap(keep);
  return done;
}

// Copies the results of finished slots into the pinned staging rows.  Waits
// for the stream.
void Engine::collect(Cohort& c, std::vector<int> slots, hipStream_t s) {
  if (slots.empty()) return;
  std::sort(slots.begin(), slots.end());
  if (kind == 1) {
    DistNetwork& net = *dist;
    std::copy(slots.begin(), slots.end(), c.harv_h);
    PFX_HIP(hipMemcpyAsync(c.harv_d.as<int32_t>(), c.harv_h, 4 * slots.size(), hipMemcpyHostToDevice, s));
    ZbusLaunch a{};
    a.batch = (int)slots.size();
    a.ld = net.n_node;
    a.v_out = v_d.as<double>();
    a.final_mismatch = mis_d.as<double>();
    a.v = ws_d.as<double>();
    a.st = st_d.as<double>();
    a.slots = c.harv_d.as<int32_t>();
    zbus_finish_slots(net, a, s);
  }
  for_runs(slots, max_slots, [&](int first, int cnt) {
    PFX_HIP(hipMemcpyAsync(v_h + (size_t)first * vrow, v_d.as<double>() + (size_t)first * vrow,
                           sizeof(double) * (size_t)cnt * vrow, hipMemcpyDeviceToHost, s));
    PFX_HIP(hipMemcpyAsync(iters_h + first, iters_d.as<int32_t>() + first, 4 * (size_t)cnt,
                           hipMemcpyDeviceToHost, s));
    PFX_HIP(hipMemcpyAsync(conv_h + first, conv_d.as<uint8_t>() + first, (size_t)cnt, hipMemcpyDeviceToHost, s));
    PFX_HIP(hipMemcpyAsync(mis_h + first, mis_d.as<double>() + first, 8 * (size_t)cnt, hipMemcpyDeviceToHost, s));
  });
  PFX_HIP(hipStreamSynchronize(s));
}

// --------------------------------------------------------- request-driven

bool Engine::can_admit() const {
  if (pending.empty() || free_slots.empty()) return false;
  const int nfree = (int)free_slots.size();
  const Request& head = reqs.at(pending.front());
  if (head.n <= nfree) return true;
  if (head.bypassed >= kMaxBypass) return false;
  for (int64_t id : pending)
    if (reqs.at(id).n <= nfree) return true;
  return false;
}

// Under mu: takes waiting requests, in order, into free slots (lowest first).
// Returns the slots taken and, for each, the request and scenario whose
// inputs stage_rows copies into the slot's pinned row.
std::vector<int> Engine::admit_pending(std::vector<std::pair<const Request*, int>>& copies) {
  std::vector<int> taken;
  copies.clear();
  auto it = pending.begin();
  while (it != pending.end() && !free_slots.empty()) {
    Request& r = reqs.at(*it);
    const bool head = it == pending.begin();
    if (r.n > (int)free_slots.size()) {
      if (head && r.bypassed >= kMaxBypass) break;
      ++it;
      continue;
    }
    if (!head) {
      Request& h = reqs.at(pending.front());
      if (h.bypassed >= kMaxBypass) break;
      ++h.bypassed;
    }
    r.admitted = true;
    r.t_launch = now();
    for (int q = 0; q < r.n; ++q) {
      const int s = *free_slots.begin();
      free_slots.erase(free_slots.begin());
      slot_st[s] = 1;
      slot_req[s] = r.id;
      slot_idx[s] = q;
      copies.emplace_back(&r, q);
      taken.push_back(s);
    }
    it = pending.erase(it);
  }
  return taken;
}

// Without mu: the admitted scenarios' inputs, from the callers' arrays into
// the slots' pinned rows.  The slots and their rows are this cohort's alone,
// and a request stays in the table (its entry does not move) until fetched,
// which cannot happen before its scenarios finish.
void Engine::stage_rows(const std::vector<int>& slots,
                        const std::vector<std::pair<const Request*, int>>& copies) {
  for (size_t k = 0; k < slots.size(); ++k) {
    const Request& r = *copies[k].first;
    const int q = copies[k].second, s = slots[k];
    for (int i = 0; i < n_in; ++i)
      std::memcpy(in_h[i] + (size_t)s * row, r.in[i] + (size_t)q * row, sizeof(double) * row);
  }
}

// Without mu: the harvested slots' results (pinned rows) into their
// requests.  The slots are still occupied, so their rows and the requests'
// entries stay put; slot_req and slot_idx of an occupied slot change only
// under this cohort's own control.
void Engine::hand_over(const std::vector<int>& slots) {
  std::vector<std::pair<Request*, int>> to;
  {
    std::lock_guard<std::mutex> lk(mu);
    to.reserve(slots.size());
    for (int s : slots) to.emplace_back(&reqs.at(slot_req[s]), slot_idx[s]);
  }
  for (size_t k = 0; k < slots.size(); ++k) {
    Request& r = *to[k].first;
    const int q = to[k].second, s = slots[k];
    std::memcpy(r.v.data() + (size_t)q * vrow, v_h + (size_t)s * vrow, sizeof(double) * vrow);
    r.iters[q] = iters_h[s];
    r.conv[q] = conv_h[s];
    r.mismatch[q] = mis_h[s];
  }
}

// Under mu: frees the harvested slots (their results already handed over,
// unless the step failed) and completes requests whose last scenario this
// was.
void Engine::complete(const std::vector<int>& slots, const std::string& err) {
  const double t = now();
  for (int s : slots) {
    Request& r = reqs.at(slot_req[s]);
    if (!err.empty() && r.error.empty()) r.error = err;
    slot_st[s] = 0;
    slot_req[s] = -1;
    free_slots.insert(s);
    if (--r.left == 0) {
      r.done = true;
      r.t_done = t;
      completed.push_back(r.id);
    }
  }
  n_scen += slots.size();
}

void Engine::cohort_loop(int ci) {
  (void)hipSetDevice(ctx->device);
  Cohort& c = cohorts[ci];
  for (;;) {
    std::vector<int> admitted;
    std::vector<std::pair<const Request*, int>> copies;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !c.active.empty() || can_admit(); });
      if (stop) return;
      admitted = admit_pending(copies);
    }
    std::vector<int> done;
    std::string err;
    try {
      // the large host copies run outside the lock, so submissions and the
      // other cohorts' admissions never wait for them
      stage_rows(admitted, copies);
      stage_in(c, admitted, c.stream);
      done = step(c, opts.step_iters, c.stream);
      collect(c, done, c.stream);
      hand_over(done);
    } catch (const std::exception& e) {
      // a failed step fails every request with a scenario in this cohort
      // (admitted slots included, whether or not staging got to add them)
      err = e.what();
      (void)hipStreamSynchronize(c.stream);
      std::vector<int> all(c.active);
      all.insert(all.end(), admitted.begin(), admitted.end());
      all.insert(all.end(), done.begin(), done.end());
      std::sort(all.begin(), all.end());
      all.erase(std::unique(all.begin(), all.end()), all.end());
      done.swap(all);
      c.active.clear();
      c.fresh.clear();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      complete(done, err);
      ++n_steps;
    }
    if (!done.empty()) {
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
}

void engine_destroy(Engine* e) { delete e; }

void* engine_network(const Engine* e) { return e->kind == 0 ? (void*)e->tx : (void*)e->dist; }

Context* engine_context(const Engine* e) { return e->ctx; }

void engine_submit(Engine* e, int64_t id, int n, const double* in0, const double* in1, const double* in2) {
  require(e->driven, "pf_engine_submit needs a request-driven engine (n_streams >= 1)");
  require(n >= 1, "a request needs at least one scenario");
  if (n > e->max_slots)
    fail(PF_NOT_ADMITTED, "request of " + std::to_string(n) + " scenarios exceeds the engine's " +
                              std::to_string(e->max_slots) + " slots");
  const double* ins[3] = {in0, in1, in2};
  Request r;
  r.id = id;
  r.n = n;
  r.left = n;
  r.t_submit = e->now();
  for (int i = 0; i < e->n_in; ++i) {
    require(ins[i] != nullptr, "null input array");
    r.in[i] = ins[i];
  }
  r.v = e->pool.get((size_t)n * e->vrow);   // every row is written when its scenario is harvested
  r.iters.assign(n, 0);
  r.conv.assign(n, 0);
  r.mismatch.assign(n, 0.0);
  {
    std::lock_guard<std::mutex> lk(e->mu);
    require(!e->reqs.count(id), "request id already in use");
    e->reqs.emplace(id, std::move(r));
    e->pending.push_back(id);
  }
  e->cv_work.notify_all();
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
  // The request leaves the table under the lock; its results are copied out
  // after, so a large copy does not hold up the cohorts' admissions.
  Request r;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->reqs.find(id);
    require(it != e->reqs.end(), "unknown request id");
    require(it->second.done, "request not finished");
    r = std::move(it->second);
    e->reqs.erase(it);
  }
  if (!r.error.empty()) {
    e->pool.put(r.v);
    fail(PF_HIP_ERROR, "request failed: " + r.error);
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
  e->pool.put(r.v);
}

void engine_info(Engine* e, int32_t* max_slots, uint64_t* slot_bytes, int32_t* queued, int32_t* occupied,
                 uint64_t* steps, uint64_t* scenarios) {
  std::lock_guard<std::mutex> lk(e->mu);
  if (max_slots) *max_slots = e->max_slots;
  if (slot_bytes) *slot_bytes = e->per_slot;
  if (queued) *queued = (int32_t)e->pending.size();
  if (occupied) *occupied = e->occupied();
  if (steps) *steps = e->n_steps;
  if (scenarios) *scenarios = e->n_scen;
}

// ---------------------------------------------------------- caller-driven

void engine_admit(Engine* e, int n, const int32_t* slots, const double* in0, const double* in1,
                  const double* in2, hipStream_t s) {
  require(!e->driven, "pf_engine_admit needs a caller-driven engine (n_streams = 0)");
  require(n >= 0, "n must be >= 0");
  if (n == 0) return;
  require(slots != nullptr, "null slot list");
  const double* ins[3] = {in0, in1, in2};
  for (int i = 0; i < e->n_in; ++i) require(ins[i] != nullptr, "null input array");
  std::lock_guard<std::mutex> dl(e->drive_mu);
  std::vector<int> v(slots, slots + n);
  {
    std::lock_guard<std::mutex> lk(e->mu);
    std::set<int> seen;
    for (int sl : v) {
      require(sl >= 0 && sl < e->max_slots, "slot " + std::to_string(sl) + " out of range");
      require(e->slot_st[sl] == 0, "slot " + std::to_string(sl) + " is occupied");
      require(seen.insert(sl).second, "slot " + std::to_string(sl) + " listed twice");
    }
    for (int q = 0; q < n; ++q) {
      const int sl = v[q];
      e->slot_st[sl] = 1;
      e->free_slots.erase(sl);
      for (int i = 0; i < e->n_in; ++i)
        std::memcpy(e->in_h[i] + (size_t)sl * e->row, ins[i] + (size_t)q * e->row, sizeof(double) * e->row);
    }
  }
  e->stage_in(e->cohorts[0], v, s);
}

int engine_step(Engine* e, int iters, int max_done, int32_t* done_slots, int32_t* n_active, hipStream_t s) {
  require(!e->driven, "pf_engine_step needs a caller-driven engine (n_streams = 0)");
  require(iters >= 1, "iters must be >= 1");
  require(max_done >= 0 && (max_done == 0 || done_slots != nullptr), "bad done-slot output");
  std::lock_guard<std::mutex> dl(e->drive_mu);
  Cohort& c = e->cohorts[0];
  require((int)c.active.size() <= max_done || max_done >= e->max_slots,
          "max_done must be at least the number of occupied, unfinished slots (" +
              std::to_string(c.active.size()) + ")");
  const std::vector<int> done = e->step(c, iters, s);
  {
    std::lock_guard<std::mutex> lk(e->mu);
    for (int sl : done) e->slot_st[sl] = 2;
    ++e->n_steps;
  }
  std::copy(done.begin(), done.end(), done_slots);
  if (n_active) *n_active = (int32_t)c.active.size();
  return (int)done.size();
}

void engine_harvest(Engine* e, int n, const int32_t* slots, double* v_out, int32_t* iters, uint8_t* conv,
                    double* mismatch, hipStream_t s) {
  require(!e->driven, "pf_engine_harvest needs a caller-driven engine (n_streams = 0)");
  require(n >= 0, "n must be >= 0");
  if (n == 0) return;
  require(slots != nullptr, "null slot list");
  std::lock_guard<std::mutex> dl(e->drive_mu);
  std::vector<int> v(slots, slots + n);
  {
    std::lock_guard<std::mutex> lk(e->mu);
    std::set<int> seen;
    for (int sl : v) {
      require(sl >= 0 && sl < e->max_slots, "slot " + std::to_string(sl) + " out of range");
      require(e->slot_st[sl] == 2, "slot " + std::to_string(sl) + " has no finished scenario");
      require(seen.insert(sl).second, "slot " + std::to_string(sl) + " listed twice");
    }
  }
  e->collect(e->cohorts[0], v, s);
  std::lock_guard<std::mutex> lk(e->mu);
  for (int q = 0; q < n; ++q) {
    const int sl = v[q];
    if (v_out) std::memcpy(v_out + (size_t)q * e->vrow, e->v_h + (size_t)sl * e->vrow, sizeof(double) * e->vrow);
    if (iters) iters[q] = e->iters_h[sl];
    if (conv) conv[q] = e->conv_h[sl];
    if (mismatch) mismatch[q] = e->mis_h[sl];
    e->slot_st[sl] = 0;
    e->free_slots.insert(sl);
  }
  e->n_scen += n;
}

}  // namespace pfx
