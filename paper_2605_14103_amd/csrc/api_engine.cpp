// C ABI: serving engine.
#include <string>

#include "common.hpp"
#include "dist.hpp"
#include "engine.hpp"
#include "tx.hpp"

using namespace pfx;

namespace {

Engine* engine_of(pf_engine* h) {
  check_handle(h, "engine");
  return reinterpret_cast<Engine*>(h);
}

// Exactly one of the two networks; returns its kind (0 transmission, 1 feeder).
int pick(pf_tx_network* tx, pf_dist_network* dist, void** net) {
  require((tx == nullptr) != (dist == nullptr), "give exactly one of a transmission or a feeder network");
  if (tx) {
    check_handle(tx, "transmission network");
    *net = tx;
    return 0;
  }
  check_handle(dist, "feeder");
  *net = dist;
  return 1;
}

}  // namespace

namespace pfx {

// Destroys every engine bound to `network` (called before a network goes away).
void destroy_engines_of(Context* ctx, void* network) {
  std::set<void*> doomed;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (void* e : ctx->engines)
      if (network == nullptr || engine_network(static_cast<Engine*>(e)) == network) doomed.insert(e);
    for (void* e : doomed) ctx->engines.erase(e);
  }
  for (void* e : doomed) {
    registry().remove(e);
    engine_destroy(static_cast<Engine*>(e));
  }
}

}  // namespace pfx

extern "C" {

pf_status pf_engine_slot_bytes(pf_tx_network* tx, pf_dist_network* dist, const pf_opts* opts,
                               uint64_t* bytes) {
  return guarded([&] {
    require(bytes != nullptr, "bytes must not be null");
    void* net = nullptr;
    const int kind = pick(tx, dist, &net);
    *bytes = engine_slot_bytes(kind, net, resolve_opts(opts));
  });
}

pf_status pf_engine_create(pf_context* c, pf_tx_network* tx, pf_dist_network* dist, uint64_t hbm_bytes,
                           int32_t n_streams, const pf_opts* opts, pf_engine** out) {
  return guarded([&] {
    require(out != nullptr, "out must not be null");
    *out = nullptr;
    check_handle(c, "context");
    auto* ctx = reinterpret_cast<Context*>(c);
    void* net = nullptr;
    const int kind = pick(tx, dist, &net);
    const Context* owner = kind == 0 ? static_cast<TxNetwork*>(net)->ctx : static_cast<DistNetwork*>(net)->ctx;
    require(owner == ctx, "the network belongs to another context");
    activate(ctx);
    const pf_opts o = resolve_opts(opts);
    require(o.nr_direct == 0, "the serving engine runs the GMRES Newton step (nr_direct must be 0)");
    Engine* e = engine_create(ctx, kind, net, hbm_bytes, n_streams, o);
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->engines.insert(e);
    }
    registry().add(e);
    *out = reinterpret_cast<pf_engine*>(e);
  });
}

void pf_engine_destroy(pf_engine* h) {
  if (!registry().has(h)) return;
  auto* e = reinterpret_cast<Engine*>(h);
  Context* ctx = engine_context(e);
  registry().remove(e);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->engines.erase(e);
  }
  engine_destroy(e);
}

pf_status pf_engine_submit(pf_engine* h, int64_t id, int32_t n, const double* in0, const double* in1,
                           const double* in2) {
  return guarded([&] { engine_submit(engine_of(h), id, n, in0, in1, in2); });
}

pf_status pf_engine_poll(pf_engine* h, int32_t max_ids, int64_t* ids, double timeout_s, int32_t* count) {
  return guarded([&] {
    require(count != nullptr && (max_ids == 0 || ids != nullptr), "null output");
    require(max_ids >= 0, "max_ids must be >= 0");
    *count = engine_poll(engine_of(h), max_ids, ids, timeout_s);
  });
}

pf_status pf_engine_request_size(pf_engine* h, int64_t id, int32_t* n) {
  return guarded([&] {
    require(n != nullptr, "null output");
    *n = engine_request_size(engine_of(h), id);
    require(*n >= 0, "unknown request id");
  });
}

pf_status pf_engine_fetch(pf_engine* h, int64_t id, double* v_out, int32_t* iters, uint8_t* converged,
                          double* final_mismatch, double* times) {
  return guarded([&] { engine_fetch(engine_of(h), id, v_out, iters, converged, final_mismatch, times); });
}

pf_status pf_engine_info(pf_engine* h, int32_t* max_slots, uint64_t* slot_bytes, int32_t* queued,
                         int32_t* occupied, uint64_t* steps, uint64_t* scenarios) {
  return guarded([&] { engine_info(engine_of(h), max_slots, slot_bytes, queued, occupied, steps, scenarios); });
}

pf_status pf_engine_admit(pf_engine* h, int32_t n, const int32_t* slot_ids, const double* in0, const double* in1,
                          const double* in2, pf_stream stream) {
  return guarded([&] {
    Engine* e = engine_of(h);
    activate(engine_context(e));
    engine_admit(e, n, slot_ids, in0, in1, in2, reinterpret_cast<hipStream_t>(stream));
  });
}

pf_status pf_engine_step(pf_engine* h, int32_t iters, int32_t max_done, int32_t* done_slots, int32_t* n_done,
                         int32_t* n_active, pf_stream stream) {
  return guarded([&] {
    require(n_done != nullptr, "n_done must not be null");
    *n_done = 0;
    Engine* e = engine_of(h);
    activate(engine_context(e));
    *n_done = engine_step(e, iters, max_done, done_slots, n_active, reinterpret_cast<hipStream_t>(stream));
  });
}

pf_status pf_engine_harvest(pf_engine* h, int32_t n, const int32_t* slot_ids, double* v_out, int32_t* iters,
                            uint8_t* converged, double* final_mismatch, pf_stream stream) {
  return guarded([&] {
    Engine* e = engine_of(h);
    activate(engine_context(e));
    engine_harvest(e, n, slot_ids, v_out, iters, converged, final_mismatch, reinterpret_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
