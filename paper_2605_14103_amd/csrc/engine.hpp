// Serving engine (step-level continuous batching); see engine.cpp.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace pfx {

struct Engine;

// Device bytes one scenario slot costs (inputs, outputs, solver workspace).
uint64_t engine_slot_bytes(int kind, void* network, const pf_opts& o);
Engine* engine_create(Context* ctx, int kind, void* network, uint64_t hbm_bytes, int n_streams,
                      const pf_opts& o);
void engine_destroy(Engine* e);
void* engine_network(const Engine* e);
Context* engine_context(const Engine* e);
// Destroys the engines bound to `network` (all of the context's if null).
void destroy_engines_of(Context* ctx, void* network);
void engine_submit(Engine* e, int64_t id, int n, const double* in0, const double* in1, const double* in2);
int engine_poll(Engine* e, int max, int64_t* ids, double timeout_s);
int engine_request_size(Engine* e, int64_t id);
void engine_fetch(Engine* e, int64_t id, double* v_out, int32_t* iters, uint8_t* conv, double* mismatch,
                  double* times);
void engine_info(Engine* e, int32_t* max_slots, uint64_t* slot_bytes, int32_t* queued, int32_t* occupied,
                 uint64_t* steps, uint64_t* scenarios);
// Caller-driven engines (n_streams = 0).
void engine_admit(Engine* e, int n, const int32_t* slots, const double* in0, const double* in1,
                  const double* in2, hipStream_t s);
int engine_step(Engine* e, int iters, int max_done, int32_t* done_slots, int32_t* n_active, hipStream_t s);
void engine_harvest(Engine* e, int n, const int32_t* slots, double* v_out, int32_t* iters, uint8_t* conv,
                    double* mismatch, hipStream_t s);

}  // namespace pfx
