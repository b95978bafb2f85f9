/*
 * pfx — batched AC power flow on AMD MI355X (gfx950).
 *
 * C ABI of the device library.  Every entry point returns a pf_status; no C++
 * exception crosses this boundary.  The text of the last failure on the
 * calling thread is available from pf_last_error().
 *
 * Method (citations are to the paper "JAX-Based Batched AC Power Flow for GPU
 * Acceleration and AI Ecosystem Integration"):
 *   - transmission grids: Newton-Raphson on the polar state of eq. (1) with the
 *     mismatch of eq. (2) and the update of eq. (3); each Newton system is
 *     solved by restarted GMRES on Jacobian-vector products (Sec. II-A) with the
 *     left preconditioner of eq. (7) applied by the forward block substitution
 *     of eqs. (8)-(9), using (B' + eps I) and (B'' + eps I);
 *   - radial three-phase feeders: the Z-bus fixed point of eq. (10) with wye
 *     and delta constant-power loads (Sec. II-B).
 *
 * Conventions shared by all calls
 *   - Per unit throughout; angles in radians, slack angle 0.
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are read (copied) before the call returns.
 *   - Per-scenario arrays are scenario-major: element (b, i) of a real array is
 *     at [b * ld + i]; a complex array stores re, im interleaved, element
 *     (b, i) at [2 * (b * ld + i)].  ld >= the row length (n_bus or n_node).
 *   - Work is enqueued on the given stream and is asynchronous; outputs are
 *     valid once the stream has been synchronised.  A null stream means the
 *     default stream.  Exceptions, stated with each call: pf_dist_solve
 *     waits on the host once per fixed-point iteration unless
 *     opts->zbus_async = 1, and the serving engine's step and harvest calls
 *     wait for their stream.
 *   - Non-convergence of a scenario is not an error: it is reported through
 *     that scenario's converged flag, iteration count and final mismatch.
 */
#ifndef PFX_H
#define PFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pf_stream;   /* a hipStream_t */

typedef enum pf_status {
  PF_OK = 0,
  PF_INVALID_ARG = 1,     /* a size, pointer or option is out of range */
  PF_OUT_OF_MEMORY = 2,   /* a device allocation failed or the context budget is exceeded */
  PF_HIP_ERROR = 3,       /* a HIP runtime call failed */
  PF_SINGULAR_SETUP = 4,  /* a network matrix could not be factorised */
  PF_NOT_ADMITTED = 5,    /* serving engine: no free slots for the request */
  PF_BAD_HANDLE = 6       /* null or destroyed handle */
} pf_status;

typedef enum pf_precision {
  PF_FP64 = 0,            /* every step in FP64 */
  PF_MIXED = 1            /* FP32 inner solves / FP32 Zbus product; FP64 mismatch, test and update */
} pf_precision;

/* Solver options.  pf_opts_default() fills the defaults listed here. */
typedef struct pf_opts {
  int32_t precision;          /* pf_precision, default PF_FP64 */
  double tol;                 /* converged when max |mismatch| <= tol (pu), default 1e-8 */
  int32_t max_newton;         /* Newton updates at most, default 20 */
  int32_t gmres_restart;      /* Krylov dimension per GMRES cycle, 1..64, default 30 */
  int32_t gmres_max_restarts; /* GMRES cycles per Newton step at most, default 10 */
  double gmres_rtol;          /* preconditioned residual reduction of each Newton step's GMRES
                                 solve (inexact Newton), default 1e-3 (0 = the default) */
  double diverge;             /* a scenario whose mismatch exceeds this is abandoned, default 1e6 */
  int32_t zbus_max_iter;      /* fixed-point updates at most, default 100 */
  /* network set-up (read by the *_network_create calls only) */
  double eps;                 /* diagonal regularisation of B' and B'' (Sec. II-A), default 1e-8 */
  int32_t precond_block;      /* 0: exact (B'+eps I)^-1, (B''+eps I)^-1 (default);
                                 k > 0: block-Jacobi over diagonal blocks of k buses */
  int32_t factor_max_levels;  /* at most this many sparse elimination levels before the dense
                                 core; the set-up picks the cheapest split, default 8 */
  int32_t factor_max_core;    /* largest dense Schur core, default 384 */
  /* feeder solve */
  int32_t zbus_sparse;        /* 0: dense product Z r on the matrix cores (default); 1: Y_NN^-1 r
                                 by level-scheduled solves with a sparse L D L^T of Y_NN (the
                                 sparse variant named as future work in Sec. II-B) */
  int32_t zbus_async;         /* 0: the host reads each iteration's active count back and stops
                                 enqueuing once none is left, waiting one iteration behind the
                                 device (default); 1: all zbus_max_iter iterations are enqueued
                                 at once and exit on the device once no scenario is active, so
                                 the call returns without waiting (each exited iteration still
                                 costs its two launches, about 3.6 us) */
  /* transmission Newton step */
  int32_t nr_direct;          /* 0: preconditioned GMRES (default); 1: exact Newton step by a
                                 per-scenario sparse LU of J on a shared symbolic analysis (the
                                 sparse direct outlook of Sec. IV), always in FP64, for networks
                                 of up to 2048 buses; the factor lives in LDS when it fits, else
                                 in network-owned device memory (8 bytes per factor value and
                                 scenario of the batch) */
  /* serving engine */
  int32_t step_iters;         /* Newton updates or fixed-point iterations per engine step of a
                                 request-driven engine, 1..1000, default 1 */
  /* inexact Newton forcing term of the GMRES Newton step */
  int32_t forcing;            /* 0: every Newton step's GMRES solve stops at gmres_rtol;
                                 1 (default): adaptive (Eisenstat-Walker choice 2): eta_0 = forcing_max,
                                 eta_k = 0.9 (|F_k| / |F_k-1|)^2, kept at least 0.9 eta_k-1^2
                                 when that exceeds 0.1, at most forcing_max, and at least
                                 gmres_rtol and 0.1 tol / |F_k| (no solve tighter than the
                                 fixed tolerance or than reaching tol needs).  The adaptive term
                                 saves GMRES steps (about 5 % of a 2000-bus batch solve) but
                                 gives some scenarios one more Newton update, which in the
                                 step-level serving engine lengthens the requests that hold
                                 them: serving engines meant for low tail latency should use 0 */
  double forcing_max;         /* largest adaptive forcing term, (0, 1), default 0.01 */
} pf_opts;

void pf_opts_default(pf_opts* out);

typedef struct pf_context pf_context;
typedef struct pf_tx_network pf_tx_network;
typedef struct pf_dist_network pf_dist_network;
typedef struct pf_engine pf_engine;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * workspace the context may hold (0 = no bound).  Errors: PF_INVALID_ARG,
 * PF_HIP_ERROR. */
pf_status pf_context_create(int32_t device, uint64_t hbm_budget_bytes, pf_context** out);
/* Destroy a context and every network created in it.  Null is ignored. */
void pf_context_destroy(pf_context* ctx);
/* Message of the last failing call on this thread ("" if none).  The pointer
 * stays valid until the next failing call on the same thread. */
const char* pf_last_error(void);
/* Device bytes currently held by the context (networks and workspaces). */
uint64_t pf_context_bytes(const pf_context* ctx);

/* ---------------------------------------------------------- transmission */

/* Build the bus admittance matrix of pi-model branches (Sec. II-A): branch k
 * from f[k] to t[k] with series impedance r[k] + j x[k] and total charging
 * b[k] adds y_s + j b/2 to both diagonal entries and -y_s to both
 * off-diagonal ones.  All pointers are host.  Output CSR (host, caller
 * allocated): row_ptr[n_bus + 1], col_idx[cap], y_re[cap], y_im[cap] with
 * columns sorted and duplicates summed; *nnz_out receives the count.
 * Errors: PF_INVALID_ARG (index out of range, zero impedance, cap too small:
 * then *nnz_out still receives the required count). */
pf_status pf_tx_ybus_from_branches(int32_t n_bus, int32_t n_branch, const int32_t* f,
                                   const int32_t* t, const double* r, const double* x,
                                   const double* b, int32_t cap, int32_t* row_ptr,
                                   int32_t* col_idx, double* y_re, double* y_im, int32_t* nnz_out);

/* Register a transmission network (Sec. II-A).  Host inputs, copied:
 *   Ybus as CSR (row_ptr[n_bus+1], col_idx[nnz], y_re[nnz], y_im[nnz]);
 *   bus_type[n_bus]: 0 = PQ, 1 = PV, 2 = slack, exactly one slack.
 *   Optional branch list (n_branch may be 0; needed only by the branch-loss
 *   calls): from/to buses, series impedance r + j x and total charging b.
 * The index sets are Theta = PV u PQ and Q = PQ (Sec. II-A); B' and B'' are
 * -Im(Ybus) on Theta x Theta and Q x Q, G = -Re(Ybus) on Q x Theta (eq. (7)).
 * Their regularised inverses are factorised here, once (Sec. II-A: the
 * inverses are precomputed).  setup_opts may be null (defaults).  Networks of
 * up to 8192 buses are supported.
 * Errors: PF_INVALID_ARG, PF_SINGULAR_SETUP, PF_OUT_OF_MEMORY, PF_HIP_ERROR. */
pf_status pf_tx_network_create(pf_context* ctx, int32_t n_bus, int32_t nnz, const int32_t* row_ptr,
                               const int32_t* col_idx, const double* y_re, const double* y_im,
                               const int8_t* bus_type, int32_t n_branch, const int32_t* br_f,
                               const int32_t* br_t, const double* br_r, const double* br_x,
                               const double* br_b, const pf_opts* setup_opts, pf_tx_network** out);
void pf_tx_network_destroy(pf_tx_network* net);
/* Sizes: n_bus, |Theta|, |Q|, nnz(Ybus), stored sparse entries of the
 * explicit (B' + eps I)^-1 and (B'' + eps I)^-1 passes, and the dense core
 * sizes of the two inverses (any pointer may be null). */
pf_status pf_tx_network_info(const pf_tx_network* net, int32_t* n_bus, int32_t* n_theta,
                             int32_t* n_q, int32_t* nnz, int32_t* factor_nnz, int32_t* core_bp,
                             int32_t* core_bpp);

/* Batched Newton-Raphson (eqs. (1)-(3)) from a flat start for `batch`
 * scenarios.  Device inputs [batch][ld]: p_inj, q_inj (scheduled injections,
 * generation minus load) and vm_set (|V| set-points at PV buses and the slack;
 * read only there).  Device outputs: v_out complex [batch][ld] (all buses),
 * newton_iters[batch] (updates taken), gmres_iters[batch] (Arnoldi steps over
 * all Newton steps), converged[batch] (1 when max |F| <= tol),
 * final_mismatch[batch] (max |F| at v_out), work_bytes[batch] (algorithmic
 * HBM bytes of the scenario's solve under the byte model: per Jacobian-vector
 * product 2wm + 4wn (V and I in the inner solve's precision), per
 * preconditioner application 2wm + 8n, per Gram-Schmidt pass of Arnoldi step
 * j (2j + 3)wm (a second pass, when taken, counts again), per GMRES cycle
 * start 8m + wm and end (k + 2)wm for k steps, per mismatch evaluation
 * 32n + 16m, per Newton update 16m, with w = 8 (PF_FP64) or 4 (PF_MIXED) and
 * m = |Theta| + |Q|).  Optional outputs
 * may be null: gmres_iters, final_mismatch, work_bytes.  batch may be 0.
 * With opts->nr_direct = 1 each Newton step is solved exactly by a sparse LU
 * of J (FP64 whatever opts->precision says; gmres_iters reports 0; the
 * byte model counts the mismatch plus 40m per step); the network's shared
 * analysis is built on the first such call, and a network above 2048 buses
 * is refused with PF_INVALID_ARG.
 * Errors: PF_INVALID_ARG (ld < n_bus, batch < 0, bad options),
 * PF_OUT_OF_MEMORY, PF_HIP_ERROR. */
pf_status pf_tx_solve(pf_tx_network* net, const pf_opts* opts, int32_t batch, int64_t ld,
                      const double* p_inj, const double* q_inj, const double* vm_set,
                      double* v_out, int32_t* newton_iters, int32_t* gmres_iters,
                      uint8_t* converged, double* final_mismatch, double* work_bytes,
                      pf_stream stream);

/* Batched Newton-Raphson as pf_tx_solve, with each scenario's own Ybus values
 * on the network's sparsity pattern: topology and parameter actions such as
 * branch switching, one per scenario (the batches of candidate operating
 * actions that Sec. I motivates).  y_vals: device, [batch][ldy] complex
 * (re, im interleaved, 2 ldy doubles per scenario, ldy >= the nnz given at
 * network creation), the values of the CSR entries given at creation, in
 * that order (duplicates are summed as at creation; an entry may be zero).
 * The mismatch (eq. (2)) and the Jacobian-vector products use the scenario's
 * values; the preconditioner of eq. (7) stays the one factorised from the
 * network's own values (an approximate left preconditioner only changes
 * how fast GMRES converges, not the Newton step it converges to).  The values
 * are first copied into the kernel's layout (FP64, plus an FP32 copy for
 * PF_MIXED) in network-owned workspace, which grows to batch x the stored
 * entries of Ybus.  work_bytes adds the scenario's Ybus entries per
 * mismatch (16 bytes each) and per Jacobian-vector product (2w bytes each).
 * A scenario whose actions leave the Jacobian singular (an islanded bus)
 * reports converged = 0.
 * Errors: as pf_tx_solve; PF_INVALID_ARG for ldy < nnz or null y_vals. */
pf_status pf_tx_solve_yvals(pf_tx_network* net, const pf_opts* opts, int32_t batch, int64_t ld,
                            const double* p_inj, const double* q_inj, const double* vm_set, int64_t ldy,
                            const double* y_vals, double* v_out, int32_t* newton_iters,
                            int32_t* gmres_iters, uint8_t* converged, double* final_mismatch,
                            double* work_bytes, pf_stream stream);

/* Per-scenario Ybus values for branch switching, for pf_tx_solve_yvals: for
 * each scenario s, y_vals[s] = the given Ybus (CSR as for
 * pf_tx_network_create) minus the pi-model stamps (Sec. II-A) of the branches
 * k with branch_on[s * n_branch + k] == 0.  The pattern is kept: the entries
 * of a switched-out branch keep their places (zero off the diagonal when no
 * other branch is parallel to it).  All pointers host; y_vals
 * [batch][2 ldy] doubles, caller allocated, ldy >= nnz.
 * Errors: PF_INVALID_ARG (bus index out of range, a branch whose four entries
 * are not all in the pattern, zero impedance, ldy < nnz). */
pf_status pf_tx_ybus_switch(int32_t n_bus, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                            const double* y_re, const double* y_im, int32_t n_branch, const int32_t* f,
                            const int32_t* t, const double* r, const double* x, const double* b,
                            int32_t batch, const uint8_t* branch_on, int64_t ldy, double* y_vals);

/* Bytes of the fixed device array behind pf_tx_solve_noalloc (64 MiB). */
#define PF_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* pf_tx_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results, bit for bit, as pf_tx_solve with
 * the same arguments, with the per-scenario workspace (Newton state, GMRES
 * vectors, Krylov basis) taken from one fixed array of
 * PF_NOALLOC_SCRATCH_BYTES that each device holds from library load until
 * the process ends.  The call makes no hipMalloc/hipFree or other
 * allocating call; the caller still provides every input and output as for
 * pf_tx_solve (all device memory).  The array must hold
 * align256(batch * 13 nbp * 8) + batch * (gmres_restart + 1) * 2 nbp * w
 * bytes (nbp = the padded bus count of the kernel's shape, w = 8 for PF_FP64,
 * 4 for PF_MIXED): on a 2000-bus grid (nbp 2048) about 52 scenarios in FP64
 * and 99 in mixed precision, on a 30-bus grid about 1700.  The kernels
 * overwrite every workspace element before reading it, so the array needs
 * no clearing between calls.  All calls on one device share its array:
 * the library makes each call's kernels wait on the device for the previous
 * call's (on whatever stream), so calls enqueued from several streams
 * serialise rather than corrupt each other; work outside this entry point
 * never touches the array.  The network's direct Newton step is not
 * available here (nr_direct must be 0).
 * Errors: PF_INVALID_ARG (as pf_tx_solve; nr_direct = 1; a batch whose
 * workspace exceeds the array, with the byte count in the message),
 * PF_BAD_HANDLE, PF_HIP_ERROR. */
pf_status pf_tx_solve_noalloc(pf_tx_network* net, const pf_opts* opts, int32_t batch, int64_t ld,
                              const double* p_inj, const double* q_inj, const double* vm_set,
                              double* v_out, int32_t* newton_iters, int32_t* gmres_iters,
                              uint8_t* converged, double* final_mismatch, double* work_bytes,
                              pf_stream stream);

/* Branch loss L_b = sum over branches of |I_f|^2 with the from-end current
 * I_f = (y_s + j b/2) V_f - y_s V_t, for voltages v (device complex
 * [batch][ld]).  Outputs (device): loss[batch] and, if dl_dv is not null, the
 * gradient in torch's convention dL/dRe V + j dL/dIm V, complex [batch][ld].
 * Needs the branch list given at network creation.
 * Errors: PF_INVALID_ARG, PF_HIP_ERROR. */
pf_status pf_tx_branch_loss(pf_tx_network* net, int32_t batch, int64_t ld, const double* v,
                            double* loss, double* dl_dv, pf_stream stream);

/* Adjoint of the solved state: for converged voltages v (device complex
 * [batch][ld]) and an upstream gradient dl_dv (device complex [batch][ld],
 * torch convention), solve J^T lambda = dL/dx by restarted GMRES on
 * transposed Jacobian-vector products with the transposed preconditioner of
 * eq. (7), and return dL/dP = lambda_P on Theta buses and dL/dQ = lambda_Q on
 * PQ buses (device [batch][ld], zero elsewhere).  Always FP64.
 * gmres_iters and converged (device, [batch]) may be null.
 * Errors: PF_INVALID_ARG, PF_OUT_OF_MEMORY, PF_HIP_ERROR. */
pf_status pf_tx_adjoint(pf_tx_network* net, const pf_opts* opts, int32_t batch, int64_t ld,
                        const double* v, const double* dl_dv, double* grad_p, double* grad_q,
                        int32_t* gmres_iters, uint8_t* converged, pf_stream stream);

/* ---------------------------------------------------------- distribution */

/* Build the three-phase admittance matrix of a radial feeder (Sec. II-B):
 * segment k joins bus seg_from[k] to seg_to[k] with 3x3 series impedance
 * z[k] (row-major, complex interleaved, 18 doubles per segment); phase node
 * 3*bus + phase.  Each segment adds inv(z) to both diagonal 3x3 blocks and
 * -inv(z) to both off-diagonal blocks.  Output CSR as for the transmission
 * builder over 3*n_bus nodes.  Errors: PF_INVALID_ARG, PF_SINGULAR_SETUP. */
pf_status pf_dist_ybus_from_segments(int32_t n_bus, int32_t n_seg, const int32_t* seg_from,
                                     const int32_t* seg_to, const double* z, int32_t cap,
                                     int32_t* row_ptr, int32_t* col_idx, double* y_re, double* y_im,
                                     int32_t* nnz_out);

/* Register a feeder.  Host inputs, copied: three-phase Ybus CSR over n_node
 * phase nodes; slack_nodes[3] with voltages v_slack (re/im interleaved, 6
 * doubles); wye_node[n_wye] (nodes that may carry a wye load);
 * delta_nodes[n_delta][3] (phase nodes a, b, c of each delta-loaded bus).
 * Computes the reduced impedance Z = inv(Y_NN) over the non-slack nodes N and
 * the no-load voltage v0 = -Z Y_NS v_S (Sec. II-B, eq. (10)) in FP64, keeps Z
 * in FP64 and FP32 on the device.  setup_opts may be null.
 * Errors: PF_INVALID_ARG, PF_SINGULAR_SETUP, PF_OUT_OF_MEMORY, PF_HIP_ERROR. */
pf_status pf_dist_network_create(pf_context* ctx, int32_t n_node, int32_t nnz, const int32_t* row_ptr,
                                 const int32_t* col_idx, const double* y_re, const double* y_im,
                                 const int32_t* slack_nodes, const double* v_slack, int32_t n_wye,
                                 const int32_t* wye_node, int32_t n_delta, const int32_t* delta_nodes,
                                 const pf_opts* setup_opts, pf_dist_network** out);
void pf_dist_network_destroy(pf_dist_network* net);
pf_status pf_dist_network_info(const pf_dist_network* net, int32_t* n_node, int32_t* n_free,
                               int32_t* n_wye, int32_t* n_delta);

/* Batched Z-bus fixed point (eq. (10)) from v = v0.  Device inputs complex
 * [batch][ld] over all phase nodes, consumption convention: s_wye (wye load on
 * each node; read at wye nodes only) and s_delta (for a delta bus with nodes
 * a, b, c: the ab, bc, ca branch loads at a, b, c; read at delta nodes only).
 * The iteration is run in residual form v <- v + Z r, r = i(v) - (Y_NN v +
 * Y_NS v_S), which equals Z i(v) + v0 exactly; a scenario is converged when
 * max |v * conj(r)| <= tol.  Device outputs: v_out complex [batch][ld] (all
 * nodes, slack included), iters[batch], converged[batch], final_mismatch
 * [batch] (may be null), sum_abs_change[batch] (the change of sum |v| over the
 * last update, the paper's stop quantity; may be null).  By default
 * (opts->zbus_async = 0) the call blocks the calling thread: it waits on
 * the host for each iteration's active count, one iteration behind the
 * device, and stops enqueuing after the last active iteration, returning
 * once the remaining work (the last update and the output kernel) is
 * enqueued.  With zbus_async = 1 it enqueues all zbus_max_iter iterations
 * and returns without waiting; once no scenario is active the remaining
 * launches exit at once on the device, at about 3.6 us per iteration (with
 * the default cap of 100 and solves converging in about 5 iterations that
 * costs 12-20 % of a 900-node batch of 4096; lower zbus_max_iter to cut it).
 * Caps above 1000 iterations always take the host-checked loop.
 * Errors: PF_INVALID_ARG, PF_OUT_OF_MEMORY, PF_HIP_ERROR. */
pf_status pf_dist_solve(pf_dist_network* net, const pf_opts* opts, int32_t batch, int64_t ld,
                        const double* s_wye, const double* s_delta, double* v_out, int32_t* iters,
                        uint8_t* converged, double* final_mismatch, double* sum_abs_change,
                        pf_stream stream);

/* ------------------------------------------------------------- serving */

/* Serving engine: step-level continuous batching of scenarios for one
 * registered network (the batched solves of Sec. II-A or II-B, served as the
 * requests of the paper's many-scenario setting arrive).  The engine owns
 * device memory for max_slots scenario slots (inputs, outputs, the
 * resumable solver state and workspace; max_slots = floor(hbm_bytes /
 * slot_bytes), a little less for a feeder engine with several streams).  A
 * step advances every occupied slot by at most a given number of Newton
 * updates (transmission) or Z-bus fixed-point iterations (feeder) in one
 * launch over the occupied slots; between steps finished scenarios are
 * harvested and waiting ones admitted into any free slots.  A scenario
 * resumes each step exactly where the previous one stopped, so its result is
 * bit-identical to pf_tx_solve / pf_dist_solve of that scenario with the
 * engine's options, whatever shares its steps.  Options (precision,
 * tolerances, step_iters) are fixed at creation; the direct Newton step is
 * not available (nr_direct must be 0).  An engine is bound to its network
 * and context: destroying either destroys the engine (waiting requests are
 * dropped).  The engine's calls are thread-safe.
 *
 * Two ways to drive an engine:
 *   caller-driven (n_streams = 0): pf_engine_admit, pf_engine_step and
 *     pf_engine_harvest on streams the caller names;
 *   request-driven (n_streams = 1..8): pf_engine_submit queues requests of
 *     any size; each of n_streams cohorts (a HIP stream run by a host thread
 *     of the engine) repeats admit -> step (opts->step_iters iterations) ->
 *     harvest.  Requests are admitted in arrival order into any free slots
 *     (not necessarily contiguous), all of a request's scenarios into one
 *     cohort; a request too large for the free slots may be passed by later
 *     requests at most 8 times.  pf_engine_poll and pf_engine_fetch report a
 *     request once its last scenario is harvested.  The cohorts' kernels
 *     overlap on the device, and so do those of engines on other networks. */

/* Device bytes of one slot for `opts` (exactly one of tx, dist non-null). */
pf_status pf_engine_slot_bytes(pf_tx_network* tx, pf_dist_network* dist, const pf_opts* opts,
                               uint64_t* bytes);
/* Create an engine over exactly one of tx or dist.  hbm_bytes bounds the slot
 * memory (PF_INVALID_ARG if below one slot); n_streams in 0..8 (0:
 * caller-driven); opts may be null.
 * Errors: PF_INVALID_ARG, PF_BAD_HANDLE, PF_OUT_OF_MEMORY, PF_HIP_ERROR. */
pf_status pf_engine_create(pf_context* ctx, pf_tx_network* tx, pf_dist_network* dist, uint64_t hbm_bytes,
                           int32_t n_streams, const pf_opts* opts, pf_engine** out);
void pf_engine_destroy(pf_engine* engine);

/* Caller-driven engines.  Place n scenarios into the free slots slot_ids[n]
 * (host, 0 <= slot < max_slots, distinct).  Host inputs, copied before
 * return, [n][row] as for pf_engine_submit.  The inputs reach the device on
 * `stream` (asynchronously); the scenarios take part from the next
 * pf_engine_step.  Errors: PF_INVALID_ARG (request-driven engine, slot out of
 * range, occupied or repeated, null input). */
pf_status pf_engine_admit(pf_engine* engine, int32_t n, const int32_t* slot_ids, const double* in0,
                          const double* in1, const double* in2, pf_stream stream);
/* One step on `stream`: every occupied slot whose scenario has not finished
 * runs at most `iters` (>= 1) Newton updates or fixed-point iterations.
 * Waits for the stream, then writes the slots whose scenario finished in this
 * step (converged, abandoned or out of iterations) to done_slots[*n_done]
 * (host, capacity max_done, which must be at least the number of unfinished
 * scenarios, or max_slots), and the number still iterating to *n_active (may
 * be null).  A finished scenario keeps its slot until harvested.
 * Errors: PF_INVALID_ARG, PF_HIP_ERROR. */
pf_status pf_engine_step(pf_engine* engine, int32_t iters, int32_t max_done, int32_t* done_slots,
                         int32_t* n_done, int32_t* n_active, pf_stream stream);
/* Copy the results of the finished scenarios in slot_ids[n] to host memory,
 * [n][...] in that order (v_out complex [n][row], iters, converged,
 * final_mismatch as for pf_engine_fetch; any output may be null), and free
 * their slots.  Waits for `stream`.  Errors: PF_INVALID_ARG (a slot not
 * holding a finished scenario, repeated slot), PF_HIP_ERROR. */
pf_status pf_engine_harvest(pf_engine* engine, int32_t n, const int32_t* slot_ids, double* v_out,
                            int32_t* iters, uint8_t* converged, double* final_mismatch, pf_stream stream);

/* Request-driven engines.  Queue request `id` (caller-chosen, unique among
 * unfetched requests) of n scenarios.  Host inputs [n][row]: transmission:
 * in0 = p_inj, in1 = q_inj, in2 = vm_set (row = n_bus, as in pf_tx_solve);
 * feeder: in0 = s_wye, in1 = s_delta complex (row = 2 n_node doubles, as in
 * pf_dist_solve), in2 unused.  Nothing is copied at submission: the engine
 * reads the inputs when it admits the request into slots, so the caller
 * keeps them valid and unchanged until pf_engine_poll reports the request
 * (or the engine is destroyed).
 * Errors: PF_NOT_ADMITTED (n exceeds the engine's slots), PF_INVALID_ARG
 * (caller-driven engine, n < 1, duplicate id, null input). */
pf_status pf_engine_submit(pf_engine* engine, int64_t id, int32_t n, const double* in0, const double* in1,
                           const double* in2);
/* Ids of up to max_ids finished requests, oldest first, each reported once;
 * waits up to timeout_s seconds for the first one (0: do not wait). */
pf_status pf_engine_poll(pf_engine* engine, int32_t max_ids, int64_t* ids, double timeout_s,
                         int32_t* count);
/* Scenario count of an unfetched request.  Errors: PF_INVALID_ARG (unknown id). */
pf_status pf_engine_request_size(pf_engine* engine, int64_t id, int32_t* n);
/* Copy a finished request's results to host memory and forget it: v_out
 * complex [n][row] (row = n_bus or n_node), iters[n] (Newton updates or Z-bus
 * iterations), converged[n], final_mismatch[n], times[3] (seconds since the
 * engine was created: submission, admission into slots, harvest of the last
 * scenario).  Any output may be null.  Errors: PF_INVALID_ARG (unknown or
 * unfinished id), PF_HIP_ERROR (a step holding the request's scenarios
 * failed; the request is forgotten). */
pf_status pf_engine_fetch(pf_engine* engine, int64_t id, double* v_out, int32_t* iters, uint8_t* converged,
                          double* final_mismatch, double* times);
/* Counters (any pointer may be null): slots, bytes per slot, requests waiting
 * for admission, occupied slots, steps run, scenarios harvested. */
pf_status pf_engine_info(pf_engine* engine, int32_t* max_slots, uint64_t* slot_bytes, int32_t* queued,
                         int32_t* occupied, uint64_t* steps, uint64_t* scenarios);

#ifdef __cplusplus
}
#endif

#endif /* PFX_H */
