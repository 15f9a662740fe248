/*
 * sts.h - C ABI of the sparse, truncated state-vector library (gfx950).
 *
 * The library keeps a quantum state as a sparse list of (basis key, complex
 * amplitude) terms in device memory and offers the operations the paper
 * builds its simulator from:
 *
 *   sts_init        - a state of n <= 64 qubits in the ground state |0...0>,
 *                     stored as a single term (Sec. I); basis keys are 64-bit
 *                     integers, so n is at most 64 (Sec. V).
 *   sts_apply_gate  - apply a 2^m x 2^m unitary to m qubits: each amplitude
 *                     multiplies the column of U picked by its bit pattern on
 *                     those qubits, the new keys follow from bit operations,
 *                     and contributions to the same key are summed (Eq. (3)
 *                     and its m-qubit generalisation, Sec. IV.A).
 *   sts_truncate    - keep the largest-|a|^2 terms: p-mass first, then top-k,
 *                     then renormalise (Sec. III; Sec. IV.B).
 *   sts_peak        - the most probable basis key (Sec. I); only this result
 *                     crosses to the host (Sec. V).
 *
 * Conventions
 *   - Qubit q is bit q of a key (qubit 0 = least significant bit).
 *   - U is row-major, 2^m x 2^m, complex, FP64, interleaved (re, im):
 *     U[2*(i*2^m + j) + 0/1]. U[i][j] maps local pattern j to local pattern i,
 *     where bit t of a local pattern is qubit qubits[t]. U is not checked for
 *     unitarity.
 *   - Amplitudes are complex128 (STS_C128) or complex64 (STS_C64). With
 *     STS_C64 the gate arithmetic and stored amplitudes are FP32 (U is
 *     rounded to FP32, nearest-even, once per call), while |a|^2, the
 *     truncation threshold, the probability-mass sums and the
 *     renormalisation scale stay FP64.
 *   - Ranking is the total order (|a|^2 descending, key ascending), with
 *     |a|^2 = fl64(fl64(re*re) + fl64(im*im)) (components promoted to FP64
 *     first). A term is dropped by gate application only when both parts
 *     are exactly zero.
 *   - Truncation keeps L = min(L_p, K, C) terms of the C present, where L_p
 *     is the shortest prefix of the ranked terms whose exact mass is
 *     >= p * W (W = exact current total). K = 0 turns top-k off; p <= 0 or
 *     p >= 1 turns p-mass off. If L = C nothing changes (no rescale);
 *     otherwise every kept amplitude is multiplied by fl64(1/sqrt(S)), with
 *     S the correctly rounded kept mass.
 *
 * Execution, ownership, errors
 *   - All calls are ordered on the stream given to sts_init and return
 *     without waiting for the GPU, except those marked "synchronises".
 *     The term count stays on the device between calls.
 *   - Host arrays passed in are read before the call returns; the caller
 *     keeps ownership. Device memory is owned by the context: either carved
 *     from the caller's arena (which must stay allocated until sts_free) or
 *     allocated by the library.
 *   - A context is not thread-safe; distinct contexts may run concurrently
 *     on distinct streams.
 *   - STS_E_ARG leaves everything as it was. STS_E_CAPACITY is decided on
 *     the host before any term is written: the gate step that did not fit
 *     is discarded, and the terms and every figure of sts_stats and
 *     sts_counters are those from before that gate; the context stays
 *     usable. STS_E_HIP and STS_E_NOMEM during a computation poison the
 *     context: afterwards only sts_free is valid (other calls return
 *     STS_E_STATE). STS_E_STATE also reports a failed internal consistency
 *     check on the device (a cut that could not be resolved, a write past a
 *     buffer), which the host's checks rule out; it poisons the context.
 */
#ifndef STS_H
#define STS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STS_OK = 0,
    STS_E_ARG = -1,      /* invalid argument; nothing changed                  */
    STS_E_NOMEM = -2,    /* device allocation failed                           */
    STS_E_CAPACITY = -3, /* the result would not fit in the context's capacity  */
    STS_E_HIP = -4,      /* a HIP runtime call failed                          */
    STS_E_STATE = -5     /* the context is poisoned or the call is out of order */
} sts_status;

typedef enum { STS_C128 = 0, STS_C64 = 1 } sts_precision;

typedef struct sts_ctx sts_ctx;

/*
 * Device bytes a context needs to hold up to cap_terms terms at the given
 * precision (for sizing an arena). Writes the size to *bytes.
 */
sts_status sts_required_bytes(uint64_t cap_terms, int precision, size_t *bytes);

/*
 * Create a state of n_qubits (1..64) in the ground state (one term, key 0,
 * amplitude 1). max_terms = K of top-k truncation (0 = off; a K above
 * 2^n_qubits never cuts and is taken as 2^n_qubits); mass = p of
 * p-mass truncation (off unless 0 < p < 1). Both may be given: p-mass first,
 * then top-k (Sec. III). hip_stream: a hipStream_t, NULL = the null stream.
 * arena/arena_bytes: device memory to carve every buffer from (NULL/0 = the
 * library allocates). cap_terms: the most terms the state may ever hold;
 * 0 = max(K, 2^20) when the library allocates, or as many as the arena holds
 * (this argument, the precision, the stream and the arena extend the
 * two-argument form sts_init(n_qubits, K_or_mass)). Gate application needs
 * room for the 2^m * N candidates only when the state is not truncated
 * right after (see sts_apply_gate). STS_E_CAPACITY if K > cap_terms.
 */
sts_status sts_init(sts_ctx **out, int n_qubits, uint64_t max_terms, double mass,
                    int precision, void *hip_stream, void *arena, size_t arena_bytes,
                    uint64_t cap_terms);

/*
 * Apply the gate U (host array, 2*4^m doubles, layout above) on the m
 * distinct qubits qubits[0..m-1] (each < n), 1 <= m <= 5. Gates of up to 3
 * qubits, and 4-qubit gates on a state holding at most about half of
 * cap_terms, run on the LDS-tiled kernels; other 4- and 5-qubit gates run on
 * slower untiled ones (same results). The result is
 * formed lazily: the grouping work runs now, and the new amplitudes are
 * produced by the following sts_truncate (so candidates are never stored),
 * or by the next call that needs them. Returns STS_E_ARG for bad arguments.
 * Whether a gate's un-truncated result must fit in cap_terms is known only
 * when the next call arrives (an sts_truncate never forms it), so its
 * overflow is reported by that next call - this one for the previous gate,
 * or sts_peak, sts_num_terms, sts_read_terms - as STS_E_CAPACITY: the
 * previous gate is discarded and the state is the one before it, while the
 * gate of this call is not applied. Checking at the gate itself would cost a
 * host synchronisation per gate.
 */
sts_status sts_apply_gate(sts_ctx *ctx, int m, const int *qubits, const double *U);

/* Truncate by the rule fixed at sts_init (see above) and renormalise.
 * STS_E_CAPACITY (the pending gate discarded, nothing else changed) when
 * the cut keeps more than cap_terms terms (possible only when p-mass alone
 * limits it), or when an untiled 4- or 5-qubit gate puts more candidates
 * into the cut's exponent than the side buffer holds (8 x cap_terms). */
sts_status sts_truncate(sts_ctx *ctx);

/* Most probable key (ties to the smaller key) and its probability
 * |a|^2 / W, W the exact current total. Synchronises. */
sts_status sts_peak(sts_ctx *ctx, uint64_t *key, double *prob);

/* Number of terms now held. Synchronises. */
sts_status sts_num_terms(sts_ctx *ctx, uint64_t *n);

/* Copy the terms to the host in ascending key order, amplitudes as FP64
 * (re, im) pairs; keys[cap], amps[2*cap]. *n receives the count; returns
 * STS_E_CAPACITY (copying nothing) if cap is too small. Synchronises. */
sts_status sts_read_terms(sts_ctx *ctx, uint64_t cap, uint64_t *keys, double *amps, uint64_t *n);

/* Replace the state with n terms from the host (keys unique and < 2^n_qubits,
 * amplitudes FP64 (re, im); rounded to FP32 for STS_C64). */
sts_status sts_load_terms(sts_ctx *ctx, uint64_t n, const uint64_t *keys, const double *amps);

/* Figures of the last sts_truncate: W = total mass before the cut (correctly
 * rounded), kept_fraction = S/W, log10_cum_kept = sum of log10 of every kept
 * fraction so far, last_candidates = number of nonzero terms before the cut.
 * Any pointer may be NULL. Synchronises. */
sts_status sts_stats(sts_ctx *ctx, double *W, double *kept_fraction, double *log10_cum_kept,
                     uint64_t *last_candidates);

/* Cumulative counters since sts_init: truncations run (gate steps), input
 * terms they processed (gate-term updates) and candidates they ranked. Any
 * pointer may be NULL. Synchronises. */
sts_status sts_counters(sts_ctx *ctx, uint64_t *gate_steps, uint64_t *term_updates, uint64_t *candidates);

/* Shapes of the grouping sort (digit bits x keys per workgroup tile). The
 * default, 8-bit digits in 4096-key tiles, suits large states: a digit's run
 * in a tile averages 16 keys, so the scatter's writes coalesce. Small states
 * sort in a chain of short launches, where 11-bit digits (fewer passes) or
 * 2048-key tiles (more workgroups) can pay. */
typedef enum {
    STS_SORT_8x16 = 0,  /* 8-bit digits, 4096-key tiles (default)  */
    STS_SORT_8x8 = 1,   /* 8-bit digits, 2048-key tiles            */
    STS_SORT_11x16 = 2, /* 11-bit digits, 4096-key tiles           */
    STS_SORT_11x8 = 3   /* 11-bit digits, 2048-key tiles           */
} sts_sort_shape;

/* From now on, sort states of at most 2^small_log2 terms with `shape` and
 * larger ones with STS_SORT_8x16 (small_log2 = 0: always the default). The
 * results do not depend on the shape. STS_E_ARG for small_log2 outside
 * 0..40 or an unknown shape; call between steps (no gate pending). */
sts_status sts_set_sort_shape(sts_ctx *ctx, int small_log2, int shape);

/* Kernel kinds timed by sts_profile (the kernels of a gate step). */
typedef enum {
    STS_K_RADIX_HIST = 0,   /* per-tile digit counts of a grouping-sort pass */
    STS_K_RADIX_SCAN = 1,   /* their scan into per-tile digit offsets        */
    STS_K_RADIX_PASS = 2,   /* one scatter pass of the grouping sort         */
    STS_K_GROUP_HIST = 3,   /* gate + weight histogram pass                  */
    STS_K_PICK1 = 4,        /* exponent-level cut                            */
    STS_K_GROUP_EXTRACT = 5,/* gate + copy of the cut's exponent             */
    STS_K_SIDE_HIST = 6,    /* mantissa-level cut                            */
    STS_K_FINAL = 7,        /* last levels and LDS sort                      */
    STS_K_GROUP_EMIT = 8,   /* gate + survivor write                         */
    STS_K_SIDE_EXTRACT = 9, /* copy of the mantissa-level subset             */
    STS_K_TILE_KEPT = 10,   /* survivors per tile                            */
    STS_K_TILE_SCAN = 11,   /* output offsets per tile                       */
    STS_K_SAMPLE = 12,      /* gate on a sample of tiles: the cut's window   */
    STS_K_COUNT = 13
} sts_kernel_kind;

/* Turn per-kernel timing on (1) or off (0). While on, every kernel launch is
 * bracketed by HIP events on the context's stream. */
sts_status sts_profile(sts_ctx *ctx, int enable);

/* Total time (ms) and number of launches of one kernel kind since timing was
 * turned on (or last reset with reset = 1). Synchronises. */
sts_status sts_kernel_time(sts_ctx *ctx, int kind, int reset, double *total_ms, uint64_t *launches);

/* ------------------------------------------------------------------------
 * Batches of independent circuits.
 *
 * At small k the cost of a gate step is a fixed overhead rather than work
 * proportional to k (Sec. VI.B), so running one circuit at a time leaves the
 * GPU mostly idle. sts_batch_run keeps several circuits in flight at once.
 * Each circuit runs through its own context exactly as it would alone
 * (sts_init, then sts_apply_gate / sts_truncate per gate, then sts_peak), so
 * its results do not depend on the rest of the batch.
 * ------------------------------------------------------------------------ */

/* One circuit: n_gates gates in order, flattened. Gate i acts on gate_m[i]
 * (1..5) qubits, listed next in gate_qubits, with the next 2*4^m doubles of
 * gate_U as its matrix (layout of sts_apply_gate); truncate_after[i] != 0
 * truncates right after it. max_terms and mass as in sts_init. The arrays
 * are the caller's and are read during the call.
 * Optional output: when out_keys and out_amps are not NULL, the final terms
 * are copied there as sts_read_terms does (ascending keys, FP64 (re, im)
 * pairs; out_keys[out_cap], out_amps[2*out_cap]); the result's n_terms says
 * how many, and a final state of more than out_cap terms is the circuit's
 * STS_E_CAPACITY. These arrays must stay valid until the result is
 * returned (sts_batch_run) or taken (sts_server_wait). */
typedef struct {
    int n_qubits;
    uint64_t max_terms;
    double mass;
    uint64_t n_gates;
    const int *gate_m;
    const int *gate_qubits;
    const double *gate_U;
    const uint8_t *truncate_after;
    uint64_t out_cap;
    uint64_t *out_keys;
    double *out_amps;
} sts_circuit;

typedef struct {
    int precision;   /* STS_C128 or STS_C64, for every circuit                 */
    int n_streams;   /* circuits in flight, 1..64: each has a host thread, a   */
                     /* HIP stream and a device arena of its own               */
    int graph_steps; /* 0: plain launches; > 0: a truncated gate step of up   */
                     /* to 3 qubits (top-k on) is captured into a HIP graph    */
                     /* once per state of the circuit's context (term buffer,  */
                     /* size bound, gate size) and replayed for later gates    */
                     /* with only the gate changed                             */
    int sort_small_log2; /* each circuit's context: sts_set_sort_shape(         */
    int sort_shape;      /* sort_small_log2, sort_shape); 0, 0 = the default    */
} sts_batch_config;

typedef struct {
    sts_status status;      /* STS_OK, or the first error of this circuit     */
    uint64_t peak_key;      /* sts_peak at the end                            */
    double peak_prob;
    uint64_t n_terms;       /* terms held at the end                          */
    uint64_t gate_steps;    /* sts_counters at the end                        */
    uint64_t term_updates;
    double log10_cum_kept;  /* sts_stats at the end                           */
    double seconds;         /* host wall time from its sts_init to its result */
    double queue_seconds;   /* server: from submission to admission (else 0)  */
    double latency_seconds; /* server: from submission to result (else        */
                            /* equal to seconds)                              */
} sts_circuit_result;

/* Run n circuits on the current device. The library allocates one arena per
 * stream (sized for the largest circuit: max(K, 1024) terms, times 2^m if an
 * untruncated gate of m qubits occurs) and frees it before returning. The
 * longest circuits (gates x min(K, 2^n)) start first. results[n] receives
 * one entry per circuit, in input order. Returns STS_E_ARG for bad arguments
 * (nothing runs), the first error of any circuit otherwise, or STS_OK.
 * Synchronises. */
sts_status sts_batch_run(int n, const sts_circuit *circuits, const sts_batch_config *cfg,
                         sts_circuit_result *results);

/* ------------------------------------------------------------------------
 * A resident server with continuous batching.
 *
 * Requests are circuits submitted at any time from any thread. Worker
 * threads (one HIP stream each) admit queued requests in submission order
 * whenever a block for the request's context fits in the server's device
 * memory budget, keep up to max_active requests each, and advance them in
 * turn by gates_per_turn gates, so a request that arrives while long ones
 * run starts at the next turn. Each request runs through its own context
 * exactly as alone (sts_init, gates, sts_peak), so its result does not
 * depend on what else is being served.
 * ------------------------------------------------------------------------ */
typedef struct sts_server sts_server;

typedef struct {
    int precision;       /* STS_C128 or STS_C64, for every request            */
    int n_streams;       /* worker threads / HIP streams, 1..64               */
    int max_active;      /* requests a worker interleaves, 1..64              */
    int gates_per_turn;  /* gates a request advances per turn, >= 1           */
    uint64_t hbm_bytes;  /* device memory for request contexts, allocated at  */
                         /* creation; 0 = half of the free device memory      */
} sts_server_config;

/* Start a server on the current device (allocates its memory budget and
 * starts its workers). */
sts_status sts_server_create(sts_server **out, const sts_server_config *cfg);

/* Queue a circuit (layout of sts_circuit; its arrays are copied before the
 * call returns) and return its ticket. STS_E_CAPACITY if the request's
 * context could never fit in the budget; STS_E_STATE once the server is
 * being destroyed. Thread-safe. */
sts_status sts_server_submit(sts_server *s, const sts_circuit *c, uint64_t *ticket);

/* Wait for a request to finish and take its result (queue_seconds and
 * latency_seconds measured from its submission). Each ticket can be taken
 * once; STS_E_ARG for an unknown ticket. Thread-safe. */
sts_status sts_server_wait(sts_server *s, uint64_t ticket, sts_circuit_result *out);

/* Requests queued, running and finished so far, and device bytes held by
 * running requests. Any pointer may be NULL. Thread-safe. */
sts_status sts_server_stats(sts_server *s, uint64_t *queued, uint64_t *active, uint64_t *done,
                            uint64_t *bytes_in_use);

/* Finish every submitted request, stop the workers and free the budget.
 * Results not taken are dropped. NULL is a no-op. */
void sts_server_destroy(sts_server *s);

/* ------------------------------------------------------------------------
 * One gate step with no allocation of any kind, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.
 *
 * Applies U (host array, layout of sts_apply_gate) on qubits[0..m-1]
 * (1 <= m <= 3) to the n_in terms in keys_in / amps_in, truncates by the
 * rule (max_terms = K >= 1, required; mass = p as in sts_init) and
 * renormalises - the results of sts_load_terms, sts_apply_gate and
 * sts_truncate on a context - and writes the kept terms to keys_out /
 * amps_out and their count to *n_out. All five arrays are the caller's
 * device memory: keys u64, amplitudes double2 (STS_C128) or float2
 * (STS_C64); the outputs need room for min(K, 2^n_qubits) terms and must
 * not overlap the inputs; n_out points to one u64 in device memory; stats,
 * if not NULL, to two doubles in device memory that receive W and the kept
 * fraction (as sts_stats). Terms come out in no particular order.
 * Every working buffer lives in one static device array of 32 MiB per
 * device (held until the process ends), laid out for at most
 * STS_STATIC_MAX_TERMS terms: n_in or K above that is STS_E_CAPACITY, with
 * nothing launched. The call only enqueues work on hip_stream (NULL = the
 * null stream) and returns without waiting; it launches kernels and
 * device-to-device copies only. Each call overwrites the array, so calls
 * that overlap in time on one device (other streams, other threads) race:
 * order them on one stream or serialise them. STS_E_ARG for bad arguments
 * (nothing launched); STS_E_HIP if a launch fails.
 * ------------------------------------------------------------------------ */
#define STS_STATIC_MAX_TERMS 65536
sts_status sts_step_static(int n_qubits, uint64_t max_terms, double mass, int precision, void *hip_stream,
                           int m, const int *qubits, const double *U,
                           const uint64_t *keys_in, const void *amps_in, uint64_t n_in,
                           uint64_t *keys_out, void *amps_out, uint64_t *n_out, double *stats);

/* Release the context and the device memory it allocated. NULL is a no-op. */
void sts_free(sts_ctx *ctx);

/* Static description of a status code. */
const char *sts_strerror(sts_status s);

#ifdef __cplusplus
}
#endif

#endif /* STS_H */
