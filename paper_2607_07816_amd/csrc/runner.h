// runner.h - host helpers shared by the batch runner and the server: checks
// and sizes of an sts_circuit, and running its gates on a context.
#pragma once
#include <algorithm>

#include "sts.h"
#include "kernels.h"

// replayed gate steps (api.hip): a per-context cache of captured steps
struct StepGraphs;
StepGraphs *step_graphs_new();
void step_graphs_free(StepGraphs *gs);
void step_graphs_counts(const StepGraphs *gs, u64 *captures, u64 *replays);
// one truncated gate step, as sts_apply_gate + sts_truncate; replayed from a
// captured graph when the context starts it in the state of an earlier step
// (same term buffer, same size bound, same gate size)
sts_status step_replayed(sts_ctx *c, StepGraphs *gs, int m, const int *qubits, const double *U);

namespace sts_runner {

inline bool circuit_valid(const sts_circuit &c)
{
    if (c.n_qubits < 1 || c.n_qubits > 64) return false;
    if (c.n_gates && (!c.gate_m || !c.gate_qubits || !c.gate_U || !c.truncate_after)) return false;
    for (u64 i = 0; i < c.n_gates; ++i)
        if (c.gate_m[i] < 1 || c.gate_m[i] > STS_MAXM) return false;
    return true;
}

// terms a circuit's context must hold: min(K, 2^n) for truncated steps, and
// room for an untruncated gate's 2^m times as many candidates
inline u64 circuit_cap(const sts_circuit &c)
{
    const u64 full = c.n_qubits >= 40 ? (1ull << 40) : (1ull << c.n_qubits);
    const u64 k = c.max_terms ? std::min<u64>(c.max_terms, full) : full;
    int m_free = 0;
    for (u64 i = 0; i < c.n_gates; ++i)
        if (!c.truncate_after[i]) m_free = std::max(m_free, c.gate_m[i]);
    const u64 cap = k > (~0ull >> m_free) ? ~0ull : (k << m_free);
    return std::min<u64>(std::max<u64>(cap, 1024), 1ull << 36);
}

// gates x min(K, 2^n): the scale of a circuit's work
inline double circuit_work(const sts_circuit &c)
{
    const double full = c.n_qubits >= 40 ? 1e12 : (double)(1ull << c.n_qubits);
    const double k = c.max_terms ? std::min((double)c.max_terms, full) : full;
    return (double)c.n_gates * k;
}

// apply gates [*gi, end) of c (advancing *gi and the qubit/U offsets)
inline sts_status run_gates(sts_ctx *ctx, const sts_circuit &c, u64 end, u64 *gi, u64 *qo, u64 *uo)
{
    sts_status st = STS_OK;
    while (st == STS_OK && *gi < end) {
        const u64 i = *gi;
        const int m = c.gate_m[i];
        st = sts_apply_gate(ctx, m, c.gate_qubits + *qo, c.gate_U + *uo);
        if (st == STS_OK && c.truncate_after[i]) st = sts_truncate(ctx);
        *qo += (u64)m;
        *uo += 2ull << (2 * m);
        *gi = i + 1;
    }
    return st;
}

// the end-of-circuit figures of a result, and the final terms if asked for
inline sts_status finish(sts_ctx *ctx, const sts_circuit &c, sts_circuit_result *r)
{
    sts_status st = sts_peak(ctx, &r->peak_key, &r->peak_prob); // synchronises
    if (st == STS_OK) st = sts_num_terms(ctx, &r->n_terms);
    if (st == STS_OK) st = sts_counters(ctx, &r->gate_steps, &r->term_updates, nullptr);
    if (st == STS_OK) st = sts_stats(ctx, nullptr, nullptr, &r->log10_cum_kept, nullptr);
    if (st == STS_OK && c.out_keys && c.out_amps) {
        uint64_t n = 0;
        st = sts_read_terms(ctx, c.out_cap, c.out_keys, c.out_amps, &n);
    }
    return st;
}

} // namespace sts_runner
