// batch.hip - many independent circuits on one GPU.
//
// At small k a gate step is a fixed cost of a dozen short kernel launches
// (the GPU overhead visible at low k in Sec. VI.B), so one circuit at a time
// leaves most of the device idle. The batch runner keeps several circuits in
// flight: each worker is a host thread with its own HIP stream and its own
// device arena, and runs whole circuits through an ordinary context carved
// from that arena, so every circuit computes exactly what it computes alone.
// Circuits are handed out longest first (work ~ gates x min(K, 2^n)).
// Optionally, truncated gate steps of up to 3 qubits are captured into HIP
// graphs, one per state of the context (term buffer, size bound, gate size),
// and replayed with only the gate changed: one graph launch per gate instead
// of a dozen kernel launches.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "runner.h"

namespace {

using namespace sts_runner;

struct BatchJob {
    int idx;
    double work;
};

// one circuit start to finish on an existing stream and arena
void run_one(const sts_circuit &c, int prec, int graph_steps, int sort_small_log2, int sort_shape, hipStream_t s,
             void *arena, size_t arena_bytes, sts_circuit_result *r)
{
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(r, 0, sizeof(*r));
    sts_ctx *ctx = nullptr;
    sts_status st = sts_init(&ctx, c.n_qubits, c.max_terms, c.mass, prec, s, arena, arena_bytes, circuit_cap(c));
    if (st == STS_OK) st = sts_set_sort_shape(ctx, sort_small_log2, sort_shape);
    StepGraphs *gs = graph_steps > 0 && st == STS_OK ? step_graphs_new() : nullptr;
    u64 qo = 0, uo = 0;
    u64 i = 0;
    while (st == STS_OK && i < c.n_gates) {
        const int m = c.gate_m[i];
        if (!gs || m > 3 || !c.truncate_after[i] || c.max_terms == 0) {
            st = run_gates(ctx, c, i + 1, &i, &qo, &uo);
            continue;
        }
        // truncated steps of up to 3 qubits: captured once per state of the
        // context, then replayed
        st = step_replayed(ctx, gs, m, c.gate_qubits + qo, c.gate_U + uo);
        qo += (u64)m;
        uo += 2ull << (2 * m);
        ++i;
    }
    if (st == STS_OK) st = finish(ctx, c, r);
    if (ctx) sts_free(ctx); // waits for the stream
    step_graphs_free(gs);
    r->status = st;
    r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    r->latency_seconds = r->seconds;
}

} // namespace

extern "C" sts_status sts_batch_run(int n, const sts_circuit *circuits, const sts_batch_config *cfg,
                                    sts_circuit_result *results)
{
    if (n < 0 || (n > 0 && (!circuits || !results)) || !cfg) return STS_E_ARG;
    if (cfg->precision != STS_C128 && cfg->precision != STS_C64) return STS_E_ARG;
    if (cfg->n_streams < 1 || cfg->n_streams > 64 || cfg->graph_steps < 0) return STS_E_ARG;
    if (cfg->sort_small_log2 < 0 || cfg->sort_small_log2 > 40 || cfg->sort_shape < 0 || cfg->sort_shape > 3)
        return STS_E_ARG;
    for (int i = 0; i < n; ++i)
        if (!circuit_valid(circuits[i])) return STS_E_ARG;
    if (n == 0) return STS_OK;
    for (int i = 0; i < n; ++i) {
        std::memset(&results[i], 0, sizeof(results[i]));
        results[i].status = STS_E_STATE; // until a worker has run it
    }

    std::vector<BatchJob> jobs(n);
    u64 cap_max = 1024;
    for (int i = 0; i < n; ++i) {
        jobs[i].idx = i;
        jobs[i].work = circuit_work(circuits[i]);
        cap_max = std::max(cap_max, circuit_cap(circuits[i]));
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const BatchJob &a, const BatchJob &b) { return a.work > b.work; });
    size_t bytes = 0;
    sts_status st = sts_required_bytes(cap_max, cfg->precision, &bytes);
    if (st != STS_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return STS_E_HIP;

    const int workers = std::min(cfg->n_streams, n);
    std::atomic<int> next{0};
    std::atomic<int> setup_err{0};
    auto worker = [&]() {
        if (hipSetDevice(dev) != hipSuccess) {
            setup_err = STS_E_HIP;
            return;
        }
        hipStream_t s = nullptr;
        void *arena = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            setup_err = STS_E_HIP;
            return;
        }
        const hipError_t e = hipMalloc(&arena, bytes);
        if (e != hipSuccess) {
            setup_err = e == hipErrorOutOfMemory ? STS_E_NOMEM : STS_E_HIP;
            (void)hipStreamDestroy(s);
            return;
        }
        for (int j = next.fetch_add(1); j < n; j = next.fetch_add(1)) {
            const int idx = jobs[j].idx;
            run_one(circuits[idx], cfg->precision, cfg->graph_steps, cfg->sort_small_log2, cfg->sort_shape, s, arena,
                    bytes, &results[idx]);
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(arena);
        (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> pool;
    pool.reserve(workers);
    for (int w = 0; w < workers; ++w) pool.emplace_back(worker);
    for (auto &t : pool) t.join();
    for (int i = 0; i < n; ++i)
        if (results[i].status == STS_E_STATE && setup_err.load()) return (sts_status)setup_err.load();
    for (int i = 0; i < n; ++i)
        if (results[i].status != STS_OK) return results[i].status;
    return STS_OK;
}
