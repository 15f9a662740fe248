// serve.hip - a resident simulation server with continuous batching.
//
// Requests (circuits) are copied on submission into a FIFO queue. Worker
// threads, each with a HIP stream of its own, admit requests between turns:
// a request is admitted when a block for its context fits in the server's
// device memory budget (first-fit over one slab allocated at creation), and
// the queue is served in order, so a large request at the head is not
// overtaken. A worker keeps up to max_active requests and advances each by
// gates_per_turn gates in turn; a request that finishes frees its block at
// once, and the next one joins at the next turn, so short requests do not
// wait for long ones to finish. Every request runs through its own context
// exactly as it would alone.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runner.h"

namespace {

using namespace sts_runner;
using Clock = std::chrono::steady_clock;

double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

struct Request {
    u64 ticket = 0;
    // owned copy of the circuit
    std::vector<int> m, q;
    std::vector<double> u;
    std::vector<uint8_t> t;
    sts_circuit c{};
    u64 cap = 0, bytes = 0, off = 0;
    sts_ctx *ctx = nullptr;
    u64 gi = 0, qo = 0, uo = 0;
    Clock::time_point arrive, admit;
    sts_circuit_result res{};
    bool done = false;
};

// first-fit allocator of aligned blocks in [0, size)
class Blocks {
public:
    void reset(u64 size)
    {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(u64 bytes, u64 *off)
    {
        bytes = (bytes + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const u64 rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(u64 off, u64 bytes)
    {
        bytes = (bytes + 255) & ~255ull;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    u64 used() const { return used_; }

private:
    std::map<u64, u64> free_;
    u64 used_ = 0;
};

} // namespace

struct sts_server {
    sts_server_config cfg{};
    int dev = 0;
    unsigned char *slab = nullptr;
    u64 slab_bytes = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<u64, Request *> all;
    Blocks blocks;
    u64 next_ticket = 1, n_active = 0, n_done = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
};

namespace {

void complete(sts_server *s, Request *r, sts_status st)
{
    if (r->ctx) {
        sts_free(r->ctx); // waits for the stream
        r->ctx = nullptr;
    }
    const auto now = Clock::now();
    r->res.status = st;
    r->res.seconds = secs(r->admit, now);
    r->res.queue_seconds = secs(r->arrive, r->admit);
    r->res.latency_seconds = secs(r->arrive, now);
    std::lock_guard<std::mutex> lk(s->mu);
    s->blocks.release(r->off, r->bytes);
    r->done = true;
    s->n_active -= 1;
    s->n_done += 1;
    s->cv_done.notify_all();
    s->cv_work.notify_all(); // memory came free
}

void worker_main(sts_server *s, int w)
{
    (void)hipSetDevice(s->dev);
    hipStream_t stream = s->streams[w];
    std::vector<Request *> active;
    for (;;) {
        std::vector<Request *> fresh;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                while ((int)active.size() + (int)fresh.size() < s->cfg.max_active && !s->queue.empty()) {
                    Request *r = s->queue.front();
                    if (!s->blocks.alloc(r->bytes, &r->off)) break; // in order: wait for memory
                    s->queue.pop_front();
                    r->admit = Clock::now();
                    s->n_active += 1;
                    fresh.push_back(r);
                }
                if (!active.empty() || !fresh.empty()) break;
                if (s->stopping && s->queue.empty()) return;
                s->cv_work.wait(lk);
            }
        }
        for (Request *r : fresh) {
            const sts_status st = sts_init(&r->ctx, r->c.n_qubits, r->c.max_terms, r->c.mass, s->cfg.precision,
                                           stream, s->slab + r->off, r->bytes, r->cap);
            if (st != STS_OK) {
                r->ctx = nullptr;
                complete(s, r, st);
            } else {
                active.push_back(r);
            }
        }
        // one turn: every active request advances by up to gates_per_turn gates
        for (size_t i = 0; i < active.size();) {
            Request *r = active[i];
            const u64 end = std::min<u64>(r->gi + (u64)s->cfg.gates_per_turn, r->c.n_gates);
            sts_status st = run_gates(r->ctx, r->c, end, &r->gi, &r->qo, &r->uo);
            if (st == STS_OK && r->gi < r->c.n_gates) {
                ++i;
                continue;
            }
            if (st == STS_OK) st = finish(r->ctx, r->c, &r->res);
            complete(s, r, st);
            active[i] = active.back();
            active.pop_back();
        }
    }
}

} // namespace

extern "C" {

sts_status sts_server_create(sts_server **out, const sts_server_config *cfg)
{
    if (!out || !cfg) return STS_E_ARG;
    *out = nullptr;
    if (cfg->precision != STS_C128 && cfg->precision != STS_C64) return STS_E_ARG;
    if (cfg->n_streams < 1 || cfg->n_streams > 64 || cfg->max_active < 1 || cfg->max_active > 64 ||
        cfg->gates_per_turn < 1)
        return STS_E_ARG;
    sts_server *s = new (std::nothrow) sts_server();
    if (!s) return STS_E_NOMEM;
    s->cfg = *cfg;
    if (hipGetDevice(&s->dev) != hipSuccess) {
        delete s;
        return STS_E_HIP;
    }
    u64 bytes = cfg->hbm_bytes;
    if (!bytes) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return STS_E_HIP;
        }
        bytes = (u64)(fr / 2);
    }
    bytes &= ~255ull;
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        delete s;
        return e == hipErrorOutOfMemory ? STS_E_NOMEM : STS_E_HIP;
    }
    s->slab = (unsigned char *)p;
    s->slab_bytes = bytes;
    s->blocks.reset(bytes);
    s->streams.resize(cfg->n_streams, nullptr);
    for (int w = 0; w < cfg->n_streams; ++w) {
        if (hipStreamCreateWithFlags(&s->streams[w], hipStreamNonBlocking) != hipSuccess) {
            for (auto st : s->streams)
                if (st) (void)hipStreamDestroy(st);
            (void)hipFree(s->slab);
            delete s;
            return STS_E_HIP;
        }
    }
    for (int w = 0; w < cfg->n_streams; ++w) s->workers.emplace_back(worker_main, s, w);
    *out = s;
    return STS_OK;
}

sts_status sts_server_submit(sts_server *s, const sts_circuit *c, uint64_t *ticket)
{
    if (!s || !c || !ticket || !circuit_valid(*c)) return STS_E_ARG;
    Request *r = new (std::nothrow) Request();
    if (!r) return STS_E_NOMEM;
    u64 nq = 0;
    for (u64 i = 0; i < c->n_gates; ++i) nq += (u64)c->gate_m[i];
    u64 nu = 0;
    for (u64 i = 0; i < c->n_gates; ++i) nu += 2ull << (2 * c->gate_m[i]);
    r->m.assign(c->gate_m, c->gate_m + c->n_gates);
    r->q.assign(c->gate_qubits, c->gate_qubits + nq);
    r->u.assign(c->gate_U, c->gate_U + nu);
    r->t.assign(c->truncate_after, c->truncate_after + c->n_gates);
    r->c = *c;
    r->c.gate_m = r->m.data();
    r->c.gate_qubits = r->q.data();
    r->c.gate_U = r->u.data();
    r->c.truncate_after = r->t.data();
    r->cap = circuit_cap(r->c);
    size_t bytes = 0;
    sts_status st = sts_required_bytes(r->cap, s->cfg.precision, &bytes);
    if (st != STS_OK || bytes > s->slab_bytes) {
        delete r;
        return st != STS_OK ? st : STS_E_CAPACITY; // could never be admitted
    }
    r->bytes = bytes;
    r->arrive = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
        delete r;
        return STS_E_STATE;
    }
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_all();
    return STS_OK;
}

sts_status sts_server_wait(sts_server *s, uint64_t ticket, sts_circuit_result *out)
{
    if (!s || !out) return STS_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return STS_E_ARG;
    Request *r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    *out = r->res;
    s->all.erase(it);
    delete r;
    return STS_OK;
}

sts_status sts_server_stats(sts_server *s, uint64_t *queued, uint64_t *active, uint64_t *done, uint64_t *bytes_in_use)
{
    if (!s) return STS_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = s->queue.size();
    if (active) *active = s->n_active;
    if (done) *done = s->n_done;
    if (bytes_in_use) *bytes_in_use = s->blocks.used();
    return STS_OK;
}

void sts_server_destroy(sts_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_work.notify_all();
    }
    for (auto &t : s->workers) t.join();
    for (auto st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    for (auto &kv : s->all) delete kv.second;
    if (s->slab) (void)hipFree(s->slab);
    delete s;
}

} // extern "C"
