// api.hip - the C ABI of libsts: context, device memory, and the order in
// which the kernels of a gate step run.
//
// A gate step (sts_apply_gate then sts_truncate) runs, on the context's
// stream and without host synchronisation:
//   1. 1..4 radix digit passes (per-tile counts, per-digit scan, scatter):
//      group the state by the hash bucket of the bits outside the gate
//      (radix.hip);
//   2. histogram pass: recompute every new amplitude, histogram its weight by
//      exponent field with exact mantissa sums (group.hip);
//   3. level-1 pick: exact prefix over exponent bins (select.hip);
//   4. extraction pass: copy the candidates of the cut's exponent to the side
//      buffer (group.hip);
//   5. level-2 histogram + pick over the side buffer, then the final levels
//      and an LDS sort of the last <= 4096 candidates (select.hip);
//   6. write pass: recompute once more and write the survivors, rescaled
//      (group.hip).
// Without a truncation rule (or when the next gate arrives first) step 6
// alone runs, keeping every nonzero candidate.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "sts.h"
#include "kernels.h"

namespace {

constexpr u64 kAlign = 256;
constexpr int kULen = 32 * 32 * 2; // doubles of the largest U

u64 align_up(u64 x) { return (x + kAlign - 1) & ~(kAlign - 1); }

u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }

struct Layout {
    u64 ctl, ctl_save, keys[3], amps[3], side_key, side_w, side_amp, sub_key, sub_w, h1, h2, h2w, h3, best, rcount, rprefix, rtotal, look_comp,
        t_above, t_side, t_off, tctr, dU, sub_cnt, wpart, sbins, gate, total;
};

// tiles of the LDS-tiled passes (2048 terms each) and the side-buffer entries:
// one slab of 2048 << m entries per tile, m <= 3
u64 tiled_tiles(u64 cap) { return (cap + 2047) / 2048 + 1; }
u64 side_capacity(u64 cap) { return tiled_tiles(cap) * (2048ull << 3); }

Layout make_layout(u64 cap, int prec)
{
    const u64 asz = prec == STS_C128 ? 16 : 8;
    const u64 scap = side_capacity(cap);
    const u64 ttiles = tiled_tiles(cap);
    const u64 tiles = ceil_div(cap, 2048) + 1; // the smallest grouping-sort tile
    const u64 gtiles = ceil_div(cap, STS_GTILE);
    Layout L;
    u64 o = 0;
    auto take = [&](u64 bytes) {
        const u64 at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.ctl = take(sizeof(DevCtl));
    L.ctl_save = take(sizeof(DevCtl));
    for (int i = 0; i < 3; ++i) L.keys[i] = take(cap * 8);
    for (int i = 0; i < 3; ++i) L.amps[i] = take(cap * asz);
    L.side_key = take(scap * 8);
    L.side_w = take(scap * 8);
    L.side_amp = take(scap * asz);
    L.sub_key = take((u64)STS_SUB_CAP * 8);
    L.sub_w = take((u64)STS_SUB_CAP * 8);
    L.h1 = take(3 * STS_NBIN * 8);
    L.h2 = take(3 * STS_NBIN * 8);
    L.h2w = take(3 * STS_NBIN * 8);
    L.h3 = take(3 * STS_NBIN * 8);
    L.best = take(2 * STS_MAX_GROUPS * 8);
    L.rcount = take(2048 * tiles * 4); // per digit (up to 11-bit digits) and tile
    L.rprefix = take(2048 * tiles * 8);
    L.rtotal = take(2048 * 8);
    L.look_comp = take(gtiles * 8);
    L.t_above = take(ttiles * 4 * 4); // up to 4 slabs per tile
    L.t_side = take(ttiles * 4 * 4);
    L.t_off = take(ttiles * 8);
    L.tctr = take(16 * 4);
    L.dU = take(kULen * 8 + kULen * 4); // U in FP64, then its FP32 rounding
    L.sub_cnt = take((STS_SUB_REGIONS + 1) * 128);
    L.wpart = take(6 * STS_MAX_GROUPS * 8);
    L.sbins = take(STS_SW_BANKS * (STS_SW_NB + 4) * 8);
    L.gate = take(2 * sizeof(GateArg)); // the current gate, and the identity
    L.total = o;
    return L;
}

// the working memory of sts_step_static: one array per device, holding a
// context laid out for STS_STATIC_MAX_TERMS terms of either precision
constexpr size_t kStaticBytes = 32ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// its address on the current device (the array's name is a host-side
// stand-in, never a device address); looked up once per device
hipError_t static_scratch(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

} // namespace

struct sts_ctx {
    int n_qubits = 0;
    int prec = 0;
    u64 K = 0;
    double p = 0.0;
    hipStream_t stream = nullptr;
    bool own_mem = false;
    unsigned char *mem = nullptr;
    u64 cap = 0, scap = 0, tiles_cap = 0, gtiles_cap = 0;
    u64 *keys[3] = {nullptr, nullptr, nullptr};
    void *amps[3] = {nullptr, nullptr, nullptr};
    int cur = 0;            // buffer with the state, or the sorted input of the pending gate
    int radix_small_log2 = 0;               // states of at most 2^this terms are sorted with
    int radix_small_shape = STS_RADIX_8x16; // this shape; larger ones with 8x16
    bool pending = false;   // a gate whose new amplitudes are not written yet
    GateArg gate;
    u64 n_bound = 1;        // upper bound on the terms in buffer cur
    DevCtl *ctl = nullptr;
    DevCtl *ctl_save = nullptr; // the control block as it was before a step that may be refused
    u64 *h1 = nullptr, *h2 = nullptr, *h2w = nullptr, *h3 = nullptr, *best = nullptr;
    u64 *side_key = nullptr, *side_w = nullptr, *sub_key = nullptr, *sub_w = nullptr;
    void *side_amp = nullptr;
    u32 *rcount = nullptr;                          // per-tile digit counts of a scatter pass
    u64 *rprefix = nullptr, *rtotal = nullptr, *look_comp = nullptr;
    u32 *t_above = nullptr, *t_side = nullptr;
    u64 *t_off = nullptr;
    u32 *tctr = nullptr;
    double *dU = nullptr;
    u32 *sub_cnt = nullptr;
    u64 *wpart = nullptr, *sbins = nullptr;
    GateArg *dgate = nullptr, *dgate_id = nullptr; // device copies of the gate and of the identity
    const GateArg *gate_dev = nullptr;              // the one the pending step's kernels read
    double *hU = nullptr;    // pinned staging of U for m >= 4
    hipEvent_t u_event = nullptr;
    bool u_event_live = false;
    DevCtl *hctl = nullptr;  // pinned mirror of the control block
    u32 epoch = 0;
    bool poisoned = false;
    // optional per-kernel timing
    bool prof = false;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    double prof_ms[STS_K_COUNT] = {};
    u64 prof_n[STS_K_COUNT] = {};
};

namespace {

sts_status fail_hip(sts_ctx *c, hipError_t e)
{
    if (e == hipSuccess) return STS_OK;
    if (c) c->poisoned = true;
    return e == hipErrorOutOfMemory ? STS_E_NOMEM : STS_E_HIP;
}

#define STS_TRY(c, expr)                                   \
    do {                                                   \
        const hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return fail_hip((c), _e);    \
    } while (0)

hipEvent_t prof_event(sts_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// a kernel launch, bracketed by events when timing is on
#define STS_LAUNCH(c, kind, expr)                                                  \
    do {                                                                           \
        hipEvent_t _a = nullptr, _b = nullptr;                                     \
        if ((c)->prof) {                                                           \
            _a = prof_event(c);                                                    \
            _b = prof_event(c);                                                    \
            if (_a && _b) STS_TRY(c, hipEventRecord(_a, (c)->stream));             \
        }                                                                          \
        STS_TRY(c, expr);                                                          \
        if (_a && _b) {                                                            \
            STS_TRY(c, hipEventRecord(_b, (c)->stream));                           \
            (c)->marks.push_back({(kind), _a, _b});                                \
        }                                                                          \
    } while (0)

// fold finished marks into the per-kind totals (after a synchronisation)
void prof_collect(sts_ctx *c)
{
    for (auto &m : c->marks) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
            c->prof_ms[m.kind] += ms;
            c->prof_n[m.kind] += 1;
        }
        c->pool.push_back(m.a);
        c->pool.push_back(m.b);
    }
    c->marks.clear();
}

u32 next_epoch(sts_ctx *c)
{
    if (++c->epoch >= (1u << 24)) {
        // tags wrap: clear every look-back word once
        (void)hipMemsetAsync(c->look_comp, 0, c->gtiles_cap * 8, c->stream);
        c->epoch = 1;
    }
    return c->epoch;
}

u64 sat_shl(u64 x, int m)
{
    if (m <= 0) return x;
    if (x > (~0ull >> m)) return ~0ull;
    return x << m;
}

PassBufs pass_bufs(sts_ctx *c, int in, int out)
{
    PassBufs b;
    std::memset(&b, 0, sizeof(b));
    b.gate = c->gate_dev;
    b.keys = c->keys[in];
    b.amps = c->amps[in];
    b.n_in = &c->ctl->cnt[in];
    b.n_out = out >= 0 ? &c->ctl->cnt[out] : nullptr;
    b.ctl = c->ctl;
    b.h1 = c->h1;
    b.h2w = c->h2w;
    b.h3 = c->h3;
    b.best = c->best;
    b.side_key = c->side_key;
    b.side_w = c->side_w;
    b.side_amp = c->side_amp;
    b.side_cap = c->scap;
    b.sub_key = c->sub_key;
    b.sub_w = c->sub_w;
    b.sub_cap = STS_SUB_CAP;
    b.sub_cnt = c->sub_cnt;
    if (out >= 0) {
        b.out_keys = c->keys[out];
        b.out_amps = c->amps[out];
    }
    b.out_cap = c->cap;
    b.look = c->look_comp;
    b.t_above = c->t_above;
    b.t_side = c->t_side;
    b.t_off = c->t_off;
    b.tile_ctr = c->tctr + 4;
    b.wpart = c->wpart;
    b.sbins = c->sbins;
    return b;
}

// whether a gate of m qubits takes the LDS-tiled passes: always for m <= 3;
// for m = 4 when every tile's side slab (2048 << 4 entries) fits the side
// buffer, i.e. when the state holds at most about half the capacity
bool use_tiles(const sts_ctx *c, int m)
{
    if (m <= 3) return true;
    if (m > 4) return false;
    return ceil_div(std::max<u64>(c->n_bound, 1), 2048) * (2048ull << 4) <= c->scap;
}

// workgroups of the histogram pass (persistent; the tiled pass walks
// 2048-term tiles), at most as many as are resident at once
int hist_groups(int prec, u64 n_bound, int m, bool tiled)
{
    const u64 g = ceil_div(n_bound ? n_bound : 1, tiled ? 2048 : STS_WG);
    const u64 cap = (u64)std::min(group_hist_capacity(prec, m, tiled), STS_MAX_GROUPS);
    return (int)std::min<u64>(std::max<u64>(g, 1), cap);
}

int compact_tiles(u64 n_bound, int m) { return (int)sts_compact_groups(n_bound, m); }

// point every buffer of the context into its device memory c->mem
void bind_layout(sts_ctx *c, const Layout &L)
{
    c->ctl = (DevCtl *)(c->mem + L.ctl);
    c->ctl_save = (DevCtl *)(c->mem + L.ctl_save);
    for (int i = 0; i < 3; ++i) {
        c->keys[i] = (u64 *)(c->mem + L.keys[i]);
        c->amps[i] = c->mem + L.amps[i];
    }
    c->side_key = (u64 *)(c->mem + L.side_key);
    c->side_w = (u64 *)(c->mem + L.side_w);
    c->side_amp = (void *)(c->mem + L.side_amp);
    c->sub_key = (u64 *)(c->mem + L.sub_key);
    c->sub_w = (u64 *)(c->mem + L.sub_w);
    c->h1 = (u64 *)(c->mem + L.h1);
    c->h2 = (u64 *)(c->mem + L.h2);
    c->h2w = (u64 *)(c->mem + L.h2w);
    c->h3 = (u64 *)(c->mem + L.h3);
    c->best = (u64 *)(c->mem + L.best);
    c->rcount = (u32 *)(c->mem + L.rcount);
    c->rprefix = (u64 *)(c->mem + L.rprefix);
    c->rtotal = (u64 *)(c->mem + L.rtotal);
    c->look_comp = (u64 *)(c->mem + L.look_comp);
    c->t_above = (u32 *)(c->mem + L.t_above);
    c->t_side = (u32 *)(c->mem + L.t_side);
    c->t_off = (u64 *)(c->mem + L.t_off);
    c->tctr = (u32 *)(c->mem + L.tctr);
    c->dU = (double *)(c->mem + L.dU);
    c->sub_cnt = (u32 *)(c->mem + L.sub_cnt);
    c->wpart = (u64 *)(c->mem + L.wpart);
    c->sbins = (u64 *)(c->mem + L.sbins);
    c->dgate = (GateArg *)(c->mem + L.gate);
    c->dgate_id = c->dgate + 1;
    c->gate_dev = c->dgate_id;
}

// copy the control block to the host and wait; map device-side error flags
sts_status sync_ctl(sts_ctx *c)
{
    STS_TRY(c, hipMemcpyAsync(c->hctl, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, c->stream));
    STS_TRY(c, hipStreamSynchronize(c->stream));
    // the host's checks keep every write inside its buffer and every cut
    // resolvable, so a flag here is an internal inconsistency
    if (c->hctl->flags & (STS_F_SIDE_OVERFLOW | STS_F_OUT_OVERFLOW | STS_F_UNRESOLVED)) {
        c->poisoned = true;
        return STS_E_STATE;
    }
    return STS_OK;
}

// a gate step that may still be refused for capacity keeps a copy of the
// control block (term counts, statistics, the previous cut) on the device
sts_status save_ctl(sts_ctx *c)
{
    STS_TRY(c, hipMemcpyAsync(c->ctl_save, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToDevice, c->stream));
    return STS_OK;
}

// refuse the pending gate step: the control block goes back to the saved
// copy, and the state is the sorted input, i.e. the terms before the gate
sts_status refuse_step(sts_ctx *c)
{
    STS_TRY(c, hipMemcpyAsync(c->ctl, c->ctl_save, sizeof(DevCtl), hipMemcpyDeviceToDevice, c->stream));
    STS_TRY(c, hipStreamSynchronize(c->stream));
    c->pending = false;
    return STS_E_CAPACITY;
}

// the grouping sort's shape for the state's size bound (the context's
// policy), and its digit passes: enough bucket bits for that bound
int sort_shape(const sts_ctx *c)
{
    return c->radix_small_log2 > 0 && c->n_bound <= (1ull << c->radix_small_log2) ? c->radix_small_shape
                                                                                  : STS_RADIX_8x16;
}

int sort_passes(const sts_ctx *c)
{
    const u64 nb = std::max<u64>(c->n_bound, 2);
    int lg = 0;
    while ((1ull << lg) < nb && lg < 63) ++lg;
    const int bits = sts_radix_bits(sort_shape(c));
    return std::min(std::max((lg + bits - 1) / bits, 1), 32 / bits);
}

// group the state in buffer cur by the hash bucket of key & notmask (the
// device gate's); returns
// the buffer that holds the sorted terms and the bucket bits used
sts_status sort_state(sts_ctx *c, const u64 *notmask, int *sorted, int *hb_out)
{
    const u64 nb = std::max<u64>(c->n_bound, 2);
    const int shape = sort_shape(c);
    const int bits = sts_radix_bits(shape);
    const int npass = sort_passes(c);
    const int hb = bits * npass;
    const int tiles = (int)std::max<u64>(ceil_div(nb, sts_radix_tile(shape)), 1);
    const int a = (c->cur + 1) % 3, b = (c->cur + 2) % 3;
    int src = c->cur, dst = a;
    for (int p = 0; p < npass; ++p) {
        const int shift = 64 - hb + bits * p;
        for (int what = 0; what < 3; ++what) {
            const int kind = what == 0 ? STS_K_RADIX_HIST : (what == 1 ? STS_K_RADIX_SCAN : STS_K_RADIX_PASS);
            STS_LAUNCH(c, kind, launch_radix(what, shape, c->prec, c->keys[src], c->amps[src], c->keys[dst],
                                             c->amps[dst], &c->ctl->cnt[src], &c->ctl->cnt[dst], notmask, shift,
                                             c->rcount, c->rprefix, c->rtotal, c->tiles_cap, tiles, c->stream));
        }
        src = dst;
        dst = dst == a ? b : a;
    }
    *sorted = src;
    *hb_out = hb;
    return STS_OK;
}

// number of nonzero candidates of the pending gate (synchronises)
sts_status count_candidates(sts_ctx *c, u64 *count)
{
    PassBufs b = pass_bufs(c, c->cur, -1);
    const bool tiled = use_tiles(c, c->gate.m);
    const int G = hist_groups(c->prec, c->n_bound, c->gate.m, tiled);
    STS_LAUNCH(c, STS_K_GROUP_HIST, launch_group_hist(c->prec, c->gate, b, G, tiled, c->stream));
    STS_LAUNCH(c, STS_K_PICK1, launch_pick1(b, G, 1, 0, c->stream));
    const sts_status st = sync_ctl(c);
    if (st != STS_OK) return st;
    *count = c->hctl->cand_all;
    return STS_OK;
}

// write out the pending gate's candidates without truncation
sts_status materialise(sts_ctx *c)
{
    if (!c->pending) return STS_OK;
    const u64 cb = sat_shl(c->n_bound, c->gate.m);
    u64 bound = cb;
    if (cb > c->cap) {
        u64 count = 0;
        const sts_status st = count_candidates(c, &count);
        if (st != STS_OK) return st;
        if (count > c->cap) {
            c->pending = false; // drop the gate: the sorted input is the state before it
            return STS_E_CAPACITY;
        }
        bound = count;
    }
    const int dst = (c->cur + 1) % 3;
    PassBufs b = pass_bufs(c, c->cur, dst);
    b.materialise = 1;
    if (use_tiles(c, c->gate.m)) {
        const int tt = (int)std::max<u64>(ceil_div(c->n_bound, 2048), 1);
        STS_LAUNCH(c, STS_K_GROUP_EXTRACT,
                   launch_group_extract_tiles(c->prec, c->gate, b, std::min(tt, 2048), c->stream));
        STS_LAUNCH(c, STS_K_TILE_KEPT, launch_tile_kept(b, tt, c->stream));
        STS_LAUNCH(c, STS_K_TILE_SCAN, launch_tile_scan(b, tt, c->stream));
        STS_LAUNCH(c, STS_K_GROUP_EMIT, launch_group_emit_tiles(c->prec, c->gate, b, tt, c->stream));
    } else {
        b.epoch = next_epoch(c);
        STS_LAUNCH(c, STS_K_GROUP_EMIT, launch_group_compact(c->prec, STS_KIND_EMIT, c->gate, b,
                                                             compact_tiles(c->n_bound, c->gate.m), c->stream));
    }
    c->cur = dst;
    c->n_bound = std::min(bound, c->cap);
    c->pending = false;
    return STS_OK;
}

// the gate's kernel description (everything but the bucket bits hb, and
// for m >= 4 the device pointer to U); qubits and U already checked
void fill_gate(GateArg *g, int m, const int *qubits, const double *U)
{
    std::memset(g, 0, sizeof(*g));
    g->m = m;
    u64 mask = 0;
    for (int t = 0; t < m; ++t) {
        g->q[t] = qubits[t];
        mask |= 1ull << qubits[t];
    }
    g->notmask = ~mask;
    const int dim = 1 << m;
    if (m <= 3) {
        for (int i = 0; i < dim * dim; ++i) {
            g->ur[i] = U[2 * i];
            g->ui[i] = U[2 * i + 1];
            g->fr[i] = (float)U[2 * i]; // nearest-even
            g->fi[i] = (float)U[2 * i + 1];
        }
        for (int i = 0; i < dim; ++i) {
            u64 d = 0;
            for (int t = 0; t < m; ++t)
                if ((i >> t) & 1) d |= 1ull << qubits[t];
            g->dep[i] = d;
        }
    }
}

// STS_E_ARG unless qubits are m distinct qubits of the state and U is finite
sts_status check_gate(const sts_ctx *c, int m, const int *qubits, const double *U)
{
    if (!qubits || !U || m < 1 || m > STS_MAXM || m > c->n_qubits) return STS_E_ARG;
    u64 mask = 0;
    for (int t = 0; t < m; ++t) {
        if (qubits[t] < 0 || qubits[t] >= c->n_qubits) return STS_E_ARG;
        if (mask & (1ull << qubits[t])) return STS_E_ARG;
        mask |= 1ull << qubits[t];
    }
    for (int i = 0; i < 2 << (2 * m); ++i)
        if (!std::isfinite(U[i])) return STS_E_ARG;
    return STS_OK;
}

GateArg identity_gate()
{
    GateArg g;
    std::memset(&g, 0, sizeof(g));
    g.m = 0;
    g.notmask = ~0ull;
    return g;
}

sts_status check_live(sts_ctx *c)
{
    if (!c) return STS_E_ARG;
    if (c->poisoned) return STS_E_STATE;
    return STS_OK;
}

} // namespace

extern "C" {

sts_status sts_required_bytes(uint64_t cap_terms, int precision, size_t *bytes)
{
    if (!bytes || cap_terms == 0 || (precision != STS_C128 && precision != STS_C64)) return STS_E_ARG;
    if (cap_terms > (1ull << 36)) return STS_E_ARG;
    *bytes = (size_t)make_layout(cap_terms, precision).total;
    return STS_OK;
}

sts_status sts_init(sts_ctx **out, int n_qubits, uint64_t max_terms, double mass, int precision, void *hip_stream,
                    void *arena, size_t arena_bytes, uint64_t cap_terms)
{
    if (!out) return STS_E_ARG;
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 64) return STS_E_ARG;
    if (precision != STS_C128 && precision != STS_C64) return STS_E_ARG;
    if (!(mass == mass)) return STS_E_ARG; // NaN
    if (arena && arena_bytes == 0) return STS_E_ARG;
    if (cap_terms > (1ull << 36)) return STS_E_ARG;
    // n qubits have at most 2^n basis keys, so a larger K never cuts
    if (n_qubits < 64) max_terms = std::min<u64>(max_terms, 1ull << n_qubits);
    u64 cap = cap_terms;
    if (arena) {
        if (cap == 0) {
            // largest capacity whose layout fits the arena
            u64 lo = 1, hi = 1ull << 36;
            if (make_layout(1, precision).total > arena_bytes) return STS_E_NOMEM;
            while (lo < hi) {
                const u64 mid = lo + (hi - lo + 1) / 2;
                if (make_layout(mid, precision).total <= arena_bytes) lo = mid;
                else hi = mid - 1;
            }
            cap = lo;
        }
        if (make_layout(cap, precision).total > arena_bytes) return STS_E_NOMEM;
    } else if (cap == 0) {
        cap = std::max<u64>(max_terms, 1ull << 20);
    }
    if (max_terms > cap) return STS_E_CAPACITY;

    sts_ctx *c = new (std::nothrow) sts_ctx();
    if (!c) return STS_E_NOMEM;
    c->n_qubits = n_qubits;
    c->prec = precision;
    c->K = max_terms;
    c->p = (mass > 0.0 && mass < 1.0) ? mass : 0.0;
    c->stream = (hipStream_t)hip_stream;
    c->cap = cap;
    c->scap = side_capacity(cap);
    c->tiles_cap = ceil_div(cap, 2048) + 1;
    c->gtiles_cap = ceil_div(cap, STS_GTILE);
    const Layout L = make_layout(cap, precision);
    if (arena) {
        c->mem = (unsigned char *)arena;
    } else {
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, L.total);
        if (e != hipSuccess) {
            delete c;
            return e == hipErrorOutOfMemory ? STS_E_NOMEM : STS_E_HIP;
        }
        c->mem = (unsigned char *)p;
        c->own_mem = true;
    }
    bind_layout(c, L);

    hipError_t e = hipHostMalloc((void **)&c->hctl, sizeof(DevCtl), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->hU, kULen * (sizeof(double) + sizeof(float)), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->u_event, hipEventDisableTiming);
    if (e != hipSuccess) {
        sts_free(c);
        return STS_E_HIP;
    }
    std::memset(c->hctl, 0, sizeof(DevCtl));
    c->hctl->K = c->K;
    c->hctl->p = c->p;
    c->hctl->scale = 1.0;
    c->hctl->frac = 1.0;
    c->hctl->e_pred = -1;
    // zero the bookkeeping regions (everything but the term buffers)
    e = hipMemsetAsync(c->mem + L.h1, 0, L.total - L.h1, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->ctl, c->hctl, sizeof(DevCtl), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_init_state(precision, c->keys[0], c->amps[0], &c->ctl->cnt[0], c->stream);
    if (e == hipSuccess) e = launch_set_gate(identity_gate(), c->dgate_id, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        sts_free(c);
        return e == hipErrorOutOfMemory ? STS_E_NOMEM : STS_E_HIP;
    }
    c->cur = 0;
    c->n_bound = 1;
    *out = c;
    return STS_OK;
}

sts_status sts_apply_gate(sts_ctx *c, int m, const int *qubits, const double *U)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    st = check_gate(c, m, qubits, U);
    if (st != STS_OK) return st;
    st = materialise(c);
    if (st != STS_OK) return st;

    GateArg g;
    fill_gate(&g, m, qubits, U);
    const int dim = 1 << m;
    if (m > 3) {
        // the previous copy from the staging buffer must have finished
        if (c->u_event_live) STS_TRY(c, hipEventSynchronize(c->u_event));
        // the FP64 entries, then their FP32 roundings (nearest-even) right
        // after them: one copy
        const size_t nd = (size_t)2 * dim * dim;
        std::memcpy(c->hU, U, nd * sizeof(double));
        float *hf = reinterpret_cast<float *>(c->hU + nd);
        for (size_t i = 0; i < nd; ++i) hf[i] = (float)U[i];
        STS_TRY(c, hipMemcpyAsync(c->dU, c->hU, nd * (sizeof(double) + sizeof(float)), hipMemcpyHostToDevice,
                                  c->stream));
        STS_TRY(c, hipEventRecord(c->u_event, c->stream));
        c->u_event_live = true;
        g.uptr = c->dU;
        g.uptr_f = reinterpret_cast<const float *>(c->dU + nd);
    }
    int sorted = c->cur, hb = 8;
    g.hb = sts_radix_bits(sort_shape(c)) * sort_passes(c); // the bucket bits the sort below uses
    STS_TRY(c, launch_set_gate(g, c->dgate, c->stream));
    c->gate_dev = c->dgate;
    st = sort_state(c, &c->dgate->notmask, &sorted, &hb);
    if (st != STS_OK) return st;
    c->cur = sorted;
    c->gate = g;
    c->pending = true;
    return STS_OK;
}

sts_status sts_truncate(sts_ctx *c)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (!c->pending) {
        c->gate = identity_gate();
        c->gate_dev = c->dgate_id;
        c->pending = true;
    }
    const u64 cb = sat_shl(c->n_bound, c->gate.m);
    const int out = (c->cur + 1) % 3;
    PassBufs b = pass_bufs(c, c->cur, out);
    const bool tiled = use_tiles(c, c->gate.m);
    const int G = hist_groups(c->prec, c->n_bound, c->gate.m, tiled);
    const int tiles = compact_tiles(c->n_bound, c->gate.m);
    const int tt = (int)std::max<u64>(ceil_div(c->n_bound, 2048), 1);
    u64 nb = c->K ? std::min<u64>(c->K, cb) : cb;
    // two ways a step may not fit, both found before anything is written:
    // untiled passes (4- and 5-qubit gates on a large state) copy the cut
    // exponent's candidates to the side buffer in one dense run, which may
    // exceed it; a cut limited by p-mass alone may keep more than cap terms
    const bool side_risk = !tiled && cb > c->scap;
    const bool out_risk = nb > c->cap;
    if (side_risk || out_risk) {
        st = save_ctl(c);
        if (st != STS_OK) return st;
    }
    // large states: estimate this step's cut on a sample of tiles first, so
    // that the histogram pass copies a narrow window around it
    if (tiled && c->gate.m >= 1 && c->gate.m <= 4 && c->n_bound >= STS_SAMPLE_MIN)
        STS_LAUNCH(c, STS_K_SAMPLE, launch_group_sample(c->prec, c->gate, b, c->stream));
    b.predict = tiled ? 1 : 0; // the histogram pass also extracts the predicted window
    // and keeps the candidates above it, so that a step whose cut falls in
    // the window writes its survivors without running the gate again
    b.copy = tiled ? 1 : 0;
    STS_LAUNCH(c, STS_K_GROUP_HIST, launch_group_hist(c->prec, c->gate, b, G, tiled, c->stream));
    b.predict = 0;
    STS_LAUNCH(c, STS_K_PICK1, launch_pick1(b, G, 0, tiled ? 1 : 0, c->stream));
    if (side_risk) {
        st = sync_ctl(c);
        if (st != STS_OK) return st;
        if (!c->hctl->keep_all && c->hctl->sub_count > c->scap) return refuse_step(c);
    }
    if (tiled) {
        // as many workgroups as the histogram pass keeps resident: one round
        // of launches when the window held the cut and every one exits
        STS_LAUNCH(c, STS_K_GROUP_EXTRACT,
                   launch_group_extract_tiles(c->prec, c->gate, b, std::min(tt, G), c->stream));
    } else {
        b.epoch = next_epoch(c);
        STS_LAUNCH(c, STS_K_GROUP_EXTRACT,
                   launch_group_compact(c->prec, STS_KIND_EXTRACT, c->gate, b, tiles, c->stream));
    }
    // the side passes stream the side buffer; 128 workgroups keep it moving,
    // and more would only queue more atomics on the shared bins and the
    // last-workgroup counter
    const int sg = (int)std::min<u64>(std::max<u64>(ceil_div(std::min(cb, c->scap), 256), 1), STS_SIDE_GROUPS);
    STS_LAUNCH(c, STS_K_SIDE_HIST, launch_side_hist(b, c->h2, sg, c->stream));
    // the extraction keeps no per-workgroup state: one wave per tile keeps
    // every tile's loads in flight at once
    STS_LAUNCH(c, STS_K_SIDE_EXTRACT, launch_side_extract(b, tiled ? std::max(sg, (tt + 3) / 4) : sg, c->stream));
    STS_LAUNCH(c, STS_K_FINAL, launch_final(b, c->stream));
    if (out_risk) {
        // only p-mass limits this cut: learn its size before writing
        st = sync_ctl(c);
        if (st != STS_OK) return st;
        const u64 L = c->hctl->keep_all ? c->hctl->n_cand : c->hctl->L;
        if (L > c->cap) return refuse_step(c);
        nb = L;
    }
    if (tiled) {
        STS_LAUNCH(c, STS_K_TILE_KEPT, launch_tile_kept(b, tt, c->stream));
        STS_LAUNCH(c, STS_K_TILE_SCAN, launch_tile_scan(b, tt, c->stream));
        STS_LAUNCH(c, STS_K_GROUP_EMIT, launch_group_emit_tiles(c->prec, c->gate, b, tt, c->stream));
    } else {
        b.epoch = next_epoch(c);
        STS_LAUNCH(c, STS_K_GROUP_EMIT, launch_group_compact(c->prec, STS_KIND_EMIT, c->gate, b, tiles, c->stream));
    }
    c->cur = out;
    c->n_bound = nb;
    c->pending = false;
    return STS_OK;
}

sts_status sts_set_sort_shape(sts_ctx *c, int small_log2, int shape)
{
    static_assert(STS_SORT_8x16 == STS_RADIX_8x16 && STS_SORT_8x8 == STS_RADIX_8x8 &&
                      STS_SORT_11x16 == STS_RADIX_11x16 && STS_SORT_11x8 == STS_RADIX_11x8,
                  "public and internal sort shapes agree");
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (small_log2 < 0 || small_log2 > 40 || shape < 0 || shape >= STS_RADIX_SHAPES) return STS_E_ARG;
    if (c->pending) return STS_E_STATE; // the pending gate's sort already ran with the old shape
    c->radix_small_log2 = small_log2;
    c->radix_small_shape = shape;
    return STS_OK;
}

sts_status sts_peak(sts_ctx *c, uint64_t *key, double *prob)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (!key || !prob) return STS_E_ARG;
    st = materialise(c);
    if (st != STS_OK) return st;
    const GateArg g = identity_gate();
    PassBufs b = pass_bufs(c, c->cur, -1);
    b.gate = c->dgate_id;
    const int G = hist_groups(c->prec, c->n_bound, 0, true);
    STS_LAUNCH(c, STS_K_GROUP_HIST, launch_group_hist(c->prec, g, b, G, true, c->stream));
    STS_LAUNCH(c, STS_K_PICK1, launch_pick1(b, G, 1, 0, c->stream));
    st = sync_ctl(c);
    if (st != STS_OK) return st;
    if (c->hctl->cnt[c->cur] == 0) return STS_E_STATE;
    *key = c->hctl->peak_key;
    *prob = c->hctl->peak_w / c->hctl->peak_W;
    return STS_OK;
}

sts_status sts_num_terms(sts_ctx *c, uint64_t *n)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (!n) return STS_E_ARG;
    st = materialise(c);
    if (st != STS_OK) return st;
    st = sync_ctl(c);
    if (st != STS_OK) return st;
    *n = c->hctl->cnt[c->cur];
    c->n_bound = *n;
    return STS_OK;
}

sts_status sts_read_terms(sts_ctx *c, uint64_t cap, uint64_t *keys, double *amps, uint64_t *n)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (!n || (cap && (!keys || !amps))) return STS_E_ARG;
    st = sts_num_terms(c, n);
    if (st != STS_OK) return st;
    const u64 cnt = *n;
    if (cnt > cap) return STS_E_CAPACITY;
    if (cnt == 0) return STS_OK;
    std::vector<u64> k(cnt);
    STS_TRY(c, hipMemcpyAsync(k.data(), c->keys[c->cur], cnt * 8, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> a(2 * cnt);
    std::vector<float> af;
    if (c->prec == STS_C128) {
        STS_TRY(c, hipMemcpyAsync(a.data(), c->amps[c->cur], cnt * 16, hipMemcpyDeviceToHost, c->stream));
    } else {
        af.resize(2 * cnt);
        STS_TRY(c, hipMemcpyAsync(af.data(), c->amps[c->cur], cnt * 8, hipMemcpyDeviceToHost, c->stream));
    }
    STS_TRY(c, hipStreamSynchronize(c->stream));
    if (c->prec == STS_C64)
        for (u64 i = 0; i < 2 * cnt; ++i) a[i] = (double)af[i];
    std::vector<u64> order(cnt);
    for (u64 i = 0; i < cnt; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](u64 x, u64 y) { return k[x] < k[y]; });
    for (u64 i = 0; i < cnt; ++i) {
        keys[i] = k[order[i]];
        amps[2 * i] = a[2 * order[i]];
        amps[2 * i + 1] = a[2 * order[i] + 1];
    }
    return STS_OK;
}

sts_status sts_load_terms(sts_ctx *c, uint64_t n, const uint64_t *keys, const double *amps)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (n && (!keys || !amps)) return STS_E_ARG;
    if (n > c->cap) return STS_E_CAPACITY;
    const u64 lim = c->n_qubits == 64 ? ~0ull : ((1ull << c->n_qubits) - 1);
    std::vector<u64> sk(keys, keys + n);
    for (u64 i = 0; i < n; ++i)
        if (sk[i] > lim || !std::isfinite(amps[2 * i]) || !std::isfinite(amps[2 * i + 1])) return STS_E_ARG;
    std::sort(sk.begin(), sk.end());
    for (u64 i = 1; i < n; ++i)
        if (sk[i] == sk[i - 1]) return STS_E_ARG;
    // the state is replaced: any pending gate is dropped
    c->pending = false;
    if (n) {
        STS_TRY(c, hipMemcpyAsync(c->keys[c->cur], keys, n * 8, hipMemcpyHostToDevice, c->stream));
        if (c->prec == STS_C128) {
            STS_TRY(c, hipMemcpyAsync(c->amps[c->cur], amps, n * 16, hipMemcpyHostToDevice, c->stream));
            STS_TRY(c, hipStreamSynchronize(c->stream));
        } else {
            std::vector<float> af(2 * n);
            for (u64 i = 0; i < 2 * n; ++i) af[i] = (float)amps[i];
            STS_TRY(c, hipMemcpyAsync(c->amps[c->cur], af.data(), n * 8, hipMemcpyHostToDevice, c->stream));
            STS_TRY(c, hipStreamSynchronize(c->stream));
        }
    }
    STS_TRY(c, launch_set_n(&c->ctl->cnt[c->cur], n, c->stream));
    c->n_bound = n;
    return STS_OK;
}

sts_status sts_stats(sts_ctx *c, double *W, double *kept_fraction, double *log10_cum_kept, uint64_t *last_candidates)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    st = sync_ctl(c);
    if (st != STS_OK) return st;
    if (W) *W = c->hctl->W;
    if (kept_fraction) *kept_fraction = c->hctl->frac;
    if (log10_cum_kept) *log10_cum_kept = c->hctl->log10_cum;
    if (last_candidates) *last_candidates = c->hctl->n_cand;
    return STS_OK;
}

sts_status sts_counters(sts_ctx *c, uint64_t *gate_steps, uint64_t *term_updates, uint64_t *candidates)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    st = sync_ctl(c);
    if (st != STS_OK) return st;
    if (gate_steps) *gate_steps = c->hctl->tot_steps;
    if (term_updates) *term_updates = c->hctl->tot_updates;
    if (candidates) *candidates = c->hctl->tot_cand;
    return STS_OK;
}

sts_status sts_profile(sts_ctx *c, int enable)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    c->prof = enable != 0;
    return STS_OK;
}

sts_status sts_kernel_time(sts_ctx *c, int kind, int reset, double *total_ms, uint64_t *launches)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    if (kind < 0 || kind >= STS_K_COUNT) return STS_E_ARG;
    STS_TRY(c, hipStreamSynchronize(c->stream));
    prof_collect(c);
    if (total_ms) *total_ms = c->prof_ms[kind];
    if (launches) *launches = c->prof_n[kind];
    if (reset) {
        for (int k = 0; k < STS_K_COUNT; ++k) {
            c->prof_ms[k] = 0;
            c->prof_n[k] = 0;
        }
    }
    return STS_OK;
}

sts_status sts_step_static(int n_qubits, uint64_t max_terms, double mass, int precision, void *hip_stream, int m,
                           const int *qubits, const double *U, const uint64_t *keys_in, const void *amps_in,
                           uint64_t n_in, uint64_t *keys_out, void *amps_out, uint64_t *n_out, double *stats)
{
    if (n_qubits < 1 || n_qubits > 64 || (precision != STS_C128 && precision != STS_C64)) return STS_E_ARG;
    if (!(mass == mass) || !qubits || !U || m < 1 || m > 3 || m > n_qubits) return STS_E_ARG;
    if ((n_in && (!keys_in || !amps_in)) || !keys_out || !amps_out || !n_out) return STS_E_ARG;
    if (n_qubits < 64) max_terms = std::min<u64>(max_terms, 1ull << n_qubits);
    if (max_terms == 0) return STS_E_ARG; // top-k bounds the result and the caller's output arrays
    if (max_terms > STS_STATIC_MAX_TERMS || n_in > STS_STATIC_MAX_TERMS) return STS_E_CAPACITY;
    const Layout L = make_layout(STS_STATIC_MAX_TERMS, precision);
    if (L.total > kStaticBytes) return STS_E_CAPACITY;
    void *base = nullptr;
    if (static_scratch(&base) != hipSuccess) return STS_E_HIP;

    // a context on the stack over the static array: with gates of at most 3
    // qubits and top-k within the capacity, the gate step never synchronises,
    // never allocates and is never refused
    sts_ctx c;
    c.n_qubits = n_qubits;
    c.prec = precision;
    c.K = max_terms;
    c.p = (mass > 0.0 && mass < 1.0) ? mass : 0.0;
    c.stream = (hipStream_t)hip_stream;
    c.cap = STS_STATIC_MAX_TERMS;
    c.scap = side_capacity(c.cap);
    c.tiles_cap = ceil_div(c.cap, 2048) + 1;
    c.gtiles_cap = ceil_div(c.cap, STS_GTILE);
    c.mem = (unsigned char *)base;
    bind_layout(&c, L);
    // the array keeps the last call's contents: every counter, histogram and
    // look-back word starts from zero again, and the control block anew
    STS_TRY(&c, launch_fill_zero((u64 *)(c.mem + L.h1), (L.total - L.h1) / 8, c.stream));
    STS_TRY(&c, launch_ctl_begin(c.ctl, c.K, c.p, n_in, c.stream));
    STS_TRY(&c, launch_set_gate(identity_gate(), c.dgate_id, c.stream));
    const u64 asz = precision == STS_C128 ? 16 : 8;
    if (n_in) {
        STS_TRY(&c, hipMemcpyAsync(c.keys[0], keys_in, n_in * 8, hipMemcpyDeviceToDevice, c.stream));
        STS_TRY(&c, hipMemcpyAsync(c.amps[0], amps_in, n_in * asz, hipMemcpyDeviceToDevice, c.stream));
    }
    c.cur = 0;
    c.n_bound = n_in;
    sts_status st = sts_apply_gate(&c, m, qubits, U);
    if (st != STS_OK) return st;
    st = sts_truncate(&c);
    if (st != STS_OK) return st;
    STS_TRY(&c, launch_terms_out(c.keys[c.cur], c.amps[c.cur], (int)asz, c.ctl, c.cur, (u64 *)keys_out, amps_out,
                                 max_terms, (u64 *)n_out, stats, c.stream));
    return STS_OK;
}

void sts_free(sts_ctx *c)
{
    if (!c) return;
    if (c->stream || c->mem) (void)hipStreamSynchronize(c->stream);
    for (auto &m : c->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->own_mem && c->mem) (void)hipFree(c->mem);
    if (c->hctl) (void)hipHostFree(c->hctl);
    if (c->hU) (void)hipHostFree(c->hU);
    if (c->u_event) (void)hipEventDestroy(c->u_event);
    delete c;
}

const char *sts_strerror(sts_status s)
{
    switch (s) {
    case STS_OK: return "ok";
    case STS_E_ARG: return "invalid argument";
    case STS_E_NOMEM: return "device allocation failed";
    case STS_E_CAPACITY: return "result exceeds the context's capacity";
    case STS_E_HIP: return "HIP runtime error";
    case STS_E_STATE: return "context poisoned or call out of order";
    }
    return "unknown status";
}

} // extern "C"

// ---------------------------------------------------------------------------
// Replayed gate steps (batch runner). A truncated step of up to 3 qubits
// launches the same kernels with the same grids whenever the context starts
// it from the same term buffer with the same size bound: every size the
// kernels use is read from device memory, and the gate itself from the
// context's device copy, written by one k_set_gate launch. Such a step is
// captured into a HIP graph once and afterwards replayed with only that
// launch's argument changed to the new gate.
// ---------------------------------------------------------------------------
struct StepGraph {
    int m, cur;
    u64 nb;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipGraphNode_t set_node;
    int cur_after;
    u64 nb_after;
};

struct StepGraphs {
    std::vector<StepGraph> v;
    u64 last_nb = ~0ull;
    u64 replays = 0, captures = 0;
};

StepGraphs *step_graphs_new() { return new (std::nothrow) StepGraphs(); }

void step_graphs_free(StepGraphs *gs)
{
    if (!gs) return;
    for (auto &e : gs->v) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        if (e.graph) (void)hipGraphDestroy(e.graph);
    }
    delete gs;
}

void step_graphs_counts(const StepGraphs *gs, u64 *captures, u64 *replays)
{
    *captures = gs ? gs->captures : 0;
    *replays = gs ? gs->replays : 0;
}

sts_status step_replayed(sts_ctx *c, StepGraphs *gs, int m, const int *qubits, const double *U)
{
    sts_status st = check_live(c);
    if (st != STS_OK) return st;
    st = check_gate(c, m, qubits, U);
    if (st != STS_OK) return st;
    // a steady size bound (as the previous step's) and a step that never
    // synchronises: gates of up to 3 qubits, top-k within the capacity
    const bool steady = c->n_bound == gs->last_nb;
    gs->last_nb = c->n_bound;
    if (!steady || c->pending || c->prof || m > 3 || c->K == 0 || c->K > c->cap) {
        st = sts_apply_gate(c, m, qubits, U);
        if (st == STS_OK) st = sts_truncate(c);
        return st;
    }
    StepGraph *hit = nullptr;
    for (auto &e : gs->v)
        if (e.m == m && e.cur == c->cur && e.nb == c->n_bound) hit = &e;
    if (!hit) {
        StepGraph e{};
        e.m = m;
        e.cur = c->cur;
        e.nb = c->n_bound;
        STS_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        st = sts_apply_gate(c, m, qubits, U);
        if (st == STS_OK) st = sts_truncate(c);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(c->stream, &graph);
        if (st != STS_OK || ee != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            c->poisoned = true; // the step was recorded, not run
            return st != STS_OK ? st : STS_E_HIP;
        }
        e.graph = graph;
        e.cur_after = c->cur;
        e.nb_after = c->n_bound;
        // the one launch that writes the gate
        size_t nn = 0;
        hipError_t he = hipGraphGetNodes(graph, nullptr, &nn);
        std::vector<hipGraphNode_t> nodes(nn);
        if (he == hipSuccess) he = hipGraphGetNodes(graph, nodes.data(), &nn);
        for (size_t i = 0; he == hipSuccess && i < nn; ++i) {
            hipGraphNodeType t;
            if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams p{};
            if (hipGraphKernelNodeGetParams(nodes[i], &p) == hipSuccess && p.func == set_gate_kernel())
                e.set_node = nodes[i];
        }
        if (he == hipSuccess && !e.set_node) he = hipErrorNotFound;
        if (he == hipSuccess) he = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        if (he == hipSuccess) he = hipGraphLaunch(e.exec, c->stream);
        if (he != hipSuccess) {
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
            (void)hipGraphDestroy(graph);
            return fail_hip(c, he);
        }
        gs->v.push_back(e);
        gs->captures += 1;
        return STS_OK;
    }
    // replay with the new gate: the same bucket bits (same size bound)
    GateArg g;
    fill_gate(&g, m, qubits, U);
    g.hb = sts_radix_bits(sort_shape(c)) * sort_passes(c);
    GateArg *dst = c->dgate;
    void *args[2] = {&g, &dst};
    hipKernelNodeParams p{};
    p.func = const_cast<void *>(set_gate_kernel());
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    STS_TRY(c, hipGraphExecKernelNodeSetParams(hit->exec, hit->set_node, &p));
    STS_TRY(c, hipGraphLaunch(hit->exec, c->stream));
    c->cur = hit->cur_after;
    c->n_bound = hit->nb_after;
    c->gate = g;
    c->gate_dev = c->dgate;
    c->pending = false;
    gs->replays += 1;
    return STS_OK;
}
