// group_impl.h - the gate step proper: find each group of partner terms in the
// bucket-sorted input, multiply it by U in registers, and either histogram
// the new amplitudes' weights or write the survivors.
//
// Gate rule (Eq. (3), generalised to m qubits in Sec. IV.A): for a group
// with rest-of-key r, member j (its bits on the gate's qubits) holds a_j; the
// new term with pattern i has key r | deposit(i) and amplitude
// sum_j U[i][j] a_j over the members present, summed in ascending j from +0
// with complex products (ur*vr - ui*vi, ur*vi + ui*vr), each operation
// rounded once (built with -ffp-contract=off). Exact zeros are not kept
// (Sec. I: only nonzero amplitudes are stored).
//
// The new amplitudes are never stored as candidates: the histogram pass, the
// side-buffer extraction and the final write each recompute them from the
// sorted input (reading 16-24 bytes per input term instead of writing and
// re-reading 2^m times as much).
#pragma once
#include "kernels.h"

namespace sts_group {

template <typename AT> struct Scalar;
template <> struct Scalar<double2> { typedef double T; };
template <> struct Scalar<float2> { typedef float T; };

template <typename AT, int M> struct Group {
    AT v[1 << M];
    u32 present; // bit j: member with pattern j exists (0: this thread leads no group)
    u64 rest;    // key bits outside the gate (the whole key for m = 0)
};

template <int M> __device__ __forceinline__ u32 extract_bits(u64 key, const GateArg &g)
{
    u32 j = 0;
#pragma unroll
    for (int t = 0; t < M; ++t) j |= (u32)((key >> g.q[t]) & 1ull) << t;
    return j;
}

template <int M> __device__ __forceinline__ u64 deposit_bits(u32 i, const GateArg &g)
{
    if (M <= 3) return g.dep[i];
    u64 k = 0;
#pragma unroll
    for (int t = 0; t < M; ++t) k |= (u64)((i >> t) & 1u) << g.q[t];
    return k;
}

template <typename AT, int M> __device__ __forceinline__ void group_clear(Group<AT, M> &G)
{
#pragma unroll
    for (int jj = 0; jj < (1 << M); ++jj) {
        G.v[jj].x = 0;
        G.v[jj].y = 0;
    }
}

// Complex64 groups of 3- and 4-qubit gates are built differently. A group
// has few members (about two of 8 or 16), and a member's pattern is only
// known at run time, so placing it in a register array takes a 2^m-way
// select and the product a dense 2^m x 2^m pass. Instead the group holds its
// 2^m outputs, and each member found adds its column of U (read from LDS by
// the member's pattern) times its amplitude. The outputs sum the members in
// the order the group scan finds them: the same in every pass of a step, and
// in every run, since every pass writes its terms in an order fixed by the
// input (the FP32 path is held to a tolerance, not to the FP64 operation
// order; for 1- and 2-qubit gates the dense product is the faster one).
template <typename AT, int M> struct SparseGroup {
    static constexpr bool value = false;
};
template <int M> struct SparseGroup<float2, M> {
    static constexpr bool value = M >= 3 && M <= 5;
};

// the loops over a group's outputs: unrolled for gates of up to 4 qubits,
// and for complex64 5-qubit groups, whose 32 sums are registers indexed by
// the loop (other 5-qubit groups are read by index from scratch memory)
template <typename AT, int M> struct OutUnroll {
    static constexpr int value = (M <= 4 || SparseGroup<AT, M>::value) ? (1 << M) : 1;
};

// the gate's matrix in LDS, U[i][j] at [2^m i + j] (complex64)
template <int M> __device__ __forceinline__ float2 *gate_table_c64()
{
    __shared__ float2 t[1 << (2 * M)];
    return t;
}

// every kernel that builds groups calls this first, with every thread
template <typename AT, int M> __device__ __forceinline__ void stage_gate(const GateArg &g)
{
    if constexpr (SparseGroup<AT, M>::value) {
        float2 *t = gate_table_c64<M>();
        for (int k = threadIdx.x; k < (1 << (2 * M)); k += blockDim.x) {
            float2 u;
            u.x = M <= 3 ? g.fr[k] : g.uptr_f[2 * k];
            u.y = M <= 3 ? g.fi[k] : g.uptr_f[2 * k + 1];
            t[k] = u;
        }
        __syncthreads();
    }
}

template <typename AT, int M> __device__ __forceinline__ void group_set(Group<AT, M> &G, u32 j, AT a)
{
    if constexpr (SparseGroup<AT, M>::value) {
        const float2 *t = gate_table_c64<M>();
#pragma unroll
        for (int i = 0; i < (1 << M); ++i) {
            const float2 u = t[(1 << M) * i + (int)j];
            G.v[i].x = __builtin_fmaf(u.x, a.x, G.v[i].x);
            G.v[i].x = __builtin_fmaf(-u.y, a.y, G.v[i].x);
            G.v[i].y = __builtin_fmaf(u.x, a.y, G.v[i].y);
            G.v[i].y = __builtin_fmaf(u.y, a.x, G.v[i].y);
        }
    } else {
#pragma unroll
        for (int jj = 0; jj < (1 << M); ++jj)
            if (jj == (int)j) G.v[jj] = a;
    }
    G.present |= 1u << j;
}

// Load the group led by element idx. The leader is the first element (in
// sorted order) of its group; every other member returns an empty group.
template <typename AT, int M>
__device__ __forceinline__ void load_group(const GateArg &g, const u64 *__restrict__ keys,
                                           const AT *__restrict__ amps, u64 idx, u64 n, Group<AT, M> &G)
{
    G.present = 0;
    G.rest = 0;
    if (idx >= n) return;
    const u64 key = keys[idx];
    const AT amp = amps[idx];
    if (M == 0) {
        G.rest = key;
        G.v[0] = amp;
        G.present = 1;
        return;
    }
    const u64 rest = key & g.notmask;
    const int sh = 64 - g.hb;
    const u64 b = sts_mix64(rest) >> sh;
    for (u64 p = idx; p > 0; --p) {
        const u64 mp = keys[p - 1] & g.notmask;
        if ((sts_mix64(mp) >> sh) != b) break;
        if (mp == rest) return; // an earlier member leads this group
    }
    G.rest = rest;
    group_clear<AT, M>(G);
    group_set<AT, M>(G, extract_bits<M>(key, g), amp);
    for (u64 p = idx + 1; p < n; ++p) {
        const u64 kp = keys[p];
        const u64 mp = kp & g.notmask;
        if ((sts_mix64(mp) >> sh) != b) break;
        if (mp == rest) group_set<AT, M>(G, extract_bits<M>(kp, g), amps[p]);
    }
}

// a load through the constant address space: the matrix of a 4- or 5-qubit
// gate is read-only while a kernel runs and the same in every lane, so its
// entries come in by scalar loads (a plain pointer may alias the kernel's
// stores, and its loads would each wait in the vector memory pipe)
template <typename T> __device__ __forceinline__ T ld_const(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}

// entry U[i][j] in the arithmetic type R of the amplitudes (FP32 entries
// were rounded once on the host; m >= 4 reads the copies in device memory)
template <typename R, int M> struct UEntry;
template <int M> struct UEntry<double, M> {
    static __device__ __forceinline__ double re(const GateArg &g, int i, int j)
    {
        return M <= 3 ? g.ur[i * (1 << M) + j] : ld_const(&g.uptr[2 * (i * (1 << M) + j)]);
    }
    static __device__ __forceinline__ double im(const GateArg &g, int i, int j)
    {
        return M <= 3 ? g.ui[i * (1 << M) + j] : ld_const(&g.uptr[2 * (i * (1 << M) + j) + 1]);
    }
};
template <int M> struct UEntry<float, M> {
    static __device__ __forceinline__ float re(const GateArg &g, int i, int j)
    {
        return M <= 3 ? g.fr[i * (1 << M) + j] : ld_const(&g.uptr_f[2 * (i * (1 << M) + j)]);
    }
    static __device__ __forceinline__ float im(const GateArg &g, int i, int j)
    {
        return M <= 3 ? g.fi[i * (1 << M) + j] : ld_const(&g.uptr_f[2 * (i * (1 << M) + j) + 1]);
    }
};

// new amplitude with local pattern i of the group
template <typename AT, int M>
__device__ __forceinline__ AT group_out(const GateArg &g, const Group<AT, M> &G, int i)
{
    typedef typename Scalar<AT>::T R;
    if (M == 0) return G.v[0];
    if constexpr (SparseGroup<AT, M>::value) return G.v[i]; // accumulated by group_set
    R ar = (R)0, ai = (R)0;
    if (sizeof(R) == 4) {
        // complex64: fused multiply-adds (the FP32 path is held to a
        // tolerance, not to the FP64 operation order); absent members are
        // zero and add nothing. The member loop is always unrolled, so the
        // group's registers are only indexed by constants.
#pragma unroll
        for (int j = 0; j < (1 << M); ++j) {
            const R ur = UEntry<R, M>::re(g, i, j);
            const R ui = UEntry<R, M>::im(g, i, j);
            const R vr = G.v[j].x, vi = G.v[j].y;
            ar = __builtin_fmaf(ur, vr, ar);
            ar = __builtin_fmaf(-ui, vi, ar);
            ai = __builtin_fmaf(ur, vi, ai);
            ai = __builtin_fmaf(ui, vr, ai);
        }
    } else {
        // complex128: the oracle's order - each product and sum rounded once,
        // members summed in ascending j; an absent member leaves the sum
        // untouched (selected away, not added as zero, so signed zeros match)
#pragma unroll
        for (int j = 0; j < (1 << M); ++j) {
            const R ur = UEntry<R, M>::re(g, i, j);
            const R ui = UEntry<R, M>::im(g, i, j);
            const R vr = G.v[j].x, vi = G.v[j].y;
            const R tr = ur * vr - ui * vi;
            const R ti = ur * vi + ui * vr;
            const R nr = ar + tr, ni = ai + ti;
            const bool has = (G.present >> j) & 1u;
            ar = has ? nr : ar;
            ai = has ? ni : ai;
        }
    }
    AT o;
    o.x = ar;
    o.y = ai;
    return o;
}

template <typename AT> __device__ __forceinline__ bool nonzero(AT a) { return a.x != 0 || a.y != 0; }

template <typename AT> __device__ __forceinline__ u64 weight_bits(AT a)
{
    return sts_dbits(sts_weight((double)a.x, (double)a.y));
}

// complex64: both squares are exact in binary64 (24-bit significands), so a
// fused multiply-add rounds the same sum once, with one instruction fewer
template <> __device__ __forceinline__ u64 weight_bits<float2>(float2 a)
{
    const double x = (double)a.x, y = (double)a.y;
    return sts_dbits(__builtin_fma(x, x, y * y));
}

// ---------------------------------------------------------------------------
// pass 1: histogram of the new weights by exponent field, with exact
// mantissa sums, plus each workgroup's best term (weight desc, key asc)
// ---------------------------------------------------------------------------
template <typename AT, int M>
__global__ void __launch_bounds__(STS_WG) k_group_hist(const GateArg *__restrict__ gp, PassBufs b)
{
    const GateArg &g = *gp;
    stage_gate<AT, M>(g);
    __shared__ u32 s_cnt[STS_NBIN];
    __shared__ u64 s_hi[STS_NBIN];
    __shared__ u64 s_lo[STS_NBIN];
    __shared__ u64 s_bw[STS_WG / 64], s_bk[STS_WG / 64];
    for (int i = threadIdx.x; i < STS_NBIN; i += STS_WG) {
        s_cnt[i] = 0;
        s_hi[i] = 0;
        s_lo[i] = 0;
    }
    __syncthreads();
    const u64 n = *b.n_in;
    const u64 *keys = b.keys;
    const AT *amps = (const AT *)b.amps;
    u64 bw = 0, bk = ~0ull; // bw: weight bits | 2^63 when set
    for (u64 idx = (u64)blockIdx.x * STS_WG + threadIdx.x; idx < n; idx += (u64)gridDim.x * STS_WG) {
        Group<AT, M> G;
        load_group<AT, M>(g, keys, amps, idx, n, G);
        if (!G.present) continue;
#pragma unroll OutUnroll<AT, M>::value
        for (int i = 0; i < (1 << M); ++i) {
            const AT o = group_out<AT, M>(g, G, i);
            if (M > 0 && !nonzero(o)) continue;
            const u64 wb = weight_bits(o);
            const u32 e = (u32)(wb >> 52);
            const u64 mant = sts_mant(wb);
            atomicAdd(&s_cnt[e], 1u);
            atomicAdd(&s_hi[e], mant >> 26);
            atomicAdd(&s_lo[e], mant & ((1ull << 26) - 1));
            const u64 key = G.rest | deposit_bits<M>((u32)i, g);
            const u64 tagged = wb | (1ull << 63);
            if (tagged > bw || (tagged == bw && key < bk)) {
                bw = tagged;
                bk = key;
            }
        }
    }
    // workgroup best: wave reduction then across waves
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const u64 ow = __shfl_xor(bw, d, 64);
        const u64 ok = __shfl_xor(bk, d, 64);
        if (ow > bw || (ow == bw && ok < bk)) {
            bw = ow;
            bk = ok;
        }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        s_bw[threadIdx.x >> 6] = bw;
        s_bk[threadIdx.x >> 6] = bk;
    }
    for (int i = threadIdx.x; i < STS_NBIN; i += STS_WG) {
        const u32 c = s_cnt[i];
        if (c) {
            atomicAdd(&b.h1[i], (u64)c);
            atomicAdd(&b.h1[STS_NBIN + i], s_hi[i]);
            atomicAdd(&b.h1[2 * STS_NBIN + i], s_lo[i]);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 w = s_bw[0], k = s_bk[0];
        for (int i = 1; i < STS_WG / 64; ++i) {
            if (s_bw[i] > w || (s_bw[i] == w && s_bk[i] < k)) {
                w = s_bw[i];
                k = s_bk[i];
            }
        }
        b.best[blockIdx.x] = w;
        b.best[STS_MAX_GROUPS + blockIdx.x] = k;
    }
}

// ---------------------------------------------------------------------------
// compaction passes, ordered by tile with decoupled look-back:
//   EXTRACT - candidates whose exponent field is the one holding the cut go
//             to the side buffer as (key, weight bits)
//   EMIT    - survivors (rank <= the cut term's rank) go to the new state,
//             multiplied by the renormalisation scale when terms were dropped
// ---------------------------------------------------------------------------
template <typename AT, int M, int KIND>
__device__ __forceinline__ bool keep_out(const DevCtl *ctl, int materialise, const AT &o, u64 key, int e_star,
                                         u64 thr_w, u64 thr_k)
{
    if (M > 0 && !nonzero(o)) return false;
    if (KIND == STS_KIND_EXTRACT) return (int)(weight_bits(o) >> 52) == e_star;
    if (materialise) return true;
    const u64 wb = weight_bits(o);
    return wb > thr_w || (wb == thr_w && key <= thr_k);
}

template <typename AT, int M, int KIND>
__global__ void __launch_bounds__(STS_WG) k_group_compact(const GateArg *__restrict__ gp, PassBufs b)
{
    const GateArg &g = *gp;
    stage_gate<AT, M>(g);
    typedef typename Scalar<AT>::T R;
    constexpr int IT = STS_GROUP_ITEMS;
    __shared__ u32 s_tile;
    __shared__ u32 s_scratch[STS_WG / 64];
    __shared__ u64 s_base;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const u32 t = atomicAdd(b.tile_ctr, 1u);
        if (t == gridDim.x - 1) st_agent(b.tile_ctr, 0u);
        s_tile = t;
    }
    __syncthreads();
    const u64 tile = s_tile;
    DevCtl *ctl = b.ctl;
    const int materialise = b.materialise;
    if (KIND == STS_KIND_EXTRACT && ctl->keep_all) return;
    const u64 n = *b.n_in;
    const u64 ntiles = (n + STS_GTILE - 1) / STS_GTILE;
    if (tile >= ntiles) {
        if (tile == 0) { // empty input: publish the empty result
            if (tid == 0) {
                if (KIND == STS_KIND_EXTRACT) {
                    ctl->side_n = 0;
                    ctl->side_dense = 1;
                } else {
                    *b.n_out = 0;
                }
            }
        }
        return;
    }
    const bool keep_everything = KIND == STS_KIND_EMIT && (materialise || ctl->keep_all);
    const int e_star = ctl->e_star;
    const u64 thr_w = ctl->thr_wbits, thr_k = ctl->thr_key;
    const bool rescale = KIND == STS_KIND_EMIT && !materialise && !ctl->keep_all && ctl->dropped;
    const double scale = ctl->scale;
    const u64 *keys = b.keys;
    const AT *amps = (const AT *)b.amps;

    // count this thread's outputs
    u32 mine = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const u64 idx = tile * STS_GTILE + (u64)k * STS_WG + tid;
        Group<AT, M> G;
        load_group<AT, M>(g, keys, amps, idx, n, G);
        if (!G.present) continue;
#pragma unroll OutUnroll<AT, M>::value
        for (int i = 0; i < (1 << M); ++i) {
            const AT o = group_out<AT, M>(g, G, i);
            const u64 key = G.rest | deposit_bits<M>((u32)i, g);
            const bool keep = keep_everything ? (M == 0 || nonzero(o))
                                              : keep_out<AT, M, KIND>(ctl, materialise, o, key, e_star, thr_w, thr_k);
            mine += keep ? 1u : 0u;
        }
    }
    u32 tile_total;
    const u32 my_off = block_excl_scan<u32, STS_WG>(mine, s_scratch, &tile_total);
    if (tid == 0) s_base = lb_exclusive(b.look, 1, tile, tile_total, b.epoch);
    __syncthreads();
    const u64 base = s_base + my_off;
    if (tid == 0 && tile == ntiles - 1) {
        const u64 total = base + tile_total;
        if (KIND == STS_KIND_EXTRACT) {
            ctl->side_n = total;
            ctl->side_dense = 1;
        } else {
            *b.n_out = total;
        }
    }
    if (mine == 0) return;

    // write them
    u64 pos = base;
    const u64 cap = KIND == STS_KIND_EXTRACT ? b.side_cap : b.out_cap;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const u64 idx = tile * STS_GTILE + (u64)k * STS_WG + tid;
        Group<AT, M> G;
        load_group<AT, M>(g, keys, amps, idx, n, G);
        if (!G.present) continue;
#pragma unroll OutUnroll<AT, M>::value
        for (int i = 0; i < (1 << M); ++i) {
            AT o = group_out<AT, M>(g, G, i);
            const u64 key = G.rest | deposit_bits<M>((u32)i, g);
            const bool keep = keep_everything ? (M == 0 || nonzero(o))
                                              : keep_out<AT, M, KIND>(ctl, materialise, o, key, e_star, thr_w, thr_k);
            if (!keep) continue;
            if (pos >= cap) {
                atomicOr(&ctl->flags, KIND == STS_KIND_EXTRACT ? STS_F_SIDE_OVERFLOW : STS_F_OUT_OVERFLOW);
                ++pos;
                continue;
            }
            if (KIND == STS_KIND_EXTRACT) {
                b.side_key[pos] = key;
                b.side_w[pos] = weight_bits(o);
            } else {
                if (rescale) {
                    o.x = (R)((double)o.x * scale);
                    o.y = (R)((double)o.y * scale);
                }
                b.out_keys[pos] = key;
                ((AT *)b.out_amps)[pos] = o;
            }
            ++pos;
        }
    }
}

// ---------------------------------------------------------------------------
// LDS-tiled passes (gates of up to 4 qubits). A workgroup stages a tile of
// TT_TG sorted terms plus a halo of TT_H on each side (keys and hash
// buckets) in LDS, so the partner search reads LDS; a run that crosses the
// halo continues in global memory. Tile t owns slab t of the side buffer
// (2048 << m entries) and writes its survivors at an offset from a scan of
// per-tile counts, so no pass needs atomics across workgroups.
// ---------------------------------------------------------------------------
constexpr int TT_IT = 8;
constexpr int TT_TG = STS_WG * TT_IT;   // 2048 terms per tile
constexpr int TT_H = 64;
constexpr int TT_LD = TT_TG + 2 * TT_H;
constexpr int TT_EBASE = 1023 - 127 + 8; // exponent fields [904, 1032) live in LDS bins
constexpr int TT_NB = 128;

// bkt holds the low 16 bits of each key's hash bucket: neighbouring runs in
// the sorted order have neighbouring buckets, which differ there, so a run of
// equal low bits is the run of equal buckets (the key test decides the group)
template <typename AT> struct TileSmem {
    u64 key[TT_LD];
    unsigned short bkt[TT_LD];
};

__device__ __forceinline__ u32 tile_bucket(u64 key, u64 notmask, int sh)
{
    return (u32)(sts_mix64(key & notmask) >> sh) & 0xffffu;
}

// stage the keys of global terms [lo, hi) and their hash buckets into LDS:
// every load of the thread is issued before any of them is used, so the tile
// costs one memory latency. Amplitudes stay in global memory: a thread reads
// its own term's (coalesced), and a group leader its members' (neighbours,
// already in cache), which keeps the tile small and the occupancy high.
template <typename AT, int M>
__device__ __forceinline__ void stage_tile(TileSmem<AT> &s, const GateArg &g, const u64 *__restrict__ keys,
                                           const AT *__restrict__ amps, u64 lo, u64 hi)
{
    (void)amps;
    constexpr int PER = (TT_LD + STS_WG - 1) / STS_WG;
    const int sh = 64 - g.hb;
    const int cnt = (int)(hi - lo);
    u64 kk[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int li = r * STS_WG + (int)threadIdx.x;
        if (li < cnt) kk[r] = keys[lo + li];
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int li = r * STS_WG + (int)threadIdx.x;
        if (li < cnt) {
            s.key[li] = kk[r];
            if (M > 0) s.bkt[li] = (unsigned short)tile_bucket(kk[r], g.notmask, sh);
        }
    }
}

// whether term e (global index) leads its group: no earlier term of the
// staged tile [lo, hi), or before it, has the same rest of key (the backward
// half of tile_group's scan)
template <int M>
__device__ __forceinline__ bool tile_leads(const unsigned short *bkt, const u64 *skey, const GateArg &g,
                                           const u64 *__restrict__ keys, u64 lo, u64 n, u64 e)
{
    if (e >= n) return false;
    if (M == 0) return true;
    const int li = (int)(e - lo);
    const u64 nm = g.notmask;
    const u64 rest = skey[li] & nm;
    const u32 b = bkt[li];
    int p = li - 1;
    for (; p >= 0; --p) {
        if (bkt[p] != b) return true;
        if ((skey[p] & nm) == rest) return false;
    }
    // the run goes on below the staged range
    const int sh = 64 - g.hb;
    for (u64 q = lo; q > 0; --q) {
        const u64 kq = keys[q - 1];
        if (tile_bucket(kq, nm, sh) != b) break;
        if ((kq & nm) == rest) return false;
    }
    return true;
}

// the group led by term e (global index), from the staged tile [lo, hi).
// Both scans walk LDS with 32-bit local indices; a run that reaches the edge
// of the staged range (rare: the halo is 64 terms) continues in global memory
// after the LDS loop.
template <typename AT, int M>
__device__ __forceinline__ void tile_group(const TileSmem<AT> &s, const GateArg &g, const u64 *__restrict__ keys,
                                           const AT *__restrict__ amps, u64 lo, u64 hi, u64 n, u64 e,
                                           Group<AT, M> &G)
{
    G.present = 0;
    G.rest = 0;
    if (e >= n) return;
    const int li = (int)(e - lo);
    const u64 key = s.key[li];
    const AT amp = amps[e];
    if (M == 0) {
        G.rest = key;
        G.v[0] = amp;
        G.present = 1;
        return;
    }
    const u64 nm = g.notmask;
    const u64 rest = key & nm;
    const u32 b = s.bkt[li];
    const int sh = 64 - g.hb;
    const int last = (int)(hi - lo);
    // the two nearest neighbours on each side read at once (most runs end
    // there), the rest of a run one step at a time
    const bool hp = li > 0, hp2 = li > 1, hn = li + 1 < last, hn2 = li + 2 < last;
    u32 bp = 0, bp2 = 0, bn = 0, bn2 = 0;
    u64 kp = 0, kp2 = 0, kn = 0, kn2 = 0;
    if (hp) {
        bp = s.bkt[li - 1];
        kp = s.key[li - 1];
    }
    if (hp2) {
        bp2 = s.bkt[li - 2];
        kp2 = s.key[li - 2];
    }
    if (hn) {
        bn = s.bkt[li + 1];
        kn = s.key[li + 1];
    }
    if (hn2) {
        bn2 = s.bkt[li + 2];
        kn2 = s.key[li + 2];
    }
    // backward: does an earlier member of this group lead it?
    int p = li - 1;
    if (hp && bp == b) {
        if ((kp & nm) == rest) return;
        p = li - 2;
        if (hp2 && bp2 == b) {
            if ((kp2 & nm) == rest) return;
            for (p = li - 3; p >= 0; --p) {
                if (s.bkt[p] != b) break;
                if ((s.key[p] & nm) == rest) return;
            }
        }
    }
    if (p < 0 && lo > 0) { // the run goes on below the staged range
        for (u64 q = lo; q > 0; --q) {
            const u64 kq = keys[q - 1];
            if (tile_bucket(kq, nm, sh) != b) break;
            if ((kq & nm) == rest) return;
        }
    }
    G.rest = rest;
    group_clear<AT, M>(G);
    group_set<AT, M>(G, extract_bits<M>(key, g), amp);
    // forward: collect the other members
    int f = li + 1;
    if (hn && bn == b) {
        if ((kn & nm) == rest) group_set<AT, M>(G, extract_bits<M>(kn, g), amps[lo + li + 1]);
        f = li + 2;
        if (hn2 && bn2 == b) {
            if ((kn2 & nm) == rest) group_set<AT, M>(G, extract_bits<M>(kn2, g), amps[lo + li + 2]);
            for (f = li + 3; f < last; ++f) {
                if (s.bkt[f] != b) break;
                const u64 kf = s.key[f];
                if ((kf & nm) == rest) group_set<AT, M>(G, extract_bits<M>(kf, g), amps[lo + f]);
            }
        }
    }
    if (f == last) { // the run goes on above the staged range
        for (u64 q = hi; q < n; ++q) {
            const u64 kq = keys[q];
            if (tile_bucket(kq, nm, sh) != b) break;
            if ((kq & nm) == rest) group_set<AT, M>(G, extract_bits<M>(kq, g), amps[q]);
        }
    }
}

// position of this lane's item among the lanes of its wave that keep one,
// plus a base claimed once per wave from an LDS counter
__device__ __forceinline__ u32 wave_claim(bool keep, u32 *counter)
{
    const u64 mask = __ballot(keep);
    if (!mask) return 0;
    const int leader = __ffsll((long long)mask) - 1;
    u32 base = 0;
    if (sts_lane() == leader) base = atomicAdd(counter, (u32)__popcll(mask));
    base = __shfl(base, leader, 64);
    return base + (u32)__popcll(mask & sts_lanemask_lt());
}

// first of `cnt` consecutive slots for this lane (cnt < 2^BITS), the lanes of
// the wave in lane order after a base claimed once per wave from an LDS
// counter. Every lane of the wave must take part.
template <int BITS> __device__ __forceinline__ u32 wave_claim_n(u32 cnt, u32 *counter)
{
    const u64 lt = sts_lanemask_lt();
    u32 pre = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
        const u64 m = __ballot((cnt >> bit) & 1u);
        pre += (u32)__popcll(m & lt) << bit;
        tot += (u32)__popcll(m) << bit;
    }
    if (!tot) return 0;
    const int leader = __ffsll((long long)__ballot(1)) - 1;
    u32 base = 0;
    if (sts_lane() == leader) base = atomicAdd(counter, tot);
    base = __shfl(base, leader, 64);
    return base + pre;
}

// LDS bins of the histogram pass: one per exponent field of
// [TT_EBASE, TT_EBASE + TT_NB) ("cold"), and for the TT_HOT exponent fields
// where most candidates land (from hot_lo: the predicted cut's exponent and
// the ones below it) TT_HSUB sub-bins by the top fraction bits, in
// TT_HCOPIES copies (lane % TT_HCOPIES). Lanes whose weights share a hot
// exponent then spread over TT_HSUB * TT_HCOPIES addresses instead of
// queuing on one; the sub-bins of an exponent are added up when flushed.
constexpr int TT_HOT = 16, TT_HSUB = 4, TT_HCOPIES = 2;
constexpr int TT_HPER = TT_HSUB * TT_HCOPIES;          // slots per hot exponent
constexpr int TT_SLOTS = TT_NB + TT_HOT * TT_HPER;     // 256

__device__ __forceinline__ void flush_one(const PassBufs &b, int e, u64 hi, u64 lo)
{
    const u64 cnt = lo >> 44;
    if (cnt) {
        atomicAdd(&b.h1[e], cnt);
        atomicAdd(&b.h1[STS_NBIN + e], hi);
        atomicAdd(&b.h1[2 * STS_NBIN + e], lo & ((1ull << 44) - 1));
    }
}

// add the LDS bins to the global exponent histogram and clear them
__device__ __forceinline__ void flush_bins(const PassBufs &b, u64 *s_hi, u64 *s_lo, int hot_lo)
{
    for (int i = threadIdx.x; i < TT_NB; i += STS_WG) {
        const u64 hi = s_hi[i], lo = s_lo[i];
        s_hi[i] = 0;
        s_lo[i] = 0;
        flush_one(b, TT_EBASE + i, hi, lo);
    }
    if (threadIdx.x < TT_HOT) {
        u64 hi = 0, lo = 0;
        const int at = TT_NB + (int)threadIdx.x * TT_HPER;
#pragma unroll
        for (int k = 0; k < TT_HPER; ++k) {
            hi += s_hi[at + k];
            lo += s_lo[at + k];
            s_hi[at + k] = 0;
            s_lo[at + k] = 0;
        }
        const int e = hot_lo + (int)threadIdx.x;
        if (e >= 0 && e < STS_NBIN) flush_one(b, e, hi, lo);
    }
}

// add a lane's window mantissa sums to the workgroup's (LDS) and clear them
__device__ __forceinline__ void flush_window(u64 *s_wacc, u64 &ma, u64 &mw)
{
    if (ma) {
        atomicAdd(&s_wacc[1], ma >> 26);
        atomicAdd(&s_wacc[2], ma & ((1ull << 26) - 1));
    }
    if (mw) {
        atomicAdd(&s_wacc[4], mw >> 26);
        atomicAdd(&s_wacc[5], mw & ((1ull << 26) - 1));
    }
    ma = mw = 0;
}

// Level-2 bins of a sampled window: the top 11 fraction bits of the rank
// key inside the window's exponent (as the side-buffer histogram bins them).
// A window spans three sub-bins of 1/32 octave, i.e. at most 192 of them.
constexpr int TT_W2 = 192;
constexpr int TT_W2_LOW = 20; // split of the mantissa sums, as in the side pass

// add a workgroup's level-2 window bins to the device copy and clear them
__device__ __forceinline__ void flush_w2(const PassBufs &b, u64 *s_w2hi, u64 *s_w2lo, u32 d_lo)
{
    for (int i = threadIdx.x; i < TT_W2; i += STS_WG) {
        const u64 lo = s_w2lo[i];
        const u64 c = lo >> 44;
        if (c) {
            const u128 tot = ((u128)s_w2hi[i] << TT_W2_LOW) + (u128)(lo & ((1ull << 44) - 1));
            const u32 d = d_lo + (u32)i;
            atomicAdd(&b.h2w[d], c);
            atomicAdd(&b.h2w[STS_NBIN + d], (u64)(tot >> 26));
            atomicAdd(&b.h2w[2 * STS_NBIN + d], (u64)tot & ((1ull << 26) - 1));
        }
        s_w2hi[i] = 0;
        s_w2lo[i] = 0;
    }
}

// histogram pass over tiles (static tile assignment, persistent grid). With
// b.predict, the candidates whose exponent field equals the previous step's
// cut exponent (ctl->e_pred) also go to the tile's side-buffer slab, and the
// tile's candidates above it are counted: when this step's cut exponent turns
// out the same, the extraction pass has nothing left to do.
// five workgroups per CU for gates of up to 3 qubits; a 4-qubit group (16
// members) needs more registers, and three keep it out of scratch memory
template <typename AT, int M>
__global__ void __launch_bounds__(STS_WG, M >= 4 ? 3 : 5) k_tile_hist(const GateArg *__restrict__ gp, PassBufs b)
{
    const GateArg &g = *gp;
    stage_gate<AT, M>(g);
    constexpr bool kLeadList = M >= 4;
    __shared__ TileSmem<AT> s;
    __shared__ u64 s_hi[TT_SLOTS]; // sum of mantissa >> 26
    __shared__ u64 s_lo[TT_SLOTS]; // sum of mantissa & (2^26-1), plus count << 44
    __shared__ u64 s_bw[STS_WG / 64], s_bk[STS_WG / 64];
    // window sums of the workgroup: candidates above the window, their part in
    // its exponent (mantissa sum >> 26, & (2^26-1)); candidates inside it, the
    // same two sums
    __shared__ u64 s_wacc[6];
    // 4-qubit gates: the tile's group leaders, listed so that every lane of
    // the output loop has a group (about half the terms lead one, and the
    // loop over a group's 16 outputs runs for the whole wave)
    __shared__ unsigned short s_lead[kLeadList ? TT_TG : 1];
    __shared__ u32 s_lscan[STS_WG / 64];
    // level-2 bins of a sampled window (sums split at bit 20, count << 44)
    __shared__ u64 s_w2hi[TT_W2], s_w2lo[TT_W2];
    for (int i = threadIdx.x; i < TT_SLOTS; i += STS_WG) {
        s_hi[i] = 0;
        s_lo[i] = 0;
    }
    for (int i = threadIdx.x; i < TT_W2; i += STS_WG) {
        s_w2hi[i] = 0;
        s_w2lo[i] = 0;
    }
    if (threadIdx.x < 6) s_wacc[threadIdx.x] = 0;
    DevCtl *ctl = b.ctl;
    const u64 n = *b.n_in;
    const u64 *keys = b.keys;
    const AT *amps = (const AT *)b.amps;
    const u64 ntiles = (n + TT_TG - 1) / TT_TG;
    // the window of weights [w_lo, w_hi] copied to the side buffer: the one
    // the sampling pass set for this step, else the previous cut's octave
    int e_w = -1;
    u64 w_lo = 0, w_hi = 0;
    bool fine = false; // a sampled window: also bin its candidates for level 2
    if (b.predict) {
        if (ctl->w_mode) {
            e_w = ctl->e_w;
            w_lo = ctl->w_lo;
            w_hi = ctl->w_hi;
            fine = true;
        } else if (ctl->e_pred >= 0) {
            e_w = ctl->e_pred;
            w_lo = (u64)e_w << 52;
            w_hi = w_lo | ((1ull << 52) - 1);
        }
    }
    const bool predict = e_w >= 0;
    // first level-2 bin of the window (its heaviest weights)
    const u32 d_lo = (u32)((((1ull << 52) - 1) - (w_hi & ((1ull << 52) - 1))) >> 41);
    const u32 d_top = 2047u - d_lo;
    // The window's edges are multiples of 2^47 in the weight bits, so the
    // high words decide: inside when wL <= hi < wH, above when hi >= wH,
    // above but in the window's exponent when also hi < wE1.
    const u32 wL = (u32)(w_lo >> 32), wH = (u32)((w_hi + 1) >> 32), wE1 = (u32)(e_w + 1) << 20;
    // exact mantissa sums of the candidates above the window in its exponent
    // (ma) and inside it (mw): per lane over at most 8 tiles (< 2^12
    // mantissas of < 2^53: no overflow), then added to the workgroup's sums
    // in LDS split at bit 26; their counts come from the per-tile totals
    u64 ma = 0, mw = 0;
    // each wave of a tile owns one slab of 512 << M entries (room for all its
    // candidates): the window's from its start, those above the window from
    // its end, claimed with counters the wave keeps itself
    if (predict && blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->side_dense = 0;
        ctl->side_ntiles = ntiles << 2;
        ctl->side_slab_shift = 9 + M;
        ctl->side_spt_log2 = 2;
    }
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); // uniform: kept in a scalar register
    const int copy = (int)(threadIdx.x % TT_HCOPIES);
    // the hot exponents: the window's and the ones below it (most candidates
    // fall below the cut), else around the previous cut
    const int e_ref = predict ? e_w : (ctl->e_pred >= 0 ? ctl->e_pred : TT_EBASE + 116);
    const int hot_lo = e_ref - (TT_HOT - 4);
    u64 bw = 0, bk = ~0ull;
    int since_flush = 0;
    for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        if (since_flush == 8) {
            // a tile adds at most 2048 * 8 candidates to a bin, so after 8 tiles
            // the low sums stay below 2^43 and the counts below 2^17: flush
            __syncthreads();
            flush_bins(b, s_hi, s_lo, hot_lo);
            if (predict) flush_window(s_wacc, ma, mw);
            if (fine) flush_w2(b, s_w2hi, s_w2lo, d_lo);
            since_flush = 0;
        }
        ++since_flush;
        const u64 base = tile * TT_TG;
        const u64 lo = base > (u64)TT_H ? base - TT_H : 0;
        const u64 hi = base + TT_TG + TT_H < n ? base + TT_TG + TT_H : n;
        __syncthreads(); // previous tile done with the LDS
        stage_tile<AT, M>(s, g, keys, amps, lo, hi);
        __syncthreads();
        int rounds = TT_IT;
        u32 nlead = 0; // the same in every thread
        if constexpr (kLeadList) {
            // listed in term order (a block scan, not claims): the order in
            // which the output loop meets the groups, and so the order of
            // the survivors this step writes, is the same in every run
#pragma unroll 1
            for (int k = 0; k < TT_IT; ++k) {
                const u64 e = base + (u64)k * STS_WG + threadIdx.x;
                const bool lead = tile_leads<M>(s.bkt, s.key, g, keys, lo, n, e);
                u32 tot;
                const u32 at = nlead + block_excl_scan<u32, STS_WG>(lead ? 1u : 0u, s_lscan, &tot);
                if (lead) s_lead[at] = (unsigned short)(e - base);
                nlead += tot;
            }
            __syncthreads();
            rounds = (int)((nlead + STS_WG - 1) / STS_WG);
        }
        const u64 slab = ((tile << 2) + (u64)wv) << (9 + M);
        const bool slab_fits = slab + (512ull << M) <= b.side_cap;
        const bool keep_above = predict && b.copy && slab_fits;
        // the wave's slab: bases in scalar registers, 32-bit offsets per lane
        u64 *const sk = b.side_key + slab;
        u64 *const sw = b.side_w + slab;
        AT *const sa = (AT *)b.side_amp + slab;
        u32 c_in = 0, c_ab = 0; // the wave's claims so far (the same in every lane)
#pragma unroll 1
        for (int k = 0; k < rounds; ++k) {
            u64 e = base + (u64)k * STS_WG + threadIdx.x;
            if constexpr (kLeadList) {
                const u32 j = (u32)k * STS_WG + threadIdx.x;
                e = j < nlead ? base + s_lead[j] : n; // n: no group
            }
            Group<AT, M> G;
            tile_group<AT, M>(s, g, keys, amps, lo, hi, n, e, G);
#pragma unroll OutUnroll<AT, M>::value
            for (int i = 0; i < (1 << M); ++i) {
                const AT o = group_out<AT, M>(g, G, i);
                const bool cand = G.present && (M == 0 || nonzero(o));
                const u64 wb = weight_bits(o);
                const int e_ = (int)(wb >> 52);
                bool ab = false, inw = false;
                if (cand) {
                    const u64 mant = sts_mant(wb);
                    if (predict) {
                        const u32 hw = (u32)(wb >> 32);
                        ab = hw >= wH;
                        inw = hw >= wL && !ab;
                        mw += inw ? mant : 0ull;
                        ma += (ab && hw < wE1) ? mant : 0ull;
                        if (fine && inw) {
                            // digit 2047 - (top 11 fraction bits), less the window's first
                            const u32 rel = d_top - ((hw >> 9) & 2047u);
                            if (rel < (u32)TT_W2) {
                                atomicAdd(&s_w2hi[rel], mant >> TT_W2_LOW);
                                atomicAdd(&s_w2lo[rel], (mant & ((1ull << TT_W2_LOW) - 1)) | (1ull << 44));
                            } else { // outside the window's bins: cannot happen; fail the step
                                atomicOr(&ctl->flags, STS_F_UNRESOLVED);
                            }
                        }
                    }
                    const int bin = e_ - TT_EBASE;
                    const int hd = e_ - hot_lo;
                    if ((unsigned)hd < (unsigned)TT_HOT || (unsigned)bin < (unsigned)TT_NB) {
                        const int f2 = (int)((wb >> 50) & (TT_HSUB - 1));
                        const int slot = (unsigned)hd < (unsigned)TT_HOT ? TT_NB + (hd * TT_HSUB + f2) * TT_HCOPIES + copy : bin;
                        atomicAdd(&s_hi[slot], mant >> 26);
                        atomicAdd(&s_lo[slot], (mant & ((1ull << 26) - 1)) | (1ull << 44));
                    } else { // far outside the usual range: straight to the global bins
                        atomicAdd(&b.h1[e_], 1ull);
                        atomicAdd(&b.h1[STS_NBIN + e_], mant >> 26);
                        atomicAdd(&b.h1[2 * STS_NBIN + e_], mant & ((1ull << 26) - 1));
                    }
                    if (M == 0) { // the peak is only asked of the state itself (sts_peak)
                        const u64 key = G.rest;
                        const u64 tagged = wb | (1ull << 63);
                        if (tagged > bw || (tagged == bw && key < bk)) {
                            bw = tagged;
                            bk = key;
                        }
                    }
                }
                if (predict) {
                    const u64 m_ab = __ballot(ab), m_in = __ballot(inw);
                    if (inw) {
                        if (slab_fits) {
                            const u32 at = c_in + sts_lanes_below(m_in);
                            sts_store_at(sk, at * 8u, G.rest | deposit_bits<M>((u32)i, g));
                            sts_store_at(sw, at * 8u, wb);
                            if (keep_above) sts_store_at(sa, at * (u32)sizeof(AT), o);
                        } else { // cannot happen (the side buffer holds every tile's slabs)
                            atomicOr(&ctl->flags, STS_F_SIDE_OVERFLOW);
                        }
                    } else if (ab && keep_above) {
                        const u32 at = ((512u << M) - 1u) - c_ab - sts_lanes_below(m_ab);
                        sts_store_at(sk, at * 8u, G.rest | deposit_bits<M>((u32)i, g));
                        sts_store_at(sa, at * (u32)sizeof(AT), o);
                    }
                    c_in += (u32)__popcll(m_in);
                    c_ab += (u32)__popcll(m_ab);
                }
            }
        }
        if (predict && sts_lane() == 0) {
            const u64 sl = (tile << 2) + (u64)wv;
            b.t_above[sl] = c_ab;
            b.t_side[sl] = c_in;
            atomicAdd((unsigned long long *)&s_wacc[0], (unsigned long long)c_ab);
            atomicAdd((unsigned long long *)&s_wacc[3], (unsigned long long)c_in);
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const u64 ow = __shfl_xor(bw, d, 64);
        const u64 ok = __shfl_xor(bk, d, 64);
        if (ow > bw || (ow == bw && ok < bk)) {
            bw = ow;
            bk = ok;
        }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        s_bw[threadIdx.x >> 6] = bw;
        s_bk[threadIdx.x >> 6] = bk;
    }
    flush_bins(b, s_hi, s_lo, hot_lo);
    if (fine) flush_w2(b, s_w2hi, s_w2lo, d_lo);
    if (predict) {
        // this workgroup's window sums in its own slots (the pick adds the
        // workgroups up: no global atomics)
        flush_window(s_wacc, ma, mw);
        __syncthreads();
        if (threadIdx.x < 6) b.wpart[threadIdx.x * STS_MAX_GROUPS + blockIdx.x] = s_wacc[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 w = s_bw[0], k = s_bk[0];
        for (int i = 1; i < STS_WG / 64; ++i) {
            if (s_bw[i] > w || (s_bw[i] == w && s_bk[i] < k)) {
                w = s_bw[i];
                k = s_bk[i];
            }
        }
        b.best[blockIdx.x] = w;
        b.best[STS_MAX_GROUPS + blockIdx.x] = k;
    }
}

// ---------------------------------------------------------------------------
// sampling pass (large states): the gate on the first STS_SAMPLE_SPAN inputs
// of STS_SAMPLE_TILES evenly spaced tiles, the candidates' weights counted in
// fine bins (exponent field and the top STS_SW_FB fraction bits, over the
// STS_SW_EXPS exponents around the previous cut) with their masses summed in
// FP32. The last workgroup scales the sample to the whole input, estimates
// the bin where this step's cut falls (the rule of Sec. III applied to the
// sample) and sets the window the histogram pass copies to the side buffer:
// that bin and its two neighbours inside the same exponent field. The
// estimate only decides which candidates are copied; the cut is still found
// exactly, and a window that misses it costs the extraction pass. Without a
// previous cut the pass does nothing (the histogram pass then predicts
// nothing).
// ---------------------------------------------------------------------------
template <typename AT, int M>
__global__ void __launch_bounds__(STS_WG) k_tile_sample(const GateArg *__restrict__ gp, PassBufs b)
{
    const GateArg &g = *gp;
    stage_gate<AT, M>(g);
    constexpr int SPAN = STS_SAMPLE_SPAN; // inputs per workgroup, from a tile's start
    __shared__ TileSmem<AT> s;
    __shared__ u32 s_c[STS_SW_NB];
    __shared__ float s_m[STS_SW_NB];
    __shared__ u64 s_scan_c[STS_WG / 64];
    __shared__ double s_scan_m[STS_WG / 64];
    __shared__ u32 s_flag, s_hit, s_cab;
    __shared__ float s_mab, s_mbe;
    static_assert(STS_SW_NB == STS_WG, "one bin per thread in the last workgroup");
    DevCtl *ctl = b.ctl;
    const u64 n = *b.n_in; // loaded with the control word, before the test
    const int e_prev = ctl->e_pred;
    if (e_prev < 0) return; // uniform: nothing to centre the bins on
    const int e_lo = e_prev - STS_SW_EXPS / 2; // exponent field of bin row 0
    s_c[threadIdx.x] = 0;
    s_m[threadIdx.x] = 0.f;
    if (threadIdx.x == 0) {
        s_cab = 0;
        s_mab = 0.f;
        s_mbe = 0.f;
    }
    const u64 *keys = b.keys;
    const AT *amps = (const AT *)b.amps;
    const u64 ntiles = (n + TT_TG - 1) / TT_TG;
    const u64 stride = ntiles > gridDim.x ? ntiles / gridDim.x : 1;
    const u64 tile = (u64)blockIdx.x * stride;
    // STS_SW_BANKS copies of the bins, workgroup w adding to copy w %
    // STS_SW_BANKS: atomics on one address from every workgroup would queue
    // behind each other
    const int bank = (int)(blockIdx.x % STS_SW_BANKS);
    u32 *gc = reinterpret_cast<u32 *>(b.sbins);                                   // [bank][bin] counts
    float *gm = reinterpret_cast<float *>(b.sbins + STS_SW_BANKS * STS_SW_NB / 2); // [bank][bin] masses
    // per bank: [0] inputs sampled, [1] count above the bins, [2] (float) mass
    // above, [3] (float) mass below
    u64 *gt = b.sbins + STS_SW_BANKS * STS_SW_NB;
    __syncthreads();
    if (tile < ntiles) {
        const u64 base = tile * TT_TG;
        const u64 end = base + SPAN < n ? base + SPAN : n;
        const u64 lo = base > (u64)TT_H ? base - TT_H : 0;
        const u64 hi = end + TT_H < n ? end + TT_H : n;
        stage_tile<AT, M>(s, g, keys, amps, lo, hi);
        __syncthreads();
        u32 c_above = 0;
        float m_above = 0.f, m_below = 0.f;
#pragma unroll 1
        for (int k = 0; k < SPAN / STS_WG; ++k) {
            const u64 e = base + (u64)k * STS_WG + threadIdx.x;
            Group<AT, M> G;
            tile_group<AT, M>(s, g, keys, amps, lo, hi, n, e < end ? e : n, G);
#pragma unroll OutUnroll<AT, M>::value
            for (int i = 0; i < (1 << M); ++i) {
                const AT o = group_out<AT, M>(g, G, i);
                if (!G.present || !nonzero(o)) continue;
                const u64 wb = weight_bits(o);
                const float w = (float)__longlong_as_double((long long)wb);
                const int row = (int)(wb >> 52) - e_lo;
                if (row >= STS_SW_EXPS) {
                    ++c_above;
                    m_above += w;
                } else if (row < 0) {
                    m_below += w;
                } else {
                    const int f = (row << STS_SW_FB) | (int)((wb >> (52 - STS_SW_FB)) & ((1u << STS_SW_FB) - 1));
                    atomicAdd(&s_c[f], 1u);
                    atomicAdd(&s_m[f], w);
                }
            }
        }
        // workgroup totals of the out-of-range parts (wave sums, then LDS),
        // then one global atomic per non-empty bin and per total, on the
        // workgroup's bank
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            c_above += __shfl_xor(c_above, d, 64);
            m_above += __shfl_xor(m_above, d, 64);
            m_below += __shfl_xor(m_below, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&s_cab, c_above);
            atomicAdd(&s_mab, m_above);
            atomicAdd(&s_mbe, m_below);
        }
        __syncthreads();
        const u32 cb = s_c[threadIdx.x];
        if (cb) {
            atomicAdd(&gc[bank * STS_SW_NB + threadIdx.x], cb);
            atomicAdd(&gm[bank * STS_SW_NB + threadIdx.x], s_m[threadIdx.x]);
        }
        u64 *bt = gt + 4 * bank;
        if (threadIdx.x == 0) {
            atomicAdd(&bt[0], end > base ? end - base : 0ull);
            if (s_cab) {
                atomicAdd(&bt[1], (u64)s_cab);
                atomicAdd(reinterpret_cast<float *>(&bt[2]), s_mab);
            }
            if (s_mbe != 0.f) atomicAdd(reinterpret_cast<float *>(&bt[3]), s_mbe);
        }
    }
    if (!sts_last_block(&ctl->done[2], &s_flag)) return;

    // the last workgroup: thread t owns bin STS_SW_NB-1-t, so rank order
    // (weight descending) is thread order
    const int t = threadIdx.x;
    const int f = STS_SW_NB - 1 - t;
    u32 c = 0;
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < STS_SW_BANKS; ++k) {
        c += ld_agent(&gc[k * STS_SW_NB + f]);
        m += (double)__int_as_float((int)ld_agent(reinterpret_cast<u32 *>(&gm[k * STS_SW_NB + f])));
    }
    u64 sampled = 0, c_above = 0;
    double m_above = 0.0, m_below = 0.0;
#pragma unroll
    for (int k = 0; k < STS_SW_BANKS; ++k) {
        const u64 *bt = gt + 4 * k;
        sampled += ld_agent(&bt[0]);
        c_above += ld_agent(&bt[1]);
        m_above += (double)__int_as_float((int)ld_agent(reinterpret_cast<const u32 *>(&bt[2])));
        m_below += (double)__int_as_float((int)ld_agent(reinterpret_cast<const u32 *>(&bt[3])));
    }
    u64 ctot;
    double mtot;
    const u64 cex = block_excl_scan<u64, STS_WG>((u64)c, s_scan_c, &ctot) + c_above;
    const double mex = block_excl_scan<double, STS_WG>(m, s_scan_m, &mtot) + m_above;
    mtot += m_above + m_below;
    const u64 K = ctl->K;
    const double p = ctl->p;
    const bool p_on = p > 0.0 && p < 1.0;
    // the rule scaled to the sample: K of n terms is K * sampled / n of the
    // sample; the mass target is p of the sample's own total
    const double kt = K > 0 && sampled > 0 ? (double)K * (double)sampled / (double)n : 0.0;
    const double mt = p * mtot;
    if (t == 0) s_hit = 0xffffffffu;
    __syncthreads();
    const bool met_above = (K > 0 && (double)c_above >= kt) || (p_on && m_above >= mt);
    const bool met = c && ((K > 0 && (double)(cex + c) >= kt) || (p_on && mex + m >= mt));
    if (sampled > 0 && !met_above && met) atomicMin(&s_hit, (u32)t);
    __syncthreads();
    if (t == 0) {
        const u32 r = s_hit;
        if (r == 0xffffffffu) {
            ctl->w_mode = 0;
        } else {
            const int fb = STS_SW_NB - 1 - (int)r;
            const int ex = e_lo + (fb >> STS_SW_FB);
            const int sub = fb & ((1 << STS_SW_FB) - 1);
            const int lo_sub = sub > 0 ? sub - 1 : 0;
            const int hi_sub = sub + 1 < (1 << STS_SW_FB) ? sub + 1 : sub;
            ctl->e_w = ex;
            ctl->w_lo = ((u64)ex << 52) | ((u64)lo_sub << (52 - STS_SW_FB));
            ctl->w_hi = ((u64)ex << 52) + ((u64)(hi_sub + 1) << (52 - STS_SW_FB)) - 1;
            ctl->w_mode = 1;
        }
    }
    for (int i = t; i < STS_SW_BANKS * (STS_SW_NB + 4); i += STS_WG) st_agent(&b.sbins[i], 0ull);
}

// ---------------------------------------------------------------------------
// atomic-free compaction (gates of up to 4 qubits), one workgroup per tile:
//   k_tile_extract - counts the tile's candidates ranked certainly before the
//                    cut (exponent field above e*, or all when nothing is
//                    cut) and copies those of exponent e* into the tile's own
//                    slab of the side buffer (2048 << m entries per tile)
//   (then: per-tile survivor counts, a scan into offsets - select.hip)
//   k_tile_emit    - writes the tile's survivors at its offset
// ---------------------------------------------------------------------------
template <typename AT, int M>
__global__ void __launch_bounds__(STS_WG) k_tile_extract(const GateArg *__restrict__ gp, PassBufs b)
{
    const GateArg &g = *gp;
    stage_gate<AT, M>(g);
    __shared__ TileSmem<AT> s;
    __shared__ u32 s_above, s_side;
    const int tid = threadIdx.x;
    DevCtl *ctl = b.ctl;
    const u64 n = *b.n_in;
    const u64 ntiles = (n + TT_TG - 1) / TT_TG;
    if (!b.materialise && ctl->pred_hit) return; // the histogram pass already did this
    if (blockIdx.x == 0 && tid == 0) {
        ctl->side_dense = 0;
        ctl->side_ntiles = ntiles;
        ctl->side_slab_shift = 11 + M;
        ctl->side_spt_log2 = 0;
    }
    const bool all = b.materialise || ctl->keep_all;
    const int e_star = ctl->e_star;
    const u64 *keys = b.keys;
    const AT *amps = (const AT *)b.amps;
    // a grid of at most a few thousand workgroups walks the tiles, so that
    // the launch costs little when the window held the cut and it exits
    for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const u64 base = tile * TT_TG;
        const u64 lo = base > (u64)TT_H ? base - TT_H : 0;
        const u64 hi = base + TT_TG + TT_H < n ? base + TT_TG + TT_H : n;
        if (tid == 0) {
            s_above = 0;
            s_side = 0;
        }
        stage_tile<AT, M>(s, g, keys, amps, lo, hi);
        __syncthreads();
        const u64 slab = tile << (11 + M);
        u32 above = 0;
#pragma unroll 1
        for (int k = 0; k < TT_IT; ++k) {
            const u64 e = base + (u64)k * STS_WG + tid;
            Group<AT, M> G;
            tile_group<AT, M>(s, g, keys, amps, lo, hi, n, e, G);
            u64 wbs[1 << M];
            u32 sidebits = 0;
#pragma unroll OutUnroll<AT, M>::value
            for (int i = 0; i < (1 << M); ++i) {
                const AT o = group_out<AT, M>(g, G, i);
                const bool cand = G.present && (M == 0 || nonzero(o));
                const u64 wb = weight_bits(o);
                wbs[i] = wb;
                const int ex = (int)(wb >> 52);
                above += (cand && (all || ex > e_star)) ? 1u : 0u;
                sidebits |= (cand && !all && ex == e_star) ? (1u << i) : 0u;
            }
            u32 at = wave_claim_n<M + 1>((u32)__popc(sidebits), &s_side);
#pragma unroll OutUnroll<AT, M>::value
            for (int i = 0; i < (1 << M); ++i) {
                if (!((sidebits >> i) & 1u)) continue;
                if (slab + at < b.side_cap) {
                    b.side_key[slab + at] = G.rest | deposit_bits<M>((u32)i, g);
                    b.side_w[slab + at] = wbs[i];
                }
                ++at;
            }
        }
        atomicAdd(&s_above, above);
        __syncthreads();
        if (tid == 0) {
            b.t_above[tile] = s_above;
            b.t_side[tile] = s_side;
        }
    }
}

// a survivor's amplitude as written: scaled by 1/sqrt(kept mass) when the
// cut dropped anything
template <typename AT> __device__ __forceinline__ AT out_amp(AT o, bool rescale, double scale)
{
    typedef typename Scalar<AT>::T R;
    if (rescale) {
        o.x = (R)((double)o.x * scale);
        o.y = (R)((double)o.y * scale);
    }
    return o;
}

// The survivors of a tile whose cut fell in the histogram pass's window:
// every candidate above the window (kept at the ends of the tile's slabs)
// and those of the window ranked at or above the threshold term (at their
// starts), copied rather than computed again. Same set and values as the
// computing path of k_tile_emit.
template <typename AT>
__device__ __forceinline__ void tile_copy_out(const PassBufs &b, u64 tile, int spl, int shift, u64 out0, u64 thr_w,
                                              u64 thr_k, bool rescale, double scale, u32 *s_scan)
{
    constexpr int UN = 8; // a tile's survivors above the window (about 2048) in one round of loads
    const TileSlabs ab = tile_slabs(b.t_above, tile, spl, shift, true, b.side_cap);
    const TileSlabs sd = tile_slabs(b.t_side, tile, spl, shift, false, b.side_cap);
    const u32 na = ab.n, ns = sd.n;
    const AT *sa = (const AT *)b.side_amp;
    AT *oa = (AT *)b.out_amps;
    for (u32 j0 = 0; j0 < na; j0 += UN * STS_WG) {
        u64 kk[UN];
        AT aa[UN];
#pragma unroll
        for (int r = 0; r < UN; ++r) {
            const u32 j = j0 + (u32)r * STS_WG + threadIdx.x;
            if (j < na) {
                // the slabs are read once: non-temporal loads
                const u64 i = slab_at(ab, j);
                kk[r] = __builtin_nontemporal_load(&b.side_key[i]);
                aa[r].x = __builtin_nontemporal_load(&sa[i].x);
                aa[r].y = __builtin_nontemporal_load(&sa[i].y);
            }
        }
#pragma unroll
        for (int r = 0; r < UN; ++r) {
            const u32 j = j0 + (u32)r * STS_WG + threadIdx.x;
            if (j < na && out0 + j < b.out_cap) {
                // the amplitudes bypass the caches, which then hold the keys
                // for the next step's first counting pass
                b.out_keys[out0 + j] = kk[r];
                const AT o = out_amp(aa[r], rescale, scale);
                __builtin_nontemporal_store(o.x, &oa[out0 + j].x);
                __builtin_nontemporal_store(o.y, &oa[out0 + j].y);
            }
        }
    }
    // the window's survivors after them, in slab order (a block scan, so the
    // order is the same in every run)
    u32 run = 0;
    for (u32 j0 = 0; j0 < ns; j0 += STS_WG) {
        const u32 j = j0 + threadIdx.x;
        bool keep = false;
        u64 k = 0, i = 0;
        if (j < ns) {
            i = slab_at(sd, j);
            const u64 w = b.side_w[i];
            k = b.side_key[i];
            keep = w > thr_w || (w == thr_w && k <= thr_k);
        }
        u32 tot;
        const u64 at = out0 + na + run + block_excl_scan<u32, STS_WG>(keep ? 1u : 0u, s_scan, &tot);
        if (keep && at < b.out_cap) {
            b.out_keys[at] = k;
            oa[at] = out_amp(sa[i], rescale, scale);
        }
        run += tot;
    }
}

template <typename AT, int M>
__global__ void __launch_bounds__(STS_WG) k_tile_emit(const GateArg *__restrict__ gp, PassBufs b)
{
    const GateArg &g = *gp;
    stage_gate<AT, M>(g);
    __shared__ TileSmem<AT> s;
    __shared__ u32 s_scan[STS_WG / 64];
    const int tid = threadIdx.x;
    DevCtl *ctl = b.ctl;
    const u64 tile = blockIdx.x; // below the tile arrays' length (the launch's bound)
    // every control load issued before any is used
    const u64 n = *b.n_in;
    const int keep_all = ctl->keep_all, dropped = ctl->dropped, hit = ctl->pred_hit;
    const u64 thr_w = ctl->thr_wbits, thr_k = ctl->thr_key;
    const double scale = ctl->scale;
    const int shift = ctl->side_slab_shift, spl = ctl->side_spt_log2;
    const u64 out0 = b.t_off[tile];
    const u64 ntiles = (n + TT_TG - 1) / TT_TG;
    if (tile >= ntiles) return;
    const bool all = b.materialise || keep_all;
    const bool rescale = !all && dropped;
    // the histogram pass kept this tile's survivors when its slabs fit
    if (b.copy && !all && hit && spl == 2 && shift == 9 + M && ((tile + 1) << (11 + M)) <= b.side_cap) {
        tile_copy_out<AT>(b, tile, spl, shift, out0, thr_w, thr_k, rescale, scale, s_scan);
        return;
    }
    const u64 *keys = b.keys;
    const AT *amps = (const AT *)b.amps;
    const u64 base = tile * TT_TG;
    const u64 lo = base > (u64)TT_H ? base - TT_H : 0;
    const u64 hi = base + TT_TG + TT_H < n ? base + TT_TG + TT_H : n;
    stage_tile<AT, M>(s, g, keys, amps, lo, hi);
    __syncthreads();
    // survivors in term order (a block scan per round, not claims): the new
    // state's order, and so every later step's, is the same in every run
    u32 run = 0;
#pragma unroll 1
    for (int k = 0; k < TT_IT; ++k) {
        const u64 e = base + (u64)k * STS_WG + tid;
        Group<AT, M> G;
        tile_group<AT, M>(s, g, keys, amps, lo, hi, n, e, G);
        AT os[1 << M];
        u32 keepbits = 0;
#pragma unroll OutUnroll<AT, M>::value
        for (int i = 0; i < (1 << M); ++i) {
            const AT o = group_out<AT, M>(g, G, i);
            os[i] = o;
            const u64 key = G.rest | deposit_bits<M>((u32)i, g);
            const u64 wb = weight_bits(o);
            const bool keep = G.present && (M == 0 || nonzero(o)) &&
                              (all || wb > thr_w || (wb == thr_w && key <= thr_k));
            keepbits |= keep ? (1u << i) : 0u;
        }
        u32 tot;
        u32 at = run + block_excl_scan<u32, STS_WG>((u32)__popc(keepbits), s_scan, &tot);
        run += tot;
#pragma unroll OutUnroll<AT, M>::value
        for (int i = 0; i < (1 << M); ++i) {
            if (!((keepbits >> i) & 1u)) continue;
            if (out0 + at < b.out_cap) {
                b.out_keys[out0 + at] = G.rest | deposit_bits<M>((u32)i, g);
                ((AT *)b.out_amps)[out0 + at] = out_amp(os[i], rescale, scale);
            }
            ++at;
        }
    }
}

// workgroups of the histogram pass that fit on the device at once (the pass
// is persistent: more would run as a second, mostly idle wave)
template <typename AT, int M, bool TILED> int hist_capacity()
{
    static int cap = 0;
    if (!cap) {
        int per_cu = 0, dev = 0, cus = 0;
        if constexpr (TILED)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_hist<AT, M>, STS_WG, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_group_hist<AT, M>, STS_WG, 0);
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        cap = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    }
    return cap;
}

template <typename AT, int M, bool TILED>
hipError_t hist_m(const GateArg &g, const PassBufs &b, int grid, hipStream_t s)
{
    if constexpr (TILED) hipLaunchKernelGGL((k_tile_hist<AT, M>), dim3(grid), dim3(STS_WG), 0, s, b.gate, b);
    else hipLaunchKernelGGL((k_group_hist<AT, M>), dim3(grid), dim3(STS_WG), 0, s, b.gate, b);
    return hipGetLastError();
}

template <typename AT, int M>
hipError_t compact_m(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    if (kind == STS_KIND_EXTRACT)
        hipLaunchKernelGGL((k_group_compact<AT, M, STS_KIND_EXTRACT>), dim3(tiles), dim3(STS_WG), 0, s, b.gate, b);
    else
        hipLaunchKernelGGL((k_group_compact<AT, M, STS_KIND_EMIT>), dim3(tiles), dim3(STS_WG), 0, s, b.gate, b);
    return hipGetLastError();
}

template <typename AT, int M> hipError_t extract_tiles_m(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_tile_extract<AT, M>), dim3(tiles), dim3(STS_WG), 0, s, b.gate, b);
    return hipGetLastError();
}

template <typename AT, int M> hipError_t sample_m(const GateArg &g, const PassBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL((k_tile_sample<AT, M>), dim3(STS_SAMPLE_TILES), dim3(STS_WG), 0, s, b.gate, b);
    return hipGetLastError();
}

template <typename AT, int M> hipError_t emit_tiles_m(const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    hipLaunchKernelGGL((k_tile_emit<AT, M>), dim3(tiles), dim3(STS_WG), 0, s, b.gate, b);
    return hipGetLastError();
}

} // namespace sts_group
