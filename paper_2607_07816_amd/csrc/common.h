// common.h - device-side definitions shared by the library's kernels.
//
// Layout of a state in HBM: structure-of-arrays, keys u64[cap] and amplitudes
// (double2 or float2)[cap], so every pass streams two coalesced arrays. The
// term count lives in the device control block (DevCtl), never on the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned long long u64;
typedef unsigned int u32;
typedef unsigned __int128 u128;

#define STS_WG 256            // threads per workgroup in the streaming kernels
#define STS_NBIN 2048         // histogram bins per selection level
#define STS_NL 20             // 64-bit limbs of the exact mass accumulator
#define STS_SMALL 4096        // a subset this small fits the final LDS sort
#define STS_FINAL_SORT 512    // the final workgroup adds 11-bit levels until its subset is this small
#define STS_MAXM 5            // largest gate (qubits)
#define STS_MAX_PASSES 4      // radix passes per sort (8-bit digits)
#define STS_TILE_ITEMS 16     // keys per thread in a radix tile
#define STS_TILE (STS_WG * STS_TILE_ITEMS)

// --------------------------------------------------------------------------
// exact masses: an unsigned integer count of 2^-1074 units (every binary64
// value is such a multiple), STS_NL limbs, little-endian
// --------------------------------------------------------------------------
struct Big {
    u64 l[STS_NL];
};

// decision state of a truncation and the running statistics (one per state)
struct DevCtl {
    u64 cnt[4];          // terms held by each term buffer (slot 3 unused)
    u64 n_cand;          // candidates of the last truncation (from the first pass)
    u64 cand_all;        // candidates counted by the last level-1 pass of any kind
    u64 tot_steps;       // truncations run since init
    u64 tot_updates;     // input terms of those truncations
    u64 tot_cand;        // candidates of those truncations
    u64 side_n;          // candidates copied to the side buffer (dense layout)
    u64 side_ntiles;     // tiled layout: slabs of 2^side_slab_shift entries
    int side_slab_shift;
    int side_dense;      // 1: entries [0, side_n) (look-back pass); 0: per-tile slabs
    int side_spt_log2;   // tiled layout: each tile owns 2^side_spt_log2 consecutive slabs
    // fields updated with atomics sit on cache lines of their own: every
    // workgroup of every kernel reads the fields around them, and reads of a
    // line wait behind the atomics queued on it
    alignas(128) u32 done[4]; // last-workgroup counters, one per kernel kind
    alignas(128) u32 flags;   // STS_F_* below
    // truncation rule
    alignas(128) u64 K;  // top-k (0 = off)
    double p;            // p-mass (off unless 0 < p < 1)
    // decision
    int keep_all;        // the rule keeps every candidate
    int dropped;         // L < C: rescale
    int e_star;          // exponent field of the level holding the L-th term
    int e_pred;          // cut exponent of the previous truncation (-1: none)
    int pred_hit;        // the histogram pass's side-buffer window holds this truncation's cut
    int w2_mode;         // the histogram pass binned a sampled window for level 2 (h2w)
    int l2_done;         // the level-1 pick also picked level 2 from those bins
    // window of weights [w_lo, w_hi] (bit patterns, one exponent field e_w)
    // that the histogram pass copies to the side buffer: set for this step by
    // the sampling pass (w_mode = 1), else the octave of e_pred
    int w_mode;
    int e_w;
    u64 w_lo, w_hi;
    int level;           // last resolved level
    u64 cnt_before;      // terms ranked before the current subset
    u64 mb_lo, mb_hi;    // mantissa sum (units 2^(max(e*,1)-1075)) ranked before the subset inside e*
    u64 R_lo, R_hi;      // remaining mass to reach, same units; all ones = off
    u64 sub_count;       // terms in the current subset
    u64 vpre_hi, vpre_lo;// fixed high part of the within-exponent rank key
    int vshift;          // bits of the rank key below the fixed part
    int pad1;
    u64 L;               // terms kept
    u64 thr_wbits, thr_key; // the L-th term in rank order
    double scale;        // renormalisation factor (1 when nothing dropped)
    double S;            // kept mass (correctly rounded)
    double W;            // total mass before the cut (correctly rounded)
    double frac;         // S / W
    double log10_cum;    // running sum of log10(frac)
    u64 peak_key;
    double peak_w;
    double peak_W;       // exact total of the state the peak was taken on, rounded
    Big S_excl;          // exact mass of the bins above e*
    Big T;               // exact p * W target (rounded up)
};

#define STS_F_SIDE_OVERFLOW 1u
#define STS_F_OUT_OVERFLOW 2u
#define STS_F_UNRESOLVED 4u
#define STS_F_INEXACT 8u

// --------------------------------------------------------------------------
// hashing: a bijective 64-bit mixer (splitmix64 finalisation). Equal hashes
// mean equal inputs, so grouping by hash buckets never merges distinct keys.
// --------------------------------------------------------------------------
__device__ __forceinline__ u64 sts_mix64(u64 x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// weight bits: |a|^2 = fl64(fl64(re*re) + fl64(im*im)), components in FP64
__device__ __forceinline__ double sts_weight(double re, double im)
{
    return re * re + im * im;
}

__device__ __forceinline__ u64 sts_dbits(double x) { return (u64)__double_as_longlong(x); }

// mantissa as an integer and the exponent of its unit: w = mant * 2^(max(e,1) - 1075)
__device__ __forceinline__ u64 sts_mant(u64 wbits)
{
    const u64 e = wbits >> 52;
    const u64 f = wbits & ((1ull << 52) - 1);
    return e ? (f | (1ull << 52)) : f;
}

// --------------------------------------------------------------------------
// Big helpers (single-thread use)
// --------------------------------------------------------------------------
__device__ __forceinline__ void big_zero(Big &a)
{
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) a.l[i] = 0;
}

// a += v * 2^bit, v < 2^128 (given as lo, hi). Every limb index is a
// compile-time constant, so the accumulator stays in registers.
__device__ inline void big_add_shifted(Big &a, u64 vlo, u64 vhi, int bit)
{
    const int limb = bit >> 6, off = bit & 63;
    const u64 p0 = vlo << off;
    const u64 p1 = off ? ((vhi << off) | (vlo >> (64 - off))) : vhi;
    const u64 p2 = off ? (vhi >> (64 - off)) : 0;
    u64 carry = 0;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) {
        const int k = i - limb;
        const u64 add = k == 0 ? p0 : (k == 1 ? p1 : (k == 2 ? p2 : 0));
        const u64 s = a.l[i] + add;
        const u64 c1 = s < add;
        const u64 s2 = s + carry;
        const u64 c2 = s2 < s;
        a.l[i] = s2;
        carry = c1 + c2;
    }
}

__device__ inline void big_add(Big &a, const Big &b)
{
    u64 carry = 0;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) {
        const u64 s = a.l[i] + b.l[i];
        const u64 c1 = s < b.l[i];
        const u64 s2 = s + carry;
        const u64 c2 = s2 < s;
        a.l[i] = s2;
        carry = c1 + c2;
    }
}

// a -= b (requires a >= b)
__device__ inline void big_sub(Big &a, const Big &b)
{
    u64 borrow = 0;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) {
        const u64 x = a.l[i];
        const u64 d = x - b.l[i];
        const u64 b1 = x < b.l[i];
        const u64 d2 = d - borrow;
        const u64 b2 = d < borrow;
        a.l[i] = d2;
        borrow = b1 | b2;
    }
}

__device__ inline int big_cmp(const Big &a, const Big &b)
{
    int r = 0;
#pragma unroll
    for (int i = STS_NL - 1; i >= 0; --i) {
        if (r == 0 && a.l[i] != b.l[i]) r = a.l[i] < b.l[i] ? -1 : 1;
    }
    return r;
}

__device__ inline bool big_is_zero(const Big &a)
{
    u64 o = 0;
    for (int i = 0; i < STS_NL; ++i) o |= a.l[i];
    return o == 0;
}

// a >>= 64 * k (whole limbs), with compile-time limb indices (a barrel of
// conditional shifts), so nothing spills to scratch memory
__device__ inline void big_shr_limbs(Big &a, int k)
{
#pragma unroll
    for (int b = 16; b >= 1; b >>= 1) {
        if (k & b) {
#pragma unroll
            for (int i = 0; i < STS_NL; ++i) a.l[i] = (i + b < STS_NL) ? a.l[i + b] : 0ull;
        }
    }
}

// any bit of a below bit position s set?
__device__ inline bool big_any_below(const Big &a, int s)
{
    const int wl = s >> 6, wb = s & 63;
    bool any = false;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) {
        if (i < wl) any |= a.l[i] != 0;
        if (i == wl && wb) any |= (a.l[i] & ((1ull << wb) - 1)) != 0;
    }
    return any;
}

// a >>= s (truncating)
__device__ inline void big_shr(Big &a, int s)
{
    big_shr_limbs(a, s >> 6);
    const int wb = s & 63;
    if (wb) {
#pragma unroll
        for (int i = 0; i < STS_NL; ++i) {
            const u64 nxt = (i + 1 < STS_NL) ? a.l[i + 1] : 0ull;
            a.l[i] = (a.l[i] >> wb) | (nxt << (64 - wb));
        }
    }
}

// r = ceil(a * m / 2^s)
__device__ inline void big_mul_shr_ceil(Big &r, const Big &a, u64 m, int s)
{
    u64 carry = 0;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) {
        const u128 t = (u128)a.l[i] * m + carry;
        r.l[i] = (u64)t;
        carry = (u64)(t >> 64);
    }
    const bool any = big_any_below(r, s);
    big_shr(r, s);
    if (any) big_add_shifted(r, 1, 0, 0);
}

// ceil(a / 2^s) clamped to 2^128 - 1 (returned as lo, hi)
__device__ inline void big_shr_ceil_u128(const Big &a, int s, u64 &lo, u64 &hi)
{
    Big t = a;
    const bool any = big_any_below(t, s);
    big_shr(t, s);
    bool over = false;
#pragma unroll
    for (int i = 2; i < STS_NL; ++i) over |= t.l[i] != 0;
    if (over) {
        lo = ~0ull;
        hi = ~0ull;
        return;
    }
    lo = t.l[0];
    hi = t.l[1];
    if (any) {
        lo += 1;
        if (lo == 0) {
            hi += 1;
            if (hi == 0) {
                lo = ~0ull;
                hi = ~0ull;
            }
        }
    }
}

// nearest binary64 to a (ties to even), from the top 128 bits and a sticky bit
__device__ inline double big_to_double(const Big &a)
{
    int top = -1;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i)
        if (a.l[i]) top = i;
    if (top < 0) return 0.0;
    u64 L0 = 0, L1 = 0, L2 = 0;
    bool below = false;
#pragma unroll
    for (int i = 0; i < STS_NL; ++i) {
        if (i == top) L0 = a.l[i];
        if (i == top - 1) L1 = a.l[i];
        if (i == top - 2) L2 = a.l[i];
        if (i < top - 2) below |= a.l[i] != 0;
    }
    const int lz = __clzll((long long)L0);
    const int h = top * 64 + 63 - lz; // position of the top set bit
    if (h < 53) return ldexp((double)L0, -1074);
    const u64 hi = lz ? (L0 << lz) | (L1 >> (64 - lz)) : L0; // bit 63 = bit h
    const u64 lo = lz ? (L1 << lz) | (L2 >> (64 - lz)) : L1;
    const bool rest = below || (lz ? (L2 << lz) != 0 : L2 != 0);
    u64 mant = hi >> 11;
    const bool guard = (hi >> 10) & 1ull;
    const bool sticky = (hi & 0x3ffull) != 0 || lo != 0 || rest;
    int lsb = h - 52;
    if (guard && (sticky || (mant & 1ull))) {
        mant += 1;
        if (mant == (1ull << 53)) {
            mant >>= 1;
            lsb += 1;
        }
    }
    return ldexp((double)mant, lsb - 1074);
}

// --------------------------------------------------------------------------
// wave64 / workgroup helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int sts_lane() { return __lane_id(); }

__device__ __forceinline__ u64 sts_lanemask_lt() { return (1ull << sts_lane()) - 1ull; }

// set bits of the wave mask m below this lane (two mbcnt instructions)
__device__ __forceinline__ u32 sts_lanes_below(u64 m)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
}

// store v at a byte offset below 4 GiB from a base that is the same in every
// lane: the address stays a scalar base plus a 32-bit lane offset
template <typename T> __device__ __forceinline__ void sts_store_at(T *base, u32 byte_off, const T &v)
{
    *reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(base) + byte_off) = v;
}

// The workgroups of a launch are dealt to the XCDs in turn (workgroup b to
// XCD b % 8), and each XCD has its own L2. sts_xcd_tile renumbers them so
// that every XCD works through one contiguous range of tiles: neighbouring
// tiles, whose output runs share cache lines, then meet in the same L2.
// A bijection of [0, tiles) for tiles == gridDim.x.
#define STS_XCDS 8
__device__ __forceinline__ u32 sts_xcd_tile(u32 b, u32 tiles)
{
    const u32 x = b % STS_XCDS, i = b / STS_XCDS;
    const u32 q = tiles / STS_XCDS, r = tiles % STS_XCDS;
    return x * q + (x < r ? x : r) + i;
}

// inclusive scan over the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = sts_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// exclusive scan over a workgroup of NT threads (NT/64 waves); returns the
// exclusive prefix and writes the total to *total. scratch: NT/64 entries.
template <typename T, int NT>
__device__ __forceinline__ T block_excl_scan(T v, T *scratch, T *total)
{
    const int lane = sts_lane();
    const int w = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) scratch[w] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const T s = scratch[i];
        if (i < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// "last workgroup" election: every workgroup calls this once after its global
// atomics; it returns true in exactly one workgroup (the last to arrive),
// which then sees every other workgroup's atomics. Resets the counter.
__device__ inline bool sts_last_block(u32 *counter, u32 *s_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const u32 prev = atomicAdd(counter, 1u);
        const bool last = prev == gridDim.x - 1;
        if (last) st_agent(counter, 0u);
        *s_flag = last ? 1u : 0u;
    }
    __syncthreads();
    const bool last = *s_flag != 0;
    if (last) __threadfence();
    return last;
}

// --------------------------------------------------------------------------
// decoupled look-back words: epoch (24 bits) | status (2) | value (38).
// The epoch tags the launch that wrote a word, so the arrays never need
// clearing between launches. status 1 = tile aggregate, 2 = inclusive prefix.
// --------------------------------------------------------------------------
#define STS_LB_VBITS 38
#define STS_LB_VMASK ((1ull << STS_LB_VBITS) - 1ull)

__device__ __forceinline__ u64 lb_pack(u32 epoch, u32 status, u64 val)
{
    return ((u64)(epoch & 0xffffffu) << 40) | ((u64)status << STS_LB_VBITS) | (val & STS_LB_VMASK);
}

// Publish this tile's aggregate, walk back over predecessors until an
// inclusive prefix is found, publish the inclusive prefix. Returns the
// exclusive prefix. Tiles are numbered in the order their workgroups started,
// so every predecessor is resident or finished and the wait ends.
__device__ inline u64 lb_exclusive(u64 *look, u64 stride, u64 tile, u64 local, u32 epoch)
{
    constexpr int B = 8; // predecessors read per round trip
    const u32 ep = epoch & 0xffffffu;
    if (tile == 0) {
        st_agent(&look[0], lb_pack(epoch, 2, local));
        return 0;
    }
    st_agent(&look[tile * stride], lb_pack(epoch, 1, local));
    u64 excl = 0;
    u64 j = tile - 1; // next predecessor to account for
    for (;;) {
        // tile 0 always publishes an inclusive value, so the walk ends at or
        // before it; reads below tile 0 are never issued
        u64 v[B];
#pragma unroll
        for (int b = 0; b < B; ++b) v[b] = (u64)b <= j ? ld_agent(&look[(j - b) * stride]) : 0ull;
        int used = 0;
        bool done = false;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (done || used < b) continue;           // stopped earlier in this batch
            if ((u64)b > j) continue;
            if ((u32)(v[b] >> 40) != ep) continue;  // not published yet: re-read from here
            excl += v[b] & STS_LB_VMASK;
            used = b + 1;
            if (((v[b] >> STS_LB_VBITS) & 3u) == 2u) done = true;
        }
        if (done) break;
        if (used == 0) __builtin_amdgcn_s_sleep(1);
        j -= (u64)used;
    }
    st_agent(&look[tile * stride], lb_pack(epoch, 2, excl + local));
    return excl;
}
