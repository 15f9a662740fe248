// radix.hip - grouping a state by the bits outside a gate's qubits.
//
// Every term whose key differs from another only on the gate's qubits must
// meet it (Sec. IV.A: the 2^m amplitudes of a tuple share the bits outside
// the gate). The state is sorted by a hash bucket of key & ~mask: a stable
// least-significant-digit radix sort with digits of BITS bits (8 or 11)
// taken from the top bits of a bijective 64-bit mix of the masked key. Equal
// masked keys share a bucket, so after the sort every group sits inside one
// short run of equal buckets; the hash spreads buckets evenly whatever the
// key distribution.
//
// Each digit pass is reduce-then-scan, with no waiting between workgroups:
//   k_radix_count - per tile of 256 * IT keys, the count of every digit
//   k_radix_scan  - per digit (one workgroup each), the exclusive prefix of
//                   its counts over the tiles, and its total
//   k_radix_pass  - per tile: rank the keys in registers and LDS (wave64
//                   ballots find lanes with equal digits), take the tile's
//                   output offsets from the scan (digit base = exclusive scan
//                   of the totals, done in the workgroup), stage the tile in
//                   LDS in digit order and write keys and amplitudes out in
//                   coalesced runs.
// The shape (BITS, IT) is chosen per sort by the context's policy: 8-bit
// digits in 4096-key tiles by default (a digit's run per tile averages 16
// keys, so the writes coalesce), 11-bit digits (fewer passes) or 2048-key
// tiles (more workgroups) for small states, where a sort is a chain of short
// launches. The counting and scatter workgroups take the tiles in one
// contiguous range per XCD (neighbouring tiles' output runs share cache
// lines, merged in that XCD's L2), and the scatter's input loads are
// non-temporal (the cache keeps the output, which the next pass reads).
#include <type_traits>

#include "kernels.h"

namespace {

template <int BITS> __device__ __forceinline__ u32 bucket_digit(u64 key, u64 notmask, int shift)
{
    return (u32)((sts_mix64(key & notmask) >> shift) & ((1u << BITS) - 1u));
}

// digit counts of one tile, written digit-major: counts[d * tiles_cap + tile]
template <int BITS, int IT>
__global__ void __launch_bounds__(STS_WG) k_radix_count(const u64 *__restrict__ keys, const u64 *n_in,
                                                         const u64 *gate_notmask, int shift, u32 *__restrict__ counts,
                                                         u64 tiles_cap)
{
    constexpr int ND = 1 << BITS;
    constexpr u64 TILE = (u64)STS_WG * IT;
    __shared__ u32 s_h[ND];
    const u64 n = *n_in;
    const u64 notmask = *gate_notmask;
    // the state's tiles go to the XCDs in contiguous ranges, so that the
    // counts of neighbouring tiles (adjacent in each digit's row) are written
    // through one L2; workgroups past the state's tiles write zeros
    const u64 nt = (n + TILE - 1) / TILE;
    const u64 tile = blockIdx.x < nt ? sts_xcd_tile(blockIdx.x, nt < gridDim.x ? (u32)nt : gridDim.x) : blockIdx.x;
    for (int d = threadIdx.x; d < ND; d += STS_WG) s_h[d] = 0;
    __syncthreads();
    const u64 base = tile * TILE;
    u64 kk[IT];
    if (base + TILE <= n) {
#pragma unroll
        for (int k = 0; k < IT; ++k) kk[k] = keys[base + (u64)k * STS_WG + threadIdx.x];
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const u64 i = base + (u64)k * STS_WG + threadIdx.x;
            kk[k] = i < n ? keys[i] : 0ull;
        }
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const u64 i = base + (u64)k * STS_WG + threadIdx.x;
        if (i < n) atomicAdd(&s_h[bucket_digit<BITS>(kk[k], notmask, shift)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < ND; d += STS_WG) counts[(u64)d * tiles_cap + tile] = s_h[d];
}

// per digit (workgroup d): exclusive prefix of its tile counts, and its
// total, both digit-major: prefix[d * tiles_cap + tile]. A chunk of
// STS_WG * CH counts is loaded and stored coalesced (lane-consecutive) and
// transposed through LDS, so that each thread scans CH consecutive counts
// (LDS rows padded against bank conflicts).
__global__ void __launch_bounds__(STS_WG) k_radix_scan(const u32 *__restrict__ counts, u64 *__restrict__ prefix,
                                                        u64 *__restrict__ totals, const u64 *n_in, u64 tiles_cap,
                                                        u64 tile_keys)
{
    constexpr int CH = 16;
    constexpr int CHUNK = STS_WG * CH;
    __shared__ u32 s_c[CHUNK + CHUNK / 32];
    __shared__ u64 s_p[CHUNK + CHUNK / 16];
    __shared__ u64 scratch[STS_WG / 64];
    __shared__ u64 s_carry;
    auto pc = [](u32 i) { return i + (i >> 5); }; // padded index into s_c
    auto pp = [](u32 i) { return i + (i >> 4); }; // padded index into s_p
    const u64 n = *n_in;
    const u64 ntiles = (n + tile_keys - 1) / tile_keys;
    const u64 d = blockIdx.x;
    const u32 t = threadIdx.x;
    const u32 *c = counts + d * tiles_cap;
    u64 *pr = prefix + d * tiles_cap;
    if (t == 0) s_carry = 0;
    for (u64 c0 = 0; c0 < ntiles; c0 += CHUNK) {
        u32 v[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const u64 i = c0 + (u64)k * STS_WG + t;
            v[k] = i < ntiles ? c[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) s_c[pc((u32)k * STS_WG + t)] = v[k];
        __syncthreads();
        u32 mine[CH];
        u64 sum = 0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            mine[k] = s_c[pc(t * CH + (u32)k)];
            sum += mine[k];
        }
        u64 total;
        u64 run = block_excl_scan<u64, STS_WG>(sum, scratch, &total) + s_carry;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            s_p[pp(t * CH + (u32)k)] = run;
            run += mine[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const u64 i = c0 + (u64)k * STS_WG + t;
            if (i < ntiles) pr[i] = s_p[pp((u32)k * STS_WG + t)];
        }
        if (t == 0) s_carry += total;
        __syncthreads();
    }
    if (t == 0) totals[d] = s_carry;
}

// An amplitude is moved as W plain 64-bit words (W = 1: complex64, W = 2:
// complex128), held in one register array per word (an array of HIP's
// 16-byte vector type would be left in scratch memory). Thread t owns the
// DPT = 2^BITS / 256 consecutive digits t*DPT .. t*DPT + DPT-1.
template <int W, int BITS, int IT>
__global__ void __launch_bounds__(STS_WG) k_radix_pass(const u64 *__restrict__ kin, const u64 *__restrict__ ain,
                                                        u64 *__restrict__ kout, u64 *__restrict__ aout,
                                                        const u64 *n_in, u64 *n_out, const u64 *gate_notmask,
                                                        int shift, const u64 *__restrict__ prefix,
                                                        const u64 *__restrict__ totals, u64 tiles_cap)
{
    constexpr int NW = STS_WG / 64;
    constexpr int ND = 1 << BITS;
    constexpr int DPT = ND / STS_WG;
    constexpr int TILE = STS_WG * IT;
    constexpr int ESZ = 8 * W;
    static_assert(DPT >= 1 && ND % STS_WG == 0, "whole digits per thread");
    typedef typename std::conditional<(BITS > 8), unsigned short, unsigned char>::type dig_t;
    __shared__ u32 s_cnt[NW][ND];
    __shared__ u32 s_dstart[ND];
    __shared__ u64 s_base[ND];
    __shared__ u32 s_scratch[NW];
    __shared__ u64 s_scratch64[NW];
    __shared__ dig_t s_dig[TILE];
    __shared__ __attribute__((aligned(16))) unsigned char s_buf[TILE * ESZ];

    const u64 notmask = *gate_notmask;
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const u64 n = *n_in;
    u64 tot_d[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) tot_d[q] = totals[tid * DPT + q];
    if (blockIdx.x == 0 && tid == 0) *n_out = n;
    // the launch may have more workgroups than the state has tiles; the
    // state's tiles go to the XCDs in contiguous ranges
    const u64 nt = (n + TILE - 1) / TILE;
    if (blockIdx.x >= nt) return;
    const u64 tile = sts_xcd_tile(blockIdx.x, nt < gridDim.x ? (u32)nt : gridDim.x);
    // global offset of this tile's first key of each own digit: the digit's
    // base (exclusive scan of the totals) plus the tiles before it; loaded
    // now, used after the ranking
    u64 pre_d[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) pre_d[q] = prefix[(u64)(tid * DPT + q) * tiles_cap + tile];
    for (int i = tid; i < NW * ND; i += STS_WG) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const u64 base = tile * TILE;

    // issue every key and amplitude load of the thread first. The pass
    // reads its input once, and the next pass (or the gate passes) reads its
    // output: the loads are non-temporal, so the caches keep the output just
    // written rather than the input
    u64 key[IT], a0[IT], a1[IT];
    u32 dig[IT];
    u32 rank[IT];
    if (base + TILE <= n) {
        // a full tile (uniform branch): every load issued back to back
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const u64 e = base + (u64)w * (64 * IT) + (u64)k * 64 + lane;
            key[k] = __builtin_nontemporal_load(&kin[e]);
            a0[k] = __builtin_nontemporal_load(&ain[e * W]);
            if (W == 2) a1[k] = __builtin_nontemporal_load(&ain[e * W + 1]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const u64 e = base + (u64)w * (64 * IT) + (u64)k * 64 + lane;
            if (e < n) {
                key[k] = __builtin_nontemporal_load(&kin[e]);
                a0[k] = __builtin_nontemporal_load(&ain[e * W]);
                if (W == 2) a1[k] = __builtin_nontemporal_load(&ain[e * W + 1]);
            } else {
                key[k] = 0ull;
            }
        }
    }
    // rank every key of the tile among equal digits, in index order
    const u64 lt = sts_lanemask_lt();
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const u64 e = base + (u64)w * (64 * IT) + (u64)k * 64 + lane;
        const bool valid = e < n;
        const u32 d = valid ? bucket_digit<BITS>(key[k], notmask, shift) : 0u;
        dig[k] = valid ? d : (u32)ND;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const u64 bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        u32 pre = 0;
        if (valid) pre = s_cnt[w][d];
        const u32 below = (u32)__popcll(peers & lt);
        if (valid && below == 0) s_cnt[w][d] = pre + (u32)__popcll(peers);
        rank[k] = pre + below;
    }
    __syncthreads();

    // per-digit totals of the tile and each wave's exclusive prefix
    u32 tot[DPT];
    u32 tsum = 0;
    u64 dsum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int d = tid * DPT + q;
        u32 run = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const u32 c = s_cnt[ww][d];
            s_cnt[ww][d] = run;
            run += c;
        }
        tot[q] = run;
        tsum += run;
        dsum += tot_d[q];
    }
    u32 all;
    u32 dstart = block_excl_scan<u32, STS_WG>(tsum, s_scratch, &all);
    u64 n_all;
    u64 dbase = block_excl_scan<u64, STS_WG>(dsum, s_scratch64, &n_all);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int d = tid * DPT + q;
        s_dstart[d] = dstart;
        s_base[d] = dbase + pre_d[q];
        dstart += tot[q];
        dbase += tot_d[q];
    }
    __syncthreads();

    // stage keys in digit order, then write them out
    u64 *sk = reinterpret_cast<u64 *>(s_buf);
    u32 pos[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (dig[k] < (u32)ND) {
            pos[k] = s_dstart[dig[k]] + s_cnt[w][dig[k]] + rank[k];
            sk[pos[k]] = key[k];
            s_dig[pos[k]] = (dig_t)dig[k];
        }
    }
    __syncthreads();
    const u32 count = (u32)((n - base) < (u64)TILE ? (n - base) : (u64)TILE);
    for (u32 i = tid; i < count; i += STS_WG) {
        const u32 d = s_dig[i];
        kout[s_base[d] + (i - s_dstart[d])] = sk[i];
    }
    __syncthreads();

    // same permutation for the amplitudes
    u64 *sa = reinterpret_cast<u64 *>(s_buf);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (dig[k] < (u32)ND) {
            sa[pos[k] * W] = a0[k];
            if (W == 2) sa[pos[k] * W + 1] = a1[k];
        }
    }
    __syncthreads();
    for (u32 i = tid; i < count; i += STS_WG) {
        const u32 d = s_dig[i];
        const u64 o = (s_base[d] + (i - s_dstart[d])) * W;
        aout[o] = sa[i * W];
        if (W == 2) aout[o + 1] = sa[i * W + 1];
    }
}

} // namespace

template <int BITS, int IT>
static hipError_t radix_launch(int what, int prec, const u64 *kin, const void *ain, u64 *kout, void *aout, const u64 *n_in,
                        u64 *n_out, const u64 *notmask, int shift, u32 *counts, u64 *prefix, u64 *totals,
                        u64 tiles_cap, int tiles, hipStream_t s)
{
    static_assert(sizeof(double2) == 2 * sizeof(u64) && sizeof(float2) == sizeof(u64), "amplitude words");
    if (what == 0) {
        hipLaunchKernelGGL((k_radix_count<BITS, IT>), dim3(tiles), dim3(STS_WG), 0, s, kin, n_in, notmask, shift,
                           counts, tiles_cap);
    } else if (what == 1) {
        hipLaunchKernelGGL(k_radix_scan, dim3(1u << BITS), dim3(STS_WG), 0, s, (const u32 *)counts, prefix, totals,
                           n_in, tiles_cap, (u64)STS_WG * IT);
    } else if (prec == 0) {
        hipLaunchKernelGGL((k_radix_pass<2, BITS, IT>), dim3(tiles), dim3(STS_WG), 0, s, kin, (const u64 *)ain, kout,
                           (u64 *)aout, n_in, n_out, notmask, shift, prefix, totals, tiles_cap);
    } else {
        hipLaunchKernelGGL((k_radix_pass<1, BITS, IT>), dim3(tiles), dim3(STS_WG), 0, s, kin, (const u64 *)ain, kout,
                           (u64 *)aout, n_in, n_out, notmask, shift, prefix, totals, tiles_cap);
    }
    return hipGetLastError();
}

hipError_t launch_radix(int what, int shape, int prec, const u64 *kin, const void *ain, u64 *kout, void *aout,
                        const u64 *n_in, u64 *n_out, const u64 *notmask, int shift, u32 *counts, u64 *prefix,
                        u64 *totals, u64 tiles_cap, int tiles, hipStream_t s)
{
    switch (shape) {
    case STS_RADIX_8x16:
        return radix_launch<8, 16>(what, prec, kin, ain, kout, aout, n_in, n_out, notmask, shift, counts, prefix,
                                   totals, tiles_cap, tiles, s);
    case STS_RADIX_8x8:
        return radix_launch<8, 8>(what, prec, kin, ain, kout, aout, n_in, n_out, notmask, shift, counts, prefix,
                                  totals, tiles_cap, tiles, s);
    case STS_RADIX_11x16:
        return radix_launch<11, 16>(what, prec, kin, ain, kout, aout, n_in, n_out, notmask, shift, counts, prefix,
                                    totals, tiles_cap, tiles, s);
    case STS_RADIX_11x8:
        return radix_launch<11, 8>(what, prec, kin, ain, kout, aout, n_in, n_out, notmask, shift, counts, prefix,
                                   totals, tiles_cap, tiles, s);
    }
    return hipErrorInvalidValue;
}
