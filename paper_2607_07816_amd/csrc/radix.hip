// radix.hip - grouping a state by the bits outside a gate's qubits.
//
// Every term whose key differs from another only on the gate's qubits must
// meet it (Sec. IV.A: the 2^m amplitudes of a tuple share the bits outside
// the gate). The state is sorted by a hash bucket of key & ~mask: a stable
// least-significant-digit radix sort with 8-bit digits taken from the top
// bits of a bijective 64-bit mix of the masked key. Equal masked keys share a
// bucket, so after the sort every group sits inside one short run of equal
// buckets; the hash spreads buckets evenly whatever the key distribution.
//
// Each digit pass is reduce-then-scan, with no waiting between workgroups:
//   k_radix_count - per 4096-key tile, the count of every digit
//   k_radix_scan  - per digit (one workgroup each), the exclusive prefix of
//                   its counts over the tiles, and its total
//   k_radix_pass  - per tile: rank the keys in registers and LDS (wave64
//                   ballots find lanes with equal digits), take the tile's
//                   output offsets from the scan (digit base = exclusive scan
//                   of the totals, done in the workgroup), stage the tile in
//                   LDS in digit order and write keys and amplitudes out in
//                   coalesced runs.
// The counting and scatter workgroups take the tiles in one contiguous range
// per XCD (neighbouring tiles' output runs share cache lines, merged in that
// XCD's L2), and the scatter's input loads are non-temporal (the cache keeps
// the output, which the next pass reads).
#include "kernels.h"

namespace {

__device__ __forceinline__ u32 bucket_digit(u64 key, u64 notmask, int shift)
{
    return (u32)((sts_mix64(key & notmask) >> shift) & 255u);
}

// digit counts of one tile, written digit-major: counts[d * tiles_cap + tile]
__global__ void __launch_bounds__(STS_WG) k_radix_count(const u64 *__restrict__ keys, const u64 *n_in,
                                                         const u64 *gate_notmask, int shift, u32 *__restrict__ counts,
                                                         u64 tiles_cap)
{
    __shared__ u32 s_h[256];
    const u64 n = *n_in;
    const u64 notmask = *gate_notmask;
    // the state's tiles go to the XCDs in contiguous ranges, so that the
    // counts of neighbouring tiles (adjacent in each digit's row) are written
    // through one L2; workgroups past the state's tiles write zeros
    const u64 nt = (n + STS_TILE - 1) / STS_TILE;
    const u64 tile = blockIdx.x < nt ? sts_xcd_tile(blockIdx.x, nt < gridDim.x ? (u32)nt : gridDim.x) : blockIdx.x;
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const u64 base = tile * STS_TILE;
    u64 kk[STS_TILE_ITEMS];
    if (base + STS_TILE <= n) {
#pragma unroll
        for (int k = 0; k < STS_TILE_ITEMS; ++k) kk[k] = keys[base + (u64)k * STS_WG + threadIdx.x];
    } else {
#pragma unroll
        for (int k = 0; k < STS_TILE_ITEMS; ++k) {
            const u64 i = base + (u64)k * STS_WG + threadIdx.x;
            kk[k] = i < n ? keys[i] : 0ull;
        }
    }
#pragma unroll
    for (int k = 0; k < STS_TILE_ITEMS; ++k) {
        const u64 i = base + (u64)k * STS_WG + threadIdx.x;
        if (i < n) atomicAdd(&s_h[bucket_digit(kk[k], notmask, shift)], 1u);
    }
    __syncthreads();
    counts[(u64)threadIdx.x * tiles_cap + tile] = s_h[threadIdx.x];
}

// per digit (workgroup d): exclusive prefix of its tile counts, and its
// total, both digit-major: prefix[d * tiles_cap + tile]. A chunk of
// STS_WG * CH counts is loaded and stored coalesced (lane-consecutive) and
// transposed through LDS, so that each thread scans CH consecutive counts
// (LDS rows padded against bank conflicts).
__global__ void __launch_bounds__(STS_WG) k_radix_scan(const u32 *__restrict__ counts, u64 *__restrict__ prefix,
                                                        u64 *__restrict__ totals, const u64 *n_in, u64 tiles_cap)
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
    const u64 ntiles = (n + STS_TILE - 1) / STS_TILE;
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
// 16-byte vector type would be left in scratch memory).
template <int W>
__global__ void __launch_bounds__(STS_WG) k_radix_pass(const u64 *__restrict__ kin, const u64 *__restrict__ ain,
                                                        u64 *__restrict__ kout, u64 *__restrict__ aout,
                                                        const u64 *n_in, u64 *n_out, const u64 *gate_notmask,
                                                        int shift, const u64 *__restrict__ prefix,
                                                        const u64 *__restrict__ totals, u64 tiles_cap)
{
    const u64 notmask = *gate_notmask;
    constexpr int NW = STS_WG / 64;
    constexpr int IT = STS_TILE_ITEMS;
    constexpr int ESZ = 8 * W;
    __shared__ u32 s_cnt[NW][256];
    __shared__ u32 s_dstart[256];
    __shared__ u64 s_base[256];
    __shared__ u32 s_scratch[NW];
    __shared__ u64 s_scratch64[NW];
    __shared__ unsigned char s_dig[STS_TILE];
    __shared__ __attribute__((aligned(16))) unsigned char s_buf[STS_TILE * ESZ];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const u64 n = *n_in;
    const u64 tot_d = totals[tid];
    if (blockIdx.x == 0 && tid == 0) *n_out = n;
    // the launch may have more workgroups than the state has tiles; the
    // state's tiles go to the XCDs in contiguous ranges
    const u64 nt = (n + STS_TILE - 1) / STS_TILE;
    if (blockIdx.x >= nt) return;
    const u64 tile = sts_xcd_tile(blockIdx.x, nt < gridDim.x ? (u32)nt : gridDim.x);
    // global offset of this tile's first key of digit tid: the digit's base
    // (exclusive scan of the totals) plus the tiles before it; loaded now,
    // used after the ranking
    const u64 pre_d = prefix[(u64)tid * tiles_cap + tile];
    for (int i = tid; i < NW * 256; i += STS_WG) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const u64 base = tile * STS_TILE;

    // issue every key and amplitude load of the thread first. The pass
    // reads its input once, and the next pass (or the gate passes) reads its
    // output: the loads are non-temporal, so the caches keep the output just
    // written rather than the input
    u64 key[IT], a0[IT], a1[IT];
    u32 dig[IT];
    u32 rank[IT];
    if (base + STS_TILE <= n) {
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
        const u32 d = valid ? bucket_digit(key[k], notmask, shift) : 0u;
        dig[k] = valid ? d : 256u;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
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
    u32 tot;
    {
        const int d = tid; // STS_WG == 256 digits
        u32 run = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const u32 c = s_cnt[ww][d];
            s_cnt[ww][d] = run;
            run += c;
        }
        tot = run;
    }
    u32 all;
    const u32 dstart = block_excl_scan<u32, STS_WG>(tot, s_scratch, &all);
    s_dstart[tid] = dstart;
    u64 n_all;
    const u64 dbase = block_excl_scan<u64, STS_WG>(tot_d, s_scratch64, &n_all);
    s_base[tid] = dbase + pre_d;
    __syncthreads();

    // stage keys in digit order, then write them out
    u64 *sk = reinterpret_cast<u64 *>(s_buf);
    u32 pos[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (dig[k] < 256u) {
            pos[k] = s_dstart[dig[k]] + s_cnt[w][dig[k]] + rank[k];
            sk[pos[k]] = key[k];
            s_dig[pos[k]] = (unsigned char)dig[k];
        }
    }
    __syncthreads();
    const u32 count = (u32)((n - base) < (u64)STS_TILE ? (n - base) : (u64)STS_TILE);
    for (u32 i = tid; i < count; i += STS_WG) {
        const u32 d = s_dig[i];
        kout[s_base[d] + (i - s_dstart[d])] = sk[i];
    }
    __syncthreads();

    // same permutation for the amplitudes
    u64 *sa = reinterpret_cast<u64 *>(s_buf);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (dig[k] < 256u) {
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

hipError_t launch_radix_count(const u64 *keys, const u64 *n_in, const u64 *notmask, int shift, u32 *counts,
                              u64 tiles_cap, int tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_radix_count, dim3(tiles), dim3(STS_WG), 0, s, keys, n_in, notmask, shift, counts, tiles_cap);
    return hipGetLastError();
}

hipError_t launch_radix_scan(const u32 *counts, u64 *prefix, u64 *totals, const u64 *n_in, u64 tiles_cap,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(STS_WG), 0, s, counts, prefix, totals, n_in, tiles_cap);
    return hipGetLastError();
}

hipError_t launch_radix_pass(int prec, const u64 *kin, const void *ain, u64 *kout, void *aout, const u64 *n_in,
                             u64 *n_out, const u64 *notmask, int shift, const u64 *prefix, const u64 *totals,
                             u64 tiles_cap, int tiles, hipStream_t s)
{
    static_assert(sizeof(double2) == 2 * sizeof(u64) && sizeof(float2) == sizeof(u64), "amplitude words");
    if (prec == 0)
        hipLaunchKernelGGL(k_radix_pass<2>, dim3(tiles), dim3(STS_WG), 0, s, kin, (const u64 *)ain, kout,
                           (u64 *)aout, n_in, n_out, notmask, shift, prefix, totals, tiles_cap);
    else
        hipLaunchKernelGGL(k_radix_pass<1>, dim3(tiles), dim3(STS_WG), 0, s, kin, (const u64 *)ain, kout,
                           (u64 *)aout, n_in, n_out, notmask, shift, prefix, totals, tiles_cap);
    return hipGetLastError();
}
