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
// Kernels: one histogram pass over the keys for every digit, a 256-bin scan,
// then one scatter pass per digit. Each scatter pass ranks a 4096-key tile in
// registers and LDS (wave64 ballots find lanes with equal digits), gets the
// tile's global offsets with decoupled look-back, stages the tile in LDS in
// digit order and writes keys and amplitudes out in coalesced runs.
#include "kernels.h"

namespace {

__device__ __forceinline__ u32 bucket_digit(u64 key, u64 notmask, int shift)
{
    return (u32)((sts_mix64(key & notmask) >> shift) & 255u);
}

__global__ void __launch_bounds__(STS_WG) k_radix_hist(const u64 *__restrict__ keys, const u64 *n_in,
                                                        u64 notmask, int hb, int npass,
                                                        u64 *__restrict__ hist)
{
    __shared__ u32 s_h[STS_MAX_PASSES * 256];
    for (int i = threadIdx.x; i < STS_MAX_PASSES * 256; i += STS_WG) s_h[i] = 0;
    __syncthreads();
    const u64 n = *n_in;
    const int base_shift = 64 - hb;
    constexpr int IT = 8; // keys per thread per round, loaded before use
    for (u64 r = (u64)blockIdx.x * STS_WG * IT; r < n; r += (u64)gridDim.x * STS_WG * IT) {
        u64 kk[IT];
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const u64 i = r + (u64)k * STS_WG + threadIdx.x;
            kk[k] = i < n ? keys[i] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const u64 i = r + (u64)k * STS_WG + threadIdx.x;
            if (i >= n) continue;
            const u64 h = sts_mix64(kk[k] & notmask);
            for (int p = 0; p < npass; ++p) {
                const u32 d = (u32)((h >> (base_shift + 8 * p)) & 255u);
                atomicAdd(&s_h[p * 256 + d], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += STS_WG) {
        const u32 c = s_h[i];
        if (c) atomicAdd(&hist[i], (u64)c);
    }
}

// exclusive scan of each pass's 256 digit counts; clears the histogram and
// advances the look-back tags (on the device, so a replayed graph of these
// launches never meets tags of an earlier replay)
__global__ void __launch_bounds__(256) k_radix_scan(u64 *__restrict__ hist, u64 *__restrict__ offs, int npass,
                                                    u32 *epoch)
{
    __shared__ u64 scratch[4];
    if (threadIdx.x == 0) {
        u32 e = *epoch + STS_MAX_PASSES;
        if (e >= (1u << 24) - STS_MAX_PASSES) e = 1;
        *epoch = e;
    }
    for (int p = 0; p < npass; ++p) {
        const u64 v = hist[p * 256 + threadIdx.x];
        u64 tot;
        const u64 ex = block_excl_scan<u64, 256>(v, scratch, &tot);
        offs[p * 256 + threadIdx.x] = ex;
        hist[p * 256 + threadIdx.x] = 0;
    }
}

template <typename AT>
__global__ void __launch_bounds__(STS_WG) k_radix_pass(const u64 *__restrict__ kin, const AT *__restrict__ ain,
                                                        u64 *__restrict__ kout, AT *__restrict__ aout,
                                                        const u64 *n_in, u64 *n_out, u64 notmask, int shift,
                                                        const u64 *__restrict__ offs, u64 *__restrict__ look,
                                                        u32 *tile_ctr, const u32 *epoch_base, int pass)
{
    constexpr int NW = STS_WG / 64;
    constexpr int IT = STS_TILE_ITEMS;
    constexpr int ESZ = sizeof(AT) > sizeof(u64) ? sizeof(AT) : sizeof(u64);
    __shared__ u32 s_tile;
    __shared__ u32 s_cnt[NW][256];
    __shared__ u32 s_dstart[256];
    __shared__ u64 s_base[256];
    __shared__ u32 s_scratch[NW];
    __shared__ unsigned char s_dig[STS_TILE];
    __shared__ __attribute__((aligned(16))) unsigned char s_buf[STS_TILE * ESZ];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    if (tid == 0) {
        const u32 t = atomicAdd(tile_ctr, 1u);
        if (t == gridDim.x - 1) st_agent(tile_ctr, 0u); // last id handed out: reset for the next launch
        s_tile = t;
    }
    for (int i = tid; i < NW * 256; i += STS_WG) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const u64 tile = s_tile;
    const u64 n = *n_in;
    if (tile == 0 && tid == 0) *n_out = n;
    const u64 base = tile * STS_TILE;
    if (base >= n) return;

    // issue every key and amplitude load of the thread first
    u64 key[IT];
    AT amp[IT];
    u32 dig[IT];
    u32 rank[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const u64 e = base + (u64)w * (64 * IT) + (u64)k * 64 + lane;
        if (e < n) {
            key[k] = kin[e];
            amp[k] = ain[e];
        } else {
            key[k] = 0ull;
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
    // global position of this tile's first key with digit tid
    const u64 excl = lb_exclusive(look + tid, 256, tile, tot, *epoch_base + (u32)pass);
    s_base[tid] = offs[tid] + excl;
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
    AT *sa = reinterpret_cast<AT *>(s_buf);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (dig[k] < 256u) sa[pos[k]] = amp[k];
    }
    __syncthreads();
    for (u32 i = tid; i < count; i += STS_WG) {
        const u32 d = s_dig[i];
        aout[s_base[d] + (i - s_dstart[d])] = sa[i];
    }
}

} // namespace

hipError_t launch_radix_hist(const u64 *keys, const u64 *n_in, u64 notmask, int hb, int npass, u64 *hist, int grid,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_radix_hist, dim3(grid), dim3(STS_WG), 0, s, keys, n_in, notmask, hb, npass, hist);
    return hipGetLastError();
}

hipError_t launch_radix_scan(u64 *hist, u64 *offs, int npass, u32 *epoch, hipStream_t s)
{
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(256), 0, s, hist, offs, npass, epoch);
    return hipGetLastError();
}

hipError_t launch_radix_pass(int prec, const u64 *kin, const void *ain, u64 *kout, void *aout, const u64 *n_in,
                             u64 *n_out, u64 notmask, int shift, const u64 *offs, u64 *look, u32 *tile_ctr,
                             const u32 *epoch_base, int pass, int tiles, hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL(k_radix_pass<double2>, dim3(tiles), dim3(STS_WG), 0, s, kin, (const double2 *)ain,
                           kout, (double2 *)aout, n_in, n_out, notmask, shift, offs, look, tile_ctr, epoch_base, pass);
    else
        hipLaunchKernelGGL(k_radix_pass<float2>, dim3(tiles), dim3(STS_WG), 0, s, kin, (const float2 *)ain, kout,
                           (float2 *)aout, n_in, n_out, notmask, shift, offs, look, tile_ctr, epoch_base, pass);
    return hipGetLastError();
}
