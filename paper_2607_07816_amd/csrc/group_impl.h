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

// full unrolling only for gates of up to 3 qubits (the 32x32 case would
// otherwise multiply the code size, for no gain off the hot path)
template <int M> struct Unroll {
    static constexpr int value = M <= 3 ? (1 << M) : 1;
};

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
    u64 k = 0;
#pragma unroll
    for (int t = 0; t < M; ++t) k |= (u64)((i >> t) & 1u) << g.q[t];
    return k;
}

template <typename AT, int M> __device__ __forceinline__ void group_set(Group<AT, M> &G, u32 j, AT a)
{
#pragma unroll
    for (int jj = 0; jj < (1 << M); ++jj)
        if (jj == (int)j) G.v[jj] = a;
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
    group_set<AT, M>(G, extract_bits<M>(key, g), amp);
    for (u64 p = idx + 1; p < n; ++p) {
        const u64 kp = keys[p];
        const u64 mp = kp & g.notmask;
        if ((sts_mix64(mp) >> sh) != b) break;
        if (mp == rest) group_set<AT, M>(G, extract_bits<M>(kp, g), amps[p]);
    }
}

template <int M> __device__ __forceinline__ double u_re(const GateArg &g, int i, int j)
{
    if (M <= 3) return g.ur[i * (1 << M) + j];
    return g.uptr[2 * (i * (1 << M) + j)];
}

template <int M> __device__ __forceinline__ double u_im(const GateArg &g, int i, int j)
{
    if (M <= 3) return g.ui[i * (1 << M) + j];
    return g.uptr[2 * (i * (1 << M) + j) + 1];
}

// new amplitude with local pattern i of the group
template <typename AT, int M>
__device__ __forceinline__ AT group_out(const GateArg &g, const Group<AT, M> &G, int i)
{
    typedef typename Scalar<AT>::T R;
    if (M == 0) return G.v[0];
    R ar = (R)0, ai = (R)0;
#pragma unroll Unroll<M>::value
    for (int j = 0; j < (1 << M); ++j) {
        if ((G.present >> j) & 1u) {
            const R ur = (R)u_re<M>(g, i, j);
            const R ui = (R)u_im<M>(g, i, j);
            const R vr = G.v[j].x, vi = G.v[j].y;
            const R tr = ur * vr - ui * vi;
            const R ti = ur * vi + ui * vr;
            ar = ar + tr;
            ai = ai + ti;
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

// ---------------------------------------------------------------------------
// pass 1: histogram of the new weights by exponent field, with exact
// mantissa sums, plus each workgroup's best term (weight desc, key asc)
// ---------------------------------------------------------------------------
template <typename AT, int M>
__global__ void __launch_bounds__(STS_WG) k_group_hist(GateArg g, PassBufs b)
{
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
#pragma unroll Unroll<M>::value
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
__global__ void __launch_bounds__(STS_WG) k_group_compact(GateArg g, PassBufs b)
{
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
                if (KIND == STS_KIND_EXTRACT) ctl->side_n = 0;
                else *b.n_out = 0;
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
#pragma unroll Unroll<M>::value
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
        if (KIND == STS_KIND_EXTRACT) ctl->side_n = total;
        else *b.n_out = total;
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
#pragma unroll Unroll<M>::value
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

template <typename AT, int M> hipError_t hist_m(const GateArg &g, const PassBufs &b, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_group_hist<AT, M>), dim3(grid), dim3(STS_WG), 0, s, g, b);
    return hipGetLastError();
}

template <typename AT, int M>
hipError_t compact_m(int kind, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s)
{
    if (kind == STS_KIND_EXTRACT)
        hipLaunchKernelGGL((k_group_compact<AT, M, STS_KIND_EXTRACT>), dim3(tiles), dim3(STS_WG), 0, s, g, b);
    else
        hipLaunchKernelGGL((k_group_compact<AT, M, STS_KIND_EMIT>), dim3(tiles), dim3(STS_WG), 0, s, g, b);
    return hipGetLastError();
}

} // namespace sts_group
