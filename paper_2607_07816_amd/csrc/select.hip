// select.hip - finding the cut of a truncation exactly.
//
// Truncation keeps the shortest prefix of the terms ranked by (|a|^2
// descending, key ascending) that holds at least p of the mass, and at most K
// terms (Sec. III; the ranking by decreasing |a|^2 of Sec. IV.B). Instead of
// sorting all candidates, the cut is located by most-significant-digit
// selection on the rank:
//   level 1  - the exponent field of |a|^2 (2048 bins, from the histogram
//              pass over the recomputed candidates),
//   level 2  - within that exponent, the top 11 bits of the within-exponent
//              rank key V = ((2^52 - 1 - fraction) << 64) | key, from the side
//              buffer of that exponent's candidates,
//   level 3+ - further 11-bit digits of V inside one workgroup (level 3 from
//              a histogram built while the level-2 subset is copied out),
//              until at most 512 terms remain; those are sorted in LDS.
// Masses are exact: each bin carries the exact integer sum of its weights'
// mantissas, levels >= 2 share one exponent, and level 1 prefixes are exact
// integers on the 2^-1074 grid. Every decision therefore equals the one made
// in exact arithmetic, and the kept mass S is correctly rounded.
#include <algorithm>

#include "kernels.h"

namespace {

// bit position of the unit 2^(max(e,1)-1075) on the 2^-1074 grid
__device__ __forceinline__ int unit_bit(int e) { return (e > 0 ? e : 1) - 1; }

__device__ __forceinline__ u128 make128(u64 lo, u64 hi) { return ((u128)hi << 64) | lo; }

// ---------------------------------------------------------------------------
// Exact masses, one wave wide: a number of 64 limbs of 64 bits (units
// 2^-1074), limb i held by lane i. Every lane of the wave takes part in each
// operation. Carries between limbs are resolved at once from two ballots: a
// limb generates a carry (its sum wrapped) or propagates one (its sum is all
// ones), and the carries into the limbs are the carries of the binary sum
// (G | P) + G, i.e. ((G | P) + G) ^ (G | P) ^ G.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 wl_carry_in(bool gen, bool prop)
{
    const u64 G = __ballot(gen), P = __ballot(prop);
    const u64 X = G | P;
    return (((X + G) ^ X ^ G) >> sts_lane()) & 1ull;
}

__device__ __forceinline__ u64 wl_add(u64 a, u64 b)
{
    const u64 s = a + b;
    return s + wl_carry_in(s < a, s == ~0ull);
}

// a - b, a >= b
__device__ __forceinline__ u64 wl_sub(u64 a, u64 b)
{
    const u64 d = a - b;
    return d - wl_carry_in(a < b, d == 0);
}

// this lane's limb of v * 2^bit, v < 2^128 given as (lo, hi)
__device__ __forceinline__ u64 wl_piece(u64 lo, u64 hi, int bit)
{
    const int k = sts_lane() - (bit >> 6), off = bit & 63;
    if (k == 0) return lo << off;
    if (k == 1) return off ? (hi << off) | (lo >> (64 - off)) : hi;
    if (k == 2) return off ? hi >> (64 - off) : 0ull;
    return 0ull;
}

// sign of a - b
__device__ __forceinline__ int wl_cmp(u64 a, u64 b)
{
    const u64 D = __ballot(a != b);
    if (!D) return 0;
    const int top = 63 - __clzll((long long)D);
    return ((__ballot(a > b) >> top) & 1ull) ? 1 : -1;
}

// limb `src` of the number (0 outside 0..63); src may differ between lanes
__device__ __forceinline__ u64 wl_limb(u64 a, int src)
{
    const u64 v = __shfl(a, src & 63, 64);
    return (src >= 0 && src < 64) ? v : 0ull;
}

// a >> s (s >= 0), and whether any bit below s was set
__device__ __forceinline__ u64 wl_shr(u64 a, int s, bool *sticky)
{
    const int q = s >> 6, r = s & 63, lane = sts_lane();
    const u64 a0 = wl_limb(a, lane + q), a1 = wl_limb(a, lane + q + 1);
    const u64 low = lane < q ? a : (lane == q && r ? (a & ((1ull << r) - 1)) : 0ull);
    *sticky = __ballot(low != 0) != 0;
    return r ? (a0 >> r) | (a1 << (64 - r)) : a0;
}

// ceil(a * m / 2^s), m < 2^64
__device__ __forceinline__ u64 wl_mul_shr_ceil(u64 a, u64 m, int s)
{
    const u128 pr = (u128)a * m;
    const u64 hi_below = __shfl_up((u64)(pr >> 64), 1, 64);
    const u64 t = wl_add((u64)pr, sts_lane() > 0 ? hi_below : 0ull);
    bool sticky;
    const u64 q = wl_shr(t, s, &sticky);
    return sticky ? wl_add(q, sts_lane() == 0 ? 1ull : 0ull) : q;
}

// nearest binary64 (ties to even); the result is the same in every lane
__device__ inline double wl_to_double(u64 a)
{
    const u64 NZ = __ballot(a != 0);
    if (!NZ) return 0.0;
    const int top = 63 - __clzll((long long)NZ);
    const u64 L0 = wl_limb(a, top), L1 = wl_limb(a, top - 1), L2 = wl_limb(a, top - 2);
    const bool below = top >= 3 && (NZ & ((1ull << (top - 2)) - 1)) != 0;
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

// Subset of the rank order still holding the cut: the terms of exponent e*
// whose rank key V has the high part vpre above bit vshift.
struct Sub {
    u64 cnt_before; // terms ranked before the subset
    u128 mb;        // their mantissa sum inside e* (units 2^(max(e*,1)-1075))
    u128 vpre;
    int vshift;
    u64 count;      // terms in the subset
};

__device__ inline void sub_load(Sub &s, const DevCtl *ctl)
{
    s.cnt_before = ctl->cnt_before;
    s.mb = make128(ctl->mb_lo, ctl->mb_hi);
    s.vpre = make128(ctl->vpre_lo, ctl->vpre_hi);
    s.vshift = ctl->vshift;
    s.count = ctl->sub_count;
}

__device__ inline void sub_store(const Sub &s, DevCtl *ctl)
{
    ctl->cnt_before = s.cnt_before;
    ctl->mb_lo = (u64)s.mb;
    ctl->mb_hi = (u64)(s.mb >> 64);
    ctl->vpre_lo = (u64)s.vpre;
    ctl->vpre_hi = (u64)(s.vpre >> 64);
    ctl->vshift = s.vshift;
    ctl->sub_count = s.count;
}

// Pick the first digit (ascending = rank order) where the rule is met, over
// 2048 bins held in (cnt[], hi[], lo[]) - global (agent loads) or LDS - by NT
// threads, and narrow *sub to it. K, R: the rule (R all ones = no p-mass).
// Returns false if no digit qualifies.
// inclusive scan of (count, mass) pairs over a workgroup of NT threads, in
// place: wave scans, then the wave totals through LDS (one barrier; sc, sm
// hold NT / 64 entries and are not read again before the caller's next
// barrier)
template <int NT>
__device__ __forceinline__ void block_scan_cm(u64 &c, u128 &m, u64 *sc, u128 *sm)
{
    const int lane = sts_lane(), w = (int)threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u64 oc = __shfl_up(c, d, 64);
        const u64 ol = __shfl_up((u64)m, d, 64), oh = __shfl_up((u64)(m >> 64), d, 64);
        if (lane >= d) {
            c += oc;
            m += make128(ol, oh);
        }
    }
    if (lane == 63) {
        sc[w] = c;
        sm[w] = m;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        if (i < w) {
            c += sc[i];
            m += sm[i];
        }
    }
}

template <int NT>
__device__ bool pick_digit(const u64 *cntp, const u64 *hip_, const u64 *lop, bool agent, u64 K, u128 R, int dw,
                           Sub *sub, u128 *s_m, u64 *s_c, u32 *s_hit)
{
    constexpr int PER = STS_NBIN / NT;
    const int t = threadIdx.x;
    u64 c[PER];
    u128 ms[PER];
    u64 cc = 0;
    u128 mm = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int d = PER * t + k;
        if (agent) {
            c[k] = ld_agent(&cntp[d]);
            ms[k] = ((u128)ld_agent(&hip_[d]) << 26) + (u128)ld_agent(&lop[d]);
        } else {
            c[k] = cntp[d];
            ms[k] = ((u128)hip_[d] << 26) + (u128)lop[d];
        }
        cc += c[k];
        mm += ms[k];
    }
    const u64 own_c = cc;
    const u128 own_m = mm;
    if (t == 0) *s_hit = 0xffffffffu;
    block_scan_cm<NT>(cc, mm, s_c, s_m);
    // exclusive prefix of this thread's bins, from the subset's start
    u64 cnt = sub->cnt_before + (cc - own_c);
    u128 m = sub->mb + (mm - own_m);
    u32 hit = 0xffffffffu;
    u64 cnt_hit = 0;
    u128 m_hit = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (hit == 0xffffffffu && c[k]) {
            const bool hk = K > 0 && cnt + c[k] >= K;
            const bool hp = m + ms[k] >= R;
            if (hk || hp) {
                hit = (u32)(PER * t + k);
                cnt_hit = cnt;
                m_hit = m;
            } else {
                cnt += c[k];
                m += ms[k];
            }
        }
    }
    if (hit != 0xffffffffu) atomicMin(s_hit, hit);
    __syncthreads();
    const u32 first = *s_hit;
    if (first == 0xffffffffu) {
        __syncthreads();
        return false;
    }
    if (hit == first) {
        const int k = (int)first - PER * t;
        sub->vpre = (sub->vpre << dw) | (u128)first;
        sub->vshift -= dw;
        sub->cnt_before = cnt_hit;
        sub->mb = m_hit;
        sub->count = c[k];
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------
// level 1: one workgroup of 256 threads. Thread t owns the eight exponent
// bins 2047-8t .. 2040-8t (descending weight order). The bins that hold
// candidates are listed in rank order in LDS; one wave then adds their exact
// masses up (the total W and the p-mass target), and walks them again to the
// first bin where the rule is met.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pick1(PassBufs b, int groups, int peak_only, int predicted)
{
    __shared__ u32 s_e[STS_NBIN];   // the non-empty bins in rank order: exponent field,
    __shared__ u64 s_c[STS_NBIN];   // count,
    __shared__ __attribute__((aligned(16))) u64 s_lo[STS_NBIN]; // mantissa sum (low, high words)
    __shared__ u64 s_hi[STS_NBIN];
    __shared__ u32 s_scan[4];
    __shared__ u64 s_bw[4], s_bk[4];
    __shared__ u64 s_w[6];
    __shared__ Sub s_sub;   // level 2 of a sampled window that holds the cut
    __shared__ u32 s_fine, s_hit2;
    __shared__ u64 s_sub_R_lo, s_sub_R_hi;
    __shared__ u64 s_chunk[4][64]; // exact mass of each quarter of the bin list (a limb per lane)
    __shared__ u64 s_chunk_c[4];   // and its count
    const int t = threadIdx.x;
    DevCtl *ctl = b.ctl;
    u64 *h1 = b.h1;
    // the exponent of the window the histogram pass copied (predicted steps)
    const int w_mode = ctl->w_mode;
    const int e_w = predicted ? (w_mode ? ctl->e_w : ctl->e_pred) : -1;
    if (t < 6) s_w[t] = 0;
    if (t == 0) s_fine = 0;

    // own bins: every load issued before any is used
    u64 c[8], hi[8], lo[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int e = 2047 - 8 * t - k;
        c[k] = h1[e];
        hi[k] = h1[STS_NBIN + e];
        lo[k] = h1[2 * STS_NBIN + e];
    }
    // the per-workgroup peaks too (reduced below)
    constexpr int BPT = (STS_MAX_GROUPS + 255) / 256;
    u64 bwv[BPT], bkv[BPT];
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
        const int i = t + 256 * r;
        bwv[r] = i < groups ? b.best[i] : 0ull;
        bkv[r] = i < groups ? b.best[STS_MAX_GROUPS + i] : ~0ull;
    }
    // the window sums of the histogram workgroups: count of candidates above
    // the window and mantissa sums of those in its exponent, then count and
    // sums of those inside it
    // (loaded whenever the pass predicted, before the control block says
    // whether a window was copied)
    u64 v[6] = {0, 0, 0, 0, 0, 0};
    if (predicted) {
#pragma unroll
        for (int r = 0; r < STS_MAX_GROUPS / 256; ++r) { // every load issued before any is used
            const int i = t + 256 * r;
            if (i < groups) {
#pragma unroll
                for (int f = 0; f < 6; ++f) v[f] += b.wpart[f * STS_MAX_GROUPS + i];
            }
        }
    }
    if (e_w >= 0) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) v[f] += __shfl_xor(v[f], d, 64);
        }
        __syncthreads(); // s_w cleared
        if ((t & 63) == 0) {
#pragma unroll
            for (int f = 0; f < 6; ++f) atomicAdd((unsigned long long *)&s_w[f], (unsigned long long)v[f]);
        }
    }
    // list the non-empty bins in rank order
    u32 nz = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) nz += c[k] ? 1u : 0u;
    u32 nbins;
    u32 at = block_excl_scan<u32, 256>(nz, s_scan, &nbins);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!c[k]) continue;
        s_e[at] = (u32)(2047 - 8 * t - k);
        s_c[at] = c[k];
        const u128 ms = ((u128)hi[k] << 26) + (u128)lo[k];
        s_lo[at] = (u64)ms;
        s_hi[at] = (u64)(ms >> 64);
        ++at;
    }
    // peak: reduce the per-workgroup bests (written by the identity pass of
    // sts_peak only)
    if (peak_only) {
        u64 bw = 0, bk = ~0ull;
#pragma unroll
        for (int r = 0; r < BPT; ++r) {
            const u64 w = bwv[r], k = bkv[r];
            if (w > bw || (w == bw && k < bk)) {
                bw = w;
                bk = k;
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
        if ((t & 63) == 0) {
            s_bw[t >> 6] = bw;
            s_bk[t >> 6] = bk;
        }
    }
    __syncthreads();

    // exact sums of the listed bins in four chunks, one wave each (a chain of
    // exact additions per bin, a quarter as long as over all bins)
    const u32 chunk = (nbins + 3) / 4;
    {
        const int q = t >> 6;
        const u32 j0 = (u32)q * chunk, j1 = j0 + chunk < nbins ? j0 + chunk : nbins;
        u64 C = 0, nc = 0;
        for (u32 j = j0; j < j1; ++j) {
            C = wl_add(C, wl_piece(s_lo[j], s_hi[j], unit_bit((int)s_e[j])));
            nc += s_c[j];
        }
        s_chunk[q][t & 63] = C;
        if ((t & 63) == 0) s_chunk_c[q] = nc;
    }
    __syncthreads();

    if (t < 64) { // one wave: the total, the target and the cut's bin
        const int lane = t;
        u64 W = 0, total_c = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            W = wl_add(W, s_chunk[q][lane]);
            total_c += s_chunk_c[q];
        }
        const double Wd = wl_to_double(W);
        if (peak_only) {
            if (lane == 0) {
                ctl->cand_all = total_c;
                ctl->peak_W = Wd;
                u64 w = s_bw[0], k = s_bk[0];
                for (int i = 1; i < 4; ++i)
                    if (s_bw[i] > w || (s_bw[i] == w && s_bk[i] < k)) {
                        w = s_bw[i];
                        k = s_bk[i];
                    }
                ctl->peak_key = k;
                ctl->peak_w = (w >> 63) ? __longlong_as_double((long long)(w & ~(1ull << 63))) : 0.0;
            }
        } else {
            const u64 K = ctl->K;
            const double p = ctl->p;
            const bool p_on = p > 0.0 && p < 1.0;
            // p-mass target T = ceil(p * W), exactly
            u64 T = 0;
            if (p_on) {
                const u64 pb = sts_dbits(p);
                const u64 pe = pb >> 52, pf = pb & ((1ull << 52) - 1);
                const u64 pm = pe ? (pf | (1ull << 52)) : pf;
                const int sh = pe ? (int)(1075 - pe) : 1074;
                T = wl_mul_shr_ceil(W, pm, sh);
            }
            if (lane < STS_NL) ctl->T.l[lane] = T;
            if (lane == 0) {
                ctl->cand_all = total_c;
                ctl->W = Wd;
                ctl->n_cand = total_c;
                ctl->tot_steps += 1;
                ctl->tot_updates += *b.n_in;
                ctl->tot_cand += total_c;
            }
            // the first bin in rank order where the rule is met: the first
            // chunk through which it is met (the rule only grows along the
            // ranking), then that chunk's bins
            u64 S = 0, cnt = 0;
            u32 hit = 0xffffffffu;
            for (int q = 0; q < 4; ++q) {
                const u64 inc_q = wl_add(S, s_chunk[q][lane]);
                const bool met_q = (K > 0 && cnt + s_chunk_c[q] >= K) || (p_on && wl_cmp(inc_q, T) >= 0);
                if (met_q) {
                    const u32 j0 = (u32)q * chunk, j1 = j0 + chunk < nbins ? j0 + chunk : nbins;
                    for (u32 j = j0; j < j1; ++j) {
                        const u64 inc = wl_add(S, wl_piece(s_lo[j], s_hi[j], unit_bit((int)s_e[j])));
                        const bool hk = K > 0 && cnt + s_c[j] >= K;
                        const bool hp = p_on && wl_cmp(inc, T) >= 0;
                        if (hk || hp) {
                            hit = j;
                            break;
                        }
                        S = inc;
                        cnt += s_c[j];
                    }
                    break;
                }
                S = inc_q;
                cnt += s_chunk_c[q];
            }
            if (hit == 0xffffffffu) {
                if (lane == 0) {
                    ctl->keep_all = 1;
                    ctl->dropped = 0;
                    ctl->L = total_c;
                    ctl->scale = 1.0;
                    ctl->S = Wd;
                    ctl->frac = 1.0;
                    ctl->level = 1;
                    ctl->pred_hit = 0;
                    ctl->e_pred = -1;
                }
            } else {
                const int e = (int)s_e[hit];
                const int ub = unit_bit(e);
                // does the copied window hold the cut? Exactly when the rule is
                // not met through the candidates above it and is met through it
                bool in_window = false;
                u64 ca = 0, cw = 0;
                u128 ma = 0;
                if (e == e_w) {
                    // the histogram pass counted every candidate above the window;
                    // those in exponents above e are the cnt ranked before this bin
                    ca = s_w[0] - cnt;
                    cw = s_w[3];
                    ma = ((u128)s_w[1] << 26) + (u128)s_w[2];
                    const u128 mw = ((u128)s_w[4] << 26) + (u128)s_w[5];
                    const u64 Sa = wl_add(S, wl_piece((u64)ma, (u64)(ma >> 64), ub));
                    const bool met_a = (K > 0 && cnt + ca >= K) || (p_on && wl_cmp(Sa, T) >= 0);
                    const u64 Sw = wl_add(Sa, wl_piece((u64)mw, (u64)(mw >> 64), ub));
                    const bool met_w = (K > 0 && cnt + ca + cw >= K) || (p_on && wl_cmp(Sw, T) >= 0);
                    in_window = !met_a && met_w;
                }
                // remaining mass to reach inside the bin, in its units (rounded up)
                u64 R_lo = ~0ull, R_hi = ~0ull;
                if (p_on) {
                    bool sticky;
                    const u64 q = wl_shr(wl_sub(T, S), ub, &sticky);
                    const bool over = __ballot(lane >= 2 && q != 0) != 0;
                    u128 r = ((u128)__shfl(q, 1, 64) << 64) | (u128)__shfl(q, 0, 64);
                    if (!over) {
                        if (sticky) r += 1;
                        if (r != 0 || !sticky) {
                            R_lo = (u64)r;
                            R_hi = (u64)(r >> 64);
                        }
                    }
                }
                if (lane < STS_NL) ctl->S_excl.l[lane] = S;
                if (lane == 0 && in_window && w_mode && predicted) {
                    // the histogram pass binned this window for level 2: the
                    // whole workgroup picks its digit below
                    s_fine = 1;
                    s_sub.cnt_before = cnt + ca;
                    s_sub.mb = ma;
                    s_sub.vpre = 0;
                    s_sub.vshift = 116;
                    s_sub.count = cw;
                    s_sub_R_lo = R_lo;
                    s_sub_R_hi = R_hi;
                }
                if (lane == 0) {
                    ctl->keep_all = 0;
                    ctl->pred_hit = in_window ? 1 : 0;
                    ctl->e_pred = e;
                    ctl->e_star = e;
                    ctl->cnt_before = in_window ? cnt + ca : cnt;
                    ctl->sub_count = in_window ? cw : s_c[hit];
                    ctl->mb_lo = in_window ? (u64)ma : 0;
                    ctl->mb_hi = in_window ? (u64)(ma >> 64) : 0;
                    ctl->level = 1;
                    ctl->R_lo = R_lo;
                    ctl->R_hi = R_hi;
                }
            }
            if (lane == 0) {
                ctl->w2_mode = predicted && w_mode; // the histogram pass binned the window for level 2
                ctl->w_mode = 0;                     // a window serves one step
                ctl->l2_done = 0;
            }
        }
    }
    __syncthreads();
    for (int i = t; i < 3 * STS_NBIN; i += 256) h1[i] = 0;
    if (s_fine) { // uniform
        // level 2 from the window's bins (the side pass then has nothing to
        // do); the bin lists above are done with, so their LDS serves the pick
        const u128 R = make128(s_sub_R_lo, s_sub_R_hi);
        u128 *s_m = reinterpret_cast<u128 *>(s_lo);
        u64 *s_c2 = s_hi;
        const bool ok = pick_digit<256>(b.h2w, b.h2w + STS_NBIN, b.h2w + 2 * STS_NBIN, true, ctl->K, R, 11, &s_sub,
                                        s_m, s_c2, &s_hit2);
        if (ok && t <= STS_SUB_REGIONS) st_agent(&b.sub_cnt[t * 32], 0u);
        if (t == 0) {
            if (ok) {
                sub_store(s_sub, ctl);
                ctl->level = 2;
                ctl->l2_done = 1;
            } else {
                atomicOr(&ctl->flags, STS_F_UNRESOLVED);
            }
        }
        for (int i = t; i < 3 * STS_NBIN; i += 256) st_agent(&b.h2w[i], 0ull);
    }
}

// The side buffer is either dense (entries [0, side_n)) or split into slabs
// of 2^shift entries (one per tile, or one per wave of a tile in the
// histogram pass), slab s holding t_side[s] entries from its start. Its
// entries are visited through a flat index f over the whole layout.
struct SideView {
    const u64 *key;
    const u64 *w;
    const u32 *cnt;
    u64 flat;  // flat indices to visit
    int dense;
    int shift;
};

__device__ __forceinline__ SideView side_view(const PassBufs &b, const DevCtl *ctl)
{
    SideView v;
    v.key = b.side_key;
    v.w = b.side_w;
    v.cnt = b.t_side;
    v.dense = ctl->side_dense;
    v.shift = ctl->side_slab_shift;
    const u64 f = v.dense ? ctl->side_n : (ctl->side_ntiles << v.shift);
    v.flat = f < b.side_cap ? f : b.side_cap;
    return v;
}

__device__ __forceinline__ bool side_valid(const SideView &v, u64 f)
{
    return v.dense || (f & ((1ull << v.shift) - 1)) < (u64)v.cnt[f >> v.shift];
}

// The same entries as a list of chunks: the tiles of the tiled layout (each
// the runs of its 1 or 4 slabs), or runs of 8192 entries of the dense one.
// Workgroups walk chunks; threads walk the entries of a chunk.
struct SideChunks {
    u64 nchunks;
    int dense;
    int shift;
    int spl;
    u64 n;          // dense: entries
    u64 cap;
    const u32 *cnt;
};

__device__ __forceinline__ SideChunks side_chunks(const PassBufs &b, const DevCtl *ctl)
{
    SideChunks c;
    c.dense = ctl->side_dense;
    c.shift = ctl->side_slab_shift;
    c.spl = ctl->side_spt_log2;
    c.cap = b.side_cap;
    c.cnt = b.t_side;
    c.n = ctl->side_n < b.side_cap ? ctl->side_n : b.side_cap;
    c.nchunks = c.dense ? (c.n + 8191) / 8192 : (ctl->side_ntiles >> c.spl);
    return c;
}

// the entries of chunk t (visited with slab_at)
__device__ __forceinline__ TileSlabs chunk_of(const SideChunks &c, u64 t)
{
    if (!c.dense) return tile_slabs(c.cnt, t, c.spl, c.shift, false, c.cap);
    TileSlabs s;
    const u64 base = t * 8192;
    const u32 count = (u32)(c.n - base < 8192 ? c.n - base : 8192);
    s.f0 = base;
    s.f1 = s.f2 = s.f3 = 0;
    s.p1 = s.p2 = s.p3 = s.n = count;
    return s;
}

// most entries a chunk can hold
__device__ __forceinline__ u64 chunk_max(const SideChunks &c) { return c.dense ? 8192ull : (1ull << (c.shift + c.spl)); }

// within-exponent rank key: ascending V = descending weight, then ascending key
__device__ __forceinline__ u128 rank_key(u64 wbits, u64 key)
{
    const u64 frac = wbits & ((1ull << 52) - 1);
    return ((u128)(((1ull << 52) - 1) - frac) << 64) | (u128)key;
}

__device__ __forceinline__ u64 mant_of_v(u128 v, int e)
{
    const u64 frac = ((1ull << 52) - 1) - (u64)(v >> 64);
    return e ? (frac | (1ull << 52)) : frac;
}


// ---------------------------------------------------------------------------
// level 2 over the side buffer (many workgroups), pick by the last one
// ---------------------------------------------------------------------------
// LDS bins of the level-2 histogram: s_hi sums mantissa >> 20, s_lo sums
// mantissa & (2^20 - 1) plus count << 44. A workgroup flushes them before
// 2^19 entries have gone in, so neither field can overflow into the next.
constexpr int SH_LOW = 20;
constexpr u64 SH_FLUSH = 1ull << 19;

__device__ __forceinline__ void side_flush(u64 *h2, u64 *s_hi, u64 *s_lo)
{
    for (int i = threadIdx.x; i < STS_NBIN; i += 256) {
        const u64 lo = s_lo[i];
        const u64 c = lo >> 44;
        if (c) {
            const u128 tot = ((u128)s_hi[i] << SH_LOW) + (u128)(lo & ((1ull << 44) - 1));
            atomicAdd(&h2[i], c);
            atomicAdd(&h2[STS_NBIN + i], (u64)(tot >> 26));
            atomicAdd(&h2[2 * STS_NBIN + i], (u64)tot & ((1ull << 26) - 1));
        }
        s_hi[i] = 0;
        s_lo[i] = 0;
    }
}

// this workgroup's share of the level-2 histogram of the side buffer, added
// to h2
__device__ __forceinline__ void side_bins(const PassBufs &b, DevCtl *ctl, u64 *h2, u64 *s_hi, u64 *s_lo)
{
    constexpr int UN = 16; // entries in flight per lane
    for (int i = threadIdx.x; i < STS_NBIN; i += 256) {
        s_hi[i] = 0;
        s_lo[i] = 0;
    }
    __syncthreads();
    const SideChunks sc = side_chunks(b, ctl);
    // each wave takes a chunk of its own, so a workgroup has four chunks'
    // loads in flight; a round of four chunks adds at most 4 * chunk_max
    // entries, and the bins are flushed before they could overflow
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const u64 cmax = chunk_max(sc);
    u64 since = 0;
    for (u64 r0 = (u64)blockIdx.x * 4; r0 < sc.nchunks; r0 += (u64)gridDim.x * 4) {
        if (since + 4 * cmax > SH_FLUSH) { // uniform across the workgroup
            __syncthreads();
            side_flush(h2, s_hi, s_lo);
            __syncthreads();
            since = 0;
        }
        since += 4 * cmax;
        const u64 t = r0 + wv;
        if (t >= sc.nchunks) continue;
        const TileSlabs ch = chunk_of(sc, t);
        const u32 count = ch.n;
        for (u32 i0 = 0; i0 < count; i0 += UN * 64) {
            u64 w[UN];
#pragma unroll
            for (int r = 0; r < UN; ++r) {
                const u32 i = i0 + (u32)r * 64 + lane;
                w[r] = i < count ? b.side_w[slab_at(ch, i)] : ~0ull;
            }
#pragma unroll
            for (int r = 0; r < UN; ++r) {
                if (w[r] == ~0ull) continue; // past the chunk (no weight has all bits set)
                const u64 vh = ((1ull << 52) - 1) - (w[r] & ((1ull << 52) - 1));
                const u32 d = (u32)(vh >> 41);
                const u64 mant = sts_mant(w[r]);
                atomicAdd(&s_hi[d], mant >> SH_LOW);
                atomicAdd(&s_lo[d], (mant & ((1ull << SH_LOW) - 1)) | (1ull << 44));
            }
        }
    }
    __syncthreads();
    side_flush(h2, s_hi, s_lo);
}

__global__ void __launch_bounds__(256) k_side_hist(PassBufs b, u64 *h2)
{
    __shared__ u64 s_hi[STS_NBIN];
    __shared__ u64 s_lo[STS_NBIN];
    __shared__ u128 s_m[256];
    __shared__ u64 s_c[256];
    __shared__ u32 s_hit, s_flag;
    __shared__ Sub s_sub;
    DevCtl *ctl = b.ctl;
    const int keep_all = ctl->keep_all, w2 = ctl->w2_mode;
    // the level-1 pick already picked level 2 from the histogram pass's
    // window bins
    if (ctl->l2_done) return;
    // the histogram pass binned a sampled window that holds the cut: its
    // level-2 bins are complete, and only the pick is left
    const bool fine = w2 && ctl->pred_hit && !keep_all;
    if (keep_all && !w2) return;
    if (!keep_all && !fine) side_bins(b, ctl, h2, s_hi, s_lo);
    if (!sts_last_block(&ctl->done[1], &s_flag)) return;
    if (!keep_all) {
        const u64 *hs = fine ? b.h2w : h2;
        if (threadIdx.x == 0) {
            s_sub.cnt_before = ctl->cnt_before;
            s_sub.mb = make128(ctl->mb_lo, ctl->mb_hi); // the window's exponent above it, or 0
            s_sub.vpre = 0;
            s_sub.vshift = 116;
            s_sub.count = ctl->sub_count;
        }
        __syncthreads();
        const u128 R = make128(ctl->R_lo, ctl->R_hi);
        if (pick_digit<256>(hs, hs + STS_NBIN, hs + 2 * STS_NBIN, true, ctl->K, R, 11, &s_sub, s_m, s_c, &s_hit)) {
            if (threadIdx.x <= STS_SUB_REGIONS) st_agent(&b.sub_cnt[threadIdx.x * 32], 0u);
            if (threadIdx.x == 0) {
                sub_store(s_sub, ctl);
                ctl->level = 2;
            }
        } else if (threadIdx.x == 0) {
            atomicOr(&ctl->flags, STS_F_UNRESOLVED);
        }
        if (!fine)
            for (int i = threadIdx.x; i < 3 * STS_NBIN; i += 256) st_agent(&h2[i], 0ull);
    }
    if (w2)
        for (int i = threadIdx.x; i < 3 * STS_NBIN; i += 256) st_agent(&b.h2w[i], 0ull);
}


// ---------------------------------------------------------------------------
// copy the level-2 subset out of the side buffer (many workgroups), so the
// final workgroup reads a few thousand terms instead of the whole buffer
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_side_extract(PassBufs b)
{
    constexpr int UN = 4;
    DevCtl *ctl = b.ctl;
    // every control load issued before any is used
    const int keep_all = ctl->keep_all;
    const u32 flags = ctl->flags;
    const u64 sub_count = ctl->sub_count;
    const SideChunks sc = side_chunks(b, ctl);
    const int vshift = ctl->vshift;
    const u128 vpre = make128(ctl->vpre_lo, ctl->vpre_hi);
    const int e = ctl->e_star;
    if (keep_all || (flags & (STS_F_UNRESOLVED | STS_F_SIDE_OVERFLOW))) return;
    if (sub_count > b.sub_cap) return; // the final kernel reads the side buffer itself
    // the subset's histogram for the next level (the digit below vshift),
    // with exact mantissa sums, as the final workgroup's first level would
    // bin it: that workgroup then starts from the pick
    const int dw = vshift < 11 ? vshift : 11;
    // each wave fills one of STS_SUB_REGIONS regions, whose counters sit on
    // separate cache lines (one shared counter would serialise every wave)
    const u32 region = (blockIdx.x * 4u + (threadIdx.x >> 6)) % STS_SUB_REGIONS;
    const u32 region_len = (u32)(b.sub_cap / STS_SUB_REGIONS);
    const u64 region_base = (u64)region * region_len;
    u32 *cnt = &b.sub_cnt[region * 32];
    const u64 lt = sts_lanemask_lt();
    // tiles (a few hundred window entries each): one wave per tile, so that
    // every tile's wave is resident at once; dense runs: a workgroup per run
    const bool per_wave = !sc.dense;
    const u32 wv = threadIdx.x >> 6;
    const u64 t0 = per_wave ? (u64)blockIdx.x * 4 + wv : (u64)blockIdx.x;
    const u64 tstep = per_wave ? (u64)gridDim.x * 4 : (u64)gridDim.x;
    const u32 nth = per_wave ? 64u : 256u, me = per_wave ? (u32)sts_lane() : (u32)threadIdx.x;
    for (u64 t = t0; t < sc.nchunks; t += tstep) {
        const TileSlabs ch = chunk_of(sc, t);
        const u32 count = ch.n;
        for (u32 i0 = 0; i0 < count; i0 += UN * nth) {
            u64 w[UN];
#pragma unroll
            for (int r = 0; r < UN; ++r) {
                const u32 j = i0 + (u32)r * nth + me;
                w[r] = j < count ? b.side_w[slab_at(ch, j)] : ~0ull;
            }
#pragma unroll
            for (int r = 0; r < UN; ++r) {
                const u32 j = i0 + (u32)r * nth + me;
                const u64 i = j < count ? slab_at(ch, j) : 0ull;
                bool take = false;
                u64 k = 0;
                if (w[r] != ~0ull) {
                    if (vshift >= 64) { // the fixed part lies in the weight half of V
                        const u64 vh = ((1ull << 52) - 1) - (w[r] & ((1ull << 52) - 1));
                        take = (vh >> (vshift - 64)) == (u64)vpre;
                        if (take) k = b.side_key[i];
                    } else {
                        k = b.side_key[i];
                        take = (rank_key(w[r], k) >> vshift) == vpre;
                    }
                }
                const u64 mask = __ballot(take);
                if (!mask) continue;
                const int leader = __ffsll((long long)mask) - 1;
                u32 pos = 0;
                if (sts_lane() == leader) {
                    pos = atomicAdd(cnt, (u32)__popcll(mask));
                    if (pos + (u32)__popcll(mask) > region_len) atomicOr(&b.sub_cnt[STS_SUB_REGIONS * 32], 1u);
                }
                pos = __shfl(pos, leader, 64) + (u32)__popcll(mask & lt);
                if (take && pos < region_len) {
                    b.sub_key[region_base + pos] = k;
                    b.sub_w[region_base + pos] = w[r];
                }
                if (take && dw > 0) {
                    const u128 v = rank_key(w[r], k);
                    const u32 d = (u32)((v >> (vshift - dw)) & (u128)((1u << dw) - 1));
                    const u64 mant = mant_of_v(v, e);
                    atomicAdd(&b.h3[d], 1ull);
                    atomicAdd(&b.h3[STS_NBIN + d], mant >> 26);
                    atomicAdd(&b.h3[2 * STS_NBIN + d], mant & ((1ull << 26) - 1));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// final levels and the exact cut, one workgroup of 1024 threads
// ---------------------------------------------------------------------------
constexpr int FT = 1024;
constexpr int FB = 8; // subset entries a thread of the final workgroup loads at a time

__global__ void __launch_bounds__(FT) k_final(PassBufs b)
{
    // LDS: the level histograms and the sort buffer share one region
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[STS_SMALL * sizeof(u128)];
    __shared__ u128 s_m[FT];
    __shared__ u64 s_c[FT];
    __shared__ u32 s_hit, s_n;
    u64 *h_cnt = reinterpret_cast<u64 *>(s_raw);
    u64 *h_hi = h_cnt + STS_NBIN;
    u64 *h_lo = h_hi + STS_NBIN;
    u128 *sv = reinterpret_cast<u128 *>(s_raw);
    static_assert(3 * STS_NBIN * sizeof(u64) <= STS_SMALL * sizeof(u128), "LDS union");

    __shared__ Sub s_sub;
    DevCtl *ctl = b.ctl;
    if (ctl->keep_all) return;
    if (ctl->flags & (STS_F_UNRESOLVED | STS_F_SIDE_OVERFLOW)) return;
    const int t = threadIdx.x;
    const int e = ctl->e_star;
    // the subset and what the cut's thread needs at the end, loaded now
    // (visible after the barrier below)
    __shared__ u64 s_Sx[STS_NL], s_ncand;
    __shared__ double s_W, s_l10;
    if (t == 0) {
        sub_load(s_sub, ctl);
        s_ncand = ctl->n_cand;
        s_W = ctl->W;
        s_l10 = ctl->log10_cum;
    }
    if (t < STS_NL) s_Sx[t] = ctl->S_excl.l[t];
    // the subset regions when they hold the whole subset, else the side buffer
    // (entries of region r at r * region_len + [0, count_r); visited through
    // an exclusive prefix of the counts, so only filled slots are read)
    __shared__ u32 s_regpre[STS_SUB_REGIONS + 1];
    const u32 region_len = (u32)(b.sub_cap / STS_SUB_REGIONS);
    const bool small = ctl->sub_count <= b.sub_cap && ld_agent(&b.sub_cnt[STS_SUB_REGIONS * 32]) == 0u;
    if (t < 64) { // one wave scans the region counts
        static_assert(STS_SUB_REGIONS == 64, "one lane per region");
        const u32 c0 = ld_agent(&b.sub_cnt[t * 32]);
        const u32 c = c0 < region_len ? c0 : region_len;
        const u32 inc = (u32)wave_incl_scan((u64)c);
        s_regpre[t + 1] = inc;
        if (t == 0) s_regpre[0] = 0;
    }
    __syncthreads();
    const u64 *src_w = small ? b.sub_w : b.side_w;
    const u64 *src_k = small ? b.sub_key : b.side_key;
    const SideView view = side_view(b, ctl);
    const u64 n = small ? (u64)s_regpre[STS_SUB_REGIONS] : view.flat;
    // physical index of visited entry f (false: an empty slot of the side buffer)
    auto entry = [&](u64 f, u64 &i) -> bool {
        if (small) {
            int lo = 0; // the last region r with pre[r] <= f (then f < pre[r + 1])
#pragma unroll
            for (int step = STS_SUB_REGIONS / 2; step > 0; step >>= 1)
                if (s_regpre[lo + step] <= f) lo += step;
            i = (u64)lo * region_len + (f - s_regpre[lo]);
            return true;
        }
        i = f;
        return side_valid(view, f);
    };
    // body(V) for every visited entry whose V lies under the prefix: FB
    // entries per thread at a time, their loads in flight together (a loop
    // of one entry at a time waits on a load per entry)
    auto each_in_subset = [&](int vshift, u128 vpre, auto body) {
        for (u64 f0 = t; f0 < n; f0 += (u64)FT * FB) {
            u64 w[FB], k[FB], at[FB];
            bool ok[FB];
#pragma unroll
            for (int r = 0; r < FB; ++r) {
                const u64 f = f0 + (u64)FT * r;
                u64 i = 0;
                ok[r] = f < n && entry(f, i);
                at[r] = ok[r] ? i : 0ull; // entry 0 exists: a harmless load
            }
#pragma unroll
            for (int r = 0; r < FB; ++r) {
                w[r] = src_w[at[r]];
                k[r] = src_k[at[r]];
            }
#pragma unroll
            for (int r = 0; r < FB; ++r) {
                const u128 v = rank_key(w[r], k[r]);
                if (ok[r] && (v >> vshift) == vpre) body(v);
            }
        }
    };
    const u64 K = ctl->K;
    const u128 R = make128(ctl->R_lo, ctl->R_hi);
    // the subset copy binned the first of the levels below (the condition
    // under which it copies the subset); the bins are cleared here for the
    // next step, whether or not a level is needed
    bool from_h3 = ctl->sub_count <= b.sub_cap;

    // further levels until the subset is small (a level is a pass over the
    // subset and a block scan; the bitonic sort below costs a barrier per
    // stage, so levels are the cheaper way down)
    while (s_sub.count > STS_FINAL_SORT && s_sub.vshift > 0) {
        const int vshift = s_sub.vshift;
        const int dw = vshift < 11 ? vshift : 11;
        const u128 vpre = s_sub.vpre;
        bool ok;
        if (from_h3) {
            ok = pick_digit<FT>(b.h3, b.h3 + STS_NBIN, b.h3 + 2 * STS_NBIN, true, K, R, dw, &s_sub, s_m, s_c,
                                &s_hit);
            for (int i = t; i < 3 * STS_NBIN; i += FT) st_agent(&b.h3[i], 0ull);
            from_h3 = false;
        } else {
            for (int i = t; i < 3 * STS_NBIN; i += FT) h_cnt[i] = 0;
            __syncthreads();
            each_in_subset(vshift, vpre, [&](const u128 v) {
                const u32 d = (u32)((v >> (vshift - dw)) & (u128)((1u << dw) - 1));
                const u64 mant = mant_of_v(v, e);
                atomicAdd((unsigned long long *)&h_cnt[d], 1ull);
                atomicAdd((unsigned long long *)&h_hi[d], mant >> 26);
                atomicAdd((unsigned long long *)&h_lo[d], mant & ((1ull << 26) - 1));
            });
            __syncthreads();
            ok = pick_digit<FT>(h_cnt, h_hi, h_lo, false, K, R, dw, &s_sub, s_m, s_c, &s_hit);
        }
        if (!ok) {
            if (t == 0) atomicOr(&ctl->flags, STS_F_UNRESOLVED);
            return;
        }
    }
    if (from_h3) // binned, but the subset was small enough already
        for (int i = t; i < 3 * STS_NBIN; i += FT) st_agent(&b.h3[i], 0ull);

    // gather the subset and sort it by V
    const int vshift = s_sub.vshift;
    const u128 vpre = s_sub.vpre;
    if (t == 0) s_n = 0;
    __syncthreads();
    each_in_subset(vshift, vpre, [&](const u128 v) {
        const u32 slot = atomicAdd(&s_n, 1u);
        if (slot < STS_SMALL) sv[slot] = v;
    });
    __syncthreads();
    const u32 m = s_n;
    if (m == 0 || m > STS_SMALL) {
        if (t == 0) atomicOr(&ctl->flags, STS_F_UNRESOLVED);
        return;
    }
    u32 P = 1;
    while (P < m) P <<= 1;
    for (u32 i = m + t; i < P; i += FT) sv[i] = ~(u128)0;
    __syncthreads();
    for (u32 k = 2; k <= P; k <<= 1) {
        for (u32 j = k >> 1; j > 0; j >>= 1) {
            for (u32 i = t; i < P; i += FT) {
                const u32 ixj = i ^ j;
                if (ixj > i) {
                    const u128 a = sv[i], c = sv[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > c) == up) {
                        sv[i] = c;
                        sv[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }

    // exact prefix in rank order: thread t owns elements 4t .. 4t+3
    constexpr int PER = STS_SMALL / FT;
    u128 loc[PER];
    u128 acc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const u32 r = PER * t + k;
        if (r < m) acc += (u128)mant_of_v(sv[r], e);
        loc[k] = acc;
    }
    if (t == 0) s_hit = 0xffffffffu;
    u64 none = 0;
    u128 inc = acc;
    block_scan_cm<FT>(none, inc, s_c, s_m);
    const u128 excl = inc - acc;
    const u64 cb = s_sub.cnt_before;
    const u128 mb = s_sub.mb;
    u32 hit = 0xffffffffu;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const u32 r = PER * t + k;
        if (hit == 0xffffffffu && r < m) {
            const bool hk = K > 0 && cb + r + 1 >= K;
            const bool hp = mb + excl + loc[k] >= R;
            if (hk || hp) hit = r;
        }
    }
    if (hit != 0xffffffffu) atomicMin(&s_hit, hit);
    __syncthreads();
    const u32 first = s_hit;
    if (first == 0xffffffffu) {
        if (t == 0) atomicOr(&ctl->flags, STS_F_UNRESOLVED);
        return;
    }
    if (hit == first) {
        const int k = (int)first - PER * t;
        const u128 v = sv[first];
        const u64 frac = ((1ull << 52) - 1) - (u64)(v >> 64);
        const u128 mk = mb + excl + loc[k];
        Big S;
#pragma unroll
        for (int i = 0; i < STS_NL; ++i) S.l[i] = s_Sx[i];
        big_add_shifted(S, (u64)mk, (u64)(mk >> 64), unit_bit(e));
        const double Sd = big_to_double(S);
        const u64 L = cb + first + 1;
        const int dropped = L < s_ncand;
        ctl->L = L;
        ctl->thr_wbits = ((u64)e << 52) | frac;
        ctl->thr_key = (u64)v;
        ctl->dropped = dropped;
        ctl->S = Sd;
        ctl->scale = dropped ? 1.0 / sqrt(Sd) : 1.0;
        const double frac_kept = Sd / s_W;
        ctl->frac = frac_kept;
        if (dropped) ctl->log10_cum = s_l10 + log10(frac_kept);
    }
}

// ---------------------------------------------------------------------------
// per-tile survivors of the tiled passes, then their exclusive scan
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tile_kept(PassBufs b)
{
    // one wave per tile: a tile's window entries (a few hundred) take one
    // round of loads, and every tile's wave is resident at once
    constexpr int UN = 4;
    DevCtl *ctl = b.ctl;
    const u64 tile = (u64)blockIdx.x * 4 + (threadIdx.x >> 6); // below the tile arrays' length
    // every control load issued before any is used
    const u64 n = *b.n_in;
    const u64 thr_w = ctl->thr_wbits, thr_k = ctl->thr_key;
    const int shift = ctl->side_slab_shift, spl = ctl->side_spt_log2;
    const u64 ntiles = (n + 2047) / 2048;
    if (tile >= ntiles) return; // the whole wave
    // the tile's window entries (one slab, or one per wave of the histogram
    // pass), and its candidates certain before the cut
    const TileSlabs sd = tile_slabs(b.t_side, tile, spl, shift, false, b.side_cap);
    u64 na = 0;
    for (int w = 0; w < (1 << spl); ++w) na += b.t_above[(tile << spl) + (u64)w];
    const u32 ns = sd.n;
    const u32 lane = (u32)sts_lane();
    u32 c = 0;
    for (u32 i0 = 0; i0 < ns; i0 += UN * 64) {
        u64 w[UN], k[UN];
#pragma unroll
        for (int r = 0; r < UN; ++r) {
            const u32 j = i0 + (u32)r * 64 + lane;
            const u64 i = j < ns ? slab_at(sd, j) : slab_at(sd, 0);
            w[r] = b.side_w[i];
            k[r] = b.side_key[i];
        }
#pragma unroll
        for (int r = 0; r < UN; ++r) {
            const u32 j = i0 + (u32)r * 64 + lane;
            // ranked at or above the threshold term; the key decides only a tie
            c += (j < ns && (w[r] > thr_w || (w[r] == thr_w && k[r] <= thr_k))) ? 1u : 0u;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane == 0) b.t_off[tile] = na + c;
}

__global__ void __launch_bounds__(1024) k_tile_scan(PassBufs b)
{
    constexpr int CH = 8; // tiles per thread per round, loaded before use
    __shared__ u64 s_scratch[16];
    __shared__ u64 s_carry;
    DevCtl *ctl = b.ctl;
    const u64 n = *b.n_in;
    const u64 ntiles = (n + 2047) / 2048;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (u64 c0 = 0; c0 < ntiles; c0 += 1024ull * CH) {
        const u64 lo = c0 + (u64)threadIdx.x * CH;
        u64 v[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) v[k] = lo + k < ntiles ? b.t_off[lo + k] : 0ull;
        u64 sum = 0;
#pragma unroll
        for (int k = 0; k < CH; ++k) sum += v[k];
        u64 total;
        u64 run = block_excl_scan<u64, 1024>(sum, s_scratch, &total) + s_carry;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (lo + k < ntiles) b.t_off[lo + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) s_carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const u64 total = s_carry;
        *b.n_out = total;
        if (total > b.out_cap) atomicOr(&ctl->flags, STS_F_OUT_OVERFLOW);
    }
}

__global__ void k_init_state(u64 *keys, double2 *amps64, float2 *amps32, u64 *n_out)
{
    keys[0] = 0;
    if (amps64) amps64[0] = make_double2(1.0, 0.0);
    if (amps32) amps32[0] = make_float2(1.0f, 0.0f);
    *n_out = 1;
}

__global__ void k_set_n(u64 *n_out, u64 n) { *n_out = n; }

// the gate's description into device memory, where every kernel of its step
// reads it (a captured step is replayed for another gate by changing this
// one launch's argument)
__global__ void __launch_bounds__(64) k_set_gate(GateArg g, GateArg *dst)
{
    static_assert(sizeof(GateArg) % sizeof(u32) == 0, "GateArg is a whole number of words");
    const u32 *src = reinterpret_cast<const u32 *>(&g);
    u32 *d = reinterpret_cast<u32 *>(dst);
    for (u32 i = threadIdx.x; i < sizeof(GateArg) / sizeof(u32); i += 64) d[i] = src[i];
}

// zero n words (a kernel rather than a memset, so the work can sit in a
// captured graph)
__global__ void __launch_bounds__(256) k_fill_zero(u64 *p, u64 n)
{
    for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256) p[i] = 0;
}

// a fresh control block: the rule, nothing cut yet, n_in terms in buffer 0
__global__ void __launch_bounds__(64) k_ctl_begin(DevCtl *ctl, u64 K, double p, u64 n_in)
{
    u64 *w = reinterpret_cast<u64 *>(ctl);
    constexpr u64 words = sizeof(DevCtl) / sizeof(u64);
    static_assert(sizeof(DevCtl) % sizeof(u64) == 0, "DevCtl is a whole number of words");
    for (u64 i = threadIdx.x; i < words; i += 64) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->K = K;
        ctl->p = p;
        ctl->scale = 1.0;
        ctl->frac = 1.0;
        ctl->e_pred = -1;
        ctl->cnt[0] = n_in;
    }
}

// copy the cnt[slot] terms of (keys, amps) to the caller's arrays (at most
// out_cap), their count to *n_out and, if stats is set, W and the kept
// fraction to stats[0..1]
__global__ void __launch_bounds__(256) k_terms_out(const u64 *keys, const void *amps, int amp_bytes,
                                                   const DevCtl *ctl, int slot, u64 *keys_out, void *amps_out,
                                                   u64 out_cap, u64 *n_out, double *stats)
{
    const u64 n0 = ctl->cnt[slot];
    const u64 n = n0 < out_cap ? n0 : out_cap;
    for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += (u64)gridDim.x * 256) {
        keys_out[i] = keys[i];
        if (amp_bytes == 16) reinterpret_cast<double2 *>(amps_out)[i] = reinterpret_cast<const double2 *>(amps)[i];
        else reinterpret_cast<float2 *>(amps_out)[i] = reinterpret_cast<const float2 *>(amps)[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *n_out = n;
        if (stats) {
            stats[0] = ctl->W;
            stats[1] = ctl->frac;
        }
    }
}

} // namespace

hipError_t launch_pick1(const PassBufs &b, int groups, int peak_only, int predicted, hipStream_t s)
{
    hipLaunchKernelGGL(k_pick1, dim3(1), dim3(256), 0, s, b, groups, peak_only, predicted);
    return hipGetLastError();
}

hipError_t launch_side_hist(const PassBufs &b, u64 *h2, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_side_hist, dim3(grid), dim3(256), 0, s, b, h2);
    return hipGetLastError();
}

hipError_t launch_side_extract(const PassBufs &b, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_side_extract, dim3(grid), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_tile_kept(const PassBufs &b, int tiles, hipStream_t s)
{
    hipLaunchKernelGGL(k_tile_kept, dim3((tiles + 3) / 4), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_tile_scan(const PassBufs &b, u64 ntiles_bound, hipStream_t s)
{
    (void)ntiles_bound;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_final(const PassBufs &b, hipStream_t s)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(FT), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_init_state(int prec, u64 *keys, void *amps, u64 *n_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, keys, prec == 0 ? (double2 *)amps : nullptr,
                       prec == 0 ? nullptr : (float2 *)amps, n_out);
    return hipGetLastError();
}

hipError_t launch_set_gate(const GateArg &g, GateArg *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_gate, dim3(1), dim3(64), 0, s, g, dst);
    return hipGetLastError();
}

const void *set_gate_kernel() { return reinterpret_cast<const void *>(&k_set_gate); }

hipError_t launch_set_n(u64 *n_out, u64 n, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_n, dim3(1), dim3(1), 0, s, n_out, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero(u64 *p, u64 n, hipStream_t s)
{
    const u64 blocks = std::min<u64>((n + 255) / 256, 1024);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_ctl_begin(DevCtl *ctl, u64 K, double p, u64 n_in, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_begin, dim3(1), dim3(64), 0, s, ctl, K, p, n_in);
    return hipGetLastError();
}

hipError_t launch_terms_out(const u64 *keys, const void *amps, int amp_bytes, const DevCtl *ctl, int slot,
                            u64 *keys_out, void *amps_out, u64 out_cap, u64 *n_out, double *stats, hipStream_t s)
{
    const u64 blocks = std::max<u64>(std::min<u64>((out_cap + 255) / 256, 1024), 1);
    hipLaunchKernelGGL(k_terms_out, dim3((unsigned)blocks), dim3(256), 0, s, keys, amps, amp_bytes, ctl, slot,
                       keys_out, amps_out, out_cap, n_out, stats);
    return hipGetLastError();
}
