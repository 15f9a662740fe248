// kernels.h - launchers for the library's kernels (host side) and the
// argument blocks they take. Everything here is internal to libsts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

// Gate description passed by value to the grouping kernels. For m <= 3 the
// matrix travels in the argument block itself (no device copy per gate);
// for m = 4, 5 it is read from uptr (device, interleaved re/im).
struct GateArg {
    int m;
    int q[STS_MAXM];
    u64 notmask;        // ~(sum of 2^q)
    int hb;             // hash-bucket bits the input was sorted by (m >= 1)
    int pad;
    double ur[64];      // row-major U, real parts (m <= 3)
    double ui[64];      // imaginary parts
    float fr[64];       // the same rounded to FP32 (nearest-even), for complex64 states
    float fi[64];
    u64 dep[8];         // dep[i]: pattern i deposited on the gate's qubits (m <= 3)
    const double *uptr; // m >= 4
    const float *uptr_f; // m >= 4: the same rounded to FP32 (nearest-even)
};

// Device buffers a grouping pass reads and writes.
struct PassBufs {
    const GateArg *gate;  // the gate (device memory: written by k_set_gate per gate)
    const u64 *keys;      // sorted input keys (or the state, m = 0)
    const void *amps;     // sorted input amplitudes
    const u64 *n_in;      // number of input terms (device)
    u64 *n_out;           // number of terms written to out_keys/out_amps (device)
    DevCtl *ctl;
    // level-1 histogram (per exponent field) and per-workgroup best term
    u64 *h1;              // [3][STS_NBIN]: count, mantissa>>26, mantissa & (2^26-1)
    u64 *h2w;             // the same for level 2 of a sampled window (histogram pass)
    u64 *h3;              // the same for the next level of the level-2 subset (the subset copy)
    u64 *best;            // [2][max groups]: (wbits | 2^63), key
    // compaction targets
    u64 *side_key;        // side buffer: candidates of the exponent holding the cut
    u64 *side_w;
    void *side_amp;       // their amplitudes (histogram pass with `copy`)
    u64 side_cap;
    u64 *sub_key;         // the level-2 subset of the side buffer, in STS_SUB_REGIONS
    u64 *sub_w;           // regions of sub_cap / STS_SUB_REGIONS entries
    u64 sub_cap;
    u32 *sub_cnt;         // per region its fill count, 32 words (a cache line) apart; then an
                          // overflow word at STS_SUB_REGIONS * 32
    u64 *out_keys;        // new state
    void *out_amps;
    u64 out_cap;
    u32 *t_above;         // per slab: survivors certain before the cut (tiled passes)
    u32 *t_side;          // per slab: side-buffer entries in it
    u64 *t_off;           // per tile: output offset of its survivors
    u64 *look;            // look-back words, one per tile
    u32 *tile_ctr;
    u32 epoch;            // tags look-back words of this launch
    int materialise;      // 1: keep every candidate, no rescale (no truncation)
    int predict;          // histogram pass: also extract the window of the predicted cut
    int copy;             // histogram pass: also keep every candidate above the window, with
                          // the window's amplitudes, in the tile's slab; emit pass: when the
                          // window held the cut, copy the survivors out of the slabs
    u64 *wpart;           // [6][STS_MAX_GROUPS]: per histogram workgroup, the count of candidates
                          // above the window and the mantissa sums (>> 26, & (2^26-1)) of those in
                          // the window's exponent; then the count and sums of those inside it
    u64 *sbins;           // sampling pass: STS_SW_BANKS x STS_SW_NB counts (u32), as many masses
                          // (float), then 4 totals per bank
};

// The slabs of one tile in the tiled side-buffer layout: 2^spl (1 or 4)
// consecutive slabs of 2^shift entries, slab s holding cnt[s] entries of one
// kind, at its start (window entries) or at its end (entries above the
// window). A tile's entries of that kind are visited through one flat index.
// (Scalar fields rather than arrays, so that the struct stays in registers.)
struct TileSlabs {
    u64 f0, f1, f2, f3; // first entry of each slab's run
    u32 p1, p2, p3, n;  // ends of the first three runs in the flat index; entries in all
};

__device__ __forceinline__ TileSlabs tile_slabs(const u32 *cnt, u64 tile, int spl, int shift, bool at_end, u64 cap)
{
    u64 f[4];
    u32 c[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        c[w] = 0;
        f[w] = 0;
        if (w < (1 << spl)) {
            const u64 sl = (tile << spl) + (u64)w;
            const u64 base = sl << shift, end = base + (1ull << shift);
            u32 k = cnt[sl];
            if (at_end) {
                if (end > cap) k = 0;
                f[w] = end - k;
            } else {
                if (base >= cap) k = 0;
                else if ((u64)k > cap - base) k = (u32)(cap - base);
                f[w] = base;
            }
            c[w] = k;
        }
    }
    TileSlabs t;
    t.f0 = f[0];
    t.f1 = f[1];
    t.f2 = f[2];
    t.f3 = f[3];
    t.p1 = c[0];
    t.p2 = t.p1 + c[1];
    t.p3 = t.p2 + c[2];
    t.n = t.p3 + c[3];
    return t;
}

// physical index of a tile's j-th entry (j < n)
__device__ __forceinline__ u64 slab_at(const TileSlabs &t, u32 j)
{
    if (j < t.p1) return t.f0 + j;
    if (j < t.p2) return t.f1 + (j - t.p1);
    if (j < t.p3) return t.f2 + (j - t.p2);
    return t.f3 + (j - t.p3);
}

// launch helpers (return hipError_t of the launch)
// grouping-sort shapes (digit bits x keys per thread): 8x16 is the default
#define STS_RADIX_8x16 0   // 8-bit digits, 4096-key tiles
#define STS_RADIX_8x8 1    // 8-bit digits, 2048-key tiles
#define STS_RADIX_11x16 2  // 11-bit digits, 4096-key tiles
#define STS_RADIX_11x8 3   // 11-bit digits, 2048-key tiles
#define STS_RADIX_SHAPES 4
inline int sts_radix_bits(int shape) { return shape >= STS_RADIX_11x16 ? 11 : 8; }
inline u64 sts_radix_tile(int shape) { return (shape & 1) ? 2048ull : 4096ull; }

// one step of a grouping-sort pass: what = 0 digit counts per tile, 1 their
// scan (one workgroup per digit), 2 the scatter
hipError_t launch_radix(int what, int shape, int prec, const u64 *kin, const void *ain, u64 *kout, void *aout,
                        const u64 *n_in, u64 *n_out, const u64 *notmask, int shift, u32 *counts, u64 *prefix,
                        u64 *totals, u64 tiles_cap, int tiles, hipStream_t s);

hipError_t launch_group_hist(int prec, const GateArg &g, const PassBufs &b, int grid, bool tiled, hipStream_t s);
int group_hist_capacity(int prec, int m, bool tiled); // resident workgroups of the histogram pass
hipError_t launch_group_compact(int prec, int kind, const GateArg &g, const PassBufs &b, int tiles,
                                hipStream_t s);
hipError_t launch_pick1(const PassBufs &b, int groups, int peak_only, int predicted, hipStream_t s);
hipError_t launch_side_hist(const PassBufs &b, u64 *h2, int grid, hipStream_t s);
hipError_t launch_side_extract(const PassBufs &b, int grid, hipStream_t s);
hipError_t launch_tile_kept(const PassBufs &b, int tiles, hipStream_t s);
hipError_t launch_tile_scan(const PassBufs &b, u64 ntiles_bound, hipStream_t s);
hipError_t launch_group_extract_tiles(int prec, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t launch_group_sample(int prec, const GateArg &g, const PassBufs &b, hipStream_t s);
hipError_t launch_group_emit_tiles(int prec, const GateArg &g, const PassBufs &b, int tiles, hipStream_t s);
hipError_t launch_final(const PassBufs &b, hipStream_t s);
hipError_t launch_init_state(int prec, u64 *keys, void *amps, u64 *n_out, hipStream_t s);
hipError_t launch_set_n(u64 *n_out, u64 n, hipStream_t s);
hipError_t launch_set_gate(const GateArg &g, GateArg *dst, hipStream_t s);
const void *set_gate_kernel(); // the kernel launch_set_gate launches (to find its node in a captured graph)
hipError_t launch_fill_zero(u64 *p, u64 n, hipStream_t s);
hipError_t launch_ctl_begin(DevCtl *ctl, u64 K, double p, u64 n_in, hipStream_t s);
hipError_t launch_terms_out(const u64 *keys, const void *amps, int amp_bytes, const DevCtl *ctl, int slot,
                            u64 *keys_out, void *amps_out, u64 out_cap, u64 *n_out, double *stats, hipStream_t s);

// workgroups to launch for a compaction pass over n terms with an m-qubit
// gate: m <= 3 uses LDS tiles of 2048 terms, larger
// gates one tile of STS_GTILE terms per workgroup
inline u64 sts_compact_groups(u64 n, int m)
{
    const u64 per = m <= 3 ? 2048ull : 1024ull;
    const u64 g = (n + per - 1) / per;
    return g ? g : 1;
}

#define STS_KIND_EXTRACT 0
#define STS_KIND_EMIT 1
#define STS_GROUP_ITEMS 4                       // elements per thread in a compaction tile
#define STS_GTILE (STS_WG * STS_GROUP_ITEMS)     // elements per compaction tile
#define STS_MAX_GROUPS 2048                      // workgroups of a histogram pass (best-term slots)
#define STS_SIDE_GROUPS 128
#define STS_SUB_REGIONS 64                        // fill counters of the level-2 subset buffer
#define STS_SUB_CAP (1u << 16)                   // level-2 subset buffer (terms)
#define STS_SW_FB 5                              // fraction bits of a sampling bin
#define STS_SW_EXPS 8                            // exponent fields the sampling bins cover
#define STS_SW_NB (STS_SW_EXPS << STS_SW_FB)     // sampling bins (256)
#define STS_SW_BANKS 16                          // copies of the sampling bins in device memory
#define STS_SAMPLE_TILES 256                     // tiles the sampling pass runs the gate on
#define STS_SAMPLE_SPAN 512                      // inputs of each, from the tile's start
#define STS_SAMPLE_MIN (1ull << 22)              // terms from which a step samples first
