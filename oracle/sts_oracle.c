/*
 * sts_oracle.c - plain C FP64 oracle for the sparse, truncated state vector.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never does.
 * It shares no code, header or helper with the HIP library.
 *
 * It computes exactly what oracle/dict_oracle.py computes (and is checked
 * against it bit for bit), in plain C so that it reaches sizes the Python
 * oracle cannot. It is deliberately simple: grouping is done by sorting
 * (rest-of-key, local index) records with qsort, ranking by sorting all terms
 * with qsort, and probability masses are summed exactly in a wide integer.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fused multiply-add, so
 * every product and sum is rounded once, as in IEEE binary64 arithmetic).
 *
 * Operations and the passages they follow:
 *   orc_apply     - Eq. (3) generalised to m qubits (Sec. IV.A): each present
 *                   amplitude of a group multiplies the column of U picked by
 *                   its local bit pattern; the new key is the rest of the key
 *                   with the output pattern deposited on the gate's bits;
 *                   contributions to one new key are summed (segmented sum).
 *   orc_truncate  - Sec. III and Sec. IV.B: sort by decreasing |a|^2 (ties by
 *                   ascending key), keep the shortest prefix reaching p of the
 *                   mass (p-mass) and at most K terms (top-k), renormalise.
 *   orc_peak      - the most probable key (Sec. I, Sec. V).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* exact non-negative sums of doubles: an integer count of 2^-1074 units     */
/* ------------------------------------------------------------------------ */

#define NL 24 /* 64-bit limbs; values < 2^(64*NL - 1074) */

typedef struct { uint64_t l[NL]; } big;

static void big_zero(big *a) { memset(a, 0, sizeof(*a)); }

static void big_add_at(big *a, uint64_t v, int limb, int off)
{
    /* a += v * 2^(64*limb + off) */
    unsigned __int128 lo = (unsigned __int128)v << off;
    uint64_t parts[3];
    parts[0] = (uint64_t)lo;
    parts[1] = (uint64_t)(lo >> 64);
    parts[2] = 0;
    unsigned carry = 0;
    for (int i = limb; i < NL; ++i) {
        uint64_t add = (i - limb < 3) ? parts[i - limb] : 0;
        uint64_t s = a->l[i] + add;
        unsigned c1 = s < add;
        uint64_t s2 = s + carry;
        unsigned c2 = s2 < s;
        a->l[i] = s2;
        carry = c1 + c2;
        if (i - limb >= 2 && carry == 0) break;
    }
}

/* add a non-negative finite double exactly */
static void big_add_double(big *a, double w)
{
    uint64_t bits;
    memcpy(&bits, &w, 8);
    uint64_t e = (bits >> 52) & 0x7ff;
    uint64_t f = bits & ((1ull << 52) - 1);
    uint64_t mant;
    int shift; /* value = mant * 2^(shift - 1074) */
    if (e == 0) { mant = f; shift = 0; }
    else { mant = f | (1ull << 52); shift = (int)e - 1; }
    if (mant == 0) return;
    if (shift / 64 + 2 >= NL) abort(); /* weight far beyond any normalised state */
    big_add_at(a, mant, shift / 64, shift % 64);
}

static void big_add(big *a, const big *b)
{
    unsigned carry = 0;
    for (int i = 0; i < NL; ++i) {
        uint64_t s = a->l[i] + b->l[i];
        unsigned c1 = s < b->l[i];
        uint64_t s2 = s + carry;
        unsigned c2 = s2 < s;
        a->l[i] = s2;
        carry = c1 + c2;
    }
}

static int big_cmp(const big *a, const big *b)
{
    for (int i = NL - 1; i >= 0; --i) {
        if (a->l[i] != b->l[i]) return a->l[i] < b->l[i] ? -1 : 1;
    }
    return 0;
}

/* r = ceil(a * m / 2^s) for a 64-bit multiplier m (a*m must fit in NL limbs) */
static void big_mul_shr_ceil(big *r, const big *a, uint64_t m, int s)
{
    big prod;
    unsigned __int128 carry = 0;
    for (int i = 0; i < NL; ++i) {
        unsigned __int128 t = (unsigned __int128)a->l[i] * m + carry;
        prod.l[i] = (uint64_t)t;
        carry = t >> 64;
    }
    /* sticky: any bit below position s set? */
    int any = 0;
    int wl = s / 64, wb = s % 64;
    for (int i = 0; i < wl && i < NL; ++i) any |= prod.l[i] != 0;
    if (wl < NL && wb) any |= (prod.l[wl] & ((1ull << wb) - 1)) != 0;
    big_zero(r);
    for (int i = 0; i < NL; ++i) {
        int src = i + wl;
        if (src >= NL) break;
        uint64_t v = prod.l[src] >> wb;
        if (wb && src + 1 < NL) v |= prod.l[src + 1] << (64 - wb);
        r->l[i] = v;
    }
    if (any) big_add_at(r, 1, 0, 0);
}

static int big_top_bit(const big *a)
{
    for (int i = NL - 1; i >= 0; --i)
        if (a->l[i]) return i * 64 + 63 - __builtin_clzll(a->l[i]);
    return -1;
}

static int big_bit(const big *a, int pos)
{
    if (pos < 0) return 0;
    return (int)((a->l[pos / 64] >> (pos % 64)) & 1);
}

static int big_any_below(const big *a, int pos)
{
    /* any bit strictly below pos set? */
    if (pos <= 0) return 0;
    int wl = pos / 64, wb = pos % 64;
    for (int i = 0; i < wl; ++i) if (a->l[i]) return 1;
    if (wb && (a->l[wl] & ((1ull << wb) - 1))) return 1;
    return 0;
}

/* the double nearest to a (round half to even) */
static double big_to_double(const big *a)
{
    int h = big_top_bit(a);
    if (h < 0) return 0.0;
    if (h < 53) {
        /* fewer than 54 significant bits at the 2^-1074 grid: exact */
        uint64_t v = a->l[0];
        return ldexp((double)v, -1074);
    }
    int lo = h - 52; /* lowest kept bit */
    uint64_t mant = 0;
    for (int b = h; b >= lo; --b) mant = (mant << 1) | (uint64_t)big_bit(a, b);
    int guard = big_bit(a, lo - 1);
    int sticky = big_any_below(a, lo - 1);
    if (guard && (sticky || (mant & 1))) {
        mant += 1;
        if (mant == (1ull << 53)) { mant >>= 1; lo += 1; }
    }
    return ldexp((double)mant, lo - 1074);
}

/* ------------------------------------------------------------------------ */
/* gate application                                                          */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t rest; uint32_t j; uint32_t pad; uint64_t idx; } member;

static int cmp_member(const void *pa, const void *pb)
{
    const member *a = pa, *b = pb;
    if (a->rest != b->rest) return a->rest < b->rest ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

/*
 * keys[n], amps[2n] (re, im interleaved) -> keys_out, amps_out (capacity cap).
 * U: row-major 2^m x 2^m complex, interleaved (re, im); U[i][j] maps local
 * pattern j to local pattern i. Returns 0, or -1 for bad arguments / duplicate
 * keys, -2 when the output does not fit in cap.
 */
int orc_apply(uint64_t n, const uint64_t *keys, const double *amps, int m,
              const int *qubits, const double *U, uint64_t cap,
              uint64_t *n_out, uint64_t *keys_out, double *amps_out)
{
    if (m < 0 || m > 16) return -1;
    uint64_t mask = 0;
    for (int t = 0; t < m; ++t) {
        if (qubits[t] < 0 || qubits[t] > 63) return -1;
        if (mask & (1ull << qubits[t])) return -1;
        mask |= 1ull << qubits[t];
    }
    member *mem = (member *)malloc((n ? n : 1) * sizeof(member));
    if (!mem) return -1;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t j = 0;
        for (int t = 0; t < m; ++t) j |= (uint32_t)((keys[i] >> qubits[t]) & 1) << t;
        mem[i].rest = keys[i] & ~mask;
        mem[i].j = j;
        mem[i].pad = 0;
        mem[i].idx = i;
    }
    qsort(mem, n, sizeof(member), cmp_member);
    const uint32_t dim = 1u << m;
    uint64_t out = 0;
    int rc = 0;
    uint64_t g0 = 0;
    while (g0 < n) {
        uint64_t g1 = g0 + 1;
        while (g1 < n && mem[g1].rest == mem[g0].rest) {
            if (mem[g1].j == mem[g1 - 1].j) { rc = -1; goto done; } /* duplicate key */
            ++g1;
        }
        for (uint32_t i = 0; i < dim; ++i) {
            double acc_r = 0.0, acc_i = 0.0;
            for (uint64_t g = g0; g < g1; ++g) { /* ascending j */
                const double vr = amps[2 * mem[g].idx], vi = amps[2 * mem[g].idx + 1];
                const double ur = U[2 * ((uint64_t)i * dim + mem[g].j)];
                const double ui = U[2 * ((uint64_t)i * dim + mem[g].j) + 1];
                const double tr = ur * vr - ui * vi;
                const double ti = ur * vi + ui * vr;
                acc_r = acc_r + tr;
                acc_i = acc_i + ti;
            }
            if (acc_r != 0.0 || acc_i != 0.0) {
                if (out >= cap) { rc = -2; goto done; }
                uint64_t dep = 0;
                for (int t = 0; t < m; ++t) dep |= (uint64_t)((i >> t) & 1) << qubits[t];
                keys_out[out] = mem[g0].rest | dep;
                amps_out[2 * out] = acc_r;
                amps_out[2 * out + 1] = acc_i;
                ++out;
            }
        }
        g0 = g1;
    }
done:
    free(mem);
    *n_out = out;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* truncation and peak                                                       */
/* ------------------------------------------------------------------------ */

typedef struct { double w; uint64_t key; uint64_t idx; } ritem;

static int cmp_rank(const void *pa, const void *pb)
{
    const ritem *a = pa, *b = pb;
    if (a->w != b->w) return a->w > b->w ? -1 : 1; /* weight descending */
    if (a->key != b->key) return a->key < b->key ? -1 : 1; /* key ascending */
    return 0;
}

static ritem *rank_terms(uint64_t n, const uint64_t *keys, const double *amps)
{
    ritem *it = (ritem *)malloc((n ? n : 1) * sizeof(ritem));
    if (!it) return NULL;
    for (uint64_t i = 0; i < n; ++i) {
        const double re = amps[2 * i], im = amps[2 * i + 1];
        it[i].w = re * re + im * im;
        it[i].key = keys[i];
        it[i].idx = i;
    }
    qsort(it, n, sizeof(ritem), cmp_rank);
    return it;
}

/*
 * In place: on return keys/amps hold the kept terms (in rank order when
 * something was dropped, untouched otherwise). K = 0 turns top-k off;
 * p <= 0 or p >= 1 turns p-mass off. Outputs: n_out, W (correctly rounded
 * total weight), S (correctly rounded kept weight), frac = S / W, dropped.
 */
int orc_truncate(uint64_t n, uint64_t *keys, double *amps, uint64_t K, double p,
                 uint64_t *n_out, double *W_out, double *S_out, double *frac_out,
                 int *dropped_out)
{
    ritem *it = rank_terms(n, keys, amps);
    if (!it) return -1;
    big W;
    big_zero(&W);
    for (uint64_t i = 0; i < n; ++i) big_add_double(&W, it[i].w);
    const double Wd = big_to_double(&W);

    uint64_t L = n;
    if (p > 0.0 && p < 1.0) {
        /* target T = ceil(p * W) in 2^-1074 units; p = pm * 2^(pe - 1075) */
        uint64_t pb;
        memcpy(&pb, &p, 8);
        uint64_t pe = (pb >> 52) & 0x7ff, pf = pb & ((1ull << 52) - 1);
        uint64_t pm = pe ? (pf | (1ull << 52)) : pf;
        int shift = pe ? (int)(1075 - pe) : 1074;
        big T, run;
        big_mul_shr_ceil(&T, &W, pm, shift);
        big_zero(&run);
        for (uint64_t i = 0; i < n; ++i) {
            big_add_double(&run, it[i].w);
            if (big_cmp(&run, &T) >= 0) { L = i + 1; break; }
        }
    }
    if (K > 0 && K < L) L = K;

    if (L >= n) {
        *n_out = n;
        *W_out = Wd;
        *S_out = Wd;
        *frac_out = 1.0;
        *dropped_out = 0;
        free(it);
        return 0;
    }
    big S;
    big_zero(&S);
    for (uint64_t i = 0; i < L; ++i) big_add_double(&S, it[i].w);
    const double Sd = big_to_double(&S);
    const double scale = 1.0 / sqrt(Sd);

    uint64_t *nk = (uint64_t *)malloc(L * sizeof(uint64_t));
    double *na = (double *)malloc(2 * L * sizeof(double));
    if (!nk || !na) { free(it); free(nk); free(na); return -1; }
    for (uint64_t r = 0; r < L; ++r) {
        const uint64_t i = it[r].idx;
        nk[r] = keys[i];
        na[2 * r] = amps[2 * i] * scale;
        na[2 * r + 1] = amps[2 * i + 1] * scale;
    }
    memcpy(keys, nk, L * sizeof(uint64_t));
    memcpy(amps, na, 2 * L * sizeof(double));
    free(nk);
    free(na);
    free(it);
    *n_out = L;
    *W_out = Wd;
    *S_out = Sd;
    *frac_out = Sd / Wd;
    *dropped_out = 1;
    return 0;
}

/* most probable key (ties to the smaller key), prob = w / (sum of w) */
int orc_peak(uint64_t n, const uint64_t *keys, const double *amps, uint64_t *key, double *prob)
{
    if (n == 0) return -1;
    big W;
    big_zero(&W);
    uint64_t best = 0;
    double bw = -1.0;
    for (uint64_t i = 0; i < n; ++i) {
        const double re = amps[2 * i], im = amps[2 * i + 1];
        const double w = re * re + im * im;
        big_add_double(&W, w);
        if (w > bw || (w == bw && keys[i] < keys[best])) { bw = w; best = i; }
    }
    *key = keys[best];
    *prob = bw / big_to_double(&W);
    return 0;
}

/* exact sum of weights, correctly rounded (exported for the tests) */
double orc_weight_sum(uint64_t n, const double *amps)
{
    big W;
    big_zero(&W);
    for (uint64_t i = 0; i < n; ++i) {
        const double re = amps[2 * i], im = amps[2 * i + 1];
        big_add_double(&W, re * re + im * im);
    }
    return big_to_double(&W);
}

/* correctly rounded sum of arbitrary non-negative doubles (for the tests) */
double orc_fsum_nonneg(uint64_t n, const double *x)
{
    big W;
    big_zero(&W);
    for (uint64_t i = 0; i < n; ++i) big_add_double(&W, x[i]);
    return big_to_double(&W);
}

/* ------------------------------------------------------------------------ */
/* parallel twin (OpenMP)                                                    */
/*                                                                          */
/* The same two operations with the work split over host threads, for the  */
/* sizes where the plain functions above take minutes. Gate application    */
/* spreads the terms over buckets by a hash of their rest-of-key, so every */
/* group lies in one bucket, and treats each bucket exactly as orc_apply   */
/* treats the whole state. Truncation sorts chunks in parallel and merges  */
/* them into the same total order (weight descending, key ascending; keys  */
/* are unique, so the order is unique), and splits every exact sum into    */
/* partial integer sums, which add up to the same integer. The results     */
/* therefore equal those of orc_apply / orc_truncate bit for bit; only the */
/* order of the terms after a gate without truncation differs (it is       */
/* unspecified there). The tests check both against each other.            */
/* ------------------------------------------------------------------------ */
#include <omp.h>

static uint32_t mt_bucket(uint64_t rest, uint32_t nb)
{
    /* Fibonacci hashing: the top 32 bits of rest * 2^64/phi, reduced */
    const uint64_t h = rest * 0x9e3779b97f4a7c15ull;
    return (uint32_t)((h >> 32) % nb);
}

int orc_apply_mt(uint64_t n, const uint64_t *keys, const double *amps, int m,
                 const int *qubits, const double *U, uint64_t cap,
                 uint64_t *n_out, uint64_t *keys_out, double *amps_out, int threads)
{
    if (m < 0 || m > 8) return -1;
    if (threads < 1) threads = 1;
    uint64_t mask = 0;
    for (int t = 0; t < m; ++t) {
        if (qubits[t] < 0 || qubits[t] > 63) return -1;
        if (mask & (1ull << qubits[t])) return -1;
        mask |= 1ull << qubits[t];
    }
    const int C = threads;                 /* input chunks */
    const uint32_t NB = 256u * (uint32_t)threads; /* buckets */
    const uint32_t dim = 1u << m;
    member *mem = (member *)malloc((n ? n : 1) * sizeof(member));
    member *srt = (member *)malloc((n ? n : 1) * sizeof(member));
    uint32_t *bid = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t *cnt = (uint64_t *)calloc((size_t)C * NB, sizeof(uint64_t));
    uint64_t *bstart = (uint64_t *)malloc(((size_t)NB + 1) * sizeof(uint64_t));
    uint64_t *bout = (uint64_t *)calloc(NB, sizeof(uint64_t));
    uint64_t *tk = (uint64_t *)malloc(((n ? n : 1) << m) * sizeof(uint64_t));
    double *ta = (double *)malloc(((n ? n : 1) << m) * 2 * sizeof(double));
    int rc = 0;
    if (!mem || !srt || !bid || !cnt || !bstart || !bout || !tk || !ta) { rc = -1; goto out; }

    /* members, bucket ids and per-chunk bucket counts */
#pragma omp parallel for num_threads(threads) schedule(static, 1)
    for (int c = 0; c < C; ++c) {
        const uint64_t lo = n * (uint64_t)c / C, hi = n * (uint64_t)(c + 1) / C;
        for (uint64_t i = lo; i < hi; ++i) {
            uint32_t j = 0;
            for (int t = 0; t < m; ++t) j |= (uint32_t)((keys[i] >> qubits[t]) & 1) << t;
            mem[i].rest = keys[i] & ~mask;
            mem[i].j = j;
            mem[i].pad = 0;
            mem[i].idx = i;
            bid[i] = mt_bucket(mem[i].rest, NB);
            cnt[(size_t)c * NB + bid[i]] += 1;
        }
    }
    /* bucket-major offsets; within a bucket, chunk order */
    {
        uint64_t run = 0;
        for (uint32_t b = 0; b < NB; ++b) {
            bstart[b] = run;
            for (int c = 0; c < C; ++c) {
                const uint64_t v = cnt[(size_t)c * NB + b];
                cnt[(size_t)c * NB + b] = run;
                run += v;
            }
        }
        bstart[NB] = run;
    }
#pragma omp parallel for num_threads(threads) schedule(static, 1)
    for (int c = 0; c < C; ++c) {
        const uint64_t lo = n * (uint64_t)c / C, hi = n * (uint64_t)(c + 1) / C;
        for (uint64_t i = lo; i < hi; ++i) srt[cnt[(size_t)c * NB + bid[i]]++] = mem[i];
    }
    /* every bucket as orc_apply treats a whole state; its outputs go to a
     * region of 2^m slots per member */
#pragma omp parallel for num_threads(threads) schedule(dynamic, 16) reduction(min : rc)
    for (uint32_t b = 0; b < NB; ++b) {
        const uint64_t b0 = bstart[b], b1 = bstart[b + 1];
        member *g = srt + b0;
        const uint64_t gn = b1 - b0;
        qsort(g, gn, sizeof(member), cmp_member);
        uint64_t o = b0 << m;
        uint64_t g0 = 0;
        while (g0 < gn) {
            uint64_t g1 = g0 + 1;
            while (g1 < gn && g[g1].rest == g[g0].rest) {
                if (g[g1].j == g[g1 - 1].j) rc = -1; /* duplicate key */
                ++g1;
            }
            for (uint32_t i = 0; i < dim; ++i) {
                double acc_r = 0.0, acc_i = 0.0;
                for (uint64_t q = g0; q < g1; ++q) { /* ascending j */
                    const double vr = amps[2 * g[q].idx], vi = amps[2 * g[q].idx + 1];
                    const double ur = U[2 * ((uint64_t)i * dim + g[q].j)];
                    const double ui = U[2 * ((uint64_t)i * dim + g[q].j) + 1];
                    const double tr = ur * vr - ui * vi;
                    const double ti = ur * vi + ui * vr;
                    acc_r = acc_r + tr;
                    acc_i = acc_i + ti;
                }
                if (acc_r != 0.0 || acc_i != 0.0) {
                    uint64_t dep = 0;
                    for (int t = 0; t < m; ++t) dep |= (uint64_t)((i >> t) & 1) << qubits[t];
                    tk[o] = g[g0].rest | dep;
                    ta[2 * o] = acc_r;
                    ta[2 * o + 1] = acc_i;
                    ++o;
                }
            }
            g0 = g1;
        }
        bout[b] = o - (b0 << m);
    }
    if (rc != 0) goto out;
    {
        uint64_t total = 0;
        for (uint32_t b = 0; b < NB; ++b) {
            const uint64_t v = bout[b];
            bout[b] = total;
            total += v;
        }
        if (total > cap) { rc = -2; goto out; }
#pragma omp parallel for num_threads(threads) schedule(dynamic, 64)
        for (uint32_t b = 0; b < NB; ++b) {
            const uint64_t src = bstart[b] << m;
            const uint64_t len = (b + 1 < NB ? bout[b + 1] : total) - bout[b];
            memcpy(keys_out + bout[b], tk + src, len * sizeof(uint64_t));
            memcpy(amps_out + 2 * bout[b], ta + 2 * src, len * 2 * sizeof(double));
        }
        *n_out = total;
    }
out:
    free(mem); free(srt); free(bid); free(cnt); free(bstart); free(bout); free(tk); free(ta);
    if (rc != 0) *n_out = 0;
    return rc;
}

/* merge the sorted runs a[s1, s1 + n1) and a[s2, s2 + n2) into d[s1, ...),
 * keeping only the first `limit` terms of the merged order; returns its length */
static uint64_t merge_runs(const ritem *a, ritem *d, uint64_t s1, uint64_t n1, uint64_t s2, uint64_t n2,
                           uint64_t limit)
{
    uint64_t i = s1, j = s2, o = s1;
    const uint64_t e1 = s1 + n1, e2 = s2 + n2, eo = s1 + limit;
    while (o < eo && i < e1 && j < e2) d[o++] = cmp_rank(&a[j], &a[i]) < 0 ? a[j++] : a[i++];
    while (o < eo && i < e1) d[o++] = a[i++];
    while (o < eo && j < e2) d[o++] = a[j++];
    return o - s1;
}

int orc_truncate_mt(uint64_t n, uint64_t *keys, double *amps, uint64_t K, double p,
                    uint64_t *n_out, double *W_out, double *S_out, double *frac_out,
                    int *dropped_out, int threads)
{
    if (threads < 1) threads = 1;
    const int C = threads;
    /* with top-k on, only the first K of the ranked list can be kept, and
     * the first K of a union of sorted runs lie in the first K of each run */
    const uint64_t need = (K > 0 && K < n) ? K : n;
    ritem *it = (ritem *)malloc((n ? n : 1) * sizeof(ritem));
    ritem *buf = (ritem *)malloc((n ? n : 1) * sizeof(ritem));
    big *part = (big *)malloc((size_t)C * sizeof(big));
    uint64_t *rs = (uint64_t *)malloc(((size_t)C + 1) * sizeof(uint64_t)); /* run starts */
    uint64_t *rl = (uint64_t *)malloc(((size_t)C + 1) * sizeof(uint64_t)); /* run lengths */
    if (!it || !buf || !part || !rs || !rl) { free(it); free(buf); free(part); free(rs); free(rl); return -1; }
    /* weights, chunk sorts and exact partial totals */
#pragma omp parallel for num_threads(threads) schedule(static, 1)
    for (int c = 0; c < C; ++c) {
        const uint64_t lo = n * (uint64_t)c / C, hi = n * (uint64_t)(c + 1) / C;
        big_zero(&part[c]);
        for (uint64_t i = lo; i < hi; ++i) {
            const double re = amps[2 * i], im = amps[2 * i + 1];
            it[i].w = re * re + im * im;
            it[i].key = keys[i];
            it[i].idx = i;
            big_add_double(&part[c], it[i].w);
        }
        qsort(it + lo, hi - lo, sizeof(ritem), cmp_rank);
        rs[c] = lo;
        rl[c] = hi - lo;
    }
    big W;
    big_zero(&W);
    for (int c = 0; c < C; ++c) big_add(&W, &part[c]);
    const double Wd = big_to_double(&W);
    /* pairwise merge rounds; run c absorbs run c + w */
    for (int w = 1; w < C; w *= 2) {
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
        for (int c = 0; c < C; c += 2 * w) {
            const uint64_t n2 = c + w < C ? rl[c + w] : 0;
            const uint64_t s2 = c + w < C ? rs[c + w] : rs[c];
            const uint64_t lim = rl[c] + n2 < need ? rl[c] + n2 : need;
            rl[c] = merge_runs(it, buf, rs[c], rl[c], s2, n2, lim);
        }
        ritem *t = it; it = buf; buf = t;
    }
    const uint64_t nr = rl[0]; /* the first `need` terms in rank order, from it[0] */

    uint64_t L = n;
    if (p > 0.0 && p < 1.0) {
        uint64_t pb;
        memcpy(&pb, &p, 8);
        uint64_t pe = (pb >> 52) & 0x7ff, pf = pb & ((1ull << 52) - 1);
        uint64_t pm = pe ? (pf | (1ull << 52)) : pf;
        int shift = pe ? (int)(1075 - pe) : 1074;
        big T, run;
        big_mul_shr_ceil(&T, &W, pm, shift);
        /* exact masses of contiguous ranges of the ranked list; the first
         * range whose inclusive prefix reaches T holds the cut */
#pragma omp parallel for num_threads(threads) schedule(static, 1)
        for (int c = 0; c < C; ++c) {
            big_zero(&part[c]);
            for (uint64_t i = nr * (uint64_t)c / C; i < nr * (uint64_t)(c + 1) / C; ++i)
                big_add_double(&part[c], it[i].w);
        }
        big_zero(&run);
        for (int c = 0; c < C; ++c) {
            big inc = run;
            big_add(&inc, &part[c]);
            if (big_cmp(&inc, &T) >= 0) {
                for (uint64_t i = nr * (uint64_t)c / C; i < nr * (uint64_t)(c + 1) / C; ++i) {
                    big_add_double(&run, it[i].w);
                    if (big_cmp(&run, &T) >= 0) { L = i + 1; break; }
                }
                break;
            }
            run = inc;
        }
        /* not reached within the first K terms: L_p > K, and top-k decides */
    }
    if (K > 0 && K < L) L = K;

    if (L >= n) {
        *n_out = n;
        *W_out = Wd;
        *S_out = Wd;
        *frac_out = 1.0;
        *dropped_out = 0;
        free(it); free(buf); free(part); free(rs); free(rl);
        return 0;
    }
#pragma omp parallel for num_threads(threads) schedule(static, 1)
    for (int c = 0; c < C; ++c) {
        const uint64_t lo = L * (uint64_t)c / C, hi = L * (uint64_t)(c + 1) / C;
        big_zero(&part[c]);
        for (uint64_t i = lo; i < hi; ++i) big_add_double(&part[c], it[i].w);
    }
    big S;
    big_zero(&S);
    for (int c = 0; c < C; ++c) big_add(&S, &part[c]);
    const double Sd = big_to_double(&S);
    const double scale = 1.0 / sqrt(Sd);

    uint64_t *nk = (uint64_t *)malloc(L * sizeof(uint64_t));
    double *na = (double *)malloc(2 * L * sizeof(double));
    if (!nk || !na) { free(it); free(buf); free(part); free(rs); free(rl); free(nk); free(na); return -1; }
#pragma omp parallel for num_threads(threads) schedule(static)
    for (uint64_t r = 0; r < L; ++r) {
        const uint64_t i = it[r].idx;
        nk[r] = keys[i];
        na[2 * r] = amps[2 * i] * scale;
        na[2 * r + 1] = amps[2 * i + 1] * scale;
    }
    memcpy(keys, nk, L * sizeof(uint64_t));
    memcpy(amps, na, 2 * L * sizeof(double));
    free(nk); free(na); free(it); free(buf); free(part); free(rs); free(rl);
    *n_out = L;
    *W_out = Wd;
    *S_out = Sd;
    *frac_out = Sd / Wd;
    *dropped_out = 1;
    return 0;
}
