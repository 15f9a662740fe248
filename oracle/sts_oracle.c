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
