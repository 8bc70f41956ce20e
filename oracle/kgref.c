/*
 * kgref -- CPU oracle for communication-free Erdos-Renyi generation
 * (Funke et al., "Communication-free Massively Distributed Graph Generation",
 *  arXiv 1710.07565, Sections 2.1.1, 2.2 and 4).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * definition of what the GPU library computes, bit for bit.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no source with the GPU library and includes none of its headers.
 *
 * What the paper fixes and what is our reading of it:
 *   - G(n,m): a uniform m-subset of the n(n-1) directed slots, or of the
 *     n(n-1)/2 undirected slots (Sec. 2.1.1).  We use the strict upper
 *     triangle (u < v); the paper draws the lower one, the law is the same.
 *   - G(n,p): every slot independently with probability p (Sec. 2.1.1).
 *   - The sample count of a sub-universe is hypergeometric; a recursion tree
 *     over the chunks splits the count, every subtree drawing from its own
 *     pseudorandom stream keyed by the subtree, not by the processor
 *     (Sec. 2.2, Sec. 4.1, Sec. 4.2 quadrant recursion, split l = ceil(P/2)).
 *   - G(n,p) chunk counts are binomial, keyed by the chunk id (Sec. 4.3).
 *   - Below a threshold a sequential sampler draws the chunk's sample
 *     (Sec. 2.2); our threshold is a tile of 2^s slots holding 560..1120
 *     expected samples (1024 whenever the density is a power of two),
 *     itself split by a hypergeometric tree, and the base case draws until
 *     k distinct slots are seen.
 *   - Variates by acceptance-rejection (Sec. 2.2): discrete ratio of
 *     uniforms for the hypergeometric and binomial laws, direct simulation
 *     for small hypergeometric samples, geometric waiting times for
 *     binomials of small mean.  The hash + Mersenne Twister of Sec. 8.1 is
 *     replaced by the Philox4x32-10 counter generator (Salmon et al., SC'11),
 *     whose keyed bijection of the counter plays the role of the hash.
 *
 * Floating point: IEEE binary64 + - * / sqrt only, no FMA contraction
 * (built with -ffp-contract=off), no libm log: log and log1p are written out
 * below so that any other implementation following the same operation order
 * obtains the same bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 3)           */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void kgref_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags: every recursion node, chunk and tile owns one stream
 * (Sec. 2.2: one seed per recursion subtree, independent of the PE). */
enum { TAG_DTREE = 1, TAG_UTREE = 2, TAG_CBIN = 3, TAG_TTREE = 4, TAG_TLEAF = 5, TAG_INST = 6, TAG_SKIP = 7 };

/* A stream is Philox keyed by the seed with counter (a, j, b, tag);
 * j counts 128-bit blocks. */
typedef struct {
    uint32_t key[2];
    uint32_t a, b, tag;
    uint64_t next;      /* index of the next 64-bit draw */
    uint64_t cached_j;  /* block held in buf, or UINT64_MAX */
    uint32_t buf[4];
} stream_t;

static void stream_init(stream_t *s, uint64_t seed, uint32_t a, uint32_t b, uint32_t tag)
{
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    s->a = a; s->b = b; s->tag = tag;
    s->next = 0;
    s->cached_j = UINT64_MAX;
}

static void stream_block(stream_t *s, uint64_t j, uint32_t out[4])
{
    uint32_t ctr[4] = { s->a, (uint32_t)j, s->b, s->tag };
    kgref_philox(ctr, s->key, out);
}

/* 64-bit draw number d lives in block d/2: (w1:w0) for even d, (w3:w2) for odd d. */
static uint64_t stream_u64(stream_t *s)
{
    uint64_t d = s->next++;
    uint64_t j = d >> 1;
    if (j != s->cached_j) { stream_block(s, j, s->buf); s->cached_j = j; }
    if ((d & 1) == 0) return ((uint64_t)s->buf[1] << 32) | s->buf[0];
    return ((uint64_t)s->buf[3] << 32) | s->buf[2];
}

/* Uniform in (0,1) from 64 random bits: the top 52 bits plus one half ulp,
 * exact in binary64, never 0 or 1. */
static double u64_to_unit(uint64_t x)
{
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

/* Integer uniform on [0, R), R >= 1, by masking to the next power of two and
 * rejecting (exact, integer only). */
static uint64_t stream_below(stream_t *s, uint64_t R)
{
    uint64_t mask = 0;
    while (mask < R - 1) mask = (mask << 1) | 1;
    for (;;) {
        uint64_t x = stream_u64(s) & mask;
        if (x < R) return x;
    }
}

/* ------------------------------------------------------------------ */
/* Logarithms from + - * / only                                        */
/* log(1+u) = 2 atanh(s), s = u/(2+u), written as                       */
/*   u - (u^2/2 - s (u^2/2 + R(s^2))),  R(z) = sum_{i>=1} 2 z^i/(2i+1)  */
/* x = 2^e f with f in [sqrt(1/2), sqrt(2)); ln 2 split in a hi part    */
/* with 32 fraction bits (so e*hi is exact) and the rounded remainder.  */
/* ------------------------------------------------------------------ */
static const double LN2_HI = 0x1.62e42fee00000p-1;
static const double LN2_LO = 0x1.a39ef35793c76p-33;

static double atanh_tail(double z)
{
    /* R(z) = z (2/3 + z (2/5 + ... + z (2/23))), eleven terms, Horner. */
    double r = 2.0 / 23.0;
    r = 2.0 / 21.0 + z * r;
    r = 2.0 / 19.0 + z * r;
    r = 2.0 / 17.0 + z * r;
    r = 2.0 / 15.0 + z * r;
    r = 2.0 / 13.0 + z * r;
    r = 2.0 / 11.0 + z * r;
    r = 2.0 / 9.0 + z * r;
    r = 2.0 / 7.0 + z * r;
    r = 2.0 / 5.0 + z * r;
    r = 2.0 / 3.0 + z * r;
    return z * r;
}

double kgref_log(double x)
{
    /* Valid for finite x >= DBL_MIN (the variates never need more). */
    uint64_t bits;
    memcpy(&bits, &x, 8);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    uint64_t mant = bits & 0x000FFFFFFFFFFFFFull;
    /* sqrt(2) = 0x3FF6A09E667F3BCD: mantissa fields above it go to [1/sqrt2, 1). */
    uint64_t fbits;
    if (mant > 0x6A09E667F3BCDull) { fbits = mant | (1022ull << 52); e += 1; }
    else                           { fbits = mant | (1023ull << 52); }
    double f;
    memcpy(&f, &fbits, 8);
    double u = f - 1.0;
    double s = u / (2.0 + u);
    double z = s * s;
    double R = atanh_tail(z);
    double hfsq = 0.5 * u * u;
    double dk = (double)e;
    return dk * LN2_HI - ((hfsq - (s * (hfsq + R) + dk * LN2_LO)) - u);
}

double kgref_log1p(double x)
{
    if (x > -0.25 && x < 0.25) {
        double s = x / (2.0 + x);
        double z = s * s;
        double R = atanh_tail(z);
        double hfsq = 0.5 * x * x;
        return x - (hfsq - s * (hfsq + R));
    }
    return kgref_log(1.0 + x);
}

/* ------------------------------------------------------------------ */
/* ln k!  -- table for k <= 1024 by forward summation of log, Stirling  */
/* series (three correction terms) for differences above.               */
/* ------------------------------------------------------------------ */
#define LNF_TAB 1024
static double lnf_tab[LNF_TAB + 1];
static int lnf_ready = 0;

static void lnf_init(void)
{
    if (lnf_ready) return;
    double acc = 0.0;
    lnf_tab[0] = 0.0;
    for (int i = 1; i <= LNF_TAB; i++) {
        acc = acc + kgref_log((double)i);
        lnf_tab[i] = acc;
    }
    lnf_ready = 1;
}

/* Stirling correction 1/(12z) - 1/(360 z^3) + 1/(1260 z^5). */
static double stirling_corr(double z)
{
    double r = 1.0 / z;
    double r2 = r * r;
    return r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));
}

/* ln((a+d)!) - ln(a!) for a >= 1024, d >= 1, a + d < 2^64 (above 2^53 the
 * conversions to binary64 round to nearest, even).  With z = a+1:
 * (z - 1/2) log1p(d/z) + d (log(z+d) - 1) + corr(z+d) - corr(z),
 * which never subtracts two large log-factorials. */
static double stirling_diff(uint64_t a, uint64_t d)
{
    double z = (double)(a + 1);
    double zd = (double)(a + d + 1);
    double dd = (double)d;
    double t1 = (z - 0.5) * kgref_log1p(dd / z);
    double t2 = dd * (kgref_log(zd) - 1.0);
    double t3 = stirling_corr(zd) - stirling_corr(z);
    return (t1 + t2) + t3;
}

/* lnf(y) - lnf(x) for 0 <= x, y < 2^64. */
double kgref_lnf_diff(uint64_t x, uint64_t y)
{
    lnf_init();
    if (x == y) return 0.0;
    if (x > y) return -kgref_lnf_diff(y, x);
    if (y <= LNF_TAB) return lnf_tab[y] - lnf_tab[x];
    if (x >= LNF_TAB) return stirling_diff(x, y - x);
    return (lnf_tab[LNF_TAB] - lnf_tab[x]) + stirling_diff(LNF_TAB, y - LNF_TAB);
}

double kgref_lnf(uint64_t k)
{
    return kgref_lnf_diff(0, k);
}

/* ------------------------------------------------------------------ */
/* Hypergeometric and binomial variates (Sec. 2.2: acceptance-rejection */
/* in expected constant time; ratio of uniforms after Kinderman and     */
/* Monahan, with Stadlober's centre and half-width for discrete laws).  */
/* ------------------------------------------------------------------ */
/* 2 sqrt(2/e) and 3 - 2 sqrt(3/e) */
static const double ROU_D1 = 0x1.b72cd3f331398p+0;
static const double ROU_D2 = 0x1.cc3ebd3bc711ap-1;

/* One ratio-of-uniforms proposal per 128-bit block j: U from (w1:w0),
 * V from (w3:w2).  Returns 1 and sets *x on acceptance. */
typedef double (*logratio_fn)(uint64_t x, const void *ctx);

static uint64_t rou_sample(stream_t *s, double a, double h, uint64_t upper,
                           logratio_fn lr, const void *ctx)
{
    double upper_excl = (double)upper + 1.0;
    for (uint64_t j = 0;; j++) {
        uint32_t w[4];
        stream_block(s, j, w);
        double U = u64_to_unit(((uint64_t)w[1] << 32) | w[0]);
        double V = u64_to_unit(((uint64_t)w[3] << 32) | w[2]);
        double t = a + h * (V - 0.5) / U;
        if (!(t >= 0.0) || t >= upper_excl) continue;
        uint64_t X = (uint64_t)floor(t);
        /* above 2^53, upper + 1 rounds in binary64: keep X in range exactly */
        if (X > upper) continue;
        double T = lr(X, ctx);
        if (U * (4.0 - U) - 3.0 <= T) return X;     /* 2 log U <= 4U - U^2 - 3 */
        if (U * (U - T) >= 1.0) continue;            /* 2 log U >  U - 1/U      */
        if (2.0 * kgref_log(U) <= T) return X;
    }
}

typedef struct { uint64_t N, K, k, M; } hyp_ctx;

/* log f(x) - log f(M) for the hypergeometric pmf
 * f(x) = C(K,x) C(N-K,k-x) / C(N,k). */
static double hyp_logratio(uint64_t X, const void *vctx)
{
    const hyp_ctx *c = (const hyp_ctx *)vctx;
    uint64_t N = c->N, K = c->K, k = c->k, M = c->M;
    double T = kgref_lnf_diff(X, M);
    T = T + kgref_lnf_diff(k - X, k - M);
    T = T + kgref_lnf_diff(K - X, K - M);
    T = T + kgref_lnf_diff(N - K - k + X, N - K - k + M);
    return T;
}

/* Number of the k draws (without replacement, from N items) that fall among
 * K marked items; here k <= K <= N/2. */
static uint64_t hyp_core(stream_t *s, uint64_t N, uint64_t K, uint64_t k)
{
    if (k == 0) return 0;
    if (k <= 16) {
        /* Direct simulation: draw i takes one of the N - i remaining items. */
        uint64_t X = 0;
        for (uint64_t i = 0; i < k; i++) {
            uint64_t r = stream_below(s, N - i);
            if (r < K - X) X++;
        }
        return X;
    }
    double Nd = (double)N, Kd = (double)K, kd = (double)k;
    double pp = Kd / Nd;
    double mu = kd * pp;
    double var = (((Nd - kd) * kd) * pp) * (1.0 - pp) / (Nd - 1.0);
    double c = sqrt(var + 0.5);
    double h = ROU_D1 * c + ROU_D2;
    double a = mu + 0.5;
    hyp_ctx ctx;
    ctx.N = N; ctx.K = K; ctx.k = k;
    ctx.M = (uint64_t)(((u128)(k + 1) * (u128)(K + 1)) / (u128)(N + 2));
    return rou_sample(s, a, h, k, hyp_logratio, &ctx);
}

uint64_t kgref_hyp_stream(stream_t *s, uint64_t N, uint64_t K, uint64_t k)
{
    /* Symmetries, in this order: take the complement of the draws if they are
     * more than half of N, the complement of the marked set likewise, then
     * exchange the roles of draws and marked items so that k <= K. */
    uint64_t k1 = k, K1 = K;
    int c1 = 0, c2 = 0;
    if (k1 > N - k1) { k1 = N - k1; c1 = 1; }
    if (K1 > N - K1) { K1 = N - K1; c2 = 1; }
    uint64_t lo = k1 < K1 ? k1 : K1;
    uint64_t hi = k1 < K1 ? K1 : k1;
    uint64_t x = hyp_core(s, N, hi, lo);
    if (c2) x = k1 - x;
    if (c1) x = K - x;
    return x;
}

uint64_t kgref_hyp(uint64_t N, uint64_t K, uint64_t k, uint64_t seed,
                   uint32_t a, uint32_t b, uint32_t tag)
{
    stream_t s;
    stream_init(&s, seed, a, b, tag);
    return kgref_hyp_stream(&s, N, K, k);
}

typedef struct { uint64_t N, M; double lq; } bin_ctx;

/* log f(x) - log f(M) for f(x) = C(N,x) p^x (1-p)^(N-x). */
static double bin_logratio(uint64_t X, const void *vctx)
{
    const bin_ctx *c = (const bin_ctx *)vctx;
    double T = kgref_lnf_diff(X, c->M);
    T = T + kgref_lnf_diff(c->N - X, c->N - c->M);
    T = T + ((double)X - (double)c->M) * c->lq;
    return T;
}

static uint64_t bin_core(stream_t *s, uint64_t N, double p)
{
    /* 0 < p <= 1/2 */
    double Nd = (double)N;
    if (Nd * p < 16.0) {
        /* Waiting times: the gap before the next success is
         * floor(log U / log(1-p)) failures (geometric law). */
        double L = kgref_log1p(-p);
        uint64_t X = 0, pos = 0;
        for (;;) {
            double U = u64_to_unit(stream_u64(s));
            double g = floor(kgref_log(U) / L);
            if (g >= (double)(N - pos)) return X;
            pos += (uint64_t)g + 1;
            X++;
        }
    }
    double q = 1.0 - p;
    double mu = Nd * p;
    double var = mu * q;
    double c = sqrt(var + 0.5);
    double h = ROU_D1 * c + ROU_D2;
    double a = mu + 0.5;
    bin_ctx ctx;
    ctx.N = N;
    ctx.M = (uint64_t)floor((Nd + 1.0) * p);
    ctx.lq = kgref_log(p) - kgref_log1p(-p);
    return rou_sample(s, a, h, N, bin_logratio, &ctx);
}

uint64_t kgref_bin_stream(stream_t *s, uint64_t N, double p)
{
    if (N == 0 || p <= 0.0) return 0;
    if (p >= 1.0) return N;
    if (p > 0.5) return N - bin_core(s, N, 1.0 - p);
    return bin_core(s, N, p);
}

uint64_t kgref_bin(uint64_t N, double p, uint64_t seed, uint32_t a, uint32_t b, uint32_t tag)
{
    stream_t s;
    stream_init(&s, seed, a, b, tag);
    return kgref_bin_stream(&s, N, p);
}

/* ------------------------------------------------------------------ */
/* Instances, chunks and the index space                               */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t n;        /* vertices */
    uint64_t m;        /* edges (G(n,m)) */
    double   p;        /* edge probability (G(n,p)) */
    uint64_t seed;
    uint32_t model;    /* 0 = G(n,m), 1 = G(n,p) */
    uint32_t directed;
    uint32_t P;        /* the paper's P: chunks (directed) or sections (undirected) */
    uint32_t pad;
} kgref_inst;

enum { KGREF_OK = 0, KGREF_EINVAL = -1, KGREF_ERANGE = -2, KGREF_ENOSPC = -3 };

#define LAMBDA 560u   /* expected samples per tile in [560, 1120); 1024 when the density is a power of two */

static uint64_t slots_total(const kgref_inst *I)
{
    if (I->n < 2) return 0;
    return I->directed ? I->n * (I->n - 1) : I->n * (I->n - 1) / 2;
}

uint32_t kgref_tile_exponent(const kgref_inst *I);

int kgref_validate(const kgref_inst *I)
{
    if (I->n < 1 || I->P < 1 || (uint64_t)I->P > I->n) return KGREF_EINVAL;
    if (I->model > 1) return KGREF_EINVAL;
    if (I->n > (1ull << 32)) return KGREF_ERANGE;
    u128 N = I->directed ? (u128)I->n * (I->n - 1) : (u128)I->n * (I->n - 1) / 2;
    if (I->directed ? (I->P > (1u << 31)) : (I->P > (1u << 15))) return KGREF_ERANGE;
    if (I->model == 0 && I->m > (uint64_t)N) return KGREF_EINVAL;
    if (I->model == 1 && !(I->p >= 0.0 && I->p <= 1.0)) return KGREF_EINVAL;
    if (N >= ((u128)1 << 53)) {
        /* Universes of 2^53 slots and more (n <= 2^32, so N < 2^64): slot
         * indices stay 64-bit integers; counts must stay below 2^53 (the
         * variates convert them exactly), the slot counts that are converted
         * round to nearest. */
        if (I->model == 0 && I->m >= ((uint64_t)1 << 53)) return KGREF_ERANGE;
        if (I->model == 1 && (double)N * I->p >= 0x1p52) return KGREF_ERANGE;
    }
    /* every chunk has fewer than 2^31 tiles (the tile index is a 32-bit
     * stream word) */
    uint64_t s = kgref_tile_exponent(I);
    uint64_t rows = (I->n + I->P - 1) / I->P;               /* rows of the largest section */
    u128 Nc = I->directed ? (u128)rows * (I->n - 1) : (u128)rows * rows;
    if ((Nc >> s) >= ((u128)1 << 31)) return KGREF_ERANGE;
    return KGREF_OK;
}

/* Tile exponent: the smallest s in [9, 32] whose tiles of 2^s slots hold at
 * least LAMBDA samples in expectation. */
uint32_t kgref_tile_exponent(const kgref_inst *I)
{
    uint64_t N = slots_total(I);
    for (uint32_t s = 9; s <= 32; s++) {
        if (I->model == 0) {
            if (((u128)I->m << s) >= (u128)LAMBDA * N) return s;
        } else {
            if (ldexp(I->p, (int)s) >= (double)LAMBDA) return s;
        }
    }
    return 32;
}

uint64_t kgref_num_chunks(const kgref_inst *I)
{
    return I->directed ? (uint64_t)I->P : (uint64_t)I->P * (I->P + 1) / 2;
}

/* Section boundary floor(i n / P) (Sec. 4.1 rows, Sec. 4.2 sections). */
static uint64_t bound(const kgref_inst *I, uint64_t i)
{
    return (uint64_t)(((u128)i * I->n) / I->P);
}

/* Undirected chunk (I, J), I <= J, in row-major order over the upper
 * triangle of the P x P chunk matrix. */
static uint64_t uordinal(uint64_t P, uint64_t i, uint64_t j)
{
    return i * P - i * (i - 1) / 2 + (j - i);
}

static void uchunk_of(uint64_t P, uint64_t ord, uint64_t *pi, uint64_t *pj)
{
    uint64_t i = 0;
    while (i + 1 < P && uordinal(P, i + 1, i + 1) <= ord) i++;
    *pi = i;
    *pj = i + (ord - uordinal(P, i, i));
}

/* Slot count of chunk with canonical ordinal c. */
static uint64_t chunk_slots(const kgref_inst *I, uint64_t c)
{
    if (I->directed) return (bound(I, c + 1) - bound(I, c)) * (I->n - 1);
    uint64_t i, j;
    uchunk_of(I->P, c, &i, &j);
    uint64_t hi = bound(I, i + 1) - bound(I, i);
    if (i == j) return hi * (hi - (hi > 0)) / 2;
    return hi * (bound(I, j + 1) - bound(I, j));
}

/* ---- Directed chunk tree (Sec. 4.1 with the split of Sec. 4.2) ---- */
static void dtree(const kgref_inst *I, uint64_t lo, uint64_t hi, uint64_t k,
                  uint64_t heap, uint64_t *counts)
{
    if (hi - lo == 1) { counts[lo] = k; return; }
    uint64_t mid = lo + (hi - lo + 1) / 2;
    uint64_t Nn = (bound(I, hi) - bound(I, lo)) * (I->n - 1);
    uint64_t Nl = (bound(I, mid) - bound(I, lo)) * (I->n - 1);
    uint64_t X = kgref_hyp(Nn, Nl, k, I->seed, (uint32_t)heap, 0, TAG_DTREE);
    dtree(I, lo, mid, X, 2 * heap, counts);
    dtree(I, mid, hi, k - X, 2 * heap + 1, counts);
}

/* ---- Undirected quadrant recursion (Sec. 4.2) ----
 * A triangle node T[a,b) covers all pairs of vertices u < v inside sections
 * a..b-1; a rectangle node R[a,b)x[c,d) covers row sections a..b-1 against
 * column sections c..d-1 (entirely above the diagonal).  Node codes: root 1,
 * child = 4 * parent + quadrant. */
static uint64_t tri_slots(const kgref_inst *I, uint64_t a, uint64_t b)
{
    uint64_t A = bound(I, b) - bound(I, a);
    return A * (A - (A > 0)) / 2;
}

static uint64_t rect_slots(const kgref_inst *I, uint64_t a, uint64_t b, uint64_t c, uint64_t d)
{
    return (bound(I, b) - bound(I, a)) * (bound(I, d) - bound(I, c));
}

static void rtree(const kgref_inst *I, uint64_t a, uint64_t b, uint64_t c, uint64_t d,
                  uint64_t k, uint64_t code, uint64_t *counts)
{
    uint64_t P = I->P;
    if (b - a == 1 && d - c == 1) { counts[uordinal(P, a, c)] = k; return; }
    uint64_t Nn = rect_slots(I, a, b, c, d);
    if (d - c == 1) {                       /* split rows only */
        uint64_t l = a + (b - a + 1) / 2;
        uint64_t X = kgref_hyp(Nn, rect_slots(I, a, l, c, d), k, I->seed, (uint32_t)code, 0, TAG_UTREE);
        rtree(I, a, l, c, d, X, 4 * code + 0, counts);
        rtree(I, l, b, c, d, k - X, 4 * code + 1, counts);
        return;
    }
    if (b - a == 1) {                       /* split columns only */
        uint64_t q = c + (d - c + 1) / 2;
        uint64_t X = kgref_hyp(Nn, rect_slots(I, a, b, c, q), k, I->seed, (uint32_t)code, 0, TAG_UTREE);
        rtree(I, a, b, c, q, X, 4 * code + 0, counts);
        rtree(I, a, b, q, d, k - X, 4 * code + 1, counts);
        return;
    }
    uint64_t l = a + (b - a + 1) / 2, q = c + (d - c + 1) / 2;
    uint64_t N00 = rect_slots(I, a, l, c, q), N01 = rect_slots(I, a, l, q, d);
    uint64_t N10 = rect_slots(I, l, b, c, q);
    uint64_t X00 = kgref_hyp(Nn, N00, k, I->seed, (uint32_t)code, 0, TAG_UTREE);
    uint64_t X01 = kgref_hyp(Nn - N00, N01, k - X00, I->seed, (uint32_t)code, 1, TAG_UTREE);
    uint64_t X10 = kgref_hyp(Nn - N00 - N01, N10, k - X00 - X01, I->seed, (uint32_t)code, 2, TAG_UTREE);
    rtree(I, a, l, c, q, X00, 4 * code + 0, counts);
    rtree(I, a, l, q, d, X01, 4 * code + 1, counts);
    rtree(I, l, b, c, q, X10, 4 * code + 2, counts);
    rtree(I, l, b, q, d, k - X00 - X01 - X10, 4 * code + 3, counts);
}

static void ttree(const kgref_inst *I, uint64_t a, uint64_t b, uint64_t k, uint64_t code,
                  uint64_t *counts)
{
    uint64_t P = I->P;
    if (b - a == 1) { counts[uordinal(P, a, a)] = k; return; }
    uint64_t l = a + (b - a + 1) / 2;
    uint64_t Nn = tri_slots(I, a, b);
    uint64_t N1 = tri_slots(I, a, l);
    uint64_t NR = rect_slots(I, a, l, l, b);
    uint64_t X0 = kgref_hyp(Nn, N1, k, I->seed, (uint32_t)code, 0, TAG_UTREE);
    uint64_t X1 = kgref_hyp(Nn - N1, NR, k - X0, I->seed, (uint32_t)code, 1, TAG_UTREE);
    ttree(I, a, l, X0, 4 * code + 0, counts);
    rtree(I, a, l, l, b, X1, 4 * code + 1, counts);
    ttree(I, l, b, k - X0 - X1, 4 * code + 2, counts);
}

/* Counts of all chunks in canonical order (whole-tree expansion). */
int kgref_chunk_counts(const kgref_inst *I, uint64_t *counts)
{
    int st = kgref_validate(I);
    if (st) return st;
    uint64_t C = kgref_num_chunks(I);
    if (I->model == 1) {
        /* Sec. 4.3: a binomial per chunk, keyed by the chunk id. */
        for (uint64_t c = 0; c < C; c++)
            counts[c] = kgref_bin(chunk_slots(I, c), I->p, I->seed, (uint32_t)c, 0, TAG_CBIN);
        return KGREF_OK;
    }
    if (I->directed) dtree(I, 0, I->P, I->m, 1, counts);
    else             ttree(I, 0, I->P, I->m, 1, counts);
    return KGREF_OK;
}

/* Count of a single chunk by walking only its root-to-leaf path, as one PE
 * does in the paper (Sec. 2.2, 4.1, 4.2).  Used to check that every chunk
 * obtains the same count without seeing the others. */
uint64_t kgref_chunk_count_path(const kgref_inst *I, uint64_t c)
{
    if (I->model == 1)
        return kgref_bin(chunk_slots(I, c), I->p, I->seed, (uint32_t)c, 0, TAG_CBIN);
    uint64_t k = I->m;
    if (I->directed) {
        uint64_t lo = 0, hi = I->P, heap = 1;
        while (hi - lo > 1) {
            uint64_t mid = lo + (hi - lo + 1) / 2;
            uint64_t Nn = (bound(I, hi) - bound(I, lo)) * (I->n - 1);
            uint64_t Nl = (bound(I, mid) - bound(I, lo)) * (I->n - 1);
            uint64_t X = kgref_hyp(Nn, Nl, k, I->seed, (uint32_t)heap, 0, TAG_DTREE);
            if (c < mid) { hi = mid; k = X; heap = 2 * heap; }
            else         { lo = mid; k = k - X; heap = 2 * heap + 1; }
        }
        return k;
    }
    uint64_t ci, cj;
    uchunk_of(I->P, c, &ci, &cj);
    uint64_t a = 0, b = I->P, cc = 0, d = 0, code = 1;
    int tri = 1;
    for (;;) {
        if (tri) {
            if (b - a == 1) return k;
            uint64_t l = a + (b - a + 1) / 2;
            uint64_t Nn = tri_slots(I, a, b), N1 = tri_slots(I, a, l), NR = rect_slots(I, a, l, l, b);
            uint64_t X0 = kgref_hyp(Nn, N1, k, I->seed, (uint32_t)code, 0, TAG_UTREE);
            if (cj < l) { b = l; k = X0; code = 4 * code; continue; }
            uint64_t X1 = kgref_hyp(Nn - N1, NR, k - X0, I->seed, (uint32_t)code, 1, TAG_UTREE);
            if (ci < l) { tri = 0; cc = l; d = b; b = l; k = X1; code = 4 * code + 1; continue; }
            a = l; k = k - X0 - X1; code = 4 * code + 2;
            continue;
        }
        if (b - a == 1 && d - cc == 1) return k;
        uint64_t Nn = rect_slots(I, a, b, cc, d);
        if (d - cc == 1) {
            uint64_t l = a + (b - a + 1) / 2;
            uint64_t X = kgref_hyp(Nn, rect_slots(I, a, l, cc, d), k, I->seed, (uint32_t)code, 0, TAG_UTREE);
            if (ci < l) { b = l; k = X; code = 4 * code; }
            else        { a = l; k = k - X; code = 4 * code + 1; }
            continue;
        }
        if (b - a == 1) {
            uint64_t q = cc + (d - cc + 1) / 2;
            uint64_t X = kgref_hyp(Nn, rect_slots(I, a, b, cc, q), k, I->seed, (uint32_t)code, 0, TAG_UTREE);
            if (cj < q) { d = q; k = X; code = 4 * code; }
            else        { cc = q; k = k - X; code = 4 * code + 1; }
            continue;
        }
        uint64_t l = a + (b - a + 1) / 2, q = cc + (d - cc + 1) / 2;
        uint64_t N00 = rect_slots(I, a, l, cc, q), N01 = rect_slots(I, a, l, q, d);
        uint64_t N10 = rect_slots(I, l, b, cc, q);
        int quad = (ci >= l) * 2 + (cj >= q);
        uint64_t X00 = kgref_hyp(Nn, N00, k, I->seed, (uint32_t)code, 0, TAG_UTREE);
        uint64_t X01 = 0, X10 = 0;
        if (quad >= 1) X01 = kgref_hyp(Nn - N00, N01, k - X00, I->seed, (uint32_t)code, 1, TAG_UTREE);
        if (quad >= 2) X10 = kgref_hyp(Nn - N00 - N01, N10, k - X00 - X01, I->seed, (uint32_t)code, 2, TAG_UTREE);
        uint64_t kk = quad == 0 ? X00 : quad == 1 ? X01 : quad == 2 ? X10 : k - X00 - X01 - X10;
        if (quad < 2) b = l; else a = l;
        if (quad & 1) cc = q; else d = q;
        k = kk;
        code = 4 * code + (uint64_t)quad;
    }
}

/* ------------------------------------------------------------------ */
/* Tiles: the sequential-sampling threshold (Sec. 2.2)                 */
/* ------------------------------------------------------------------ */
static uint64_t tile_range_slots(uint64_t lo, uint64_t hi, uint32_t s, uint64_t Nc)
{
    u128 end = (u128)hi << s;
    uint64_t e = end > Nc ? Nc : (uint64_t)end;
    return e - (lo << s);
}

static void tile_tree(const kgref_inst *I, uint64_t ordinal, uint32_t s, uint64_t Nc,
                      uint64_t lo, uint64_t hi, uint64_t k, uint64_t heap, uint64_t *tcounts)
{
    if (hi - lo == 1) { tcounts[lo] = k; return; }
    uint64_t mid = lo + (hi - lo + 1) / 2;
    uint64_t X = kgref_hyp(tile_range_slots(lo, hi, s, Nc), tile_range_slots(lo, mid, s, Nc), k,
                           I->seed, (uint32_t)ordinal, (uint32_t)heap, TAG_TTREE);
    tile_tree(I, ordinal, s, Nc, lo, mid, X, 2 * heap, tcounts);
    tile_tree(I, ordinal, s, Nc, mid, hi, k - X, 2 * heap + 1, tcounts);
}

uint64_t kgref_chunk_num_tiles(const kgref_inst *I, uint64_t c)
{
    uint32_t s = kgref_tile_exponent(I);
    uint64_t Nc = chunk_slots(I, c);
    return (Nc + ((1ull << s) - 1)) >> s;
}

/* Tile counts of chunk c given its count Kc; returns the number of tiles. */
uint64_t kgref_tile_counts(const kgref_inst *I, uint64_t c, uint64_t Kc, uint64_t *tcounts)
{
    uint32_t s = kgref_tile_exponent(I);
    uint64_t Nc = chunk_slots(I, c);
    uint64_t T = (Nc + ((1ull << s) - 1)) >> s;
    if (T == 0) return 0;
    tile_tree(I, c, s, Nc, 0, T, Kc, 1, tcounts);
    return T;
}

/* ---- Base case: draw until k distinct slots, output ascending ---- */
typedef struct { uint64_t *slot; uint64_t cap; } hset;   /* open addressing, key+1 stored */

static int hset_insert(hset *h, uint64_t key)
{
    uint64_t i = (key * 0x9E3779B97F4A7C15ull) & (h->cap - 1);
    for (;;) {
        if (h->slot[i] == 0) { h->slot[i] = key + 1; return 1; }
        if (h->slot[i] == key + 1) return 0;
        i = (i + 1) & (h->cap - 1);
    }
}

static int hset_has(const hset *h, uint64_t key)
{
    uint64_t i = (key * 0x9E3779B97F4A7C15ull) & (h->cap - 1);
    for (;;) {
        if (h->slot[i] == 0) return 0;
        if (h->slot[i] == key + 1) return 1;
        i = (i + 1) & (h->cap - 1);
    }
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Sorted k-subset of [0, St) for tile `tile` of chunk `ordinal`.  Draw t is
 * word t mod 4 of block t/4 of the stream, masked to ceil(log2 St) bits;
 * values >= St are rejected; repeats are skipped; sampling stops at the
 * k-th distinct value.  If 2k > St the St - k excluded slots are drawn
 * that way and the complement is returned.  keys must hold k entries. */
int kgref_leaf(uint64_t k, uint64_t St, uint64_t seed, uint32_t ordinal, uint32_t tile,
               uint64_t *keys)
{
    if (k > St) return KGREF_EINVAL;
    if (k == 0) return KGREF_OK;
    int comp = 2 * k > St;
    uint64_t want = comp ? St - k : k;
    uint64_t cap = 16;
    while (cap < 2 * want + 2) cap <<= 1;
    hset h;
    h.cap = cap;
    h.slot = (uint64_t *)calloc(cap, sizeof(uint64_t));
    uint64_t *drawn = (uint64_t *)malloc((want + 1) * sizeof(uint64_t));
    if (!h.slot || !drawn) { free(h.slot); free(drawn); return KGREF_ENOSPC; }
    uint64_t mask = 0;
    while (mask < St - 1) mask = (mask << 1) | 1;
    stream_t s;
    stream_init(&s, seed, ordinal, tile, TAG_TLEAF);
    uint64_t got = 0;
    uint32_t w[4];
    uint64_t curj = UINT64_MAX;
    for (uint64_t t = 0; got < want; t++) {
        uint64_t j = t >> 2;
        if (j != curj) { stream_block(&s, j, w); curj = j; }
        uint64_t x = (uint64_t)w[t & 3] & mask;
        if (x >= St) continue;
        if (hset_insert(&h, x)) drawn[got++] = x;
    }
    if (!comp) {
        qsort(drawn, want, sizeof(uint64_t), cmp_u64);
        memcpy(keys, drawn, want * sizeof(uint64_t));
    } else {
        uint64_t o = 0;
        for (uint64_t x = 0; x < St; x++)
            if (!hset_has(&h, x)) keys[o++] = x;
    }
    free(h.slot);
    free(drawn);
    return KGREF_OK;
}

/* ---- Offset computations: slot -> edge (Sec. 4.1, 4.2) ---- */
typedef struct {
    int directed, diag;
    uint64_t n, row0;      /* directed: first row of the chunk */
    uint64_t a, h;         /* undirected: row section start and size */
    uint64_t b, w;         /* undirected: column section start and size */
} chunk_geo;

static void chunk_geometry(const kgref_inst *I, uint64_t c, chunk_geo *g)
{
    memset(g, 0, sizeof(*g));
    g->directed = (int)I->directed;
    g->n = I->n;
    if (I->directed) { g->row0 = bound(I, c); return; }
    uint64_t ci, cj;
    uchunk_of(I->P, c, &ci, &cj);
    g->diag = ci == cj;
    g->a = bound(I, ci); g->h = bound(I, ci + 1) - g->a;
    g->b = bound(I, cj); g->w = bound(I, cj + 1) - g->b;
}

static void decode(const chunk_geo *g, uint64_t l, uint32_t *u, uint32_t *v)
{
    if (g->directed) {
        /* Row-major over the n x n matrix without its diagonal. */
        uint64_t i = g->row0 * (g->n - 1) + l;
        uint64_t uu = i / (g->n - 1), w = i % (g->n - 1);
        *u = (uint32_t)uu;
        *v = (uint32_t)(w + (w >= uu));
        return;
    }
    if (!g->diag) {
        /* Rectangle: row-major over h rows of w columns. */
        *u = (uint32_t)(g->a + l / g->w);
        *v = (uint32_t)(g->b + l % g->w);
        return;
    }
    /* Triangle: row r holds the h-1-r pairs (r, r+1..h-1) and starts at
     * r h - r(r+1)/2; find the last start <= l by bisection. */
    uint64_t h = g->h, lo = 0, hi = h - 1;
    while (hi - lo > 1) {
        uint64_t mid = (lo + hi) / 2;
        u128 st = (u128)mid * h - (u128)mid * (mid + 1) / 2;
        if (st <= l) lo = mid; else hi = mid;
    }
    uint64_t st = lo * h - lo * (lo + 1) / 2;
    *u = (uint32_t)(g->a + lo);
    *v = (uint32_t)(g->a + lo + 1 + (l - st));
}

/* Edges of chunk c in ascending local order; returns the count written or a
 * negative status. out must hold Kc pairs. */
int64_t kgref_chunk_edges_given(const kgref_inst *I, uint64_t c, uint64_t Kc, uint32_t *out)
{
    uint32_t s = kgref_tile_exponent(I);
    uint64_t Nc = chunk_slots(I, c);
    uint64_t T = (Nc + ((1ull << s) - 1)) >> s;
    if (Kc == 0) return 0;
    if (Kc > Nc) return KGREF_EINVAL;
    uint64_t *tc = (uint64_t *)malloc(T * sizeof(uint64_t));
    uint64_t *toff = (uint64_t *)malloc((T + 1) * sizeof(uint64_t));
    kgref_tile_counts(I, c, Kc, tc);
    toff[0] = 0;
    for (uint64_t t = 0; t < T; t++) toff[t + 1] = toff[t] + tc[t];
    chunk_geo g;
    chunk_geometry(I, c, &g);
    int err = 0;
    /* Tiles are independent given their counts: a chunk with many tiles
     * that is generated alone spreads them over threads (each tile still
     * writes at its own offset, so the order of the work does not matter). */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 8) reduction(| : err) if (T >= 256 && !omp_in_parallel())
#endif
    for (int64_t ti = 0; ti < (int64_t)T; ti++) {
        uint64_t t = (uint64_t)ti;
        uint64_t St = tile_range_slots(t, t + 1, s, Nc);
        uint64_t *keys = (uint64_t *)malloc((tc[t] + 1) * sizeof(uint64_t));
        int st = kgref_leaf(tc[t], St, I->seed, (uint32_t)c, (uint32_t)t, keys);
        if (st) {
            err |= 1;
        } else {
            uint64_t o = toff[t];
            for (uint64_t e = 0; e < tc[t]; e++, o++) {
                uint32_t u, v;
                decode(&g, (t << s) + keys[e], &u, &v);
                out[2 * o] = u;
                out[2 * o + 1] = v;
            }
        }
        free(keys);
    }
    uint64_t total = toff[T];
    free(tc);
    free(toff);
    return err ? KGREF_EINVAL : (int64_t)total;
}

int64_t kgref_chunk_edges(const kgref_inst *I, uint64_t c, uint32_t *out)
{
    int st = kgref_validate(I);
    if (st) return st;
    return kgref_chunk_edges_given(I, c, kgref_chunk_count_path(I, c), out);
}

/* Whole edge list: chunks in canonical order (Sec. 4.1 rows ascending;
 * Sec. 4.2 chunk matrix row-major), each chunk's edges at the exclusive
 * prefix sum of the counts.  Chunks are independent (communication-free),
 * so they are generated in parallel.  Returns the number of edges, or a
 * negative status (KGREF_ENOSPC if it exceeds cap; nothing written then). */
int64_t kgref_generate(const kgref_inst *I, uint32_t *out, uint64_t cap, int threads)
{
    int st = kgref_validate(I);
    if (st) return st;
    uint64_t C = kgref_num_chunks(I);
    uint64_t *counts = (uint64_t *)malloc(C * sizeof(uint64_t));
    uint64_t *off = (uint64_t *)malloc((C + 1) * sizeof(uint64_t));
    kgref_chunk_counts(I, counts);
    off[0] = 0;
    for (uint64_t c = 0; c < C; c++) off[c + 1] = off[c] + counts[c];
    uint64_t total = off[C];
    if (total > cap) { free(counts); free(off); return KGREF_ENOSPC; }
    int err = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
#endif
    for (int64_t c = 0; c < (int64_t)C; c++) {
        int64_t r = kgref_chunk_edges_given(I, (uint64_t)c, counts[c], out + 2 * off[c]);
        if (r < 0 || (uint64_t)r != counts[c]) err |= 1;
    }
    (void)threads;
    free(counts);
    free(off);
    return err ? KGREF_EINVAL : (int64_t)total;
}

/* ------------------------------------------------------------------------
 * The geometric-skip G(n,p) variant (a second sampler for the same law,
 * with its own bits).  Every slot is an independent Bernoulli(p) trial
 * (Sec. 2.1.1, 4.3); instead of a binomial count per chunk and a sample of
 * that size, each tile of the chunk (the same 2^s-slot tiles) runs the
 * trials itself by waiting times: the number of failures before the next
 * success is floor(log U / log(1 - p)) (geometric law), U from the tile's
 * stream (seed, chunk ordinal, tile, TAG_SKIP), one 64-bit draw per gap.
 * For p > 1/2 the waiting times are those of the failures (probability
 * 1 - p) and every other slot is a success.  Keys come out ascending.
 * ------------------------------------------------------------------------ */

/* Successes of one tile of St slots: their number; the tile-local keys go to
 * keys[] when keys is not NULL. */
static uint64_t skip_tile(uint64_t St, double p, uint64_t seed, uint32_t c, uint32_t t, uint64_t *keys)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) {
        if (keys) for (uint64_t x = 0; x < St; x++) keys[x] = x;
        return St;
    }
    const int flip = p > 0.5;
    const double L = kgref_log1p(flip ? -(1.0 - p) : -p);
    stream_t s;
    stream_init(&s, seed, c, t, TAG_SKIP);
    uint64_t pos = 0, k = 0;
    for (;;) {
        double U = u64_to_unit(stream_u64(&s));
        double g = floor(kgref_log(U) / L);
        uint64_t next = g >= (double)(St - pos) ? St : pos + (uint64_t)g;   /* the next trial event, or the end */
        if (flip) {
            /* slots pos .. next-1 are successes, next (if inside) a failure */
            for (uint64_t x = pos; x < next; x++) { if (keys) keys[k] = x; k++; }
        } else if (next < St) {
            if (keys) keys[k] = next;
            k++;
        }
        if (next >= St) return k;
        pos = next + 1;
    }
}

static uint64_t skip_chunk(const kgref_inst *I, uint64_t c, uint32_t *out)
{
    uint32_t s = kgref_tile_exponent(I);
    uint64_t Nc = chunk_slots(I, c);
    uint64_t T = (Nc + ((1ull << s) - 1)) >> s;
    chunk_geo g;
    chunk_geometry(I, c, &g);
    uint64_t o = 0, room = 0;
    uint64_t *keys = NULL;
    for (uint64_t t = 0; t < T; t++) {
        uint64_t St = tile_range_slots(t, t + 1, s, Nc);
        uint64_t k = skip_tile(St, I->p, I->seed, (uint32_t)c, (uint32_t)t, NULL);
        if (out && k > 0) {
            if (k > room) {
                free(keys);
                room = k;
                keys = (uint64_t *)malloc(room * sizeof(uint64_t));
            }
            skip_tile(St, I->p, I->seed, (uint32_t)c, (uint32_t)t, keys);
            for (uint64_t e = 0; e < k; e++) {
                uint32_t u, v;
                decode(&g, (t << s) + keys[e], &u, &v);
                out[2 * (o + e)] = u;
                out[2 * (o + e) + 1] = v;
            }
        }
        o += k;
    }
    free(keys);
    return o;
}

/* Edges of chunk c under the skip variant (out may be NULL: count only). */
int64_t kgref_skip_chunk_edges(const kgref_inst *I, uint64_t c, uint32_t *out)
{
    int st = kgref_validate(I);
    if (st) return st;
    if (I->model != 1) return KGREF_EINVAL;
    return (int64_t)skip_chunk(I, c, out);
}

/* Whole edge list under the skip variant, chunks in canonical order; returns
 * the number of edges (KGREF_ENOSPC if above cap: nothing written). */
int64_t kgref_skip_generate(const kgref_inst *I, uint32_t *out, uint64_t cap, int threads)
{
    int st = kgref_validate(I);
    if (st) return st;
    if (I->model != 1) return KGREF_EINVAL;
    uint64_t C = kgref_num_chunks(I);
    uint64_t *off = (uint64_t *)malloc((C + 1) * sizeof(uint64_t));
    off[0] = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < (int64_t)C; c++) off[c + 1] = skip_chunk(I, (uint64_t)c, NULL);
    for (uint64_t c = 0; c < C; c++) off[c + 1] += off[c];
    uint64_t total = off[C];
    if (total > cap) { free(off); return KGREF_ENOSPC; }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < (int64_t)C; c++) skip_chunk(I, (uint64_t)c, out + 2 * off[c]);
    (void)threads;
    free(off);
    return (int64_t)total;
}

/* Per-instance seed of a batch: the Philox image of (0, i, 0, INST) under the
 * base seed, words (w1:w0). */
uint64_t kgref_instance_seed(uint64_t base, uint32_t i)
{
    uint32_t ctr[4] = { 0, i, 0, TAG_INST };
    uint32_t key[2] = { (uint32_t)base, (uint32_t)(base >> 32) };
    uint32_t w[4];
    kgref_philox(ctr, key, w);
    return ((uint64_t)w[1] << 32) | w[0];
}

int kgref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Array evaluation of the building blocks for element-wise comparisons
 * (record layouts as in the tests): fn 1 philox, 2 log, 3 log1p,
 * 4 lnf_diff, 5 hyp, 6 bin. */
void kgref_eval_many(int fn, const void *in, void *out, uint64_t n)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < (int64_t)n; i++) {
        switch (fn) {
        case 1: {
            const uint32_t *r = (const uint32_t *)in + 6 * i;
            kgref_philox(r, r + 4, (uint32_t *)out + 4 * i);
            break;
        }
        case 2: ((double *)out)[i] = kgref_log(((const double *)in)[i]); break;
        case 3: ((double *)out)[i] = kgref_log1p(((const double *)in)[i]); break;
        case 4: {
            const uint64_t *r = (const uint64_t *)in + 2 * i;
            ((double *)out)[i] = kgref_lnf_diff(r[0], r[1]);
            break;
        }
        case 5: {
            const uint64_t *r = (const uint64_t *)in + 6 * i;
            ((uint64_t *)out)[i] = kgref_hyp(r[0], r[1], r[2], r[3], (uint32_t)r[4], (uint32_t)(r[4] >> 32),
                                             (uint32_t)r[5]);
            break;
        }
        case 6: {
            const uint64_t *r = (const uint64_t *)in + 6 * i;
            double p;
            memcpy(&p, &r[1], 8);
            ((uint64_t *)out)[i] = kgref_bin(r[0], p, r[3], (uint32_t)r[4], (uint32_t)(r[4] >> 32),
                                             (uint32_t)r[5]);
            break;
        }
        default: break;
        }
    }
}

/* Edges of the chunks [c0, c1), concatenated in canonical order, given all
 * chunk counts; chunks in parallel.  Returns the number of edges written or a
 * negative status (KGREF_ENOSPC if they exceed cap). */
int64_t kgref_generate_chunks(const kgref_inst *I, const uint64_t *counts, uint64_t c0, uint64_t c1,
                              uint32_t *out, uint64_t cap, int threads)
{
    int st = kgref_validate(I);
    if (st) return st;
    uint64_t C = kgref_num_chunks(I);
    if (c0 > c1 || c1 > C) return KGREF_EINVAL;
    uint64_t *off = (uint64_t *)malloc((c1 - c0 + 1) * sizeof(uint64_t));
    off[0] = 0;
    for (uint64_t c = c0; c < c1; c++) off[c - c0 + 1] = off[c - c0] + counts[c];
    uint64_t total = off[c1 - c0];
    if (total > cap) { free(off); return KGREF_ENOSPC; }
    int err = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
#endif
    for (int64_t c = (int64_t)c0; c < (int64_t)c1; c++) {
        int64_t r = kgref_chunk_edges_given(I, (uint64_t)c, counts[c], out + 2 * off[c - c0]);
        if (r < 0 || (uint64_t)r != counts[c]) err |= 1;
    }
    (void)threads;
    free(off);
    return err ? KGREF_EINVAL : (int64_t)total;
}

/* ------------------------------------------------------------------ */
/* Random geometric graphs in two dimensions (Sec. 2.1.2 model; Sec. 5 */
/* generator: grid of cells of side >= r, a divide-and-conquer count   */
/* of the points per sub-square by binomial variates keyed by the      */
/* subtree, points per cell from the cell's own stream, edges between  */
/* a cell and its neighbours, each pair tested once).                  */
/*                                                                     */
/* Our reading: the unit square is split recursively into quadrants   */
/* down to 4^L cells of side 2^-L, L the largest level with            */
/* 2^L r <= 1 and 4^L <= n (cells of side >= max(r, n^-1/2), Sec. 5),  */
/* at most KGREF_RGG_MAX_LEVEL.  A node at level l, Morton index z,    */
/* holding k points splits them as: lower half (y) Bin(k, 1/2), its    */
/* left quadrant Bin(lower, 1/2), the upper-left quadrant              */
/* Bin(k - lower, 1/2); every probability is exactly 1/2, so the four  */
/* counts are multinomial(k; 1/4 each) with no rounding of the law.    */
/* Streams: (seed; j, z, 3 l + slot, TAG_RTREE) for the three draws,   */
/* (seed; j, cell, 0, TAG_RPTS) for the points, block j = point j.     */
/* Vertex ids follow the cells in Morton order; edges are the pairs    */
/* u < v with dx^2 + dy^2 < r^2 (binary64, each operation rounded),    */
/* listed in ascending (u, v).                                         */
/* ------------------------------------------------------------------ */
#define TAG_RTREE 8
#define TAG_RPTS 9
#define KGREF_RGG_MAX_LEVEL 14

uint32_t kgref_rgg_level(uint64_t n, double r)
{
    uint32_t L = 0;
    while (L < KGREF_RGG_MAX_LEVEL && ldexp(r, (int)L + 1) <= 1.0 && ((uint64_t)1 << (2 * (L + 1))) <= n) L++;
    return L;
}

/* the three binomial draws of node (l, z) holding k points -> the four
 * quadrant counts in Morton order (x bit low, y bit high) */
static void rgg_split(uint64_t seed, uint32_t l, uint64_t z, uint64_t k, uint64_t q[4])
{
    uint64_t lower = kgref_bin(k, 0.5, seed, (uint32_t)z, 3 * l + 0, TAG_RTREE);
    uint64_t ll = kgref_bin(lower, 0.5, seed, (uint32_t)z, 3 * l + 1, TAG_RTREE);
    uint64_t ul = kgref_bin(k - lower, 0.5, seed, (uint32_t)z, 3 * l + 2, TAG_RTREE);
    q[0] = ll;
    q[1] = lower - ll;
    q[2] = ul;
    q[3] = k - lower - ul;
}

static void rgg_tree(uint64_t seed, uint32_t L, uint32_t l, uint64_t z, uint64_t k, uint64_t *cells)
{
    if (l == L) { cells[z] = k; return; }
    uint64_t q[4];
    rgg_split(seed, l, z, k, q);
    for (int i = 0; i < 4; i++) rgg_tree(seed, L, l + 1, 4 * z + (uint64_t)i, q[i], cells);
}

/* Point counts of all 4^L cells, Morton order. */
int kgref_rgg_cells(uint64_t n, double r, uint64_t seed, uint64_t *cells)
{
    uint32_t L = kgref_rgg_level(n, r);
    rgg_tree(seed, L, 0, 0, n, cells);
    return (int)L;
}

/* One cell's count by walking only its root path, as a processor that owns
 * the cell (or needs it as a neighbour) does without communication. */
uint64_t kgref_rgg_cell_count_path(uint64_t n, double r, uint64_t seed, uint64_t cell)
{
    uint32_t L = kgref_rgg_level(n, r);
    uint64_t k = n, z = 0;
    for (uint32_t l = 0; l < L; l++) {
        uint64_t q[4];
        rgg_split(seed, l, z, k, q);
        uint64_t d = (cell >> (2 * (L - 1 - l))) & 3;
        z = 4 * z + d;
        k = q[d];
    }
    return k;
}

static void rgg_cell_xy(uint64_t z, uint32_t L, uint64_t *cx, uint64_t *cy)
{
    uint64_t x = 0, y = 0;
    for (uint32_t i = 0; i < L; i++) {
        x |= ((z >> (2 * i)) & 1) << i;
        y |= ((z >> (2 * i + 1)) & 1) << i;
    }
    *cx = x;
    *cy = y;
}

static uint64_t rgg_morton(uint64_t x, uint64_t y, uint32_t L)
{
    uint64_t z = 0;
    for (uint32_t i = 0; i < L; i++) z |= (((x >> i) & 1) << (2 * i)) | (((y >> i) & 1) << (2 * i + 1));
    return z;
}

/* Point j of cell z: (cx + U, cy + V) 2^-L, U and V the two uniforms of
 * block j of the cell's stream. */
static void rgg_point(uint64_t seed, uint32_t L, uint64_t z, uint64_t j, double *x, double *y)
{
    stream_t s;
    stream_init(&s, seed, (uint32_t)z, 0, TAG_RPTS);
    uint32_t w[4];
    stream_block(&s, j, w);
    double U = u64_to_unit(((uint64_t)w[1] << 32) | w[0]);
    double V = u64_to_unit(((uint64_t)w[3] << 32) | w[2]);
    uint64_t cx, cy;
    rgg_cell_xy(z, L, &cx, &cy);
    double h = ldexp(1.0, -(int)L);
    *x = ((double)cx + U) * h;
    *y = ((double)cy + V) * h;
}

static int rgg_adjacent(const double *a, const double *b, double r2)
{
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    return dx * dx + dy * dy < r2;
}

static int cmp_u64r(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

/* The whole graph: points (2n doubles, vertex order) and the edges in
 * ascending (u, v), at most cap of them written.  Returns the edge count
 * (which may exceed cap: then only the first cap are written), or a
 * negative status. */
int64_t kgref_rgg2d(uint64_t n, double r, uint64_t seed, double *pts, uint32_t *edges, uint64_t cap)
{
    if (!(r >= 0.0) || n > 0xFFFFFFFFull) return KGREF_EINVAL;
    uint32_t L = kgref_rgg_level(n, r);
    uint64_t G = (uint64_t)1 << L, C = G * G;
    uint64_t *cells = (uint64_t *)calloc(C, sizeof(uint64_t));
    uint64_t *off = (uint64_t *)malloc((C + 1) * sizeof(uint64_t));
    double *P = pts ? pts : (double *)malloc((2 * n + 2) * sizeof(double));
    rgg_tree(seed, L, 0, 0, n, cells);
    off[0] = 0;
    for (uint64_t z = 0; z < C; z++) off[z + 1] = off[z] + cells[z];
    for (uint64_t z = 0; z < C; z++)
        for (uint64_t j = 0; j < cells[z]; j++) rgg_point(seed, L, z, j, &P[2 * (off[z] + j)], &P[2 * (off[z] + j) + 1]);
    const double r2 = r * r;
    uint64_t E = 0;
    for (uint64_t z = 0; z < C; z++) {
        uint64_t cx, cy, nb[9];
        int nn = 0;
        rgg_cell_xy(z, L, &cx, &cy);
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int64_t x = (int64_t)cx + dx, y = (int64_t)cy + dy;
                if (x < 0 || y < 0 || x >= (int64_t)G || y >= (int64_t)G) continue;
                uint64_t zz = rgg_morton((uint64_t)x, (uint64_t)y, L);
                if (zz >= z) nb[nn++] = zz;
            }
        qsort(nb, (size_t)nn, sizeof(uint64_t), cmp_u64r);
        for (uint64_t a = off[z]; a < off[z + 1]; a++)
            for (int i = 0; i < nn; i++)
                for (uint64_t b = off[nb[i]]; b < off[nb[i] + 1]; b++) {
                    if (b <= a || !rgg_adjacent(&P[2 * a], &P[2 * b], r2)) continue;
                    if (edges && E < cap) { edges[2 * E] = (uint32_t)a; edges[2 * E + 1] = (uint32_t)b; }
                    E++;
                }
    }
    free(cells);
    free(off);
    if (!pts) free(P);
    return (int64_t)E;
}

/* The k points of cell z (2k doubles), as the whole generator makes them. */
void kgref_rgg_cell_points(uint64_t n, double r, uint64_t seed, uint64_t z, uint64_t k, double *out)
{
    uint32_t L = kgref_rgg_level(n, r);
    for (uint64_t j = 0; j < k; j++) rgg_point(seed, L, z, j, &out[2 * j], &out[2 * j + 1]);
}

/* ------------------------------------------------------------------ */
/* Three-dimensional random geometric graphs (Sec. 2.1.2, Sec. 5 with  */
/* d = 3): n points uniform in the unit cube, an edge between every     */
/* two points closer than r.  Cells of side 2^-L >= max(r, n^-1/3), L   */
/* at most 10, from an octant recursion: a node (level l, Morton index  */
/* z) holding k points draws 2^3 - 1 = 7 Bin(., 1/2) variates (the      */
/* paper's 2^d - 1 binomials per split, Sec. 5.1): the lower z half     */
/* (slot 0); the lower y halves of the lower and the upper z half       */
/* (slots 1, 2); the lower x halves of the four (z, y) quarters (slots  */
/* 3..6, in Morton order); stream (j, z, 7 l + slot, TAG_RTREE3).       */
/* Point j of cell z: ((cx + U) h, (cy + V) h, (cz + W) h), U, V, W the */
/* 64-bit draws 3j, 3j + 1, 3j + 2 of (z, 0, TAG_RPTS3).  Vertex ids in */
/* Morton order of the cells (x bit low, then y, then z), then the      */
/* points of a cell; an edge iff ((dx^2 + dy^2) + dz^2) < r^2 in        */
/* binary64, each operation rounded; each pair once as u < v, in        */
/* ascending (u, v).                                                    */
/* ------------------------------------------------------------------ */
#define TAG_RTREE3 10
#define TAG_RPTS3 11
#define KGREF_RGG3_MAX_LEVEL 10

uint32_t kgref_rgg3_level(uint64_t n, double r)
{
    uint32_t L = 0;
    while (L < KGREF_RGG3_MAX_LEVEL && ldexp(r, (int)L + 1) <= 1.0 && ((uint64_t)1 << (3 * (L + 1))) <= n) L++;
    return L;
}

/* the seven binomial draws of node (l, z) holding k points -> the eight
 * octant counts in Morton order (index x + 2 y + 4 z of the octant) */
static void rgg3_split(uint64_t seed, uint32_t l, uint64_t z, uint64_t k, uint64_t q[8])
{
    uint32_t a = (uint32_t)z, b = 7 * l;
    uint64_t lz = kgref_bin(k, 0.5, seed, a, b + 0, TAG_RTREE3);          /* z = 0 half */
    uint64_t y0 = kgref_bin(lz, 0.5, seed, a, b + 1, TAG_RTREE3);         /* z = 0, y = 0 */
    uint64_t y1 = kgref_bin(k - lz, 0.5, seed, a, b + 2, TAG_RTREE3);     /* z = 1, y = 0 */
    uint64_t quarter[4] = {y0, lz - y0, y1, k - lz - y1};                  /* (y, z) = 00, 10, 01, 11 */
    for (int i = 0; i < 4; i++) {
        uint64_t x0 = kgref_bin(quarter[i], 0.5, seed, a, b + 3 + (uint32_t)i, TAG_RTREE3);
        q[2 * i] = x0;
        q[2 * i + 1] = quarter[i] - x0;
    }
}

static void rgg3_tree(uint64_t seed, uint32_t L, uint32_t l, uint64_t z, uint64_t k, uint64_t *cells)
{
    if (l == L) { cells[z] = k; return; }
    uint64_t q[8];
    rgg3_split(seed, l, z, k, q);
    for (int i = 0; i < 8; i++) rgg3_tree(seed, L, l + 1, 8 * z + (uint64_t)i, q[i], cells);
}

/* Point counts of all 8^L cells, Morton order. */
int kgref_rgg3_cells(uint64_t n, double r, uint64_t seed, uint64_t *cells)
{
    uint32_t L = kgref_rgg3_level(n, r);
    rgg3_tree(seed, L, 0, 0, n, cells);
    return (int)L;
}

/* One cell's count from its root path only (no other node is drawn). */
uint64_t kgref_rgg3_cell_count_path(uint64_t n, double r, uint64_t seed, uint64_t cell)
{
    uint32_t L = kgref_rgg3_level(n, r);
    uint64_t k = n, z = 0;
    for (uint32_t l = 0; l < L; l++) {
        uint64_t q[8];
        rgg3_split(seed, l, z, k, q);
        uint64_t d = (cell >> (3 * (L - 1 - l))) & 7;
        z = 8 * z + d;
        k = q[d];
    }
    return k;
}

static void rgg3_cell_xyz(uint64_t z, uint32_t L, uint64_t c[3])
{
    c[0] = c[1] = c[2] = 0;
    for (uint32_t i = 0; i < L; i++)
        for (int d = 0; d < 3; d++) c[d] |= ((z >> (3 * i + (uint32_t)d)) & 1) << i;
}

static uint64_t rgg3_morton(const int64_t c[3], uint32_t L)
{
    uint64_t z = 0;
    for (uint32_t i = 0; i < L; i++)
        for (int d = 0; d < 3; d++) z |= (((uint64_t)c[d] >> i) & 1) << (3 * i + (uint32_t)d);
    return z;
}

/* Point j of cell z. */
static void rgg3_point(uint64_t seed, uint32_t L, uint64_t z, uint64_t j, double *out)
{
    stream_t s;
    stream_init(&s, seed, (uint32_t)z, 0, TAG_RPTS3);
    uint64_t c[3];
    rgg3_cell_xyz(z, L, c);
    double h = ldexp(1.0, -(int)L);
    for (int d = 0; d < 3; d++) {
        uint64_t t = 3 * j + (uint64_t)d;      /* 64-bit draw t: half t % 2 of block t / 2 */
        uint32_t w[4];
        stream_block(&s, t / 2, w);
        uint64_t x = (t & 1) ? (((uint64_t)w[3] << 32) | w[2]) : (((uint64_t)w[1] << 32) | w[0]);
        out[d] = ((double)c[d] + u64_to_unit(x)) * h;
    }
}

static int rgg3_adjacent(const double *a, const double *b, double r2)
{
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    double dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz < r2;
}

/* The whole graph: points (3n doubles, vertex order) and the edges in
 * ascending (u, v), at most cap of them written.  Returns the edge count
 * (which may exceed cap: then only the first cap are written), or a
 * negative status. */
int64_t kgref_rgg3d(uint64_t n, double r, uint64_t seed, double *pts, uint32_t *edges, uint64_t cap)
{
    if (!(r >= 0.0) || n > 0xFFFFFFFFull) return KGREF_EINVAL;
    uint32_t L = kgref_rgg3_level(n, r);
    uint64_t G = (uint64_t)1 << L, C = G * G * G;
    uint64_t *cells = (uint64_t *)calloc(C, sizeof(uint64_t));
    uint64_t *off = (uint64_t *)malloc((C + 1) * sizeof(uint64_t));
    double *P = pts ? pts : (double *)malloc((3 * n + 3) * sizeof(double));
    rgg3_tree(seed, L, 0, 0, n, cells);
    off[0] = 0;
    for (uint64_t z = 0; z < C; z++) off[z + 1] = off[z] + cells[z];
    for (uint64_t z = 0; z < C; z++)
        for (uint64_t j = 0; j < cells[z]; j++) rgg3_point(seed, L, z, j, &P[3 * (off[z] + j)]);
    const double r2 = r * r;
    uint64_t E = 0;
    for (uint64_t z = 0; z < C; z++) {
        uint64_t c[3], nb[27];
        int nn = 0;
        rgg3_cell_xyz(z, L, c);
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int64_t w[3] = {(int64_t)c[0] + dx, (int64_t)c[1] + dy, (int64_t)c[2] + dz};
                    if (w[0] < 0 || w[1] < 0 || w[2] < 0 || w[0] >= (int64_t)G || w[1] >= (int64_t)G ||
                        w[2] >= (int64_t)G)
                        continue;
                    uint64_t zz = rgg3_morton(w, L);
                    if (zz >= z) nb[nn++] = zz;
                }
        qsort(nb, (size_t)nn, sizeof(uint64_t), cmp_u64r);
        for (uint64_t a = off[z]; a < off[z + 1]; a++)
            for (int i = 0; i < nn; i++)
                for (uint64_t b = off[nb[i]]; b < off[nb[i] + 1]; b++) {
                    if (b <= a || !rgg3_adjacent(&P[3 * a], &P[3 * b], r2)) continue;
                    if (edges && E < cap) { edges[2 * E] = (uint32_t)a; edges[2 * E + 1] = (uint32_t)b; }
                    E++;
                }
    }
    free(cells);
    free(off);
    if (!pts) free(P);
    return (int64_t)E;
}

/* The k points of cell z (3k doubles), as the whole generator makes them. */
void kgref_rgg3_cell_points(uint64_t n, double r, uint64_t seed, uint64_t z, uint64_t k, double *out)
{
    uint32_t L = kgref_rgg3_level(n, r);
    for (uint64_t j = 0; j < k; j++) rgg3_point(seed, L, z, j, &out[3 * j]);
}
