// kg_device.hpp -- device building blocks of the generator: counter-based
// random streams, the binary64 logarithm kernel, hypergeometric and binomial
// variates, and the geometry of chunks, tiles and edge slots.
//
// Method: Funke et al., "Communication-free Massively Distributed Graph
// Generation" (arXiv 1710.07565).  Every recursion node draws from its own
// stream so that any chunk can recompute its sample size alone (Sec. 2.2);
// sample sizes of sub-universes are hypergeometric (Sec. 2.2) or binomial
// (Sec. 4.3); variates come from acceptance-rejection (Sec. 2.2).
//
// Bit reproducibility: only IEEE binary64 + - * / sqrt and exact conversions
// are used, in a fixed order, with contraction disabled at build time
// (-ffp-contract=off).  log is computed here from those operations; no
// device math library routine decides a variate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kg {

// ---------------------------------------------------------------------------
// Constants of the method
// ---------------------------------------------------------------------------
constexpr uint32_t kLambda = 560;       // tiles hold [560, 1120) samples in expectation (1024 at power-of-two densities)
constexpr uint32_t kUnitTiles = 64;     // most tiles of one planner unit (one lane expands it)
constexpr uint32_t kLnfTab = 1024;      // ln k! tabulated for k <= kLnfTab

enum : uint32_t { TAG_DTREE = 1, TAG_UTREE = 2, TAG_CBIN = 3, TAG_TTREE = 4, TAG_TLEAF = 5, TAG_INST = 6 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplications with the bijection keyed by (k0, k1), bumped by the Weyl
// constants between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__host__ __device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The same rounds for a key held in scalar registers (the same key in every
// lane of the wave): the three-way xor of a round is one v_bitop3_b32 (a
// three-input bitwise function given by its truth table; 0x96 is a ^ b ^ c)
// with the round key as its scalar operand.
__device__ __forceinline__ uint32_t xor3_sk(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// Philox4x32-10 of counter (a, j, b, tag) under a wave-uniform key, with a,
// b and tag wave-uniform and the block j per lane: the first round's products
// are both uniform, the second and third have one uniform product each, so
// they are formed by the scalar unit.
__device__ __forceinline__ U4 philox_wave(uint32_t a, uint32_t j, uint32_t b, uint32_t tag, uint32_t k0,
                                         uint32_t k1)
{
    uint32_t z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    k0 += z;
    k1 += z;
    // round 1: c0 = a, c1 = j, c2 = b, c3 = tag
    uint64_t p0 = (uint64_t)0xD2511F53u * a;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * b;
    uint32_t c0 = ((uint32_t)(p1 >> 32) ^ k0) ^ j;     // lane
    uint32_t c1 = (uint32_t)p1;                        // uniform
    uint32_t c2 = (uint32_t)(p0 >> 32) ^ tag ^ k1;     // uniform
    uint32_t c3 = (uint32_t)p0;                        // uniform
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // round 2: c0 lane, c2 uniform
    p0 = (uint64_t)0xD2511F53u * c0;
    p1 = (uint64_t)0xCD9E8D57u * c2;
    {
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;        // uniform
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);      // lane
        c1 = (uint32_t)p1;                                       // uniform
        c3 = (uint32_t)p0;                                       // lane
        c0 = n0;
        c2 = n2;
    }
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // round 3: c0 uniform, c2 lane
    p0 = (uint64_t)0xD2511F53u * c0;
    p1 = (uint64_t)0xCD9E8D57u * c2;
    {
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);      // lane
        const uint32_t n2 = c3 ^ ((uint32_t)(p0 >> 32) ^ k1);      // lane
        c1 = (uint32_t)p1;                                       // lane
        c3 = (uint32_t)p0;                                       // uniform
        c0 = n0;
        c2 = n2;
    }
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        p0 = (uint64_t)0xD2511F53u * c0;
        p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_sk((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = r == 3 ? (uint32_t)(p0 >> 32) ^ (c3 ^ k1) : xor3_sk((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// A random stream: Philox keyed by the seed, counter (a, block, b, tag).
struct Stream {
    uint32_t k0, k1, a, b, tag;
    __device__ __forceinline__ U4 block(uint32_t j) const { return philox(a, j, b, tag, k0, k1); }
    // only when k0, k1 are wave-uniform (scalar registers)
    __device__ __forceinline__ U4 block_uniform_key(uint32_t j) const
    {
        return philox_wave(a, j, b, tag, k0, k1);
    }
};

__device__ __forceinline__ Stream make_stream(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag)
{
    return Stream{(uint32_t)seed, (uint32_t)(seed >> 32), a, b, tag};
}

// Sequential 64-bit draws: draw d is (w1:w0) of block d/2 if d is even,
// (w3:w2) otherwise.
struct Draws64 {
    Stream s;
    uint64_t next;
    uint32_t cj;
    U4 buf;
    __device__ __forceinline__ explicit Draws64(const Stream &st) : s(st), next(0), cj(0xFFFFFFFFu), buf{0, 0, 0, 0} {}
    __device__ __forceinline__ uint64_t get()
    {
        const uint64_t d = next++;
        const uint32_t j = (uint32_t)(d >> 1);
        if (j != cj) { buf = s.block(j); cj = j; }
        return (d & 1) ? (((uint64_t)buf.w << 32) | buf.z) : (((uint64_t)buf.y << 32) | buf.x);
    }
};

// Top 52 bits plus half an ulp: exact, strictly inside (0, 1).
__device__ __forceinline__ double unit_of(uint64_t x)
{
    return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

// Uniform integer in [0, R) by power-of-two mask and rejection.
__device__ __forceinline__ uint64_t draw_below(Draws64 &d, uint64_t R)
{
    const uint64_t mask = R <= 1 ? 0ull : (~0ull >> __clzll(R - 1));
    for (;;) {
        const uint64_t x = d.get() & mask;
        if (x < R) return x;
    }
}

// ---------------------------------------------------------------------------
// Natural logarithm from + - * / (binary64).  x = 2^e f, f in [sqrt(1/2),
// sqrt(2)); with u = f - 1 (exact) and s = u / (2 + u),
//   log f = 2 atanh(s) = u - (u^2/2 - s (u^2/2 + R(s^2))),
//   R(z) = sum_{i=1..11} 2 z^i / (2i + 1)  (Horner, innermost term first);
// e ln 2 is added as e*hi (exact: hi has 32 fraction bits) and e*lo.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double atanh_series(double z)
{
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

__device__ __forceinline__ double log_f64(double x)
{
    const double kLn2Hi = 0x1.62e42fee00000p-1;
    const double kLn2Lo = 0x1.a39ef35793c76p-33;
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ffu) - 1023;
    const uint64_t mant = bits & 0x000FFFFFFFFFFFFFull;
    uint64_t fb;
    if (mant > 0x6A09E667F3BCDull) { fb = mant | (1022ull << 52); e += 1; }   // above sqrt(2)
    else                           { fb = mant | (1023ull << 52); }
    const double f = __longlong_as_double((long long)fb);
    const double u = f - 1.0;
    const double s = u / (2.0 + u);
    const double z = s * s;
    const double R = atanh_series(z);
    const double hfsq = 0.5 * u * u;
    const double dk = (double)e;
    return dk * kLn2Hi - ((hfsq - (s * (hfsq + R) + dk * kLn2Lo)) - u);
}

__device__ __forceinline__ double log1p_f64(double x)
{
    if (x > -0.25 && x < 0.25) {
        const double s = x / (2.0 + x);
        const double z = s * s;
        const double R = atanh_series(z);
        const double hfsq = 0.5 * x * x;
        return x - (hfsq - s * (hfsq + R));
    }
    return log_f64(1.0 + x);
}

// ---------------------------------------------------------------------------
// ln k!: table T[k] = T[k-1] + log k for k <= 1024 (built on the device by
// kg_lnf_init_kernel); above it only differences are needed, from Stirling's
// series with three correction terms in z = k + 1:
//   lnf(a+d) - lnf(a) = (z - 1/2) log1p(d/z) + d (log(z + d) - 1)
//                       + corr(z + d) - corr(z),
//   corr(z) = 1/(12 z) - 1/(360 z^3) + 1/(1260 z^5),
// so that two large log-factorials are never subtracted.
// ---------------------------------------------------------------------------
extern __device__ double g_lnf_tab[kLnfTab + 1];

__device__ __forceinline__ double stirling_corr(double z)
{
    const double r = 1.0 / z;
    const double r2 = r * r;
    return r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0)));
}

__device__ __forceinline__ double stirling_diff(uint64_t a, uint64_t d)
{
    const double z = (double)(a + 1);
    const double zd = (double)(a + d + 1);
    const double dd = (double)d;
    const double t1 = (z - 0.5) * log1p_f64(dd / z);
    const double t2 = dd * (log_f64(zd) - 1.0);
    const double t3 = stirling_corr(zd) - stirling_corr(z);
    return (t1 + t2) + t3;
}

// lnf(y) - lnf(x).  Both cases above the table go through one Stirling
// difference (lanes of a wave often differ in the case): from x itself, or
// from the end of the table with the tabulated part below it added; in the
// first case the added part is +0.0, which leaves the value unchanged.
__device__ __forceinline__ double lnf_diff(uint64_t x, uint64_t y)
{
    if (x == y) return 0.0;
    const bool neg = x > y;
    const uint64_t lo = neg ? y : x, hi = neg ? x : y;
    double r;
    if (hi <= kLnfTab) {
        r = g_lnf_tab[hi] - g_lnf_tab[lo];
    } else {
        const bool part = lo < kLnfTab;
        const uint64_t a = part ? (uint64_t)kLnfTab : lo;
        const double tp = part ? g_lnf_tab[kLnfTab] - g_lnf_tab[part ? lo : 0] : 0.0;
        r = tp + stirling_diff(a, hi - a);
    }
    return neg ? -r : r;
}

// floor(a * b / d) for a*b < 2^106, d >= 1, exactly: estimate in binary64,
// correct with 128-bit products.
__device__ __forceinline__ uint64_t muldiv_floor(uint64_t a, uint64_t b, uint64_t d)
{
    typedef unsigned __int128 u128;
    const u128 num = (u128)a * b;
    double est = floor(((double)a * (double)b) / (double)d);
    uint64_t q = est <= 0.0 ? 0ull : (uint64_t)est;
    while ((u128)q * d > num) --q;
    while ((u128)(q + 1) * d <= num) ++q;
    return q;
}

// ---------------------------------------------------------------------------
// Discrete ratio of uniforms (Kinderman-Monahan; centre mu + 1/2 and
// half-width (D1 sqrt(var + 1/2) + D2)/2 as in Stadlober's samplers).
// Proposal j uses block j: U from (w1:w0), V from (w3:w2);
// X = floor(a + h (V - 1/2) / U), accepted iff 2 log U <= log f(X)/f(M),
// with the squeezes 4U - U^2 - 3 <= T (accept) and T <= U - 1/U (reject).
// ---------------------------------------------------------------------------
constexpr double kRouD1 = 0x1.b72cd3f331398p+0;   // 2 sqrt(2/e)
constexpr double kRouD2 = 0x1.cc3ebd3bc711ap-1;   // 3 - 2 sqrt(3/e)

// log f(x) - log f(M) of the hypergeometric law.
struct HypRatio {
    uint64_t N, K, k, M;
    __device__ __forceinline__ double operator()(uint64_t X) const
    {
        double T = lnf_diff(X, M);
        T = T + lnf_diff(k - X, k - M);
        T = T + lnf_diff(K - X, K - M);
        T = T + lnf_diff(N - K - k + X, N - K - k + M);
        return T;
    }
    // the t-th difference of the sum above, and the sum in the same order
    __device__ __forceinline__ double term(uint32_t t, uint64_t X) const
    {
        const uint64_t b = t == 0 ? 0 : t == 1 ? k : t == 2 ? K : N - K - k;
        const bool up = t == 0 || t == 3;
        return lnf_diff(up ? b + X : b - X, up ? b + M : b - M);
    }
    __device__ __forceinline__ double combine(double d0, double d1, double d2, double d3, uint64_t) const
    {
        return ((d0 + d1) + d2) + d3;
    }
};

// log f(x) - log f(M) of the binomial law; lq = log p - log(1-p).
struct BinRatio {
    uint64_t N, M;
    double lq;
    __device__ __forceinline__ double operator()(uint64_t X) const
    {
        double T = lnf_diff(X, M);
        T = T + lnf_diff(N - X, N - M);
        T = T + ((double)X - (double)M) * lq;
        return T;
    }
    __device__ __forceinline__ double term(uint32_t t, uint64_t X) const
    {
        const bool up = t != 1;
        const uint64_t b = t == 1 ? N : 0;
        return t < 2 ? lnf_diff(up ? b + X : b - X, up ? b + M : b - M) : 0.0;
    }
    __device__ __forceinline__ double combine(double d0, double d1, double, double, uint64_t X) const
    {
        return (d0 + d1) + ((double)X - (double)M) * lq;
    }
};

// Broadcast within aligned lane groups of G = 2 or 4 lanes: the value of lane
// T of each group, to the whole group (DPP quad_perm; the group's lanes are
// active together).
template <int G, int T>
__device__ __forceinline__ double group_bcast(double v)
{
    static_assert((G == 2 && T < 2) || (G == 4 && T < 4), "lane within a group of 2 or 4");
    constexpr int ctrl = G == 4 ? T * 0x55 : (T | T << 2 | (T + 2) << 4 | (T + 2) << 6);
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, ctrl, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// PAR = 1, TERMS = 1: one proposal at a time in one lane.  Otherwise an
// aligned group of PAR * TERMS lanes works on one variate (the same
// arguments in every lane of the group): it tries proposals j0 .. j0 + PAR - 1
// at once, and with TERMS = 2 or 4 the four log-factorial differences of a
// proposal's ratio are spread over TERMS lanes (lane t forms differences t,
// t + TERMS, ...) and summed in the sequential order.  The lowest accepted proposal wins, so the variate is
// the one the sequential loop returns.  Used where a variate's latency, not
// the lanes' throughput, bounds a kernel.
template <int PAR, int TERMS, class Ratio>
__device__ __forceinline__ uint64_t rou_sample(const Stream &s, double a, double h, uint64_t upper,
                                               const Ratio &ratio)
{
    static_assert(PAR == 1 || PAR == 2 || PAR == 4 || PAR == 8, "1, 2, 4 or 8 proposals at once");
    static_assert(TERMS == 1 || TERMS == 2 || TERMS == 4, "ratio in one, two or four lanes");
    constexpr uint32_t GL = PAR * TERMS;     // lanes per variate
    const double upper_excl = (double)upper + 1.0;
    const uint32_t lane = __lane_id();
    const uint32_t q = (lane & (GL - 1)) / TERMS;
    const uint32_t tq = lane & (TERMS - 1);
    for (uint32_t j0 = 0;; j0 += PAR) {
        const U4 w = s.block(j0 + q);
        const double U = unit_of(((uint64_t)w.y << 32) | w.x);
        const double V = unit_of(((uint64_t)w.w << 32) | w.z);
        const double t = a + h * (V - 0.5) / U;
        bool acc = false;
        uint64_t X = 0;
        if (t >= 0.0 && t < upper_excl) {
            X = (uint64_t)floor(t);
            if (X <= upper) {           // upper + 1 rounds in binary64 above 2^53
                double T;
                if (TERMS == 1) {
                    T = ratio(X);
                } else if (TERMS == 2) {
                    const double da = ratio.term(tq, X), db = ratio.term(tq + 2, X);
                    T = ratio.combine(group_bcast<2, 0>(da), group_bcast<2, 1>(da), group_bcast<2, 0>(db),
                                      group_bcast<2, 1>(db), X);
                } else {
                    const double d = ratio.term(tq, X);
                    T = ratio.combine(group_bcast<4, 0>(d), group_bcast<4, 1>(d), group_bcast<4, 2>(d),
                                      group_bcast<4, 3>(d), X);
                }
                if (U * (4.0 - U) - 3.0 <= T) acc = true;
                else if (U * (U - T) >= 1.0) acc = false;
                else acc = 2.0 * log_f64(U) <= T;
            }
        }
        if (GL == 1) {
            if (acc) return X;
        } else {
            const uint32_t base = lane & ~(GL - 1);
            const uint32_t won = (uint32_t)(__ballot(acc) >> base) & (uint32_t)((1ull << GL) - 1);
            if (won) {
                const int src = (int)(base + __builtin_ctz(won));
                const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)X, src);
                const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(X >> 32), src);
                return ((uint64_t)hi << 32) | lo;
            }
        }
    }
}

// Hypergeometric: how many of k draws without replacement from N items land
// among K marked ones (the sample size of a sub-universe, Sec. 2.2).
template <int PAR = 1, int TERMS = 1>
__device__ __forceinline__ uint64_t hyp(const Stream &s, uint64_t N, uint64_t K, uint64_t k)
{
    // symmetries: complement the draws, complement the marked set, swap roles
    uint64_t k1 = k, K1 = K;
    bool c1 = false, c2 = false;
    if (k1 > N - k1) { k1 = N - k1; c1 = true; }
    if (K1 > N - K1) { K1 = N - K1; c2 = true; }
    const uint64_t lo = k1 < K1 ? k1 : K1;   // draws
    const uint64_t hi = k1 < K1 ? K1 : k1;   // marked
    uint64_t x;
    if (lo == 0) {
        x = 0;
    } else if (lo <= 16) {
        // direct simulation: the i-th draw picks one of the N - i items left
        Draws64 d(s);
        x = 0;
        for (uint64_t i = 0; i < lo; ++i)
            if (draw_below(d, N - i) < hi - x) ++x;
    } else {
        const double Nd = (double)N, Kd = (double)hi, kd = (double)lo;
        const double pp = Kd / Nd;
        const double mu = kd * pp;
        const double var = (((Nd - kd) * kd) * pp) * (1.0 - pp) / (Nd - 1.0);
        const double c = sqrt(var + 0.5);
        const double h = kRouD1 * c + kRouD2;
        const double a = mu + 0.5;
        HypRatio r{N, hi, lo, muldiv_floor(lo + 1, hi + 1, N + 2)};
        x = rou_sample<PAR, TERMS>(s, a, h, lo, r);
    }
    if (c2) x = k1 - x;
    if (c1) x = K - x;
    return x;
}

// The same hypergeometric variate as hyp(), consumed one ratio-of-uniforms
// proposal per step() so that lanes of a wave working on different variates
// do not wait for each other's rejection loops.  Identical draws and result.
struct HypRun {
    Stream s;
    uint64_t N, K, k1, hi, lo, M, x;
    double a, h, upper_excl;
    uint32_t j;
    bool c1, c2, done;

    __device__ __forceinline__ void init(const Stream &st, uint64_t N_, uint64_t K_, uint64_t k)
    {
        s = st;
        N = N_;
        K = K_;
        k1 = k;
        uint64_t K1 = K_;
        c1 = c2 = false;
        if (k1 > N - k1) { k1 = N - k1; c1 = true; }
        if (K1 > N - K1) { K1 = N - K1; c2 = true; }
        lo = k1 < K1 ? k1 : K1;
        hi = k1 < K1 ? K1 : k1;
        j = 0;
        done = true;
        if (lo == 0) {
            x = 0;
        } else if (lo <= 16) {
            Draws64 d(s);
            x = 0;
            for (uint64_t i = 0; i < lo; ++i)
                if (draw_below(d, N - i) < hi - x) ++x;
        } else {
            const double Nd = (double)N, Kd = (double)hi, kd = (double)lo;
            const double pp = Kd / Nd;
            const double mu = kd * pp;
            const double var = (((Nd - kd) * kd) * pp) * (1.0 - pp) / (Nd - 1.0);
            const double c = sqrt(var + 0.5);
            h = kRouD1 * c + kRouD2;
            a = mu + 0.5;
            M = muldiv_floor(lo + 1, hi + 1, N + 2);
            upper_excl = (double)lo + 1.0;
            done = false;
        }
    }

    // one proposal; true once the variate is known.  TERMS = 2 or 4: the
    // aligned group of TERMS lanes holding the same state forms the ratio's
    // four differences together (same value in every lane of the group).
    template <int TERMS = 1>
    __device__ __forceinline__ bool step()
    {
        if (done) return true;
        const U4 w = s.block(j++);
        const double U = unit_of(((uint64_t)w.y << 32) | w.x);
        const double V = unit_of(((uint64_t)w.w << 32) | w.z);
        const double t = a + h * (V - 0.5) / U;
        if (!(t >= 0.0) || t >= upper_excl) return false;
        const uint64_t X = (uint64_t)floor(t);
        if (X > lo) return false;
        const HypRatio ratio{N, hi, lo, M};
        double T;
        if (TERMS == 1) {
            T = ratio(X);
        } else if (TERMS == 2) {
            const uint32_t tq = __lane_id() & 1;
            const double da = ratio.term(tq, X), db = ratio.term(tq + 2, X);
            T = ratio.combine(group_bcast<2, 0>(da), group_bcast<2, 1>(da), group_bcast<2, 0>(db),
                              group_bcast<2, 1>(db), X);
        } else {
            const double d = ratio.term(__lane_id() & 3, X);
            T = ratio.combine(group_bcast<4, 0>(d), group_bcast<4, 1>(d), group_bcast<4, 2>(d),
                              group_bcast<4, 3>(d), X);
        }
        bool acc = false;
        if (U * (4.0 - U) - 3.0 <= T) acc = true;
        else if (U * (U - T) >= 1.0) acc = false;
        else acc = 2.0 * log_f64(U) <= T;
        if (acc) { x = X; done = true; }
        return done;
    }

    __device__ __forceinline__ uint64_t result() const
    {
        uint64_t r = x;
        if (c2) r = k1 - r;
        if (c1) r = K - r;
        return r;
    }
};

// Binomial(N, p): a G(n,p) chunk's edge count (Sec. 4.3).  Small means by
// geometric waiting times floor(log U / log(1-p)); otherwise ratio of uniforms.
template <int PAR = 1, int TERMS = 1>
__device__ __forceinline__ uint64_t bin_core(const Stream &s, uint64_t N, double p)
{
    const double Nd = (double)N;
    if (Nd * p < 16.0) {
        const double L = log1p_f64(-p);
        Draws64 d(s);
        uint64_t X = 0, pos = 0;
        for (;;) {
            const double U = unit_of(d.get());
            const double g = floor(log_f64(U) / L);
            if (g >= (double)(N - pos)) return X;
            pos += (uint64_t)g + 1;
            ++X;
        }
    }
    const double q = 1.0 - p;
    const double mu = Nd * p;
    const double var = mu * q;
    const double c = sqrt(var + 0.5);
    const double h = kRouD1 * c + kRouD2;
    const double a = mu + 0.5;
    BinRatio r{N, (uint64_t)floor((Nd + 1.0) * p), log_f64(p) - log1p_f64(-p)};
    return rou_sample<PAR, TERMS>(s, a, h, N, r);
}

template <int PAR = 1, int TERMS = 1>
__device__ __forceinline__ uint64_t binom(const Stream &s, uint64_t N, double p)
{
    if (N == 0 || p <= 0.0) return 0;
    if (p >= 1.0) return N;
    if (p > 0.5) return N - bin_core<PAR, TERMS>(s, N, 1.0 - p);
    return bin_core<PAR, TERMS>(s, N, p);
}

// ---------------------------------------------------------------------------
// Instances and chunk geometry (Sec. 4.1 row chunks; Sec. 4.2 sections and
// the upper-triangular chunk matrix, ordered row-major).
// ---------------------------------------------------------------------------
struct Inst {
    uint64_t n, m;
    double p;
    uint64_t seed;
    uint32_t model, directed, P, s;   // s: tile exponent, tiles of 2^s slots
    uint64_t nchunks;                 // chunks generated: P (directed) or P(P+1)/2; 1 or P for a view
    uint64_t chunk_base;              // first global chunk index of the instance
    uint32_t view;                    // 0: the whole graph; r + 1: the edges incident to section r
    uint32_t pad_;
};

__host__ __device__ __forceinline__ uint64_t section_bound(const Inst &I, uint64_t i)
{
    // floor(i n / P); i n < 2^64 because i <= P <= 2^31 and n <= 2^32
    return (i * I.n) / I.P;
}

__host__ __device__ __forceinline__ uint64_t uord(uint64_t P, uint64_t i)
{
    return i * P - i * (i - 1) / 2;   // ordinal of diagonal chunk (i, i)
}

struct Chunk {
    uint64_t N;       // slots
    uint64_t row0;    // directed: first row
    uint64_t a, h;    // undirected: row section start / size
    uint64_t b, w;    // undirected: column section start / size
    uint32_t diag;    // undirected triangle chunk
};

// Ordinal (in the instance's canonical chunk order) of the instance's k-th
// generated chunk.  A view of section r (the per-PE partition of Sec. 4.1
// and 4.2) generates, directed, row chunk r alone; undirected, the chunks
// (i, r) for i < r and (r, j) for j >= r of the upper-triangular chunk
// matrix, in canonical order -- every edge with an endpoint in section r.
__host__ __device__ __forceinline__ uint64_t chunk_ordinal(const Inst &I, uint64_t k)
{
    if (I.view == 0) return k;
    const uint64_t r = I.view - 1;
    if (I.directed) return r;
    return k < r ? uord(I.P, k) + (r - k) : uord(I.P, r) + (k - r);
}

__device__ __forceinline__ Chunk chunk_geometry(const Inst &I, uint64_t c)
{
    Chunk g;
    g.diag = 0; g.a = g.h = g.b = g.w = 0; g.row0 = 0;
    if (I.directed) {
        g.row0 = section_bound(I, c);
        g.N = (section_bound(I, c + 1) - g.row0) * (I.n - 1);
        return g;
    }
    // row of the chunk matrix: largest i with uord(i) <= c
    uint64_t lo = 0, hi = I.P;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (uord(I.P, mid) <= c) lo = mid; else hi = mid;
    }
    const uint64_t ci = lo, cj = lo + (c - uord(I.P, lo));
    g.a = section_bound(I, ci); g.h = section_bound(I, ci + 1) - g.a;
    g.b = section_bound(I, cj); g.w = section_bound(I, cj + 1) - g.b;
    g.diag = ci == cj;
    g.N = g.diag ? g.h * (g.h - (g.h > 0)) / 2 : g.h * g.w;
    return g;
}

// Tiles of chunk with N slots; planner units (subtrees of <= kUnitTiles
// tiles): 2^d with d minimal such that ceil(T / 2^d) <= kUnitTiles.
__device__ __forceinline__ uint64_t tiles_of(uint64_t N, uint32_t s)
{
    return (N + ((1ull << s) - 1)) >> s;
}

__device__ __forceinline__ uint32_t unit_depth(uint64_t T, uint32_t ulog)
{
    uint32_t d = 0;
    while (((T + (1ull << d) - 1) >> d) > (1ull << ulog)) ++d;
    return d;
}

// ---------------------------------------------------------------------------
// Chunk counts by walking one root-to-leaf path (what a single PE does in the
// paper; Sec. 2.2, 4.1, 4.2).  The split of a range [lo, hi) of chunks or
// sections is at lo + ceil((hi - lo)/2).
// ---------------------------------------------------------------------------
template <int PAR = 1, int TERMS = 1>
__device__ __forceinline__ uint64_t dtree_count(const Inst &I, uint64_t c)
{
    uint64_t k = I.m, lo = 0, hi = I.P;
    uint32_t heap = 1;
    const uint64_t w = I.n - 1;
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        const uint64_t blo = section_bound(I, lo);
        const uint64_t Nn = (section_bound(I, hi) - blo) * w;
        const uint64_t Nl = (section_bound(I, mid) - blo) * w;
        const uint64_t X = hyp<PAR, TERMS>(make_stream(I.seed, heap, 0, TAG_DTREE), Nn, Nl, k);
        if (c < mid) { hi = mid; k = X; heap = 2 * heap; }
        else         { lo = mid; k = k - X; heap = 2 * heap + 1; }
    }
    return k;
}

__device__ __forceinline__ uint64_t tri_slots(const Inst &I, uint64_t a, uint64_t b)
{
    const uint64_t A = section_bound(I, b) - section_bound(I, a);
    return A * (A - (A > 0)) / 2;
}

__device__ __forceinline__ uint64_t rect_slots(const Inst &I, uint64_t a, uint64_t b, uint64_t c, uint64_t d)
{
    return (section_bound(I, b) - section_bound(I, a)) * (section_bound(I, d) - section_bound(I, c));
}

template <int PAR = 1, int TERMS = 1>
__device__ __forceinline__ uint64_t utree_count(const Inst &I, uint64_t ci, uint64_t cj)
{
    uint64_t k = I.m, a = 0, b = I.P, cc = 0, d = 0;
    uint32_t code = 1;
    bool tri = true;
    for (;;) {
        if (tri) {
            if (b - a == 1) return k;
            const uint64_t l = a + (b - a + 1) / 2;
            const uint64_t Nn = tri_slots(I, a, b), N1 = tri_slots(I, a, l), NR = rect_slots(I, a, l, l, b);
            const uint64_t X0 = hyp<PAR, TERMS>(make_stream(I.seed, code, 0, TAG_UTREE), Nn, N1, k);
            if (cj < l) { b = l; k = X0; code = 4 * code; continue; }
            const uint64_t X1 = hyp<PAR, TERMS>(make_stream(I.seed, code, 1, TAG_UTREE), Nn - N1, NR, k - X0);
            if (ci < l) { tri = false; cc = l; d = b; b = l; k = X1; code = 4 * code + 1; continue; }
            a = l; k = k - X0 - X1; code = 4 * code + 2;
            continue;
        }
        if (b - a == 1 && d - cc == 1) return k;
        const uint64_t Nn = rect_slots(I, a, b, cc, d);
        if (d - cc == 1) {
            const uint64_t l = a + (b - a + 1) / 2;
            const uint64_t X = hyp<PAR, TERMS>(make_stream(I.seed, code, 0, TAG_UTREE), Nn, rect_slots(I, a, l, cc, d), k);
            if (ci < l) { b = l; k = X; code = 4 * code; }
            else        { a = l; k = k - X; code = 4 * code + 1; }
            continue;
        }
        if (b - a == 1) {
            const uint64_t q = cc + (d - cc + 1) / 2;
            const uint64_t X = hyp<PAR, TERMS>(make_stream(I.seed, code, 0, TAG_UTREE), Nn, rect_slots(I, a, b, cc, q), k);
            if (cj < q) { d = q; k = X; code = 4 * code; }
            else        { cc = q; k = k - X; code = 4 * code + 1; }
            continue;
        }
        const uint64_t l = a + (b - a + 1) / 2, q = cc + (d - cc + 1) / 2;
        const uint64_t N00 = rect_slots(I, a, l, cc, q), N01 = rect_slots(I, a, l, q, d);
        const uint64_t N10 = rect_slots(I, l, b, cc, q);
        const uint32_t quad = (ci >= l ? 2u : 0u) + (cj >= q ? 1u : 0u);
        const uint64_t X00 = hyp<PAR, TERMS>(make_stream(I.seed, code, 0, TAG_UTREE), Nn, N00, k);
        uint64_t X01 = 0, X10 = 0;
        if (quad >= 1) X01 = hyp<PAR, TERMS>(make_stream(I.seed, code, 1, TAG_UTREE), Nn - N00, N01, k - X00);
        if (quad >= 2) X10 = hyp<PAR, TERMS>(make_stream(I.seed, code, 2, TAG_UTREE), Nn - N00 - N01, N10, k - X00 - X01);
        const uint64_t kk = quad == 0 ? X00 : quad == 1 ? X01 : quad == 2 ? X10 : k - X00 - X01 - X10;
        if (quad < 2) b = l; else a = l;
        if (quad & 1) cc = q; else d = q;
        k = kk;
        code = 4 * code + quad;
    }
}

// Slots of tile range [lo, hi) of a chunk with Nc slots.
__device__ __forceinline__ uint64_t tile_range_slots(uint64_t lo, uint64_t hi, uint32_t s, uint64_t Nc)
{
    const uint64_t e = hi << s;
    return (e > Nc ? Nc : e) - (lo << s);
}

}  // namespace kg
