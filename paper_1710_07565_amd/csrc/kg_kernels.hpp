// kg_kernels.hpp -- the four kernels of one generation pass:
//   count  : each chunk recomputes its own edge count (root path of the
//            hypergeometric chunk tree, or one binomial per chunk),
//   scan   : exclusive prefix sums give every chunk its output offset,
//   plan   : each chunk's count is split over its tiles by a hypergeometric
//            tile tree, expanded level by level in LDS,
//   sample : one wavefront per tile draws its slots, sorts them in LDS,
//            decodes them to (u, v) and streams them out.
// All kernels read sizes from device memory, so one launch shape serves any
// instance list of the same bounds.
#pragma once
#include "kg_device.hpp"

namespace kg {

struct Job {
    uint32_t ninst;
    uint32_t leaf_cap;       // samples sorted per LDS pass, <= kCapMax
    uint64_t G;              // chunks over all instances
    uint64_t capacity;       // output room in edges
    uint64_t tile_cap;       // tile_off has tile_cap + 1 entries
    const Inst *insts;       // ninst > 1: device array
    Inst one;                // ninst == 1
    uint64_t *off;           // G + 1: counts, then exclusive offsets
    uint64_t *tstart;        // G + 1: tiles per chunk, then first tile
    uint64_t *ustart;        // G + 1: planner units per chunk, then first unit
    uint64_t *tile_off;      // output offset of every tile, + total
    uint64_t *status;        // [0] edges [1] overflow [2] tiles [3] units
    uint64_t *out_total;     // optional: edge total
    uint64_t *inst_off;      // optional: ninst + 1 instance offsets
    uint32_t *edges;
};

constexpr int kCapMax = 1024;            // LDS sort capacity of a wave

__device__ __forceinline__ const Inst &inst_at(const Job &job, uint32_t i)
{
    return job.ninst == 1 ? job.one : job.insts[i];
}

// instance owning global chunk g: last i with chunk_base <= g
__device__ __forceinline__ uint32_t inst_of_chunk(const Job &job, uint64_t g)
{
    if (job.ninst == 1) return 0;
    uint32_t lo = 0, hi = job.ninst;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (job.insts[mid].chunk_base <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// last index g in [0, G) with a[g] <= x, for nondecreasing a with a[G] > x
__device__ __forceinline__ uint64_t last_le(const uint64_t *a, uint64_t G, uint64_t x)
{
    uint64_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// lnf table: T[0] = 0, T[k] = T[k-1] + log k (sequential, one lane).
// ---------------------------------------------------------------------------
__global__ void lnf_init_kernel()
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    g_lnf_tab[0] = 0.0;
    for (uint32_t i = 1; i <= kLnfTab; ++i) {
        acc = acc + log_f64((double)i);
        g_lnf_tab[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// count: one lane per chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void count_kernel(Job job)
{
    const uint64_t g = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    if (g >= job.G) return;
    const uint32_t i = inst_of_chunk(job, g);
    const Inst &I = inst_at(job, i);
    const uint64_t c = g - I.chunk_base;
    const Chunk ch = chunk_geometry(I, c);
    uint64_t cnt;
    if (I.model == 1) {
        cnt = binom(make_stream(I.seed, (uint32_t)c, 0, TAG_CBIN), ch.N, I.p);
    } else if (I.directed) {
        cnt = dtree_count(I, c);
    } else {
        uint64_t lo = 0, hi = I.P;
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (uord(I.P, mid) <= c) lo = mid; else hi = mid;
        }
        cnt = utree_count(I, lo, lo + (c - uord(I.P, lo)));
    }
    const uint64_t T = tiles_of(ch.N, I.s);
    job.off[g] = cnt;
    job.tstart[g] = T;
    job.ustart[g] = T ? (1ull << unit_depth(T)) : 0;
}

// ---------------------------------------------------------------------------
// scan: one workgroup of 1024 lanes, exclusive scans of the three per-chunk
// arrays (each lane owns a contiguous segment), then the totals.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void scan_kernel(Job job)
{
    __shared__ uint64_t s_part[3][1024];
    const uint32_t t = threadIdx.x;
    const uint64_t G = job.G;
    const uint64_t seg = (G + 1023) / 1024;
    const uint64_t b0 = t * seg < G ? t * seg : G;
    const uint64_t b1 = b0 + seg < G ? b0 + seg : G;
    uint64_t sc = 0, st = 0, su = 0;
    for (uint64_t g = b0; g < b1; ++g) { sc += job.off[g]; st += job.tstart[g]; su += job.ustart[g]; }
    s_part[0][t] = sc; s_part[1][t] = st; s_part[2][t] = su;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        uint64_t a0 = 0, a1 = 0, a2 = 0;
        if (t >= d) { a0 = s_part[0][t - d]; a1 = s_part[1][t - d]; a2 = s_part[2][t - d]; }
        __syncthreads();
        s_part[0][t] += a0; s_part[1][t] += a1; s_part[2][t] += a2;
        __syncthreads();
    }
    uint64_t pc = t ? s_part[0][t - 1] : 0, pt = t ? s_part[1][t - 1] : 0, pu = t ? s_part[2][t - 1] : 0;
    for (uint64_t g = b0; g < b1; ++g) {
        const uint64_t c0 = job.off[g], t0 = job.tstart[g], u0 = job.ustart[g];
        job.off[g] = pc; job.tstart[g] = pt; job.ustart[g] = pu;
        pc += c0; pt += t0; pu += u0;
    }
    __syncthreads();
    if (t == 0) {
        const uint64_t E = s_part[0][1023], T = s_part[1][1023], U = s_part[2][1023];
        job.off[G] = E; job.tstart[G] = T; job.ustart[G] = U;
        const uint64_t overflow = (E > job.capacity || T > job.tile_cap) ? 1 : 0;
        job.status[0] = E; job.status[1] = overflow; job.status[2] = T; job.status[3] = U;
        if (T <= job.tile_cap) job.tile_off[T] = E;
        if (job.out_total) *job.out_total = E;
    }
}

// Instance offsets need the scanned array; a second tiny kernel keeps the
// scan free of a grid-wide dependency.
__global__ __launch_bounds__(256) void inst_offsets_kernel(Job job)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i > job.ninst) return;
    job.inst_off[i] = i == job.ninst ? job.off[job.G] : job.off[inst_at(job, i).chunk_base];
}

// ---------------------------------------------------------------------------
// plan: one wavefront per unit, a subtree of <= 256 tiles of one chunk's tile
// tree.  Lane 0 walks from the tile-tree root to the unit's root (the
// communication-free path); the wave then expands the subtree level by level.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void plan_kernel(Job job)
{
    __shared__ uint32_t s_lo[2][kUnitTiles], s_hi[2][kUnitTiles], s_heap[2][kUnitTiles];
    __shared__ uint64_t s_k[2][kUnitTiles];
    __shared__ uint64_t s_tc[kUnitTiles];
    __shared__ uint64_t s_root[4];
    const uint32_t lane = threadIdx.x;
    if (job.status[1]) return;
    const uint64_t U = job.status[3];
    const uint64_t G = job.G;
    for (uint64_t u = blockIdx.x; u < U; u += gridDim.x) {
        const uint64_t g = last_le(job.ustart, G, u);
        const Inst &I = inst_at(job, inst_of_chunk(job, g));
        const uint64_t c = g - I.chunk_base;
        const Chunk ch = chunk_geometry(I, c);
        const uint32_t s = I.s;
        const uint64_t T = tiles_of(ch.N, s);
        const uint64_t units = job.ustart[g + 1] - job.ustart[g];
        const uint32_t d = 63 - __clzll(units);
        const uint64_t j = u - job.ustart[g];
        if (lane == 0) {
            uint64_t lo = 0, hi = T, k = job.off[g + 1] - job.off[g], base = 0;
            uint32_t heap = 1;
            for (uint32_t lev = 0; lev < d; ++lev) {
                const uint64_t mid = lo + (hi - lo + 1) / 2;
                const uint64_t X = hyp(make_stream(I.seed, (uint32_t)c, heap, TAG_TTREE),
                                       tile_range_slots(lo, hi, s, ch.N), tile_range_slots(lo, mid, s, ch.N), k);
                if (((j >> (d - 1 - lev)) & 1) == 0) { hi = mid; k = X; heap = 2 * heap; }
                else { lo = mid; k = k - X; base += X; heap = 2 * heap + 1; }
            }
            s_root[0] = lo; s_root[1] = hi; s_root[2] = k; s_root[3] = base;
            s_lo[0][0] = 0; s_hi[0][0] = (uint32_t)(hi - lo); s_k[0][0] = k; s_heap[0][0] = heap;
        }
        __syncthreads();
        const uint64_t rlo = s_root[0], nt = s_root[1] - s_root[0], base = s_root[3];
        uint32_t cur = 0, cnt = 1;
        for (;;) {
            int internal = 0;
            for (uint32_t e = lane; e < cnt; e += 64) {
                const uint32_t a = s_lo[cur][e], b = s_hi[cur][e];
                const uint64_t kk = s_k[cur][e];
                const uint32_t h = s_heap[cur][e];
                uint32_t la = 0, lb = 0, ra = 0, rb = 0;
                uint64_t lk = 0, rk = 0;
                if (b - a == 1) {
                    s_tc[a] = kk;
                } else if (b - a > 1) {
                    const uint32_t mid = a + (b - a + 1) / 2;
                    const uint64_t X = hyp(make_stream(I.seed, (uint32_t)c, h, TAG_TTREE),
                                           tile_range_slots(rlo + a, rlo + b, s, ch.N),
                                           tile_range_slots(rlo + a, rlo + mid, s, ch.N), kk);
                    la = a; lb = mid; lk = X; ra = mid; rb = b; rk = kk - X;
                    internal = 1;
                }
                if (2 * e + 1 < kUnitTiles) {
                    s_lo[cur ^ 1][2 * e] = la; s_hi[cur ^ 1][2 * e] = lb; s_k[cur ^ 1][2 * e] = lk;
                    s_heap[cur ^ 1][2 * e] = 2 * h;
                    s_lo[cur ^ 1][2 * e + 1] = ra; s_hi[cur ^ 1][2 * e + 1] = rb; s_k[cur ^ 1][2 * e + 1] = rk;
                    s_heap[cur ^ 1][2 * e + 1] = 2 * h + 1;
                }
            }
            if (!__syncthreads_or(internal)) break;
            cur ^= 1;
            cnt *= 2;
        }
        // exclusive scan of the tile counts (4 per lane), then the offsets
        uint64_t v[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t tt = lane * 4 + q;
            v[q] = tt < nt ? s_tc[tt] : 0;
            sum += v[q];
        }
        uint64_t incl = sum;
#pragma unroll
        for (int dlt = 1; dlt < 64; dlt <<= 1) {
            const uint64_t o = __shfl_up(incl, dlt, 64);
            if (lane >= (uint32_t)dlt) incl += o;
        }
        uint64_t run = job.off[g] + base + (incl - sum);
        const uint64_t t0 = job.tstart[g] + rlo;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t tt = lane * 4 + q;
            if (tt < nt) job.tile_off[t0 + tt] = run;
            run += v[q];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// sample: wave-per-tile leaf sampling.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t lanemask_lt(uint32_t lane)
{
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Slot -> edge of one tile (Sec. 4.1 and 4.2 offset computations).
struct Decoder {
    uint32_t type;      // 0 directed, 1 rectangle, 2 triangle
    uint64_t dv;        // directed: n - 1; rectangle: section width
    double rcp;         // 1 / dv
    uint64_t u0, w0;    // directed: row and column offset of the tile start
    uint64_t a, b, c0;  // rectangle: first row, first column, column offset of the tile start
    uint64_t h, Ttri, lbase;  // triangle: section size, its slots, tile start

    __device__ __forceinline__ uint64_t fdiv(uint64_t x, uint64_t &rem) const
    {
        uint64_t q = (uint64_t)((double)x * rcp);
        int64_t r = (int64_t)(x - q * dv);
        if (r < 0) { --q; r += (int64_t)dv; }
        else if ((uint64_t)r >= dv) { ++q; r -= (int64_t)dv; }
        rem = (uint64_t)r;
        return q;
    }

    __device__ __forceinline__ uint2 operator()(uint32_t x) const
    {
        if (type == 0) {
            uint64_t r;
            const uint64_t q = fdiv(w0 + x, r);
            const uint64_t u = u0 + q;
            return make_uint2((uint32_t)u, (uint32_t)(r + (r >= u)));
        }
        if (type == 1) {
            uint64_t r;
            const uint64_t q = fdiv(c0 + x, r);
            return make_uint2((uint32_t)(a + q), (uint32_t)(b + r));
        }
        // triangle: rows counted from the bottom hold 1, 2, 3, ... slots
        const uint64_t l = lbase + x;
        const uint64_t lr = Ttri - 1 - l;
        uint64_t q = (uint64_t)((sqrt(8.0 * (double)lr + 1.0) - 1.0) * 0.5);
        while (q * (q + 1) / 2 > lr) --q;
        while ((q + 1) * (q + 2) / 2 <= lr) ++q;
        const uint64_t r = h - 2 - q;
        const uint64_t st = r * h - r * (r + 1) / 2;
        return make_uint2((uint32_t)(a + r), (uint32_t)(a + r + 1 + (l - st)));
    }
};

struct TileCtx {
    uint64_t S;         // slots of the tile
    uint32_t bits;      // ceil(log2 S)
    uint32_t mask;
    uint32_t full;      // S == 2^bits: no draw is rejected
    Stream st;          // (seed, chunk ordinal, tile, TLEAF)
    uint64_t o0;        // output offset of the tile
    uint32_t *edges;
    Decoder dec;
};

// wave-uniform values, kept in scalar registers
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x)
{
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}
__device__ __forceinline__ double unid(double x)
{
    return __longlong_as_double((long long)uni64((uint64_t)__double_as_longlong(x)));
}

__device__ __forceinline__ void store_edge(uint32_t *edges, uint64_t idx, uint2 e)
{
    *reinterpret_cast<uint2 *>(edges + 2 * idx) = e;
}

// word q of a Philox block
__device__ __forceinline__ uint32_t word_of(const U4 &w, int q)
{
    return q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
}

// Output the complement of the sorted excluded set ex[0..ne) within
// [rlo, rhi), ranks starting at r0; returns the number written.
__device__ uint64_t emit_complement(const TileCtx &t, const uint32_t *ex, uint32_t ne, uint64_t rlo,
                                    uint64_t rhi, uint64_t r0)
{
    const uint32_t lane = threadIdx.x;
    uint32_t e = 0;
    uint64_t out = 0;
    for (uint64_t base = rlo; base < rhi; base += 64) {
        const uint32_t ej = e + lane;
        uint64_t bit = 0;
        bool in = false;
        if (ej < ne) {
            const uint64_t xv = ex[ej];
            if (xv < base + 64) { in = true; bit = 1ull << (xv - base); }
        }
        const uint64_t msk = wave_or64(bit);
        e += __popcll(__ballot(in));
        const uint64_t p = base + lane;
        const uint64_t valid = __ballot(p < rhi);
        const uint64_t keepm = ~msk & valid;
        if ((keepm >> lane) & 1) store_edge(t.edges, t.o0 + r0 + out + __popcll(keepm & lanemask_lt(lane)),
                                            t.dec((uint32_t)p));
        out += __popcll(keepm);
    }
    return out;
}

// Sorted distinct valid draws lying in [rlo, rhi) among the first J draws of
// the tile's stream, left in s[0..n); returns n, or 0xFFFFFFFF when more
// than cap draws fall in the range.  Draw d is word d mod 4 of block d/4,
// masked to `bits` bits; values >= S are rejected.
//   1. blocks are generated 64 at a time (one per lane) and the kept words
//      appended to s[] in draw order by ballot prefix counts;
//   2. counting sort on the top bits of (x - rlo): LDS histogram (atomic
//      slot per key), exclusive scan, scatter back into s[];
//   3. each key's rank inside its bucket gives its sorted position
//      (ties broken by position, so repeats land next to each other);
//   4. repeats, if any, are squeezed out.
template <int CAP>
__device__ uint32_t collect_sorted(const TileCtx &t, uint32_t *s, uint32_t *hist, uint64_t J, uint64_t rlo,
                                   uint64_t rhi, uint32_t cap)
{
    constexpr int E = CAP / 64;          // kept keys per lane, at most
    const uint32_t lane = threadIdx.x;
    uint32_t n = 0;
    const uint64_t nblk = (J + 3) >> 2;
    for (uint64_t b0 = 0; b0 < nblk; b0 += 64) {
        const uint64_t blk = b0 + lane;
        U4 w{0, 0, 0, 0};
        if (blk < nblk) w = t.st.block((uint32_t)blk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t d = 4 * blk + q;
            const uint32_t x = word_of(w, q) & t.mask;
            const bool ok = d < J && (t.full || x < t.S) && x >= rlo && x < rhi;
            const uint64_t bal = __ballot(ok);
            const uint32_t pos = n + __popcll(bal & lanemask_lt(lane));
            if (ok && pos < cap) s[pos] = x;
            n += __popcll(bal);
        }
        if (n > cap) return 0xFFFFFFFFu;
    }
    if (n == 0) return 0;
    // bucket count: a power of two near n, at most CAP/2 and 2^(range bits)
    const uint64_t width = rhi - rlo;
    const uint32_t rbits = width <= 1 ? 0 : 64 - __clzll(width - 1);
    uint32_t nbb = n <= 1 ? 0 : 32 - __clz(n - 1);
    const uint32_t nbmax = 31 - __clz((uint32_t)(CAP / 2));
    if (nbb > nbmax) nbb = nbmax;
    if (nbb > rbits) nbb = rbits;
    const uint32_t NB = 1u << nbb;
    const uint32_t shift = rbits - nbb;
    for (uint32_t b = lane; b <= NB; b += 64) hist[b] = 0;
    __syncthreads();
    uint32_t xs[E], sl[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t p = lane + 64u * e;
        sl[e] = 0xFFFFFFFFu;
        xs[e] = 0;
        if (p < n) {
            xs[e] = s[p];
            sl[e] = atomicAdd(&hist[(uint32_t)((xs[e] - rlo) >> shift)], 1u);
        }
    }
    __syncthreads();
    {
        // exclusive scan of hist[0..NB)
        const uint32_t per = (NB + 63) / 64;
        const uint32_t h0 = lane * per;
        uint32_t sum = 0;
        for (uint32_t i = 0; i < per; ++i) if (h0 + i < NB) sum += hist[h0 + i];
        uint32_t incl = sum;
#pragma unroll
        for (int dlt = 1; dlt < 64; dlt <<= 1) {
            const uint32_t o = __shfl_up(incl, dlt, 64);
            if (lane >= (uint32_t)dlt) incl += o;
        }
        uint32_t run = incl - sum;
        for (uint32_t i = 0; i < per; ++i)
            if (h0 + i < NB) { const uint32_t v = hist[h0 + i]; hist[h0 + i] = run; run += v; }
        if (lane == 63) hist[NB] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (sl[e] != 0xFFFFFFFFu) s[hist[(uint32_t)((xs[e] - rlo) >> shift)] + sl[e]] = xs[e];
    __syncthreads();
    uint32_t ndup = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (sl[e] != 0xFFFFFFFFu) {
            const uint32_t x = xs[e];
            const uint32_t b = (uint32_t)((x - rlo) >> shift);
            const uint32_t st0 = hist[b], en = hist[b + 1], mp = st0 + sl[e];
            uint32_t rank = 0;
            uint32_t dup = 0;
            for (uint32_t jj = st0; jj < en; ++jj) {
                const uint32_t y = s[jj];
                const uint32_t eqb = (y == x) & (jj < mp);
                rank += (y < x) | eqb;
                dup |= eqb;
            }
            sl[e] = st0 + rank;
            ndup += dup;
        }
    }
    ndup = wave_sum32(ndup);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (sl[e] != 0xFFFFFFFFu) s[sl[e]] = xs[e];
    __syncthreads();
    if (ndup == 0) return n;
    // squeeze out repeats (they are adjacent)
    uint32_t kept = 0;
    for (uint32_t b0 = 0; b0 < n; b0 += 64) {
        const uint32_t p = b0 + lane;
        uint32_t x = 0;
        bool keep = false;
        if (p < n) {
            x = s[p];
            keep = p == 0 || s[p - 1] != x;
        }
        const uint64_t bal = __ballot(keep);
        __syncthreads();
        if (keep) s[kept + __popcll(bal & lanemask_lt(lane))] = x;
        kept += __popcll(bal);
        __syncthreads();
    }
    return kept;
}

// Base case of the sampler for one tile: the sorted set of k distinct slots
// of [0, S) obtained by drawing until k distinct values are seen (the draws
// that reach k distinct values are found by growing J: each draw adds at
// most one new value, so with D(J) < k distinct among J draws at least
// k - D(J) more draws are needed).  When 2k > S the S - k excluded slots are
// drawn instead and the complement is written.  Key sub-ranges keep every
// pass within the LDS capacity.
template <int CAP>
__device__ void leaf_sample(const TileCtx &t, uint32_t *s, uint32_t *hist, uint64_t k, uint32_t cap)
{
    const bool comp = 2 * k > t.S;
    const uint64_t ke = comp ? t.S - k : k;
    if (ke == 0) {
        emit_complement(t, s, 0, 0, t.S, 0);
        return;
    }
    const uint64_t span = 1ull << t.bits;
    uint64_t nsub = 1;
    while (nsub < span && nsub * cap < ke) nsub <<= 1;
    uint64_t J = ke;
    uint32_t last_n = 0;
    for (;;) {
        const uint64_t W = span / nsub;
        uint64_t D = 0;
        bool over = false;
        for (uint64_t sb = 0; sb < nsub; ++sb) {
            const uint32_t n = collect_sorted<CAP>(t, s, hist, J, sb * W, (sb + 1) * W, cap);
            if (n == 0xFFFFFFFFu) { over = true; break; }
            if (!comp) {
                // speculative: if D(J) < k these ranks are rewritten later,
                // and D(J) <= k keeps them inside the tile's output range
                for (uint32_t p = threadIdx.x; p < n; p += 64) store_edge(t.edges, t.o0 + D + p, t.dec(s[p]));
            }
            D += n;
            last_n = n;
            __syncthreads();
        }
        if (over) {
            __syncthreads();
            nsub <<= 1;
            continue;
        }
        if (D == ke) break;
        J += ke - D;
    }
    if (!comp) return;
    if (nsub == 1) {
        emit_complement(t, s, last_n, 0, t.S, 0);
        return;
    }
    const uint64_t W = span / nsub;
    uint64_t r = 0;
    for (uint64_t sb = 0; sb < nsub; ++sb) {
        const uint32_t n = collect_sorted<CAP>(t, s, hist, J, sb * W, (sb + 1) * W, cap);
        const uint64_t hi = (sb + 1) * W < t.S ? (sb + 1) * W : t.S;
        if (sb * W < hi) r += emit_complement(t, s, n, sb * W, hi, r);
        __syncthreads();
    }
}

template <int CAP>
__global__ __launch_bounds__(64) void sample_kernel(Job job)
{
    __shared__ uint32_t s_bkt[CAP];
    __shared__ uint32_t s_hist[CAP / 2 + 1];
    if (job.status[1]) return;
    const uint64_t T = job.status[2];
    const uint64_t W = gridDim.x;
    const uint64_t per = (T + W - 1) / W;
    const uint64_t t0 = (uint64_t)blockIdx.x * per;
    const uint64_t t1 = t0 + per < T ? t0 + per : T;
    uint64_t g = ~0ull, gend = 0, gstart = 0;
    Inst I;
    Chunk ch;
    uint64_t c = 0;
    for (uint64_t t = t0; t < t1; ++t) {
        const uint64_t o0 = job.tile_off[t];
        const uint64_t k = job.tile_off[t + 1] - o0;
        if (k == 0) continue;
        if (g == ~0ull || t >= gend) {
            g = last_le(job.tstart, job.G, t);
            gstart = job.tstart[g];
            gend = job.tstart[g + 1];
            I = inst_at(job, inst_of_chunk(job, g));
            c = g - I.chunk_base;
            ch = chunk_geometry(I, c);
        }
        const uint64_t tl = t - gstart;
        const uint32_t s = I.s;
        const uint64_t lstart = tl << s;
        TileCtx tc;
        tc.S = uni64((ch.N - lstart) < (1ull << s) ? (ch.N - lstart) : (1ull << s));
        tc.bits = uni(tc.S <= 1 ? 0 : 64 - __clzll(tc.S - 1));
        tc.mask = uni(tc.bits >= 32 ? 0xFFFFFFFFu : ((1u << tc.bits) - 1));
        tc.full = uni(tc.S == (1ull << tc.bits));
        tc.st = Stream{uni((uint32_t)I.seed), uni((uint32_t)(I.seed >> 32)), uni((uint32_t)c), uni((uint32_t)tl),
                       TAG_TLEAF};
        tc.o0 = uni64(o0);
        tc.edges = job.edges;
        Decoder &dd = tc.dec;
        dd.type = 0; dd.dv = 1; dd.rcp = 1.0; dd.u0 = dd.w0 = dd.a = dd.b = dd.c0 = dd.h = dd.Ttri = dd.lbase = 0;
        if (I.directed) {
            dd.type = 0;
            dd.dv = I.n - 1;
            dd.rcp = 1.0 / (double)dd.dv;
            const uint64_t bi = ch.row0 * dd.dv + lstart;
            dd.u0 = bi / dd.dv;
            dd.w0 = bi - dd.u0 * dd.dv;
        } else if (!ch.diag) {
            dd.type = 1;
            dd.dv = ch.w;
            dd.rcp = 1.0 / (double)dd.dv;
            const uint64_t r0 = lstart / ch.w;
            dd.c0 = lstart - r0 * ch.w;
            dd.a = ch.a + r0;
            dd.b = ch.b;
        } else {
            dd.type = 2;
            dd.h = ch.h;
            dd.a = ch.a;
            dd.Ttri = ch.N;
            dd.lbase = lstart;
        }
        dd.type = uni(dd.type);
        dd.dv = uni64(dd.dv); dd.rcp = unid(dd.rcp);
        dd.u0 = uni64(dd.u0); dd.w0 = uni64(dd.w0);
        dd.a = uni64(dd.a); dd.b = uni64(dd.b); dd.c0 = uni64(dd.c0);
        dd.h = uni64(dd.h); dd.Ttri = uni64(dd.Ttri); dd.lbase = uni64(dd.lbase);
        leaf_sample<CAP>(tc, s_bkt, s_hist, k, job.leaf_cap < CAP ? job.leaf_cap : CAP);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// element-wise evaluation of the building blocks (for parity checks)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void eval_kernel(int fn, const void *in, void *out, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    switch (fn) {
    case 1: {
        const uint32_t *r = (const uint32_t *)in + 6 * i;
        const U4 w = philox(r[0], r[1], r[2], r[3], r[4], r[5]);
        uint32_t *o = (uint32_t *)out + 4 * i;
        o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = w.w;
        break;
    }
    case 2: ((double *)out)[i] = log_f64(((const double *)in)[i]); break;
    case 3: ((double *)out)[i] = log1p_f64(((const double *)in)[i]); break;
    case 4: {
        const uint64_t *r = (const uint64_t *)in + 2 * i;
        ((double *)out)[i] = lnf_diff(r[0], r[1]);
        break;
    }
    case 5: {
        const uint64_t *r = (const uint64_t *)in + 6 * i;
        const Stream st = make_stream(r[3], (uint32_t)r[4], (uint32_t)(r[4] >> 32), (uint32_t)r[5]);
        ((uint64_t *)out)[i] = hyp(st, r[0], r[1], r[2]);
        break;
    }
    case 6: {
        const uint64_t *r = (const uint64_t *)in + 6 * i;
        const Stream st = make_stream(r[3], (uint32_t)r[4], (uint32_t)(r[4] >> 32), (uint32_t)r[5]);
        ((uint64_t *)out)[i] = binom(st, r[0], __longlong_as_double((long long)r[1]));
        break;
    }
    case 7: {
        const double *r = (const double *)in + 2 * i;
        double *o = (double *)out + 2 * i;
        o[0] = sqrt(r[0]);
        o[1] = r[0] / r[1];
        break;
    }
    default: break;
    }
}

}  // namespace kg
