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
    uint32_t fast_cap;       // draws of the register base case (tile_kernel); larger tiles are queued
    uint32_t unit_log;       // planner units hold <= 2^unit_log tiles (launch shape only)
    uint64_t G;              // chunks over all instances
    uint64_t capacity;       // output room in edges
    uint64_t tile_cap;       // tile_off has tile_cap + 1 entries
    const Inst *insts;       // ninst > 1: device array
    Inst one;                // ninst == 1
    uint64_t *off;           // G + 1: counts, then exclusive offsets
    uint64_t *tstart;        // G + 1: tiles per chunk, then first tile
    uint64_t *ustart;        // G + 1: planner units per chunk, then first unit
    uint64_t *bsum;          // 3 x (G / 64 rounded up): per 64 chunks the sums of
                             // off, tstart, ustart, then their exclusive prefixes
    uint64_t *tile_off;      // output offset of every tile, + total
    uint64_t *status;        // [0] edges [1] overflow [2] tiles [3] units [4] queued tiles [5] tile ranges handed out
    uint64_t *queue;         // tile_cap entries: tiles left to the general base case
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

// Inclusive sum over the 64 lanes of a wave (shuffles up by 1, 2, ..., 32).
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v)
{
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

// ---------------------------------------------------------------------------
// count: a group of PAR * TERMS lanes per chunk, a workgroup per 64 chunks.
// The count of a chunk is a root path of dependent variates (Sec. 4.1, 4.2)
// or one binomial (Sec. 4.3), so the kernel's time is the latency of that
// chain: the lanes of a chunk try PAR ratio-of-uniforms proposals of each
// variate at once and, with TERMS = 4, form each proposal's log-factorial
// differences in four lanes (the first accepted proposal in proposal order
// wins, so the counts are those of the one-proposal loop).  Writes the
// chunk's edge count, tile count and planner-unit count, and the workgroup's
// three sums to bsum (the first phase of the offset scan).
// ---------------------------------------------------------------------------
template <int PAR, int TERMS>
__global__ __launch_bounds__(64 * PAR * TERMS) void count_kernel(Job job)
{
    constexpr int kCountPar = PAR, kCountTerms = TERMS;
    constexpr int kCountLanes = PAR * TERMS, kCountWaves = PAR * TERMS;   // 64 chunks per workgroup
    __shared__ uint64_t s_sum[kCountWaves][3];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t g = (uint64_t)blockIdx.x * 64 + threadIdx.x / kCountLanes;
    const bool lead = (threadIdx.x & (kCountLanes - 1)) == 0;
    uint64_t cnt = 0, T = 0, Us = 0;
    if (g < job.G) {
        const uint32_t i = inst_of_chunk(job, g);
        const Inst &I = inst_at(job, i);
        const uint64_t c = chunk_ordinal(I, g - I.chunk_base);
        const Chunk ch = chunk_geometry(I, c);
        if (I.model == 1) {
            cnt = binom<kCountPar, kCountTerms>(make_stream(I.seed, (uint32_t)c, 0, TAG_CBIN), ch.N, I.p);
        } else if (I.directed) {
            cnt = dtree_count<kCountPar, kCountTerms>(I, c);
        } else {
            uint64_t lo = 0, hi = I.P;
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) >> 1;
                if (uord(I.P, mid) <= c) lo = mid; else hi = mid;
            }
            cnt = utree_count<kCountPar, kCountTerms>(I, lo, lo + (c - uord(I.P, lo)));
        }
        T = tiles_of(ch.N, I.s);
        Us = T ? (1ull << unit_depth(T, job.unit_log)) : 0;
        if (lead) {
            job.off[g] = cnt;
            job.tstart[g] = T;
            job.ustart[g] = Us;
        }
    }
    if (!lead) cnt = T = Us = 0;
    const uint64_t sc = wave_incl_scan64(cnt), st = wave_incl_scan64(T), su = wave_incl_scan64(Us);
    if (lane == 63) {
        s_sum[wv][0] = sc;
        s_sum[wv][1] = st;
        s_sum[wv][2] = su;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const uint32_t a = threadIdx.x;
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < kCountWaves; ++w) t += s_sum[w][a];
        const uint64_t nb = (job.G + 63) / 64;
        job.bsum[a * nb + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// scan, second phase: one workgroup of 1024 lanes turns the wave sums into
// exclusive prefixes in rounds of 4096 entries (four consecutive entries per
// lane, coalesced): per-lane sums, wave scans, a scan of the 16 wave totals,
// a running carry.  The next round's entries are loaded before the current
// round is scanned.  It also writes the totals and the status words.
// Third phase (fix_kernel): every chunk adds its wave's prefix to the
// in-wave prefix of its own values.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void scan_kernel(Job job)
{
    __shared__ uint64_t s_wave[3][16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint64_t G = (job.G + 63) / 64;     // wave sums to scan
    uint64_t *arr[3] = {job.bsum, job.bsum + G, job.bsum + 2 * G};
    uint64_t carry[3] = {0, 0, 0};
    uint64_t cur[3][4], nxt[3][4];
    auto load = [&](uint64_t base, uint64_t (&dst)[3][4]) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t g = base + 4 * (uint64_t)t + i;
                dst[a][i] = g < G ? arr[a][g] : 0;
            }
    };
    load(0, cur);
    for (uint64_t base = 0; base < G; base += 4096) {
        if (base + 4096 < G) load(base + 4096, nxt);
        uint64_t incl[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint64_t sum = cur[a][0] + cur[a][1] + cur[a][2] + cur[a][3];
            incl[a] = wave_incl_scan64(sum);
            if (lane == 63) s_wave[a][wv] = incl[a];
            incl[a] -= sum;                       // exclusive within the wave
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uint64_t before = carry[a], total = 0;
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const uint64_t x = s_wave[a][w];
                if ((uint32_t)w < wv) before += x;
                total += x;
            }
            uint64_t run = before + incl[a];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t g = base + 4 * (uint64_t)t + i;
                const uint64_t c = cur[a][i];
                if (g < G) arr[a][g] = run;
                run += c;
            }
            carry[a] += total;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) cur[a][i] = nxt[a][i];
    }
    if (t == 0) {
        const uint64_t E = carry[0], T = carry[1], U = carry[2];
        job.off[job.G] = E; job.tstart[job.G] = T; job.ustart[job.G] = U;
        const uint64_t overflow = (E > job.capacity || T > job.tile_cap) ? 1 : 0;
        job.status[0] = E; job.status[1] = overflow; job.status[2] = T; job.status[3] = U;
        job.status[4] = 0;
        job.status[5] = 0;
        if (T <= job.tile_cap) job.tile_off[T] = E;
        if (job.out_total) *job.out_total = E;
    }
}

// Third phase: exclusive offsets of every chunk (one wave per 64 chunks).
__global__ __launch_bounds__(64) void fix_kernel(Job job)
{
    const uint64_t g = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    const uint64_t nb = (job.G + 63) / 64;
    const bool in = g < job.G;
    const uint64_t c = in ? job.off[g] : 0, t = in ? job.tstart[g] : 0, u = in ? job.ustart[g] : 0;
    const uint64_t sc = wave_incl_scan64(c), st = wave_incl_scan64(t), su = wave_incl_scan64(u);
    if (in) {
        job.off[g] = job.bsum[blockIdx.x] + sc - c;
        job.tstart[g] = job.bsum[nb + blockIdx.x] + st - t;
        job.ustart[g] = job.bsum[2 * nb + blockIdx.x] + su - u;
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
// plan: each lane takes a contiguous range of planner units (a unit is a
// subtree of <= 64 tiles of one chunk's tile tree, at depth d, index j), so
// the chunk of its next unit is found by stepping forward.  For each unit
// the lane walks from the tile-tree root
// to the unit (the communication-free path: the count of the unit and the
// counts left of it), then traverses the unit depth first, left child first,
// so leaves come in tile order and each tile's output offset is a running
// sum.  Every split is one HypRun, advanced by one proposal per loop trip;
// pending right children wait on a small per-lane stack in LDS.  With
// TERMS = 2 or 4 a unit belongs to a group of that many lanes, which keep
// the same state and spread each proposal's four log-factorial differences
// over the group (for launches with few units, where one unit's chain of
// variates, not the lanes' throughput, sets the time).
// ---------------------------------------------------------------------------
constexpr int kPlanStack = 8;   // > depth of a unit subtree (6 for 64 tiles)

template <int TERMS>
__global__ __launch_bounds__(64) void plan_kernel(Job job)
{
    __shared__ uint64_t st_k[kPlanStack][64];
    __shared__ uint32_t st_lo[kPlanStack][64], st_hi[kPlanStack][64], st_heap[kPlanStack][64];
    const uint32_t lane = threadIdx.x;
    if (job.status[1]) return;
    const uint64_t U = job.status[3];
    // blocked unit ranges: a lane group's next unit is the following one, so
    // the chunk index only moves forward (one binary search per group)
    const uint64_t TL = (uint64_t)gridDim.x * (64 / TERMS);
    const uint64_t per = (U + TL - 1) / TL;
    uint64_t u = ((uint64_t)blockIdx.x * 64 + lane) / TERMS * per;
    const uint64_t uend = u + per < U ? u + per : U;
    bool active = u < uend;
    uint64_t g = 0;
    // unit state
    uint64_t seed = 0, Nc = 0, tbase = 0, obase = 0, run = 0, j = 0;
    uint32_t c = 0, s = 0, d = 0, lev = 0;
    // current node (tile range within the chunk, count, heap id); path mode
    // while lev < d
    uint64_t lo = 0, hi = 0, k = 0;
    uint32_t heap = 1;
    int sp = 0;
    bool need_node = true, running = false;
    HypRun hr;
    hr.done = true;
    if (active) {
        g = last_le(job.ustart, job.G, u);
        const Inst &I = inst_at(job, inst_of_chunk(job, g));
        const uint64_t cc = chunk_ordinal(I, g - I.chunk_base);
        const Chunk ch = chunk_geometry(I, cc);
        seed = I.seed; c = (uint32_t)cc; s = I.s; Nc = ch.N;
        const uint64_t units = job.ustart[g + 1] - job.ustart[g];
        d = 63 - __clzll(units);
        j = u - job.ustart[g];
        tbase = job.tstart[g];
        obase = job.off[g];
        lo = 0; hi = tiles_of(Nc, s); k = job.off[g + 1] - obase; heap = 1; lev = 0; run = 0; sp = 0;
        need_node = false;
    }
    while (__any(active)) {
        if (active) {
            if (need_node) {
                if (sp > 0) {
                    --sp;
                    lo = st_lo[sp][lane]; hi = st_hi[sp][lane]; k = st_k[sp][lane]; heap = st_heap[sp][lane];
                    need_node = false;
                } else {
                    ++u;
                    if (u >= uend) {
                        active = false;
                    } else {
                        while (job.ustart[g + 1] <= u) ++g;
                        const Inst &I = inst_at(job, inst_of_chunk(job, g));
                        const uint64_t cc = chunk_ordinal(I, g - I.chunk_base);
                        const Chunk ch = chunk_geometry(I, cc);
                        seed = I.seed; c = (uint32_t)cc; s = I.s; Nc = ch.N;
                        const uint64_t units = job.ustart[g + 1] - job.ustart[g];
                        d = 63 - __clzll(units);
                        j = u - job.ustart[g];
                        tbase = job.tstart[g];
                        obase = job.off[g];
                        lo = 0; hi = tiles_of(Nc, s); k = job.off[g + 1] - obase; heap = 1; lev = 0; run = 0;
                        need_node = false;
                    }
                }
            }
            if (active && !need_node && !running) {
                if (lev >= d && hi - lo == 1) {
                    job.tile_off[tbase + lo] = obase + run;
                    run += k;
                    need_node = true;
                } else {
                    const uint64_t mid = lo + (hi - lo + 1) / 2;
                    hr.init(make_stream(seed, c, heap, TAG_TTREE), tile_range_slots(lo, hi, s, Nc),
                            tile_range_slots(lo, mid, s, Nc), k);
                    running = true;
                }
            }
            if (active && running && hr.template step<TERMS>()) {
                const uint64_t X = hr.result();
                const uint64_t mid = lo + (hi - lo + 1) / 2;
                running = false;
                if (lev < d) {
                    // on the path to the unit: follow bit (d-1-lev) of j
                    if (((j >> (d - 1 - lev)) & 1) == 0) { hi = mid; k = X; heap = 2 * heap; }
                    else { lo = mid; k = k - X; run += X; heap = 2 * heap + 1; }
                    ++lev;
                } else {
                    st_lo[sp][lane] = (uint32_t)mid; st_hi[sp][lane] = (uint32_t)hi;
                    st_k[sp][lane] = k - X; st_heap[sp][lane] = 2 * heap + 1;
                    ++sp;
                    hi = mid; k = X; heap = 2 * heap;
                }
            }
        }
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

// Inclusive prefix sum over the 64 lanes with DPP moves: shifts by 1, 2, 4
// and 8 inside rows of 16 lanes, then the last lane of row 0 / 2 is added to
// row 1 / 3 and the last lane of row 1 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Slot -> edge of one tile (Sec. 4.1 and 4.2 offset computations).
// Directed: slot w of row u (w in [0, n-1)) is column w + [w >= u].
// Rectangle: local l -> (row r0 + l / width, column b + l % width).
// Triangle: rows counted from the bottom hold 1, 2, 3, ... slots.
// Because n <= 2^32, rows, columns, section sizes and the divisor fit 32
// bits.  The dividend c0 + x fits 32 bits unless the tile has close
// to 2^32 slots ("wide").  Divisions use a binary64 reciprocal estimate
// corrected by one step (exact for dividends below 2^33), or a shift when
// the divisor is a power of two.
struct Decoder {
    uint32_t type;      // 0 directed, 1 rectangle, 2 triangle
    uint32_t pow2;      // divisor is 2^sh
    uint32_t sh;
    uint32_t wide;      // some dividend c0 + x of the tile needs 33 bits
    uint32_t dv;        // directed: n - 1; rectangle: section width
    uint32_t r0, c0;    // row of the tile start and its offset in that row
    uint32_t b;         // rectangle: first column
    uint32_t a, h;      // triangle: section start and size
    double rcp;         // 1 / dv
    uint64_t Ttri, lbase;  // triangle: its slots, tile start

    __device__ __forceinline__ uint32_t divmod(uint32_t x, uint32_t &rem) const
    {
        if (!wide) {
            const uint32_t y = c0 + x;
            if (pow2) { rem = y & (dv - 1); return y >> sh; }
            uint32_t q = (uint32_t)((double)y * rcp);
            int32_t r = (int32_t)(y - q * dv);
            if (r < 0) { --q; r += (int32_t)dv; }
            else if ((uint32_t)r >= dv) { ++q; r -= (int32_t)dv; }
            rem = (uint32_t)r;
            return q;
        }
        const uint64_t y = (uint64_t)c0 + x;
        if (pow2) { rem = (uint32_t)(y & (dv - 1)); return (uint32_t)(y >> sh); }
        uint64_t q = (uint64_t)((double)y * rcp);
        int64_t r = (int64_t)(y - q * dv);
        if (r < 0) { --q; r += (int64_t)dv; }
        else if ((uint64_t)r >= dv) { ++q; r -= (int64_t)dv; }
        rem = (uint32_t)r;
        return (uint32_t)q;
    }

    __device__ __forceinline__ uint2 operator()(uint32_t x) const
    {
        if (type != 2) {
            uint32_t r;
            const uint32_t q = divmod(x, r);
            const uint32_t u = r0 + q;
            return type == 0 ? make_uint2(u, r + (r >= u)) : make_uint2(u, b + r);
        }
        const uint64_t l = lbase + x;
        const uint64_t lr = Ttri - 1 - l;
        // largest q with q(q+1)/2 <= lr: the binary64 estimate is within one
        // of it (lr < 2^63: the rounding of lr moves the square root by far
        // less than one), so each correction runs at most twice
        uint64_t q = (uint64_t)((sqrt(8.0 * (double)lr + 1.0) - 1.0) * 0.5);
        for (int i = 0; i < 2 && q * (q + 1) / 2 > lr; ++i) --q;
        for (int i = 0; i < 2 && (q + 1) * (q + 2) / 2 <= lr; ++i) ++q;
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

// A lane's run of `per` consecutive counters starting at h0 (per is 1, 2, 4,
// 8 or 16; runs of 4 or more are 16-byte aligned).
__device__ __forceinline__ void load_run(const uint32_t *h, uint32_t h0, uint32_t per, uint32_t NB, uint32_t *v)
{
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = 0;
    if (h0 >= NB) return;
    if (per >= 4) {
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
            if ((uint32_t)i < per) {
                const uint4 q = *reinterpret_cast<const uint4 *>(h + h0 + i);
                v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) if ((uint32_t)i < per) v[i] = h[h0 + i];
    }
}

__device__ __forceinline__ void store_run(uint32_t *h, uint32_t h0, uint32_t per, uint32_t NB, const uint32_t *v)
{
    if (h0 >= NB) return;
    if (per >= 4) {
#pragma unroll
        for (int i = 0; i < 16; i += 4)
            if ((uint32_t)i < per) *reinterpret_cast<uint4 *>(h + h0 + i) = make_uint4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) if ((uint32_t)i < per) h[h0 + i] = v[i];
    }
}

// W consecutive LDS words starting at p0 (W = 4, 8 or 16; p0 a multiple of
// W/2), loaded into / stored from registers, and a bitonic network that sorts
// them ascending.
template <int W>
__device__ __forceinline__ void win_load(const uint32_t *s, uint32_t p0, uint32_t *v)
{
    if ((p0 & 3) == 0) {
#pragma unroll
        for (int i = 0; i < W; i += 4) {
            const uint4 q = *reinterpret_cast<const uint4 *>(s + p0 + i);
            v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < W; i += 2) {
            const uint2 q = *reinterpret_cast<const uint2 *>(s + p0 + i);
            v[i] = q.x; v[i + 1] = q.y;
        }
    }
}

template <int W>
__device__ __forceinline__ void win_store(uint32_t *s, uint32_t p0, const uint32_t *v)
{
    if ((p0 & 3) == 0) {
#pragma unroll
        for (int i = 0; i < W; i += 4)
            *reinterpret_cast<uint4 *>(s + p0 + i) = make_uint4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < W; i += 2) *reinterpret_cast<uint2 *>(s + p0 + i) = make_uint2(v[i], v[i + 1]);
    }
}

template <int W>
__device__ __forceinline__ void win_sort(uint32_t *v)
{
#pragma unroll
    for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t a = v[i], b = v[l];
                    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    if ((i & k) == 0) { v[i] = lo; v[l] = hi; } else { v[i] = hi; v[l] = lo; }
                }
            }
        }
    }
}

// Merge of two ascending runs v[0..4) and v[4..8): the second run reversed
// makes the sequence bitonic, and three compare-exchange stages sort it.
__device__ __forceinline__ void win_merge8(uint32_t *v)
{
    uint32_t t = v[4]; v[4] = v[7]; v[7] = t;
    t = v[5]; v[5] = v[6]; v[6] = t;
#pragma unroll
    for (int j = 4; j > 0; j >>= 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if ((i & j) == 0) {
                const uint32_t a = v[i], b = v[i + j];
                v[i] = a < b ? a : b;
                v[i + j] = a < b ? b : a;
            }
        }
    }
}

// Two window passes over s[0..V) with windows of 8 keys, R (1 or 2)
// consecutive windows per lane (s padded with ~0 up to 512 R + 4): lane L
// sorts windows [8 (R L + r), +8), then the windows shifted by 4.  The result
// is sorted whenever no bucket of more than 5 keys straddles a window
// boundary; order and repeats are checked from the registers of the second
// pass (one shuffle for the boundary between lanes).  Returns
// (bad ? 1 : 0) | (repeats << 1).
__device__ __forceinline__ uint32_t window_passes(uint32_t *s, uint32_t V, uint32_t R)
{
    const uint32_t lane = threadIdx.x;
    uint32_t v[8], head[4];
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
        if (r < R) {
            const uint32_t p0 = 8 * (R * lane + r);
            win_load<8>(s, p0, v);
            win_sort<8>(v);
            win_store<8>(s, p0, v);
            if (r == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) head[i] = v[i];
            }
        }
    }
    __syncthreads();
    uint32_t bad = 0, dup = 0, prev_last = 0, first = 0;
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
        if (r < R) {
            const uint32_t p0 = 8 * (R * lane + r) + 4;
            win_load<8>(s, p0, v);
            win_merge8(v);          // both halves come sorted from the first pass
            win_store<8>(s, p0, v);
#pragma unroll
            for (int i = 0; i < 7; ++i)
                if (p0 + i + 1 < V) { bad |= v[i] > v[i + 1]; dup += v[i] == v[i + 1]; }
            if (r == 0) first = v[0];
            else if (p0 < V) { bad |= prev_last > v[0]; dup += prev_last == v[0]; }
            prev_last = v[7];
        }
    }
    const uint32_t last_p = 8 * (R * lane + R - 1) + 4 + 7;     // position of prev_last
    const uint32_t nxt = __shfl_down(first, 1, 64);
    if (lane < 63 && last_p + 1 < V) { bad |= prev_last > nxt; dup += prev_last == nxt; }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t y = i + 1 < 4 ? head[i + 1] : first;
            if ((uint32_t)i + 1 < V) { bad |= head[i] > y; dup += head[i] == y; }
        }
    }
    return bad | (dup << 1);
}

// Write sorted keys s[0..n) as edges o0 .. o0+n-1: lane-strided, four keys
// per lane per round so that their LDS reads overlap.
__device__ __forceinline__ void emit_sorted(const TileCtx &t, const uint32_t *s, uint32_t n)
{
    const uint32_t lane = threadIdx.x;
    for (uint32_t b = 0; b < n; b += 256) {
        uint32_t x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t p = b + lane + 64 * i;
            x[i] = p < n ? s[p] : 0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t p = b + lane + 64 * i;
            if (p < n) store_edge(t.edges, t.o0 + p, t.dec(x[i]));
        }
    }
}

// Fast base case for tiles whose draws fit one LDS pass (J <= cap): lane L
// keeps in registers the words of blocks L, L + 64, ... (draw d = 4 block + q),
// so the histogram atomics run while the words are produced and nothing is
// staged.  Counting sort on the top bits of the key with about two buckets
// per key: exclusive scan, scatter, then every lane sorts the buckets it owns
// (a contiguous range it knows from the scan) in place and counts repeats.
// Leaves the sorted distinct set in s[0..ke) and returns true, or false when
// J would exceed cap (the caller then uses key sub-ranges).
template <int CAP>
__device__ __forceinline__ bool leaf_fast(const TileCtx &t, uint32_t *s, uint32_t *hist, uint32_t ke, uint32_t cap)
{
    constexpr int R = CAP / 256;
    const uint32_t lane = threadIdx.x;
    uint32_t nbb = 33 - __clz(ke | 1);                  // ~2 buckets per key
    const uint32_t nbmax = 31 - __clz((uint32_t)CAP);
    if (nbb > nbmax) nbb = nbmax;
    if (nbb > t.bits) nbb = t.bits;
    const uint32_t NB = 1u << nbb;
    const uint32_t shift = t.bits - nbb;
    const uint32_t per = NB >= 64 ? NB / 64 : 1;        // buckets owned by a lane
    const uint32_t h0 = lane * per;
    uint32_t J = ke;
    for (;;) {
        if (J > cap) return false;
        {
            uint32_t z[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            store_run(hist, h0, per, NB, z);
        }
        {
            // draws straight to LDS: s[d] = word d masked, or ~0 if rejected
            const uint32_t nblk = (J + 3) >> 2;
#pragma unroll 1
            for (uint32_t blk = lane; blk < nblk; blk += 64) {
                const U4 w = t.st.block(blk);
                uint32_t v[4] = {w.x & t.mask, w.y & t.mask, w.z & t.mask, w.w & t.mask};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (!(4 * blk + q < J && (t.full || v[q] < t.S))) v[q] = 0xFFFFFFFFu;
                *reinterpret_cast<uint4 *>(s + 4 * blk) = make_uint4(v[0], v[1], v[2], v[3]);
            }
            __syncthreads();
            uint32_t xs[4 * R], sl[4 * R];
            const bool allv = t.full;   // with S = 2^bits no draw is rejected
#pragma unroll
            for (int e = 0; e < 4 * R; ++e) {
                const uint32_t d = lane + 64u * e;
                xs[e] = 0;
                sl[e] = 0xFFFFFFFFu;
                if (d < J) {
                    const uint32_t x = s[d];
                    if (allv || x != 0xFFFFFFFFu) {
                        xs[e] = x;
                        sl[e] = atomicAdd(&hist[x >> shift], 1u);
                    }
                }
            }
            __syncthreads();
            // exclusive scan of hist[0..NB): lane owns per = NB/64 consecutive
            // buckets, read and written with 16-byte LDS accesses
            {
                uint32_t cv[16];
                load_run(hist, h0, per, NB, cv);
                uint32_t sum = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) if ((uint32_t)i < per) sum += cv[i];
                uint32_t incl = sum;
#pragma unroll
                for (int dlt = 1; dlt < 64; dlt <<= 1) {
                    const uint32_t o = __shfl_up(incl, dlt, 64);
                    if (lane >= (uint32_t)dlt) incl += o;
                }
                uint32_t run = incl - sum;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    if ((uint32_t)i < per) { const uint32_t c = cv[i]; cv[i] = run; run += c; }
                }
                store_run(hist, h0, per, NB, cv);
                if (lane == 63) hist[NB] = incl;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 4 * R; ++e)
                if (sl[e] != 0xFFFFFFFFu) s[hist[xs[e] >> shift] + sl[e]] = xs[e];
        }
        __syncthreads();
        const uint32_t V = hist[NB];
        // The array is now ordered by bucket.  Sort by value: every lane sorts
        // its PL consecutive keys in registers (bitonic network), then the
        // windows shifted by PL/2 (any bucket of <= PL/2 + 1 keys lying across
        // a window boundary falls inside one shifted window); a check pass
        // counts repeats and repeats both passes in the rare case that a
        // longer bucket left the order broken.
        uint32_t ndup = 0;
        {
            const uint32_t R = V <= 512 ? 1 : 2;
            const uint32_t span = 512 * R + 4;
            for (uint32_t p = V + lane; p < span; p += 64) s[p] = 0xFFFFFFFFu;
            for (;;) {
                __syncthreads();
                const uint32_t r = window_passes(s, V, R);
                ndup = r >> 1;
                if (!__syncthreads_or(r & 1)) break;
            }
        }
        ndup = wave_sum32(ndup);
        __syncthreads();
        const uint32_t D = V - ndup;
        if (D == ke) {
            if (ndup) {
                uint32_t kept = 0;
                for (uint32_t b0 = 0; b0 < V; b0 += 64) {
                    const uint32_t p = b0 + lane;
                    uint32_t x = 0;
                    bool keep = false;
                    if (p < V) {
                        x = s[p];
                        keep = p == 0 || s[p - 1] != x;
                    }
                    const uint64_t bal = __ballot(keep);
                    __syncthreads();
                    if (keep) s[kept + __popcll(bal & lanemask_lt(lane))] = x;
                    kept += __popcll(bal);
                    __syncthreads();
                }
            }
            return true;
        }
        J += ke - D;
    }
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
    if (ke <= cap && leaf_fast<CAP>(t, s, hist, (uint32_t)ke, cap)) {
        if (!comp) emit_sorted(t, s, (uint32_t)ke);
        else {
            emit_complement(t, s, (uint32_t)ke, 0, t.S, 0);
        }
        return;
    }
    __syncthreads();
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
