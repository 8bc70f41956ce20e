// kg_skip.hpp -- the geometric-skip G(n,p) variant: a second sampler for the
// law of Sec. 2.1.1 / 4.3 (every slot an independent Bernoulli(p) trial)
// with its own bits.  Each tile of each chunk (the 2^s-slot tiles of the
// main path) runs its trials by waiting times: the number of failures before
// the next success is floor(log U / log(1 - p)), one 64-bit draw of the
// tile's stream (seed, chunk ordinal, tile, TAG_SKIP) per gap; for p > 1/2
// the waiting times are those of the failures and the other slots are the
// successes.  Count pass -> scan of the tile counts -> write pass.  When
// the workspace holds a row of positions per tile, the count pass keeps the
// events' positions and the write pass only decodes them (skip_gen_kernel,
// skip_emit_kernel); otherwise the count pass runs one lane per tile and the
// write pass generates the same trials again (skip_count_kernel,
// skip_write_kernel).  The chunk and tile layout comes from the main path's
// count and offset kernels.
#pragma once
#include "kg_tile.hpp"

namespace kg {

constexpr uint32_t TAG_SKIP = 7;

// Trials of one tile of St slots; `emit(x)` receives the tile-local keys of
// the successes in ascending order.  Returns their number.
template <class Emit>
__device__ __forceinline__ uint64_t skip_trials(const Stream &st, uint64_t St, double p, Emit emit)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) {
        for (uint64_t x = 0; x < St; ++x) emit(x);
        return St;
    }
    const bool flip = p > 0.5;
    const double L = log1p_f64(flip ? -(1.0 - p) : -p);
    Draws64 d(st);
    uint64_t pos = 0, k = 0;
    for (;;) {
        const double U = unit_of(d.get());
        const double g = floor(log_f64(U) / L);
        const uint64_t next = g >= (double)(St - pos) ? St : pos + (uint64_t)g;
        if (flip) {
            for (uint64_t x = pos; x < next; ++x) { emit(x); ++k; }
        } else if (next < St) {
            emit(next);
            ++k;
        }
        if (next >= St) return k;
        pos = next + 1;
    }
}

// Edge of chunk-local slot l (canonical local order of Sec. 4.1 / 4.2).
__device__ __forceinline__ uint2 skip_decode(const Inst &I, const Chunk &ch, uint64_t l)
{
    if (I.directed) {
        const uint64_t i = ch.row0 * (I.n - 1) + l;
        const uint64_t u = i / (I.n - 1), w = i % (I.n - 1);
        return make_uint2((uint32_t)u, (uint32_t)(w + (w >= u)));
    }
    if (!ch.diag) return make_uint2((uint32_t)(ch.a + l / ch.w), (uint32_t)(ch.b + l % ch.w));
    // triangle: row r starts at r h - r (r + 1) / 2; the last start <= l
    const uint64_t h = ch.h;
    uint64_t lo = 0, hi = h - 1;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (mid * h - mid * (mid + 1) / 2 <= l) lo = mid; else hi = mid;
    }
    const uint64_t st = lo * h - lo * (lo + 1) / 2;
    return make_uint2((uint32_t)(ch.a + lo), (uint32_t)(ch.a + lo + 1 + (l - st)));
}

// The tile's chunk, geometry, stream and slot count.
struct SkipTile {
    Inst I;
    Chunk ch;
    Stream st;
    uint64_t S, lbase;
};

__device__ __forceinline__ SkipTile skip_tile_at(const Job &job, uint64_t t)
{
    SkipTile r;
    const uint64_t g = last_le(job.tstart, job.G, t);
    r.I = inst_at(job, inst_of_chunk(job, g));
    const uint64_t c = chunk_ordinal(r.I, g - r.I.chunk_base);
    r.ch = chunk_geometry(r.I, c);
    const uint64_t tl = t - job.tstart[g];
    r.lbase = tl << r.I.s;
    const uint64_t full = 1ull << r.I.s;
    r.S = r.ch.N - r.lbase < full ? r.ch.N - r.lbase : full;
    r.st = make_stream(r.I.seed, (uint32_t)c, (uint32_t)tl, TAG_SKIP);
    return r;
}

// Count pass: one lane per tile; the count goes to tile_off[t] and the wave's
// sum to queue[wave] (the main path's queue is free in this mode).
__global__ __launch_bounds__(64) void skip_count_kernel(Job job)
{
    const uint64_t t = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    const uint64_t T = job.status[2];
    uint64_t k = 0;
    if (!job.status[1] && t < T) {
        const SkipTile r = skip_tile_at(job, t);
        k = skip_trials(r.st, r.S, r.I.p, [](uint64_t) {});
        job.tile_off[t] = k;
    }
    const uint64_t incl = wave_incl_scan64(k);
    if (threadIdx.x == 63) job.queue[blockIdx.x] = incl;
}

// Scan of the wave sums (one workgroup of 1024 lanes, rounds of 1024); the
// total edges and the overflow flag.
__global__ __launch_bounds__(1024) void skip_scan_kernel(Job job, uint64_t nwaves)
{
    __shared__ uint64_t s_w[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nwaves; base += 1024) {
        const uint64_t i = base + t;
        const uint64_t v = i < nwaves ? job.queue[i] : 0;
        const uint64_t incl = wave_incl_scan64(v);
        if (lane == 63) s_w[wv] = incl;
        __syncthreads();
        uint64_t before = carry, total = 0;
        for (int w = 0; w < 16; ++w) {
            const uint64_t x = s_w[w];
            if ((uint32_t)w < wv) before += x;
            total += x;
        }
        if (i < nwaves) job.queue[i] = before + incl - v;
        carry += total;
        __syncthreads();
    }
    if (t == 0) {
        job.status[0] = carry;
        job.status[1] = carry > job.capacity ? 1 : 0;
        job.status[5] = 0;
        if (job.out_total) *job.out_total = carry;
    }
}

// The scanned counts as tile offsets: tile_off[t] = the wave's prefix plus
// the in-wave prefix of the counts, tile_off[T] = the total (the layout the
// write pass walks, as the main path's sampler does).
__global__ __launch_bounds__(64) void skip_fix_kernel(Job job)
{
    const uint64_t t = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    const uint64_t T = job.status[2];
    const uint64_t k = t < T ? job.tile_off[t] : 0;
    const uint64_t ex = wave_incl_scan64(k) - k;
    if (t < T) job.tile_off[t] = job.queue[blockIdx.x] + ex;
    else if (t == T) job.tile_off[T] = job.status[0];
}

// Write pass: a persistent grid walks ranges of tiles chunk by chunk, each
// workgroup taking the next range from the shared counter (as the main
// sampler does, with its decoders).  The waiting times of a tile are
// independent draws, so the positions of its events (successes, or
// failures when p > 1/2) are prefix sums: x_d = x_{d-1} + 1 + g_d.  A round
// takes 128 draws (lane L: block 64 r + L, draws 128 r + 2 L and + 1), forms
// the gaps, scans them across the wave and appends the events below S to
// LDS; full batches and the tile's last one are decoded and stored with
// consecutive lanes on consecutive edges (the main sampler's emission).
// The positions are those of skip_trials: the same draws, gaps and sums.
constexpr uint32_t kSkipKeys = 1408;   // LDS batch (11 rounds of 128 events)

// One round of a tile's waiting times: the positions x0, x1 of lane L's two
// events (tile-local, counted from `pos`), whether they fall below S, how
// many of the round's 128 events do (they are a prefix in lane order), and
// the wave's inclusive sum of the advances for the next round's `pos`.
struct SkipRound {
    uint64_t x0, x1, next;
    bool v0, v1;
    uint32_t nv;
};

__device__ __forceinline__ SkipRound skip_round(const TileCtx &tc, uint32_t r, uint64_t pos, double L)
{
    const uint32_t lane = threadIdx.x;
    const uint64_t S = tc.S;
    const U4 q = tc.st.block_uniform_key(64 * r + lane);
    const double U0 = unit_of(((uint64_t)q.y << 32) | q.x);
    const double U1 = unit_of(((uint64_t)q.w << 32) | q.z);
    const double g0 = floor(log_f64(U0) / L), g1 = floor(log_f64(U1) / L);
    const double cap = (double)S;
    const uint64_t a0 = (uint64_t)(g0 < cap ? g0 : cap) + 1;
    const uint64_t a1 = (uint64_t)(g1 < cap ? g1 : cap) + 1;
    const uint64_t sum = a0 + a1;
    const uint64_t incl = wave_incl_scan64(sum);
    SkipRound o;
    o.x0 = pos + (incl - sum) + a0 - 1;
    o.x1 = o.x0 + a1;
    o.v0 = o.x0 < S;
    o.v1 = o.x1 < S;
    o.nv = (uint32_t)(__popcll(__ballot(o.v0)) + __popcll(__ballot(o.v1)));
    o.next = pos + (__builtin_amdgcn_readlane((uint32_t)incl, 63) |
                    ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(incl >> 32), 63) << 32));
    return o;
}

// A tile's events generated and stored at output offset o0, in LDS batches
// of up to kSkipKeys (for p > 1/2 the complement of the failures is stored).
__device__ __forceinline__ void skip_write_tile(TileCtx &tc, uint32_t *s_key, uint64_t o0, bool flip, double L)
{
    const uint32_t lane = threadIdx.x;
    const uint64_t S = tc.S;
    uint64_t pos = 0, rlo = 0, done = 0;
    uint32_t nb = 0;
    for (uint32_t r = 0;; ++r) {
        const SkipRound R = skip_round(tc, r, pos, L);
        if (nb + R.nv > kSkipKeys) {
            // batch full: out with it (a wave-uniform decision)
            __syncthreads();
            if (!flip) {
                TileCtx tb = tc;
                tb.o0 = o0 + done;
                emit_tile(tb, s_key, nb);
                done += nb;
            } else {
                const uint64_t rhi = (uint64_t)s_key[nb - 1] + 1;
                done += emit_complement(tc, s_key, nb, rlo, rhi, done);
                rlo = rhi;
            }
            __syncthreads();
            nb = 0;
        }
        if (R.v0) s_key[nb + 2 * lane] = (uint32_t)R.x0;
        if (R.v1) s_key[nb + 2 * lane + 1] = (uint32_t)R.x1;
        nb += R.nv;
        if (R.nv < 128) break;
        pos = R.next;
    }
    __syncthreads();
    if (!flip) {
        TileCtx tb = tc;
        tb.o0 = o0 + done;
        emit_tile(tb, s_key, nb);
    } else {
        emit_complement(tc, s_key, nb, rlo, S, done);
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void skip_write_kernel(Job job)
{
    __shared__ __attribute__((aligned(16))) uint32_t s_key[kSkipKeys];
    if (ld_uni(job.status + 1)) return;
    const uint64_t T = ld_uni(job.status + 2);
    const double p = job.one.p;
    const bool flip = p > 0.5;
    const bool all = p >= 1.0;
    const double L = log1p_f64(flip ? -(1.0 - p) : -p);
    TileWalk w;
    TileCtx &tc = w.tc;
    tc.edges = job.edges;
    TileGrab grab(T);
    uint64_t t, t1;
    while (grab.next(job, t, t1)) {
        uint64_t g = chunk_of_tile(job, t);
        for (;;) {
            w.enter(job, g);
            const uint64_t tend = w.gend < t1 ? w.gend : t1;
            for (; t < tend; ++t) {
                const uint64_t o0 = ld_uni(job.tile_off + t);
                const uint64_t k = ld_uni(job.tile_off + t + 1) - o0;
                if (k == 0) continue;
                w.tile(t);
                tc.st.tag = TAG_SKIP;
                tc.o0 = o0;
                if (all) emit_complement(tc, s_key, 0, 0, tc.S, 0);
                else skip_write_tile(tc, s_key, o0, flip, L);
            }
            if (t >= t1) break;
            ++g;
            while (ld_uni(job.tstart + g + 1) <= t) ++g;
        }
    }
}

// Slab variant (when the workspace holds it): a gap pass generates each
// tile's events once, keeps the positions of up to `cap` of them in the
// tile's slab row (slab + t cap, ascending) and writes the tile's edge count;
// after the scan an emission pass only decodes the stored positions, so the
// FP64 log and division of a gap are paid once instead of twice.  A tile
// with more events than its row holds is generated again by the write path.
__global__ __launch_bounds__(64) void skip_gen_kernel(Job job, uint32_t *slab, uint32_t cap)
{
    const uint64_t T = ld_uni(job.status + 2);
    const double p = job.one.p;
    const bool flip = p > 0.5;
    const bool all = p >= 1.0;
    const double L = all ? 0.0 : log1p_f64(flip ? -(1.0 - p) : -p);
    const uint32_t lane = threadIdx.x;
    TileWalk w;
    TileCtx &tc = w.tc;
    TileGrab grab(T);
    uint64_t t, t1;
    while (grab.next(job, t, t1)) {
        uint64_t g = chunk_of_tile(job, t);
        for (;;) {
            w.enter(job, g);
            const uint64_t tend = w.gend < t1 ? w.gend : t1;
            for (; t < tend; ++t) {
                w.tile(t);
                tc.st.tag = TAG_SKIP;
                const uint64_t S = tc.S;
                uint64_t nev = 0;
                if (!all && p > 0.0) {
                    uint32_t *row = slab + t * (uint64_t)cap;
                    uint64_t pos = 0;
                    for (uint32_t r = 0;; ++r) {
                        const SkipRound R = skip_round(tc, r, pos, L);
                        const uint64_t i0 = nev + 2 * lane;
                        if (R.v0 && i0 < cap) row[i0] = (uint32_t)R.x0;
                        if (R.v1 && i0 + 1 < cap) row[i0 + 1] = (uint32_t)R.x1;
                        nev += R.nv;
                        if (R.nv < 128) break;
                        pos = R.next;
                    }
                }
                const uint64_t k = all ? S : !(p > 0.0) ? 0 : flip ? S - nev : nev;
                if (lane == 0) job.tile_off[t] = k;
            }
            if (t >= t1) break;
            ++g;
            while (ld_uni(job.tstart + g + 1) <= t) ++g;
        }
    }
}

// The gap pass's tile counts summed per wave of 64 tiles (for the scan).
__global__ __launch_bounds__(64) void skip_sums_kernel(Job job)
{
    const uint64_t t = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    const uint64_t T = job.status[2];
    const uint64_t k = t < T ? job.tile_off[t] : 0;
    const uint64_t incl = wave_incl_scan64(k);
    if (threadIdx.x == 63) job.queue[blockIdx.x] = incl;
}

// Emission pass of the slab variant: each tile's stored positions through
// LDS to the decoders (the complement of them for p > 1/2).
__global__ __launch_bounds__(64) void skip_emit_kernel(Job job, const uint32_t *slab, uint32_t cap)
{
    __shared__ __attribute__((aligned(16))) uint32_t s_key[kSkipKeys];
    if (ld_uni(job.status + 1)) return;
    const uint64_t T = ld_uni(job.status + 2);
    const double p = job.one.p;
    const bool flip = p > 0.5;
    const bool all = p >= 1.0;
    const double L = all ? 0.0 : log1p_f64(flip ? -(1.0 - p) : -p);
    const uint32_t lane = threadIdx.x;
    TileWalk w;
    TileCtx &tc = w.tc;
    tc.edges = job.edges;
    TileGrab grab(T);
    uint64_t t, t1;
    while (grab.next(job, t, t1)) {
        uint64_t g = chunk_of_tile(job, t);
        for (;;) {
            w.enter(job, g);
            const uint64_t tend = w.gend < t1 ? w.gend : t1;
            for (; t < tend; ++t) {
                const uint64_t o0 = ld_uni(job.tile_off + t);
                const uint64_t k = ld_uni(job.tile_off + t + 1) - o0;
                if (k == 0) continue;
                w.tile(t);
                tc.st.tag = TAG_SKIP;
                tc.o0 = o0;
                const uint64_t S = tc.S;
                if (all) {
                    emit_complement(tc, s_key, 0, 0, S, 0);
                    continue;
                }
                const uint64_t nev = flip ? S - k : k;
                if (nev > cap) {
                    skip_write_tile(tc, s_key, o0, flip, L);
                    continue;
                }
                // the row to LDS, 16 bytes per lane (rows start 16-byte
                // aligned: cap is a multiple of 4), then the tail word by word
                const uint32_t *row = slab + t * (uint64_t)cap;
                const uint32_t n4 = (uint32_t)nev & ~3u;
                for (uint32_t i = 4 * lane; i < n4; i += 256)
                    *reinterpret_cast<uint4 *>(s_key + i) = *reinterpret_cast<const uint4 *>(row + i);
                if (n4 + lane < (uint32_t)nev) s_key[n4 + lane] = row[n4 + lane];
                __syncthreads();
                if (!flip) emit_tile(tc, s_key, (uint32_t)nev);
                else emit_complement(tc, s_key, (uint32_t)nev, 0, S, 0);
                __syncthreads();
            }
            if (t >= t1) break;
            ++g;
            while (ld_uni(job.tstart + g + 1) <= t) ++g;
        }
    }
}

}  // namespace kg
