// kg_skip.hpp -- the geometric-skip G(n,p) variant: a second sampler for the
// law of Sec. 2.1.1 / 4.3 (every slot an independent Bernoulli(p) trial)
// with its own bits.  Each tile of each chunk (the 2^s-slot tiles of the
// main path) runs its trials by waiting times: the number of failures before
// the next success is floor(log U / log(1 - p)), one 64-bit draw of the
// tile's stream (seed, chunk ordinal, tile, TAG_SKIP) per gap; for p > 1/2
// the waiting times are those of the failures and the other slots are the
// successes.  Count pass (one lane per tile) -> scan of the tile counts ->
// write pass (the same trials again, decoded and stored at the tile's
// offset).  The chunk and tile layout comes from the main path's count and
// offset kernels.
#pragma once
#include "kg_kernels.hpp"

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
        if (job.out_total) *job.out_total = carry;
    }
}

// Write pass: the same trials, each success decoded and stored at the tile's
// offset (the wave's prefix plus the in-wave prefix of the counts).
__global__ __launch_bounds__(64) void skip_write_kernel(Job job)
{
    if (job.status[1]) return;
    const uint64_t t = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    const uint64_t T = job.status[2];
    const uint64_t k = t < T ? job.tile_off[t] : 0;
    const uint64_t o = job.queue[blockIdx.x] + wave_incl_scan64(k) - k;
    if (t >= T || k == 0) return;
    const SkipTile r = skip_tile_at(job, t);
    uint2 *out = reinterpret_cast<uint2 *>(job.edges) + o;
    uint64_t e = 0;
    if (r.ch.diag) {
        skip_trials(r.st, r.S, r.I.p, [&](uint64_t x) { out[e++] = skip_decode(r.I, r.ch, r.lbase + x); });
        return;
    }
    // directed rows and rectangles: keys ascend, so the row and column of a
    // key follow from the previous ones by adding the gap (a division only
    // when the gap spans a whole row)
    const uint64_t W = r.I.directed ? r.I.n - 1 : r.ch.w;
    const uint64_t first = r.I.directed ? r.ch.row0 * W + r.lbase : r.lbase;
    uint64_t row = first / W, col = first % W, last = 0;
    skip_trials(r.st, r.S, r.I.p, [&](uint64_t x) {
        const uint64_t gap = x - last;
        last = x;
        if (gap >= W) { row += gap / W; col += gap % W; }
        else col += gap;
        if (col >= W) { col -= W; ++row; }
        out[e++] = r.I.directed ? make_uint2((uint32_t)row, (uint32_t)(col + (col >= row)))
                                : make_uint2((uint32_t)(r.ch.a + row), (uint32_t)(r.ch.b + col));
    });
}

}  // namespace kg
