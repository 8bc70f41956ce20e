// kg_rgg.hpp -- two-dimensional random geometric graphs: n points uniform in
// the unit square, an edge between every two points closer than r
// (Sec. 2.1.2), generated as in Sec. 5: a grid of 4^L cells of side
// 2^-L >= max(r, n^-1/2); the points per cell by a quadrant recursion of
// binomial variates, each node drawing from a stream keyed by the node
// (Sec. 5.1); the points of a cell from the cell's own stream; edges by
// comparing each point with the points of its cell and the eight neighbours,
// counted, prefix-summed and written in a second pass (Sec. 5.3).
//
// A node at level l (Morton index z) holding k points splits them with three
// Bin(., 1/2) variates: the lower half (slot 0), its left quadrant (slot 1),
// the upper half's left quadrant (slot 2); stream (seed; j, z, 3 l + slot,
// TAG_RTREE).  Every node is computed once here, level by level; its value is
// the one any root path to it would give, since it depends only on its own
// count and stream.  Point j of cell z is ((cx + U) 2^-L, (cy + V) 2^-L), U
// and V the two 64-bit uniforms of block j of (seed; j, z, 0, TAG_RPTS).
// Vertex ids follow the cells in Morton order (x bit low, y bit high) and
// the points within a cell; edges (u, v), u < v, with dx^2 + dy^2 < r^2 in
// binary64 (each operation rounded), in ascending (u, v).
#pragma once
#include "kg_kernels.hpp"

namespace kg {

constexpr uint32_t TAG_RTREE = 8;
constexpr uint32_t TAG_RPTS = 9;
constexpr uint32_t kRggMaxLevel = 14;
constexpr uint32_t kRggNone = 0xFFFFFFFFu;

struct RggJob {
    uint64_t n, seed, capacity;
    double r2, h;              // r * r, cell side 2^-L
    uint32_t L, G;             // level, cells per side
    uint64_t C;                // cells
    uint64_t *tree;            // node counts, level l at (4^l - 1) / 3, Morton order
    uint64_t *coff;            // C + 1 first vertex id of every cell
    uint32_t *pcell;           // n: cell of every vertex
    uint32_t *ecnt;            // n: edges (u, v > u) of every vertex u; top bit: more candidates than recorded
    uint64_t *bits;            // kRggBitWords x n (word-major): the count pass's test results per candidate
    uint64_t *wsum;            // ceil(n / 64) + 1: edges per wave of vertices, then their offsets
    uint64_t *woff;
    uint64_t *sums;            // scan partials
    uint64_t *status;          // [0] edges [1] overflow
    uint64_t *out_total;
    double2 *pts;
    uint2 *edges;
};

__device__ __forceinline__ uint64_t rgg_level_base(uint32_t l) { return ((1ull << (2 * l)) - 1) / 3; }

// Morton index <-> cell coordinates (L <= 14, so 28 bits)
__device__ __forceinline__ uint32_t spread_bits(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__device__ __forceinline__ uint32_t gather_bits(uint32_t z)
{
    z &= 0x55555555u;
    z = (z | (z >> 1)) & 0x33333333u;
    z = (z | (z >> 2)) & 0x0F0F0F0Fu;
    z = (z | (z >> 4)) & 0x00FF00FFu;
    z = (z | (z >> 8)) & 0x0000FFFFu;
    return z;
}

__global__ __launch_bounds__(64) void rgg_root_kernel(RggJob J)
{
    if (threadIdx.x == 0) J.tree[0] = J.n;
}

// One level of the quadrant recursion: lane per node of level l.
__global__ __launch_bounds__(64) void rgg_split_kernel(RggJob J, uint32_t l)
{
    const uint64_t z = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    if (z >= (1ull << (2 * l))) return;
    const uint64_t k = J.tree[rgg_level_base(l) + z];
    const uint64_t lower = binom(make_stream(J.seed, (uint32_t)z, 3 * l + 0, TAG_RTREE), k, 0.5);
    const uint64_t ll = binom(make_stream(J.seed, (uint32_t)z, 3 * l + 1, TAG_RTREE), lower, 0.5);
    const uint64_t ul = binom(make_stream(J.seed, (uint32_t)z, 3 * l + 2, TAG_RTREE), k - lower, 0.5);
    uint64_t *ch = J.tree + rgg_level_base(l + 1) + 4 * z;
    ch[0] = ll;
    ch[1] = lower - ll;
    ch[2] = ul;
    ch[3] = k - lower - ul;
}

// ---------------------------------------------------------------------------
// Exclusive scan of a u64 array of any length in three launches: tiles of
// 4096 (256 threads x 16 consecutive items) reduced, the tile sums scanned by
// one workgroup, the tiles scanned again with their prefix.  out[len] = total.
// ---------------------------------------------------------------------------
constexpr uint32_t kScanItems = 16;
constexpr uint64_t kScanTile = 256 * kScanItems;

__device__ __forceinline__ uint64_t block256_excl_scan(uint64_t v, uint64_t &total)
{
    __shared__ uint64_t s_w[4];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t incl = wave_incl_scan64(v);
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        const uint64_t x = s_w[i];
        if (i < w) before += x;
        tot += x;
    }
    total = tot;
    return before + incl - v;
}

// Loads and stores of a tile are lane-strided (item i x 256 + thread), so a
// wave's access covers 512 contiguous bytes; the apply pass goes through LDS
// to give each thread its 16 consecutive items.
__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint64_t *a, uint64_t len, uint64_t *sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x;
    uint64_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i)
        if (base + 256ull * i < len) s += a[base + 256ull * i];
    uint64_t total;
    (void)block256_excl_scan(s, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// in place over sums[0, nb); sums[nb] = total
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint64_t *sums, uint64_t nb)
{
    __shared__ uint64_t s_w[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += 1024) {
        const uint64_t i = base + t;
        const uint64_t v = i < nb ? sums[i] : 0;
        const uint64_t incl = wave_incl_scan64(v);
        if (lane == 63) s_w[wv] = incl;
        __syncthreads();
        uint64_t before = carry, total = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            const uint64_t x = s_w[w];
            if (w < wv) before += x;
            total += x;
        }
        if (i < nb) sums[i] = before + incl - v;
        carry += total;
        __syncthreads();
    }
    if (t == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const uint64_t *a, uint64_t len, const uint64_t *sums,
                                                         uint64_t *out)
{
    // item j of the tile at LDS word j + j / 16 (thread t's 16 items spread
    // over the banks)
    __shared__ uint64_t s_t[kScanTile + kScanTile / kScanItems];
    const uint32_t t = threadIdx.x;
    const uint64_t tb = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i) {
        const uint32_t j = 256 * i + t;
        s_t[j + j / kScanItems] = tb + j < len ? a[tb + j] : 0;
    }
    __syncthreads();
    const uint32_t p0 = t * (kScanItems + 1);
    uint64_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i) s += s_t[p0 + i];
    uint64_t total;
    uint64_t run = block256_excl_scan(s, total) + sums[blockIdx.x];
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i) {
        const uint64_t v = s_t[p0 + i];
        s_t[p0 + i] = run;
        run += v;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t i = 0; i < kScanItems; ++i) {
        const uint32_t j = 256 * i + t;
        if (tb + j < len) out[tb + j] = s_t[j + j / kScanItems];
    }
    if (blockIdx.x == 0 && t == 0) out[len] = sums[gridDim.x];
}

// ---------------------------------------------------------------------------
// Points: a wave per 64 consecutive cells, whose points are consecutive
// vertices; lane per point (stores of consecutive lanes are contiguous).  A
// point's cell is the last of the wave's cells whose first vertex is <= it
// (a binary search over the 64 offsets held one per lane).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void rgg_points_kernel(RggJob J)
{
    const uint64_t z0 = (uint64_t)blockIdx.x * 64;
    const uint32_t lane = threadIdx.x;
    const uint64_t first = J.coff[min(z0 + lane, J.C)];
    const uint64_t start = J.coff[z0], end = J.coff[min(z0 + 64, J.C)];
    for (uint64_t base = start; base < end; base += 64) {
        const uint64_t p = base + lane;
        uint32_t l = 0;
#pragma unroll
        for (uint32_t step = 32; step >= 1; step >>= 1) {
            const uint64_t v = __shfl(first, (int)(l + step), 64);
            if (v <= p) l += step;
        }
        const uint64_t j = p - __shfl(first, (int)l, 64);
        if (p < end) {
            const uint32_t z = (uint32_t)(z0 + l);
            const double cx = (double)gather_bits(z), cy = (double)gather_bits(z >> 1);
            const U4 w = make_stream(J.seed, z, 0, TAG_RPTS).block((uint32_t)j);
            const double U = unit_of(((uint64_t)w.y << 32) | w.x);
            const double V = unit_of(((uint64_t)w.w << 32) | w.z);
            J.pts[p] = make_double2((cx + U) * J.h, (cy + V) * J.h);
            J.pcell[p] = z;
        }
    }
}

// ---------------------------------------------------------------------------
// Edges: lane per vertex u.  The neighbour cells with Morton index >= u's
// cell, in ascending index, hold the ids above u's cell in ascending order;
// within u's own cell the candidates start at u + 1.
//
// Count pass (WRITE = false): every candidate is tested, four at a time.
// The wave first gathers the cells its vertices need (the windows of its at
// most seven cells, deduplicated by a sort across the lanes) and, if their
// points fit, copies them to LDS once; the tests then read LDS instead of
// global memory.  The results of the first 64 kRggBitWords candidates are kept as
// a bit mask per vertex (word w of vertex u at bits[w n + u], so a wave's
// stores are contiguous), the edge count per vertex and per wave of 64
// vertices are stored; a vertex with more candidates is flagged.
// Write pass (WRITE = true): at the wave's offset plus the in-wave prefix,
// the edges are read off the mask (candidate order again, set bits only);
// flagged vertices test their candidates again.  A wave's edges are
// contiguous in the output: they are gathered in LDS and stored with
// consecutive lanes on consecutive edges, unless they exceed the buffer.
// ---------------------------------------------------------------------------
constexpr uint32_t kRggStage = 640;    // edges per wave gathered in LDS (5 KB)
constexpr uint32_t kRggBitWords = 4;   // candidates recorded per vertex: 256
constexpr uint32_t kRggMore = 0x80000000u;
constexpr uint32_t kRggWinPts = 320;   // window points a count-pass wave copies to LDS (5 KB)

template <bool WRITE>
__global__ __launch_bounds__(64) void rgg_edges_kernel(RggJob J)
{
    __shared__ uint2 s_e[WRITE ? kRggStage : 1];
    const uint64_t u = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    uint64_t o = 0, wtotal = 0, lo = 0;
    bool more = false;
    if (WRITE) {
        if (J.status[1]) return;
        const uint32_t e = u < J.n ? J.ecnt[u] : 0;
        more = (e & kRggMore) != 0;
        const uint64_t k = e & ~kRggMore;
        const uint64_t incl = wave_incl_scan64(k);
        lo = incl - k;
        wtotal = __shfl(incl, 63, 64);
        o = J.woff[blockIdx.x];
    }
    const bool staged = wtotal <= kRggStage;
    // count pass: the points of every cell some lane of the wave needs
    // (the windows of the wave's cells, Morton index >= the cell), copied
    // to LDS once, if they fit: the candidate tests then read LDS
    __shared__ double2 s_p[WRITE ? 1 : kRggWinPts];
    __shared__ uint32_t s_cz[WRITE ? 1 : 64], s_co[WRITE ? 1 : 65];
    __shared__ uint64_t s_cs[WRITE ? 1 : 64];
    uint32_t U = 0;
    bool win = false;
    if (!WRITE && (uint64_t)blockIdx.x * 64 < J.n) {
        const uint32_t l = threadIdx.x;
        const uint64_t u0 = (uint64_t)blockIdx.x * 64;
        const uint64_t ul = u0 + 63 < J.n ? u0 + 63 : J.n - 1;
        const uint32_t zlo = J.pcell[u0], zhi = J.pcell[ul];
        if (9ull * (zhi - zlo + 1) <= 64) {
            uint32_t v = kRggNone;
            if (l < 9 * (zhi - zlo + 1)) {
                const uint32_t zc = zlo + l / 9;
                const int i = (int)(l % 9);
                const int x = (int)gather_bits(zc) + i % 3 - 1, y = (int)gather_bits(zc >> 1) + i / 3 - 1;
                if (x >= 0 && y >= 0 && x < (int)J.G && y < (int)J.G) {
                    const uint32_t zz = spread_bits((uint32_t)x) | (spread_bits((uint32_t)y) << 1);
                    if (zz >= zc) v = zz;
                }
            }
            // bitonic sort of the 64 lane values, ascending
#pragma unroll
            for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    const uint32_t w = (uint32_t)__shfl_xor((int)v, (int)j, 64);
                    v = (((l & j) == 0) == ((l & k) == 0)) ? min(v, w) : max(v, w);
                }
            }
            const uint32_t prev = (uint32_t)__shfl_up((int)v, 1, 64);
            const bool uniq = v != kRggNone && (l == 0 || v != prev);
            const uint64_t m = __ballot(uniq);
            U = (uint32_t)__popcll(m);
            const uint32_t idx = (uint32_t)__popcll(m & lanemask_lt(l));
            uint64_t st = 0, ct = 0;
            if (uniq) {
                st = J.coff[v];
                ct = J.coff[v + 1] - st;
            }
            const uint64_t incl = wave_incl_scan64(ct);
            const uint64_t total = __shfl(incl, 63, 64);
            if (total <= kRggWinPts) {
                if (uniq) {
                    s_cz[idx] = v;
                    s_cs[idx] = st;
                    s_co[idx] = (uint32_t)(incl - ct);
                }
                if (l == 0) s_co[U] = (uint32_t)total;
                __syncthreads();
                for (uint32_t i = 0; i < U; ++i) {
                    const uint32_t ob = s_co[i], len = s_co[i + 1] - ob;
                    const uint64_t sb = s_cs[i];
                    for (uint32_t t = l; t < len; t += 64) s_p[ob + t] = J.pts[sb + t];
                }
                __syncthreads();
                win = true;
            }
        }
    }
    uint32_t cnt = 0;
    uint64_t c = 0;       // candidates seen
    if (u < J.n) {
        const uint32_t z = J.pcell[u];
        const int cx = (int)gather_bits(z), cy = (int)gather_bits(z >> 1);
        uint32_t nb[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int x = cx + i % 3 - 1, y = cy + i / 3 - 1;
            const bool in = x >= 0 && y >= 0 && x < (int)J.G && y < (int)J.G;
            const uint32_t zz = in ? (spread_bits((uint32_t)x) | (spread_bits((uint32_t)y) << 1)) : kRggNone;
            nb[i] = zz >= z ? zz : kRggNone;
        }
        // odd-even transposition sort of the nine indices
#pragma unroll
        for (int r = 0; r < 9; ++r) {
#pragma unroll
            for (int i = r & 1; i + 1 < 9; i += 2) {
                const uint32_t a = min(nb[i], nb[i + 1]), b = max(nb[i], nb[i + 1]);
                nb[i] = a;
                nb[i + 1] = b;
            }
        }
        auto emit = [&](uint64_t b) {
            const uint2 e = make_uint2((uint32_t)u, (uint32_t)b);
            if (staged) s_e[lo + cnt] = e;
            else J.edges[o + lo + cnt] = e;
            ++cnt;
        };
        if (!WRITE) {
            const double2 p = J.pts[u];
            const double r2 = J.r2;
            uint64_t cur = 0;
            auto hit = [&](const double2 q) -> uint32_t {
                const double dx = p.x - q.x, dy = p.y - q.y;
                return dx * dx + dy * dy < r2 ? 1u : 0u;
            };
            // append nbits (1..4) result bits v to the mask: a full word is
            // stored (if recorded), a word boundary inside v carries over
            auto put = [&](uint32_t v, uint32_t nbits) {
                const uint32_t off = (uint32_t)(c & 63);
                const uint64_t w = c >> 6;
                cur |= (uint64_t)v << off;
                c += nbits;
                if (off + nbits >= 64) {
                    if (w < kRggBitWords) J.bits[w * J.n + u] = cur;
                    cur = off + nbits > 64 ? (uint64_t)(v >> (64 - off)) : 0;
                }
            };
            if (win) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const uint32_t zz = nb[i];
                    if (zz == kRggNone) continue;
                    uint32_t a = 0, e = U;
                    while (e - a > 1) {
                        const uint32_t mid = (a + e) >> 1;
                        if (s_cz[mid] <= zz) a = mid;
                        else e = mid;
                    }
                    const uint64_t sb = s_cs[a];
                    const uint32_t ob = s_co[a];
                    const uint32_t t1 = s_co[a + 1] - ob;
                    uint32_t t = zz == z ? (uint32_t)(u + 1 - sb) : 0;
                    for (; t + 4 <= t1; t += 4) {
                        const double2 q0 = s_p[ob + t], q1 = s_p[ob + t + 1], q2 = s_p[ob + t + 2],
                                      q3 = s_p[ob + t + 3];
                        const uint32_t v = hit(q0) | (hit(q1) << 1) | (hit(q2) << 2) | (hit(q3) << 3);
                        cnt += (uint32_t)__builtin_popcount(v);
                        put(v, 4);
                    }
                    for (; t < t1; ++t) {
                        const uint32_t v = hit(s_p[ob + t]);
                        cnt += v;
                        put(v, 1);
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const uint32_t zz = nb[i];
                    if (zz == kRggNone) continue;
                    const uint64_t b1 = J.coff[zz + 1];
                    uint64_t b = zz == z ? u + 1 : J.coff[zz];
                    for (; b + 4 <= b1; b += 4) {
                        const double2 q0 = J.pts[b], q1 = J.pts[b + 1], q2 = J.pts[b + 2], q3 = J.pts[b + 3];
                        const uint32_t v = hit(q0) | (hit(q1) << 1) | (hit(q2) << 2) | (hit(q3) << 3);
                        cnt += (uint32_t)__builtin_popcount(v);
                        put(v, 4);
                    }
                    for (; b < b1; ++b) {
                        const uint32_t v = hit(J.pts[b]);
                        cnt += v;
                        put(v, 1);
                    }
                }
            }
            if ((c & 63) != 0 && (c >> 6) < kRggBitWords) J.bits[(c >> 6) * J.n + u] = cur;
        } else if (more) {
            const double2 p = J.pts[u];
            const double r2 = J.r2;
            auto test = [&](const double2 q, uint64_t b) {
                const double dx = p.x - q.x, dy = p.y - q.y;
                if (dx * dx + dy * dy < r2) emit(b);
            };
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint32_t zz = nb[i];
                if (zz == kRggNone) continue;
                const uint64_t b1 = J.coff[zz + 1];
                uint64_t b = zz == z ? u + 1 : J.coff[zz];
                for (; b + 4 <= b1; b += 4) {
                    const double2 q0 = J.pts[b], q1 = J.pts[b + 1], q2 = J.pts[b + 2], q3 = J.pts[b + 3];
                    test(q0, b);
                    test(q1, b + 1);
                    test(q2, b + 2);
                    test(q3, b + 3);
                }
                for (; b < b1; ++b) test(J.pts[b], b);
            }
        } else {
            // the recorded results: walk the candidates in the same order,
            // a word at a time, and emit the set bits
            uint32_t wcur = kRggNone;
            uint64_t word = 0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint32_t zz = nb[i];
                if (zz == kRggNone) continue;
                const uint64_t b1 = J.coff[zz + 1];
                uint64_t b = zz == z ? u + 1 : J.coff[zz];
                while (b < b1) {
                    const uint32_t w = (uint32_t)(c >> 6), off = (uint32_t)(c & 63);
                    if (w != wcur) {
                        word = J.bits[(uint64_t)w * J.n + u];
                        wcur = w;
                    }
                    const uint64_t take = min((uint64_t)(64 - off), b1 - b);
                    uint64_t m = word >> off;
                    if (take < 64) m &= (1ull << take) - 1;
                    while (m) {
                        emit(b + (uint64_t)__builtin_ctzll(m));
                        m &= m - 1;
                    }
                    b += take;
                    c += take;
                }
            }
        }
    }
    if (!WRITE) {
        if (u < J.n) J.ecnt[u] = cnt | (c > 64ull * kRggBitWords ? kRggMore : 0u);
        const uint64_t incl = wave_incl_scan64((uint64_t)cnt);
        if (threadIdx.x == 63) J.wsum[blockIdx.x] = incl;
    } else if (staged) {
        __syncthreads();
        for (uint64_t i = threadIdx.x; i < wtotal; i += 64) J.edges[o + i] = s_e[i];
    }
}

// The total, the overflow flag and the caller's copy of the total.
__global__ __launch_bounds__(64) void rgg_total_kernel(RggJob J, uint64_t nw)
{
    if (threadIdx.x != 0) return;
    const uint64_t E = J.woff[nw];
    J.status[0] = E;
    J.status[1] = E > J.capacity ? 1 : 0;
    if (J.out_total) *J.out_total = E;
}

}  // namespace kg
