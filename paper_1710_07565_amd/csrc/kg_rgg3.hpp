// kg_rgg3.hpp -- three-dimensional random geometric graphs: n points uniform
// in the unit cube, an edge between every two points closer than r (Sec.
// 2.1.2, d = 3), generated as in Sec. 5: a grid of 8^L cells of side
// 2^-L >= max(r, n^-1/3); the points per cell by an octant recursion of
// binomial variates, each node drawing from a stream keyed by the node (Sec.
// 5.1, 2^d - 1 = 7 variates per split); the points of a cell from the cell's
// own stream; edges by comparing each point with the points of its cell and
// the 26 neighbours, counted, prefix-summed and written in a second pass
// (Sec. 5.3).
//
// A node at level l (Morton index z) holding k points draws seven
// Bin(., 1/2) variates, stream (seed; j, z, 7 l + slot, TAG_RTREE3): the
// lower z half (slot 0), the lower y halves of the lower and the upper z half
// (slots 1, 2), the lower x halves of the four (y, z) quarters in Morton
// order (slots 3..6).  Every node is computed once, level by level; its value
// is the one any root path to it gives, since it depends only on its own
// count and stream.  Point j of cell z is ((c + U) 2^-L per axis), U the
// 64-bit uniforms 3j (x), 3j + 1 (y), 3j + 2 (z) of (seed; ., z, 0,
// TAG_RPTS3), 64-bit draw t being the half t mod 2 of block floor(t / 2).
// Vertex ids follow the cells in Morton order (x bit lowest, then y, then
// z) and the points within a cell; edges (u, v), u < v, with
// (dx^2 + dy^2) + dz^2 < r^2 in binary64 (each operation rounded), in
// ascending (u, v).
#pragma once
#include "kg_rgg.hpp"

namespace kg {

constexpr uint32_t TAG_RTREE3 = 10;
constexpr uint32_t TAG_RPTS3 = 11;
constexpr uint32_t kRgg3MaxLevel = 10;     // 8^10 cells: Morton indices below 2^30
constexpr uint32_t kRgg3Win = 27;          // cells of a 3 x 3 x 3 window
constexpr uint32_t kRgg3BitWords = 2;      // candidates recorded per vertex: 128 (about 54 on average)

struct Rgg3Job {
    uint64_t n, seed, capacity;
    double r2, h;              // r * r, cell side 2^-L
    uint32_t L, G;             // level, cells per side
    uint64_t C;                // cells
    uint64_t *tree;            // node counts, level l at (8^l - 1) / 7, Morton order
    uint64_t *coff;            // C + 1 first vertex id of every cell
    uint32_t *pcell;           // n: cell of every vertex
    uint32_t *ecnt;            // n: edges (u, v > u) of every vertex u; top bit: more candidates than recorded
    uint64_t *bits;            // kRgg3BitWords x n (word-major): the count pass's test results per candidate
    uint64_t *wsum;            // ceil(n / 64) + 1: edges per wave of vertices, then their offsets
    uint64_t *woff;
    uint64_t *sums;            // scan partials
    uint64_t *status;          // [0] edges [1] overflow
    uint64_t *out_total;
    double *pts;               // 3 n: x, y, z of every vertex
    uint2 *edges;
};

__device__ __forceinline__ uint64_t rgg3_level_base(uint32_t l) { return ((1ull << (3 * l)) - 1) / 7; }

// Morton index <-> cell coordinates (L <= 10, so 30 bits): every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t x)
{
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t gather3(uint32_t z)
{
    z &= 0x09249249u;
    z = (z | (z >> 2)) & 0x030C30C3u;
    z = (z | (z >> 4)) & 0x0300F00Fu;
    z = (z | (z >> 8)) & 0x030000FFu;
    z = (z | (z >> 16)) & 0x3FFu;
    return z;
}

__global__ __launch_bounds__(64) void rgg3_root_kernel(Rgg3Job J)
{
    if (threadIdx.x == 0) J.tree[0] = J.n;
}

// One level of the octant recursion: lane per node of level l.
__global__ __launch_bounds__(64) void rgg3_split_kernel(Rgg3Job J, uint32_t l)
{
    const uint64_t z = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    if (z >= (1ull << (3 * l))) return;
    const uint64_t k = J.tree[rgg3_level_base(l) + z];
    const uint32_t a = (uint32_t)z, b = 7 * l;
    const uint64_t lz = binom(make_stream(J.seed, a, b + 0, TAG_RTREE3), k, 0.5);
    const uint64_t y0 = binom(make_stream(J.seed, a, b + 1, TAG_RTREE3), lz, 0.5);
    const uint64_t y1 = binom(make_stream(J.seed, a, b + 2, TAG_RTREE3), k - lz, 0.5);
    const uint64_t quarter[4] = {y0, lz - y0, y1, k - lz - y1};     // (y, z) = 00, 10, 01, 11
    uint64_t *ch = J.tree + rgg3_level_base(l + 1) + 8 * z;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t x0 = binom(make_stream(J.seed, a, b + 3 + (uint32_t)i, TAG_RTREE3), quarter[i], 0.5);
        ch[2 * i] = x0;
        ch[2 * i + 1] = quarter[i] - x0;
    }
}

// Points: a wave per 64 consecutive cells, lane per point (as in two
// dimensions); point j draws blocks floor(3j / 2) and the next one.
__global__ __launch_bounds__(64) void rgg3_points_kernel(Rgg3Job J)
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
            const Stream st = make_stream(J.seed, z, 0, TAG_RPTS3);
            const uint64_t t0 = 3 * j;
            const U4 w0 = st.block((uint32_t)(t0 >> 1)), w1 = st.block((uint32_t)(t0 >> 1) + 1);
            // the six 64-bit halves of the two blocks; draws t0, t0 + 1, t0 + 2
            // start at half t0 mod 2
            uint64_t d[3];
            if ((t0 & 1) == 0) {
                d[0] = ((uint64_t)w0.y << 32) | w0.x;
                d[1] = ((uint64_t)w0.w << 32) | w0.z;
                d[2] = ((uint64_t)w1.y << 32) | w1.x;
            } else {
                d[0] = ((uint64_t)w0.w << 32) | w0.z;
                d[1] = ((uint64_t)w1.y << 32) | w1.x;
                d[2] = ((uint64_t)w1.w << 32) | w1.z;
            }
            double *q = J.pts + 3 * p;
#pragma unroll
            for (int a = 0; a < 3; ++a) q[a] = ((double)gather3(z >> a) + unit_of(d[a])) * J.h;
            J.pcell[p] = z;
        }
    }
}

// The window of cell z: the cells of its 3 x 3 x 3 neighbourhood with Morton
// index >= z, ascending (kRggNone past the last), by odd-even transposition.
__device__ __forceinline__ void rgg3_window(uint32_t z, uint32_t G, uint32_t (&nb)[kRgg3Win])
{
    const int cx = (int)gather3(z), cy = (int)gather3(z >> 1), cz = (int)gather3(z >> 2);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int x = cx + i % 3 - 1, y = cy + (i / 3) % 3 - 1, w = cz + i / 9 - 1;
        const bool in = x >= 0 && y >= 0 && w >= 0 && x < (int)G && y < (int)G && w < (int)G;
        const uint32_t zz = in ? (spread3((uint32_t)x) | (spread3((uint32_t)y) << 1) | (spread3((uint32_t)w) << 2))
                               : kRggNone;
        nb[i] = zz >= z ? zz : kRggNone;
    }
#pragma unroll
    for (int r = 0; r < 27; ++r) {
#pragma unroll
        for (int i = r & 1; i + 1 < 27; i += 2) {
            const uint32_t a = min(nb[i], nb[i + 1]), b = max(nb[i], nb[i + 1]);
            nb[i] = a;
            nb[i + 1] = b;
        }
    }
}

// Edges: lane per vertex u; the window cells, in ascending Morton index,
// hold the ids above u's cell in ascending order; within u's own cell the
// candidates start at u + 1.  The windows of the (at most 64) cells a wave's
// vertices lie in are sorted once, one lane per cell, into LDS.  Count pass
// (WRITE = false): per-vertex and per-wave edge counts, and the results of
// the vertex's first 128 candidate tests as a bit mask (word-major, so a
// wave's stores are contiguous; a vertex with more candidates is flagged).
// Write pass: the same walk reading the mask (flagged vertices test again),
// the edges stored at the wave's offset plus the in-wave prefix, gathered in
// LDS and stored with consecutive lanes on consecutive edges unless they
// exceed the buffer.
template <bool WRITE>
__global__ __launch_bounds__(64) void rgg3_edges_kernel(Rgg3Job J)
{
    __shared__ uint2 s_e[WRITE ? kRggStage : 1];
    __shared__ uint32_t s_win[64][kRgg3Win];
    const uint32_t lane = threadIdx.x;
    const uint64_t u = (uint64_t)blockIdx.x * 64 + lane;
    uint64_t o = 0, wtotal = 0, lo = 0;
    if (WRITE) {
        if (J.status[1]) return;
        const uint64_t k = u < J.n ? (J.ecnt[u] & ~kRggMore) : 0;
        const uint64_t incl = wave_incl_scan64(k);
        lo = incl - k;
        wtotal = __shfl(incl, 63, 64);
        o = J.woff[blockIdx.x];
    }
    const bool staged = wtotal <= kRggStage;
    const uint64_t u0 = (uint64_t)blockIdx.x * 64;
    // (a wave without vertices -- n = 0 -- only stores its zero sum)
    const uint64_t ul = u0 + 63 < J.n ? u0 + 63 : J.n - 1;
    const uint32_t zlo = u0 < J.n ? J.pcell[u0] : 0, zhi = u0 < J.n ? J.pcell[ul] : 0;
    // the windows in LDS: one per cell of the wave (sorted once per cell), or,
    // when the wave's vertices spread over more than 64 cells, one per lane
    const bool shared = u0 < J.n && zhi - zlo < 64;
    if (u0 < J.n) {
        const bool mine = shared ? lane <= zhi - zlo : u < J.n;
        if (mine) {
            uint32_t nb[kRgg3Win];
            rgg3_window(shared ? zlo + lane : J.pcell[u], J.G, nb);
#pragma unroll
            for (int i = 0; i < 27; ++i) s_win[lane][i] = nb[i];
        }
        __syncthreads();
    }
    uint32_t cnt = 0;
    uint64_t c = 0;       // candidates seen
    bool more = false;
    if (WRITE && u < J.n) more = (J.ecnt[u] & kRggMore) != 0;
    if (u < J.n) {
        const uint32_t z = J.pcell[u];
        const uint32_t *nb = s_win[shared ? z - zlo : lane];
        auto emit = [&](uint64_t b) {
            const uint2 e = make_uint2((uint32_t)u, (uint32_t)b);
            if (staged) s_e[lo + cnt] = e;
            else J.edges[o + lo + cnt] = e;
            ++cnt;
        };
        if (!WRITE || more) {
            const double *p = J.pts + 3 * u;
            const double px = p[0], py = p[1], pz = p[2];
            const double r2 = J.r2;
            uint64_t cur = 0;
            // count pass: append nbits (1..4) result bits v to the vertex's
            // mask; a full word is stored if recorded, a word boundary inside
            // v carries over
            auto put = [&](uint32_t v, uint32_t nbits) {
                const uint32_t off = (uint32_t)(c & 63);
                const uint64_t w = c >> 6;
                cur |= (uint64_t)v << off;
                c += nbits;
                if (off + nbits >= 64) {
                    if (w < kRgg3BitWords) J.bits[w * J.n + u] = cur;
                    cur = off + nbits > 64 ? (uint64_t)(v >> (64 - off)) : 0;
                }
            };
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                const uint32_t zz = nb[i];
                if (zz == kRggNone) continue;
                const uint64_t b1 = J.coff[zz + 1];
                // four candidates' loads in flight per trip (a cell holds a
                // few points, so most cells take one trip)
                for (uint64_t b = zz == z ? u + 1 : J.coff[zz]; b < b1; b += 4) {
                    double q[4][3];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (b + t < b1) {
                            const double *src = J.pts + 3 * (b + t);
                            q[t][0] = src[0];
                            q[t][1] = src[1];
                            q[t][2] = src[2];
                        }
                    }
                    uint32_t v = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (b + t >= b1) break;
                        const double dx = px - q[t][0], dy = py - q[t][1], dz = pz - q[t][2];
                        if ((dx * dx + dy * dy) + dz * dz < r2) {
                            if (WRITE) emit(b + t);
                            else v |= 1u << t;
                        }
                    }
                    if (!WRITE) {
                        cnt += (uint32_t)__builtin_popcount(v);
                        put(v, (uint32_t)min((uint64_t)4, b1 - b));
                    }
                }
            }
            if (!WRITE && (c & 63) != 0 && (c >> 6) < kRgg3BitWords) J.bits[(c >> 6) * J.n + u] = cur;
        } else {
            // the recorded results: walk the candidates in the same order, a
            // word at a time, and emit the set bits
            uint32_t wcur = kRggNone;
            uint64_t word = 0;
#pragma unroll
            for (int i = 0; i < 27; ++i) {
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
        if (u < J.n) J.ecnt[u] = cnt | (c > 64ull * kRgg3BitWords ? kRggMore : 0u);
        const uint64_t incl = wave_incl_scan64((uint64_t)cnt);
        if (lane == 63) J.wsum[blockIdx.x] = incl;
    } else if (staged) {
        __syncthreads();
        for (uint64_t i = lane; i < wtotal; i += 64) J.edges[o + i] = s_e[i];
    }
}

// The total, the overflow flag and the caller's copy of the total.
__global__ __launch_bounds__(64) void rgg3_total_kernel(Rgg3Job J, uint64_t nw)
{
    if (threadIdx.x != 0) return;
    const uint64_t E = J.woff[nw];
    J.status[0] = E;
    J.status[1] = E > J.capacity ? 1 : 0;
    if (J.out_total) *J.out_total = E;
}

}  // namespace kg
