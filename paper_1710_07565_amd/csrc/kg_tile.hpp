// kg_tile.hpp -- the sampler's two kernels.
//
//   tile_kernel  : the common case.  One wavefront per tile; a tile whose
//                  base case needs at most kFastDraws draws keeps them in
//                  registers (16 per lane), sorts them in LDS and streams the
//                  decoded edges out.  Any other tile is appended to a queue.
//   queue_kernel : the queued tiles, with the general base case (key
//                  sub-ranges when the draws exceed the LDS capacity).
//
// Both produce the same bits for a tile: the sorted distinct set of the
// first J draws of the tile's stream with J the smallest count giving k
// distinct valid values (Sec. 2.2 base case; Sec. 4.1, 4.2 offsets).
#pragma once
#include "kg_kernels.hpp"

namespace kg {

constexpr uint32_t kFastDraws = 1280;   // draws of one wave's base case (at most 5 Philox blocks per lane)
constexpr uint32_t kFastRounds = 5;     // rounds of 256 draws (one Philox block per lane each)
constexpr uint32_t kKeyWords = 1288;    // LDS key words: >= kFastDraws + 3 and >= the widest sort span (64 x 20)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kGrabBig = 32;       // tiles per range a workgroup takes from the shared counter ...
constexpr uint64_t kGrabSmall = 8;      // ... and near the end of the walk
constexpr uint64_t kTailTiles = 64;     // tiles per workgroup handed out in small ranges

// Wave-uniform 64-bit load through the scalar data cache.  Only for data
// that no lane writes while the kernel runs (sizes and offsets written by
// the earlier kernels of the pass).
__device__ __forceinline__ uint64_t ld_uni(const uint64_t *p)
{
    return *(const __attribute__((address_space(4))) uint64_t *)p;
}

// The chunk of tile t (wave-uniform): the last g with tstart[g] <= t.  A
// 64-way search: at each level the lanes probe 64 evenly spaced entries of
// the candidate range and the count of those <= t (a prefix of the lanes,
// the starts being sorted) picks the sub-range, so the wave waits for
// ceil(log64 G) loads, not log2 G.  Keeps tstart[lo] <= t (tstart[0] = 0).
__device__ __forceinline__ uint64_t chunk_of_tile(const Job &job, uint64_t t)
{
    const uint64_t lane = threadIdx.x & 63;
    uint64_t lo = 0, n = job.G;
    while (n > 1) {
        const uint64_t step = (n + 63) >> 6;
        const uint64_t p = lo + lane * step;
        const bool le = p < lo + n && job.tstart[p] <= t;
        const uint64_t c = (uint64_t)__popcll(__ballot(le));   // >= 1: lane 0 probes lo
        const uint64_t end = lo + n;
        lo += (c - 1) * step;
        n = end - lo < step ? end - lo : step;
    }
    return lo;
}

// Ranges of tiles for a persistent grid, in tile order: workgroup b takes
// range b first, then the next one not yet handed out, from the counter
// status[5] (cleared by the scan kernel), so a workgroup whose tiles were
// cheap takes more and none waits on a slow tail.  Ranges of kGrabBig tiles
// first, then, for the last kTailTiles tiles per workgroup of the grid,
// ranges of kGrabSmall, so that the walk ends evenly and the counter, the
// chunk search and the chunk set-up are paid once per kGrabBig tiles for
// most of it.  Walks with fewer than 4 x kGrabBig tiles per workgroup take
// smaller ranges (down to one tile) so that small jobs still spread over the
// grid; when the grid holds every range, no workgroup touches the counter.
struct TileGrab {
    uint64_t T, head, qh, Q;   // tiles, tiles in large ranges, large ranges, all ranges
    uint64_t big, small;       // range sizes
    bool first;

    __device__ __forceinline__ TileGrab(uint64_t tiles)
    {
        T = tiles;
        const uint64_t W = gridDim.x;
        const uint64_t fair = T / (4 * W);
        small = fair >= kGrabSmall ? kGrabSmall : fair > 0 ? fair : 1;
        big = fair >= kGrabBig ? kGrabBig : fair > small ? fair : small;
        const uint64_t tail = W * kTailTiles;
        head = T > tail ? T - tail : 0;
        qh = (head + big - 1) / big;
        Q = qh + (T - head + small - 1) / small;
        first = true;
    }

    // the next range [t0, t1); false once every range has been handed out
    __device__ __forceinline__ bool next(const Job &job, uint64_t &t0, uint64_t &t1)
    {
        const uint64_t W = gridDim.x;
        uint64_t q;
        if (first) {
            q = blockIdx.x;
            first = false;
        } else if (Q <= W) {
            return false;
        } else {
            uint64_t b = 0;
            if (threadIdx.x == 0) b = atomicAdd((unsigned long long *)(job.status + 5), 1ull);
            q = W + uni64(b);
        }
        if (q >= Q) return false;
        if (q < qh) {
            t0 = q * big;
            t1 = t0 + big < head ? t0 + big : head;
        } else {
            t0 = head + (q - qh) * small;
            t1 = t0 + small < T ? t0 + small : T;
        }
        return true;
    }
};

// The chunk a wave is in: chunk constants, the stream and the decoder of
// its tiles (enter), the chunk of a tile (locate) and the context of one
// tile (tile).  The tile kernel advances the decoder from tile to tile itself;
// the queue kernel places every tile from scratch.
struct TileWalk {
    uint64_t g, gstart, gend;   // current chunk, its first tile, first tile of the next
    uint64_t N;                 // slots of the chunk
    uint64_t qs;                // 2^s = qs * dv + rs
    uint32_t s;                 // tile exponent
    uint32_t row0;              // first row of the chunk (directed) or its row section
    uint32_t rs;
    TileCtx tc;

    __device__ __forceinline__ void enter(const Job &job, uint64_t gg)
    {
        g = gg;
        gstart = ld_uni(job.tstart + g);
        gend = ld_uni(job.tstart + g + 1);
        // the fields the sampler needs, through the scalar cache for batches
        Inst I;
        memset(&I, 0, sizeof(I));
        if (job.ninst == 1) {
            I.n = job.one.n; I.seed = job.one.seed; I.chunk_base = job.one.chunk_base;
            I.directed = job.one.directed; I.P = job.one.P; I.s = job.one.s; I.view = job.one.view;
        } else {
            const __attribute__((address_space(4))) Inst *q =
                (const __attribute__((address_space(4))) Inst *)(job.insts + inst_of_chunk(job, g));
            I.n = q->n; I.seed = q->seed; I.chunk_base = q->chunk_base;
            I.directed = q->directed; I.P = q->P; I.s = q->s; I.view = q->view;
        }
        const uint32_t c = uni((uint32_t)chunk_ordinal(I, g - I.chunk_base));
        s = uni(I.s);
        const Chunk ch = chunk_geometry(I, c);
        N = uni64(ch.N);
        Decoder &d = tc.dec;
        d.r0 = d.c0 = d.b = d.a = d.h = 0;
        d.Ttri = d.lbase = 0;
        d.wide = 0;
        uint64_t dv;
        if (I.directed) {
            d.type = 0; dv = I.n - 1; row0 = uni((uint32_t)ch.row0);
        } else if (!ch.diag) {
            d.type = 1; dv = ch.w; d.b = uni((uint32_t)ch.b); row0 = uni((uint32_t)ch.a);
        } else {
            d.type = 2; dv = 1; row0 = uni((uint32_t)ch.a);
            d.a = row0; d.h = uni((uint32_t)ch.h); d.Ttri = N;
        }
        if (dv == 0) dv = 1;
        d.type = uni(d.type);
        d.dv = uni((uint32_t)dv);
        d.pow2 = uni((dv & (dv - 1)) == 0);
        d.sh = uni(63 - __clzll(dv));
        d.rcp = unid(1.0 / (double)dv);
        qs = uni64((1ull << s) / dv);
        rs = uni((uint32_t)((1ull << s) - qs * dv));
        tc.st = Stream{uni((uint32_t)I.seed), uni((uint32_t)(I.seed >> 32)), c, 0, TAG_TLEAF};
    }

    // the chunk of tile t, entered
    __device__ __forceinline__ void locate(const Job &job, uint64_t t) { enter(job, chunk_of_tile(job, t)); }

    // slot count, stream counter and decoding constants of tile t (of the
    // current chunk)
    __device__ __forceinline__ void tile(uint64_t t)
    {
        Decoder &d = tc.dec;
        const uint64_t tl = t - gstart;
        const uint64_t lstart = tl << s;
        if (d.type == 2) {
            d.lbase = lstart;
        } else {
            const uint64_t q = lstart / d.dv;
            d.c0 = uni((uint32_t)(lstart - q * d.dv));
            d.r0 = uni(row0 + (uint32_t)q);
        }
        d.lbase = uni64(d.lbase);
        tc.S = uni64((N - lstart) < (1ull << s) ? (N - lstart) : (1ull << s));
        tc.bits = uni(tc.S <= 1 ? 0 : 64 - __clzll(tc.S - 1));
        tc.mask = uni(tc.bits >= 32 ? 0xFFFFFFFFu : ((1u << tc.bits) - 1));
        tc.full = uni(tc.S == (1ull << tc.bits));
        tc.st.b = uni((uint32_t)tl);
        d.wide = uni((uint64_t)d.c0 + tc.S > (1ull << 32));
    }
};

// Lane-to-lane moves of the sort (wave-wide DPP shifts by one lane); the
// lane without a source keeps `edge`.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t x, uint32_t edge)
{
    return __builtin_amdgcn_update_dpp(edge, x, 0x130, 0xF, 0xF, false);   // wave_shl:1, lane 63 keeps edge
}
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t x, uint32_t edge)
{
    return __builtin_amdgcn_update_dpp(edge, x, 0x138, 0xF, 0xF, false);   // wave_shr:1, lane 0 keeps edge
}

template <int W>
__device__ __forceinline__ void wload(const uint32_t *s, uint32_t p0, uint32_t *v)
{
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = s[p0 + i];
}
template <int W>
__device__ __forceinline__ void wstore(uint32_t *s, uint32_t p0, const uint32_t *v)
{
#pragma unroll
    for (int i = 0; i < W; ++i) s[p0 + i] = v[i];
}

// The lane index as a fresh register value: addresses derived from it are
// formed where they are used instead of being kept (and spilled) across the
// whole tile loop.
__device__ __forceinline__ uint32_t lane_here()
{
    uint32_t r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(threadIdx.x));
    return r;
}

__device__ __forceinline__ void cx(uint32_t &a, uint32_t &b)
{
    const uint32_t x = a, y = b;
    a = x < y ? x : y;
    b = x < y ? y : x;
}

// Sort of s[0, 64 W) (W even) after the bucket placement: the keys are in
// bucket order (bucket = top bits), arbitrary inside a bucket, and no bucket
// holds more than R keys.  Lane L holds positions [W L, W L + W) in
// registers and the wave runs R rounds of odd-even transposition sort:
// even rounds compare-exchange the pairs (2j, 2j + 1), all inside a lane;
// odd rounds the pairs (2j + 1, 2j + 2), the pair across two lanes by DPP
// (each lane computes its own side from the old values).  A pair of keys
// from two buckets is already in order and never exchanged, so every bucket
// is sorted on its own, as a sequence of at most R elements, which R rounds
// of odd-even transposition sort (Knuth, TAOCP vol. 3, 5.3.4) always sort.
// Returns the number of equal adjacent pairs among the first V positions.
template <int W>
__device__ __forceinline__ uint32_t oddeven(uint32_t *s, uint32_t V, uint32_t R)
{
    const uint32_t lane = lane_here();
    const uint32_t p0 = W * lane;
    uint32_t v[W];
    wload<W>(s, p0, v);
    // rounds in pairs (an extra round leaves a sorted sequence sorted)
    for (uint32_t r = 0; r < R; r += 2) {
#pragma unroll
        for (int i = 0; i < W; i += 2) cx(v[i], v[i + 1]);
        const uint32_t nx = from_next_lane(v[0], kNone);     // lane 63: the padding bound
        const uint32_t pv = from_prev_lane(v[W - 1], 0u);    // lane 0: no predecessor
#pragma unroll
        for (int i = 1; i + 1 < W; i += 2) cx(v[i], v[i + 1]);
        v[W - 1] = v[W - 1] < nx ? v[W - 1] : nx;
        v[0] = v[0] > pv ? v[0] : pv;
    }
    wstore<W>(s, p0, v);
    uint32_t eq = 0;
#pragma unroll
    for (int i = 0; i + 1 < W; ++i) eq += __popcll(__ballot(v[i] == v[i + 1]));
    const uint32_t nx = from_next_lane(v[0], ~v[W - 1]);       // lane 63: a value unequal to its last key
    eq += __popcll(__ballot(v[W - 1] == nx));
    // the pairs inside the padding [V, 64 W) are all equal; (V - 1, V) is not
    constexpr uint32_t span = 64 * W;
    return V < span ? eq - (span - 1 - V) : eq;
}

// Maximum over the 64 lanes (DPP row shifts, then row broadcasts; lane 63
// ends with the maximum).
__device__ __forceinline__ uint32_t wave_max32(uint32_t v)
{
    uint32_t t;
    t = __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xF, 0xF, false); v = v > t ? v : t;   // row_shr:1
    t = __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xF, 0xF, false); v = v > t ? v : t;   // row_shr:2
    t = __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xF, 0xF, false); v = v > t ? v : t;   // row_shr:4
    t = __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xF, 0xF, false); v = v > t ? v : t;   // row_shr:8
    t = __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false); v = v > t ? v : t;   // row_bcast:15
    t = __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false); v = v > t ? v : t;   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Base case of the common tiles.  Pass 1 (one Philox block per lane and
// round; lane L computes blocks L + 64 e, i.e. draws 256 e + 4 L + q) counts
// every valid draw in its bucket -- the top min(9, bits) bits of the key,
// 512 32-bit counters -- and keeps the draws in registers (rejected ones as
// ~0), together with its rank among the draws of its bucket (the value
// the LDS atomic returned).  An exclusive scan turns the counters into bucket
// starts; pass 2 places each draw at its bucket start plus its rank; as
// many rounds of odd-even transposition as the fullest bucket has keys (8 to
// 14 keys per lane) then sort inside buckets, and repeats are counted.
// While fewer than ke distinct values are seen, J grows by the shortfall
// (each draw adds at most one new value).  Leaves the sorted set in s[0..ke)
// and returns true, or returns false once J would exceed lim (or in the rare
// cases the queue kernel handles); the counters are zero again whenever it
// returns.
constexpr uint32_t kBucketWords = 512;   // one 32-bit counter per bucket
constexpr uint32_t kMaxRounds = 32;      // a fuller bucket sends the tile to the queue

__device__ __forceinline__ bool fast_set(const TileCtx &t, uint32_t *s, uint32_t *cnt, uint32_t ke, uint32_t lim)
{
    const uint32_t lane = threadIdx.x;
    const uint32_t S32 = (uint32_t)t.S;                 // used only when S < 2^bits <= 2^32
    const uint32_t shift = t.bits > 9 ? t.bits - 9 : 0;
    uint4 *cw = reinterpret_cast<uint4 *>(cnt) + 2 * lane;   // this lane's 8 counter words
    uint32_t J = ke;
    for (;;) {
        if (J > lim) return false;
        // the counters are zero here: cleared at the start of the kernel and
        // after every use (below)
        const uint32_t nit = uni((J + 255) >> 8);
        // rounds whose 256 draws all lie below J: in a full tile with keys
        // below 2^31 every such draw is valid and needs no checks
        const bool nclean_tile = t.full && t.bits < 32;
        const uint32_t nclean = nclean_tile ? uni(J >> 8) : 0u;
        uint64_t coll = 0;      // a valid key equal to ~0 (2^32-slot tiles only)
        bool hit = false;
        // the draws stay in registers (x[4 e + q] = draw 256 e + 4 lane + q)
        uint32_t x[4 * kFastRounds], rk[4 * kFastRounds];
#pragma unroll
        for (int e = 0; e < (int)kFastRounds; ++e) {
#pragma unroll
            for (int q = 0; q < 4; ++q) { x[4 * e + q] = kNone; rk[4 * e + q] = 0; }
            const uint32_t blk = lane + 64u * e;
            if ((uint32_t)e < nclean) {
                const U4 w = t.st.block_uniform_key(blk);     // the tile's key is wave-uniform
                const uint32_t v[4] = {w.x & t.mask, w.y & t.mask, w.z & t.mask, w.w & t.mask};
#pragma unroll
                for (int q = 0; q < 4; ++q) rk[4 * e + q] = atomicAdd(&cnt[v[q] >> shift], 1u);
#pragma unroll
                for (int q = 0; q < 4; ++q) x[4 * e + q] = v[q];
            } else if ((uint32_t)e < nit && 4 * blk < J) {
                // only the lanes whose block holds draws below J compute it
                const U4 w = t.st.block_uniform_key(blk);
                uint32_t v[4] = {w.x & t.mask, w.y & t.mask, w.z & t.mask, w.w & t.mask};
                if (nclean_tile) {
                    // a full tile with keys below 2^31: only draws past J drop out
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool ok = 4 * blk + q < J;
                        rk[4 * e + q] = atomicAdd(&cnt[v[q] >> shift], ok ? 1u : 0u);
                        v[q] = ok ? v[q] : kNone;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // a draw past J or rejected adds 0 and is kept as ~0
                        const bool ok = (4 * blk + q < J) & (t.full | (v[q] < S32));
                        hit |= ok & (v[q] == kNone);
                        rk[4 * e + q] = atomicAdd(&cnt[v[q] >> shift], ok ? 1u : 0u);
                        v[q] = ok ? v[q] : kNone;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) x[4 * e + q] = v[q];
            }
        }
        coll = __ballot(hit);
        __syncthreads();
        if (coll) {
            cw[0] = make_uint4(0, 0, 0, 0);
            cw[1] = make_uint4(0, 0, 0, 0);
            return false;
        }
        uint32_t V;             // valid draws
        uint32_t R;             // keys in the fullest bucket
        {
            const uint4 c0 = cw[0], c1 = cw[1];
            uint32_t w[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
            uint32_t sum = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) sum += w[i];
            uint32_t mx = w[0];
#pragma unroll
            for (int i = 1; i < 8; ++i) mx = mx > w[i] ? mx : w[i];
            R = wave_max32(mx);
            const uint32_t incl = wave_incl_scan32(sum);
            uint32_t run = incl - sum;
#pragma unroll
            for (int i = 0; i < 8; ++i) { const uint32_t c = w[i]; w[i] = run; run += c; }
            cw[0] = make_uint4(w[0], w[1], w[2], w[3]);
            cw[1] = make_uint4(w[4], w[5], w[6], w[7]);
            V = __builtin_amdgcn_readlane(incl, 63);
        }
        __syncthreads();
        {
#pragma unroll
            for (int e = 0; e < (int)kFastRounds; ++e) {
                if ((uint32_t)e < nclean) {
                    // every entry of a clean round is a valid key
                    uint32_t old[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) old[q] = cnt[x[4 * e + q] >> shift] + rk[4 * e + q];
#pragma unroll
                    for (int q = 0; q < 4; ++q) s[old[q]] = x[4 * e + q];
                } else if ((uint32_t)e < nit) {
                    uint32_t old[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t xv = x[4 * e + q];
                        const bool ok = xv != kNone;
                        old[q] = cnt[ok ? xv >> shift : 0u] + rk[4 * e + q];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t xv = x[4 * e + q];
                        // a ~0 entry lands in the padding after the V keys, which is
                        // rewritten below or lies past the sorted span (kKeyWords >= V + 4)
                        const uint32_t pos = xv != kNone ? old[q] : V + (lane & 3);
                        s[pos] = xv;
                    }
                }
            }
        }
        // the wave's LDS operations complete in order, so the bucket starts
        // read above are read before they are cleared here
        cw[0] = make_uint4(0, 0, 0, 0);
        cw[1] = make_uint4(0, 0, 0, 0);
        __syncthreads();
        if (R > kMaxRounds) return false;
        uint32_t ndup;
        {
            // keys per lane from V: 4, 8, 12, 16, 18 or 20; [V, 64 W) is padded with ~0
            const int mode = V <= 256 ? 0 : V <= 512 ? 1 : V <= 768 ? 2 : V <= 1024 ? 3 : V <= 1152 ? 4 : 5;
            constexpr uint32_t kSpan[6] = {256, 512, 768, 1024, 1152, 1280};
            const uint32_t span = kSpan[mode];
            for (uint32_t p = V + lane; p < span; p += 64) s[p] = kNone;
            __syncthreads();
            if (mode == 0) ndup = oddeven<4>(s, V, R);
            else if (mode == 1) ndup = oddeven<8>(s, V, R);
            else if (mode == 2) ndup = oddeven<12>(s, V, R);
            else if (mode == 3) ndup = oddeven<16>(s, V, R);
            else if (mode == 4) ndup = oddeven<18>(s, V, R);
            else ndup = oddeven<20>(s, V, R);
            __syncthreads();
        }
        const uint32_t D = V - ndup;
        if (D == ke) {
            if (ndup) {
                uint32_t kept = 0;
                for (uint32_t b0 = 0; b0 < V; b0 += 64) {
                    const uint32_t p = b0 + lane;
                    uint32_t xv = 0;
                    bool keep = false;
                    if (p < V) {
                        xv = s[p];
                        keep = p == 0 || s[p - 1] != xv;
                    }
                    const uint64_t bal = __ballot(keep);
                    __syncthreads();
                    if (keep) s[kept + __popcll(bal & lanemask_lt(lane))] = xv;
                    kept += __popcll(bal);
                    __syncthreads();
                }
            }
            return true;
        }
        J += ke - D;
    }
}

// Decoding constants of a tile copied into vector registers: they are read
// by every key of the emission loop, and scalar registers are scarce there.
__device__ __forceinline__ uint32_t vreg(uint32_t x)
{
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

struct DecV {
    uint32_t dv, r0, c0, b, sh, msk;
    double rcp;
};

__device__ __forceinline__ DecV dec_vregs(const Decoder &d)
{
    DecV v;
    v.dv = vreg(d.dv); v.r0 = vreg(d.r0); v.c0 = vreg(d.c0); v.b = vreg(d.b);
    v.sh = vreg(d.sh); v.msk = vreg(d.dv - 1);
    const uint64_t rb = (uint64_t)__double_as_longlong(d.rcp);
    v.rcp = __longlong_as_double((long long)(((uint64_t)vreg((uint32_t)(rb >> 32)) << 32) | vreg((uint32_t)rb)));
    return v;
}

// Directed (TYPE 0) or rectangle (TYPE 1) slot with a 32-bit dividend:
// quotient by shift or by the binary64 reciprocal estimate, corrected once
// without branches.
template <int TYPE, bool POW2, bool ALIGNED = false>
__device__ __forceinline__ uint2 dec_narrow(const DecV &d, uint32_t x)
{
    if (ALIGNED) {
        // rectangle, width 2^sh, tile starting at a row start, first column a
        // multiple of the width: row offset by shift, column by mask and OR
        return make_uint2(d.r0 + (x >> d.sh), d.b | (x & d.msk));
    }
    const uint32_t y = d.c0 + x;
    uint32_t q, r;
    if (POW2) {
        q = y >> d.sh;
        r = y & d.msk;
    } else {
        q = (uint32_t)((double)y * d.rcp);
        int32_t rr = (int32_t)(y - q * d.dv);
        const bool neg = rr < 0;
        q -= neg ? 1u : 0u;
        rr += neg ? (int32_t)d.dv : 0;
        const bool big = (uint32_t)rr >= d.dv;
        q += big ? 1u : 0u;
        rr -= big ? (int32_t)d.dv : 0;
        r = (uint32_t)rr;
    }
    const uint32_t u = d.r0 + q;
    return TYPE == 0 ? make_uint2(u, r + (r >= u ? 1u : 0u)) : make_uint2(u, d.b + r);
}

// Sorted keys s[0..n) out as edges o0 .. o0 + n - 1, four keys per lane per
// round (lane-strided, so each store instruction covers 512 contiguous bytes).
template <int TYPE, bool POW2, bool ALIGNED = false>
__device__ __forceinline__ void emit_narrow(const TileCtx &t, const uint32_t *s, uint32_t n)
{
    const DecV d = dec_vregs(t.dec);
    uint2 *out = reinterpret_cast<uint2 *>(t.edges) + t.o0;
    const uint32_t lane = lane_here();
    const uint32_t nfull = n & ~255u;
    // one 64-bit lane pointer advanced per round; the four stores of a round
    // sit at fixed byte offsets from it (0, 512, 1024, 1536)
    uint2 *ol = out + lane;
    for (uint32_t b = 0; b < nfull; b += 256, ol += 256) {
        uint32_t x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = s[b + lane + 64 * i];
#pragma unroll
        for (int i = 0; i < 4; ++i) ol[64 * i] = dec_narrow<TYPE, POW2, ALIGNED>(d, x[i]);
    }
    if (nfull < n) {
        uint32_t x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t p = nfull + lane + 64 * i;
            x[i] = p < n ? s[p] : 0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t p = nfull + lane + 64 * i;
            if (p < n) out[p] = dec_narrow<TYPE, POW2, ALIGNED>(d, x[i]);
        }
    }
}

__device__ __forceinline__ void emit_tile(const TileCtx &t, const uint32_t *s, uint32_t n)
{
    const Decoder &d = t.dec;
    if (d.type == 2 || d.wide) emit_sorted(t, s, n);
    else if (d.type == 0) {
        if (d.pow2) emit_narrow<0, true>(t, s, n); else emit_narrow<0, false>(t, s, n);
    } else {
        if (d.pow2 && d.c0 == 0 && (d.b & (d.dv - 1)) == 0) emit_narrow<1, true, true>(t, s, n);
        else if (d.pow2) emit_narrow<1, true>(t, s, n);
        else emit_narrow<1, false>(t, s, n);
    }
}

// 4 waves per SIMD (up to 128 VGPRs, no spills); the LDS of a wave (keys of
// up to 1280 draws and 512 bucket counters, 7.2 KB) would allow 5
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void tile_kernel(Job job)
{
    __shared__ __attribute__((aligned(16))) uint32_t s_key[kKeyWords];
    __shared__ __attribute__((aligned(16))) uint32_t s_cnt[kBucketWords];   // bucket counters, then starts
    if (ld_uni(job.status + 1)) return;
    const uint64_t T = ld_uni(job.status + 2);
    {
        uint4 *cw = reinterpret_cast<uint4 *>(s_cnt) + 2 * threadIdx.x;
        cw[0] = make_uint4(0, 0, 0, 0);
        cw[1] = make_uint4(0, 0, 0, 0);
        __syncthreads();
    }
    const uint32_t lim = job.fast_cap < kFastDraws ? job.fast_cap : kFastDraws;
    TileWalk w;
    TileCtx &tc = w.tc;
    Decoder &d = tc.dec;
    tc.edges = job.edges;
    TileGrab grab(T);
    uint64_t t, t1;
    while (grab.next(job, t, t1)) {
        uint64_t g = chunk_of_tile(job, t);
        // tile offsets are read two tiles ahead: they come from HBM (the output
        // stream evicts them from the caches), so a tile never waits for its own
        uint64_t o_next = ld_uni(job.tile_off + t);
        uint64_t o_pre = ld_uni(job.tile_off + t + 1);
        for (;;) {
            // chunk constants, then the decoder at the wave's first tile of the chunk
            w.enter(job, g);
            const uint64_t tend = w.gend < t1 ? w.gend : t1;
            const uint32_t s = w.s;
            const uint64_t full_S = 1ull << s;
            uint64_t lstart = (t - w.gstart) << s;
            if (d.type != 2) {
                const uint64_t q = lstart / d.dv;
                d.c0 = uni((uint32_t)(lstart - q * d.dv));
                d.r0 = uni(w.row0 + (uint32_t)q);
            }
            const uint32_t qs32 = (uint32_t)w.qs;
            for (; t < tend; ++t) {
                const uint64_t o0 = o_next;
                o_next = o_pre;
                if (t + 2 <= T) o_pre = ld_uni(job.tile_off + t + 2);
                const uint64_t k = o_next - o0;
                if (k != 0) {
                    // slots of the tile: 2^s except for the chunk's last tile
                    if (t + 1 < w.gend) {
                        tc.S = full_S;
                        tc.bits = s;
                        tc.mask = s >= 32 ? 0xFFFFFFFFu : (1u << s) - 1;
                        tc.full = 1;
                    } else {
                        tc.S = uni64(w.N - lstart);
                        tc.bits = uni(tc.S <= 1 ? 0 : 64 - __clzll(tc.S - 1));
                        tc.mask = uni(tc.bits >= 32 ? 0xFFFFFFFFu : ((1u << tc.bits) - 1));
                        tc.full = uni(tc.S == (1ull << tc.bits));
                    }
                    tc.st.b = uni((uint32_t)(t - w.gstart));
                    d.lbase = lstart;
                    d.wide = s == 32 ? uni((uint64_t)d.c0 + tc.S > (1ull << 32)) : 0u;
                    tc.o0 = o0;
                    const bool comp = 2 * k > tc.S;
                    const uint64_t ke = comp ? tc.S - k : k;
                    if (ke == 0) {
                        emit_complement(tc, s_key, 0, 0, tc.S, 0);
                    } else if (ke <= lim && fast_set(tc, s_key, s_cnt, (uint32_t)ke, lim)) {
                        if (!comp) emit_tile(tc, s_key, (uint32_t)ke);
                        else emit_complement(tc, s_key, (uint32_t)ke, 0, tc.S, 0);
                    } else if (threadIdx.x == 0) {
                        const uint64_t q = atomicAdd((unsigned long long *)(job.status + 4), 1ull);
                        job.queue[q] = t;
                    }
                    __syncthreads();
                }
                // next tile of the chunk: 2^s = qs dv + rs slots further
                lstart += full_S;
                if (d.type != 2) {
                    uint32_t c0 = d.c0 + w.rs, r0 = d.r0 + qs32;
                    if (c0 >= d.dv) { c0 -= d.dv; ++r0; }
                    d.c0 = c0;
                    d.r0 = r0;
                }
            }
            if (t >= t1) break;
            // next chunk that has tiles
            ++g;
            while (ld_uni(job.tstart + g + 1) <= t) ++g;
        }
    }
}

// Tiles the fast kernel queued: one wave per queued tile, general base case.
template <int CAP>
__global__ __launch_bounds__(64) void queue_kernel(Job job)
{
    __shared__ __attribute__((aligned(16))) uint32_t s_bkt[CAP + 8];
    __shared__ __attribute__((aligned(16))) uint32_t s_hist[CAP + 8];
    if (ld_uni(job.status + 1)) return;
    const uint64_t nq = ld_uni(job.status + 4);
    const uint32_t cap = job.leaf_cap < CAP ? job.leaf_cap : CAP;
    for (uint64_t i = blockIdx.x; i < nq; i += gridDim.x) {
        const uint64_t t = ld_uni(job.queue + i);
        const uint64_t o0 = ld_uni(job.tile_off + t);
        const uint64_t k = ld_uni(job.tile_off + t + 1) - o0;
        TileWalk w;
        w.locate(job, t);
        w.tile(t);
        TileCtx &tc = w.tc;
        tc.o0 = o0;
        tc.edges = job.edges;
        leaf_sample<CAP>(tc, s_bkt, s_hist, k, cap);
        __syncthreads();
    }
}

}  // namespace kg
