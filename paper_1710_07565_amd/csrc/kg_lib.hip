// kg_lib.hip -- host side of the C ABI declared in include/kg.h: argument
// checks, the per-instance plan (chunk count, tile exponent), workspace
// layout, and the launch sequence count -> scan -> plan -> sample.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/kg.h"
#include "kg_tile.hpp"
#include "kg_skip.hpp"
#include "kg_rgg.hpp"
#include "kg_rgg3.hpp"
#include "kg_hash.hpp"

namespace kg {
__device__ double g_lnf_tab[kLnfTab + 1];
}

// Static scratch of kg_gnm_static (KG_STATIC_SCRATCH_BYTES, kg.h): the
// workspace of callers that cannot allocate.  Each device the library runs on holds one copy of it for the
// life of the process.  Host code must use the device address looked up
// with hipGetSymbolAddress (g_scratch_ptr), never the array's name.
static __device__ __align__(256) uint8_t scratch[KG_STATIC_SCRATCH_BYTES];

using namespace kg;

namespace {

typedef unsigned __int128 u128;

constexpr uint32_t kSpecVersion = 1;
constexpr uint64_t kMaxChunks = 1ull << 36;   // chunks of one call (a batch: all instances)

// Non-semantic knobs.
int64_t g_leaf_cap = 0;        // 0: default
int64_t g_sample_waves = 0;    // per CU
int64_t g_plan_waves = 0;      // per CU
int64_t g_count_lanes = 0;     // lanes per chunk in the count kernel (0: chosen per call)
int64_t g_skip_row = 0;        // positions kept per tile by kg_gnp_skip (0: kSkipKeys)

// The HIP error behind the most recent KG_EDEVICE from a launch on this
// thread (kg_last_hip_error).
thread_local int t_last_hip_error = 0;

// Whether the launches since the last check were accepted; a failure's
// HIP error code is kept for kg_last_hip_error.
bool launched_ok()
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return true;
    t_last_hip_error = (int)e;
    return false;
}
int64_t g_time_kernels = 0;

// Event pairs recorded around kernel launches while timing is on.
std::mutex g_time_mu;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events[5];

// True while `s` is being recorded into a graph: such a call must only
// enqueue kernels (no allocation, synchronisation or host-memory copies).
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Set while kg_gnm_static runs on this thread: its calls record no timer
// events (creating and keeping them allocates).
thread_local bool t_no_timers = false;

struct KernelTimer {
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(int kid, hipStream_t st) : id(kid), s(st)
    {
        if (!g_time_kernels || t_no_timers || capturing(s)) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, s);
    }
    ~KernelTimer()
    {
        if (!a) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_time_mu);
        g_events[id].emplace_back(a, b);
    }
};


std::mutex g_init_mu;
bool g_init_done[64];
int g_num_cu[64];
void *g_scratch_ptr[64];        // device address of `scratch` on each device (set up by ensure_init)

// Workspaces registered with kg_set_workspace, per device: calls given no
// workspace of their own use it instead of a stream-ordered allocation.
std::mutex g_ws_mu;
void *g_reg_ws[64];
uint64_t g_reg_bytes[64];

// A call that passes no workspace gets the one registered for the current
// device, if any (d_ws and bytes are left alone otherwise).
void registered_workspace(void *&d_ws, uint64_t &bytes)
{
    if (d_ws) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (g_reg_ws[dev]) {
        d_ws = g_reg_ws[dev];
        bytes = g_reg_bytes[dev];
    }
}

// While `s` is being recorded into a graph a call may enqueue kernels only:
// the library must already be set up on the device (the first call launches
// a table kernel and synchronises) and the workspace must not come from the
// stream-ordered allocator.
kg_status capture_check(hipStream_t s, const void *d_ws)
{
    if (!capturing(s)) return KG_OK;
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return KG_EDEVICE;
    bool ready;
    {
        std::lock_guard<std::mutex> lk(g_init_mu);
        ready = g_init_done[d];
    }
    return ready && d_ws ? KG_OK : KG_EINVAL;
}

int g_sample_blocks_per_cu[64];
int g_plan_blocks_per_cu[64];
int g_skip_blocks_per_cu[64];
int g_gen_blocks_per_cu[64];
int g_emit_blocks_per_cu[64];
int g_queue_blocks_per_cu[64];
constexpr int kCountVariants = 4;   // count kernel with 1, 2, 4, 8 lanes per chunk
int g_count_blocks_per_cu[64][kCountVariants];

kg_status ensure_init(int *dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KG_EDEVICE;
    *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_init_done[dev]) return KG_OK;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return KG_EDEVICE;
    g_num_cu[dev] = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    // resident one-wave workgroups per compute unit: a grid of exactly that
    // many avoids a partial second round of workgroups
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tile_kernel, 64, 0) != hipSuccess || nb < 1) nb = 8;
    g_sample_blocks_per_cu[dev] = nb;
    nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, plan_kernel<1>, 64, 0) != hipSuccess || nb < 1) nb = 8;
    g_plan_blocks_per_cu[dev] = nb;
    nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, skip_write_kernel, 64, 0) != hipSuccess || nb < 1) nb = 8;
    g_skip_blocks_per_cu[dev] = nb;
    nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, skip_gen_kernel, 64, 0) != hipSuccess || nb < 1) nb = 8;
    g_gen_blocks_per_cu[dev] = nb;
    nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, skip_emit_kernel, 64, 0) != hipSuccess || nb < 1) nb = 8;
    g_emit_blocks_per_cu[dev] = nb;
    nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, queue_kernel<kCapMax>, 64, 0) != hipSuccess || nb < 1) nb = 1;
    g_queue_blocks_per_cu[dev] = nb;
    {
        const void *fk[kCountVariants] = {(const void *)count_kernel<1, 1>, (const void *)count_kernel<1, 2>,
                                          (const void *)count_kernel<1, 4>, (const void *)count_kernel<2, 4>};
        const int threads[kCountVariants] = {64, 128, 256, 512};
        for (int v = 0; v < kCountVariants; ++v) {
            nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk[v], threads[v], 0) != hipSuccess || nb < 0) nb = 0;
            g_count_blocks_per_cu[dev][v] = nb;
        }
    }
    // this device's copy of the static scratch (its own address per device)
    void *sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) return KG_EDEVICE;
    g_scratch_ptr[dev] = sp;
    hipLaunchKernelGGL(lnf_init_kernel, dim3(1), dim3(64), 0, 0);
    if (!launched_ok()) return KG_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return KG_EDEVICE;
    g_init_done[dev] = true;
    return KG_OK;
}

// Validation and the per-instance plan.
kg_status plan_instance(const kg_instance &in, Inst &out, uint64_t &tile_bound)
{
    if (in.model > 1 || in.directed > 1) return KG_EINVAL;
    if (in.n < 1 || in.chunks < 1 || (uint64_t)in.chunks > in.n) return KG_EINVAL;
    if (in.flags > in.chunks) return KG_EINVAL;     // 0, or 1 + the section of a view
    if (in.n > (1ull << 32)) return KG_ERANGE;
    const u128 N128 = in.directed ? (u128)in.n * (in.n - 1) : (u128)in.n * (in.n - 1) / 2;
    if (in.directed ? (in.chunks > (1u << 31)) : (in.chunks > (1u << 15))) return KG_ERANGE;
    const uint64_t N = (uint64_t)N128;     // < 2^64 since n <= 2^32
    if (in.model == KG_GNM && in.m > N) return KG_EINVAL;
    if (in.model == KG_GNP && !(in.p >= 0.0 && in.p <= 1.0)) return KG_EINVAL;
    if (N128 >= ((u128)1 << 53)) {
        // universes of 2^53 slots and more: counts stay below 2^53 (the
        // variates convert them exactly); slot counts round to nearest
        if (in.model == KG_GNM && in.m >= (1ull << 53)) return KG_ERANGE;
        if (in.model == KG_GNP && (double)N * in.p >= 0x1p52) return KG_ERANGE;
    }
    // tile exponent: smallest s in [9, 32] with 2^s m >= lambda N (G(n,m)) or
    // 2^s p >= lambda (G(n,p))
    uint32_t s = 32;
    for (uint32_t t = 9; t <= 32; ++t) {
        const bool ok = in.model == KG_GNM ? (((u128)in.m << t) >= (u128)kLambda * N)
                                            : (ldexp(in.p, (int)t) >= (double)kLambda);
        if (ok) { s = t; break; }
    }
    {
        // every chunk has fewer than 2^31 tiles (the tile index is a 32-bit
        // stream word): bounded through the largest section
        const uint64_t rows = (in.n + in.chunks - 1) / in.chunks;
        const u128 Nc = in.directed ? (u128)rows * (in.n - 1) : (u128)rows * rows;
        if ((Nc >> s) >= ((u128)1 << 31)) return KG_ERANGE;
    }
    memset(&out, 0, sizeof(out));
    out.n = in.n;
    out.m = in.model == KG_GNM ? in.m : 0;
    out.p = in.model == KG_GNP ? in.p : 0.0;
    out.seed = in.seed;
    out.model = in.model;
    out.directed = in.directed;
    out.P = in.chunks;
    out.s = s;
    out.view = in.flags;
    if (in.flags == 0) {
        out.nchunks = in.directed ? (uint64_t)in.chunks : (uint64_t)in.chunks * (in.chunks + 1) / 2;
        // sum over chunks of ceil(N_c / 2^s) <= N / 2^s + chunks
        tile_bound = (N >> s) + out.nchunks;
    } else {
        // the chunks incident to section r hold at most h_r n slots
        const uint64_t r = in.flags - 1;
        const uint64_t h = section_bound(out, r + 1) - section_bound(out, r);
        out.nchunks = in.directed ? 1 : (uint64_t)in.chunks;
        tile_bound = (uint64_t)(((u128)h * in.n) >> s) + out.nchunks;
    }
    return KG_OK;
}

struct Layout {
    uint64_t status, insts, off, tstart, ustart, bsum, tile_off, queue, total;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

Layout layout_for(uint32_t ninst, uint64_t G, uint64_t Tb)
{
    Layout L;
    uint64_t o = 0;
    L.status = o; o = align256(o + 8 * sizeof(uint64_t));
    L.insts = o; o = align256(o + (ninst > 1 ? ninst * sizeof(Inst) : 0));
    L.off = o; o = align256(o + (G + 1) * 8);
    L.tstart = o; o = align256(o + (G + 1) * 8);
    L.ustart = o; o = align256(o + (G + 1) * 8);
    L.bsum = o; o = align256(o + 3 * ((G + 63) / 64) * 8);
    L.tile_off = o; o = align256(o + (Tb + 1) * 8);
    L.queue = o; o = align256(o + (Tb + 1) * 8);
    L.total = o;
    return L;
}

// The planned instances of a call.  A single instance lives inside the
// object, so a one-instance call makes no heap allocation.
struct InstList {
    Inst first;
    std::vector<Inst> many;     // a batch (more than one instance)
    uint32_t count = 0;
    void resize(uint32_t c)
    {
        count = c;
        if (c > 1) many.resize(c);
    }
    size_t size() const { return count; }
    Inst *data() { return count > 1 ? many.data() : &first; }
    const Inst *data() const { return count > 1 ? many.data() : &first; }
    Inst &operator[](size_t i) { return data()[i]; }
    const Inst &operator[](size_t i) const { return data()[i]; }
};

struct Prepared {
    InstList insts;
    uint64_t G = 0, Tb = 0;
    Layout L;
};

kg_status prepare(const kg_instance *in, uint32_t count, Prepared &P)
{
    if (!in || count == 0) return KG_EINVAL;
    P.insts.resize(count);
    P.G = 0;
    P.Tb = 0;
    for (uint32_t i = 0; i < count; ++i) {
        uint64_t tb = 0;
        const kg_status st = plan_instance(in[i], P.insts[i], tb);
        if (st) return st;
        P.insts[i].chunk_base = P.G;
        P.G += P.insts[i].nchunks;
        P.Tb += tb;
        // one-dimensional grids of one wave per 64 chunks
        if (P.G > kMaxChunks) return KG_ERANGE;
    }
    P.L = layout_for(count, P.G, P.Tb);
    return KG_OK;
}

int64_t opt_or(int64_t v, int64_t dflt) { return v > 0 ? v : dflt; }

struct Workspace {
    char *base = nullptr;
    bool owned = false;
};

kg_status acquire(Workspace &ws, void *d_ws, uint64_t ws_bytes, uint64_t need, hipStream_t s)
{
    if (d_ws) {
        if (ws_bytes < need) return KG_ENOSPC;
        ws.base = (char *)d_ws;
        ws.owned = false;
        return KG_OK;
    }
    void *p = nullptr;
    if (hipMallocAsync(&p, need, s) != hipSuccess) return KG_EDEVICE;
    ws.base = (char *)p;
    ws.owned = true;
    return KG_OK;
}

void release(Workspace &ws, hipStream_t s)
{
    if (ws.owned && ws.base) (void)hipFreeAsync(ws.base, s);
    ws.base = nullptr;
}

Job make_job(const Prepared &P, const Workspace &ws, uint32_t *edges, uint64_t capacity)
{
    Job job;
    memset(&job, 0, sizeof(job));
    job.ninst = (uint32_t)P.insts.size();
    int64_t cap = opt_or(g_leaf_cap, kCapMax);
    if (cap > kCapMax) cap = kCapMax;
    if (cap < 128) cap = 128;
    job.leaf_cap = (uint32_t)cap;
    // a leaf capacity set by the caller also bounds the register base case
    // (tests force the general path with it); by default it takes all it can
    job.fast_cap = g_leaf_cap > 0 ? (uint32_t)std::min<int64_t>(cap, kFastDraws) : kFastDraws;
    // planner units: enough of them to give every resident lane one (one lane
    // expands a unit), at most kUnitTiles tiles each
    {
        const uint64_t lanes = 256ull * 16 * 64;
        uint32_t ulog = 1;
        while (ulog < 6 && (P.Tb >> (ulog + 1)) >= lanes) ++ulog;
        job.unit_log = ulog;
    }
    job.G = P.G;
    job.capacity = capacity;
    job.tile_cap = P.Tb;
    job.insts = job.ninst > 1 ? (const Inst *)(ws.base + P.L.insts) : nullptr;
    job.one = P.insts[0];
    job.off = (uint64_t *)(ws.base + P.L.off);
    job.tstart = (uint64_t *)(ws.base + P.L.tstart);
    job.ustart = (uint64_t *)(ws.base + P.L.ustart);
    job.bsum = (uint64_t *)(ws.base + P.L.bsum);
    job.tile_off = (uint64_t *)(ws.base + P.L.tile_off);
    job.status = (uint64_t *)(ws.base + P.L.status);
    job.queue = (uint64_t *)(ws.base + P.L.queue);
    job.edges = edges;
    return job;
}

// The count kernel's lanes per chunk: its time is the latency of each
// chunk's chain of variates, so a chunk gets as many lanes (8, 4, then 2) as
// keep every workgroup of the launch resident at once; a launch too large
// for that takes one lane per chunk (the least work per variate).  Launch
// shape only: the counts are the same for every choice.
void launch_count(const Job &job, uint64_t nb, int dev, hipStream_t s)
{
    int v = 0;
    if (g_count_lanes) {
        v = g_count_lanes == 8 ? 3 : g_count_lanes == 4 ? 2 : g_count_lanes == 2 ? 1 : 0;
    } else {
        const uint64_t cu = (uint64_t)g_num_cu[dev];
        for (int c = kCountVariants - 1; c >= 1; --c)
            if (nb <= cu * (uint64_t)g_count_blocks_per_cu[dev][c]) { v = c; break; }
    }
    if (v == 3) hipLaunchKernelGGL((count_kernel<2, 4>), dim3((uint32_t)nb), dim3(512), 0, s, job);
    else if (v == 2) hipLaunchKernelGGL((count_kernel<1, 4>), dim3((uint32_t)nb), dim3(256), 0, s, job);
    else if (v == 1) hipLaunchKernelGGL((count_kernel<1, 2>), dim3((uint32_t)nb), dim3(128), 0, s, job);
    else hipLaunchKernelGGL((count_kernel<1, 1>), dim3((uint32_t)nb), dim3(64), 0, s, job);
}

// count + scan (+ instance offsets).  `resident`: the descriptor table is
// already in the workspace (kg_batch_upload).
kg_status launch_counts(const Prepared &P, Job &job, int dev, hipStream_t s, bool resident)
{
    if (job.ninst > 1 && !resident) {
        if (hipMemcpyAsync((void *)job.insts, P.insts.data(), P.insts.size() * sizeof(Inst),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return KG_EDEVICE;
    }
    const uint64_t nb = (P.G + 63) / 64;
    {
        KernelTimer tm(KG_KERNEL_COUNT, s);
        launch_count(job, nb, dev, s);
    }
    {
        KernelTimer tm(KG_KERNEL_SCAN, s);
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, job);
        hipLaunchKernelGGL(fix_kernel, dim3((uint32_t)nb), dim3(64), 0, s, job);
    }
    if (job.inst_off)
        hipLaunchKernelGGL(inst_offsets_kernel, dim3((job.ninst + 1 + 255) / 256), dim3(256), 0, s, job);
    return launched_ok() ? KG_OK : KG_EDEVICE;
}

kg_status launch_generate(const Prepared &P, Job &job, int dev, hipStream_t s)
{
    const int64_t cu = g_num_cu[dev];
    // planner units: at most 2 per 2^unit_log tiles plus one per chunk; one lane each
    const uint64_t ub = 2 * (P.Tb >> job.unit_log) + P.G + 1;
    uint64_t pgrid = (uint64_t)(cu * opt_or(g_plan_waves, g_plan_blocks_per_cu[dev]));
    // few units (their bound fits the resident lanes 4 or 2 times over): a
    // group of lanes per unit shortens each unit's chain of variates
    const int terms = ub * 4 <= pgrid * 64 ? 4 : ub * 2 <= pgrid * 64 ? 2 : 1;
    if (pgrid > (ub * terms + 63) / 64) pgrid = (ub * terms + 63) / 64;
    {
        KernelTimer tm(KG_KERNEL_PLAN, s);
        if (terms == 4) hipLaunchKernelGGL(plan_kernel<4>, dim3((uint32_t)pgrid), dim3(64), 0, s, job);
        else if (terms == 2) hipLaunchKernelGGL(plan_kernel<2>, dim3((uint32_t)pgrid), dim3(64), 0, s, job);
        else hipLaunchKernelGGL(plan_kernel<1>, dim3((uint32_t)pgrid), dim3(64), 0, s, job);
    }
    uint64_t sgrid = (uint64_t)(cu * opt_or(g_sample_waves, g_sample_blocks_per_cu[dev]));
    if (sgrid > P.Tb + 1) sgrid = P.Tb + 1;
    // the queued tiles (more draws than the register base case holds, or a
    // bucket too full to sort): rare, the tiles expecting at most 1120
    // samples; a grid that fills the chip drains them in parallel (every
    // wave exits at once when the queue is empty)
    uint64_t qgrid = (uint64_t)(cu * g_queue_blocks_per_cu[dev]);
    if (qgrid > P.Tb + 1) qgrid = P.Tb + 1;
    {
        KernelTimer tm(KG_KERNEL_SAMPLE, s);
        hipLaunchKernelGGL(tile_kernel, dim3((uint32_t)sgrid), dim3(64), 0, s, job);
    }
    {
        KernelTimer tm(KG_KERNEL_QUEUE, s);
        hipLaunchKernelGGL(queue_kernel<kCapMax>, dim3((uint32_t)qgrid), dim3(64), 0, s, job);
    }
    return launched_ok() ? KG_OK : KG_EDEVICE;
}

kg_status run(const kg_instance *inst, uint32_t count, uint32_t *edges, uint64_t capacity,
              uint64_t *d_total, uint64_t *d_inst_off, void *d_ws, uint64_t ws_bytes, void *stream,
              bool counts_only, uint64_t *h_total, uint64_t *d_counts, bool resident = false)
{
    Prepared P;
    kg_status st = prepare(inst, count, P);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    registered_workspace(d_ws, ws_bytes);
    st = capture_check(s, d_ws);
    if (st) return st;
    // nothing may be read back, and a batch's descriptor table must already
    // be resident
    if (capturing(s) && (counts_only || (count > 1 && !resident))) return KG_EINVAL;
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    Workspace ws;
    st = acquire(ws, d_ws, ws_bytes, P.L.total, s);
    if (st) return st;
    Job job = make_job(P, ws, edges, capacity);
    job.out_total = d_total;
    job.inst_off = d_inst_off;
    if (d_counts) {
        // counts only: run the count kernel and copy the per-chunk counts out
        const uint64_t nb = (P.G + 63) / 64;
        launch_count(job, nb, dev, s);
        if (!launched_ok()) st = KG_EDEVICE;
        else if (hipMemcpyAsync(d_counts, job.off, P.G * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = KG_EDEVICE;
        release(ws, s);
        return st;
    }
    st = launch_counts(P, job, dev, s, resident);
    if (!st && counts_only) {
        uint64_t tot = 0;
        if (hipMemcpyAsync(&tot, job.status, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = KG_EDEVICE;
        else
            *h_total = tot;
    } else if (!st) {
        st = launch_generate(P, job, dev, s);
    }
    release(ws, s);
    return st;
}

kg_instance make_inst(uint64_t n, uint32_t model, int directed, uint64_t m, double p, uint64_t seed,
                      uint32_t chunks)
{
    kg_instance I;
    memset(&I, 0, sizeof(I));
    I.n = n;
    I.model = model;
    I.directed = directed ? 1u : 0u;
    I.m = m;
    I.p = p;
    I.seed = seed;
    I.chunks = chunks;
    return I;
}

// ---------------------------------------------------------------------------
// Random geometric graphs: level rule and workspace layout.
// ---------------------------------------------------------------------------
uint32_t rgg_level(uint64_t n, double r)
{
    uint32_t L = 0;
    while (L < kRggMaxLevel && ldexp(r, (int)L + 1) <= 1.0 && (1ull << (2 * (L + 1))) <= n) ++L;
    return L;
}

struct RggLayout {
    uint32_t L;
    uint64_t C, nw, nbc, nbw;
    uint64_t tree, coff, pcell, ecnt, bits, wsum, woff, sums, status, total;
};

RggLayout rgg_layout(uint64_t n, double r)
{
    RggLayout Y;
    Y.L = rgg_level(n, r);
    Y.C = 1ull << (2 * Y.L);
    Y.nw = (n + 63) / 64;
    Y.nbc = (Y.C + kScanTile - 1) / kScanTile;
    Y.nbw = Y.nw ? (Y.nw + kScanTile - 1) / kScanTile : 1;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) { const uint64_t at = o; o += (bytes + 255) & ~255ull; return at; };
    Y.tree = take(((1ull << (2 * (Y.L + 1))) - 1) / 3 * 8);
    Y.coff = take((Y.C + 1) * 8);
    Y.pcell = take(n * 4);
    Y.ecnt = take(n * 4);
    Y.bits = take(n * 8 * kRggBitWords);
    Y.wsum = take((Y.nw + 1) * 8);
    Y.woff = take((Y.nw + 1) * 8);
    Y.sums = take((std::max(Y.nbc, Y.nbw) + 1) * 8);
    Y.status = take(4 * 8);
    Y.total = o;
    return Y;
}

uint32_t rgg3_level(uint64_t n, double r)
{
    uint32_t L = 0;
    while (L < kRgg3MaxLevel && ldexp(r, (int)L + 1) <= 1.0 && (1ull << (3 * (L + 1))) <= n) ++L;
    return L;
}

struct Rgg3Layout {
    uint32_t L;
    uint64_t C, nw, nbc, nbw;
    uint64_t tree, coff, pcell, ecnt, bits, wsum, woff, sums, status, total;
};

Rgg3Layout rgg3_layout(uint64_t n, double r)
{
    Rgg3Layout Y;
    Y.L = rgg3_level(n, r);
    Y.C = 1ull << (3 * Y.L);
    Y.nw = (n + 63) / 64;
    Y.nbc = (Y.C + kScanTile - 1) / kScanTile;
    Y.nbw = Y.nw ? (Y.nw + kScanTile - 1) / kScanTile : 1;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) { const uint64_t at = o; o += (bytes + 255) & ~255ull; return at; };
    Y.tree = take(((1ull << (3 * (Y.L + 1))) - 1) / 7 * 8);
    Y.coff = take((Y.C + 1) * 8);
    Y.pcell = take(n * 4);
    Y.ecnt = take(n * 4);
    Y.bits = take(n * 8 * kRgg3BitWords);
    Y.wsum = take((Y.nw + 1) * 8);
    Y.woff = take((Y.nw + 1) * 8);
    Y.sums = take((std::max(Y.nbc, Y.nbw) + 1) * 8);
    Y.status = take(4 * 8);
    Y.total = o;
    return Y;
}

kg_status rgg3_check(uint64_t n, double r)
{
    if (!(r >= 0.0)) return KG_EINVAL;
    if (n > 0xFFFFFFFFull) return KG_ERANGE;
    const uint32_t L = rgg3_level(n, r);
    // points per cell times points: the per-point pass's work
    if ((double)n * (double)n > ldexp(1.0, 36 + 3 * (int)L)) return KG_ERANGE;
    return KG_OK;
}

kg_status rgg_check(uint64_t n, double r)
{
    if (!(r >= 0.0)) return KG_EINVAL;
    if (n > 0xFFFFFFFFull) return KG_ERANGE;
    const uint32_t L = rgg_level(n, r);
    // expected points per cell times points: the per-point pass's work
    if ((double)n * (double)n > ldexp(1.0, 36 + 2 * (int)L)) return KG_ERANGE;
    return KG_OK;
}

void rgg_scan(const uint64_t *a, uint64_t len, uint64_t *sums, uint64_t *out, hipStream_t s)
{
    const uint64_t nb = len ? (len + kScanTile - 1) / kScanTile : 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((uint32_t)nb), dim3(256), 0, s, a, len, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums, nb);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((uint32_t)nb), dim3(256), 0, s, a, len, (const uint64_t *)sums, out);
}

}  // namespace

extern "C" {

uint32_t kg_spec_version(void) { return kSpecVersion; }

const char *kg_strerror(kg_status st)
{
    switch (st) {
    case KG_OK: return "ok";
    case KG_EINVAL: return "invalid argument";
    case KG_ERANGE: return "argument outside the supported range";
    case KG_ENOSPC: return "output or workspace too small";
    case KG_EDEVICE: return "HIP runtime error";
    case KG_ESCRATCH: return "the instance needs more workspace than the static scratch holds (96 MiB)";
    default: return "unknown status";
    }
}

kg_status kg_workspace_bytes(const kg_instance *inst, uint32_t count, uint64_t *bytes)
{
    if (!bytes) return KG_EINVAL;
    Prepared P;
    const kg_status st = prepare(inst, count, P);
    if (st) return st;
    *bytes = P.L.total;
    return KG_OK;
}

kg_status kg_gnm(uint64_t n, uint64_t m, int directed, uint64_t seed, uint32_t chunks, uint32_t *d_edges,
                 uint64_t capacity_edges, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    const kg_instance I = make_inst(n, KG_GNM, directed, m, 0.0, seed, chunks);
    if (!d_edges && m > 0) return KG_EINVAL;
    if (((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    Prepared P;
    kg_status st = prepare(&I, 1, P);
    if (st) return st;
    if (capacity_edges < m) return KG_ENOSPC;
    return run(&I, 1, d_edges, capacity_edges, nullptr, nullptr, d_workspace, workspace_bytes, stream, false,
               nullptr, nullptr);
}

kg_status kg_gnm_static(uint64_t n, uint64_t m, int directed, uint64_t seed, uint32_t chunks, uint32_t *d_edges,
                        uint64_t capacity_edges, void *stream)
{
    const kg_instance I = make_inst(n, KG_GNM, directed, m, 0.0, seed, chunks);
    if (!d_edges && m > 0) return KG_EINVAL;
    if (((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    Prepared P;
    kg_status st = prepare(&I, 1, P);
    if (st) return st;
    if (capacity_edges < m) return KG_ENOSPC;
    if (P.L.total > KG_STATIC_SCRATCH_BYTES) return KG_ESCRATCH;
    // the device's scratch address is looked up once, by the set-up of the
    // first call on the device (which, like every first call, synchronises)
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    void *sp;
    {
        std::lock_guard<std::mutex> lk(g_init_mu);
        sp = g_scratch_ptr[dev];
    }
    if (!sp) return KG_EDEVICE;
    t_no_timers = true;
    st = run(&I, 1, d_edges, capacity_edges, nullptr, nullptr, sp, KG_STATIC_SCRATCH_BYTES, stream, false,
             nullptr, nullptr);
    t_no_timers = false;
    return st;
}

kg_status kg_gnp(uint64_t n, double p, int directed, uint64_t seed, uint32_t chunks, uint32_t *d_edges,
                 uint64_t capacity_edges, uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes,
                 void *stream)
{
    const kg_instance I = make_inst(n, KG_GNP, directed, 0, p, seed, chunks);
    if (((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    if (!d_edges) capacity_edges = 0;
    return run(&I, 1, d_edges, capacity_edges, d_total, nullptr, d_workspace, workspace_bytes, stream, false,
               nullptr, nullptr);
}

kg_status kg_gnp_count(uint64_t n, double p, int directed, uint64_t seed, uint32_t chunks, uint64_t *h_total,
                       void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_total) return KG_EINVAL;
    const kg_instance I = make_inst(n, KG_GNP, directed, 0, p, seed, chunks);
    return run(&I, 1, nullptr, 0, nullptr, nullptr, d_workspace, workspace_bytes, stream, true, h_total,
               nullptr);
}

kg_status kg_chunk_counts(const kg_instance *inst, uint64_t *d_counts, void *d_workspace,
                          uint64_t workspace_bytes, void *stream)
{
    if (!inst || !d_counts) return KG_EINVAL;
    return run(inst, 1, nullptr, 0, nullptr, nullptr, d_workspace, workspace_bytes, stream, false, nullptr,
               d_counts);
}

kg_status kg_batch(const kg_instance *h_inst, uint32_t count, uint32_t *d_arena, uint64_t arena_edges,
                   uint64_t *d_inst_offsets, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_inst || count == 0 || !d_inst_offsets) return KG_EINVAL;
    if (((uintptr_t)d_arena & 7) != 0) return KG_EINVAL;
    if (!d_arena) arena_edges = 0;
    return run(h_inst, count, d_arena, arena_edges, nullptr, d_inst_offsets, d_workspace, workspace_bytes,
               stream, false, nullptr, nullptr);
}

kg_status kg_pe_view(const kg_instance *inst, uint32_t rank, uint32_t *d_edges, uint64_t capacity_edges,
                     uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!inst || inst->flags != 0 || rank >= inst->chunks) return KG_EINVAL;
    if (((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    kg_instance I = *inst;
    I.flags = rank + 1;
    if (!d_edges) capacity_edges = 0;
    return run(&I, 1, d_edges, capacity_edges, d_total, nullptr, d_workspace, workspace_bytes, stream, false,
               nullptr, nullptr);
}

// Workspace of kg_gnp_skip's position rows: the chunk layout, then one row
// of kSkipKeys 32-bit positions per tile (tile bound Tb).
uint64_t skip_rows_offset(const Prepared &P) { return align256(P.L.total); }
uint64_t skip_rows_bytes(const Prepared &P) { return skip_rows_offset(P) + P.Tb * (uint64_t)kSkipKeys * 4; }

kg_status kg_gnp_skip_workspace_bytes(uint64_t n, double p, int directed, uint32_t chunks, uint64_t *bytes)
{
    if (!bytes) return KG_EINVAL;
    const kg_instance I = make_inst(n, KG_GNP, directed, 0, p, 1, chunks);
    Prepared P;
    const kg_status st = prepare(&I, 1, P);
    if (st) return st;
    *bytes = skip_rows_bytes(P);
    return KG_OK;
}

kg_status kg_gnp_skip(uint64_t n, double p, int directed, uint64_t seed, uint32_t chunks, uint32_t *d_edges,
                      uint64_t capacity_edges, uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes,
                      void *stream)
{
    const kg_instance I = make_inst(n, KG_GNP, directed, 0, p, seed, chunks);
    if (((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    if (!d_edges) capacity_edges = 0;
    Prepared P;
    kg_status st = prepare(&I, 1, P);
    if (st) return st;
    const uint64_t nw = (P.Tb + 63) / 64;          // one wave per 64 tiles
    if (nw > 0x7FFFFFFFull || nw > P.Tb + 1) return KG_ERANGE;
    hipStream_t s = (hipStream_t)stream;
    registered_workspace(d_workspace, workspace_bytes);
    st = capture_check(s, d_workspace);
    if (st) return st;
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    // a call that writes edges keeps the count pass's positions when the
    // workspace holds a row per tile (or the library allocates it)
    const uint64_t rows_bytes = skip_rows_bytes(P);
    const bool rows = d_edges && (!d_workspace || workspace_bytes >= rows_bytes);
    Workspace ws;
    st = acquire(ws, d_workspace, workspace_bytes, rows ? rows_bytes : P.L.total, s);
    if (st) return st;
    // the chunk and tile layout from the main path's count and offset
    // kernels; their binomial total is not this sampler's, so no capacity
    // check and no total there
    Job job = make_job(P, ws, d_edges, ~0ull);
    st = launch_counts(P, job, dev, s, false);
    if (!st) {
        uint32_t *row0 = rows ? (uint32_t *)(ws.base + skip_rows_offset(P)) : nullptr;
        // positions kept per tile: a multiple of 4 (16-byte aligned rows)
        const uint32_t cap = (uint32_t)opt_or(g_skip_row, kSkipKeys) & ~3u;
        {
            KernelTimer tm(KG_KERNEL_PLAN, s);
            if (rows) {
                uint64_t ggrid = (uint64_t)g_num_cu[dev] * (uint64_t)g_gen_blocks_per_cu[dev];
                if (ggrid > P.Tb + 1) ggrid = P.Tb + 1;
                hipLaunchKernelGGL(skip_gen_kernel, dim3((uint32_t)ggrid), dim3(64), 0, s, job, row0, cap);
                hipLaunchKernelGGL(skip_sums_kernel, dim3((uint32_t)nw), dim3(64), 0, s, job);
            } else {
                hipLaunchKernelGGL(skip_count_kernel, dim3((uint32_t)nw), dim3(64), 0, s, job);
            }
        }
        Job jw = job;
        jw.capacity = capacity_edges;
        jw.out_total = d_total;
        hipLaunchKernelGGL(skip_scan_kernel, dim3(1), dim3(1024), 0, s, jw, nw);
        hipLaunchKernelGGL(skip_fix_kernel, dim3((uint32_t)((P.Tb + 1 + 63) / 64)), dim3(64), 0, s, jw);
        {
            KernelTimer tm(KG_KERNEL_SAMPLE, s);
            if (rows) {
                uint64_t egrid = (uint64_t)g_num_cu[dev] * (uint64_t)g_emit_blocks_per_cu[dev];
                if (egrid > P.Tb + 1) egrid = P.Tb + 1;
                hipLaunchKernelGGL(skip_emit_kernel, dim3((uint32_t)egrid), dim3(64), 0, s, jw,
                                   (const uint32_t *)row0, cap);
            } else {
                uint64_t wgrid = (uint64_t)g_num_cu[dev] * (uint64_t)g_skip_blocks_per_cu[dev];
                if (wgrid > P.Tb + 1) wgrid = P.Tb + 1;
                hipLaunchKernelGGL(skip_write_kernel, dim3((uint32_t)wgrid), dim3(64), 0, s, jw);
            }
        }
        if (!launched_ok()) st = KG_EDEVICE;
    }
    release(ws, s);
    return st;
}

kg_status kg_rgg2d_workspace_bytes(uint64_t n, double r, uint64_t *bytes)
{
    if (!bytes) return KG_EINVAL;
    const kg_status st = rgg_check(n, r);
    if (st) return st;
    *bytes = rgg_layout(n, r).total;
    return KG_OK;
}

kg_status kg_rgg2d(uint64_t n, double r, uint64_t seed, double *d_points, uint32_t *d_edges,
                   uint64_t capacity_edges, uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes,
                   void *stream)
{
    kg_status st = rgg_check(n, r);
    if (st) return st;
    if (n > 0 && !d_points) return KG_EINVAL;
    if (((uintptr_t)d_points & 15) != 0 || ((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    if (!d_edges) capacity_edges = 0;
    hipStream_t s = (hipStream_t)stream;
    registered_workspace(d_workspace, workspace_bytes);
    st = capture_check(s, d_workspace);
    if (st) return st;
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    const RggLayout Y = rgg_layout(n, r);
    Workspace ws;
    st = acquire(ws, d_workspace, workspace_bytes, Y.total, s);
    if (st) return st;
    RggJob J;
    memset(&J, 0, sizeof(J));
    J.n = n;
    J.seed = seed;
    J.capacity = capacity_edges;
    J.r2 = r * r;
    J.h = ldexp(1.0, -(int)Y.L);
    J.L = Y.L;
    J.G = 1u << Y.L;
    J.C = Y.C;
    J.tree = (uint64_t *)(ws.base + Y.tree);
    J.coff = (uint64_t *)(ws.base + Y.coff);
    J.pcell = (uint32_t *)(ws.base + Y.pcell);
    J.ecnt = (uint32_t *)(ws.base + Y.ecnt);
    J.bits = (uint64_t *)(ws.base + Y.bits);
    J.wsum = (uint64_t *)(ws.base + Y.wsum);
    J.woff = (uint64_t *)(ws.base + Y.woff);
    J.sums = (uint64_t *)(ws.base + Y.sums);
    J.status = (uint64_t *)(ws.base + Y.status);
    J.out_total = d_total;
    J.pts = (double2 *)d_points;
    J.edges = (uint2 *)d_edges;
    {
        KernelTimer tm(KG_KERNEL_COUNT, s);
        hipLaunchKernelGGL(rgg_root_kernel, dim3(1), dim3(64), 0, s, J);
        for (uint32_t l = 0; l < Y.L; ++l)
            hipLaunchKernelGGL(rgg_split_kernel, dim3((uint32_t)(((1ull << (2 * l)) + 63) / 64)), dim3(64), 0, s,
                               J, l);
    }
    {
        KernelTimer tm(KG_KERNEL_SCAN, s);
        rgg_scan(J.tree + ((Y.C - 1) / 3), Y.C, J.sums, J.coff, s);
    }
    {
        KernelTimer tm(KG_KERNEL_QUEUE, s);
        hipLaunchKernelGGL(rgg_points_kernel, dim3((uint32_t)((Y.C + 63) / 64)), dim3(64), 0, s, J);
    }
    const uint64_t nwg = Y.nw ? Y.nw : 1;
    {
        KernelTimer tm(KG_KERNEL_PLAN, s);
        hipLaunchKernelGGL(rgg_edges_kernel<false>, dim3((uint32_t)nwg), dim3(64), 0, s, J);
    }
    {
        KernelTimer tm(KG_KERNEL_SCAN, s);
        rgg_scan(J.wsum, Y.nw, J.sums, J.woff, s);
        hipLaunchKernelGGL(rgg_total_kernel, dim3(1), dim3(64), 0, s, J, Y.nw);
    }
    {
        KernelTimer tm(KG_KERNEL_SAMPLE, s);
        hipLaunchKernelGGL(rgg_edges_kernel<true>, dim3((uint32_t)nwg), dim3(64), 0, s, J);
    }
    if (!launched_ok()) st = KG_EDEVICE;
    release(ws, s);
    return st;
}

kg_status kg_rgg3d_workspace_bytes(uint64_t n, double r, uint64_t *bytes)
{
    if (!bytes) return KG_EINVAL;
    const kg_status st = rgg3_check(n, r);
    if (st) return st;
    *bytes = rgg3_layout(n, r).total;
    return KG_OK;
}

kg_status kg_rgg3d(uint64_t n, double r, uint64_t seed, double *d_points, uint32_t *d_edges,
                   uint64_t capacity_edges, uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes,
                   void *stream)
{
    kg_status st = rgg3_check(n, r);
    if (st) return st;
    if (n > 0 && !d_points) return KG_EINVAL;
    if (((uintptr_t)d_points & 7) != 0 || ((uintptr_t)d_edges & 7) != 0) return KG_EINVAL;
    if (!d_edges) capacity_edges = 0;
    hipStream_t s = (hipStream_t)stream;
    registered_workspace(d_workspace, workspace_bytes);
    st = capture_check(s, d_workspace);
    if (st) return st;
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    const Rgg3Layout Y = rgg3_layout(n, r);
    Workspace ws;
    st = acquire(ws, d_workspace, workspace_bytes, Y.total, s);
    if (st) return st;
    Rgg3Job J;
    memset(&J, 0, sizeof(J));
    J.n = n;
    J.seed = seed;
    J.capacity = capacity_edges;
    J.r2 = r * r;
    J.h = ldexp(1.0, -(int)Y.L);
    J.L = Y.L;
    J.G = 1u << Y.L;
    J.C = Y.C;
    J.tree = (uint64_t *)(ws.base + Y.tree);
    J.coff = (uint64_t *)(ws.base + Y.coff);
    J.pcell = (uint32_t *)(ws.base + Y.pcell);
    J.ecnt = (uint32_t *)(ws.base + Y.ecnt);
    J.bits = (uint64_t *)(ws.base + Y.bits);
    J.wsum = (uint64_t *)(ws.base + Y.wsum);
    J.woff = (uint64_t *)(ws.base + Y.woff);
    J.sums = (uint64_t *)(ws.base + Y.sums);
    J.status = (uint64_t *)(ws.base + Y.status);
    J.out_total = d_total;
    J.pts = d_points;
    J.edges = (uint2 *)d_edges;
    {
        KernelTimer tm(KG_KERNEL_COUNT, s);
        hipLaunchKernelGGL(rgg3_root_kernel, dim3(1), dim3(64), 0, s, J);
        for (uint32_t l = 0; l < Y.L; ++l)
            hipLaunchKernelGGL(rgg3_split_kernel, dim3((uint32_t)(((1ull << (3 * l)) + 63) / 64)), dim3(64), 0, s,
                               J, l);
    }
    {
        KernelTimer tm(KG_KERNEL_SCAN, s);
        rgg_scan(J.tree + ((Y.C - 1) / 7), Y.C, J.sums, J.coff, s);
    }
    {
        KernelTimer tm(KG_KERNEL_QUEUE, s);
        hipLaunchKernelGGL(rgg3_points_kernel, dim3((uint32_t)((Y.C + 63) / 64)), dim3(64), 0, s, J);
    }
    const uint64_t nwg = Y.nw ? Y.nw : 1;
    {
        KernelTimer tm(KG_KERNEL_PLAN, s);
        hipLaunchKernelGGL(rgg3_edges_kernel<false>, dim3((uint32_t)nwg), dim3(64), 0, s, J);
    }
    {
        KernelTimer tm(KG_KERNEL_SCAN, s);
        rgg_scan(J.wsum, Y.nw, J.sums, J.woff, s);
        hipLaunchKernelGGL(rgg3_total_kernel, dim3(1), dim3(64), 0, s, J, Y.nw);
    }
    {
        KernelTimer tm(KG_KERNEL_SAMPLE, s);
        hipLaunchKernelGGL(rgg3_edges_kernel<true>, dim3((uint32_t)nwg), dim3(64), 0, s, J);
    }
    if (!launched_ok()) st = KG_EDEVICE;
    release(ws, s);
    return st;
}

kg_status kg_batch_upload(const kg_instance *h_inst, uint32_t count, void *d_workspace,
                          uint64_t workspace_bytes, void *stream)
{
    if (!h_inst || count == 0 || !d_workspace) return KG_EINVAL;
    Prepared P;
    kg_status st = prepare(h_inst, count, P);
    if (st) return st;
    if (workspace_bytes < P.L.total) return KG_ENOSPC;
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return KG_EINVAL;
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    if (count == 1) return KG_OK;          // one instance travels in the kernel arguments
    if (hipMemcpyAsync((char *)d_workspace + P.L.insts, P.insts.data(), P.insts.size() * sizeof(Inst),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return KG_EDEVICE;
    return KG_OK;
}

kg_status kg_batch_launch(const kg_instance *h_inst, uint32_t count, uint32_t *d_arena, uint64_t arena_edges,
                          uint64_t *d_inst_offsets, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_inst || count == 0 || !d_inst_offsets || !d_workspace) return KG_EINVAL;
    if (((uintptr_t)d_arena & 7) != 0) return KG_EINVAL;
    if (!d_arena) arena_edges = 0;
    return run(h_inst, count, d_arena, arena_edges, nullptr, d_inst_offsets, d_workspace, workspace_bytes,
               stream, false, nullptr, nullptr, true);
}

kg_status kg_edge_hash(const uint32_t *d_edges, uint64_t n_edges, uint64_t *d_hash, void *stream)
{
    if (!d_hash || (n_edges > 0 && !d_edges)) return KG_EINVAL;
    if (((uintptr_t)d_edges & 7) != 0 || ((uintptr_t)d_hash & 7) != 0) return KG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KG_EDEVICE;
    hipLaunchKernelGGL(hash_clear_kernel, dim3(1), dim3(64), 0, s, d_hash);
    uint64_t grid = (n_edges / 2 + 255) / 256;
    if (grid < 1) grid = 1;
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(hash_kernel, dim3((uint32_t)grid), dim3(256), 0, s, d_edges, n_edges, d_hash);
    return launched_ok() ? KG_OK : KG_EDEVICE;
}

kg_status kg_set_workspace(void *d_workspace, uint64_t workspace_bytes)
{
    if (!d_workspace && workspace_bytes != 0) return KG_EINVAL;
    if (d_workspace && (workspace_bytes == 0 || ((uintptr_t)d_workspace & 255) != 0)) return KG_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KG_EDEVICE;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_reg_ws[dev] = d_workspace;
    g_reg_bytes[dev] = workspace_bytes;
    return KG_OK;
}

uint64_t kg_instance_seed(uint64_t base, uint32_t i)
{
    const U4 w = philox(0, i, 0, TAG_INST, (uint32_t)base, (uint32_t)(base >> 32));
    return ((uint64_t)w.y << 32) | w.x;
}

kg_status kg_set_option(int option, int64_t value)
{
    if (value < 0) return KG_EINVAL;
    switch (option) {
    case KG_OPT_LEAF_CAP:
        if (value != 0 && (value < 128 || value > kCapMax)) return KG_ERANGE;
        g_leaf_cap = value;
        return KG_OK;
    case KG_OPT_SAMPLE_WAVES:
        if (value > 32) return KG_ERANGE;
        g_sample_waves = value;
        return KG_OK;
    case KG_OPT_PLAN_WAVES:
        if (value > 64) return KG_ERANGE;
        g_plan_waves = value;
        return KG_OK;
    case KG_OPT_TIME_KERNELS:
        if (value > 1) return KG_ERANGE;
        g_time_kernels = value;
        return KG_OK;
    case KG_OPT_COUNT_LANES:
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8) return KG_ERANGE;
        g_count_lanes = value;
        return KG_OK;
    case KG_OPT_SKIP_ROW:
        if (value != 0 && (value < 64 || value > kSkipKeys)) return KG_ERANGE;
        g_skip_row = value;
        return KG_OK;
    default:
        return KG_EINVAL;
    }
}

kg_status kg_kernel_time_read(int kernel, double *ms_total, uint64_t *launches)
{
    if (kernel < 0 || kernel > 4 || !ms_total || !launches) return KG_EINVAL;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_time_mu);
        ev.swap(g_events[kernel]);
    }
    double tot = 0.0;
    kg_status st = KG_OK;
    for (auto &e : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(e.second) != hipSuccess || hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess)
            st = KG_EDEVICE;
        tot += ms;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    *ms_total = tot;
    *launches = ev.size();
    return st;
}

kg_status kg_eval(int fn, const void *d_in, void *d_out, uint64_t n, void *stream)
{
    if (fn < KG_EVAL_PHILOX || fn > KG_EVAL_SQRT_DIV) return KG_EINVAL;
    if (n == 0) return KG_OK;
    if (!d_in || !d_out) return KG_EINVAL;
    kg_status st = capture_check((hipStream_t)stream, d_in);
    if (st) return st;
    int dev = 0;
    st = ensure_init(&dev);
    if (st) return st;
    const uint64_t nb = (n + 255) / 256;
    if (nb > 0x7FFFFFFFull) return KG_ERANGE;
    hipLaunchKernelGGL(eval_kernel, dim3((uint32_t)nb), dim3(256), 0, (hipStream_t)stream, fn, d_in, d_out, n);
    return launched_ok() ? KG_OK : KG_EDEVICE;
}

int kg_last_hip_error(void)
{
    return t_last_hip_error;
}

int64_t kg_get_option(int option)
{
    switch (option) {
    case KG_OPT_LEAF_CAP: return opt_or(g_leaf_cap, kCapMax);
    case KG_OPT_SAMPLE_WAVES: return g_sample_waves;     // 0: as many as fit on a compute unit
    case KG_OPT_PLAN_WAVES: return g_plan_waves;
    case KG_OPT_TIME_KERNELS: return g_time_kernels;
    case KG_OPT_COUNT_LANES: return g_count_lanes;
    case KG_OPT_SKIP_ROW: return opt_or(g_skip_row, kSkipKeys);
    default: return -1;
    }
}

}  // extern "C"
