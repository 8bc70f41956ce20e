/*
 * kg.h -- C ABI of the MI355X generator for Erdos-Renyi graphs G(n,m) and
 * G(n,p), directed or undirected, following the communication-free method of
 * Funke et al., "Communication-free Massively Distributed Graph Generation"
 * (arXiv 1710.07565, Sec. 4).
 *
 * Conventions shared by every entry point:
 *   - Inputs are the problem as the paper states it: n vertices; m edges
 *     (G(n,m), Sec. 2.1.1: a graph uniform among those with m edges) or a
 *     probability p (G(n,p), Sec. 2.1.1: every slot independently); directed
 *     or undirected; a seed; and the paper's P: the number of row chunks
 *     (directed, Sec. 4.1) or of sections per matrix dimension (undirected,
 *     Sec. 4.2, giving P(P+1)/2 chunks).
 *   - Output edges are uint32 pairs [u0, v0, u1, v1, ...] in device memory.
 *     Chunks come in canonical order (directed: rows ascending; undirected:
 *     the upper-triangular chunk matrix row-major), each chunk ascending by
 *     its local slot index.  Directed output is therefore sorted by (u, v);
 *     undirected output always has u < v.
 *   - The bytes are a pure function of (n, m or p, directed, seed, P): they do
 *     not depend on the stream, the launch shape, tuning knobs or the device.
 *   - Limits: n <= 2^32 (so the slot count N = n(n-1) directed or
 *     n(n-1)/2 undirected is below 2^64), 1 <= P <= n, P <= 2^31 directed,
 *     P <= 2^15 undirected; fewer than 2^31 tiles in every chunk; at most
 *     2^36 chunks in one call (a batch counts the chunks of all its
 *     instances).  For N >= 2^53 (Sec. 1: universes beyond binary64's exact
 *     integers) the edge count must stay below 2^53 (G(n,m): m < 2^53;
 *     G(n,p): N p < 2^52); slot counts are then converted to binary64 by
 *     rounding to nearest, identically in every implementation of the
 *     bits.
 *   - Every device pointer is owned by the caller; the library never frees
 *     caller memory.  `stream` is a hipStream_t (NULL = default stream).
 *     Calls are asynchronous on `stream` unless stated otherwise; argument
 *     errors are returned synchronously and then nothing is enqueued.
 *   - Scratch: each generation call takes a device workspace of at least the
 *     size kg_workspace_bytes() reports.  Passing d_workspace = NULL makes the
 *     library use the workspace registered for the current device with
 *     kg_set_workspace, or, if none is, take it from the stream-ordered
 *     allocator (hipMallocAsync / hipFreeAsync on `stream`).  Two calls in
 *     flight at once must not share a workspace.
 *   - Output capacity: G(n,m) checks it on the host (KG_ENOSPC, nothing
 *     enqueued).  Where the edge total is only known on the device (G(n,p),
 *     views, the skip sampler, geometric graphs) an undersized output is
 *     detected there: nothing is written to the edge buffer, the call still
 *     returns KG_OK (it returns before the kernels run) and the required
 *     total is stored at d_total, which the caller reads in stream order.
 *   - Statuses are returned, never thrown across the ABI.
 */
#ifndef KG_H
#define KG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kg_status;
enum {
    KG_OK = 0,
    KG_EINVAL = -1,   /* bad argument: n, m, p, P, model, NULL pointer */
    KG_ERANGE = -2,   /* outside the limits above */
    KG_ENOSPC = -3,   /* output or workspace too small; nothing enqueued */
    KG_EDEVICE = -4,  /* a HIP call failed */
    KG_ESCRATCH = -5  /* kg_gnm_static: the instance needs more workspace than
                       * KG_STATIC_SCRATCH_BYTES; nothing enqueued */
};
enum { KG_GNM = 0, KG_GNP = 1 };

/* One graph instance.  `chunks` is the paper's P. */
typedef struct {
    uint64_t n;
    uint32_t model;      /* KG_GNM or KG_GNP */
    uint32_t directed;   /* 0 or 1 */
    uint64_t m;          /* G(n,m) edge count */
    double p;            /* G(n,p) edge probability in [0, 1] */
    uint64_t seed;
    uint32_t chunks;
    uint32_t flags;      /* 0: the whole graph; r + 1 (r < chunks): only the edges
                          * incident to section r, the per-PE view of Sec. 4.1
                          * (directed: row chunk r) and Sec. 4.2 (undirected: the
                          * chunks (i, r), i < r, and (r, j), j >= r, of the
                          * chunk matrix), in canonical chunk order and with the
                          * bytes those chunks have in the whole graph */
} kg_instance;

/* Spec version of the output bits (changes whenever any output could). */
uint32_t kg_spec_version(void);
const char *kg_strerror(kg_status st);

/* Device workspace needed by a call on `count` instances.  Host only. */
kg_status kg_workspace_bytes(const kg_instance *inst, uint32_t count, uint64_t *bytes);

/* Register a caller-owned device buffer (256-byte aligned, `workspace_bytes`
 * long) as the workspace of the current device: every later call on that
 * device that passes d_workspace = NULL uses it instead of the
 * stream-ordered allocator, and fails with KG_ENOSPC if it is smaller than
 * the call needs.  kg_set_workspace(NULL, 0) removes the registration.  The
 * library never frees the buffer; the caller keeps it alive while it is
 * registered.  Calls that use the registered buffer must not overlap in
 * time (issue them on one stream).  KG_EINVAL for NULL with a nonzero size,
 * a zero size or a misaligned pointer; KG_EDEVICE if no device is current. */
kg_status kg_set_workspace(void *d_workspace, uint64_t workspace_bytes);

/* G(n,m) (Sec. 4.1 directed, Sec. 4.2 undirected): writes exactly m edges to
 * d_edges (room for capacity_edges pairs).  KG_ENOSPC if capacity < m. */
kg_status kg_gnm(uint64_t n, uint64_t m, int directed, uint64_t seed, uint32_t chunks,
                 uint32_t *d_edges, uint64_t capacity_edges,
                 void *d_workspace, uint64_t workspace_bytes, void *stream);

/* kg_gnm for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call the allocator, harnesses
 * that forbid it).  Same arguments, checks and output bytes as kg_gnm, but the
 * workspace is a static scratch area of KG_STATIC_SCRATCH_BYTES (96 MiB) in
 * the library, one per device, held from the library's first call on that
 * device until the process ends; the call itself allocates nothing (no
 * hipMalloc, no stream-ordered allocation, no heap).  An instance whose
 * workspace (kg_workspace_bytes) exceeds that size returns KG_ESCRATCH before
 * anything is enqueued; the headline size (undirected n = 2^26, m = 2^31,
 * P = 256) needs 65.3 MiB.  Every call on one device shares that device's
 * area, so calls on one device that overlap in time race: issue them on one
 * stream.  The library's first call on a device (any entry point) sets the
 * device up and synchronises; under stream capture that first call must
 * already have happened. */
#define KG_STATIC_SCRATCH_BYTES (96ull << 20)
kg_status kg_gnm_static(uint64_t n, uint64_t m, int directed, uint64_t seed, uint32_t chunks,
                        uint32_t *d_edges, uint64_t capacity_edges, void *stream);

/* G(n,p) (Sec. 4.3: binomial chunk counts keyed by chunk id, then the G(n,m)
 * sampler per chunk).  The edge total is stored at the device address
 * d_total (may be NULL).  If it exceeds capacity_edges nothing is written to
 * d_edges; the caller detects this by reading *d_total after the stream
 * completes. */
kg_status kg_gnp(uint64_t n, double p, int directed, uint64_t seed, uint32_t chunks,
                 uint32_t *d_edges, uint64_t capacity_edges, uint64_t *d_total,
                 void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Edge total of a G(n,p) instance: runs only the count and offset steps and
 * synchronises `stream`; *h_total is host memory. */
kg_status kg_gnp_count(uint64_t n, double p, int directed, uint64_t seed, uint32_t chunks,
                       uint64_t *h_total, void *d_workspace, uint64_t workspace_bytes,
                       void *stream);

/* Per-chunk edge counts of one instance (canonical order) into d_counts
 * (device, one uint64 per chunk).  Asynchronous. */
kg_status kg_chunk_counts(const kg_instance *inst, uint64_t *d_counts,
                          void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Many instances in one pass over one arena.  Instance i is written at
 * edge index d_inst_offsets[i] (device, count+1 entries, the last one the
 * total), and its bytes equal those of kg_gnm / kg_gnp with the same
 * arguments.  If the total exceeds arena_edges nothing is written to the
 * arena (read d_inst_offsets[count] to see the need). */
kg_status kg_batch(const kg_instance *h_inst, uint32_t count, uint32_t *d_arena,
                   uint64_t arena_edges, uint64_t *d_inst_offsets,
                   void *d_workspace, uint64_t workspace_bytes, void *stream);

/* G(n,p) by geometric skips, a second sampler for the same law with its own
 * bits (Sec. 2.1.1, 4.3): each 2^s-slot tile of each chunk runs its Bernoulli
 * trials by waiting times, floor(log U / log(1 - p)) failures before the next
 * success (for p > 1/2: the waiting times of the failures), one 64-bit draw
 * of Philox counter (chunk ordinal, draw/2, tile, 7) per gap; a count pass,
 * a scan of the tile counts and a write pass.  Output order and arguments as
 * kg_gnp: the total goes to d_total (device, may be NULL); if it exceeds
 * capacity_edges nothing is written.  The workspace needs at least
 * kg_workspace_bytes of the G(n,p) instance; with at least
 * kg_gnp_skip_workspace_bytes (or none passed: the library allocates that
 * much) a call that writes edges keeps each tile's event positions from the
 * count pass in the workspace and the write pass only decodes them (the
 * same bytes, each gap's logarithm computed once). */
kg_status kg_gnp_skip(uint64_t n, double p, int directed, uint64_t seed, uint32_t chunks,
                      uint32_t *d_edges, uint64_t capacity_edges, uint64_t *d_total,
                      void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Workspace bytes with which kg_gnp_skip keeps the event positions (about 5.6
 * KB per tile of up to 1408 events: the chunk layout plus one row of 32-bit
 * tile-local positions per tile).  Host only. */
kg_status kg_gnp_skip_workspace_bytes(uint64_t n, double p, int directed, uint32_t chunks, uint64_t *bytes);

/* The per-PE view of one instance (inst->flags must be 0): the edges
 * incident to section `rank` (< chunks), i.e. what processing element `rank`
 * of the paper's distributed run generates without communication (Sec. 4.1,
 * Sec. 4.2 with the chunk row and column of the section; off-diagonal chunks
 * appear in the views of both their sections).  Byte-identical to the same
 * chunks of the whole graph.  The edge total, random for G(n,m) as for
 * G(n,p), is stored at d_total (device, may be NULL); if it exceeds
 * capacity_edges nothing is written.  Views are also accepted by kg_batch
 * (flags = rank + 1), e.g. all P views of a graph in one pass. */
kg_status kg_pe_view(const kg_instance *inst, uint32_t rank, uint32_t *d_edges, uint64_t capacity_edges,
                     uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Two-dimensional random geometric graph (Sec. 2.1.2 model, Sec. 5
 * generator): n points uniform in [0,1)^2 and an edge between every two
 * points at distance below r.  The square is cut into 4^L cells of side
 * 2^-L, L the largest level <= 14 with 2^L r <= 1 and 4^L <= n (cells of
 * side >= max(r, n^-1/2), Sec. 5); the points per cell come from a
 * quadrant recursion of three Bin(k, 1/2) variates per node, keyed by the
 * node (Philox counter (Morton index, j, 3 level + slot, 8), Sec. 5.1); the
 * points of a cell from counter (cell, j, 0, 9); the edges from a count
 * pass, a scan and a write pass over each point's cell and its eight
 * neighbours (Sec. 5.3).  The output does not depend on any launch setting.
 *   d_points  device, n x (double x, double y), 16-byte aligned, written in
 *             vertex order: cells in Morton order (x bit low), then the
 *             cell's points.  May be NULL only if n == 0.
 *   d_edges   device, capacity_edges x (uint32 u, uint32 v), u < v, in
 *             ascending (u, v); (x_u - x_v)^2 + (y_u - y_v)^2 < r^2 in
 *             binary64 with every operation rounded.  Nothing is written
 *             if the total exceeds capacity_edges.
 *   d_total   device uint64, may be NULL: the edge total.
 * n < 2^32, r >= 0 (KG_EINVAL for NaN or negative r); KG_ERANGE if
 * n^2 / 4^L > 2^36 (points per cell too many for the per-point pass: r > 1/2
 * with large n).  Asynchronous on `stream`; the workspace (or, if d_workspace
 * is NULL, a stream-ordered allocation) holds kg_rgg2d_workspace_bytes. */
kg_status kg_rgg2d_workspace_bytes(uint64_t n, double r, uint64_t *bytes);
kg_status kg_rgg2d(uint64_t n, double r, uint64_t seed, double *d_points, uint32_t *d_edges,
                   uint64_t capacity_edges, uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes,
                   void *stream);

/* Three-dimensional random geometric graph (Sec. 2.1.2 model with d = 3,
 * Sec. 5 generator): n points uniform in [0,1)^3 and an edge between every
 * two points at distance below r.  The cube is cut into 8^L cells of side
 * 2^-L, L the largest level <= 10 with 2^L r <= 1 and 8^L <= n; the points
 * per cell come from an octant recursion of seven Bin(k, 1/2) variates per
 * node (the 2^d - 1 binomials of Sec. 5.1; Philox counter (Morton index, j,
 * 7 level + slot, 10): slot 0 the lower z half, 1 and 2 the lower y halves
 * of the lower and upper z half, 3..6 the lower x halves of the four (y, z)
 * quarters); point j of a cell takes the 64-bit draws 3j, 3j + 1, 3j + 2 of
 * counter (cell, ., 0, 11) for x, y, z; the edges come from a count pass,
 * a scan and a write pass over each point's cell and its 26 neighbours
 * (Sec. 5.3).  The output does not depend on any launch setting.
 *   d_points  device, n x (double x, double y, double z), 8-byte aligned,
 *             in vertex order: cells in Morton order (x bit lowest, then y,
 *             then z), then the cell's points.  May be NULL only if n == 0.
 *   d_edges   device, capacity_edges x (uint32 u, uint32 v), u < v, in
 *             ascending (u, v); ((x_u - x_v)^2 + (y_u - y_v)^2) +
 *             (z_u - z_v)^2 < r^2 in binary64 with every operation rounded.
 *             Nothing is written if the total exceeds capacity_edges.
 *   d_total   device uint64, may be NULL: the edge total.
 * n < 2^32, r >= 0 (KG_EINVAL for NaN or negative r); KG_ERANGE if
 * n^2 / 8^L > 2^36.  Asynchronous on `stream`; the workspace (or, if
 * d_workspace is NULL, a stream-ordered allocation) holds
 * kg_rgg3d_workspace_bytes. */
kg_status kg_rgg3d_workspace_bytes(uint64_t n, double r, uint64_t *bytes);
kg_status kg_rgg3d(uint64_t n, double r, uint64_t seed, double *d_points, uint32_t *d_edges,
                   uint64_t capacity_edges, uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes,
                   void *stream);

/* kg_batch in two parts, so that the generating part can be recorded into a
 * HIP graph (stream capture) and replayed.  kg_batch_upload writes the
 * descriptor table of the list into d_workspace (required, at least
 * kg_workspace_bytes) and synchronises `stream`; it must not be called while
 * `stream` is capturing.  kg_batch_launch then does what kg_batch does with
 * the same arguments and output, but reads the descriptor table from the
 * workspace and enqueues kernels only: no allocation, no host copy, no
 * synchronisation.  It must be given the same list (h_inst is read on the
 * host for the launch sizes) and a workspace that the upload filled and that
 * nothing else has used since.  While `stream` is capturing, the library must
 * already have been used once on the device (any call), and only these calls
 * are accepted, each with a caller workspace (passed, or registered with
 * kg_set_workspace): kg_batch_launch, kg_gnm, kg_gnp, kg_pe_view,
 * kg_chunk_counts, kg_gnp_skip, kg_rgg2d, kg_rgg3d and kg_eval; the others return
 * KG_EINVAL before enqueuing anything.  A replayed graph rewrites the same
 * bytes; replays that overlap in time must not share the arena or the
 * workspace. */
kg_status kg_batch_upload(const kg_instance *h_inst, uint32_t count, void *d_workspace,
                          uint64_t workspace_bytes, void *stream);
kg_status kg_batch_launch(const kg_instance *h_inst, uint32_t count, uint32_t *d_arena,
                          uint64_t arena_edges, uint64_t *d_inst_offsets,
                          void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Order-independent 64-bit checksum of an edge list, for a consumer (the
 * serving client) that checks what it received without copying it to the
 * host: *d_hash = sum over i < n_edges of mix(i * 0x9E3779B97F4A7C15 +
 * (u_i << 32 | v_i)) mod 2^64, mix being the SplitMix64 finaliser.  d_edges
 * is device memory, 8-byte aligned (any edge of a list the library wrote),
 * d_hash one device uint64 (8-byte aligned).  Asynchronous on `stream`; kernels only, so it may be recorded
 * into a graph. */
kg_status kg_edge_hash(const uint32_t *d_edges, uint64_t n_edges, uint64_t *d_hash, void *stream);

/* Per-instance seed of a batch drawn from a base seed: the Philox4x32-10
 * image of counter (0, i, 0, 6) under key `base`, words (w1:w0). Host only. */
uint64_t kg_instance_seed(uint64_t base, uint32_t i);

/* Non-semantic launch knobs (never change output bits).  A value of 0
 * restores the default (for the wave counts: as many workgroups as fit on a
 * compute unit at once).  Process-wide; set them before issuing calls. */
enum {
    KG_OPT_LEAF_CAP = 1,        /* samples a wave sorts in LDS per pass (128..1024) */
    KG_OPT_SAMPLE_WAVES = 2,    /* resident sampler waves per compute unit (1..32) */
    KG_OPT_PLAN_WAVES = 3,      /* resident tile-planner waves per compute unit (1..64) */
    KG_OPT_TIME_KERNELS = 4,    /* 1: bracket every kernel launch with hipEvents (not under capture) */
    KG_OPT_COUNT_LANES = 5,     /* lanes per chunk in the count kernel (1, 2, 4 or 8; 0: the most for
                                   which every workgroup of the launch is resident at once) */
    KG_OPT_SKIP_ROW = 6         /* kg_gnp_skip: positions kept per tile (64..1408; tiles with more
                                   events are generated again in the write pass) */
};
kg_status kg_set_option(int option, int64_t value);
int64_t kg_get_option(int option);

/* The hipError_t code behind the most recent KG_EDEVICE that a rejected
 * kernel launch caused on the calling thread (0 if none yet); for error
 * messages.  Host only. */
int kg_last_hip_error(void);

/* Kernel timing for measurement.  While KG_OPT_TIME_KERNELS is 1 every launch
 * of kernel `kernel` (KG_KERNEL_*) is bracketed by two hipEvents recorded on
 * the launch stream.  kg_kernel_time_read waits for the recorded events,
 * returns the summed milliseconds and the number of launches, and forgets
 * them.  Host only; synchronises with the recorded events. */
enum {
    KG_KERNEL_COUNT = 0,   /* per-chunk counts (kg_rgg2d: the quadrant recursion) */
    KG_KERNEL_SCAN = 1,    /* offsets (the scan of the wave sums and the fix-up; kg_rgg2d: both scans) */
    KG_KERNEL_PLAN = 2,    /* tile plan (kg_gnp_skip: count pass; kg_rgg2d: edge count pass) */
    KG_KERNEL_SAMPLE = 3,  /* common-case tile sampler (kg_gnp_skip, kg_rgg2d: write pass) */
    KG_KERNEL_QUEUE = 4    /* general base case for the tiles the sampler queued (kg_rgg2d: points) */
};
kg_status kg_kernel_time_read(int kernel, double *ms_total, uint64_t *launches);

/* Element-wise evaluation of the device building blocks, for checking them
 * against an independent implementation.  d_in / d_out are device arrays of
 * n records; the call is asynchronous on `stream`.
 *   KG_EVAL_PHILOX    in: 6 x uint32 (c0 c1 c2 c3 k0 k1)   out: 4 x uint32
 *   KG_EVAL_LOG       in: double x                          out: double log x
 *   KG_EVAL_LOG1P     in: double x                          out: double log(1+x)
 *   KG_EVAL_LNF_DIFF  in: 2 x uint64 (x, y)                 out: double ln y! - ln x!
 *   KG_EVAL_HYP       in: 6 x uint64 (N, K, k, seed, a | b << 32, tag)  out: uint64
 *   KG_EVAL_BIN       in: 6 x uint64 (N, p bits, 0, seed, a | b << 32, tag) out: uint64
 *   KG_EVAL_SQRT_DIV  in: 2 x double (a, b)                 out: 2 x double (sqrt a, a / b)
 * The variates follow Sec. 2.2 / 4.3 exactly as the generator uses them. */
enum {
    KG_EVAL_PHILOX = 1, KG_EVAL_LOG = 2, KG_EVAL_LOG1P = 3, KG_EVAL_LNF_DIFF = 4,
    KG_EVAL_HYP = 5, KG_EVAL_BIN = 6, KG_EVAL_SQRT_DIV = 7
};
kg_status kg_eval(int fn, const void *d_in, void *d_out, uint64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KG_H */
