/*
 * glt.h -- exact 2-, 3- and 4-node graphlet (network motif) counts on an AMD MI355X.
 *
 * C ABI of libglt.  The library counts, for a simple undirected graph, the number of
 * induced embeddings of every graphlet H1..H17 of the paper's Table 1 (global counts,
 * Section 3 "Problem Formulation", global graphlet counting problem), and optionally the
 * number of those embeddings that contain each edge (per-edge or "micro" counts,
 * Section 4.3 and Section 4.5 "Unrestricted counts").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graph input is a symmetric CSR: row_ptr has n+1 offsets, col holds 2m neighbour ids,
 * both directions of every edge, neighbours in any order within a row.  Self-loops,
 * duplicate entries, asymmetric entries and out-of-range ids are rejected with an error;
 * the library never reads outside [row_ptr[0], row_ptr[n]) of col.
 *
 * Edge numbering for per-edge output: edge k is the k-th CSR entry (i, col[j]) with
 * i < col[j], scanning rows i = 0..n-1 and, within a row, entries in storage order.
 *
 * Per-edge output layout: 13 slots x m, slot-major (slot s of edge k at s*m + k),
 * uint64, slots in graphlet order
 *   0 H3 triangle        1 H4 2-star          2 H5 3-node-1-edge     3 H7 4-clique
 *   4 H8 chordal-cycle   5 H9 tailed-triangle 6 H10 4-cycle          7 H11 3-star
 *   8 H12 4-path         9 H13 4-node-1-tri  10 H14 4-node-2-edge   11 H15 4-node-2-star
 *  12 H16 4-node-1-edge
 * (H1 is the edge itself; H2, H6 and H17 contain no edge.)
 *
 * Global output: 17 unsigned 128-bit counts X1..X17 (index i-1), exact for any n < 2^31.
 *
 * Ownership: every buffer passed in belongs to the caller and is never freed or retained
 * past the call.  Library state lives only in the handles created here and is released
 * by the matching destroy call.  Errors are returned as negative glt_status values; the
 * message is available from glt_last_error() until the next call on the same handle.
 * On error, outputs are unspecified.  No C++ exception crosses this interface.
 *
 * Streams: "stream" is a hipStream_t (passed as void*).  A call's device work is ordered
 * after the work already queued on that stream.  NULL selects the handle's own stream,
 * which is then made to wait for the work already queued on the device's legacy default
 * (NULL) stream, so inputs written there (e.g. by PyTorch's default stream) are complete
 * before they are read.  Every call in this header returns only after its results are
 * complete and visible to the host (global counts) and on the device (per-edge counts).
 */
#ifndef GLT_H
#define GLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { uint64_t lo, hi; } glt_u128;

typedef struct {
    int64_t n;                 /* vertices, isolated ones included; 0 <= n < 2^31        */
    int64_t m;                 /* undirected edges; row_ptr[n] - row_ptr[0] == 2*m        */
    const void* row_ptr;       /* int32[n+1] or int64[n+1] (see offsets_are_64bit)        */
    const int32_t* col;        /* int32[2m] neighbour ids                                 */
    int32_t offsets_are_64bit; /* 0: row_ptr is int32, 1: int64                           */
    int32_t on_device;         /* 1: row_ptr/col/out_per_edge are device pointers (hipMalloc
                                  or a torch CUDA tensor on the handle's device); 0: host  */
} glt_csr;

typedef enum {
    GLT_OK = 0,
    GLT_E_INVALID_ARG = -1,    /* null pointer, bad size, offsets not monotone, id out of range */
    GLT_E_NOT_SIMPLE = -2,     /* self-loop or duplicate entry                                  */
    GLT_E_NOT_SYMMETRIC = -3,  /* an entry (i,j) without its (j,i)                              */
    GLT_E_OOM = -4,            /* device workspace would exceed the handle's HBM budget         */
    GLT_E_DEVICE = -5,         /* a HIP runtime error                                           */
    GLT_E_UNSUPPORTED = -6,    /* n >= 2^31 or 2m >= 2^31                                       */
    GLT_E_INTERNAL = -7,       /* an internal consistency check failed (a library bug)          */
    GLT_E_BUSY = -8            /* the server's request queue is full                            */
} glt_status;

enum {
    GLT_GLOBAL = 1,            /* compute X1..X17 (always done; the flag is accepted for clarity) */
    GLT_PER_EDGE = 2           /* also write the 13 per-edge counts                               */
};

typedef struct glt_ctx glt_ctx;

/* Create a handle bound to HIP device `device`.  hbm_budget_bytes caps the device
 * workspace the handle may hold (0 = no cap beyond the device's free memory). */
glt_status glt_create(int device, size_t hbm_budget_bytes, glt_ctx** out);

/* Release the handle and all device memory it holds.  NULL is ignored. */
void glt_destroy(glt_ctx* ctx);

/* Message of the last error on this handle ("" if none).  Valid until the next call. */
const char* glt_last_error(const glt_ctx* ctx);

/* Library version string. */
const char* glt_version(void);

/*
 * Count graphlets of one graph (Problem 1 of Section 3 for the global counts, the
 * edge-centric decomposition of Sections 4.3-4.6 for the per-edge counts).
 *   g             graph (see conventions); validated before any count is computed
 *   flags         GLT_GLOBAL | optional GLT_PER_EDGE
 *   out_global    host array of 17 glt_u128 (X1..X17); required
 *   out_per_edge  NULL, or uint64[13*m] (device memory if g->on_device, else host);
 *                 required when GLT_PER_EDGE is set
 *   stream        hipStream_t or NULL
 * Errors: GLT_E_INVALID_ARG, GLT_E_NOT_SIMPLE, GLT_E_NOT_SYMMETRIC, GLT_E_OOM,
 *         GLT_E_DEVICE, GLT_E_UNSUPPORTED, GLT_E_INTERNAL.
 */
glt_status glt_count(glt_ctx* ctx, const glt_csr* g, uint32_t flags,
                     glt_u128 out_global[17], uint64_t* out_per_edge, void* stream);

/*
 * glt_count for callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same counts
 * as glt_count, computed with no hipMalloc, hipFree or other allocating call.  Its
 * workspace is one fixed array of GLT_NOALLOC_MAX_BYTES per device, reserved when the
 * library is loaded on that device and held until the process ends; every call on a device
 * shares it (calls that overlap on one device, on any handles or streams, race and must be
 * serialised by the caller), and each call clears what it needs before use.  Arguments as
 * glt_count, except that g->on_device must be 1 (inputs and out_per_edge in device memory).
 * The triangle passes re-scan out-lists instead of storing triangle records.
 * Errors as glt_count; GLT_E_INVALID_ARG for host inputs; GLT_E_UNSUPPORTED when the graph's
 * workspace exceeds GLT_NOALLOC_MAX_BYTES (roughly 400,000 edges), with the size needed in
 * the message.
 */
#define GLT_NOALLOC_MAX_BYTES ((size_t)128 << 20)
glt_status glt_count_noalloc(glt_ctx* ctx, const glt_csr* g, uint32_t flags,
                             glt_u128 out_global[17], uint64_t* out_per_edge, void* stream);

/*
 * A batch of independent graphs packed back to back.  Graph g owns packed vertices
 * [vtx_base[g], vtx_base[g+1]) and packed column entries [slot_base[g], slot_base[g+1]);
 * its n_g + 1 local row offsets start at row_ptr[vtx_base[g] + g] and count from 0 to
 * 2 m_g; its column entries hold local vertex ids in [0, n_g).  Edge numbering within a
 * graph follows the single-graph convention.
 */
typedef struct {
    int64_t num_graphs;        /* B >= 0                                                     */
    const int64_t* vtx_base;   /* host int64[B+1], vtx_base[0] == 0                          */
    const int64_t* slot_base;  /* host int64[B+1], slot_base[0] == 0, each difference even   */
    const int32_t* row_ptr;    /* int32[vtx_base[B] + B] local offsets                       */
    const int32_t* col;        /* int32[slot_base[B]] local neighbour ids                    */
    int32_t on_device;         /* 1: row_ptr and col are device pointers, 0: host            */
} glt_batch;

/*
 * Global counts X1..X17 of every graph of a batch (Problem 1 of Section 3 per graph; the
 * graphs are independent, so their edge neighbourhoods are processed together in one pass
 * over the packed graph, Section 4.1).  flags must be GLT_GLOBAL.
 *   out  host array of B*17 glt_u128, graph g's counts at out[17*g .. 17*g+16]
 * Errors as glt_count; any invalid graph fails the whole call.  A large batch (at least 64
 * graphs and 2^26 column entries, on a handle created without a memory budget) is counted
 * as four parts (graph g in part g mod 4) by helper handles the handle creates on first use,
 * on their own streams and host threads at the same time; the counts are the same, the
 * handle's glt_last_work entries become the parts' sums (maxima for entries [10]-[15]) and
 * its glt_last_timing entries the longest part's.
 */
glt_status glt_count_batch(glt_ctx* ctx, const glt_batch* b, uint32_t flags, glt_u128* out, void* stream);

/*
 * Timing breakdown of the last successful glt_count or glt_count_batch on this handle, in
 * milliseconds measured with HIP events, one entry per kernel group (each one kernel, the
 * workgroup triangle and gather groups one kernel per out-degree bucket):
 * [0] validation + preprocessing (degree order, sorted oriented CSR, work lists),
 * [1] triangle / 4-clique pass, one wavefront per vertex, [2] the same, one workgroup per
 * vertex, [3] per-edge gather pass, wavefront path, [4] the same, workgroup path,
 * [5]-[8] 4-cycle wedge pass, wave / mid / workgroup / huge class, [9] vertex sums, combine
 * and reduction, [10] the whole call.  In stream mode 1 (the schedule's wedge_stream, or its
 * automatic choice) the wedge pass runs on a second stream beside entries [1]-[4]; in mode 2
 * entries [2] and [4]
 * run beside [1] and [3], and [6] (mid class, second stream) beside [5] (wave class, after
 * the vertex sums on the call's stream); overlapping entries share the chip.  Returns the
 * number of entries written (<= cap, at most 11).
 */
int glt_last_timing(const glt_ctx* ctx, float* ms, int cap);

/*
 * Work counters of the last successful glt_count or glt_count_batch on this handle:
 * [0] n, [1] m, [2] wedges y - w - x (x ranked above y and w; the 4-cycle pass's unit of
 * work) counted by the wave class, [3] by the workgroup class, [4] out-list entries scanned
 * by the triangle pass (sum over oriented edges (a,b) of |N+(b)|), wavefront path, [5] the
 * same, workgroup path, [6] triangles found by the wavefront path, [7] by the workgroup
 * path, [8] wedges of the mid class, [9] of the huge class; with the schedule's
 * record_balance, [10] the tail of the 4-cycle pass's workgroup class in nanoseconds (from
 * the time 95 % of its list entries were done to the time the last one was) and [11] the
 * span from the first entry done to the last (0 otherwise); [12]-[15] the most wedges of one
 * bottom vertex among those the schedule's bounds place in the wave, mid, workgroup and huge
 * class (as bucketed: a bottom a class hands over to the next one counts in the first).
 * Returns the number of entries written (<= cap, at most 16).  Used to state the
 * algorithmic bytes of each kernel group and the balance of the work lists (Section 4.3,
 * Table 4's orderings).
 */
int glt_last_work(const glt_ctx* ctx, uint64_t* out, int cap);

/*
 * Work schedule of a handle: how the counting passes split their work among size classes
 * (Section 4.3 splits edges by cost between workers; here vertices are split by their work
 * between wavefront and workgroup kernels).  Every schedule yields the same counts; only
 * the speed differs.  Defaults: 128, 2048, 16384, 4096, 1, 2^30, -1, -1, 0.
 */
typedef struct {
    int32_t wedge_wave_max;    /* 4-cycle pass: bottom vertices with at most this many wedges
                                  run one per wavefront with an LDS hash only (0..256)        */
    int32_t wedge_mid_max;     /* up to this many: one per wavefront with a dense window of
                                  16-bit top counters and a hash (>= 0; at most 65,535 apply) */
    int32_t wedge_dense;       /* width of the dense window of highest-ranked tops (0..16384;
                                  each class caps it at its own table: 1024, 4096, 16384)     */
    int32_t wedge_range_limit; /* distinct hashed tops per range before it is halved (1..4096;
                                  each class caps it at half its hash: 256, 512, 1024, 4096)  */
    int32_t tri_records;       /* 1: store each triangle once for the 4-clique sweep and the
                                  gather pass when the record buffer fits; 0: re-scan lists  */
    int32_t wedge_wg_max;      /* up to this many: one per 256-thread workgroup, moving to the
                                  1024-thread class with the largest tables if its distinct
                                  tops overflow the workgroup's tables; more: straight there */
    int32_t wedge_stream;      /* streams: 0 all passes on the call's stream; 1 the 4-cycle
                                  pass on a second stream beside the triangle and gather
                                  passes; 2 the workgroup paths of the triangle and gather
                                  passes on a second stream beside their wavefront paths,
                                  then the mid 4-cycle class there beside the vertex sums
                                  and the wave class, the larger classes alone after both;
                                  -1 (default): 2                                              */
    int32_t list_order;        /* order of the workgroup work lists (Section 4.3's edge order,
                                  Table 4's ordering study): 0 largest work first, 1 largest
                                  degree first, 2 ascending rank (no sort), 3 pseudo-random,
                                  4 largest volume first (volume: the sum of the neighbours'
                                  degrees), 5 smallest degree first, 6 smallest volume first;
                                  -1 (default) chosen per call: 1 for a single graph of at
                                  least 2^25 edges, else 2                                   */
    int32_t record_balance;    /* 1: time when each entry of the 4-cycle pass's workgroup-class
                                  list is done (one clock read per entry) and report the
                                  spread in glt_last_work entries [10], [11]; 0: off         */
} glt_schedule;

/* The handle's current schedule. */
glt_status glt_get_schedule(const glt_ctx* ctx, glt_schedule* out);

/* Replace the handle's schedule; GLT_E_INVALID_ARG (and no change) if a field is outside its
 * range. */
glt_status glt_set_schedule(glt_ctx* ctx, const glt_schedule* s);

/*
 * Autotuner for batches: counts the batch once per candidate schedule (a fixed 36-point grid
 * over the wedge class bounds, the dense window and the stream mode wedge_stream, after one
 * warm-up call), checks that all candidates give identical counts (GLT_E_INTERNAL
 * otherwise), installs the candidate with the least device time (the whole call,
 * glt_last_timing's last entry) on the handle and returns it.
 *   best     out: the chosen schedule
 *   best_ms  out (may be NULL): its device time in milliseconds
 * Errors as glt_count_batch.
 */
glt_status glt_autotune_batch(glt_ctx* ctx, const glt_batch* b, glt_schedule* best, float* best_ms, void* stream);

/*
 * Calibration of the roofline (measurement only; counts nothing).  Allocates `bytes` of
 * device memory on `device`, runs one untimed and `reps` timed launches of a probe kernel
 * over it and frees it:
 *   kind 0  global atomic adds, each wavefront to a run of 64 consecutive 32-bit words at a
 *           pseudo-random 256-byte-aligned place (the pattern of the counting passes' credits
 *           to the out-edges of one vertex)
 *   kind 1  global atomic adds, each lane to a pseudo-random 32-bit word
 *   kind 2  one read of every byte (16-byte loads, grid-stride), no stores besides one
 *           word per workgroup
 *   kind 3, 4  as 0 and 1 with 64-bit words (runs of 64 words are 512 bytes)
 *   ms   out: average time of one launch in milliseconds (HIP events)
 *   ops  out: atomic adds (kinds 0, 1, 3, 4) or bytes read (kind 2) per launch
 * Errors: GLT_E_INVALID_ARG (null output, reps < 1, unknown kind, bytes outside
 * [16 KiB, 16 GiB)), GLT_E_OOM, GLT_E_DEVICE.
 */
glt_status glt_probe(int device, int kind, size_t bytes, int reps, float* ms, uint64_t* ops);

/*
 * The 4-cycle (wedge) pass of the last successful single-graph glt_count on this handle,
 * run again on host threads: the CPU worker of Section 4.3's hybrid scheme (CPU workers take
 * jobs from the front of the ordered queue in small chunks; here bottoms in rank order, 16 at
 * a time, to whichever thread is free), for measuring what a host share of the work would
 * cost beside the device.  Counts nothing for the caller: the per-edge credits land in a
 * scratch host array and only totals are reported.  Copies the relabelled graph it needs
 * from the handle's device workspace (pinned host memory, allocated and freed by the call).
 *   threads  host threads (<= 0: all hardware threads)
 *   r        out: the report below
 * Errors: GLT_E_INVALID_ARG (null argument, or no single-graph count on the handle since its
 * creation or its last batch call), GLT_E_OOM (host memory), GLT_E_DEVICE.
 */
typedef struct {
    int32_t threads;        /* host threads used                                            */
    uint64_t wedges;        /* wedges y - w - x (x above y) visited, each once per sweep     */
    uint64_t cycles4;       /* non-induced 4-cycles found: sum over (y, x) of C(c(y, x), 2)  */
    uint64_t gpu_cycles4;   /* the same total from the device's wedge pass of that call      */
    uint64_t credit_sum;    /* sum of the per-edge 4-cycle credits (4 x cycles4 if correct)  */
    uint64_t bytes_copied;  /* bytes copied from the device (offsets, wedge ranges, columns) */
    double copy_ms;         /* wall time of those copies                                    */
    double count_ms;        /* wall time of both sweeps over every bottom vertex            */
} glt_host_wedge_report;
glt_status glt_host_wedges(glt_ctx* ctx, int threads, glt_host_wedge_report* r);

/* ------------------------------------------------------------------------------------ */
/* Request server: continuous batching of graph-count requests on one device.            */
/* Requests are admitted in arrival order into a device-resident pool as its budget      */
/* allows (copied on a copy stream), and every admitted request whose copy has finished   */
/* joins the next batched launch (global counts, as glt_count_batch) on a compute stream, */
/* so requests arriving during a launch overlap with it.  A request whose graph is        */
/* invalid fails alone.                                                                    */
/* ------------------------------------------------------------------------------------ */

typedef struct glt_server glt_server;

typedef struct {
    int32_t device;            /* HIP device                                                   */
    int32_t max_batch_graphs;  /* requests per launch; 0 = no limit, 1 = one request per launch */
    int64_t max_batch_edges;   /* edges per launch (a larger request runs alone); 0 = 8,388,608 */
    size_t resident_bytes;     /* device pool for admitted graphs (the admission budget); 0 = 4 GiB */
    size_t workspace_bytes;    /* cap of the counting workspace (0 = none)                      */
    int32_t max_pending;       /* queued, not yet admitted requests before GLT_E_BUSY; 0 = 2^20 */
    int32_t large_edges;       /* requests with more edges run on a second compute lane (its own
                                  stream and workspace), overlapping the small-request batches
                                  instead of holding them up; 0 = 262,144, -1 = one lane       */
} glt_server_opts;

typedef struct {
    uint64_t req_id;           /* as passed to glt_server_submit                               */
    int32_t status;            /* glt_status of this request                                   */
    int32_t batch_graphs;      /* number of requests in the launch that counted it             */
    glt_u128 X[17];            /* X1..X17 when status == GLT_OK                                 */
    double t_submit, t_admit, t_start, t_done;   /* seconds on glt_server_clock()              */
} glt_result;

/* Create a server (starts its admission and compute threads).  opts may be NULL. */
glt_status glt_server_create(const glt_server_opts* opts, glt_server** out);

/* Queue one request.  g must describe host memory (on_device == 0); it is copied before the
 * call returns.  Returns GLT_E_BUSY when max_pending requests are already queued, and
 * GLT_E_INVALID_ARG / GLT_E_UNSUPPORTED for malformed sizes (n, 2m < 2^30 per request). */
glt_status glt_server_submit(glt_server* s, const glt_csr* g, uint64_t req_id);

/* Move up to max completed results to out, waiting up to timeout_us for the first one.
 * Returns the number written. */
int glt_server_poll(glt_server* s, glt_result* out, int max, int timeout_us);

/* Requests submitted and not yet completed. */
int64_t glt_server_inflight(glt_server* s);

/* Monotonic clock (seconds) used for the result timestamps. */
double glt_server_clock(void);

/* Stop the threads and release everything; results not yet polled are discarded. */
void glt_server_destroy(glt_server* s);

#ifdef __cplusplus
}
#endif

#endif /* GLT_H */
