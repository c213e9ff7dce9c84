// glt_internal.h -- internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prims.h"

// Error bits raised by device-side validation.
enum {
    ERR_RANGE = 1,       // neighbour id outside [0, n) or offsets not monotone
    ERR_SELF = 2,        // self-loop
    ERR_DUP = 4,         // duplicate entry
    ERR_ASYM = 8,        // entry without its reverse
    ERR_NEG = 16,        // a per-edge count came out negative (internal)
    ERR_CAP = 32,        // an LDS table or range stack bound was exceeded (internal)
};
// d.err words: [0] error bits, [1] maximum degree, [2 + c] rows of sort class c (from the
// validation), [2 + RS_N + c] append counters of the row lists (preprocessing).
#define ERR_WORDS 16

// Size classes of the per-row sort of P2 (entries per row).
enum { RS_TINY = 0, RS_WAVE, RS_WMID, RS_BLK, RS_BIG, RS_N };
#ifndef RT_MAX
#define RT_MAX 32       // thread per row (sorting network in registers)
#endif
#define RW_MAX 64       // wavefront per row (bitonic over lanes)
#ifndef RM_MAX
#define RM_MAX 256      // wavefront per row (bitonic in the wavefront's LDS)
#endif
#define RB_MAX 2048     // workgroup per row (bitonic in LDS); longer rows: radix passes
__host__ __device__ inline int row_class(int64_t len) {
    return len <= 1 ? -1 : len <= RT_MAX ? RS_TINY : len <= RW_MAX ? RS_WAVE : len <= RM_MAX ? RS_WMID
                                     : len <= RB_MAX ? RS_BLK : RS_BIG;
}

// Per oriented edge (u -> v, u before v in the degree order) accumulators, one dense
// array per quantity indexed by the oriented index k.  Credits to the out-edges of one
// vertex land on consecutive k, so a wavefront's atomics coalesce into few cache lines.
// Widths: an edge u -> v (d_u <= d_v <= dmax) has K < d_u^2 / 2, P < d_u d_v, g < 2 d_u d_v and
// sig < d_u dmax, so every value stays below 2^32 when d_u dmax < 2^31.  Such "narrow" edges
// keep K and P as 32-bit words and g, sig packed in one 64-bit word (g low, sig high).  In
// the degree order the other, "wide" edges are a suffix [kw, m) of the oriented index (their
// lower endpoint has degree >= 2^31 / dmax); they keep four 64-bit words each in the arrays
// Kw, Pw, gw, sw indexed by k - kw.  kw is settled during preprocessing: m when no edge is wide
// (32-bit kernels), the first wide edge when the wide suffix is at most m / 4 (its arrays then
// live in the sig buffer), else 0 (every edge wide; Kw..sw are K, P, g, sig themselves).
struct EdgeArrays {
    u32* t;      // triangles on the edge
    u64* K;      // 4-cliques on the edge (edges inside T): u32 words below kw
    u64* P;      // non-induced 4-cycles through the edge: u32 words below kw
    u64* g;      // below kw: sum over w in T of t(w,u) + t(w,v) (low half) and of d_w (high half)
    u64* sig;    // storage of the wide arrays (see above)
    int* u;      // lower-ranked endpoint (relabelled id); the other one is ocol[k]
    int kw;      // first wide edge (m: none)
    u64* Kw; u64* Pw; u64* gw; u64* sw;   // wide edges' K, P, g, sig at k - kw
};

// Wide-edge storage for a given split point (the same on host and device).
__host__ __device__ inline void wide_arrays(EdgeArrays& e, int m, int kw) {
    e.kw = kw;
    if (kw <= 0) {
        e.Kw = e.K; e.Pw = e.P; e.gw = e.g; e.sw = e.sig;
    } else {
        const int64_t nw = (int64_t)m - kw;
        e.Kw = e.sig; e.Pw = e.sig + nw; e.gw = e.sig + 2 * nw; e.sw = e.sig + 3 * nw;
    }
}

// Sums produced by the counting passes, all reduced to 128 bits at the end.
// Index layout of the per-block partials and of the final reduction:
//   0..13  : unrestricted sums C3,C4,C5,C7,C8,C9,C10,C11,C12,C13,C14,C15,C16 (13 used)
//   14     : 3 x (number of 4-cliques), from the triangle pass
//   15     : number of non-induced 4-cycles, from the wedge pass
#define NSUMS 16
#define NWORK 12   // device work counters (glt_last_work entries [2]-[9], then [12]-[15])
#define NSEG 11     // timed groups: prep, tri wave, tri wg, gather wave, gather wg, wedge wave, wedge mid,
                    // wedge wg, wedge huge, combine, total
#define NEV 17      // events of one call (see count_passes)
enum { S_C3 = 0, S_C4, S_C5, S_C7, S_C8, S_C9, S_C10, S_C11, S_C12, S_C13, S_C14, S_C15, S_C16,
       S_SPARE, S_K4x3, S_NC4 };
// The per-group totals array (gsum) holds NSUMS words per line and uses S_K4x3, S_NC4 and
// the triangle counts of the two triangle-pass paths (measurement only).
enum { GS_TRI_WAVE = 0, GS_TRI_WG = 1 };
#define GLT_REDUCE_BLOCKS 256   // first-stage workgroups of the 128-bit partial-sum reduction
#define GSPREAD 64   // lines of gsum a single graph's groups spread their atomics over
#define WSPREAD_WORDS 12  // u64 per line of the spread work counters (folded into work[])
// gsum line of a group: its graph in a batch, else spread by workgroup index
__device__ __forceinline__ int64_t gslot(const int* ngid, int v) {
    return ngid ? (int64_t)ngid[v] : (int64_t)(blockIdx.x & (GSPREAD - 1));
}

// Orders of the workgroup work lists (the paper's study of edge orderings, Section 4.3 and
// Table 4, applied to vertex work lists): largest work, degree or volume (sum of the
// neighbours' degrees) first, their inverses (smallest first), ascending rank (the bucketing
// order, no sort) and pseudo-random.
enum { LO_WORK = 0, LO_DEGREE = 1, LO_NONE = 2, LO_RANDOM = 3, LO_VOLUME = 4, LO_DEGREE_INV = 5,
       LO_VOLUME_INV = 6, LO_N = 7 };

// Bucket ids for the vertex work lists.
enum { TB_WAVE = 0, TB_BLK1, TB_BLK2, TB_GLOBAL, TB_N };   // triangle / gather passes
// segments of n entries in the triangle-pass list area, which holds the row-sort lists first
#define TL_SEGS (TB_N > RS_N ? TB_N : RS_N)
// Largest out-degree whose adjacency rows the workgroup triangle pass keeps in LDS (bucket
// TB_BLK2): 896 rows of 28 words, the hash, the per-neighbour arrays and the run tables of a
// 1024-thread group fill about 152 KB of the CU's 160 KB.
#ifndef TB_LDS_ROWS
#define TB_LDS_ROWS 896
#endif
// Oriented edges per combine workgroup of a batch (each graph's edges are cut into chunks of
// this many, so a few large graphs still spread over many workgroups).
#define CG_CHUNK 8192
enum { WB_WAVE = 0, WB_MID, WB_BLK, WB_HUGE, WB_N };        // wedge pass
// d.counts words: TB_N triangle-list counts, WB_N wedge-list counts, TB_N largest out-degrees
// per triangle list, the accumulator split point kw (EdgeArrays), and the number of bottoms
// the mid wedge class handed to the workgroup class (appended after the latter's own list).
#define CNT_KW (TB_N + WB_N + TB_N)
#define CNT_MID_TO_WG (CNT_KW + 1)
#define CNT_WORDS (CNT_KW + 2)
// Padded accumulation of the work-list counters and largest out-degrees (then copied into
// counts): APAD_SLOTS counters, APAD_STRIDE ints (4 KiB) apart.
#define APAD_STRIDE 1024
#define APAD_SLOTS (TB_N + WB_N + TB_N)

// Device pointers of one graph's workspace.
struct Dev {
    int n;            // vertices
    int m;            // undirected edges
    int S;            // 2m CSR slots
    int* err;         // error bits
    int* deg;         // original ids: degree
    int* order;       // rank -> original id
    int* rank;        // original id -> rank (relabelled id)
    int* ndeg;        // relabelled id -> degree
    int* nrp;         // relabelled CSR offsets [n+1]
    int* ncol;        // relabelled CSR columns [S], ascending within a row
    int* dlo;         // number of lower-ranked neighbours of each vertex
    int* optr;        // oriented (upward) CSR offsets [n+1]
    int4* vinf;       // per vertex: first upward slot, row end, optr, original id [n]
    int* ocol;        // oriented CSR columns [m], ascending
    int* s2k;         // CSR slot -> oriented edge index [S]
    int* eid2k;       // caller edge id -> oriented edge index [m]
    int2* wb;         // CSR slot s of row y (w = ncol[s]) -> oriented range [k0, k1) of the tops x > y of
                      // the wedges y - w - x: N+(w), or its part after y when w < y [S]
    EdgeArrays e;     // per-edge accumulators [m] each
    u64* tri;         // twice the triangles at each relabelled vertex [n]
    u64* erec;        // per-edge combine records, 32 bytes per oriented edge [4m] (single graphs)
    u64* vrec;        // per-vertex combine records, 32 bytes per vertex [4n] (single graphs)
    u64* sdeg;        // sum of neighbour degrees [n]
    int* tlist;       // triangle-pass vertex lists, TB_N segments of n
    u64* toff;        // [n+1] triangle-record slots before vertex a: prefix of C(|N+(a)|, 2)
    int* tcnt;        // [n] triangle records written for lowest vertex a
    u64* tmp64;       // scan scratch for toff
    u64* wspread;     // [GSPREAD][WSPREAD_WORDS] work counters, folded into work[] after the passes
    u64* trec;        // triangle records (null: the passes re-scan the out-lists instead)
    int* wlist;       // wedge-pass vertex lists, WB_N segments of n
    int* counts;      // bucket counts and maxima (TB_N + WB_N + TB_N)
    int* apad;        // [APAD_SLOTS * APAD_STRIDE] the same, accumulated apart (see k_pad_to_counts)
    u64* work;        // work counters [NWORK]: wedges (wave / workgroup class), triangle-pass list
                      // entries (wave / workgroup path), triangles found (wave / workgroup path),
                      // wedges (mid / huge class)
    u64* wcnt;        // wedges per vertex [n] (wedge-pass bucketing)
    u32* rowx;        // [S+1] exclusive prefix of row starts of the input CSR: row of entry s = rowx[s+1]-1
    int* nsrow;       // [S] row of each relabelled CSR entry
    u64* sums;        // per-block partial sums, 13 (lo, hi) pairs per entry, then GLT_REDUCE_BLOCKS entries
    int nsum_slots;   // combine blocks' entries of sums (the reduction stage's follow)
    u64* final_sums;  // 2*NSUMS u64 (lo,hi) reduced 128-bit sums
    u32* gscratch;    // global-memory adjacency bitmaps for very high out-degree
    int64_t gscratch_words;
    // preprocessing scratch
    u64* key0; u64* key1; u32* val0; u32* val1;
    u32* upx;         // prefix of "upward" flags over the caller's slots [S+1]
    u32* rs_counts; u32* rs_tmp;
    int* itmp; int64_t* ltmp;
    // per-graph accumulation (batched mode: the input is a disjoint union of graphs)
    int ngraphs;          // 0 for a single graph
    int* gid;             // original vertex -> graph (batched mode)
    int* ngid;            // relabelled vertex -> graph (batched mode), else null
    int* vtop;            // relabelled vertex -> end of its graph's rank range (batched mode), else null
    u64* gsum;            // [max(1, ngraphs)][NSUMS] 4-clique / 4-cycle accumulators
    const int64_t* gvb;   // device copy of the per-graph vertex bases [ngraphs+1]
    const int64_t* gsb;   // device copy of the per-graph slot bases [ngraphs+1]
    u64* gparts;          // [ngraphs][13][2] per-graph unrestricted sums (128-bit)
    int* gcb;             // [ngraphs+1] first combine chunk of each graph (CG_CHUNK oriented edges each)
    int ncchunks;         // combine chunks of the batch (gcb[ngraphs])
    u64* cparts;          // [chunks][13][2] per-chunk unrestricted sums
    const int** glrp;     // device array of per-graph local-offset pointers [ngraphs]
    const int** glcol;    // device array of per-graph local-column pointers [ngraphs]
    // tuning (defaults; overridable per handle for testing)
    int wedge_wave_max;   // wedge-pass vertices with at most this many wedges: wave class (hash only)
    int wedge_mid_max;    // up to this many: mid class (one wavefront, dense window + hash)
    int wedge_wg_max;     // up to this many: workgroup class; more: huge class (1024 threads, big tables)
    int num_cu;           // compute units (resident grid of the huge class)
    int list_order;       // LO_*: order of the workgroup work lists
    int wedge_limit;      // distinct hashed tops per range before the range is split
    int wedge_dense;      // width of the dense window of highest-ranked tops
    int acc32;            // 32-bit accumulator kernels: no wide edge (EdgeArrays), or global counts only
    int wide_degree;      // > 0: lower endpoint degree from which edges are wide, if below the bound (tests)
    u64* tstamp;          // null, or per workgroup-class wedge list entry the wall clock when it was done
                          // (load-balance measurement; the preprocessing scratch key1 is reused)
    int per_edge;         // per-edge output requested (global counts need neither caller edge
                          // ids nor the K, P, g, sigma accumulators)
};

// Host-side entry points of the device pipeline (count.hip).
struct Timing { float ms[5]; };

int glt_union_build(const Dev& d, int* urp, int* ucol, hipStream_t st);
int glt_prep_validate(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st);
int glt_prep_build(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st,
                   const int* vinfo /* max degree, then RS_N row-class counts */);
void glt_count_passes(const Dev& d, int per_edge, const int* host_counts, u64* out_pe,
                      hipStream_t st, hipStream_t side, hipEvent_t* ev /* NEV events, ev[0] recorded by the caller */,
                      int mode /* streams: 0 one, 1 wedge pass on `side`, 2 workgroup paths on `side` */);

// The device arrays of the handle's last successful single-graph count (false if there is
// none) and the 4-cycle total of its wedge pass; the handle's device.
struct glt_ctx;
bool glt_last_graph(const glt_ctx* ctx, Dev* d, uint64_t* cycles4);
int glt_ctx_device(const glt_ctx* ctx);
