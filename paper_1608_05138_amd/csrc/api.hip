// api.hip -- the C ABI of libglt: handles, workspace, validation, the exact combination of
// the unrestricted counts into global frequencies (Section 4.6).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/glt.h"
#include "glt_internal.h"

typedef __int128 i128;
typedef unsigned __int128 u128;

int glt_combine_blocks(int m);
int64_t glt_slab_words(int smax);
int glt_wedge_table();
int glt_wave_table();
int glt_wedge_dense();

// Large batches (at least GLT_BATCH_SPLIT_GRAPHS graphs and 2^26 entries, on a handle without
// a memory budget) are dealt round-robin to GLT_BATCH_PARTS parts counted at the same time.
#define GLT_BATCH_PARTS 4
#define GLT_BATCH_SPLIT_GRAPHS 64
#define GLT_BATCH_SPLIT_SLOTS ((int64_t)1 << 26)

struct glt_ctx {
    int device = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    float timing[NSEG] = {};
    hipEvent_t ev[NEV] = {};
    hipStream_t side = nullptr;       // second stream: the wedge pass runs beside the triangle passes
    u64* hbuf = nullptr;   // pinned host buffer for small read-backs (4 KiB)
    int wedge_wave_max = 0;
    int wedge_mid_max = 0;
    int wedge_wg_max = 0;
    int num_cu = 256;
    int wedge_limit = 0;
    int wedge_dense = 0;
    // n, m, device work counters 0-7, the workgroup class's tail and span, device counters 8-11
    uint64_t work[2 + NWORK + 2] = {};
    int record_balance = 0;            // schedule: time the entries of the workgroup wedge class
    int bal_count = 0;                 // entries of that list in the last call
    int clock_khz = 100000;            // device wall-clock rate
    void* stage = nullptr;             // device staging of host batch inputs
    size_t stage_bytes = 0;
    void* trec = nullptr;              // triangle records (grown on demand)
    size_t trec_bytes = 0;
    size_t trec_cap = 0;               // largest record buffer the handle allocates
    int tri_records = 1;               // schedule: use triangle records when they fit
    int wedge_stream = -1;             // schedule: stream mode (-1 chosen per call, see resolve_schedule;
                                       // 0 one stream: each kernel group has
                                       // the chip alone; 1 wedge pass on the side stream; 2 the
                                       // workgroup triangle / gather paths on the side stream, the
                                       // wedge pass alone)
    int list_order = -1;               // schedule: order of the workgroup work lists (LO_*; -1 chosen
                                       // per call, see resolve_schedule)
    int last_mode = 0;                 // the stream mode the last call's timing was taken in
    int wide_degree = 0;               // GLT_WIDE_DEGREE (tests): widen edges from this lower-endpoint degree
    void* slab = nullptr;              // larger global slab for the highest out-degrees (grown on demand)
    size_t slab_bytes = 0;
    hipEvent_t ev_null = nullptr;      // orders the handle's stream after the legacy default stream
    void* scratch = nullptr;           // device address of this device's glt_count_noalloc workspace
    glt_ctx* part[GLT_BATCH_PARTS] = {};   // helper handles of large batches (created on first use)
    hipEvent_t ev_part = nullptr;      // the parts' streams start after the caller's stream reaches it
    Dev last;                          // device arrays of the last single-graph count (glt_host_wedges)
    bool last_valid = false;
    uint64_t last_cycles4 = 0;         // its wedge pass's 4-cycle total
};

#define GLT_VERSION "glt 0.2 (gfx950)"

// Workspace of glt_count_noalloc: one fixed array per device (each device that loads the
// library holds its own copy until the process ends).  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress, once per device, at handle
// creation (scratch_address).
#define GLT_SCRATCH_BYTES GLT_NOALLOC_MAX_BYTES
static __device__ __align__(256) unsigned char scratch[GLT_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up once per device.
hipError_t scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

constexpr size_t kAlign = 256;
constexpr int64_t kGScratchWords = 8 << 20;   // 32 MiB of global bitmap rows / accumulators

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(int64_t count) {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T* p = (T*)(base ? base + off : nullptr);
        off += (size_t)(count > 0 ? count : 1) * sizeof(T);
        return p;
    }
};

// Input-side buffers of one call besides the pipeline arrays.
struct Staging {
    void* rp = nullptr;     // host-copied offsets (single graph) or union offsets (batched)
    int* col = nullptr;     // host-copied columns (single) or union columns (batched)
    u64* out = nullptr;     // device per-edge output when the caller's is host memory
    int* lrp = nullptr;     // batched: host-copied local offsets
    int* lcol = nullptr;    // batched: host-copied local columns
};

// Lays out every array of one call's workspace (with base == nullptr: only sizes it).
// ngraphs > 0 selects the batched layout (union offsets/columns and per-graph arrays).
size_t carve(void* base, int n, int m, int rp64, bool host_in, bool host_out, int ngraphs,
             int64_t local_rp_len, Dev& d, Staging& sg) {
    Carver c(base);
    const int64_t S = 2 * (int64_t)m;
    const int64_t big = S > n ? S : n;
    d.n = n; d.m = m; d.S = (int)S;
    d.err = c.take<int>(ERR_WORDS);
    d.counts = c.take<int>(CNT_WORDS);
    d.work = c.take<u64>(NWORK);
    d.final_sums = c.take<u64>(2 * 13);
    d.apad = c.take<int>((int64_t)APAD_SLOTS * APAD_STRIDE);   // (after err..work: one read-back takes those)
    d.deg = c.take<int>(n);
    d.order = c.take<int>(n);
    d.rank = c.take<int>(n);
    d.ndeg = c.take<int>(n);
    d.nrp = c.take<int>(n + 1);
    d.dlo = c.take<int>(n);
    d.optr = c.take<int>(n + 1);
    d.vinf = c.take<int4>(n);
    d.ncol = c.take<int>(S);
    d.ocol = c.take<int>(m);
    d.s2k = c.take<int>(S);
    d.eid2k = c.take<int>(m);
    d.wb = c.take<int2>(S);
    d.e.t = c.take<u32>(m);
    d.e.K = c.take<u64>(m);
    d.e.P = c.take<u64>(m);
    d.e.g = c.take<u64>(m);
    d.e.sig = c.take<u64>(m);
    d.e.u = c.take<int>(m);
    d.wcnt = c.take<u64>(n);
    d.toff = c.take<u64>(n + 1);
    d.tcnt = c.take<int>(n);
    d.tmp64 = c.take<u64>(scan_tmp_elems(n + 1));
    d.wspread = c.take<u64>((int64_t)GSPREAD * WSPREAD_WORDS);
    d.rowx = c.take<u32>(S + 1);
    d.nsrow = c.take<int>(S);
    d.tri = c.take<u64>(n);
    d.sdeg = c.take<u64>(n);
    d.tlist = c.take<int>((int64_t)TL_SEGS * n);
    d.wlist = c.take<int>((int64_t)WB_N * n);
    d.nsum_slots = glt_combine_blocks(m > 0 ? m : 1);
    d.sums = c.take<u64>((int64_t)(d.nsum_slots + GLT_REDUCE_BLOCKS) * 13 * 2);   // + reduction stage
    d.gscratch_words = kGScratchWords;
    d.gscratch = c.take<u32>(kGScratchWords);
    d.key0 = c.take<u64>(big);
    d.key1 = c.take<u64>(big);
    d.val0 = c.take<u32>(big);
    d.val1 = c.take<u32>(big);
    d.upx = c.take<u32>(S + 1);
    const int64_t rsc = rs_counts_elems(big);
    d.rs_counts = c.take<u32>(rsc);
    d.rs_tmp = c.take<u32>(scan_tmp_elems(rsc > big ? rsc : big));
    d.itmp = c.take<int>(scan_tmp_elems(S + n + 1) + n + 1);
    d.ltmp = nullptr;
    d.ngraphs = ngraphs;
    d.gsum = c.take<u64>((int64_t)(ngraphs > 0 ? ngraphs : GSPREAD) * NSUMS);
    if (ngraphs > 0) {
        d.gparts = c.take<u64>((int64_t)ngraphs * 13 * 2);   // right after gsum: one read-back takes both
        d.gid = c.take<int>(n);
        d.ngid = c.take<int>(n);
        d.vtop = c.take<int>(n);
        d.ncchunks = 0;
        d.cparts = c.take<u64>(((int64_t)m / CG_CHUNK + ngraphs + 1) * 13 * 2);
        // the per-graph tables the host fills, side by side (one copy writes all five)
        d.gvb = c.take<int64_t>(ngraphs + 1);
        d.gsb = c.take<int64_t>(ngraphs + 1);
        d.gcb = c.take<int>(ngraphs + 1);
        d.glrp = (const int**)c.take<int*>(ngraphs);
        d.glcol = (const int**)c.take<int*>(ngraphs);
        sg.rp = c.take<int>(n + 1);
        sg.col = c.take<int>(S);
        sg.lrp = sg.lcol = nullptr;
        sg.out = nullptr;
        (void)host_in;
        (void)local_rp_len;
        d.erec = d.vrec = nullptr;
    } else {
        d.erec = c.take<u64>(4 * (int64_t)m);
        d.vrec = c.take<u64>(4 * (int64_t)n);
        d.gid = d.ngid = d.vtop = nullptr;
        d.gvb = d.gsb = nullptr;
        d.gparts = nullptr;
        d.gcb = nullptr;
        d.ncchunks = 0;
        d.cparts = nullptr;
        d.glrp = d.glcol = nullptr;
        sg.rp = host_in ? (void*)c.take<char>((int64_t)(n + 1) * (rp64 ? 8 : 4)) : nullptr;
        sg.col = host_in ? c.take<int>(S) : nullptr;
        sg.out = host_out ? c.take<u64>(13 * (int64_t)m) : nullptr;
        sg.lrp = sg.lcol = nullptr;
    }
    return c.off + kAlign;
}

glt_status fail(glt_ctx* ctx, glt_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return s;
}

#define HIPCHK(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(ctx, GLT_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_));       \
    } while (0)

i128 ch2(i128 x) { return x < 2 ? 0 : x * (x - 1) / 2; }
i128 ch3(i128 x) { return x < 3 ? 0 : x * (x - 1) * (x - 2) / 6; }
i128 ch4(i128 x) { return x < 4 ? 0 : x * (x - 1) / 2 * (x - 2) * (x - 3) / 12; }

// Global frequencies from the unrestricted counts (Section 4.6, with C9 = sum |T|(|S_u|+|S_v|)
// and X11 from C11).  k4 is the number of 4-cliques and nc4 the number of non-induced
// 4-cycles (each counted once by the triangle and wedge passes).  In per-edge mode C7 and C10
// come from the per-edge counts too and must agree.  Returns false if a division that must
// be exact is not, or a count is negative: both indicate a library bug.
bool globals(int64_t n, int64_t m, const i128 C[17], i128 k4, i128 nc4, bool per_edge, i128 X[18],
             std::string& why) {
    auto exact = [&](i128 num, int den, i128& dst, const char* name) {
        if (num < 0 || num % den != 0) { why = std::string("inexact ") + name; return false; }
        dst = num / den;
        return true;
    };
    X[1] = m;
    X[2] = ch2(n) - m;
    if (!exact(C[3], 3, X[3], "X3")) return false;
    if (!exact(C[4], 2, X[4], "X4")) return false;
    X[5] = C[5];
    X[6] = ch3(n) - X[3] - X[4] - X[5];
    X[7] = k4;
    if (per_edge && C[7] != 6 * k4) { why = "4-clique totals disagree"; return false; }
    X[8] = C[8] - 6 * X[7];
    if (!exact(C[9] - 4 * X[8], 2, X[9], "X9")) return false;
    X[10] = nc4 - X[8] - 3 * X[7];   // a chordal cycle holds one 4-cycle, a 4-clique three
    if (per_edge && C[10] != 4 * X[10]) { why = "4-cycle totals disagree"; return false; }
    if (!exact(C[11] - X[9], 3, X[11], "X11")) return false;
    X[12] = C[12] - 4 * X[10];
    if (!exact(C[13] - X[9], 3, X[13], "X13")) return false;
    if (!exact(C[14] - 6 * X[7] - 4 * X[8] - 2 * X[9] - 4 * X[10] - 2 * X[12], 2, X[14], "X14")) return false;
    if (!exact(C[15] - 2 * X[12], 2, X[15], "X15")) return false;
    X[16] = C[16] - 2 * X[14];
    i128 s = 0;
    for (int i = 7; i <= 16; i++) s += X[i];
    X[17] = ch4(n) - s;
    for (int i = 1; i <= 17; i++)
        if (X[i] < 0) { why = "negative global count"; return false; }
    return true;
}

// The unrestricted sums C3..C16 from 13 (lo,hi) pairs in the order C3,C4,C5,C7,...,C16.
void unpack_c(const u64* fs, i128 C[17]) {
    static const int cidx[13] = {3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};
    for (int i = 0; i < 17; i++) C[i] = 0;
    for (int c = 0; c < 13; c++) C[cidx[c]] = (i128)(((u128)fs[2 * c + 1] << 64) | (u128)fs[2 * c]);
}

void store_x(const i128 X[18], glt_u128* out) {
    for (int i = 0; i < 17; i++) {
        u128 v = (u128)X[i + 1];
        out[i].lo = (uint64_t)v;
        out[i].hi = (uint64_t)(v >> 64);
    }
}

// Grows the handle's workspace to `need` bytes (respecting the budget).
glt_status ensure_ws(glt_ctx* ctx, size_t need, hipStream_t st) {
    if (ctx->budget && need > ctx->budget)
        return fail(ctx, GLT_E_OOM, "workspace of %zu bytes exceeds the budget of %zu", need, ctx->budget);
    if (need <= ctx->ws_bytes) return GLT_OK;
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->ws) { (void)hipFree(ctx->ws); ctx->ws = nullptr; ctx->ws_bytes = 0; }
    if (hipMalloc(&ctx->ws, need) != hipSuccess) {
        ctx->ws = nullptr;
        (void)hipGetLastError();
        return fail(ctx, GLT_E_OOM, "hipMalloc of %zu bytes failed", need);
    }
    ctx->ws_bytes = need;
    return GLT_OK;
}

// Triangle records need 8 bytes per slot (sum over vertices of C(out-degree, 2)).  They are
// used when that fits the handle's record cap and budget; otherwise the passes re-scan the
// out-lists, with the same results.
// The workgroup passes for out-degrees above the LDS limit keep their rows (or accumulators)
// in a global slab, one region per workgroup, launched in groups that fit it.  The built-in
// 32 MiB slab is replaced by one that holds every such workgroup at once when that fits
// 1 GiB and the budget (one launch instead of dozens on heavy-tailed graphs).
void grow_slab(glt_ctx* ctx, Dev& d, int count, int smax, hipStream_t st) {
    if (count <= 0 || smax <= 0) return;
    const int64_t per = glt_slab_words(smax);   // one workgroup's region (triangle and gather passes)
    const int64_t want = std::min<int64_t>(std::max<int64_t>(per * count, per), (int64_t)1 << 28);   // words (1 GiB)
    if (want <= d.gscratch_words) return;
    const size_t need = (size_t)want * 4;
    if (need > ctx->slab_bytes) {
        if (ctx->budget && ctx->ws_bytes + ctx->trec_bytes + need > ctx->budget) return;
        if (hipStreamSynchronize(st) != hipSuccess) return;
        if (ctx->slab) { (void)hipFree(ctx->slab); ctx->slab = nullptr; ctx->slab_bytes = 0; }
        if (hipMalloc(&ctx->slab, need) != hipSuccess) {
            ctx->slab = nullptr;
            (void)hipGetLastError();
            return;
        }
        ctx->slab_bytes = need;
    }
    d.gscratch = (u32*)ctx->slab;
    d.gscratch_words = (int64_t)(ctx->slab_bytes / 4);
}

u64* ensure_trec(glt_ctx* ctx, u64 slots, hipStream_t st) {
    if (slots == 0 || ctx->trec_cap == 0 || !ctx->tri_records) return nullptr;
    if (slots > (u64)(ctx->trec_cap / 8)) return nullptr;
    const size_t need = (size_t)slots * 8;
    if (ctx->budget && ctx->ws_bytes + need > ctx->budget) return nullptr;
    if (need <= ctx->trec_bytes) return (u64*)ctx->trec;
    if (hipStreamSynchronize(st) != hipSuccess) return nullptr;
    if (ctx->trec) { (void)hipFree(ctx->trec); ctx->trec = nullptr; ctx->trec_bytes = 0; }
    if (hipMalloc(&ctx->trec, need) != hipSuccess) {
        ctx->trec = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    ctx->trec_bytes = need;
    return (u64*)ctx->trec;
}

// The schedule's automatic fields (-1): stream mode 2, and the work lists of a single graph
// of at least 2^25 edges ordered largest degree first, of smaller graphs and batches left in
// the bucketing order.  Measured: R-MAT scale 22 (6.4*10^7 edges) 414 ms in rank order, 406
// with degree order; the Chung-Lu graph (10^7 edges) 17.1 ms in rank order, 17.6 with degree
// order.  (Mode 1 takes R-MAT to 402-404 ms, but shares the chip between the triangle and
// wedge passes, so no kernel's time is its own; it stays a schedule choice.)
#define GLT_AUTO_LARGE_EDGES (1 << 25)
void resolve_schedule(const glt_ctx* ctx, const Dev& d, int& mode, int& order) {
    const bool large = d.ngraphs == 0 && d.m >= GLT_AUTO_LARGE_EDGES;
    mode = ctx->wedge_stream >= 0 ? ctx->wedge_stream : 2;
    order = ctx->list_order >= 0 ? ctx->list_order : (large ? LO_DEGREE : LO_NONE);
}

// Validation, preprocessing and the counting passes on a prepared CSR (rp, col) on the
// device.  Host read-backs: validation flags after the row check and after the build.
glt_status run_pipeline(glt_ctx* ctx, Dev& d, const void* rp, int rp64, const int* col, bool per_edge,
                        u64* pe_dev, hipStream_t st, bool noalloc = false) {
    const int n = d.n, m = d.m;
    d.wedge_wave_max = ctx->wedge_wave_max;
    d.wedge_mid_max = ctx->wedge_mid_max;
    d.wedge_wg_max = ctx->wedge_wg_max;
    d.num_cu = ctx->num_cu;
    int mode = 0;
    resolve_schedule(ctx, d, mode, d.list_order);
    d.wedge_limit = ctx->wedge_limit;
    d.wedge_dense = ctx->wedge_dense;
    d.wide_degree = ctx->wide_degree;
    d.tstamp = ctx->record_balance ? d.key1 : nullptr;   // key1 is free once preprocessing is done
    d.per_edge = per_edge ? 1 : 0;
    HIPCHK(hipEventRecord(ctx->ev[0], st));
    glt_prep_validate(d, rp, rp64, col, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->hbuf, d.err, (2 + RS_N) * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int hc[CNT_WORDS];
    int vinfo[1 + RS_N];
    {
        const int e = ((int*)ctx->hbuf)[0];
        if (e & ERR_RANGE)
            return fail(ctx, GLT_E_INVALID_ARG,
                        "row offsets not non-decreasing from 0 to 2m, or a neighbour id out of range");
        if (e & ERR_SELF) return fail(ctx, GLT_E_NOT_SIMPLE, "self-loop");
        for (int i = 0; i < 1 + RS_N; i++) vinfo[i] = ((int*)ctx->hbuf)[1 + i];   // max degree, row classes
    }
    glt_prep_build(d, rp, rp64, col, st, vinfo);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->hbuf, d.err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 8, d.optr + n, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 16, d.counts, sizeof(int) * CNT_WORDS, hipMemcpyDeviceToHost, st));
    if (n > 0) HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 128, d.toff + n, sizeof(u64), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    {
        const int e = ((int*)ctx->hbuf)[0];
        const int up = n > 0 ? ((int*)ctx->hbuf)[2] : 0;
        if (e & ERR_DUP) return fail(ctx, GLT_E_NOT_SIMPLE, "duplicate entry");
        if ((e & ERR_ASYM) || up != m) return fail(ctx, GLT_E_NOT_SYMMETRIC, "adjacency is not symmetric");
        memcpy(hc, (char*)ctx->hbuf + 16, sizeof(int) * CNT_WORDS);
    }
    if (noalloc) {
        d.trec = nullptr;   // the passes re-scan the out-lists; the carved 32 MiB slab serves
    } else {
        d.trec = ensure_trec(ctx, n > 0 ? *(u64*)((char*)ctx->hbuf + 128) : 0, st);
        grow_slab(ctx, d, hc[TB_GLOBAL], hc[TB_N + WB_N + TB_GLOBAL], st);
    }
    // the workgroup passes above the LDS rows need at least one slab region
    if (hc[TB_GLOBAL] > 0 && glt_slab_words(hc[TB_N + WB_N + TB_GLOBAL]) > d.gscratch_words)
        return fail(ctx, GLT_E_OOM, "out-degree %d needs %lld bytes of slab per workgroup, more than available",
                    hc[TB_N + WB_N + TB_GLOBAL], (long long)glt_slab_words(hc[TB_N + WB_N + TB_GLOBAL]) * 4);
    // per-edge accumulators: 32-bit kernels when no edge is wide (or no per-edge output),
    // else 64-bit in-kernel sums with the narrow / wide storage split at kw (EdgeArrays)
    ctx->bal_count = ctx->record_balance ? hc[TB_N + WB_BLK] : 0;
    wide_arrays(d.e, m, hc[CNT_KW]);
    d.acc32 = (!per_edge || hc[CNT_KW] >= m) ? 1 : 0;
    ctx->last_mode = mode;
    glt_count_passes(d, per_edge ? 1 : 0, hc, pe_dev, st, ctx->side, ctx->ev, mode);
    HIPCHK(hipGetLastError());
    return GLT_OK;
}

// Kernel groups as (begin, end) events; the wedge groups (side stream) overlap the
// triangle and gather groups, so the groups do not add up to the total.
// The device work counters of a call into the handle's glt_last_work entries: counters 0-7
// at [2]-[9], 8-11 at [12]-[15] (entries [10], [11] are the balance summary's).
void set_work(glt_ctx* ctx, const u64* dev_work, bool valid) {
    for (int i = 0; i < NWORK; i++) ctx->work[i < 8 ? 2 + i : 4 + i] = valid ? dev_work[i] : 0;
}

void record_timing(glt_ctx* ctx) {
    // group i runs from event be[i][0] to event be[i][1] (events as in count_passes)
    int be[NSEG][2] = {{0, 1}, {1, 2}, {2, 3}, {12, 4}, {4, 5}, {14, 6},
                       {6, 7}, {15, 8}, {8, 9}, {10, 11}, {0, 11}};
    if (ctx->last_mode == 1) be[5][0] = 1;   // the wedge pass starts at the fork, beside the others
    if (ctx->last_mode == 2) {               // workgroup paths on the second stream from the fork
        be[2][0] = 1;
        be[4][0] = 13;
        be[6][0] = 5;                        // the mid class follows the gather workgroup path
    }
    for (int i = 0; i < NSEG; i++) {
        const int b0 = be[i][0];
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ctx->ev[b0], ctx->ev[be[i][1]]);
        ctx->timing[i] = ms;
    }
}

// Load-balance summary of the last call's workgroup wedge class (record_balance): from the
// wall-clock times at which its list entries were done, the tail (95th percentile to the
// last) and the span (first to last), in nanoseconds, into work[10], work[11].
glt_status balance_summary(glt_ctx* ctx, const u64* tstamp, hipStream_t st) {
    ctx->work[10] = ctx->work[11] = 0;
    const int c = ctx->bal_count;
    if (c <= 0 || !tstamp) return GLT_OK;
    std::vector<u64> t((size_t)c);
    HIPCHK(hipMemcpyAsync(t.data(), tstamp, (size_t)c * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::sort(t.begin(), t.end());
    const double ns = 1e6 / (double)ctx->clock_khz;
    const u64 p95 = t[(size_t)((int64_t)(c - 1) * 95 / 100)];
    ctx->work[10] = (uint64_t)((double)(t.back() - p95) * ns);
    ctx->work[11] = (uint64_t)((double)(t.back() - t.front()) * ns);
    return GLT_OK;
}

// The stream a call runs on.  With no stream given, the handle's own (non-blocking) stream,
// made to wait for the work already queued on the device's legacy default stream: device
// inputs (and the per-edge output buffer) may come from work still pending there.
glt_status call_stream(glt_ctx* ctx, void* stream_, hipStream_t& st) {
    if (stream_) {
        st = (hipStream_t)stream_;
        return GLT_OK;
    }
    st = ctx->stream;
    HIPCHK(hipEventRecord(ctx->ev_null, nullptr));
    HIPCHK(hipStreamWaitEvent(st, ctx->ev_null, 0));
    return GLT_OK;
}

}  // namespace

// Global counts of B graphs given per-graph device pointers to their local offsets
// (n_g + 1 entries, 0 .. 2 m_g) and local columns; vb/sb are host bases (sizes of each graph).
glt_status glt_run_batch_ptrs(glt_ctx* ctx, int64_t B, const int64_t* vb, const int64_t* sb,
                              const int* const* rp_ptrs, const int* const* col_ptrs, glt_u128* out,
                              hipStream_t st) {
    ctx->err.clear();
    ctx->last_valid = false;
    for (int64_t g = 0; g < B; g++)
        if (vb[g + 1] < vb[g] || sb[g + 1] < sb[g] || ((sb[g + 1] - sb[g]) & 1))
            return fail(ctx, GLT_E_INVALID_ARG, "graph %lld: bases not monotone or odd slot count", (long long)g);
    const int64_t N = vb[B], S = sb[B];
    if (N >= ((int64_t)1 << 31) || S >= ((int64_t)1 << 31))
        return fail(ctx, GLT_E_UNSUPPORTED, "packed vertices or slots do not fit 31 bits");
    const int n = (int)N, m = (int)(S / 2);
    HIPCHK(hipSetDevice(ctx->device));
    Dev d;
    Staging sg;
    const size_t need = carve(nullptr, n, m, 0, false, false, (int)B, 0, d, sg);
    glt_status rc = ensure_ws(ctx, need, st);
    if (rc) return rc;
    carve(ctx->ws, n, m, 0, false, false, (int)B, 0, d, sg);
    // The per-graph tables (vertex and slot bases, combine chunks, offset and column
    // pointers) are carved side by side: one host image at the same offsets, one copy.
    // Combine chunks: graph g's oriented edges (m_g of them) in pieces of CG_CHUNK.
    char* const d0 = (char*)d.gvb;
    const size_t img_bytes = (size_t)((char*)(d.glcol + B) - d0);
    std::vector<char> img(img_bytes, 0);
    memcpy(img.data() + ((char*)d.gvb - d0), vb, (size_t)(B + 1) * 8);
    memcpy(img.data() + ((char*)d.gsb - d0), sb, (size_t)(B + 1) * 8);
    memcpy(img.data() + ((char*)d.glrp - d0), rp_ptrs, (size_t)B * sizeof(void*));
    memcpy(img.data() + ((char*)d.glcol - d0), col_ptrs, (size_t)B * sizeof(void*));
    int* cb = (int*)(img.data() + ((char*)d.gcb - d0));
    for (int64_t g = 0; g < B; g++) cb[g + 1] = cb[g] + (int)(((sb[g + 1] - sb[g]) / 2 + CG_CHUNK - 1) / CG_CHUNK);
    d.ncchunks = cb[B];
    HIPCHK(hipMemcpyAsync(d0, img.data(), img_bytes, hipMemcpyHostToDevice, st));
    glt_union_build(d, (int*)sg.rp, sg.col, st);
    HIPCHK(hipGetLastError());
    rc = run_pipeline(ctx, d, sg.rp, 0, sg.col, false, nullptr, st);
    if (rc) return rc;
    // two read-backs: the per-graph sums (gsum, then gparts, carved side by side) and the
    // flag / counter words (err through work, carved side by side at the start)
    const size_t res_bytes = (size_t)((char*)(d.gparts + (size_t)B * 26) - (char*)d.gsum);
    const size_t flag_bytes = (size_t)((char*)(d.work + NWORK) - (char*)d.err);
    if (1024 + flag_bytes > 4096) return fail(ctx, GLT_E_INTERNAL, "flag words exceed the read-back buffer");
    std::vector<u64> res(res_bytes / 8);
    HIPCHK(hipMemcpyAsync(res.data(), d.gsum, res_bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 1024, d.err, flag_bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const u64* gs = res.data();
    const u64* parts = res.data() + ((u64*)d.gparts - (u64*)d.gsum);
    if (((int*)((char*)ctx->hbuf + 1024))[0] & ERR_CAP)
        return fail(ctx, GLT_E_INTERNAL, "an on-chip table bound of the wedge pass was exceeded");
    ctx->work[0] = (uint64_t)n;
    ctx->work[1] = (uint64_t)m;
    set_work(ctx, (const u64*)((char*)ctx->hbuf + 1024 + ((char*)d.work - (char*)d.err)), true);
    record_timing(ctx);
    rc = balance_summary(ctx, d.tstamp, st);
    if (rc) return rc;
    for (int64_t g = 0; g < B; g++) {
        i128 C[17];
        unpack_c(&parts[(size_t)g * 26], C);
        const i128 k4x3 = (i128)gs[(size_t)g * NSUMS + S_K4x3];
        if (k4x3 % 3 != 0) return fail(ctx, GLT_E_INTERNAL, "graph %lld: 4-clique total not divisible by 3", (long long)g);
        i128 X[18];
        std::string why;
        if (!globals(vb[g + 1] - vb[g], (sb[g + 1] - sb[g]) / 2, C, k4x3 / 3, (i128)gs[(size_t)g * NSUMS + S_NC4],
                     false, X, why))
            return fail(ctx, GLT_E_INTERNAL, "graph %lld: global combination failed: %s", (long long)g, why.c_str());
        store_x(X, out + g * 17);
    }
    return GLT_OK;
}

extern "C" {

const char* glt_version(void) { return GLT_VERSION; }

glt_status glt_create(int device, size_t hbm_budget_bytes, glt_ctx** out) {
    glt_ctx* ctx = nullptr;
    if (!out) return GLT_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GLT_E_INVALID_ARG;
    ctx = new (std::nothrow) glt_ctx();
    if (!ctx) return GLT_E_OOM;
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    // default schedule; the environment may change it within the same ranges as
    // glt_set_schedule (used by tests to force classes and range splitting on small graphs)
    ctx->wedge_wave_max = 128;   // (<= glt_wave_table() / 2; 128 measured best on the Chung-Lu graph)
    ctx->wedge_limit = glt_wedge_table() / 2;
    if (const char* e = getenv("GLT_WEDGE_WAVE_MAX")) {
        int v = atoi(e);
        if (v >= 0 && v <= glt_wave_table() / 2) ctx->wedge_wave_max = v;
    }
    ctx->wedge_mid_max = 2048;
    if (const char* e = getenv("GLT_WEDGE_MID_MAX")) {
        int v = atoi(e);
        if (v >= 0) ctx->wedge_mid_max = v;
    }
    ctx->wedge_wg_max = 1 << 30;   // bottoms move to the huge class when their tops overflow
    if (const char* e = getenv("GLT_WEDGE_WG_MAX")) {
        int v = atoi(e);
        if (v >= 0) ctx->wedge_wg_max = v;
    }
    if (const char* e = getenv("GLT_WEDGE_STREAM")) {
        const int v = atoi(e);
        ctx->wedge_stream = (v >= 0 && v <= 2) ? v : 0;
    }
    if (const char* e = getenv("GLT_WEDGE_RANGE_LIMIT")) {
        int v = atoi(e);
        if (v >= 1 && v < ctx->wedge_limit) ctx->wedge_limit = v;
    }
    if (const char* e = getenv("GLT_WIDE_DEGREE")) ctx->wide_degree = atoi(e) > 0 ? atoi(e) : 0;
    ctx->wedge_dense = glt_wedge_dense();
    if (const char* e = getenv("GLT_WEDGE_DENSE")) {
        int v = atoi(e);
        if (v >= 0 && v < ctx->wedge_dense) ctx->wedge_dense = v;
    }
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
        delete ctx;
        return GLT_E_DEVICE;
    }
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            ctx->num_cu = cus;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
            ctx->clock_khz = khz;
    }
    {
        // triangle records may take up to a quarter of the device's memory (0 disables them)
        size_t fr = 0, total = 0;
        if (hipMemGetInfo(&fr, &total) == hipSuccess) ctx->trec_cap = total / 4;
        if (const char* e = getenv("GLT_TRI_RECORD_BYTES")) ctx->trec_cap = (size_t)strtoull(e, nullptr, 10);
    }
    for (int i = 0; i < NEV; i++)
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) { glt_destroy(ctx); return GLT_E_DEVICE; }
    if (hipEventCreateWithFlags(&ctx->ev_null, hipEventDisableTiming) != hipSuccess) {
        glt_destroy(ctx);
        return GLT_E_DEVICE;
    }
    // the device's glt_count_noalloc workspace (device current); a failure here only
    // disables that entry point
    if (scratch_address(device, &ctx->scratch) != hipSuccess) {
        ctx->scratch = nullptr;
        (void)hipGetLastError();
    }
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess) {
        glt_destroy(ctx);
        return GLT_E_DEVICE;
    }
    if (hipHostMalloc((void**)&ctx->hbuf, 4096, hipHostMallocDefault) != hipSuccess) {
        glt_destroy(ctx);
        return GLT_E_DEVICE;
    }
    *out = ctx;
    return GLT_OK;
}

void glt_destroy(glt_ctx* ctx) {
    if (!ctx) return;
    for (glt_ctx*& p : ctx->part) {
        glt_destroy(p);
        p = nullptr;
    }
    (void)hipSetDevice(ctx->device);
    if (ctx->ev_part) (void)hipEventDestroy(ctx->ev_part);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->stage) (void)hipFree(ctx->stage);
    if (ctx->trec) (void)hipFree(ctx->trec);
    if (ctx->slab) (void)hipFree(ctx->slab);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    for (int i = 0; i < NEV; i++)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    if (ctx->ev_null) (void)hipEventDestroy(ctx->ev_null);
    if (ctx->hbuf) (void)hipHostFree(ctx->hbuf);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* glt_last_error(const glt_ctx* ctx) { return ctx ? ctx->err.c_str() : "null handle"; }

int glt_last_work(const glt_ctx* ctx, uint64_t* out, int cap) {
    if (!ctx || !out) return 0;
    const int k = cap < 4 + NWORK ? cap : 4 + NWORK;
    for (int i = 0; i < k; i++) out[i] = ctx->work[i];
    return k;
}

int glt_last_timing(const glt_ctx* ctx, float* ms, int cap) {
    if (!ctx || !ms) return 0;
    int k = cap < NSEG ? cap : NSEG;
    for (int i = 0; i < k; i++) ms[i] = ctx->timing[i];
    return k;
}

}  // extern "C"

namespace {

// One graph: glt_count, or with noalloc glt_count_noalloc (device inputs only, the
// workspace carved from the device's scratch array, no triangle records, no slab growth).
glt_status count_one(glt_ctx* ctx, const glt_csr* g, uint32_t flags, glt_u128 out_global[17],
                     uint64_t* out_per_edge, void* stream_, bool noalloc) {
    if (!ctx) return GLT_E_INVALID_ARG;
    ctx->err.clear();
    ctx->last_valid = false;
    if (!g || !out_global) return fail(ctx, GLT_E_INVALID_ARG, "null graph or output");
    const bool per_edge = (flags & GLT_PER_EDGE) != 0;
    if (flags & ~(uint32_t)(GLT_GLOBAL | GLT_PER_EDGE)) return fail(ctx, GLT_E_INVALID_ARG, "unknown flags");
    if (g->n < 0 || g->m < 0) return fail(ctx, GLT_E_INVALID_ARG, "negative size");
    if (g->n >= ((int64_t)1 << 31) || 2 * g->m >= ((int64_t)1 << 31))
        return fail(ctx, GLT_E_UNSUPPORTED, "n or 2m does not fit 31 bits");
    if (!g->row_ptr || (g->m > 0 && !g->col)) return fail(ctx, GLT_E_INVALID_ARG, "null row_ptr or col");
    if (per_edge && g->m > 0 && !out_per_edge) return fail(ctx, GLT_E_INVALID_ARG, "per-edge output missing");
    const int n = (int)g->n, m = (int)g->m;
    const int64_t S = 2 * (int64_t)m;
    const int rp64 = g->offsets_are_64bit ? 1 : 0;
    const bool host_in = !g->on_device;
    const bool host_out = per_edge && !g->on_device && m > 0;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = nullptr;
    glt_status rc = call_stream(ctx, stream_, st);
    if (rc) return rc;

    Dev d;
    Staging sg;
    const size_t need = carve(nullptr, n, m, rp64, host_in, host_out, 0, 0, d, sg);
    if (noalloc) {
        if (host_in) return fail(ctx, GLT_E_INVALID_ARG, "glt_count_noalloc takes device inputs only");
        if (!ctx->scratch) return fail(ctx, GLT_E_DEVICE, "no scratch address for device %d", ctx->device);
        if (need > GLT_SCRATCH_BYTES)
            return fail(ctx, GLT_E_UNSUPPORTED, "graph needs %zu bytes of workspace, the fixed scratch holds %zu",
                        need, (size_t)GLT_SCRATCH_BYTES);
        carve(ctx->scratch, n, m, rp64, false, false, 0, 0, d, sg);
    } else {
        rc = ensure_ws(ctx, need, st);
        if (rc) return rc;
        carve(ctx->ws, n, m, rp64, host_in, host_out, 0, 0, d, sg);
    }

    const void* rp = g->row_ptr;
    const int* col = g->col;
    if (host_in) {
        HIPCHK(hipMemcpyAsync(sg.rp, g->row_ptr, (size_t)(n + 1) * (rp64 ? 8 : 4), hipMemcpyHostToDevice, st));
        if (S > 0) HIPCHK(hipMemcpyAsync(sg.col, g->col, (size_t)S * 4, hipMemcpyHostToDevice, st));
        rp = sg.rp;
        col = sg.col;
    }
    u64* pe_dev = per_edge ? (host_out ? sg.out : (u64*)out_per_edge) : nullptr;
    // offsets must start at 0 and end at 2m: checked on the device with the rows (for n = 0
    // the single offset is checked here, from host memory when the input is there)
    if (n == 0 && S != 0) return fail(ctx, GLT_E_INVALID_ARG, "no vertices but 2m = %lld entries", (long long)S);
    if (n == 0 && host_in) {
        const int64_t r0 = rp64 ? ((const int64_t*)g->row_ptr)[0] : ((const int32_t*)g->row_ptr)[0];
        if (r0 != 0) return fail(ctx, GLT_E_INVALID_ARG, "row_ptr[0] = %lld, expected 0", (long long)r0);
    }
    rc = run_pipeline(ctx, d, rp, rp64, col, per_edge, pe_dev, st, noalloc);
    if (rc) return rc;
    if (host_out)
        HIPCHK(hipMemcpyAsync(out_per_edge, sg.out, (size_t)13 * m * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->hbuf, d.final_sums, sizeof(u64) * 2 * 13, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 512, d.gsum, sizeof(u64) * NSUMS, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 1024, d.err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((char*)ctx->hbuf + 1032, d.work, NWORK * sizeof(u64), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (((int*)((char*)ctx->hbuf + 1024))[0] & ERR_NEG)
        return fail(ctx, GLT_E_INTERNAL, "a per-edge count came out negative");
    if (((int*)((char*)ctx->hbuf + 1024))[0] & ERR_CAP)
        return fail(ctx, GLT_E_INTERNAL, "an on-chip table bound of the wedge pass was exceeded");
    ctx->work[0] = (uint64_t)n;
    ctx->work[1] = (uint64_t)m;
    set_work(ctx, (const u64*)((char*)ctx->hbuf + 1032), n > 0);
    record_timing(ctx);
    rc = balance_summary(ctx, d.tstamp, st);
    if (rc) return rc;
    i128 C[17];
    unpack_c(ctx->hbuf, C);
    const u64* gs = (const u64*)((char*)ctx->hbuf + 512);
    const i128 k4x3 = (i128)gs[S_K4x3];
    if (k4x3 % 3 != 0) return fail(ctx, GLT_E_INTERNAL, "4-clique total not divisible by 3");
    i128 X[18];
    std::string why;
    if (!globals(n, m, C, k4x3 / 3, (i128)gs[S_NC4], per_edge, X, why))
        return fail(ctx, GLT_E_INTERNAL, "global combination failed: %s", why.c_str());
    store_x(X, out_global);
    ctx->last = d;
    ctx->last_valid = !noalloc;
    ctx->last_cycles4 = gs[S_NC4];
    return GLT_OK;
}

}  // namespace

bool glt_last_graph(const glt_ctx* ctx, Dev* d, uint64_t* cycles4) {
    if (!ctx || !ctx->last_valid) return false;
    *d = ctx->last;
    *cycles4 = ctx->last_cycles4;
    return true;
}

int glt_ctx_device(const glt_ctx* ctx) { return ctx->device; }

extern "C" {

glt_status glt_count(glt_ctx* ctx, const glt_csr* g, uint32_t flags, glt_u128 out_global[17],
                     uint64_t* out_per_edge, void* stream) {
    return count_one(ctx, g, flags, out_global, out_per_edge, stream, false);
}

glt_status glt_count_noalloc(glt_ctx* ctx, const glt_csr* g, uint32_t flags, glt_u128 out_global[17],
                             uint64_t* out_per_edge, void* stream) {
    return count_one(ctx, g, flags, out_global, out_per_edge, stream, true);
}

// A large batch as GLT_BATCH_PARTS parts (graph g in part g mod K, in order), each counted by
// a helper handle on its own stream and host thread, all at the same time: one part's
// preprocessing (bound by scattered loads) overlaps the others' counting passes (bound by
// instruction issue).  Every graph's counts are those of the whole batch's call.  The
// handle's work counters become the parts' sums (maxima for the per-class maxima and the
// balance entries), its kernel-group times the longest part's.
static glt_status run_batch_parts(glt_ctx* ctx, int64_t B, const int64_t* vb, const int64_t* sb,
                                  const int* const* rps, const int* const* cols, glt_u128* out, hipStream_t st) {
    constexpr int K = GLT_BATCH_PARTS;
    for (glt_ctx*& p : ctx->part)
        if (!p) {
            const glt_status rc = glt_create(ctx->device, 0, &p);
            if (rc) return fail(ctx, rc, "creating a helper handle for the batch parts failed");
        }
    if (!ctx->ev_part) HIPCHK(hipEventCreateWithFlags(&ctx->ev_part, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ctx->ev_part, st));
    std::vector<int64_t> pv[K], ps[K];
    std::vector<const int*> pr[K], pc[K];
    std::vector<glt_u128> po[K];
    for (int k = 0; k < K; k++) { pv[k].assign(1, 0); ps[k].assign(1, 0); }
    for (int64_t g = 0; g < B; g++) {
        const int k = (int)(g % K);
        pv[k].push_back(pv[k].back() + (vb[g + 1] - vb[g]));
        ps[k].push_back(ps[k].back() + (sb[g + 1] - sb[g]));
        pr[k].push_back(rps[g]);
        pc[k].push_back(cols[g]);
    }
    glt_status rc[K];
    std::vector<std::thread> th;
    for (int k = 0; k < K; k++) {
        glt_ctx* p = ctx->part[k];
        p->wedge_wave_max = ctx->wedge_wave_max;
        p->wedge_mid_max = ctx->wedge_mid_max;
        p->wedge_wg_max = ctx->wedge_wg_max;
        p->wedge_limit = ctx->wedge_limit;
        p->wedge_dense = ctx->wedge_dense;
        p->tri_records = ctx->tri_records;
        p->wedge_stream = ctx->wedge_stream;
        p->list_order = ctx->list_order;
        p->record_balance = ctx->record_balance;
        p->wide_degree = ctx->wide_degree;
        HIPCHK(hipStreamWaitEvent(p->stream, ctx->ev_part, 0));
        po[k].assign(pr[k].size() * 17, glt_u128{0, 0});
        rc[k] = GLT_OK;
    }
    for (int k = 0; k < K; k++)
        th.emplace_back([&, k] {
            glt_ctx* p = ctx->part[k];
            const int64_t Bk = (int64_t)pr[k].size();
            rc[k] = Bk > 0 ? glt_run_batch_ptrs(p, Bk, pv[k].data(), ps[k].data(), pr[k].data(), pc[k].data(),
                                               po[k].data(), p->stream)
                           : GLT_OK;
        });
    for (std::thread& t : th) t.join();
    for (int k = 0; k < K; k++)
        if (rc[k]) return fail(ctx, rc[k], "%s", ctx->part[k]->err.c_str());
    for (int64_t g = 0; g < B; g++) memcpy(&out[(size_t)g * 17], &po[g % K][(size_t)(g / K) * 17], 17 * sizeof(glt_u128));
    ctx->work[0] = (uint64_t)vb[B];
    ctx->work[1] = (uint64_t)(sb[B] / 2);
    for (int i = 2; i < 2 + NWORK + 2; i++) {
        uint64_t v = 0;
        const bool maxed = i >= 10;   // the balance entries and the per-class maxima
        for (int k = 0; k < K; k++) v = maxed ? std::max(v, ctx->part[k]->work[i]) : v + ctx->part[k]->work[i];
        ctx->work[i] = v;
    }
    for (int i = 0; i < NSEG; i++) {
        float t = 0.f;
        for (int k = 0; k < K; k++) t = std::max(t, ctx->part[k]->timing[i]);
        ctx->timing[i] = t;
    }
    ctx->last_mode = ctx->part[0]->last_mode;
    return GLT_OK;
}

glt_status glt_count_batch(glt_ctx* ctx, const glt_batch* b, uint32_t flags, glt_u128* out, void* stream_) {
    if (!ctx) return GLT_E_INVALID_ARG;
    ctx->err.clear();
    if (!b || (b->num_graphs > 0 && (!out || !b->vtx_base || !b->slot_base)))
        return fail(ctx, GLT_E_INVALID_ARG, "null batch, bases or output");
    if (flags & ~(uint32_t)GLT_GLOBAL)
        return fail(ctx, GLT_E_INVALID_ARG, "batched counting supports GLT_GLOBAL only");
    const int64_t B = b->num_graphs;
    if (B < 0 || B >= ((int64_t)1 << 31)) return fail(ctx, GLT_E_INVALID_ARG, "bad number of graphs");
    if (B == 0) return GLT_OK;
    const int64_t* vb = b->vtx_base;
    const int64_t* sb = b->slot_base;
    if (vb[0] != 0 || sb[0] != 0) return fail(ctx, GLT_E_INVALID_ARG, "bases must start at 0");
    for (int64_t g = 0; g < B; g++)
        if (vb[g + 1] < vb[g] || sb[g + 1] < sb[g])
            return fail(ctx, GLT_E_INVALID_ARG, "graph %lld: bases not monotone", (long long)g);
    const int64_t N = vb[B], S = sb[B];
    if (N >= ((int64_t)1 << 31) || S >= ((int64_t)1 << 31))
        return fail(ctx, GLT_E_UNSUPPORTED, "packed vertices or slots do not fit 31 bits");
    if (!b->row_ptr || (S > 0 && !b->col)) return fail(ctx, GLT_E_INVALID_ARG, "null row_ptr or col");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = nullptr;
    glt_status rc0 = call_stream(ctx, stream_, st);
    if (rc0) return rc0;
    const int* rp = b->row_ptr;
    const int* col = b->col;
    if (!b->on_device) {
        const size_t need = (size_t)(N + B) * 4 + (size_t)S * 4 + 512;
        if (need > ctx->stage_bytes) {
            HIPCHK(hipStreamSynchronize(st));
            if (ctx->stage) { (void)hipFree(ctx->stage); ctx->stage = nullptr; ctx->stage_bytes = 0; }
            if (hipMalloc(&ctx->stage, need) != hipSuccess) {
                ctx->stage = nullptr;
                (void)hipGetLastError();
                return fail(ctx, GLT_E_OOM, "hipMalloc of %zu staging bytes failed", need);
            }
            ctx->stage_bytes = need;
        }
        int* drp = (int*)ctx->stage;
        int* dcol = drp + ((N + B + 63) / 64) * 64;
        HIPCHK(hipMemcpyAsync(drp, b->row_ptr, (size_t)(N + B) * 4, hipMemcpyHostToDevice, st));
        if (S > 0) HIPCHK(hipMemcpyAsync(dcol, b->col, (size_t)S * 4, hipMemcpyHostToDevice, st));
        rp = drp;
        col = dcol;
    }
    std::vector<const int*> rps((size_t)B), cols((size_t)B);
    for (int64_t g = 0; g < B; g++) {
        rps[(size_t)g] = rp + vb[g] + g;
        cols[(size_t)g] = col + sb[g];
    }
    ctx->last_valid = false;
    if (B >= GLT_BATCH_SPLIT_GRAPHS && S >= GLT_BATCH_SPLIT_SLOTS && ctx->budget == 0)
        return run_batch_parts(ctx, B, vb, sb, rps.data(), cols.data(), out, st);
    return glt_run_batch_ptrs(ctx, B, vb, sb, rps.data(), cols.data(), out, st);
}

}  // extern "C"

glt_status glt_get_schedule(const glt_ctx* ctx, glt_schedule* out) {
    if (!ctx || !out) return GLT_E_INVALID_ARG;
    memset(out, 0, sizeof(*out));
    out->wedge_wave_max = ctx->wedge_wave_max;
    out->wedge_mid_max = ctx->wedge_mid_max;
    out->wedge_wg_max = ctx->wedge_wg_max;
    out->wedge_stream = ctx->wedge_stream;
    out->list_order = ctx->list_order;
    out->wedge_dense = ctx->wedge_dense;
    out->wedge_range_limit = ctx->wedge_limit;
    out->tri_records = ctx->tri_records;
    out->record_balance = ctx->record_balance;
    return GLT_OK;
}

glt_status glt_set_schedule(glt_ctx* ctx, const glt_schedule* s) {
    if (!ctx) return GLT_E_INVALID_ARG;
    ctx->err.clear();
    if (!s) return fail(ctx, GLT_E_INVALID_ARG, "null schedule");
    if (s->wedge_wave_max < 0 || s->wedge_wave_max > glt_wave_table() / 2)
        return fail(ctx, GLT_E_INVALID_ARG, "wedge_wave_max must be in [0, %d]", glt_wave_table() / 2);
    if (s->wedge_mid_max < 0) return fail(ctx, GLT_E_INVALID_ARG, "wedge_mid_max must be >= 0");
    if (s->wedge_wg_max < 0) return fail(ctx, GLT_E_INVALID_ARG, "wedge_wg_max must be >= 0");
    if (s->wedge_dense < 0 || s->wedge_dense > glt_wedge_dense())
        return fail(ctx, GLT_E_INVALID_ARG, "wedge_dense must be in [0, %d]", glt_wedge_dense());
    if (s->wedge_range_limit < 1 || s->wedge_range_limit > glt_wedge_table() / 2)
        return fail(ctx, GLT_E_INVALID_ARG, "wedge_range_limit must be in [1, %d]", glt_wedge_table() / 2);
    if (s->tri_records != 0 && s->tri_records != 1) return fail(ctx, GLT_E_INVALID_ARG, "tri_records must be 0 or 1");
    if (s->wedge_stream < -1 || s->wedge_stream > 2)
        return fail(ctx, GLT_E_INVALID_ARG, "wedge_stream must be -1 (automatic), 0, 1 or 2");
    if (s->record_balance != 0 && s->record_balance != 1)
        return fail(ctx, GLT_E_INVALID_ARG, "record_balance must be 0 or 1");
    if (s->list_order < -1 || s->list_order >= LO_N)
        return fail(ctx, GLT_E_INVALID_ARG, "list_order must be -1 (automatic) or in [0, %d]", LO_N - 1);
    ctx->wedge_wave_max = s->wedge_wave_max;
    ctx->wedge_mid_max = s->wedge_mid_max;
    ctx->wedge_wg_max = s->wedge_wg_max;
    ctx->wedge_dense = s->wedge_dense;
    ctx->wedge_limit = s->wedge_range_limit;
    ctx->tri_records = s->tri_records;
    ctx->wedge_stream = s->wedge_stream;
    ctx->list_order = s->list_order;
    ctx->record_balance = s->record_balance;
    return GLT_OK;
}

glt_status glt_autotune_batch(glt_ctx* ctx, const glt_batch* b, glt_schedule* best, float* best_ms, void* stream) {
    if (!ctx) return GLT_E_INVALID_ARG;
    ctx->err.clear();
    if (!b || !best) return fail(ctx, GLT_E_INVALID_ARG, "null batch or output");
    const int64_t B = b->num_graphs;
    if (B <= 0) return fail(ctx, GLT_E_INVALID_ARG, "empty batch");
    glt_schedule base;
    glt_get_schedule(ctx, &base);
    std::vector<glt_u128> ref((size_t)B * 17), got((size_t)B * 17);
    glt_status rc = glt_count_batch(ctx, b, GLT_GLOBAL, ref.data(), stream);   // warm-up, reference counts
    if (rc) return rc;
    // candidate grid: wedge class bounds x dense window x stream mode
    static const int wave_c[2] = {128, 256};
    static const int mid_c[3] = {1024, 2048, 4096};
    static const int dense_c[2] = {4096, 16384};
    glt_schedule win = base;
    float win_ms = -1.f;
    for (int a = 0; a < 2; a++)
        for (int c = 0; c < 3; c++)
            for (int e = 0; e < 6; e++) {
                glt_schedule cand = base;
                cand.wedge_wave_max = wave_c[a];
                cand.wedge_mid_max = mid_c[c];
                cand.wedge_dense = dense_c[e & 1];
                cand.wedge_stream = e >> 1;
                rc = glt_set_schedule(ctx, &cand);
                if (rc) { glt_set_schedule(ctx, &base); return rc; }
                rc = glt_count_batch(ctx, b, GLT_GLOBAL, got.data(), stream);
                if (rc) { glt_set_schedule(ctx, &base); return rc; }
                if (memcmp(got.data(), ref.data(), got.size() * sizeof(glt_u128)) != 0) {
                    glt_set_schedule(ctx, &base);
                    return fail(ctx, GLT_E_INTERNAL, "schedule (%d, %d, %d, %d) changed the counts", wave_c[a], mid_c[c],
                                dense_c[e & 1], e >> 1);
                }
                const float ms = ctx->timing[NSEG - 1];   // the whole call
                if (win_ms < 0 || ms < win_ms) { win_ms = ms; win = cand; }
            }
    glt_set_schedule(ctx, &win);
    *best = win;
    if (best_ms) *best_ms = win_ms;
    return GLT_OK;
}
