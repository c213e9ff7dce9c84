// Stand-ins for the HIP runtime and for the library's counting calls that the request
// server uses (see hip/hip_runtime.h here).  The stub "count" of a packed batch returns, per
// graph, X1 = m, X2 = n, X3 = sum of its column entries and X4 = its first column entry, so
// the test can check that every result belongs to its own request; a graph whose first
// column entry is -7 is "invalid" (the batch fails with GLT_E_NOT_SYMMETRIC, as a failed
// validation does).  Each batch sleeps in proportion to its edges, so admission and compute
// overlap as on a device.
#include <atomic>
#include <chrono>
#include <mutex>
#include <stdlib.h>
#include <string.h>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
#include "../../include/glt.h"

struct stub_event { std::atomic<int> recorded{0}; std::atomic<int> bad{0}; };
struct stub_stream { int unused = 0; };

static std::atomic<int64_t> g_copies{0};
static std::atomic<int64_t> g_fail_copy{-1};   // index of the copy whose event reports an error
static std::atomic<int64_t> g_batches{0};
static std::atomic<int64_t> g_max_batch{0};
static std::atomic<int64_t> g_ns_per_edge{20};

extern "C" {
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) { *p = malloc(n ? n : 1); return *p ? hipSuccess : hipErrorUnknown; }
hipError_t hipFree(void* p) { free(p); return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new stub_stream(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new stub_event(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
// the server records one event per request, after its copy: the chosen copy's event reports
// an error when queried
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    const int64_t idx = g_copies++;
    e->bad = (idx == g_fail_copy) ? 1 : 0;
    e->recorded = 1;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    if (e->bad) return hipErrorUnknown;
    return e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return hipEventQuery(e); }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, int, hipStream_t) {
    memcpy(dst, src, n);
    return hipSuccess;
}

glt_status glt_create(int, size_t, glt_ctx** out) { *out = (glt_ctx*)new int(0); return GLT_OK; }
void glt_destroy(glt_ctx* c) { delete (int*)c; }

void stub_configure(int64_t fail_copy, int64_t ns_per_edge) {
    g_fail_copy = fail_copy;
    g_ns_per_edge = ns_per_edge;
    g_copies = 0;
    g_batches = 0;
    g_max_batch = 0;
}
int64_t stub_batches(void) { return g_batches; }
int64_t stub_max_batch(void) { return g_max_batch; }
}

glt_status glt_run_batch_ptrs(glt_ctx*, int64_t B, const int64_t* vb, const int64_t* sb,
                              const int* const* rp_ptrs, const int* const* col_ptrs, glt_u128* out, hipStream_t) {
    g_batches++;
    int64_t mb = g_max_batch.load();
    while (B > mb && !g_max_batch.compare_exchange_weak(mb, B)) {}
    int64_t edges = 0;
    for (int64_t g = 0; g < B; g++) {
        const int64_t n = vb[g + 1] - vb[g], S = sb[g + 1] - sb[g];
        edges += S / 2;
        if (rp_ptrs[g][0] != 0 || rp_ptrs[g][n] != S) return GLT_E_INVALID_ARG;
        if (S > 0 && col_ptrs[g][0] == -7) return GLT_E_NOT_SYMMETRIC;
        int64_t sum = 0;
        for (int64_t j = 0; j < S; j++) sum += col_ptrs[g][j];
        memset(out + 17 * g, 0, sizeof(glt_u128) * 17);
        out[17 * g + 0].lo = (uint64_t)(S / 2);
        out[17 * g + 1].lo = (uint64_t)n;
        out[17 * g + 2].lo = (uint64_t)sum;
        out[17 * g + 3].lo = S > 0 ? (uint64_t)(int64_t)col_ptrs[g][0] : 0;
    }
    std::this_thread::sleep_for(std::chrono::nanoseconds(edges * g_ns_per_edge.load()));
    return GLT_OK;
}
