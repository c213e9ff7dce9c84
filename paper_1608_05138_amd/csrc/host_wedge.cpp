// host_wedge.cpp -- the 4-cycle (wedge) pass on host threads: the CPU side of the paper's
// hybrid scheme (Section 4.3, "Hybrid CPU-GPU": CPU workers take edges from the front of the
// ordered job queue in chunks, GPUs from the back; Section 4.4, work stealing), built to
// measure what such a worker achieves on this machine's host beside the device.  It works on
// the relabelled, oriented graph of the handle's last single-graph call, which lives in
// device memory: the copies it needs are timed apart from the counting.
//
// For every bottom vertex y (taken in rank order, a chunk of bottoms at a time, by however
// many threads are free) and every wedge y - w - x with x ranked above y, the count sweep
// counts c(y, x) in a dense per-thread array, the credit sweep credits c(y, x) - 1 to the
// edges (w, x) and (y, w), and the 4-cycles with lowest vertex y and opposite vertex x number
// C(c(y, x), 2) -- the same decomposition as the device's wedge pass, in plain loops.
#include <hip/hip_runtime.h>
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "../../include/glt.h"
#include "glt_internal.h"

namespace {

struct HostGraph {
    int n = 0, m = 0, S = 0;
    int* nrp = nullptr;    // [n + 1] relabelled CSR offsets
    int2* wb = nullptr;    // [S] oriented range of the tops of slot s's wedges
    int* ocol = nullptr;   // [m] oriented columns
    int* s2k = nullptr;    // [S] slot -> oriented edge index
};

void free_host(HostGraph& h) {
    if (h.nrp) (void)hipHostFree(h.nrp);
    if (h.wb) (void)hipHostFree(h.wb);
    if (h.ocol) (void)hipHostFree(h.ocol);
    if (h.s2k) (void)hipHostFree(h.s2k);
    h = HostGraph();
}

constexpr int kChunk = 16;   // bottoms a thread takes at a time

struct Totals {
    uint64_t wedges = 0, cycles = 0;
};

void worker(const HostGraph& h, std::atomic<int>& next, uint64_t* P, Totals& out) {
    std::vector<uint32_t> cnt((size_t)h.n, 0);
    std::vector<int> touched;
    Totals t;
    while (true) {
        const int y0 = next.fetch_add(kChunk, std::memory_order_relaxed);
        if (y0 >= h.n) break;
        const int y1 = std::min(h.n, y0 + kChunk);
        for (int y = y0; y < y1; y++) {
            const int rb = h.nrp[y], re = h.nrp[y + 1];
            for (int s = rb; s < re; s++)
                for (int k = h.wb[s].x; k < h.wb[s].y; k++) {
                    const int x = h.ocol[k];
                    if (cnt[x]++ == 0) touched.push_back(x);
                }
            for (int s = rb; s < re; s++) {
                uint64_t sum = 0;
                for (int k = h.wb[s].x; k < h.wb[s].y; k++) {
                    const uint64_t c = cnt[h.ocol[k]] - 1;
                    if (c) __atomic_fetch_add(&P[k], c, __ATOMIC_RELAXED);   // top edge (w, x)
                    sum += c;
                }
                t.wedges += (uint64_t)(h.wb[s].y - h.wb[s].x);
                if (sum) __atomic_fetch_add(&P[h.s2k[s]], sum, __ATOMIC_RELAXED);   // bottom edge (y, w)
            }
            for (const int x : touched) {
                const uint64_t c = cnt[x];
                t.cycles += c * (c - 1) / 2;
                cnt[x] = 0;
            }
            touched.clear();
        }
    }
    out = t;
}

}  // namespace

extern "C" glt_status glt_host_wedges(glt_ctx* ctx, int threads, glt_host_wedge_report* r) {
    if (!ctx || !r) return GLT_E_INVALID_ARG;
    Dev d;
    uint64_t gpu_cycles = 0;
    if (!glt_last_graph(ctx, &d, &gpu_cycles)) return GLT_E_INVALID_ARG;
    if (threads <= 0) {   // the threads this process may run on
        cpu_set_t set;
        CPU_ZERO(&set);
        threads = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set) : 0;
        if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    }
    *r = glt_host_wedge_report();
    HostGraph h;
    h.n = d.n;
    h.m = d.m;
    h.S = d.S;
    if (hipSetDevice(glt_ctx_device(ctx)) != hipSuccess) return GLT_E_DEVICE;
    if (hipHostMalloc((void**)&h.nrp, (size_t)(h.n + 1) * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h.wb, (size_t)std::max(h.S, 1) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h.ocol, (size_t)std::max(h.m, 1) * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h.s2k, (size_t)std::max(h.S, 1) * 4, hipHostMallocDefault) != hipSuccess) {
        free_host(h);
        return GLT_E_OOM;
    }
    std::vector<uint64_t> P((size_t)h.m, 0);
    // the device arrays the host side reads, copied once (the part of a hybrid step that
    // moves the relabelled graph to the host)
    const auto c0 = std::chrono::steady_clock::now();
    bool ok = hipDeviceSynchronize() == hipSuccess &&
              hipMemcpy(h.nrp, d.nrp, (size_t)(h.n + 1) * 4, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok && h.S > 0)
        ok = hipMemcpy(h.wb, d.wb, (size_t)h.S * 8, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(h.s2k, d.s2k, (size_t)h.S * 4, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(h.ocol, d.ocol, (size_t)h.m * 4, hipMemcpyDeviceToHost) == hipSuccess;
    const auto c1 = std::chrono::steady_clock::now();
    if (!ok) {
        free_host(h);
        return GLT_E_DEVICE;
    }
    std::atomic<int> next(0);
    std::vector<Totals> tot((size_t)threads);
    std::vector<std::thread> pool;
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < threads; i++) pool.emplace_back(worker, std::cref(h), std::ref(next), P.data(), std::ref(tot[i]));
    for (auto& th : pool) th.join();
    const auto t1 = std::chrono::steady_clock::now();
    for (const Totals& t : tot) {
        r->wedges += t.wedges;
        r->cycles4 += t.cycles;
    }
    uint64_t psum = 0;
    for (const uint64_t v : P) psum += v;
    r->credit_sum = psum;
    r->gpu_cycles4 = gpu_cycles;
    r->threads = threads;
    r->bytes_copied = (uint64_t)(h.n + 1) * 4 + (uint64_t)h.S * 12 + (uint64_t)h.m * 4;
    r->copy_ms = std::chrono::duration<double, std::milli>(c1 - c0).count();
    r->count_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    free_host(h);
    return GLT_OK;
}
