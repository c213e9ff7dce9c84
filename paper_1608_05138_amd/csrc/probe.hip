// probe.hip -- calibration kernels for the roofline of the counting passes: the device's
// rate of global atomic adds in the access patterns the passes issue (runs of consecutive
// words per wavefront, as the per-edge credits to one vertex's out-edges; single scattered
// words, as credits to unrelated edges) and a read-only stream (a second calibration point
// of the traffic counters besides a copy).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/glt.h"

namespace {

// 32-bit mix of a counter (Murmur3's finaliser); only spreads addresses, any mixing works.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

constexpr int kThreads = 256;
constexpr int kRounds = 64;   // atomics per lane per launch

// Each wavefront adds 1 to a run of 64 consecutive words starting at a pseudo-random
// multiple of 64, kRounds times.  lines = words / 64 (every run is in bounds).
template <typename W>
__global__ __launch_bounds__(kThreads) void k_probe_runs(W* __restrict__ a, uint32_t lines) {
    const uint32_t wave = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    for (int r = 0; r < kRounds; r++) {
        const uint32_t line = mix32(wave * kRounds + r) % lines;
        atomicAdd(a + (size_t)line * 64 + lane, (W)1);
    }
}

// Each lane adds 1 to a pseudo-random word, kRounds times.
template <typename W>
__global__ __launch_bounds__(kThreads) void k_probe_scatter(W* __restrict__ a, uint32_t words) {
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    for (int r = 0; r < kRounds; r++) atomicAdd(a + mix32(t * kRounds + r) % words, (W)1);
}

// Reads words [0, n16 * 4) once in 16-byte loads (grid-stride) and writes one sum per block.
__global__ __launch_bounds__(kThreads) void k_probe_read(const uint4* __restrict__ a, size_t n16,
                                                         uint32_t* __restrict__ out) {
    uint32_t s = 0;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += (size_t)gridDim.x * kThreads) {
        const uint4 v = a[i];
        s += v.x ^ v.y ^ v.z ^ v.w;
    }
    __shared__ uint32_t red[kThreads];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int d = kThreads / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

extern "C" glt_status glt_probe(int device, int kind, size_t bytes, int reps, float* ms, uint64_t* ops) {
    if (!ms || !ops || reps < 1 || kind < 0 || kind > 4) return GLT_E_INVALID_ARG;
    const size_t words = bytes / 4;              // 32-bit words
    const size_t words64 = bytes / 8;            // 64-bit words (kinds 3, 4)
    if (words < 64 * 64 || words > ((size_t)1 << 32) - 64) return GLT_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return GLT_E_INVALID_ARG;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    uint32_t* a = nullptr;
    uint32_t* out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    glt_status rc = GLT_OK;
    const unsigned grid = (unsigned)cus * 32;   // 8192 workgroups of 256 lanes on 256 CUs
    if (hipMalloc(&a, words * 4) != hipSuccess || hipMalloc(&out, (size_t)grid * 4) != hipSuccess) {
        (void)hipGetLastError();
        rc = GLT_E_OOM;
        goto done;
    }
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(a, 0, words * 4, st) != hipSuccess) {
        rc = GLT_E_DEVICE;
        goto done;
    }
    for (int it = 0; it <= reps; it++) {   // launch 0 warms up, launches 1..reps are timed
        if (it == 1 && hipEventRecord(e0, st) != hipSuccess) { rc = GLT_E_DEVICE; goto done; }
        if (kind == 0)
            hipLaunchKernelGGL(k_probe_runs<uint32_t>, dim3(grid), dim3(kThreads), 0, st, a, (uint32_t)(words / 64));
        else if (kind == 1)
            hipLaunchKernelGGL(k_probe_scatter<uint32_t>, dim3(grid), dim3(kThreads), 0, st, a, (uint32_t)words);
        else if (kind == 2)
            hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(kThreads), 0, st, (const uint4*)a, words / 4, out);
        else if (kind == 3)
            hipLaunchKernelGGL(k_probe_runs<unsigned long long>, dim3(grid), dim3(kThreads), 0, st,
                               (unsigned long long*)a, (uint32_t)(words64 / 64));
        else
            hipLaunchKernelGGL(k_probe_scatter<unsigned long long>, dim3(grid), dim3(kThreads), 0, st,
                               (unsigned long long*)a, (uint32_t)words64);
    }
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipGetLastError() != hipSuccess) {
        rc = GLT_E_DEVICE;
        goto done;
    }
    {
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t / (float)reps;
        *ops = kind == 2 ? (uint64_t)(words / 4) * 16 : (uint64_t)grid * kThreads * kRounds;
    }
done:
    if (st) (void)hipStreamSynchronize(st);
    if (a) (void)hipFree(a);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    return rc;
}
