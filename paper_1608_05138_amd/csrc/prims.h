// prims.h -- device primitives for gfx950 (wave64): wave scans and segmented sums by DPP,
// block scans and reductions, a device-wide exclusive scan, a stable LSD radix sort of
// (u64 key, u32 value) pairs, and fill kernels.  Used by the graph preprocessing (degree
// order, sorted CSR) and the counting passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned long long u64;
typedef unsigned int u32;

#define GLT_WAVE 64

__device__ __forceinline__ int glt_lane() { return (int)__lane_id(); }

// Orders LDS accesses of one wavefront: writes before the call are visible to every lane
// of the same wavefront after it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves by DPP (GFX9 data-parallel primitives; no LDS traffic).  Lanes whose
// source is outside the row (row_shr), in a row not named by the row mask (row_bcast), or
// off the wave's ends (wave_shr / wave_shl) read 0.  Every lane of the wave must be active.
#define GLT_DPP_ROW_SHR(n) (0x110 + (n))
#define GLT_DPP_ROW_BCAST15 0x142
#define GLT_DPP_ROW_BCAST31 0x143
#define GLT_DPP_WAVE_SHL1 0x130
#define GLT_DPP_WAVE_SHR1 0x138
template <int CTRL, int ROWM, bool BC>
__device__ __forceinline__ u32 dpp_u32(u32 v) {
    return (u32)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWM, 0xf, BC);
}
template <typename T, int CTRL, int ROWM, bool BC>
__device__ __forceinline__ T dpp_move(T v) {
    if constexpr (sizeof(T) == 8) {
        const u32 lo = dpp_u32<CTRL, ROWM, BC>((u32)(u64)v);
        const u32 hi = dpp_u32<CTRL, ROWM, BC>((u32)((u64)v >> 32));
        return (T)(((u64)hi << 32) | lo);
    } else {
        return (T)dpp_u32<CTRL, ROWM, BC>((u32)v);
    }
}
// Inclusive sum over the lanes of a wavefront (every lane active): shifts by 1, 2, 4, 8
// inside rows of 16 lanes, then the last lane of row 0 / row 2 into rows 1 / 3 and of row 1
// into rows 2 and 3.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    v += dpp_move<T, GLT_DPP_ROW_SHR(1), 0xf, true>(v);
    v += dpp_move<T, GLT_DPP_ROW_SHR(2), 0xf, true>(v);
    v += dpp_move<T, GLT_DPP_ROW_SHR(4), 0xf, true>(v);
    v += dpp_move<T, GLT_DPP_ROW_SHR(8), 0xf, true>(v);
    v += dpp_move<T, GLT_DPP_ROW_BCAST15, 0xa, false>(v);
    v += dpp_move<T, GLT_DPP_ROW_BCAST31, 0xc, false>(v);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = GLT_WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, GLT_WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int d = GLT_WAVE / 2; d >= 1; d >>= 1) {
        T o = __shfl_xor(v, d, GLT_WAVE);
        v = o > v ? o : v;
    }
    return v;
}

// one step of the segmented scan: (v, f) := (v_src, f_src) (+) (v, f), where
// (a, fa) (+) (b, fb) = (fb ? b : a + b, fa | fb)
template <typename T, int CTRL, int ROWM, bool BC>
__device__ __forceinline__ void seg_step(T& v, u32& f) {
    const T o = dpp_move<T, CTRL, ROWM, BC>(v);
    const u32 of = dpp_u32<CTRL, ROWM, BC>(f);
    if (!f) v += o;
    f |= of;
}
// Segmented inclusive sum over the lanes of a wavefront (the moves of wave_incl_scan):
// `start` marks the first lane of a segment (lane 0 always begins one).
template <typename T>
__device__ __forceinline__ T wave_seg_sum(T v, bool start) {
    u32 f = start ? 1u : 0u;
    seg_step<T, GLT_DPP_ROW_SHR(1), 0xf, true>(v, f);
    seg_step<T, GLT_DPP_ROW_SHR(2), 0xf, true>(v, f);
    seg_step<T, GLT_DPP_ROW_SHR(4), 0xf, true>(v, f);
    seg_step<T, GLT_DPP_ROW_SHR(8), 0xf, true>(v, f);
    seg_step<T, GLT_DPP_ROW_BCAST15, 0xa, false>(v, f);
    seg_step<T, GLT_DPP_ROW_BCAST31, 0xc, false>(v, f);
    return v;
}

// Segmented sum over maximal runs of equal consecutive keys in a wavefront (a key may recur
// in separate runs; each run is summed on its own).  is_last marks the last lane of each
// run, which holds the run's total.  Every lane must call it (idle lanes: a sentinel key).
template <typename T>
__device__ __forceinline__ T seg_run_sum_last(T v, int key, bool& is_last) {
    const int l = glt_lane();
    const int kp = (int)dpp_u32<GLT_DPP_WAVE_SHR1, 0xf, true>((u32)key);
    const int kn = (int)dpp_u32<GLT_DPP_WAVE_SHL1, 0xf, true>((u32)key);
    is_last = (l == GLT_WAVE - 1) || (kn != key);
    return wave_seg_sum(v, l == 0 || kp != key);
}

// The same for keys that are non-decreasing in lane order.
template <typename T>
__device__ __forceinline__ T seg_sum_last(T v, int key, bool& is_last) {
    return seg_run_sum_last(v, key, is_last);
}

// Exclusive scan over a block of BLOCK threads.  lds must hold BLOCK/64 elements.  All
// threads of the block must call it (contains __syncthreads).
template <typename T, int BLOCK>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T& total) {
    const int l = glt_lane(), w = threadIdx.x / GLT_WAVE;
    T inc = wave_incl_scan(v);
    if (l == GLT_WAVE - 1) lds[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / GLT_WAVE; i++) {
        T s = lds[i];
        if (i < w) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// first index in [lo, hi) with a[idx] >= x (hi if none)
__device__ __forceinline__ int lower_bound_i32(const int* a, int lo, int hi, int x) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <typename T>
static inline void launch_fill(T* p, int64_t n, T v, hipStream_t st) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

// ---------------------------------------------------------------------------------------
// device-wide exclusive scan (tile = 256 threads x 16 items)
// ---------------------------------------------------------------------------------------
#define SCAN_THREADS 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_THREADS * SCAN_ITEMS)

template <typename Tin, typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_sums(const Tin* in, int64_t n, T* sums) {
    __shared__ T lds[SCAN_THREADS / GLT_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
    for (int r = 0; r < SCAN_ITEMS; r++) {
        int64_t i = base + r * SCAN_THREADS + threadIdx.x;
        if (i < n) acc += (T)in[i];
    }
    T tot;
    block_excl_scan<T, SCAN_THREADS>(acc, lds, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block of 1024 threads: exclusive scan of nb sums in place; writes grand total
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_sums(T* sums, int64_t nb, T* total_out) {
    __shared__ T lds[1024 / GLT_WAVE];
    int64_t per = (nb + 1023) / 1024;
    int64_t b0 = (int64_t)threadIdx.x * per;
    T acc = 0;
    for (int64_t i = 0; i < per; i++)
        if (b0 + i < nb) acc += sums[b0 + i];
    T tot;
    T off = block_excl_scan<T, 1024>(acc, lds, tot);
    for (int64_t i = 0; i < per; i++)
        if (b0 + i < nb) { T s = sums[b0 + i]; sums[b0 + i] = off; off += s; }
    if (threadIdx.x == 0 && total_out) *total_out = tot;
}

template <typename Tin, typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_apply(const Tin* in, T* out, int64_t n,
                                                                  const T* sums) {
    __shared__ T tile[SCAN_TILE];
    __shared__ T lds[SCAN_THREADS / GLT_WAVE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int r = 0; r < SCAN_ITEMS; r++) {
        int idx = r * SCAN_THREADS + threadIdx.x;
        int64_t i = base + idx;
        tile[idx] = (i < n) ? (T)in[i] : (T)0;
    }
    __syncthreads();
    T loc[SCAN_ITEMS];
    T acc = 0;
    for (int r = 0; r < SCAN_ITEMS; r++) { loc[r] = tile[threadIdx.x * SCAN_ITEMS + r]; acc += loc[r]; }
    T tot;
    T off = block_excl_scan<T, SCAN_THREADS>(acc, lds, tot) + sums[blockIdx.x];
    for (int r = 0; r < SCAN_ITEMS; r++) { tile[threadIdx.x * SCAN_ITEMS + r] = off; off += loc[r]; }
    __syncthreads();
    for (int r = 0; r < SCAN_ITEMS; r++) {
        int idx = r * SCAN_THREADS + threadIdx.x;
        int64_t i = base + idx;
        if (i < n) out[i] = tile[idx];
    }
}

// Inputs of at most SCAN_SMALL elements: one workgroup scans them in one launch (small
// calls, such as the batches of a served stream, are bound by their launch count).  Thread
// t owns up to SCAN_SMALL_ITEMS consecutive elements and reads all of them before writing
// any, so out may alias in.
#define SCAN_SMALL_THREADS 1024
#define SCAN_SMALL_ITEMS 16
#define SCAN_SMALL (SCAN_SMALL_THREADS * SCAN_SMALL_ITEMS)
template <typename Tin, typename T>
__global__ __launch_bounds__(SCAN_SMALL_THREADS) void k_scan_small(const Tin* in, T* out, int64_t n, T* total) {
    __shared__ T lds[SCAN_SMALL_THREADS / GLT_WAVE];
    const int per = (int)((n + SCAN_SMALL_THREADS - 1) / SCAN_SMALL_THREADS);   // <= SCAN_SMALL_ITEMS
    const int64_t b0 = (int64_t)threadIdx.x * per;
    T loc[SCAN_SMALL_ITEMS];
    T acc = 0;
#pragma unroll
    for (int r = 0; r < SCAN_SMALL_ITEMS; r++) {
        loc[r] = (r < per && b0 + r < n) ? (T)in[b0 + r] : (T)0;
        acc += loc[r];
    }
    T tot;
    T off = block_excl_scan<T, SCAN_SMALL_THREADS>(acc, lds, tot);
#pragma unroll
    for (int r = 0; r < SCAN_SMALL_ITEMS; r++)
        if (r < per && b0 + r < n) { out[b0 + r] = off; off += loc[r]; }
    if (threadIdx.x == 0 && total) *total = tot;
}

// out[i] = sum_{j<i} in[i]; out may alias in; total (device) optional.  tmp holds
// ceil(n / SCAN_TILE) elements.
template <typename Tin, typename T>
static inline void launch_excl_scan(const Tin* in, T* out, int64_t n, T* tmp, T* total,
                                    hipStream_t st) {
    if (n <= SCAN_SMALL) {
        hipLaunchKernelGGL((k_scan_small<Tin, T>), dim3(1), dim3(SCAN_SMALL_THREADS), 0, st, in, out, n, total);
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL((k_scan_tile_sums<Tin, T>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, n, tmp);
    hipLaunchKernelGGL((k_scan_sums<T>), dim3(1), dim3(1024), 0, st, tmp, nb, total);
    hipLaunchKernelGGL((k_scan_tile_apply<Tin, T>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, out, n, tmp);
}

static inline int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// ---------------------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, keys u64 and values u32
// ---------------------------------------------------------------------------------------
#define RS_THREADS 256
#define RS_ITEMS 16
#define RS_TILE (RS_THREADS * RS_ITEMS)

static __global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const u64* keys, int64_t n, int shift,
                                                        u32* counts, int64_t nblocks) {
    __shared__ u32 hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t i = base + r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&hist[(u32)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

static __global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const u64* kin, const u32* vin, u64* kout,
                                                           u32* vout, int64_t n, int shift,
                                                           const u32* offs, int64_t nblocks) {
    __shared__ u32 base[256];
    __shared__ u32 wcnt[RS_THREADS / GLT_WAVE][256];
    const int t = threadIdx.x, lane = glt_lane(), w = t / GLT_WAVE;
    base[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    for (int q = 0; q < RS_THREADS / GLT_WAVE; q++) wcnt[q][t] = 0;
    __syncthreads();
    const u64 lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (GLT_WAVE - lane));
    int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; r++) {
        int64_t i = tile0 + r * RS_THREADS + t;
        bool valid = i < n;
        u64 k = valid ? kin[i] : 0;
        u32 v = valid ? vin[i] : 0;
        u32 d = (u32)(k >> shift) & 255u;
        u64 peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            u64 bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        u32 rank = (u32)__popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[w][d] = (u32)__popcll(peers);
        __syncthreads();
        if (valid) {
            u32 off = base[d];
            for (int q = 0; q < w; q++) off += wcnt[q][d];
            kout[off + rank] = k;
            vout[off + rank] = v;
        }
        __syncthreads();
        u32 add = 0;
        for (int q = 0; q < RS_THREADS / GLT_WAVE; q++) { add += wcnt[q][t]; wcnt[q][t] = 0; }
        base[t] += add;
        __syncthreads();
    }
}

// Sorts (keys, vals) of length n (< 2^32) by key bits [0, bits).  Ping-pongs between the
// (k0,v0) and (k1,v1) buffers; returns 0 if the result is in (k0,v0), 1 if in (k1,v1).
// counts: 256 * ceil(n/RS_TILE) u32; tmp: scan scratch for that many elements.
static inline int launch_radix_sort(u64* k0, u32* v0, u64* k1, u32* v1, int64_t n, int bits,
                                    u32* counts, u32* tmp, hipStream_t st) {
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    int cur = 0;
    if (n <= 1) return 0;
    for (int shift = 0; shift < bits; shift += 8) {
        u64* ki = cur ? k1 : k0; u32* vi = cur ? v1 : v0;
        u64* ko = cur ? k0 : k1; u32* vo = cur ? v0 : v1;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_THREADS), 0, st, ki, n, shift, counts, nb);
        launch_excl_scan<u32, u32>(counts, counts, 256 * nb, tmp, (u32*)nullptr, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_THREADS), 0, st, ki, vi, ko, vo, n,
                           shift, counts, nb);
        cur ^= 1;
    }
    return cur;
}

static inline int64_t rs_counts_elems(int64_t n) { return 256 * ((n + RS_TILE - 1) / RS_TILE) + 1; }
