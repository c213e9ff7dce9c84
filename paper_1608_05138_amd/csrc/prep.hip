// prep.hip -- input validation and preprocessing (Section 4.2, P1-P3) on the device.
//
// P1: vertices are ordered by (degree, id) ascending and relabelled with their rank, so
//     that comparing relabelled ids compares degrees (ties by original id).
// P2: every adjacency list is sorted by relabelled id; ascending relabelled id is
//     ascending degree, i.e. the reverse of the paper's largest-first order, which only
//     changes the direction lists are walked in.
// P3: each edge is oriented from its lower-ranked endpoint u to its higher-ranked endpoint
//     v (d_v >= d_u).  The upward lists N+(x) form an oriented CSR whose entry index k is
//     the edge's index in every per-edge accumulator.
#include "glt_internal.h"

__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int d = GLT_WAVE / 2; d >= 1; d >>= 1) v |= __shfl_xor(v, d, GLT_WAVE);
    return v;
}

// One wavefront per row: offsets monotone and inside [0, S], ids in range, no self-loop.
template <typename RP>
__global__ __launch_bounds__(256) void k_validate_rows(const RP* __restrict__ rp, const int* __restrict__ col,
                                                       int n, int64_t S, int* __restrict__ deg,
                                                       int* __restrict__ err, int* __restrict__ maxdeg) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    if (wid >= n) return;
    const int x = (int)wid;
    int64_t b = (int64_t)rp[x], e = (int64_t)rp[x + 1];
    if (b < 0 || e < b || e > S) {
        if (lane == 0) { deg[x] = 0; atomicOr(err, ERR_RANGE); }
        return;
    }
    if (lane == 0) { deg[x] = (int)(e - b); atomicMax(maxdeg, (int)(e - b)); }
    int bad = 0;
    for (int64_t j = b + lane; j < e; j += GLT_WAVE) {
        int c = col[j];
        if (c < 0 || c >= n) bad |= ERR_RANGE;
        else if (c == x) bad |= ERR_SELF;
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(err, bad);
}

__global__ void k_iota_keys(const int* __restrict__ deg, int n, u64* __restrict__ keys, u32* __restrict__ vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { keys[i] = (u64)(u32)deg[i]; vals[i] = (u32)i; }
}

__global__ void k_apply_order(const u32* __restrict__ sorted_ids, const int* __restrict__ deg, int n,
                              int* __restrict__ order, int* __restrict__ rank, int* __restrict__ ndeg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int x = (int)sorted_ids[i];
        order[i] = x;
        rank[x] = i;
        ndeg[i] = deg[x];
    }
}

// One wavefront per row of the caller's CSR: emit the relabelled (src, dst) key of every
// slot, its caller slot index as payload, and the "upward in caller ids" flag whose
// prefix sum numbers the caller's edges.
template <typename RP>
__global__ __launch_bounds__(256) void k_emit(const RP* __restrict__ rp, const int* __restrict__ col, int n,
                                              const int* __restrict__ rank, int B, u64* __restrict__ keys,
                                              u32* __restrict__ vals, u32* __restrict__ upflag) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    if (wid >= n) return;
    const int x = (int)wid;
    const int64_t b = (int64_t)rp[x], e = (int64_t)rp[x + 1];
    const u64 rx = (u64)(u32)rank[x] << B;
    for (int64_t j = b + lane; j < e; j += GLT_WAVE) {
        int y = col[j];
        keys[j] = rx | (u64)(u32)rank[y];
        vals[j] = (u32)j;
        upflag[j] = (y > x) ? 1u : 0u;
    }
}

// Sorted keys -> relabelled columns; adjacent equal keys are duplicate entries.
__global__ void k_unpack_cols(const u64* __restrict__ keys, int64_t S, u64 mask, int* __restrict__ ncol,
                              int* __restrict__ err) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    u64 k = keys[s];
    ncol[s] = (int)(k & mask);
    if (s > 0 && keys[s - 1] == k) atomicOr(err, ERR_DUP);
}

// dlo[x] = number of neighbours ranked below x (the row is ascending, binary search).
__global__ void k_dlo(const int* __restrict__ nrp, const int* __restrict__ ncol, int n, int* __restrict__ dlo,
                      int* __restrict__ dplus) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int b = nrp[x], e = nrp[x + 1];
    int p = lower_bound_i32(ncol, b, e, x);
    dlo[x] = p - b;
    dplus[x] = e - p;
}

// One wavefront per relabelled row: copy the upward part into the oriented CSR, map every
// upward slot to its oriented index k, find the matching downward slot of the other
// endpoint (binary search) and map it to k too, name the caller's edge id of k, and
// initialise the edge's accumulator record.
__global__ __launch_bounds__(256) void k_edge_index(const int* __restrict__ nrp, const int* __restrict__ ncol,
                                                    const int* __restrict__ dlo, const int* __restrict__ optr,
                                                    const int* __restrict__ order, const u32* __restrict__ oslot,
                                                    const u32* __restrict__ upx, int n, int m, int* __restrict__ ocol,
                                                    int* __restrict__ s2k, int* __restrict__ eid2k,
                                                    EdgeAcc* __restrict__ acc, int* __restrict__ err) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    if (wid >= n) return;
    const int x = (int)wid;
    const int ub = nrp[x] + dlo[x], e = nrp[x + 1];
    const int k0 = optr[x];
    const int ox = order[x];
    int bad = 0;
    for (int s = ub + lane; s < e; s += GLT_WAVE) {
        const int k = k0 + (s - ub);
        if (k >= m) { bad |= ERR_ASYM; continue; }   // more upward than downward entries
        const int y = ncol[s];
        ocol[k] = y;
        s2k[s] = k;
        const int yb = nrp[y], ye = yb + dlo[y];
        const int sp = lower_bound_i32(ncol, yb, ye, x);
        EdgeAcc r;
        r.t = 0; r.u = x; r.v = y; r.pad = 0; r.K = 0; r.P = 0; r.gu = 0; r.gv = 0; r.sig = 0;
        acc[k] = r;
        if (sp >= ye || ncol[sp] != x) { bad |= ERR_ASYM; continue; }
        s2k[sp] = k;
        const int oy = order[y];
        const u32 j = (ox < oy) ? oslot[s] : oslot[sp];
        const u32 eid = upx[j];
        if (eid >= (u32)m) { bad |= ERR_ASYM; continue; }
        eid2k[eid] = k;
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(err, bad);
}

// Triangle / gather pass buckets by out-degree s = |N+(x)|.
__device__ __forceinline__ int tbucket(int s) {
    if (s < 2) return -1;
    if (s <= 64) return TB_WAVE;
    if (s <= 256) return TB_BLK1;
    if (s <= 640) return TB_BLK2;
    return TB_GLOBAL;
}

__device__ __forceinline__ void wave_append(int* counter, int* list, bool pred, int value) {
    const int lane = glt_lane();
    u64 mask = __ballot(pred);
    if (mask == 0) return;
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader, GLT_WAVE);
    u64 lt = (lane == 0) ? 0ull : ((~0ull) >> (GLT_WAVE - lane));
    if (pred) list[base + __popcll(mask & lt)] = value;
}

__global__ __launch_bounds__(256) void k_tbuckets(const int* __restrict__ optr, int n, int* __restrict__ tlist,
                                                  int* __restrict__ counts, int* __restrict__ tmax) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int s = (x < n) ? optr[x + 1] - optr[x] : 0;
    int b = (x < n) ? tbucket(s) : -1;
    for (int q = 0; q < TB_N; q++) {
        wave_append(&counts[q], tlist + (int64_t)q * n, b == q, x);
        if (b == q) atomicMax(&tmax[q], s);
    }
}

// Wedge pass: wc[y] = number of wedges y - w - x with x above both y and w
// (w in N(y), x in N+(w), x > y).  One wavefront per vertex; buckets by wc.
__global__ __launch_bounds__(256) void k_wbuckets(const int* __restrict__ nrp, const int* __restrict__ ncol,
                                                  const int* __restrict__ optr, const int* __restrict__ s2k, int n,
                                                  int wave_max, int* __restrict__ wlist, int* __restrict__ counts,
                                                  u64* __restrict__ work) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    if (wid >= n) return;
    const int y = (int)wid;
    int64_t wc = 0, ls = 0;
    for (int s = nrp[y] + lane; s < nrp[y + 1]; s += GLT_WAVE) {
        int w = ncol[s];
        const int dpw = optr[w + 1] - optr[w];
        wc += (w > y) ? dpw : (optr[w + 1] - s2k[s] - 1);
        ls += (w > y) ? dpw : 0;
    }
    wc = wave_sum(wc);
    ls = wave_sum(ls);
    if (lane == 0) {
        if (wc) atomicAdd(&work[0], (u64)wc);
        if (ls) atomicAdd(&work[1], (u64)ls);
    }
    if (lane == 0 && wc > 0) {
        int q = (wc <= wave_max) ? WB_WAVE : WB_BLK;
        int pos = atomicAdd(&counts[q], 1);
        wlist[(int64_t)q * n + pos] = y;
    }
}

// ---------------------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------------------
static inline unsigned nblk(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

int glt_prep_validate(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st) {
    // err[0] error bits, err[1] max degree
    (void)hipMemsetAsync(d.err, 0, 4 * sizeof(int), st);
    if (d.n > 0) {
        unsigned g = nblk((int64_t)d.n * GLT_WAVE, 256);
        if (rp64)
            hipLaunchKernelGGL(k_validate_rows<int64_t>, dim3(g), dim3(256), 0, st, (const int64_t*)rp, col, d.n,
                               (int64_t)d.S, d.deg, d.err, d.err + 1);
        else
            hipLaunchKernelGGL(k_validate_rows<int32_t>, dim3(g), dim3(256), 0, st, (const int32_t*)rp, col, d.n,
                               (int64_t)d.S, d.deg, d.err, d.err + 1);
    }
    return 0;
}

static inline int bitlen(u64 x) { int b = 0; while (x) { b++; x >>= 1; } return b; }

int glt_prep_build(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st, int* host_counts) {
    const int n = d.n;
    const int64_t S = d.S;
    int maxdeg = host_counts[0];
    (void)hipMemsetAsync(d.counts, 0, sizeof(int) * (TB_N + WB_N + TB_N), st);
    (void)hipMemsetAsync(d.work, 0, sizeof(u64) * 2, st);
    if (n == 0) return 0;
    // P1: stable sort of vertices by degree (ties keep id order)
    hipLaunchKernelGGL(k_iota_keys, dim3(nblk(n, 256)), dim3(256), 0, st, d.deg, n, d.key0, d.val0);
    int cur = launch_radix_sort(d.key0, d.val0, d.key1, d.val1, n, bitlen((u64)maxdeg), d.rs_counts, d.rs_tmp, st);
    hipLaunchKernelGGL(k_apply_order, dim3(nblk(n, 256)), dim3(256), 0, st, cur ? d.val1 : d.val0, d.deg, n,
                       d.order, d.rank, d.ndeg);
    // relabelled CSR offsets
    launch_excl_scan<int, int>(d.ndeg, d.nrp, n, d.itmp, d.nrp + n, st);
    // P2: sort every slot by (relabelled src, relabelled dst)
    const int B = bitlen((u64)(n > 1 ? n - 1 : 1));
    if (S > 0) {
        unsigned g = nblk((int64_t)n * GLT_WAVE, 256);
        if (rp64)
            hipLaunchKernelGGL(k_emit<int64_t>, dim3(g), dim3(256), 0, st, (const int64_t*)rp, col, n, d.rank, B,
                               d.key0, d.val0, d.upx);
        else
            hipLaunchKernelGGL(k_emit<int32_t>, dim3(g), dim3(256), 0, st, (const int32_t*)rp, col, n, d.rank, B,
                               d.key0, d.val0, d.upx);
        launch_excl_scan<u32, u32>(d.upx, d.upx, S, d.rs_tmp, (u32*)nullptr, st);
        cur = launch_radix_sort(d.key0, d.val0, d.key1, d.val1, S, 2 * B, d.rs_counts, d.rs_tmp, st);
        u64* ks = cur ? d.key1 : d.key0;
        hipLaunchKernelGGL(k_unpack_cols, dim3(nblk(S, 256)), dim3(256), 0, st, ks, S, (u64)((1ull << B) - 1),
                           d.ncol, d.err);
    }
    const u32* oslot = cur ? d.val1 : d.val0;
    // P3: orientation
    int* dplus = d.itmp + scan_tmp_elems(S + n + 1);  // past the scan scratch
    hipLaunchKernelGGL(k_dlo, dim3(nblk(n, 256)), dim3(256), 0, st, d.nrp, d.ncol, n, d.dlo, dplus);
    launch_excl_scan<int, int>(dplus, d.optr, n, d.itmp, d.optr + n, st);
    if (S > 0)
        hipLaunchKernelGGL(k_edge_index, dim3(nblk((int64_t)n * GLT_WAVE, 256)), dim3(256), 0, st, d.nrp, d.ncol,
                           d.dlo, d.optr, d.order, oslot, d.upx, n, d.m, d.ocol, d.s2k, d.eid2k, d.acc, d.err);
    // work lists
    {
        hipLaunchKernelGGL(k_tbuckets, dim3(nblk(n, 256)), dim3(256), 0, st, d.optr, n, d.tlist, d.counts,
                           d.counts + TB_N + WB_N);
        hipLaunchKernelGGL(k_wbuckets, dim3(nblk((int64_t)n * GLT_WAVE, 256)), dim3(256), 0, st, d.nrp, d.ncol,
                           d.optr, d.s2k, n, d.wedge_wave_max, d.wlist, d.counts + TB_N, d.work);
    }
    return 0;
}
