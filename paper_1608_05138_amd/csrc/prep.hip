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
                                                       int* __restrict__ err) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    if (wid >= n) return;
    const int x = (int)wid;
    int64_t b = (int64_t)rp[x], e = (int64_t)rp[x + 1];
    if (b < 0 || e < b || e > S) {
        if (lane == 0) { deg[x] = 0; atomicOr(err, ERR_RANGE); }
        return;
    }
    if (lane == 0) deg[x] = (int)(e - b);
    int bad = 0;
    for (int64_t j = b + lane; j < e; j += GLT_WAVE) {
        int c = col[j];
        if (c < 0 || c >= n) bad |= ERR_RANGE;
        else if (c == x) bad |= ERR_SELF;
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(err, bad);
}

// Maximum degree: one atomic per workgroup.
__global__ __launch_bounds__(256) void k_max_deg(const int* __restrict__ deg, int n, int* __restrict__ maxdeg) {
    __shared__ int red[256 / GLT_WAVE];
    int v = 0;
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < n; x += (int64_t)gridDim.x * 256)
        v = max(v, deg[x]);
    v = wave_max(v);
    if (glt_lane() == 0) red[threadIdx.x / GLT_WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = 0;
        for (int q = 0; q < 256 / GLT_WAVE; q++) b = max(b, red[q]);
        if (b) atomicMax(maxdeg, b);
    }
}

__global__ void k_iota_keys(const int* __restrict__ deg, int n, u64* __restrict__ keys, u32* __restrict__ vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { keys[i] = (u64)(u32)deg[i]; vals[i] = (u32)i; }
}

__global__ void k_apply_order(const u32* __restrict__ sorted_ids, const int* __restrict__ deg, int n,
                              int* __restrict__ order, int* __restrict__ rank, int* __restrict__ ndeg,
                              const int* __restrict__ gid, int* __restrict__ ngid) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int x = (int)sorted_ids[i];
        order[i] = x;
        rank[x] = i;
        ndeg[i] = deg[x];
        if (ngid) ngid[i] = gid[x];
    }
}

// ---------------------------------------------------------------------------------------
// batched input: graphs packed with per-graph bases become one disjoint union
// ---------------------------------------------------------------------------------------
// One workgroup per graph: union offsets from the graph's local offsets, graph id per vertex.
// Local offsets outside [0, 2 m_g] or not starting at 0 / ending at 2 m_g are flagged and
// replaced by in-range values so later kernels stay inside the arrays.
__global__ __launch_bounds__(256) void k_union_rows(const int64_t* __restrict__ vb, const int64_t* __restrict__ sb,
                                                    const int* __restrict__ lrp, int* __restrict__ urp,
                                                    int* __restrict__ gid, int* __restrict__ err) {
    const int g = blockIdx.x;
    const int64_t v0 = vb[g], ng = vb[g + 1] - v0;
    const int64_t s0 = sb[g], sg = sb[g + 1] - s0;
    const int* lr = lrp + v0 + g;
    int bad = 0;
    for (int64_t i = threadIdx.x; i <= ng; i += blockDim.x) {
        int64_t o = lr[i];
        if (o < 0 || o > sg || (i == 0 && o != 0) || (i == ng && o != sg)) {
            bad = ERR_RANGE;
            o = (i == ng) ? sg : 0;
        }
        if (i < ng) { urp[v0 + i] = (int)(s0 + o); gid[v0 + i] = g; }
    }
    if (bad) atomicOr(err, bad);
}

// One wavefront per union vertex: local neighbour ids -> union ids (out-of-range local ids
// are flagged and replaced by the vertex itself, which the self-loop check then rejects too).
__global__ __launch_bounds__(256) void k_union_cols(const int64_t* __restrict__ vb, const int* __restrict__ urp,
                                                    const int* __restrict__ gid, const int* __restrict__ lcol,
                                                    int N, int64_t S, int* __restrict__ ucol, int* __restrict__ err) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    if (wid >= N) return;
    const int v = (int)wid;
    const int g = gid[v];
    const int64_t v0 = vb[g], ng = vb[g + 1] - v0;
    int64_t b = urp[v], e = urp[v + 1];
    if (b < 0 || e < b || e > S) {
        if (lane == 0) atomicOr(err, ERR_RANGE);
        return;
    }
    int bad = 0;
    for (int64_t j = b + lane; j < e; j += GLT_WAVE) {
        const int c = lcol[j];
        if (c < 0 || c >= ng) { bad = ERR_RANGE; ucol[j] = v; }
        else ucol[j] = (int)(v0 + c);
    }
    bad = wave_or(bad);
    if (lane == 0 && bad) atomicOr(err, bad);
}

int glt_union_build(const Dev& d, const int* lrp, const int* lcol, int* urp, int* ucol, hipStream_t st) {
    (void)hipMemsetAsync(d.err, 0, 4 * sizeof(int), st);
    if (d.ngraphs <= 0 || d.n <= 0) return 0;
    hipLaunchKernelGGL(k_union_rows, dim3(d.ngraphs), dim3(256), 0, st, d.gvb, d.gsb, lrp, urp, d.gid, d.err);
    launch_fill<int>(urp + d.n, 1, d.S, st);
    hipLaunchKernelGGL(k_union_cols, dim3((unsigned)(((int64_t)d.n * GLT_WAVE + 255) / 256)), dim3(256), 0, st,
                       d.gvb, urp, d.gid, lcol, d.n, (int64_t)d.S, ucol, d.err);
    return 0;
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
                                                    EdgeArrays ea, int* __restrict__ err) {
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
        ea.t[k] = 0; ea.K[k] = 0; ea.P[k] = 0; ea.gu[k] = 0; ea.gv[k] = 0; ea.sig[k] = 0; ea.u[k] = x;
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
        const int mx = wave_max(b == q ? s : 0);
        if (glt_lane() == 0 && mx) atomicMax(&tmax[q], mx);
    }
}

// Wedge pass: wc[y] = number of wedges y - w - x with x above both y and w
// (w in N(y), x in N+(w), x > y), and the triangle pass's list length sum over the
// out-neighbours w of y of |N+(w)|.  One wavefront per vertex; work totals reduced per
// workgroup before one atomic.
__global__ __launch_bounds__(256) void k_wcount(const int* __restrict__ nrp, const int* __restrict__ ncol,
                                                const int* __restrict__ optr, const int* __restrict__ s2k, int n,
                                                int64_t* __restrict__ wcnt, u64* __restrict__ work) {
    __shared__ u64 red[2][256 / GLT_WAVE];
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GLT_WAVE;
    const int lane = glt_lane();
    int64_t wc = 0, ls = 0;
    if (wid < n) {
        const int y = (int)wid;
        for (int s = nrp[y] + lane; s < nrp[y + 1]; s += GLT_WAVE) {
            const int w = ncol[s];
            const int dpw = optr[w + 1] - optr[w];
            wc += (w > y) ? dpw : (optr[w + 1] - s2k[s] - 1);
            ls += (w > y) ? dpw : 0;
        }
        wc = wave_sum(wc);
        ls = wave_sum(ls);
        if (lane == 0) wcnt[y] = wc;
    }
    if (lane == 0) { red[0][threadIdx.x / GLT_WAVE] = (u64)wc; red[1][threadIdx.x / GLT_WAVE] = (u64)ls; }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 a = 0, b = 0;
        for (int q = 0; q < 256 / GLT_WAVE; q++) { a += red[0][q]; b += red[1][q]; }
        if (a) atomicAdd(&work[0], a);
        if (b) atomicAdd(&work[1], b);
    }
}

__global__ __launch_bounds__(256) void k_wappend(const int64_t* __restrict__ wcnt, int n, int wave_max,
                                                 int* __restrict__ wlist, int* __restrict__ counts) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t wc = (y < n) ? wcnt[y] : 0;
    const int q = (wc == 0) ? -1 : (wc <= wave_max ? WB_WAVE : WB_BLK);
    for (int b = 0; b < WB_N; b++) wave_append(&counts[b], wlist + (int64_t)b * n, q == b, y);
}

// ---------------------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------------------
static inline unsigned nblk(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

int glt_prep_validate(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st) {
    // err[0] error bits (kept from the union build in batched mode), err[1] max degree
    if (d.ngraphs <= 0) (void)hipMemsetAsync(d.err, 0, 4 * sizeof(int), st);
    if (d.n > 0) {
        unsigned g = nblk((int64_t)d.n * GLT_WAVE, 256);
        if (rp64)
            hipLaunchKernelGGL(k_validate_rows<int64_t>, dim3(g), dim3(256), 0, st, (const int64_t*)rp, col, d.n,
                               (int64_t)d.S, d.deg, d.err);
        else
            hipLaunchKernelGGL(k_validate_rows<int32_t>, dim3(g), dim3(256), 0, st, (const int32_t*)rp, col, d.n,
                               (int64_t)d.S, d.deg, d.err);
        unsigned gm = nblk(d.n, 256);
        if (gm > 2048) gm = 2048;
        hipLaunchKernelGGL(k_max_deg, dim3(gm), dim3(256), 0, st, d.deg, d.n, d.err + 1);
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
                       d.order, d.rank, d.ndeg, d.gid, d.ngid);
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
                           d.dlo, d.optr, d.order, oslot, d.upx, n, d.m, d.ocol, d.s2k, d.eid2k, d.e, d.err);
    // work lists
    {
        hipLaunchKernelGGL(k_tbuckets, dim3(nblk(n, 256)), dim3(256), 0, st, d.optr, n, d.tlist, d.counts,
                           d.counts + TB_N + WB_N);
        hipLaunchKernelGGL(k_wcount, dim3(nblk((int64_t)n * GLT_WAVE, 256)), dim3(256), 0, st, d.nrp, d.ncol,
                           d.optr, d.s2k, n, d.wcnt, d.work);
        hipLaunchKernelGGL(k_wappend, dim3(nblk(n, 256)), dim3(256), 0, st, d.wcnt, n, d.wedge_wave_max, d.wlist,
                           d.counts + TB_N);
    }
    return 0;
}
