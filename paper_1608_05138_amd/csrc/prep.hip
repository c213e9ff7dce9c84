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
//
// Kernels over CSR entries run one thread per entry.  The row of an entry of the caller's
// CSR comes from a counting pass: with cnt[p] = number of rows starting at offset p,
// E = exclusive prefix of cnt, the row of entry s is E[s+1] - 1 (the last row whose start
// is <= s).  The row of an entry of the relabelled CSR is the high half of its sort key.
#include "glt_internal.h"

__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int d = GLT_WAVE / 2; d >= 1; d >>= 1) v |= __shfl_xor(v, d, GLT_WAVE);
    return v;
}

static inline unsigned nblk(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

// ---------------------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------------------
// One thread per row: offsets inside [0, S] and monotone; degree; row-start counts.
template <typename RP>
__global__ __launch_bounds__(256) void k_check_rows(const RP* __restrict__ rp, int n, int64_t S,
                                                    int* __restrict__ deg, u32* __restrict__ cnt,
                                                    int* __restrict__ err) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = false;
    int64_t b = 0;
    if (x < n) {
        b = (int64_t)rp[x];
        const int64_t e = (int64_t)rp[x + 1];
        ok = b >= 0 && e >= b && e <= S;
        deg[x] = ok ? (int)(e - b) : 0;
    }
    const int bad = wave_or((x < n && !ok) ? ERR_RANGE : 0);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
    // rows of a wavefront start at non-decreasing offsets: count each offset once per run
    bool last;
    const int key = ok ? (int)b : 0x7fffffff;
    const u32 c = seg_sum_last(ok ? 1u : 0u, key, last);
    if (last && c && ok) atomicAdd(&cnt[b], c);
}

// One thread per entry of the caller's CSR: its row (from the row-start prefix), the
// neighbour id in range, no self-loop.
__global__ __launch_bounds__(256) void k_check_cols(const u32* __restrict__ rowx, const int* __restrict__ col,
                                                    int n, int64_t S, int* __restrict__ err) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (s < S) {
        const int x = (int)rowx[s + 1] - 1;
        const int c = col[s];
        if (x < 0 || x >= n || c < 0 || c >= n) bad = ERR_RANGE;
        else if (c == x) bad = ERR_SELF;
    }
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
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

// ---------------------------------------------------------------------------------------
// batched input: graphs packed with per-graph bases become one disjoint union
// ---------------------------------------------------------------------------------------
// One workgroup per graph: union offsets from the graph's local offsets, graph id per vertex.
// Local offsets outside [0, 2 m_g] or not starting at 0 / ending at 2 m_g are flagged and
// replaced by in-range values so later kernels stay inside the arrays.
__global__ __launch_bounds__(256) void k_union_rows(const int64_t* __restrict__ vb, const int64_t* __restrict__ sb,
                                                    const int* const* __restrict__ glrp, int* __restrict__ urp,
                                                    int* __restrict__ gid, int* __restrict__ err) {
    const int g = blockIdx.x;
    const int64_t v0 = vb[g], ng = vb[g + 1] - v0;
    const int64_t s0 = sb[g], sg = sb[g + 1] - s0;
    const int* lr = glrp[g];
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

// One thread per union entry: local neighbour id -> union id (an out-of-range local id is
// flagged and replaced by the entry's own row, which the self-loop check rejects too).
__global__ __launch_bounds__(256) void k_union_cols(const int64_t* __restrict__ vb, const int64_t* __restrict__ sb,
                                                    const u32* __restrict__ rowx, const int* __restrict__ gid,
                                                    const int* const* __restrict__ glcol, int N, int64_t S,
                                                    int* __restrict__ ucol, int* __restrict__ err) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (s < S) {
        const int v = (int)rowx[s + 1] - 1;
        if (v < 0 || v >= N) {
            bad = ERR_RANGE;
            ucol[s] = 0;
        } else {
            const int g = gid[v];
            const int64_t v0 = vb[g], ng = vb[g + 1] - v0;
            const int64_t j = s - sb[g];
            if (j < 0 || j >= sb[g + 1] - sb[g]) {
                bad = ERR_RANGE;
                ucol[s] = v;
            } else {
                const int c = glcol[g][j];
                if (c < 0 || c >= ng) { bad = ERR_RANGE; ucol[s] = v; }
                else ucol[s] = (int)(v0 + c);
            }
        }
    }
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
}

int glt_union_build(const Dev& d, int* urp, int* ucol, hipStream_t st) {
    (void)ucol;
    (void)hipMemsetAsync(d.err, 0, 4 * sizeof(int), st);
    if (d.ngraphs <= 0) return 0;
    hipLaunchKernelGGL(k_union_rows, dim3(d.ngraphs), dim3(256), 0, st, d.gvb, d.gsb, d.glrp, urp, d.gid, d.err);
    launch_fill<int>(urp + d.n, 1, d.S, st);
    return 0;
}

// ---------------------------------------------------------------------------------------
// P1 / P2 / P3
// ---------------------------------------------------------------------------------------
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

// One thread per entry of the caller's CSR: the relabelled (src, dst) key, the caller's
// entry index as payload, and the "upward in caller ids" flag whose prefix sum numbers the
// caller's edges.
__global__ __launch_bounds__(256) void k_emit(const u32* __restrict__ rowx, const int* __restrict__ col, int64_t S,
                                              const int* __restrict__ rank, int B, u64* __restrict__ keys,
                                              u32* __restrict__ vals, u32* __restrict__ upflag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int x = (int)rowx[s + 1] - 1;
    const int y = col[s];
    keys[s] = ((u64)(u32)rank[x] << B) | (u64)(u32)rank[y];
    vals[s] = (u32)s;
    upflag[s] = (y > x) ? 1u : 0u;
}

// Sorted keys -> relabelled rows and columns; adjacent equal keys are duplicate entries.
__global__ void k_unpack_cols(const u64* __restrict__ keys, int64_t S, int B, int* __restrict__ ncol,
                              int* __restrict__ nsrow, int* __restrict__ err) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const u64 k = keys[s];
    ncol[s] = (int)(k & ((1ull << B) - 1));
    nsrow[s] = (int)(k >> B);
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

// One thread per relabelled entry; upward entries (x -> y, y > x) copy themselves into the
// oriented CSR at index k, map both their own entry and the matching downward entry of y
// (binary search) to k, name the caller's edge id of k and clear the edge's accumulators.
__global__ __launch_bounds__(256) void k_edge_index(const int* __restrict__ nrp, const int* __restrict__ ncol,
                                                    const int* __restrict__ nsrow, const int* __restrict__ dlo,
                                                    const int* __restrict__ optr, const int* __restrict__ order,
                                                    const u32* __restrict__ oslot, const u32* __restrict__ upx,
                                                    int64_t S, int m, int* __restrict__ ocol, int* __restrict__ s2k,
                                                    int* __restrict__ eid2k, EdgeArrays ea, int* __restrict__ err) {
    const int64_t s64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (s64 < S) {
        const int s = (int)s64;
        const int x = nsrow[s];
        const int ub = nrp[x] + dlo[x];
        const int y = ncol[s];
        if (s >= ub) {
            const int k = optr[x] + (s - ub);
            if (k >= m) {
                bad = ERR_ASYM;   // more upward than downward entries
            } else {
                ocol[k] = y;
                s2k[s] = k;
                ea.t[k] = 0; ea.K[k] = 0; ea.P[k] = 0; ea.g[k] = 0; ea.sig[k] = 0; ea.u[k] = x;
                const int yb = nrp[y], ye = yb + dlo[y];
                const int sp = lower_bound_i32(ncol, yb, ye, x);
                if (sp >= ye || ncol[sp] != x) {
                    bad = ERR_ASYM;
                } else {
                    s2k[sp] = k;
                    const u32 j = (order[x] < order[y]) ? oslot[s] : oslot[sp];
                    const u32 eid = upx[j];
                    if (eid >= (u32)m) bad = ERR_ASYM;
                    else eid2k[eid] = k;
                }
            }
        }
    }
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
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

// Wedge pass work: per relabelled entry (y -> w) the wedges y - w - x with x above both y
// and w (x in N+(w), x > y), summed per y; and the triangle pass's list lengths |N+(w)|
// over upward entries.  One thread per entry, runs of one row summed in the wavefront.
__global__ __launch_bounds__(256) void k_wcount(const int* __restrict__ ncol, const int* __restrict__ nsrow,
                                                const int* __restrict__ optr, const int* __restrict__ s2k, int64_t S,
                                                u64* __restrict__ wcnt, u64* __restrict__ work) {
    __shared__ u64 red[2][256 / GLT_WAVE];
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u64 wc = 0, ls = 0;
    int y = 0x7fffffff;
    if (s < S) {
        y = nsrow[s];
        const int w = ncol[s];
        const int dpw = optr[w + 1] - optr[w];
        wc = (u64)((w > y) ? dpw : (optr[w + 1] - s2k[s] - 1));
        ls = (u64)((w > y) ? dpw : 0);
    }
    bool last;
    const u64 run = seg_sum_last(wc, y, last);
    if (last && run && y != 0x7fffffff) atomicAdd(&wcnt[y], run);
    const u64 a = wave_sum(wc), b = wave_sum(ls);
    if (glt_lane() == 0) { red[0][threadIdx.x / GLT_WAVE] = a; red[1][threadIdx.x / GLT_WAVE] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 ta = 0, tb = 0;
        for (int q = 0; q < 256 / GLT_WAVE; q++) { ta += red[0][q]; tb += red[1][q]; }
        if (ta) atomicAdd(&work[0], ta);
        if (tb) atomicAdd(&work[1], tb);
    }
}

__global__ __launch_bounds__(256) void k_wappend(const u64* __restrict__ wcnt, int n, int wave_max,
                                                 int* __restrict__ wlist, int* __restrict__ counts) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    const u64 wc = (y < n) ? wcnt[y] : 0;
    const int q = (wc == 0) ? -1 : (wc <= (u64)wave_max ? WB_WAVE : WB_BLK);
    for (int b = 0; b < WB_N; b++) wave_append(&counts[b], wlist + (int64_t)b * n, q == b, y);
}

// ---------------------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------------------
int glt_prep_validate(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st) {
    // err[0] error bits (kept from the union build in batched mode), err[1] max degree
    if (d.ngraphs <= 0) (void)hipMemsetAsync(d.err, 0, 4 * sizeof(int), st);
    if (d.n <= 0) return 0;
    const int64_t S = d.S;
    launch_fill<u32>(d.rowx, S + 1, 0u, st);
    if (rp64)
        hipLaunchKernelGGL(k_check_rows<int64_t>, dim3(nblk(d.n, 256)), dim3(256), 0, st, (const int64_t*)rp, d.n, S,
                           d.deg, d.rowx, d.err);
    else
        hipLaunchKernelGGL(k_check_rows<int32_t>, dim3(nblk(d.n, 256)), dim3(256), 0, st, (const int32_t*)rp, d.n, S,
                           d.deg, d.rowx, d.err);
    launch_excl_scan<u32, u32>(d.rowx, d.rowx, S + 1, d.rs_tmp, (u32*)nullptr, st);
    if (S > 0) {
        if (d.ngraphs > 0)
            hipLaunchKernelGGL(k_union_cols, dim3(nblk(S, 256)), dim3(256), 0, st, d.gvb, d.gsb, d.rowx, d.gid,
                               d.glcol, d.n, S, (int*)col, d.err);
        hipLaunchKernelGGL(k_check_cols, dim3(nblk(S, 256)), dim3(256), 0, st, d.rowx, col, d.n, S, d.err);
    }
    unsigned gm = nblk(d.n, 256);
    if (gm > 2048) gm = 2048;
    hipLaunchKernelGGL(k_max_deg, dim3(gm), dim3(256), 0, st, d.deg, d.n, d.err + 1);
    return 0;
}

static inline int bitlen(u64 x) { int b = 0; while (x) { b++; x >>= 1; } return b; }

int glt_prep_build(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st, int* host_counts) {
    (void)rp;
    (void)rp64;
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
    // P2: sort every entry by (relabelled src, relabelled dst)
    const int B = bitlen((u64)(n > 1 ? n - 1 : 1));
    if (S > 0) {
        hipLaunchKernelGGL(k_emit, dim3(nblk(S, 256)), dim3(256), 0, st, d.rowx, col, S, d.rank, B, d.key0, d.val0,
                           d.upx);
        launch_excl_scan<u32, u32>(d.upx, d.upx, S, d.rs_tmp, (u32*)nullptr, st);
        cur = launch_radix_sort(d.key0, d.val0, d.key1, d.val1, S, 2 * B, d.rs_counts, d.rs_tmp, st);
        u64* ks = cur ? d.key1 : d.key0;
        hipLaunchKernelGGL(k_unpack_cols, dim3(nblk(S, 256)), dim3(256), 0, st, ks, S, B, d.ncol, d.nsrow, d.err);
    }
    const u32* oslot = cur ? d.val1 : d.val0;
    // P3: orientation
    int* dplus = d.itmp + scan_tmp_elems(S + n + 1);  // past the scan scratch
    hipLaunchKernelGGL(k_dlo, dim3(nblk(n, 256)), dim3(256), 0, st, d.nrp, d.ncol, n, d.dlo, dplus);
    launch_excl_scan<int, int>(dplus, d.optr, n, d.itmp, d.optr + n, st);
    if (S > 0)
        hipLaunchKernelGGL(k_edge_index, dim3(nblk(S, 256)), dim3(256), 0, st, d.nrp, d.ncol, d.nsrow, d.dlo, d.optr,
                           d.order, oslot, d.upx, S, d.m, d.ocol, d.s2k, d.eid2k, d.e, d.err);
    // work lists
    hipLaunchKernelGGL(k_tbuckets, dim3(nblk(n, 256)), dim3(256), 0, st, d.optr, n, d.tlist, d.counts,
                       d.counts + TB_N + WB_N);
    launch_fill<u64>(d.wcnt, n, 0ull, st);
    if (S > 0)
        hipLaunchKernelGGL(k_wcount, dim3(nblk(S, 256)), dim3(256), 0, st, d.ncol, d.nsrow, d.optr, d.s2k, S, d.wcnt,
                           d.work);
    hipLaunchKernelGGL(k_wappend, dim3(nblk(n, 256)), dim3(256), 0, st, d.wcnt, n, d.wedge_wave_max, d.wlist,
                       d.counts + TB_N);
    return 0;
}
