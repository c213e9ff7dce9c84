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

// Appends value[r] to list cls[r] (one of NL lists, `stride` apart) for every entry whose
// class is in [0, NL).  A workgroup of 256 threads holds R sub-tiles of 256 consecutive
// indices (thread t holds entry t of each); within the workgroup's tile the entries keep
// their index order, and each list takes one global atomic per workgroup (hundreds of
// thousands of workgroups on a few counters would serialise).  Every thread of the
// workgroup must call it, once per kernel.
template <int NL, int R, int CS = 1>   // CS: ints between consecutive list counters
__device__ __forceinline__ void block_append(int* counters, int* lists, int64_t stride, const int (&cls)[R],
                                             const int (&value)[R]) {
    __shared__ int wc[R][NL][256 / GLT_WAVE];
    __shared__ int base[NL];
    const int lane = glt_lane(), w = threadIdx.x / GLT_WAVE;
    const u64 lt = (lane == 0) ? 0ull : ((~0ull) >> (GLT_WAVE - lane));
    u64 mine[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        mine[r] = 0;
#pragma unroll
        for (int c = 0; c < NL; c++) {
            const u64 msk = __ballot(cls[r] == c);
            if (cls[r] == c) mine[r] = msk;
            if (lane == 0) wc[r][c][w] = (int)__popcll(msk);
        }
    }
    __syncthreads();
    if (threadIdx.x < NL) {   // per list: exclusive prefix over (sub-tile, wavefront), then one atomic
        const int c = threadIdx.x;
        int tot = 0;
        for (int r = 0; r < R; r++)
            for (int q = 0; q < 256 / GLT_WAVE; q++) {
                const int v = wc[r][c][q];
                wc[r][c][q] = tot;
                tot += v;
            }
        base[c] = tot ? atomicAdd(&counters[c * CS], tot) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int c = cls[r];
        if (c >= 0 && c < NL)
            lists[(int64_t)c * stride + base[c] + wc[r][c][w] + (int)__popcll(mine[r] & lt)] = value[r];
    }
}

// Sub-tiles per workgroup of the list and counter kernels: 8 on large inputs (eight times
// fewer same-address atomics), 1 on small ones (more workgroups, shorter per-thread chains).
#ifndef TILE_R_LARGE
#define TILE_R_LARGE 8
#endif
static inline int tile_r(int64_t n) { return n >= (1 << 20) ? TILE_R_LARGE : 1; }

static inline unsigned nblk(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

// ---------------------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------------------
// One thread per row (R sub-tiles of 256 rows per workgroup): offsets inside [0, S] and
// monotone; degree; row-start counts (when cnt is given); rows per sort class.
template <typename RP, int R>
__global__ __launch_bounds__(256) void k_check_rows(const RP* __restrict__ rp, int n, int64_t S,
                                                    int* __restrict__ deg, u32* __restrict__ cnt,
                                                    int* __restrict__ err) {
    // rows per sort class of P2, summed per workgroup before one atomic per class
    __shared__ int cls_cnt[RS_N];
    if (threadIdx.x < RS_N) cls_cnt[threadIdx.x] = 0;
    __syncthreads();
    int bad = 0;
    for (int r = 0; r < R; r++) {
        const int x = (blockIdx.x * R + r) * 256 + threadIdx.x;
        bool ok = false;
        int64_t b = 0;
        if (x < n) {
            b = (int64_t)rp[x];
            const int64_t e = (int64_t)rp[x + 1];
            // offsets non-decreasing inside [0, S], starting at 0 and ending at S = 2m
            ok = b >= 0 && e >= b && e <= S && (x > 0 || b == 0) && (x < n - 1 || e == S);
            deg[x] = ok ? (int)(e - b) : 0;
            if (!ok) bad = ERR_RANGE;
        }
        const int cls = ok ? row_class(deg[x]) : -1;
#pragma unroll
        for (int c = 0; c < RS_N; c++) {
            const u64 msk = __ballot(cls == c);
            if (glt_lane() == 0 && msk) atomicAdd(&cls_cnt[c], (int)__popcll(msk));
        }
        // rows of a wavefront start at non-decreasing offsets: count each offset once per run
        bool last;
        const int key = ok ? (int)b : 0x7fffffff;
        const u32 c = seg_sum_last(ok ? 1u : 0u, key, last);
        if (cnt && last && c && ok) atomicAdd(&cnt[b], c);
    }
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
    __syncthreads();
    if (threadIdx.x < RS_N && cls_cnt[threadIdx.x]) atomicAdd(&err[2 + threadIdx.x], cls_cnt[threadIdx.x]);
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

// Batch: per sub-chunk of US_SUB entries of one graph (its chunks of 2 CG_CHUNK entries are
// numbered by gcb; one workgroup per sub-chunk) the union row of every entry, in the form
// the relabelling reads (rowx[s + 1] = row + 1), its union column, and the checks of every
// entry (id in range, no self-loop).  The sub-chunk's first row is found by rounds of 256
// probes, its rows are expanded into LDS (one thread per row, from the union offsets) and
// written out coalesced, so the union needs no row-start counting pass and no scan over all
// entries.  Entries no row covers (offsets not monotone, which the row check flags too) are
// flagged as well.
#define US_SLOTS (2 * CG_CHUNK)
#define US_SUB 4096   // entries expanded in LDS at a time
__global__ __launch_bounds__(256) void k_union_slots(const int64_t* __restrict__ vb, const int64_t* __restrict__ sb,
                                                     const int* __restrict__ gcb, int ngraphs,
                                                     const int* __restrict__ urp,
                                                     const int* const* __restrict__ glcol,
                                                     u32* __restrict__ rowx, int* __restrict__ ucol,
                                                     int* __restrict__ err) {
    static_assert(US_SLOTS % US_SUB == 0, "sub-chunks tile a chunk");
    __shared__ int srow[US_SUB];
    __shared__ u64 sprobe[256 / GLT_WAVE];
    __shared__ int64_t slo;
    const int b = blockIdx.x / (US_SLOTS / US_SUB), t = threadIdx.x;   // chunk b, one sub-chunk of it
    int glo = 0, ghi = ngraphs;   // the chunk's graph: the last g with gcb[g] <= b
    while (ghi - glo > 1) {
        const int mid = (glo + ghi) >> 1;
        if (gcb[mid] <= b) glo = mid; else ghi = mid;
    }
    const int g = glo;
    const int64_t v0 = vb[g], ng = vb[g + 1] - v0, s0 = sb[g];
    const int64_t j0 = (int64_t)(b - gcb[g]) * US_SLOTS;
    const int64_t j1 = min(j0 + US_SLOTS, sb[g + 1] - s0);
    const int* lc = glcol[g];
    int bad = 0;
    {
        const int64_t q0 = j0 + (int64_t)(blockIdx.x % (US_SLOTS / US_SUB)) * US_SUB;
        if (q0 >= j1) return;   // past the graph's last entry (whole workgroup)
        const int64_t c0 = s0 + q0, c1 = s0 + min(q0 + US_SUB, j1);   // union entries [c0, c1)
        // the row holding entry c0: the last row of the graph with offset <= c0 (the graph's
        // first offset is its slot base s0 <= c0), by rounds of 256 probes at once
        int64_t lo = v0, hi = v0 + ng;   // urp[lo] <= c0; the answer lies in [lo, hi)
        while (hi - lo > 1) {
            const int64_t step = (hi - lo + 255) / 256;
            const int64_t p = lo + (int64_t)t * step;
            const bool le = p < hi && (int64_t)urp[p] <= c0;   // probes <= c0 form a prefix
            const u64 m = __ballot(le);
            if (glt_lane() == 0) sprobe[t / GLT_WAVE] = m;
            __syncthreads();
            int cntle = 0;
            for (int w = 0; w < 256 / GLT_WAVE; w++) cntle += __popcll(sprobe[w]);
            __syncthreads();
            const int64_t nlo = lo + (int64_t)(cntle - 1) * step;   // the last probe <= c0
            hi = min(hi, nlo + step);
            lo = nlo;
        }
        if (t == 0) slo = lo;
        for (int i = t; i < US_SUB; i += 256) srow[i] = -1;
        __syncthreads();
        for (int64_t r = slo + t; r < v0 + ng; r += 256) {
            const int64_t rb = urp[r], re = urp[r + 1];
            if (rb >= c1) break;   // offsets ascend: every later row starts past the sub-chunk too
            const int64_t e0 = rb > c0 ? rb : c0, e1 = re < c1 ? re : c1;
            for (int64_t e = e0; e < e1; e++) srow[e - c0] = (int)r;
        }
        __syncthreads();
        for (int64_t e = c0 + t; e < c1; e += 256) {
            const int v = srow[e - c0];
            const int c = lc[e - s0];
            rowx[e + 1] = (u32)(v + 1);
            if (v < 0 || c < 0 || c >= ng) {
                bad |= ERR_RANGE;
                ucol[e] = (int)v0;
            } else {
                ucol[e] = (int)(v0 + c);
                if (v0 + c == v) bad |= ERR_SELF;
            }
        }
    }
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
}

int glt_union_build(const Dev& d, int* urp, int* ucol, hipStream_t st) {
    (void)ucol;
    (void)hipMemsetAsync(d.err, 0, ERR_WORDS * sizeof(int), st);
    if (d.ngraphs <= 0) return 0;
    hipLaunchKernelGGL(k_union_rows, dim3(d.ngraphs), dim3(256), 0, st, d.gvb, d.gsb, d.glrp, urp, d.gid, d.err);
    launch_fill<int>(urp + d.n, 1, d.S, st);
    return 0;
}

// ---------------------------------------------------------------------------------------
// P1 / P2 / P3
// ---------------------------------------------------------------------------------------
// P1 sort keys: the degree; in a batch (graph, degree), so that every graph's vertices keep
// the contiguous rank range of their union ids, degree-ordered inside it.
__global__ void k_iota_keys(const int* __restrict__ deg, const int* __restrict__ gid, int degbits, int n,
                            u64* __restrict__ keys, u32* __restrict__ vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        keys[i] = (gid ? ((u64)(u32)gid[i] << degbits) : 0ull) | (u64)(u32)deg[i];
        vals[i] = (u32)i;
    }
}

// Rank i -> original id; also appends i to the list of its row's sort class.  In a batch
// also rank i's graph and the end of that graph's rank range (graphs keep contiguous ranges,
// the ones their packed vertices had).
template <int R>
__global__ __launch_bounds__(256) void k_apply_order(const u32* __restrict__ sorted_ids, const int* __restrict__ deg,
                                                     int n, int* __restrict__ order, int* __restrict__ rank,
                                                     int* __restrict__ ndeg, const int* __restrict__ gid,
                                                     int* __restrict__ ngid, const int64_t* __restrict__ gvb,
                                                     int* __restrict__ vtop, int* __restrict__ rlist,
                                                     int* __restrict__ rcnt) {
    int cls[R], idx[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = (blockIdx.x * R + r) * 256 + threadIdx.x;
        cls[r] = -1;
        idx[r] = i;
        if (i < n) {
            const int x = (int)sorted_ids[i];
            order[i] = x;
            rank[x] = i;
            ndeg[i] = deg[x];
            if (ngid) {
                ngid[i] = gid[x];
                vtop[i] = (int)gvb[gid[x] + 1];
            }
            cls[r] = row_class(deg[x]);
        }
    }
    block_append<RS_N, R>(rcnt, rlist, n, cls, idx);
}

// P2 without a global sort: row x of the caller's CSR becomes row rank[x] with the same
// length, so every entry goes straight to nrp[rank[x]] + (its offset within the row), keyed by
// its neighbour's rank and carrying its caller index; then each row is sorted on its own.
// Also sets the "upward in caller ids" flag whose prefix sum numbers the caller's edges.
template <typename RP>
__global__ __launch_bounds__(256) void k_place(const RP* __restrict__ rp, const u32* __restrict__ rowx,
                                               const int* __restrict__ col, int64_t S, const int* __restrict__ rank,
                                               const int* __restrict__ nrp, u32* __restrict__ key,
                                               u32* __restrict__ val, int* __restrict__ nsrow,
                                               u32* __restrict__ upflag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const int x = (int)rowx[s + 1] - 1;
    const int y = col[s];
    const int r = rank[x];
    const int64_t pos = (int64_t)nrp[r] + (s - (int64_t)rp[x]);
    key[pos] = (u32)rank[y];
    nsrow[pos] = r;
    if (val) {   // per-edge output: the caller's slot rides along, and upward slots are flagged
        val[pos] = (u32)s;
        upflag[s] = (y > x) ? 1u : 0u;
    }
}

#define PAD_KEY 0xffffffffu   // sorts after every rank (ranks are < 2^31)

// The row sorts below order each relabelled row by neighbour rank in place (keys at the
// row's own positions of the relabelled column array), carrying the caller's slot index when
// KV (per-edge output needs it), and flag equal neighbours side by side: duplicate entries.
__device__ __forceinline__ void flag_dups(int bad, int* err) {
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
}

// Rows of 2..RT_MAX entries: one thread per row, bitonic network over RT_MAX registers.
template <bool KV>
__global__ __launch_bounds__(256) void k_sort_tiny(const int* __restrict__ list, int cnt, const int* __restrict__ nrp,
                                                   u32* __restrict__ key, u32* __restrict__ val,
                                                   int* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < cnt) {
        const int r = list[i];
        const int b = nrp[r], len = nrp[r + 1] - b;
        u32 k[RT_MAX], v[RT_MAX];
#pragma unroll
        for (int j = 0; j < RT_MAX; j++) {
            k[j] = (j < len) ? key[b + j] : PAD_KEY;
            if (KV) v[j] = (j < len) ? val[b + j] : 0u;
        }
#pragma unroll
        for (int kk = 2; kk <= RT_MAX; kk <<= 1) {
#pragma unroll
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
#pragma unroll
                for (int a = 0; a < RT_MAX; a++) {
                    const int c = a ^ jj;
                    if (c > a) {
                        const bool up = (a & kk) == 0;
                        if ((k[a] > k[c]) == up) {
                            const u32 tk = k[a]; k[a] = k[c]; k[c] = tk;
                            if (KV) { const u32 tv = v[a]; v[a] = v[c]; v[c] = tv; }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RT_MAX; j++)
            if (j < len) {
                key[b + j] = k[j];
                if (KV) val[b + j] = v[j];
                if (j > 0 && k[j] == k[j - 1]) bad = ERR_DUP;
            }
    }
    flag_dups(bad, err);
}

// Rows of RT_MAX+1..RW_MAX entries: one wavefront per row, bitonic over the lanes.
template <bool KV>
__global__ __launch_bounds__(256) void k_sort_wave(const int* __restrict__ list, int cnt, const int* __restrict__ nrp,
                                                   u32* __restrict__ key, u32* __restrict__ val,
                                                   int* __restrict__ err) {
    const int i = blockIdx.x * (256 / GLT_WAVE) + threadIdx.x / GLT_WAVE;
    if (i >= cnt) return;   // whole wavefronts
    const int l = glt_lane();
    const int r = list[i];
    const int b = nrp[r], len = nrp[r + 1] - b;
    u32 k = (l < len) ? key[b + l] : PAD_KEY;
    u32 v = (KV && l < len) ? val[b + l] : 0u;
#pragma unroll
    for (int kk = 2; kk <= GLT_WAVE; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const u32 ok = __shfl_xor(k, jj, GLT_WAVE);
            const u32 ov = KV ? __shfl_xor(v, jj, GLT_WAVE) : 0u;
            const bool up = (l & kk) == 0;
            const bool lower = (l & jj) == 0;
            // lower lane of an ascending pair keeps the minimum, upper the maximum
            const bool take = lower ? ((k > ok) == up) : ((k < ok) == up);
            if (take) { k = ok; v = ov; }
        }
    }
    const u32 prev = __shfl_up(k, 1, GLT_WAVE);
    if (l < len) {
        key[b + l] = k;
        if (KV) val[b + l] = v;
    }
    flag_dups((l > 0 && l < len && prev == k) ? ERR_DUP : 0, err);
}

// Rows of RW_MAX+1..RM_MAX entries: one wavefront per row (four rows per workgroup), bitonic
// in the wavefront's own LDS.  A wavefront's LDS accesses complete in issue order, so its
// stages need no workgroup barrier.
template <bool KV>
__global__ __launch_bounds__(256) void k_sort_wmid(const int* __restrict__ list, int cnt, const int* __restrict__ nrp,
                                                   u32* __restrict__ key, u32* __restrict__ val,
                                                   int* __restrict__ err) {
    constexpr int NW = 256 / GLT_WAVE;
    __shared__ u32 skw[NW][RM_MAX], svw[NW][KV ? RM_MAX : 1];
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
    const int i = blockIdx.x * NW + w;
    if (i >= cnt) return;   // whole wavefronts
    u32* sk = skw[w];
    u32* sv = svw[KV ? w : 0];
    const int r = list[i];
    const int b = nrp[r], len = nrp[r + 1] - b;
    int P = 2 * RW_MAX;
    while (P < len) P <<= 1;   // <= RM_MAX
    for (int j = l; j < P; j += GLT_WAVE) {
        sk[j] = (j < len) ? key[b + j] : PAD_KEY;
        if (KV) sv[j] = (j < len) ? val[b + j] : 0u;
    }
    wave_sync();
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int q = l; q < P / 2; q += GLT_WAVE) {
                const int lo = ((q & ~(jj - 1)) << 1) | (q & (jj - 1));
                const int hi = lo + jj;
                const bool up = (lo & kk) == 0;
                const u32 a = sk[lo], c = sk[hi];
                if ((a > c) == up) {
                    sk[lo] = c; sk[hi] = a;
                    if (KV) { const u32 tv = sv[lo]; sv[lo] = sv[hi]; sv[hi] = tv; }
                }
            }
            wave_sync();
        }
    }
    int bad = 0;
    for (int j = l; j < len; j += GLT_WAVE) {
        key[b + j] = sk[j];
        if (KV) val[b + j] = sv[j];
        if (j > 0 && sk[j] == sk[j - 1]) bad = ERR_DUP;
    }
    flag_dups(bad, err);
}

// Rows of RM_MAX+1..RB_MAX entries: one workgroup per row, bitonic in LDS.
template <bool KV>
__global__ __launch_bounds__(256) void k_sort_blk(const int* __restrict__ list, int cnt, const int* __restrict__ nrp,
                                                  u32* __restrict__ key, u32* __restrict__ val,
                                                  int* __restrict__ err) {
    __shared__ u32 sk[RB_MAX], sv[KV ? RB_MAX : 1];
    const int t = threadIdx.x;
    const int r = list[blockIdx.x];
    const int b = nrp[r], len = nrp[r + 1] - b;
    int P = 2 * RW_MAX;
    while (P < len) P <<= 1;   // <= RB_MAX
    for (int j = t; j < P; j += 256) {
        sk[j] = (j < len) ? key[b + j] : PAD_KEY;
        if (KV) sv[j] = (j < len) ? val[b + j] : 0u;
    }
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int q = t; q < P / 2; q += 256) {
                const int lo = ((q & ~(jj - 1)) << 1) | (q & (jj - 1));
                const int hi = lo + jj;
                const bool up = (lo & kk) == 0;
                const u32 a = sk[lo], c = sk[hi];
                if ((a > c) == up) {
                    sk[lo] = c; sk[hi] = a;
                    if (KV) { const u32 tv = sv[lo]; sv[lo] = sv[hi]; sv[hi] = tv; }
                }
            }
            __syncthreads();
        }
    }
    int bad = 0;
    for (int j = t; j < len; j += 256) {
        key[b + j] = sk[j];
        if (KV) val[b + j] = sv[j];
        if (j > 0 && sk[j] == sk[j - 1]) bad = ERR_DUP;
    }
    flag_dups(bad, err);
}

// Rows longer than RB_MAX: one 1024-thread workgroup per row, stable LSD radix passes over
// `bits` key bits, ping-ponging between (kA, vA) and (kB, vB) at the row's own positions;
// the result ends in (kA, vA).  The passes are as few as digits of at most SB_DMAX bits
// allow (20-bit ranks: two passes of 10 bits), the digits as even as possible.  Each pass:
// a digit histogram, its exclusive scan, then tiles of 1024 entries in order, ranked
// within each wavefront by ballots and across wavefronts by per-wavefront digit counts.
#define SB_T 1024
#define SB_DMAX 10
#define SB_NB (1 << SB_DMAX)
template <bool KV>
__global__ __launch_bounds__(SB_T) void k_sort_big(const int* __restrict__ list, int cnt, const int* __restrict__ nrp,
                                                   u32* __restrict__ kA, u32* __restrict__ vA, u32* __restrict__ kB,
                                                   u32* __restrict__ vB, int bits, int* __restrict__ err) {
    static_assert(SB_NB <= SB_T, "one bucket per thread in the bucket loops");
    __shared__ u32 base[SB_NB];
    __shared__ u32 wcnt[SB_T / GLT_WAVE][SB_NB];
    __shared__ u32 sscan[SB_T / GLT_WAVE];
    const int t = threadIdx.x, lane = glt_lane(), w = t / GLT_WAVE;
    const int r = list[blockIdx.x];
    const int64_t b = nrp[r];
    const int len = nrp[r + 1] - (int)b;
    u32* ki = kA + b; u32* vi = KV ? vA + b : nullptr;
    u32* ko = kB + b; u32* vo = KV ? vB + b : nullptr;
    const u64 lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (GLT_WAVE - lane));
    const int npass_all = (bits + SB_DMAX - 1) / SB_DMAX;
    const int dbits = npass_all > 0 ? (bits + npass_all - 1) / npass_all : 0;   // <= SB_DMAX
    const u32 dmask = (1u << dbits) - 1u;
    const int nb = 1 << dbits;                                                   // buckets in use
    int npass = 0;
    for (int shift = 0; shift < bits; shift += dbits, npass++) {
        if (t < nb) {
            base[t] = 0;
            for (int q = 0; q < SB_T / GLT_WAVE; q++) wcnt[q][t] = 0;
        }
        __syncthreads();
        for (int j = t; j < len; j += SB_T) atomicAdd(&base[(ki[j] >> shift) & dmask], 1u);
        __syncthreads();
        u32 tot;
        const u32 ex = block_excl_scan<u32, SB_T>(t < nb ? base[t] : 0u, sscan, tot);
        if (t < nb) base[t] = ex;
        __syncthreads();
        for (int j0 = 0; j0 < len; j0 += SB_T) {
            const int j = j0 + t;
            const bool valid = j < len;
            const u32 k = valid ? ki[j] : 0u;
            const u32 v = (KV && valid) ? vi[j] : 0u;
            const u32 d = (k >> shift) & dmask;
            u64 peers = __ballot(valid);
            for (int bit = 0; bit < dbits; bit++) {
                const u64 bb = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? bb : ~bb;
            }
            const u32 rk = (u32)__popcll(peers & lt_mask);
            if (valid && rk == 0) wcnt[w][d] = (u32)__popcll(peers);
            __syncthreads();
            if (valid) {
                u32 off = base[d];
                for (int q = 0; q < w; q++) off += wcnt[q][d];
                ko[off + rk] = k;
                if (KV) vo[off + rk] = v;
            }
            __syncthreads();
            if (t < nb) {
                u32 add = 0;
                for (int q = 0; q < SB_T / GLT_WAVE; q++) { add += wcnt[q][t]; wcnt[q][t] = 0; }
                base[t] += add;
            }
            __syncthreads();
        }
        u32* tk = ki; ki = ko; ko = tk;
        u32* tv = vi; vi = vo; vo = tv;
    }
    // ki holds the sorted row (every thread's writes of the last pass are ordered before
    // these reads by the pass's final barrier)
    int bad = 0;
    for (int j = t; j < len; j += SB_T) {
        const u32 k = ki[j];
        if (j > 0 && ki[j - 1] == k) bad = ERR_DUP;
        if (npass & 1) {
            kA[b + j] = k;
            if (KV) vA[b + j] = vi[j];
        }
    }
    flag_dups(bad, err);
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

// Per vertex x: (first upward slot nrp[x] + dlo[x], row end nrp[x + 1], optr[x], order[x]),
// one 16-byte record, so that an entry's scattered look-up of its other endpoint reads one
// line instead of four arrays.
__global__ __launch_bounds__(256) void k_vinfo(const int* __restrict__ nrp, const int* __restrict__ dlo,
                                               const int* __restrict__ optr, const int* __restrict__ order, int n,
                                               int4* __restrict__ vinf) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) vinf[x] = make_int4(nrp[x] + dlo[x], nrp[x + 1], optr[x], order[x]);
}

// One thread per relabelled entry s of row x (y = ncol[s]).  Upward entries (y > x) copy
// themselves into the oriented CSR at index k and clear the edge's accumulators; downward
// entries find their edge's k by binary search of x in N+(y), map themselves to k and (PE:
// per-edge output) name the caller's edge id of k.  Global counts need only t and u of an
// edge, and no caller edge ids.  Every entry also records, for the wedge pass, the oriented
// range [k0, k1) of the tops of the wedges x - y - top (top above x: all of N+(y) when y > x,
// the part after x when y < x) and adds its length to wcnt[x] (runs of one row summed in the
// wavefront first); upward entries add |N+(y)| to the triangle-list totals of x's path.
template <bool PE>
__global__ __launch_bounds__(256) void k_edge_index(const int* __restrict__ ncol, const int* __restrict__ nsrow,
                                                    const int4* __restrict__ vinf, const u32* __restrict__ oslot,
                                                    const u32* __restrict__ upx, int64_t S, int m,
                                                    int* __restrict__ ocol, int* __restrict__ s2k,
                                                    int* __restrict__ eid2k, EdgeArrays ea,
                                                    const int* __restrict__ kwp,
                                                    int2* __restrict__ wb, u64* __restrict__ wcnt,
                                                    u64* __restrict__ wspread, int* __restrict__ err) {
    __shared__ u64 red[2][256 / GLT_WAVE];
    const int64_t s64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    u64 wc = 0, lw = 0, lb = 0;
    int x = 0x7fffffff;
    if (s64 < S) {
        const int s = (int)s64;
        x = nsrow[s];
        const int4 vx = vinf[x];
        const int ub = vx.x;
        const int y = ncol[s];
        const int4 vy = vinf[y];
        const int y1 = vy.z + (vy.y - vy.x);   // optr[y + 1]
        int2 r = make_int2(0, 0);
        if (s >= ub) {
            // upward x -> y: its own oriented slot
            const int k = vx.z + (s - ub);
            if (k >= m) {
                bad = ERR_ASYM;   // more upward than downward entries
            } else {
                ocol[k] = y;
                s2k[s] = k;
                ea.t[k] = 0; ea.u[k] = x;
                if (PE) {
                    // narrow edges: K and P are u32 words and one word of g holds g and sigma;
                    // wide edges: four u64 words (EdgeArrays)
                    const int kw = *kwp;
                    if (k < kw) {
                        reinterpret_cast<u32*>(ea.K)[k] = 0;
                        reinterpret_cast<u32*>(ea.P)[k] = 0;
                        ea.g[k] = 0;
                    } else {
                        wide_arrays(ea, m, kw);
                        ea.Kw[k - kw] = 0; ea.Pw[k - kw] = 0; ea.gw[k - kw] = 0; ea.sw[k - kw] = 0;
                    }
                }
                r = make_int2(vy.z, y1);
                const int dpx = vx.y - vx.x;   // |N+(x)|: the triangle-pass path of x
                if (dpx >= 2 && dpx <= 64) lw = (u64)(y1 - vy.z);
                else if (dpx > 64) lb = (u64)(y1 - vy.z);
            }
        } else {
            // downward x -> y (y ranked below x): the edge's slot is x's place in N+(y), a short
            // list (out-degrees are bounded by sqrt(2m) in the degree order)
            const int yb = vy.x, ye = vy.y;
            const int sp = lower_bound_i32(ncol, yb, ye, x);
            const int k = vy.z + (sp - yb);
            if (sp >= ye || ncol[sp] != x || k >= m) {
                bad = ERR_ASYM;
            } else {
                s2k[s] = k;
                r = make_int2(k + 1, y1);
                if (PE) {
                    const u32 j = (vx.w < vy.w) ? oslot[s] : oslot[sp];
                    const u32 eid = upx[j];
                    if (eid >= (u32)m) bad = ERR_ASYM;
                    else eid2k[eid] = k;
                }
            }
        }
        wb[s] = r;
        wc = (u64)(r.y - r.x);
    }
    bool last;
    const u64 run = seg_sum_last(wc, x, last);
    if (last && run && x != 0x7fffffff) atomicAdd(&wcnt[x], run);
    const u64 ta = wave_sum(lw), tb = wave_sum(lb);
    if (glt_lane() == 0) { red[0][threadIdx.x / GLT_WAVE] = ta; red[1][threadIdx.x / GLT_WAVE] = tb; }
    bad = wave_or(bad);
    if (glt_lane() == 0 && bad) atomicOr(err, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 sa = 0, sb = 0;
        for (int q = 0; q < 256 / GLT_WAVE; q++) { sa += red[0][q]; sb += red[1][q]; }
        u64* line = wspread + (blockIdx.x & (GSPREAD - 1)) * WSPREAD_WORDS;
        if (sa) atomicAdd(&line[2], sa);
        if (sb) atomicAdd(&line[3], sb);
    }
}

// Triangle / gather pass buckets by out-degree s = |N+(x)|.
__device__ __forceinline__ int tbucket(int s) {
    if (s < 2) return -1;
    if (s <= 64) return TB_WAVE;
    if (s <= 256) return TB_BLK1;
    if (s <= TB_LDS_ROWS) return TB_BLK2;
    return TB_GLOBAL;
}


// Triangle-pass lists by out-degree; toff[x] = C(|N+(x)|, 2), the most triangles x can be
// the lowest vertex of (its prefix sum places x's triangle records).
template <int R>
__global__ __launch_bounds__(256) void k_tbuckets(const int* __restrict__ optr, int n, int* __restrict__ tlist,
                                                  int* __restrict__ counts, int* __restrict__ tmax,
                                                  u64* __restrict__ toff) {
    __shared__ int bmax[TB_N];
    if (threadIdx.x < TB_N) bmax[threadIdx.x] = 0;
    int cls[R], idx[R], sz[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int x = (blockIdx.x * R + r) * 256 + threadIdx.x;
        const int s = (x < n) ? optr[x + 1] - optr[x] : 0;
        cls[r] = (x < n) ? tbucket(s) : -1;
        idx[r] = x;
        sz[r] = s;
        if (x < n) toff[x] = (u64)s * (u64)(s > 0 ? s - 1 : 0) / 2;
    }
    block_append<TB_N, R, APAD_STRIDE>(counts, tlist, n, cls, idx);   // (its barriers also order bmax's clearing)
#pragma unroll
    for (int r = 0; r < R; r++) {
        for (int q = 0; q < TB_N; q++) {
            const int mx = wave_max(cls[r] == q ? sz[r] : 0);
            if (glt_lane() == 0 && mx) atomicMax(&bmax[q], mx);
        }
    }
    __syncthreads();
    if (threadIdx.x < TB_N && bmax[threadIdx.x]) atomicMax(&tmax[threadIdx.x * APAD_STRIDE], bmax[threadIdx.x]);
}

// Bucket the wedge pass by wedges per vertex; per-class wedge totals go to the spread work
// counters.
template <int R>
__global__ __launch_bounds__(256) void k_wappend(const u64* __restrict__ wcnt, int n, int wave_max, int mid_max,
                                                 int wg_max, int* __restrict__ wlist, int* __restrict__ counts,
                                                 u64* __restrict__ wspread) {
    int cls[R], idx[R];
    u64 wsum[WB_N], wmax[WB_N];
#pragma unroll
    for (int c = 0; c < WB_N; c++) { wsum[c] = 0; wmax[c] = 0; }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int y = (blockIdx.x * R + r) * 256 + threadIdx.x;
        const u64 wc = (y < n) ? wcnt[y] : 0;
        const int q = (wc == 0)                 ? -1
                      : (wc <= (u64)wave_max)   ? WB_WAVE
                      : (wc <= (u64)mid_max)    ? WB_MID
                      : (wc <= (u64)wg_max)     ? WB_BLK
                                                : WB_HUGE;
        cls[r] = q;
        idx[r] = y;
#pragma unroll
        for (int c = 0; c < WB_N; c++) {
            wsum[c] += q == c ? wc : 0ull;
            wmax[c] = (q == c && wc > wmax[c]) ? wc : wmax[c];
        }
    }
    block_append<WB_N, R, APAD_STRIDE>(counts, wlist, n, cls, idx);
    // wedges per class, summed per workgroup: wspread words 0 (wave), 1 (workgroup), 4 (mid),
    // 5 (huge); the most wedges of one bottom per class: words 8 + class
    __shared__ u64 cred[WB_N][256 / GLT_WAVE];
    __shared__ u64 cmax[WB_N][256 / GLT_WAVE];
#pragma unroll
    for (int c = 0; c < WB_N; c++) {
        const u64 v = wave_sum(wsum[c]);
        const u64 x = ::wave_max(wmax[c]);   // (the parameter wave_max shadows it)
        if (glt_lane() == 0) {
            cred[c][threadIdx.x / GLT_WAVE] = v;
            cmax[c][threadIdx.x / GLT_WAVE] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x < WB_N) {
        u64 t = 0, x = 0;
        for (int k = 0; k < 256 / GLT_WAVE; k++) {
            t += cred[threadIdx.x][k];
            x = cmax[threadIdx.x][k] > x ? cmax[threadIdx.x][k] : x;
        }
        const int wd = threadIdx.x == WB_WAVE ? 0 : threadIdx.x == WB_MID ? 4 : threadIdx.x == WB_BLK ? 1 : 5;
        u64* line = wspread + (blockIdx.x & (GSPREAD - 1)) * WSPREAD_WORDS;
        if (t) atomicAdd(&line[wd], t);
        if (x) atomicMax(&line[8 + threadIdx.x], x);
    }
}

// The work-list counters and the triangle lists' largest out-degrees, accumulated APAD_STRIDE
// ints apart (each in its own stretch of memory, so that the atomics of 10^5 workgroups on
// different counters proceed in parallel instead of queueing on one line), into their
// places in counts.
__global__ void k_pad_to_counts(const int* __restrict__ apad, int* __restrict__ counts) {
    const int t = threadIdx.x;
    if (t < TB_N) counts[t] = apad[t * APAD_STRIDE];                                     // triangle lists
    if (t < WB_N) counts[TB_N + t] = apad[(TB_N + t) * APAD_STRIDE];                     // wedge lists
    if (t < TB_N) counts[TB_N + WB_N + t] = apad[(TB_N + WB_N + t) * APAD_STRIDE];       // largest out-degrees
}

// Split point kw of the per-edge accumulators (EdgeArrays): the first oriented edge whose
// lower endpoint u has d_u dmax >= 2^31 (a suffix in the degree order); m if there is none;
// 0 (every edge wide) when that suffix holds more than m / 4 edges, too many for the wide
// arrays' place in the sig buffer.  Batches (global counts only) use no accumulator: m.
// wide_degree > 0 lowers the threshold to that degree (tests: more edges take the wide path;
// a lower threshold only widens edges, which is always exact).
__global__ void k_wide_split(const int* __restrict__ ndeg, const int* __restrict__ optr, int n, int m,
                             int batched, int wide_degree, int* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int kw = m;
    if (!batched && n > 0) {
        const int64_t dmax = ndeg[n - 1];   // ranks ascend by degree
        if (dmax > 0) {
            int64_t dw = ((int64_t)1 << 31) / dmax + ((((int64_t)1 << 31) % dmax) ? 1 : 0);   // ceil
            if (wide_degree > 0 && wide_degree < dw) dw = wide_degree;
            int lo = 0, hi = n;               // first rank with degree >= dw
            while (lo < hi) {
                const int mid = lo + (hi - lo) / 2;
                if ((int64_t)ndeg[mid] < dw) lo = mid + 1;
                else hi = mid;
            }
            kw = optr[lo];
            if ((int64_t)(m - kw) * 4 > (int64_t)m) kw = 0;
        }
    }
    *out = kw;
}

// ---------------------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------------------
template <int R>
static void launch_check_rows(const Dev& d, const void* rp, int rp64, u32* cnt, hipStream_t st) {
    if (rp64)
        hipLaunchKernelGGL((k_check_rows<int64_t, R>), dim3(nblk(d.n, 256 * R)), dim3(256), 0, st,
                           (const int64_t*)rp, d.n, (int64_t)d.S, d.deg, cnt, d.err);
    else
        hipLaunchKernelGGL((k_check_rows<int32_t, R>), dim3(nblk(d.n, 256 * R)), dim3(256), 0, st,
                           (const int32_t*)rp, d.n, (int64_t)d.S, d.deg, cnt, d.err);
}

int glt_prep_validate(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st) {
    // err[0] error bits (kept from the union build in batched mode), err[1] max degree
    if (d.ngraphs <= 0) (void)hipMemsetAsync(d.err, 0, ERR_WORDS * sizeof(int), st);
    if (d.n <= 0) return 0;
    const int64_t S = d.S;
    // the row of every entry: in a batch written per chunk from the union offsets, else a
    // prefix sum of row-start counts
    u32* cnt = d.ngraphs > 0 ? nullptr : d.rowx;
    if (cnt) launch_fill<u32>(d.rowx, S + 1, 0u, st);
    if (tile_r(d.n) == 1) launch_check_rows<1>(d, rp, rp64, cnt, st);
    else launch_check_rows<TILE_R_LARGE>(d, rp, rp64, cnt, st);
    if (cnt) launch_excl_scan<u32, u32>(d.rowx, d.rowx, S + 1, d.rs_tmp, (u32*)nullptr, st);
    if (S > 0) {
        if (d.ngraphs > 0)   // the union's rows and columns, checked as they are written
            hipLaunchKernelGGL(k_union_slots, dim3(d.ncchunks * (US_SLOTS / US_SUB)), dim3(256), 0, st, d.gvb, d.gsb, d.gcb, d.ngraphs,
                               (const int*)rp, d.glcol, d.rowx, (int*)col, d.err);
        else
            hipLaunchKernelGGL(k_check_cols, dim3(nblk(S, 256)), dim3(256), 0, st, d.rowx, col, d.n, S, d.err);
    }
    unsigned gm = nblk(d.n, 256);
    if (gm > 2048) gm = 2048;
    hipLaunchKernelGGL(k_max_deg, dim3(gm), dim3(256), 0, st, d.deg, d.n, d.err + 1);
    return 0;
}

static inline int bitlen(u64 x) { int b = 0; while (x) { b++; x >>= 1; } return b; }

template <bool KV>
static void launch_row_sorts(const Dev& d, const int* rows, const int* rlist, u32* key, u32* val, hipStream_t st) {
    const int n = d.n;
    if (rows[RS_TINY] > 0)
        hipLaunchKernelGGL(k_sort_tiny<KV>, dim3(nblk(rows[RS_TINY], 256)), dim3(256), 0, st,
                           rlist + (int64_t)RS_TINY * n, rows[RS_TINY], d.nrp, key, val, d.err);
    if (rows[RS_WAVE] > 0)
        hipLaunchKernelGGL(k_sort_wave<KV>, dim3(nblk(rows[RS_WAVE], 256 / GLT_WAVE)), dim3(256), 0, st,
                           rlist + (int64_t)RS_WAVE * n, rows[RS_WAVE], d.nrp, key, val, d.err);
    if (rows[RS_WMID] > 0)
        hipLaunchKernelGGL(k_sort_wmid<KV>, dim3(nblk(rows[RS_WMID], 256 / GLT_WAVE)), dim3(256), 0, st,
                           rlist + (int64_t)RS_WMID * n, rows[RS_WMID], d.nrp, key, val, d.err);
    if (rows[RS_BLK] > 0)
        hipLaunchKernelGGL(k_sort_blk<KV>, dim3(rows[RS_BLK]), dim3(256), 0, st, rlist + (int64_t)RS_BLK * n,
                           rows[RS_BLK], d.nrp, key, val, d.err);
    if (rows[RS_BIG] > 0)
        hipLaunchKernelGGL(k_sort_big<KV>, dim3(rows[RS_BIG]), dim3(SB_T), 0, st, rlist + (int64_t)RS_BIG * n,
                           rows[RS_BIG], d.nrp, key, val, (u32*)d.key1, d.val1, bitlen((u64)(n > 1 ? n - 1 : 1)),
                           d.err);
}

int glt_prep_build(const Dev& d, const void* rp, int rp64, const int* col, hipStream_t st, const int* vinfo) {
    static_assert(RS_N <= TL_SEGS, "row-sort lists live in the triangle-pass list area");
    const int n = d.n;
    const int64_t S = d.S;
    const int maxdeg = vinfo[0];
    const int* rows = vinfo + 1;   // rows per sort class
    (void)hipMemsetAsync(d.counts, 0, sizeof(int) * CNT_WORDS, st);
    launch_fill<u64>(d.work, NWORK, 0ull, st);
    launch_fill<u64>(d.wspread, (int64_t)GSPREAD * WSPREAD_WORDS, 0ull, st);
    if (n == 0) return 0;
    // P1: stable sort of vertices by degree (ties keep id order); rows listed by sort class
    const int degbits = bitlen((u64)maxdeg);
    const int keybits = degbits + (d.ngraphs > 0 ? bitlen((u64)(d.ngraphs - 1)) : 0);
    hipLaunchKernelGGL(k_iota_keys, dim3(nblk(n, 256)), dim3(256), 0, st, d.deg, d.ngraphs > 0 ? d.gid : nullptr,
                       degbits, n, d.key0, d.val0);
    const int cur = launch_radix_sort(d.key0, d.val0, d.key1, d.val1, n, keybits, d.rs_counts, d.rs_tmp, st);
    int* rlist = d.tlist;
    int* rcnt = d.err + 2 + RS_N;
    if (tile_r(n) == 1)
        hipLaunchKernelGGL(k_apply_order<1>, dim3(nblk(n, 256)), dim3(256), 0, st, cur ? d.val1 : d.val0, d.deg, n,
                           d.order, d.rank, d.ndeg, d.gid, d.ngid, d.gvb, d.vtop, rlist, rcnt);
    else
        hipLaunchKernelGGL(k_apply_order<TILE_R_LARGE>, dim3(nblk(n, 256 * TILE_R_LARGE)), dim3(256), 0, st,
                           cur ? d.val1 : d.val0, d.deg, n, d.order, d.rank, d.ndeg, d.gid, d.ngid, d.gvb, d.vtop,
                           rlist, rcnt);
    // relabelled CSR offsets
    launch_excl_scan<int, int>(d.ndeg, d.nrp, n, d.itmp, d.nrp + n, st);
    // P2: entries placed in their relabelled rows, then every row sorted by neighbour rank in
    // place in the relabelled column array (duplicates flagged by the sorts).  The caller's
    // slot index is carried and the caller's edges numbered only for per-edge output.
    u32* key = (u32*)d.ncol;
    u32* val = d.per_edge ? d.val0 : nullptr;
    if (S > 0) {
        if (rp64)
            hipLaunchKernelGGL(k_place<int64_t>, dim3(nblk(S, 256)), dim3(256), 0, st, (const int64_t*)rp, d.rowx, col,
                               S, d.rank, d.nrp, key, val, d.nsrow, d.upx);
        else
            hipLaunchKernelGGL(k_place<int32_t>, dim3(nblk(S, 256)), dim3(256), 0, st, (const int32_t*)rp, d.rowx, col,
                               S, d.rank, d.nrp, key, val, d.nsrow, d.upx);
        if (d.per_edge) {
            launch_excl_scan<u32, u32>(d.upx, d.upx, S, d.rs_tmp, (u32*)nullptr, st);
            launch_row_sorts<true>(d, rows, rlist, key, val, st);
        } else {
            launch_row_sorts<false>(d, rows, rlist, key, val, st);
        }
    }
    const u32* oslot = val;
    // P3: orientation
    int* dplus = d.itmp + scan_tmp_elems(S + n + 1);  // past the scan scratch
    hipLaunchKernelGGL(k_dlo, dim3(nblk(n, 256)), dim3(256), 0, st, d.nrp, d.ncol, n, d.dlo, dplus);
    launch_excl_scan<int, int>(dplus, d.optr, n, d.itmp, d.optr + n, st);
    hipLaunchKernelGGL(k_wide_split, dim3(1), dim3(64), 0, st, d.ndeg, d.optr, n, d.m, d.ngraphs > 0 ? 1 : 0,
                       d.wide_degree, d.counts + CNT_KW);
    launch_fill<u64>(d.wcnt, n, 0ull, st);
    if (S > 0) {
        hipLaunchKernelGGL(k_vinfo, dim3(nblk(n, 256)), dim3(256), 0, st, d.nrp, d.dlo, d.optr, d.order, n, d.vinf);
        if (d.per_edge)
            hipLaunchKernelGGL(k_edge_index<true>, dim3(nblk(S, 256)), dim3(256), 0, st, d.ncol, d.nsrow, d.vinf,
                               oslot, d.upx, S, d.m, d.ocol, d.s2k, d.eid2k, d.e, d.counts + CNT_KW, d.wb, d.wcnt,
                               d.wspread,
                               d.err);
        else
            hipLaunchKernelGGL(k_edge_index<false>, dim3(nblk(S, 256)), dim3(256), 0, st, d.ncol, d.nsrow, d.vinf,
                               oslot, d.upx, S, d.m, d.ocol, d.s2k, d.eid2k, d.e, d.counts + CNT_KW, d.wb, d.wcnt,
                               d.wspread,
                               d.err);
    }
    // work lists
    // The counting passes walk these lists in append order.  Appended in tiles of 2048
    // consecutive ranks (TILE_R_LARGE sub-tiles) instead of 256, the batch's triangle wave
    // path and mid wedge class ran 2.6 and 1.4 ms slower, more than the 3 ms that fewer
    // counter atomics save here, so the work lists keep one sub-tile per workgroup.
    const int mid_max = d.wedge_mid_max < 65535 ? d.wedge_mid_max : 65535;
    launch_fill<int>(d.apad, (int64_t)APAD_SLOTS * APAD_STRIDE, 0, st);
    hipLaunchKernelGGL(k_tbuckets<1>, dim3(nblk(n, 256)), dim3(256), 0, st, d.optr, n, d.tlist, d.apad,
                       d.apad + (TB_N + WB_N) * APAD_STRIDE, d.toff);
    launch_excl_scan<u64, u64>(d.toff, d.toff, n, d.tmp64, d.toff + n, st);
    hipLaunchKernelGGL(k_wappend<1>, dim3(nblk(n, 256)), dim3(256), 0, st, d.wcnt, n, d.wedge_wave_max, mid_max,
                       d.wedge_wg_max, d.wlist, d.apad + TB_N * APAD_STRIDE, d.wspread);
    hipLaunchKernelGGL(k_pad_to_counts, dim3(1), dim3(64), 0, st, d.apad, d.counts);
    return 0;
}
