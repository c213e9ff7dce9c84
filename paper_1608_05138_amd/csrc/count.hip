// count.hip -- the counting passes on the relabelled, oriented graph.
//
// The paper derives every 2-, 3- and 4-node count from per-edge triangles |T|, 4-cliques
// and 4-cycles (Section 4.5) plus degrees.  Its GPU kernels (Alg. 2-4) search T and S_u
// of every edge by binary search, which repeats work on hub edges.  Here the same per-edge
// quantities are produced by passes that touch each triangle, 4-clique and ranked wedge a
// bounded number of times:
//
//  * triangle pass (per lowest-ranked vertex a): S = N+(a).  The adjacency among S is
//    built as bit rows M_i; every edge (b_i, b_j) of M is a triangle (a, b_i, b_j) and
//    popcount(M_i & M_j) is the number of 4-cliques {a, b_i, b_j, c} with a lowest.  Each
//    triangle credits its three edges once (t), each 4-clique its six edges once (K).
//  * gather pass (per-edge mode): for every triangle (a, b_i, b_j) the third vertex w of
//    each edge contributes t(w,u) + t(w,v) and d_w, giving the number of edges between T and
//    S_u or S_v and the degree sum over T needed for the remaining per-edge 4-node counts
//    (every per-edge count depends on the T-S_u and T-S_v edge counts only through their sum).
//  * wedge pass (per bottom vertex y): wedges y - w - x with x ranked above y and w are
//    grouped by x in an LDS hash; a group of c wedges closes C(c,2) 4-cycles whose top
//    vertex is x.  Each wedge's edges (y,w) and (w,x) lie on c-1 of them, which gives every
//    edge's number of (non-induced) 4-cycles P; the induced count is
//    P - 2K - a_u - a_v (edges S_u-S_v, the paper's cycle count).
//  * vertex pass: triangles at each vertex and sums of neighbour degrees.
//  * combine: the 13 per-edge counts and the unrestricted sums C3..C16 (Section 4.5),
//    reduced exactly in 128 bits; the global frequencies (Section 4.6) follow on the host.
//
// Work items inside a wavefront are enumerated as flattened (source, offset) pairs with
// consecutive lanes on consecutive entries of one out-list, so credits to the edges of one
// list are coalesced atomics to consecutive oriented indices, and credits that all lanes of
// a run send to the same source are first summed with a segmented wave reduction.
#include "glt_internal.h"

// Per-edge accumulators K, P, g, sig are 64-bit, or 32-bit when the maximum degree bounds
// every value below 2^32 (the host picks AT); the buffers are sized for 64-bit either way.
template <typename AT>
__device__ __forceinline__ void acc_add(u64* base, int64_t k, u64 v) {
    atomicAdd(&((AT*)base)[k], (AT)v);
}
template <typename AT>
__device__ __forceinline__ u64 acc_get(const u64* base, int64_t k) {
    return (u64)((const AT*)base)[k];
}

#define TB_THREADS 256

// ---------------------------------------------------------------------------------------
// triangle / 4-clique pass, out-degree 2..64: one wavefront per vertex, M rows in one word
// ---------------------------------------------------------------------------------------
// Membership of a vertex id in S = N+(a) (s <= 64) through a 128-entry LDS hash per
// wavefront mapping id -> position in S.
#define SH_SIZE 128
__device__ __forceinline__ u32 shash(int x) { return ((u32)x * 2654435761u >> 9) & (SH_SIZE - 1); }

__device__ __forceinline__ void sh_insert(int* hk, unsigned char* hv, int x, int pos) {
    u32 h = shash(x);
    while (atomicCAS(&hk[h], -1, x) != -1) h = (h + 1) & (SH_SIZE - 1);
    hv[h] = (unsigned char)pos;
}

__device__ __forceinline__ int sh_find(const int* hk, const unsigned char* hv, int x) {
    u32 h = shash(x);
    while (true) {
        const int k = hk[h];
        if (k == x) return hv[h];
        if (k == -1) return -1;
        h = (h + 1) & (SH_SIZE - 1);
    }
}

template <bool PE, typename AT>
__global__ __launch_bounds__(TB_THREADS) void k_tri_wave(const int* __restrict__ list, int nlist,
                                                        const int* __restrict__ optr, const int* __restrict__ ocol,
                                                        EdgeArrays e, u64* __restrict__ gsum,
                                                        const int* __restrict__ ngid) {
    __shared__ int sOb[4][GLT_WAVE];
    __shared__ int sPre[4][GLT_WAVE];
    __shared__ u64 sM[4][GLT_WAVE];
    __shared__ u64 sK[4][GLT_WAVE];
    __shared__ int hk[4][SH_SIZE];
    __shared__ unsigned char hv[4][SH_SIZE];
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
    const int idx = blockIdx.x * 4 + w;
    const bool active = idx < nlist;
    const int a = active ? list[idx] : 0;
    const int o0 = active ? optr[a] : 0;
    const int s = active ? optr[a + 1] - o0 : 0;
    int b = 0, ob = 0, db = 0;
    if (l < s) { b = ocol[o0 + l]; ob = optr[b]; db = optr[b + 1] - ob; }
    const int inc = wave_incl_scan(db);
    const int total = __shfl(inc, GLT_WAVE - 1, GLT_WAVE);
    sOb[w][l] = ob; sPre[w][l] = inc - db; sM[w][l] = 0; sK[w][l] = 0;
    hk[w][l] = -1; hk[w][l + GLT_WAVE] = -1;
    __syncthreads();
    if (l < s) sh_insert(hk[w], hv[w], b, l);
    __syncthreads();
    // build the adjacency rows among S
    int i = 0;
    for (int q0 = 0; q0 < total; q0 += GLT_WAVE) {
        const int q = q0 + l;
        if (q < total) {
            i = advance_idx(sPre[w], s, q, i);
            const int x = ocol[sOb[w][i] + (q - sPre[w][i])];
            const int j = sh_find(hk[w], hv[w], x);
            if (j >= 0) {
                atomicOr(&sM[w][i], 1ull << j);
                atomicOr(&sM[w][j], 1ull << i);
            }
        }
    }
    __syncthreads();
    u64 k4 = 0;
    i = 0;
    for (int q0 = 0; q0 < total; q0 += GLT_WAVE) {
        const int q = q0 + l;
        int key = 0x7fffffff;
        u64 tk = 0;
        if (q < total) {
            i = advance_idx(sPre[w], s, q, i);
            key = i;
            const int k = sOb[w][i] + (q - sPre[w][i]);
            const int j = sh_find(hk[w], hv[w], ocol[k]);
            if (j >= 0) {
                tk = (u64)__popcll(sM[w][i] & sM[w][j]);
                atomicAdd(&e.t[k], 1u);
                if (PE && tk) {
                    acc_add<AT>(e.K, k, tk);
                    atomicAdd(&sK[w][j], tk);
                }
                k4 += tk;
            }
        }
        if (PE) {
            bool last;
            const u64 ssum = seg_sum_last(tk, key, last);
            if (last && ssum) atomicAdd(&sK[w][key], ssum);
        }
    }
    __syncthreads();
    if (l < s) {
        const u32 tl = (u32)__popcll(sM[w][l]);
        if (tl) atomicAdd(&e.t[o0 + l], tl);
        if (PE) {
            const u64 kl = sK[w][l] >> 1;
            if (kl) acc_add<AT>(e.K, o0 + l, kl);
        }
    }
    k4 = wave_sum(k4);
    if (l == 0 && k4) atomicAdd(&gsum[(ngid ? ngid[a] : 0) * NSUMS + S_K4x3], k4);
}

// ---------------------------------------------------------------------------------------
// triangle / 4-clique pass, out-degree > 64: one workgroup per vertex, M rows of W words
// in LDS (GM = false) or in a per-workgroup global slab (GM = true)
// ---------------------------------------------------------------------------------------
template <bool PE, bool GM, typename AT>
__global__ __launch_bounds__(TB_THREADS) void k_tri_blk(const int* __restrict__ list, int nlist, int smax,
                                                       const int* __restrict__ optr, const int* __restrict__ ocol,
                                                       EdgeArrays e, u64* __restrict__ gsum,
                                                       u32* __restrict__ gscratch, const int* __restrict__ ngid) {
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    __shared__ int sScan[TB_THREADS / GLT_WAVE];
    __shared__ u64 sRed[TB_THREADS / GLT_WAVE];
    u64* sK = (u64*)dyn;
    int* sS = (int*)(sK + smax);
    int* sOb = sS + smax;
    int* sPre = sOb + smax;
    const int Wmax = (smax + 31) / 32;
    u32* M = GM ? gscratch + (int64_t)blockIdx.x * smax * Wmax : (u32*)(sPre + smax);
    const int tid = threadIdx.x;
    const int a = list[blockIdx.x];
    const int o0 = optr[a];
    const int s = optr[a + 1] - o0;
    const int W = (s + 31) / 32;
    // S, its out-list offsets and the exclusive prefix of their lengths
    int carry = 0;
    for (int c0 = 0; c0 < s; c0 += TB_THREADS) {
        const int i = c0 + tid;
        int db = 0;
        if (i < s) {
            const int b = ocol[o0 + i];
            const int ob = optr[b];
            db = optr[b + 1] - ob;
            sS[i] = b; sOb[i] = ob; sK[i] = 0;
        }
        int tot;
        const int ex = block_excl_scan<int, TB_THREADS>(db, sScan, tot);
        if (i < s) sPre[i] = carry + ex;
        carry += tot;
    }
    const int total = carry;
    for (int q = tid; q < s * W; q += TB_THREADS) M[q] = 0;
    __syncthreads();
    int ii = 0;
    for (int q = tid; q < total; q += TB_THREADS) {
        const int i = ii = advance_idx(sPre, s, q, ii);
        const int x = ocol[sOb[i] + (q - sPre[i])];
        const int j = lower_bound_i32(sS, i + 1, s, x);
        if (j < s && sS[j] == x) {
            atomicOr(&M[i * W + (j >> 5)], 1u << (j & 31));
            atomicOr(&M[j * W + (i >> 5)], 1u << (i & 31));
        }
    }
    __syncthreads();
    u64 k4 = 0;
    // every thread runs the same number of iterations so the wave reductions see full waves
    const int rounds = (total + TB_THREADS - 1) / TB_THREADS;
    ii = 0;
    for (int r = 0; r < rounds; r++) {
        const int q = r * TB_THREADS + tid;
        int i = 0x7fffffff;
        u64 tk = 0;
        if (q < total) {
            i = ii = advance_idx(sPre, s, q, ii);
            const int k = sOb[i] + (q - sPre[i]);
            const int x = ocol[k];
            const int j = lower_bound_i32(sS, i + 1, s, x);
            if (j < s && sS[j] == x) {
                for (int wd = 0; wd < W; wd++) tk += (u64)__popc(M[i * W + wd] & M[j * W + wd]);
                atomicAdd(&e.t[k], 1u);
                if (PE && tk) {
                    acc_add<AT>(e.K, k, tk);
                    atomicAdd(&sK[j], tk);
                }
                k4 += tk;
            }
        }
        if (PE) {
            bool last;
            const u64 ssum = seg_sum_last(tk, i, last);
            if (last && ssum) atomicAdd(&sK[i], ssum);
        }
    }
    __syncthreads();
    for (int i = tid; i < s; i += TB_THREADS) {
        u32 tl = 0;
        for (int wd = 0; wd < W; wd++) tl += (u32)__popc(M[i * W + wd]);
        if (tl) atomicAdd(&e.t[o0 + i], tl);
        if (PE) {
            const u64 kl = sK[i] >> 1;
            if (kl) acc_add<AT>(e.K, o0 + i, kl);
        }
    }
    k4 = wave_sum(k4);
    if (glt_lane() == 0) sRed[tid / GLT_WAVE] = k4;
    __syncthreads();
    if (tid == 0) {
        u64 tot = 0;
        for (int q = 0; q < TB_THREADS / GLT_WAVE; q++) tot += sRed[q];
        if (tot) atomicAdd(&gsum[(ngid ? ngid[a] : 0) * NSUMS + S_K4x3], tot);
    }
}

static inline size_t tri_blk_lds(int smax, bool gm) {
    const int Wmax = (smax + 31) / 32;
    size_t b = (size_t)smax * (8 + 4 + 4 + 4);
    if (!gm) b += (size_t)smax * Wmax * 4;
    return b;
}

// ---------------------------------------------------------------------------------------
// gather pass (per-edge mode): for every triangle (a, b_i, b_j), a lowest
// ---------------------------------------------------------------------------------------
// Credits of one triangle found at (i, j, edge k = (b_i, b_j)):
//   edge (a, b_i): g += t(a, b_j) + t(b_i, b_j), sig += d(b_j)   [local, run-summed]
//   edge (a, b_j): g += t(a, b_i) + t(b_i, b_j), sig += d(b_i)   [local]
//   edge (b_i, b_j): g += t(a, b_i) + t(a, b_j), sig += d(a)     [global, coalesced]
template <typename AT>
__device__ __forceinline__ void gather_credit(bool found, int i, int j, int k, const u32* sT, const int* sD, int da,
                                              EdgeArrays& e, u64* sG, u64* sSg) {
    u64 gi = 0, di = 0;
    if (found) {
        const u64 tij = e.t[k];
        const u64 tai = sT[i], taj = sT[j];
        gi = taj + tij;
        di = (u64)sD[j];
        atomicAdd(&sG[j], tai + tij);
        atomicAdd(&sSg[j], (u64)sD[i]);
        acc_add<AT>(e.g, k, tai + taj);
        acc_add<AT>(e.sig, k, (u64)da);
    }
    // lanes of a wavefront hold non-decreasing i (idle lanes a larger sentinel, zero values)
    bool last;
    const u64 a1 = seg_sum_last(gi, i, last);
    const u64 a3 = seg_sum_last(di, i, last);
    if (last) {
        if (a1) atomicAdd(&sG[i], a1);
        if (a3) atomicAdd(&sSg[i], a3);
    }
}

template <typename AT>
__global__ __launch_bounds__(TB_THREADS) void k_gather_wave(const int* __restrict__ list, int nlist,
                                                           const int* __restrict__ optr,
                                                           const int* __restrict__ ocol,
                                                           const int* __restrict__ ndeg, EdgeArrays e) {
    __shared__ int sOb[4][GLT_WAVE];
    __shared__ int sPre[4][GLT_WAVE];
    __shared__ u32 sT[4][GLT_WAVE];
    __shared__ int sD[4][GLT_WAVE];
    __shared__ u64 sG[4][GLT_WAVE];
    __shared__ u64 sSg[4][GLT_WAVE];
    __shared__ int hk[4][SH_SIZE];
    __shared__ unsigned char hv[4][SH_SIZE];
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
    const int idx = blockIdx.x * 4 + w;
    const bool active = idx < nlist;
    const int a = active ? list[idx] : 0;
    const int o0 = active ? optr[a] : 0;
    const int s = active ? optr[a + 1] - o0 : 0;
    const int da = active ? ndeg[a] : 0;
    int b = 0, ob = 0, db = 0;
    u32 tb = 0;
    int degb = 0;
    if (l < s) {
        b = ocol[o0 + l]; ob = optr[b]; db = optr[b + 1] - ob;
        tb = e.t[o0 + l]; degb = ndeg[b];
    }
    const int inc = wave_incl_scan(db);
    const int total = __shfl(inc, GLT_WAVE - 1, GLT_WAVE);
    sOb[w][l] = ob; sPre[w][l] = inc - db; sT[w][l] = tb; sD[w][l] = degb;
    sG[w][l] = 0; sSg[w][l] = 0;
    hk[w][l] = -1; hk[w][l + GLT_WAVE] = -1;
    __syncthreads();
    if (l < s) sh_insert(hk[w], hv[w], b, l);
    __syncthreads();
    int i = 0;
    for (int q0 = 0; q0 < total; q0 += GLT_WAVE) {
        const int q = q0 + l;
        int key = 0x3fffffff, j = -1, k = 0;
        if (q < total) {
            i = advance_idx(sPre[w], s, q, i);
            key = i;
            k = sOb[w][i] + (q - sPre[w][i]);
            j = sh_find(hk[w], hv[w], ocol[k]);
        }
        gather_credit<AT>(j >= 0, key, j, k, sT[w], sD[w], da, e, sG[w], sSg[w]);
    }
    __syncthreads();
    if (l < s) {
        if (sG[w][l]) acc_add<AT>(e.g, o0 + l, sG[w][l]);
        if (sSg[w][l]) acc_add<AT>(e.sig, o0 + l, sSg[w][l]);
    }
}

template <bool GM, typename AT>
__global__ __launch_bounds__(TB_THREADS) void k_gather_blk(const int* __restrict__ list, int nlist, int smax,
                                                          const int* __restrict__ optr,
                                                          const int* __restrict__ ocol,
                                                          const int* __restrict__ ndeg, EdgeArrays e,
                                                          u64* __restrict__ gslab) {
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    __shared__ int sScan[TB_THREADS / GLT_WAVE];
    int* sS = (int*)dyn;
    int* sOb = sS + smax;
    int* sPre = sOb + smax;
    u32* sT = (u32*)(sPre + smax);
    int* sD = (int*)(sT + smax);
    u64* sG = GM ? gslab + (int64_t)blockIdx.x * 2 * smax : (u64*)(sD + smax + (smax & 1));
    u64* sSg = sG + smax;
    const int tid = threadIdx.x;
    const int a = list[blockIdx.x];
    const int o0 = optr[a];
    const int s = optr[a + 1] - o0;
    const int da = ndeg[a];
    int carry = 0;
    for (int c0 = 0; c0 < s; c0 += TB_THREADS) {
        const int i = c0 + tid;
        int db = 0;
        if (i < s) {
            const int b = ocol[o0 + i];
            const int ob = optr[b];
            db = optr[b + 1] - ob;
            sS[i] = b; sOb[i] = ob; sT[i] = e.t[o0 + i]; sD[i] = ndeg[b];
            sG[i] = 0; sSg[i] = 0;
        }
        int tot;
        const int ex = block_excl_scan<int, TB_THREADS>(db, sScan, tot);
        if (i < s) sPre[i] = carry + ex;
        carry += tot;
    }
    const int total = carry;
    __syncthreads();
    const int rounds = (total + TB_THREADS - 1) / TB_THREADS;
    int ii = 0;
    for (int r = 0; r < rounds; r++) {
        const int q = r * TB_THREADS + tid;
        int i = 0x3fffffff, j = 0, k = 0;
        bool found = false;
        if (q < total) {
            i = ii = advance_idx(sPre, s, q, ii);
            k = sOb[i] + (q - sPre[i]);
            const int x = ocol[k];
            j = lower_bound_i32(sS, i + 1, s, x);
            found = (j < s && sS[j] == x);
        }
        gather_credit<AT>(found, i, j, k, sT, sD, da, e, sG, sSg);
    }
    __syncthreads();
    for (int i = tid; i < s; i += TB_THREADS) {
        if (sG[i]) acc_add<AT>(e.g, o0 + i, sG[i]);
        if (sSg[i]) acc_add<AT>(e.sig, o0 + i, sSg[i]);
    }
}

static inline size_t gather_blk_lds(int smax, bool gm) {
    return (size_t)(smax + 1) * 4 * 5 + (gm ? 0 : (size_t)smax * 8 * 2);
}

// ---------------------------------------------------------------------------------------
// wedge / 4-cycle pass
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ u32 hslot(int x, u32 mask) { return ((u32)x * 2654435761u >> 7) & mask; }

// Range of oriented indices k (x = ocol[k]) of the wedges y - w - x for CSR slot s of row y.
__device__ __forceinline__ void wedge_range(int y, int s, const int* __restrict__ ncol, const int* __restrict__ optr,
                                            const int* __restrict__ s2k, int& w, int& k0, int& k1) {
    w = ncol[s];
    k1 = optr[w + 1];
    k0 = (w > y) ? optr[w] : s2k[s] + 1;
}

#define WW_TABLE 512   // per-wave hash entries; wave-path vertices have <= WW_TABLE/2 wedges

// One wavefront per bottom vertex y with at most WW_TABLE/2 wedges.
template <bool PE, typename AT>
__global__ __launch_bounds__(256) void k_wedge_wave(const int* __restrict__ list, int nlist,
                                                    const int* __restrict__ nrp, const int* __restrict__ ncol,
                                                    const int* __restrict__ optr, const int* __restrict__ ocol,
                                                    const int* __restrict__ s2k, EdgeArrays e,
                                                    u64* __restrict__ gsum, const int* __restrict__ ngid) {
    __shared__ int hkey[4][WW_TABLE];
    __shared__ u32 hcnt[4][WW_TABLE];
    __shared__ int sK0[4][GLT_WAVE];
    __shared__ int sPre[4][GLT_WAVE];
    __shared__ u32 sB[4][GLT_WAVE];
    const int w4 = threadIdx.x / GLT_WAVE, l = glt_lane();
    const int idx = blockIdx.x * 4 + w4;
    const bool active = idx < nlist;
    const int y = active ? list[idx] : 0;
    const int rb = active ? nrp[y] : 0, re = active ? nrp[y + 1] : 0;
    for (int q = l; q < WW_TABLE; q += GLT_WAVE) { hkey[w4][q] = -1; hcnt[w4][q] = 0; }
    __syncthreads();
    const u32 mask = WW_TABLE - 1;
    // count phase
    for (int c0 = rb; c0 < re; c0 += GLT_WAVE) {
        const int s = c0 + l;
        int wv = 0, k0 = 0, k1 = 0;
        if (s < re) wedge_range(y, s, ncol, optr, s2k, wv, k0, k1);
        const int len = k1 - k0;
        const int inc = wave_incl_scan(len);
        const int tot = __shfl(inc, GLT_WAVE - 1, GLT_WAVE);
        const int nsrc = min(GLT_WAVE, re - c0);
        wave_sync();
        sK0[w4][l] = k0; sPre[w4][l] = inc - len;
        wave_sync();
        int ii = 0;
        for (int q0 = 0; q0 < tot; q0 += GLT_WAVE) {
            const int q = q0 + l;
            if (q < tot) {
                const int i = ii = advance_idx(sPre[w4], nsrc, q, ii);
                const int x = ocol[sK0[w4][i] + (q - sPre[w4][i])];
                u32 h = hslot(x, mask);
                while (true) {
                    int cur = hkey[w4][h];
                    if (cur == -1) cur = atomicCAS(&hkey[w4][h], -1, x);
                    if (cur == -1 || cur == x) { atomicAdd(&hcnt[w4][h], 1u); break; }
                    h = (h + 1) & mask;
                }
            }
        }
    }
    __syncthreads();
    u64 c4 = 0;
    for (int q = l; q < WW_TABLE; q += GLT_WAVE) {
        const u64 c = hcnt[w4][q];
        c4 += c * (c - (c > 0)) / 2;
    }
    // credit phase
    if (PE) {
        for (int c0 = rb; c0 < re; c0 += GLT_WAVE) {
            const int s = c0 + l;
            int wv = 0, k0 = 0, k1 = 0;
            if (s < re) wedge_range(y, s, ncol, optr, s2k, wv, k0, k1);
            const int len = k1 - k0;
            const int inc = wave_incl_scan(len);
            const int tot = __shfl(inc, GLT_WAVE - 1, GLT_WAVE);
            const int nsrc = min(GLT_WAVE, re - c0);
            wave_sync();
            sK0[w4][l] = k0; sPre[w4][l] = inc - len; sB[w4][l] = 0;
            wave_sync();
            int ii = 0;
            for (int q0 = 0; q0 < tot; q0 += GLT_WAVE) {
                const int q = q0 + l;
                int i = 0x7fffffff;
                u32 c = 0;
                if (q < tot) {
                    i = ii = advance_idx(sPre[w4], nsrc, q, ii);
                    const int k = sK0[w4][i] + (q - sPre[w4][i]);
                    const int x = ocol[k];
                    u32 h = hslot(x, mask);
                    while (hkey[w4][h] != x) h = (h + 1) & mask;
                    c = hcnt[w4][h] - 1;
                    if (c) acc_add<AT>(e.P, k, (u64)c);
                }
                bool last;
                const u32 ssum = seg_sum_last(c, i, last);
                if (last && ssum) atomicAdd(&sB[w4][i], ssum);
            }
            wave_sync();
            if (s < re && sB[w4][l]) acc_add<AT>(e.P, s2k[s], (u64)sB[w4][l]);
        }
    }
    c4 = wave_sum(c4);
    if (l == 0 && c4) atomicAdd(&gsum[(ngid ? ngid[y] : 0) * NSUMS + S_NC4], c4);
}

#define WB_THREADS 256
#define WB_TABLE 2048           // LDS hash entries per workgroup (tops below the dense window)
#define WB_DENSE 8192           // dense LDS counters for the highest-ranked tops
#define WB_STACK 96

// One workgroup per bottom vertex with many wedges.  Tops x in the dense window
// [n - dense, n) (the highest-ranked vertices, which close most wedges of a degree-ordered
// graph) are counted in a dense LDS array; lower tops go to an LDS hash.  The x-range
// [lo, hi) is split in halves whenever its hashed part holds more distinct tops than
// `limit` (<= WB_TABLE/2); a range is credited only after its count phase completed without
// overflow, so no wedge is credited twice.
template <bool PE, typename AT>
__global__ __launch_bounds__(WB_THREADS) void k_wedge_blk(const int* __restrict__ list, int nlist, int n, int limit,
                                                         int dense, const int* __restrict__ nrp,
                                                         const int* __restrict__ ncol, const int* __restrict__ optr,
                                                         const int* __restrict__ ocol, const int* __restrict__ s2k,
                                                         EdgeArrays e, u64* __restrict__ gsum,
                                                         const int* __restrict__ ngid) {
    __shared__ u32 dcnt[WB_DENSE];
    __shared__ int hkey[WB_TABLE];
    __shared__ u32 hcnt[WB_TABLE];
    __shared__ int sK0[WB_THREADS];
    __shared__ int sPre[WB_THREADS];
    __shared__ u64 sB[WB_THREADS];
    __shared__ int sScan[WB_THREADS / GLT_WAVE];
    __shared__ u64 sRed[WB_THREADS / GLT_WAVE];
    __shared__ int stLo[WB_STACK], stHi[WB_STACK];
    __shared__ int sp, distinct, ovf;
    const int tid = threadIdx.x;
    const int y = list[blockIdx.x];
    const int rb = nrp[y], re = nrp[y + 1];
    const u32 mask = WB_TABLE - 1;
    const int base = max(n - dense, y + 1);   // tops >= base are counted densely
    const int nd = n - base;                  // dense counters in use (<= dense <= WB_DENSE)
    if (tid == 0) { stLo[0] = y + 1; stHi[0] = n; sp = 1; }
    u64 c4 = 0;
    __syncthreads();
    while (true) {
        if (sp == 0) break;
        const int lo = stLo[sp - 1], hi = stHi[sp - 1];
        const bool full = (lo == y + 1) && (hi == n);
        __syncthreads();
        if (tid == 0) { sp--; distinct = 0; ovf = 0; }
        for (int q = tid; q < WB_TABLE; q += WB_THREADS) { hkey[q] = -1; hcnt[q] = 0; }
        for (int q = tid; q < nd; q += WB_THREADS) dcnt[q] = 0;
        __syncthreads();
        // count phase
        for (int c0 = rb; c0 < re; c0 += WB_THREADS) {
            const int s = c0 + tid;
            int wv = 0, k0 = 0, k1 = 0;
            if (s < re) {
                wedge_range(y, s, ncol, optr, s2k, wv, k0, k1);
                if (!full) {
                    k0 = lower_bound_i32(ocol, k0, k1, lo);
                    k1 = lower_bound_i32(ocol, k0, k1, hi);
                }
            }
            const int len = k1 - k0;
            int tot;
            const int ex = block_excl_scan<int, WB_THREADS>(len, sScan, tot);
            const int nsrc = min(WB_THREADS, re - c0);
            sK0[tid] = k0; sPre[tid] = ex;
            __syncthreads();
            int ii = 0;
            for (int q = tid; q < tot; q += WB_THREADS) {
                if (*(volatile int*)&ovf) break;
                const int i = ii = advance_idx(sPre, nsrc, q, ii);
                const int x = ocol[sK0[i] + (q - sPre[i])];
                if (x >= base) {
                    atomicAdd(&dcnt[x - base], 1u);
                    continue;
                }
                u32 h = hslot(x, mask);
                while (true) {
                    int cur = hkey[h];
                    if (cur == -1) {
                        cur = atomicCAS(&hkey[h], -1, x);
                        if (cur == -1) {
                            atomicAdd(&hcnt[h], 1u);
                            if (atomicAdd(&distinct, 1) + 1 > limit) ovf = 1;
                            break;
                        }
                    }
                    if (cur == x) { atomicAdd(&hcnt[h], 1u); break; }
                    h = (h + 1) & mask;
                }
            }
            __syncthreads();
        }
        if (ovf) {
            if (tid == 0) {
                const int mid = lo + (hi - lo) / 2;
                stLo[sp] = mid; stHi[sp] = hi; sp++;
                stLo[sp] = lo; stHi[sp] = mid; sp++;
            }
            __syncthreads();
            continue;
        }
        for (int q = tid; q < WB_TABLE; q += WB_THREADS) {
            const u64 c = hcnt[q];
            c4 += c * (c - (c > 0)) / 2;
        }
        for (int q = tid; q < nd; q += WB_THREADS) {
            const u64 c = dcnt[q];
            c4 += c * (c - (c > 0)) / 2;
        }
        if (PE) {
            for (int c0 = rb; c0 < re; c0 += WB_THREADS) {
                const int s = c0 + tid;
                int wv = 0, k0 = 0, k1 = 0;
                if (s < re) {
                    wedge_range(y, s, ncol, optr, s2k, wv, k0, k1);
                    if (!full) {
                        k0 = lower_bound_i32(ocol, k0, k1, lo);
                        k1 = lower_bound_i32(ocol, k0, k1, hi);
                    }
                }
                const int len = k1 - k0;
                int tot;
                const int ex = block_excl_scan<int, WB_THREADS>(len, sScan, tot);
                const int nsrc = min(WB_THREADS, re - c0);
                sK0[tid] = k0; sPre[tid] = ex; sB[tid] = 0;
                __syncthreads();
                const int rounds = (tot + WB_THREADS - 1) / WB_THREADS;
                int ii = 0;
                for (int r = 0; r < rounds; r++) {
                    const int q = r * WB_THREADS + tid;
                    int i = 0x7fffffff;
                    u64 c = 0;
                    if (q < tot) {
                        i = ii = advance_idx(sPre, nsrc, q, ii);
                        const int k = sK0[i] + (q - sPre[i]);
                        const int x = ocol[k];
                        if (x >= base) {
                            c = dcnt[x - base] - 1;
                        } else {
                            u32 h = hslot(x, mask);
                            while (hkey[h] != x) h = (h + 1) & mask;
                            c = hcnt[h] - 1;
                        }
                        if (c) acc_add<AT>(e.P, k, c);
                    }
                    bool last;
                    const u64 ssum = seg_sum_last(c, i, last);
                    if (last && ssum) atomicAdd(&sB[i], ssum);
                }
                __syncthreads();
                if (s < re && sB[tid]) acc_add<AT>(e.P, s2k[s], sB[tid]);
                __syncthreads();
            }
        }
        __syncthreads();
    }
    c4 = wave_sum(c4);
    if (glt_lane() == 0) sRed[tid / GLT_WAVE] = c4;
    __syncthreads();
    if (tid == 0) {
        u64 tot = 0;
        for (int q = 0; q < WB_THREADS / GLT_WAVE; q++) tot += sRed[q];
        if (tot) atomicAdd(&gsum[(ngid ? ngid[y] : 0) * NSUMS + S_NC4], tot);
    }
}

// ---------------------------------------------------------------------------------------
// vertex pass: per relabelled entry (x -> y) the edge's t and d_y, summed per x (runs of one
// row are summed in the wavefront first): tri[x] = 2 x (triangles at x), sdeg[x] = sum of
// neighbour degrees.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vertex(const int* __restrict__ nsrow, const int* __restrict__ ncol,
                                                const int* __restrict__ s2k, const int* __restrict__ ndeg,
                                                const u32* __restrict__ et, int64_t S, u64* __restrict__ tri,
                                                u64* __restrict__ sdeg) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u64 t = 0, sd = 0;
    int x = 0x7fffffff;
    if (s < S) {
        x = nsrow[s];
        t = et[s2k[s]];
        sd = (u64)ndeg[ncol[s]];
    }
    bool last;
    const u64 rt = seg_sum_last(t, x, last);
    const u64 rs = seg_sum_last(sd, x, last);
    if (last && x != 0x7fffffff) {
        if (rt) atomicAdd(&tri[x], rt);
        if (rs) atomicAdd(&sdeg[x], rs);
    }
}

// ---------------------------------------------------------------------------------------
// combine: per-edge counts and unrestricted sums, 128-bit per-block partials
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void add128(u64& lo, u64& hi, u64 v) {
    const u64 o = lo;
    lo += v;
    hi += (lo < o) ? 1ull : 0ull;
}

__device__ __forceinline__ void wave_sum128(u64& lo, u64& hi) {
#pragma unroll
    for (int d = GLT_WAVE / 2; d >= 1; d >>= 1) {
        const u64 olo = __shfl_xor(lo, d, GLT_WAVE);
        const u64 ohi = __shfl_xor(hi, d, GLT_WAVE);
        const u64 o = lo;
        lo += olo;
        hi += ohi + ((lo < o) ? 1ull : 0ull);
    }
}

#define CB_THREADS 256
#define CB_EPT 4
#define NCS 13

template <bool PE, typename AT>
__global__ __launch_bounds__(CB_THREADS) void k_combine(const int* __restrict__ eid2k, EdgeArrays e,
                                                        const int* __restrict__ ocol,
                                                        const int* __restrict__ ndeg, const u64* __restrict__ tri,
                                                        const u64* __restrict__ sdeg, int n, int m,
                                                        u64* __restrict__ out, u64* __restrict__ part,
                                                        int* __restrict__ err) {
    __shared__ u64 red[CB_THREADS / GLT_WAVE][NCS][2];
    u64 lo[NCS], hi[NCS];
#pragma unroll
    for (int c = 0; c < NCS; c++) { lo[c] = 0; hi[c] = 0; }
    int bad = 0;
    const int64_t e0 = (int64_t)blockIdx.x * CB_THREADS * CB_EPT;
    for (int r = 0; r < CB_EPT; r++) {
        const int64_t eid = e0 + (int64_t)r * CB_THREADS + threadIdx.x;
        if (eid >= m) break;
        const int k = eid2k[eid];
        const int u = e.u[k], v = ocol[k];
        const int64_t du = ndeg[u], dv = ndeg[v];
        const int64_t t = e.t[k];
        const int64_t su = du - 1 - t, sv = dv - 1 - t;
        const int64_t D = (int64_t)n - 2 - t - su - sv;
        int64_t K = 0, Q = 0;
        if (PE) {
            K = (int64_t)acc_get<AT>(e.K, k);
            const int64_t P = (int64_t)acc_get<AT>(e.P, k);
            const int64_t A = (int64_t)acc_get<AT>(e.g, k) - 2 * t - 4 * K;     // edges T-S_u plus T-S_v
            Q = P - 2 * K - A;                                      // edges S_u-S_v
            const int64_t sigT = (int64_t)acc_get<AT>(e.sig, k);
            const int64_t E2 = (int64_t)((tri[u] + tri[v]) >> 1) - 2 * t - 2 * K - A;   // inside S_u plus inside S_v
            const int64_t ETD = sigT - 2 * t - 2 * K - A;           // edges T-D
            const int64_t ESD = ((int64_t)sdeg[u] - dv - sigT) + ((int64_t)sdeg[v] - du - sigT) - su - sv - 2 * E2 - A -
                                2 * Q;                              // edges S_u-D plus S_v-D
            const int64_t EDD = (int64_t)m - 1 - 2 * t - su - sv - (K + E2 + A + Q + ETD + ESD);
            int64_t x[13];
            x[0] = t;
            x[1] = su + sv;
            x[2] = D;
            x[3] = K;
            x[4] = (t * (t - 1) / 2 - K) + A;
            x[5] = t * (su + sv) - A + ETD + E2;
            x[6] = Q;
            x[7] = su * (su - 1) / 2 + sv * (sv - 1) / 2 - E2;
            x[8] = (su * sv - Q) + ESD;
            x[9] = t * D - ETD;
            x[10] = EDD;
            x[11] = (su + sv) * D - ESD;
            x[12] = D * (D - 1) / 2 - EDD;
            int neg = (A < 0) | (Q < 0) | (E2 < 0) | (ETD < 0) | (ESD < 0) | (EDD < 0);
#pragma unroll
            for (int c = 0; c < 13; c++) {
                neg |= (x[c] < 0);
                out[(int64_t)c * m + eid] = (u64)x[c];
            }
            if (neg) bad = ERR_NEG;
        }
        // unrestricted counts (Section 4.5): C3,C4,C5,C7,C8,C9,C10,C11,C12,C13,C14,C15,C16
        add128(lo[0], hi[0], (u64)t);
        add128(lo[1], hi[1], (u64)(su + sv));
        add128(lo[2], hi[2], (u64)D);
        add128(lo[3], hi[3], (u64)K);
        add128(lo[4], hi[4], (u64)(t * (t - 1) / 2));
        add128(lo[5], hi[5], (u64)(t * (su + sv)));
        add128(lo[6], hi[6], (u64)Q);
        add128(lo[7], hi[7], (u64)(su * (su - 1) / 2 + sv * (sv - 1) / 2));
        add128(lo[8], hi[8], (u64)(su * sv));
        add128(lo[9], hi[9], (u64)(t * D));
        add128(lo[10], hi[10], (u64)((int64_t)m - du - dv + 1));
        add128(lo[11], hi[11], (u64)((su + sv) * D));
        add128(lo[12], hi[12], (u64)(D * (D - 1) / 2));
    }
    if (bad) atomicOr(err, bad);
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
#pragma unroll
    for (int c = 0; c < NCS; c++) {
        wave_sum128(lo[c], hi[c]);
        if (l == 0) { red[w][c][0] = lo[c]; red[w][c][1] = hi[c]; }
    }
    __syncthreads();
    if (threadIdx.x < NCS) {
        const int c = threadIdx.x;
        u64 L = 0, H = 0;
        for (int q = 0; q < CB_THREADS / GLT_WAVE; q++) {
            const u64 o = L;
            L += red[q][c][0];
            H += red[q][c][1] + ((L < o) ? 1ull : 0ull);
        }
        part[((int64_t)blockIdx.x * NCS + c) * 2] = L;
        part[((int64_t)blockIdx.x * NCS + c) * 2 + 1] = H;
    }
}

// one workgroup: final 128-bit reduction of the per-block partials
__global__ __launch_bounds__(256) void k_reduce_parts(const u64* __restrict__ part, int nparts,
                                                      u64* __restrict__ fin) {
    __shared__ u64 red[256 / GLT_WAVE][2];
    for (int c = 0; c < NCS; c++) {
        u64 lo = 0, hi = 0;
        for (int b = threadIdx.x; b < nparts; b += 256) {
            const u64 o = lo;
            lo += part[((int64_t)b * NCS + c) * 2];
            hi += part[((int64_t)b * NCS + c) * 2 + 1] + ((lo < o) ? 1ull : 0ull);
        }
        wave_sum128(lo, hi);
        if (glt_lane() == 0) { red[threadIdx.x / GLT_WAVE][0] = lo; red[threadIdx.x / GLT_WAVE][1] = hi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 L = 0, H = 0;
            for (int q = 0; q < 256 / GLT_WAVE; q++) {
                const u64 o = L;
                L += red[q][0];
                H += red[q][1] + ((L < o) ? 1ull : 0ull);
            }
            fin[2 * c] = L;
            fin[2 * c + 1] = H;
        }
        __syncthreads();
    }
}

// Batched global mode: one workgroup per graph over its edges (edge ids of graph g are
// [slot_base[g]/2, slot_base[g+1]/2) in the packed numbering), unrestricted sums with the
// graph's own n and m.
__global__ __launch_bounds__(CB_THREADS) void k_combine_graphs(const int64_t* __restrict__ vb,
                                                               const int64_t* __restrict__ sb,
                                                               const int* __restrict__ eid2k, EdgeArrays e,
                                                               const int* __restrict__ ocol,
                                                               const int* __restrict__ ndeg,
                                                               u64* __restrict__ gparts) {
    __shared__ u64 red[CB_THREADS / GLT_WAVE][NCS][2];
    const int g = blockIdx.x;
    const int64_t ng = vb[g + 1] - vb[g];
    const int64_t e0 = sb[g] / 2, e1 = sb[g + 1] / 2, mg = e1 - e0;
    u64 lo[NCS], hi[NCS];
#pragma unroll
    for (int c = 0; c < NCS; c++) { lo[c] = 0; hi[c] = 0; }
    for (int64_t eid = e0 + threadIdx.x; eid < e1; eid += CB_THREADS) {
        const int k = eid2k[eid];
        const int64_t du = ndeg[e.u[k]], dv = ndeg[ocol[k]];
        const int64_t t = e.t[k];
        const int64_t su = du - 1 - t, sv = dv - 1 - t;
        const int64_t D = ng - 2 - t - su - sv;
        add128(lo[0], hi[0], (u64)t);
        add128(lo[1], hi[1], (u64)(su + sv));
        add128(lo[2], hi[2], (u64)D);
        add128(lo[4], hi[4], (u64)(t * (t - 1) / 2));
        add128(lo[5], hi[5], (u64)(t * (su + sv)));
        add128(lo[7], hi[7], (u64)(su * (su - 1) / 2 + sv * (sv - 1) / 2));
        add128(lo[8], hi[8], (u64)(su * sv));
        add128(lo[9], hi[9], (u64)(t * D));
        add128(lo[10], hi[10], (u64)(mg - du - dv + 1));
        add128(lo[11], hi[11], (u64)((su + sv) * D));
        add128(lo[12], hi[12], (u64)(D * (D - 1) / 2));
    }
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
#pragma unroll
    for (int c = 0; c < NCS; c++) {
        wave_sum128(lo[c], hi[c]);
        if (l == 0) { red[w][c][0] = lo[c]; red[w][c][1] = hi[c]; }
    }
    __syncthreads();
    if (threadIdx.x < NCS) {
        const int c = threadIdx.x;
        u64 L = 0, H = 0;
        for (int q = 0; q < CB_THREADS / GLT_WAVE; q++) {
            const u64 o = L;
            L += red[q][c][0];
            H += red[q][c][1] + ((L < o) ? 1ull : 0ull);
        }
        gparts[((int64_t)g * NCS + c) * 2] = L;
        gparts[((int64_t)g * NCS + c) * 2 + 1] = H;
    }
}

// ---------------------------------------------------------------------------------------
// heaviest-first order of the workgroup work lists (the paper's edge order: hardest jobs
// first, Section 4.3), so the longest jobs do not start last and run alone
// ---------------------------------------------------------------------------------------
// mode 0: work = wedges of y (wcnt); mode 1: work = out-degree of x
__global__ void k_work_keys(const int* __restrict__ list, int nlist, int mode, const u64* __restrict__ wcnt,
                            const int* __restrict__ optr, u64* __restrict__ keys, u32* __restrict__ vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlist) return;
    const int x = list[i];
    const u64 w = mode == 0 ? wcnt[x] : (u64)(optr[x + 1] - optr[x]);
    keys[i] = ((1ull << 40) - 1) - (w < (1ull << 40) ? w : (1ull << 40) - 1);
    vals[i] = (u32)x;
}

__global__ void k_copy_list(const u32* __restrict__ vals, int nlist, int* __restrict__ list) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nlist) list[i] = (int)vals[i];
}

static void sort_heaviest_first(const Dev& d, int* list, int nlist, int mode, hipStream_t st) {
    if (nlist < 2) return;
    const unsigned g = (unsigned)((nlist + 255) / 256);
    hipLaunchKernelGGL(k_work_keys, dim3(g), dim3(256), 0, st, list, nlist, mode, d.wcnt, d.optr, d.key0, d.val0);
    const int cur = launch_radix_sort(d.key0, d.val0, d.key1, d.val1, nlist, 40, d.rs_counts, d.rs_tmp, st);
    hipLaunchKernelGGL(k_copy_list, dim3(g), dim3(256), 0, st, cur ? d.val1 : d.val0, nlist, list);
}

static inline int combine_blocks(int m) { return (int)(((int64_t)m + CB_THREADS * CB_EPT - 1) / (CB_THREADS * CB_EPT)); }

// ---------------------------------------------------------------------------------------
// host orchestration of the passes
// ---------------------------------------------------------------------------------------
static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <typename AT>
static void count_passes(const Dev& d, int per_edge, const int* hc, u64* out_pe, hipStream_t st, hipEvent_t* ev) {
    const int n = d.n, m = d.m;
    u64* gsum = d.gsum;                   // [graph][NSUMS]: 3 x 4-cliques and non-induced 4-cycles
    launch_fill<u64>(gsum, (int64_t)(d.ngraphs > 0 ? d.ngraphs : 1) * NSUMS, 0ull, st);
    const int* tl = d.tlist;
    const int* cnt = hc;                  // TB_N counts, WB_N counts, TB_N maxima
    const EdgeArrays e = d.e;
    for (int bkt = TB_BLK1; bkt <= TB_GLOBAL; bkt++) sort_heaviest_first(d, d.tlist + (int64_t)bkt * n, cnt[bkt], 1, st);
    sort_heaviest_first(d, d.wlist + (int64_t)WB_BLK * n, hc[TB_N + WB_BLK], 0, st);
    // triangle / 4-clique pass
    if (cnt[TB_WAVE] > 0) {
        if (per_edge)
            hipLaunchKernelGGL((k_tri_wave<true, AT>), dim3(cdiv(cnt[TB_WAVE], 4)), dim3(TB_THREADS), 0, st,
                               tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], d.optr, d.ocol, e, gsum, d.ngid);
        else
            hipLaunchKernelGGL((k_tri_wave<false, AT>), dim3(cdiv(cnt[TB_WAVE], 4)), dim3(TB_THREADS), 0, st,
                               tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], d.optr, d.ocol, e, gsum, d.ngid);
    }
    for (int bkt = TB_BLK1; bkt <= TB_GLOBAL; bkt++) {
        const int c = cnt[bkt];
        if (c <= 0) continue;
        const int smax = cnt[TB_N + WB_N + bkt];
        const bool gm = (bkt == TB_GLOBAL);
        const size_t lds = tri_blk_lds(smax, gm);
        const int* lst = tl + (int64_t)bkt * n;
        if (gm) {
            // the global slab holds one M per workgroup: launch in groups that fit it
            const int64_t per = (int64_t)smax * ((smax + 31) / 32);
            int64_t grp = d.gscratch_words / per;
            if (grp < 1) grp = 1;
            for (int64_t off = 0; off < c; off += grp) {
                const int cc = (int)((c - off < grp) ? (c - off) : grp);
                if (per_edge)
                    hipLaunchKernelGGL((k_tri_blk<true, true, AT>), dim3(cc), dim3(TB_THREADS), lds, st, lst + off, cc,
                                       smax, d.optr, d.ocol, e, gsum, d.gscratch, d.ngid);
                else
                    hipLaunchKernelGGL((k_tri_blk<false, true, AT>), dim3(cc), dim3(TB_THREADS), lds, st, lst + off, cc,
                                       smax, d.optr, d.ocol, e, gsum, d.gscratch, d.ngid);
            }
        } else {
            if (per_edge)
                hipLaunchKernelGGL((k_tri_blk<true, false, AT>), dim3(c), dim3(TB_THREADS), lds, st, lst, c, smax,
                                   d.optr, d.ocol, e, gsum, d.gscratch, d.ngid);
            else
                hipLaunchKernelGGL((k_tri_blk<false, false, AT>), dim3(c), dim3(TB_THREADS), lds, st, lst, c, smax,
                                   d.optr, d.ocol, e, gsum, d.gscratch, d.ngid);
        }
    }
    if (ev) (void)hipEventRecord(ev[0], st);
    // gather pass
    if (per_edge) {
        if (cnt[TB_WAVE] > 0)
            hipLaunchKernelGGL(k_gather_wave<AT>, dim3(cdiv(cnt[TB_WAVE], 4)), dim3(TB_THREADS), 0, st,
                               tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], d.optr, d.ocol, d.ndeg, e);
        for (int bkt = TB_BLK1; bkt <= TB_GLOBAL; bkt++) {
            const int c = cnt[bkt];
            if (c <= 0) continue;
            const int smax = cnt[TB_N + WB_N + bkt];
            const int* lst = tl + (int64_t)bkt * n;
            if (bkt == TB_GLOBAL) {
                const int64_t per = 2 * (int64_t)smax * 2;   // u64 accumulators, in u32 words
                int64_t grp = d.gscratch_words / per;
                if (grp < 1) grp = 1;
                for (int64_t off = 0; off < c; off += grp) {
                    const int cc = (int)((c - off < grp) ? (c - off) : grp);
                    hipLaunchKernelGGL((k_gather_blk<true, AT>), dim3(cc), dim3(TB_THREADS), gather_blk_lds(smax, true), st,
                                       lst + off, cc, smax, d.optr, d.ocol, d.ndeg, e, (u64*)d.gscratch);
                }
            } else {
                hipLaunchKernelGGL((k_gather_blk<false, AT>), dim3(c), dim3(TB_THREADS), gather_blk_lds(smax, false), st,
                                   lst, c, smax, d.optr, d.ocol, d.ndeg, e, (u64*)d.gscratch);
            }
        }
    }
    if (ev) (void)hipEventRecord(ev[1], st);
    // wedge pass
    const int* wc = hc + TB_N;
    if (wc[WB_WAVE] > 0) {
        if (per_edge)
            hipLaunchKernelGGL((k_wedge_wave<true, AT>), dim3(cdiv(wc[WB_WAVE], 4)), dim3(256), 0, st,
                               d.wlist + (int64_t)WB_WAVE * n, wc[WB_WAVE], d.nrp, d.ncol, d.optr, d.ocol, d.s2k,
                               e, gsum, d.ngid);
        else
            hipLaunchKernelGGL((k_wedge_wave<false, AT>), dim3(cdiv(wc[WB_WAVE], 4)), dim3(256), 0, st,
                               d.wlist + (int64_t)WB_WAVE * n, wc[WB_WAVE], d.nrp, d.ncol, d.optr, d.ocol, d.s2k,
                               e, gsum, d.ngid);
    }
    if (wc[WB_BLK] > 0) {
        if (per_edge)
            hipLaunchKernelGGL((k_wedge_blk<true, AT>), dim3(wc[WB_BLK]), dim3(WB_THREADS), 0, st,
                               d.wlist + (int64_t)WB_BLK * n, wc[WB_BLK], n, d.wedge_limit, d.wedge_dense, d.nrp,
                               d.ncol, d.optr, d.ocol, d.s2k, e, gsum, d.ngid);
        else
            hipLaunchKernelGGL((k_wedge_blk<false, AT>), dim3(wc[WB_BLK]), dim3(WB_THREADS), 0, st,
                               d.wlist + (int64_t)WB_BLK * n, wc[WB_BLK], n, d.wedge_limit, d.wedge_dense, d.nrp,
                               d.ncol, d.optr, d.ocol, d.s2k, e, gsum, d.ngid);
    }
    if (ev) (void)hipEventRecord(ev[2], st);
    // vertex pass + combine
    if (per_edge && n > 0 && m > 0) {
        launch_fill<u64>(d.tri, n, 0ull, st);
        launch_fill<u64>(d.sdeg, n, 0ull, st);
        hipLaunchKernelGGL(k_vertex, dim3(cdiv(2 * (int64_t)m, 256)), dim3(256), 0, st, d.nsrow, d.ncol, d.s2k,
                           d.ndeg, e.t, 2 * (int64_t)m, d.tri, d.sdeg);
    }
    const int nb = combine_blocks(m);
    if (d.ngraphs > 0) {
        hipLaunchKernelGGL(k_combine_graphs, dim3(d.ngraphs), dim3(CB_THREADS), 0, st, d.gvb, d.gsb, d.eid2k, e,
                           d.ocol, d.ndeg, d.gparts);
    } else if (m > 0) {
        if (per_edge)
            hipLaunchKernelGGL((k_combine<true, AT>), dim3(nb), dim3(CB_THREADS), 0, st, d.eid2k, e, d.ocol, d.ndeg, d.tri,
                               d.sdeg, n, m, out_pe, d.sums, d.err);
        else
            hipLaunchKernelGGL((k_combine<false, AT>), dim3(nb), dim3(CB_THREADS), 0, st, d.eid2k, e, d.ocol, d.ndeg, d.tri,
                               d.sdeg, n, m, out_pe, d.sums, d.err);
        hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, st, d.sums, nb, d.final_sums);
    } else {
        launch_fill<u64>(d.final_sums, 2 * NCS, 0ull, st);
    }
    if (ev) (void)hipEventRecord(ev[3], st);
}

void glt_count_passes(const Dev& d, int per_edge, const int* hc, u64* out_pe, hipStream_t st, hipEvent_t* ev) {
    if (d.acc32)
        count_passes<u32>(d, per_edge, hc, out_pe, st, ev);
    else
        count_passes<u64>(d, per_edge, hc, out_pe, st, ev);
}

int glt_combine_blocks(int m) { return combine_blocks(m); }
// largest out-degree the block passes accept (LDS holds 5 ints per neighbour of a)
int glt_max_out_degree() { return 3200; }
int glt_wedge_table() { return WB_TABLE; }
int glt_wedge_dense() { return WB_DENSE; }
int glt_wave_table() { return WW_TABLE; }
