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
// Work items inside a group are enumerated as flattened (source, offset) pairs with
// consecutive lanes on consecutive entries of one out-list (run tables map a position to
// its source in O(1)), so credits to the edges of one list are coalesced atomics to
// consecutive oriented indices, and credits that all lanes of a run send to the same source
// are first summed across the wavefront (DPP) before one atomic per run.
#include "glt_internal.h"

// Per-edge accumulators (EdgeArrays): 32-bit words for narrow edges (k < kw), 64-bit words
// for wide ones.  With AT = u32 (no wide edge) the 64-bit side is compiled out.  Every credit
// of a narrow edge is at most its final value, so it fits 32 bits; sums that kernels form
// in AT before crediting are exact modulo 2^32, and so is the narrow word they land in.
enum { ACC_K = 0, ACC_P = 1 };
template <typename AT, int WHICH>
__device__ __forceinline__ void acc_add(const EdgeArrays& e, int64_t k, u64 v) {
    if (sizeof(AT) == 8 && k >= e.kw) atomicAdd(&(WHICH == ACC_K ? e.Kw : e.Pw)[k - e.kw], v);
    else atomicAdd(&((u32*)(WHICH == ACC_K ? e.K : e.P))[k], (u32)v);
}
template <typename AT, int WHICH>
__device__ __forceinline__ u64 acc_get(const EdgeArrays& e, int64_t k) {
    if (sizeof(AT) == 8 && k >= e.kw) return (WHICH == ACC_K ? e.Kw : e.Pw)[k - e.kw];
    return (u64)((const u32*)(WHICH == ACC_K ? e.K : e.P))[k];
}

// g and sigma of an edge: for a narrow edge the pair shares one 64-bit word of the g buffer
// (g low, sigma high), so both move with one atomic; each half stays below 2^32, so no carry
// crosses the halves.  A wide edge has them in separate 64-bit words.
template <typename AT>
__device__ __forceinline__ void gsig_add(const EdgeArrays& e, int64_t k, u64 g, u64 sig) {
    if (sizeof(AT) == 8 && k >= e.kw) {
        if (g) atomicAdd(&e.gw[k - e.kw], g);
        if (sig) atomicAdd(&e.sw[k - e.kw], sig);
    } else {
        const u64 v = (sig << 32) | (g & 0xffffffffull);
        if (v) atomicAdd(&e.g[k], v);
    }
}
template <typename AT>
__device__ __forceinline__ void gsig_get(const EdgeArrays& e, int64_t k, u64& g, u64& sig) {
    if (sizeof(AT) == 8 && k >= e.kw) {
        g = e.gw[k - e.kw];
        sig = e.sw[k - e.kw];
    } else {
        const u64 v = e.g[k];
        g = v & 0xffffffffull;
        sig = v >> 32;
    }
}

// Triangle and 4-clique credits of one edge.  In per-edge mode a narrow edge accumulates
// (K << 32 | t) in its g word during the triangle pass, one atomic for both (t and K stay
// below 2^32, so the halves never carry into each other); k_unpack_tk then moves them to t
// and K and clears g before the gather pass.  Wide edges, and global counting (no K), credit
// t and K separately.
template <bool PE, typename AT>
__device__ __forceinline__ void tk_add(const EdgeArrays& e, int64_t k, u32 dt, u64 dk) {
    if (PE && !(sizeof(AT) == 8 && k >= e.kw)) {
        const u64 v = (dk << 32) | (u64)dt;
        if (v) atomicAdd(&e.g[k], v);
    } else {
        if (dt) atomicAdd(&e.t[k], dt);
        if (PE && dk) acc_add<AT, ACC_K>(e, k, dk);
    }
}

__global__ __launch_bounds__(256) void k_unpack_tk(EdgeArrays e, int m) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m || k >= e.kw) return;
    const u64 v = e.g[k];
    e.t[k] = (u32)v;
    reinterpret_cast<u32*>(e.K)[k] = (u32)(v >> 32);
    e.g[k] = 0;
}

#define TB_THREADS 256
#ifndef TW_G
#define TW_G 4         // wavefronts per block in the wavefront triangle and gather passes
#endif
#define TW_THREADS (TW_G * GLT_WAVE)
#ifndef TRI_BIG_MINB
#define TRI_BIG_MINB 1 // resident 1024-thread triangle workgroups per CU the registers are sized for
#endif
#ifndef TRI_ILP
#define TRI_ILP 4      // out-list entries per lane in flight in the triangle passes (8: more registers, slower)
#endif

template <int T>
__device__ __forceinline__ void grp_sync() {
    if constexpr (T == GLT_WAVE) wave_sync(); else __syncthreads();
}

// Flattened enumeration of the entries of up to T runs (sources) by a group of T threads,
// with consecutive threads on consecutive positions.  Thread i of the group owns run i of
// the current chunk (len_i entries starting at column offset k0_i); positions are
// numbered 0 .. sum(len) - 1 in run order.  For every super-tile of SPOS = 64 T positions
// the group marks the first position of each non-empty run in a bit mask (one 64-bit word
// per thread) and keeps the number of runs begun before each word; the run of a position
// is then (runs begun before its word) + popcount(earlier bits of its word) - 1, found with
// two broadcast LDS reads and one lookup, instead of a search over the run prefix sums.
template <int T>
struct RunTables {
    static constexpr int SPOS = 64 * T;
    u64 msk[T];        // bit p of word w: a non-empty run begins at super-tile position 64 w + p
    int pc[T];         // non-empty runs begun before word w (including earlier super-tiles)
    int2 nz[T];        // per non-empty run in order: (column offset - position, run index)
    u64 scan[T / GLT_WAVE > 0 ? T / GLT_WAVE : 1];
};

template <int T, typename V>
__device__ __forceinline__ V grp_excl_scan_t(V v, V* lds, V& tot) {
    if constexpr (T == GLT_WAVE) {
        const V inc = wave_incl_scan(v);
        tot = __shfl(inc, GLT_WAVE - 1, GLT_WAVE);
        return inc - v;
    } else {
        return block_excl_scan<V, T>(v, lds, tot);
    }
}

// Group-cooperative (every thread of the group calls it, uniformly): sets up a chunk whose
// run tid has `len` entries at column offset k0; returns the chunk's total entries and
// this thread's first position `pre`; the tables describe super-tile 0 and `carry` counts
// the non-empty runs begun in it.  The caller has passed a group barrier since the tables
// were last read.
template <int T>
__device__ __forceinline__ int runs_begin(RunTables<T>& rt, int len, int k0, int& pre, int& carry) {
    const int tid = threadIdx.x % T;
    rt.msk[tid] = 0;
    u64 tot2;
    // run lengths (<= the out-degree limit) and non-empty flags, one packed scan
    const u64 ex = grp_excl_scan_t<T, u64>(((u64)(u32)len << 32) | (u64)(len > 0), rt.scan, tot2);
    grp_sync<T>();   // the cleared words are visible before any bit is set
    pre = (int)(ex >> 32);
    if (len > 0) {
        rt.nz[(int)(u32)ex] = make_int2(k0 - pre, tid);
        if (pre < RunTables<T>::SPOS) atomicOr(&rt.msk[pre >> 6], 1ull << (pre & 63));
    }
    grp_sync<T>();
    u64 ptot;
    rt.pc[tid] = (int)grp_excl_scan_t<T, u64>((u64)__popcll(rt.msk[tid]), rt.scan, ptot);
    carry = (int)ptot;
    grp_sync<T>();
    return (int)(tot2 >> 32);
}

// Group-cooperative: moves the tables to the super-tile starting at position sb0.
template <int T>
__device__ __forceinline__ void runs_next(RunTables<T>& rt, int sb0, int len, int pre, int& carry) {
    const int tid = threadIdx.x % T;
    grp_sync<T>();   // readers of the previous super-tile are done
    rt.msk[tid] = 0;
    grp_sync<T>();
    const int p = pre - sb0;
    if (len > 0 && p >= 0 && p < RunTables<T>::SPOS) atomicOr(&rt.msk[p >> 6], 1ull << (p & 63));
    grp_sync<T>();
    u64 ptot;
    rt.pc[tid] = carry + (int)grp_excl_scan_t<T, u64>((u64)__popcll(rt.msk[tid]), rt.scan, ptot);
    carry += (int)ptot;
    grp_sync<T>();
}

// (column offset - position, run index) of super-tile position p
template <int T>
__device__ __forceinline__ int2 runs_at(const RunTables<T>& rt, int p) {
    const int w = p >> 6;
    const u64 m = rt.msk[w] & ((2ull << (p & 63)) - 1ull);
    return rt.nz[rt.pc[w] + __popcll(m) - 1];
}


// ---------------------------------------------------------------------------------------
// triangle / 4-clique pass, out-degree 2..64: one wavefront per vertex, M rows in one word
// ---------------------------------------------------------------------------------------
// Membership of a vertex id in S = N+(a) (s <= 64) through an LDS hash per wavefront mapping
// id -> position in S.  Most probes miss, so the table is kept sparse (a miss usually costs
// one read).
#ifndef SH_SIZE
#define SH_SIZE 256
#endif
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

// Entries of the LDS hash over S = N+(a) in the workgroup triangle pass: a power of two
// >= F |S| (load <= 1/F), sparser for the smaller buckets where LDS allows.
#ifndef TRI_HT_F
#define TRI_HT_F 2
#endif
#ifndef TRI_HT_F2
#define TRI_HT_F2 2
#endif
// Words per adjacency row M_i in the workgroup triangle pass.  Rows in the global slab are
// padded to a multiple of four words, so they are 16-byte aligned and the 4-clique sweep
// reads them in 16-byte loads (the padding words stay zero); rows in LDS are not (16-byte LDS
// reads at scattered rows measured slower there).
__host__ __device__ inline int tri_row_words(int s, bool gm) {
    const int w = (s + 31) / 32;
    return gm ? ((w + 3) & ~3) : w;
}

__host__ __device__ inline int tri_blk_ht(int smax) {
    const int f = smax <= 256 ? TRI_HT_F : smax <= TB_LDS_ROWS ? TRI_HT_F2 : 2;
    int h = 64;
    while (h < f * smax) h <<= 1;
    return h;
}

// Out-degrees above TB_LDS_SMAX (rare: the degree order bounds them by sqrt(2m)) keep the
// workgroup passes' per-neighbour arrays and membership hash in the workgroup's region of
// the global slab too (GX), besides the rows.  Positions in N+(a) are 16-bit fields of the
// triangle records and of the hash; 2m < 2^31 keeps every out-degree below 46,341.
#define TB_LDS_SMAX 3200
// u32 words of one workgroup's slab region: triangle pass (rows; GX: sK, sS, sOb, sLen, hash)
__host__ __device__ inline int64_t tri_slab_words(int smax, bool gx) {
    int64_t w = (int64_t)smax * tri_row_words(smax, true);
    if (gx) w += 5 * (int64_t)smax + tri_blk_ht(smax) + (tri_blk_ht(smax) + 1) / 2;
    return (w + 3) & ~(int64_t)3;
}
// gather pass (sG, sSg; GX: sS, sOb, sLen, sT, sD)
__host__ __device__ inline int64_t gather_slab_words(int smax, bool gx) {
    int64_t w = 4 * (int64_t)smax;
    if (gx) w += 5 * (int64_t)(smax + 1);
    return (w + 3) & ~(int64_t)3;
}

// Membership of S = N+(a) for the workgroup triangle pass: LDS open addressing, id -> position.
__device__ __forceinline__ u32 bhash(int x, u32 mask) { return ((u32)x * 2654435761u >> 7) & mask; }
__device__ __forceinline__ int bh_find(const int* hk, const unsigned short* hp, u32 mask, int x) {
    u32 h = bhash(x, mask);
    while (true) {
        const int k = hk[h];
        if (k == x) return (int)hp[h];
        if (k == -1) return -1;
        h = (h + 1) & mask;
    }
}

// A bit filter over S in LDS ahead of the hash: most out-list entries of the neighbours are
// not in S (on the R-MAT graph 97.5 % in the 65..256 bucket), and a clear bit rejects one
// with a single read.  BITS bits, indexed by the top bits of a multiplicative hash; at most
// 1/32 of them are set for out-degrees up to 256 and 1/36 up to 896.
#ifndef TRI_FILTER
#define TRI_FILTER 1
#endif
template <int NT>
struct TriFilter {
    static constexpr int BITS = NT <= 256 ? 8192 : 32768;
    static constexpr int LG = NT <= 256 ? 13 : 15;
    static constexpr int WORDS = TRI_FILTER ? BITS / 32 : 1;
};
template <int LG>
__device__ __forceinline__ u32 fhash(int x) { return ((u32)x * 0x9E3779B1u) >> (32 - LG); }

// Triangle records (REC): every triangle (a, b_i, b_j) found while the rows are built is
// written as (k << 32 | j << 16 | i), k the oriented index of (b_i, b_j), into a's slots
// [toff[a], toff[a] + C(|N+(a)|, 2)) (each pair i < j at most once), and tcnt[a] holds
// their number.  The 4-clique sweep and the gather pass then walk the records instead of
// re-scanning every out-list of N+(a).
__device__ __forceinline__ u64 tri_rec(int i, int j, int k) {
    return ((u64)(u32)k << 32) | (u64)(u32)(i | (j << 16));
}
__device__ __forceinline__ void tri_unrec(u64 v, int& i, int& j, int& k) {
    i = (int)(v & 0xffffu);
    j = (int)((v >> 16) & 0xffffu);
    k = (int)(v >> 32);
}

template <bool PE, bool REC, typename AT>
__global__ __launch_bounds__(TW_THREADS) void k_tri_wave(const int* __restrict__ list, int nlist,
                                                        const int* __restrict__ optr, const int* __restrict__ ocol,
                                                        EdgeArrays e, u64* __restrict__ gsum,
                                                        const int* __restrict__ ngid, u64* __restrict__ trec,
                                                        const u64* __restrict__ toff, int* __restrict__ tcnt) {
    constexpr int SPOS = RunTables<GLT_WAVE>::SPOS;
    __shared__ RunTables<GLT_WAVE> sRT[TW_G];
    __shared__ u64 sM[TW_G][GLT_WAVE];
    __shared__ u64 sK[TW_G][GLT_WAVE];
    __shared__ int hk[TW_G][SH_SIZE];
    __shared__ unsigned char hv[TW_G][SH_SIZE];
    // every LDS array is per wavefront: wavefronts synchronise only with themselves
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
    const int idx = blockIdx.x * TW_G + w;
    if (idx >= nlist) return;
    const int a = list[idx];
    const int o0 = optr[a];
    const int s = optr[a + 1] - o0;
    int b = 0, ob = 0, db = 0;
    if (l < s) { b = ocol[o0 + l]; ob = optr[b]; db = optr[b + 1] - ob; }
    RunTables<GLT_WAVE>& rt = sRT[w];
    sM[w][l] = 0; sK[w][l] = 0;
    for (int q = l; q < SH_SIZE; q += GLT_WAVE) hk[w][q] = -1;
    // runs: the out-list of b_l for every l; positions enumerate N+(b_0), N+(b_1), ...
    int pre, carry;
    const int total = runs_begin<GLT_WAVE>(rt, db, ob, pre, carry);
    if (l < s) sh_insert(hk[w], hv[w], b, l);
    wave_sync();
    // build the adjacency rows among S (and record the triangles)
    u64* rec = REC ? trec + toff[a] : nullptr;
    const u64 lt = (l == 0) ? 0ull : ((~0ull) >> (GLT_WAVE - l));
    int nh = 0;   // records so far (wave-uniform)
    for (int sb0 = 0; sb0 < total; sb0 += SPOS) {
        if (sb0 > 0) runs_next<GLT_WAVE>(rt, sb0, db, pre, carry);
        const int se = min(total, sb0 + SPOS);
        for (int q0 = sb0; q0 < se; q0 += TRI_ILP * GLT_WAVE) {
            // TRI_ILP entries per lane in flight: indices and loads first, then the probes
            int is[TRI_ILP], ks[TRI_ILP], xs[TRI_ILP];
#pragma unroll
            for (int u = 0; u < TRI_ILP; u++) {
                const int q = q0 + u * GLT_WAVE + l;
                xs[u] = -1;
                is[u] = 0;
                ks[u] = 0;
                if (q < se) {
                    const int2 r = runs_at(rt, q - sb0);
                    is[u] = r.y;
                    ks[u] = q + r.x;
                    xs[u] = ocol[ks[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < TRI_ILP; u++) {
                const int j = (xs[u] >= 0) ? sh_find(hk[w], hv[w], xs[u]) : -1;
                if (j >= 0) {
                    atomicOr(&sM[w][is[u]], 1ull << j);
                    atomicOr(&sM[w][j], 1ull << is[u]);
                }
                if (REC) {   // entries in scan order: records stay sorted by i
                    const u64 hm = __ballot(j >= 0);
                    if (j >= 0) rec[nh + __popcll(hm & lt)] = tri_rec(is[u], j, ks[u]);
                    nh += __popcll(hm);
                }
            }
        }
    }
    wave_sync();
    // 4-cliques of every triangle (a, b_i, b_j): popcount(M_i & M_j); each credits the
    // triangle's three edges (the two at a are summed per source in LDS)
    u64 k4 = 0;
    if (REC) {
        for (int r0 = 0; r0 < nh; r0 += GLT_WAVE) {
            const int r = r0 + l;
            int ri = 0x7fffffff;
            u64 tk = 0;
            if (r < nh) {
                int rj, k;
                tri_unrec(rec[r], ri, rj, k);
                tk = (u64)__popcll(sM[w][ri] & sM[w][rj]);
                tk_add<PE, AT>(e, k, 1u, PE ? tk : 0ull);
                if (PE && tk) atomicAdd(&sK[w][rj], tk);
                k4 += tk;
            }
            if (PE) {   // records are in scan order: runs of equal i summed first
                bool last;
                const u64 ssum = seg_sum_last(tk, ri, last);
                if (last && ssum) atomicAdd(&sK[w][ri], ssum);
            }
        }
        if (l == 0) tcnt[a] = nh;
    } else {
        runs_begin<GLT_WAVE>(rt, db, ob, pre, carry);
        for (int sb0 = 0; sb0 < total; sb0 += SPOS) {
            if (sb0 > 0) runs_next<GLT_WAVE>(rt, sb0, db, pre, carry);
            const int se = min(total, sb0 + SPOS);
            for (int q0 = sb0; q0 < se; q0 += GLT_WAVE) {
                const int q = q0 + l;
                if (q < se) {
                    const int2 r = runs_at(rt, q - sb0);
                    const int i = r.y, k = q + r.x;
                    const int j = sh_find(hk[w], hv[w], ocol[k]);
                    if (j >= 0) {
                        const u64 tk = (u64)__popcll(sM[w][i] & sM[w][j]);
                        tk_add<PE, AT>(e, k, 1u, PE ? tk : 0ull);
                        if (PE && tk) {
                            atomicAdd(&sK[w][i], tk);
                            atomicAdd(&sK[w][j], tk);
                        }
                        k4 += tk;
                    }
                }
            }
        }
    }
    wave_sync();
    if (l < s) tk_add<PE, AT>(e, o0 + l, (u32)__popcll(sM[w][l]), PE ? (sK[w][l] >> 1) : 0ull);
    k4 = wave_sum(k4);
    const u64 ntri = wave_sum((l < s) ? (u64)__popcll(sM[w][l]) : 0ull) / 2;
    if (l == 0) {
        u64* gs = gsum + gslot(ngid, a) * NSUMS;
        if (k4) atomicAdd(&gs[S_K4x3], k4);
        if (ntri) atomicAdd(&gs[GS_TRI_WAVE], ntri);
    }
}

// ---------------------------------------------------------------------------------------
// triangle / 4-clique pass, out-degree > 64: one workgroup per vertex, M rows of W words
// in LDS (GM = false) or in a per-workgroup global slab (GM = true)
// ---------------------------------------------------------------------------------------
// popcount(M_i & M_j) over W words (GM: 16-byte loads of padded rows)
template <bool GM>
__device__ __forceinline__ u64 row_and_count(const u32* M, int W, int i, int j) {
    u64 c = 0;
    if constexpr (GM) {
        const uint4* mi = reinterpret_cast<const uint4*>(M + (int64_t)i * W);
        const uint4* mj = reinterpret_cast<const uint4*>(M + (int64_t)j * W);
        for (int wd = 0; wd < W / 4; wd++) {
            const uint4 x = mi[wd], y = mj[wd];
            c += (u64)(__popc(x.x & y.x) + __popc(x.y & y.y) + __popc(x.z & y.z) + __popc(x.w & y.w));
        }
    } else {
        for (int wd = 0; wd < W; wd++) c += (u64)__popc(M[i * W + wd] & M[j * W + wd]);
    }
    return c;
}

// GM: rows M in the workgroup's slab region (gstride u32 words per workgroup); GX (with GM):
// also the per-neighbour arrays and the hash there.  A launch takes the list entries with
// out-degree <= smax, or with GX those above TB_LDS_SMAX (each group skips the rest).
template <bool PE, bool GM, bool REC, typename AT, int NT, bool GX>
__global__ __launch_bounds__(NT, NT <= 256 ? 8 : TRI_BIG_MINB) void k_tri_blk(const int* __restrict__ list, int nlist, int smax,
                                                       const int* __restrict__ optr, const int* __restrict__ ocol,
                                                       EdgeArrays e, u64* __restrict__ gsum,
                                                       u32* __restrict__ gscratch, int64_t gstride,
                                                       const int* __restrict__ ngid,
                                                       u64* __restrict__ trec, const u64* __restrict__ toff,
                                                       int* __restrict__ tcnt) {
    static_assert(GM || !GX, "global per-neighbour arrays only on the global-row path");
    constexpr int SPOS = RunTables<NT>::SPOS;
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    __shared__ RunTables<NT> rt;
    __shared__ u64 sRed[NT / GLT_WAVE];
    __shared__ int sNrec;
    __shared__ u32 sF[TriFilter<NT>::WORDS];
    const int a = list[blockIdx.x];
    const int o0 = optr[a];
    const int s = optr[a + 1] - o0;
    if (GX ? (s <= TB_LDS_SMAX) : (s > smax)) return;   // not this launch's entry (uniform per workgroup)
    const int Wmax = tri_row_words(smax, GM);
    u32* gb = GM ? gscratch + (int64_t)blockIdx.x * gstride : nullptr;
    unsigned char* xb = GX ? (unsigned char*)(gb + (int64_t)smax * Wmax) : dyn;
    u64* sK = (u64*)xb;
    int* sS = (int*)(sK + smax);
    int* sOb = sS + smax;
    int* sLen = sOb + smax;
    u32* M = GM ? gb : (u32*)(sLen + smax);
    const int HT = tri_blk_ht(smax);
    const u32 hmask = (u32)HT - 1;
    int* hk = GM ? (sLen + smax) : (int*)(M + (int64_t)smax * Wmax);
    unsigned short* hp = (unsigned short*)(hk + HT);
    const int tid = threadIdx.x;
    const int W = tri_row_words(s, GM);
    constexpr int FLG = TriFilter<NT>::LG;
    for (int q = tid; q < HT; q += NT) hk[q] = -1;
    if (TRI_FILTER) for (int q = tid; q < TriFilter<NT>::WORDS; q += NT) sF[q] = 0;
    __syncthreads();
    // S, its out-list offsets and lengths; S into the hash and the filter
    for (int i = tid; i < s; i += NT) {
        const int b = ocol[o0 + i];
        const int ob = optr[b];
        sS[i] = b; sOb[i] = ob; sLen[i] = optr[b + 1] - ob; sK[i] = 0;
        u32 h = bhash(b, hmask);
        while (atomicCAS(&hk[h], -1, b) != -1) h = (h + 1) & hmask;
        hp[h] = (unsigned short)i;
        if (TRI_FILTER) {
            const u32 f = fhash<FLG>(b);
            atomicOr(&sF[f >> 5], 1u << (f & 31));
        }
    }
    for (int q = tid; q < s * W; q += NT) M[q] = 0;
    if (tid == 0) sNrec = 0;
    __syncthreads();
    u64* rec = REC ? trec + toff[a] : nullptr;
    const u64 lt = (glt_lane() == 0) ? 0ull : ((~0ull) >> (GLT_WAVE - glt_lane()));
    // scan the out-lists of b_c0 .. b_{c0+255}, one chunk of runs at a time
    for (int c0 = 0; c0 < s; c0 += NT) {
        const int len = (c0 + tid < s) ? sLen[c0 + tid] : 0;
        const int ob = (c0 + tid < s) ? sOb[c0 + tid] : 0;
        int pre, carry;
        const int total = runs_begin<NT>(rt, len, ob, pre, carry);
        for (int sb0 = 0; sb0 < total; sb0 += SPOS) {
            if (sb0 > 0) runs_next<NT>(rt, sb0, len, pre, carry);
            const int se = min(total, sb0 + SPOS);
            for (int q0 = sb0; q0 < se; q0 += TRI_ILP * NT) {
                int is[TRI_ILP], ks[TRI_ILP], xs[TRI_ILP];
#pragma unroll
                for (int u = 0; u < TRI_ILP; u++) {
                    const int q = q0 + u * NT + tid;
                    xs[u] = -1;
                    is[u] = 0;
                    ks[u] = 0;
                    if (q < se) {
                        const int2 r = runs_at(rt, q - sb0);
                        is[u] = c0 + r.y;
                        ks[u] = q + r.x;
                        xs[u] = ocol[ks[u]];
                    }
                }
#pragma unroll
                for (int u = 0; u < TRI_ILP; u++) {
                    const int i = is[u];
                    int j = s;
                    bool maybe = xs[u] >= 0;
                    if (TRI_FILTER && maybe) {
                        const u32 f = fhash<FLG>(xs[u]);
                        maybe = (sF[f >> 5] >> (f & 31)) & 1u;
                    }
                    if (maybe) {
                        const int jj = bh_find(hk, hp, hmask, xs[u]);   // x in S lies above b_i: jj > i
                        if (jj >= 0) {
                            j = jj;
                            atomicOr(&M[i * W + (j >> 5)], 1u << (j & 31));
                            // rows in global memory are filled above the diagonal only (the
                            // lanes of a run set bits of one row); the mirror bits follow by
                            // tile transposes below
                            if (!GM) atomicOr(&M[j * W + (i >> 5)], 1u << (i & 31));
                        }
                    }
                    if (REC) {   // one slot reservation per wavefront and entry batch
                        const u64 hm = __ballot(j < s);
                        int base = 0;
                        if (glt_lane() == 0 && hm) base = atomicAdd(&sNrec, __popcll(hm));
                        base = __shfl(base, 0, GLT_WAVE);
                        if (j < s) rec[base + __popcll(hm & lt)] = tri_rec(i, j, ks[u]);
                    }
                }
            }
        }
        __syncthreads();   // the run tables are rebuilt for the next chunk
    }
    if constexpr (GM) {
        // M = U | U^T: every 32 x 32 bit tile (I, J), I <= J, of the upper part U is transposed
        // by one wavefront (32 ballots) into its mirror tile (J, I), which only it writes (an
        // off-diagonal mirror holds no bit yet; a diagonal tile ORs into itself)
        const int TWn = (s + 31) >> 5;
        const int npairs = TWn * (TWn + 1) / 2;
        const int ln = glt_lane();
        for (int p = tid / GLT_WAVE; p < npairs; p += NT / GLT_WAVE) {
            int I = 0, rem = p;
            while (rem >= TWn - I) { rem -= TWn - I; I++; }
            const int J = I + rem;
            const int r = 32 * I + (ln & 31);
            u32 u = 0;
            if (ln < 32 && r < s) u = M[(int64_t)r * W + J];
            u32 tr = 0;
#pragma unroll 8
            for (int c = 0; c < 32; c++) {
                const u32 b = (u32)__ballot((u >> c) & 1u);   // bit q: row 32I + q has column 32J + c
                if (ln == c) tr = b;
            }
            const int rr = 32 * J + ln;
            if (ln < 32 && rr < s) M[(int64_t)rr * W + I] = (I == J) ? (tr | u) : tr;
        }
        __syncthreads();
    }
    u64 k4 = 0;
    // 4-cliques of every triangle (a, b_i, b_j): popcount(M_i & M_j); each credits the
    // triangle's three edges (the two at a are summed per source in LDS)
    if (REC) {
        const int nrec = sNrec;
        constexpr int CR = 4;   // records per thread and round, loaded together
        for (int r0 = 0; r0 < nrec; r0 += CR * NT) {
            int ri[CR], rj[CR], rk[CR];
#pragma unroll
            for (int u = 0; u < CR; u++) {
                const int r = r0 + u * NT + tid;
                ri[u] = 0x7fffffff; rj[u] = 0; rk[u] = -1;
                if (r < nrec) tri_unrec(rec[r], ri[u], rj[u], rk[u]);
            }
#pragma unroll
            for (int u = 0; u < CR; u++) {
                u64 tk = 0;
                if (rk[u] >= 0) {
                    tk = row_and_count<GM>(M, W, ri[u], rj[u]);
                    tk_add<PE, AT>(e, rk[u], 1u, PE ? tk : 0ull);
                    if (PE && tk) atomicAdd(&sK[rj[u]], tk);
                    k4 += tk;
                }
                if (PE) {   // records come in runs of equal i (per writing wavefront)
                    bool last;
                    const u64 ssum = seg_run_sum_last(tk, ri[u], last);
                    if (last && ssum) atomicAdd(&sK[ri[u]], ssum);
                }
            }
        }
        if (tid == 0) tcnt[a] = nrec;
    } else {
        for (int c0 = 0; c0 < s; c0 += NT) {
            const int len = (c0 + tid < s) ? sLen[c0 + tid] : 0;
            const int ob = (c0 + tid < s) ? sOb[c0 + tid] : 0;
            int pre, carry;
            const int total = runs_begin<NT>(rt, len, ob, pre, carry);
            for (int sb0 = 0; sb0 < total; sb0 += SPOS) {
                if (sb0 > 0) runs_next<NT>(rt, sb0, len, pre, carry);
                const int se = min(total, sb0 + SPOS);
                for (int q = sb0 + tid; q < se; q += NT) {
                    const int2 r = runs_at(rt, q - sb0);
                    const int i = c0 + r.y, k = q + r.x;
                    const int j = bh_find(hk, hp, hmask, ocol[k]);
                    if (j >= 0) {
                        const u64 tk = row_and_count<GM>(M, W, i, j);
                        tk_add<PE, AT>(e, k, 1u, PE ? tk : 0ull);
                        if (PE && tk) {
                            atomicAdd(&sK[i], tk);
                            atomicAdd(&sK[j], tk);
                        }
                        k4 += tk;
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    u64 ntri = 0;
    for (int i = tid; i < s; i += NT) {
        u32 tl = 0;
        for (int wd = 0; wd < W; wd++) tl += (u32)__popc(M[i * W + wd]);
        ntri += tl;
        tk_add<PE, AT>(e, o0 + i, tl, PE ? (sK[i] >> 1) : 0ull);
    }
    k4 = wave_sum(k4);
    if (glt_lane() == 0) sRed[tid / GLT_WAVE] = k4;
    __syncthreads();
    if (tid == 0) {
        u64 tot = 0;
        for (int q = 0; q < NT / GLT_WAVE; q++) tot += sRed[q];
        if (tot) atomicAdd(&gsum[gslot(ngid, a) * NSUMS + S_K4x3], tot);
    }
    ntri = wave_sum(ntri) / 2;
    if (glt_lane() == 0 && ntri) atomicAdd(&gsum[gslot(ngid, a) * NSUMS + GS_TRI_WG], ntri);
}

static inline size_t tri_blk_lds(int smax, bool gm, bool gx) {
    if (gx) return 0;
    size_t b = (size_t)smax * (8 + 4 + 4 + 4);
    if (!gm) b += (size_t)smax * tri_row_words(smax, false) * 4;
    b += (size_t)tri_blk_ht(smax) * (4 + 2);
    return b;
}

// ---------------------------------------------------------------------------------------
// gather pass (per-edge mode): for every triangle (a, b_i, b_j), a lowest
// ---------------------------------------------------------------------------------------
// Credits of one triangle found at (i, j, edge k = (b_i, b_j)):
//   edge (a, b_i): g += t(a, b_j) + t(b_i, b_j), sig += d(b_j)   [local, run-summed]
//   edge (a, b_j): g += t(a, b_i) + t(b_i, b_j), sig += d(b_i)   [local]
//   edge (b_i, b_j): g += t(a, b_i) + t(a, b_j), sig += d(a)     [global, coalesced]
// tij = t of edge k = (b_i, b_j).  Runs of equal i in the wavefront are summed first (every
// lane must call; idle lanes pass a sentinel key and found = false).
template <typename AT>
__device__ __forceinline__ void gather_credit(bool found, int i, int j, int k, u64 tij, const u32* sT, const int* sD,
                                              int da, EdgeArrays& e, u64* sG, u64* sSg) {
    u64 gi = 0, di = 0;
    if (found) {
        const u64 tai = sT[i], taj = sT[j];
        gi = taj + tij;
        di = (u64)sD[j];
        atomicAdd(&sG[j], tai + tij);
        atomicAdd(&sSg[j], (u64)sD[i]);
        gsig_add<AT>(e, k, tai + taj, (u64)da);
    }
    bool last;
    const u64 a1 = seg_run_sum_last(gi, i, last);
    const u64 a3 = seg_run_sum_last(di, i, last);
    if (last) {
        if (a1) atomicAdd(&sG[i], a1);
        if (a3) atomicAdd(&sSg[i], a3);
    }
}

template <bool REC, typename AT>
__global__ __launch_bounds__(TW_THREADS) void k_gather_wave(const int* __restrict__ list, int nlist,
                                                           const int* __restrict__ optr,
                                                           const int* __restrict__ ocol,
                                                           const int* __restrict__ ndeg, EdgeArrays e,
                                                           const u64* __restrict__ trec,
                                                           const u64* __restrict__ toff,
                                                           const int* __restrict__ tcnt) {
    constexpr int SPOS = RunTables<GLT_WAVE>::SPOS;
    __shared__ RunTables<GLT_WAVE> sRT[REC ? 1 : TW_G];
    __shared__ u32 sT[TW_G][GLT_WAVE];
    __shared__ int sD[TW_G][GLT_WAVE];
    __shared__ u64 sG[TW_G][GLT_WAVE];
    __shared__ u64 sSg[TW_G][GLT_WAVE];
    __shared__ int hk[TW_G][SH_SIZE];
    __shared__ unsigned char hv[TW_G][SH_SIZE];
    // every LDS array is per wavefront: wavefronts synchronise only with themselves and leave
    // as soon as their vertex is done
    const int w = threadIdx.x / GLT_WAVE, l = glt_lane();
    const int idx = blockIdx.x * TW_G + w;
    if (idx >= nlist) return;
    const int a = list[idx];
    const int nh = REC ? tcnt[a] : 0;
    if (REC && nh == 0) return;   // no triangle has a as its lowest vertex
    const int o0 = optr[a];
    const int s = optr[a + 1] - o0;
    const int da = ndeg[a];
    // REC: GR rounds of records (and the t of each triangle's third edge) are loaded before
    // the setup, so that both chains of loads are in flight together
    constexpr int GR = 2;
    int ri[GR], rj[GR], rk[GR];
    u32 rt3[GR];
    const u64* rec = REC ? trec + toff[a] : nullptr;
    if (REC) {
#pragma unroll
        for (int u = 0; u < GR; u++) {
            const int r = u * GLT_WAVE + l;
            ri[u] = 0x3fffffff; rj[u] = -1; rk[u] = 0;
            if (r < nh) tri_unrec(rec[r], ri[u], rj[u], rk[u]);
        }
#pragma unroll
        for (int u = 0; u < GR; u++) rt3[u] = (u * GLT_WAVE + l < nh) ? e.t[rk[u]] : 0u;
    }
    int b = 0, ob = 0, db = 0;
    u32 tb = 0;
    int degb = 0;
    if (l < s) {
        b = ocol[o0 + l];
        tb = e.t[o0 + l];
        degb = ndeg[b];
        if (!REC) { ob = optr[b]; db = optr[b + 1] - ob; }
    }
    sT[w][l] = tb; sD[w][l] = degb;
    sG[w][l] = 0; sSg[w][l] = 0;
    if (REC) {
        wave_sync();
#pragma unroll
        for (int u = 0; u < GR; u++)
            gather_credit<AT>(u * GLT_WAVE + l < nh, ri[u], rj[u], rk[u], rt3[u], sT[w], sD[w], da, e, sG[w],
                              sSg[w]);
        for (int r0 = GR * GLT_WAVE; r0 < nh; r0 += GLT_WAVE) {
            const int r = r0 + l;
            int i = 0x3fffffff, j = -1, k = 0;
            if (r < nh) tri_unrec(rec[r], i, j, k);
            gather_credit<AT>(r < nh, i, j, k, r < nh ? (u64)e.t[k] : 0ull, sT[w], sD[w], da, e, sG[w], sSg[w]);
        }
    } else {
        RunTables<GLT_WAVE>& rt = sRT[REC ? 0 : w];
        for (int q = l; q < SH_SIZE; q += GLT_WAVE) hk[w][q] = -1;
        int pre, carry;
        const int total = runs_begin<GLT_WAVE>(rt, db, ob, pre, carry);
        if (l < s) sh_insert(hk[w], hv[w], b, l);
        wave_sync();
        for (int sb0 = 0; sb0 < total; sb0 += SPOS) {
            if (sb0 > 0) runs_next<GLT_WAVE>(rt, sb0, db, pre, carry);
            const int se = min(total, sb0 + SPOS);
            for (int q0 = sb0; q0 < se; q0 += GLT_WAVE) {
                const int q = q0 + l;
                int i = 0x3fffffff, j = -1, k = 0;
                if (q < se) {
                    const int2 r = runs_at(rt, q - sb0);
                    i = r.y;
                    k = q + r.x;
                    j = sh_find(hk[w], hv[w], ocol[k]);
                }
                gather_credit<AT>(j >= 0, i, j, k, j >= 0 ? (u64)e.t[k] : 0ull, sT[w], sD[w], da, e, sG[w], sSg[w]);
            }
        }
    }
    wave_sync();
    if (l < s) {
        gsig_add<AT>(e, o0 + l, sG[w][l], sSg[w][l]);
    }
}

// GM: the accumulators sG, sSg in the workgroup's slab region (gstride u32 words per
// workgroup); GX (with GM): the per-neighbour arrays there too.  A launch takes the list
// entries with out-degree <= smax, or with GX those above TB_LDS_SMAX.
template <bool GM, bool REC, typename AT, bool GX>
__global__ __launch_bounds__(TB_THREADS) void k_gather_blk(const int* __restrict__ list, int nlist, int smax,
                                                          const int* __restrict__ optr,
                                                          const int* __restrict__ ocol,
                                                          const int* __restrict__ ndeg, EdgeArrays e,
                                                          u64* __restrict__ gslab, int64_t gstride,
                                                          const u64* __restrict__ trec,
                                                          const u64* __restrict__ toff,
                                                          const int* __restrict__ tcnt) {
    static_assert(GM || !GX, "global per-neighbour arrays only on the global-accumulator path");
    constexpr int SPOS = RunTables<TB_THREADS>::SPOS;
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    __shared__ RunTables<REC ? GLT_WAVE : TB_THREADS> rt;
    const int tid = threadIdx.x;
    const int a = list[blockIdx.x];
    const int o0 = optr[a];
    const int s = optr[a + 1] - o0;
    if (GX ? (s <= TB_LDS_SMAX) : (s > smax)) return;   // not this launch's entry (uniform per workgroup)
    const int nh = REC ? tcnt[a] : 0;
    if (REC && nh == 0) return;   // no triangle has a as its lowest vertex (uniform per block)
    u64* gb = GM ? gslab + (int64_t)blockIdx.x * (gstride / 2) : nullptr;
    int* sS = GX ? (int*)(gb + 2 * (int64_t)smax) : (int*)dyn;
    int* sOb = sS + smax;
    int* sLen = sOb + smax;
    u32* sT = (u32*)(sLen + smax);
    int* sD = (int*)(sT + smax);
    u64* sG = GM ? gb : (u64*)(sD + smax + (smax & 1));
    u64* sSg = sG + smax;
    const int da = ndeg[a];
    // REC: GR records per thread and round, each with the t of its third edge; the first
    // round's loads go out before the setup
    constexpr int GR = 4;
    const u64* rec = REC ? trec + toff[a] : nullptr;
    int ri[GR], rj[GR], rk[GR];
    u32 rt3[GR];
    auto load_round = [&](int r0) {
#pragma unroll
        for (int u = 0; u < GR; u++) {
            const int r = r0 + u * TB_THREADS + tid;
            ri[u] = 0x3fffffff; rj[u] = -1; rk[u] = 0;
            if (r < nh) tri_unrec(rec[r], ri[u], rj[u], rk[u]);
        }
#pragma unroll
        for (int u = 0; u < GR; u++) rt3[u] = (r0 + u * TB_THREADS + tid < nh) ? e.t[rk[u]] : 0u;
    };
    if (REC) load_round(0);
    for (int i = tid; i < s; i += TB_THREADS) {
        const int b = ocol[o0 + i];
        const int ob = optr[b];
        sS[i] = b; sOb[i] = ob; sLen[i] = optr[b + 1] - ob; sT[i] = e.t[o0 + i]; sD[i] = ndeg[b];
        sG[i] = 0; sSg[i] = 0;
    }
    __syncthreads();
    if (REC) {
        // records come in runs of equal i (per writing wavefront), summed per run
        for (int r0 = 0; r0 < nh; r0 += GR * TB_THREADS) {
            if (r0 > 0) load_round(r0);
#pragma unroll
            for (int u = 0; u < GR; u++)
                gather_credit<AT>(r0 + u * TB_THREADS + tid < nh, ri[u], rj[u], rk[u], rt3[u], sT, sD, da, e, sG,
                                  sSg);
        }
    } else {
        if constexpr (!REC) {
            for (int c0 = 0; c0 < s; c0 += TB_THREADS) {
                const int len = (c0 + tid < s) ? sLen[c0 + tid] : 0;
                const int ob = (c0 + tid < s) ? sOb[c0 + tid] : 0;
                int pre, carry;
                const int total = runs_begin<TB_THREADS>(rt, len, ob, pre, carry);
                for (int sb0 = 0; sb0 < total; sb0 += SPOS) {
                    if (sb0 > 0) runs_next<TB_THREADS>(rt, sb0, len, pre, carry);
                    const int se = min(total, sb0 + SPOS);
                    // every thread runs the same number of rounds (runs are summed across the wave)
                    for (int q0 = sb0; q0 < se; q0 += TB_THREADS) {
                        const int q = q0 + tid;
                        int i = 0x3fffffff, j = 0, k = 0;
                        bool found = false;
                        if (q < se) {
                            const int2 r = runs_at(rt, q - sb0);
                            i = c0 + r.y;
                            k = q + r.x;
                            const int x = ocol[k];
                            j = lower_bound_i32(sS, i + 1, s, x);
                            found = (j < s && sS[j] == x);
                        }
                        gather_credit<AT>(found, i, j, k, found ? (u64)e.t[k] : 0ull, sT, sD, da, e, sG, sSg);
                    }
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < s; i += TB_THREADS) {
        gsig_add<AT>(e, o0 + i, sG[i], sSg[i]);
    }
}

static inline size_t gather_blk_lds(int smax, bool gm, bool gx) {
    if (gx) return 0;
    return (size_t)(smax + 1) * 4 * 5 + (gm ? 0 : (size_t)smax * 8 * 2);
}

// ---------------------------------------------------------------------------------------
// wedge / 4-cycle pass
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ u32 hslot(int x, u32 mask) { return ((u32)x * 2654435761u >> 7) & mask; }

// Oriented index range [k0, k1) of the wedges y - w - x for CSR slot s of row y (w = ncol[s]),
// restricted to tops x in [lo, hi) unless the range is the full [y + 1, n).
__device__ __forceinline__ void wedge_bounds(int s, int lo, int hi, bool full, const int2* __restrict__ wb,
                                             const int* __restrict__ ocol, int& k0, int& k1) {
    const int2 r = wb[s];
    k0 = r.x;
    k1 = r.y;
    if (!full) {
        k0 = lower_bound_i32(ocol, k0, k1, lo);
        k1 = lower_bound_i32(ocol, k0, k1, hi);
    }
}

#ifndef WEDGE_NORET
#define WEDGE_NORET 1
#endif
#define WEDGE_STACK 40   // x-range stack per group (halving depth <= 32 for 31-bit ids)
#ifndef WEDGE_ILP
#define WEDGE_ILP 2      // wedges per lane and batch; two batches are in flight (4 per batch: slower)
#endif
#ifndef WEDGE_ILP_HUGE
#define WEDGE_ILP_HUGE 2 // the same for the 1024-thread class (at most 128 registers per lane)
#endif
#ifndef WEDGE_PF
#define WEDGE_PF 1       // each sweep loads the next batch's tops before it works on the current one
#endif

// Size classes of the wedge pass (wedges per bottom vertex y): threads per group, groups per
// block, hash entries, dense top counters.
#define WW_T 64
#ifndef WW_G
#define WW_G 4
#endif
#define WW_HT 512        // wave class: <= WW_HT / 2 wedges, so the hash never overflows
#define WM_T 64
#ifndef WM_G
#define WM_G 1       // mid class: 16-bit counters (its bottoms have at most 65,535 wedges)
#endif
#ifndef WM_HT
#define WM_HT 1024
#endif
#ifndef WM_DW
#define WM_DW 1024
#endif
#define WB_T 256
#ifndef WB_MINB
#define WB_MINB 1        // workgroup class: resident groups per CU the registers are sized for
#endif
#ifndef WEDGE_ILP_WG
#define WEDGE_ILP_WG WEDGE_ILP
#endif
#define WB_RESIDENT 4    // resident workgroup-class groups per CU for the bottoms the mid class hands over
#ifndef WB_HT
#define WB_HT 2048
#endif
#ifndef WB_DW
#define WB_DW 4096
#endif
#define WH_T 1024        // huge class: a whole CU's LDS for bottom vertices with the most wedges
#ifndef WH_HT
#define WH_HT 8192
#endif
#ifndef WH_DW
#define WH_DW 16384
#endif
#ifndef WH_PER_CU
#define WH_PER_CU 1      // resident huge-class workgroups per CU
#endif

// One group of T threads per bottom vertex y (G groups per block).  For every wedge
// y - w - x with x above y the group counts c(y, x) = number of such w in LDS: tops x in
// the dense window [n - dense, n) (the highest-ranked vertices, which close most wedges of a
// degree-ordered graph) in a direct array, lower tops in an open-addressing hash.  The
// non-induced 4-cycles with lowest vertex y and opposite vertex x number C(c, 2), summed
// from the values the counter increments return (0 + 1 + ... + c - 1).  With PE, a second
// sweep credits c(y, x) - 1 to each wedge's two edges (the top edge (w, x) directly, the
// bottom edge (y, w) summed per source first).  Whenever more than `limit` distinct hashed
// tops appear, the x-range [lo, hi) is halved and redone; a range is credited only after its
// count sweep completed without overflow, so no wedge is credited twice.
// Top counters: u32 each, or (P16) two 16-bit counters per u32 word when every count is
// known to stay below 2^16 (the count of a top never exceeds the bottom vertex's wedges).
template <bool P16>
__device__ __forceinline__ u32 cnt_inc(u32* a, int i) {
    if constexpr (P16) {
        const u32 sh = (u32)(i & 1) << 4;
        return (atomicAdd(&a[i >> 1], 1u << sh) >> sh) & 0xffffu;
    } else {
        return atomicAdd(&a[i], 1u);
    }
}
template <bool P16>
__device__ __forceinline__ void cnt_add(u32* a, int i) {
    if constexpr (P16) atomicAdd(&a[i >> 1], 1u << ((u32)(i & 1) << 4));
    else atomicAdd(&a[i], 1u);
}
template <bool P16>
__device__ __forceinline__ u32 cnt_get(const u32* a, int i) {
    if constexpr (P16) return (a[i >> 1] >> ((u32)(i & 1) << 4)) & 0xffffu;
    else return a[i];
}

// Tops x (ocol at the wedge's oriented index, -1 past the end) of the IL super-tile
// positions q, q + T, ... of a sweep; with the oriented index k and the run (source) i too.
// Every lane loads (lanes past the end at position se - 1, which exists while se > sb0), so
// the number of loads in flight is fixed and a later wait can leave the next batch's loads
// pending.
template <int T, int IL>
__device__ __forceinline__ void wedge_tops(const RunTables<T>& rt, const int* __restrict__ ocol, int sb0, int se,
                                           int q, int (&xs)[IL]) {
#pragma unroll
    for (int j = 0; j < IL; j++, q += T) {
        const int qc = min(q, se - 1);
        const int x = ocol[qc + runs_at(rt, qc - sb0).x];
        xs[j] = q < se ? x : -1;
    }
}
template <int T, int IL>
__device__ __forceinline__ void wedge_slots(const RunTables<T>& rt, const int* __restrict__ ocol, int sb0, int se,
                                            int q, int (&xs)[IL], int (&ks)[IL], int (&is)[IL]) {
#pragma unroll
    for (int j = 0; j < IL; j++, q += T) {
        const int qc = min(q, se - 1);
        const int2 r = runs_at(rt, qc - sb0);
        ks[j] = qc + r.x;
        is[j] = r.y;
        const int x = ocol[ks[j]];
        xs[j] = q < se ? x : -1;
    }
}

template <bool PE, typename AT, int T, int G, int HT, int DW, bool P16, int IL>
__global__ __launch_bounds__(T * G, T == WB_T ? WB_MINB : 1) void k_wedge(const int* __restrict__ list, int nlist, int n, int limit,
                                                 int dense, const int* __restrict__ nrp,
                                                 const int2* __restrict__ wb,
                                                 const int* __restrict__ ocol, const int* __restrict__ s2k,
                                                 const u64* __restrict__ wcnt, EdgeArrays e,
                                                 u64* __restrict__ gsum, const int* __restrict__ ngid,
                                                 const int* __restrict__ vtop, int* __restrict__ err,
                                                 const int* __restrict__ dcount, int* __restrict__ defer_list,
                                                 int* __restrict__ defer_cnt, u64* __restrict__ defer_work,
                                                 u64* __restrict__ tstamp) {
    static_assert(T == GLT_WAVE || G == 1, "multi-wave groups own the whole block");
    static_assert(HT % 4 == 0 && DW % 4 == 0 && (HT & (HT - 1)) == 0, "table sizes");
    constexpr int DWA = DW > 0 ? DW : 8;
    constexpr int DCW = P16 ? DWA / 2 : DWA;   // u32 words of dense counters
    constexpr int HCW = P16 ? HT / 2 : HT;     // u32 words of hash counters
    constexpr int SPOS = RunTables<T>::SPOS;
    constexpr u32 mask = HT - 1;
    // NR: with per-edge credits the counting sweep increments without reading back (the
    // credit sweep sees every final count and sums the 4-cycles there)
    constexpr bool NR = PE && WEDGE_NORET;
    __shared__ __align__(16) u32 s_dc[G][DCW];
    __shared__ __align__(16) int s_hk[G][HT];
    __shared__ __align__(16) u32 s_hc[G][HCW];
    __shared__ RunTables<T> s_rt[G];
    __shared__ AT s_b[G][T];
    __shared__ int s_lo[G][WEDGE_STACK], s_hi[G][WEDGE_STACK];
    __shared__ int s_sp[G], s_dist[G], s_ovf[G];
    const int g = threadIdx.x / T, tid = threadIdx.x % T;
    // one list entry per group, or (dcount given) a resident grid walking a list whose length
    // a previous launch settled on the device
    const int first = blockIdx.x * G + g;
    const int count = dcount ? *dcount : nlist;
    const int stride = dcount ? (int)gridDim.x * G : count;
    if (first >= count) return;   // whole groups leave together (G == 1 when T > one wave)
    RunTables<T>& rt = s_rt[g];
    u32* dc = s_dc[g];
    int* hk = s_hk[g];
    u32* hc = s_hc[g];
    AT* sb = s_b[g];
    // A group walking several entries loads the next entry's row bounds and the entry after
    // that one ahead, while it works on the current one.  Tops lie above y inside y's
    // graph: a batch keeps each graph's ranks contiguous, vtop holds the end.
    int y1 = list[first];
    int y2 = first + stride < count ? list[first + stride] : 0;
    int rb1 = nrp[y1], re1 = nrp[y1 + 1], top1 = vtop ? vtop[y1] : n;
    for (int item = first; item < count; item += stride) {
    grp_sync<T>();   // the previous entry's last reads of the group's LDS are done
    const int y = y1, rb = rb1, re = re1, top = top1;
    if (item + stride < count) {
        y1 = y2;
        rb1 = nrp[y1]; re1 = nrp[y1 + 1]; top1 = vtop ? vtop[y1] : n;
        if (item + 2 * stride < count) y2 = list[item + 2 * stride];
    }
    const int base = max(top - min(dense, DW), y + 1);   // tops >= base are counted densely
    const int nd = top - base;                            // dense counters in use, <= DW
    // a top's count is at most the row length (one wedge per source), so below 2^25 the
    // wavefront prefix of 64 counts stays below 2^31
    const bool scan32 = (re - rb) < (1 << 25);
    if (tid == 0) { s_lo[g][0] = y + 1; s_hi[g][0] = top; s_sp[g] = 1; }
    u64 c4 = 0;
    grp_sync<T>();
    while (true) {
        const int sp = s_sp[g];
        if (sp == 0) break;
        const int lo = s_lo[g][sp - 1], hi = s_hi[g][sp - 1];
        const bool full = (lo == y + 1) && (hi == top);
        grp_sync<T>();
        if (tid == 0) { s_sp[g] = sp - 1; s_dist[g] = 0; s_ovf[g] = 0; }
        for (int q = tid; q < HT / 4; q += T) reinterpret_cast<int4*>(hk)[q] = make_int4(-1, -1, -1, -1);
        for (int q = tid; q < HCW / 4; q += T) reinterpret_cast<int4*>(hc)[q] = make_int4(0, 0, 0, 0);
        const int ndw = P16 ? (nd + 1) / 2 : nd;   // dense counter words in use
        for (int q = tid; q < (ndw + 3) / 4; q += T) reinterpret_cast<int4*>(dc)[q] = make_int4(0, 0, 0, 0);
        grp_sync<T>();
        // count sweep, over chunks of T sources; source tid of a chunk has `len` wedges
        u64 c4r = 0;
        // the overflow flag, read from LDS (a volatile access through a generic pointer would
        // be a flat load, which waits for every global load in flight)
        auto ovf_set = [&]() {
            return __hip_atomic_load(&s_ovf[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
        };
        // counts the tops of one batch (-1: no wedge)
        auto count_batch = [&](const int (&xs)[IL]) {
#pragma unroll
            for (int j = 0; j < IL; j++) {
                const int x = xs[j];
                if (x < 0) continue;
                if (x >= base) {
                    if (NR) cnt_add<P16>(dc, x - base);
                    else c4r += cnt_inc<P16>(dc, x - base);
                } else {
                    u32 h = hslot(x, mask);
                    bool done = false;
                    for (int p = 0; p < HT; p++) {   // bounded probe: a full table is an overflow
                        int cur = hk[h];
                        if (cur == -1) {
                            cur = atomicCAS(&hk[h], -1, x);
                            if (cur == -1) {
                                if (NR) cnt_add<P16>(hc, (int)h);
                                else c4r += cnt_inc<P16>(hc, (int)h);
                                if (atomicAdd(&s_dist[g], 1) >= limit) s_ovf[g] = 1;
                                done = true;
                                break;
                            }
                        }
                        if (cur == x) {
                            if (NR) cnt_add<P16>(hc, (int)h);
                            else c4r += cnt_inc<P16>(hc, (int)h);
                            done = true;
                            break;
                        }
                        h = (h + 1) & mask;
                    }
                    if (!done) s_ovf[g] = 1;
                }
            }
        };
        int tot1 = 0, len = 0, pre = 0;
        for (int c0 = rb; c0 < re; c0 += T) {
            const int s = c0 + tid;
            int k0 = 0, k1 = 0;
            if (s < re) wedge_bounds(s, lo, hi, full, wb, ocol, k0, k1);
            len = k1 - k0;
            int carry;
            const int tot = runs_begin<T>(rt, len, k0, pre, carry);
            for (int sb0 = 0; sb0 < tot; sb0 += SPOS) {
                if (sb0 > 0) runs_next<T>(rt, sb0, len, pre, carry);
                const int se = min(tot, sb0 + SPOS);
                // batches of IL * T positions; with WEDGE_PF two batches alternate between two
                // register sets, the next one's tops in flight while the current one is counted
                int xa[IL], xb[IL];
                wedge_tops<T, IL>(rt, ocol, sb0, se, sb0 + tid, xa);
                for (int q0 = sb0; q0 < se; q0 += (WEDGE_PF ? 2 : 1) * IL * T) {
                    if (ovf_set()) break;
                    if constexpr (WEDGE_PF) {
                        wedge_tops<T, IL>(rt, ocol, sb0, se, q0 + IL * T + tid, xb);
                        count_batch(xa);
                        if (q0 + IL * T >= se || ovf_set()) break;
                        wedge_tops<T, IL>(rt, ocol, sb0, se, q0 + 2 * IL * T + tid, xa);
                        count_batch(xb);
                    } else {
                        if (q0 > sb0) wedge_tops<T, IL>(rt, ocol, sb0, se, q0 + tid, xa);
                        count_batch(xa);
                    }
                }
            }
            tot1 = tot;
            grp_sync<T>();
        }
        if (s_ovf[g]) {
            if (defer_cnt && full) {
                // too many distinct tops for this class: y moves, uncredited, to the list of
                // the class with the largest tables
                if (tid == 0) {
                    defer_list[atomicAdd(defer_cnt, 1)] = y;
                    if (defer_work) atomicAdd(defer_work, wcnt[y]);   // wedges that changed class
                }
                grp_sync<T>();
                break;
            }
            if (tid == 0) {
                if (sp + 1 <= WEDGE_STACK && hi - lo >= 2) {
                    const int mid = lo + (hi - lo) / 2;
                    s_lo[g][sp - 1] = mid; s_hi[g][sp - 1] = hi;
                    s_lo[g][sp] = lo; s_hi[g][sp] = mid;
                    s_sp[g] = sp + 1;
                } else {
                    atomicOr(err, ERR_CAP);   // cannot happen while limit >= 1; reported, not hung
                }
            }
            grp_sync<T>();
            continue;
        }
        c4 += c4r;
        if (PE) {
            // credit sweep: the counts of this range are final.  With one chunk of sources in
            // one super-tile the count sweep's run tables are still in place.
            const bool one = (re - rb) <= T && tot1 <= SPOS;
            // credits the wedges of one batch starting at position q0 (x = -1: no wedge; the
            // lane still takes part in the wavefront's prefix sums)
            auto credit_batch = [&](int q0, int sb0, int se, const int (&xs)[IL], const int (&ks)[IL],
                                    const int (&is)[IL]) {
#pragma unroll
                for (int j = 0; j < IL; j++) {
                    const int x = xs[j], kj = ks[j], ij = is[j];
                    u32 c = 0;
                    if (x >= 0) {
                        u32 cnt = 1;
                        if (x >= base) {
                            cnt = cnt_get<P16>(dc, x - base);
                        } else {
                            u32 h = hslot(x, mask);
                            int p = 0;
                            while (p < HT && hk[h] != x) { h = (h + 1) & mask; p++; }
                            if (p < HT) cnt = cnt_get<P16>(hc, (int)h);
                            else atomicOr(err, ERR_CAP);
                        }
                        c = cnt - 1;
                        if (NR) c4 += (u64)c;   // sums to 2 x sum over tops of C(c, 2)
                    }
                    // the wavefront's lanes cover one word of the run tables, whose start
                    // bits (and every idle lane) delimit the sources
                    const int qw = q0 + j * T + (tid & ~(GLT_WAVE - 1));
                    const int idle = se - qw;   // lanes >= idle have no wedge
                    u64 F = rt.msk[(qw - sb0) >> 6] | 1ull;
                    if (idle <= 0) F = ~0ull;
                    else if (idle < GLT_WAVE) F |= ~0ull << idle;
                    const int l = glt_lane();
                    const bool first = (F >> l) & 1;
                    const bool last = (l == GLT_WAVE - 1) || (((F >> l) >> 1) & 1);
                    if (c) acc_add<AT, ACC_P>(e, kj, (u64)c);   // top edge (w, x)
                    // bottom edge (y, w): with P the wave's inclusive prefix of c, a
                    // source's sum is P(last lane) - P(first lane - 1): its first lane
                    // subtracts its exclusive prefix and its last lane adds its inclusive
                    // one (modular arithmetic, exact once both have landed).  While the
                    // row is short enough that 64 counts sum below 2^31 the prefix is
                    // formed in 32 bits and each lane's term sign-extended.
                    AT v;
                    if (sizeof(AT) == 4 || scan32) {
                        const u32 P = wave_incl_scan<u32>(c);
                        v = (AT)(int64_t)(int32_t)((last ? P : 0u) - (first ? P - c : 0u));
                    } else {
                        const AT P = wave_incl_scan<AT>((AT)c);
                        v = (last ? P : (AT)0) - (first ? (AT)(P - c) : (AT)0);
                    }
                    if (v) atomicAdd(&sb[ij], v);
                }
            };
            for (int c0 = rb; c0 < re; c0 += T) {
                const int s = c0 + tid;
                int tot = tot1, carry = 0;
                if (!one) {
                    int k0 = 0, k1 = 0;
                    if (s < re) wedge_bounds(s, lo, hi, full, wb, ocol, k0, k1);
                    len = k1 - k0;
                    tot = runs_begin<T>(rt, len, k0, pre, carry);
                }
                sb[tid] = 0;
                grp_sync<T>();
                for (int sb0 = 0; sb0 < tot; sb0 += SPOS) {
                    if (sb0 > 0) runs_next<T>(rt, sb0, len, pre, carry);
                    const int se = min(tot, sb0 + SPOS);
                    // the same two alternating register sets as the count sweep
                    int xa[IL], ka[IL], ia[IL], xb[IL], kb[IL], ib[IL];
                    wedge_slots<T, IL>(rt, ocol, sb0, se, sb0 + tid, xa, ka, ia);
                    for (int q0 = sb0; q0 < se; q0 += (WEDGE_PF ? 2 : 1) * IL * T) {
                        if constexpr (WEDGE_PF) {
                            wedge_slots<T, IL>(rt, ocol, sb0, se, q0 + IL * T + tid, xb, kb, ib);
                            credit_batch(q0, sb0, se, xa, ka, ia);
                            if (q0 + IL * T >= se) break;
                            wedge_slots<T, IL>(rt, ocol, sb0, se, q0 + 2 * IL * T + tid, xa, ka, ia);
                            credit_batch(q0 + IL * T, sb0, se, xb, kb, ib);
                        } else {
                            if (q0 > sb0) wedge_slots<T, IL>(rt, ocol, sb0, se, q0 + tid, xa, ka, ia);
                            credit_batch(q0, sb0, se, xa, ka, ia);
                        }
                    }
                }
                grp_sync<T>();
                if (s < re && sb[tid]) acc_add<AT, ACC_P>(e, s2k[s], (u64)sb[tid]);
                grp_sync<T>();
            }
        }
        grp_sync<T>();
    }
    // the group's total (with NR twice the 4-cycles of y, even), added once
    c4 = wave_sum(c4);
    if constexpr (T > GLT_WAVE) {
        grp_sync<T>();
        if (glt_lane() == 0) rt.scan[tid / GLT_WAVE] = c4;
        grp_sync<T>();
        c4 = 0;
        for (int q = 0; q < T / GLT_WAVE; q++) c4 += rt.scan[q];
    }
    if (NR) c4 >>= 1;
    if (tid == 0 && c4) atomicAdd(&gsum[gslot(ngid, y) * NSUMS + S_NC4], c4);
    // load-balance measurement (when asked): the wall clock at which this list entry is done
    if (tstamp && tid == 0) tstamp[item] = (u64)wall_clock64();
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

// The combine walks the edges in the caller's order, so its reads of the edge and vertex
// arrays are scattered.  With 32-bit accumulators they are first packed, in oriented-edge
// and vertex order (coalesced), into one 32-byte record per edge and per vertex: the
// combine then gathers three records per edge instead of a dozen scattered words.
struct __align__(32) ERec {
    int u, v;
    u32 t, K, P, pad;
    u64 gsig;   // g (low half), sigma (high half)
};
struct __align__(32) VRec {
    u64 tri, sdeg;
    int deg, pad[3];
};

__global__ __launch_bounds__(256) void k_pack_edges(EdgeArrays e, const int* __restrict__ ocol, int m,
                                                    ERec* __restrict__ er) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    ERec r;
    r.u = e.u[k];
    r.v = ocol[k];
    r.t = e.t[k];
    r.K = ((const u32*)e.K)[k];
    r.P = ((const u32*)e.P)[k];
    r.pad = 0;
    r.gsig = e.g[k];
    er[k] = r;
}

__global__ __launch_bounds__(256) void k_pack_vertices(const u64* __restrict__ tri, const u64* __restrict__ sdeg,
                                                       const int* __restrict__ ndeg, int n, VRec* __restrict__ vr) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    VRec r;
    r.tri = tri[x];
    r.sdeg = sdeg[x];
    r.deg = ndeg[x];
    r.pad[0] = r.pad[1] = r.pad[2] = 0;
    vr[x] = r;
}

// PK: per-edge inputs from the packed records (per-edge mode with 32-bit accumulators).
template <bool PE, typename AT, bool PK>
__global__ __launch_bounds__(CB_THREADS) void k_combine(const int* __restrict__ eid2k, EdgeArrays e,
                                                        const int* __restrict__ ocol,
                                                        const int* __restrict__ ndeg, const u64* __restrict__ tri,
                                                        const u64* __restrict__ sdeg, const ERec* __restrict__ er,
                                                        const VRec* __restrict__ vr, int n, int m,
                                                        u64* __restrict__ out, u64* __restrict__ part,
                                                        int* __restrict__ err) {
    static_assert(!PK || (PE && sizeof(AT) == 4), "packed records hold 32-bit accumulators");
    __shared__ u64 red[CB_THREADS / GLT_WAVE][NCS][2];
    u64 lo[NCS], hi[NCS];
#pragma unroll
    for (int c = 0; c < NCS; c++) { lo[c] = 0; hi[c] = 0; }
    int bad = 0;
    const int64_t e0 = (int64_t)blockIdx.x * CB_THREADS * CB_EPT;
    for (int r = 0; r < CB_EPT; r++) {
        const int64_t eid = e0 + (int64_t)r * CB_THREADS + threadIdx.x;
        if (eid >= m) break;
        const int k = PE ? eid2k[eid] : (int)eid;   // global sums: any edge order, here oriented
        int u, v;
        int64_t du, dv, t, Kk = 0, Pk = 0, triu = 0, triv = 0, sdu = 0, sdv = 0;
        u64 gk = 0, sk = 0;
        if constexpr (PK) {
            const ERec r = er[k];
            u = r.u; v = r.v;
            const VRec a = vr[u], b = vr[v];
            du = a.deg; dv = b.deg;
            t = r.t; Kk = r.K; Pk = r.P;
            gk = r.gsig & 0xffffffffull; sk = r.gsig >> 32;
            triu = (int64_t)a.tri; triv = (int64_t)b.tri; sdu = (int64_t)a.sdeg; sdv = (int64_t)b.sdeg;
        } else {
            u = e.u[k]; v = ocol[k];
            du = ndeg[u]; dv = ndeg[v];
            t = e.t[k];
            if (PE) {
                Kk = (int64_t)acc_get<AT, ACC_K>(e, k);
                Pk = (int64_t)acc_get<AT, ACC_P>(e, k);
                gsig_get<AT>(e, k, gk, sk);
                triu = (int64_t)tri[u]; triv = (int64_t)tri[v]; sdu = (int64_t)sdeg[u]; sdv = (int64_t)sdeg[v];
            }
        }
        const int64_t su = du - 1 - t, sv = dv - 1 - t;
        const int64_t D = (int64_t)n - 2 - t - su - sv;
        int64_t K = 0, Q = 0;
        if (PE) {
            K = Kk;
            const int64_t P = Pk;
            const int64_t A = (int64_t)gk - 2 * t - 4 * K;     // edges T-S_u plus T-S_v
            Q = P - 2 * K - A;                                      // edges S_u-S_v
            const int64_t sigT = (int64_t)sk;
            const int64_t E2 = ((triu + triv) >> 1) - 2 * t - 2 * K - A;   // inside S_u plus inside S_v
            const int64_t ETD = sigT - 2 * t - 2 * K - A;           // edges T-D
            const int64_t ESD = (sdu - dv - sigT) + (sdv - du - sigT) - su - sv - 2 * E2 - A -
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

// 128-bit reduction of per-block partial records (NCS (lo, hi) pairs each) into one record
// per workgroup at out.  The records are read as 16-byte (lo, hi) items in address order;
// a workgroup's 1014 = 78 x NCS active threads step by a multiple of NCS items, so every
// thread keeps to one column (its index mod NCS) and the loads stay coalesced.
#define RP_ACT ((1024 / NCS) * NCS)
__global__ __launch_bounds__(1024) void k_reduce_parts(const u64* __restrict__ part, int nparts,
                                                       u64* __restrict__ out) {
    __shared__ u64 red[RP_ACT][2];
    const int t = threadIdx.x;
    if (t < RP_ACT) {
        u64 lo = 0, hi = 0;
        const int64_t items = (int64_t)nparts * NCS;
        const int64_t stride = (int64_t)gridDim.x * RP_ACT;
        const ulonglong2* p = reinterpret_cast<const ulonglong2*>(part);
        for (int64_t q = (int64_t)blockIdx.x * RP_ACT + t; q < items; q += stride) {
            const ulonglong2 v = p[q];
            add128(lo, hi, v.x);
            hi += v.y;
        }
        red[t][0] = lo;
        red[t][1] = hi;
    }
    __syncthreads();
    if (t < NCS) {
        u64 L = 0, H = 0;
        for (int q = t; q < RP_ACT; q += NCS) {
            add128(L, H, red[q][0]);
            H += red[q][1];
        }
        out[((int64_t)blockIdx.x * NCS + t) * 2] = L;
        out[((int64_t)blockIdx.x * NCS + t) * 2 + 1] = H;
    }
}

// Partial records of nb combine blocks -> final_sums: one workgroup per RP_ACT x 2 items
// (at most GLT_REDUCE_BLOCKS) writing records behind the partials, then one workgroup.
static void reduce_parts(const Dev& d, int nb, hipStream_t st) {
    const int64_t items = (int64_t)nb * NCS;
    int r = (int)((items + 2 * RP_ACT - 1) / (2 * RP_ACT));
    if (r > GLT_REDUCE_BLOCKS) r = GLT_REDUCE_BLOCKS;
    if (r <= 1) {
        hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(1024), 0, st, d.sums, nb, d.final_sums);
        return;
    }
    u64* mid = d.sums + (int64_t)d.nsum_slots * NCS * 2;
    hipLaunchKernelGGL(k_reduce_parts, dim3(r), dim3(1024), 0, st, d.sums, nb, mid);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(1024), 0, st, mid, r, d.final_sums);
}

// Batched global mode: one workgroup per graph over its oriented edges, unrestricted sums
// with the graph's own n and m.
__global__ __launch_bounds__(CB_THREADS) void k_combine_graphs(const int64_t* __restrict__ vb,
                                                               const int* __restrict__ gcb, int ngraphs,
                                                               const int* __restrict__ optr, EdgeArrays e,
                                                               const int* __restrict__ ocol,
                                                               const int* __restrict__ ndeg,
                                                               u64* __restrict__ cparts) {
    __shared__ u64 red[CB_THREADS / GLT_WAVE][NCS][2];
    const int b = blockIdx.x;
    // this chunk's graph: the last g with gcb[g] <= b (graphs without edges own no chunk)
    int glo = 0, ghi = ngraphs;
    while (ghi - glo > 1) {
        const int mid = (glo + ghi) >> 1;
        if (gcb[mid] <= b) glo = mid; else ghi = mid;
    }
    const int g = glo;
    const int64_t ng = vb[g + 1] - vb[g];
    // graph g's vertices hold the ranks [vb[g], vb[g + 1]), so its oriented edges are the
    // contiguous range below (the sums do not depend on the edge order)
    const int64_t eg0 = optr[vb[g]], eg1 = optr[vb[g + 1]], mg = eg1 - eg0;
    const int64_t e0 = eg0 + (int64_t)(b - gcb[g]) * CG_CHUNK;
    const int64_t e1 = min(e0 + (int64_t)CG_CHUNK, eg1);
    u64 lo[NCS], hi[NCS];
#pragma unroll
    for (int c = 0; c < NCS; c++) { lo[c] = 0; hi[c] = 0; }
    for (int64_t k = e0 + threadIdx.x; k < e1; k += CB_THREADS) {
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
        cparts[((int64_t)b * NCS + c) * 2] = L;
        cparts[((int64_t)b * NCS + c) * 2 + 1] = H;
    }
}

// Per graph (one wave each), the sum of its chunks' 128-bit partials (zero for a graph
// without edges): lanes stride over the chunks, then a wave reduction.
__global__ __launch_bounds__(GLT_WAVE) void k_fold_graph_parts(const int* __restrict__ gcb,
                                                               const u64* __restrict__ cparts,
                                                               u64* __restrict__ gparts) {
    const int g = blockIdx.x, l = threadIdx.x;
    const int b0 = gcb[g], b1 = gcb[g + 1];
    for (int c = 0; c < NCS; c++) {
        u64 L = 0, H = 0;
        for (int b = b0 + l; b < b1; b += GLT_WAVE) {
            const u64 o = L;
            L += cparts[((int64_t)b * NCS + c) * 2];
            H += cparts[((int64_t)b * NCS + c) * 2 + 1] + ((L < o) ? 1ull : 0ull);
        }
        wave_sum128(L, H);
        if (l == 0) {
            gparts[((int64_t)g * NCS + c) * 2] = L;
            gparts[((int64_t)g * NCS + c) * 2 + 1] = H;
        }
    }
}

// ---------------------------------------------------------------------------------------
// heaviest-first order of the workgroup work lists (the paper's edge order: hardest jobs
// first, Section 4.3), so the longest jobs do not start last and run alone
// ---------------------------------------------------------------------------------------
// mode 0: work = wedges of y (wcnt); mode 1: work = out-degree of x.  The sort key is a
// 13-bit monotone code of the work (exact below 256, else exponent and the 7 bits after the
// leading one), so two 8-bit radix passes order the list.
__device__ __forceinline__ u32 work_code(u64 w) {
    if (w < 256) return (u32)w;
    const int ex = 63 - __clzll((long long)w);          // >= 8
    const u32 top = (u32)(w >> (ex - 7));               // [128, 256)
    return 256u + (u32)(ex - 8) * 128u + (top - 128u);  // < 7424
}

// order: LO_WORK sorts by the work (mode 0: wedges of y, mode 1: out-degree of x), LO_DEGREE
// by the vertex's degree, LO_VOLUME by its volume (vol), all largest first; LO_DEGREE_INV and
// LO_VOLUME_INV smallest first; LO_RANDOM by a hash of the vertex.
__global__ void k_work_keys(const int* __restrict__ list, int nlist, int mode, int order,
                            const u64* __restrict__ wcnt, const int* __restrict__ optr,
                            const int* __restrict__ ndeg, const u64* __restrict__ vol,
                            u64* __restrict__ keys, u32* __restrict__ vals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlist) return;
    const int x = list[i];
    u32 key;
    if (order == LO_RANDOM) {
        key = ((u32)x * 2654435761u) >> 16;
    } else {
        const bool deg = order == LO_DEGREE || order == LO_DEGREE_INV;
        const bool vl = order == LO_VOLUME || order == LO_VOLUME_INV;
        const u64 w = deg ? (u64)ndeg[x] : vl ? vol[x] : mode == 0 ? wcnt[x] : (u64)(optr[x + 1] - optr[x]);
        const bool inv = order == LO_DEGREE_INV || order == LO_VOLUME_INV;
        key = inv ? work_code(w) : 0xffffu - work_code(w);   // ascending sort
    }
    keys[i] = (u64)key;
    vals[i] = (u32)x;
}

// Volume of every relabelled vertex, vol(x) = sum of its neighbours' degrees (the vertex form
// of Table 4's vol(e)), for the volume orders of the work lists.
__global__ __launch_bounds__(256) void k_volume(const int* __restrict__ nsrow, const int* __restrict__ ncol,
                                                const int* __restrict__ ndeg, int64_t S, u64* __restrict__ vol) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    u64 d = 0;
    int x = 0x7fffffff;
    if (s < S) {
        x = nsrow[s];
        d = (u64)ndeg[ncol[s]];
    }
    bool last;   // runs of one row are summed in the wavefront first
    const u64 r = seg_sum_last(d, x, last);
    if (last && x != 0x7fffffff && r) atomicAdd(&vol[x], r);
}

__global__ void k_copy_list(const u32* __restrict__ vals, int nlist, int* __restrict__ list) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nlist) list[i] = (int)vals[i];
}

static void sort_heaviest_first(const Dev& d, int* list, int nlist, int mode, hipStream_t st) {
    if (nlist < 2 || d.list_order == LO_NONE) return;   // LO_NONE: the bucketing order (ascending rank)
    const unsigned g = (unsigned)((nlist + 255) / 256);
    hipLaunchKernelGGL(k_work_keys, dim3(g), dim3(256), 0, st, list, nlist, mode, d.list_order, d.wcnt, d.optr,
                       d.ndeg, d.sdeg, d.key0, d.val0);
    const int cur = launch_radix_sort(d.key0, d.val0, d.key1, d.val1, nlist, 16, d.rs_counts, d.rs_tmp, st);
    hipLaunchKernelGGL(k_copy_list, dim3(g), dim3(256), 0, st, cur ? d.val1 : d.val0, nlist, list);
}

// Per-group totals (4-cliques x 3, 4-cycles, triangles per path) are added with one atomic
// per group into GSPREAD cache lines (single graph) or one line per graph (batch), so that
// hundreds of thousands of groups do not contend on one address.  One workgroup folds the
// lines: the single-graph sums land in line 0; the triangle totals go to work[4], work[5],
// and the other work counters (spread the same way) to work[0..3], work[6], work[7].
__global__ __launch_bounds__(256) void k_fold_gsum(u64* __restrict__ gsum, int ngraphs, u64* __restrict__ work,
                                                   const u64* __restrict__ wspread) {
    __shared__ u64 red[2][256 / GLT_WAVE];
    const int t = threadIdx.x;
    // spread work counters: words 0, 1, 4, 5 wedges of the wave, workgroup, mid and huge
    // classes as bucketed, 2, 3 triangle-pass list entries per path, 6 wedges of bottoms that
    // moved from the workgroup to the huge class, 7 from the mid to the workgroup class,
    // 8-11 the most wedges of one bottom bucketed to the wave, mid, workgroup, huge class
    // (folded by maximum, work[8..11])
    __shared__ u64 wsum[WSPREAD_WORDS];
    if (t < WSPREAD_WORDS) {
        u64 v = 0;
        for (int q = 0; q < GSPREAD; q++) {
            const u64 x = wspread[q * WSPREAD_WORDS + t];
            v = t < 8 ? v + x : (x > v ? x : v);
        }
        wsum[t] = v;
    }
    __syncthreads();
    if (t == 0) {
        work[0] = wsum[0];
        work[1] = wsum[1] - wsum[6] + wsum[7];
        work[2] = wsum[2];
        work[3] = wsum[3];
        work[6] = wsum[4] - wsum[7];
        work[7] = wsum[5] + wsum[6];
        for (int c = 0; c < 4; c++) work[8 + c] = wsum[8 + c];
    }
    if (ngraphs <= 0) {
        u64 v = 0;
        if (t < NSUMS)
            for (int q = 0; q < GSPREAD; q++) v += gsum[q * NSUMS + t];
        __syncthreads();
        if (t < NSUMS) gsum[t] = v;
        if (t == GS_TRI_WAVE) work[4] = v;
        if (t == GS_TRI_WG) work[5] = v;
        return;
    }
    u64 a = 0, b = 0;
    for (int g = t; g < ngraphs; g += 256) { a += gsum[(int64_t)g * NSUMS + GS_TRI_WAVE]; b += gsum[(int64_t)g * NSUMS + GS_TRI_WG]; }
    a = wave_sum(a);
    b = wave_sum(b);
    if (glt_lane() == 0) { red[0][t / GLT_WAVE] = a; red[1][t / GLT_WAVE] = b; }
    __syncthreads();
    if (t == 0) {
        u64 ta = 0, tb = 0;
        for (int q = 0; q < 256 / GLT_WAVE; q++) { ta += red[0][q]; tb += red[1][q]; }
        work[4] = ta;
        work[5] = tb;
    }
}

static inline int combine_blocks(int m) { return (int)(((int64_t)m + CB_THREADS * CB_EPT - 1) / (CB_THREADS * CB_EPT)); }

// ---------------------------------------------------------------------------------------
// host orchestration of the passes
// ---------------------------------------------------------------------------------------
static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <bool PE, typename AT>
static void launch_tri_wave(const Dev& d, const int* lst, int c, hipStream_t st) {
    if (d.trec)
        hipLaunchKernelGGL((k_tri_wave<PE, true, AT>), dim3(cdiv(c, TW_G)), dim3(TW_THREADS), 0, st, lst, c, d.optr, d.ocol,
                           d.e, d.gsum, d.ngid, d.trec, d.toff, d.tcnt);
    else
        hipLaunchKernelGGL((k_tri_wave<PE, false, AT>), dim3(cdiv(c, TW_G)), dim3(TW_THREADS), 0, st, lst, c, d.optr,
                           d.ocol, d.e, d.gsum, d.ngid, d.trec, d.toff, d.tcnt);
}

// Threads per workgroup of the triangle pass: 256 for out-degrees up to 256 (small LDS
// tables, many workgroups per CU), TB_BIG_THREADS above, where the rows' LDS allows only a
// few workgroups per CU and larger groups keep more out-list loads in flight.
#ifndef TB_BIG_THREADS
#define TB_BIG_THREADS 1024
#endif
template <bool PE, bool GM, typename AT, int NT, bool GX>
static void launch_tri_blk_nt(const Dev& d, const int* lst, int c, int smax, int64_t gstride, hipStream_t st) {
    const size_t lds = tri_blk_lds(smax, GM, GX);
    if (d.trec)
        hipLaunchKernelGGL((k_tri_blk<PE, GM, true, AT, NT, GX>), dim3(c), dim3(NT), lds, st, lst, c, smax, d.optr,
                           d.ocol, d.e, d.gsum, d.gscratch, gstride, d.ngid, d.trec, d.toff, d.tcnt);
    else
        hipLaunchKernelGGL((k_tri_blk<PE, GM, false, AT, NT, GX>), dim3(c), dim3(NT), lds, st, lst, c, smax, d.optr,
                           d.ocol, d.e, d.gsum, d.gscratch, gstride, d.ngid, d.trec, d.toff, d.tcnt);
}
template <bool PE, bool GM, typename AT, bool GX = false>
static void launch_tri_blk(const Dev& d, const int* lst, int c, int smax, int64_t gstride, hipStream_t st) {
    if (smax <= 256) launch_tri_blk_nt<PE, GM, AT, TB_THREADS, GX>(d, lst, c, smax, gstride, st);
    else launch_tri_blk_nt<PE, GM, AT, TB_BIG_THREADS, GX>(d, lst, c, smax, gstride, st);
}

template <bool GM, typename AT, bool GX = false>
static void launch_gather_blk(const Dev& d, const int* lst, int c, int smax, int64_t gstride, hipStream_t st) {
    const size_t lds = gather_blk_lds(smax, GM, GX);
    if (d.trec)
        hipLaunchKernelGGL((k_gather_blk<GM, true, AT, GX>), dim3(c), dim3(TB_THREADS), lds, st, lst, c, smax, d.optr,
                           d.ocol, d.ndeg, d.e, (u64*)d.gscratch, gstride, d.trec, d.toff, d.tcnt);
    else
        hipLaunchKernelGGL((k_gather_blk<GM, false, AT, GX>), dim3(c), dim3(TB_THREADS), lds, st, lst, c, smax, d.optr,
                           d.ocol, d.ndeg, d.e, (u64*)d.gscratch, gstride, d.trec, d.toff, d.tcnt);
}

// Words per workgroup of the global slab for the out-degree bucket above the LDS rows, whose
// largest out-degree is smax: its triangle and gather launches share the regions.
static inline int64_t gm_slab_words(int smax) {
    const int s0 = smax < TB_LDS_SMAX ? smax : TB_LDS_SMAX;
    int64_t w = tri_slab_words(s0, false);
    const int64_t g0 = gather_slab_words(s0, false);
    if (g0 > w) w = g0;
    if (smax > TB_LDS_SMAX) {
        const int64_t t1 = tri_slab_words(smax, true), g1 = gather_slab_words(smax, true);
        if (t1 > w) w = t1;
        if (g1 > w) w = g1;
    }
    return w;
}

// Where a wedge class sends the bottoms whose distinct tops overflow its tables: a list, its
// device counter, and the work counter that moves their wedges between classes.
struct WedgeDefer {
    int* list = nullptr;
    int* cnt = nullptr;
    u64* work = nullptr;
};

// One group per list entry (grid from the host's count), or, with `resident` blocks, a grid
// that walks the list up to the device count at `dcount`; overflowing entries go to `df`.
// Resident grids (workgroups per CU; 0: one group per list entry).  A resident group walks
// several list entries and loads the next entry's bounds while it counts the current one:
// the wave class, whose bottoms have at most 128 wedges, spends most of an entry's time on
// that chain of dependent loads (10,000-graph batch: 41 -> 7 ms).  The mid class measured
// slower resident (38 -> 51..68 ms: its heavier entries, walked with a fixed stride, balance
// worse than one group per entry).
#ifndef WEDGE_RES_WAVE
#define WEDGE_RES_WAVE 8
#endif
#ifndef WEDGE_RES_MID
#define WEDGE_RES_MID 0
#endif
// Workgroups for a list of cnt entries, G per workgroup: one per entry up to `cap`.
static inline int resident_grid(int cnt, int G, int cap) {
    const int64_t need = ((int64_t)cnt + G - 1) / G;
    return (int)(need < cap ? need : cap);
}

template <bool PE, typename AT, int T, int G, int HT, int DW, bool P16 = false, int IL = WEDGE_ILP>
static void launch_wedge_list(const Dev& d, const int* list, int cnt, const int* dcount, hipStream_t st, int resident,
                              WedgeDefer df, u64* tstamp) {
    if (cnt <= 0 && resident <= 0) return;
    const int limit = d.wedge_limit < HT / 2 ? d.wedge_limit : HT / 2;
    const unsigned grid = resident > 0 ? (unsigned)resident : cdiv(cnt, G);
    hipLaunchKernelGGL((k_wedge<PE, AT, T, G, HT, DW, P16, IL>), dim3(grid), dim3(T * G), 0, st, list, cnt, d.n,
                       limit, d.wedge_dense, d.nrp, d.wb, d.ocol, d.s2k, d.wcnt, d.e, d.gsum, d.ngid, d.vtop, d.err,
                       resident > 0 ? dcount : nullptr, df.list, df.cnt, df.work, tstamp);
}

// One class's own list (grid from the host's count, or resident walking the device count),
// overflowing bottoms sent to class `defer` (>= 0).
template <bool PE, typename AT, int T, int G, int HT, int DW, bool P16 = false, int IL = WEDGE_ILP>
static void launch_wedge(const Dev& d, int bkt, int cnt, hipStream_t st, int resident = 0, int defer = -1) {
    int* counts = d.counts + TB_N;
    WedgeDefer df;
    if (defer >= 0) {
        df.list = d.wlist + (int64_t)defer * d.n;
        df.cnt = counts + defer;
        df.work = d.wspread + 6;
    }
    launch_wedge_list<PE, AT, T, G, HT, DW, P16, IL>(d, d.wlist + (int64_t)bkt * d.n, cnt, counts + bkt, st, resident,
                                                     df, bkt == WB_BLK ? d.tstamp : nullptr);
}

// Events of one call (all recorded, also used to fork and join; the stream modes are
// described at count_passes):
//   ev[0] start                            ev[1] end of preprocessing (fork)
//   ev[2..5] after tri wave / tri wg / gather wave / gather wg
//   ev[12], ev[13] start of the gather wavefront / workgroup path (after their joins)
//   ev[14] start of the wave class          ev[6], ev[7] after the wave / mid classes
//   ev[15] start of the workgroup class     ev[8], ev[9] after the workgroup / huge classes
//   ev[10] after the last join              ev[11] after the combine
//   ev[16] after the (t, K) unpack (mode 2: the second stream's gather path waits for it)
// The passes share only read-only inputs and write distinct accumulators, so the streams
// join only where a pass needs another's final values (the gather pass needs every t).
// Wave class, and mid class, on stream s (ev[6], ev[7] after each).
template <typename AT>
static void wedge_wave_class(const Dev& d, int per_edge, const int* hc, hipStream_t s, hipEvent_t* ev) {
    const int* wc = hc + TB_N;
    const int res = wc[WB_WAVE] > 0 ? resident_grid(wc[WB_WAVE], WW_G, d.num_cu * WEDGE_RES_WAVE) : 0;
    if (per_edge) launch_wedge<true, AT, WW_T, WW_G, WW_HT, 0, false>(d, WB_WAVE, wc[WB_WAVE], s, res);
    else launch_wedge<false, AT, WW_T, WW_G, WW_HT, 0>(d, WB_WAVE, wc[WB_WAVE], s, res);
    (void)hipEventRecord(ev[6], s);
}

// The mid class hands a bottom whose distinct tops overflow its tables on the first try to
// the workgroup class (appended after that class's own entries, counted in CNT_MID_TO_WG)
// instead of splitting its top range: on R-MAT most such bottoms would need several splits,
// each re-scanning their sources (mid class 40.7 -> 1.3 ms, workgroup class 44.5 -> 52 ms).
template <typename AT>
static void wedge_mid_class(const Dev& d, int per_edge, const int* hc, hipStream_t s, hipEvent_t* ev) {
    const int* wc = hc + TB_N;
    WedgeDefer df;
    df.list = d.wlist + (int64_t)WB_BLK * d.n + wc[WB_BLK];
    df.cnt = d.counts + CNT_MID_TO_WG;
    df.work = d.wspread + 7;
    const int* lst = d.wlist + (int64_t)WB_MID * d.n;
    const int* dc = d.counts + TB_N + WB_MID;
    const int res = wc[WB_MID] > 0 ? resident_grid(wc[WB_MID], WM_G, d.num_cu * WEDGE_RES_MID) : 0;
    if (per_edge) launch_wedge_list<true, AT, WM_T, WM_G, WM_HT, WM_DW, true>(d, lst, wc[WB_MID], dc, s, res, df, nullptr);
    else launch_wedge_list<false, AT, WM_T, WM_G, WM_HT, WM_DW, true>(d, lst, wc[WB_MID], dc, s, res, df, nullptr);
    (void)hipEventRecord(ev[7], s);
}

// Workgroup class first: its bottoms whose tops overflow its tables join the huge list,
// which one resident workgroup per CU then walks (ev[15] before, ev[8], ev[9] after each).
template <typename AT>
static void wedge_large(const Dev& d, int per_edge, const int* hc, hipStream_t s, hipEvent_t* ev) {
    const int* wc = hc + TB_N;
    const int huge_grid = (wc[WB_MID] + wc[WB_BLK] + wc[WB_HUGE] > 0) ? d.num_cu * WH_PER_CU : 0;
    (void)hipEventRecord(ev[15], s);
    if (per_edge) launch_wedge<true, AT, WB_T, 1, WB_HT, WB_DW, false, WEDGE_ILP_WG>(d, WB_BLK, wc[WB_BLK], s, 0, WB_HUGE);
    else launch_wedge<false, AT, WB_T, 1, WB_HT, WB_DW, false, WEDGE_ILP_WG>(d, WB_BLK, wc[WB_BLK], s, 0, WB_HUGE);
    if (wc[WB_MID] > 0) {
        // the bottoms the mid class handed over: a resident grid walks them up to their device
        // count (unknown to the host), overflowing ones go on to the huge class
        WedgeDefer df;
        df.list = d.wlist + (int64_t)WB_HUGE * d.n;
        df.cnt = d.counts + TB_N + WB_HUGE;
        df.work = d.wspread + 6;
        const int* lst = d.wlist + (int64_t)WB_BLK * d.n + wc[WB_BLK];
        const int res = d.num_cu * WB_RESIDENT;
        if (per_edge)
            launch_wedge_list<true, AT, WB_T, 1, WB_HT, WB_DW, false, WEDGE_ILP_WG>(d, lst, 0, d.counts + CNT_MID_TO_WG, s, res, df, nullptr);
        else
            launch_wedge_list<false, AT, WB_T, 1, WB_HT, WB_DW, false, WEDGE_ILP_WG>(d, lst, 0, d.counts + CNT_MID_TO_WG, s, res, df, nullptr);
    }
    (void)hipEventRecord(ev[8], s);
    if (per_edge) launch_wedge<true, AT, WH_T, 1, WH_HT, WH_DW, false, WEDGE_ILP_HUGE>(d, WB_HUGE, wc[WB_HUGE], s, huge_grid);
    else launch_wedge<false, AT, WH_T, 1, WH_HT, WH_DW, false, WEDGE_ILP_HUGE>(d, WB_HUGE, wc[WB_HUGE], s, huge_grid);
    (void)hipEventRecord(ev[9], s);
}

template <typename AT>
static void wedge_pass(const Dev& d, int per_edge, const int* hc, hipStream_t s, hipEvent_t* ev) {
    wedge_wave_class<AT>(d, per_edge, hc, s, ev);
    wedge_mid_class<AT>(d, per_edge, hc, s, ev);
    wedge_large<AT>(d, per_edge, hc, s, ev);
}

// Vertex pass (needs final t only): triangles and neighbour-degree sums per vertex, and with
// packed combine records (per-edge mode, 32-bit accumulators) the per-vertex records.
template <typename AT>
static void vertex_sums(const Dev& d, hipStream_t s) {
    const int n = d.n, m = d.m;
    launch_fill<u64>(d.tri, n, 0ull, s);
    launch_fill<u64>(d.sdeg, n, 0ull, s);
    hipLaunchKernelGGL(k_vertex, dim3(cdiv(2 * (int64_t)m, 256)), dim3(256), 0, s, d.nsrow, d.ncol, d.s2k, d.ndeg,
                       d.e.t, 2 * (int64_t)m, d.tri, d.sdeg);
    if (sizeof(AT) == 4 && d.erec && d.vrec)
        hipLaunchKernelGGL(k_pack_vertices, dim3(cdiv(n, 256)), dim3(256), 0, s, d.tri, d.sdeg, d.ndeg, n,
                           (VRec*)d.vrec);
}

// Stream modes: 0 everything on st; 1 the wedge pass on `side`, beside the triangle and
// gather passes on st; 2 the workgroup paths of the triangle and gather passes on `side`,
// beside their wavefront paths on st (each gather path starts once both triangle paths
// are done), then the mid wedge class on `side` and the vertex pass and wave wedge class on
// st, and the workgroup and huge wedge classes alone on st after both.
template <typename AT>
static void count_passes(const Dev& d, int per_edge, const int* hc, u64* out_pe, hipStream_t st, hipStream_t side,
                         hipEvent_t* ev, int mode) {
    const bool overlap = mode == 1, split = mode == 2;
    const hipStream_t sw = split ? side : st;   // stream of the workgroup paths
    const int n = d.n, m = d.m;
    u64* gsum = d.gsum;                   // [graph][NSUMS]: 3 x 4-cliques and non-induced 4-cycles
    launch_fill<u64>(gsum, (int64_t)(d.ngraphs > 0 ? d.ngraphs : GSPREAD) * NSUMS, 0ull, st);
    const int* tl = d.tlist;
    const int* cnt = hc;                  // TB_N counts, WB_N counts, TB_N maxima
    const EdgeArrays e = d.e;
    if (d.list_order == LO_VOLUME || d.list_order == LO_VOLUME_INV) {
        // volumes for the sort keys (sdeg is recomputed by the vertex pass later)
        launch_fill<u64>(d.sdeg, n, 0ull, st);
        if (m > 0)
            hipLaunchKernelGGL(k_volume, dim3(cdiv(2 * (int64_t)m, 256)), dim3(256), 0, st, d.nsrow, d.ncol, d.ndeg,
                               2 * (int64_t)m, d.sdeg);
    }
    for (int bkt = TB_BLK1; bkt <= TB_GLOBAL; bkt++) sort_heaviest_first(d, d.tlist + (int64_t)bkt * n, cnt[bkt], 1, st);
    for (int bkt = WB_MID; bkt <= WB_HUGE; bkt++) sort_heaviest_first(d, d.wlist + (int64_t)bkt * n, hc[TB_N + bkt], 0, st);
    (void)hipEventRecord(ev[1], st);
    if (split) (void)hipStreamWaitEvent(side, ev[1], 0);
    if (overlap) {
        // the wedge pass on the side stream, beside the triangle and gather passes
        (void)hipStreamWaitEvent(side, ev[1], 0);
        (void)hipEventRecord(ev[14], side);
        wedge_pass<AT>(d, per_edge, hc, side, ev);
    }
    // triangle / 4-clique pass
    if (cnt[TB_WAVE] > 0) {
        if (per_edge) launch_tri_wave<true, AT>(d, tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], st);
        else launch_tri_wave<false, AT>(d, tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], st);
    }
    (void)hipEventRecord(ev[2], st);
    for (int bkt = TB_BLK1; bkt <= TB_GLOBAL; bkt++) {
        const int c = cnt[bkt];
        if (c <= 0) continue;
        const int smax = cnt[TB_N + WB_N + bkt];
        const bool gm = (bkt == TB_GLOBAL);
        const int* lst = tl + (int64_t)bkt * n;
        // the global slab holds one region per workgroup: launch in groups that fit it; the
        // out-degrees above TB_LDS_SMAX get a second launch over the same entries (GX)
        int64_t grp = c;
        const int64_t per = gm ? gm_slab_words(smax) : 0;
        const int s0 = smax < TB_LDS_SMAX ? smax : TB_LDS_SMAX;
        if (gm) {
            grp = d.gscratch_words / per;
            if (grp < 1) grp = 1;
        }
        for (int64_t off = 0; off < c; off += grp) {
            const int cc = (int)((c - off < grp) ? (c - off) : grp);
            if (per_edge) {
                if (gm) {
                    launch_tri_blk<true, true, AT>(d, lst + off, cc, s0, per, sw);
                    if (smax > TB_LDS_SMAX) launch_tri_blk<true, true, AT, true>(d, lst + off, cc, smax, per, sw);
                } else {
                    launch_tri_blk<true, false, AT>(d, lst + off, cc, smax, 0, sw);
                }
            } else {
                if (gm) {
                    launch_tri_blk<false, true, AT>(d, lst + off, cc, s0, per, sw);
                    if (smax > TB_LDS_SMAX) launch_tri_blk<false, true, AT, true>(d, lst + off, cc, smax, per, sw);
                } else {
                    launch_tri_blk<false, false, AT>(d, lst + off, cc, smax, 0, sw);
                }
            }
        }
    }
    (void)hipEventRecord(ev[3], sw);
    // the gather passes need every triangle's t: the call's stream waits for the workgroup
    // path, unpacks the narrow edges' (t, K) words, and the second stream waits for that
    if (split) (void)hipStreamWaitEvent(st, ev[3], 0);
    if (per_edge && m > 0)
        hipLaunchKernelGGL(k_unpack_tk, dim3(cdiv(m, 256)), dim3(256), 0, st, e, m);
    if (split) {
        (void)hipEventRecord(ev[16], st);
        (void)hipStreamWaitEvent(side, ev[16], 0);
    }
    (void)hipEventRecord(ev[12], st);
    (void)hipEventRecord(ev[13], sw);
    // gather pass
    if (per_edge && cnt[TB_WAVE] > 0) {
        if (d.trec)
            hipLaunchKernelGGL((k_gather_wave<true, AT>), dim3(cdiv(cnt[TB_WAVE], TW_G)), dim3(TW_THREADS), 0, st,
                               tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], d.optr, d.ocol, d.ndeg, e, d.trec, d.toff,
                               d.tcnt);
        else
            hipLaunchKernelGGL((k_gather_wave<false, AT>), dim3(cdiv(cnt[TB_WAVE], TW_G)), dim3(TW_THREADS), 0, st,
                               tl + (int64_t)TB_WAVE * n, cnt[TB_WAVE], d.optr, d.ocol, d.ndeg, e, d.trec, d.toff,
                               d.tcnt);
    }
    (void)hipEventRecord(ev[4], st);
    if (per_edge) {
        for (int bkt = TB_BLK1; bkt <= TB_GLOBAL; bkt++) {
            const int c = cnt[bkt];
            if (c <= 0) continue;
            const int smax = cnt[TB_N + WB_N + bkt];
            const int* lst = tl + (int64_t)bkt * n;
            const bool gm = (bkt == TB_GLOBAL);
            // the gather pass keeps its accumulators in LDS up to TB_LDS_SMAX (36 bytes per
            // neighbour); only the out-degrees above it use slab regions (GX)
            if (!gm || smax <= TB_LDS_SMAX) {
                launch_gather_blk<false, AT>(d, lst, c, smax, 0, sw);
                continue;
            }
            const int64_t per = gm_slab_words(smax);
            int64_t grp = d.gscratch_words / per;
            if (grp < 1) grp = 1;
            for (int64_t off = 0; off < c; off += grp) {
                const int cc = (int)((c - off < grp) ? (c - off) : grp);
                launch_gather_blk<false, AT>(d, lst + off, cc, TB_LDS_SMAX, 0, sw);
                launch_gather_blk<true, AT, true>(d, lst + off, cc, smax, per, sw);
            }
        }
    }
    (void)hipEventRecord(ev[5], sw);
    // mode 2: the mid wedge class follows the gather workgroup path on the second stream;
    // the vertex pass (t is final once st waited for both triangle paths; in no timed group)
    // and the wave wedge class follow the gather wavefront path on st
    const bool vsplit = split && per_edge && n > 0 && m > 0;
    if (split) {
        wedge_mid_class<AT>(d, per_edge, hc, side, ev);
        if (vsplit) vertex_sums<AT>(d, st);
        (void)hipEventRecord(ev[14], st);
        wedge_wave_class<AT>(d, per_edge, hc, st, ev);
        (void)hipStreamWaitEvent(st, ev[7], 0);   // join: the large classes run alone
        wedge_large<AT>(d, per_edge, hc, st, ev);
    } else if (overlap) {
        (void)hipStreamWaitEvent(st, ev[9], 0);   // join the wedge pass
    } else {
        (void)hipEventRecord(ev[14], st);
        wedge_pass<AT>(d, per_edge, hc, st, ev);
    }
    (void)hipEventRecord(ev[10], st);
    // vertex pass (unless done beside the gather pass) + combine
    if (per_edge && n > 0 && m > 0 && !vsplit) vertex_sums<AT>(d, st);
    const int nb = combine_blocks(m);
    if (d.ngraphs > 0) {
        if (d.ncchunks > 0)
            hipLaunchKernelGGL(k_combine_graphs, dim3(d.ncchunks), dim3(CB_THREADS), 0, st, d.gvb, d.gcb, d.ngraphs,
                               d.optr, e, d.ocol, d.ndeg, d.cparts);
        hipLaunchKernelGGL(k_fold_graph_parts, dim3(d.ngraphs), dim3(GLT_WAVE), 0, st, d.gcb, d.cparts, d.gparts);
    } else if (m > 0) {
        ERec* er = (ERec*)d.erec;
        VRec* vr = (VRec*)d.vrec;
        if (per_edge && sizeof(AT) == 4 && er && vr) {
            hipLaunchKernelGGL(k_pack_edges, dim3(cdiv(m, 256)), dim3(256), 0, st, e, d.ocol, m, er);
            if constexpr (sizeof(AT) == 4)
                hipLaunchKernelGGL((k_combine<true, AT, true>), dim3(nb), dim3(CB_THREADS), 0, st, d.eid2k, e, d.ocol,
                                   d.ndeg, d.tri, d.sdeg, er, vr, n, m, out_pe, d.sums, d.err);
        } else if (per_edge) {
            hipLaunchKernelGGL((k_combine<true, AT, false>), dim3(nb), dim3(CB_THREADS), 0, st, d.eid2k, e, d.ocol,
                               d.ndeg, d.tri, d.sdeg, er, vr, n, m, out_pe, d.sums, d.err);
        } else {
            hipLaunchKernelGGL((k_combine<false, AT, false>), dim3(nb), dim3(CB_THREADS), 0, st, d.eid2k, e, d.ocol,
                               d.ndeg, d.tri, d.sdeg, er, vr, n, m, out_pe, d.sums, d.err);
        }
        reduce_parts(d, nb, st);
    } else {
        launch_fill<u64>(d.final_sums, 2 * NCS, 0ull, st);
    }
    (void)hipEventRecord(ev[11], st);
    hipLaunchKernelGGL(k_fold_gsum, dim3(1), dim3(256), 0, st, gsum, d.ngraphs, d.work, d.wspread);
}

void glt_count_passes(const Dev& d, int per_edge, const int* hc, u64* out_pe, hipStream_t st, hipStream_t side,
                      hipEvent_t* ev, int mode) {
    if (d.acc32)
        count_passes<u32>(d, per_edge, hc, out_pe, st, side, ev, mode);
    else
        count_passes<u64>(d, per_edge, hc, out_pe, st, side, ev, mode);
}

int glt_combine_blocks(int m) { return combine_blocks(m); }
// words per workgroup of the global slab for the bucket above the LDS rows (largest out-degree smax)
int64_t glt_slab_words(int smax) { return gm_slab_words(smax); }
int glt_wedge_table() { return WH_HT; }
int glt_wedge_dense() { return WH_DW; }
int glt_wave_table() { return WW_HT; }
