// K3: LSD post-processing (paper Sec. III.C; order 0 and higher), one wavefront per shot.
//
// Clusters start as the flipped checks.  In every round each cluster that is
// still invalid adds its best boundary column (lowest soft value, then lowest
// index), judged on the state at the start of the round; clusters that come
// to share a check merge (union-find, smallest slot is the root).  A cluster
// is valid when s restricted to its checks lies in the span of its columns.
// Validity uses one pool of bit-packed basis vectors over the checks:
// vectors of different clusters have disjoint supports, so reducing a
// cluster's syndrome by the whole pool only ever touches that cluster's own
// vectors.  At the end, the columns of valid clusters are ranked and
// eliminated in rank order; a column is a pivot iff it is independent of
// the earlier ones, and every basis vector carries its combination of pivot
// columns, so reducing s yields the solution.  Both bases are kept in
// reduced echelon form (each vector is 1 at its own pivot and 0 at every
// other vector's pivot): a reduction then takes exactly the vectors whose
// pivot bit is set in the input and forms their sum in parallel.  The
// reduced vector, the pivots, the solution and the combinations are those
// of the elimination in insertion order, since a vector of the span is fixed
// by its bits at the pivots.
//
// Higher orders (lsd_order > 0) add the higher-order search that LSD-0
// leaves out (Sec. III.D.1 step 5), read as the combination sweep of ordered
// statistics decoding on every valid cluster.  Its non-pivot columns F, in
// rank order, give the candidates: none of F, each single column of F, each
// pair among the first lsd_order columns of F (lexicographic).  Setting the
// columns J of F moves the pivot solution by the xor of their pivot
// combinations, which the elimination leaves in the combination words of a
// non-pivot column.  The candidate of least prior weight (FP64, summed in
// ascending column index) replaces the cluster's OSD-0 solution; ties keep
// the earlier candidate.
#include "internal.h"

namespace vibe {

namespace {

// cluster state bits; kDirty: the cluster took a column or merged this round,
// so its validity must be computed again (an unchanged cluster keeps it)
constexpr uint32_t kValid = 1u, kFailed = 2u, kDirty = 4u;
constexpr size_t kLsdLds = 150 * 1024;  // LDS budget of one LSD wavefront
// row cache entries: the row's least column not yet held is unknown / none
constexpr int32_t kRowStale = -2, kRowEmpty = -1;

// Per-shot state.  Everything one lane writes and another reads lives in
// LDS.  The global part holds the large arrays: the basis vectors, which
// each lane only ever touches in its own words (w = lane mod 64), and the
// column lists of the final solve, which are read across lanes only through
// agent-scope loads (they bypass the CU's L1, whose copy of a line another
// lane just wrote is not refreshed by a workgroup barrier).
struct LsdMem {
    // LDS
    int32_t* chk_cl;    // m
    int32_t* parent;    // m
    uint32_t* cstate;   // m
    int64_t* best_q;    // m
    int32_t* best_v;    // m
    int32_t* ccount;    // m
    int32_t* picks;     // 2m (slot, column)
    int32_t* added;     // m
    int32_t* pool_piv;  // m
    int32_t* piv2;      // m
    int32_t* pivcol;    // m
    int64_t* row_q;     // m: key of the row's least column not yet held (lane 0 only)
    int32_t* row_v;     // m: that column, kRowEmpty or kRowStale (lane 0 only)
    int32_t* clist;     // m: the checks held by clusters, in the order they joined (lane 0 only)
    uint64_t* in_bits;  // words_n
    uint64_t* ebits;    // words_n
    uint64_t* xbuf;     // words_m
    uint64_t* cbuf;     // words_m
    uint64_t* dbuf;     // words_m: a candidate's change of the pivot solution
    uint64_t* hbuf;     // words_m: one bit per basis vector (a reduction's vectors)
    uint64_t* fbuf;     // words_m: one bit per basis vector (vectors to clear a new pivot from)
    // global
    int32_t* cols;      // n
    int32_t* sorted;    // n
    int64_t* ckey;      // n
    uint64_t* pool;     // m x words_m
    uint64_t* basis2;   // m x 2 words_m (vector, combination)
    // global, lsd_order > 0 only
    int32_t* npc;       // n: non-pivot columns in rank order
    int32_t* nproot;    // n: their clusters
    int32_t* pidx;      // n: pivot index of a column, -1 if none (lane 0 only)
    int32_t* ck;        // n: one cluster's columns, ascending (lane 0 only)
    int32_t* fl;        // n: one cluster's non-pivot ordinals, rank order (lane 0 only)
    uint64_t* reps;     // n x words_m: pivot combination of each non-pivot column
    int priv_lds;       // the per-check arrays marked "lane 0 only" are in LDS too
};

__host__ __device__ inline size_t al8(size_t x) { return (x + 7) & ~(size_t)7; }

// Lays out the LDS part at `lds` and the global part at `glob` (either may
// be null to measure); returns the two sizes.
__host__ __device__ inline void lsd_layout(const DevGraph& g, unsigned char* lds, unsigned char* glob,
                                           LsdMem* out, size_t* lds_bytes, size_t* glob_bytes) {
    const size_t m = g.m ? g.m : 1, n = g.n, wn = g.words_n, wm = g.words_m ? g.words_m : 1;
    size_t lo = 0, go = 0;
    auto tl = [&](size_t bytes) {
        unsigned char* p = lds ? lds + lo : nullptr;
        lo += al8(bytes);
        return p;
    };
    auto tg = [&](size_t bytes) {
        unsigned char* p = glob ? glob + go : nullptr;
        go += al8(bytes);
        return p;
    };
    // The arrays only lane 0 touches (best_q, best_v, ccount, picks, added,
    // pivcol, row_q, row_v, clist: 48 bytes per check) move to global memory when everything
    // would not fit in kLsdLds bytes of LDS (graphs with several thousand
    // checks).  Reads and writes by one lane need no cross-lane visibility.
    const size_t all_lds = al8(8 * m) + 2 * al8(8 * wn) + 5 * al8(8 * wm) + 5 * al8(4 * m) + al8(8 * m) +
                           4 * al8(4 * m) + al8(8 * m) + 2 * al8(4 * m);
    const bool priv_glob = all_lds > kLsdLds;
    auto tp = [&](size_t bytes) { return priv_glob ? tg(bytes) : tl(bytes); };
    LsdMem M;
    M.priv_lds = priv_glob ? 0 : 1;
    M.best_q = (int64_t*)tp(8 * m);
    M.in_bits = (uint64_t*)tl(8 * wn);
    M.ebits = (uint64_t*)tl(8 * wn);
    M.xbuf = (uint64_t*)tl(8 * wm);
    M.cbuf = (uint64_t*)tl(8 * wm);
    M.dbuf = (uint64_t*)tl(8 * wm);
    M.hbuf = (uint64_t*)tl(8 * wm);
    M.fbuf = (uint64_t*)tl(8 * wm);
    M.chk_cl = (int32_t*)tl(4 * m);
    M.parent = (int32_t*)tl(4 * m);
    M.cstate = (uint32_t*)tl(4 * m);
    M.best_v = (int32_t*)tp(4 * m);
    M.ccount = (int32_t*)tp(4 * m);
    M.picks = (int32_t*)tp(8 * m);
    M.added = (int32_t*)tp(4 * m);
    M.pool_piv = (int32_t*)tl(4 * m);
    M.piv2 = (int32_t*)tl(4 * m);
    M.pivcol = (int32_t*)tp(4 * m);
    M.row_q = (int64_t*)tp(8 * m);
    M.row_v = (int32_t*)tp(4 * m);
    M.clist = (int32_t*)tp(4 * m);
    M.ckey = (int64_t*)tg(8 * n);
    M.pool = (uint64_t*)tg(8 * wm * m);
    M.basis2 = (uint64_t*)tg(16 * wm * m);
    M.cols = (int32_t*)tg(4 * n);
    M.sorted = (int32_t*)tg(4 * n);
    const size_t nh = g.lsd_order ? n : 0;
    M.npc = (int32_t*)tg(4 * nh);
    M.nproot = (int32_t*)tg(4 * nh);
    M.pidx = (int32_t*)tg(4 * nh);
    M.ck = (int32_t*)tg(4 * nh);
    M.fl = (int32_t*)tg(4 * nh);
    M.reps = (uint64_t*)tg(8 * wm * nh);
    if (out) *out = M;
    if (lds_bytes) *lds_bytes = lo;
    if (glob_bytes) *glob_bytes = go;
}

__device__ inline int32_t ald32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int64_t ald64(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// order-preserving map of a float to int64 (-0 and +0 map to the same key)
__device__ inline int64_t float_key(float f) {
    uint32_t b = __float_as_uint(f);
    int64_t mag = (int64_t)(b & 0x7fffffffu);
    return (b >> 31) ? -mag : mag;
}

__device__ inline int32_t find_root(int32_t* parent, int32_t x) {
    while (parent[x] != x) x = parent[x];
    return x;
}

__device__ inline bool key_less(int64_t qa, int32_t a, int64_t qb, int32_t b) {
    return qa < qb || (qa == qb && a < b);
}

__device__ inline uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

// x ^= the basis vectors whose pivot bit is set in x, comb (if given) ^=
// their combination words.  The basis is in reduced echelon form, so these
// are the vectors that the reduction in insertion order adds, and their sum
// does not depend on the order.  hit (LDS) receives one bit per vector.
// Word w of every vector is read and written only by lane w mod 64, so the
// basis needs no cross-lane visibility in global memory.
__device__ void reduce_by(uint64_t* x, uint64_t* comb, const uint64_t* vecs, size_t stride,
                          const int32_t* piv, int count, uint32_t wm, uint64_t* hit, int lane) {
    __syncthreads();
    const int nblk = (count + kWave - 1) / kWave;
    for (int b = 0; b < nblk; b++) {
        const int j = b * kWave + lane;
        bool h = false;
        if (j < count) {
            const int32_t p = piv[j];
            h = (x[p >> 6] >> (p & 63)) & 1ull;
        }
        const uint64_t mask = __ballot(h);
        if (lane == 0) hit[b] = mask;
    }
    __syncthreads();
    for (uint32_t w = lane; w < wm; w += kWave) {
        uint64_t acc = 0, cacc = 0;
        for (int b = 0; b < nblk; b++) {
            uint64_t mask = uni64(hit[b]);
            while (mask) {
                // up to eight vectors per step, their loads in flight together
                uint64_t t[8], c[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    t[u] = 0;
                    c[u] = 0;
                    if (mask) {
                        const size_t i = (size_t)b * kWave + (size_t)(__ffsll((long long)mask) - 1);
                        mask &= mask - 1;
                        t[u] = vecs[i * stride + w];
                        if (comb) c[u] = vecs[i * stride + wm + w];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    acc ^= t[u];
                    cacc ^= c[u];
                }
            }
        }
        x[w] ^= acc;
        if (comb) comb[w] ^= cacc;
    }
    __syncthreads();
}

// Appends x (reduced by the basis of count vectors, lowest set bit p) with
// its combination words comb (if given) as vector count, pivot p, and clears
// bit p from every earlier vector that has it (xor x and comb), so the
// basis stays in reduced echelon form.  flag (LDS) receives one bit per
// earlier vector; the lane that holds word p / 64 of the vectors finds them.
__device__ void basis_append(uint64_t* vecs, size_t stride, int32_t* piv, int count, const uint64_t* x,
                             const uint64_t* comb, int p, uint32_t wm, uint64_t* flag, int lane) {
    const uint32_t W = (uint32_t)p >> 6;
    const uint64_t bit = 1ull << (p & 63);
    const int nblk = (count + kWave - 1) / kWave;
    for (uint32_t w = lane; w < wm; w += kWave) {
        if (w != W) continue;
        for (int b = 0; b < nblk; b++) {
            uint64_t f = 0;
#pragma unroll 8
            for (int u = 0; u < kWave; u++) {
                const int j = b * kWave + u;
                if (j < count && (vecs[(size_t)j * stride + w] & bit)) f |= 1ull << u;
            }
            flag[b] = f;
        }
    }
    __syncthreads();
    for (uint32_t w = lane; w < wm; w += kWave) {
        const uint64_t xw = x[w], cw = comb ? comb[w] : 0;
        for (int b = 0; b < nblk; b++) {
            uint64_t mask = uni64(flag[b]);
            while (mask) {
                const size_t i = (size_t)b * kWave + (size_t)(__ffsll((long long)mask) - 1);
                mask &= mask - 1;
                vecs[i * stride + w] ^= xw;
                if (comb) vecs[i * stride + wm + w] ^= cw;
            }
        }
        vecs[(size_t)count * stride + w] = xw;
        if (comb) vecs[(size_t)count * stride + wm + w] = cw;
    }
    if (lane == 0) piv[count] = p;
    __syncthreads();
}

// lowest set bit of a words_m vector, or -1
__device__ int lowest_bit(const uint64_t* x, uint32_t wm, int lane) {
    int best = 0x7fffffff;
    for (uint32_t w = lane; w < wm; w += kWave)
        if (x[w]) {
            int b = (int)(w * 64 + __ffsll((long long)x[w]) - 1);
            if (b < best) best = b;
        }
    for (int off = kWave / 2; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
    best = uni(best);
    return best == 0x7fffffff ? -1 : best;
}

__device__ void column_vector(const DevGraph& g, uint64_t* x, uint32_t v, int lane) {
    for (uint32_t w = lane; w < g.words_m; w += kWave) x[w] = 0;
    __syncthreads();
    if (lane == 0)
        for (uint32_t j = g.cp[v]; j < g.cp[v + 1]; j++) {
            uint32_t c = g.ci[j];
            x[c >> 6] |= 1ull << (c & 63);
        }
    __syncthreads();
}

// dbuf = pivot combination of non-pivot ordinals oa and ob (-1 = none)
__device__ void candidate_delta(const LsdMem& S, int32_t oa, int32_t ob, uint32_t wm, int lane) {
    for (uint32_t w = lane; w < wm; w += kWave) {
        uint64_t d = 0;
        if (oa >= 0) d ^= S.reps[(size_t)oa * wm + w];
        if (ob >= 0) d ^= S.reps[(size_t)ob * wm + w];
        S.dbuf[w] = d;
    }
    __syncthreads();
}

// Is column v set in the cluster's solution for the candidate whose pivot
// change is in dbuf and whose non-pivot columns are va, vb?  (lane 0)
__device__ inline bool cand_bit(const LsdMem& S, int32_t v, int32_t va, int32_t vb) {
    bool b = (S.ebits[v >> 6] >> (v & 63)) & 1ull;
    const int32_t k = S.pidx[v];
    if (k >= 0) b ^= (S.dbuf[k >> 6] >> (k & 63)) & 1ull;
    return b ^ (v == va) ^ (v == vb);
}

// The combination sweep on every valid cluster that has non-pivot columns.
// ebits holds the OSD-0 solution on entry and the chosen one on return.
__device__ void combination_sweep(const DevGraph& g, const LsdMem& S, int nk, int ncol, int nnp, uint32_t wm,
                                  int lane) {
    for (int K = 0; K < nk; K++) {
        if (uni(S.parent[K]) != K || !(uni(S.cstate[K]) & kValid)) continue;
        int nf = 0, nck = 0;
        if (lane == 0) {
            for (int f = 0; f < nnp; f++)
                if (S.nproot[f] == K) S.fl[nf++] = f;
            if (nf)
                for (int i = 0; i < ncol; i++) {
                    const int32_t v = S.cols[i];
                    if (find_root(S.parent, S.chk_cl[g.ci[g.cp[v]]]) == K) S.ck[nck++] = v;
                }
        }
        nf = uni(__shfl(nf, 0));
        nck = uni(__shfl(nck, 0));
        __syncthreads();
        if (!nf) continue;
        const int lo = min(nf, (int)g.lsd_order);
        const int ncand = 1 + nf + lo * (lo - 1) / 2;
        double bw = 0.0;
        int bt = 0;
        int pa = 0, pb = 1;  // the next pair among the first lo columns of F
        int32_t best_oa = -1, best_ob = -1;
        for (int t = 0; t < ncand; t++) {
            int fa = -1, fb = -1;  // positions in F
            if (t >= 1 && t <= nf) {
                fa = t - 1;
            } else if (t > nf) {
                fa = pa;
                fb = pb;
                if (++pb == lo) {
                    pa++;
                    pb = pa + 1;
                }
            }
            int32_t oa = -1, ob = -1;
            if (lane == 0) {
                oa = fa >= 0 ? S.fl[fa] : -1;
                ob = fb >= 0 ? S.fl[fb] : -1;
            }
            oa = uni(__shfl(oa, 0));
            ob = uni(__shfl(ob, 0));
            candidate_delta(S, oa, ob, wm, lane);
            if (lane == 0) {
                const int32_t va = oa >= 0 ? S.npc[oa] : -1, vb = ob >= 0 ? S.npc[ob] : -1;
                double w = 0.0;
                for (int i = 0; i < nck; i++) {
                    const int32_t v = S.ck[i];
                    if (cand_bit(S, v, va, vb)) w += g.lam64[v];
                }
                if (t == 0 || w < bw) {
                    bw = w;
                    bt = t;
                    best_oa = oa;
                    best_ob = ob;
                }
            }
            __syncthreads();
        }
        bt = uni(__shfl(bt, 0));
        best_oa = uni(__shfl(best_oa, 0));
        best_ob = uni(__shfl(best_ob, 0));
        if (bt == 0) continue;
        candidate_delta(S, best_oa, best_ob, wm, lane);
        if (lane == 0) {
            const int32_t va = best_oa >= 0 ? S.npc[best_oa] : -1, vb = best_ob >= 0 ? S.npc[best_ob] : -1;
            for (int i = 0; i < nck; i++) {
                const int32_t v = S.ck[i];
                const bool b = cand_bit(S, v, va, vb);
                const uint64_t bit = 1ull << (v & 63);
                S.ebits[v >> 6] = b ? (S.ebits[v >> 6] | bit) : (S.ebits[v >> 6] & ~bit);
            }
        }
        __syncthreads();
    }
}

// The least (key, column) over the columns of row c not yet held, formed by
// the whole wavefront (every lane receives it; column INT32_MAX: none).
template <class KeyF>
__device__ inline void row_least(const DevGraph& g, const LsdMem& S, uint32_t c, KeyF key, int lane, int64_t& bq,
                                 int32_t& bv) {
    bq = INT64_MAX;
    bv = 0x7fffffff;
    for (uint32_t p = g.rp[c] + lane; p < g.rp[c + 1]; p += kWave) {
        const uint32_t v = g.ri[p];
        if ((S.in_bits[v >> 6] >> (v & 63)) & 1ull) continue;
        const int64_t kq = key(v);
        if (key_less(kq, (int32_t)v, bq, bv)) {
            bq = kq;
            bv = (int32_t)v;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int64_t oq = __shfl_xor(bq, off);
        const int32_t ov = __shfl_xor(bv, off);
        if (key_less(oq, ov, bq, bv)) {
            bq = oq;
            bv = ov;
        }
    }
}

__global__ __launch_bounds__(kWave) void lsd_kernel(DevGraph g, LsdLaunch a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x;
    LsdMem S;
    lsd_layout(g, lds, static_cast<unsigned char*>(a.scratch) + a.scratch_per_block * blockIdx.x, &S,
               nullptr, nullptr);
    const uint32_t count = uni(a.list ? *a.list_count : a.n_list);
    const uint32_t wm = g.words_m;
    for (uint32_t it = blockIdx.x; it < count && it < a.n_list; it += gridDim.x) {
        const uint32_t local = uni(a.list ? a.list[it] : it);
        const uint64_t gshot = a.shot0 + local;
        const uint8_t* s = a.syndromes + gshot * g.m;
        auto key = [&](uint32_t v) -> int64_t {
            return a.soft_f32 ? float_key(a.soft_f32[gshot * g.n + v]) : a.soft_fix[(size_t)local * g.n + v];
        };

        // ---- one cluster per flipped check, slots in ascending check order
        int nk = 0, ncl = 0;  // ncl: length of clist (kept by lane 0, broadcast per round)
        for (uint32_t base = 0; base < g.m; base += kWave) {
            const uint32_t c = base + lane;
            const bool f = c < g.m && s[c] != 0;
            const uint64_t mask = __ballot(f);
            if (lane == 0)
                for (uint64_t mm = mask; mm; mm &= mm - 1)
                    S.clist[ncl++] = (int32_t)(base + __ffsll((long long)mm) - 1);
            const int pre = __popcll(mask & ((1ull << lane) - 1ull));
            if (c < g.m) {
                if (f) {
                    const int slot = nk + pre;
                    S.chk_cl[c] = slot;
                    S.parent[slot] = slot;
                    S.cstate[slot] = 0;
                } else {
                    S.chk_cl[c] = -1;
                }
            }
            nk += __popcll(mask);
        }
        for (uint32_t w = lane; w < g.words_n; w += kWave) {
            S.in_bits[w] = 0;
            S.ebits[w] = 0;
        }
        if (lane == 0)
            for (uint32_t c = 0; c < g.m; c++) S.row_v[c] = kRowStale;
        __syncthreads();
        int pool_n = 0, rounds = 0;

        for (;;) {
            // 1. best boundary column of every invalid, growing cluster: the
            //    least (key, column) over its checks' rows.  Each row's least
            //    column not yet held is cached across rounds; it changes only
            //    when that column joins, and step 3 marks such rows stale
            //    (another column of the row joining leaves the least where it
            //    is).
            // 2. clusters with an empty boundary fail; the others pick, in
            //    cluster order.
            ncl = uni(__shfl(ncl, 0));
            int npick = 0;
            if (S.priv_lds) {
                // Every per-check array is in LDS: each lane takes its own
                // checks of the list, the whole wavefront scans each stale
                // row, and the least (key, column) of a cluster is formed by
                // LDS atomics, the key first, then the column among the
                // checks that reach that key.
                for (int K = lane; K < nk; K += kWave) {
                    S.best_q[K] = INT64_MAX;
                    S.best_v[K] = 0x7fffffff;
                }
                __syncthreads();
                for (int kb = 0; kb < ncl; kb += kWave) {
                    const int i = kb + lane;
                    int32_t c = 0, R = 0;
                    bool act = false;
                    if (i < ncl) {
                        c = S.clist[i];
                        R = find_root(S.parent, S.chk_cl[c]);
                        act = !(S.cstate[R] & (kValid | kFailed));
                    }
                    uint64_t stale = __ballot(act && S.row_v[c] == kRowStale);
                    while (stale) {
                        const int b = __ffsll((long long)stale) - 1;
                        stale &= stale - 1;
                        const uint32_t cc = (uint32_t)uni(__shfl(c, b));
                        int64_t bq;
                        int32_t bv;
                        row_least(g, S, cc, key, lane, bq, bv);
                        if (lane == 0) {
                            S.row_q[cc] = bq;
                            S.row_v[cc] = bv == 0x7fffffff ? kRowEmpty : bv;
                        }
                    }
                    __syncthreads();
                    if (act && S.row_v[c] >= 0)
                        __hip_atomic_fetch_min(&S.best_q[R], S.row_q[c], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                __syncthreads();
                for (int kb = 0; kb < ncl; kb += kWave) {
                    const int i = kb + lane;
                    if (i < ncl) {
                        const int32_t c = S.clist[i];
                        const int32_t R = find_root(S.parent, S.chk_cl[c]);
                        const int32_t v = S.row_v[c];
                        if (!(S.cstate[R] & (kValid | kFailed)) && v >= 0 && S.row_q[c] == S.best_q[R])
                            __hip_atomic_fetch_min(&S.best_v[R], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                __syncthreads();
                for (int kb = 0; kb < nk; kb += kWave) {
                    const int K = kb + lane;
                    bool pick = false;
                    int32_t v = 0;
                    if (K < nk && S.parent[K] == K && !(S.cstate[K] & (kValid | kFailed))) {
                        v = S.best_v[K];
                        pick = v != 0x7fffffff;
                        if (!pick) S.cstate[K] |= kFailed;
                    }
                    const uint64_t pm = __ballot(pick);
                    if (pick) {
                        const int at = npick + __popcll(pm & ((1ull << lane) - 1ull));
                        S.picks[2 * at] = K;
                        S.picks[2 * at + 1] = v;
                    }
                    npick += __popcll(pm);
                }
                __syncthreads();
            } else {
            // The per-check arrays are in global memory: lane 0 keeps them,
            // and only lane 0's copy of a cache entry is used (readfirstlane).
            for (int i = 0; i < ncl; i++) {
                const uint32_t c = (uint32_t)uni(S.clist[i]);
                const int32_t R = uni(find_root(S.parent, S.chk_cl[c]));
                if (uni(S.cstate[R]) & (kValid | kFailed)) continue;
                if (uni(S.row_v[c]) != kRowStale) continue;
                int64_t bq;
                int32_t bv;
                row_least(g, S, c, key, lane, bq, bv);
                if (lane == 0) {
                    S.row_q[c] = bq;
                    S.row_v[c] = bv == 0x7fffffff ? kRowEmpty : bv;
                }
            }
            if (lane == 0) {
                for (int K = 0; K < nk; K++) {
                    S.best_q[K] = INT64_MAX;
                    S.best_v[K] = -1;
                }
                for (int i = 0; i < ncl; i++) {
                    const int32_t c = S.clist[i];
                    const int32_t R = find_root(S.parent, S.chk_cl[c]);
                    if (S.cstate[R] & (kValid | kFailed)) continue;
                    const int32_t v = S.row_v[c];
                    if (v < 0) continue;
                    const int64_t q = S.row_q[c];
                    if (S.best_v[R] < 0 || key_less(q, v, S.best_q[R], S.best_v[R])) {
                        S.best_q[R] = q;
                        S.best_v[R] = v;
                    }
                }
            }
            __syncthreads();
            if (lane == 0) {
                for (int K = 0; K < nk; K++) {
                    if (S.parent[K] != K || (S.cstate[K] & (kValid | kFailed))) continue;
                    if (S.best_v[K] < 0) {
                        S.cstate[K] |= kFailed;
                    } else {
                        S.picks[2 * npick] = K;
                        S.picks[2 * npick + 1] = S.best_v[K];
                        npick++;
                    }
                }
            }
            npick = uni(__shfl(npick, 0));
            __syncthreads();
            }
            if (!npick) break;
            rounds++;
            // 3. apply every pick: the column joins, its checks join, clusters
            //    that now share a check merge
            int nadd = 0;
            if (lane == 0) {
                for (int i = 0; i < npick; i++) {
                    const int32_t K = S.picks[2 * i];
                    const uint32_t j = (uint32_t)S.picks[2 * i + 1];
                    if (!((S.in_bits[j >> 6] >> (j & 63)) & 1ull)) {
                        S.in_bits[j >> 6] |= 1ull << (j & 63);
                        S.added[nadd++] = (int32_t)j;
                    }
                    for (uint32_t q = g.cp[j]; q < g.cp[j + 1]; q++) {
                        const uint32_t c = g.ci[q];
                        if (S.row_v[c] == (int32_t)j) S.row_v[c] = kRowStale;  // j is held now
                        if (S.chk_cl[c] < 0) {
                            S.chk_cl[c] = K;
                            S.clist[ncl++] = (int32_t)c;
                        } else {
                            int32_t ra = find_root(S.parent, K), rb = find_root(S.parent, S.chk_cl[c]);
                            if (ra != rb) {
                                const int32_t lo = min(ra, rb), hi = max(ra, rb);
                                S.parent[hi] = lo;
                                S.cstate[lo] |= (S.cstate[hi] & kFailed) | kDirty;
                            }
                        }
                    }
                    S.cstate[find_root(S.parent, K)] |= kDirty;
                }
            }
            nadd = uni(__shfl(nadd, 0));
            __syncthreads();
            // 4. extend the basis pool with the new columns
            for (int i = 0; i < nadd; i++) {
                int32_t col = 0;
                if (lane == 0) col = S.added[i];
                column_vector(g, S.xbuf, (uint32_t)uni(__shfl(col, 0)), lane);
                reduce_by(S.xbuf, nullptr, S.pool, wm, S.pool_piv, pool_n, wm, S.hbuf, lane);
                const int p = lowest_bit(S.xbuf, wm, lane);
                if (p >= 0) {
                    basis_append(S.pool, wm, S.pool_piv, pool_n, S.xbuf, nullptr, p, wm, S.fbuf, lane);
                    pool_n++;
                }
                __syncthreads();
            }
            // 5. validity of every live cluster that changed and has not failed
            //    (found 64 clusters at a time, taken in cluster order)
            for (int kb = 0; kb < nk; kb += kWave) {
              const int K0 = kb + lane;
              uint64_t dm = __ballot(K0 < nk && S.parent[K0] == K0 &&
                                     (S.cstate[K0] & (kFailed | kDirty)) == kDirty);
              while (dm) {
                const int K = kb + __ffsll((long long)dm) - 1;
                dm &= dm - 1;
                for (uint32_t base = 0; base < g.m; base += kWave) {
                    const uint32_t c = base + lane;
                    bool in = false;
                    if (c < g.m && s[c]) {
                        const int32_t cl = S.chk_cl[c];
                        in = cl >= 0 && find_root(S.parent, cl) == K;
                    }
                    const uint64_t mask = __ballot(in);
                    if (lane == 0) S.xbuf[base / kWave] = mask;
                }
                __syncthreads();
                reduce_by(S.xbuf, nullptr, S.pool, wm, S.pool_piv, pool_n, wm, S.hbuf, lane);
                const bool valid = lowest_bit(S.xbuf, wm, lane) < 0;
                if (lane == 0) S.cstate[K] = (valid ? (S.cstate[K] | kValid) : (S.cstate[K] & ~kValid)) & ~kDirty;
                __syncthreads();
              }
            }
        }

        // ---- gather the columns of valid clusters, rank them, solve
        int ncol = 0;
        bool failed = false;
        if (lane == 0) {
            for (int K = 0; K < nk; K++) S.ccount[K] = 0;
            for (uint32_t w = 0; w < g.words_n; w++) {
                uint64_t x = S.in_bits[w];
                while (x) {
                    const int b = __ffsll((long long)x) - 1;
                    x &= x - 1;
                    const uint32_t v = w * 64 + b;
                    const int32_t R = find_root(S.parent, S.chk_cl[g.ci[g.cp[v]]]);
                    S.ccount[R]++;
                    if (S.cstate[R] & kValid) {
                        S.cols[ncol++] = (int32_t)v;
                        if (g.lsd_order) S.pidx[v] = -1;
                    }
                }
            }
        }
        ncol = uni(__shfl(ncol, 0));
        __syncthreads();
        for (int i = lane; i < ncol; i += kWave) S.ckey[i] = key((uint32_t)ald32(&S.cols[i]));
        __syncthreads();
        for (int i = lane; i < ncol; i += kWave) {
            const int64_t qi = ald64(&S.ckey[i]);
            const int32_t vi = ald32(&S.cols[i]);
            int r = 0;
            for (int j = 0; j < ncol; j++)
                if (key_less(ald64(&S.ckey[j]), ald32(&S.cols[j]), qi, vi)) r++;
            S.sorted[r] = vi;
        }
        __syncthreads();
        int nb = 0, nnp = 0;
        for (int i = 0; i < ncol; i++) {
            const uint32_t v = (uint32_t)uni(ald32(&S.sorted[i]));
            column_vector(g, S.xbuf, v, lane);
            for (uint32_t w = lane; w < wm; w += kWave) S.cbuf[w] = 0;
            reduce_by(S.xbuf, S.cbuf, S.basis2, 2 * (size_t)wm, S.piv2, nb, wm, S.hbuf, lane);
            const int p = lowest_bit(S.xbuf, wm, lane);
            if (p >= 0) {
                if (lane == 0) S.cbuf[nb >> 6] ^= 1ull << (nb & 63);
                __syncthreads();
                basis_append(S.basis2, 2 * (size_t)wm, S.piv2, nb, S.xbuf, S.cbuf, p, wm, S.fbuf, lane);
                if (lane == 0) {
                    S.pivcol[nb] = (int32_t)v;
                    if (g.lsd_order) S.pidx[v] = nb;
                }
                nb++;
            } else if (g.lsd_order) {
                // a non-pivot column: cbuf holds its combination of pivots
                for (uint32_t w = lane; w < wm; w += kWave) S.reps[(size_t)nnp * wm + w] = S.cbuf[w];
                if (lane == 0) {
                    S.npc[nnp] = (int32_t)v;
                    S.nproot[nnp] = find_root(S.parent, S.chk_cl[g.ci[g.cp[v]]]);
                }
                nnp++;
            }
            __syncthreads();
        }
        // target: s on the checks of valid clusters
        for (uint32_t base = 0; base < g.m; base += kWave) {
            const uint32_t c = base + lane;
            bool in = false;
            if (c < g.m && s[c]) {
                const int32_t cl = S.chk_cl[c];
                in = cl >= 0 && (S.cstate[find_root(S.parent, cl)] & kValid);
            }
            const uint64_t mask = __ballot(in);
            if (lane == 0) S.xbuf[base / kWave] = mask;
        }
        for (uint32_t w = lane; w < wm; w += kWave) S.cbuf[w] = 0;
        __syncthreads();
        reduce_by(S.xbuf, S.cbuf, S.basis2, 2 * (size_t)wm, S.piv2, nb, wm, S.hbuf, lane);
        if (lane == 0)
            for (int i = 0; i < nb; i++)
                if ((S.cbuf[i >> 6] >> (i & 63)) & 1ull) {
                    const uint32_t v = (uint32_t)S.pivcol[i];
                    S.ebits[v >> 6] |= 1ull << (v & 63);
                }
        __syncthreads();
        if (g.lsd_order && nnp) combination_sweep(g, S, nk, ncol, nnp, wm, lane);
        uint64_t* out = a.corrections + gshot * g.words_n;
        for (uint32_t w = lane; w < g.words_n; w += kWave) out[w] = S.ebits[w];
        int nclus = 0, largest = 0;
        if (lane == 0) {
            for (int K = 0; K < nk; K++) {
                if (S.parent[K] != K) continue;
                nclus++;
                largest = max(largest, S.ccount[K]);
                if (!(S.cstate[K] & kValid)) failed = true;
            }
            if (a.stats) {
                vibe_shot_stats* st = a.stats + gshot;
                if (!a.list) {
                    st->winner = -1;
                    st->t_win = 0;
                    st->n_conv = 0;
                    st->member_iters = 0;
                }
                // keep the saturation flag the selection wrote for this shot
                st->flags = (a.list ? (st->flags & VIBE_FLAG_SATURATED) : 0u) | VIBE_FLAG_LSD_USED |
                            (failed ? VIBE_FLAG_LSD_FAILED : 0u);
                st->lsd_clusters = (uint32_t)nclus;
                st->lsd_largest = (uint32_t)largest;
                st->lsd_rounds = (uint32_t)rounds;
            }
        }
        __syncthreads();
    }
}

}  // namespace

size_t lsd_scratch_per_block(const DevGraph& g) {
    size_t gb = 0;
    lsd_layout(g, nullptr, nullptr, nullptr, nullptr, &gb);
    return al8(gb) + 256;
}

size_t lsd_lds_bytes(const DevGraph& g) {
    size_t lb = 0;
    lsd_layout(g, nullptr, nullptr, nullptr, &lb, nullptr);
    return lb;
}

int launch_lsd(const DevGraph& g, const LsdLaunch& a, hipStream_t st) {
    if (!a.n_list) return VIBE_OK;
    const size_t lds = lsd_lds_bytes(g);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)lsd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(lsd)");
    }
    hipLaunchKernelGGL(lsd_kernel, dim3(a.grid), dim3(kWave), lds, st, g, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "lsd_kernel launch");
}

}  // namespace vibe
