// Adjoint of K unrolled min-sum iterations: gradients of the soft-syndrome
// loss with respect to the channel LLRs lambda_v and the per-iteration
// scaling factors alpha_t (the differentiable decoder; Algorithm 1 unrolled).
//
// Forward: K iterations of the serial (or parallel) schedule without early
// stop, from lambda and alpha given as inputs.  Every iteration records, per
// edge e = (c, v), its check message q_e (r_e = alpha_t q_e), the edge u*
// attaining the minimum with the sign factor of dq_e / dmu_{u*}, and whether
// the new message was clamped (these records are the checkpoints: the
// reverse pass needs nothing else).  Loss: with the final posteriors L_v,
// shat_c = (1 - prod_{v in N(c)} tanh(L_v / 2)) / 2 clamped to [eps, 1 - eps],
// loss = sum_c BCE(s_c, shat_c), in FP64.
//
// Reverse, iteration t = K .. 1, chunks in reverse order.  Edge e's new
// message feeds the other messages of its column (and L_v after the last
// iteration), so
//   rbar_e = sum_{e' in column, e' != e} mubar_e' + Lbar_v,
//   lambdabar_v += sum_{e' in column} mubar_e' + Lbar_v,
//   alphabar_t += rbar_e q_e,
//   mubar_{u*} += rbar_e alpha_t (1 - 2 s_c) prod sign * sign(mu_{u*}),
// where mu_{u*} is u*'s new message of iteration t if u* comes earlier in
// the sweep and its message of iteration t - 1 otherwise.  At t = 1 the old
// messages are lambda itself.  Sign products, argmin choices and clamps are
// piecewise constant: where they do not change this is the exact gradient.
//
// The argmin adjoints of one row are summed in LDS, not in memory.  In the
// serial schedule, the prefix argmin of the row's edges, visited in reverse,
// only moves to earlier edges, and every edge before the current prefix
// argmin is still to come: one accumulator per row collects the adjoint of
// that argmin and hands it over when the reverse pass reaches it.  The
// suffix argmin (an old message) also only moves to earlier edges as the
// pass goes on, so a second accumulator is written out once, when its
// target changes or the pass ends.  In the parallel schedule the argmin
// over a row without the edge itself is the row's first minimum for every
// edge but that one, and the next minimum for it: two accumulators.
//
// One wavefront per (shot, member) item.  Items go to blocks statically
// (block b takes items b, b + grid, ...); a block sums its items' loss and
// gradients in item order into a row of its own, and the rows are summed in
// a fixed order, so the result does not depend on timing.  Slot arrays are
// private to their lane except for the argmin adjoints written out by
// another lane and the per-column values of the loss stage; those are read
// with agent-scope loads after a barrier.  Every pass loads the next chunk's
// slot data while it works on the current one.
#include "internal.h"

#pragma clang fp contract(off)

namespace vibe {

namespace {

template <class F>
struct GP;
template <>
struct GP<float> {
    using B = uint32_t;
    static constexpr B kSign = 0x80000000u;
    __device__ static B bits(float x) { return __float_as_uint(x); }
    __device__ static float val(B b) { return __uint_as_float(b); }
    __device__ static B ident(const DevGraph& g) { return g.ident32; }
};
template <>
struct GP<double> {
    using B = uint64_t;
    static constexpr B kSign = 0x8000000000000000ull;
    __device__ static B bits(double x) { return (uint64_t)__double_as_longlong(x); }
    __device__ static double val(B b) { return __longlong_as_double((long long)b); }
    __device__ static B ident(const DevGraph& g) { return g.ident64; }
};

// A row state with its argmin: magnitude bits with the parity of the signs
// in the sign position, and the slot of the edge attaining the minimum with
// that edge's own sign in bit 31 (kNoArg: none).  On equal magnitudes the
// earlier operand's slot is kept.
constexpr uint32_t kNoArg = 0x7fffffffu;

// Per-edge record word: argmin slot (kSlotMask: none) and flags.
constexpr uint32_t kSlotMask = 0x00ffffffu;
constexpr uint32_t kSneg = 1u << 24;  // dq_e / dmu_{u*} is negative
constexpr uint32_t kNcm = 1u << 25;   // the new message was not clamped
constexpr uint32_t kLnc = 1u << 26;   // lambda_v was not clamped

template <class F>
struct RS {
    typename GP<F>::B st;
    uint32_t arg;
};

template <class F>
__device__ inline RS<F> rs_join(RS<F> a, RS<F> b) {
    using B = typename GP<F>::B;
    constexpr B kS = GP<F>::kSign;
    const B ma = a.st & ~kS, mb = b.st & ~kS;
    RS<F> o;
    o.st = (ma <= mb ? ma : mb) | ((a.st ^ b.st) & kS);
    o.arg = ma <= mb ? a.arg : b.arg;
    return o;
}

template <class F>
__device__ inline RS<F> rs_of(F x, uint32_t slot) {
    using B = typename GP<F>::B;
    RS<F> o;
    o.st = (GP<F>::bits(x) & ~GP<F>::kSign) | (x < F(0) ? GP<F>::kSign : (B)0);
    o.arg = slot | (x < F(0) ? 0x80000000u : 0u);
    return o;
}

template <class F>
__device__ inline F clampv(F x, F lim) {
    return x > lim ? lim : (x < -lim ? -lim : x);
}

// Reads of words that another lane of the wavefront wrote to the block's
// scratch.  A buffer load with the first cache-policy bit set misses the
// vector L1 and reads the L2, which this CU's stores write through to (an
// agent-scope atomic load would also leave this XCD's L2 behind).  The
// scratch of one block is addressed as a wave-uniform descriptor plus a byte
// offset.
struct Scr {
    __amdgpu_buffer_rsrc_t r;
    const unsigned char* base;
};
constexpr int kBufFlags = 0x00020000;  // 32-bit data format: plain dword access

__device__ __forceinline__ Scr make_scr(const void* base, uint32_t bytes) {
    return Scr{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufFlags),
               static_cast<const unsigned char*>(base)};
}

template <class T>
__device__ __forceinline__ T xload(const Scr& sc, const T* p) {
    const int off = (int)(reinterpret_cast<const unsigned char*>(p) - sc.base);
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(sc.r, off, 0, 1));
    } else {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(sc.r, off, 0, 1);
        return __builtin_bit_cast(T, u);
    }
}

template <class F>
__device__ inline F wave_sum(F x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ inline uint32_t deg_of(uint32_t meta) { return (meta >> kMetaDegShift) & 15u; }

// edges in a chunk (its first lanes), from every lane's meta word
__device__ inline uint32_t edges_of(uint32_t meta) { return uni((uint32_t)__popcll(__ballot(deg_of(meta) != 0))); }

// XCDs of the device: workgroups are dispatched to them round-robin
constexpr uint32_t kXcds = 8;

// keeps the compiler from moving LDS traffic of one chunk past the next's,
// or scheduling a later chunk's work into this one
__device__ inline void chunk_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

// v of the lane at byte address addr (lane * 4, taken mod 256)
__device__ __forceinline__ float perm(uint32_t addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((int)addr, __float_as_int(v)));
}
__device__ __forceinline__ double perm(uint32_t addr, double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute((int)addr, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute((int)addr, (int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// acc + the sum of v over the column's other positions, in position order.
// Position j of the column is the lane at byte address b0x4 + 4 P j; the
// reads go eight at a time at constant offsets from that base, and
// positions past the column and the edge's own add an exact zero.
template <class F, int P>
__device__ __forceinline__ F column_others(F acc, F v, uint32_t b0x4, uint32_t deg, uint32_t seg, uint32_t dmax) {
    if (dmax <= 8) {
        F vj[8];
#pragma unroll
        for (int q = 0; q < 8; q++) vj[q] = perm(b0x4 + 4u * P * (uint32_t)q, v);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            if ((uint32_t)q >= dmax) break;
            acc += ((uint32_t)q < deg && (uint32_t)q != seg) ? vj[q] : F(0);
        }
    } else {
        for (uint32_t j0 = 0; j0 < dmax; j0 += 8) {
            F vj[8];
#pragma unroll
            for (int q = 0; q < 8; q++) vj[q] = perm(b0x4 + 4u * P * (j0 + (uint32_t)q), v);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const uint32_t j = j0 + (uint32_t)q;
                if (j >= dmax) break;
                acc += (j < deg && j != seg) ? vj[q] : F(0);
            }
        }
    }
    return acc;
}

struct GradBufs {
    size_t msgA, msgB, sufst, sufarg, rq, rw, mbA, mbB, Lfin, Lbar, colA, colB, cS, csg, dl;
    size_t bytes;
};

// Per-block scratch layout, for E edges (slot arrays are compact: a chunk's
// edges sit on its first lanes, so the edge of lane l in chunk k has index
// base_k + l, base_k = edges in the member's earlier chunks), n columns,
// m checks and K iterations, message size fb.
__host__ __device__ inline GradBufs grad_layout(size_t S, size_t n, size_t m, uint32_t K, size_t fb) {
    GradBufs b;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    b.msgA = take(fb * S);       // messages, double-buffered over iterations
    b.msgB = take(fb * S);
    b.sufst = take(fb * S);      // suffix row states of this iteration's sweep
    b.sufarg = take(4 * S);
    b.rq = take(fb * S * K);     // records: q_e per iteration
    b.rw = take(4 * S * K);      // records: argmin slot and flags per iteration
    b.mbA = take(fb * S);        // message adjoints, double-buffered
    b.mbB = take(fb * S);
    b.Lfin = take(fb * n);       // final posteriors (unclamped)
    b.Lbar = take(fb * n);       // d loss / d L_v (0 where L_v was clamped)
    b.colA = take(fb * n);       // per-column terms of the loss stage
    b.colB = take(fb * n);
    b.cS = take(fb * m);         // per-check terms of the loss stage
    b.csg = take(4 * m);
    b.dl = take(8 * m);          // d loss / d shat_c
    b.bytes = off;
    return b;
}

}  // namespace

struct GradLaunch {
    const uint8_t* syndromes;       // B x m
    uint32_t B;                     // shots
    uint32_t K;
    const void* lam;                // n, message precision
    const void* alpha;              // K
    double eps;
    const unsigned char* recs;      // gradient schedule: per chunk meta[W] then v[W]
    const uint32_t* member_chunk;   // L + 1
    double* loss_rows;              // grid: per-block sums
    double* lbar_rows;              // grid x n
    double* abar_rows;              // grid x K
    void* scratch;
    size_t scratch_per_block;
    int grid;
};

namespace {

// The loss of the P items of a wavefront (item p of column v at v * P + p,
// of check c at c * P + p; items p >= nact are idle) from their final
// posteriors L (unclamped) and the gradient Lbar = d loss / d L_v (0 where
// L_v was clamped); returns the summed loss (every lane).
// shat_c = (1 - prod_v t_v) / 2 with t_v = tanh(L_v / 2).  FP64 messages:
// the product in the row's column order, as the definition reads.  FP32
// messages: in the log domain, which keeps shat_c accurate when it is tiny:
// with a_v = |L_v| and e_v = exp(-a_v),
//   log tanh(a_v / 2) = log1p(-e_v) - log1p(e_v) = l_v,  |prod| = exp(S_c),
//   S_c = sum_v l_v, shat_c = -expm1(S_c) / 2 if the sign product is +1,
// and dt_v / dL_v = (1 - t_v^2) / 2 = 2 e_v / (1 + e_v)^2.  l_v is bounded
// below by -80 so that exp(S_c - l_v), the product without v, stays finite.
template <class F, int P>
__device__ double loss_stage(const DevGraph& g, const Scr& sc, const uint64_t* sb, uint32_t nact, double eps,
                             const F* Lfin, F* Lbar, F* colA, F* colB, F* cS, uint32_t* csg, double* dl) {
    const uint32_t lane = threadIdx.x;
    const F lim = (F)g.clamp;
    double loss = 0.0;
    // per column: FP64 t_v; FP32 l_v and e_v
    for (uint32_t x = lane; x < g.n * P; x += kWave) {
        const uint32_t v = x / P;
        if (g.cp[v + 1] == g.cp[v]) continue;  // in no check
        const F L = clampv(xload(sc, &Lfin[x]), lim);
        if constexpr (sizeof(F) == 8) {
            colA[x] = tanh(L / 2.0);
        } else {
            const float e = expf(-fabsf(L));
            colA[x] = fmaxf(log1pf(-e) - log1pf(e), -80.0f);
            colB[x] = e;
        }
    }
    __syncthreads();
    for (uint32_t x = lane; x < g.m * P; x += kWave) {
        const uint32_t c = x / P, p = x % P;
        const bool sbit = ((sb[(c >> 6) * P + p] >> (c & 63)) & 1ull) != 0;
        double sh, sh1;  // shat_c and 1 - shat_c
        if constexpr (sizeof(F) == 8) {
            double prod = 1.0;
            for (uint32_t kk = g.rp[c]; kk < g.rp[c + 1]; kk++) prod *= xload(sc, &colA[g.ri[kk] * P + p]);
            sh = 0.5 * (1.0 - prod);
            sh1 = 1.0 - sh;
        } else {
            float S = 0.0f;
            uint32_t neg = 0;
            for (uint32_t kk = g.rp[c]; kk < g.rp[c + 1]; kk++) {
                const uint32_t u = g.ri[kk] * P + p;
                S += xload(sc, &colA[u]);
                neg ^= xload(sc, &Lfin[u]) < 0.0f ? 1u : 0u;
            }
            cS[x] = S;
            csg[x] = neg;
            const float small = -0.5f * expm1f(S), big = 0.5f * (1.0f + expf(S));
            sh = neg ? big : small;
            sh1 = neg ? small : big;
        }
        double d = 0.0;
        if (sh < eps || sh1 < eps) {
            if (sh < eps) {
                sh = eps;
                sh1 = 1.0 - eps;
            } else {
                sh1 = eps;
                sh = 1.0 - eps;
            }
        } else {
            d = sbit ? -1.0 / sh : 1.0 / sh1;
        }
        double term;
        if constexpr (sizeof(F) == 8)
            term = sbit ? log(sh) : log(sh1);
        else
            term = (double)logf((float)(sbit ? sh : sh1));
        if (p < nact) loss -= term;
        dl[x] = d;
    }
    __syncthreads();
    for (uint32_t x = lane; x < g.n * P; x += kWave) {
        const uint32_t v = x / P, p = x % P;
        const F Lv = xload(sc, &Lfin[x]);
        double gsum = 0.0;
        if (g.cp[v + 1] > g.cp[v] && Lv <= lim && Lv >= -lim) {
            for (uint32_t j = g.cp[v]; j < g.cp[v + 1]; j++) {
                const uint32_t c = g.ci[j];
                if constexpr (sizeof(F) == 8) {
                    const double tv = xload(sc, &colA[x]);
                    double ex = 1.0;
                    for (uint32_t kk = g.rp[c]; kk < g.rp[c + 1]; kk++) {
                        const uint32_t u = g.ri[kk];
                        if (u != v) ex *= xload(sc, &colA[u * P + p]);
                    }
                    gsum += xload(sc, &dl[c * P + p]) * (-0.25 * ex * (1.0 - tv * tv));
                } else {
                    const float e = xload(sc, &colB[x]);
                    const float sech2_half = 2.0f * e / ((1.0f + e) * (1.0f + e));  // dt_v / dL_v
                    const bool neg = (xload(sc, &csg[c * P + p]) != 0) != (Lv < 0.0f);
                    const float ex = expf(xload(sc, &cS[c * P + p]) - xload(sc, &colA[x]));  // |prod without v|
                    gsum += xload(sc, &dl[c * P + p]) * (-0.5 * (double)sech2_half * (double)(neg ? -ex : ex));
                }
            }
        }
        Lbar[x] = (F)gsum;
    }
    return wave_sum(loss);
}

// waves per SIMD the register allocation aims at (FP32: 6 fit without spills)
template <class F>
constexpr int grad_waves() {
    return sizeof(F) == 4 ? 6 : 3;
}

// One wavefront runs P items: P consecutive shots of one member, on the
// gradient schedule whose chunks hold at most W = 64 / P edges.  Lane l
// serves item p = l mod P at chunk position l / P, so every per-edge array
// is indexed base_k * P + l (base_k: edges in the member's earlier chunks)
// and a chunk's data for all P items is one contiguous run.
template <class F, bool FLOOD, int P>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(grad_waves<F>()))) void bp_grad_kernel(
    DevGraph g, GradLaunch a) {
    using Pr = GP<F>;
    using B = typename Pr::B;
    constexpr uint32_t W = kWave / P;
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t mP = g.m * P;
    uint64_t* sb = reinterpret_cast<uint64_t*>(lds);      // syndrome bits, word w of item p at w * P + p
    B* pst = reinterpret_cast<B*>(sb + g.words_m * P);    // running row states, m * P
    F* pacc = reinterpret_cast<F*>(pst + mP);             // row accumulators (reverse)
    F* sacc = pacc + mP;
    uint32_t* parg = reinterpret_cast<uint32_t*>(sacc + mP);
    uint32_t* ptgt = parg + mP;
    uint32_t* stgt = ptgt + mP;
    const uint32_t lane = threadIdx.x, p = lane % P, sl = lane / P;
    const F* lam = reinterpret_cast<const F*>(a.lam);
    const F* alpha = reinterpret_cast<const F*>(a.alpha);
    const F lim = (F)g.clamp;
    const B ident = Pr::ident(g);
    // per-edge slots of the P items, plus one wavefront of padding: the
    // loads of the next chunk are issued whatever its size (a conditional
    // load makes the compiler wait for every load in flight at each use),
    // and the last chunk's unused lanes read past the end
    const uint32_t S = g.E * P + kWave;
    const GradBufs lay = grad_layout(S, g.n * P, mP, a.K, sizeof(F));
    unsigned char* base = static_cast<unsigned char*>(a.scratch) + (size_t)blockIdx.x * a.scratch_per_block;
    const Scr sc = make_scr(base, (uint32_t)a.scratch_per_block);
    F* msgA = reinterpret_cast<F*>(base + lay.msgA);
    F* msgB = reinterpret_cast<F*>(base + lay.msgB);
    B* sufst = reinterpret_cast<B*>(base + lay.sufst);
    uint32_t* sufarg = reinterpret_cast<uint32_t*>(base + lay.sufarg);
    F* rq = reinterpret_cast<F*>(base + lay.rq);
    uint32_t* rw = reinterpret_cast<uint32_t*>(base + lay.rw);
    F* mbA = reinterpret_cast<F*>(base + lay.mbA);
    F* mbB = reinterpret_cast<F*>(base + lay.mbB);
    F* Lfin = reinterpret_cast<F*>(base + lay.Lfin);
    F* Lbar = reinterpret_cast<F*>(base + lay.Lbar);
    F* colA = reinterpret_cast<F*>(base + lay.colA);
    F* colB = reinterpret_cast<F*>(base + lay.colB);
    F* cS = reinterpret_cast<F*>(base + lay.cS);
    uint32_t* csg = reinterpret_cast<uint32_t*>(base + lay.csg);
    double* dl = reinterpret_cast<double*>(base + lay.dl);
    const uint32_t K = a.K;
    constexpr uint32_t rb = 8 * W;  // gradient chunk record: meta[W], v[W]
    // work units (group of P shots, member): with at least one member per
    // XCD, the blocks of one XCD (dispatched round-robin, block b to XCD
    // b mod 8) take the members of one eighth of the ensemble, so the chunk
    // records they read stay in that XCD's L2
    const uint32_t n_groups = (a.B + P - 1) / P;
    const bool grouped = g.L >= kXcds && gridDim.x >= kXcds;
    const uint32_t xcd = blockIdx.x % kXcds;
    const uint32_t mlo = grouped ? xcd * g.L / kXcds : 0u;
    const uint32_t gsz = grouped ? (xcd + 1) * g.L / kXcds - mlo : g.L;
    const uint32_t z0 = grouped ? blockIdx.x / kXcds : blockIdx.x;
    const uint32_t zstep = grouped ? (gridDim.x - xcd + kXcds - 1) / kXcds : gridDim.x;
    const uint32_t n_z = n_groups * gsz;
    double* lbar_row = a.lbar_rows + (size_t)blockIdx.x * g.n;
    for (uint32_t v = lane; v < g.n; v += kWave) lbar_row[v] = 0.0;
    double loss_acc = 0.0, abar_acc = 0.0;  // abar_acc: iteration lane + 1

    for (uint32_t z = z0; z < n_z; z += zstep) {
        const uint32_t grp = z / gsz, mem = mlo + z % gsz;
        const uint32_t shot0 = grp * P, nact = min((uint32_t)P, a.B - shot0);
        const bool act = p < nact;  // idle items repeat shot0 and contribute nothing
        for (uint32_t q = 0; q < P; q++) {
            const uint8_t* sq = a.syndromes + (size_t)(shot0 + (q < nact ? q : 0u)) * g.m;
            for (uint32_t b0 = 0; b0 < g.m; b0 += kWave) {
                const uint32_t c = b0 + lane;
                const uint64_t mk = __ballot(c < g.m && sq[c] != 0);
                if (lane == 0) sb[(b0 / kWave) * P + q] = mk;
            }
        }
        const uint32_t c0 = uni(a.member_chunk[mem]), nch = uni(a.member_chunk[mem + 1]) - c0;
        const unsigned char* recs = a.recs + (size_t)c0 * rb;
        auto meta_of = [&](uint32_t k) { return *reinterpret_cast<const uint32_t*>(recs + (size_t)k * rb + 4u * sl); };
        auto v_of = [&](uint32_t k) { return *reinterpret_cast<const uint32_t*>(recs + (size_t)k * rb + 4u * W + 4u * sl); };
        auto synd_bit = [&](uint32_t c) { return ((sb[(c >> 6) * P + p] >> (c & 63)) & 1ull) != 0; };
        auto edges = [&](uint32_t meta) { return edges_of(meta) / P; };  // per item
        __syncthreads();

        // the messages before iteration 1
        for (uint32_t k = 0, base0 = 0; k < nch; k++) {
            const uint32_t meta = meta_of(k);
            if (deg_of(meta)) msgA[base0 * P + lane] = clampv(lam[v_of(k)], lim);
            base0 += edges(meta);
        }
        __syncthreads();

        // ---- forward, recording every iteration
        for (uint32_t t = 1; t <= K; t++) {
            const F* old = (t & 1) ? msgA : msgB;
            F* nw = (t & 1) ? msgB : msgA;
            F* rqt = rq + (size_t)(t - 1) * S;
            uint32_t* rwt = rw + (size_t)(t - 1) * S;
            const F al = alpha[t - 1];

            // suffix states of the old messages: chunks in reverse
            for (uint32_t x = lane; x < mP; x += kWave) {
                pst[x] = ident;
                parg[x] = kNoArg;
            }
            __syncthreads();
            if (nch) {
                uint32_t mA = meta_of(nch - 1);
                uint32_t bA = g.E - edges(mA);
                F xA = old[bA * P + lane];
                uint32_t mB = meta_of(nch > 1 ? nch - 2 : 0u);
                for (uint32_t k = nch; k-- > 0;) {
                    const uint32_t meta = mA, base_k = bA;
                    const F x = xA;
                    mA = mB;  // chunk k - 1 (chunk 0 again at the end)
                    if (k > 0) bA = base_k - edges(mA);
                    xA = old[bA * P + lane];
                    mB = meta_of(k > 1 ? k - 2 : 0u);
                    if (deg_of(meta)) {
                        const uint32_t r = (meta & 0xffffu) * P + p, i = base_k * P + lane;
                        RS<F> run{pst[r], parg[r]};
                        sufst[i] = run.st;
                        sufarg[i] = run.arg;
                        run = rs_join(rs_of(x, i), run);
                        pst[r] = run.st;
                        parg[r] = run.arg;
                    }
                    chunk_fence();
                }
            }
            for (uint32_t x = lane; x < mP; x += kWave) {
                pst[x] = ident;
                parg[x] = kNoArg;
            }
            __syncthreads();

            // the sweep
            if (nch) {
                uint32_t mA = meta_of(0), vA = v_of(0), bA = 0;
                B sA = sufst[lane];
                uint32_t aA = sufarg[lane];
                F lA = lam[vA];  // lambda is small and stays in the caches
                F oA = FLOOD ? old[lane] : F(0);
                const uint32_t k1 = nch > 1 ? 1u : 0u;
                uint32_t mB = meta_of(k1), vB = v_of(k1);
                for (uint32_t k = 0; k < nch; k++) {
                    const uint32_t meta = mA, v = vA, base_k = bA;
                    const B sst = sA;
                    const uint32_t sarg = aA;
                    const F lr = lA, xo = oA;
                    bA = base_k + edges(meta);  // chunk k + 1 (past the end after the last)
                    mA = mB;
                    vA = vB;
                    {
                        const uint32_t i1 = bA * P + lane;
                        sA = sufst[i1];
                        aA = sufarg[i1];
                        lA = lam[vA];
                        if (FLOOD) oA = old[i1];
                    }
                    const uint32_t k2 = min(k + 2, nch - 1);
                    mB = meta_of(k2);
                    vB = v_of(k2);
                    const uint32_t deg = deg_of(meta), dmax = uni((meta >> kMetaDmaxShift) & 15u);
                    const uint32_t c = meta & 0xffffu, seg = (meta >> 16) & 15u;
                    const uint32_t r = c * P + p, i = base_k * P + lane;
                    F q = F(0);
                    uint32_t w = 0;
                    const RS<F> pre{pst[r], parg[r]};
                    if (deg) {
                        const RS<F> j = rs_join(pre, RS<F>{sst, sarg});
                        const bool neg = ((j.st & Pr::kSign) != 0) != synd_bit(c);
                        const F mag = Pr::val(j.st & ~Pr::kSign);
                        q = neg ? -mag : mag;
                        const uint32_t u = j.arg & 0x7fffffffu;
                        w = (u == kNoArg ? kSlotMask : u) | ((neg != ((j.arg >> 31) != 0)) ? kSneg : 0u);
                    }
                    const F rr = al * q;
                    const F lv = clampv(lr, lim);
                    // mu = lambda + the column's other r in check order; on
                    // the column's last position that is L without its own r
                    const uint32_t b0x4 = (uint32_t)((int)lane - (int)(seg * P)) << 2;
                    F mu = column_others<F, P>(lv, rr, b0x4, deg, seg, dmax);
                    const F L = perm(b0x4 + 4u * P * (deg - 1u), mu + rr);
                    if (deg) {
                        w |= (mu <= lim && mu >= -lim) ? kNcm : 0u;
                        w |= (lr <= lim && lr >= -lim) ? kLnc : 0u;
                        mu = clampv(mu, lim);
                        rqt[i] = q;
                        rwt[i] = w;
                        if (t < K) nw[i] = mu;
                        // serial: the row's later edges see the new message;
                        // parallel: the previous one
                        const RS<F> np = rs_join(pre, FLOOD ? rs_of(xo, i) : rs_of(mu, i));
                        pst[r] = np.st;
                        parg[r] = np.arg;
                        if (t == K && seg == 0) Lfin[v * P + p] = L;
                    }
                    chunk_fence();
                }
            }
            __syncthreads();
        }

        // ---- loss and d loss / d L (Lfin was written by other lanes)
        loss_acc += loss_stage<F, P>(g, sc, sb, nact, a.eps, Lfin, Lbar, colA, colB, cS, csg, dl);
        __syncthreads();

        // ---- reverse
        const F* mbp = mbA;  // adjoint of iteration t's new messages from iteration t + 1
        F* mbn = mbB;        // adjoint of iteration t's old messages, written out here
        for (uint32_t t = K; t >= 1; t--) {
            const F* rqt = rq + (size_t)(t - 1) * S;
            const uint32_t* rwt = rw + (size_t)(t - 1) * S;
            const F al = alpha[t - 1];
            const bool last = t == K;  // no later iteration; L enters the loss
            for (uint32_t x = lane; x < mP; x += kWave) {
                ptgt[x] = kSlotMask;
                stgt[x] = kSlotMask;
                pacc[x] = F(0);
                sacc[x] = F(0);
            }
            __syncthreads();
            double abar = 0.0;
            if (nch) {
                // mbp is not read at the last iteration (no adjoint comes
                // from later) and Lbar only there, but both loads are issued
                // every step (in bounds either way)
                uint32_t mA = meta_of(nch - 1), vA = v_of(nch - 1);
                uint32_t bA = g.E - edges(mA);
                F qA = rqt[bA * P + lane], gA = xload(sc, &mbp[bA * P + lane]), glA = xload(sc, &Lbar[vA * P + p]);
                uint32_t wA = rwt[bA * P + lane];
                const uint32_t km = nch > 1 ? nch - 2 : 0u;
                uint32_t mB = meta_of(km), vB = v_of(km);
                for (uint32_t k = nch; k-- > 0;) {
                    const uint32_t meta = mA, v = vA, w = wA, base_k = bA;
                    const F q = qA, gprev = gA, GLv = glA;
                    mA = mB;  // chunk k - 1 (chunk 0 again at the end)
                    vA = vB;
                    if (k > 0) bA = base_k - edges(mA);
                    {
                        const uint32_t i1 = bA * P + lane;
                        qA = rqt[i1];
                        wA = rwt[i1];
                        gA = xload(sc, &mbp[i1]);
                        glA = xload(sc, &Lbar[vA * P + p]);
                    }
                    const uint32_t k2 = k > 1 ? k - 2 : 0u;
                    mB = meta_of(k2);
                    vB = v_of(k2);
                    const uint32_t deg = deg_of(meta), dmax = uni((meta >> kMetaDmaxShift) & 15u);
                    const uint32_t c = meta & 0xffffu, seg = (meta >> 16) & 15u;
                    const uint32_t r = c * P + p, i = base_k * P + lane;
                    F gin = last ? F(0) : gprev;
                    if (deg) {
                        if (!FLOOD && ptgt[r] == i) {  // the prefix argmin reached: take its adjoint
                            gin += pacc[r];
                            ptgt[r] = kSlotMask;
                        }
                        mbn[i] = F(0);  // written out later if this edge is a suffix argmin
                    }
                    const F gm = (deg && (w & kNcm)) ? gin : F(0);
                    const F GL = (deg && last) ? GLv : F(0);
                    const uint32_t b0x4 = (uint32_t)((int)lane - (int)(seg * P)) << 2;
                    const F others = column_others<F, P>(F(0), gm, b0x4, deg, seg, dmax);
                    if (deg) {
                        const F rbar = others + GL;
                        // the column's last position adds its own term last:
                        // the sum over the column in check order
                        if (act && seg + 1 == deg && (w & kLnc)) unsafeAtomicAdd(&lbar_row[v], (double)((others + gm) + GL));
                        if (act) abar += (double)(rbar * q);
                        const uint32_t u = w & kSlotMask;
                        if (u != kSlotMask) {
                            const F d = (w & kSneg) ? -(rbar * al) : rbar * al;
                            if (FLOOD) {
                                if (ptgt[r] == u || ptgt[r] == kSlotMask) {
                                    ptgt[r] = u;
                                    pacc[r] += d;
                                } else {
                                    stgt[r] = u;
                                    sacc[r] += d;
                                }
                            } else if (u < i) {
                                pacc[r] = ptgt[r] == kSlotMask ? d : pacc[r] + d;
                                ptgt[r] = u;
                            } else if (stgt[r] != u) {
                                if (stgt[r] != kSlotMask) mbn[stgt[r]] = sacc[r];
                                stgt[r] = u;
                                sacc[r] = d;
                            } else {
                                sacc[r] += d;
                            }
                        }
                    }
                    chunk_fence();
                }
            }
            __syncthreads();
            for (uint32_t x = lane; x < mP; x += kWave) {
                if (stgt[x] != kSlotMask) mbn[stgt[x]] = sacc[x];
                if (FLOOD && ptgt[x] != kSlotMask) mbn[ptgt[x]] = pacc[x];
            }
            abar = wave_sum(abar);
            if (lane == t - 1) abar_acc += abar;
            __syncthreads();
            F* tmp = const_cast<F*>(mbp);
            mbp = mbn;
            mbn = tmp;
        }
        // the old messages of iteration 1 are lambda itself
        for (uint32_t k = 0, base0 = 0; k < nch; k++) {
            const uint32_t meta = meta_of(k), v = v_of(k);
            const uint32_t deg = deg_of(meta), dmax = uni((meta >> kMetaDmaxShift) & 15u);
            const uint32_t seg = (meta >> 16) & 15u;
            const uint32_t i = base0 * P + lane;
            base0 += edges(meta);
            const F x = deg ? xload(sc, &mbp[i]) : F(0);
            const F gm = (deg && (rw[i] & kLnc)) ? x : F(0);
            const uint32_t b0x4 = (uint32_t)((int)lane - (int)(seg * P)) << 2;
            const F others = column_others<F, P>(F(0), gm, b0x4, deg, seg, dmax);
            if (act && deg && seg + 1 == deg) unsafeAtomicAdd(&lbar_row[v], (double)(others + gm));
        }
        // (a column without checks is in no check's product: its gradient is 0)
        __syncthreads();
    }
    if (lane == 0) a.loss_rows[blockIdx.x] = loss_acc;
    if (lane < K) a.abar_rows[(size_t)blockIdx.x * K + lane] = abar_acc;
}

// out[j] = sum over rows r of in[r * width + j]: eight partial sums over the
// rows r = p (mod 8), each in ascending r, then the eight in order of p
__global__ __launch_bounds__(256) void reduce_rows_kernel(const double* in, uint32_t rows, uint32_t width,
                                                          double* out) {
    __shared__ double part[8][32];
    const uint32_t jl = threadIdx.x & 31u, p = threadIdx.x >> 5;
    const uint32_t j = blockIdx.x * 32u + jl;
    double acc = 0.0;
    if (j < width)
        for (uint32_t r = p; r < rows; r += 8) acc += in[(size_t)r * width + j];
    part[p][jl] = acc;
    __syncthreads();
    if (p == 0 && j < width) {
        double sum = part[0][jl];
        for (int q = 1; q < 8; q++) sum += part[q][jl];
        out[j] = sum;
    }
}

template <class F, bool FLOOD>
const void* grad_fn(uint32_t P) {
    return P == 4 ? (const void*)bp_grad_kernel<F, FLOOD, 4>
                  : P == 2 ? (const void*)bp_grad_kernel<F, FLOOD, 2> : (const void*)bp_grad_kernel<F, FLOOD, 1>;
}

}  // namespace

// grad launch limits: blocks (one wavefront each) and their scratch in total
constexpr uint64_t kGradMaxGrid = 8192;
constexpr uint64_t kGradScratchBudget = 40ull << 30;
constexpr size_t kGradMaxLds = 160 * 1024;  // LDS of one workgroup on gfx950

size_t grad_scratch_per_block(const DevGraph& g, uint32_t K, uint32_t P) {
    return grad_layout((size_t)g.E * P + kWave, (size_t)g.n * P, (size_t)g.m * P, K, g.fp64 ? 8 : 4).bytes;
}

size_t grad_lds_bytes(const DevGraph& g, uint32_t P) {
    const size_t fb = g.fp64 ? 8 : 4;
    return (8ull * g.words_m + (3 * fb + 12) * g.m) * P + 16;
}

const void* grad_kernel_for(const DevGraph& g, uint32_t P) {
    return g.fp64 ? (g.flood ? grad_fn<double, true>(P) : grad_fn<double, false>(P))
                  : (g.flood ? grad_fn<float, true>(P) : grad_fn<float, false>(P));
}

// blocks of the gradient kernel resident on the whole device at once
int grad_resident_blocks(const DevGraph& g, uint32_t P) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, grad_kernel_for(g, P), kWave, grad_lds_bytes(g, P)) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu * cus;
}

int launch_grad(const DevGraph& g, uint32_t P, const GradLaunch& a, hipStream_t st) {
    const void* fn = grad_kernel_for(g, P);
    const size_t lds = grad_lds_bytes(g, P);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(grad)");
    }
    void* args[] = {const_cast<DevGraph*>(&g), const_cast<GradLaunch*>(&a)};
    hipError_t e = hipLaunchKernel(fn, dim3(a.grid), dim3(kWave), args, lds, st);
    if (e != hipSuccess) return hip_fail(e, "bp_grad_kernel launch");
    return VIBE_OK;
}

// The gradient schedule.  The decode schedule's chunks (at most 64 edges,
// whole columns, no two columns sharing a check) are recut into chunks of
// at most W edges, columns kept whole and in lane order: a part of an
// independent set is independent, so the sweep is unchanged.  W = 64 / P
// lets one wavefront run P shots side by side; W is the one of 64, 32, 16
// that gives the least estimated time per shot (on graphs whose chunks are
// far from full, most of a 64-lane chunk is idle).  Built once per graph.
int build_grad_schedule(vibe_graph* G) {
    if (G->grad_width) return VIBE_OK;
    const DevGraph& d = G->h.dg;
    const uint32_t L = d.L;
    std::vector<uint32_t> mc(L + 1);
    hipError_t e = hipMemcpy(mc.data(), d.member_chunk, 4ull * (L + 1), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(member_chunk)");
    const size_t nrec = mc[L];
    const uint32_t rb = rec_bytes(d.fp64 != 0);
    std::vector<unsigned char> recs(std::max<size_t>(nrec, 1) * rb);
    if (nrec) {
        e = hipMemcpy(recs.data(), d.sched, nrec * rb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(schedule)");
    }
    auto meta_at = [&](size_t k, uint32_t q) { return reinterpret_cast<const uint32_t*>(recs.data() + k * rb)[q]; };
    auto v_at = [&](size_t k, uint32_t q) { return reinterpret_cast<const uint32_t*>(recs.data() + k * rb + kRecV)[q]; };
    // the columns of chunk k as (first lane, degree)
    auto columns = [&](size_t k, std::vector<std::pair<uint32_t, uint32_t>>& out) {
        out.clear();
        for (uint32_t q = 0; q < (uint32_t)kWave;) {
            const uint32_t deg = (meta_at(k, q) >> kMetaDegShift) & 15u;
            if (!deg) break;
            out.push_back({q, deg});
            q += deg;
        }
    };
    std::vector<std::pair<uint32_t, uint32_t>> cols;
    uint32_t bestW = kWave;
    double best = -1.0;
    for (uint32_t W : {64u, 32u, 16u}) {
        // P shots per wavefront multiply the LDS row state by P
        if (W < (uint32_t)kWave && grad_lds_bytes(G->h.dg, kWave / W) > kGradMaxLds) continue;
        size_t cnt = 0;
        for (uint32_t i = 0; i < L; i++) {
            size_t ci = 0;
            for (size_t k = mc[i]; k < mc[i + 1]; k++) {
                columns(k, cols);
                uint32_t fill = W + 1;
                for (auto& cd : cols) {
                    if (fill + cd.second > W) {
                        ci++;
                        fill = 0;
                    }
                    fill += cd.second;
                }
            }
            cnt += ci;
        }
        // chunk steps per shot, weighted by the cost of a step with P shots
        // side by side (measured on the d = 5 and d = 7 circuit graphs: a
        // step takes 1.2-1.7x as long with P = 2 and 1.6-2.0x with P = 4;
        // the larger factors are used)
        const uint32_t P = kWave / W;
        const double step = P == 1 ? 1.0 : P == 2 ? 1.7 : 2.0;
        const double cost = (double)cnt * step / P;
        if (best < 0 || cost < best) {
            best = cost;
            bestW = W;
        }
    }
#ifdef VIBE_GRAD_WIDTH
    bestW = VIBE_GRAD_WIDTH;  // build-time override, for measurements
#endif
    if (G->grad_force) bestW = G->grad_force;
    const uint32_t W = bestW;
    std::vector<uint32_t> out;  // per chunk: meta[W], v[W]
    std::vector<uint32_t> gmc(L + 1, 0);
    uint32_t maxc = 0;
    for (uint32_t i = 0; i < L; i++) {
        gmc[i] = (uint32_t)(out.size() / (2 * W));
        for (size_t k = mc[i]; k < mc[i + 1]; k++) {
            columns(k, cols);
            size_t a = 0;
            while (a < cols.size()) {
                size_t b = a;
                uint32_t fill = 0, dmax = 0;
                while (b < cols.size() && fill + cols[b].second <= W) {
                    fill += cols[b].second;
                    dmax = std::max(dmax, cols[b].second);
                    b++;
                }
                const size_t at = out.size();
                out.resize(at + 2 * W, 0);
                uint32_t lane = 0;
                for (size_t cc = a; cc < b; cc++)
                    for (uint32_t j = 0; j < cols[cc].second; j++, lane++) {
                        const uint32_t q = cols[cc].first + j;
                        out[at + lane] = (meta_at(k, q) & ~(15u << kMetaDmaxShift)) | (dmax << kMetaDmaxShift);
                        out[at + W + lane] = v_at(k, q);
                    }
                for (; lane < W; lane++) out[at + lane] = dmax << kMetaDmaxShift;  // unused slots
                a = b;
            }
        }
        maxc = std::max(maxc, (uint32_t)(out.size() / (2 * W)) - gmc[i]);
    }
    gmc[L] = (uint32_t)(out.size() / (2 * W));
    if (out.empty()) out.assign(2 * W, 0);
    void* pr = nullptr;
    void* pm = nullptr;
    if (hipMalloc(&pr, 4 * out.size()) != hipSuccess) return fail(VIBE_ENOMEM, "gradient schedule allocation failed");
    G->h.allocations.push_back(pr);
    if (hipMalloc(&pm, 4 * gmc.size()) != hipSuccess) return fail(VIBE_ENOMEM, "gradient schedule allocation failed");
    G->h.allocations.push_back(pm);
    G->h.device_bytes += 4 * (out.size() + gmc.size());
    if ((e = hipMemcpy(pr, out.data(), 4 * out.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pm, gmc.data(), 4 * gmc.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(gradient schedule)");
    G->grad_recs = static_cast<const unsigned char*>(pr);
    G->grad_member_chunk = static_cast<const uint32_t*>(pm);
    G->grad_P = kWave / W;
    G->grad_max_chunks = maxc;
    G->grad_width = W;
    return VIBE_OK;
}

int launch_reduce_rows(const double* in, uint32_t rows, uint32_t width, double* out, hipStream_t st) {
    if (!width) return VIBE_OK;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3((width + 31) / 32), dim3(256), 0, st, in, rows, width, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "reduce_rows_kernel launch");
}

}  // namespace vibe

using namespace vibe;

extern "C" int vibe_grad_set_width(vibe_graph* G, uint32_t width) {
    set_error("");
    if (!G) return fail(VIBE_EINVAL, "graph handle is NULL");
    if (width != 0 && width != 16 && width != 32 && width != 64)
        return fail(VIBE_EINVAL, "width must be 0 (automatic), 16, 32 or 64");
    if (width == G->grad_force) return VIBE_OK;
    if (G->grad_width) {  // drop the schedule built for the previous setting
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        auto& al = G->h.allocations;
        for (const void* p : {static_cast<const void*>(G->grad_recs), static_cast<const void*>(G->grad_member_chunk)})
            for (size_t i = 0; i < al.size(); i++)
                if (al[i] == p) {
                    (void)hipFree(al[i]);
                    al.erase(al.begin() + (long)i);
                    break;
                }
        G->grad_recs = nullptr;
        G->grad_member_chunk = nullptr;
        G->grad_width = 0;
    }
    G->grad_force = width;
    return VIBE_OK;
}

extern "C" int vibe_bp_grad(vibe_graph* G, const uint8_t* syndromes, uint64_t B, uint32_t K, const void* lam,
                            const void* alpha, double eps, double* loss, double* dlam, double* dalpha,
                            void* stream) {
    set_error("");
    if (!G) return fail(VIBE_EINVAL, "graph handle is NULL");
    if (K < 1 || K > 64) return fail(VIBE_EINVAL, "K must be in 1..64");
    if (!B) return fail(VIBE_EINVAL, "B must be >= 1");
    if (!syndromes || !lam || !alpha || !loss || !dlam || !dalpha) return fail(VIBE_EINVAL, "NULL argument");
    if (!(eps > 0.0 && eps < 0.5)) return fail(VIBE_EINVAL, "eps must be in (0, 0.5)");
    const DevGraph& g = G->h.dg;
    if (g.layered) return fail(VIBE_EUNSUPPORTED, "the gradient covers the serial-V and parallel schedules");
    if ((uint64_t)g.E >= kSlotMask) return fail(VIBE_EUNSUPPORTED, "graph too large for the gradient (E >= 2^24 - 1)");
    const uint64_t items64 = B * g.L;
    if (items64 > (1u << 24)) return fail(VIBE_EINVAL, "B x L must be at most 2^24");
    int rc = build_grad_schedule(G);
    if (rc) return rc;
    const uint32_t P = G->grad_P;
    if (grad_lds_bytes(g, P) > kGradMaxLds)
        return fail(VIBE_EUNSUPPORTED, "the gradient's LDS row state exceeds 160 KB (too many checks for this width)");
    const uint64_t units = (B + P - 1) / P * g.L;  // (group of P shots, member)
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t per = grad_scratch_per_block(g, K, P);
    if (per >= (1ull << 31)) return fail(VIBE_EUNSUPPORTED, "gradient scratch per wavefront exceeds 2 GB (graph x K too large)");
    // as many blocks as can be resident at once (work is assigned
    // statically, so more would only queue), within the scratch budget
    const uint64_t fit = std::max<uint64_t>(1, kGradScratchBudget / std::max<size_t>(per, 1));
    const uint64_t resident = std::max<uint64_t>(1, (uint64_t)grad_resident_blocks(g, P));
    const uint32_t grid = (uint32_t)std::min<uint64_t>(units, std::min<uint64_t>(std::min(kGradMaxGrid, resident), fit));
    // workspace: per-block loss, lambda-bar and alpha-bar rows | scratch
    auto round256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_loss = off;
    off += round256(8ull * grid);
    const size_t o_lbar = off;
    off += round256(8ull * grid * g.n);
    const size_t o_abar = off;
    off += round256(8ull * grid * K);
    const size_t o_scr = off;
    off += per * grid;
    if (G->ws.bytes < off) {
        if (G->ws.base) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
            (void)hipFree(G->ws.base);
            G->ws.base = nullptr;
            G->ws.bytes = 0;
        }
        if (hipMalloc(&G->ws.base, off) != hipSuccess) return fail(VIBE_ENOMEM, "grad workspace allocation failed");
        G->ws.bytes = off;
    }
    unsigned char* base = static_cast<unsigned char*>(G->ws.base);
    GradLaunch a{};
    a.syndromes = syndromes;
    a.B = (uint32_t)B;
    a.K = K;
    a.lam = lam;
    a.alpha = alpha;
    a.eps = eps;
    a.recs = G->grad_recs;
    a.member_chunk = G->grad_member_chunk;
    a.loss_rows = reinterpret_cast<double*>(base + o_loss);
    a.lbar_rows = reinterpret_cast<double*>(base + o_lbar);
    a.abar_rows = reinterpret_cast<double*>(base + o_abar);
    a.scratch = base + o_scr;
    a.scratch_per_block = per;
    a.grid = (int)grid;
    if ((rc = launch_grad(g, P, a, st))) return rc;
    if ((rc = launch_reduce_rows(a.loss_rows, grid, 1, loss, st))) return rc;
    if ((rc = launch_reduce_rows(a.lbar_rows, grid, g.n, dlam, st))) return rc;
    return launch_reduce_rows(a.abar_rows, grid, K, dalpha, st);
}
