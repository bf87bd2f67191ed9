// Adjoint of K unrolled min-sum iterations: gradients of the soft-syndrome
// loss with respect to the channel LLRs lambda_v and the per-iteration
// scaling factors alpha_t (the differentiable decoder; Algorithm 1 unrolled).
//
// Forward: K iterations of the serial (or parallel) schedule without early
// stop, from lambda and alpha given as inputs, keeping the messages at the
// start of every iteration (checkpoints).  Loss: with the final posteriors
// L_v, shat_c = (1 - prod_{v in N(c)} tanh(L_v / 2)) / 2 clamped to
// [eps, 1 - eps], loss = sum_c BCE(s_c, shat_c).
//
// Reverse, iteration t = K .. 1: the iteration is recomputed from its
// checkpoint, recording for every edge e = (c, v) its check message
// r_e = alpha_t q_e, the edge u* that attains the minimum (with its sign) and
// whether the new message was clamped.  Then the chunks are visited in
// reverse order.  Edge e's new message feeds the other edges' messages of
// its column (and L_v after the last iteration), so
//   rbar_e = sum_{e' in column, e' != e} mubar_e' + Lbar_v,
//   lambdabar_v += sum_{e' in column} mubar_e' + Lbar_v,
//   alphabar_t += rbar_e q_e,
//   mubar_{u*} += rbar_e alpha_t (1 - 2 s_c) prod sign * sign(mu_{u*}),
// where mu_{u*} is u*'s new message of iteration t if u* comes earlier in
// the sweep (its adjoint is completed later in the reverse order) and its
// message of iteration t - 1 otherwise (the adjoint passed on to iteration
// t - 1).  At t = 1 the messages are lambda itself.  Sign products, argmin
// choices and clamps are piecewise constant: where they do not change, this
// is the exact gradient of the loss.
//
// One wavefront per (shot, member) item.  Items go to blocks statically
// (block b takes items b, b + grid, ...); a block sums its items' loss and
// gradients in item order into a row of its own, and the rows are summed in
// a fixed order, so the result does not depend on timing.  Adjoints that one
// lane adds into a slot that another lane reads go through device atomics,
// issued by one wavefront in program order, and are read back with
// agent-scope loads.
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
// that edge's own sign in bit 31 (kNoArg: none).
constexpr uint32_t kNoArg = 0x7fffffffu;

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

template <class F>
__device__ inline F shfl_f(F v, int src) {
    return __shfl(v, src);
}

__device__ inline double aload(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline float aload(const float* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

template <class F>
__device__ inline F wave_sum(F x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

struct GradItemBufs {
    size_t ckpt, mu_new, sufst, sufarg, rq, rarg, flags, mubar_a, mubar_b, Lfin, Lbar, dl;
    size_t bytes;
};

// Per-block scratch layout, for S slots (max_chunks * 64), n columns, m checks
// and K iterations, element size fb.
__host__ __device__ inline GradItemBufs grad_layout(size_t S, size_t n, size_t m, uint32_t K, size_t fb) {
    GradItemBufs b;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    b.ckpt = take(fb * S * K);   // messages at the start of iterations 1..K
    b.mu_new = take(fb * S);     // this iteration's new messages (recompute)
    b.sufst = take(fb * S);      // suffix states of the recompute
    b.sufarg = take(4 * S);
    b.rq = take(fb * S);         // q_e, r_e = alpha_t q_e
    b.rarg = take(4 * S);        // argmin slot | its sign, or kNoArg
    b.flags = take(4 * S);       // bit 0: new message not clamped; bit 1: sign factor negative
    b.mubar_a = take(fb * S);
    b.mubar_b = take(fb * S);
    b.Lfin = take(fb * n);
    b.Lbar = take(fb * n);
    b.dl = take(8 * m);          // d loss / d shat_c (the loss stage runs in FP64)
    b.bytes = off;
    return b;
}

}  // namespace

struct GradLaunch {
    const uint8_t* syndromes;  // B x m
    uint32_t B;                // shots
    uint32_t K;
    const void* lam;           // n, message precision
    const void* alpha;         // K
    double eps;
    double* loss_rows;         // grid: per-block sums
    double* lbar_rows;         // grid x n
    double* abar_rows;         // grid x K
    void* scratch;
    size_t scratch_per_block;
    int grid;
};

namespace {

template <class F, bool FLOOD>
__global__ __launch_bounds__(kWave) void bp_grad_kernel(DevGraph g, GradLaunch a) {
    using P = GP<F>;
    using B = typename P::B;
    extern __shared__ __align__(16) unsigned char lds[];
    uint64_t* sb = reinterpret_cast<uint64_t*>(lds);
    B* pst = reinterpret_cast<B*>(sb + g.words_m);  // prefix states, m
    uint32_t* parg = reinterpret_cast<uint32_t*>(pst + g.m);
    const int lane = threadIdx.x;
    const F* lam = reinterpret_cast<const F*>(a.lam);
    const F* alpha = reinterpret_cast<const F*>(a.alpha);
    const F lim = (F)g.clamp;
    const B ident = P::ident(g);
    const uint32_t S = g.max_chunks * kWave;
    const GradItemBufs lay = grad_layout(S, g.n, g.m, a.K, sizeof(F));
    unsigned char* base = static_cast<unsigned char*>(a.scratch) + (size_t)blockIdx.x * a.scratch_per_block;
    F* ckpt = reinterpret_cast<F*>(base + lay.ckpt);
    F* mu_new = reinterpret_cast<F*>(base + lay.mu_new);
    B* sufst = reinterpret_cast<B*>(base + lay.sufst);
    uint32_t* sufarg = reinterpret_cast<uint32_t*>(base + lay.sufarg);
    F* rq = reinterpret_cast<F*>(base + lay.rq);
    uint32_t* rarg = reinterpret_cast<uint32_t*>(base + lay.rarg);
    uint32_t* flags = reinterpret_cast<uint32_t*>(base + lay.flags);
    F* mbA = reinterpret_cast<F*>(base + lay.mubar_a);
    F* mbB = reinterpret_cast<F*>(base + lay.mubar_b);
    F* Lfin = reinterpret_cast<F*>(base + lay.Lfin);
    F* Lbar = reinterpret_cast<F*>(base + lay.Lbar);
    double* dl = reinterpret_cast<double*>(base + lay.dl);
    const uint32_t n_items = a.B * g.L;
    double* lbar_row = a.lbar_rows + (size_t)blockIdx.x * g.n;
    for (uint32_t v = lane; v < g.n; v += kWave) lbar_row[v] = 0.0;
    double loss_acc = 0.0, abar_acc = 0.0;  // abar_acc: iteration lane + 1

    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint32_t shot = item / g.L, mem = item % g.L;
        const uint8_t* s = a.syndromes + (size_t)shot * g.m;
        for (uint32_t b0 = 0; b0 < g.m; b0 += kWave) {
            const uint32_t c = b0 + lane;
            const uint64_t mk = __ballot(c < g.m && s[c] != 0);
            if (lane == 0) sb[b0 / kWave] = mk;
        }
        const uint32_t c0 = uni(g.member_chunk[mem]), nch = uni(g.member_chunk[mem + 1]) - c0;
        const uint32_t rb = rec_bytes(sizeof(F) == 8);
        const unsigned char* recs = g.sched + (size_t)c0 * rb;
        auto meta_of = [&](uint32_t k) { return *reinterpret_cast<const uint32_t*>(recs + (size_t)k * rb + 4u * lane); };
        auto v_of = [&](uint32_t k) { return *reinterpret_cast<const uint32_t*>(recs + (size_t)k * rb + kRecV + 4u * lane); };
        __syncthreads();

        // the iteration from messages `old` (slot order): records q, argmin,
        // flags and the new messages; at the last iteration also L
        auto iterate = [&](const F* old, uint32_t t, bool last) {
            const F al = alpha[t - 1];
            // suffix states (with argmin) of the old messages
            for (uint32_t c = lane; c < g.m; c += kWave) {
                pst[c] = ident;
                parg[c] = kNoArg;
            }
            __syncthreads();
            for (uint32_t k = nch; k-- > 0;) {
                const uint32_t meta = meta_of(k);
                const uint32_t i = k * kWave + lane;
                if ((meta >> kMetaDegShift) & 15u) {
                    const uint32_t c = meta & 0xffffu;
                    RS<F> run{pst[c], parg[c]};
                    sufst[i] = run.st;
                    sufarg[i] = run.arg;
                    run = rs_join(rs_of(old[i], i), run);
                    pst[c] = run.st;
                    parg[c] = run.arg;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            for (uint32_t c = lane; c < g.m; c += kWave) {
                pst[c] = ident;
                parg[c] = kNoArg;
            }
            __syncthreads();
            // the sweep
            for (uint32_t k = 0; k < nch; k++) {
                const uint32_t meta = meta_of(k), v = v_of(k);
                const uint32_t deg = (meta >> kMetaDegShift) & 15u, dmax = uni((meta >> kMetaDmaxShift) & 15u);
                const uint32_t c = meta & 0xffffu, seg = (meta >> 16) & 15u;
                const uint32_t i = k * kWave + lane;
                F q = F(0);
                RS<F> pre{pst[c], parg[c]};
                if (deg) {
                    const RS<F> j = rs_join(pre, RS<F>{sufst[i], sufarg[i]});
                    const bool neg = ((j.st & P::kSign) != 0) != (((sb[c >> 6] >> (c & 63)) & 1ull) != 0);
                    const F mag = P::val(j.st & ~P::kSign);
                    q = neg ? -mag : mag;
                    rq[i] = q;
                    rarg[i] = j.arg;
                    // sign factor of dr/dmu_{u*}: (1 - 2 s_c) prod sign * sign(mu_{u*})
                    const bool sneg = neg != ((j.arg & 0x80000000u) != 0);
                    flags[i] = sneg ? 2u : 0u;
                }
                const F r = al * q;
                const F lv = deg ? clampv(lam[v], lim) : F(0);
                F L = lv, mu = lv;
                const int b0 = lane - (int)seg;
                for (uint32_t jj = 0; jj < dmax; jj++) {
                    const F rj = shfl_f(r, (b0 + (int)jj) & (kWave - 1));
                    if (jj < deg) {
                        L += rj;
                        if (jj != seg) mu += rj;
                    }
                }
                if (deg) {
                    const bool ncm = mu <= lim && mu >= -lim;
                    mu = clampv(mu, lim);
                    mu_new[i] = mu;
                    flags[i] |= ncm ? 1u : 0u;
                    // serial: the row's later edges see the new message
                    // parallel: they see the previous one
                    const RS<F> mine = FLOOD ? rs_of(old[i], i) : rs_of(mu, i);
                    const RS<F> np = rs_join(pre, mine);
                    pst[c] = np.st;
                    parg[c] = np.arg;
                    if (last && seg == 0) Lfin[v] = L;  // unclamped (flags of L in Lbar)
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
        };

        // ---- forward with checkpoints
        for (uint32_t k = 0; k < nch; k++) {
            const uint32_t i = k * kWave + lane;
            const uint32_t meta = meta_of(k);
            ckpt[i] = ((meta >> kMetaDegShift) & 15u) ? clampv(lam[v_of(k)], lim) : F(0);
        }
        for (uint32_t v = lane; v < g.n; v += kWave) Lfin[v] = clampv(lam[v], lim);  // columns without checks
        __syncthreads();
        for (uint32_t t = 1; t <= a.K; t++) {
            iterate(ckpt + (size_t)(t - 1) * S, t, t == a.K);
            if (t < a.K)
                for (uint32_t k = 0; k < nch; k++) {
                    const uint32_t i = k * kWave + lane;
                    ckpt[(size_t)t * S + i] = mu_new[i];
                }
            __syncthreads();
        }
        // ---- loss and d loss / d L, in FP64 whatever the message precision
        // (Lfin was written by other lanes)
        double loss = 0.0;
        const double dlim = g.clamp;
        for (uint32_t c = lane; c < g.m; c += kWave) {
            double prod = 1.0;
            for (uint32_t kk = g.rp[c]; kk < g.rp[c + 1]; kk++)
                prod *= tanh(clampv((double)aload(&Lfin[g.ri[kk]]), dlim) / 2.0);
            double sh = 0.5 * (1.0 - prod), d = 0.0;
            const bool sc = s[c] != 0;
            if (sh < a.eps || sh > 1.0 - a.eps) {
                sh = sh < a.eps ? a.eps : 1.0 - a.eps;
            } else {
                d = sc ? -1.0 / sh : 1.0 / (1.0 - sh);
            }
            loss -= sc ? log(sh) : log(1.0 - sh);
            dl[c] = d;
        }
        loss_acc += wave_sum(loss);
        __syncthreads();
        for (uint32_t v = lane; v < g.n; v += kWave) {
            const double Lv = (double)aload(&Lfin[v]);
            double gsum = 0.0;
            if (Lv <= dlim && Lv >= -dlim) {
                const double tv = tanh(Lv / 2.0);
                for (uint32_t j = g.cp[v]; j < g.cp[v + 1]; j++) {
                    const uint32_t c = g.ci[j];
                    double ex = 1.0;
                    for (uint32_t kk = g.rp[c]; kk < g.rp[c + 1]; kk++) {
                        const uint32_t u = g.ri[kk];
                        if (u != v) ex *= tanh(clampv((double)aload(&Lfin[u]), dlim) / 2.0);
                    }
                    gsum += aload(&dl[c]) * (-0.25 * ex * (1.0 - tv * tv));
                }
            }
            Lbar[v] = (F)gsum;
        }
        __syncthreads();

        // ---- reverse
        for (uint32_t k = 0; k < nch; k++) mbA[k * kWave + lane] = F(0);
        __syncthreads();
        F* mb_new = mbA;  // adjoint of iteration t's new messages
        F* mb_old = mbB;  // adjoint of its old messages (iteration t - 1's)
        for (uint32_t t = a.K; t >= 1; t--) {
            iterate(ckpt + (size_t)(t - 1) * S, t, t == a.K);
            const F al = alpha[t - 1];
            for (uint32_t k = 0; k < nch; k++) mb_old[k * kWave + lane] = F(0);
            __syncthreads();
            double abar = 0.0;
            for (uint32_t k = nch; k-- > 0;) {
                const uint32_t meta = meta_of(k), v = v_of(k);
                const uint32_t deg = (meta >> kMetaDegShift) & 15u, dmax = uni((meta >> kMetaDmaxShift) & 15u);
                const uint32_t seg = (meta >> 16) & 15u;
                const uint32_t i = k * kWave + lane;
                const uint32_t fl = deg ? flags[i] : 0u;
                const F gm = deg && (fl & 1u) ? aload(&mb_new[i]) : F(0);
                F GL = F(0);
                if (deg && t == a.K) {
                    const F Lv = aload(&Lfin[v]);
                    GL = (Lv <= lim && Lv >= -lim) ? aload(&Lbar[v]) : F(0);
                }
                // column sums of the message adjoints
                F all = F(0), others = F(0);
                const int b0 = lane - (int)seg;
                for (uint32_t jj = 0; jj < dmax; jj++) {
                    const F gj = shfl_f(gm, (b0 + (int)jj) & (kWave - 1));
                    if (jj < deg) {
                        all += gj;
                        if (jj != seg) others += gj;
                    }
                }
                if (deg) {
                    const F rbar = others + GL;
                    const F lr = lam[v];
                    if (seg == 0 && lr <= lim && lr >= -lim) unsafeAtomicAdd(&lbar_row[v], (double)(all + GL));
                    const F q = rq[i];
                    abar += (double)(rbar * q);
                    const uint32_t u = rarg[i] & 0x7fffffffu;
                    if (u != kNoArg) {
                        const F d = rbar * al * ((fl & 2u) ? F(-1) : F(1));
                        // serial: an earlier slot holds this iteration's new
                        // message; parallel: every slot its previous one
                        F* tgt = (!FLOOD && u < i) ? mb_new : mb_old;
                        unsafeAtomicAdd(&tgt[u], d);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            abar = wave_sum(abar);
            if (lane == t - 1) abar_acc += abar;
            __syncthreads();
            F* tmp = mb_new;
            mb_new = mb_old;
            mb_old = tmp;
        }
        // the messages before iteration 1 are lambda itself
        for (uint32_t k = 0; k < nch; k++) {
            const uint32_t meta = meta_of(k), v = v_of(k);
            const uint32_t deg = (meta >> kMetaDegShift) & 15u, dmax = uni((meta >> kMetaDmaxShift) & 15u);
            const uint32_t seg = (meta >> 16) & 15u;
            const uint32_t i = k * kWave + lane;
            const F x = deg ? aload(&mb_new[i]) : F(0);
            const F lv = deg ? lam[v] : F(0);
            const F gm = (lv <= lim && lv >= -lim) ? x : F(0);
            F all = F(0);
            const int b0 = lane - (int)seg;
            for (uint32_t jj = 0; jj < dmax; jj++) {
                const F gj = shfl_f(gm, (b0 + (int)jj) & (kWave - 1));
                if (jj < deg) all += gj;
            }
            if (deg && seg == 0) unsafeAtomicAdd(&lbar_row[v], (double)all);
        }
        // (a column without checks is in no check's product: its gradient is 0)
        __syncthreads();
    }
    if (lane == 0) a.loss_rows[blockIdx.x] = loss_acc;
    if (lane < a.K) a.abar_rows[(size_t)blockIdx.x * a.K + lane] = abar_acc;
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
const void* grad_fn() {
    return (const void*)bp_grad_kernel<F, FLOOD>;
}

}  // namespace

// grad launch limits: blocks (one wavefront each) and their scratch in total
constexpr uint64_t kGradMaxGrid = 8192;
constexpr uint64_t kGradScratchBudget = 16ull << 30;

size_t grad_scratch_per_block(const DevGraph& g, uint32_t K) {
    return grad_layout((size_t)g.max_chunks * kWave, g.n, g.m, K, g.fp64 ? 8 : 4).bytes;
}

size_t grad_lds_bytes(const DevGraph& g) {
    const size_t fb = g.fp64 ? 8 : 4;
    return 8ull * g.words_m + (fb + 4) * g.m + 16;
}

int launch_grad(const DevGraph& g, const GradLaunch& a, hipStream_t st) {
    const void* fn = g.fp64 ? (g.flood ? grad_fn<double, true>() : grad_fn<double, false>())
                            : (g.flood ? grad_fn<float, true>() : grad_fn<float, false>());
    const size_t lds = grad_lds_bytes(g);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(grad)");
    }
    void* args[] = {const_cast<DevGraph*>(&g), const_cast<GradLaunch*>(&a)};
    hipError_t e = hipLaunchKernel(fn, dim3(a.grid), dim3(kWave), args, lds, st);
    if (e != hipSuccess) return hip_fail(e, "bp_grad_kernel launch");
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
    const uint64_t items64 = B * g.L;
    if (items64 > (1u << 24)) return fail(VIBE_EINVAL, "B x L must be at most 2^24");
    const uint32_t items = (uint32_t)items64;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t per = grad_scratch_per_block(g, K);
    // one block per resident wavefront slot at most, within the scratch budget
    const uint64_t fit = std::max<uint64_t>(1, kGradScratchBudget / std::max<size_t>(per, 1));
    const uint32_t grid = (uint32_t)std::min<uint64_t>(items, std::min<uint64_t>(kGradMaxGrid, fit));
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
    a.loss_rows = reinterpret_cast<double*>(base + o_loss);
    a.lbar_rows = reinterpret_cast<double*>(base + o_lbar);
    a.abar_rows = reinterpret_cast<double*>(base + o_abar);
    a.scratch = base + o_scr;
    a.scratch_per_block = per;
    a.grid = (int)grid;
    int rc = launch_grad(g, a, st);
    if (rc) return rc;
    if ((rc = launch_reduce_rows(a.loss_rows, grid, 1, loss, st))) return rc;
    if ((rc = launch_reduce_rows(a.lbar_rows, grid, g.n, dlam, st))) return rc;
    return launch_reduce_rows(a.abar_rows, grid, K, dalpha, st);
}
