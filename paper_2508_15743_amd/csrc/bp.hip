// K1: the ensemble of serial-V min-sum decoders (paper Appendix A, Algorithm 1;
// ensemble and correction limit, Sec. III.D).
//
// One wavefront decodes one work item = (shot, member).
//
// Exact serial sweep without row rescans.  When column v is visited, the
// edges of a row that come before v in the sweep carry this sweep's messages
// and those after v still hold the previous sweep's.  So min and sign parity
// over N(c) \ v split into
//   * a prefix state per check (running min and parity of this sweep's new
//     messages), 4 bytes of LDS per check, and
//   * a suffix state (min and parity of the previous sweep's messages on the
//     row's later edges), kept in the edge's own slot of the message slab.
// The slab follows the member's sweep order, so a chunk reads the suffix
// states of its edges and overwrites them with the new messages in one
// contiguous run.  After the sweep, a backward pass over the chunks with a
// running state per check (LDS) turns the new messages into the next sweep's
// suffix states, again one contiguous run per chunk.
//
// Columns that share no check commute, so the host grouped the sweep into
// dependency levels and chunks of at most 64 edges holding whole columns;
// a chunk runs with one lane per edge and the result is bit-identical to the
// column-by-column sweep.  Sums over a column's edges run in ascending check
// order through wave shuffles.  Hard decisions, the residual syndrome
// s + H e and the syndrome are bit-packed in LDS; convergence is a ballot.
#include "internal.h"

namespace vibe {

namespace {

__device__ inline float clampf(float x, float lim) { return fminf(fmaxf(x, -lim), lim); }

__device__ inline uint32_t rs_encode(float x) {
    return (__float_as_uint(x) & 0x7fffffffu) | (x < 0.0f ? 0x80000000u : 0u);
}

__device__ inline uint64_t load_mask(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double wave_sum_f64(double x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ inline uint32_t wave_sum_u32(uint32_t x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return uni(x);
}

__device__ inline uint32_t wave_max_u32(uint32_t x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off));
    return uni(x);
}

// Members known to precede `mem` in (convergence iteration, index) order:
// converged before iteration t, or at t with a lower index.
__device__ inline uint32_t preceding_converged(const uint64_t* mask, uint32_t t, uint32_t mem, int lane) {
    uint32_t cnt = 0;
    for (uint32_t tt = lane + 1; tt < t; tt += kWave) cnt += __popcll(load_mask(&mask[tt]));
    const uint32_t own = __popcll(load_mask(&mask[t]) & ((1ull << mem) - 1ull));
    cnt += lane == 0 ? own : 0u;  // a select, not a branch on the lane
    return wave_sum_u32(cnt);
}

// Backward pass: turn the slab's new messages (float bits) into the suffix
// states of the next sweep.  Chunks from last to first; running[c] is the
// state of the part of row c already passed.  Edges of one chunk sit in
// distinct rows, so a chunk is one parallel step.
__device__ void suffix_pass(const DevGraph& g, uint32_t* slab, uint32_t* running, uint32_t ch_lo,
                            uint32_t ch_hi, size_t mbase, int lane) {
    for (uint32_t c = lane; c < g.m; c += kWave) running[c] = g.ident;
    __syncthreads();
    uint32_t nmeta = 0, nx = 0, nlen = 0;
    size_t npos = 0;
    if (ch_hi > ch_lo) {
        const uint32_t beg = g.chunk_off[ch_hi - 1];
        nlen = g.chunk_off[ch_hi] - beg;
        npos = beg - mbase + lane;
        if ((uint32_t)lane < nlen) {
            nmeta = g.slots[beg + lane].meta;
            nx = slab[npos];
        }
    }
    for (uint32_t ch = ch_hi; ch-- > ch_lo;) {
        const uint32_t meta = nmeta, x = nx, len = nlen;
        const size_t pos = npos;
        if (ch > ch_lo) {
            const uint32_t beg = g.chunk_off[ch - 1];
            nlen = g.chunk_off[ch] - beg;
            npos = beg - mbase + lane;
            if ((uint32_t)lane < nlen) {
                nmeta = g.slots[beg + lane].meta;
                nx = slab[npos];
            }
        }
        if ((uint32_t)lane < len) {
            const uint32_t c = meta & 0xffffu;
            const uint32_t st = running[c];
            slab[pos] = st;
            running[c] = rs_combine(rs_encode(__uint_as_float(x)), st);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

template <bool SLAB_LDS>
__global__ __launch_bounds__(kWave) void bp_ensemble_kernel(DevGraph g, BpLaunch a) {
    extern __shared__ __align__(16) unsigned char lds[];
    uint64_t* sb = reinterpret_cast<uint64_t*>(lds);
    uint64_t* res = sb + g.words_m;
    uint64_t* eb = res + g.words_m;
    uint32_t* pref = reinterpret_cast<uint32_t*>(eb + g.words_n);
    uint32_t* slab = SLAB_LDS ? pref + g.m : a.slab + (size_t)blockIdx.x * g.E;

    const int lane = threadIdx.x;
    float* post = a.post_slab + (size_t)blockIdx.x * g.n;
    const uint32_t n_items = a.n_shots * g.L;
    const float lim = g.clamp;
    const float al = g.alpha;

    for (;;) {
        const uint32_t item = wave_ticket(a.counter, 1u);
        if (item >= n_items) break;
        uint32_t shot, mem;
        if (a.member_major) {
            mem = item / a.n_shots;
            shot = item % a.n_shots;
        } else {
            shot = item / g.L;
            mem = item % g.L;
        }
        const uint32_t rec = shot * g.L + mem;  // output record of this item
        const uint8_t* s = a.syndromes + (size_t)(a.shot0 + shot) * g.m;
        uint64_t* cmask = a.conv_mask + (size_t)shot * (kMaxT + 1);

        // ---- syndrome bits; the residual s + H e starts at s (e = 0)
        uint64_t any = 0;
        for (uint32_t base = 0; base < g.m; base += kWave) {
            const uint32_t c = base + lane;
            const uint64_t mask = __ballot(c < g.m && s[c] != 0);
            if (lane == 0) {
                sb[base / kWave] = mask;
                res[base / kWave] = mask;
            }
            any |= mask;
        }
        if (a.use_M && preceding_converged(cmask, 1, mem, lane) >= g.M) {
            // M members of lower index converged at the first iteration: this
            // one cannot be among the first M
            if (lane == 0) a.t_conv[rec] = 0;
            continue;
        }
        if (!any && a.fast_zero && g.all_lam_positive) {
            // s = 0 with every lambda > 0: the first sweep leaves every message
            // positive, so the decision is e = 0 and it satisfies s at t = 1.
            if (a.cand)
                for (uint32_t w = lane; w < g.words_n; w += kWave) a.cand[(size_t)rec * g.words_n + w] = 0;
            if (lane == 0) {
                a.t_conv[rec] = 1;
                if (a.weight) a.weight[rec] = 0.0;
                atomicOr(reinterpret_cast<unsigned long long*>(&cmask[1]), 1ull << mem);
                atomicAdd(&a.iters[shot], 1u);
            }
            continue;
        }
        // The slab is only ever re-read by the lane that wrote it: a slot's
        // position is (chunk start + lane) in the sweep and in the backward
        // pass alike.  The first sweep reads the suffix states of the initial
        // messages from the graph itself.
        const size_t mbase = (size_t)mem * g.E;  // this member's first slot
        const uint32_t* init = g.init_suf + mbase;
        for (uint32_t w = lane; w < g.words_n; w += kWave) eb[w] = g.e0[w];
        __syncthreads();

        const uint32_t ch_lo = g.member_chunk[mem], ch_hi = g.member_chunk[mem + 1];
        uint32_t conv_t = 0, ran = 0;
        bool stopped = false;
        for (uint32_t t = 1; t <= a.T_run; t++) {
            if (a.use_M && t >= 2 && preceding_converged(cmask, t, mem, lane) >= g.M) {
                stopped = true;  // cannot be among the first M any more
                break;
            }
            const bool want_post = a.post_out != nullptr || (a.accumulate_q && t == a.T_run);
            if (want_post) {
                // columns without checks keep L_v = lambda_v
                for (uint32_t v = lane; v < g.n; v += kWave) {
                    const float l = g.lam[v];
                    post[v] = l;
                    if (a.post_out) a.post_out[(size_t)rec * g.n + v] = l;
                }
            }
            for (uint32_t c = lane; c < g.m; c += kWave) pref[c] = g.ident;
            __syncthreads();

            // software pipeline: the slots and suffix states of the next chunk
            // are loaded while the current chunk is processed (suffix states
            // of later slots are final for the whole sweep)
            Slot nsl{0, 0};
            uint32_t nsuf = g.ident, nlen = 0;
            size_t npos = 0;
            if (ch_lo < ch_hi) {
                const uint32_t nbeg = g.chunk_off[ch_lo];
                nlen = g.chunk_off[ch_lo + 1] - nbeg;
                npos = nbeg - mbase + lane;
                if ((uint32_t)lane < nlen) {
                    nsl = g.slots[nbeg + lane];
                    nsuf = t == 1 ? init[npos] : slab[npos];
                }
            }
            for (uint32_t ch = ch_lo; ch < ch_hi; ch++) {
                const Slot sl = nsl;
                const uint32_t suf = nsuf;
                const uint32_t len = nlen;
                const size_t pos = npos;
                if (ch + 1 < ch_hi) {
                    const uint32_t nbeg = g.chunk_off[ch + 1];
                    nlen = g.chunk_off[ch + 2] - nbeg;
                    npos = nbeg - mbase + lane;
                    if ((uint32_t)lane < nlen) {
                        nsl = g.slots[nbeg + lane];
                        nsuf = t == 1 ? init[npos] : slab[npos];
                    }
                }
                const bool act = (uint32_t)lane < len;
                const uint32_t c = sl.meta & 0xffffu;
                const uint32_t seg = (sl.meta >> 16) & 15u;
                const uint32_t deg = act ? (sl.meta >> 20) & 15u : 0u;
                float r = 0.0f, lv = 0.0f;
                uint32_t pre = 0;
                if (act) {
                    lv = g.lam[sl.v];
                    pre = pref[c];
                    // r_{c->v} = (1 - 2 s_c) alpha prod sign min |mu|, over N(c) \ v
                    const uint32_t st = rs_combine(pre, suf);
                    const uint32_t neg = (st >> 31) ^ (uint32_t)((sb[c >> 6] >> (c & 63)) & 1ull);
                    const float rr = al * __uint_as_float(st & 0x7fffffffu);
                    r = neg ? -rr : rr;
                }
                // sums over the column's edges in ascending check order
                const uint32_t dmax = wave_max_u32(deg);
                const int b0 = lane - (int)seg;
                float L = lv, x = lv;
                for (uint32_t j = 0; j < dmax; j++) {
                    const float rj = __shfl(r, (b0 + (int)j) & (kWave - 1));
                    if (j < deg) {
                        L += rj;
                        if (j != seg) x += rj;
                    }
                }
                if (act) {
                    L = clampf(L, lim);
                    x = clampf(x, lim);
                    slab[pos] = __float_as_uint(x);
                    pref[c] = rs_combine(pre, rs_encode(x));
                    const uint32_t v = sl.v;
                    const bool enew = L <= 0.0f;
                    const bool eold = (eb[v >> 6] >> (v & 63)) & 1ull;
                    if (enew != eold) {
                        if (seg == 0) atomicXor(reinterpret_cast<unsigned long long*>(&eb[v >> 6]), 1ull << (v & 63));
                        atomicXor(reinterpret_cast<unsigned long long*>(&res[c >> 6]), 1ull << (c & 63));
                    }
                    if (want_post && seg == 0) {
                        post[v] = L;
                        if (a.post_out) a.post_out[(size_t)rec * g.n + v] = L;
                    }
                }
                // LDS writes of this chunk precede the next chunk's reads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();  // every new message stored
            ran = t;
            // converged iff the residual s + H e is zero
            bool nz = false;
            for (uint32_t w = lane; w < g.words_m; w += kWave) nz |= res[w] != 0;
            if (__ballot(nz) == 0) {
                if (!conv_t) conv_t = t;
                if (a.stop_on_converge) break;
            }
            if (t < a.T_run) {
                suffix_pass(g, slab, pref, ch_lo, ch_hi, mbase, lane);
                __syncthreads();
            }
        }

        if (lane == 0) {
            a.t_conv[rec] = (int32_t)conv_t;
            atomicAdd(&a.iters[shot], ran);
        }
        if (a.cand && (conv_t || !a.use_M))
            for (uint32_t w = lane; w < g.words_n; w += kWave) a.cand[(size_t)rec * g.words_n + w] = eb[w];
        if (a.weight && conv_t) {
            // W(e) = sum_v e_v lambda_v in FP64, ascending v
            double W = 0.0;
            for (uint32_t base = 0; base < g.words_n; base += kWave) {
                const uint32_t w = base + lane;
                uint64_t nzw = __ballot(w < g.words_n && eb[w] != 0);
                if (lane == 0) {
                    while (nzw) {
                        const int bi = __ffsll((long long)nzw) - 1;
                        nzw &= nzw - 1;
                        uint64_t xw = eb[base + bi];
                        while (xw) {
                            const int bb = __ffsll((long long)xw) - 1;
                            xw &= xw - 1;
                            W += g.lam64[(size_t)(base + bi) * 64 + bb];
                        }
                    }
                }
            }
            if (lane == 0) a.weight[rec] = W;
        }
        if (lane == 0 && conv_t) atomicOr(reinterpret_cast<unsigned long long*>(&cmask[conv_t]), 1ull << mem);
        if (a.accumulate_q && !conv_t && !stopped && ran == a.T_run) {
            // normalised posterior, summed over the members of a shot with no
            // converged member, in 2^-56 fixed point (order-independent)
            uint32_t cnt = 0;
            for (uint32_t tt = lane + 1; tt <= a.T_run; tt += kWave) cnt += __popcll(load_mask(&cmask[tt]));
            if (wave_sum_u32(cnt) == 0) {
                // post[v] was written by the lane that swept v: read it past the L1
                double ss = 0.0;
                for (uint32_t v = lane; v < g.n; v += kWave) {
                    const double xv = __hip_atomic_load(&post[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ss += xv * xv;
                }
                ss = wave_sum_f64(ss);
                if (uni(ss > 0.0 ? 1u : 0u)) {
                    const double scale = kQScale / sqrt(ss);
                    int64_t* q = a.qfix + (size_t)shot * g.n;
                    for (uint32_t v = lane; v < g.n; v += kWave) {
                        const double xv = __hip_atomic_load(&post[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        atomicAdd(reinterpret_cast<unsigned long long*>(&q[v]), (unsigned long long)llrint(xv * scale));
                    }
                }
            }
        }
        __syncthreads();
    }
}

__global__ void zero_kernel(uint32_t* p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

size_t bp_lds_bytes(const DevGraph& g, bool slab_in_lds) {
    size_t b = sizeof(uint64_t) * (2 * (size_t)g.words_m + g.words_n) + sizeof(uint32_t) * g.m;
    if (slab_in_lds) b += sizeof(uint32_t) * (size_t)g.E;
    return b;
}

bool bp_slab_fits_lds(const DevGraph& g) { return bp_lds_bytes(g, true) <= 96 * 1024; }

int bp_grid(const DevGraph& g, bool slab_in_lds) {
    static int cached_cus = 0;
    if (!cached_cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
        cached_cus = prop.multiProcessorCount;
    }
    const size_t lds = bp_lds_bytes(g, slab_in_lds);
    int per_cu = 0;
    hipError_t e = slab_in_lds
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bp_ensemble_kernel<true>, kWave, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bp_ensemble_kernel<false>, kWave, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    if (per_cu > 16) per_cu = 16;
    return per_cu * cached_cus;
}

int launch_bp(const DevGraph& g, const BpLaunch& a, hipStream_t st) {
    const size_t lds = bp_lds_bytes(g, a.slab_in_lds != 0);
    const void* fn = a.slab_in_lds ? (const void*)bp_ensemble_kernel<true> : (const void*)bp_ensemble_kernel<false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(bp)");
    }
    if (a.slab_in_lds)
        hipLaunchKernelGGL(bp_ensemble_kernel<true>, dim3(a.grid), dim3(kWave), lds, st, g, a);
    else
        hipLaunchKernelGGL(bp_ensemble_kernel<false>, dim3(a.grid), dim3(kWave), lds, st, g, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bp_ensemble_kernel launch");
    return VIBE_OK;
}

int launch_zero(void* p, size_t bytes, hipStream_t st) {
    if (!bytes) return VIBE_OK;
    const size_t words = (bytes + 3) / 4;
    const int blocks = (int)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, static_cast<uint32_t*>(p), words);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "zero_kernel launch");
}

}  // namespace vibe
