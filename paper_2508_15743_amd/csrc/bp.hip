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
//     messages), one word of LDS per check, and
//   * a suffix state (min and parity of the previous sweep's messages on the
//     row's later edges), kept in the edge's own slot of the message slab.
// The slab follows the member's schedule, so a chunk reads the suffix states
// of its edges and overwrites them with the new messages in one contiguous
// run of 64 slots.  After the sweep, a backward pass over the chunks with a
// running state per check (LDS) turns the new messages into the next sweep's
// suffix states, again one run per chunk.
//
// Columns that share no check commute, so the host packed each member's
// sweep into chunks of mutually independent columns with at most 64 edges;
// a chunk runs with one lane per edge and the result is bit-identical to the
// column-by-column sweep.  Sums over a column's edges run in ascending check
// order through wave shuffles, as in a column-by-column decoder, and nothing
// is contracted into fused multiply-adds, so the FP64 variant reproduces a
// plain FP64 decoder bit for bit.  The chain of chunks is the critical path:
// both passes load their slots three chunks ahead (six in the latency
// variant).  The residual syndrome
// s + H e and the syndrome are bit-packed in LDS, and so are the hard
// decisions (or, on graphs where that bitmap would cap residency, they sit
// in global memory: a mask per chunk read with the chunk's slots, and a
// bitmap updated on flips); convergence is a ballot.
//
// Launch variants (none changes a result): the slab in LDS for small
// graphs; P = 2 or 4 shots of a member per wavefront on the member's
// schedule recut into chunks of 64 / P edges; several requests on
// different graphs in one persistent launch (ragged); and, for a launch
// whose items all reside at once, the deeper prefetch ring at four waves
// per SIMD (the latency variant).
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

#pragma clang fp contract(off)

namespace vibe {

namespace {

template <class F>
struct Prec;

template <>
struct Prec<float> {
    using B = uint32_t;
    static constexpr B kSign = 0x80000000u;
    __device__ static B bits(float x) { return __float_as_uint(x); }
    __device__ static float val(B b) { return __uint_as_float(b); }
    __device__ static float clamp(float x, float lim) { return __builtin_amdgcn_fmed3f(x, -lim, lim); }
    __device__ static B ident(const DevGraph& g) { return g.ident32; }
};

template <>
struct Prec<double> {
    using B = uint64_t;
    static constexpr B kSign = 0x8000000000000000ull;
    __device__ static B bits(double x) { return (uint64_t)__double_as_longlong(x); }
    __device__ static double val(B b) { return __longlong_as_double((long long)b); }
    __device__ static double clamp(double x, double lim) { return fmin(fmax(x, -lim), lim); }
    __device__ static B ident(const DevGraph& g) { return g.ident64; }
};

// value of the lane whose index is byte_addr / 4 (mod 64)
__device__ __forceinline__ float bperm(uint32_t byte_addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((int)byte_addr, __float_as_int(v)));
}
__device__ __forceinline__ double bperm(uint32_t byte_addr, double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute((int)byte_addr, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute((int)byte_addr, (int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <class F>
__device__ inline typename Prec<F>::B rs_encode(F x) {
    using P = Prec<F>;
    return (P::bits(x) & ~P::kSign) | (x < F(0) ? P::kSign : (typename P::B)0);
}

__device__ inline uint64_t load_mask(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lane j's value, broadcast (j wave-uniform)
__device__ inline double readlane_f64(double x, int j) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ inline uint32_t wave_sum_u32(uint32_t x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return uni(x);
}

// Members known to precede `mem` in (convergence iteration, index) order:
// converged before iteration t, or at t with a lower index.
__device__ uint32_t preceding_converged(const uint64_t* mask, uint32_t t, uint32_t mem, int lane) {
    uint32_t cnt = 0;
    for (uint32_t tt = lane + 1; tt < t; tt += kWave) cnt += __popcll(load_mask(&mask[tt]));
    const uint32_t own = __popcll(load_mask(&mask[t]) & ((1ull << mem) - 1ull));
    cnt += lane == 0 ? own : 0u;  // a select, not a branch on the lane
    return wave_sum_u32(cnt);
}

// Buffer resources: the schedule of one member and the message slab of one
// block are addressed as a wave-uniform descriptor plus a per-lane byte
// offset, so no 64-bit address is formed per lane and load.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kBufFlags = 0x00020000;  // 32-bit data format: plain dword access

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufFlags);
}

template <class T>
__device__ __forceinline__ T bload(Rsrc r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
        return __builtin_bit_cast(T, u);
    } else {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
        return __builtin_bit_cast(T, u);
    }
}

// the same, missing the vector L1: for words another lane wrote
template <class T>
__device__ __forceinline__ T bloadx(Rsrc r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 1);
        return __builtin_bit_cast(T, u);
    } else {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 1);
        return __builtin_bit_cast(T, u);
    }
}

template <class T>
__device__ __forceinline__ void bstore(T v, Rsrc r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
    } else {
        using V2 = __attribute__((ext_vector_type(2))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)voff, (int)soff, 0);
    }
}

// What one work item's passes need.
template <class F>
struct Ctx {
    using B = typename Prec<F>::B;
    Rsrc sch;       // the member's chunk records
    Rsrc slb;       // the block's slab (global variant)
    B* lslab;       // the block's slab (LDS variant)
    Rsrc mslb;      // parallel schedule: the block's message slab (global variant)
    B* lmslab;      // parallel schedule: the block's message slab (LDS variant)
    B* pref;
    const uint64_t* sb;
    uint64_t* res;
    uint64_t* eb;
    F* post;        // n posteriors
    F* trash;       // 64 slots that absorb the posterior stores of lanes that
                    // own no column
    F al, lim;
    int lane;
    uint32_t lane4, laneF;  // lane * 4, lane * sizeof(F)
    uint32_t rec4, recF;    // several shots per wavefront: the lane's slot in
                            // a record of W = 64 / P entries, * 4, * sizeof(F)
    Rsrc dsl;               // decisions in global memory: the block's decision
                            // mask of each chunk (bit q: the decision of the
                            // column that slot q belongs to)
};

// Byte offsets of the fields in a chunk record of W entries per field.
template <class F, uint32_t W>
struct RecW {
    static constexpr uint32_t kV = 4 * W, kLam = 8 * W, kInit = 8 * W + W * (uint32_t)sizeof(F);
    static constexpr uint32_t kBytes = W * (8 + 2 * (uint32_t)sizeof(F));
};
static_assert(RecW<float, 64>::kV == kRecV && RecW<float, 64>::kLam == kRecLam &&
                  RecW<float, 64>::kInit == rec_init(false) && RecW<float, 64>::kBytes == rec_bytes(false) &&
                  RecW<double, 64>::kInit == rec_init(true) && RecW<double, 64>::kBytes == rec_bytes(true),
              "record geometry");

// Every vector memory operation of a chunk step is issued unconditionally
// (prefetch indices are clamped instead of tested, unused slots store junk
// into their own slab slot), so the compiler can count the loads still in
// flight and wait only for the oldest stage instead of draining all of them.
#ifndef VIBE_BP_DEPTH
#define VIBE_BP_DEPTH 3
#endif
constexpr int kDepth = VIBE_BP_DEPTH;  // chunks loaded ahead of the one being processed
// The latency variant: a launch whose work items all reside at once is bound
// by each item's chain of chunk steps, not by the slab stream, and loading
// six chunks ahead shortens each step (single shots of the d = 9 and d = 13
// circuit graphs: 8% and 12% faster); the deeper ring needs the registers
// of 4 waves per SIMD, which such a launch does not miss.
constexpr int kLatDepth = 6;
// occupancy the register allocator aims for (waves per SIMD): 6 keeps the
// production kernel (FP32, serial schedule, global slab, one request, or
// several requests none of which is layered) within 80 VGPRs (with
// decisions in global memory a few registers spill, outside the chunk
// loops); the other FP32 variants need more registers and aim for 5, the
// FP64 ones for 4
#ifndef VIBE_BP_WAVES_PER_EU
#define VIBE_BP_WAVES_PER_EU 6
#endif
template <class F, bool SLAB_LDS, bool FLOOD, bool RAGGED, bool WITH_LAYERED = false, bool DG = false>
constexpr int waves_target() {
    return sizeof(F) == 8 ? 4 : (!SLAB_LDS && !FLOOD && !(RAGGED && WITH_LAYERED) ? VIBE_BP_WAVES_PER_EU : 5);
}

// Slot data of one chunk for the sweep, loaded ahead of use.
template <class F>
struct Stage {
    uint32_t meta, v;
    F lam;
    typename Prec<F>::B suf;
    F old;        // parallel schedule: the edge's message of the previous iteration
    uint32_t dm;  // decisions in global memory: the half of the chunk's decision
                  // mask of the previous sweep that holds this lane's bit
};

// W: entries per record field (64 / shots per wavefront).  The slab slot
// of a lane is always chunk * 64 + lane.
template <class F, bool SLAB_LDS, bool FLOOD, uint32_t W = kWave, bool DG = false>
__device__ __forceinline__ void fetch(const Ctx<F>& x, Stage<F>& s, uint32_t k, bool first) {
    using P = Prec<F>;
    using B = typename P::B;
    using R = RecW<F, W>;
    // chunk offset added to the lane offset (a short-lived VGPR); field
    // offsets become instruction immediates
    const uint32_t base = k * R::kBytes;
    const uint32_t o4 = (W == kWave ? x.lane4 : x.rec4) + base, oF = (W == kWave ? x.laneF : x.recF) + base;
    s.meta = bload<uint32_t>(x.sch, o4, 0);
    s.v = bload<uint32_t>(x.sch, o4 + R::kV, 0);
    s.lam = bload<F>(x.sch, oF + R::kLam, 0);
    if constexpr (SLAB_LDS) {
        s.suf = x.lslab[k * kWave + x.lane];
    } else {
        // first sweep: the initial suffix states of the schedule record
        const Rsrc r = first ? x.sch : x.slb;
        const uint32_t o = first ? oF + R::kInit : x.laneF + k * kWave * (uint32_t)sizeof(B);
        s.suf = bload<B>(r, o, 0);
    }
    if constexpr (FLOOD) {
        // the previous message (lambda before the first iteration); the
        // load is issued either way so that every step issues the same
        // memory operations
        B m;
        if constexpr (SLAB_LDS)
            m = x.lmslab[k * kWave + x.lane];
        else
            m = bload<B>(x.mslb, x.laneF + k * kWave * (uint32_t)sizeof(B), 0);
        s.old = first ? s.lam : P::val(m);
    }
    if constexpr (DG) {
        // written by this wavefront's previous sweep (read past the L1);
        // every chunk column starts at e = 0 in the first sweep
        const uint32_t m = bloadx<uint32_t>(x.dsl, k * 8u + (((uint32_t)x.lane >> 5) << 2), 0);
        s.dm = first ? 0u : m;
    }
}

// One chunk of the sweep: r_{c->v} = (1 - 2 s_c) alpha prod sign min |mu|
// over N(c) \ v for each edge, then L_v and the new mu_{v->c}.  Serial
// schedule: the row's earlier edges contribute their new messages (the
// prefix state accumulates them).  Parallel schedule (FLOOD): they
// contribute their previous messages, so every message of the iteration
// comes from the previous iteration's.
template <class F, bool SLAB_LDS, bool WANT_POST, bool FLOOD, bool DG = false>
__device__ __forceinline__ void sweep_chunk(const Ctx<F>& x, const Stage<F>& s, uint32_t k, uint64_t& sat) {
    using P = Prec<F>;
    using B = typename P::B;
    const uint32_t meta = s.meta, v = s.v;
    const uint32_t deg = (meta >> kMetaDegShift) & 15u;  // 0: unused slot (c = 0, v = 0)
    const uint32_t dmax = uni((meta >> kMetaDmaxShift) & 15u);
    const uint32_t c = meta & 0xffffu, seg = (meta >> 16) & 15u;
    // the LDS words this edge needs, issued together
    const B pre = x.pref[c];
    const uint64_t sw = x.sb[c >> 6];
    uint64_t ew = 0;
    if constexpr (!DG) ew = x.eb[v >> 6];
    const B stt = rs_combine<B>(pre, s.suf);
    const bool neg = ((stt & P::kSign) != 0) != (((sw >> (c & 63)) & 1ull) != 0);
    const F rr = x.al * P::val(stt & ~P::kSign);
    const F r = deg ? (neg ? -rr : rr) : F(0);
    // mu_{v->c} = lambda_v + sum_{c' != c} r and L_v = lambda_v + sum_c r, in
    // ascending check order over the column's consecutive lanes.  Position
    // j of the column is lane b0 + j, read at a constant offset from one
    // base address, eight positions per batch with all reads issued first;
    // positions outside the column and the edge's own position add an
    // exact zero (which changes no value, only possibly the sign of a zero
    // result).  On the column's last lane the partial sums of mu are those
    // of L, so L = mu + r there exactly, and one more read hands it to the
    // whole column.
    const uint32_t b0x4 = (uint32_t)(x.lane - (int)seg) << 2;
    F mu = s.lam;
    if (dmax <= 8) {
        // one batch, offsets fixed at compile time
        F rj[8];
#pragma unroll
        for (int q = 0; q < 8; q++) rj[q] = bperm(b0x4 + 4u * (uint32_t)q, r);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            if ((uint32_t)q >= dmax) break;
            mu += ((uint32_t)q < deg && (uint32_t)q != seg) ? rj[q] : F(0);
        }
    } else {
        for (uint32_t j0 = 0; j0 < dmax; j0 += 8) {
            F rj[8];
#pragma unroll
            for (int q = 0; q < 8; q++) rj[q] = bperm(b0x4 + 4u * (j0 + (uint32_t)q), r);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const uint32_t j = j0 + (uint32_t)q;
                if (j >= dmax) break;
                mu += (j < deg && j != seg) ? rj[q] : F(0);
            }
        }
    }
    F L = bperm(b0x4 + 4u * (deg - 1u), mu + r);
    L = P::clamp(L, x.lim);
    mu = P::clamp(mu, x.lim);
    // saturation witness: lanes whose posterior or message reached the clamp
    sat |= __ballot(deg && (fabs(L) >= x.lim || fabs(mu) >= x.lim));
    if constexpr (FLOOD) {
        if constexpr (SLAB_LDS)
            x.lmslab[k * kWave + x.lane] = P::bits(mu);
        else
            bstore<B>(P::bits(mu), x.mslb, x.laneF + k * kWave * (uint32_t)sizeof(B), 0);
    } else {
        if constexpr (SLAB_LDS)
            x.lslab[k * kWave + x.lane] = P::bits(mu);
        else
            bstore<B>(P::bits(mu), x.slb, x.laneF + k * kWave * (uint32_t)sizeof(B), 0);
    }
    const bool enew = L <= F(0);
    // the column's previous decision: its bit of the decision bitmap, or
    // this lane's bit of the chunk's decision mask
    bool eold;
    if constexpr (DG)
        eold = ((s.dm >> ((uint32_t)x.lane & 31u)) & 1u) != 0;
    else
        eold = (ew >> (v & 63)) & 1ull;
    if (deg) {
        x.pref[c] = rs_combine<B>(pre, rs_encode(FLOOD ? s.old : mu));
        if (enew != eold) {
            if (seg == 0) atomicXor(reinterpret_cast<unsigned long long*>(&x.eb[v >> 6]), 1ull << (v & 63));
            atomicXor(reinterpret_cast<unsigned long long*>(&x.res[c >> 6]), 1ull << (c & 63));
        }
    }
    if constexpr (WANT_POST) {
        F* dst = (deg && seg == 0) ? x.post + v : x.trash + x.lane;
        *dst = L;
    }
    if constexpr (DG) {
        // the chunk's new decision mask, stored by every lane (the same
        // value, so that the store is unconditional)
        bstore<uint64_t>(__ballot(deg && enew), x.dsl, k * 8u, 0);
    }
    // LDS writes of this chunk precede the next chunk's reads; nothing of a
    // later chunk is scheduled into this one (that would keep every stage's
    // derived values live at once)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

// The whole sweep: chunks 0 .. nch-1 (nch >= 1), each one's slots loaded
// kDepth chunks ahead (the suffix states of later chunks are final for the
// whole sweep).
template <class F, bool SLAB_LDS, bool WANT_POST, bool FLOOD, uint32_t W = kWave, bool DG = false, int D = kDepth>
__device__ __forceinline__ void sweep(const Ctx<F>& x, uint32_t nch, bool first, uint64_t& sat) {
    const uint32_t last = nch - 1;
    Stage<F> ring[D];
#pragma unroll
    for (int d = 0; d < D; d++) fetch<F, SLAB_LDS, FLOOD, W, DG>(x, ring[d], min((uint32_t)d, last), first);
    for (uint32_t k = 0; k < nch; k += D) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            if (k + d >= nch) break;
            sweep_chunk<F, SLAB_LDS, WANT_POST, FLOOD, DG>(x, ring[d], k + d, sat);
            fetch<F, SLAB_LDS, FLOOD, W, DG>(x, ring[d], min(k + d + D, last), first);
        }
    }
}

template <class F>
struct BStage {
    uint32_t meta;
    typename Prec<F>::B msg;
};

template <class F, bool SLAB_LDS, bool FLOOD, uint32_t W = kWave>
__device__ __forceinline__ void bfetch(const Ctx<F>& x, BStage<F>& s, uint32_t k) {
    using B = typename Prec<F>::B;
    s.meta = bload<uint32_t>(x.sch, (W == kWave ? x.lane4 : x.rec4) + k * RecW<F, W>::kBytes, 0);
    // the sweep's new messages: in the state slab itself (serial), or in the
    // message slab (parallel)
    if constexpr (SLAB_LDS)
        s.msg = (FLOOD ? x.lmslab : x.lslab)[k * kWave + x.lane];
    else
        s.msg = bload<B>(FLOOD ? x.mslb : x.slb, x.laneF + k * kWave * (uint32_t)sizeof(B), 0);
}

// One chunk of the backward pass: the slot receives the state of its row's
// later edges, then its own message joins the running state.
template <class F, bool SLAB_LDS>
__device__ __forceinline__ void back_chunk(const Ctx<F>& x, const BStage<F>& s, uint32_t k,
                                           typename Prec<F>::B* running) {
    using B = typename Prec<F>::B;
    const uint32_t c = s.meta & 0xffffu;
    const B stt = running[c];
    if constexpr (SLAB_LDS)
        x.lslab[k * kWave + x.lane] = stt;
    else
        bstore<B>(stt, x.slb, x.laneF + k * kWave * (uint32_t)sizeof(B), 0);
    if ((s.meta >> kMetaDegShift) & 15u) running[c] = rs_combine<B>(rs_encode(Prec<F>::val(s.msg)), stt);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_sched_barrier(0);
}

// Backward pass over chunks nch-1 .. 0 (nch >= 1) with loads kDepth chunks
// ahead.  Edges of one chunk sit in distinct rows, so a chunk is one
// parallel step.
template <class F, bool SLAB_LDS, bool FLOOD, uint32_t W = kWave, int D = kDepth>
__device__ __forceinline__ void backward(const Ctx<F>& x, uint32_t nch, typename Prec<F>::B* running) {
    BStage<F> ring[D];
    auto at = [nch](uint32_t d) { return d < nch ? nch - 1 - d : 0u; };  // d chunks from the end
#pragma unroll
    for (int d = 0; d < D; d++) bfetch<F, SLAB_LDS, FLOOD, W>(x, ring[d], at(d));
    for (uint32_t e = 0; e < nch; e += D) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            if (e + d >= nch) break;
            back_chunk<F, SLAB_LDS>(x, ring[d], nch - 1 - e - d, running);
            bfetch<F, SLAB_LDS, FLOOD, W>(x, ring[d], at(e + d + D));
        }
    }
}

// One work item = (shot, member) of one request: the member's BP run on the
// shot's syndrome, its convergence record, candidate and contribution to
// the normalised average.  `lds` is the block's dynamic LDS; the slabs and
// posteriors are the block's own.
// One sweep of the layered (check-serial) schedule: the checks one at a
// time in the member's order cord.  The slab holds the check messages r by
// CSR position (position k of a row is always handled by lane (k - row
// start) mod 64, so each lane reads back only what it wrote) and, from byte
// offset E * sizeof(F), the running posteriors L_v, which any lane writes
// and which are therefore read past the L1.  At check c every edge forms
// mu = L_v - r (clamped); the row's smallest and next smallest magnitude,
// the position of the smallest and the sign parity are reduced over the
// wavefront; then r_{c->v} = (1 - 2 s_c) alpha prod sign min over the
// others (the next smallest for the position of the smallest, the clamp
// for a row of one) and L_v = (L_v - r_old) + r_new.  Afterwards every
// decision is refreshed from the clamped L and the residual updated.
// A row of the layered sweep as held in registers: up to kRowRegs edges per
// lane (rows of up to 64 * kRowRegs edges); longer rows take a slower path
// that reloads.
constexpr int kRowRegs = 4;
template <class F>
struct LRow {
    uint32_t c, k0, k1;
    uint32_t v[kRowRegs];
    F r[kRowRegs];
};

template <class F>
__device__ __forceinline__ void layered_load_row(const DevGraph& g, const Ctx<F>& x, const uint32_t* cord,
                                                 uint32_t idx, LRow<F>& row) {
    row.c = uni(cord[idx]);
    row.k0 = uni(g.rp[row.c]);
    row.k1 = uni(g.rp[row.c + 1]);
    // every load is issued, at a clamped position, so that the compiler
    // counts them instead of waiting for all loads at each use
    const uint32_t kmax = g.E ? g.E - 1 : 0;
#pragma unroll
    for (int q = 0; q < kRowRegs; q++) {
        const uint32_t k = min(row.k0 + x.lane + (uint32_t)q * kWave, kmax);
        row.v[q] = g.ri[k];
        row.r[q] = bload<F>(x.slb, k * (uint32_t)sizeof(F), 0);
    }
}

// the smallest and next smallest magnitude, position of the smallest and
// sign parity over the wavefront
template <class F>
__device__ __forceinline__ void row_reduce(F& m1, F& m2, uint32_t& arg, uint32_t& par) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const F om1 = __shfl_xor(m1, off), om2 = __shfl_xor(m2, off);
        const uint32_t oarg = __shfl_xor(arg, off), opar = __shfl_xor(par, off);
        const bool take = om1 < m1 || (om1 == m1 && oarg < arg);
        const F hi1 = m1 < om1 ? om1 : m1, lo2 = m2 < om2 ? m2 : om2;
        m2 = hi1 < lo2 ? hi1 : lo2;
        m1 = take ? om1 : m1;
        arg = take ? oarg : arg;
        par ^= opar;
    }
}

// One sweep of the layered (check-serial) schedule: the checks one at a
// time in the member's order cord.  The slab holds the check messages r by
// CSR position (position k of a row is always handled by lane (k - row
// start) mod 64, so each lane reads back only what it wrote) and, from byte
// offset E * sizeof(F), the running posteriors L_v, which any lane writes
// and which are therefore read past the L1.  At check c every edge forms
// mu = L_v - r (clamped); the row's smallest and next smallest magnitude,
// the position of the smallest and the sign parity are reduced over the
// wavefront; then r_{c->v} = (1 - 2 s_c) alpha prod sign min over the
// others (the next smallest for the position of the smallest, the clamp
// for a row of one) and L_v = (L_v - r_old) + r_new.  The next check's
// columns and messages are loaded while the current one is worked on (no
// other check touches them); its posteriors are not, since the current
// check may update them.  Afterwards every decision is refreshed from the
// clamped L and the residual updated.
template <class F>
__device__ __forceinline__ void layered_sweep(const DevGraph& g, const Ctx<F>& x, const uint32_t* cord,
                                              bool want_post, uint64_t& sat) {
    using P = Prec<F>;
    const uint32_t lane = x.lane;
    constexpr uint32_t fb = sizeof(F);
    const uint32_t oL = g.E * fb;
    const F lim = x.lim, al = x.al;
    if (g.m) {
        LRow<F> cur, nxt;
        layered_load_row<F>(g, x, cord, 0, cur);
        for (uint32_t idx = 0; idx < g.m; idx++) {
            layered_load_row<F>(g, x, cord, idx + 1 < g.m ? idx + 1 : idx, nxt);
            const uint32_t c = cur.c, k0 = cur.k0, k1 = cur.k1;
            const bool sc = ((x.sb[c >> 6] >> (c & 63)) & 1ull) != 0;
            F m1 = lim, m2 = lim;
            uint32_t arg = 0xffffffffu, par = 0;
            if (k1 - k0 <= (uint32_t)(kRowRegs * kWave)) {
                F mraw[kRowRegs];
#pragma unroll
                for (int q = 0; q < kRowRegs; q++) {
                    const uint32_t k = k0 + lane + (uint32_t)q * kWave;
                    mraw[q] = bloadx<F>(x.slb, oL + cur.v[q] * fb, 0) - cur.r[q];
                    if (k < k1) {
                        const F mu = P::clamp(mraw[q], lim);
                        const F aa = fabs(mu);
                        sat |= __ballot(aa >= lim);
                        par ^= mu < F(0) ? 1u : 0u;
                        if (aa < m1) {
                            m2 = m1;
                            m1 = aa;
                            arg = k;
                        } else if (aa < m2) {
                            m2 = aa;
                        }
                    }
                }
                row_reduce<F>(m1, m2, arg, par);
#pragma unroll
                for (int q = 0; q < kRowRegs; q++) {
                    const uint32_t k = k0 + lane + (uint32_t)q * kWave;
                    if (k < k1) {
                        const F mu = P::clamp(mraw[q], lim);
                        const F mag = k == arg ? m2 : m1;
                        const bool neg = ((par ^ (mu < F(0) ? 1u : 0u)) != 0) != sc;
                        const F rn = al * (neg ? -mag : mag);
                        bstore<F>(rn, x.slb, k * fb, 0);
                        bstore<F>(mraw[q] + rn, x.slb, oL + cur.v[q] * fb, 0);
                    }
                }
            } else {
                // a long row: reload in the second pass
                for (uint32_t k = k0 + lane; k < k1; k += kWave) {
                    const uint32_t v = g.ri[k];
                    const F mu = P::clamp(bloadx<F>(x.slb, oL + v * fb, 0) - bload<F>(x.slb, k * fb, 0), lim);
                    const F aa = fabs(mu);
                    sat |= __ballot(aa >= lim);
                    par ^= mu < F(0) ? 1u : 0u;
                    if (aa < m1) {
                        m2 = m1;
                        m1 = aa;
                        arg = k;
                    } else if (aa < m2) {
                        m2 = aa;
                    }
                }
                row_reduce<F>(m1, m2, arg, par);
                for (uint32_t k = k0 + lane; k < k1; k += kWave) {
                    const uint32_t v = g.ri[k];
                    const F mraw = bloadx<F>(x.slb, oL + v * fb, 0) - bload<F>(x.slb, k * fb, 0);
                    const F mu = P::clamp(mraw, lim);
                    const F mag = k == arg ? m2 : m1;
                    const bool neg = ((par ^ (mu < F(0) ? 1u : 0u)) != 0) != sc;
                    const F rn = al * (neg ? -mag : mag);
                    bstore<F>(rn, x.slb, k * fb, 0);
                    bstore<F>(mraw + rn, x.slb, oL + v * fb, 0);
                }
            }
            cur = nxt;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    for (uint32_t v = lane; v < g.n; v += kWave) {
        const uint32_t j0 = g.cp[v], j1 = g.cp[v + 1];
        if (j0 == j1) continue;  // no check: L_v = lambda_v, decision fixed
        const F L = P::clamp(bloadx<F>(x.slb, oL + v * fb, 0), lim);
        sat |= __ballot(fabs(L) >= lim);
        if (want_post) x.post[v] = L;
        const bool enew = L <= F(0);
        const bool eold = (x.eb[v >> 6] >> (v & 63)) & 1ull;
        if (enew != eold) {
            atomicXor(reinterpret_cast<unsigned long long*>(&x.eb[v >> 6]), 1ull << (v & 63));
            for (uint32_t j = j0; j < j1; j++) {
                const uint32_t c = g.ci[j];
                atomicXor(reinterpret_cast<unsigned long long*>(&x.res[c >> 6]), 1ull << (c & 63));
            }
        }
    }
}

// The outputs of a work item whose syndrome is zero, with every lambda > 0:
// the first sweep leaves every message positive, so the decision is e = 0
// and it satisfies s at t = 1.
__device__ __forceinline__ void zero_item(const DevGraph& g, const BpLaunch& a, uint32_t shot, uint32_t mem,
                                          int lane) {
    const uint32_t rec = shot * g.L + mem;
    uint64_t* cmask = a.conv_mask + (size_t)shot * (kMaxT + 1);
    if (a.cand)
        for (uint32_t w = lane; w < g.words_n; w += kWave) a.cand[(size_t)rec * g.words_n + w] = 0;
    if (lane == 0) {
        a.t_conv[rec] = 1;
        if (a.weight) a.weight[rec] = 0.0;
        atomicOr(reinterpret_cast<unsigned long long*>(&cmask[1]), 1ull << mem);
        atomicAdd(&a.iters[shot], 1u);
    }
}

// The outputs of a finished work item (member mem on shot `shot`): its
// convergence record, candidate and weight, saturation mark, and its
// contribution to the normalised average.  eb: its decisions (LDS); post:
// its posteriors of the last sweep, written by any lane of the wavefront.
// DG: the decision bitmap is in global memory, updated by atomics, and is
// read past the L1.
template <class F, bool DG = false>
__device__ __forceinline__ void finish_item(const DevGraph& g, const BpLaunch& a, uint32_t shot, uint32_t mem,
                                            uint32_t conv_t, uint32_t ran, bool stopped, bool saturated,
                                            const uint64_t* eb, const F* post, int lane) {
    auto ebw = [&](uint32_t w) { return DG ? load_mask(&eb[w]) : eb[w]; };
    const uint32_t rec = shot * g.L + mem;
    uint64_t* cmask = a.conv_mask + (size_t)shot * (kMaxT + 1);
    // a run that reached the clamp marks its member in word 0 of the shot's
    // convergence masks (iterations count from 1, so that word is free)
    if (lane == 0) {
        a.t_conv[rec] = (int32_t)conv_t;
        atomicAdd(&a.iters[shot], ran);
        if (saturated) atomicOr(reinterpret_cast<unsigned long long*>(&cmask[0]), 1ull << mem);
    }
    if (a.cand && (conv_t || !a.use_M))
        for (uint32_t w = lane; w < g.words_n; w += kWave) a.cand[(size_t)rec * g.words_n + w] = ebw(w);
    if (a.weight && conv_t) {
        // W(e) = sum_v e_v lambda_v in FP64, ascending v
        double W = 0.0;
        for (uint32_t base = 0; base < g.words_n; base += kWave) {
            const uint32_t w = base + lane;
            uint64_t nzw = __ballot(w < g.words_n && ebw(w) != 0);
            if (lane == 0) {
                while (nzw) {
                    const int bi = __ffsll((long long)nzw) - 1;
                    nzw &= nzw - 1;
                    uint64_t xw = ebw(base + bi);
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
            // ||L||^2 summed in ascending v: each lane squares one value of
            // a block of 64 and the running sum takes them in order (every
            // lane holds the same sum).  post[v] was written by the lane
            // that swept v: read it past the L1.
            double ss = 0.0;
            for (uint32_t base = 0; base < g.n; base += kWave) {
                const uint32_t v = base + lane;
                double sq = 0.0;
                if (v < g.n) {
                    const double xv = (double)__hip_atomic_load(&post[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sq = xv * xv;
                }
                const uint32_t cnt_b = min((uint32_t)kWave, g.n - base);
                for (uint32_t j = 0; j < cnt_b; j++) ss += readlane_f64(sq, (int)j);
            }
            if (uni(ss > 0.0 ? 1u : 0u)) {
                const double scale = kQScale / sqrt(ss);
                int64_t* q = a.qfix + (size_t)shot * g.n;
                for (uint32_t v = lane; v < g.n; v += kWave) {
                    const double xv = (double)__hip_atomic_load(&post[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    atomicAdd(reinterpret_cast<unsigned long long*>(&q[v]), (unsigned long long)llrint(xv * scale));
                }
            }
        }
    }
}

// DG: decisions in global memory (the chunk decision masks and the bitmap
// after the block's posteriors, see bp_post_elems), not in LDS.
template <class F, bool SLAB_LDS, bool FLOOD, bool LAYERED = false, bool DG = false, int D = kDepth>
__device__ __forceinline__ void run_item(const DevGraph& g, const BpLaunch& a, uint32_t item, unsigned char* lds,
                                         Ctx<F> x) {
    using P = Prec<F>;
    using B = typename P::B;
    static_assert(!DG || (!SLAB_LDS && !LAYERED), "decisions in global memory: chunked sweeps, global slab");
    uint64_t* sb = reinterpret_cast<uint64_t*>(lds);
    uint64_t* res = sb + g.words_m;
    uint64_t* eb = res + g.words_m;
    B* pref = reinterpret_cast<B*>(DG ? eb : eb + g.words_n);
    if constexpr (DG) {
        F* aux = x.post + bp_post_head(g);
        x.dsl = make_rsrc(aux, g.max_chunks * 8u);
        eb = reinterpret_cast<uint64_t*>(aux) + g.max_chunks;
    }
    // LDS variant: the state slab, then (parallel schedule) the message slab;
    // the global slabs are buffer resources set up by the caller
    B* slab = SLAB_LDS ? pref + g.m : nullptr;
    B* mslab = SLAB_LDS && FLOOD ? slab + (size_t)g.max_chunks * kWave : nullptr;
    const int lane = x.lane;
    F* post = x.post;
    const F* lamv = reinterpret_cast<const F*>(g.lam);
    const B ident = P::ident(g);
    constexpr bool kF64 = sizeof(F) == 8;
    x.lslab = slab;
    x.lmslab = mslab;
    x.pref = pref;
    x.sb = sb;
    x.res = res;
    x.eb = eb;
    x.trash = post + g.n;
    x.al = (F)g.alpha;
    x.lim = (F)g.clamp;

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
        return;
    }
    if (!any && a.fast_zero && g.all_lam_positive) {
        zero_item(g, a, shot, mem, lane);
        return;
    }
    for (uint32_t w = lane; w < g.words_n; w += kWave) eb[w] = g.e0[w];

    // The slab is only ever re-read by the lane that wrote it: a slot's
    // position is (chunk * 64 + lane) in the sweep and in the backward
    // pass alike.  The first sweep reads the suffix states of the initial
    // messages from the graph itself.
    const uint32_t c0 = uni(g.member_chunk[mem]), nch = uni(g.member_chunk[mem + 1]) - c0;
    const unsigned char* recs = g.sched + (size_t)c0 * rec_bytes(kF64);
    x.sch = make_rsrc(recs, nch * rec_bytes(kF64));
    F* post_out = a.post_out ? reinterpret_cast<F*>(a.post_out) + (size_t)rec * g.n : nullptr;
    if constexpr (LAYERED) {
        // check messages 0, each position stored by the lane that will use
        // it; posteriors lambda (clamped)
        for (uint32_t c = 0; c < g.m; c++) {
            const uint32_t k0 = uni(g.rp[c]), k1 = uni(g.rp[c + 1]);
            for (uint32_t k = k0 + lane; k < k1; k += kWave) bstore<F>(F(0), x.slb, k * (uint32_t)sizeof(F), 0);
        }
        for (uint32_t v = lane; v < g.n; v += kWave)
            bstore<F>(P::clamp(lamv[v], x.lim), x.slb, (g.E + v) * (uint32_t)sizeof(F), 0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (SLAB_LDS) {
        // the first sweep reads the initial suffix states from the slab
        for (uint32_t q = 0; q < nch; q++)
            slab[q * kWave + lane] = *reinterpret_cast<const B*>(recs + (size_t)q * rec_bytes(kF64) +
                                                                 rec_init(kF64) + (size_t)lane * sizeof(B));
    }

    uint32_t conv_t = 0, ran = 0;
    bool stopped = false;
    uint64_t sat = 0;  // lanes that saw a posterior or message reach the clamp (saturation witness)
    for (uint32_t t = 1; t <= a.T_run; t++) {
        if (a.use_M && t >= 2 && preceding_converged(cmask, t, mem, lane) >= g.M) {
            stopped = true;  // cannot be among the first M any more
            break;
        }
        if (g.alpha_t) x.al = (F)g.alpha_t[t - 1];  // one scaling factor per iteration
        const bool want_post = post_out != nullptr || (a.accumulate_q && t == a.T_run);
        if (want_post) {
            // columns without checks keep L_v = lambda_v
            for (uint32_t v = lane; v < g.n; v += kWave) post[v] = lamv[v];
        }
        for (uint32_t c = lane; c < g.m; c += kWave) pref[c] = ident;
        __syncthreads();
        if constexpr (LAYERED) {
            layered_sweep<F>(g, x, g.cperm + (size_t)mem * g.m, want_post, sat);
        } else if (nch) {
            if (want_post)
                sweep<F, SLAB_LDS, true, FLOOD, kWave, DG, D>(x, nch, t == 1, sat);
            else
                sweep<F, SLAB_LDS, false, FLOOD, kWave, DG, D>(x, nch, t == 1, sat);
        }
        __syncthreads();  // every new message stored
        if (post_out) {
            // post[v] was written by the lane that swept v: read it past the L1
            for (uint32_t v = lane; v < g.n; v += kWave)
                post_out[v] = __hip_atomic_load(&post[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ran = t;
        // converged iff the residual s + H e is zero
        bool nz = false;
        for (uint32_t w = lane; w < g.words_m; w += kWave) nz |= res[w] != 0;
        if (__ballot(nz) == 0) {
            if (!conv_t) conv_t = t;
            if (a.stop_on_converge) break;
        }
        if (!LAYERED && t < a.T_run && nch) {
            for (uint32_t c = lane; c < g.m; c += kWave) pref[c] = ident;
            __syncthreads();
            backward<F, SLAB_LDS, FLOOD, kWave, D>(x, nch, pref);
            __syncthreads();
        }
    }

    finish_item<F, DG>(g, a, shot, mem, conv_t, ran, stopped, uni(sat != 0 ? 1u : 0u) != 0, eb, post, lane);
}

// One work item of the multi-shot launch: member mem on the P shots
// grp * P .. grp * P + P - 1 (those below n_shots) side by side, on the
// member's schedule recut into chunks of W = 64 / P edges.  Lanes
// p * W .. p * W + W - 1 run shot p: every lane does what it does for one
// shot, on its shot's row states, decisions and posteriors (LDS, shot p's
// copy), so a column's edges are still consecutive lanes.  Each shot
// finishes on its own (converged, or out of the first M): its outputs are
// written then, and its lanes go on with work that is never read.  The
// item ends when every shot has finished.  Global slab, serial schedule,
// stop on convergence (so a shot's convergence iteration is the iteration
// it finishes at, and its iterations run are those before it finishes).
template <class F, int P, bool DG = false>
__device__ __forceinline__ void run_group(const DevGraph& g, const BpLaunch& a, uint32_t item, unsigned char* lds,
                                          Ctx<F> x) {
    using PR = Prec<F>;
    using B = typename PR::B;
    constexpr uint32_t W = kWave / P;
    constexpr uint32_t kAll = (1u << P) - 1u;
    const int lane = x.lane;
    const uint32_t p = (uint32_t)lane / W;
    uint64_t* sb0 = reinterpret_cast<uint64_t*>(lds);
    uint64_t* res0 = sb0 + P * g.words_m;
    uint64_t* eb0 = res0 + P * g.words_m;
    B* pref0 = reinterpret_cast<B*>(DG ? eb0 : eb0 + P * g.words_n);
    F* post0 = x.post;  // P x n posteriors, then 64 trash slots
    if constexpr (DG) {  // chunk decision masks, then P decision bitmaps
        F* aux = post0 + bp_post_head(g);
        x.dsl = make_rsrc(aux, g.max_chunks * 8u);
        eb0 = reinterpret_cast<uint64_t*>(aux) + g.max_chunks;
    }
    const F* lamv = reinterpret_cast<const F*>(g.lam);
    const B ident = PR::ident(g);
    x.lslab = nullptr;
    x.lmslab = nullptr;
    x.sb = sb0 + p * g.words_m;
    x.res = res0 + p * g.words_m;
    x.eb = eb0 + p * g.words_n;
    x.pref = pref0 + p * g.m;
    x.post = post0 + p * g.n;
    x.trash = post0 + P * g.n;
    x.rec4 = ((uint32_t)lane % W) * 4u;
    x.recF = ((uint32_t)lane % W) * (uint32_t)sizeof(F);
    x.al = (F)g.alpha;
    x.lim = (F)g.clamp;

    const uint32_t groups = (a.n_shots + P - 1) / P;
    uint32_t grp, mem;
    if (a.member_major) {
        mem = item / groups;
        grp = item % groups;
    } else {
        grp = item / g.L;
        mem = item % g.L;
    }
    const uint32_t first = grp * P;
    const uint32_t nact = uni(min((uint32_t)P, a.n_shots - first));  // shots present (>= 1)

    // ---- syndrome bits of each shot; absent shots read shot `first`'s
    // bytes and count as finished
    uint32_t done = 0, nonzero = 0;
#pragma unroll
    for (int q = 0; q < P; q++) {
        const bool act = (uint32_t)q < nact;
        const uint8_t* s = a.syndromes + (size_t)(a.shot0 + first + (act ? (uint32_t)q : 0u)) * g.m;
        uint64_t any = 0;
        for (uint32_t base = 0; base < g.m; base += kWave) {
            const uint32_t c = base + lane;
            const uint64_t mask = __ballot(act && c < g.m && s[c] != 0);
            if (lane == 0) {
                sb0[q * g.words_m + base / kWave] = mask;
                res0[q * g.words_m + base / kWave] = mask;
            }
            any |= mask;
        }
        if (!act) {
            done |= 1u << q;
        } else {
            uint64_t* cm = a.conv_mask + (size_t)(first + q) * (kMaxT + 1);
            if (a.use_M && preceding_converged(cm, 1, mem, lane) >= g.M) {
                // M members of lower index converged at the first iteration
                if (lane == 0) a.t_conv[(first + q) * g.L + mem] = 0;
                done |= 1u << q;
            } else if (!any && a.fast_zero && g.all_lam_positive) {
                zero_item(g, a, first + q, mem, lane);
                done |= 1u << q;
            }
        }
    }
    done = uni(done);
    if (done == kAll) return;
    for (uint32_t w = lane; w < P * g.words_n; w += kWave) eb0[w] = g.e0[w % g.words_n];

    const uint32_t c0 = uni(g.member_chunk[mem]), nch = uni(g.member_chunk[mem + 1]) - c0;
    x.sch = make_rsrc(g.sched + (size_t)c0 * RecW<F, W>::kBytes, nch * RecW<F, W>::kBytes);

    uint64_t sat = 0;  // lanes that saw a posterior or message reach the clamp
    auto sat_of = [&](int q) {
        const uint64_t mask = ((W == kWave ? ~0ull : (1ull << W) - 1ull)) << (q * W);
        return uni((sat & mask) != 0 ? 1u : 0u) != 0;
    };
    for (uint32_t t = 1; t <= a.T_run; t++) {
        if (a.use_M && t >= 2) {
#pragma unroll
            for (int q = 0; q < P; q++) {
                if ((done >> q) & 1u) continue;
                uint64_t* cm = a.conv_mask + (size_t)(first + q) * (kMaxT + 1);
                if (preceding_converged(cm, t, mem, lane) >= g.M) {
                    // cannot be among the first M any more
                    finish_item<F, DG>(g, a, first + q, mem, 0u, t - 1, true, sat_of(q), eb0 + q * g.words_n,
                                   post0 + q * g.n, lane);
                    done |= 1u << q;
                }
            }
            done = uni(done);
            if (done == kAll) return;
        }
        if (g.alpha_t) x.al = (F)g.alpha_t[t - 1];
        const bool want_post = a.accumulate_q && t == a.T_run;
        if (want_post)  // columns without checks keep L_v = lambda_v
            for (uint32_t i = lane; i < P * g.n; i += kWave) post0[i] = lamv[i % g.n];
        for (uint32_t i = lane; i < P * g.m; i += kWave) pref0[i] = ident;
        __syncthreads();
        if (nch) {
            if (want_post)
                sweep<F, false, true, false, W, DG>(x, nch, t == 1, sat);
            else
                sweep<F, false, false, false, W, DG>(x, nch, t == 1, sat);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; q++) {
            if ((done >> q) & 1u) continue;
            // converged iff the shot's residual s + H e is zero
            bool nz = false;
            for (uint32_t w = lane; w < g.words_m; w += kWave) nz |= res0[q * g.words_m + w] != 0;
            if (__ballot(nz) == 0) {
                finish_item<F, DG>(g, a, first + q, mem, t, t, false, sat_of(q), eb0 + q * g.words_n,
                               post0 + q * g.n, lane);
                done |= 1u << q;
            }
        }
        done = uni(done);
        if (done == kAll) return;
        if (t < a.T_run && nch) {
            for (uint32_t i = lane; i < P * g.m; i += kWave) pref0[i] = ident;
            __syncthreads();
            backward<F, false, false, W>(x, nch, x.pref);
            __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < P; q++) {
        if ((done >> q) & 1u) continue;
        finish_item<F, DG>(g, a, first + q, mem, 0u, a.T_run, false, sat_of(q), eb0 + q * g.words_n,
                       post0 + q * g.n, lane);
    }
}

// Pass context fields that depend only on the block: lane offsets, the
// block's global slabs and posterior area.
template <class F>
__device__ __forceinline__ Ctx<F> block_ctx(typename Prec<F>::B* gslab, typename Prec<F>::B* gmslab,
                                           uint32_t slab_elems, F* post) {
    using B = typename Prec<F>::B;
    Ctx<F> x;
    x.slb = make_rsrc(gslab, slab_elems * (uint32_t)sizeof(B));
    x.mslb = make_rsrc(gmslab, slab_elems * (uint32_t)sizeof(B));
    x.post = post;
    x.lane = threadIdx.x;
    x.lane4 = (uint32_t)threadIdx.x * 4u;
    x.laneF = (uint32_t)threadIdx.x * (uint32_t)sizeof(F);
    return x;
}

// A read-only struct copied into registers through the constant address
// space (scalar loads), one dword at a time.
template <class T>
__device__ __forceinline__ T load_const(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized struct");
    T v;
    const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)p;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; i++) dst[i] = src[i];
    return v;
}

// One launch over the items of one request.  DG: decisions in global
// memory; D: chunks loaded ahead (kLatDepth: the latency variant).
template <class F, bool SLAB_LDS, bool FLOOD, bool LAYERED = false, bool DG = false, int D = kDepth>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(D > kDepth ? 4 : waves_target<F, SLAB_LDS, FLOOD, false, false, DG>()))) void bp_ensemble_kernel(DevGraph g, BpLaunch a) {
    using B = typename Prec<F>::B;
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t slab_elems = g.max_chunks * kWave;
    B* gslab = a.slab ? reinterpret_cast<B*>(a.slab) + (size_t)blockIdx.x * slab_elems : nullptr;
    B* gmslab = FLOOD && a.slab ? reinterpret_cast<B*>(a.slab) + ((size_t)gridDim.x + blockIdx.x) * slab_elems : nullptr;
    F* post = reinterpret_cast<F*>(a.post_slab) + (size_t)blockIdx.x * bp_post_elems(g);
    const Ctx<F> x = block_ctx<F>(gslab, gmslab, slab_elems, post);
    const uint32_t n_items = a.n_shots * g.L;
    for (;;) {
        const uint32_t item = wave_ticket(a.counter, 1u);
        if (item >= n_items) break;
        run_item<F, SLAB_LDS, FLOOD, LAYERED, DG, D>(g, a, item, lds, x);
        __syncthreads();
    }
}

// One persistent launch over the items of several requests, on different
// graphs (ragged batching).  Items are numbered request after request;
// segs[j].item0 is request j's first.  Every block owns slabs and
// posteriors sized for the largest graph.  The segment table is read-only
// for the launch and read through the constant address space, so its
// fields load as wave-uniform scalars.  WITH_LAYERED: some segment may be
// on the layered schedule (the variant without that item body needs fewer
// registers).  DG: the other segments keep decisions in global memory.
template <class F, bool SLAB_LDS, bool FLOOD, bool WITH_LAYERED, bool DG = false, int D = kDepth>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(D > kDepth ? 4 : waves_target<F, SLAB_LDS, FLOOD, true, WITH_LAYERED, DG>()))) void bp_ragged_kernel(RaggedLaunch r) {
    using B = typename Prec<F>::B;
    using CSeg = const __attribute__((address_space(4))) BpSeg;
    extern __shared__ __align__(16) unsigned char lds[];
    CSeg* segs = (CSeg*)r.segs;
    B* gslab = r.slab ? reinterpret_cast<B*>(r.slab) + (size_t)blockIdx.x * r.slab_elems : nullptr;
    B* gmslab = FLOOD && r.slab ? reinterpret_cast<B*>(r.slab) + ((size_t)gridDim.x + blockIdx.x) * r.slab_elems : nullptr;
    F* post = reinterpret_cast<F*>(r.post_slab) + (size_t)blockIdx.x * r.post_elems;
    const Ctx<F> x = block_ctx<F>(gslab, gmslab, r.slab_elems, post);
    for (;;) {
        const uint32_t item = wave_ticket(r.counter, 1u);
        if (item >= r.n_items) break;
        uint32_t j = 0;
        while (j + 1 < r.n_segs && segs[j + 1].item0 <= item) j++;
        const DevGraph g = load_const(&r.segs[j].g);
        const BpLaunch a = load_const(&r.segs[j].a);
        // one launch may mix schedules: parallel items need the launch's
        // second slab, serial ones use the first only, and layered ones
        // (global slabs only) keep messages and posteriors in the first
        if constexpr (!SLAB_LDS && WITH_LAYERED) {
            if (g.layered) {
                run_item<F, false, false, true>(g, a, item - segs[j].item0, lds, x);
                __syncthreads();
                continue;
            }
        }
        if constexpr (FLOOD) {
            if (g.flood)
                run_item<F, SLAB_LDS, true, false, DG>(g, a, item - segs[j].item0, lds, x);
            else
                run_item<F, SLAB_LDS, false, false, DG>(g, a, item - segs[j].item0, lds, x);
        } else {
            run_item<F, SLAB_LDS, false, false, DG, D>(g, a, item - segs[j].item0, lds, x);
        }
        __syncthreads();
    }
}

// One launch over the items of one request, P = 2 or 4 shots per
// wavefront (serial schedule, slab in global memory).
// occupancy the register allocator aims for with P shots per wavefront
// (waves per SIMD): the FP32 variants fit it without spills, the FP64 ones
// spill a few registers
template <class F, int P>
constexpr int multi_waves_target() {
    return sizeof(F) == 8 || P == 4 ? 4 : 5;
}

template <class F, int P, bool DG>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(multi_waves_target<F, P>()))) void bp_multi_kernel(DevGraph g, BpLaunch a) {
    using B = typename Prec<F>::B;
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t slab_elems = g.max_chunks * kWave;
    B* gslab = reinterpret_cast<B*>(a.slab) + (size_t)blockIdx.x * slab_elems;
    F* post = reinterpret_cast<F*>(a.post_slab) + (size_t)blockIdx.x * bp_post_elems(g);
    const Ctx<F> x = block_ctx<F>(gslab, nullptr, slab_elems, post);
    const uint32_t n_items = (a.n_shots + P - 1) / P * g.L;
    for (;;) {
        const uint32_t item = wave_ticket(a.counter, 1u);
        if (item >= n_items) break;
        run_group<F, P, DG>(g, a, item, lds, x);
        __syncthreads();
    }
}

// The ragged launch when some request runs several shots per wavefront:
// every segment on the serial or layered schedule, slabs in global memory;
// each segment's items follow its own shots per wavefront.  DG: the
// serial segments keep decisions in global memory.
template <class F, bool DG>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4))) void bp_ragged_multi_kernel(RaggedLaunch r) {
    using B = typename Prec<F>::B;
    using CSeg = const __attribute__((address_space(4))) BpSeg;
    extern __shared__ __align__(16) unsigned char lds[];
    CSeg* segs = (CSeg*)r.segs;
    B* gslab = reinterpret_cast<B*>(r.slab) + (size_t)blockIdx.x * r.slab_elems;
    F* post = reinterpret_cast<F*>(r.post_slab) + (size_t)blockIdx.x * r.post_elems;
    const Ctx<F> x = block_ctx<F>(gslab, nullptr, r.slab_elems, post);
    for (;;) {
        const uint32_t item = wave_ticket(r.counter, 1u);
        if (item >= r.n_items) break;
        uint32_t j = 0;
        while (j + 1 < r.n_segs && segs[j + 1].item0 <= item) j++;
        const DevGraph g = load_const(&r.segs[j].g);
        const BpLaunch a = load_const(&r.segs[j].a);
        const uint32_t it = item - segs[j].item0;
        if (g.layered)
            run_item<F, false, false, true>(g, a, it, lds, x);
        else if (g.P == 2)
            run_group<F, 2, DG>(g, a, it, lds, x);
        else if (g.P == 4)
            run_group<F, 4, DG>(g, a, it, lds, x);
        else
            run_item<F, false, false, false, DG>(g, a, it, lds, x);
        __syncthreads();
    }
}

__global__ void zero_kernel(uint32_t* p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <class F, bool FLOOD>
const void* kernel_for_t(bool slab_in_lds, bool ragged, bool layered, bool dg) {
    if (ragged) {  // layered segments run with global slabs only
        if (slab_in_lds) return (const void*)bp_ragged_kernel<F, true, FLOOD, false>;
        if (layered) return (const void*)bp_ragged_kernel<F, false, FLOOD, true>;
        return dg ? (const void*)bp_ragged_kernel<F, false, FLOOD, false, true>
                  : (const void*)bp_ragged_kernel<F, false, FLOOD, false>;
    }
    if (slab_in_lds) return (const void*)bp_ensemble_kernel<F, true, FLOOD>;
    return dg ? (const void*)bp_ensemble_kernel<F, false, FLOOD, false, true>
              : (const void*)bp_ensemble_kernel<F, false, FLOOD>;
}

template <class F, bool DG>
const void* multi_kernel_for(bool ragged, uint32_t P) {
    if (ragged) return (const void*)bp_ragged_multi_kernel<F, DG>;
    return P == 2 ? (const void*)bp_multi_kernel<F, 2, DG> : (const void*)bp_multi_kernel<F, 4, DG>;
}

// ragged: layered = some segment is layered, P > 1 = some segment runs
// several shots per wavefront; dg: decisions in global memory (the
// non-layered items; the slab in global memory)
const void* kernel_for(bool fp64, bool flood, bool slab_in_lds, bool ragged, bool layered = false, uint32_t P = 1,
                       bool dg = false, bool latency = false) {
    // the latency variant: FP32, serial schedule, global slab, one shot per
    // wavefront, decisions in LDS
    if (latency && !fp64 && !flood && !slab_in_lds && !layered && P == 1 && !dg)
        return ragged ? (const void*)bp_ragged_kernel<float, false, false, false, false, kLatDepth>
                      : (const void*)bp_ensemble_kernel<float, false, false, false, false, kLatDepth>;
    // several shots per wavefront: serial schedule, slab in global memory
    if (P > 1) {
        if (fp64) return dg ? multi_kernel_for<double, true>(ragged, P) : multi_kernel_for<double, false>(ragged, P);
        return dg ? multi_kernel_for<float, true>(ragged, P) : multi_kernel_for<float, false>(ragged, P);
    }
    // the layered schedule: one request at a time, slab in global memory
    if (layered && !ragged) return fp64 ? (const void*)bp_ensemble_kernel<double, false, false, true>
                                        : (const void*)bp_ensemble_kernel<float, false, false, true>;
    if (fp64)
        return flood ? kernel_for_t<double, true>(slab_in_lds, ragged, layered, dg)
                     : kernel_for_t<double, false>(slab_in_lds, ragged, layered, dg);
    return flood ? kernel_for_t<float, true>(slab_in_lds, ragged, layered, dg)
                 : kernel_for_t<float, false>(slab_in_lds, ragged, layered, dg);
}

int launch_fn(const void* fn, int grid, size_t lds, void** args, hipStream_t st) {
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(bp)");
    }
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, lds, st);
    if (e != hipSuccess) return hip_fail(e, "bp kernel launch");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bp kernel launch");
    return VIBE_OK;
}

}  // namespace

int bp_slabs(const DevGraph& g) { return g.flood ? 2 : 1; }

size_t bp_lds_bytes(const DevGraph& g, bool slab_in_lds) {
    const size_t mb = g.fp64 ? 8 : 4;
    // per shot of the wavefront: syndrome, residual, decisions (unless in
    // global memory: never with the slab in LDS), row states
    const bool dec_lds = slab_in_lds || !g.dec_global;
    const size_t words = 2 * (size_t)g.words_m + (dec_lds ? g.words_n : 0);
    size_t b = (size_t)g.P * (sizeof(uint64_t) * words + mb * g.m);
    if (slab_in_lds) b += bp_slabs(g) * mb * (size_t)g.max_chunks * kWave;
    return b;
}



bool bp_slab_fits_lds(const DevGraph& g) { return !g.layered && g.P == 1 && bp_lds_bytes(g, true) <= 96 * 1024; }

int bp_grid_for(bool fp64, bool flood, bool slab_in_lds, size_t lds_bytes, bool ragged, bool layered, uint32_t P,
                bool dec_global, bool latency) {
    // resident blocks of a kernel variant at an LDS size, per device: an
    // occupancy query per launch plan is cheap but not free, so the answers
    // are kept (a few variants and sizes per graph)
    static std::mutex mu;
    static std::map<std::tuple<int, const void*, size_t>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const void* fn = kernel_for(fp64, flood, slab_in_lds, ragged, layered, P, dec_global, latency);
    const auto key = std::make_tuple(dev, fn, lds_bytes);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWave, lds_bytes);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    if (per_cu > 32) per_cu = 32;
    const int grid = per_cu * prop.multiProcessorCount;
    cache[key] = grid;
    return grid;
}

bool use_lds_slab(const vibe_graph* G, const DevGraph& g) {
    if (G->tune_lds == 0 || !bp_slab_fits_lds(g)) return false;
    if (G->tune_lds > 0) return true;
    DevGraph d = g;
    d.dec_global = 0;
    return bp_grid(d, true) >= bp_grid(d, false);
}

bool dec_global_pays(const DevGraph& g) {
    if (g.layered) return false;
    DevGraph a = g, b = g;
    a.dec_global = 0;
    b.dec_global = 1;
    // the LDS slab variant keeps decisions in LDS: compare global slabs
    return bp_grid(b, false) > bp_grid(a, false);
}

int bp_grid(const DevGraph& g, bool slab_in_lds) {
    return bp_grid_for(g.fp64 != 0, g.flood != 0, slab_in_lds, bp_lds_bytes(g, slab_in_lds), false, g.layered != 0,
                       g.P, g.dec_global != 0);
}

int bp_latency_grid(const DevGraph& g, bool slab_in_lds) {
    if (g.fp64 || g.flood || g.layered || slab_in_lds || g.P != 1 || g.dec_global) return 0;
    return bp_grid_for(false, false, false, bp_lds_bytes(g, false), false, false, 1, false, true);
}

int launch_bp(const DevGraph& g, const BpLaunch& a, hipStream_t st) {
    const bool in_lds = a.slab_in_lds != 0;
    void* args[] = {const_cast<DevGraph*>(&g), const_cast<BpLaunch*>(&a)};
    if (g.P > 1 && (g.flood || g.layered || in_lds || a.post_out || !a.stop_on_converge))
        return fail(VIBE_EINVAL, "internal: several shots per wavefront need the serial schedule, a global slab "
                                 "and stop on convergence");
    if (g.dec_global && (g.layered || in_lds))
        return fail(VIBE_EINVAL, "internal: decisions in global memory need a chunked schedule and a global slab");
    if (a.latency && !bp_latency_grid(g, in_lds))
        return fail(VIBE_EINVAL, "internal: the latency variant needs FP32, the serial schedule, a global slab, "
                                 "one shot per wavefront and decisions in LDS");
    return launch_fn(kernel_for(g.fp64 != 0, g.flood != 0, in_lds, false, g.layered != 0, g.P, g.dec_global != 0,
                                a.latency != 0),
                     a.grid, bp_lds_bytes(g, in_lds), args, st);
}

int launch_bp_ragged(const RaggedLaunch& r, hipStream_t st) {
    void* args[] = {const_cast<RaggedLaunch*>(&r)};
    if (r.multi && (r.flood || r.slab_in_lds))
        return fail(VIBE_EINVAL, "internal: several shots per wavefront need the serial schedule and a global slab");
    if (r.dec_global && (r.slab_in_lds || (r.layered && !r.multi)))
        return fail(VIBE_EINVAL, "internal: decisions in global memory need global slabs (and no layered segment "
                                 "outside the multi-shot launch)");
    if (r.latency && (r.fp64 || r.flood || r.slab_in_lds || r.layered || r.multi || r.dec_global))
        return fail(VIBE_EINVAL, "internal: the latency variant needs FP32, the serial schedule, global slabs, "
                                 "one shot per wavefront and decisions in LDS");
    return launch_fn(kernel_for(r.fp64 != 0, r.flood != 0, r.slab_in_lds != 0, true, r.layered != 0,
                                r.multi ? 2u : 1u, r.dec_global != 0, r.latency != 0),
                     r.grid, r.lds_bytes, args, st);
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
