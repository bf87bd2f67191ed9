// Online stage (paper Sec. III.D.2): launch sequences of the C ABI.
//
// Batched decode, per chunk of shots: K1 (BP ensemble, persistent grid, one
// wavefront per (shot, member), correction limit applied on the fly, the
// normalised posteriors of unconverged members accumulated in fixed point),
// K2 (selection by prior weight; shots with no converged member are queued),
// K3 (LSD-0 on the queued shots); then K4 (observables) over the whole batch.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace vibe {

namespace {

struct ChunkBufs {
    int32_t* t_conv;
    double* weight;
    uint64_t* cand;
    uint64_t* cmask;     // per shot: members converged at each iteration
    uint32_t* iters;
    int64_t* qfix;
    uint32_t* fail_list;
    uint32_t* counters;  // [0] BP work counter, [1] failed-shot count
    void* slab;
    void* post_slab;
    void* lsd_scratch;
};

inline size_t msg_bytes(const DevGraph& g) { return g.fp64 ? 8 : 4; }

size_t per_shot_bytes(const DevGraph& g, bool decode) {
    size_t b = 4ull * g.L + 8ull * (kMaxT + 1) + 4 + 4;
    if (decode) b += 8ull * g.L + 8ull * g.L * g.words_n + 8ull * g.n;
    return b;
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int ensure_workspace(vibe_graph* G, size_t bytes) {
    if (G->ws.bytes >= bytes) return VIBE_OK;
    if (G->ws.base) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before growing the workspace");
        (void)hipFree(G->ws.base);
        G->ws.base = nullptr;
        G->ws.bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(VIBE_ENOMEM, "workspace allocation failed");
    G->ws.base = p;
    G->ws.bytes = bytes;
    return VIBE_OK;
}

// Sizes of the per-chunk buffers for chunks of up to `bc` shots.
// slab_blocks: blocks that need a message slab in global memory (0 when the
// slab lives in LDS); post_blocks: blocks of the BP grid (posterior slabs).
constexpr int kBufs = 11;
size_t carve_sizes(const DevGraph& g, uint32_t bc, bool decode, int slab_blocks, int post_blocks, int lsd_grid,
                   size_t* sizes) {
    const size_t s[kBufs] = {
        4ull * bc * g.L,                                   // t_conv
        decode ? 8ull * bc * g.L : 0,                      // weight
        decode ? 8ull * bc * g.L * g.words_n : 0,          // cand
        8ull * bc * (kMaxT + 1),                           // convergence masks
        4ull * bc,                                         // iters
        decode ? 8ull * bc * g.n : 0,                      // qfix
        4ull * bc,                                         // fail_list
        64,                                                // counters
        msg_bytes(g) * bp_slabs(g) * slab_blocks * std::max<size_t>((size_t)g.max_chunks * kWave, 1),  // slabs
        msg_bytes(g) * post_blocks * bp_post_elems(g),     // posterior slabs
        decode ? lsd_scratch_per_block(g) * lsd_grid : 0,  // LSD scratch
    };
    size_t total = 0;
    for (int i = 0; i < kBufs; i++) {
        sizes[i] = s[i];
        total += al256(s[i]);
    }
    return total;
}

// Point the buffers of B into memory at `base` (256-byte aligned) laid out
// by carve_sizes.
void carve_at(unsigned char* p, const size_t* sizes, ChunkBufs* B) {
    void* ptrs[kBufs];
    for (int i = 0; i < kBufs; i++) {
        ptrs[i] = sizes[i] ? p : nullptr;
        p += al256(sizes[i]);
    }
    B->t_conv = (int32_t*)ptrs[0];
    B->weight = (double*)ptrs[1];
    B->cand = (uint64_t*)ptrs[2];
    B->cmask = (uint64_t*)ptrs[3];
    B->iters = (uint32_t*)ptrs[4];
    B->qfix = (int64_t*)ptrs[5];
    B->fail_list = (uint32_t*)ptrs[6];
    B->counters = (uint32_t*)ptrs[7];
    B->slab = ptrs[8];
    B->post_slab = ptrs[9];
    B->lsd_scratch = ptrs[10];
}

// Carve the handle's workspace (grown on demand) for chunks of up to `bc`
// shots.
int carve(const DevGraph& g, vibe_graph* G, uint32_t bc, bool decode, int slab_blocks, int post_blocks,
          int lsd_grid, ChunkBufs* B) {
    size_t sizes[kBufs];
    const size_t total = carve_sizes(g, bc, decode, slab_blocks, post_blocks, lsd_grid, sizes);
    int rc = ensure_workspace(G, total);
    if (rc) return rc;
    carve_at(static_cast<unsigned char*>(G->ws.base), sizes, B);
    return VIBE_OK;
}

int lsd_grid_for(uint64_t B) {
    uint64_t g = std::min<uint64_t>(B ? B : 1, 512);
    return (int)g;
}

int memset_async(void* p, size_t bytes, hipStream_t st) { return launch_zero(p, bytes, st); }

// One chunk of the decoder: shots [shot0, shot0 + n), on g (the handle's
// graph, or its view with a recut schedule).
int decode_chunk(vibe_graph* G, const DevGraph& g, const ChunkBufs& W, const uint8_t* synd, uint64_t shot0,
                 uint32_t n, uint64_t* corr, vibe_shot_stats* stats, int bp_blocks, int lsd_grid, hipStream_t st,
                 bool in_lds, bool timed = true) {
    int rc;
    if ((rc = memset_async(W.cmask, 8ull * n * (kMaxT + 1), st)) ||
        (rc = memset_async(W.iters, 4ull * n, st)) || (rc = memset_async(W.qfix, 8ull * n * g.n, st)) ||
        (rc = memset_async(W.counters, 64, st)))
        return rc;
    BpLaunch b{};
    b.member_major = 1;
    b.slab_in_lds = in_lds ? 1 : 0;
    b.syndromes = synd;
    b.shot0 = shot0;
    b.n_shots = n;
    b.T_run = g.T;
    b.use_M = 1;
    b.stop_on_converge = 1;
    b.accumulate_q = 1;
    b.fast_zero = 1;
    b.t_conv = W.t_conv;
    b.weight = W.weight;
    b.cand = W.cand;
    b.post_out = nullptr;
    b.conv_mask = W.cmask;
    b.iters = W.iters;
    b.qfix = W.qfix;
    b.slab = W.slab;
    b.post_slab = W.post_slab;
    b.counter = W.counters;
    const uint64_t items = bp_items(g, n);
    b.grid = (int)std::min<uint64_t>((uint64_t)bp_blocks, items);
    // every item resident at once: the deeper prefetch ring pays
    b.latency = items <= (uint64_t)std::min(bp_blocks, bp_latency_grid(g, in_lds)) ? 1 : 0;
    if (timed) begin_timed(G, 0, st);
    if ((rc = launch_bp(g, b, st))) return rc;
    if (timed) end_timed(G, 0, st);
    SelectLaunch s{};
    s.n_shots = n;
    s.shot0 = shot0;
    s.t_conv = W.t_conv;
    s.weight = W.weight;
    s.cand = W.cand;
    s.iters = W.iters;
    s.conv_mask = W.cmask;
    s.corrections = corr;
    s.stats = stats;
    s.fail_list = W.fail_list;
    s.fail_count = W.counters + 1;
    if (timed) begin_timed(G, 1, st);
    if ((rc = launch_select(g, s, st))) return rc;
    if (timed) end_timed(G, 1, st);
    LsdLaunch l{};
    l.syndromes = synd;
    l.shot0 = shot0;
    l.list = W.fail_list;
    l.list_count = W.counters + 1;
    l.n_list = n;
    l.soft_f32 = nullptr;
    l.soft_fix = W.qfix;
    l.corrections = corr;
    l.stats = stats;
    l.scratch = W.lsd_scratch;
    l.scratch_per_block = lsd_scratch_per_block(g);
    l.grid = std::min(lsd_grid, (int)n);
    if (timed) begin_timed(G, 2, st);
    if ((rc = launch_lsd(g, l, st))) return rc;
    if (timed) end_timed(G, 2, st);
    return VIBE_OK;
}

// Bit-packed syndromes (B x words_m uint64, check c in bit c % 64 of word
// c / 64) to one byte per check, for shots [0, n).
__global__ void unpack_kernel(const uint64_t* words, uint32_t wm, uint32_t m, uint64_t n, uint8_t* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * m) return;
    const uint64_t shot = i / m;
    const uint32_t c = (uint32_t)(i % m);
    out[i] = (uint8_t)((words[shot * wm + (c >> 6)] >> (c & 63)) & 1ull);
}

int check_common(vibe_graph* G, const void* synd, uint64_t B) {
    if (!G) return fail(VIBE_EINVAL, "graph handle is NULL");
    if (B && !synd) return fail(VIBE_EINVAL, "syndromes is NULL");
    if (B > (1ull << 40)) return fail(VIBE_EINVAL, "B is too large");
    return VIBE_OK;
}

uint32_t chunk_for(const DevGraph& g, uint64_t B, bool decode) {
    // workspace of the per-chunk buffers: 8 GB holds ~40k shots of the d = 9
    // circuit graph, so a 32768-shot batch is one persistent launch (each
    // launch ends in a tail of long items)
    const size_t budget = 8ull << 30;
    uint64_t bc = budget / per_shot_bytes(g, decode);
    bc = std::max<uint64_t>(256, std::min<uint64_t>(bc, 65536));
    bc = std::min<uint64_t>(bc, (uint64_t)UINT32_MAX / std::max<uint32_t>(g.L, 1));
    return (uint32_t)std::min<uint64_t>(bc, B);
}

}  // namespace

void begin_timed(vibe_graph* G, int which, hipStream_t st) {
    if (!G->profiling) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(a, st);
    G->ev[which].push_back({a, b});
}

void end_timed(vibe_graph* G, int which, hipStream_t st) {
    if (!G->profiling || G->ev[which].empty()) return;
    (void)hipEventRecord(G->ev[which].back().second, st);
}

}  // namespace vibe

using namespace vibe;

extern "C" int vibe_profile_enable(vibe_graph* G, int enable) {
    if (!G) return fail(VIBE_EINVAL, "graph handle is NULL");
    G->profiling = enable != 0;
    return VIBE_OK;
}

extern "C" int vibe_profile_read(vibe_graph* G, double* ms, uint64_t* launches) {
    if (!G || !ms || !launches) return fail(VIBE_EINVAL, "NULL argument");
    for (int k = 0; k < 3; k++) {
        double tot = 0.0;
        for (auto& pr : G->ev[k]) {
            hipError_t e = hipEventSynchronize(pr.second);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            float t = 0.0f;
            e = hipEventElapsedTime(&t, pr.first, pr.second);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            tot += t;
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        ms[k] = tot;
        launches[k] = G->ev[k].size();
        G->ev[k].clear();
    }
    return VIBE_OK;
}

namespace vibe {
namespace {

// The batched decode of vibe_decode (bytes != NULL) and vibe_decode_packed
// (words != NULL): chunks of shots through K1-K3, then K4 over the batch.
// Packed syndromes are expanded chunk by chunk into the handle's input
// buffer, and that chunk is then decoded as shots 0..n-1 of it.
int decode_batch(vibe_graph* G, const uint8_t* bytes, const uint64_t* words, uint64_t B, uint64_t* corrections,
                 uint8_t* observables, vibe_shot_stats* stats, void* stream) {
    set_error("");
    int rc = check_common(G, bytes ? (const void*)bytes : (const void*)words, B);
    if (rc) return rc;
    if (B && (!corrections || (!observables && G->h.k))) return fail(VIBE_EINVAL, "an output pointer is NULL");
    if (!B) return VIBE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevGraph g = decode_view(G, true, B);
    const uint32_t bc = chunk_for(g, B, true);
    if (bc < B) g = decode_view(G, true, bc);
    uint8_t* u = nullptr;
    if (words) {
        const size_t in_bytes = al256((size_t)bc * (g.m ? g.m : 1));
        if (G->ws_in.bytes < in_bytes) {
            if (G->ws_in.base) {
                hipError_t e = hipDeviceSynchronize();
                if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before growing the input buffer");
                (void)hipFree(G->ws_in.base);
                G->ws_in.base = nullptr;
                G->ws_in.bytes = 0;
            }
            void* p = nullptr;
            if (hipMalloc(&p, in_bytes) != hipSuccess) return fail(VIBE_ENOMEM, "input buffer allocation failed");
            G->ws_in.base = p;
            G->ws_in.bytes = in_bytes;
        }
        u = static_cast<uint8_t*>(G->ws_in.base);
    }
    const bool in_lds = use_lds_slab(G, g);
    if (in_lds) g.dec_global = 0;  // the LDS slab variant keeps decisions in LDS
    const int bpg = G->tune_grid > 0 ? std::min(G->tune_grid, bp_grid(g, in_lds)) : bp_grid(g, in_lds);
    const int lg = lsd_grid_for(bc);
    ChunkBufs W;
    if ((rc = carve(g, G, bc, true, in_lds ? 0 : bpg, bpg, lg, &W))) return rc;
    const uint32_t wm = g.words_m ? g.words_m : 1;
    for (uint64_t s0 = 0; s0 < B; s0 += bc) {
        const uint32_t n = (uint32_t)std::min<uint64_t>(bc, B - s0);
        if (!words) {
            rc = decode_chunk(G, g, W, bytes, s0, n, corrections, stats, bpg, lg, st, in_lds);
        } else {
            const uint64_t cells = (uint64_t)n * g.m;
            if (cells) {
                hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st,
                                   words + s0 * g.words_m, wm, g.m, (uint64_t)n, u);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return hip_fail(e, "unpack_kernel launch");
            }
            rc = decode_chunk(G, g, W, u, 0, n, corrections + s0 * g.words_n, stats ? stats + s0 : nullptr, bpg,
                              lg, st, in_lds);
        }
        if (rc) return rc;
    }
    return launch_observables(g, corrections, 0, (uint32_t)std::min<uint64_t>(B, UINT32_MAX), observables, st);
}

}  // namespace
}  // namespace vibe

extern "C" int vibe_decode(vibe_graph* G, const uint8_t* syndromes, uint64_t B, uint64_t* corrections,
                           uint8_t* observables, vibe_shot_stats* stats, void* stream) {
    return decode_batch(G, syndromes, nullptr, B, corrections, observables, stats, stream);
}

extern "C" int vibe_decode_packed(vibe_graph* G, const uint64_t* syndromes, uint64_t B, uint64_t* corrections,
                                  uint8_t* observables, vibe_shot_stats* stats, void* stream) {
    return decode_batch(G, nullptr, syndromes, B, corrections, observables, stats, stream);
}

extern "C" int vibe_decode_plain(vibe_graph* G, const uint8_t* syndromes, uint64_t B,
                                 uint64_t* corrections, uint8_t* observables, vibe_shot_stats* stats,
                                 void* stream) {
    set_error("");
    int rc = check_common(G, syndromes, B);
    if (rc) return rc;
    if (B && (!corrections || (!observables && G->h.k))) return fail(VIBE_EINVAL, "an output pointer is NULL");
    if (!B) return VIBE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGraph& g = G->h.dg;
    ChunkBufs W;
    const int blocks = (int)g.L;  // one block per member of the one shot
    const bool in_lds = bp_slab_fits_lds(g);
    if ((rc = carve(g, G, 1, true, in_lds ? 0 : blocks, blocks, 1, &W))) return rc;
    for (uint64_t s0 = 0; s0 < B; s0++) {
        if ((rc = decode_chunk(G, g, W, syndromes, s0, 1, corrections, stats, blocks, 1, st, in_lds))) return rc;
        if ((rc = launch_observables(g, corrections, s0, 1, observables, st))) return rc;
    }
    return VIBE_OK;
}

extern "C" int vibe_bp_ensemble(vibe_graph* G, const uint8_t* syndromes, uint64_t B, uint32_t T_run,
                                int stop_on_converge, int32_t* t_conv, void* posteriors,
                                uint64_t* ehat, void* stream) {
    set_error("");
    int rc = check_common(G, syndromes, B);
    if (rc) return rc;
    if (T_run < 1 || T_run > (uint32_t)kMaxT) return fail(VIBE_EINVAL, "T_run must be in 1..64");
    if (B && !t_conv) return fail(VIBE_EINVAL, "t_conv is NULL");
    if (!B) return VIBE_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGraph& g = G->h.dg;
    const uint32_t bc = chunk_for(g, B, false);
    const bool in_lds = bp_slab_fits_lds(g);
    const int bpg = bp_grid(g, in_lds);
    ChunkBufs W;
    if ((rc = carve(g, G, bc, false, in_lds ? 0 : bpg, bpg, 0, &W))) return rc;
    for (uint64_t s0 = 0; s0 < B; s0 += bc) {
        const uint32_t n = (uint32_t)std::min<uint64_t>(bc, B - s0);
        if ((rc = memset_async(W.cmask, 8ull * n * (kMaxT + 1), st)) ||
            (rc = memset_async(W.iters, 4ull * n, st)) || (rc = memset_async(W.counters, 64, st)))
            return rc;
        BpLaunch b{};
        b.member_major = 0;
        b.slab_in_lds = in_lds ? 1 : 0;
        b.syndromes = syndromes;
        b.shot0 = s0;
        b.n_shots = n;
        b.T_run = T_run;
        b.use_M = 0;
        b.stop_on_converge = stop_on_converge ? 1 : 0;
        b.accumulate_q = 0;
        b.fast_zero = 0;
        b.t_conv = t_conv + s0 * g.L;
        b.weight = nullptr;
        b.cand = ehat ? ehat + s0 * g.L * g.words_n : nullptr;
        b.post_out = posteriors ? static_cast<unsigned char*>(posteriors) + s0 * g.L * g.n * msg_bytes(g)
                                : nullptr;
        b.conv_mask = W.cmask;
        b.iters = W.iters;
        b.qfix = nullptr;
        b.slab = W.slab;
        b.post_slab = W.post_slab;
        b.counter = W.counters;
        b.grid = (int)std::min<uint64_t>((uint64_t)bpg, (uint64_t)n * g.L);
        if ((rc = launch_bp(g, b, st))) return rc;
    }
    return VIBE_OK;
}

extern "C" int vibe_lsd(vibe_graph* G, const uint8_t* syndromes, const float* soft, uint64_t B,
                        uint64_t* corrections, vibe_shot_stats* stats, void* stream) {
    set_error("");
    int rc = check_common(G, syndromes, B);
    if (rc) return rc;
    if (B && (!soft || !corrections)) return fail(VIBE_EINVAL, "soft or corrections is NULL");
    if (!B) return VIBE_OK;
    if (B > UINT32_MAX) return fail(VIBE_EINVAL, "B must be < 2^32 for vibe_lsd");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGraph& g = G->h.dg;
    const int lg = lsd_grid_for(B);
    const size_t per = lsd_scratch_per_block(g);
    if ((rc = ensure_workspace(G, per * lg))) return rc;
    LsdLaunch l{};
    l.syndromes = syndromes;
    l.shot0 = 0;
    l.list = nullptr;
    l.list_count = nullptr;
    l.n_list = (uint32_t)B;
    l.soft_f32 = soft;
    l.soft_fix = nullptr;
    l.corrections = corrections;
    l.stats = stats;
    l.scratch = G->ws.base;
    l.scratch_per_block = per;
    l.grid = lg;
    return launch_lsd(g, l, st);
}

// ---------------------------------------------------------------------------
// vibe_decode_noalloc: the batched decode with every buffer beyond the
// caller's inputs and outputs carved from one static device array.  In host
// code the array's name is only a stand-in; its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.

namespace vibe {
namespace {

constexpr size_t kNoallocBytes = (size_t)VIBE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoallocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on each device, with that device current).
int scratch_for_device(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(VIBE_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(VIBE_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return VIBE_OK;
}

// A launch plan whose buffers fit `cap` bytes: BP blocks (message and
// posterior slabs) get at most half of it, LSD blocks at most a quarter and
// the shots of one chunk the rest.  Returns false if not even one block of
// each and one shot fit.
bool noalloc_plan(const DevGraph& g, bool in_lds, int full_grid, uint64_t B, size_t cap, int* bpg, int* lg,
                  uint32_t* bc, size_t* sizes) {
    const size_t slab = in_lds ? 0 : msg_bytes(g) * bp_slabs(g) * std::max<size_t>((size_t)g.max_chunks * kWave, 1);
    const size_t per_block = al256(slab) + al256(msg_bytes(g) * bp_post_elems(g));
    const size_t per_lsd = lsd_scratch_per_block(g);
    int grid = (int)std::min<size_t>((size_t)full_grid, (cap / 2) / per_block);
    int lsd = (int)std::min<size_t>(512, (cap / 4) / per_lsd);
    if (grid < 1 || lsd < 1) return false;
    const size_t fixed = carve_sizes(g, 0, true, in_lds ? 0 : grid, grid, lsd, sizes);
    if (fixed >= cap) return false;
    // per-shot bytes plus the 256-byte rounding of each buffer
    const size_t per_shot = per_shot_bytes(g, true);
    uint64_t n = (cap - fixed - 256 * kBufs) / per_shot;
    n = std::min<uint64_t>(n, chunk_for(g, B, true));
    if (n < 1) return false;
    lsd = std::min<int>(lsd, (int)std::min<uint64_t>(n, 512));
    if (carve_sizes(g, (uint32_t)n, true, in_lds ? 0 : grid, grid, lsd, sizes) > cap) return false;
    *bpg = grid;
    *lg = lsd;
    *bc = (uint32_t)n;
    return true;
}

}  // namespace
}  // namespace vibe

extern "C" int vibe_decode_noalloc(vibe_graph* G, const uint8_t* syndromes, uint64_t B, uint64_t* corrections,
                                   uint8_t* observables, vibe_shot_stats* stats, void* stream) {
    using namespace vibe;
    set_error("");
    int rc = check_common(G, syndromes, B);
    if (rc) return rc;
    if (B && (!corrections || (!observables && G->h.k))) return fail(VIBE_EINVAL, "an output pointer is NULL");
    if (!B) return VIBE_OK;
    DevGraph g = decode_view(G, true, B);
    const bool in_lds = use_lds_slab(G, g);
    if (in_lds) g.dec_global = 0;  // the LDS slab variant keeps decisions in LDS
    const int full = G->tune_grid > 0 ? std::min(G->tune_grid, bp_grid(g, in_lds)) : bp_grid(g, in_lds);
    int bpg = 0, lg = 0;
    uint32_t bc = 0;
    size_t sizes[kBufs];
    if (!noalloc_plan(g, in_lds, full, B, kNoallocBytes, &bpg, &lg, &bc, sizes))
        return fail(VIBE_EUNSUPPORTED, "the graph needs more buffer space than the " +
                                           std::to_string(kNoallocBytes >> 20) +
                                           " MiB static scratch of vibe_decode_noalloc holds for one shot");
    unsigned char* base = nullptr;
    if ((rc = scratch_for_device(G->device, &base))) return rc;
    ChunkBufs W;
    carve_at(base, sizes, &W);
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (uint64_t s0 = 0; s0 < B; s0 += bc) {
        const uint32_t n = (uint32_t)std::min<uint64_t>(bc, B - s0);
        if ((rc = decode_chunk(G, g, W, syndromes, s0, n, corrections, stats, bpg, lg, st, in_lds, false)))
            return rc;
    }
    return launch_observables(g, corrections, 0, (uint32_t)std::min<uint64_t>(B, UINT32_MAX), observables, st);
}
