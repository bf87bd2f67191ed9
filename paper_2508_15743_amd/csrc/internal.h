// Internal definitions shared by the HIP translation units of libvibelsd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/vibelsd.h"

namespace vibe {

constexpr int kWave = 64;
constexpr int kMaxColDeg = 15;
constexpr int kMaxL = 64;
constexpr int kMaxT = 64;
constexpr uint32_t kMaxLsdOrder = 64;  // pairs among the first 64 non-pivot columns: 2016
constexpr double kQScale = 72057594037927936.0;  // 2^56: fixed point of the LLR average

// Member schedules.  Member i's serial sweep (its permutation of the columns)
// is regrouped into chunks: sets of whole columns, no two sharing a check,
// with at most 64 edges, in an order that keeps every pair of columns sharing
// a check in their permutation order.  A chunk has 64 slots, one lane of a
// wavefront per slot; the edges of one column sit in consecutive slots in
// ascending check order, and unused slots have deg = 0 (and c = v = 0).
// Slot q of the member's chunk k is also position k*64 + q of the member's
// message slab.  The schedule of all members is one array of chunk records;
// a record holds 64 entries of each field, field by field:
//   meta (u32) : c | seg << 16 | deg << 20 | dmax << 24   (seg = index of the
//                edge inside its column, deg = the column's check count,
//                dmax = the largest deg in the chunk, in all 64 slots)
//   v    (u32) : the column
//   lam  (F)   : its channel LLR in the message precision F
//   init (B)   : the suffix state of the slot for the initial messages
//                mu = lambda (row state bits, same width as F)
// so a record is 64 * (8 + 2 sizeof(F)) bytes: 1024 for FP32, 1536 for FP64.
// A recut schedule for P shots per wavefront has records of W = 64 / P
// entries per field (the same fields, at 4W, 8W and 8W + W sizeof(F)).
constexpr uint32_t kMetaDegShift = 20, kMetaDmaxShift = 24;
constexpr uint32_t kRecV = 256, kRecLam = 512;  // byte offsets of fields in a record
inline constexpr uint32_t rec_bytes(bool fp64) { return fp64 ? 1536u : 1024u; }
inline constexpr uint32_t rec_init(bool fp64) { return fp64 ? 1024u : 768u; }
inline constexpr uint32_t rec_bytes_w(bool fp64, uint32_t W) { return W * (fp64 ? 24u : 16u); }

// Wave-uniform values.  A value every lane computes identically (a shuffle
// broadcast, a wave reduction, an LDS word all lanes read) still lives in a
// vector register, and the compiler may then treat branches on it as
// divergent and split loops per lane, so that a later shuffle reads a lane
// that is on another path.  Every such control value goes through
// readfirstlane, which makes it a scalar the compiler knows is uniform.
__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline int32_t uni(int32_t x) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)x); }

// One ticket per wave from a global counter.  Every lane executes the atomic
// (lane 0 adds v, the others 0), so no branch on the lane index precedes the
// broadcast: a branch there lets the compiler route lanes 1..63 around the
// atomic and run the broadcast with lane 0 inactive.
__device__ inline uint32_t wave_ticket(uint32_t* counter, uint32_t v) {
    const uint32_t got = atomicAdd(counter, __lane_id() == 0 ? v : 0u);
    return uni(__shfl(got, 0));
}

// Row state word: the bits of a magnitude (>= 0) in the message precision
// with a parity bit in the sign position.  Magnitudes compare like unsigned
// integers, so combining two states is an integer min of the magnitude bits
// and an xor of the sign bits.  B = uint32_t for FP32 messages, uint64_t for
// FP64.
template <class B>
__host__ __device__ inline B rs_combine(B a, B b) {
    constexpr B kSign = (B)1 << (8 * sizeof(B) - 1);
    const B ma = a & ~kSign, mb = b & ~kSign;
    return (ma < mb ? ma : mb) | ((a ^ b) & kSign);
}

// Everything a kernel needs to know about a resident graph (passed by value).
struct DevGraph {
    uint32_t m, n, k, L, M, T;
    uint32_t E;
    uint32_t words_n, words_m;  // ceil(n/64), ceil(m/64)
    uint32_t max_chunks;        // largest chunk count of a member (slab = max_chunks * 64)
    uint32_t P;                 // shots per wavefront of the schedule in sched: 1 (64-edge
                                // chunks), or 2 and 4 (chunks recut to 64 / P edges)
    int dec_global;             // BP decisions in global memory (per-chunk decision
                                // masks and a bitmap, after the block's posteriors)
                                // instead of a bitmap in LDS
    int fp64;                   // message precision: 0 = FP32, 1 = FP64
    int flood;                  // schedule: 0 = serial-V, 1 = parallel (flooding)
    int layered;                // 1: layered (check-serial) schedule; cperm holds the check orders
    uint32_t lsd_order;         // 0 = LSD-0; > 0: combination sweep over the first lsd_order non-pivots
    double alpha, clamp;
    const double* alpha_t;      // kMaxT scaling factors, one per iteration, or null (alpha throughout)
    uint32_t ident32;           // row state of "no message": clamp, parity 0 (FP32 bits)
    uint64_t ident64;           // the same in FP64 bits
    int all_lam_positive;
    const uint32_t* rp;           // m + 1
    const uint32_t* ri;           // E, CSR column of each edge
    const uint32_t* cp;           // n + 1
    const uint32_t* ci;           // E, CSC check of each edge
    const double* lam64;          // n, FP64 channel LLR (candidate weights)
    const void* lam;              // n, channel LLR in the message precision
    const uint64_t* e0;           // words_n: decisions of columns without checks
    const unsigned char* sched;   // chunk records of all members, see above (W = 64 / P
                                  // entries per field for the recut schedules)
    const uint32_t* member_chunk; // L + 1: chunk range of each member
    const uint32_t* cperm;        // layered schedule: L x m check orders (else unused)
    const uint64_t* lobs;         // k x words_n, bit-packed observable rows
};

struct GraphHost {
    vibe_config cfg;
    uint32_t m, n, k;
    uint64_t E;
    uint32_t max_row, max_col;
    uint32_t levels_min, levels_max;
    uint32_t chunks_min, chunks_max;
    uint64_t device_bytes;
    DevGraph dg;
    std::vector<void*> allocations;
    std::vector<uint32_t> perms;  // the member schedules as given (L x n, or L x m layered)
};

// Per-handle workspace, grown on demand and reused across calls.
struct Workspace {
    size_t bytes = 0;
    void* base = nullptr;
};

}  // namespace vibe

struct vibe_graph {
    vibe::GraphHost h;
    vibe::Workspace ws;
    vibe::Workspace ws_in;  // unpacked syndromes of vibe_decode_packed
    int device = 0;
    // launch settings chosen by vibe_autotune or vibe_set_launch: slab in
    // LDS (-1 = not tuned, use LDS whenever it fits; 0 = global; 1 = LDS),
    // BP grid (0 = full occupancy) and shots per wavefront (1, 2 or 4)
    int tune_lds = -1;
    int tune_grid = 0;
    uint32_t tune_P = 1;
    int tune_dec = -1;  // decisions in global memory: -1 = where that raises occupancy
    // decode schedules recut for 2 and 4 shots per wavefront (index P / 4),
    // built on first use
    const unsigned char* multi_recs[2] = {nullptr, nullptr};
    const uint32_t* multi_member_chunk[2] = {nullptr, nullptr};
    uint32_t multi_max_chunks[2] = {0, 0};
    // gradient schedule, built by the first vibe_bp_grad call: the member
    // sweeps recut into chunks of at most grad_width edges, so that one
    // wavefront runs grad_P = 64 / grad_width shots of a member side by side
    uint32_t grad_width = 0, grad_P = 1, grad_max_chunks = 0;
    uint32_t grad_force = 0;  // width set by vibe_grad_set_width (0: chosen per graph)
    const unsigned char* grad_recs = nullptr;
    const uint32_t* grad_member_chunk = nullptr;
    // kernel timing (vibe_profile_enable): event pairs per kernel class
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
};

namespace vibe {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// launchers (each returns VIBE_OK or VIBE_EHIP)
struct BpLaunch {
    const uint8_t* syndromes;  // B x m
    uint64_t shot0;            // first shot of this launch (index into syndromes)
    uint32_t n_shots;
    uint32_t T_run;
    int use_M;                 // apply the correction limit
    int stop_on_converge;
    int accumulate_q;          // add normalised posteriors of unconverged members
    int fast_zero;             // decide s = 0 shots without running BP
    int member_major;          // work item order: member-major (1) or shot-major (0)
    // outputs, indexed by local shot (0 .. n_shots-1) and member
    int32_t* t_conv;           // n_shots x L
    double* weight;            // n_shots x L (candidate weight), may be null
    uint64_t* cand;            // n_shots x L x words_n, may be null
    void* post_out;            // n_shots x L x n in the message precision, may be
                               // null (written every iteration)
    uint64_t* conv_mask;       // n_shots x (kMaxT + 1): members converged at t
    uint32_t* iters;           // n_shots: iterations run, summed over members
    int64_t* qfix;             // n_shots x n, may be null
    // scratch
    void* slab;                // bp_slabs x grid x max_chunks x 64 row states /
                               // messages (global variant), message precision
    void* post_slab;           // grid x n, message precision
    uint32_t* counter;         // work counter
    int grid;
    int slab_in_lds;           // which kernel variant to launch
    int latency;               // the latency variant (every item resident at once)
};
int launch_bp(const DevGraph& g, const BpLaunch& a, hipStream_t st);

// Ragged batching: one BP launch over the items of several requests, each on
// its own graph (all with the same message precision and schedule).
struct BpSeg {
    DevGraph g;
    BpLaunch a;       // that request's inputs and outputs (slab fields unused)
    uint32_t item0;   // its first item in the launch's numbering
};
struct RaggedLaunch {
    const BpSeg* segs;     // device array, n_segs entries, item0 ascending
    uint32_t n_segs;
    uint32_t n_items;      // total over the segments
    void* slab;            // bp_slabs x grid x slab_elems
    void* post_slab;       // grid x post_elems
    uint32_t slab_elems;   // largest max_chunks * 64 over the segments
    uint32_t post_elems;   // largest n + 64 over the segments
    uint32_t* counter;
    int grid;
    int slab_in_lds;
    int fp64, flood;
    int multi;             // some segment runs several shots per wavefront
    int layered;           // some segment is on the layered schedule
    int dec_global;        // the non-layered segments keep decisions in global memory
    int latency;           // the latency variant (every item resident at once)
    size_t lds_bytes;      // largest bp_lds_bytes over the segments
};
int launch_bp_ragged(const RaggedLaunch& r, hipStream_t st);
int bp_grid_for(bool fp64, bool flood, bool slab_in_lds, size_t lds_bytes, bool ragged, bool layered = false,
                uint32_t P = 1, bool dec_global = false, bool latency = false);
// Resident blocks of the latency variant of K1 for g (0 where g has none:
// FP64, another schedule, slab in LDS, several shots per wavefront,
// decisions in global memory).
int bp_latency_grid(const DevGraph& g, bool slab_in_lds);
int bp_grid(const DevGraph& g, bool slab_in_lds);
size_t bp_lds_bytes(const DevGraph& g, bool slab_in_lds);
int bp_slabs(const DevGraph& g);  // slabs per block: 1 (serial), 2 (parallel: states and messages)
bool bp_slab_fits_lds(const DevGraph& g);
// posterior slab of one BP block, in message-precision elements: P x n
// posteriors, then 64 slots that absorb the stores of lanes that own no
// column, padded to 8 bytes; with decisions in global memory, then one
// decision mask per chunk and P decision bitmaps of words_n words.  Every
// size is a multiple of 8 bytes, so that each block's area (and, in a
// ragged launch, the largest of them) keeps 8-byte alignment.
__host__ __device__ inline size_t bp_post_head(const DevGraph& g) {
    const size_t per8 = g.fp64 ? 1 : 2;  // elements per 8 bytes
    return ((size_t)g.P * g.n + kWave + per8 - 1) / per8 * per8;
}
__host__ __device__ inline size_t bp_post_elems(const DevGraph& g) {
    if (!g.dec_global) return bp_post_head(g);
    return bp_post_head(g) + ((size_t)g.max_chunks + (size_t)g.P * g.words_n) * (g.fp64 ? 1 : 2);
}
// BP work items of n shots: (member, group of P shots)
inline uint64_t bp_items(const DevGraph& g, uint64_t n) { return (n + g.P - 1) / g.P * g.L; }

// The graph as the decoder launches it for `shots` shots: the handle's graph
// with the schedule recut for tune_P shots per wavefront when that is above
// 1 (and allow_multi), else the 64-edge schedule; decisions in global memory
// as tune_dec says (automatic: where that lets more wavefronts reside and
// the work items outnumber those that reside with decisions in LDS).
DevGraph decode_view(const vibe_graph* G, bool allow_multi = true, uint64_t shots = UINT64_MAX);
// Whether decisions in global memory let more BP wavefronts reside than a
// decision bitmap in LDS (g.dec_global ignored).
bool dec_global_pays(const DevGraph& g);
// Whether the decoder keeps g's message slab in LDS: where it fits and the
// handle says so; automatic (tune_lds < 0): where it fits and costs no
// residency (a slab in LDS that leaves room for fewer wavefronts than a
// global slab runs slower: the chunk chain's latency then binds).
bool use_lds_slab(const vibe_graph* G, const DevGraph& g);
// Build (once) the decode schedule recut for P = 2 or 4 shots per wavefront.
int build_multi_schedule(vibe_graph* G, uint32_t P);
int launch_zero(void* p, size_t bytes, hipStream_t st);

struct SelectLaunch {
    uint32_t n_shots;
    uint64_t shot0;
    const int32_t* t_conv;
    const double* weight;
    const uint64_t* cand;
    const uint32_t* iters;
    const uint64_t* conv_mask;    // n_shots x (kMaxT + 1); word 0 = members that saturated, may be null
    uint64_t* corrections;        // global B x words_n (indexed by shot0 + i)
    vibe_shot_stats* stats;       // global, may be null
    uint32_t* fail_list;          // local shot indices that need LSD
    uint32_t* fail_count;
};
int launch_select(const DevGraph& g, const SelectLaunch& a, hipStream_t st);

struct LsdLaunch {
    const uint8_t* syndromes;     // global B x m
    uint64_t shot0;
    const uint32_t* list;         // local shot indices, or null = all n_list shots
    const uint32_t* list_count;   // device count (if list != null)
    uint32_t n_list;              // upper bound on the list length
    const float* soft_f32;        // global B x n (indexed by shot0 + i), or
    const int64_t* soft_fix;      // local n_shots x n fixed point
    uint64_t* corrections;        // global B x words_n
    vibe_shot_stats* stats;       // global, may be null
    void* scratch;
    size_t scratch_per_block;
    int grid;
};
int launch_lsd(const DevGraph& g, const LsdLaunch& a, hipStream_t st);
size_t lsd_scratch_per_block(const DevGraph& g);
size_t lsd_lds_bytes(const DevGraph& g);

// Record a start event before a launch of kernel class `which` (0 BP,
// 1 selection, 2 LSD) when profiling is on; end_timed records the end event.
void begin_timed(vibe_graph* G, int which, hipStream_t st);
void end_timed(vibe_graph* G, int which, hipStream_t st);

int launch_observables(const DevGraph& g, const uint64_t* corrections, uint64_t shot0,
                       uint32_t n_shots, uint8_t* observables, hipStream_t st);

}  // namespace vibe
