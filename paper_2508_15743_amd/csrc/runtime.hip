// Ragged batching, captured launch sequences and autotuning.
//
// A ragged call decodes several requests, possibly on graphs of different
// codes, with one persistent BP launch over all of their (shot, member)
// items, then selection, LSD and observables per request.  Per request the
// results are those of vibe_decode on that request alone: every kernel's
// output for a shot depends only on that shot's syndrome and graph.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "internal.h"

struct vibe_runtime {
    int device = 0;
    vibe::Workspace ws;
    // host copy of the last segment table: kept until its upload has run
    std::vector<vibe::BpSeg> table;
    hipEvent_t table_done = nullptr;
};

struct vibe_exec {
    int device = 0;
    vibe::Workspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace vibe {

// One device-to-device copy of a list (server gather and scatter).
struct CopyEntry {
    const unsigned char* src;
    unsigned char* dst;
    uint64_t bytes;
};

namespace {

// gridDim.x entries, gridDim.y blocks per entry
__global__ void copy_entries_kernel(const CopyEntry* tab) {
    const CopyEntry e = tab[blockIdx.x];
    const uint64_t step = (uint64_t)blockDim.x * gridDim.y;
    const uint64_t start = (uint64_t)blockIdx.y * blockDim.x + threadIdx.x;
    const bool w8 = ((reinterpret_cast<uintptr_t>(e.src) | reinterpret_cast<uintptr_t>(e.dst) | e.bytes) & 7) == 0;
    if (w8) {
        const uint64_t* s8 = reinterpret_cast<const uint64_t*>(e.src);
        uint64_t* d8 = reinterpret_cast<uint64_t*>(e.dst);
        for (uint64_t i = start; i < e.bytes / 8; i += step) d8[i] = s8[i];
    } else {
        for (uint64_t i = start; i < e.bytes; i += step) e.dst[i] = e.src[i];
    }
}

int launch_copies(const CopyEntry* dev_tab, uint32_t n, hipStream_t st) {
    if (!n) return VIBE_OK;
    hipLaunchKernelGGL(copy_entries_kernel, dim3(n, 8), dim3(256), 0, st, dev_tab);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "copy_entries_kernel launch");
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int grow(Workspace& ws, size_t bytes) {
    if (ws.bytes >= bytes) return VIBE_OK;
    if (ws.base) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize before growing the workspace");
        (void)hipFree(ws.base);
        ws.base = nullptr;
        ws.bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(VIBE_ENOMEM, "workspace allocation failed");
    ws.base = p;
    ws.bytes = bytes;
    return VIBE_OK;
}

// One request's part of a round: shots [shot0, shot0 + n) of request `req`.
struct Seg {
    uint32_t req;
    uint64_t shot0;
    uint32_t n;
    DevGraph g;  // the graph as launched (schedule for its shots per wavefront)
    // workspace offsets of its buffers
    size_t t_conv, weight, cand, cmask, iters, qfix, fail_list;
};

struct Round {
    std::vector<Seg> segs;
    size_t zero_off = 0, zero_bytes = 0;  // counters, masks, iteration counts, averages
    size_t segs_off = 0, slab_off = 0, post_off = 0, lsd_off = 0;
    size_t bytes = 0;
    uint32_t slab_elems = 0, post_elems = 0;
    size_t lds_bytes = 0, lsd_per_block = 0;
    int grid = 0, lsd_grid = 0;
    bool slab_in_lds = false;
    bool flood = false;  // some segment uses the parallel schedule
    bool multi = false;  // some segment runs several shots per wavefront
    bool layered = false;  // some segment is on the layered schedule
    bool dec_global = false;  // chunked segments keep decisions in global memory
    bool latency = false;     // every item resident at once: the deeper prefetch ring
};

size_t seg_bytes(const DevGraph& g, uint32_t n) {
    return al256(4ull * n * g.L) + al256(8ull * n * g.L) + al256(8ull * n * g.L * g.words_n) +
           al256(8ull * n * (kMaxT + 1)) + al256(4ull * n) + al256(8ull * n * g.n) + al256(4ull * n);
}

int check_requests(const vibe_request* reqs, uint32_t n) {
    if (!reqs && n) return fail(VIBE_EINVAL, "reqs is NULL");
    for (uint32_t i = 0; i < n; i++) {
        const vibe_request& r = reqs[i];
        if (!r.graph) return fail(VIBE_EINVAL, "a request has no graph");
        if (r.B && (!r.syndromes || !r.corrections || (!r.observables && r.graph->h.k)))
            return fail(VIBE_EINVAL, "a request has a NULL device pointer");
        if (r.B > (1ull << 40)) return fail(VIBE_EINVAL, "a request is too large");
        const DevGraph& g = r.graph->h.dg;
        const DevGraph& g0 = reqs[0].graph->h.dg;
        if (g.fp64 != g0.fp64) return fail(VIBE_EINVAL, "all graphs of a ragged call need the same message_bits");
        if (r.graph->device != reqs[0].graph->device) return fail(VIBE_EINVAL, "all graphs must be on one device");
    }
    return VIBE_OK;
}

// Split the requests into rounds whose per-shot buffers fit the budget, and
// lay out each round's workspace.
std::vector<Round> plan(const vibe_request* reqs, uint32_t n_reqs, size_t budget) {
    std::vector<Round> rounds;
    Round cur;
    size_t used = 0;
    for (uint32_t i = 0; i < n_reqs; i++) {
        const DevGraph& g = reqs[i].graph->h.dg;
        const size_t per = seg_bytes(g, 1);
        uint64_t s0 = 0;
        while (s0 < reqs[i].B) {
            uint64_t room = used < budget ? (budget - used) / per : 0;
            if (room == 0 && !cur.segs.empty()) {
                rounds.push_back(cur);
                cur = Round();
                used = 0;
                continue;
            }
            room = std::max<uint64_t>(room, 1);
            const uint32_t n = (uint32_t)std::min<uint64_t>({room, reqs[i].B - s0, (uint64_t)65536,
                                                              (uint64_t)(UINT32_MAX / 2) / std::max<uint32_t>(g.L, 1)});
            Seg sg{};
            sg.req = i;
            sg.shot0 = s0;
            sg.n = n;
            cur.segs.push_back(sg);
            used += seg_bytes(g, n);
            s0 += n;
        }
    }
    if (!cur.segs.empty()) rounds.push_back(cur);
    for (Round& r : rounds) {
        // longest items first (edges x iteration limit), so that the long
        // serial chains do not start last and leave the GPU idle in the
        // round's tail; results do not depend on the order
        std::stable_sort(r.segs.begin(), r.segs.end(), [&](const Seg& a, const Seg& b) {
            const DevGraph& ga = reqs[a.req].graph->h.dg;
            const DevGraph& gb = reqs[b.req].graph->h.dg;
            return (uint64_t)ga.E * ga.T > (uint64_t)gb.E * gb.T;
        });
        bool lds_ok = true;
        bool fp64 = false, flood = false, multi = false;
        size_t lds_global = 0, lds_l = 0;
        bool layered = false;
        for (const Seg& sg : r.segs) {
            flood = flood || reqs[sg.req].graph->h.dg.flood != 0;
            layered = layered || reqs[sg.req].graph->h.dg.layered != 0;
        }
        // several shots per wavefront (the autotuner's choice per graph)
        // only in rounds where every serial segment runs them: the launch
        // then needs the multi-shot kernel, whose lower occupancy would slow
        // the other segments' items
        bool all_multi = !flood;
        for (Seg& sg : r.segs) {
            const vibe_graph* G = reqs[sg.req].graph;
            if (!G->h.dg.layered) all_multi = all_multi && decode_view(G).P > 1;
        }
        for (Seg& sg : r.segs) {
            sg.g = decode_view(reqs[sg.req].graph, all_multi, sg.n);
            multi = multi || sg.g.P > 1;
        }
        // slabs in LDS only if every segment's fits (with its decisions in
        // LDS) and no graph was tuned otherwise
        for (const Seg& sg : r.segs) {
            DevGraph g = sg.g;
            g.dec_global = 0;
            lds_ok = lds_ok && !multi && use_lds_slab(reqs[sg.req].graph, g);
        }
        // decisions in global memory for every chunked segment if one of
        // them wants it (a graph whose decision bitmap would cap the
        // launch's occupancy); not with LDS slabs, and the launch without
        // several shots per wavefront has no such variant with layered
        // segments
        bool dg = false;
        for (const Seg& sg : r.segs) dg = dg || (!sg.g.layered && sg.g.dec_global);
        if (lds_ok || (layered && !multi)) dg = false;
        for (Seg& sg : r.segs) sg.g.dec_global = (dg && !sg.g.layered) ? 1 : 0;
        for (const Seg& sg : r.segs) {
            const DevGraph& g = sg.g;
            fp64 = g.fp64 != 0;
            r.slab_elems = std::max<uint32_t>(r.slab_elems, std::max<uint32_t>(g.max_chunks, 1) * kWave);
            r.post_elems = std::max<uint32_t>(r.post_elems, (uint32_t)bp_post_elems(g));
            lds_global = std::max(lds_global, bp_lds_bytes(g, false));
            lds_l = std::max(lds_l, bp_lds_bytes(g, true));
            r.lsd_per_block = std::max(r.lsd_per_block, lsd_scratch_per_block(g));
        }
        r.slab_in_lds = lds_ok;
        r.flood = flood;
        r.multi = multi;
        r.layered = layered;
        r.dec_global = dg;
        r.lds_bytes = lds_ok ? lds_l : lds_global;
        r.grid = bp_grid_for(fp64, flood, lds_ok, r.lds_bytes, true, layered, multi ? 2u : 1u, r.dec_global);
        uint64_t total_items = 0, max_n = 0;
        for (const Seg& sg : r.segs) {
            total_items += bp_items(sg.g, sg.n);
            max_n = std::max<uint64_t>(max_n, sg.n);
        }
        r.grid = (int)std::min<uint64_t>((uint64_t)r.grid, std::max<uint64_t>(total_items, 1));
        if (!fp64 && !flood && !lds_ok && !layered && !multi && !dg)
            r.latency = total_items <= (uint64_t)r.grid &&
                        total_items <= (uint64_t)bp_grid_for(false, false, false, r.lds_bytes, true, false, 1u,
                                                             false, true);
        r.lsd_grid = (int)std::min<uint64_t>(512, std::max<uint64_t>(max_n, 1));
        // layout: [zeroed: counters | per-segment cmask, iters, qfix, fail count]
        //         [per-segment t_conv, weight, cand, fail_list] [segment table]
        //         [slabs] [posteriors] [LSD scratch]
        size_t off = 0;
        r.zero_off = off;
        off += 256;  // [0] BP ticket counter, then one fail count per segment at 4 * (1 + j)
        off += al256(4ull * r.segs.size());
        for (Seg& sg : r.segs) {
            const DevGraph& g = reqs[sg.req].graph->h.dg;
            sg.cmask = off;
            off += al256(8ull * sg.n * (kMaxT + 1));
            sg.iters = off;
            off += al256(4ull * sg.n);
            sg.qfix = off;
            off += al256(8ull * sg.n * g.n);
        }
        r.zero_bytes = off - r.zero_off;
        for (Seg& sg : r.segs) {
            const DevGraph& g = reqs[sg.req].graph->h.dg;
            sg.t_conv = off;
            off += al256(4ull * sg.n * g.L);
            sg.weight = off;
            off += al256(8ull * sg.n * g.L);
            sg.cand = off;
            off += al256(8ull * sg.n * g.L * g.words_n);
            sg.fail_list = off;
            off += al256(4ull * sg.n);
        }
        r.segs_off = off;
        off += al256(sizeof(BpSeg) * r.segs.size());
        const size_t mb = fp64 ? 8 : 4;
        r.slab_off = off;
        if (!lds_ok) off += al256(mb * (flood ? 2 : 1) * (size_t)r.grid * r.slab_elems);
        r.post_off = off;
        off += al256(mb * (size_t)r.grid * r.post_elems);
        r.lsd_off = off;
        off += al256(r.lsd_per_block * r.lsd_grid);
        r.bytes = off;
    }
    return rounds;
}

// The segment table of a round, for the device.
std::vector<BpSeg> seg_table(const vibe_request* reqs, const Round& r, unsigned char* base) {
    std::vector<BpSeg> t(r.segs.size());
    uint32_t item0 = 0;
    for (size_t j = 0; j < r.segs.size(); j++) {
        const Seg& sg = r.segs[j];
        const vibe_request& q = reqs[sg.req];
        const DevGraph& g = sg.g;
        BpSeg& b = t[j];
        std::memset(&b, 0, sizeof(b));
        b.g = g;
        b.item0 = item0;
        item0 += (uint32_t)bp_items(g, sg.n);
        BpLaunch& a = b.a;
        a.member_major = 1;
        a.syndromes = q.syndromes;
        a.shot0 = sg.shot0;
        a.n_shots = sg.n;
        a.T_run = g.T;
        a.use_M = 1;
        a.stop_on_converge = 1;
        a.accumulate_q = 1;
        a.fast_zero = 1;
        a.t_conv = reinterpret_cast<int32_t*>(base + sg.t_conv);
        a.weight = reinterpret_cast<double*>(base + sg.weight);
        a.cand = reinterpret_cast<uint64_t*>(base + sg.cand);
        a.post_out = nullptr;
        a.conv_mask = reinterpret_cast<uint64_t*>(base + sg.cmask);
        a.iters = reinterpret_cast<uint32_t*>(base + sg.iters);
        a.qfix = reinterpret_cast<int64_t*>(base + sg.qfix);
    }
    return t;
}

// Queue one round on `st`.  The segment table must already be on the device.
int run_round(const vibe_request* reqs, const Round& r, unsigned char* base, hipStream_t st) {
    int rc;
    if ((rc = launch_zero(base + r.zero_off, r.zero_bytes, st))) return rc;
    RaggedLaunch L{};
    L.segs = reinterpret_cast<const BpSeg*>(base + r.segs_off);
    L.n_segs = (uint32_t)r.segs.size();
    uint64_t items = 0;
    for (const Seg& sg : r.segs) items += bp_items(sg.g, sg.n);
    L.n_items = (uint32_t)items;
    L.slab = r.slab_in_lds ? nullptr : base + r.slab_off;
    L.post_slab = base + r.post_off;
    L.slab_elems = r.slab_elems;
    L.post_elems = r.post_elems;
    L.counter = reinterpret_cast<uint32_t*>(base + r.zero_off);
    L.grid = r.grid;
    L.slab_in_lds = r.slab_in_lds ? 1 : 0;
    L.fp64 = reqs[r.segs[0].req].graph->h.dg.fp64;
    L.flood = r.flood ? 1 : 0;
    L.multi = r.multi ? 1 : 0;
    L.layered = r.layered ? 1 : 0;
    L.dec_global = r.dec_global ? 1 : 0;
    L.latency = r.latency ? 1 : 0;
    L.lds_bytes = r.lds_bytes;
    if ((rc = launch_bp_ragged(L, st))) return rc;
    for (size_t j = 0; j < r.segs.size(); j++) {
        const Seg& sg = r.segs[j];
        const vibe_request& q = reqs[sg.req];
        const DevGraph& g = q.graph->h.dg;
        uint32_t* fail_count = reinterpret_cast<uint32_t*>(base + r.zero_off + 256) + j;
        SelectLaunch s{};
        s.n_shots = sg.n;
        s.shot0 = sg.shot0;
        s.t_conv = reinterpret_cast<const int32_t*>(base + sg.t_conv);
        s.weight = reinterpret_cast<const double*>(base + sg.weight);
        s.cand = reinterpret_cast<const uint64_t*>(base + sg.cand);
        s.iters = reinterpret_cast<const uint32_t*>(base + sg.iters);
        s.conv_mask = reinterpret_cast<const uint64_t*>(base + sg.cmask);
        s.corrections = q.corrections;
        s.stats = q.stats;
        s.fail_list = reinterpret_cast<uint32_t*>(base + sg.fail_list);
        s.fail_count = fail_count;
        if ((rc = launch_select(g, s, st))) return rc;
        LsdLaunch l{};
        l.syndromes = q.syndromes;
        l.shot0 = sg.shot0;
        l.list = s.fail_list;
        l.list_count = fail_count;
        l.n_list = sg.n;
        l.soft_f32 = nullptr;
        l.soft_fix = reinterpret_cast<const int64_t*>(base + sg.qfix);
        l.corrections = q.corrections;
        l.stats = q.stats;
        l.scratch = base + r.lsd_off;
        l.scratch_per_block = lsd_scratch_per_block(g);
        l.grid = std::min<int>(r.lsd_grid, (int)sg.n);
        if ((rc = launch_lsd(g, l, st))) return rc;
        if ((rc = launch_observables(g, q.corrections, sg.shot0, sg.n, q.observables, st))) return rc;
    }
    return VIBE_OK;
}

// per-shot buffers of one round: large batches of large codes run as few
// rounds (each ends in a launch tail) within a fraction of the 288 GB HBM
constexpr size_t kRaggedBudget = 32ull << 30;

}  // namespace

}  // namespace vibe

using namespace vibe;

extern "C" int vibe_runtime_create(vibe_runtime** out) {
    set_error("");
    if (!out) return fail(VIBE_EINVAL, "out is NULL");
    vibe_runtime* rt = new (std::nothrow) vibe_runtime();
    if (!rt) return fail(VIBE_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&rt->device);
    *out = rt;
    return VIBE_OK;
}

extern "C" void vibe_runtime_destroy(vibe_runtime* rt) {
    if (!rt) return;
    (void)hipDeviceSynchronize();
    if (rt->table_done) (void)hipEventDestroy(rt->table_done);
    if (rt->ws.base) (void)hipFree(rt->ws.base);
    delete rt;
}

extern "C" int vibe_decode_ragged(vibe_runtime* rt, const vibe_request* reqs, uint32_t n_reqs, void* stream) {
    set_error("");
    if (!rt) return fail(VIBE_EINVAL, "runtime is NULL");
    int rc = check_requests(reqs, n_reqs);
    if (rc) return rc;
    if (n_reqs && reqs[0].graph->device != rt->device) return fail(VIBE_EINVAL, "graphs and runtime on different devices");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<Round> rounds = plan(reqs, n_reqs, kRaggedBudget);
    size_t need = 0;
    for (const Round& r : rounds) need = std::max(need, r.bytes);
    if (!need) return VIBE_OK;
    if ((rc = grow(rt->ws, need))) return rc;
    unsigned char* base = static_cast<unsigned char*>(rt->ws.base);
    if (!rt->table_done) {
        hipError_t e = hipEventCreateWithFlags(&rt->table_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    for (const Round& r : rounds) {
        // the previous upload from the host table must have run before the
        // table is rewritten
        hipError_t e = hipEventSynchronize(rt->table_done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        rt->table = seg_table(reqs, r, base);
        e = hipMemcpyAsync(base + r.segs_off, rt->table.data(), sizeof(BpSeg) * rt->table.size(),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(segment table)");
        if ((e = hipEventRecord(rt->table_done, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((rc = run_round(reqs, r, base, st))) return rc;
    }
    return VIBE_OK;
}

extern "C" int vibe_exec_create(const vibe_request* reqs, uint32_t n_reqs, vibe_exec** out) {
    set_error("");
    if (!out) return fail(VIBE_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_requests(reqs, n_reqs);
    if (rc) return rc;
    if (!n_reqs) return fail(VIBE_EINVAL, "no requests");
    std::vector<Round> rounds = plan(reqs, n_reqs, kRaggedBudget);
    if (rounds.size() != 1) return fail(VIBE_EUNSUPPORTED, "the requests exceed one round's workspace budget");
    const Round& r = rounds[0];
    vibe_exec* ex = new (std::nothrow) vibe_exec();
    if (!ex) return fail(VIBE_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&ex->device);
    if ((rc = grow(ex->ws, r.bytes))) {
        delete ex;
        return rc;
    }
    unsigned char* base = static_cast<unsigned char*>(ex->ws.base);
    std::vector<BpSeg> t = seg_table(reqs, r, base);
    hipError_t e = hipMemcpy(base + r.segs_off, t.data(), sizeof(BpSeg) * t.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        vibe_exec_destroy(ex);
        return hip_fail(e, "hipMemcpy(segment table)");
    }
    hipStream_t cs = nullptr;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
        vibe_exec_destroy(ex);
        return hip_fail(e, "hipStreamCreate");
    }
    // every launch sets its LDS limit before capture begins
    rc = run_round(reqs, r, base, cs);
    if (!rc && (e = hipStreamSynchronize(cs)) != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    if (!rc && (e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        rc = hip_fail(e, "hipStreamBeginCapture");
    if (!rc) {
        rc = run_round(reqs, r, base, cs);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cs, &gr);
        if (!rc && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        ex->graph = gr;
        if (!rc && (e = hipGraphInstantiate(&ex->exec, gr, nullptr, nullptr, 0)) != hipSuccess)
            rc = hip_fail(e, "hipGraphInstantiate");
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
        vibe_exec_destroy(ex);
        return rc;
    }
    *out = ex;
    return VIBE_OK;
}

extern "C" int vibe_exec_launch(vibe_exec* ex, void* stream) {
    set_error("");
    if (!ex || !ex->exec) return fail(VIBE_EINVAL, "exec is NULL");
    hipError_t e = hipGraphLaunch(ex->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "hipGraphLaunch");
}

extern "C" void vibe_exec_destroy(vibe_exec* ex) {
    if (!ex) return;
    (void)hipDeviceSynchronize();
    if (ex->exec) (void)hipGraphExecDestroy(ex->exec);
    if (ex->graph) (void)hipGraphDestroy(ex->graph);
    if (ex->ws.base) (void)hipFree(ex->ws.base);
    delete ex;
}

namespace vibe {
namespace {

// Launch settings found by vibe_autotune, per graph shape and batch size
// class (process-wide): a graph of the same shape reuses them untimed.
struct TuneKey {
    int device;
    uint32_t m, n, E, L, M, T, chunks, levels, lsd_order;
    int fp64, flood, layered;
    uint32_t b_log2;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, m, n, E, L, M, T, chunks, levels, lsd_order, fp64, flood, layered, b_log2) <
               std::tie(o.device, o.m, o.n, o.E, o.L, o.M, o.T, o.chunks, o.levels, o.lsd_order, o.fp64, o.flood,
                        o.layered, o.b_log2);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, vibe_launch_t> g_tune_cache;

TuneKey tune_key(const vibe_graph* g, uint64_t B) {
    const DevGraph& d = g->h.dg;
    uint32_t lb = 0;
    while (lb < 63 && (2ull << lb) <= B) lb++;
    return TuneKey{g->device, d.m, d.n, d.E, d.L, d.M, d.T, g->h.chunks_max, g->h.levels_max, d.lsd_order,
                   d.fp64, d.flood, d.layered, lb};
}

// Whether P shots per wavefront are available for the graph (serial
// schedule, row state within 96 KB of LDS).
bool multi_ok(const vibe_graph* g, uint32_t P) {
    const DevGraph& d = g->h.dg;
    if (d.flood || d.layered) return false;
    DevGraph v = d;
    v.P = P;
    return bp_lds_bytes(v, false) <= 96 * 1024;
}

int apply_launch(vibe_graph* g, const vibe_launch_t& s) {
    const uint32_t P = (uint32_t)s.shots_per_wave;
    if (P != 1 && P != 2 && P != 4) return fail(VIBE_EINVAL, "shots_per_wave must be 1, 2 or 4");
    if (s.grid < 0) return fail(VIBE_EINVAL, "grid must be >= 0");
    if (s.decisions_global < -1 || s.decisions_global > 1) return fail(VIBE_EINVAL, "decisions_global must be -1, 0 or 1");
    if (s.decisions_global == 1 && s.slab_in_lds)
        return fail(VIBE_EINVAL, "decisions in global memory need the slab in global memory");
    if (s.decisions_global == 1 && g->h.dg.layered)
        return fail(VIBE_EUNSUPPORTED, "the layered schedule keeps its decisions in LDS");
    if (P > 1) {
        if (!multi_ok(g, P)) return fail(VIBE_EUNSUPPORTED, "several shots per wavefront need the serial schedule "
                                                             "and row states within 96 KB of LDS");
        if (s.slab_in_lds) return fail(VIBE_EINVAL, "several shots per wavefront keep the slab in global memory");
        int rc = build_multi_schedule(g, P);
        if (rc) return rc;
    }
    g->tune_lds = s.slab_in_lds ? 1 : 0;
    g->tune_grid = s.grid;
    g->tune_P = P;
    g->tune_dec = s.decisions_global;
    return VIBE_OK;
}

}  // namespace
}  // namespace vibe

extern "C" int vibe_set_launch(vibe_graph* g, const vibe_launch_t* s) {
    set_error("");
    if (!g || !s) return fail(VIBE_EINVAL, "NULL argument");
    return apply_launch(g, *s);
}

extern "C" int vibe_get_launch(const vibe_graph* g, vibe_launch_t* s) {
    set_error("");
    if (!g || !s) return fail(VIBE_EINVAL, "NULL argument");
    s->slab_in_lds = use_lds_slab(g, g->h.dg) ? 1 : 0;
    s->grid = g->tune_grid;
    s->shots_per_wave = (int)g->tune_P;
    s->decisions_global = g->tune_dec;
    s->from_cache = 0;
    s->ms = 0.0;
    return VIBE_OK;
}

extern "C" int vibe_autotune(vibe_graph* g, const uint8_t* syndromes, uint64_t B, void* stream, vibe_launch_t* out) {
    set_error("");
    if (!g || (B && !syndromes)) return fail(VIBE_EINVAL, "NULL argument");
    if (!B) return fail(VIBE_EINVAL, "B must be >= 1");
    const TuneKey key = tune_key(g, B);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            vibe_launch_t c = it->second;
            int rc = apply_launch(g, c);
            if (rc) return rc;
            c.from_cache = 1;
            if (out) *out = c;
            return VIBE_OK;
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGraph& d = g->h.dg;
    uint64_t* corr = nullptr;
    uint8_t* obs = nullptr;
    if (hipMalloc(&corr, 8 * B * d.words_n) != hipSuccess || hipMalloc(&obs, B * std::max<uint32_t>(d.k, 1)) != hipSuccess) {
        if (corr) (void)hipFree(corr);
        return fail(VIBE_ENOMEM, "autotune buffers");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int saved_lds = g->tune_lds, saved_grid = g->tune_grid, saved_dec = g->tune_dec;
    const uint32_t saved_P = g->tune_P;
    int rc = VIBE_OK;
    // decode time of the sample with setting s (the first of two runs warms
    // up); *skip: the setting could not be applied for want of memory (a
    // recut schedule), so it is no candidate
    auto time_it = [&](const vibe_launch_t& s, float* ms, bool* skip) {
        int r = apply_launch(g, s);
        *skip = r == VIBE_ENOMEM;
        if (*skip) return VIBE_OK;
        for (int rep = 0; rep < 2 && !r; rep++) {
            (void)hipEventRecord(e0, st);
            r = vibe_decode(g, syndromes, B, corr, obs, nullptr, stream);
            (void)hipEventRecord(e1, st);
            if (!r && hipEventSynchronize(e1) != hipSuccess) r = fail(VIBE_EHIP, "hipEventSynchronize");
            if (!r) (void)hipEventElapsedTime(ms, e0, e1);
        }
        return r;
    };
    // first the slab placement and shots per wavefront at full occupancy,
    // then the grid for the best of them
    std::vector<vibe_launch_t> first;
    if (bp_slab_fits_lds(d)) first.push_back(vibe_launch_t{1, 0, 1, 0, 0, 0.0});
    for (int P : {1, 2, 4})
        if (P == 1 || multi_ok(g, (uint32_t)P))
            for (int dec : {0, 1})
                if (!d.layered || dec == 0) first.push_back(vibe_launch_t{0, 0, P, dec, 0, 0.0});
    vibe_launch_t best{0, 0, 1, 0, 0, 1e30};
    bool timed = false;
    for (const vibe_launch_t& s : first) {
        float ms = 0.0f;
        bool skip = false;
        if ((rc = time_it(s, &ms, &skip))) break;
        if (skip) continue;
        timed = true;
        if (ms < best.ms) {
            best = s;
            best.ms = ms;
        }
    }
    if (!rc && !timed) rc = fail(VIBE_ENOMEM, "autotune: no launch setting could be applied");
    if (!rc) {
        (void)apply_launch(g, best);
        DevGraph v = decode_view(g, true, B);
        if (best.slab_in_lds) v.dec_global = 0;
        const int full = bp_grid(v, best.slab_in_lds != 0);
        const vibe_launch_t base = best;
        for (int eighths : {7, 6, 5, 4}) {
            vibe_launch_t s = base;
            s.grid = full * eighths / 8;
            if (s.grid < 1) continue;
            float ms = 0.0f;
            bool skip = false;
            if ((rc = time_it(s, &ms, &skip))) break;
            if (!skip && ms < best.ms) {
                best = s;
                best.ms = ms;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(corr);
    (void)hipFree(obs);
    if (rc) {
        g->tune_lds = saved_lds;
        g->tune_grid = saved_grid;
        g->tune_P = saved_P;
        g->tune_dec = saved_dec;
        return rc;
    }
    if ((rc = apply_launch(g, best))) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (out) *out = best;
    return VIBE_OK;
}

// ---------------------------------------------------------------------------
// Serving: continuous batching over resident graphs, admitted by footprint.
//
// The server owns one device pool of hbm_budget bytes.  Every batch holds
// requests on one graph, so a batch of a small code never waits for the
// long serial chains of a large one, and takes a block of the pool sized by
// its own footprint: the decode workspace of its shots (per-shot buffers;
// message and posterior slabs for a BP grid no larger than its items; LSD
// scratch), the staging of its syndromes and outputs, and its copy table.
// A server thread keeps up to `slots` batches in flight, each on its own
// stream.  Whenever a slot is free it takes the oldest queued request and,
// in order, the later queued requests on the same graph, while the batch
// still fits the largest free block of the pool (and the batch limits);
// if the oldest request does not fit yet it waits for batches to retire.
// The last free slot goes only to the cheapest graphs (per-shot work
// E x T x L within twice the smallest), so short batches never queue behind
// the long serial chains of large codes.
// Requests that arrive while others run are thus admitted as slots and
// memory free up, and their work overlaps on the device.

namespace {

using Clock = std::chrono::steady_clock;

struct SrvReq {
    uint64_t ticket;
    uint32_t gi;  // graph index
    vibe_request req;
    Clock::time_point t_submit;
};

struct SrvSlot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
    size_t blk_off = 0, blk_bytes = 0;  // the batch's block of the pool
    // host tables of the batch in flight (kept until the slot retires)
    std::vector<vibe::BpSeg> segs;
    std::vector<vibe::CopyEntry> copies;
};

struct SrvDone {
    bool done = false;
    int rc = VIBE_OK;
    double latency_ms = 0.0;
};

// First-fit allocator over the pool's byte range (host bookkeeping only).
struct PoolMap {
    std::map<size_t, size_t> free_;  // offset -> bytes, no two adjacent
    void reset(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    size_t largest() const {
        size_t b = 0;
        for (const auto& kv : free_) b = std::max(b, kv.second);
        return b;
    }
    bool take(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Where a batch of `shots` shots from `n_req` requests on one graph keeps
// its buffers, relative to its block.
struct BatchLayout {
    vibe::Round round;
    size_t synd = 0, corr = 0, obs = 0, stats = 0, tab = 0, bytes = 0;
    bool one_round = false;
};

BatchLayout batch_layout(vibe_graph* G, uint64_t shots, uint32_t n_req) {
    BatchLayout L;
    const vibe::DevGraph& g = G->h.dg;
    vibe_request r{};
    r.graph = G;
    r.syndromes = reinterpret_cast<const uint8_t*>(1);
    r.corrections = reinterpret_cast<uint64_t*>(1);
    r.observables = reinterpret_cast<uint8_t*>(1);
    r.B = std::max<uint64_t>(shots, 1);
    std::vector<vibe::Round> rs = vibe::plan(&r, 1, vibe::kRaggedBudget);
    L.one_round = rs.size() == 1;
    L.round = rs[0];
    size_t off = vibe::al256(L.round.bytes);
    L.synd = off;
    off += vibe::al256(r.B * g.m);
    L.corr = off;
    off += vibe::al256(r.B * 8ull * g.words_n);
    L.obs = off;
    off += vibe::al256(r.B * std::max<uint32_t>(g.k, 1));
    L.stats = off;
    off += vibe::al256(r.B * sizeof(vibe_shot_stats));
    L.tab = off;
    off += vibe::al256(sizeof(vibe::CopyEntry) * 4ull * std::max<uint32_t>(n_req, 1));
    L.bytes = off;
    return L;
}

}  // namespace

struct vibe_server {
    std::vector<vibe_graph*> graphs;
    vibe_server_config cfg{};
    int device = 0;
    std::vector<SrvSlot> slots;
    std::vector<bool> cheap;  // per graph: per-shot work within twice the smallest
    vibe::Workspace pool;
    PoolMap map;
    size_t in_use = 0, peak = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvReq> queue;
    std::unordered_map<uint64_t, SrvDone> status;
    std::unordered_map<uint64_t, Clock::time_point> t_submit;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    uint64_t batches = 0, requests = 0;
};

namespace {

void finish_tickets(vibe_server* S, const std::vector<uint64_t>& tickets, int rc) {
    const auto now = Clock::now();
    for (uint64_t t : tickets) {
        SrvDone& d = S->status[t];
        d.done = true;
        d.rc = rc;
        d.latency_ms = std::chrono::duration<double, std::milli>(now - S->t_submit[t]).count();
        S->t_submit.erase(t);
    }
    S->cv_done.notify_all();
}

void server_loop(vibe_server* S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<SrvReq> batch;
        int slot = -1;
        BatchLayout lay;
        size_t blk = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // retire finished batches and return their blocks to the pool
            for (SrvSlot& sl : S->slots) {
                if (!sl.busy) continue;
                hipError_t q = hipEventQuery(sl.done);
                if (q == hipErrorNotReady) continue;
                finish_tickets(S, sl.tickets, q == hipSuccess ? VIBE_OK : VIBE_EHIP);
                sl.tickets.clear();
                sl.busy = false;
                S->map.give(sl.blk_off, sl.blk_bytes);
                S->in_use -= sl.blk_bytes;
            }
            bool any_busy = false;
            for (size_t i = 0; i < S->slots.size(); i++) {
                if (!S->slots[i].busy && slot < 0) slot = (int)i;
                any_busy = any_busy || S->slots[i].busy;
            }
            if (S->stop && S->queue.empty() && !any_busy) return;
            size_t n_free = 0;
            for (const SrvSlot& sl2 : S->slots) n_free += sl2.busy ? 0 : 1;
            // the graph of the oldest request that may take the free slot:
            // the last free slot is kept for the cheapest graphs (per-shot
            // work E x T x L within twice the smallest), so that their short
            // batches never wait for the long serial chains of large codes
            size_t head = S->queue.size();
            for (size_t i = 0; i < S->queue.size(); i++) {
                if (n_free > 1 || S->slots.size() == 1 || S->cheap[S->queue[i].gi]) {
                    head = i;
                    break;
                }
            }
            if (slot >= 0 && head < S->queue.size()) {
                // that request's graph, then later requests on it in order,
                // while the batch fits the largest free block
                const uint32_t gi = S->queue[head].gi;
                vibe_graph* G = S->graphs[gi];
                const size_t room = S->map.largest();
                // candidates within the batch limits, then the longest
                // prefix of them whose footprint fits (it grows with the
                // prefix, so a binary search finds it)
                std::vector<size_t> pick;
                std::vector<uint64_t> upto;  // shots of the first k + 1 candidates
                uint64_t shots = 0;
                for (size_t i = head; i < S->queue.size() && pick.size() < S->cfg.max_batch_requests; i++) {
                    const SrvReq& r = S->queue[i];
                    if (r.gi != gi) continue;
                    if (!pick.empty() && shots + r.req.B > S->cfg.max_batch_shots) break;
                    pick.push_back(i);
                    shots += r.req.B;
                    upto.push_back(shots);
                }
                auto fits = [&](size_t k, BatchLayout* out) {  // the first k candidates
                    BatchLayout t = batch_layout(G, upto[k - 1], (uint32_t)k);
                    if (out) *out = t;
                    return t.one_round && t.bytes <= room;
                };
                size_t lo = 0, hi = pick.size();  // fits(lo) (or lo = 0), !fits(hi + 1)
                while (lo < hi) {
                    const size_t mid = (lo + hi + 1) / 2;
                    if (fits(mid, nullptr))
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                pick.resize(lo);
                if (lo) fits(lo, &lay);
                if (pick.empty() && !any_busy) {
                    // cannot happen for admitted requests (each fits the
                    // whole pool alone), kept as a guard against a stall
                    std::vector<uint64_t> t1{S->queue[head].ticket};
                    S->queue.erase(S->queue.begin() + (std::ptrdiff_t)head);
                    finish_tickets(S, t1, VIBE_ENOMEM);
                    continue;
                }
                if (!pick.empty() && S->map.take(lay.bytes, &blk)) {
                    std::deque<SrvReq> rest;
                    size_t k = 0;
                    for (size_t i = 0; i < S->queue.size(); i++) {
                        if (k < pick.size() && pick[k] == i) {
                            batch.push_back(S->queue[i]);
                            k++;
                        } else {
                            rest.push_back(S->queue[i]);
                        }
                    }
                    S->queue.swap(rest);
                    S->in_use += lay.bytes;
                    S->peak = std::max(S->peak, S->in_use);
                }
            }
            if (batch.empty()) {
                // wait for a submission, or poll the batches in flight
                S->cv_work.wait_for(lk, std::chrono::microseconds(any_busy ? 20 : 2000));
                continue;
            }
        }
        // Launch outside the lock: gather the batch's syndromes into one
        // contiguous block, decode it as one request, scatter the outputs
        // back to the requests' buffers.
        SrvSlot& sl = S->slots[slot];
        sl.blk_off = blk;
        sl.blk_bytes = lay.bytes;
        unsigned char* base = static_cast<unsigned char*>(S->pool.base) + blk;
        vibe_graph* Gr = S->graphs[batch[0].gi];
        const vibe::DevGraph& g = Gr->h.dg;
        sl.copies.clear();
        std::vector<vibe::CopyEntry> scatter;
        uint64_t rows = 0;
        for (const SrvReq& r : batch) {
            const uint64_t r0 = rows;
            rows += r.req.B;
            if (!r.req.B) continue;
            sl.copies.push_back({r.req.syndromes, base + lay.synd + r0 * g.m, r.req.B * g.m});
            const uint64_t cw = 8ull * g.words_n;
            scatter.push_back({base + lay.corr + r0 * cw, reinterpret_cast<unsigned char*>(r.req.corrections),
                               r.req.B * cw});
            if (g.k) scatter.push_back({base + lay.obs + r0 * g.k, r.req.observables, r.req.B * g.k});
            if (r.req.stats)
                scatter.push_back({base + lay.stats + r0 * sizeof(vibe_shot_stats),
                                   reinterpret_cast<unsigned char*>(r.req.stats), r.req.B * sizeof(vibe_shot_stats)});
        }
        const uint32_t n_gather = (uint32_t)sl.copies.size();
        sl.copies.insert(sl.copies.end(), scatter.begin(), scatter.end());
        int rc = VIBE_OK;
        if (rows) {
            vibe_request q{};
            q.graph = Gr;
            q.syndromes = base + lay.synd;
            q.B = rows;
            q.corrections = reinterpret_cast<uint64_t*>(base + lay.corr);
            q.observables = base + lay.obs;
            q.stats = reinterpret_cast<vibe_shot_stats*>(base + lay.stats);
            std::vector<vibe::Round> rounds = vibe::plan(&q, 1, vibe::kRaggedBudget);
            vibe::CopyEntry* dtab = reinterpret_cast<vibe::CopyEntry*>(base + lay.tab);
            if (rounds.size() != 1 || rounds[0].bytes > lay.round.bytes) {
                rc = vibe::fail(VIBE_ENOMEM, "internal: a batch outgrew its block");
            } else {
                const vibe::Round& rd = rounds[0];
                sl.segs = vibe::seg_table(&q, rd, base);
                hipError_t e = hipMemcpyAsync(dtab, sl.copies.data(), sizeof(vibe::CopyEntry) * sl.copies.size(),
                                              hipMemcpyHostToDevice, sl.st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(base + rd.segs_off, sl.segs.data(), sizeof(vibe::BpSeg) * sl.segs.size(),
                                       hipMemcpyHostToDevice, sl.st);
                if (e != hipSuccess) rc = vibe::hip_fail(e, "hipMemcpyAsync(server tables)");
                if (!rc) rc = vibe::launch_copies(dtab, n_gather, sl.st);
                if (!rc) rc = vibe::run_round(&q, rd, base, sl.st);
                if (!rc) rc = vibe::launch_copies(dtab + n_gather, (uint32_t)scatter.size(), sl.st);
            }
        }
        std::unique_lock<std::mutex> lk(S->mu);
        if (rc) {
            // the stream may still hold work of this batch: wait before the
            // block goes back to the pool
            (void)hipStreamSynchronize(sl.st);
            std::vector<uint64_t> ts;
            for (const SrvReq& r : batch) ts.push_back(r.ticket);
            finish_tickets(S, ts, rc);
            S->map.give(sl.blk_off, sl.blk_bytes);
            S->in_use -= sl.blk_bytes;
            continue;
        }
        (void)hipEventRecord(sl.done, sl.st);
        for (const SrvReq& r : batch) sl.tickets.push_back(r.ticket);
        sl.busy = true;
        S->batches++;
        S->requests += batch.size();
    }
}

}  // namespace

extern "C" int vibe_server_create(vibe_graph* const* graphs, uint32_t n_graphs, const vibe_server_config* cfg,
                                  vibe_server** out) {
    set_error("");
    if (!out || !graphs || !n_graphs || !cfg) return fail(VIBE_EINVAL, "NULL argument");
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 16) return fail(VIBE_EINVAL, "slots must be in 1..16");
    if (cfg->max_batch_shots < 1 || cfg->max_batch_requests < 1) return fail(VIBE_EINVAL, "batch limits must be >= 1");
    for (uint32_t i = 0; i < n_graphs; i++) {
        if (!graphs[i]) return fail(VIBE_EINVAL, "a graph is NULL");
        const DevGraph& g = graphs[i]->h.dg;
        const DevGraph& g0 = graphs[0]->h.dg;
        if (g.fp64 != g0.fp64) return fail(VIBE_EINVAL, "all graphs of a server need the same message_bits");
        if (graphs[i]->device != graphs[0]->device) return fail(VIBE_EINVAL, "all graphs must be on one device");
    }
    // the pool: hbm_budget, or room for `slots` full batches of the graph
    // with the largest full batch
    size_t pool = cfg->hbm_budget;
    if (!pool) {
        size_t worst = 0;
        for (uint32_t i = 0; i < n_graphs; i++) {
            uint64_t b = cfg->max_batch_shots;
            BatchLayout L = batch_layout(graphs[i], b, cfg->max_batch_requests);
            while (!L.one_round && b > 1) L = batch_layout(graphs[i], b /= 2, cfg->max_batch_requests);
            worst = std::max(worst, L.bytes);
        }
        pool = worst * cfg->slots;
    }
    vibe_server* S = new (std::nothrow) vibe_server();
    if (!S) return fail(VIBE_ENOMEM, "host allocation failed");
    S->graphs.assign(graphs, graphs + n_graphs);
    S->cfg = *cfg;
    S->device = graphs[0]->device;
    S->slots.resize(cfg->slots);
    {
        double least = 0.0;
        std::vector<double> work(n_graphs);
        for (uint32_t i = 0; i < n_graphs; i++) {
            const DevGraph& g = graphs[i]->h.dg;
            work[i] = (double)g.E * g.T * g.L;
            least = i ? std::min(least, work[i]) : work[i];
        }
        S->cheap.resize(n_graphs);
        for (uint32_t i = 0; i < n_graphs; i++) S->cheap[i] = work[i] <= 2.0 * least;
    }
    int rc = grow(S->pool, pool);
    if (!rc) S->map.reset(S->pool.bytes);
    for (SrvSlot& sl : S->slots) {
        if (rc) break;
        hipError_t e;
        // default priority: streams of other priorities are avoided on purpose
        if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
            rc = hip_fail(e, "server stream or event");
    }
    if (rc) {
        for (SrvSlot& sl : S->slots) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.st) (void)hipStreamDestroy(sl.st);
        }
        if (S->pool.base) (void)hipFree(S->pool.base);
        delete S;
        return rc;
    }
    S->th = std::thread(server_loop, S);
    *out = S;
    return VIBE_OK;
}

extern "C" int vibe_server_submit(vibe_server* S, uint32_t graph_index, const uint8_t* syndromes, uint64_t B,
                                  uint64_t* corrections, uint8_t* observables, vibe_shot_stats* stats,
                                  uint64_t* ticket) {
    set_error("");
    if (!S || !ticket) return fail(VIBE_EINVAL, "NULL argument");
    if (graph_index >= S->graphs.size()) return fail(VIBE_EINVAL, "graph_index out of range");
    if (B > S->cfg.max_batch_shots) return fail(VIBE_EINVAL, "a request is larger than max_batch_shots");
    vibe_request r{};
    r.graph = S->graphs[graph_index];
    r.syndromes = syndromes;
    r.B = B;
    r.corrections = corrections;
    r.observables = observables;
    r.stats = stats;
    int rc = check_requests(&r, 1);
    if (rc) return rc;
    // admission by footprint: the request alone must fit the pool (and one
    // round of per-shot buffers); it is queued until that much is free
    const BatchLayout L = batch_layout(r.graph, B, 1);
    if (!L.one_round) return fail(VIBE_EINVAL, "a request needs more than one round of per-shot buffers");
    if (L.bytes > S->pool.bytes)
        return fail(VIBE_ENOMEM, "the request's footprint (" + std::to_string(L.bytes) +
                                     " bytes) exceeds the server's HBM pool (" + std::to_string(S->pool.bytes) +
                                     " bytes)");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(VIBE_EINVAL, "the server is shutting down");
    const uint64_t t = S->next_ticket++;
    const auto now = Clock::now();
    S->queue.push_back(SrvReq{t, graph_index, r, now});
    S->t_submit[t] = now;
    S->status[t] = SrvDone{};
    *ticket = t;
    S->cv_work.notify_one();
    return VIBE_OK;
}

extern "C" int vibe_server_wait(vibe_server* S, uint64_t ticket, double* latency_ms) {
    set_error("");
    if (!S) return fail(VIBE_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->status.find(ticket);
    if (it == S->status.end()) return fail(VIBE_EINVAL, "unknown ticket");
    S->cv_done.wait(lk, [&] { return S->status[ticket].done; });
    const SrvDone d = S->status[ticket];
    S->status.erase(ticket);
    if (latency_ms) *latency_ms = d.latency_ms;
    if (d.rc) return fail(d.rc, "the batch of this request failed");
    return VIBE_OK;
}

extern "C" int vibe_server_info(vibe_server* S, uint64_t* batches, uint64_t* requests, uint64_t* pool_bytes,
                                uint64_t* peak_bytes) {
    if (!S) return fail(VIBE_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (batches) *batches = S->batches;
    if (requests) *requests = S->requests;
    if (pool_bytes) *pool_bytes = S->pool.bytes;
    if (peak_bytes) *peak_bytes = S->peak;
    return VIBE_OK;
}

extern "C" void vibe_server_destroy(vibe_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    for (SrvSlot& sl : S->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    if (S->pool.base) (void)hipFree(S->pool.base);
    delete S;
}
