// Ragged batching, captured launch sequences and autotuning.
//
// A ragged call decodes several requests, possibly on graphs of different
// codes, with one persistent BP launch over all of their (shot, member)
// items, then selection, LSD and observables per request.  Per request the
// results are those of vibe_decode on that request alone: every kernel's
// output for a shot depends only on that shot's syndrome and graph.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

struct vibe_runtime {
    int device = 0;
    vibe::Workspace ws;
};

struct vibe_exec {
    int device = 0;
    vibe::Workspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace vibe {

namespace {

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
        if (g.fp64 != g0.fp64 || g.flood != g0.flood)
            return fail(VIBE_EINVAL, "all graphs of a ragged call need the same message_bits and schedule");
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
        bool lds_ok = true;
        bool fp64 = false, flood = false;
        size_t lds_global = 0, lds_l = 0;
        for (const Seg& sg : r.segs) {
            const vibe_graph* G = reqs[sg.req].graph;
            const DevGraph& g = G->h.dg;
            fp64 = g.fp64 != 0;
            flood = g.flood != 0;
            r.slab_elems = std::max<uint32_t>(r.slab_elems, std::max<uint32_t>(g.max_chunks, 1) * kWave);
            r.post_elems = std::max<uint32_t>(r.post_elems, g.n + kWave);
            lds_ok = lds_ok && bp_slab_fits_lds(g) && G->tune_lds != 0;
            lds_global = std::max(lds_global, bp_lds_bytes(g, false));
            lds_l = std::max(lds_l, bp_lds_bytes(g, true));
            r.lsd_per_block = std::max(r.lsd_per_block, lsd_scratch_per_block(g));
        }
        r.slab_in_lds = lds_ok;
        r.lds_bytes = lds_ok ? lds_l : lds_global;
        r.grid = bp_grid_for(fp64, flood, lds_ok, r.lds_bytes, true);
        uint64_t total_items = 0, max_n = 0;
        for (const Seg& sg : r.segs) {
            total_items += (uint64_t)sg.n * reqs[sg.req].graph->h.dg.L;
            max_n = std::max<uint64_t>(max_n, sg.n);
        }
        r.grid = (int)std::min<uint64_t>((uint64_t)r.grid, std::max<uint64_t>(total_items, 1));
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
        const DevGraph& g = q.graph->h.dg;
        BpSeg& b = t[j];
        std::memset(&b, 0, sizeof(b));
        b.g = g;
        b.item0 = item0;
        item0 += sg.n * g.L;
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
    for (const Seg& sg : r.segs) items += (uint64_t)sg.n * reqs[sg.req].graph->h.dg.L;
    L.n_items = (uint32_t)items;
    L.slab = r.slab_in_lds ? nullptr : base + r.slab_off;
    L.post_slab = base + r.post_off;
    L.slab_elems = r.slab_elems;
    L.post_elems = r.post_elems;
    L.counter = reinterpret_cast<uint32_t*>(base + r.zero_off);
    L.grid = r.grid;
    L.slab_in_lds = r.slab_in_lds ? 1 : 0;
    L.fp64 = reqs[r.segs[0].req].graph->h.dg.fp64;
    L.flood = reqs[r.segs[0].req].graph->h.dg.flood;
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

constexpr size_t kRaggedBudget = 4ull << 30;  // per-shot buffers of one round

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
    for (const Round& r : rounds) {
        std::vector<BpSeg> t = seg_table(reqs, r, base);
        // pageable source: the call returns once the table has been taken
        hipError_t e = hipMemcpyAsync(base + r.segs_off, t.data(), sizeof(BpSeg) * t.size(), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(segment table)");
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

extern "C" int vibe_autotune(vibe_graph* g, const uint8_t* syndromes, uint64_t B, void* stream, int* slab_in_lds,
                             int* grid) {
    set_error("");
    if (!g || (B && !syndromes)) return fail(VIBE_EINVAL, "NULL argument");
    if (!B) return fail(VIBE_EINVAL, "B must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const DevGraph& d = g->h.dg;
    const uint64_t words = d.words_n;
    uint64_t* corr = nullptr;
    uint8_t* obs = nullptr;
    if (hipMalloc(&corr, 8 * B * words) != hipSuccess || hipMalloc(&obs, B * std::max<uint32_t>(d.k, 1)) != hipSuccess) {
        if (corr) (void)hipFree(corr);
        return fail(VIBE_ENOMEM, "autotune buffers");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int saved_lds = g->tune_lds, saved_grid = g->tune_grid;
    const bool fits = bp_slab_fits_lds(d);
    int best_lds = fits ? 1 : 0, best_grid = 0, rc = VIBE_OK;
    float best_ms = 1e30f;
    for (int lds = fits ? 1 : 0; lds >= 0 && !rc; lds--) {
        const int full = bp_grid(d, lds != 0);
        const int cand[3] = {full, (full * 3) / 4, full / 2};
        for (int c = 0; c < 3 && !rc; c++) {
            if (cand[c] < 1) continue;
            g->tune_lds = lds;
            g->tune_grid = cand[c];
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && !rc; rep++) {  // the first run warms up
                (void)hipEventRecord(e0, st);
                rc = vibe_decode(g, syndromes, B, corr, obs, nullptr, stream);
                (void)hipEventRecord(e1, st);
                if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(VIBE_EHIP, "hipEventSynchronize");
                if (!rc) (void)hipEventElapsedTime(&ms, e0, e1);
            }
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best_lds = lds;
                best_grid = cand[c];
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
        return rc;
    }
    g->tune_lds = best_lds;
    g->tune_grid = best_grid;
    if (slab_in_lds) *slab_in_lds = best_lds;
    if (grid) *grid = best_grid;
    return VIBE_OK;
}
