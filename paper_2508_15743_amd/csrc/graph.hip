// Offline stage (paper Sec. III.D.1): validate the detector error model, derive
// the channel LLRs, build the member schedules and upload everything once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <queue>

#include "internal.h"

namespace vibe {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(VIBE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

template <class T>
int upload(GraphHost& h, const T* src, size_t count, const T** dst) {
    if (count == 0) count = 1;  // keep every pointer valid
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(T) * count);
    if (e != hipSuccess) return fail(VIBE_ENOMEM, "hipMalloc of graph data failed");
    h.allocations.push_back(p);
    h.device_bytes += sizeof(T) * count;
    if (src) {
        e = hipMemcpy(p, src, sizeof(T) * count, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy of graph data");
    }
    *dst = static_cast<const T*>(p);
    return VIBE_OK;
}

void free_all(GraphHost& h) {
    for (void* p : h.allocations) (void)hipFree(p);
    h.allocations.clear();
}

}  // namespace

// Decode schedules for P = 2 or 4 shots per wavefront.  The 64-edge chunks
// are recut into chunks of at most W = 64 / P edges, columns kept whole and
// in slot order; a subset of an independent set of columns is independent,
// so the sweep computes the same messages.  Two edges of one row lie in
// different 64-edge chunks, whose order the recut keeps, so the suffix
// state of every slot for the initial messages (the row's later edges) is
// the one of the 64-edge schedule and is copied over.  Each recut chunk
// carries its own largest column degree.
int build_multi_schedule(vibe_graph* G, uint32_t P) {
    if (P != 2 && P != 4) return fail(VIBE_EINVAL, "shots per wavefront must be 1, 2 or 4");
    const uint32_t idx = P / 4;
    if (G->multi_recs[idx]) return VIBE_OK;
    const DevGraph& d = G->h.dg;
    if (d.layered) return fail(VIBE_EUNSUPPORTED, "the layered schedule runs one shot per wavefront");
    const bool f64 = d.fp64 != 0;
    const uint32_t W = kWave / P, L = d.L, mb = f64 ? 8u : 4u;
    std::vector<uint32_t> mc(L + 1);
    hipError_t e = hipMemcpy(mc.data(), d.member_chunk, 4ull * (L + 1), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(member_chunk)");
    const size_t nrec = mc[L];
    const uint32_t rb = rec_bytes(f64), ri0 = rec_init(f64), wrb = rec_bytes_w(f64, W);
    std::vector<unsigned char> recs(std::max<size_t>(nrec, 1) * rb);
    if (nrec && (e = hipMemcpy(recs.data(), d.sched, nrec * rb, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(schedule)");
    std::vector<unsigned char> out;
    std::vector<uint32_t> gmc(L + 1, 0);
    std::vector<std::pair<uint32_t, uint32_t>> cols;  // (first slot, degree)
    uint32_t maxc = 0;
    for (uint32_t i = 0; i < L; i++) {
        gmc[i] = (uint32_t)(out.size() / wrb);
        for (size_t k = mc[i]; k < mc[i + 1]; k++) {
            const unsigned char* r = recs.data() + k * rb;
            uint32_t meta[kWave], vv[kWave];
            std::memcpy(meta, r, sizeof(meta));
            std::memcpy(vv, r + kRecV, sizeof(vv));
            cols.clear();
            for (uint32_t q = 0; q < (uint32_t)kWave;) {
                const uint32_t deg = (meta[q] >> kMetaDegShift) & 15u;
                if (!deg) break;
                cols.push_back({q, deg});
                q += deg;
            }
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
                out.resize(at + wrb, 0);
                unsigned char* o = out.data() + at;
                uint32_t slot = 0;
                auto put = [&](uint32_t mw, uint32_t v, const unsigned char* lam, const void* init) {
                    std::memcpy(o + 4 * slot, &mw, 4);
                    std::memcpy(o + 4 * W + 4 * slot, &v, 4);
                    if (lam) std::memcpy(o + 8 * W + mb * slot, lam, mb);
                    std::memcpy(o + 8 * W + mb * W + mb * slot, init, mb);
                    slot++;
                };
                for (size_t cc = a; cc < b; cc++)
                    for (uint32_t j = 0; j < cols[cc].second; j++) {
                        const uint32_t q = cols[cc].first + j;
                        put((meta[q] & ~(15u << kMetaDmaxShift)) | (dmax << kMetaDmaxShift), vv[q],
                            r + kRecLam + mb * q, r + ri0 + mb * q);
                    }
                while (slot < W)  // unused slots: c = v = 0, lambda 0, no message
                    put(dmax << kMetaDmaxShift, 0u, nullptr, f64 ? (const void*)&d.ident64 : (const void*)&d.ident32);
                a = b;
            }
        }
        maxc = std::max(maxc, (uint32_t)(out.size() / wrb) - gmc[i]);
    }
    gmc[L] = (uint32_t)(out.size() / wrb);
    if (out.empty()) {  // no edges: one unused record
        out.assign(wrb, 0);
        for (uint32_t q = 0; q < W; q++)
            std::memcpy(out.data() + 8 * W + mb * W + mb * q, f64 ? (const void*)&d.ident64 : (const void*)&d.ident32, mb);
    }
    const unsigned char* dr = nullptr;
    const uint32_t* dm = nullptr;
    int rc;
    if ((rc = upload(G->h, out.data(), out.size(), &dr)) || (rc = upload(G->h, gmc.data(), gmc.size(), &dm)))
        return rc;
    G->multi_recs[idx] = dr;
    G->multi_member_chunk[idx] = dm;
    G->multi_max_chunks[idx] = maxc;
    return VIBE_OK;
}

DevGraph decode_view(const vibe_graph* G, bool allow_multi, uint64_t shots) {
    DevGraph d = G->h.dg;
    const uint32_t P = G->tune_P;
    if (allow_multi && (P == 2 || P == 4) && G->multi_recs[P / 4]) {
        d.sched = G->multi_recs[P / 4];
        d.member_chunk = G->multi_member_chunk[P / 4];
        d.max_chunks = G->multi_max_chunks[P / 4];
        d.P = P;
    }
    if (!d.layered) {
        if (G->tune_dec >= 0) {
            d.dec_global = G->tune_dec;
        } else {
            // automatic: only a launch with more items than fit at once with
            // the decisions in LDS gains from more residency (a small batch
            // is bound by its chains, which the global masks lengthen)
            d.dec_global = 0;
            const uint64_t items = shots == UINT64_MAX ? UINT64_MAX : bp_items(d, shots);
            if (items > (uint64_t)bp_grid(d, false) && dec_global_pays(d)) d.dec_global = 1;
        }
    }
    return d;
}

}  // namespace vibe

using namespace vibe;

extern "C" const char* vibe_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* vibe_version(void) { return "vibelsd-gfx950 0.1.0"; }

extern "C" int vibe_graph_create(uint32_t m, uint32_t n, const uint32_t* h_indptr,
                                 const uint32_t* h_indices, const double* priors, uint32_t k,
                                 const uint32_t* l_indptr, const uint32_t* l_indices,
                                 const uint32_t* perms, const vibe_config* cfg, vibe_graph** out) {
    set_error("");
    if (!out) return fail(VIBE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!h_indptr || !priors || !perms || !cfg || (k && !l_indptr))
        return fail(VIBE_EINVAL, "a required pointer is NULL");
    if (n == 0) return fail(VIBE_EINVAL, "n must be >= 1");
    if (m >= 65536u) return fail(VIBE_EUNSUPPORTED, "m must be < 65536");
    if (n >= (1u << 24)) return fail(VIBE_EUNSUPPORTED, "n must be < 2^24");
    const vibe_config c = *cfg;
    if (c.L < 1 || c.L > (uint32_t)kMaxL) return fail(VIBE_EINVAL, "L must be in 1..64");
    if (c.M < 1 || c.M > c.L) return fail(VIBE_EINVAL, "M must be in 1..L");
    if (c.T_max < 1 || c.T_max > (uint32_t)kMaxT) return fail(VIBE_EINVAL, "T_max must be in 1..64");
    if (c.lsd_order > kMaxLsdOrder) return fail(VIBE_EINVAL, "lsd_order must be in 0..64");
    if (!(c.alpha > 0.0) || !(c.alpha <= 1e6)) return fail(VIBE_EINVAL, "alpha must be in (0, 1e6]");
    if (!(c.clamp >= 1.0) || !(c.clamp <= 1e30)) return fail(VIBE_EINVAL, "clamp must be in [1, 1e30]");
    if (c.message_bits != 0 && c.message_bits != 32 && c.message_bits != 64)
        return fail(VIBE_EINVAL, "message_bits must be 0, 32 or 64");
    if (c.schedule > 2) return fail(VIBE_EINVAL, "schedule must be 0 (serial), 1 (parallel) or 2 (layered)");
    const bool layered = c.schedule == 2;
    if (m && (size_t)m * (c.message_bits == 64 ? 8 : 4) + 8 * (2 * (size_t)((m + 63) / 64) + (n + 63) / 64) >
                 150 * 1024)
        return fail(VIBE_EUNSUPPORTED, "per-decoder LDS state exceeds 150 KB");

    // ---- H in CSR: validate
    if (h_indptr[0] != 0) return fail(VIBE_EINVAL, "h_indptr[0] must be 0");
    for (uint32_t r = 0; r < m; r++)
        if (h_indptr[r + 1] < h_indptr[r]) return fail(VIBE_EINVAL, "h_indptr must be non-decreasing");
    const uint64_t E = h_indptr[m];
    if (E >= (1ull << 31)) return fail(VIBE_EUNSUPPORTED, "nnz must be < 2^31");
    if (E && !h_indices) return fail(VIBE_EINVAL, "h_indices is NULL");
    uint32_t max_row = 0;
    for (uint32_t r = 0; r < m; r++) {
        uint32_t lo = h_indptr[r], hi = h_indptr[r + 1];
        if (hi - lo >= 65536u) return fail(VIBE_EUNSUPPORTED, "a row has >= 65536 entries");
        max_row = std::max(max_row, hi - lo);
        for (uint32_t a = lo; a < hi; a++) {
            if (h_indices[a] >= n) return fail(VIBE_EINVAL, "a column index is >= n");
            if (a > lo && h_indices[a] <= h_indices[a - 1])
                return fail(VIBE_EINVAL, "column indices must be strictly ascending in each row");
        }
    }
    for (uint32_t v = 0; v < n; v++)
        if (!(priors[v] > 0.0 && priors[v] < 1.0))
            return fail(VIBE_EINVAL, "every prior must lie strictly between 0 and 1");
    if (k) {
        if (l_indptr[0] != 0) return fail(VIBE_EINVAL, "l_indptr[0] must be 0");
        for (uint32_t r = 0; r < k; r++) {
            if (l_indptr[r + 1] < l_indptr[r]) return fail(VIBE_EINVAL, "l_indptr must be non-decreasing");
            for (uint32_t a = l_indptr[r]; a < l_indptr[r + 1]; a++)
                if (!l_indices || l_indices[a] >= n) return fail(VIBE_EINVAL, "bad observable column");
        }
    }
    // ---- permutations: of the n columns, or of the m checks (layered)
    {
        const uint32_t len = layered ? m : n;
        std::vector<uint8_t> seen(len);
        for (uint32_t i = 0; i < c.L; i++) {
            std::fill(seen.begin(), seen.end(), 0);
            for (uint32_t a = 0; a < len; a++) {
                uint32_t v = perms[(size_t)i * len + a];
                if (v >= len || seen[v])
                    return fail(VIBE_EINVAL, layered ? "perms rows must be permutations of 0..m-1 (layered)"
                                                     : "perms rows must be permutations of 0..n-1");
                seen[v] = 1;
            }
        }
    }

    // ---- CSC with the CSR position of every edge
    std::vector<uint32_t> cp(n + 1, 0), ci(E), ce(E);
    for (uint64_t a = 0; a < E; a++) cp[h_indices[a] + 1]++;
    for (uint32_t v = 0; v < n; v++) cp[v + 1] += cp[v];
    {
        std::vector<uint32_t> fill(cp.begin(), cp.end() - 1);
        for (uint32_t r = 0; r < m; r++)
            for (uint32_t a = h_indptr[r]; a < h_indptr[r + 1]; a++) {
                uint32_t v = h_indices[a];
                ci[fill[v]] = r;  // rows visited ascending -> checks ascending per column
                ce[fill[v]] = a;
                fill[v]++;
            }
    }
    uint32_t max_col = 0;
    for (uint32_t v = 0; v < n; v++) max_col = std::max(max_col, cp[v + 1] - cp[v]);
    if (max_col > (uint32_t)kMaxColDeg) return fail(VIBE_EUNSUPPORTED, "a column is in more than 15 checks");

    // ---- channel LLRs, in FP64 with the C library's log
    const double lim = c.clamp;
    const bool fp64 = c.message_bits == 64;
    std::vector<double> lam64(n);
    std::vector<float> lam32(n);
    int all_pos = 1;
    for (uint32_t v = 0; v < n; v++) {
        double l = std::log((1.0 - priors[v]) / priors[v]);
        l = std::min(std::max(l, -lim), lim);
        lam64[v] = l;
        lam32[v] = (float)l;
        if (!(fp64 ? l > 0.0 : lam32[v] > 0.0f)) all_pos = 0;
    }
    const uint32_t words_n = (n + 63) / 64, words_m = (m + 63) / 64;
    std::vector<uint64_t> e0(words_n, 0);
    for (uint32_t v = 0; v < n; v++)
        if (cp[v + 1] == cp[v] && !(fp64 ? lam64[v] > 0.0 : lam32[v] > 0.0f)) e0[v / 64] |= 1ull << (v % 64);
    std::vector<uint64_t> lobs((size_t)std::max<uint32_t>(k, 1) * words_n, 0);
    for (uint32_t r = 0; r < k; r++)
        for (uint32_t a = l_indptr[r]; a < l_indptr[r + 1]; a++) {
            uint32_t v = l_indices[a];
            lobs[(size_t)r * words_n + v / 64] ^= 1ull << (v % 64);
        }
    // row states (magnitude bits with the sign of the message as parity)
    auto enc32 = [](float x) -> uint32_t {
        float a = std::fabs(x);
        uint32_t bits;
        std::memcpy(&bits, &a, 4);
        return bits | (x < 0.0f ? 0x80000000u : 0u);
    };
    auto enc64 = [](double x) -> uint64_t {
        double a = std::fabs(x);
        uint64_t bits;
        std::memcpy(&bits, &a, 8);
        return bits | (x < 0.0 ? 1ull << 63 : 0ull);
    };
    const float limf = (float)lim;
    uint32_t ident32;
    uint64_t ident64;
    std::memcpy(&ident32, &limf, 4);
    std::memcpy(&ident64, &lim, 8);

    // ---- member schedules (Sec. III.D.1: one fixed serial order per member).
    //      Two columns that share a check must keep their permutation order:
    //      the later one reads the earlier one's new message, and the earlier
    //      one reads the later one's previous message.  Columns that share no
    //      check commute.  So the sweep is any topological order of the DAG
    //      whose arcs join consecutive columns of each row, cut into chunks
    //      of columns that are mutually independent.  Chunks are packed by
    //      list scheduling (ready columns by decreasing height, the longest
    //      chain of successors below them, then by permutation position) into
    //      at most 64 edges each, which reaches max(#levels, ceil(E / 64))
    //      chunks on the workloads here.
    std::vector<uint32_t> s_meta, s_v, init32;
    std::vector<float> s_lam32;
    std::vector<double> s_lam64;
    std::vector<uint64_t> init64;
    std::vector<uint32_t> member_chunk(c.L + 1, 0);
    uint32_t lev_min = UINT32_MAX, lev_max = 0, ch_min = UINT32_MAX, ch_max = 0;
    {
        const uint32_t kNone = UINT32_MAX;
        std::vector<uint32_t> last(m), level(n), height(n), npred(n), pos(n), succ(E);
        std::vector<uint32_t> taken;
        std::vector<uint64_t> skipped;
        std::vector<uint32_t> running32(m);
        std::vector<uint64_t> running64(m);
        size_t nchunks = 0;
        for (uint32_t i = 0; i < (layered ? 0u : c.L); i++) {  // the layered schedule has no chunks
            const uint32_t* pi = perms + (size_t)i * n;
            std::fill(last.begin(), last.end(), kNone);
            std::fill(succ.begin(), succ.end(), kNone);
            uint32_t nlev = 0, ncols = 0;
            for (uint32_t a = 0; a < n; a++) {
                const uint32_t v = pi[a];
                pos[v] = a;
                npred[v] = 0;
                uint32_t lv = 0;
                for (uint32_t j = cp[v]; j < cp[v + 1]; j++) {
                    const uint32_t r = ci[j], u = last[r];
                    if (u != kNone) {
                        // arc u -> v through row r; u's edge on r is the one
                        // whose check is r
                        uint32_t ju = cp[u];
                        while (ci[ju] != r) ju++;
                        succ[ju] = v;
                        bool dup = false;
                        for (uint32_t j2 = cp[v]; j2 < j; j2++) dup |= last[ci[j2]] == u;
                        if (!dup) npred[v]++;
                        lv = std::max(lv, level[u]);
                    }
                }
                for (uint32_t j = cp[v]; j < cp[v + 1]; j++) last[ci[j]] = v;
                level[v] = lv + 1;
                if (cp[v + 1] > cp[v]) {
                    nlev = std::max(nlev, level[v]);
                    ncols++;
                }
            }
            for (uint32_t a = n; a-- > 0;) {
                const uint32_t u = pi[a];
                uint32_t h = 0;
                for (uint32_t j = cp[u]; j < cp[u + 1]; j++)
                    if (succ[j] != kNone) h = std::max(h, height[succ[j]]);
                height[u] = h + 1;
            }
            lev_min = std::min(lev_min, nlev);
            lev_max = std::max(lev_max, nlev);
            // ready queue keyed by (larger height, earlier position)
            auto key = [&](uint32_t v) { return ((uint64_t)(~height[v]) << 32) | pos[v]; };
            std::priority_queue<uint64_t, std::vector<uint64_t>, std::greater<uint64_t>> ready;
            for (uint32_t a = 0; a < n; a++) {
                const uint32_t v = pi[a];
                if (cp[v + 1] > cp[v] && npred[v] == 0) ready.push(key(v));
            }
            member_chunk[i] = (uint32_t)nchunks;
            const size_t first_slot = nchunks * kWave;
            uint32_t placed = 0;
            while (!ready.empty()) {
                uint32_t cap = kWave, dmax = 0;
                taken.clear();
                skipped.clear();
                while (!ready.empty() && cap > 0 && skipped.size() < (size_t)kWave) {
                    const uint64_t kv = ready.top();
                    ready.pop();
                    const uint32_t v = pi[(uint32_t)kv];
                    const uint32_t d = cp[v + 1] - cp[v];
                    if (d <= cap) {
                        taken.push_back(v);
                        cap -= d;
                        dmax = std::max(dmax, d);
                    } else {
                        skipped.push_back(kv);
                    }
                }
                for (uint64_t kv : skipped) ready.push(kv);
                for (uint32_t v : taken) {
                    const uint32_t d = cp[v + 1] - cp[v];
                    for (uint32_t j = 0; j < d; j++) {
                        s_meta.push_back(ci[cp[v] + j] | (j << 16) | (d << kMetaDegShift) | (dmax << kMetaDmaxShift));
                        s_v.push_back(v);
                        if (fp64) s_lam64.push_back(lam64[v]);
                        else s_lam32.push_back(lam32[v]);
                    }
                }
                for (uint32_t q = kWave - cap; q < (uint32_t)kWave; q++) {  // unused slots
                    s_meta.push_back(dmax << kMetaDmaxShift);
                    s_v.push_back(0);
                    if (fp64) s_lam64.push_back(0.0);
                    else s_lam32.push_back(0.0f);
                }
                nchunks++;
                placed += (uint32_t)taken.size();
                // successors become ready once this chunk is complete
                for (uint32_t u : taken)
                    for (uint32_t j = cp[u]; j < cp[u + 1]; j++) {
                        const uint32_t v = succ[j];
                        if (v == kNone) continue;
                        bool dup = false;
                        for (uint32_t j2 = cp[u]; j2 < j; j2++) dup |= succ[j2] == v;
                        if (!dup && --npred[v] == 0) ready.push(key(v));
                    }
            }
            if (placed != ncols) return fail(VIBE_EINVAL, "internal: schedule does not cover every column");
            const uint32_t nch = (uint32_t)(nchunks - member_chunk[i]);
            ch_min = std::min(ch_min, nch);
            ch_max = std::max(ch_max, nch);
            // suffix states of the initial messages mu = lambda, from the end
            // of the sweep backwards
            const size_t end_slot = nchunks * kWave;
            if (fp64) {
                init64.resize(end_slot);
                std::fill(running64.begin(), running64.end(), ident64);
                for (size_t q = end_slot; q-- > first_slot;) {
                    if (!((s_meta[q] >> kMetaDegShift) & 15u)) {
                        init64[q] = ident64;
                        continue;
                    }
                    const uint32_t r = s_meta[q] & 0xffffu;
                    init64[q] = running64[r];
                    running64[r] = rs_combine<uint64_t>(enc64(lam64[s_v[q]]), running64[r]);
                }
            } else {
                init32.resize(end_slot);
                std::fill(running32.begin(), running32.end(), ident32);
                for (size_t q = end_slot; q-- > first_slot;) {
                    if (!((s_meta[q] >> kMetaDegShift) & 15u)) {
                        init32[q] = ident32;
                        continue;
                    }
                    const uint32_t r = s_meta[q] & 0xffffu;
                    init32[q] = running32[r];
                    running32[r] = rs_combine<uint32_t>(enc32(lam32[s_v[q]]), running32[r]);
                }
            }
            if (nchunks * kWave >= (1ull << 32)) return fail(VIBE_EUNSUPPORTED, "schedules exceed 2^32 slots");
        }
        member_chunk[c.L] = (uint32_t)nchunks;
        if (nchunks == 0) {  // no edges at all: keep one (unused) record
            s_meta.assign(kWave, 0);
            s_v.assign(kWave, 0);
            s_lam32.assign(kWave, 0.0f);
            s_lam64.assign(kWave, 0.0);
            init32.assign(kWave, ident32);
            init64.assign(kWave, ident64);
        }
        if (ch_min == UINT32_MAX) ch_min = 0;
    }

    vibe_graph* g = new (std::nothrow) vibe_graph();
    if (!g) return fail(VIBE_ENOMEM, "host allocation failed");
    GraphHost& h = g->h;
    (void)hipGetDevice(&g->device);
    h.cfg = c;
    h.m = m;
    h.n = n;
    h.k = k;
    h.E = E;
    h.max_row = max_row;
    h.max_col = max_col;
    h.levels_min = lev_min == UINT32_MAX ? 0 : lev_min;
    h.levels_max = lev_max;
    h.chunks_min = ch_min;
    h.chunks_max = ch_max;
    h.device_bytes = 0;
    h.perms.assign(perms, perms + (size_t)c.L * (layered ? m : n));
    DevGraph& d = h.dg;
    d.m = m;
    d.n = n;
    d.k = k;
    d.L = c.L;
    d.M = c.M;
    d.T = c.T_max;
    d.E = (uint32_t)E;
    d.words_n = words_n;
    d.words_m = words_m;
    // the layered schedule keeps its check messages (E) and running
    // posteriors (n) in the slab
    d.max_chunks = layered ? (uint32_t)((E + n + kWave - 1) / kWave) : ch_max;
    d.P = 1;
    d.dec_global = 0;
    d.fp64 = fp64 ? 1 : 0;
    d.flood = c.schedule == 1 ? 1 : 0;
    d.layered = layered ? 1 : 0;
    d.lsd_order = c.lsd_order;
    d.alpha = c.alpha;
    d.alpha_t = nullptr;
    d.clamp = lim;
    d.ident32 = ident32;
    d.ident64 = ident64;
    d.all_lam_positive = all_pos;
    std::vector<uint32_t> rp(h_indptr, h_indptr + m + 1);
    std::vector<uint32_t> ri(h_indices, h_indices + E);
    if (lsd_lds_bytes(d) > 150 * 1024) {
        delete g;
        return fail(VIBE_EUNSUPPORTED, "the per-shot LSD state exceeds 150 KB of LDS");
    }
    // interleave the schedule fields into chunk records
    const size_t nrec = s_meta.size() / kWave;
    const uint32_t rb = rec_bytes(fp64), ri0 = rec_init(fp64);
    std::vector<unsigned char> sched(nrec * rb);
    for (size_t j = 0; j < nrec; j++) {
        unsigned char* r = sched.data() + j * rb;
        std::memcpy(r, &s_meta[j * kWave], 4 * kWave);
        std::memcpy(r + kRecV, &s_v[j * kWave], 4 * kWave);
        if (fp64) {
            std::memcpy(r + kRecLam, &s_lam64[j * kWave], 8 * kWave);
            std::memcpy(r + ri0, &init64[j * kWave], 8 * kWave);
        } else {
            std::memcpy(r + kRecLam, &s_lam32[j * kWave], 4 * kWave);
            std::memcpy(r + ri0, &init32[j * kWave], 4 * kWave);
        }
    }
    int rc = VIBE_OK;
    const float* lam32_d = nullptr;
    if ((rc = upload(h, rp.data(), rp.size(), &d.rp)) ||
        (rc = upload(h, ri.data(), ri.size(), &d.ri)) ||
        (rc = upload(h, cp.data(), cp.size(), &d.cp)) ||
        (rc = upload(h, ci.data(), ci.size(), &d.ci)) ||
        (rc = upload(h, lam64.data(), lam64.size(), &d.lam64)) ||
        (!fp64 && (rc = upload(h, lam32.data(), lam32.size(), &lam32_d))) ||
        (rc = upload(h, e0.data(), e0.size(), &d.e0)) ||
        (rc = upload(h, sched.data(), sched.size(), &d.sched)) ||
        (rc = upload(h, member_chunk.data(), member_chunk.size(), &d.member_chunk)) ||
        (rc = upload(h, layered ? perms : (const uint32_t*)nullptr, layered ? (size_t)c.L * m : 1, &d.cperm)) ||
        (rc = upload(h, lobs.data(), lobs.size(), &d.lobs))) {
        free_all(h);
        delete g;
        return rc;
    }
    d.lam = fp64 ? (const void*)d.lam64 : (const void*)lam32_d;
    *out = g;
    return VIBE_OK;
}

extern "C" void vibe_graph_destroy(vibe_graph* g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    for (auto& v : g->ev)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    free_all(g->h);
    if (g->ws.base) (void)hipFree(g->ws.base);
    if (g->ws_in.base) (void)hipFree(g->ws_in.base);
    delete g;
}

extern "C" int vibe_graph_set_alpha(vibe_graph* g, const double* alpha, uint32_t count) {
    set_error("");
    if (!g) return fail(VIBE_EINVAL, "graph handle is NULL");
    if (count > (uint32_t)kMaxT) return fail(VIBE_EINVAL, "count must be in 0..64");
    if (count == 0) {
        g->h.dg.alpha_t = nullptr;
        return VIBE_OK;
    }
    if (!alpha) return fail(VIBE_EINVAL, "alpha is NULL");
    double table[kMaxT];
    for (uint32_t t = 0; t < (uint32_t)kMaxT; t++) {
        const double a = alpha[t < count ? t : count - 1];
        if (!(a > 0.0) || !(a <= 1e6)) return fail(VIBE_EINVAL, "every alpha must be in (0, 1e6]");
        table[t] = a;
    }
    // a new table every call: launches already queued and captured
    // sequences keep reading the table they were given (512 bytes each,
    // freed with the graph)
    const double* dev = nullptr;
    int rc = upload(g->h, table, kMaxT, &dev);
    if (rc) return rc;
    g->h.dg.alpha_t = dev;
    return VIBE_OK;
}

extern "C" int vibe_graph_get_schedules(const vibe_graph* g, uint32_t* perms) {
    if (!g || !perms) return fail(VIBE_EINVAL, "NULL argument");
    std::memcpy(perms, g->h.perms.data(), 4 * g->h.perms.size());
    return VIBE_OK;
}

extern "C" int vibe_graph_info(const vibe_graph* g, vibe_graph_info_t* info) {
    if (!g || !info) return fail(VIBE_EINVAL, "NULL argument");
    const GraphHost& h = g->h;
    info->m = h.m;
    info->n = h.n;
    info->k = h.k;
    info->L = h.cfg.L;
    info->M = h.cfg.M;
    info->T_max = h.cfg.T_max;
    info->nnz = h.E;
    info->max_row_degree = h.max_row;
    info->max_col_degree = h.max_col;
    info->levels_min = h.levels_min;
    info->levels_max = h.levels_max;
    info->chunks_min = h.chunks_min;
    info->chunks_max = h.chunks_max;
    info->message_bits = h.dg.fp64 ? 64 : 32;
    info->grad_width = g->grad_width;
    info->device_bytes = h.device_bytes;
    return VIBE_OK;
}
