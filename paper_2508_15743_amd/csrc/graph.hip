// Offline stage (paper Sec. III.D.1): validate the detector error model, derive
// the channel LLRs, build the member schedules and upload everything once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

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
    if (c.lsd_order != 0) return fail(VIBE_EUNSUPPORTED, "only LSD order 0 is implemented");
    if (!(c.alpha > 0.0) || !(c.alpha <= 1e6)) return fail(VIBE_EINVAL, "alpha must be in (0, 1e6]");
    if (!(c.clamp >= 1.0) || !(c.clamp <= 1e30)) return fail(VIBE_EINVAL, "clamp must be in [1, 1e30]");
    if (m && (size_t)m * 4 + 8 * (2 * (size_t)((m + 63) / 64) + (n + 63) / 64) > 150 * 1024)
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
    // ---- permutations
    {
        std::vector<uint8_t> seen(n);
        for (uint32_t i = 0; i < c.L; i++) {
            std::fill(seen.begin(), seen.end(), 0);
            for (uint32_t a = 0; a < n; a++) {
                uint32_t v = perms[(size_t)i * n + a];
                if (v >= n || seen[v]) return fail(VIBE_EINVAL, "perms rows must be permutations of 0..n-1");
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

    // ---- channel LLRs
    const double lim = c.clamp;
    std::vector<double> lam64(n);
    std::vector<float> lam(n);
    int all_pos = 1;
    for (uint32_t v = 0; v < n; v++) {
        double l = std::log((1.0 - priors[v]) / priors[v]);
        l = std::min(std::max(l, -lim), lim);
        lam64[v] = l;
        lam[v] = (float)l;
        if (!(lam[v] > 0.0f)) all_pos = 0;
    }
    const float limf = (float)lim;
    const uint32_t words_n = (n + 63) / 64, words_m = (m + 63) / 64;
    std::vector<uint64_t> e0(words_n, 0);
    for (uint32_t v = 0; v < n; v++)
        if (cp[v + 1] == cp[v] && !(lam[v] > 0.0f)) e0[v / 64] |= 1ull << (v % 64);
    std::vector<uint64_t> lobs((size_t)std::max<uint32_t>(k, 1) * words_n, 0);
    for (uint32_t r = 0; r < k; r++)
        for (uint32_t a = l_indptr[r]; a < l_indptr[r + 1]; a++) {
            uint32_t v = l_indices[a];
            lobs[(size_t)r * words_n + v / 64] ^= 1ull << (v % 64);
        }
    auto enc = [](float x) -> uint32_t {
        float a = std::fabs(x);
        uint32_t bits;
        std::memcpy(&bits, &a, 4);
        return bits | (x < 0.0f ? 0x80000000u : 0u);
    };
    uint32_t ident;
    std::memcpy(&ident, &limf, 4);

    // ---- member schedules.  The serial sweep of member i visits the columns
    //      in perms[i]; columns that share no check commute, so the sweep is
    //      regrouped into dependency levels (level(v) = 1 + the largest level
    //      of an earlier column sharing a check), each level cut into chunks
    //      of at most 64 edges holding whole columns.  The member's message
    //      slab follows the same slot order.  At column v's turn, the edges of
    //      a row that come before v in the sweep carry this sweep's messages
    //      and those after v the previous sweep's; init_suf holds, at every
    //      slot, the state (min |mu|, sign parity) of the row's later edges
    //      for the initial messages mu = lambda.
    std::vector<Slot> slots((size_t)c.L * E);
    std::vector<uint32_t> init_suf((size_t)c.L * E);
    std::vector<uint32_t> chunk_off;
    std::vector<uint32_t> member_chunk(c.L + 1, 0);
    uint32_t lev_min = UINT32_MAX, lev_max = 0;
    {
        std::vector<uint32_t> last(m), level(n), count, start, order(n), running(m);
        for (uint32_t i = 0; i < c.L; i++) {
            const uint32_t* pi = perms + (size_t)i * n;
            std::fill(last.begin(), last.end(), 0);
            uint32_t nlev = 0;
            for (uint32_t a = 0; a < n; a++) {
                uint32_t v = pi[a], lv = 0;
                for (uint32_t j = cp[v]; j < cp[v + 1]; j++) lv = std::max(lv, last[ci[j]]);
                lv += 1;
                level[v] = lv;
                for (uint32_t j = cp[v]; j < cp[v + 1]; j++) last[ci[j]] = lv;
                if (cp[v + 1] > cp[v]) nlev = std::max(nlev, lv);
            }
            lev_min = std::min(lev_min, nlev);
            lev_max = std::max(lev_max, nlev);
            count.assign(nlev + 2, 0);
            for (uint32_t a = 0; a < n; a++) {
                uint32_t v = pi[a];
                if (cp[v + 1] > cp[v]) count[level[v]]++;
            }
            start.assign(nlev + 2, 0);
            for (uint32_t l = 1; l <= nlev; l++) start[l + 1] = start[l] + count[l];
            {
                std::vector<uint32_t> fillp(start.begin(), start.end());
                for (uint32_t a = 0; a < n; a++) {
                    uint32_t v = pi[a];
                    if (cp[v + 1] > cp[v]) order[fillp[level[v]]++] = v;  // sweep order
                }
            }
            member_chunk[i] = (uint32_t)chunk_off.size();
            const size_t sbase = (size_t)i * E;
            size_t spos = 0;
            for (uint32_t l = 1; l <= nlev; l++) {
                uint32_t in_chunk = 0;
                chunk_off.push_back((uint32_t)(sbase + spos));
                for (uint32_t a = start[l]; a < start[l + 1]; a++) {
                    const uint32_t v = order[a], deg = cp[v + 1] - cp[v];
                    if (in_chunk + deg > (uint32_t)kWave) {
                        chunk_off.push_back((uint32_t)(sbase + spos));
                        in_chunk = 0;
                    }
                    for (uint32_t j = cp[v]; j < cp[v + 1]; j++) {
                        Slot sl;
                        sl.meta = ci[j] | ((j - cp[v]) << 16) | (deg << 20);
                        sl.v = v;
                        slots[sbase + spos++] = sl;
                    }
                    in_chunk += deg;
                }
            }
            if (spos != E) return fail(VIBE_EINVAL, "internal: schedule does not cover every edge");
            // suffix states of the initial messages, from the end of the sweep
            std::fill(running.begin(), running.end(), ident);
            for (size_t q = E; q-- > 0;) {
                const Slot& sl = slots[sbase + q];
                const uint32_t r = sl.meta & 0xffffu;
                init_suf[sbase + q] = running[r];
                running[r] = rs_combine(enc(lam[sl.v]), running[r]);
            }
        }
        member_chunk[c.L] = (uint32_t)chunk_off.size();
        chunk_off.push_back((uint32_t)((size_t)c.L * E));  // end of the last chunk
        if ((size_t)c.L * E >= (1ull << 32)) return fail(VIBE_EUNSUPPORTED, "L * nnz must be < 2^32");
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
    h.device_bytes = 0;
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
    d.alpha = (float)c.alpha;
    d.clamp = limf;
    d.ident = ident;
    d.all_lam_positive = all_pos;
    std::vector<uint32_t> rp(h_indptr, h_indptr + m + 1);
    std::vector<uint32_t> ri(h_indices, h_indices + E);
    if (lsd_lds_bytes(d) > 150 * 1024) {
        delete g;
        return fail(VIBE_EUNSUPPORTED, "the per-shot LSD state exceeds 150 KB of LDS");
    }
    int rc = VIBE_OK;
    if ((rc = upload(h, rp.data(), rp.size(), &d.rp)) ||
        (rc = upload(h, ri.data(), ri.size(), &d.ri)) ||
        (rc = upload(h, cp.data(), cp.size(), &d.cp)) ||
        (rc = upload(h, ci.data(), ci.size(), &d.ci)) ||
        (rc = upload(h, lam.data(), lam.size(), &d.lam)) ||
        (rc = upload(h, lam64.data(), lam64.size(), &d.lam64)) ||
        (rc = upload(h, e0.data(), e0.size(), &d.e0)) ||
        (rc = upload(h, init_suf.data(), init_suf.size(), &d.init_suf)) ||
        (rc = upload(h, slots.data(), slots.size(), &d.slots)) ||
        (rc = upload(h, chunk_off.data(), chunk_off.size(), &d.chunk_off)) ||
        (rc = upload(h, member_chunk.data(), member_chunk.size(), &d.member_chunk)) ||
        (rc = upload(h, lobs.data(), lobs.size(), &d.lobs))) {
        free_all(h);
        delete g;
        return rc;
    }
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
    delete g;
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
    info->device_bytes = h.device_bytes;
    return VIBE_OK;
}
