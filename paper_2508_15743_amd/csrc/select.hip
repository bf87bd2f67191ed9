// K2: candidate selection (paper Sec. III.D.2).  Among the members that
// converged, the first M in (iteration, member index) order are the
// candidates; the one of least prior weight W(e) = sum_v e_v lambda_v wins,
// ties going to the earlier candidate.  Shots with no converged member are
// queued for LSD.
// K4: observables Lobs * e mod 2 (paper Sec. II.B), bit-packed AND + popcount.
#include "internal.h"

namespace vibe {

namespace {

__global__ __launch_bounds__(kWave) void select_kernel(DevGraph g, SelectLaunch a) {
    const uint32_t shot = blockIdx.x;
    if (shot >= a.n_shots) return;
    const int lane = threadIdx.x;
    const size_t base = (size_t)shot * g.L;
    // one lane per member: key = t * 64 + i for converged members
    const bool have = (uint32_t)lane < g.L;
    const int32_t t = have ? a.t_conv[base + lane] : 0;
    const bool conv = have && t > 0;
    const uint32_t key = conv ? (uint32_t)t * kWave + lane : 0xffffffffu;
    const uint64_t cmask = __ballot(conv);
    const uint32_t nconv = __popcll(cmask);
    // rank of this member among the converged ones in (t, i) order
    uint32_t rank = 0;
    for (int j = 0; j < kWave; j++) {
        uint32_t kj = __shfl(key, j);
        if (kj < key) rank++;
    }
    const bool cand = conv && rank < g.M;
    double w = cand ? a.weight[base + lane] : INFINITY;
    // argmin of (W, rank): ties go to the earlier candidate
    uint32_t r = cand ? rank : 0xffffffffu;
    int who = cand ? lane : -1;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        double ow = __shfl_xor(w, off);
        uint32_t orr = __shfl_xor(r, off);
        int owho = __shfl_xor(who, off);
        if (ow < w || (ow == w && orr < r)) {
            w = ow;
            r = orr;
            who = owho;
        }
    }
    who = uni(who);
    const size_t gshot = a.shot0 + shot;
    // members whose run reached the clamp (word 0 of the shot's masks)
    const uint64_t sat = a.conv_mask ? a.conv_mask[(size_t)shot * (kMaxT + 1)] : 0ull;
    uint64_t* out = a.corrections + gshot * g.words_n;
    if (nconv) {
        const uint32_t tw = (uint32_t)__shfl(t, who);
        const uint64_t* src = a.cand + (base + (uint32_t)who) * g.words_n;
        for (uint32_t i = lane; i < g.words_n; i += kWave) out[i] = src[i];
        if (lane == 0 && a.stats) {
            vibe_shot_stats st;
            st.flags = VIBE_FLAG_BP_CONVERGED | (((sat >> who) & 1ull) ? VIBE_FLAG_SATURATED : 0u);
            st.winner = who;
            st.t_win = tw;
            st.n_conv = nconv;
            st.lsd_clusters = st.lsd_largest = st.lsd_rounds = 0;
            st.member_iters = a.iters[shot];
            a.stats[gshot] = st;
        }
    } else if (lane == 0) {
        uint32_t slot = atomicAdd(a.fail_count, 1u);
        a.fail_list[slot] = shot;
        if (a.stats) {
            vibe_shot_stats st;
            st.flags = VIBE_FLAG_LSD_USED | (sat ? VIBE_FLAG_SATURATED : 0u);
            st.winner = -1;
            st.t_win = 0;
            st.n_conv = 0;
            st.lsd_clusters = st.lsd_largest = st.lsd_rounds = 0;
            st.member_iters = a.iters[shot];
            a.stats[gshot] = st;
        }
    }
}

__global__ __launch_bounds__(kWave) void observables_kernel(DevGraph g, const uint64_t* corr,
                                                            uint64_t shot0, uint32_t n_shots,
                                                            uint8_t* obs) {
    const uint32_t shot = blockIdx.x;
    if (shot >= n_shots) return;
    const int lane = threadIdx.x;
    const uint64_t* e = corr + (shot0 + shot) * g.words_n;
    for (uint32_t r = 0; r < g.k; r++) {
        const uint64_t* row = g.lobs + (size_t)r * g.words_n;
        uint32_t par = 0;
        for (uint32_t i = lane; i < g.words_n; i += kWave) par ^= __popcll(e[i] & row[i]) & 1u;
        for (int off = kWave / 2; off > 0; off >>= 1) par ^= __shfl_xor(par, off);
        if (lane == 0) obs[(shot0 + shot) * g.k + r] = (uint8_t)par;
    }
}

}  // namespace

int launch_select(const DevGraph& g, const SelectLaunch& a, hipStream_t st) {
    if (!a.n_shots) return VIBE_OK;
    hipLaunchKernelGGL(select_kernel, dim3(a.n_shots), dim3(kWave), 0, st, g, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "select_kernel launch");
}

int launch_observables(const DevGraph& g, const uint64_t* corrections, uint64_t shot0,
                       uint32_t n_shots, uint8_t* observables, hipStream_t st) {
    if (!n_shots || !g.k) return VIBE_OK;
    hipLaunchKernelGGL(observables_kernel, dim3(n_shots), dim3(kWave), 0, st, g, corrections, shot0,
                       n_shots, observables);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "observables_kernel launch");
}

}  // namespace vibe
