// Measurement: the HBM ceiling of the BP kernel's memory access pattern.
//
// The BP ensemble kernel streams each resident wavefront's message slab
// through HBM: a sweep reads and rewrites one 256-byte run per chunk step in
// increasing order, the backward pass the same in decreasing order, with
// loads three steps ahead.  This kernel does exactly that on a buffer of
// `waves` private regions with no arithmetic between, so its rate is the
// most that pattern can move at that concurrency on the device (as a plain
// device copy is for sequential streams).
#include "internal.h"

namespace vibe {
namespace {

constexpr int kAhead = 3;

__global__ __launch_bounds__(kWave) void slab_stream_kernel(float* base, uint32_t region_words, uint32_t passes) {
    float* r = base + (size_t)blockIdx.x * region_words;
    const uint32_t lane = threadIdx.x;
    const int steps = (int)(region_words / kWave);
    for (uint32_t p = 0; p < passes; p++) {
        const bool fwd = (p & 1u) == 0;
        auto at = [&](int s) {
            const int k = fwd ? s : steps - 1 - s;
            return r + (size_t)k * kWave + lane;
        };
        float ring[kAhead];
#pragma unroll
        for (int d = 0; d < kAhead; d++) ring[d] = *at(d < steps ? d : steps - 1);
        for (int s = 0; s < steps; s += kAhead) {
#pragma unroll
            for (int d = 0; d < kAhead; d++) {
                if (s + d >= steps) break;
                const float v = ring[d];
                const int nx = s + d + kAhead;
                ring[d] = *at(nx < steps ? nx : steps - 1);
                *at(s + d) = v + 1.0f;
            }
        }
    }
}

}  // namespace
}  // namespace vibe

using namespace vibe;

extern "C" int vibe_measure_slab_stream(float* buf, uint64_t region_bytes, uint32_t waves, uint32_t passes,
                                        void* stream) {
    set_error("");
    if (!buf || !waves || !passes) return fail(VIBE_EINVAL, "NULL buffer or zero waves / passes");
    if (region_bytes < 256 || region_bytes % 256 || region_bytes / 4 > UINT32_MAX)
        return fail(VIBE_EINVAL, "region_bytes must be a positive multiple of 256 below 16 GiB");
    hipLaunchKernelGGL(slab_stream_kernel, dim3(waves), dim3(kWave), 0, static_cast<hipStream_t>(stream), buf,
                       (uint32_t)(region_bytes / 4), passes);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VIBE_OK : hip_fail(e, "slab_stream_kernel launch");
}
