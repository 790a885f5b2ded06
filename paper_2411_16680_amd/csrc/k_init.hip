// k_init.hip -- the learned initialisation of a layered depth map (Sec. 3.2,
// "Initialization"): one C-channel feature broadcast over every
// layer-pixel, each layer flat at its depth anchor, alpha one half.
//
// The anchor of storage layer i (0 = nearest) is the paper's layer
// l = L - i at disparity fraction delta = (l - 1/2) / L of the band between
// the far and near planes: d = 1 / (delta (1/near - 1/far) + 1/far).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "uf_params.h"

namespace qk {
namespace {

// One thread per layer-pixel: C channels of F (16-byte stores; bfloat16 LDMs
// get f0 rounded to nearest even by each thread) and the two scalars.
template <bool BF16>
__global__ void __launch_bounds__(256) k_ldm_init(const InitParams p) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= p.N) return;
    const int li = (int)(e / p.npix);
    const float delta = ((float)(p.L - li) - 0.5f) / (float)p.L;
    p.depth[e] = 1.0f / fmaf(delta, p.inv_near - p.inv_far, p.inv_far);
    p.alpha[e] = 0.5f;
    const float4 *src = reinterpret_cast<const float4 *>(p.f0);
    if (BF16) {
        uint4 *dst = reinterpret_cast<uint4 *>(static_cast<uint16_t *>(p.F) + e * p.C);
        for (int c8 = 0; c8 < p.C / 8; ++c8) {
            const float4 a = src[2 * c8], b = src[2 * c8 + 1];
            const float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
            uint32_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t lo = __builtin_bit_cast(uint16_t, (__bf16)f[2 * i]);
                const uint32_t hi = __builtin_bit_cast(uint16_t, (__bf16)f[2 * i + 1]);
                w[i] = lo | (hi << 16);
            }
            dst[c8] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    } else {
        float4 *dst = reinterpret_cast<float4 *>(static_cast<float *>(p.F) + e * p.C);
        for (int c4 = 0; c4 < p.C / 4; ++c4) dst[c4] = src[c4];
    }
}

}  // namespace

hipError_t launch_ldm_init(const InitParams &p, bool bf16, hipStream_t s) {
    const unsigned blocks = (unsigned)((p.N + 255) / 256);
    if (bf16)
        hipLaunchKernelGGL((k_ldm_init<true>), dim3(blocks), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_ldm_init<false>), dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
