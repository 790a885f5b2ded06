// k_resample.hip -- the resolution transition between LDM levels and the
// decode that starts a step (Sec. 3.2.2: the steps where the LDM grows
// upsample the feature volume and the rendered views by two in each
// spatial dimension; every step begins by decoding the feature volume into
// an LDM; the absolute decode of Sec. 3.2.3 with its depth anchors).
//
// k_upsample2x: bilinear upsampling by exactly two with half-pixel centres
// and the border extended.  Output row 2y sits at source row y - 1/4 and
// row 2y + 1 at y + 1/4, so every output is a blend of two rows with
// weights 1/4, 3/4 (the edge row clamps onto itself), likewise for
// columns.  One thread per (source pixel, 8 channels) reads the 3 x 3 source
// neighbourhood and writes the 2 x 2 output block it centres: 9 reads per
// 4 writes, and consecutive lanes write consecutive output pixels.
// Channel counts that are not a multiple of 8 take one thread per
// (source pixel, channel).  Float32 arithmetic, one rounding at the store.
//
// k_ldm_decode: per layer-pixel of layer l (0 nearest) of L,
//   alpha = sigmoid(F w_sigma), colour = sigmoid(F W_color),
//   depth = 1 / ((delta_l + (0.5/L) tanh(F w_depth)) (1/near - 1/far) + 1/far)
// with the anchor delta_l = (L - l - 0.5) / L; the 5 C weights staged in
// LDS and read as broadcasts.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <bool BF16>
__device__ inline void ld8(const void *base, int64_t off, float a[8]) {
    if constexpr (BF16) {
        const uint4 r = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(base) + off);
        const unsigned wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[2 * j] = bf2f((uint16_t)(wd[j] & 0xffffu));
            a[2 * j + 1] = bf2f((uint16_t)(wd[j] >> 16));
        }
    } else {
        const float4 *p = reinterpret_cast<const float4 *>(static_cast<const float *>(base) + off);
        const float4 r0 = p[0], r1 = p[1];
        a[0] = r0.x; a[1] = r0.y; a[2] = r0.z; a[3] = r0.w;
        a[4] = r1.x; a[5] = r1.y; a[6] = r1.z; a[7] = r1.w;
    }
}

template <bool BF16>
__device__ inline void st8(void *base, int64_t off, const float a[8]) {
    if constexpr (BF16) {
        uint4 r;
        r.x = f2bf(a[0]) | ((unsigned)f2bf(a[1]) << 16);
        r.y = f2bf(a[2]) | ((unsigned)f2bf(a[3]) << 16);
        r.z = f2bf(a[4]) | ((unsigned)f2bf(a[5]) << 16);
        r.w = f2bf(a[6]) | ((unsigned)f2bf(a[7]) << 16);
        *reinterpret_cast<uint4 *>(static_cast<uint16_t *>(base) + off) = r;
    } else {
        float4 *p = reinterpret_cast<float4 *>(static_cast<float *>(base) + off);
        p[0] = make_float4(a[0], a[1], a[2], a[3]);
        p[1] = make_float4(a[4], a[5], a[6], a[7]);
    }
}

template <bool BF16>
__device__ inline float ld1(const void *base, int64_t off) {
    if constexpr (BF16) return bf2f(static_cast<const uint16_t *>(base)[off]);
    else return static_cast<const float *>(base)[off];
}

template <bool BF16>
__device__ inline void st1(void *base, int64_t off, float v) {
    if constexpr (BF16) static_cast<uint16_t *>(base)[off] = f2bf(v);
    else static_cast<float *>(base)[off] = v;
}

// VEC = 8 channels per thread (C a multiple of 8) or 1
template <int VEC, bool BF16>
__global__ void __launch_bounds__(256) k_upsample2x(const Up2Params p) {
    const int NC = p.C / VEC;
    const int64_t total = (int64_t)p.N * p.H * p.W * NC;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int64_t pix = i / NC;
    const int c0 = VEC * (int)(i - pix * NC);
    const int64_t hw = (int64_t)p.H * p.W;
    const int n = (int)(pix / hw);
    const int64_t r = pix - (int64_t)n * hw;
    const int y = (int)(r / p.W), x = (int)(r - (int64_t)y * p.W);
    const int ys[3] = {y > 0 ? y - 1 : 0, y, y + 1 < p.H ? y + 1 : p.H - 1};
    const int xs[3] = {x > 0 ? x - 1 : 0, x, x + 1 < p.W ? x + 1 : p.W - 1};
    const int64_t sbase = (int64_t)n * hw;
    // vertical blends of the three source columns: top (row 2y), bottom (2y + 1)
    float top[3][VEC], bot[3][VEC];
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
        float a[VEC], b[VEC], c[VEC];
        const int64_t o0 = (sbase + (int64_t)ys[0] * p.W + xs[cx]) * p.C + c0;
        const int64_t o1 = (sbase + (int64_t)ys[1] * p.W + xs[cx]) * p.C + c0;
        const int64_t o2 = (sbase + (int64_t)ys[2] * p.W + xs[cx]) * p.C + c0;
        if constexpr (VEC == 8) {
            ld8<BF16>(p.src, o0, a);
            ld8<BF16>(p.src, o1, b);
            ld8<BF16>(p.src, o2, c);
        } else {
            a[0] = ld1<BF16>(p.src, o0);
            b[0] = ld1<BF16>(p.src, o1);
            c[0] = ld1<BF16>(p.src, o2);
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            top[cx][j] = fmaf(0.25f, a[j], 0.75f * b[j]);
            bot[cx][j] = fmaf(0.25f, c[j], 0.75f * b[j]);
        }
    }
    const int W2 = 2 * p.W;
    const int64_t dbase = (int64_t)n * (4 * hw);
    const int64_t d00 = (dbase + (int64_t)(2 * y) * W2 + 2 * x) * p.C + c0;
    const int64_t d10 = d00 + (int64_t)W2 * p.C;            // row 2y + 1
    float o[4][VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        o[0][j] = fmaf(0.25f, top[0][j], 0.75f * top[1][j]);
        o[1][j] = fmaf(0.25f, top[2][j], 0.75f * top[1][j]);
        o[2][j] = fmaf(0.25f, bot[0][j], 0.75f * bot[1][j]);
        o[3][j] = fmaf(0.25f, bot[2][j], 0.75f * bot[1][j]);
    }
    if constexpr (VEC == 8) {
        st8<BF16>(p.dst, d00, o[0]);
        st8<BF16>(p.dst, d00 + p.C, o[1]);
        st8<BF16>(p.dst, d10, o[2]);
        st8<BF16>(p.dst, d10 + p.C, o[3]);
    } else {
        st1<BF16>(p.dst, d00, o[0][0]);
        st1<BF16>(p.dst, d00 + p.C, o[1][0]);
        st1<BF16>(p.dst, d10, o[2][0]);
        st1<BF16>(p.dst, d10 + p.C, o[3][0]);
    }
}

__device__ inline float sigmoid_(float x) { return 1.0f / (1.0f + __expf(-x)); }

template <int C, bool BF16>
__global__ void __launch_bounds__(256) k_ldm_decode(const DecodeParams p) {
    // weights staged in LDS, read as broadcasts: [c] = (sigma, depth, r, g, b)
    __shared__ float w[C * 5];
    for (int i = threadIdx.x; i < C * 5; i += 256) {
        const int c = i / 5, k = i - 5 * c;
        w[i] = k == 0 ? p.w_sigma[c] : k == 1 ? p.w_depth[c]
             : p.logits ? 0.0f : p.W_color[3 * c + k - 2];
    }
    __syncthreads();
    const int64_t hw = (int64_t)p.H * p.W;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)p.L * hw) return;
    const int li = (int)(q / hw);
    float xs = 0.0f, xd = 0.0f, x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
#pragma unroll 1
    for (int c8 = 0; c8 < C / 8; ++c8) {                // rolled: weights stay in LDS
        float f[8];
        ld8<BF16>(p.F, q * C + 8 * c8, f);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float *wc = w + 5 * (8 * c8 + j);
            xs = fmaf(f[j], wc[0], xs);
            xd = fmaf(f[j], wc[1], xd);
            x0 = fmaf(f[j], wc[2], x0);
            x1 = fmaf(f[j], wc[3], x1);
            x2 = fmaf(f[j], wc[4], x2);
        }
    }
    if (p.logits) {                  // the unactivated depth and density
        p.depth[q] = xd;
        p.alpha[q] = xs;
        return;
    }
    const float L = (float)p.L;
    const float delta = ((float)(p.L - li) - 0.5f) / L;
    const float t = tanhf(xd);
    p.depth[q] = 1.0f / fmaf(fmaf(0.5f / L, t, delta), p.inv_near - p.inv_far, p.inv_far);
    p.alpha[q] = sigmoid_(xs);
    if (p.color != nullptr) {
        p.color[3 * q + 0] = sigmoid_(x0);
        p.color[3 * q + 1] = sigmoid_(x1);
        p.color[3 * q + 2] = sigmoid_(x2);
    }
}

template <bool BF16>
hipError_t launch_decode_t(const DecodeParams &p, dim3 g, hipStream_t s) {
    switch (p.C) {
        case 8: hipLaunchKernelGGL((k_ldm_decode<8, BF16>), g, dim3(256), 0, s, p); break;
        case 16: hipLaunchKernelGGL((k_ldm_decode<16, BF16>), g, dim3(256), 0, s, p); break;
        case 32: hipLaunchKernelGGL((k_ldm_decode<32, BF16>), g, dim3(256), 0, s, p); break;
        case 64: hipLaunchKernelGGL((k_ldm_decode<64, BF16>), g, dim3(256), 0, s, p); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_upsample2x(const Up2Params &p, hipStream_t s) {
    const bool v8 = p.C % 8 == 0;
    const int64_t threads = (int64_t)p.N * p.H * p.W * (v8 ? p.C / 8 : p.C);
    const dim3 g((unsigned)((threads + 255) / 256));
    if (v8) {
        if (p.bf16) hipLaunchKernelGGL((k_upsample2x<8, true>), g, dim3(256), 0, s, p);
        else hipLaunchKernelGGL((k_upsample2x<8, false>), g, dim3(256), 0, s, p);
    } else {
        if (p.bf16) hipLaunchKernelGGL((k_upsample2x<1, true>), g, dim3(256), 0, s, p);
        else hipLaunchKernelGGL((k_upsample2x<1, false>), g, dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_ldm_decode(const DecodeParams &p, hipStream_t s) {
    const dim3 g((unsigned)(((int64_t)p.L * p.H * p.W + 255) / 256));
    return p.bf16 ? launch_decode_t<true>(p, g, s) : launch_decode_t<false>(p, g, s);
}

}  // namespace qk
