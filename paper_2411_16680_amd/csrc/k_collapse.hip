// k_collapse.hip -- layer collapse (Sec. 3.2.2, "Layer Collapse"): each new
// layer is the mean of a pair of adjacent layers plus a residual MLP of their
// concatenation, out[j] = (F[2j] + F[2j+1]) / 2 + relu([F[2j], F[2j+1]] W1) W2,
// C = 32, bfloat16 storage and MFMA operands, float32 accumulation.
//
// A wave takes 16 output pixels as the columns of v_mfma_f32_16x16x32_bf16:
// the pair's two 16-byte channel chunks per lane are the B operands of the
// first product (K = 64 = two K blocks), its ReLU output crosses to the B
// layout of the second product through the wave's LDS slice (rounded to
// bfloat16 as the operand), the second product's output crosses back to the
// load layout the same way (in float32), and each lane adds the mean of its
// own two input chunks and stores 16 bytes: a wave writes its 16 pixels as
// one contiguous 1 KiB.  The weight fragments are built once per
// (persistent) workgroup in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32, HS = 40;             // LDS pixel stride of the ReLU output (bf16)
constexpr int YS = 36;                       // LDS pixel stride of the MLP output (float)

__device__ inline f32x4 mma(const uint4 &a, const uint4 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__global__ void __launch_bounds__(256) k_layer_collapse(const CollapseParams p) {
    // fragments 0..3: W1 K block kb (rows 32 kb ..), output half t at 2 kb + t;
    // 4..5: W2 output half t.  Lane (c, g) holds W[8g .. 8g+7 of the block][16 t + c].
    __shared__ uint4 s_w[6 * 64];
    __shared__ uint16_t s_h[4][16 * HS];
    __shared__ float s_y[4][16 * YS];            // the MLP output, to the load layout
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    for (int i = tid; i < 6 * 64; i += 256) {
        const int f = i >> 6, ln = i & 63, c = ln & 15, gg = ln >> 4;
        bf16x8 v;
        if (f < 4) {
            const int kb = f >> 1, t = f & 1;
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = (__bf16)p.W1[(32 * kb + 8 * gg + k) * kC + 16 * t + c];
        } else {
            const int t = f - 4;
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = (__bf16)p.W2[(8 * gg + k) * kC + 16 * t + c];
        }
        s_w[i] = __builtin_bit_cast(uint4, v);
    }
    const int64_t bpl = (p.npix + 15) / 16;
    uint16_t *hs = s_h[wave];
    for (int64_t base = (int64_t)blockIdx.x * 4; base < p.n_blocks; base += (int64_t)gridDim.x * 4) {
        __syncthreads();                         // fragments in; the previous block's reads done
        const int64_t blk = base + wave;
        const bool active = blk < p.n_blocks;
        const int64_t j = active ? blk / bpl : 0;
        const int64_t pix = active ? (blk - j * bpl) * 16 + n : 0;
        const bool ok = active && pix < p.npix;
        const uint16_t *fa = p.F + ((2 * j) * p.npix + pix) * kC;
        const uint16_t *fb = fa + p.npix * kC;
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
        const uint4 xa = ok ? *reinterpret_cast<const uint4 *>(fa + 8 * g) : z;
        const uint4 xb = ok ? *reinterpret_cast<const uint4 *>(fb + 8 * g) : z;
        f32x4 h0 = {0.0f, 0.0f, 0.0f, 0.0f}, h1 = {0.0f, 0.0f, 0.0f, 0.0f};
        h0 = mma(s_w[0 * 64 + lane], xa, h0);
        h0 = mma(s_w[2 * 64 + lane], xb, h0);
        h1 = mma(s_w[1 * 64 + lane], xa, h1);
        h1 = mma(s_w[3 * 64 + lane], xb, h1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            hs[n * HS + 4 * g + i] = f2bf(fmaxf(h0[i], 0.0f));
            hs[n * HS + 16 + 4 * g + i] = f2bf(fmaxf(h1[i], 0.0f));
        }
        __syncthreads();
        const uint4 hb = *reinterpret_cast<const uint4 *>(&hs[n * HS + 8 * g]);
        f32x4 y0 = {0.0f, 0.0f, 0.0f, 0.0f}, y1 = {0.0f, 0.0f, 0.0f, 0.0f};
        y0 = mma(s_w[4 * 64 + lane], hb, y0);
        y1 = mma(s_w[5 * 64 + lane], hb, y1);
        // the MLP output crosses to the load layout (lane (g, n): channels
        // 8g .. 8g+7 of pixel n), where the pair's inputs already are, so a
        // lane adds the mean from its registers and stores 16 whole bytes:
        // one instruction writes the 16 pixels' 1 KiB contiguously
        float *ys = s_y[wave];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ys[n * YS + 4 * g + i] = y0[i];
            ys[n * YS + 16 + 4 * g + i] = y1[i];
        }
        __syncthreads();
        if (ok) {
            const float4 ya = *reinterpret_cast<const float4 *>(&ys[n * YS + 8 * g]);
            const float4 yb = *reinterpret_cast<const float4 *>(&ys[n * YS + 8 * g + 4]);
            const float yv[8] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y, yb.z, yb.w};
            const unsigned wa[4] = {xa.x, xa.y, xa.z, xa.w}, wb[4] = {xb.x, xb.y, xb.z, xb.w};
            unsigned o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float lo = 0.5f * (bf2f((uint16_t)(wa[k] & 0xffffu)) + bf2f((uint16_t)(wb[k] & 0xffffu))) + yv[2 * k];
                const float hi = 0.5f * (bf2f((uint16_t)(wa[k] >> 16)) + bf2f((uint16_t)(wb[k] >> 16))) + yv[2 * k + 1];
                o[k] = f2bf(lo) | ((unsigned)f2bf(hi) << 16);
            }
            *reinterpret_cast<uint4 *>(p.F_out + (j * p.npix + pix) * kC + 8 * g) =
                make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
}

}  // namespace

hipError_t launch_layer_collapse(const CollapseParams &p, int num_cu, hipStream_t s) {
    int64_t blocks = (p.n_blocks + 3) / 4;
    const int64_t cap = 8 * (int64_t)(num_cu > 0 ? num_cu : 256);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_layer_collapse, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
