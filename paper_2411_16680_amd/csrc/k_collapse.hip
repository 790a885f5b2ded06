// k_collapse.hip -- layer collapse (Sec. 3.2.2, "Layer Collapse"): each new
// layer is the mean of a pair of adjacent layers plus a residual MLP of their
// concatenation, out[j] = (F[2j] + F[2j+1]) / 2 + relu([F[2j], F[2j+1]] W1) W2,
// C = 32, bfloat16 storage and MFMA operands, float32 accumulation.
//
// A wave takes 16 output pixels as the columns of v_mfma_f32_16x16x32_bf16:
// the pair's two 16-byte channel chunks per lane are the B operands of the
// first product (K = 64 = two K blocks), its ReLU output crosses to the B
// layout of the second product through the wave's LDS slice (rounded to
// bfloat16 as the operand), and the mean is added in float32 from the
// bfloat16 inputs before the single rounding at the store.  The weight
// fragments are built once per (persistent) workgroup in LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32, HS = 40;             // LDS pixel stride of the ReLU output (bf16)

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
        if (ok) {
            uint16_t *dst = p.F_out + (j * p.npix + pix) * kC;
            const uint2 a0 = *reinterpret_cast<const uint2 *>(fa + 4 * g);
            const uint2 b0 = *reinterpret_cast<const uint2 *>(fb + 4 * g);
            const uint2 a1 = *reinterpret_cast<const uint2 *>(fa + 16 + 4 * g);
            const uint2 b1 = *reinterpret_cast<const uint2 *>(fb + 16 + 4 * g);
            const uint16_t *pa0 = reinterpret_cast<const uint16_t *>(&a0);
            const uint16_t *pb0 = reinterpret_cast<const uint16_t *>(&b0);
            const uint16_t *pa1 = reinterpret_cast<const uint16_t *>(&a1);
            const uint16_t *pb1 = reinterpret_cast<const uint16_t *>(&b1);
            uint16_t o0[4], o1[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                o0[i] = f2bf(0.5f * (bf2f(pa0[i]) + bf2f(pb0[i])) + y0[i]);
                o1[i] = f2bf(0.5f * (bf2f(pa1[i]) + bf2f(pb1[i])) + y1[i]);
            }
            *reinterpret_cast<uint2 *>(dst + 4 * g) =
                make_uint2(o0[0] | ((unsigned)o0[1] << 16), o0[2] | ((unsigned)o0[3] << 16));
            *reinterpret_cast<uint2 *>(dst + 16 + 4 * g) =
                make_uint2(o1[0] | ((unsigned)o1[1] << 16), o1[2] | ((unsigned)o1[3] << 16));
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
