// k_conv.hip -- residual CNN block of a fusion block (Sec. 3.3: the
// one-to-many attention is interleaved with residual 3x3 convolutional
// blocks, mirroring a Transformer's MLP block): per layer,
// F_out = F + W2 * gelu(W1 * N(F)) with N the per-pixel RMS normalisation
// over the channels (unit gain, eps 1e-6, as the attention's pre-norm),
// 3x3 kernels and zero padding, gelu(x) = x Phi(x) (erf by Hastings'
// approximation, 1.5e-7), C = 32 channels,
// bfloat16 storage and MFMA operands, float32 accumulation.
//
// An implicit GEMM on v_mfma_f32_16x16x32_bf16: for each of the 9 taps, the
// A operand is the tap's W^T (16 output channels x 32 input channels, one
// fragment per half of the outputs) and the B operand 16 pixels x 32 input
// channels -- one 16-byte LDS read per lane, since pixels are channel-last.
// A persistent workgroup keeps both kernels' fragments in LDS and walks
// 16 x 8 output tiles: it stages the 20 x 12 input region normalised (2-pixel
// halo, zeros outside the image; a quad of lanes holds one pixel's four
// 8-channel chunks and sums its squares with two lane exchanges), computes
// the first convolution on the 18 x 10 region the second one needs (GELU,
// zeros outside the image -- the second convolution pads with zeros too --
// rounded to bfloat16 as its operand), then the second convolution, adds
// the un-normalised input (each lane's two pixels loaded into registers at
// the start of the tile, so their latency hides behind the convolutions) and
// stores bfloat16.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32, TX = 16, TY = 8;
constexpr int IX = TX + 4, IY = TY + 4;          // staged input region
constexpr int MX = TX + 2, MY = TY + 2;          // first convolution's region
constexpr int NMID = MX * MY;                    // 180 pixels
constexpr int MID_TILES = (NMID + 15) / 16;      // 12 pixel tiles of 16
constexpr int NFRAG = 2 * 9 * 2 * 64;            // [conv][tap][half of C_out][lane]

__device__ inline f32x4 mma(const uint4 &a, const uint4 &b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// gelu(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2, with erf from Hastings'
// rational approximation (Abramowitz and Stegun 7.1.26): for z >= 0,
// erf z = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^{-z^2},
// t = 1 / (1 + p z), |error| <= 1.5e-7 -- far below the bfloat16 rounding the
// result gets as an operand; odd in z.
__device__ inline float gelu(float x) {
    const float z = fabsf(x) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
    float poly = fmaf(1.061405429f, t, -1.453152027f);
    poly = fmaf(poly, t, 1.421413741f);
    poly = fmaf(poly, t, -0.284496736f);
    poly = fmaf(poly, t, 0.254829592f);
    const float e = 1.0f - poly * t * __expf(-z * z);      // erf |x| / sqrt 2
    return 0.5f * x * (1.0f + copysignf(e, x));
}

// Weight fragments: lane (c, g) of fragment (conv, tap, half) holds
// W[tap][8g .. 8g+7][16 half + c] (input channels along K).
__global__ void __launch_bounds__(256) k_conv_frag(const ConvParams p) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= NFRAG) return;
    const int lane = i & 63, half = (i >> 6) & 1, tap = (i >> 7) % 9, conv = (i >> 7) / 9;
    const float *Wm = conv ? p.W2 : p.W1;
    const int c = lane & 15, g = lane >> 4;
    bf16x8 v;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (__bf16)Wm[(tap * kC + 8 * g + k) * kC + 16 * half + c];
    p.frag[i] = __builtin_bit_cast(uint4, v);
}

__global__ void __launch_bounds__(256) k_residual_conv(const ConvParams p) {
    __shared__ uint4 s_w[NFRAG];                 // 36 KiB
    // pixels are 5 16-byte chunks apart (4 used): a stride of 80 bytes
    // spreads a column block's 16-byte operand reads over the LDS banks
    __shared__ uint4 s_in[IY * IX * 5];          // 18.75 KiB: [row][col][8-channel chunk]
    __shared__ uint4 s_mid[NMID * 5];            // 14 KiB
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    for (int i = tid; i < NFRAG; i += 256) s_w[i] = p.frag[i];
    const int64_t per_layer = (int64_t)p.tiles_x * p.tiles_y;
    uint16_t *mid16 = reinterpret_cast<uint16_t *>(s_mid);

    for (int64_t t = blockIdx.x; t < p.n_tiles; t += gridDim.x) {
        const int l = (int)(t / per_layer);
        const int rem = (int)(t - (int64_t)l * per_layer);
        const int ty = rem / p.tiles_x, tx = rem - ty * p.tiles_x;
        const int x0 = tx * TX, y0 = ty * TY;
        const uint16_t *Fl = p.F + (int64_t)l * p.H * p.W * kC;
        // the residual (un-normalised input) of this lane's two output
        // pixels, loaded now so that its latency hides behind the convolutions
        uint2 resv[2][2];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int y = y0 + 2 * wave + rr, x = x0 + n;
            resv[rr][0] = resv[rr][1] = make_uint2(0u, 0u);
            if (y < p.H && x < p.W) {
                const uint16_t *src = Fl + ((int64_t)y * p.W + x) * kC;
                resv[rr][0] = *reinterpret_cast<const uint2 *>(src + 4 * g);
                resv[rr][1] = *reinterpret_cast<const uint2 *>(src + 16 + 4 * g);
            }
        }
        __syncthreads();                         // weights in; the previous tile is done

        // the 4 lanes of a quad hold one pixel (256 and the last pass's cut,
        // 192, are multiples of 4, so quads stay whole; whole waves skip the
        // last pass); all loads are issued before the first is used
        constexpr int NSTAGE = (IY * IX * 4 + 255) / 256;
        uint4 v[NSTAGE];
#pragma unroll
        for (int k = 0; k < NSTAGE; ++k) {
            const int i = tid + 256 * k;
            const int pix = i >> 2, q = i & 3;
            const int r = pix / IX, c = pix - r * IX;
            const int y = y0 - 2 + r, x = x0 - 2 + c;
            v[k] = make_uint4(0u, 0u, 0u, 0u);
            if (i < IY * IX * 4 && y >= 0 && y < p.H && x >= 0 && x < p.W)
                v[k] = *reinterpret_cast<const uint4 *>(Fl + ((int64_t)y * p.W + x) * kC + 8 * q);
        }
#pragma unroll
        for (int k = 0; k < NSTAGE; ++k) {
            const int i = tid + 256 * k;
            if (k == NSTAGE - 1 && i >= IY * IX * 4) break;      // wave-uniform
            const unsigned wd[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
            float f[8], ss = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                f[2 * j] = bf2f((uint16_t)(wd[j] & 0xffffu));
                f[2 * j + 1] = bf2f((uint16_t)(wd[j] >> 16));
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) ss = fmaf(f[j], f[j], ss);
            ss += __shfl_xor(ss, 1);
            ss += __shfl_xor(ss, 2);
            const float rn = rsqrtf(ss * (1.0f / kC) + 1e-6f);   // outside: 0 * rn = 0
            uint4 o;
            o.x = f2bf(f[0] * rn) | ((unsigned)f2bf(f[1] * rn) << 16);
            o.y = f2bf(f[2] * rn) | ((unsigned)f2bf(f[3] * rn) << 16);
            o.z = f2bf(f[4] * rn) | ((unsigned)f2bf(f[5] * rn) << 16);
            o.w = f2bf(f[6] * rn) | ((unsigned)f2bf(f[7] * rn) << 16);
            s_in[(i >> 2) * 5 + (i & 3)] = o;
        }
        __syncthreads();

        // first convolution on the 18 x 10 region, 16 pixels per MFMA column block
        for (int mt = wave; mt < MID_TILES; mt += 4) {
            const int pm = 16 * mt + n;
            const int pmc = pm < NMID ? pm : 0;
            const int mr = pmc / MX, mc = pmc - mr * MX;
            f32x4 a0 = {0.0f, 0.0f, 0.0f, 0.0f}, a1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap - 3 * (tap / 3);
                const uint4 b = s_in[((mr + dy) * IX + (mc + dx)) * 5 + g];
                a0 = mma(s_w[(tap * 2 + 0) * 64 + lane], b, a0);
                a1 = mma(s_w[(tap * 2 + 1) * 64 + lane], b, a1);
            }
            if (pm < NMID) {
                const int y = y0 - 1 + mr, x = x0 - 1 + mc;
                const bool inside = y >= 0 && y < p.H && x >= 0 && x < p.W;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    mid16[pm * 40 + 4 * g + i] = inside ? f2bf(gelu(a0[i])) : (uint16_t)0;
                    mid16[pm * 40 + 16 + 4 * g + i] = inside ? f2bf(gelu(a1[i])) : (uint16_t)0;
                }
            }
        }
        __syncthreads();

        // second convolution, residual, store: output rows 2 wave, 2 wave + 1
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int r = 2 * wave + rr;
            f32x4 a0 = {0.0f, 0.0f, 0.0f, 0.0f}, a1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap - 3 * (tap / 3);
                const uint4 b = s_mid[((r + dy) * MX + (n + dx)) * 5 + g];
                a0 = mma(s_w[((9 + tap) * 2 + 0) * 64 + lane], b, a0);
                a1 = mma(s_w[((9 + tap) * 2 + 1) * 64 + lane], b, a1);
            }
            const int y = y0 + r, x = x0 + n;
            if (y < p.H && x < p.W) {
                const uint16_t r0[4] = {(uint16_t)(resv[rr][0].x & 0xffffu), (uint16_t)(resv[rr][0].x >> 16),
                                        (uint16_t)(resv[rr][0].y & 0xffffu), (uint16_t)(resv[rr][0].y >> 16)};
                const uint16_t r1[4] = {(uint16_t)(resv[rr][1].x & 0xffffu), (uint16_t)(resv[rr][1].x >> 16),
                                        (uint16_t)(resv[rr][1].y & 0xffffu), (uint16_t)(resv[rr][1].y >> 16)};
                uint16_t o0[4], o1[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    o0[i] = f2bf(a0[i] + bf2f(r0[i]));
                    o1[i] = f2bf(a1[i] + bf2f(r1[i]));
                }
                uint16_t *dst = p.F_out + (((int64_t)l * p.H + y) * p.W + x) * kC;
                *reinterpret_cast<uint2 *>(dst + 4 * g) =
                    make_uint2(o0[0] | ((unsigned)o0[1] << 16), o0[2] | ((unsigned)o0[3] << 16));
                *reinterpret_cast<uint2 *>(dst + 16 + 4 * g) =
                    make_uint2(o1[0] | ((unsigned)o1[1] << 16), o1[2] | ((unsigned)o1[3] << 16));
            }
        }
    }
}

}  // namespace

hipError_t launch_residual_conv(const ConvParams &pin, int num_cu, bool frag_ready, hipStream_t s) {
    ConvParams p = pin;
    p.tiles_x = (p.W + TX - 1) / TX;
    p.tiles_y = (p.H + TY - 1) / TY;
    p.n_tiles = (int64_t)p.L * p.tiles_x * p.tiles_y;
    hipError_t e;
    if (!frag_ready) {                           // else p.frag already holds them
        hipLaunchKernelGGL(k_conv_frag, dim3((NFRAG + 255) / 256), dim3(256), 0, s, p);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    int64_t blocks = 2 * (int64_t)(num_cu > 0 ? num_cu : 256);
    if (blocks > p.n_tiles) blocks = p.n_tiles;
    hipLaunchKernelGGL(k_residual_conv, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
