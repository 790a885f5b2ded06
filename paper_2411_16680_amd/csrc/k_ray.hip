// k_ray.hip -- ray-direction encoding added to the input views' feature maps
// (Sec. 3.2.1 and "Encode Input Images" of Sec. 3.2.2): the ray of a pixel
// of view m is cut by the planes z = near and z = far of the novel camera's
// frustum, both points are projected by the novel camera, and their
// difference (far minus near, in normalised device coordinates) goes
// through tanh, 8 octaves of sinusoids and a linear map to C channels.
//
// With o view m's centre and d the pixel's ray direction, both in the novel
// frame, the ray meets the plane z at P = o + (z - o_z)/d_z d, so
//   P_x / z = d_x / d_z + (o_x - o_z d_x / d_z) / z
// and the difference of P_x / z between the far and the near plane is
// (1/far - 1/near)(o_x - o_z d_x / d_z), likewise for y; the NDC
// difference applies the first two rows of the novel K (on its own grid,
// NDC = 2 (u, v) / (W_n, H_n) up to a constant that cancels).
//
// One thread per pixel; the geometry and tanh run in double (the top octave
// scales its argument by 128 pi), each octave's argument is reduced modulo 2
// in double -- exactly -- and its sine and cosine taken by sinpi / cospi in
// float.  The projection reads the 32 x C weights from LDS (one address per
// wave: a broadcast) and accumulates on top of the feature, which is
// rounded once at the store.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <int C, bool BF16>
__global__ void __launch_bounds__(256) k_ray_encoding(const RayParams p) {
    __shared__ float4 w4[8 * C];                 // [32][C] floats
    for (int i = threadIdx.x; i < 8 * C; i += 256) w4[i] = reinterpret_cast<const float4 *>(p.Wr)[i];
    __syncthreads();
    const int m = blockIdx.y;
    const int fw = p.fW[m];
    const int64_t np = (int64_t)p.fH[m] * fw;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= np) return;                         // no barrier below
    const int y = (int)(q / fw), x = (int)(q - (int64_t)y * fw);
    const double u = (double)x + 0.5, v = (double)y + 0.5;
    const double *D = p.D[m], *o = p.o[m];
    const double dx = fma(D[0], u, fma(D[1], v, D[2]));
    const double dy = fma(D[3], u, fma(D[4], v, D[5]));
    const double dz = fma(D[6], u, fma(D[7], v, D[8]));
    const double rz = o[2] / dz;
    const double ax = p.inv_band * fma(-rz, dx, o[0]);
    const double ay = p.inv_band * fma(-rz, dy, o[1]);
    const double tx = tanh(fma(p.kx0, ax, p.kx1 * ay));
    const double ty = tanh(fma(p.ky0, ax, p.ky1 * ay));
    float e[32];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double sx = (double)(1 << k) * tx, sy = (double)(1 << k) * ty;
        const float rx = (float)(sx - 2.0 * floor(0.5 * sx));
        const float ry = (float)(sy - 2.0 * floor(0.5 * sy));
        e[4 * k + 0] = sinpif(rx);
        e[4 * k + 1] = cospif(rx);
        e[4 * k + 2] = sinpif(ry);
        e[4 * k + 3] = cospif(ry);
    }
    const float *w = reinterpret_cast<const float *>(w4);
#pragma unroll
    for (int c8 = 0; c8 < C / 8; ++c8) {
        float a[8];
        if constexpr (BF16) {
            uint4 *ptr = reinterpret_cast<uint4 *>(static_cast<uint16_t *>(p.feat[m]) + q * C) + c8;
            const uint4 r = *ptr;
            const unsigned wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[2 * j] = bf2f((uint16_t)(wd[j] & 0xffffu));
                a[2 * j + 1] = bf2f((uint16_t)(wd[j] >> 16));
            }
        } else {
            const float4 *ptr = reinterpret_cast<const float4 *>(static_cast<float *>(p.feat[m]) + q * C) + 2 * c8;
            const float4 r0 = ptr[0], r1 = ptr[1];
            a[0] = r0.x; a[1] = r0.y; a[2] = r0.z; a[3] = r0.w;
            a[4] = r1.x; a[5] = r1.y; a[6] = r1.z; a[7] = r1.w;
        }
#pragma unroll
        for (int i = 0; i < 32; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = fmaf(e[i], w[i * C + 8 * c8 + j], a[j]);
        if constexpr (BF16) {
            uint4 r;
            r.x = f2bf(a[0]) | ((unsigned)f2bf(a[1]) << 16);
            r.y = f2bf(a[2]) | ((unsigned)f2bf(a[3]) << 16);
            r.z = f2bf(a[4]) | ((unsigned)f2bf(a[5]) << 16);
            r.w = f2bf(a[6]) | ((unsigned)f2bf(a[7]) << 16);
            reinterpret_cast<uint4 *>(static_cast<uint16_t *>(p.feat[m]) + q * C)[c8] = r;
        } else {
            float4 *ptr = reinterpret_cast<float4 *>(static_cast<float *>(p.feat[m]) + q * C) + 2 * c8;
            ptr[0] = make_float4(a[0], a[1], a[2], a[3]);
            ptr[1] = make_float4(a[4], a[5], a[6], a[7]);
        }
    }
}

template <int C>
void launch_c(const RayParams &p, dim3 grid, hipStream_t s) {
    if (p.bf16)
        hipLaunchKernelGGL((k_ray_encoding<C, true>), grid, dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_ray_encoding<C, false>), grid, dim3(256), 0, s, p);
}

}  // namespace

hipError_t launch_ray_encoding(const RayParams &p, hipStream_t s) {
    const dim3 grid((unsigned)((p.max_pixels + 255) / 256), (unsigned)p.V);
    switch (p.C) {
        case 8: launch_c<8>(p, grid, s); break;
        case 16: launch_c<16>(p, grid, s); break;
        case 32: launch_c<32>(p, grid, s); break;
        case 64: launch_c<64>(p, grid, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qk
