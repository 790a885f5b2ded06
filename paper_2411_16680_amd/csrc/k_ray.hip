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
// Two forms.  Per pixel (k_ray_encoding): one thread per map pixel
// evaluates its own encoding.  Low resolution, as the paper does it
// (k_ray_lowres + k_ray_upsample_add): the projected encoding is evaluated
// once per pixel of a coarse grid, then every map pixel adds its bilinear
// upsampling -- projection and bilinear interpolation are both linear, so
// projecting first gives the same values and leaves C channels, not 32, to
// interpolate; the second pass is bound by the feature maps' HBM traffic.
//
// The encoding runs in double up to the sinusoids (the top octave scales
// its argument by 128 pi): sin(pi t) and cos(pi t) from their Taylor
// series on a quarter period after an exact quadrant reduction, then each
// higher octave by the double-angle identities sin 2a = 2 sin a cos a,
// cos 2a = (cos a - sin a)(cos a + sin a) -- the angle error doubles per
// octave, about 1e-14 at the top.  The projection, in float, reads the
// 32 x C weights as wave-uniform operands (scalar loads or LDS broadcasts)
// and accumulates on top of the feature, which is rounded once at the store.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

// pi^n / n!, for the Taylor coefficients
__host__ __device__ constexpr double pi_pow_over_fact(int n) {
    double r = 1.0;
    for (int i = 1; i <= n; ++i) r *= 3.141592653589793 / (double)i;
    return r;
}

// sin(pi x) and cos(pi x) for |x| <= 1/4 (|pi x| <= 0.79): Taylor series to
// x^17 and x^16, the first omitted terms below 1e-17
__device__ inline void sincospi_quarter(double x, double &s, double &c) {
    constexpr double P1 = pi_pow_over_fact(1), P2 = pi_pow_over_fact(2),
                     P3 = pi_pow_over_fact(3), P4 = pi_pow_over_fact(4),
                     P5 = pi_pow_over_fact(5), P6 = pi_pow_over_fact(6),
                     P7 = pi_pow_over_fact(7), P8 = pi_pow_over_fact(8),
                     P9 = pi_pow_over_fact(9), P10 = pi_pow_over_fact(10),
                     P11 = pi_pow_over_fact(11), P12 = pi_pow_over_fact(12),
                     P13 = pi_pow_over_fact(13), P14 = pi_pow_over_fact(14),
                     P15 = pi_pow_over_fact(15), P16 = pi_pow_over_fact(16),
                     P17 = pi_pow_over_fact(17);
    const double z = x * x;
    double ps = fma(P17, z, -P15);
    ps = fma(ps, z, P13);
    ps = fma(ps, z, -P11);
    ps = fma(ps, z, P9);
    ps = fma(ps, z, -P7);
    ps = fma(ps, z, P5);
    ps = fma(ps, z, -P3);
    ps = fma(ps, z, P1);
    s = ps * x;
    double pc = fma(P16, z, -P14);
    pc = fma(pc, z, P12);
    pc = fma(pc, z, -P10);
    pc = fma(pc, z, P8);
    pc = fma(pc, z, -P6);
    pc = fma(pc, z, P4);
    pc = fma(pc, z, -P2);
    c = fma(pc, z, 1.0);
}

// sin(pi t), cos(pi t) for |t| <= 1: t = f + q/2 with q = rint(2t) and
// |f| <= 1/4 (both exact), then a rotation by q quarter turns
__device__ inline void sincospi_unit(double t, double &s, double &c) {
    const double q = rint(2.0 * t);
    double sf, cf;
    sincospi_quarter(fma(-0.5, q, t), sf, cf);
    const int qi = ((int)q) & 3;
    s = qi == 0 ? sf : qi == 1 ? cf : qi == 2 ? -sf : -cf;
    c = qi == 0 ? cf : qi == 1 ? -sf : qi == 2 ? -cf : sf;
}

// 1 / n!
__host__ __device__ constexpr double inv_fact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r /= (double)i;
    return r;
}

// tanh(x) = 1 - 2 / (e^(2x) + 1), to an absolute error near 1e-16 (the
// octaves need absolute accuracy in t, so the cancellation near x = 0 costs
// nothing): e^y = 2^n e^r with n = rint(y / ln 2), r = y - n ln 2,
// |r| <= 0.35, e^r by its Taylor series to r^14; y is clamped to [-40, 40],
// where tanh is +-1 to double precision; the quotient by a reciprocal and
// two Newton steps.
__device__ inline double tanh_abs(double x) {
    constexpr double kLn2 = 0.6931471805599453, kLog2e = 1.4426950408889634;
    const double y = fmin(fmax(2.0 * x, -40.0), 40.0);
    const double n = rint(y * kLog2e);
    const double r = fma(-n, kLn2, y);
    double p = inv_fact(14);
#pragma unroll
    for (int k = 13; k >= 0; --k) p = fma(p, r, inv_fact(k));
    const double d = ldexp(p, (int)n) + 1.0;
    double q = __builtin_amdgcn_rcp(d);
    q = fma(q, fma(-d, q, 1.0), q);
    q = fma(q, fma(-d, q, 1.0), q);
    return fma(-2.0, q, 1.0);
}

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// The 32 sinusoids of pixel (x, y) of view m's grid (the grid the
// composed D[m] was made for).
__device__ inline void ray_sinusoids(const RayParams &p, int m, int x, int y, float e[32]) {
    const double u = (double)x + 0.5, v = (double)y + 0.5;
    const double *D = p.D[m], *o = p.o[m];
    const double dx = fma(D[0], u, fma(D[1], v, D[2]));
    const double dy = fma(D[3], u, fma(D[4], v, D[5]));
    const double dz = fma(D[6], u, fma(D[7], v, D[8]));
    const double rz = o[2] / dz;
    const double ax = p.inv_band * fma(-rz, dx, o[0]);
    const double ay = p.inv_band * fma(-rz, dy, o[1]);
    const double tx = tanh_abs(fma(p.kx0, ax, p.kx1 * ay));
    const double ty = tanh_abs(fma(p.ky0, ax, p.ky1 * ay));
    double sx, cx, sy, cy;
    sincospi_unit(tx, sx, cx);
    sincospi_unit(ty, sy, cy);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        e[4 * k + 0] = (float)sx;
        e[4 * k + 1] = (float)cx;
        e[4 * k + 2] = (float)sy;
        e[4 * k + 3] = (float)cy;
        if (k < 7) {
            const double s2x = 2.0 * sx * cx, c2x = (cx - sx) * (cx + sx);
            const double s2y = 2.0 * sy * cy, c2y = (cy - sy) * (cy + sy);
            sx = s2x; cx = c2x; sy = s2y; cy = c2y;
        }
    }
}

// 8 channels of a feature pixel as float, and back (rounded once)
template <bool BF16>
__device__ inline void load8(const void *base, int64_t off, float a[8]) {
    if constexpr (BF16) {
        const uint4 r = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(base) + off);
        const unsigned wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[2 * j] = bf2f((uint16_t)(wd[j] & 0xffffu));
            a[2 * j + 1] = bf2f((uint16_t)(wd[j] >> 16));
        }
    } else {
        const float4 *ptr = reinterpret_cast<const float4 *>(static_cast<const float *>(base) + off);
        const float4 r0 = ptr[0], r1 = ptr[1];
        a[0] = r0.x; a[1] = r0.y; a[2] = r0.z; a[3] = r0.w;
        a[4] = r1.x; a[5] = r1.y; a[6] = r1.z; a[7] = r1.w;
    }
}

template <bool BF16>
__device__ inline void store8(void *base, int64_t off, const float a[8]) {
    if constexpr (BF16) {
        uint4 r;
        r.x = f2bf(a[0]) | ((unsigned)f2bf(a[1]) << 16);
        r.y = f2bf(a[2]) | ((unsigned)f2bf(a[3]) << 16);
        r.z = f2bf(a[4]) | ((unsigned)f2bf(a[5]) << 16);
        r.w = f2bf(a[6]) | ((unsigned)f2bf(a[7]) << 16);
        *reinterpret_cast<uint4 *>(static_cast<uint16_t *>(base) + off) = r;
    } else {
        float4 *ptr = reinterpret_cast<float4 *>(static_cast<float *>(base) + off);
        ptr[0] = make_float4(a[0], a[1], a[2], a[3]);
        ptr[1] = make_float4(a[4], a[5], a[6], a[7]);
    }
}

// The 32 x C weights: for C <= 16 through the scalar unit (a wave-uniform
// index into the constant address space compiles to scalar loads and the
// FMAs take the weight as an SGPR operand); for wider C the scalar loads
// come in small pieces that stall, so the workgroup stages the weights in
// LDS and every read is a broadcast.
typedef const __attribute__((address_space(4))) float *wptr_t;

template <int C>
struct Weights {
    static constexpr bool kLds = C >= 32;
    static constexpr int kBuf = kLds ? 8 * C : 1;    // float4s of LDS
    __device__ static void stage(const RayParams &p, float4 *buf) {
        if constexpr (kLds) {
            for (int i = threadIdx.x; i < 8 * C; i += 256) buf[i] = reinterpret_cast<const float4 *>(p.Wr)[i];
            __syncthreads();
        }
    }
};

// a[j] += sum_i e[i] w[i][c0 + j], j < 8
template <int C, typename WP>
__device__ inline void project8(const float e[32], WP w, int c0, float a[8]) {
#pragma unroll
    for (int i = 0; i < 32; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = fmaf(e[i], w[i * C + c0 + j], a[j]);
}

template <int C>
__device__ inline void project8_w(const float e[32], const RayParams &p, const float4 *lds, int c0,
                                  float a[8]) {
    if constexpr (Weights<C>::kLds)
        project8<C>(e, reinterpret_cast<const float *>(lds), c0, a);
    else
        project8<C>(e, (wptr_t)p.Wr, c0, a);
}

// Per-pixel form: every pixel of every map evaluates its own encoding.
template <int C, bool BF16>
__global__ void __launch_bounds__(256) k_ray_encoding(const RayParams p) {
    __shared__ float4 wbuf[Weights<C>::kBuf];
    Weights<C>::stage(p, wbuf);                  // the only barrier
    const int m = blockIdx.y;
    const int fw = p.fW[m];
    const int64_t np = (int64_t)p.fH[m] * fw;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= np) return;
    const int y = (int)(q / fw), x = (int)(q - (int64_t)y * fw);
    float e[32];
    ray_sinusoids(p, m, x, y, e);
    // all of the pixel's channels are read before any is written: the source
    // may be the map itself, and the compiler cannot move a load of one
    // pointer above a store through another that may alias it
    float a[C / 8][8];
#pragma unroll
    for (int c8 = 0; c8 < C / 8; ++c8) load8<BF16>(p.src[m], q * C + 8 * c8, a[c8]);
#pragma unroll
    for (int c8 = 0; c8 < C / 8; ++c8) {
        project8_w<C>(e, p, wbuf, 8 * c8, a[c8]);
        store8<BF16>(p.feat[m], q * C + 8 * c8, a[c8]);
    }
}

// Low-resolution form, first pass: the projected encoding P = e Wr of every
// pixel of the (lH, lW) grid, float32, into the workspace [V][lH][lW][C].
template <int C>
__global__ void __launch_bounds__(256) k_ray_lowres(const RayParams p) {
    __shared__ float4 wbuf[Weights<C>::kBuf];
    Weights<C>::stage(p, wbuf);                  // the only barrier
    const int m = blockIdx.y;
    const int64_t np = (int64_t)p.lH * p.lW;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= np) return;
    const int y = (int)(q / p.lW), x = (int)(q - (int64_t)y * p.lW);
    float e[32];
    ray_sinusoids(p, m, x, y, e);
    float *dst = p.P + ((int64_t)m * np + q) * C;
#pragma unroll
    for (int c8 = 0; c8 < C / 8; ++c8) {
        float a[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        project8_w<C>(e, p, wbuf, 8 * c8, a);
        store8<false>(dst, 8 * c8, a);
    }
}

// Low-resolution form, second pass, for a low-resolution grid no finer than
// the map (lH <= fH, lW <= fW): a workgroup takes a segment of 256 / (C/8)
// pixels of one map row, one thread per (pixel, 8 channels).  Bilinear
// interpolation is separable: the workgroup first blends the two low-res
// rows its map row falls between into LDS (the segment spans at most
// 256 / (C/8) + 2 low-res columns), then every thread interpolates between
// two LDS columns and adds the result to its feature.  P is a few MB and
// stays in L2; the feature maps are read and written once.
template <int C, bool BF16>
__global__ void __launch_bounds__(256) k_ray_upsample_add(const RayParams p) {
    constexpr int NC = C / 8, SEG = 256 / NC, MAXCOL = SEG + 3;
    __shared__ float4 rowb[MAXCOL * C / 4];      // blended low-res row segment [col][C]
    const int m = blockIdx.z;
    const int fw = p.fW[m], fh = p.fH[m];
    const int y = blockIdx.y, xs = blockIdx.x * SEG;
    if (y >= fh || xs >= fw) return;             // uniform over the workgroup
    const int lh = p.lH, lw = p.lW;
    const float ry = (float)lh / (float)fh, rx = (float)lw / (float)fw;
    const float sy = fmaxf(((float)y + 0.5f) * ry - 0.5f, 0.0f);
    const int y0 = min((int)sy, lh - 1), y1 = min(y0 + 1, lh - 1);
    const float ly = sy - (float)y0;
    const int xe = min(xs + SEG, fw) - 1;
    const int cx_lo = min((int)fmaxf(((float)xs + 0.5f) * rx - 0.5f, 0.0f), lw - 1);
    const int cx_hi = min(min((int)fmaxf(((float)xe + 0.5f) * rx - 0.5f, 0.0f), lw - 1) + 1, lw - 1);
    const int ncol = cx_hi - cx_lo + 1;          // <= SEG + 2 when lW <= fW
    const float4 *P0 = reinterpret_cast<const float4 *>(p.P + (((int64_t)m * lh + y0) * lw + cx_lo) * C);
    const float4 *P1 = reinterpret_cast<const float4 *>(p.P + (((int64_t)m * lh + y1) * lw + cx_lo) * C);
    for (int k = threadIdx.x; k < ncol * (C / 4); k += 256) {
        const float4 a = P0[k], b = P1[k];
        rowb[k] = make_float4(fmaf(ly, b.x - a.x, a.x), fmaf(ly, b.y - a.y, a.y),
                              fmaf(ly, b.z - a.z, a.z), fmaf(ly, b.w - a.w, a.w));
    }
    __syncthreads();
    const int x = xs + threadIdx.x / NC, c0 = 8 * (threadIdx.x % NC);
    if (x > xe) return;
    const float sx = fmaxf(((float)x + 0.5f) * rx - 0.5f, 0.0f);
    const int x0 = min((int)sx, lw - 1), x1 = min(x0 + 1, lw - 1);
    const float lx = sx - (float)x0;
    const float *R = reinterpret_cast<const float *>(rowb);
    float t0[8], t1[8], a[8];
    load8<false>(R, (x0 - cx_lo) * C + c0, t0);
    load8<false>(R, (x1 - cx_lo) * C + c0, t1);
    const int64_t q = (int64_t)y * fw + x;
    load8<BF16>(p.src[m], q * C + c0, a);
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] += fmaf(lx, t1[j] - t0[j], t0[j]);
    store8<BF16>(p.feat[m], q * C + c0, a);
}

// The same for any low-resolution grid (also one finer than the map): one
// thread per (map pixel, 8 channels) reads the four taps of P directly.
template <int C, bool BF16>
__global__ void __launch_bounds__(256) k_ray_upsample_add_any(const RayParams p) {
    constexpr int NC = C / 8;
    const int m = blockIdx.y;
    const int fw = p.fW[m], fh = p.fH[m];
    const int64_t np = (int64_t)fh * fw;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= np * NC) return;
    const int64_t q = i / NC;
    const int c0 = 8 * (int)(i - q * NC);
    const int y = (int)(q / fw), x = (int)(q - (int64_t)y * fw);
    const int lh = p.lH, lw = p.lW;
    const float sy = fmaxf(((float)y + 0.5f) * ((float)lh / (float)fh) - 0.5f, 0.0f);
    const float sx = fmaxf(((float)x + 0.5f) * ((float)lw / (float)fw) - 0.5f, 0.0f);
    const int y0 = min((int)sy, lh - 1), x0 = min((int)sx, lw - 1);
    const int y1 = min(y0 + 1, lh - 1), x1 = min(x0 + 1, lw - 1);
    const float ly = sy - (float)y0, lx = sx - (float)x0;
    const float *Pm = p.P + (int64_t)m * lh * lw * C + c0;
    float t00[8], t10[8], t01[8], t11[8], a[8];
    load8<false>(Pm, ((int64_t)y0 * lw + x0) * C, t00);
    load8<false>(Pm, ((int64_t)y0 * lw + x1) * C, t10);
    load8<false>(Pm, ((int64_t)y1 * lw + x0) * C, t01);
    load8<false>(Pm, ((int64_t)y1 * lw + x1) * C, t11);
    load8<BF16>(p.src[m], q * C + c0, a);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float top = fmaf(lx, t10[j] - t00[j], t00[j]);
        const float bot = fmaf(lx, t11[j] - t01[j], t01[j]);
        a[j] += fmaf(ly, bot - top, top);
    }
    store8<BF16>(p.feat[m], q * C + c0, a);
}

template <int C>
hipError_t launch_c(const RayParams &p, hipStream_t s) {
    const unsigned V = (unsigned)p.V;
    bool same = p.lH > 0;                        // low grid == every map grid: nothing to upsample
    for (int m = 0; m < p.V; ++m) same = same && p.lH == p.fH[m] && p.lW == p.fW[m];
    if (p.lH > 0 && !same) {
        hipLaunchKernelGGL((k_ray_lowres<C>), dim3((unsigned)(((int64_t)p.lH * p.lW + 255) / 256), V),
                           dim3(256), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        bool coarse = true;                      // the grid is no finer than any map
        int maxh = 0, maxw = 0;
        for (int m = 0; m < p.V; ++m) {
            coarse = coarse && p.lH <= p.fH[m] && p.lW <= p.fW[m];
            maxh = p.fH[m] > maxh ? p.fH[m] : maxh;
            maxw = p.fW[m] > maxw ? p.fW[m] : maxw;
        }
        if (coarse) {
            constexpr int SEG = 256 / (C / 8);
            const dim3 g((unsigned)((maxw + SEG - 1) / SEG), (unsigned)maxh, V);
            if (p.bf16)
                hipLaunchKernelGGL((k_ray_upsample_add<C, true>), g, dim3(256), 0, s, p);
            else
                hipLaunchKernelGGL((k_ray_upsample_add<C, false>), g, dim3(256), 0, s, p);
        } else {
            const dim3 g((unsigned)((p.max_pixels * (C / 8) + 255) / 256), V);
            if (p.bf16)
                hipLaunchKernelGGL((k_ray_upsample_add_any<C, true>), g, dim3(256), 0, s, p);
            else
                hipLaunchKernelGGL((k_ray_upsample_add_any<C, false>), g, dim3(256), 0, s, p);
        }
        return hipGetLastError();
    }
    const dim3 g((unsigned)((p.max_pixels + 255) / 256), V);
    if (p.bf16)
        hipLaunchKernelGGL((k_ray_encoding<C, true>), g, dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_ray_encoding<C, false>), g, dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ray_encoding(const RayParams &p, hipStream_t s) {
    switch (p.C) {
        case 8: return launch_c<8>(p, s);
        case 16: return launch_c<16>(p, s);
        case 32: return launch_c<32>(p, s);
        case 64: return launch_c<64>(p, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qk
