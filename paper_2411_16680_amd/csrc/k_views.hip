// k_views.hip -- render of a decoded intermediate LDM into every input view
// (Sec. 3.2.2 "Decoding and rendering the intermediate LDM", Eq. 2): the
// projection operator, the transpose of the bilinear back-projection, splats
// each layer-pixel's colour and density into the four view pixels around its
// reprojection (per layer, per view, unnormalised), then each view composites
// its projected layers front to back.
//
// Three launches: a fill kernel clears the projected layers (no
// hipMemsetAsync, so the call can be captured in a graph); k_splat, one
// thread per (view, layer-pixel), scatters with float atomics regrouped
// through LDS so that eight adjacent lanes add the four channels of a tap
// and of its right neighbour (32 contiguous bytes) instead of 64 lanes
// hitting 64 scattered words;
// k_views_composite, one thread per view pixel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

__global__ void __launch_bounds__(256) k_views_zero(const ViewsParams p) {
    const int64_t n4 = p.ws_floats >> 2;
    float4 *w = reinterpret_cast<float4 *>(p.ws);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256)
        w[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Per wave: 64 layer-pixels x 2 tap rows = 128 entries -- the float index
// in ws of the row's left and right taps (-1 = dropped) and their weights --
// and the 64 payloads (r, g, b, alpha).  A row's two taps are neighbours in
// the plane, so one entry is 32 contiguous bytes.
struct SplatSlice {
    int4 e[128];         // dst_left, dst_right, weight bits left, right
    float4 val[64];
};

__global__ void __launch_bounds__(256) k_splat(const ViewsParams p) {
    __shared__ SplatSlice sl[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    SplatSlice &s = sl[wave];
    // one (view, 256 layer-pixels) chunk per workgroup, views slowest, in an
    // XCD-aware order (workgroups are dispatched round-robin over the 8 XCDs:
    // workgroup i takes chunk (i % 8) * per + i / 8), so each XCD scatters
    // the rows of one layer into one view at a time and the band of the
    // view's plane those rows reach stays in its L2
    const int64_t bpv = (p.N + 255) / 256, n = bpv * p.V;
    int64_t chunk;
    {
        const int64_t i = blockIdx.x, xcd = i & 7, loc = i >> 3, q8 = n >> 3, rem = n & 7;
        chunk = (xcd < rem) ? xcd * (q8 + 1) + loc : rem * (q8 + 1) + (xcd - rem) * q8 + loc;
    }
    const int m = (int)(chunk / bpv);
    const int64_t q = (chunk - (int64_t)m * bpv) * 256 + threadIdx.x;   // layer-pixel
    const bool live = q < p.N;
    const int64_t hw = (int64_t)p.H * p.W;
    const int l = live ? (int)(q / hw) : 0;
    const int64_t r = live ? q - (int64_t)l * hw : 0;
    const int y = (int)(r / p.W), x = (int)(r - (int64_t)y * p.W);
    const double u = (double)x + 0.5, v = (double)y + 0.5;
    int4 row0 = make_int4(-1, -1, 0, 0), row1 = make_int4(-1, -1, 0, 0);
    if (live) {
        s.val[lane] = make_float4(p.color[q * 3 + 0], p.color[q * 3 + 1], p.color[q * 3 + 2],
                                  p.alpha[q]);
        const double invd = 1.0 / (double)p.depth[q];
        const double *A = p.cam[m];
        const int vw = p.vW[m], vh = p.vH[m];
        const double pz = fma(A[6], u, fma(A[7], v, fma(A[11], invd, A[8])));
        const double qx = fma(A[0], u, fma(A[1], v, fma(A[9], invd, A[2])));
        const double qy = fma(A[3], u, fma(A[4], v, fma(A[10], invd, A[5])));
        const double rz = 1.0 / pz;
        const double fxc = qx * rz - 0.5, fyc = qy * rz - 0.5;
        if ((pz > 1e-6) && (fxc > -2.0) && (fxc < (double)(vw + 1)) && (fyc > -2.0) &&
            (fyc < (double)(vh + 1))) {
            const double xf = floor(fxc), yf = floor(fyc);
            const float fx = (float)(fxc - xf), fy = (float)(fyc - yf);
            const int ix = (int)xf, iy = (int)yf;
            const int64_t base = p.sbase[m] + (int64_t)l * vh * vw * 4;
            const bool vx0 = (unsigned)ix < (unsigned)vw, vx1 = (unsigned)(ix + 1) < (unsigned)vw;
            const bool vy0 = (unsigned)iy < (unsigned)vh, vy1 = (unsigned)(iy + 1) < (unsigned)vh;
            const int64_t o0 = base + ((int64_t)iy * vw + ix) * 4, o1 = o0 + (int64_t)vw * 4;
            row0 = make_int4((vx0 && vy0) ? (int)o0 : -1, (vx1 && vy0) ? (int)o0 + 4 : -1,
                             __float_as_int((1.0f - fx) * (1.0f - fy)),
                             __float_as_int(fx * (1.0f - fy)));
            row1 = make_int4((vx0 && vy1) ? (int)o1 : -1, (vx1 && vy1) ? (int)o1 + 4 : -1,
                             __float_as_int((1.0f - fx) * fy), __float_as_int(fx * fy));
        }
    }
    s.e[2 * lane] = row0;
    s.e[2 * lane + 1] = row1;
    __syncthreads();
    // lanes 8k..8k+7 add entry 8 j + k: the left tap's four channels, then
    // the right tap's
    const int c = lane & 3, right = (lane >> 2) & 1;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const int en = 8 * j + (lane >> 3);
        const int4 ent = s.e[en];
        const int d = right ? ent.y : ent.x;
        if (d >= 0) {
            const float4 pv = s.val[en >> 1];
            const float val = c == 0 ? pv.x : c == 1 ? pv.y : c == 2 ? pv.z : pv.w;
            unsafeAtomicAdd(p.ws + d + c, __int_as_float(right ? ent.w : ent.z) * val);
        }
    }
}

__global__ void __launch_bounds__(256) k_views_composite(const ViewsParams p) {
    const int m = blockIdx.y;
    const int64_t np = (int64_t)p.vH[m] * p.vW[m];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    const float4 *S = reinterpret_cast<const float4 *>(p.ws + p.sbase[m]);
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    for (int l = 0; l < p.L; ++l) {
        const float4 s = S[(int64_t)l * np + i];
        const float w = T * s.w;
        c0 = fmaf(w, s.x, c0);
        c1 = fmaf(w, s.y, c1);
        c2 = fmaf(w, s.z, c2);
        T *= 1.0f - s.w;
    }
    float *rgb = p.rgb[m];
    rgb[i * 3 + 0] = c0;
    rgb[i * 3 + 1] = c1;
    rgb[i * 3 + 2] = c2;
    if (p.acc[m] != nullptr) p.acc[m][i] = 1.0f - T;
}

}  // namespace

hipError_t launch_render_to_views(const ViewsParams &p, hipStream_t s) {
    const int64_t n4 = p.ws_floats / 4;
    const int zb = (int)((n4 + 255) / 256 < 8192 ? (n4 + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_views_zero, dim3(zb > 0 ? zb : 1), dim3(256), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_splat, dim3((unsigned)(((p.N + 255) / 256) * p.V)), dim3(256), 0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_views_composite, dim3((unsigned)((p.max_view_pixels + 255) / 256), p.V),
                       dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
