// k_render.hip -- the final render of an LDM (Sec. 3.1, Eq. 1, and
// Sec. 3.2.3 "Upsampling & Activation"): bilinear upsampling of the
// unactivated depth, density and blend-weight logits to the output grid,
// activation after the upsampling, back-projection of every input image onto
// every layer through the decoded depth, blending of the images with the
// blend weights and the front-to-back over composite.
//
// One thread per output pixel, 16 x 16 pixel tiles (a wave covers 16 x 4), so
// the neighbouring threads that share low-resolution logit taps and, at
// similar depths, image taps sit in the same wave.  With V a multiple of 4
// (template NV4 = V / 4) each layer first reads the four taps' V blend logits
// as float4 vectors, upsamples all of them and takes their maximum, so the
// per-view loop only exponentiates; other view counts run the softmax online
// (running maximum, rescaled sums).  Neither the weights nor the per-view
// samples are stored.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "uf_params.h"

namespace qk {
namespace {

// RGBA8 image m as a buffer resource: a load at a byte offset outside the
// image reads zero.  A tap outside the image is sent to kTapOOB, far past
// the end (images are under 1 GiB), never to a negative offset: the compiler
// may merge the loads of neighbouring taps or fold a constant into the
// instruction's immediate offset, and a negative register offset would then
// take a valid tap out of range with it.
constexpr int kTapOOB = 0x40000000;

__device__ inline __amdgpu_buffer_rsrc_t image_rsrc(const RenderParams &p, int m) {
    const int bytes = p.iH[m] * p.iW[m] * 4;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p.img[m]), 0, bytes, 0x00020000);
}

__device__ inline unsigned load_texel(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
}

// Byte c of a packed texel as a float 0..255.
__device__ inline float chan(unsigned t, int c) {
    return (float)((t >> (8 * c)) & 0xffu);
}

__device__ inline float sigmoid_(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

template <int NV4>
__global__ void __launch_bounds__(256) k_render_ibr(const RenderParams p) {
    // XCD-aware tile order: workgroups are dispatched round-robin over the
    // 8 XCDs, so workgroup i is given tile (i % 8) * per + i / 8 and each XCD
    // walks one contiguous band of 16-row tiles; with horizontal-ish
    // baselines the band's samples fall in a band of image rows that stays
    // in the XCD's L2
    const int tiles_x = (p.W + 15) >> 4;
    const int n = tiles_x * ((p.H + 15) >> 4);
    int tile;
    {
        const int i = blockIdx.x, xcd = i & 7, loc = i >> 3, q = n >> 3, rem = n & 7;
        tile = (xcd < rem) ? xcd * (q + 1) + loc : rem * (q + 1) + (xcd - rem) * q + loc;
    }
    const int x = (tile % tiles_x) * 16 + (threadIdx.x & 15);
    const int y = (tile / tiles_x) * 16 + (threadIdx.x >> 4);
    if (x >= p.W || y >= p.H) return;              // no barriers below

    // upsampling taps: source coordinate (x + 0.5) w / W - 0.5, clamped
    // below at 0; the second tap clamped to the last column / row
    double sx = ((double)x + 0.5) * p.rx - 0.5, sy = ((double)y + 0.5) * p.ry - 0.5;
    sx = sx < 0.0 ? 0.0 : sx;
    sy = sy < 0.0 ? 0.0 : sy;
    int x0 = (int)sx, y0 = (int)sy;                 // sx, sy >= 0: truncation is floor
    x0 = x0 < p.w - 1 ? x0 : p.w - 1;
    y0 = y0 < p.h - 1 ? y0 : p.h - 1;
    const int x1 = x0 + 1 < p.w ? x0 + 1 : p.w - 1, y1 = y0 + 1 < p.h ? y0 + 1 : p.h - 1;
    const double lxd = sx - x0, lyd = sy - y0;
    const float lx = (float)lxd, ly = (float)lyd;
    const int64_t hw = (int64_t)p.h * p.w;
    const int64_t t00 = (int64_t)y0 * p.w + x0, t10 = (int64_t)y0 * p.w + x1;
    const int64_t t01 = (int64_t)y1 * p.w + x0, t11 = (int64_t)y1 * p.w + x1;
    auto lerp_f = [&](float a00, float a10, float a01, float a11) {
        return (1.0f - ly) * ((1.0f - lx) * a00 + lx * a10) + ly * ((1.0f - lx) * a01 + lx * a11);
    };

    const double u = (double)x + 0.5, v = (double)y + 0.5;
    const int V = p.V, L = p.L;
    float Tr = 1.0f, out0 = 0.0f, out1 = 0.0f, out2 = 0.0f, dmap = 0.0f;

    for (int li = 0; li < L; ++li) {
        // depth: the logit is interpolated in double, since an error in it is
        // magnified by the parallax (up to ~1e3 px per unit of disparity)
        const float *D = p.depth_logit + li * hw;
        const double xd = (1.0 - lyd) * ((1.0 - lxd) * (double)D[t00] + lxd * (double)D[t10]) +
                          lyd * ((1.0 - lxd) * (double)D[t01] + lxd * (double)D[t11]);
        const double delta = ((double)(L - li) - 0.5) / (double)L;
        const double disp = (delta + (0.5 / (double)L) * (double)tanhf((float)xd)) * p.band + p.inv_far;
        const float depth = (float)(1.0 / disp);
        const float *S = p.sigma_logit + li * hw;
        const float alpha = sigmoid_(lerp_f(S[t00], S[t10], S[t01], S[t11]));

        // one view's image, back-projected through this layer's depth: the
        // four texels' loads are issued here and blended later (blend_view),
        // so the next view's loads are in flight while this one is blended
        struct Tex {
            unsigned a[4];
            float w[4];
        };
        auto issue_view = [&](int m, Tex &t) {
            const double *A = p.cam[m];
            const double pz = fma(A[6], u, fma(A[7], v, fma(A[11], disp, A[8])));
            const double qx = fma(A[0], u, fma(A[1], v, fma(A[9], disp, A[2])));
            const double qy = fma(A[3], u, fma(A[4], v, fma(A[10], disp, A[5])));
            const int iw = p.iW[m], ih = p.iH[m];
            // 1/pz: the hardware reciprocal refined by one Newton step (the
            // relative error squares, far below what the coordinates need)
            double rz = __builtin_amdgcn_rcp(pz);
            rz = fma(rz, fma(-pz, rz, 1.0), rz);
            const double fxc = qx * rz - 0.5, fyc = qy * rz - 0.5;
            const bool ok = (pz > 1e-6) && (fxc > -2.0) && (fxc < (double)(iw + 1)) &&
                            (fyc > -2.0) && (fyc < (double)(ih + 1));
            const double xf = floor(fxc), yf = floor(fyc);
            const float wx = (float)(fxc - xf), wy = (float)(fyc - yf);
            const int ix = ok ? (int)xf : -4, iy = ok ? (int)yf : -4;
            const bool vx0 = (unsigned)ix < (unsigned)iw, vx1 = (unsigned)(ix + 1) < (unsigned)iw;
            const bool vy0 = (unsigned)iy < (unsigned)ih, vy1 = (unsigned)(iy + 1) < (unsigned)ih;
            t.w[0] = (vx0 && vy0) ? (1.0f - wx) * (1.0f - wy) : 0.0f;
            t.w[1] = (vx1 && vy0) ? wx * (1.0f - wy) : 0.0f;
            t.w[2] = (vx0 && vy1) ? (1.0f - wx) * wy : 0.0f;
            t.w[3] = (vx1 && vy1) ? wx * wy : 0.0f;
            const __amdgpu_buffer_rsrc_t rs = image_rsrc(p, m);
            const int o = (iy * iw + ix) * 4;
            t.a[0] = load_texel(rs, (vx0 && vy0) ? o : kTapOOB);
            t.a[1] = load_texel(rs, (vx1 && vy0) ? o + 4 : kTapOOB);
            t.a[2] = load_texel(rs, (vx0 && vy1) ? o + 4 * iw : kTapOOB);
            t.a[3] = load_texel(rs, (vx1 && vy1) ? o + 4 * iw + 4 : kTapOOB);
        };
        // the bilinear sample of an issued view (texels 0..255)
        auto blend_view = [&](const Tex &t, float &s0, float &s1, float &s2) {
            s0 = t.w[0] * chan(t.a[0], 0) + t.w[1] * chan(t.a[1], 0) + t.w[2] * chan(t.a[2], 0) + t.w[3] * chan(t.a[3], 0);
            s1 = t.w[0] * chan(t.a[0], 1) + t.w[1] * chan(t.a[1], 1) + t.w[2] * chan(t.a[2], 1) + t.w[3] * chan(t.a[3], 1);
            s2 = t.w[0] * chan(t.a[0], 2) + t.w[1] * chan(t.a[1], 2) + t.w[2] * chan(t.a[2], 2) + t.w[3] * chan(t.a[3], 2);
        };
        auto sample_view = [&](int m, float &s0, float &s1, float &s2) {
            Tex t;
            issue_view(m, t);
            blend_view(t, s0, s1, s2);
        };

        // blend: softmax over the views of the upsampled logits
        const float *B = p.blend_logit + li * hw * V;
        float z = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
        if constexpr (NV4 > 0) {
            // all views' logits first (16-byte loads: V = 4 NV4 floats per
            // tap, and each tap's row starts on a 16-byte boundary), then
            // their maximum, then the views
            constexpr int NV = 4 * NV4;
            const float4 *B00 = reinterpret_cast<const float4 *>(B + t00 * NV);
            const float4 *B10 = reinterpret_cast<const float4 *>(B + t10 * NV);
            const float4 *B01 = reinterpret_cast<const float4 *>(B + t01 * NV);
            const float4 *B11 = reinterpret_cast<const float4 *>(B + t11 * NV);
            float xb[NV];
#pragma unroll
            for (int c = 0; c < NV4; ++c) {
                const float4 a = B00[c], b = B10[c], d = B01[c], e = B11[c];
                xb[4 * c + 0] = lerp_f(a.x, b.x, d.x, e.x);
                xb[4 * c + 1] = lerp_f(a.y, b.y, d.y, e.y);
                xb[4 * c + 2] = lerp_f(a.z, b.z, d.z, e.z);
                xb[4 * c + 3] = lerp_f(a.w, b.w, d.w, e.w);
            }
            float mx = xb[0];
#pragma unroll
            for (int m = 1; m < NV; ++m) mx = fmaxf(mx, xb[m]);
            // the views two at a time, two texel buffers in turn: the loads
            // of the next view are issued before this one is blended (not
            // unrolled further: the loop body's live values would take the
            // register file; the index is uniform)
            Tex ta, tb;
            issue_view(0, ta);
#pragma unroll 1
            for (int m = 0; m < NV; m += 2) {
                float s0, s1, s2;
                issue_view(m + 1, tb);               // NV is even
                const float e0 = __expf(xb[m] - mx);
                blend_view(ta, s0, s1, s2);
                z += e0;
                c0 = fmaf(e0, s0, c0);
                c1 = fmaf(e0, s1, c1);
                c2 = fmaf(e0, s2, c2);
                if (m + 2 < NV) issue_view(m + 2, ta);
                const float e1 = __expf(xb[m + 1] - mx);
                blend_view(tb, s0, s1, s2);
                z += e1;
                c0 = fmaf(e1, s0, c0);
                c1 = fmaf(e1, s1, c1);
                c2 = fmaf(e1, s2, c2);
            }
        } else {
            // online: running maximum, sums rescaled when it moves
            float mx = -3.0e38f;
            for (int m = 0; m < V; ++m) {
                const float xb = lerp_f(B[t00 * V + m], B[t10 * V + m], B[t01 * V + m], B[t11 * V + m]);
                if (xb > mx) {                       // move the reference
                    const float r = __expf(mx - xb);
                    z *= r; c0 *= r; c1 *= r; c2 *= r;
                    mx = xb;
                }
                const float e = __expf(xb - mx);
                float s0, s1, s2;
                sample_view(m, s0, s1, s2);
                z += e;
                c0 = fmaf(e, s0, c0);
                c1 = fmaf(e, s1, c1);
                c2 = fmaf(e, s2, c2);
            }
        }
        const float k = Tr * alpha * (1.0f / 255.0f) / z;   // beta = e / z; texels v / 255
        out0 = fmaf(k, c0, out0);
        out1 = fmaf(k, c1, out1);
        out2 = fmaf(k, c2, out2);
        dmap = fmaf(Tr * alpha, depth, dmap);
        Tr *= 1.0f - alpha;
    }
    const int64_t q = (int64_t)y * p.W + x;
    p.rgb[q * 3 + 0] = out0;
    p.rgb[q * 3 + 1] = out1;
    p.rgb[q * 3 + 2] = out2;
    if (p.acc != nullptr) p.acc[q] = 1.0f - Tr;
    if (p.depth != nullptr) p.depth[q] = dmap;
}

}  // namespace

hipError_t launch_render_ibr(const RenderParams &p, hipStream_t s) {
    const int tiles = ((p.W + 15) / 16) * ((p.H + 15) / 16);
    const dim3 g(tiles), b(256);
    // the vector path reads 16 bytes at a time: V a multiple of 4 and the
    // logits 16-byte aligned (the C-ABI asks only for 4)
    const bool vec = p.V % 4 == 0 && (reinterpret_cast<uintptr_t>(p.blend_logit) & 15) == 0;
    switch (vec ? p.V / 4 : 0) {
    case 1: hipLaunchKernelGGL(k_render_ibr<1>, g, b, 0, s, p); break;
    case 2: hipLaunchKernelGGL(k_render_ibr<2>, g, b, 0, s, p); break;
    case 3: hipLaunchKernelGGL(k_render_ibr<3>, g, b, 0, s, p); break;
    case 4: hipLaunchKernelGGL(k_render_ibr<4>, g, b, 0, s, p); break;
    default: hipLaunchKernelGGL(k_render_ibr<0>, g, b, 0, s, p); break;
    }
    return hipGetLastError();
}

}  // namespace qk
