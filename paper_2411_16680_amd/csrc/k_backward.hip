// k_backward.hip -- adjoint of the float32 Update & Fuse step and of the
// front-to-back composite (gfx950).
//
// The paper trains through generic differentiable rendering and prints no
// adjoint; this one is derived by the chain rule from the forward of
// Sec. 3.1-3.3 (reprojection, bilinear back-projection, attention across
// views, decode heads, over composite).  Nothing is taped: each layer-pixel
// re-gathers its samples and recomputes its attention, so the extra memory
// is 16 bytes per layer-pixel plus per-workgroup weight-gradient partials.
//
// Four launches on the caller's stream:
//   k_zero_maps         clear the feature-map gradients (scatter targets)
//   k_composite_adjoint one thread per pixel: for every layer, the gradient
//                       of rgb with respect to its colour and alpha
//                       (dc = g T a, da = g . T (c - B_behind))
//   k_uf_backward<C>    one thread per layer-pixel, persistent workgroups:
//                       forward recompute with the key folded into the query
//                       (a_m = (scale W_k q) . s_m) and the value folded out
//                       (o = (sum_m p_m s_m) W_v), then the adjoint of
//                       decode, residual, W_o, W_v, softmax, W_k, W_q and
//                       RMSNorm; a second pass over the views scatters dI
//                       with float atomics (rows of C channels regrouped
//                       through LDS so that each atomic instruction covers
//                       whole rows) and differentiates the sample
//                       position with respect to depth.  Weight gradients are
//                       sums over layer-pixels of outer products; each wave
//                       forms them on the matrix cores (v_mfma_f32_16x16x4_f32,
//                       pixels along K), each workgroup writes one partial.
//   k_reduce_wgrad      sums the partials in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "uf_params.h"

namespace qk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(3))) float lds_f32;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ inline float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }

// ---------------------------------------------------------------------------
// Feature-map gradients start at zero: blockIdx.y is the view.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_zero_maps(const BwdParams p) {
    const int m = blockIdx.y;
    const int64_t n4 = (int64_t)p.fH[m] * p.fW[m] * p.C / 4;
    float4 *d = reinterpret_cast<float4 *>(p.dfeat[m]);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kBlock)
        d[i] = z;
}

// ---------------------------------------------------------------------------
// Composite adjoint, one thread per pixel.  rgb = sum_l T_l a_l c_l with
// T_l = prod_{j<l} (1 - a_j).  With B_l the composite of layers l..L-1 on
// their own, d rgb / d c_l = T_l a_l and d rgb / d a_l = T_l (c_l - B_{l+1}).
// The front-to-back pass stores (c_l, T_l); the back-to-front pass replaces
// them by (g T_l a_l, g . T_l (c_l - B_{l+1})).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_composite_adjoint(const BwdParams p) {
    const int64_t npix = (int64_t)p.H * p.W;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= npix) return;
    const int C = p.C;
    float T = 1.0f;
    for (int l = 0; l < p.L; ++l) {
        const int64_t e = (int64_t)l * npix + q;
        const float4 *f = reinterpret_cast<const float4 *>(p.F_out + e * C);
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        for (int c4 = 0; c4 < C / 4; ++c4) {
            const float4 v = f[c4];
            const float fv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float *wc = p.W_color + (4 * c4 + i) * 3;
                x0 = fmaf(fv[i], wc[0], x0);
                x1 = fmaf(fv[i], wc[1], x1);
                x2 = fmaf(fv[i], wc[2], x2);
            }
        }
        reinterpret_cast<float4 *>(p.comp)[e] = make_float4(sigm(x0), sigm(x1), sigm(x2), T);
        T *= 1.0f - p.alpha_out[e];
    }
    const float g0 = p.d_rgb[q * 3 + 0], g1 = p.d_rgb[q * 3 + 1], g2 = p.d_rgb[q * 3 + 2];
    float B0 = 0.f, B1 = 0.f, B2 = 0.f;
    for (int l = p.L - 1; l >= 0; --l) {
        const int64_t e = (int64_t)l * npix + q;
        const float4 ct = reinterpret_cast<const float4 *>(p.comp)[e];
        const float a = p.alpha_out[e];
        const float Ta = ct.w * a;
        const float da = ct.w * (g0 * (ct.x - B0) + g1 * (ct.y - B1) + g2 * (ct.z - B2));
        reinterpret_cast<float4 *>(p.comp)[e] = make_float4(g0 * Ta, g1 * Ta, g2 * Ta, da);
        B0 = fmaf(a, ct.x - B0, B0);
        B1 = fmaf(a, ct.y - B1, B1);
        B2 = fmaf(a, ct.z - B2, B2);
    }
}

// ---------------------------------------------------------------------------
// Standalone composite adjoint (the operator O on its own), one thread per
// pixel: d rgb / d c_l = T_l a_l, d rgb / d a_l = T_l (c_l - B_{l+1}) and
// d acc / d a_l = T_l P_{l+1}, with B_{l+1} the composite of the layers
// behind l and P_{l+1} the product of their (1 - a).  The front-to-back
// pass parks T_l in d_alpha (each thread touches only its own pixel); the
// back-to-front pass accumulates B and P and overwrites it.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_composite_backward(const CompBwdParams p) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= p.npix) return;
    float T = 1.0f;
    for (int l = 0; l < p.L; ++l) {
        const int64_t e = (int64_t)l * p.npix + q;
        p.d_alpha[e] = T;
        T *= 1.0f - p.alpha[e];
    }
    const float g0 = p.d_rgb[q * 3 + 0], g1 = p.d_rgb[q * 3 + 1], g2 = p.d_rgb[q * 3 + 2];
    const float gA = p.d_acc != nullptr ? p.d_acc[q] : 0.0f;
    float B0 = 0.f, B1 = 0.f, B2 = 0.f, P = 1.0f;
    for (int l = p.L - 1; l >= 0; --l) {
        const int64_t e = (int64_t)l * p.npix + q;
        const float Tl = p.d_alpha[e];
        const float a = p.alpha[e];
        const float c0 = p.color[e * 3 + 0], c1 = p.color[e * 3 + 1], c2 = p.color[e * 3 + 2];
        if (p.d_color != nullptr) {
            const float Ta = Tl * a;
            p.d_color[e * 3 + 0] = g0 * Ta;
            p.d_color[e * 3 + 1] = g1 * Ta;
            p.d_color[e * 3 + 2] = g2 * Ta;
        }
        p.d_alpha[e] = Tl * (g0 * (c0 - B0) + g1 * (c1 - B1) + g2 * (c2 - B2) + gA * P);
        B0 = fmaf(a, c0 - B0, B0);
        B1 = fmaf(a, c1 - B1, B1);
        B2 = fmaf(a, c2 - B2, B2);
        P *= 1.0f - a;
    }
}

// ---------------------------------------------------------------------------
// One view's sample of one layer-pixel: position (double, as in the float32
// forward), its derivative with respect to depth, the four clamped taps and
// their bilinear weights (zero for taps outside the map).
// ---------------------------------------------------------------------------
template <int C>
struct Sample {
    float t[4][C];       // taps 00, 10, 01, 11 (zero outside the map)
    float fx, fy;        // fractional position
    float dXdd, dYdd;    // d(position) / d(depth)
    int off[4];          // element offsets of the taps
    bool in[4];          // tap inside the map
    bool ok;             // the point is in front of view m
};

template <int C>
__device__ inline void sample_view(const BwdParams &p, int m, double uc, double vc, double d,
                                   Sample<C> &S) {
    const double *A = p.camd[m];
    const double invd = 1.0 / d;
    const double pz = fma(A[6], uc, fma(A[7], vc, fma(A[11], invd, A[8])));
    const double qx = fma(A[0], uc, fma(A[1], vc, fma(A[9], invd, A[2])));
    const double qy = fma(A[3], uc, fma(A[4], vc, fma(A[10], invd, A[5])));
    const double rz = 1.0 / pz;
    const double X = qx * rz - 0.5, Y = qy * rz - 0.5;
    S.ok = (pz > 1e-6) && (fabs(X) < 1e7) && (fabs(Y) < 1e7);
    // d p / d d = -b / d^2;  d(q / pz) / d d = (dq pz - q dpz) / pz^2
    const double k = invd * invd * rz * rz;
    S.dXdd = (float)((qx * A[11] - A[9] * pz) * k);
    S.dYdd = (float)((qy * A[11] - A[10] * pz) * k);
    const double xf = floor(X), yf = floor(Y);
    S.fx = (float)(X - xf);
    S.fy = (float)(Y - yf);
    const int fw = p.fW[m], fh = p.fH[m];
    const int ix = S.ok ? (int)xf : -4, iy = S.ok ? (int)yf : -4;
    const bool vx0 = (unsigned)ix < (unsigned)fw, vx1 = (unsigned)(ix + 1) < (unsigned)fw;
    const bool vy0 = (unsigned)iy < (unsigned)fh, vy1 = (unsigned)(iy + 1) < (unsigned)fh;
    S.in[0] = vx0 && vy0;
    S.in[1] = vx1 && vy0;
    S.in[2] = vx0 && vy1;
    S.in[3] = vx1 && vy1;
    const int cx0 = min(max(ix, 0), fw - 1), cx1 = min(max(ix + 1, 0), fw - 1);
    const int cy0 = min(max(iy, 0), fh - 1), cy1 = min(max(iy + 1, 0), fh - 1);
    S.off[0] = (cy0 * fw + cx0) * C;
    S.off[1] = (cy0 * fw + cx1) * C;
    S.off[2] = (cy1 * fw + cx0) * C;
    S.off[3] = (cy1 * fw + cx1) * C;
    const float *fm = p.feat[m];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float4 *src = reinterpret_cast<const float4 *>(fm + S.off[t]);
        const float keep = S.in[t] ? 1.0f : 0.0f;
#pragma unroll
        for (int c4 = 0; c4 < C / 4; ++c4) {
            const float4 v = src[c4];
            S.t[t][4 * c4 + 0] = v.x * keep;
            S.t[t][4 * c4 + 1] = v.y * keep;
            S.t[t][4 * c4 + 2] = v.z * keep;
            S.t[t][4 * c4 + 3] = v.w * keep;
        }
    }
}

template <int C>
__device__ inline void blend(const Sample<C> &S, float *s) {
    const float w00 = (1.f - S.fx) * (1.f - S.fy), w10 = S.fx * (1.f - S.fy);
    const float w01 = (1.f - S.fx) * S.fy, w11 = S.fx * S.fy;
#pragma unroll
    for (int c = 0; c < C; ++c)
        s[c] = fmaf(w00, S.t[0][c], fmaf(w10, S.t[1][c], fmaf(w01, S.t[2][c], w11 * S.t[3][c])));
}

// Sum over the wave's 64 layer-pixels of a_p (x) b_p, added to a 16 x 16
// accumulator (rows: index of a, columns: index of b; vectors zero-padded to
// 16).  The wave's vectors go through its own LDS slice: lane l feeds the
// matrix cores a_{4s + l/16}[l % 16] and b_{4s + l/16}[l % 16] at step s.
template <int NA, int NB>
__device__ inline void outer_accumulate(float *sa, float *sb, int lane, const float *a,
                                        const float *b, bool live, f32x4 &acc) {
    __syncthreads();   // the previous pair's reads are done
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
        float va[4], vb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = 4 * c4 + i;
            va[i] = (live && c < NA) ? a[c < NA ? c : 0] : 0.0f;
            vb[i] = (live && c < NB) ? b[c < NB ? c : 0] : 0.0f;
        }
        reinterpret_cast<float4 *>(sa + lane * 16)[c4] = make_float4(va[0], va[1], va[2], va[3]);
        reinterpret_cast<float4 *>(sb + lane * 16)[c4] = make_float4(vb[0], vb[1], vb[2], vb[3]);
    }
    __syncthreads();
    const int r = lane & 15, k = lane >> 4;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int idx = (4 * s + k) * 16 + r;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[idx], sb[idx], acc, 0, 0, 0);
    }
}

// Per-use view of the weights in LDS.  Every use site takes a fresh opaque
// base address, so the compiler neither keeps a whole matrix live across
// uses nor hoists it out of the loops; rows are read contiguously, the same
// address in every lane (a broadcast).
__device__ inline lds_f32 *weights_at(lds_f32 *base, int offset) {
    lds_f32 *w = base + offset;
    asm volatile("" : "+v"(w));
    return w;
}

// y[j] = sum_c x[c] W[c][j]   (W row-major R x K)
template <int R, int K>
__device__ inline void vec_mat(const float *x, lds_f32 *W, float *y) {
#pragma unroll
    for (int j = 0; j < K; ++j) y[j] = 0.f;
#pragma unroll 2
    for (int c = 0; c < R; ++c) {
        lds_f32 *row = W + c * K;
#pragma unroll
        for (int j = 0; j < K; ++j) y[j] = fmaf(x[c], row[j], y[j]);
        __builtin_amdgcn_sched_barrier(0);      // one row in flight at a time
    }
}

// y[c] = sum_j W[c][j] x[j]   (W row-major R x K)
template <int R, int K>
__device__ inline void mat_vec(lds_f32 *W, const float *x, float *y) {
#pragma unroll 2
    for (int c = 0; c < R; ++c) {
        lds_f32 *row = W + c * K;
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < K; ++j) acc = fmaf(row[j], x[j], acc);
        y[c] = acc;
        __builtin_amdgcn_sched_barrier(0);      // one row in flight at a time
    }
}

// Loads a layer-pixel's feature vector and returns its RMS-normalised form
// and the RMS r (unit gain, eps 1e-6 inside the root).
template <int C>
__device__ inline float load_normalised(const float *F, int64_t e, float *xn) {
    const float4 *f4 = reinterpret_cast<const float4 *>(F + e * C);
#pragma unroll
    for (int c4 = 0; c4 < C / 4; ++c4) {
        const float4 v = f4[c4];
        xn[4 * c4 + 0] = v.x;
        xn[4 * c4 + 1] = v.y;
        xn[4 * c4 + 2] = v.z;
        xn[4 * c4 + 3] = v.w;
    }
    float ss = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) ss = fmaf(xn[c], xn[c], ss);
    const float r = sqrtf(ss * (1.0f / (float)C) + 1e-6f);
    const float ir = 1.0f / r;
#pragma unroll
    for (int c = 0; c < C; ++c) xn[c] *= ir;
    return r;
}

template <int C>
__device__ inline void load_vec(const float *src, int64_t e, float *v) {
    const float4 *s4 = reinterpret_cast<const float4 *>(src + e * C);
#pragma unroll
    for (int c4 = 0; c4 < C / 4; ++c4) {
        const float4 t = s4[c4];
        v[4 * c4 + 0] = t.x;
        v[4 * c4 + 1] = t.y;
        v[4 * c4 + 2] = t.z;
        v[4 * c4 + 3] = t.w;
    }
}

template <int C>
__device__ inline void store_vec(float *dst, int64_t e, const float *v) {
    float4 *d4 = reinterpret_cast<float4 *>(dst + e * C);
#pragma unroll
    for (int c4 = 0; c4 < C / 4; ++c4)
        d4[c4] = make_float4(v[4 * c4 + 0], v[4 * c4 + 1], v[4 * c4 + 2], v[4 * c4 + 3]);
}

// One thread per layer-pixel.  Live ranges are kept short: the input
// feature is re-read where it is needed again, and dF' is parked in the dF
// output across the second pass over the views.
template <int C>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_uf_backward(const BwdParams p) {
    static_assert(C == 8 || C == 16, "the backward kernel holds C <= 16 channels per thread");
    __shared__ float s_a[kWaves][64 * 16];
    __shared__ float s_b[kWaves][64 * 16];
    __shared__ int s_o[kWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *sa = s_a[wave], *sb = s_b[wave];
    int *so = s_o[wave];

    // The weights live in LDS for the whole kernel; every lane reads the same
    // address (a broadcast).
    constexpr int NW = 4 * C * C + 5 * C;
    __shared__ __attribute__((aligned(16))) float s_w[NW];
    for (int i = threadIdx.x; i < NW; i += kBlock) {
        float v;
        if (i < C * C) v = p.Wq[i];
        else if (i < 2 * C * C) v = p.Wk[i - C * C];
        else if (i < 3 * C * C) v = p.Wv[i - 2 * C * C];
        else if (i < 4 * C * C) v = p.Wo[i - 3 * C * C];
        else if (i < 4 * C * C + C) v = p.w_sigma[i - 4 * C * C];
        else if (i < 4 * C * C + 2 * C) v = p.w_depth[i - 4 * C * C - C];
        else v = p.W_color[i - 4 * C * C - 2 * C];
        s_w[i] = v;
    }
    __syncthreads();
    lds_f32 *wb = (lds_f32 *)(s_w);
    constexpr int OQ = 0, OK = C * C, OV = 2 * C * C, OO = 3 * C * C, OH = 4 * C * C;

    f32x4 gQ = {0.f, 0.f, 0.f, 0.f}, gK = gQ, gV = gQ, gO = gQ, gH = gQ;
    const int32_t npix = p.H * p.W;
    const int32_t N = (int32_t)p.N;
    const float half_l = 0.5f / (float)p.L;
    const float band = p.inv_near - p.inv_far;
    const float kap = half_l * band;
    const float scale = p.scale;

    for (int32_t base = blockIdx.x * kBlock; base < N; base += gridDim.x * kBlock) {
        const bool live = base + (int32_t)threadIdx.x < N;
        const int32_t e = live ? base + (int32_t)threadIdx.x : N - 1;
        const int32_t li = e / npix;
        const int32_t rem = e - li * npix;
        const int32_t y = rem / p.W, x = rem - y * p.W;
        const double uc = x + 0.5, vc = y + 0.5;
        const float d = p.depth_in[e];

        // ---- query folded with the key: q~ = scale W_k (N(F) W_q)
        float qt[C];
        {
            float xn[C], q[C];
            load_normalised<C>(p.F_in, e, xn);
            vec_mat<C, C>(xn, weights_at(wb, OQ), q);
            mat_vec<C, C>(weights_at(wb, OK), q, qt);
#pragma unroll
            for (int c = 0; c < C; ++c) qt[c] *= scale;
        }

        // ---- pass 1 over the views: online softmax of a_m = q~ . s_m and
        //      ob = sum_m p_m s_m.  The weights are exp(a_m - mx) for a
        //      reference mx moved only when a logit passes it by more than 8
        //      (always at the first view), as in the forward kernel; pass 2
        //      uses the same reference.
        float mx = -1e30f, z = 0.f, ob[C];
#pragma unroll
        for (int c = 0; c < C; ++c) ob[c] = 0.f;
#pragma unroll 1
        for (int m = 0; m < p.V; ++m) {
            Sample<C> S;
            sample_view<C>(p, m, uc, vc, (double)d, S);
            float s[C];
            blend<C>(S, s);
            float a = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c) a = fmaf(qt[c], s[c], a);
            float diff = a - mx;
            if (diff > 8.0f) {
                const float r = __expf(-diff);
                z *= r;
#pragma unroll
                for (int c = 0; c < C; ++c) ob[c] *= r;
                mx = a;
                diff = 0.0f;
            }
            const float pw = __expf(diff);
            z += pw;
#pragma unroll
            for (int c = 0; c < C; ++c) ob[c] = fmaf(pw, s[c], ob[c]);
        }
        const float iz = 1.0f / z;
#pragma unroll
        for (int c = 0; c < C; ++c) ob[c] *= iz;

        // ---- o = ob W_v; F' = F + o W_o; decode and its adjoint; back
        //      through W_o and W_v to dob = W_v W_o^T dF'
        float dob[C], dd_in = 0.f, da_in = 0.f;
        {
            float o[C], fp[C];
            vec_mat<C, C>(ob, weights_at(wb, OV), o);
            vec_mat<C, C>(o, weights_at(wb, OO), fp);
            {
                float f[C];
                load_vec<C>(p.F_in, e, f);
#pragma unroll
                for (int c = 0; c < C; ++c) fp[c] += f[c];
            }
            float xs = 0.f, xd = 0.f, xc[3] = {0.f, 0.f, 0.f};
            {
                lds_f32 *wh = weights_at(wb, OH);            // w_sigma, w_depth, W_color
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    xs = fmaf(fp[c], wh[c], xs);
                    xd = fmaf(fp[c], wh[C + c], xd);
                    xc[0] = fmaf(fp[c], wh[2 * C + c * 3 + 0], xc[0]);
                    xc[1] = fmaf(fp[c], wh[2 * C + c * 3 + 1], xc[1]);
                    xc[2] = fmaf(fp[c], wh[2 * C + c * 3 + 2], xc[2]);
                }
            }
            float dco[3] = {0.f, 0.f, 0.f}, dal = 0.f, ddn = 0.f;
            if (p.comp) {
                const float4 cg = reinterpret_cast<const float4 *>(p.comp)[e];
                dco[0] = cg.x;
                dco[1] = cg.y;
                dco[2] = cg.z;
                dal = cg.w;
            }
            if (p.d_alpha_out) dal += p.d_alpha_out[e];
            if (p.d_depth_out) ddn = p.d_depth_out[e];
            // sigma'(z) = sigma(z) sigma(-z): the second factor is not taken as
            // 1 - sigma(z), which loses its digits when sigma(z) is near one
            float h[5];                                   // d x_sigma, d x_depth, d x_color
#pragma unroll
            for (int j = 0; j < 3; ++j) h[2 + j] = dco[j] * sigm(xc[j]) * sigm(-xc[j]);
            const float th = tanhf(xd);
            if (p.mode == 0) {
                const float a_in = p.alpha_in[e];
                const float ac = fminf(fmaxf(a_in, 1e-6f), 1.0f - 1e-6f);
                const float z = logf(ac / (1.0f - ac)) + xs;
                h[0] = dal * sigm(z) * sigm(-z);
                if (a_in > 1e-6f && a_in < 1.0f - 1e-6f) da_in = h[0] / (a_in * (1.0f - a_in));
                const float disp = 1.0f / d + kap * th;
                h[1] = 0.f;
                if (disp > p.inv_far && disp < p.inv_near) {
                    const float dn = 1.0f / disp;
                    const float ddisp = -ddn * dn * dn;
                    dd_in = -ddisp / (d * d);
                    h[1] = ddisp * kap * (1.0f - th * th);
                }
            } else {
                h[0] = dal * sigm(xs) * sigm(-xs);
                const float delta = ((float)(p.L - li) - 0.5f) / (float)p.L;
                const float dn = 1.0f / fmaf(delta + half_l * th, band, p.inv_far);
                h[1] = -ddn * dn * dn * kap * (1.0f - th * th);
            }
            outer_accumulate<C, 5>(sa, sb, lane, fp, h, live, gH);
            float dfp[C];
            {
                lds_f32 *wh = weights_at(wb, OH);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    float g = fmaf(wh[c], h[0], wh[C + c] * h[1]);
                    g = fmaf(wh[2 * C + c * 3 + 0], h[2], g);
                    g = fmaf(wh[2 * C + c * 3 + 1], h[3], g);
                    g = fmaf(wh[2 * C + c * 3 + 2], h[4], g);
                    dfp[c] = g;
                }
            }
            if (p.dF_out) {
                float u[C];
                load_vec<C>(p.dF_out, e, u);
#pragma unroll
                for (int c = 0; c < C; ++c) dfp[c] += u[c];
            }
            outer_accumulate<C, C>(sa, sb, lane, o, dfp, live, gO);
            float dov[C];
            mat_vec<C, C>(weights_at(wb, OO), dfp, dov);
            if (live) store_vec<C>(p.dF, e, dfp);        // the residual path; RMSNorm term added below
            outer_accumulate<C, C>(sa, sb, lane, ob, dov, live, gV);
            mat_vec<C, C>(weights_at(wb, OV), dov, dob);
        }
        float delta = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) delta = fmaf(ob[c], dob[c], delta);

        // ---- pass 2 over the views: softmax adjoint, dI scatter, depth
        //      through the sample position.  ds_m = p_m dob + da_m q~
        float sh[C];                                      // sum_m da_m s_m
#pragma unroll
        for (int c = 0; c < C; ++c) sh[c] = 0.f;
#pragma unroll 1
        for (int m = 0; m < p.V; ++m) {
            Sample<C> S;
            sample_view<C>(p, m, uc, vc, (double)d, S);
            float s[C];
            blend<C>(S, s);
            float a = 0.f, sd = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                a = fmaf(qt[c], s[c], a);
                sd = fmaf(s[c], dob[c], sd);
            }
            const float pm = __expf(a - mx) * iz;
            const float da = pm * (sd - delta);
            const float w[4] = {(1.f - S.fx) * (1.f - S.fy), S.fx * (1.f - S.fy),
                                (1.f - S.fx) * S.fy, S.fx * S.fy};
            // ds goes straight to the wave's LDS slice (row of this lane),
            // the tap offsets and weights beside it
            float gX = 0.f, gY = 0.f;
#pragma unroll
            for (int c4 = 0; c4 < C / 4; ++c4) {
                float d4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = 4 * c4 + i;
                    sh[c] = fmaf(da, s[c], sh[c]);
                    const float ds = fmaf(pm, dob[c], da * qt[c]);
                    d4[i] = ds;
                    gX = fmaf(ds, (1.f - S.fy) * (S.t[1][c] - S.t[0][c]) + S.fy * (S.t[3][c] - S.t[2][c]), gX);
                    gY = fmaf(ds, (1.f - S.fx) * (S.t[2][c] - S.t[0][c]) + S.fx * (S.t[3][c] - S.t[1][c]), gY);
                }
                reinterpret_cast<float4 *>(sa + lane * C)[c4] = make_float4(d4[0], d4[1], d4[2], d4[3]);
            }
            if (S.ok) dd_in = fmaf(gX, S.dXdd, fmaf(gY, S.dYdd, dd_in));
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                so[4 * lane + t] = (live && S.ok && S.in[t]) ? S.off[t] : -1;
                sb[4 * lane + t] = w[t];
            }
            __syncthreads();
            // dI scatter, channel-coalesced: one atomic instruction covers
            // 64 / C whole (pixel, tap) rows of C consecutive floats instead
            // of 64 scattered addresses
            {
                float *dI = p.dfeat[m];
                constexpr int RPI = 64 / C;               // rows per instruction
                const int c_l = lane % C, r_l = lane / C;
#pragma unroll 2
                for (int j = 0; j < C; ++j) {
                    const int row = r_l + RPI * j;
                    const float dsr = sa[row * C + c_l];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int o = so[4 * row + t];
                        if (o >= 0) unsafeAtomicAdd(dI + o + c_l, sb[4 * row + t] * dsr);
                    }
                }
            }
            __syncthreads();
        }

        // ---- dq = scale W_k^T sh; key and query weight gradients; RMSNorm
        //      adjoint dF += (dxn - xn (xn . dxn) / C) / r
        {
            float xn[C], q[C], dq[C];
            const float r = load_normalised<C>(p.F_in, e, xn);
            vec_mat<C, C>(xn, weights_at(wb, OQ), q);
#pragma unroll
            for (int c = 0; c < C; ++c) sh[c] *= scale;
            vec_mat<C, C>(sh, weights_at(wb, OK), dq);
            outer_accumulate<C, C>(sa, sb, lane, sh, q, live, gK);
            outer_accumulate<C, C>(sa, sb, lane, xn, dq, live, gQ);
            float dxn[C], xdx = 0.f;
            mat_vec<C, C>(weights_at(wb, OQ), dq, dxn);
#pragma unroll
            for (int c = 0; c < C; ++c) xdx = fmaf(xn[c], dxn[c], xdx);
            if (live) {
                const float ir = 1.0f / r, k = xdx * (1.0f / (float)C);
                float g[C];
                load_vec<C>(p.dF, e, g);
#pragma unroll
                for (int c = 0; c < C; ++c) g[c] += (dxn[c] - xn[c] * k) * ir;
                store_vec<C>(p.dF, e, g);
                p.d_depth[e] = dd_in;
                p.d_alpha[e] = da_in;
            }
        }
    }

    // ---- workgroup partial of every weight-gradient tile.  The D layout of
    //      a 16 x 16 tile: lane l holds column l % 16, rows 4 (l / 16) + i.
    __syncthreads();
    float *red = &s_a[0][0];                            // kWaves x 256 floats used
    const f32x4 *acc[kGradTiles] = {&gQ, &gK, &gV, &gO, &gH};
    float *part = p.partials + (size_t)blockIdx.x * kGradTiles * kGradTileElems;
#pragma unroll
    for (int t = 0; t < kGradTiles; ++t) {
        const int col = lane & 15, row0 = 4 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wave * 256 + (row0 + i) * 16 + col] = (*acc[t])[i];
        __syncthreads();
        {
            const int idx = threadIdx.x;               // 256 entries, one per thread
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += red[w * 256 + idx];
            part[t * kGradTileElems + idx] = s;
        }
        __syncthreads();
    }
}

// Deterministic sum of the workgroup partials into the weight gradients.
// A block takes 16 consecutive entries of one tile; its 16 lanes per entry
// sum interleaved partials, then one lane combines the 16 sums in order.
__global__ void __launch_bounds__(kBlock) k_reduce_wgrad(const BwdParams p) {
    __shared__ double red[16][17];
    const int e16 = threadIdx.x & 15, part = threadIdx.x >> 4;
    const int gid = blockIdx.x * 16 + e16;                 // entry in [0, 5 * 256)
    const int t = gid / kGradTileElems, rc = gid % kGradTileElems;
    double s = 0.0;
    for (int b = part; b < p.blocks; b += 16)
        s += (double)p.partials[((size_t)b * kGradTiles + t) * kGradTileElems + rc];
    red[e16][part] = s;
    __syncthreads();
    if (part != 0) return;
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) tot += red[e16][k];
    const int row = rc / 16, col = rc % 16;
    const int C = p.C;
    float *dst = nullptr;
    switch (t) {
        case 0: if (row < C && col < C) dst = p.dWq + row * C + col; break;
        case 1: if (row < C && col < C) dst = p.dWk + row * C + col; break;
        case 2: if (row < C && col < C) dst = p.dWv + row * C + col; break;
        case 3: if (row < C && col < C) dst = p.dWo + row * C + col; break;
        default:
            if (row < C) {
                if (col == 0) dst = p.dw_sigma + row;
                else if (col == 1) dst = p.dw_depth + row;
                else if (col < 5) dst = p.dW_color + row * 3 + (col - 2);
            }
            break;
    }
    if (dst != nullptr) *dst = (float)tot;
}

}  // namespace

hipError_t launch_composite_backward(const CompBwdParams &p, hipStream_t s) {
    const int64_t blocks = (p.npix + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_composite_backward, dim3((unsigned)blocks), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_update_fuse_backward(const BwdParams &p, hipStream_t s) {
    if (p.C != 8 && p.C != 16) return hipErrorInvalidValue;
    int64_t zero_blocks = 1;
    for (int m = 0; m < p.V; ++m) {
        const int64_t n4 = (int64_t)p.fH[m] * p.fW[m] * p.C / 4;
        zero_blocks = std::max<int64_t>(zero_blocks, std::min<int64_t>(1024, (n4 + kBlock - 1) / kBlock));
    }
    hipLaunchKernelGGL(k_zero_maps, dim3((unsigned)zero_blocks, (unsigned)p.V), dim3(kBlock), 0, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p.comp != nullptr) {
        const int64_t npix = (int64_t)p.H * p.W;
        hipLaunchKernelGGL(k_composite_adjoint, dim3((unsigned)((npix + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, p);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p.C == 8)
        hipLaunchKernelGGL((k_uf_backward<8>), dim3((unsigned)p.blocks), dim3(kBlock), 0, s, p);
    else
        hipLaunchKernelGGL((k_uf_backward<16>), dim3((unsigned)p.blocks), dim3(kBlock), 0, s, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_wgrad, dim3(kGradTiles * kGradTileElems / 16), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
