// k_update_fuse.hip -- fused Update & Fuse step (+ optional composite) for
// gfx950 (CDNA4).  One kernel per LDM level: reproject -> bilinear gather ->
// RMSNorm -> Q/K/V projections on MFMA -> softmax over views -> output
// projection + residual -> decode -> (front-to-back composite).
//
// The operation is the paper's Update & Fuse step (Sec. 3.2.2) with the
// fusion-block attention of Sec. 3.3 and the decode of Sec. 3.2.2-3.2.3; the
// composite is the over operator of Sec. 3.1.
//
// Work decomposition (wave64):
//   * a workgroup is 4 waves; it covers 64 G consecutive pixels of one LDM row
//     and a chunk of layers; each wave owns 16 G pixels and walks the layers
//     of its chunk front to back (so the composite accumulates in registers);
//   * projections are computed transposed, out^T = W^T x^T, on
//     v_mfma_f32_16x16x32_bf16 (bfloat16) or v_mfma_f32_16x16x4_f32 (float32):
//     the weights are the A operand and the per-pixel vectors the B operand,
//     so pixels run along the output columns.  Lane l = 16 g + n holds, in
//     the operand layout, K-slots 8g..8g+7 of pixel column n, and in the
//     accumulator layout output rows 4g..4g+3 of column n.  A pixel's logit
//     is then a sum inside the lane and across at most four lanes (one or two
//     permlane swaps), and every lane keeps one or two softmax states;
//   * the bilinear gather of view m writes straight into the B operand: lane
//     (n, g) reprojects its pixel and loads 8 channels per tap (16 B in
//     bfloat16, 32 B in float32);
//   * for C < 32 a 32-wide K chunk holds G = 32 / C independent 16-pixel
//     sub-tiles side by side and every weight is block-diagonal, so a wave
//     covers 16 G pixels and all its lanes sample the same view at a time
//     (camera parameters and the feature base stay scalar);
//   * for C = 8 the four bilinear taps run along K instead (lane (n, g) loads
//     tap g), so the two taps of a row come from adjacent lanes of one load,
//     and the MFMA forms the weighted tap sum with the weight stacked 4x;
//   * taps are clamped into the map with zero weight when outside, so the
//     gather has no divergent branches; the loads of view m + 1 are issued
//     before view m is projected;
//   * softmax over views is an online update whose reference moves only when
//     a logit exceeds it by more than 8 (one exp per state and view);
//   * weights arrive as float32 masters; each workgroup converts them once
//     into operand fragments in LDS; the K/V fragments then stay in registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "uf_params.h"

// Multiply-adds are fused only within one expression (never across
// statements), so every variant of the kernel body -- one level, one level
// with blend logits, a batch -- rounds alike and gives bit-identical results.
#pragma clang fp contract(on)

namespace qk {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int C>
struct Shape {
    static constexpr int G = (C >= 32) ? 1 : 32 / C;    // 16-pixel sub-tiles packed along K
    static constexpr int KC = (C >= 32) ? C / 32 : 1;   // 32-wide K chunks of an operand
    static constexpr int NT = (G * C) / 16;             // 16-row output tiles of Q/K/V/O
    static constexpr int ND = (G == 1) ? 1 : G / 2;     // output tiles of the decode
    static constexpr int PIX = 16 * G;                  // pixels per wave
    static constexpr int P = C + 4;                     // LDS floats per pixel (padded)
    // C = 8: the four bilinear taps run along the MFMA K dimension
    static constexpr bool TAPK = (C == 8);
};

// Weight-fragment slots in LDS: Q, [K, V,] O, decode.  The K/V slots exist
// only when the view loop projects per-sample keys and values on MFMA.
template <int C, bool KV, int HQ = 1>
struct Frags {
    // HQ query blocks (the heads of the one-to-many form, 1 otherwise); the
    // output projection reads their HQ C-channel concatenation
    static constexpr int KC = Shape<C>::KC, NT = Shape<C>::NT, ND = Shape<C>::ND;
    static constexpr int KCO = HQ * KC;
    static constexpr int OFF_Q = 0;
    static constexpr int OFF_K = HQ * KC * NT;
    static constexpr int OFF_V = OFF_K + (KV ? KC * NT : 0);
    static constexpr int OFF_O = OFF_V + (KV ? KC * NT : 0);
    static constexpr int OFF_D = OFF_O + KCO * NT;
    static constexpr int N = OFF_D + KC * ND;
};

// ---------------------------------------------------------------------------
// Arithmetic form: bfloat16 operands on v_mfma_f32_16x16x32_bf16, or float32
// operands on eight v_mfma_f32_16x16x4_f32 (same lane layout: step i feeds
// the K-slot 8g + i of every lane).
// ---------------------------------------------------------------------------
template <bool BF16>
struct Op;

template <>
struct Op<true> {
    typedef uint16_t T;                          // storage element (bf16 bits)
    struct __attribute__((aligned(16))) A {
        bf16x8_t v;
    };
    __device__ static inline A make(const float *f) {
        A a;
#pragma unroll
        for (int i = 0; i < 8; ++i) a.v[i] = (__bf16)f[i];
        return a;
    }
    __device__ static inline f32x4 mma(const A &a, const A &b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
    }
    __device__ static inline void load8(const T *p, float *f) {
        const uint4 u = *reinterpret_cast<const uint4 *>(p);
        f[0] = __uint_as_float(u.x << 16);
        f[1] = __uint_as_float(u.x & 0xffff0000u);
        f[2] = __uint_as_float(u.y << 16);
        f[3] = __uint_as_float(u.y & 0xffff0000u);
        f[4] = __uint_as_float(u.z << 16);
        f[5] = __uint_as_float(u.z & 0xffff0000u);
        f[6] = __uint_as_float(u.w << 16);
        f[7] = __uint_as_float(u.w & 0xffff0000u);
    }
    __device__ static inline void store8(T *p, const float *f) {
        A a = make(f);
        *reinterpret_cast<uint4 *>(p) = __builtin_bit_cast(uint4, a.v);
    }
};

template <>
struct Op<false> {
    typedef float T;
    struct __attribute__((aligned(16))) A {
        float v[8];
    };
    __device__ static inline A make(const float *f) {
        A a;
#pragma unroll
        for (int i = 0; i < 8; ++i) a.v[i] = f[i];
        return a;
    }
    __device__ static inline f32x4 mma(const A &a, const A &b, f32x4 c) {
#pragma unroll
        for (int i = 0; i < 8; ++i) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[i], b.v[i], c, 0, 0, 0);
        return c;
    }
    __device__ static inline void load8(const T *p, float *f) {
        const float4 a = reinterpret_cast<const float4 *>(p)[0];
        const float4 b = reinterpret_cast<const float4 *>(p)[1];
        f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
        f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
    }
    __device__ static inline void store8(T *p, const float *f) {
        reinterpret_cast<float4 *>(p)[0] = make_float4(f[0], f[1], f[2], f[3]);
        reinterpret_cast<float4 *>(p)[1] = make_float4(f[4], f[5], f[6], f[7]);
    }
};

// FP8 projection operands (OCP e4m3, the gfx950 format): 8 values per lane
// in the K-slot layout of v_mfma_f32_16x16x32_fp8_fp8 (the same slots as the
// bfloat16 16x16x32 product).  Values are multiplied by an inverse
// per-tensor scale before rounding (round to nearest even); the caller
// applies the scales to the float32 result.
struct OpF8 {
    struct __attribute__((aligned(8))) A {
        long v;
    };
    __device__ static inline A make(const float *f, float inv) {
        int lo = 0, hi = 0;
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(f[0] * inv, f[1] * inv, lo, false);
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(f[2] * inv, f[3] * inv, lo, true);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(f[4] * inv, f[5] * inv, hi, false);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(f[6] * inv, f[7] * inv, hi, true);
        A a;
        a.v = (long)(((unsigned long)(unsigned)hi << 32) | (unsigned)lo);
        return a;
    }
    __device__ static inline f32x4 mma(const A &a, const A &b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a.v, b.v, c, 0, 0, 0);
    }
};

// Projection operands: bfloat16 / float32 (the storage form), or e4m3.
template <bool BF16, bool F8>
struct Mm {
    using A = typename Op<BF16>::A;
    __device__ static inline A make(const float *f, float) { return Op<BF16>::make(f); }
    __device__ static inline f32x4 mma(const A &a, const A &b, f32x4 c) { return Op<BF16>::mma(a, b, c); }
};
template <>
struct Mm<true, true> {
    using A = OpF8::A;
    __device__ static inline A make(const float *f, float inv) { return OpF8::make(f, inv); }
    __device__ static inline f32x4 mma(const A &a, const A &b, f32x4 c) { return OpF8::mma(a, b, c); }
};

// Reprojection arithmetic: float in the bfloat16 form; double in the float32
// form, whose budget (1e-4 on RGB) the float representation of absolute
// pixel coordinates (half an ulp = 6e-5 px at 1920) would use up.
template <bool BF16>
struct CoordT {
    typedef double type;
};
template <>
struct CoordT<true> {
    typedef float type;
};

template <bool BF16>
__device__ inline typename CoordT<BF16>::type cam_entry(const UFParams &p, int m, int k) {
    if constexpr (BF16) return p.cam[m][k];
    else return p.camd[m][k];
}

template <bool BF16>
__device__ inline const typename CoordT<BF16>::type *cam_row(const UFParams &p, int m) {
    if constexpr (BF16) return p.cam[m];
    else return p.camd[m];
}

__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
// double: the hardware's reciprocal estimate refined by one Newton step (the
// relative error squares, to about an ulp), instead of the IEEE division
__device__ inline double recip(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}


__device__ inline void lds_read8(const float *src, float *f) {
    const float4 a = *reinterpret_cast<const float4 *>(src);
    const float4 b = *reinterpret_cast<const float4 *>(src + 4);
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
    f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
}

// Blended sample from the load layout (pixel pl_ld, channels ch_ld + 32 kc)
// to the operand layout (pixel pl_b, channels ch0 + 32 kc) through the
// wave's LDS slice (rows of P floats per pixel).  One wave writes and reads
// its own slice, in order, so no barrier is needed.
template <int C>
__device__ inline void stage_sample(float *slice, int pl_ld, int ch_ld, int pl_b, int ch0,
                                    float (&sv)[Shape<C>::KC][8]) {
    constexpr int KC = Shape<C>::KC, P = Shape<C>::P;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        float *dst = &slice[pl_ld * P + ch_ld + 32 * kc];
        *reinterpret_cast<float4 *>(dst) = make_float4(sv[kc][0], sv[kc][1], sv[kc][2], sv[kc][3]);
        *reinterpret_cast<float4 *>(dst + 4) = make_float4(sv[kc][4], sv[kc][5], sv[kc][6], sv[kc][7]);
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const float *src = &slice[pl_b * P + ch0 + 32 * kc];
        const float4 a = *reinterpret_cast<const float4 *>(src);
        const float4 b = *reinterpret_cast<const float4 *>(src + 4);
        sv[kc][0] = a.x; sv[kc][1] = a.y; sv[kc][2] = a.z; sv[kc][3] = a.w;
        sv[kc][4] = b.x; sv[kc][5] = b.y; sv[kc][6] = b.z; sv[kc][7] = b.w;
    }
}

// Raw storage of one 8-channel tap: 16 B of bfloat16 or 32 B of float.
template <bool BF16>
struct RawTap {
    uint4 v[BF16 ? 1 : 2];
};

// The four taps of one bilinear sample (this lane's channels), as loaded, and
// their weights.  Loading and blending are split so the loads of the next
// view can be in flight while the current view is projected.
template <int C, bool BF16>
struct Taps {
    RawTap<BF16> t[Shape<C>::KC][4];
    float w[4];
};

// Feature map m as a buffer resource: a load whose byte offset falls
// outside [0, bytes) returns zeros (the hardware's range check), so tap
// addresses need no clamping.  A tap outside the map is sent to kTapOOB, far
// past the end (the host keeps every map under 1 GiB), never to a negative
// offset: the compiler may fold a constant part of an offset into the
// instruction's immediate field or merge neighbouring loads, and a negative
// register offset then takes a valid tap out of range with it.
constexpr int kTapOOB = 0x40000000;

template <int C, bool BF16>
__device__ inline __amdgpu_buffer_rsrc_t feat_rsrc(const UFParams &p, int m) {
    const int bytes = p.fH[m] * p.fW[m] * C * (int)sizeof(typename Op<BF16>::T);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p.feat[m]), 0, bytes, 0x00020000);
}

template <bool BF16>
__device__ inline void buf_load(__amdgpu_buffer_rsrc_t r, int byte_off, RawTap<BF16> &t) {
    const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    t.v[0] = make_uint4(a[0], a[1], a[2], a[3]);
    if constexpr (!BF16) {
        const auto b = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off + 16, 0, 0);
        t.v[1] = make_uint4(b[0], b[1], b[2], b[3]);
    }
}

template <bool BF16>
__device__ inline void raw_unpack(const RawTap<BF16> &r, float *f) {
    if constexpr (BF16) {
        const uint4 u = r.v[0];
        f[0] = __uint_as_float(u.x << 16);
        f[1] = __uint_as_float(u.x & 0xffff0000u);
        f[2] = __uint_as_float(u.y << 16);
        f[3] = __uint_as_float(u.y & 0xffff0000u);
        f[4] = __uint_as_float(u.z << 16);
        f[5] = __uint_as_float(u.z & 0xffff0000u);
        f[6] = __uint_as_float(u.w << 16);
        f[7] = __uint_as_float(u.w & 0xffff0000u);
    } else {
        f[0] = __uint_as_float(r.v[0].x); f[1] = __uint_as_float(r.v[0].y);
        f[2] = __uint_as_float(r.v[0].z); f[3] = __uint_as_float(r.v[0].w);
        f[4] = __uint_as_float(r.v[1].x); f[5] = __uint_as_float(r.v[1].y);
        f[6] = __uint_as_float(r.v[1].z); f[7] = __uint_as_float(r.v[1].w);
    }
}

// Back-projection of one layer-pixel into one view (the first half of the
// bilinear sample): p = A (u, v, 1) + b / d from the view's camera entries
// cam[0..11]; a point with p_z <= 1e-6 (behind the view) samples zero.
// Gives the four taps' byte offsets in the view's map, without the channel
// part (half-pixel centres; a tap outside the map gets weight 0 and the
// out-of-range offset kTapOOB, so its load reads zeros), and their weights.
struct TapProj {
    int o[4];
    float w[4];
};

template <int C, bool BF16>
__device__ inline void project_view(const typename CoordT<BF16>::type *cam, int fw, int fh,
                                    typename CoordT<BF16>::type uc, typename CoordT<BF16>::type vc,
                                    typename CoordT<BF16>::type invdc, bool a_ok, TapProj &tp) {
    using Coord = typename CoordT<BF16>::type;
    constexpr int E = (int)sizeof(typename Op<BF16>::T);
    const Coord pz = fma(cam[6], uc, fma(cam[7], vc, fma(cam[11], invdc, cam[8])));
    const Coord qx = fma(cam[0], uc, fma(cam[1], vc, fma(cam[9], invdc, cam[2])));
    const Coord qy = fma(cam[3], uc, fma(cam[4], vc, fma(cam[10], invdc, cam[5])));
    const Coord rz = recip(pz);
    const Coord fxc = qx * rz - (Coord)0.5, fyc = qy * rz - (Coord)0.5;
    const bool ok = a_ok && (pz > (Coord)1e-6) && (fxc > (Coord)-2) && (fxc < (Coord)(fw + 1)) &&
                    (fyc > (Coord)-2) && (fyc < (Coord)(fh + 1));
    const Coord xf = floor(fxc), yf = floor(fyc);
    const float wx = (float)(fxc - xf), wy = (float)(fyc - yf);
    const int ix = ok ? (int)xf : -4, iy = ok ? (int)yf : -4;
    const bool vx0 = (unsigned)ix < (unsigned)fw, vx1 = (unsigned)(ix + 1) < (unsigned)fw;
    const bool vy0 = (unsigned)iy < (unsigned)fh, vy1 = (unsigned)(iy + 1) < (unsigned)fh;
    tp.w[0] = (vx0 && vy0) ? (1.0f - wx) * (1.0f - wy) : 0.0f;
    tp.w[1] = (vx1 && vy0) ? wx * (1.0f - wy) : 0.0f;
    tp.w[2] = (vx0 && vy1) ? (1.0f - wx) * wy : 0.0f;
    tp.w[3] = (vx1 && vy1) ? wx * wy : 0.0f;
    const int o = (iy * fw + ix) * C * E;
    tp.o[0] = (vx0 && vy0) ? o : kTapOOB;
    tp.o[1] = (vx1 && vy0) ? o + C * E : kTapOOB;
    tp.o[2] = (vx0 && vy1) ? o + fw * C * E : kTapOOB;
    tp.o[3] = (vx1 && vy1) ? o + (fw + 1) * C * E : kTapOOB;
}

// Projection groups (GR = 4, C >= 32): the four lanes that load one pixel's
// taps (a quad) take the views four at a time: lane k of the quad projects
// the pixel into view m0 + k, and view m0 + K reaches the whole quad from its
// lane K by a DPP quad permutation -- one projection per lane for four views
// instead of one per view.  GR = 1: each lane projects every view itself
// (C = 16, two lanes per pixel, where pairs save less than the registers
// they hold cost).  The results are identical.
template <int GR, int K>
__device__ inline int group_bcast(int v) {
    static_assert(GR == 1 || GR == 4, "a pixel's load group is one lane or a quad");
    if constexpr (GR == 1) return v;
    else return __builtin_amdgcn_update_dpp(0, v, K * 0x55, 0xf, 0xf, true);
}

// Issues the loads of view m (lane K of the group projected it): channels
// ch0 + 32 kc + [0, 8) of the four taps.
template <int C, bool BF16, int GR, int K>
__device__ inline void issue_group(const UFParams &p, int m, const TapProj &pr, int ch0,
                                   Taps<C, BF16> &tp) {
    constexpr int KC = Shape<C>::KC;
    constexpr int E = (int)sizeof(typename Op<BF16>::T);
    const __amdgpu_buffer_rsrc_t fr = feat_rsrc<C, BF16>(p, m);
    int o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        o[j] = group_bcast<GR, K>(pr.o[j]) + ch0 * E;
        tp.w[j] = __int_as_float(group_bcast<GR, K>(__float_as_int(pr.w[j])));
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int j = 0; j < 4; ++j) buf_load<BF16>(fr, o[j] + 32 * kc * E, tp.t[kc][j]);
}

// Calls f(integral_constant<int, K>) for K = B .. N - 1.
template <int B, int N, typename F>
__device__ inline void static_for(F &&f) {
    if constexpr (B < N) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, N>(f);
    }
}

// Second half of the bilinear sample: the weighted sum of the four taps in
// FP32 (tap order 00, 10, 01, 11).
template <int C, bool BF16>
__device__ inline void blend_taps(const Taps<C, BF16> &tp, float (&sv)[Shape<C>::KC][8]) {
#pragma unroll
    for (int kc = 0; kc < Shape<C>::KC; ++kc) {
        float t00[8], t10[8], t01[8], t11[8];
        raw_unpack<BF16>(tp.t[kc][0], t00);
        raw_unpack<BF16>(tp.t[kc][1], t10);
        raw_unpack<BF16>(tp.t[kc][2], t01);
        raw_unpack<BF16>(tp.t[kc][3], t11);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            sv[kc][i] = fmaf(tp.w[3], t11[i], fmaf(tp.w[2], t01[i], fmaf(tp.w[1], t10[i], tp.w[0] * t00[i])));
    }
}

// C = 8 taps-along-K: lane (r, g) reprojects its own pixel (16 g + r) into
// view m, publishes that pixel's four (tap offset, weight) pairs in LDS, and
// for each row-group j = 0..3 loads tap (l & 3) of pixel 16 j + (l >> 2)
// (l = 16 g + r); the weighted taps reach the operand layout (tap g of pixel
// 16 j + r in lane (r, g)) through the same LDS slice.
template <bool BF16>
struct TapsK {
    RawTap<BF16> t[4];
    float w[4];
};

template <int C, bool BF16>
__device__ inline void issue_tapk(const UFParams &p, int m, typename CoordT<BF16>::type uc,
                                  typename CoordT<BF16>::type vc, typename CoordT<BF16>::type invdc,
                                  bool a_ok, int r, int g, int2 *tT, TapsK<BF16> &tp) {
    using Coord = typename CoordT<BF16>::type;
    using T = typename Op<BF16>::T;
    const __amdgpu_buffer_rsrc_t fr = feat_rsrc<C, BF16>(p, m);
    const int fh = p.fH[m], fw = p.fW[m];
    const Coord pz = fma(cam_entry<BF16>(p, m, 6), uc,
                         fma(cam_entry<BF16>(p, m, 7), vc,
                             fma(cam_entry<BF16>(p, m, 11), invdc, cam_entry<BF16>(p, m, 8))));
    const Coord qx = fma(cam_entry<BF16>(p, m, 0), uc,
                         fma(cam_entry<BF16>(p, m, 1), vc,
                             fma(cam_entry<BF16>(p, m, 9), invdc, cam_entry<BF16>(p, m, 2))));
    const Coord qy = fma(cam_entry<BF16>(p, m, 3), uc,
                         fma(cam_entry<BF16>(p, m, 4), vc,
                             fma(cam_entry<BF16>(p, m, 10), invdc, cam_entry<BF16>(p, m, 5))));
    const Coord rz = recip(pz);
    const Coord fxc = qx * rz - (Coord)0.5, fyc = qy * rz - (Coord)0.5;
    const bool ok = a_ok && (pz > (Coord)1e-6) && (fxc > (Coord)-2) && (fxc < (Coord)(fw + 1)) &&
                    (fyc > (Coord)-2) && (fyc < (Coord)(fh + 1));
    const Coord xf = floor(fxc), yf = floor(fyc);
    const float wx = (float)(fxc - xf), wy = (float)(fyc - yf);
    const int ix = ok ? (int)xf : -4, iy = ok ? (int)yf : -4;
    const bool vx0 = (unsigned)ix < (unsigned)fw, vx1 = (unsigned)(ix + 1) < (unsigned)fw;
    const bool vy0 = (unsigned)iy < (unsigned)fh, vy1 = (unsigned)(iy + 1) < (unsigned)fh;
    // byte offsets as in project_view (an out-of-map tap reads zeros at kTapOOB)
    constexpr int E = (int)sizeof(T);
    const int o = (iy * fw + ix) * C * E;
    int4 ow0, ow1;       // (byte offset, weight bits) of taps 00, 10 | 01, 11
    ow0.x = (vx0 && vy0) ? o : kTapOOB;
    ow0.y = __float_as_int((vx0 && vy0) ? (1.0f - wx) * (1.0f - wy) : 0.0f);
    ow0.z = (vx1 && vy0) ? o + C * E : kTapOOB;
    ow0.w = __float_as_int((vx1 && vy0) ? wx * (1.0f - wy) : 0.0f);
    ow1.x = (vx0 && vy1) ? o + fw * C * E : kTapOOB;
    ow1.y = __float_as_int((vx0 && vy1) ? (1.0f - wx) * wy : 0.0f);
    ow1.z = (vx1 && vy1) ? o + (fw + 1) * C * E : kTapOOB;
    ow1.w = __float_as_int((vx1 && vy1) ? wx * wy : 0.0f);
    int4 *slot = reinterpret_cast<int4 *>(&tT[(g * 16 + r) * 4]);
    slot[0] = ow0;
    slot[1] = ow1;
    // row-group j: lane l loads tap (l & 3) of pixel 16 j + (l >> 2), so each
    // quad of lanes reads the four taps of one pixel (two 32-byte runs)
    const int lane = 16 * g + r;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int2 e = tT[64 * j + lane];
        tp.w[j] = __int_as_float(e.y);
        buf_load<BF16>(fr, e.x, tp.t[j]);
    }
}

// Pair sums across lane rows (a row is 16 lanes): with both operands equal,
// the two outputs of a permlane swap hold the two rows of each pair
// broadcast, so their sum is the pair sum (rows 0+1 and 2+3 for the 16-swap,
// rows 0..1 + 2..3 for the 32-swap).
__device__ inline float rows_pair_sum16(float v) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
__device__ inline float rows_pair_sum32(float v) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
// Value of the odd row of this lane's row pair (for even rows).
__device__ inline float odd_row_value(float v) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(s[1]);
}

// Sum over the lanes that hold one pixel's channels in the operand layout:
// lanes 16 apart (C = 16) or all four rows (C >= 32).
template <int C>
__device__ inline float operand_pixel_sum(float v) {
    if constexpr (C >= 16) v = rows_pair_sum16(v);
    if constexpr (C >= 32) v = rows_pair_sum32(v);
    return v;
}

// Sum over the lanes that hold one pixel's output channels in the
// accumulator layout: a row pair (C = 8) or all four rows (C >= 16).
template <int C>
__device__ inline float result_pixel_sum(float v) {
    v = rows_pair_sum16(v);
    if constexpr (C >= 16) v = rows_pair_sum32(v);
    return v;
}

// Reciprocal square root, logistic and tanh from the hardware's
// one-instruction approximations (as recip above; about 1 ulp, far inside the
// float32 form's budget): the IEEE-exact sequences take ten to thirty
// instructions each and sit on the per-layer-pixel path.
__device__ inline float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float sigmoidf_(float x) { return recip(1.0f + __expf(-x)); }
// tanh x = 1 - 2 / (1 + e^{2x}) (absolute error a few 1e-8; saturates to +-1)
__device__ inline float tanhf_(float x) { return 1.0f - 2.0f * recip(1.0f + __expf(2.0f * x)); }

__device__ inline void lds_write4(float *dst, const float *f) {
    *reinterpret_cast<float4 *>(dst) = make_float4(f[0], f[1], f[2], f[3]);
}

// Register budget per instance: the waves per SIMD each form reaches.  At
// four waves (128 VGPRs) the C = 16 standard form parks three values in
// scratch outside the view loop; the extra wave is worth more (levels 1-2:
// -7 %).  The bfloat16 one-to-many form at C = 64 is held to three waves
// (168 VGPRs), which its LDS allows too.  Float32: the one-to-many form at
// C <= 32 gets three waves (168 VGPRs; at C = 8 five values go to scratch,
// level 3 -10 %); the float32 standard form keeps the compiler's default (at
// three waves it would spill dozens of values).
template <int C, bool BF16, bool FOLD>
struct Occupancy {
    static constexpr int waves = !BF16 ? ((FOLD && C <= 32) ? 3 : 1) : (C > 32) ? (FOLD ? 3 : 2) : 4;
};

// FOLD = false: standard cross-attention (per-sample key and value
// projections on MFMA), with C / HD heads of HD channels each (C >= 32):
// head h owns output channels h HD .. (h + 1) HD - 1 of Q, K and V, which
// are whole 16-row output tiles for HD >= 16 and, for HD = 8, the upper or
// lower two lanes of a pixel's four in one tile; each lane keeps one softmax
// state per head it holds channels of.  FOLD = true: one-to-many attention -- the key
// projection folded into the query (q~ = N(F) W_q W_k^T / sqrt(d)) and the
// value projection into the output (W_v W_o); the per-view work is a dot
// product and a weighted sum on the samples themselves (for C = 8 the same
// MFMA loop, with the blended sample standing in for keys and values).
//
// VAR selects the variant: kPlain, one level, its parameters in the kernel
// argument; kBlend, the same that also writes the blend-weight logits (one
// head); kBatch, several requests (levels of different size, view count,
// cameras, maps and weights) in one launch -- request r owns the global
// tiles [tile_start[r], tile_start[r + 1]) and its parameters are read from
// device memory (uniform per workgroup).
constexpr int kPlain = 0, kBlend = 1, kBatch = 2;

template <bool BATCH>
struct UFArgs {
    UFParams p;
};
template <>
struct UFArgs<true> {
    const UFParams *reqs;
    UFBatch b;
};

// XCD-aware remap of the dispatch order: workgroups are dispatched to the 8
// XCDs round-robin; each XCD walks one contiguous band of the nt tiles (rows
// of one level, L2 locality of the epipolar bands).
__device__ __forceinline__ int xcd_tile(int i, int nt) {
    const int xcd = i & 7, loc = i >> 3, q = nt >> 3, rem = nt & 7;
    return (xcd < rem) ? xcd * (q + 1) + loc : rem * (q + 1) + (xcd - rem) * q + loc;
}

template <int C, bool BF16, bool FOLD, bool F8, int HD, int VAR>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((FOLD && HD != C) ? 2
                                   : (!BF16 && VAR == kBlend) ? 1    // its extra stores spill at 3
                                   : Occupancy<C, BF16, FOLD>::waves)))
k_update_fuse(const UFArgs<VAR == kBatch> args) {
    constexpr bool BATCH = VAR == kBatch;
    static_assert(VAR != kBlend || HD == C, "blend-weight logits: one head");
    // this workgroup's request and tile
    int req = 0, tile;
    if constexpr (BATCH) {
        const int t = xcd_tile(blockIdx.x, args.b.total_tiles);
        for (int i = 1; i < args.b.n_req; ++i) req = (t >= args.b.tile_start[i]) ? i : req;
        tile = t - args.b.tile_start[req];
    } else {
        tile = xcd_tile(blockIdx.x, args.p.n_tiles);
    }
    const UFParams &p = [&]() -> const UFParams & {
        if constexpr (BATCH) return args.reqs[req];
        else return args.p;
    }();
    static_assert(!F8 || BF16, "e4m3 projections take bfloat16 storage");
    static_assert(HD == C || (C >= 32 && (HD == 8 || (HD >= 16 && C % HD == 0))),
                  "several heads: C >= 32, head width 8 or a multiple of 16");
    static_assert(!(FOLD && HD != C && (F8 || C != 32)),
                  "several folded heads: C = 32, bfloat16 or float32 (LDS holds HQ query blocks)");
    using SH = Shape<C>;
    using OP = Op<BF16>;
    using AF = typename OP::A;
    using MM = Mm<BF16, F8>;                    // Q/K/V/O operands
    using MA = typename MM::A;
    using T = typename OP::T;
    using Coord = typename CoordT<BF16>::type;
    constexpr int G = SH::G, KC = SH::KC, NT = SH::NT, ND = SH::ND, PIX = SH::PIX, P = SH::P;
    constexpr bool TAPK = SH::TAPK;
    constexpr bool STDLOOP = !FOLD || TAPK;     // the MFMA view loop
    // softmax states per lane: one per 16-pixel sub-tile (G > 1), else one
    // per head whose channels the lane holds (TPH output tiles per head)
    constexpr int TPH = (HD >= 16) ? HD / 16 : 1;
    constexpr int NS = (G == 1) ? ((HD >= 16) ? NT / TPH : NT) : NT;
    // the state of output tile t
    auto st_of = [](int t) constexpr { return (G == 1 && HD >= 16) ? t / TPH : t; };
    // the one-to-many form with several heads keeps one C-channel query, one
    // softmax state and one running sum of the samples per head
    constexpr int HQ = FOLD ? C / HD : 1;
    using FR = Frags<C, STDLOOP, HQ>;
    static_assert(!TAPK || 64 * sizeof(MA) <= PIX * P * sizeof(float),
                  "tap staging must fit the o tile it shares");
    static_assert(TAPK || PIX * (C / 8 + (sizeof(MA) <= 16 ? 1 : 0)) * sizeof(MA) <= PIX * P * sizeof(float),
                  "sample staging must fit the o tile it shares");
    static_assert(!TAPK || 64 * 4 * sizeof(int2) <= PIX * P * sizeof(float),
                  "tap exchange must fit the o tile it shares");

    __shared__ AF sfrag[FR::N][64];    // FP8 form: Q/K/V/O slots hold e4m3 codes in their first 8 B
    // views per projection group (see group_bcast); with groups, the camera
    // entries and map sizes of every view sit in LDS (a lane projects into a
    // view of its own), in a table of their own -- except in the bfloat16
    // one-to-many form at C = 64, whose LDS allocation is at the limit of
    // three workgroups per CU: there the table (12 floats and 2 ints per
    // view) lives in the four pad floats that end every pixel row of the sF
    // slices, which nothing else touches (a table of its own cost a
    // workgroup per CU, and the pad reads cost registers elsewhere).
    constexpr int GR = (C >= 32) ? 4 : 1;
    constexpr bool PADTAB = GR > 1 && BF16 && FOLD && C == 64;
    static_assert(!PADTAB || (P == C + 4 && 4 * PIX * 4 >= kMaxViews * 14),
                  "the pad columns hold the camera table");
    __shared__ Coord scam[(GR > 1 && !PADTAB) ? kMaxViews * 12 : 1];
    __shared__ int sfwh[(GR > 1 && !PADTAB) ? kMaxViews * 2 : 1];
    __shared__ float sF[4][PIX * P];
    __shared__ float sO[4][PIX * P];   // o tile; for C = 8 also the tap exchange
    // word w of the padded table: pad row w / 4 (rows run through the four
    // slices), float w % 4; view m's entries are words 12 m .. 12 m + 11, its
    // map width and height words 12 kMaxViews + 2 m and + 1
    auto padw = [&](int w) -> float * {
        const int r = w >> 2;
        return &sF[r / PIX][(r % PIX) * P + C + (w & 3)];
    };

    const int tid = threadIdx.x;

    // e4m3 per-tensor scales (value = scale x code): query input, samples,
    // W_q, W_k, W_v, W_o, attention output
    float f8s[7] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
    if constexpr (F8) {
#pragma unroll
        for (int i = 0; i < 7; ++i) f8s[i] = p.f8_scales[i];
    }
    const float f8_inv_x = 1.0f / f8s[0], f8_inv_s = 1.0f / f8s[1], f8_inv_o = 1.0f / f8s[6];

    // ---- weight fragments from the float32 master weights, once per
    // workgroup.  Fragment lane (c, k) holds element [k-slot 8k..8k+7][c] of
    // W (the A operand of the transposed products).  Every projection is
    // block-diagonal over the G sub-tiles.
    for (int e = tid; e < FR::N * 64; e += 256) {
        const int f = e >> 6, ln = e & 63;
        const int nn = ln & 15, gg = ln >> 4;
        // kinds: 0 Q, 1 K, 2 V, 3 O, 4 decode (no K/V slots in the
        // one-to-many form: the O slots follow Q)
        const int kind = f < FR::OFF_K ? 0 : f < FR::OFF_V ? 1 : f < FR::OFF_O ? 2
                       : f < FR::OFF_D ? 3 : 4;
        int fi = f - (kind == 0 ? FR::OFF_Q : kind == 1 ? FR::OFF_K : kind == 2 ? FR::OFF_V
                      : kind == 3 ? FR::OFF_O : FR::OFF_D);
        int head = 0;                             // query block of a Q fragment
        if (HQ > 1 && kind == 0) { head = fi / (KC * NT); fi -= head * KC * NT; }
        const int ntile = (kind == 4) ? ND : NT;
        const int kc = fi / ntile, t = fi % ntile;
        const int ng = 16 * t + nn;               // output channel row of this lane
        const float *Wm = kind == 0 ? (FOLD ? p.Wqk + (size_t)head * C * C : p.Wq) : kind == 1 ? p.Wk
                        : kind == 2 ? p.Wv : (FOLD ? p.Wvo : p.Wo);
        float vals[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int kap = 32 * kc + 8 * gg + i;   // K slot: sub-tile kap / C, channel kap % C
            float w = 0.0f;
            if (TAPK && (kind == 1 || kind == 2)) {
                // K slot kap = tap (kap / 8) x channel (kap % 8); output rows
                // 8t..8t+7 of the tile hold row-group t of a pair
                if (nn / 8 == t) {
                    if (FOLD) w = (kap % 8 == nn % 8) ? 1.0f : 0.0f;     // the blended sample itself
                    else w = Wm[(kap % 8) * C + (nn % 8)];
                }
            } else if (HQ > 1 && kind == 3) {
                // output projection over the heads' concatenation: K slot kap
                // is channel kap % C of head kap / C
                w = (Wm + (size_t)(kap / C) * C * C)[(kap % C) * C + ng];
            } else if (kind < 4) {
                if (kap / C == ng / C) w = Wm[(kap % C) * C + (ng % C)];
            } else {                                // decode heads: sigma, depth, r, g, b
                const int s = (G == 1) ? 0 : ng / 8;
                const int j = (G == 1) ? ng : ng % 8;
                if (kap / C == s && j < 5) {
                    const int c = kap % C;
                    w = (j == 0) ? p.w_sigma[c] : (j == 1) ? p.w_depth[c] : p.W_color[c * 3 + (j - 2)];
                }
            }
            vals[i] = w;
        }
        if constexpr (F8) {
            if (kind < 4) {
                *reinterpret_cast<MA *>(&sfrag[f][ln]) = MM::make(vals, 1.0f / f8s[2 + kind]);
                continue;
            }
        }
        sfrag[f][ln] = OP::make(vals);
    }
    if constexpr (PADTAB) {
        for (int e = tid; e < p.V * 12; e += 256) *padw(e) = p.cam[e / 12][e % 12];
        for (int e = tid; e < p.V; e += 256) {
            *padw(12 * kMaxViews + 2 * e) = __int_as_float(p.fW[e]);
            *padw(12 * kMaxViews + 2 * e + 1) = __int_as_float(p.fH[e]);
        }
    } else if constexpr (GR > 1) {
        for (int e = tid; e < p.V * 12; e += 256) scam[e] = cam_entry<BF16>(p, e / 12, e % 12);
        for (int e = tid; e < p.V; e += 256) {
            sfwh[2 * e] = p.fW[e];
            sfwh[2 * e + 1] = p.fH[e];
        }
    }
    __syncthreads();

    // ---- the tile's place in the level
    const int wave = tid >> 6, lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const int chunk = tile % p.chunks;
    const int rest = tile / p.chunks;
    const int xb = rest % p.x_blocks;
    const int y = rest / p.x_blocks;
    const int x0w = xb * (4 * PIX) + wave * PIX;       // first pixel of this wave
    if (x0w >= p.W) return;                            // no later barrier: safe to leave
    const int l_begin = chunk * p.layers_per_chunk;
    const int l_end = min(p.L, l_begin + p.layers_per_chunk);

    // operand role of this lane: pixel column n of sub-tile sg, channels
    // ch0 + 32 kc + [0, 8)
    const int sg = (G > 1) ? (8 * g) / C : 0;
    const int ch0 = (G > 1) ? (8 * g) % C : 8 * g;
    const int pl_b = 16 * sg + n;                      // wave-local pixel
    const int xa = x0w + pl_b;
    const bool a_ok = xa < p.W;
    // load role of this lane (C >= 16): RL adjacent lanes read one pixel's
    // tap chunk as consecutive 16-byte pieces, which the texture path serves
    // together (in the operand layout the lanes of a pixel are 16 apart, so
    // every lane of a quad would hit a different line); the blended sample
    // then goes to the operand layout through the wave's LDS slice.  C = 8
    // (taps along K) keeps its own scheme.
    constexpr int RL = TAPK ? 1 : ((C >= 32) ? 4 : C / 8);
    const int pl_ld = TAPK ? pl_b : lane / RL;
    const int ch_ld = TAPK ? ch0 : 8 * (lane % RL);
    const int x_ld = x0w + pl_ld;
    const bool ld_ok = x_ld < p.W;
    // result role: output rows 4g..4g+3 of tile t belong to sub-tile sd(t),
    // channels ed(t) + [0, 4)
    auto sd = [&](int t) { return (G > 1) ? (16 * t + 4 * g) / C : 0; };
    auto ed = [&](int t) { return (G > 1) ? (16 * t + 4 * g) % C : 16 * t + 4 * g; };
    // decode owner lanes: heads 0..3 of a pixel sit in an even row, head 4 in
    // the row after it
    const bool owner = (G > 1) ? ((g & 1) == 0) : (g == 0);

    // projection fragment f of this lane (e4m3 copy in the FP8 form)
    auto pfrag = [&](int f) -> MA {
        if constexpr (F8) return *reinterpret_cast<const MA *>(&sfrag[f][lane]);
        else return sfrag[f][lane];
    };
    constexpr int KCB = STDLOOP ? KC : 1, NTB = STDLOOP ? NT : 1;
    MA Bk[KCB][NTB], Bv[KCB][NTB];
    if constexpr (STDLOOP) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                Bk[kc][t] = pfrag(FR::OFF_K + kc * NT + t);
                Bv[kc][t] = pfrag(FR::OFF_V + kc * NT + t);
            }
    }
    // scale of a key logit and of a value in the FP8 form (1 otherwise)
    const float kscale = f8s[3] * f8s[1];
    const float vscale = (TAPK && FOLD) ? kscale : f8s[4] * f8s[1];   // folded C = 8: v = k

    float *tF = sF[wave];
    float *tO = sO[wave];
    const T *Fin = reinterpret_cast<const T *>(p.F_in);
    T *Fout = reinterpret_cast<T *>(p.F_out);
    const bool do_comp = p.rgb != nullptr;
    const float scale = FOLD ? 1.0f : 1.0f / sqrtf((float)HD);  // folded: W_qk carries it
    const Coord uc = (Coord)(a_ok ? xa : 0) + (Coord)0.5, vc = (Coord)y + (Coord)0.5;
    const Coord uc_ld = (Coord)(ld_ok ? x_ld : 0) + (Coord)0.5;
    const float band = p.inv_near - p.inv_far;
    const float half_l = 0.5f / (float)p.L;

    float Tr[ND], cr[ND][3];
#pragma unroll
    for (int td = 0; td < ND; ++td) { Tr[td] = 1.0f; cr[td][0] = cr[td][1] = cr[td][2] = 0.0f; }

    for (int li = l_begin; li < l_end; ++li) {
        const size_t rowbase = ((size_t)li * p.H + y) * p.W;
        const size_t pa = rowbase + (a_ok ? xa : 0);
        const float d = a_ok ? p.depth_in[pa] : 1.0f;

        // ---- LDM features of this lane's pixel (operand layout), to LDS
        float fa[KC][8];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            if (a_ok) OP::load8(Fin + pa * C + ch0 + 32 * kc, fa[kc]);
            else
#pragma unroll
                for (int i = 0; i < 8; ++i) fa[kc][i] = 0.0f;
            float *dst = &tF[pl_b * P + ch0 + 32 * kc];
            lds_write4(dst, fa[kc]);
            lds_write4(dst + 4, fa[kc] + 4);
        }

        // ---- RMSNorm (unit gain, eps 1e-6) over the pixel's channels; query
        float ss = 0.0f;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int i = 0; i < 8; ++i) ss = fmaf(fa[kc][i], fa[kc][i], ss);
        ss = operand_pixel_sum<C>(ss);
        const float inv = rsqrt_(ss * (1.0f / (float)C) + 1e-6f);
        f32x4 Q[HQ * NT];
        {
            MA Xn[KC];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float t8[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) t8[i] = fa[kc][i] * inv;
                Xn[kc] = MM::make(t8, f8_inv_x);
            }
#pragma unroll
            for (int qt = 0; qt < HQ * NT; ++qt) {
                const int hq = qt / NT, t = qt % NT;
                Q[qt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    Q[qt] = MM::mma(pfrag(FR::OFF_Q + hq * KC * NT + kc * NT + t), Xn[kc], Q[qt]);
                if constexpr (F8) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) Q[qt][i] *= f8s[2] * f8s[0];
                }
            }
        }

        MA Ob[HQ * KC];                                // o, operand layout
        const Coord invdc = recip((Coord)d);
        const float d_ld = TAPK ? d : (ld_ok ? p.depth_in[rowbase + x_ld] : 1.0f);
        const Coord invdc_ld = TAPK ? invdc : recip((Coord)d_ld);
        // The view loop: two tap buffers in turn, so the loads of view m + 1
        // are in flight while view m is processed, and no buffer is copied.
        // The scheduling barriers keep the loads ahead of the arithmetic (left
        // alone, the scheduler moves the next view's loads after this view's
        // work, which serialises the views on memory latency).  The issues
        // are unconditional (clamped view index; the extra loads at the end
        // hit the cache) so the wait counts stay exact.
        int2 *tT = reinterpret_cast<int2 *>(sO[wave]);   // C = 8 tap exchange
        auto run_views = [&](auto &ta, auto &tb, auto &&view_step) {
            if constexpr (TAPK) {
                issue_tapk<C, BF16>(p, 0, uc_ld, vc, invdc_ld, ld_ok, n, g, tT, ta);
                __builtin_amdgcn_sched_barrier(0);
                for (int m = 0; m < p.V; m += 2) {
                    issue_tapk<C, BF16>(p, min(m + 1, p.V - 1), uc_ld, vc, invdc_ld, ld_ok, n, g, tT, tb);
                    __builtin_amdgcn_sched_barrier(0);
                    view_step(ta, m);
                    __builtin_amdgcn_sched_barrier(0);
                    issue_tapk<C, BF16>(p, min(m + 2, p.V - 1), uc_ld, vc, invdc_ld, ld_ok, n, g, tT, ta);
                    __builtin_amdgcn_sched_barrier(0);
                    if (m + 1 < p.V) view_step(tb, m + 1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                // views in groups of GR (see group_bcast); a group past the
                // last view is not projected, and its clamped issue reads
                // stale offsets through the last view's range-checked buffer
                TapProj pr;
                auto project = [&](int m0) {
                    if constexpr (PADTAB) {
                        const int mv = min(m0 + lane % GR, p.V - 1);
                        float cam[12];
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            const float4 c4 = *reinterpret_cast<const float4 *>(padw(12 * mv + 4 * r));
                            cam[4 * r] = c4.x; cam[4 * r + 1] = c4.y;
                            cam[4 * r + 2] = c4.z; cam[4 * r + 3] = c4.w;
                        }
                        const float2 wh = *reinterpret_cast<const float2 *>(padw(12 * kMaxViews + 2 * mv));
                        project_view<C, BF16>(cam, __float_as_int(wh.x), __float_as_int(wh.y), uc_ld, vc,
                                              invdc_ld, ld_ok, pr);
                    } else if constexpr (GR > 1) {
                        const int mv = min(m0 + lane % GR, p.V - 1);
                        project_view<C, BF16>(&scam[mv * 12], sfwh[2 * mv], sfwh[2 * mv + 1], uc_ld, vc,
                                              invdc_ld, ld_ok, pr);
                    } else {
                        project_view<C, BF16>(cam_row<BF16>(p, m0), p.fW[m0], p.fH[m0], uc_ld, vc,
                                              invdc_ld, ld_ok, pr);
                    }
                };
                static_assert(GR == 1 || RL == GR, "a projection group is a pixel's load group");
                constexpr int ST = (GR > 1) ? GR : 2;     // views per unrolled step
                project(0);
                issue_group<C, BF16, GR, 0>(p, 0, pr, ch_ld, ta);
                __builtin_amdgcn_sched_barrier(0);
                for (int m0 = 0; m0 < p.V; m0 += ST) {
                    static_for<0, ST>([&](auto kk) {
                        constexpr int k = decltype(kk)::value;
                        auto &cur = (k % 2 == 0) ? ta : tb;
                        auto &nxt = (k % 2 == 0) ? tb : ta;
                        const int mn = min(m0 + k + 1, p.V - 1);
                        if constexpr (GR == 1) {
                            project(mn);
                            issue_group<C, BF16, 1, 0>(p, mn, pr, ch_ld, nxt);
                        } else if constexpr (k + 1 < GR) {
                            issue_group<C, BF16, GR, k + 1>(p, mn, pr, ch_ld, nxt);
                        } else {
                            if (m0 + GR < p.V) project(m0 + GR);
                            issue_group<C, BF16, GR, 0>(p, mn, pr, ch_ld, nxt);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        if (m0 + k < p.V) view_step(cur, m0 + k);
                        __builtin_amdgcn_sched_barrier(0);
                    });
                }
            }
        };
        if constexpr (STDLOOP) {
            // ---- cross-attention over the views on MFMA: per-sample keys and
            // values (standard form) or, for C = 8 folded, the blended samples
            // themselves; online softmax (finite start, so the first view
            // always moves the reference)
            float M[NS], Z[NS];
            f32x4 acc[NT];
#pragma unroll
            for (int s = 0; s < NS; ++s) { M[s] = -1e30f; Z[s] = 0.0f; }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

            using TapsT = typename std::conditional<TAPK, TapsK<BF16>, Taps<C, BF16>>::type;
            // one view: blend -> keys -> logits -> online softmax -> values
            auto view_step = [&](const TapsT &cur, int m) {
                // B operands: the blended sample (one per K chunk), or for C = 8
                // the weighted taps of each 16-pixel row-group
                constexpr int NA = TAPK ? 4 : KC;
                MA Sb[NA];
                if constexpr (TAPK) {
                    // the slice that held the tap offsets is free again: the
                    // next view's loads have taken theirs
                    MA *stage = reinterpret_cast<MA *>(tT);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float t8[8];
                        raw_unpack<BF16>(cur.t[j], t8);
#pragma unroll
                        for (int i = 0; i < 8; ++i) t8[i] *= cur.w[j];
                        stage[16 * (lane & 3) + (lane >> 2)] = MM::make(t8, f8_inv_s);
                        Sb[j] = stage[lane];
                    }
                } else {
                    // blend and round in the load layout, then move the
                    // operand words (8 channels each) through the LDS slice;
                    // rows padded by one word where they are 16 B or less
                    float sv[KC][8];
                    blend_taps<C, BF16>(cur, sv);
                    constexpr int RW = C / 8 + (sizeof(MA) <= 16 ? 1 : 0);
                    MA *st = reinterpret_cast<MA *>(tO);
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc)
                        st[pl_ld * RW + (ch_ld + 32 * kc) / 8] = MM::make(sv[kc], f8_inv_s);
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) Sb[kc] = st[pl_b * RW + (ch0 + 32 * kc) / 8];
                }
                // keys^T and logits
                f32x4 Kt[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    Kt[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                    if constexpr (TAPK) {
                        Kt[t] = MM::mma(Bk[0][0], Sb[2 * t], Kt[t]);
                        Kt[t] = MM::mma(Bk[0][1], Sb[2 * t + 1], Kt[t]);
                    } else {
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc) Kt[t] = MM::mma(Bk[kc][t], Sb[kc], Kt[t]);
                    }
                }
                float lg[NS];
                if constexpr (G == 1 && HD >= 16) {
                    // a head's channels: TPH whole tiles, all four lanes
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        float part = 0.0f;
#pragma unroll
                        for (int t = s * TPH; t < (s + 1) * TPH; ++t)
#pragma unroll
                            for (int i = 0; i < 4; ++i) part = fmaf(Q[t][i], Kt[t][i], part);
                        lg[s] = result_pixel_sum<C>(part) * (scale * kscale);
                    }
                } else if constexpr (G == 1) {
                    // HD = 8: the lane's four rows of tile t and its row-pair
                    // partner's are one head
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        float part = 0.0f;
#pragma unroll
                        for (int i = 0; i < 4; ++i) part = fmaf(Q[t][i], Kt[t][i], part);
                        lg[t] = rows_pair_sum16(part) * (scale * kscale);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        float part = 0.0f;
#pragma unroll
                        for (int i = 0; i < 4; ++i) part = fmaf(Q[t][i], Kt[t][i], part);
                        lg[t] = result_pixel_sum<C>(part) * (scale * kscale);
                    }
                }
                if constexpr (VAR == kBlend || (VAR == kBatch && HD == C)) {
                    // blend-weight logits (one head): written by the lane that
                    // holds channel 0 of the pixel in the result layout (in a
                    // batch, for the requests that ask for them)
                    if (VAR == kBlend || p.blend_logit != nullptr) {
#pragma unroll
                        for (int s = 0; s < NS; ++s) {
                            const int t = (G == 1) ? s * TPH : s;
                            const int xe = x0w + 16 * sd(t) + n;
                            if (ed(t) == 0 && xe < p.W)
                                p.blend_logit[(rowbase + xe) * p.V + m] = lg[s];
                        }
                    }
                }
                // online softmax with a lazily moved reference: weights are
                // exp(logit - M) while the logit stays within e^8 of M; only
                // a logit beyond that (always the first view, rarely another)
                // rescales the running sums to a new reference
                float pw[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    float diff = lg[s] - M[s];
                    if (diff > 8.0f) {
                        const float r = __expf(-diff);
                        Z[s] *= r;
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            if (st_of(t) == s)
#pragma unroll
                                for (int i = 0; i < 4; ++i) acc[t][i] *= r;
                        M[s] = lg[s];
                        diff = 0.0f;
                    }
                    pw[s] = __expf(diff);
                    Z[s] += pw[s];
                }
                // values^T
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    f32x4 Vt = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                    if constexpr (TAPK && FOLD) {
                        Vt = Kt[t];                      // values are the samples themselves
                    } else if constexpr (TAPK) {
                        Vt = MM::mma(Bv[0][0], Sb[2 * t], Vt);
                        Vt = MM::mma(Bv[0][1], Sb[2 * t + 1], Vt);
                    } else {
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc) Vt = MM::mma(Bv[kc][t], Sb[kc], Vt);
                    }
                    const int s = st_of(t);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[t][i] = fmaf(pw[s], Vt[i], acc[t][i]);
                }
            };
            TapsT ta, tb;
            run_views(ta, tb, view_step);

            // o = acc / Z: result layout -> LDS -> operand layout
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float iz = vscale * recip(Z[st_of(t)]);
                float o4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) o4[i] = acc[t][i] * iz;
                lds_write4(&tO[(16 * sd(t) + n) * P + ed(t)], o4);
            }
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float t8[8];
                lds_read8(&tO[pl_b * P + ch0 + 32 * kc], t8);
                Ob[kc] = MM::make(t8, f8_inv_o);
            }
        } else {
            // ---- one-to-many attention: q~ (the query with W_k folded in) to
            // the operand layout, then per view a dot product with the FP32
            // sample and a weighted running sum of the samples themselves --
            // per head, through the same LDS slice one head after another
            float qa[HQ][KC][8], ob[HQ][KC][8];
#pragma unroll
            for (int hq = 0; hq < HQ; ++hq) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    float q4[4] = {Q[hq * NT + t][0], Q[hq * NT + t][1], Q[hq * NT + t][2],
                                   Q[hq * NT + t][3]};
                    lds_write4(&tO[(16 * sd(t) + n) * P + ed(t)], q4);
                }
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    lds_read8(&tO[pl_b * P + ch0 + 32 * kc], qa[hq][kc]);
#pragma unroll
                    for (int i = 0; i < 8; ++i) ob[hq][kc][i] = 0.0f;
                }
            }
            float Mx[HQ], Zs[HQ];
#pragma unroll
            for (int hq = 0; hq < HQ; ++hq) { Mx[hq] = -1e30f; Zs[hq] = 0.0f; }
            auto view_step = [&](const Taps<C, BF16> &cur, int m) {
                float sv[KC][8];
                blend_taps<C, BF16>(cur, sv);
                stage_sample<C>(tO, pl_ld, ch_ld, pl_b, ch0, sv);
#pragma unroll
                for (int hq = 0; hq < HQ; ++hq) {
                    float part = 0.0f;
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                        for (int i = 0; i < 8; ++i) part = fmaf(qa[hq][kc][i], sv[kc][i], part);
                    const float a = operand_pixel_sum<C>(part);
                    if constexpr (VAR == kBlend || (VAR == kBatch && HQ == 1)) {
                        // blend-weight logit: the lane holding channel 0
                        if ((VAR == kBlend || p.blend_logit != nullptr) && ch0 == 0 && a_ok)
                            p.blend_logit[(rowbase + xa) * p.V + m] = a;
                    }
                    float diff = a - Mx[hq];
                    if (diff > 8.0f) {             // lazily moved reference (see above)
                        const float r = __expf(-diff);
                        Zs[hq] *= r;
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                            for (int i = 0; i < 8; ++i) ob[hq][kc][i] *= r;
                        Mx[hq] = a;
                        diff = 0.0f;
                    }
                    const float pw = __expf(diff);
                    Zs[hq] += pw;
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                        for (int i = 0; i < 8; ++i) ob[hq][kc][i] = fmaf(pw, sv[kc][i], ob[hq][kc][i]);
                }
            };
            Taps<C, BF16> ta, tb;
            run_views(ta, tb, view_step);
#pragma unroll
            for (int hq = 0; hq < HQ; ++hq) {
                const float iz = recip(Zs[hq]);
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    float t8[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) t8[i] = ob[hq][kc][i] * iz;
                    Ob[hq * KC + kc] = MM::make(t8, f8_inv_o);
                }
            }
        }

        // ---- F'^T = W_o^T o^T + F^T (the accumulator starts from F)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float *fp = &tF[(16 * sd(t) + n) * P + ed(t)];
            const float4 f4 = *reinterpret_cast<const float4 *>(fp);
            // FP8 form: F' = F + s (W_o o)_codes with s = s_Wo s_o, accumulated
            // as s (F / s + codes product)
            const float os = f8s[5] * f8s[6], ios = 1.0f / os;
            f32x4 Fo = F8 ? f32x4{f4.x * ios, f4.y * ios, f4.z * ios, f4.w * ios}
                          : f32x4{f4.x, f4.y, f4.z, f4.w};
#pragma unroll
            for (int kc = 0; kc < FR::KCO; ++kc) Fo = MM::mma(pfrag(FR::OFF_O + kc * NT + t), Ob[kc], Fo);
            if constexpr (F8) {
#pragma unroll
                for (int i = 0; i < 4; ++i) Fo[i] *= os;
            }
            *reinterpret_cast<float4 *>(fp) = make_float4(Fo[0], Fo[1], Fo[2], Fo[3]);
        }

        // ---- F' back to the operand layout: store it and decode it
        f32x4 X[ND];
#pragma unroll
        for (int td = 0; td < ND; ++td) X[td] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            float t8[8];
            lds_read8(&tF[pl_b * P + ch0 + 32 * kc], t8);
            if (Fout != nullptr && a_ok) OP::store8(Fout + pa * C + ch0 + 32 * kc, t8);
            const AF af = OP::make(t8);
#pragma unroll
            for (int td = 0; td < ND; ++td) X[td] = OP::mma(sfrag[FR::OFF_D + kc * ND + td][lane], af, X[td]);
        }

        // ---- decode depth / alpha / colour of this lane's pixels, composite
#pragma unroll
        for (int td = 0; td < ND; ++td) {
            const float head4 = odd_row_value(X[td][0]);       // the blue head
            const int s = (G > 1) ? 2 * td + g / 2 : 0;
            const int xe = x0w + 16 * s + n;
            if (owner && xe < p.W) {
                const size_t pe = rowbase + xe;
                const float de = p.depth_in[pe];
                const float a_in = p.alpha_in[pe];
                const float xs = X[td][0], xd = X[td][1];
                float an, dn;
                if (p.mode == 0) {
                    const float a = fminf(fmaxf(a_in, 1e-6f), 1.0f - 1e-6f);
                    // sigma(logit(a) + xs) = 1 / (1 + (1 - a) / a e^{-xs})
                    an = recip(fmaf((1.0f - a) * recip(a), __expf(-xs), 1.0f));
                    float disp = recip(de) + half_l * band * tanhf_(xd);
                    disp = fminf(fmaxf(disp, p.inv_far), p.inv_near);
                    dn = recip(disp);
                } else {
                    an = sigmoidf_(xs);
                    const float delta = ((float)(p.L - li) - 0.5f) / (float)p.L;
                    dn = recip(fmaf(delta + half_l * tanhf_(xd), band, p.inv_far));
                }
                p.depth_out[pe] = dn;
                p.alpha_out[pe] = an;
                if (do_comp) {
                    const float w = Tr[td] * an;
                    cr[td][0] = fmaf(w, sigmoidf_(X[td][2]), cr[td][0]);
                    cr[td][1] = fmaf(w, sigmoidf_(X[td][3]), cr[td][1]);
                    cr[td][2] = fmaf(w, sigmoidf_(head4), cr[td][2]);
                    Tr[td] *= (1.0f - an);
                }
            }
        }
    }

    if (do_comp) {
#pragma unroll
        for (int td = 0; td < ND; ++td) {
            const int s = (G > 1) ? 2 * td + g / 2 : 0;
            const int xe = x0w + 16 * s + n;
            if (owner && xe < p.W) {
                const size_t q = (size_t)y * p.W + xe;
                p.rgb[q * 3 + 0] = cr[td][0];
                p.rgb[q * 3 + 1] = cr[td][1];
                p.rgb[q * 3 + 2] = cr[td][2];
                if (p.acc != nullptr) p.acc[q] = 1.0f - Tr[td];
            }
        }
    }
}

// Standalone front-to-back composite: one thread per pixel.
__global__ void __launch_bounds__(256) k_composite(const CompParams p) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p.npix) return;
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    for (int l = 0; l < p.L; ++l) {
        const int64_t e = (int64_t)l * p.npix + q;
        const float a = p.alpha[e];
        const float w = T * a;
        c0 = fmaf(w, p.color[e * 3 + 0], c0);
        c1 = fmaf(w, p.color[e * 3 + 1], c1);
        c2 = fmaf(w, p.color[e * 3 + 2], c2);
        T *= (1.0f - a);
    }
    p.rgb[q * 3 + 0] = c0;
    p.rgb[q * 3 + 1] = c1;
    p.rgb[q * 3 + 2] = c2;
    if (p.acc != nullptr) p.acc[q] = 1.0f - T;
}

// ---------------------------------------------------------------------------
// Launchers (host side of this translation unit)
// ---------------------------------------------------------------------------
// One level (batch == nullptr), or a batch of requests whose parameters
// are at `reqs` in device memory.
struct UFLaunch {
    const UFParams *p;          // host copy (single) or nullptr
    const UFParams *reqs;       // device array (batch) or nullptr
    const UFBatch *batch;
};

template <int C, bool BF16, bool FOLD, bool F8, int HD>
static hipError_t launch_uf(const UFLaunch &l, hipStream_t s) {
    if (l.batch != nullptr) {
        // batches: the bfloat16 forms without e4m3 projections
        if constexpr (BF16 && !F8) {
            const UFArgs<true> a{l.reqs, *l.batch};
            hipLaunchKernelGGL((k_update_fuse<C, BF16, FOLD, F8, HD, kBatch>),
                               dim3(l.batch->total_tiles), dim3(256), 0, s, a);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (l.p->blend_logit != nullptr) {
        // blend-weight logits: one head, no e4m3 projections
        if constexpr (HD == C && !F8) {
            const UFArgs<false> a{*l.p};
            hipLaunchKernelGGL((k_update_fuse<C, BF16, FOLD, F8, HD, kBlend>), dim3(l.p->n_tiles),
                               dim3(256), 0, s, a);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        const UFArgs<false> a{*l.p};
        hipLaunchKernelGGL((k_update_fuse<C, BF16, FOLD, F8, HD, kPlain>), dim3(l.p->n_tiles),
                           dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

// prec: 0 float32, 1 bfloat16, 2 bfloat16 storage with e4m3 projections
template <int C, int HD>
static hipError_t launch_c(const UFLaunch &p, int prec, bool fold, hipStream_t s) {
    if constexpr (HD != C && C != 32) {          // several heads, standard form only
        if (fold) return hipErrorInvalidValue;
        if (prec == 2) return launch_uf<C, true, false, true, HD>(p, s);
        if (prec == 1) return launch_uf<C, true, false, false, HD>(p, s);
        return launch_uf<C, false, false, false, HD>(p, s);
    } else if constexpr (HD != C) {              // C = 32: also folded (no e4m3 form)
        if (prec == 2) return fold ? hipErrorInvalidValue : launch_uf<C, true, false, true, HD>(p, s);
        if (prec == 1) return fold ? launch_uf<C, true, true, false, HD>(p, s) : launch_uf<C, true, false, false, HD>(p, s);
        return fold ? launch_uf<C, false, true, false, HD>(p, s) : launch_uf<C, false, false, false, HD>(p, s);
    } else {
        if (prec == 2) return fold ? launch_uf<C, true, true, true, C>(p, s) : launch_uf<C, true, false, true, C>(p, s);
        if (prec == 1) return fold ? launch_uf<C, true, true, false, C>(p, s) : launch_uf<C, true, false, false, C>(p, s);
        return fold ? launch_uf<C, false, true, false, C>(p, s) : launch_uf<C, false, false, false, C>(p, s);
    }
}

// hd: the width of one head (C for a single head)
static hipError_t launch_any(const UFLaunch &p, int C, int hd, int prec, bool fold, hipStream_t s) {
    switch (C * 1000 + hd) {
        case 8008: return launch_c<8, 8>(p, prec, fold, s);
        case 16016: return launch_c<16, 16>(p, prec, fold, s);
        case 32032: return launch_c<32, 32>(p, prec, fold, s);
        case 32016: return launch_c<32, 16>(p, prec, fold, s);
        case 32008: return launch_c<32, 8>(p, prec, fold, s);
        case 64064: return launch_c<64, 64>(p, prec, fold, s);
        case 64032: return launch_c<64, 32>(p, prec, fold, s);
        case 64016: return launch_c<64, 16>(p, prec, fold, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_update_fuse(const UFParams &p, int C, int hd, int prec, bool fold, hipStream_t s) {
    const UFLaunch l{&p, nullptr, nullptr};
    return launch_any(l, C, hd, prec, fold, s);
}

hipError_t launch_update_fuse_batch(const UFParams *reqs, const UFBatch &b, int C, int hd,
                                    int prec, bool fold, hipStream_t s) {
    const UFLaunch l{nullptr, reqs, &b};
    return launch_any(l, C, hd, prec, fold, s);
}

// Folded weights of one-to-many attention, per head h of width d = hd
// (channels h d .. h d + d - 1 of the Q/K/V projections):
//   Wqk[h][a][b] = sum_e Wq[a][h d + e] Wk[b][h d + e] / sqrt(d)   (C x Cf)
//   Wvo[h][b][c] = sum_e Wv[b][h d + e] Wo[h d + e][c]             (Cf x C)
// One thread per output element.  The operands of eight terms are loaded
// before any of them is used, so a thread waits on memory once per eight
// terms instead of once per term; the sum is still taken in order of e.
__device__ __forceinline__ float fold_dot(const float *x, int xs, const float *y, int ys,
                                          int n) {
    float acc = 0.0f;
    int e = 0;
    for (; e + 8 <= n; e += 8) {
        float u[8], v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            u[i] = x[(e + i) * xs];
            v[i] = y[(e + i) * ys];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = fmaf(u[i], v[i], acc);
    }
    for (; e < n; ++e) acc = fmaf(x[e * xs], y[e * ys], acc);
    return acc;
}

__global__ void __launch_bounds__(256) k_fold_weights(const FoldParams f) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = f.C * f.Cf, nqk = f.heads * per, stride = f.heads * f.hd;
    if (idx < nqk) {
        const int h = idx / per, j = idx - h * per;
        const int a = j / f.Cf, b = j % f.Cf;
        f.Wqk[idx] = fold_dot(f.Wq + a * stride + h * f.hd, 1,
                              f.Wk + b * stride + h * f.hd, 1, f.hd) * f.scale;
    } else if (idx < 2 * nqk) {
        const int k = idx - nqk;
        const int h = k / per, j = k - h * per;
        const int b = j / f.C, c = j % f.C;
        f.Wvo[k] = fold_dot(f.Wv + b * stride + h * f.hd, 1,
                            f.Wo + h * f.hd * f.C + c, f.C, f.hd);
    }
}

hipError_t launch_fold_weights(const FoldParams &f, hipStream_t s) {
    const int n = 2 * f.heads * f.C * f.Cf;
    hipLaunchKernelGGL(k_fold_weights, dim3((n + 255) / 256), dim3(256), 0, s, f);
    return hipGetLastError();
}

// Device scratch of the allocation-free entry point (folded weights, e4m3
// scales): one copy per GPU, held until the process ends; calls on one GPU
// share it.  Host code must not pass `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory): scratch_address() looks up
// each device's copy once, with that device current, and kernels take that
// address.
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {
std::mutex g_scratch_mu;
float *g_scratch_addr[kMaxDevices] = {};
}  // namespace

// Address of `scratch` on `device` (made current for the lookup, then
// restored).  Looked up on the first call for that device, cached after.
hipError_t scratch_address(int device, float **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device] == nullptr) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = static_cast<float *>(ptr);
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

hipError_t launch_composite(const CompParams &p, hipStream_t s) {
    const int64_t blocks = (p.npix + 255) / 256;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
