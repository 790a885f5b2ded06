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
//   * lane l = 16 g + r.  In the MFMA A-operand layout lane l holds row r
//     (pixel x0 + r) and K-slots 8g..8g+7 of each 32-wide K chunk; in the
//     accumulator layout it holds column r and rows 4g..4g+3.
//   * the bilinear gather of view m writes straight into the A operand: lane
//     (r, g) reprojects pixel r into the view its slots belong to and loads
//     8 channels per tap (16 B in bfloat16, 32 B in float32).
//   * for C < 32 the 32-wide K chunk holds G = 32 / C independent 16-pixel
//     sub-tiles side by side and every weight is laid out block-diagonally,
//     so a wave covers 16 G pixels and all its lanes sample the same view at
//     a time (camera parameters and the feature base stay scalar);
//   * taps are clamped into the map with zero weight when outside, so the
//     gather has no divergent branches;
//   * softmax over views is an online update (running max / sum, one exp per
//     view) on the accumulator layout; logits reduce over the head dimension
//     across the columns of a lane row with DPP.
//   * weights arrive as float32 masters; each workgroup converts them once
//     into B-operand fragments in LDS; the K/V fragments are then held in
//     registers for the whole view loop.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uf_params.h"

namespace qk {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int C>
struct Shape {
    static constexpr int G = (C >= 32) ? 1 : 32 / C;    // 16-pixel sub-tiles packed along K
    static constexpr int KC = (C >= 32) ? C / 32 : 1;   // 32-wide K chunks of an A operand
    static constexpr int NT = (G * C) / 16;             // 16-wide N tiles of Q/K/V/O outputs
    static constexpr int ND = (G == 1) ? 1 : G / 2;     // N tiles of the decode output
    static constexpr int NTS = (G == 1) ? 1 : NT;       // softmax states per accumulator row
    static constexpr int PIX = 16 * G;                  // pixels per wave
    static constexpr int SLOTS = 32 * KC;               // K slots per A row
    static constexpr int PITCH = SLOTS + 4;             // LDS tile row pitch (floats)
    static constexpr int OFF_Q = 0;
    static constexpr int OFF_K = KC * NT;
    static constexpr int OFF_V = 2 * KC * NT;
    static constexpr int OFF_O = 3 * KC * NT;
    static constexpr int OFF_D = 4 * KC * NT;
    static constexpr int NFRAG = OFF_D + KC * ND;
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

__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }

// DPP lane permutations inside a 16-lane row.
template <int CTRL>
__device__ inline float dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}
// Sum over aligned groups of W lanes (W = 8 or 16) of a row: quad xor 1,
// quad xor 2, then half-row mirror (8) and row mirror (16).
template <int W>
__device__ inline float group_sum(float v) {
    v += dpp<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);    // row_half_mirror
    if constexpr (W == 16) v += dpp<0x140>(v);   // row_mirror
    return v;
}

__device__ inline float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }

__device__ inline void lds_read8(const float *src, float *f) {
    const float4 a = *reinterpret_cast<const float4 *>(src);
    const float4 b = *reinterpret_cast<const float4 *>(src + 4);
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
    f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
}

// Back-projection of one layer-pixel into view m followed by its bilinear
// sample (half-pixel centres, zero padding): p = A_m (u, v, 1) + b_m / d; a
// point with p_z <= 1e-6 (behind the view) samples zero.  This lane's share is
// channels ch0 + 32 kc + [0, 8) of the sample, in FP32.  Taps are clamped into
// the map and keep weight 0 when outside, so the loads are unconditional.
template <int C, bool BF16>
__device__ inline void gather_sample(const UFParams &p, int m, typename CoordT<BF16>::type uc,
                                     typename CoordT<BF16>::type vc,
                                     typename CoordT<BF16>::type invdc, bool a_ok, int ch0,
                                     float (&sv)[Shape<C>::KC][8]) {
    using Coord = typename CoordT<BF16>::type;
    using OP = Op<BF16>;
    using T = typename OP::T;
    constexpr int KC = Shape<C>::KC;
    const T *fm = reinterpret_cast<const T *>(p.feat[m]);
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
    const bool ok = a_ok && (pz > (Coord)1e-6) && (fabs(fxc) < (Coord)1e7) && (fabs(fyc) < (Coord)1e7);
    const Coord xf = floor(fxc), yf = floor(fyc);
    const float wx = (float)(fxc - xf), wy = (float)(fyc - yf);
    const int ix = ok ? (int)xf : -4, iy = ok ? (int)yf : -4;
    const bool vx0 = (unsigned)ix < (unsigned)fw, vx1 = (unsigned)(ix + 1) < (unsigned)fw;
    const bool vy0 = (unsigned)iy < (unsigned)fh, vy1 = (unsigned)(iy + 1) < (unsigned)fh;
    const float w00 = (vx0 && vy0) ? (1.0f - wx) * (1.0f - wy) : 0.0f;
    const float w10 = (vx1 && vy0) ? wx * (1.0f - wy) : 0.0f;
    const float w01 = (vx0 && vy1) ? (1.0f - wx) * wy : 0.0f;
    const float w11 = (vx1 && vy1) ? wx * wy : 0.0f;
    const int cx0 = min(max(ix, 0), fw - 1), cx1 = min(max(ix + 1, 0), fw - 1);
    const int cy0 = min(max(iy, 0), fh - 1), cy1 = min(max(iy + 1, 0), fh - 1);
    const int o00 = (cy0 * fw + cx0) * C + ch0, o10 = (cy0 * fw + cx1) * C + ch0;
    const int o01 = (cy1 * fw + cx0) * C + ch0, o11 = (cy1 * fw + cx1) * C + ch0;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        float t00[8], t10[8], t01[8], t11[8];
        OP::load8(fm + o00 + 32 * kc, t00);
        OP::load8(fm + o10 + 32 * kc, t10);
        OP::load8(fm + o01 + 32 * kc, t01);
        OP::load8(fm + o11 + 32 * kc, t11);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            sv[kc][i] = fmaf(w11, t11[i], fmaf(w01, t01[i], fmaf(w10, t10[i], w00 * t00[i])));
    }
}

// Sum of a value over the lanes that share one pixel's channels in the A
// layout: lanes 16 apart (C = 16) or 16 and 32 apart (C >= 32).  With both
// operands equal, the two outputs of a permlane swap hold the two rows of each
// pair broadcast, so their sum is the pair sum.
template <int C>
__device__ inline float pixel_lane_sum(float v) {
    if constexpr (C >= 16) {
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    if constexpr (C >= 32) {
        const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    return v;
}

// FOLD = false: standard cross-attention (per-sample key and value
// projections on MFMA).  FOLD = true: one-to-many attention -- the key
// projection folded into the query (q~ = N(F) W_q W_k^T / sqrt(d)) and the
// value projection into the output (W_v W_o); the per-view work is a dot
// product and a weighted sum on the samples themselves.
template <int C, bool BF16, bool FOLD>
__global__ void __launch_bounds__(256) k_update_fuse(const UFParams p) {
    using SH = Shape<C>;
    using OP = Op<BF16>;
    using AF = typename OP::A;
    using T = typename OP::T;
    using Coord = typename CoordT<BF16>::type;
    constexpr int G = SH::G, KC = SH::KC, NT = SH::NT, ND = SH::ND, NTS = SH::NTS;
    constexpr int PIX = SH::PIX, PITCH = SH::PITCH;
    constexpr int DW = (C >= 16) ? 16 : 8;    // columns of one head inside a 16-wide tile

    __shared__ AF sfrag[SH::NFRAG][64];
    __shared__ float sF[4][16 * PITCH];
    __shared__ float sO[4][16 * PITCH];
    __shared__ float sX[4][PIX * 8];

    const int tid = threadIdx.x;

    // ---- B-operand fragments from the float32 master weights, once per
    // workgroup.  Every projection is block-diagonal over the G sub-tiles.
    for (int e = tid; e < SH::NFRAG * 64; e += 256) {
        const int f = e >> 6, ln = e & 63;
        const int nn = ln & 15, gg = ln >> 4;
        const int kind = (f < SH::OFF_D) ? f / (KC * NT) : 4;
        const int fi = (f < SH::OFF_D) ? f % (KC * NT) : f - SH::OFF_D;
        const int ntile = (kind == 4) ? ND : NT;
        const int kc = fi / ntile, t = fi % ntile;
        const int ng = 16 * t + nn;               // output column of this lane
        if (FOLD && (kind == 1 || kind == 2)) continue;   // no per-sample projections
        const float *Wm = kind == 0 ? (FOLD ? p.Wqk : p.Wq) : kind == 1 ? p.Wk
                        : kind == 2 ? p.Wv : (FOLD ? p.Wvo : p.Wo);
        float vals[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int kap = 32 * kc + 8 * gg + i;   // K slot: sub-tile kap / C, channel kap % C
            float w = 0.0f;
            if (kind < 4) {
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
        sfrag[f][ln] = OP::make(vals);
    }
    __syncthreads();

    // ---- tile of this workgroup: XCD-aware remap of the dispatch order so
    // that each XCD (dispatched round-robin) walks one contiguous band of rows
    const int wave = tid >> 6, lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    int tile;
    {
        const int nt = p.n_tiles, i = blockIdx.x;
        const int xcd = i & 7, loc = i >> 3, q = nt >> 3, rem = nt & 7;
        tile = (xcd < rem) ? xcd * (q + 1) + loc : rem * (q + 1) + (xcd - rem) * q + loc;
    }
    const int chunk = tile % p.chunks;
    const int rest = tile / p.chunks;
    const int xb = rest % p.x_blocks;
    const int y = rest / p.x_blocks;
    const int x0w = xb * (4 * PIX) + wave * PIX;       // first pixel of this wave
    if (x0w >= p.W) return;                            // no later barrier: safe to leave
    const int l_begin = chunk * p.layers_per_chunk;
    const int l_end = min(p.L, l_begin + p.layers_per_chunk);

    // A-operand row of this lane: pixel xa, channels ch0 + 32 kc + [0, 8)
    const int sg = (G > 1) ? (8 * g) / C : 0;
    const int ch0 = (G > 1) ? (8 * g) % C : 8 * g;
    const int xa = x0w + 16 * sg + r;
    const bool a_ok = xa < p.W;
    // per-pixel epilogue lane: pixel x0w + lane
    const bool e_ok = (lane < PIX) && (x0w + lane < p.W);

    constexpr int KCB = FOLD ? 1 : KC, NTB = FOLD ? 1 : NT;
    AF Bk[KCB][NTB], Bv[KCB][NTB];
    if constexpr (!FOLD) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                Bk[kc][t] = sfrag[SH::OFF_K + kc * NT + t][lane];
                Bv[kc][t] = sfrag[SH::OFF_V + kc * NT + t][lane];
            }
    }

    float *tF = sF[wave];
    float *tO = sO[wave];
    float *tX = sX[wave];
    const T *Fin = reinterpret_cast<const T *>(p.F_in);
    T *Fout = reinterpret_cast<T *>(p.F_out);
    const bool do_comp = p.rgb != nullptr;
    const float scale = 1.0f / sqrtf((float)C);
    const Coord uc = (Coord)(a_ok ? xa : 0) + (Coord)0.5, vc = (Coord)y + (Coord)0.5;
    const float band = p.inv_near - p.inv_far;
    const float half_l = 0.5f / (float)p.L;

    float Tr = 1.0f, cr0 = 0.0f, cr1 = 0.0f, cr2 = 0.0f;

    for (int li = l_begin; li < l_end; ++li) {
        const size_t rowbase = ((size_t)li * p.H + y) * p.W;
        const size_t pa = rowbase + (a_ok ? xa : 0);
        const float d = a_ok ? p.depth_in[pa] : 1.0f;

        // ---- LDM feature tile, A layout; copy to LDS for the residual
        float fa[KC][8];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            if (a_ok) OP::load8(Fin + pa * C + ch0 + 32 * kc, fa[kc]);
            else
#pragma unroll
                for (int i = 0; i < 8; ++i) fa[kc][i] = 0.0f;
            float *dst = &tF[r * PITCH + 32 * kc + 8 * g];
            *reinterpret_cast<float4 *>(dst) = make_float4(fa[kc][0], fa[kc][1], fa[kc][2], fa[kc][3]);
            *reinterpret_cast<float4 *>(dst + 4) = make_float4(fa[kc][4], fa[kc][5], fa[kc][6], fa[kc][7]);
        }

        // ---- RMSNorm (unit gain, eps 1e-6) over the pixel's channels, query
        float ss = 0.0f;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int i = 0; i < 8; ++i) ss = fmaf(fa[kc][i], fa[kc][i], ss);
        if constexpr (C >= 16) ss += __shfl_xor(ss, 16);
        if constexpr (C >= 32) ss += __shfl_xor(ss, 32);
        const float inv = 1.0f / sqrtf(ss * (1.0f / (float)C) + 1e-6f);
        f32x4 Q[NT];
        {
            AF Axn[KC];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float t8[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) t8[i] = fa[kc][i] * inv;
                Axn[kc] = OP::make(t8);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                Q[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    Q[t] = OP::mma(Axn[kc], sfrag[SH::OFF_Q + kc * NT + t][lane], Q[t]);
            }
        }

        AF Ao[KC];
        const Coord invdc = recip((Coord)d);
        if constexpr (!FOLD) {
            // ---- standard cross-attention over the views: per-sample keys and
            // values on MFMA, online softmax (finite start so the update is
            // branch-free; one exp per state and view)
            float M[NTS][4], Z[NTS][4];
            f32x4 acc[NT];
#pragma unroll
            for (int s = 0; s < NTS; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) { M[s][i] = -1e30f; Z[s][i] = 0.0f; }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

            for (int m = 0; m < p.V; ++m) {
                AF As[KC];
                {
                    float sv[KC][8];
                    gather_sample<C, BF16>(p, m, uc, vc, invdc, a_ok, ch0, sv);
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) As[kc] = OP::make(sv[kc]);
                }
                // keys and logits
                float lg[NTS][4];
                {
                    f32x4 Kt[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        Kt[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int kc = 0; kc < KC; ++kc) Kt[t] = OP::mma(As[kc], Bk[kc][t], Kt[t]);
                    }
                    if constexpr (G == 1) {
                        float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int t = 0; t < NT; ++t)
#pragma unroll
                            for (int i = 0; i < 4; ++i) s4[i] = fmaf(Q[t][i], Kt[t][i], s4[i]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) lg[0][i] = group_sum<16>(s4[i]) * scale;
                    } else {
#pragma unroll
                        for (int t = 0; t < NT; ++t)
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                lg[t][i] = group_sum<DW>(Q[t][i] * Kt[t][i]) * scale;
                    }
                }
                // values and the online softmax update
                float sc[NTS][4], ev[NTS][4];
#pragma unroll
                for (int s = 0; s < NTS; ++s)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float a = lg[s][i];
                        const float diff = a - M[s][i];
                        const float x = __expf(-fabsf(diff));
                        const bool up = diff > 0.0f;
                        sc[s][i] = up ? x : 1.0f;
                        ev[s][i] = up ? 1.0f : x;
                        M[s][i] = up ? a : M[s][i];
                        Z[s][i] = fmaf(Z[s][i], sc[s][i], ev[s][i]);
                    }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    f32x4 Vt = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) Vt = OP::mma(As[kc], Bv[kc][t], Vt);
                    const int s = (G == 1) ? 0 : t;
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[t][i] = fmaf(acc[t][i], sc[s][i], ev[s][i] * Vt[i]);
                }
            }

            // o = acc / Z: accumulator layout -> LDS -> A layout
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int s = (G == 1) ? 0 : t;
#pragma unroll
                for (int i = 0; i < 4; ++i) tO[(4 * g + i) * PITCH + 16 * t + r] = acc[t][i] / Z[s][i];
            }
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float t8[8];
                lds_read8(&tO[r * PITCH + 32 * kc + 8 * g], t8);
                Ao[kc] = OP::make(t8);
            }
        } else {
            // ---- one-to-many attention: q~ (the query with W_k folded in) to
            // the A layout, then per view a dot product with the FP32 sample and
            // a weighted running sum of the samples themselves
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) tO[(4 * g + i) * PITCH + 16 * t + r] = Q[t][i];
            float qa[KC][8], ob[KC][8];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                lds_read8(&tO[r * PITCH + 32 * kc + 8 * g], qa[kc]);
#pragma unroll
                for (int i = 0; i < 8; ++i) ob[kc][i] = 0.0f;
            }
            float Mx = -1e30f, Zs = 0.0f;
            for (int m = 0; m < p.V; ++m) {
                float sv[KC][8];
                gather_sample<C, BF16>(p, m, uc, vc, invdc, a_ok, ch0, sv);
                float part = 0.0f;
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                    for (int i = 0; i < 8; ++i) part = fmaf(qa[kc][i], sv[kc][i], part);
                const float a = pixel_lane_sum<C>(part);
                const float diff = a - Mx;
                const float x = __expf(-fabsf(diff));
                const bool up = diff > 0.0f;
                const float sc = up ? x : 1.0f, ev = up ? 1.0f : x;
                Mx = up ? a : Mx;
                Zs = fmaf(Zs, sc, ev);
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                    for (int i = 0; i < 8; ++i) ob[kc][i] = fmaf(ob[kc][i], sc, ev * sv[kc][i]);
            }
            const float iz = 1.0f / Zs;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float t8[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) t8[i] = ob[kc][i] * iz;
                Ao[kc] = OP::make(t8);
            }
        }

        // ---- F' = F + o W_o (the accumulator starts from F)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            f32x4 Fo;
#pragma unroll
            for (int i = 0; i < 4; ++i) Fo[i] = tF[(4 * g + i) * PITCH + 16 * t + r];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) Fo = OP::mma(Ao[kc], sfrag[SH::OFF_O + kc * NT + t][lane], Fo);
#pragma unroll
            for (int i = 0; i < 4; ++i) tF[(4 * g + i) * PITCH + 16 * t + r] = Fo[i];
        }

        // ---- F' back to the A layout: store it and decode it
        f32x4 X[ND];
#pragma unroll
        for (int td = 0; td < ND; ++td) X[td] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            float t8[8];
            lds_read8(&tF[r * PITCH + 32 * kc + 8 * g], t8);
            if (Fout != nullptr && a_ok) OP::store8(Fout + pa * C + ch0 + 32 * kc, t8);
            const AF af = OP::make(t8);
#pragma unroll
            for (int td = 0; td < ND; ++td) X[td] = OP::mma(af, sfrag[SH::OFF_D + kc * ND + td][lane], X[td]);
        }
#pragma unroll
        for (int td = 0; td < ND; ++td) {
            const int ng = 16 * td + r;
            const int s = (G == 1) ? 0 : ng / 8;
            const int j = (G == 1) ? ng : ng % 8;
            if (j < 5)
#pragma unroll
                for (int i = 0; i < 4; ++i) tX[(16 * s + 4 * g + i) * 8 + j] = X[td][i];
        }

        // ---- decode depth / alpha / colour of pixel x0w + lane, composite
        if (e_ok) {
            const size_t pe = rowbase + x0w + lane;
            const float de = p.depth_in[pe];
            const float a_in = p.alpha_in[pe];
            const float *xv = &tX[lane * 8];
            const float xs = xv[0], xd = xv[1];
            float an, dn;
            if (p.mode == 0) {
                const float a = fminf(fmaxf(a_in, 1e-6f), 1.0f - 1e-6f);
                an = sigmoidf_(logf(a / (1.0f - a)) + xs);
                float disp = 1.0f / de + half_l * band * tanhf(xd);
                disp = fminf(fmaxf(disp, p.inv_far), p.inv_near);
                dn = 1.0f / disp;
            } else {
                an = sigmoidf_(xs);
                const float delta = ((float)(p.L - li) - 0.5f) / (float)p.L;
                dn = 1.0f / (fmaf(delta + half_l * tanhf(xd), band, p.inv_far));
            }
            p.depth_out[pe] = dn;
            p.alpha_out[pe] = an;
            if (do_comp) {
                const float w = Tr * an;
                cr0 = fmaf(w, sigmoidf_(xv[2]), cr0);
                cr1 = fmaf(w, sigmoidf_(xv[3]), cr1);
                cr2 = fmaf(w, sigmoidf_(xv[4]), cr2);
                Tr *= (1.0f - an);
            }
        }
    }

    if (do_comp && e_ok) {
        const size_t q = (size_t)y * p.W + x0w + lane;
        p.rgb[q * 3 + 0] = cr0;
        p.rgb[q * 3 + 1] = cr1;
        p.rgb[q * 3 + 2] = cr2;
        if (p.acc != nullptr) p.acc[q] = 1.0f - Tr;
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
template <int C, bool BF16, bool FOLD>
static hipError_t launch_uf(const UFParams &p, hipStream_t s) {
    hipLaunchKernelGGL((k_update_fuse<C, BF16, FOLD>), dim3(p.n_tiles), dim3(256), 0, s, p);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_c(const UFParams &p, bool bf16, bool fold, hipStream_t s) {
    if (bf16) return fold ? launch_uf<C, true, true>(p, s) : launch_uf<C, true, false>(p, s);
    return fold ? launch_uf<C, false, true>(p, s) : launch_uf<C, false, false>(p, s);
}

hipError_t launch_update_fuse(const UFParams &p, int C, bool bf16, bool fold, hipStream_t s) {
    switch (C) {
        case 8: return launch_c<8>(p, bf16, fold, s);
        case 16: return launch_c<16>(p, bf16, fold, s);
        case 32: return launch_c<32>(p, bf16, fold, s);
        case 64: return launch_c<64>(p, bf16, fold, s);
        default: return hipErrorInvalidValue;
    }
}

// Folded weights of one-to-many attention (one head of width d = hd):
//   Wqk[a][b] = sum_e Wq[a][e] Wk[b][e] / sqrt(d)   (C x Cf)
//   Wvo[b][c] = sum_e Wv[b][e] Wo[e][c]             (Cf x C)
// One thread per output element.
__global__ void __launch_bounds__(256) k_fold_weights(const FoldParams f) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nqk = f.C * f.Cf;
    if (idx < nqk) {
        const int a = idx / f.Cf, b = idx % f.Cf;
        float acc = 0.0f;
        for (int e = 0; e < f.hd; ++e) acc = fmaf(f.Wq[a * f.hd + e], f.Wk[b * f.hd + e], acc);
        f.Wqk[idx] = acc * f.scale;
    } else if (idx < 2 * nqk) {
        const int j = idx - nqk;
        const int b = j / f.C, c = j % f.C;
        float acc = 0.0f;
        for (int e = 0; e < f.hd; ++e) acc = fmaf(f.Wv[b * f.hd + e], f.Wo[e * f.C + c], acc);
        f.Wvo[j] = acc;
    }
}

hipError_t launch_fold_weights(const FoldParams &f, hipStream_t s) {
    const int n = 2 * f.C * f.Cf;
    hipLaunchKernelGGL(k_fold_weights, dim3((n + 255) / 256), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_composite(const CompParams &p, hipStream_t s) {
    const int64_t blocks = (p.npix + 255) / 256;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
