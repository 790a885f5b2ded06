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
//   * a workgroup is 4 waves; it covers 64 consecutive pixels of one LDM row
//     and a chunk of layers; each wave owns 16 pixels and walks the layers
//     of its chunk front to back (so the composite accumulates in registers);
//   * lane l = 16 g + r.  In the MFMA A-operand layout lane l holds row r
//     (pixel x0 + r) and K-slots 8g..8g+7 of each 32-wide K chunk; in the
//     accumulator layout it holds column r and rows 4g..4g+3.
//   * the bilinear gather of view m writes straight into the A operand: lane
//     (r, g) reprojects pixel r into the view its slots belong to and loads
//     8 channels per tap (16 B in bfloat16, 32 B in float32).
//   * for C < 32 the 32-wide K chunk holds G = 32 / C views side by side and
//     the K/V weights are laid out block-diagonally, so one MFMA projects G
//     views; the view blocks are merged like split softmax partials at the
//     end.
//   * softmax over views is an online update (running max / sum) on the
//     accumulator layout; logits reduce over the head dimension across the
//     16 columns of a lane row.
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
    static constexpr int KC = (C >= 32) ? C / 32 : 1;    // 32-wide K chunks of an A operand
    static constexpr int G = (C >= 32) ? 1 : 32 / C;     // views packed side by side per chunk
    static constexpr int NT = (G * C) / 16;              // 16-wide N tiles of the K/V/Q output
    static constexpr int NTO = (C >= 16) ? C / 16 : 1;   // N tiles of the output projection
    static constexpr int NTS = (G == 1) ? 1 : NT;        // independent softmax states per row
    static constexpr int PITCH = C + 4;                  // LDS tile row pitch (floats)
    static constexpr int OFF_Q = 0;
    static constexpr int OFF_K = OFF_Q + KC * NT;
    static constexpr int OFF_V = OFF_K + KC * NT;
    static constexpr int OFF_O = OFF_V + KC * NT;
    static constexpr int OFF_D = OFF_O + KC * NTO;
    static constexpr int NFRAG = OFF_D + KC;
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

// Sum over aligned groups of W lanes (W = 8 or 16) inside a 16-lane row.
template <int W>
__device__ inline float group_sum(float v) {
#pragma unroll
    for (int o = 1; o < W; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }

// Merge two partial softmax states (running max, normaliser, weighted sum).
__device__ inline void merge_state(float &M, float &Z, float &A, float M2, float Z2, float A2) {
    const float ninf = -__builtin_inff();
    const float Mn = fmaxf(M, M2);
    const float s1 = (M == ninf) ? 0.0f : __expf(M - Mn);
    const float s2 = (M2 == ninf) ? 0.0f : __expf(M2 - Mn);
    A = A * s1 + A2 * s2;
    Z = Z * s1 + Z2 * s2;
    M = Mn;
}

template <int C, bool BF16>
__global__ void __launch_bounds__(256) k_update_fuse(const UFParams p) {
    using SH = Shape<C>;
    using OP = Op<BF16>;
    using AF = typename OP::A;
    using T = typename OP::T;
    constexpr int KC = SH::KC, G = SH::G, NT = SH::NT, NTO = SH::NTO, NTS = SH::NTS;
    constexpr int PITCH = SH::PITCH;
    const float ninf = -__builtin_inff();

    __shared__ AF sfrag[SH::NFRAG][64];
    __shared__ float sF[4][16 * PITCH];
    __shared__ float sO[4][16 * PITCH];
    __shared__ float sX[4][16 * 8];

    const int tid = threadIdx.x;

    // ---- B-operand fragments from the float32 master weights (once per workgroup)
    for (int e = tid; e < SH::NFRAG * 64; e += 256) {
        const int f = e >> 6, ln = e & 63;
        const int nn = ln & 15, gg = ln >> 4;
        int kind, kc, t;
        if (f < SH::OFF_K) { kind = 0; kc = (f - SH::OFF_Q) / NT; t = (f - SH::OFF_Q) % NT; }
        else if (f < SH::OFF_V) { kind = 1; kc = (f - SH::OFF_K) / NT; t = (f - SH::OFF_K) % NT; }
        else if (f < SH::OFF_O) { kind = 2; kc = (f - SH::OFF_V) / NT; t = (f - SH::OFF_V) % NT; }
        else if (f < SH::OFF_D) { kind = 3; kc = (f - SH::OFF_O) / NTO; t = (f - SH::OFF_O) % NTO; }
        else { kind = 4; kc = f - SH::OFF_D; t = 0; }
        const int ng = 16 * t + nn;       // output column of this lane
        float vals[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int kap = 32 * kc + 8 * gg + i;   // K slot
            float w = 0.0f;
            if (kind == 0) {                        // q, replicated in every view block
                if (kap < C) w = p.Wq[kap * C + (ng % C)];
            } else if (kind == 1 || kind == 2) {    // k / v, block-diagonal over packed views
                const float *Wm = (kind == 1) ? p.Wk : p.Wv;
                if (kap / C == ng / C) w = Wm[(kap % C) * C + (ng % C)];
            } else if (kind == 3) {                 // output projection
                if (kap < C && ng < C) w = p.Wo[kap * C + ng];
            } else {                                // decode heads: sigma, depth, rgb
                if (kap < C) {
                    if (nn == 0) w = p.w_sigma[kap];
                    else if (nn == 1) w = p.w_depth[kap];
                    else if (nn < 5) w = p.W_color[kap * 3 + (nn - 2)];
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
    const int x0 = xb * 64 + wave * 16;
    if (x0 >= p.W) return;                 // no later barrier: safe to leave
    const int x = x0 + r;
    const bool px_ok = x < p.W;
    const int l_begin = chunk * p.layers_per_chunk;
    const int l_end = min(p.L, l_begin + p.layers_per_chunk);

    AF Bk[KC][NT], Bv[KC][NT];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            Bk[kc][t] = sfrag[SH::OFF_K + kc * NT + t][lane];
            Bv[kc][t] = sfrag[SH::OFF_V + kc * NT + t][lane];
        }

    float *tF = sF[wave];
    float *tO = sO[wave];
    float *tX = sX[wave];
    const T *Fin = reinterpret_cast<const T *>(p.F_in);
    T *Fout = reinterpret_cast<T *>(p.F_out);
    const bool do_comp = p.rgb != nullptr;
    const float scale = 1.0f / sqrtf((float)C);
    const float u = (float)x + 0.5f, v = (float)y + 0.5f;
    // channel offset of this lane's K slots inside its view's vector
    const int ch0 = (G > 1) ? (8 * g) % C : 8 * g;
    const int jv = (G > 1) ? (8 * g) / C : 0;          // view inside the packed group

    float Tr = 1.0f, cr0 = 0.0f, cr1 = 0.0f, cr2 = 0.0f;

    for (int li = l_begin; li < l_end; ++li) {
        const size_t pix = ((size_t)li * p.H + y) * p.W + (px_ok ? x : 0);
        const float d = px_ok ? p.depth_in[pix] : 1.0f;

        // ---- LDM feature tile, A layout; copy to LDS for the residual
        float fa[KC][8];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int k0 = 32 * kc + 8 * g;
            if (k0 < C) {
                if (px_ok) OP::load8(Fin + pix * C + k0, fa[kc]);
                else
#pragma unroll
                    for (int i = 0; i < 8; ++i) fa[kc][i] = 0.0f;
                *reinterpret_cast<float4 *>(&tF[r * PITCH + k0]) =
                    make_float4(fa[kc][0], fa[kc][1], fa[kc][2], fa[kc][3]);
                *reinterpret_cast<float4 *>(&tF[r * PITCH + k0 + 4]) =
                    make_float4(fa[kc][4], fa[kc][5], fa[kc][6], fa[kc][7]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) fa[kc][i] = 0.0f;
            }
        }

        // ---- RMSNorm (unit gain, eps 1e-6) and the query projection
        float ss = 0.0f;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int i = 0; i < 8; ++i) ss = fmaf(fa[kc][i], fa[kc][i], ss);
        ss += __shfl_xor(ss, 16);
        ss += __shfl_xor(ss, 32);
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

        // ---- across-view attention with an online softmax
        float M[NTS][4], Z[NTS][4];
        f32x4 acc[NT];
#pragma unroll
        for (int s = 0; s < NTS; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) { M[s][i] = ninf; Z[s][i] = 0.0f; }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

        const float invd = 1.0f / d;
        for (int m0 = 0; m0 < p.V; m0 += G) {
            // view parameters of this lane's slots
            const T *fm;
            int fh, fw;
            float cm[12];
            if constexpr (G == 1) {
                fm = reinterpret_cast<const T *>(p.feat[m0]);
                fh = p.fH[m0];
                fw = p.fW[m0];
#pragma unroll
                for (int k = 0; k < 12; ++k) cm[k] = p.cam[m0][k];
            } else {
                const int mm0 = min(m0, p.V - 1);
                fm = reinterpret_cast<const T *>(p.feat[mm0]);
                fh = p.fH[mm0];
                fw = p.fW[mm0];
#pragma unroll
                for (int k = 0; k < 12; ++k) cm[k] = p.cam[mm0][k];
#pragma unroll
                for (int jj = 1; jj < G; ++jj) {
                    const int mm = min(m0 + jj, p.V - 1);
                    const bool mine = (jv == jj);
                    fm = mine ? reinterpret_cast<const T *>(p.feat[mm]) : fm;
                    fh = mine ? p.fH[mm] : fh;
                    fw = mine ? p.fW[mm] : fw;
#pragma unroll
                    for (int k = 0; k < 12; ++k) cm[k] = mine ? p.cam[mm][k] : cm[k];
                }
            }
            const bool vok = px_ok && (m0 + jv < p.V);

            // reproject: p = A (u, v, 1) + b / d
            const float pz = fmaf(cm[6], u, fmaf(cm[7], v, fmaf(cm[11], invd, cm[8])));
            const float qx = fmaf(cm[0], u, fmaf(cm[1], v, fmaf(cm[9], invd, cm[2])));
            const float qy = fmaf(cm[3], u, fmaf(cm[4], v, fmaf(cm[10], invd, cm[5])));
            bool ok = vok && (pz > 1e-6f);
            const float um = qx / pz, vm = qy / pz;
            const float fxc = um - 0.5f, fyc = vm - 0.5f;
            ok = ok && fabsf(fxc) < 1e7f && fabsf(fyc) < 1e7f;
            const float xf = floorf(fxc), yf = floorf(fyc);
            const float wx = fxc - xf, wy = fyc - yf;
            const int ix = ok ? (int)xf : -2, iy = ok ? (int)yf : -2;
            const bool x0v = (ix >= 0) && (ix < fw), x1v = (ix >= -1) && (ix + 1 < fw);
            const bool y0v = (iy >= 0) && (iy < fh), y1v = (iy >= -1) && (iy + 1 < fh);
            const float w00 = (1.0f - wx) * (1.0f - wy), w10 = wx * (1.0f - wy);
            const float w01 = (1.0f - wx) * wy, w11 = wx * wy;

            // bilinear gather straight into the A operand
            AF As[KC];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float sv[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) sv[i] = 0.0f;
                const long long off = ((long long)iy * fw + ix) * C + ch0 + 32 * kc;
                const T *base = fm + off;
                float t8[8];
                if (y0v && x0v) {
                    OP::load8(base, t8);
#pragma unroll
                    for (int i = 0; i < 8; ++i) sv[i] = fmaf(w00, t8[i], sv[i]);
                }
                if (y0v && x1v) {
                    OP::load8(base + C, t8);
#pragma unroll
                    for (int i = 0; i < 8; ++i) sv[i] = fmaf(w10, t8[i], sv[i]);
                }
                if (y1v && x0v) {
                    OP::load8(base + (long long)fw * C, t8);
#pragma unroll
                    for (int i = 0; i < 8; ++i) sv[i] = fmaf(w01, t8[i], sv[i]);
                }
                if (y1v && x1v) {
                    OP::load8(base + (long long)fw * C + C, t8);
#pragma unroll
                    for (int i = 0; i < 8; ++i) sv[i] = fmaf(w11, t8[i], sv[i]);
                }
                As[kc] = OP::make(sv);
            }

            // keys and logits
            float lg[NT][4];
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
                    for (int i = 0; i < 4; ++i) {
                        const float a = group_sum<16>(s4[i]) * scale;
#pragma unroll
                        for (int t = 0; t < NT; ++t) lg[t][i] = a;
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int jb = (16 * t + r) / C;     // view block of this column
                        const bool real = (m0 + jb) < p.V;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float a = Q[t][i] * Kt[t][i];
                            a = (C == 8) ? group_sum<8>(a) : group_sum<16>(a);
                            lg[t][i] = real ? a * scale : ninf;
                        }
                    }
                }
            }
            // values and the online softmax update
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                f32x4 Vt = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) Vt = OP::mma(As[kc], Bv[kc][t], Vt);
                const int s = (G == 1) ? 0 : t;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float a = lg[t][i];
                    const float Mo = M[s][i];
                    const float Mn = fmaxf(Mo, a);
                    const float sc = (Mo == ninf) ? 0.0f : __expf(Mo - Mn);
                    const float e = (a == ninf) ? 0.0f : __expf(a - Mn);
                    acc[t][i] = fmaf(acc[t][i], sc, e * Vt[i]);
                    if (G != 1 || t == NT - 1) {
                        Z[s][i] = fmaf(Z[s][i], sc, e);
                        M[s][i] = Mn;
                    }
                }
            }
        }

        // ---- attention output o (accumulator layout) -> LDS -> A layout
        if constexpr (G == 1) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) tO[(4 * g + i) * PITCH + 16 * t + r] = acc[t][i] / Z[0][i];
        } else {
            float Mm[4], Zm[4], Am[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { Mm[i] = M[0][i]; Zm[i] = Z[0][i]; Am[i] = acc[0][i]; }
#pragma unroll
            for (int t = 1; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) merge_state(Mm[i], Zm[i], Am[i], M[t][i], Z[t][i], acc[t][i]);
            if constexpr (C == 8) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float M2 = __shfl_xor(Mm[i], 8), Z2 = __shfl_xor(Zm[i], 8);
                    const float A2 = __shfl_xor(Am[i], 8);
                    merge_state(Mm[i], Zm[i], Am[i], M2, Z2, A2);
                }
            }
            if (r < C)
#pragma unroll
                for (int i = 0; i < 4; ++i) tO[(4 * g + i) * PITCH + r] = Am[i] / Zm[i];
        }
        AF Ao[KC];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int k0 = 32 * kc + 8 * g;
            float t8[8];
            if (k0 < C) {
                const float4 a = *reinterpret_cast<const float4 *>(&tO[r * PITCH + k0]);
                const float4 b = *reinterpret_cast<const float4 *>(&tO[r * PITCH + k0 + 4]);
                t8[0] = a.x; t8[1] = a.y; t8[2] = a.z; t8[3] = a.w;
                t8[4] = b.x; t8[5] = b.y; t8[6] = b.z; t8[7] = b.w;
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) t8[i] = 0.0f;
            }
            Ao[kc] = OP::make(t8);
        }

        // ---- F' = F + o W_o (accumulator starts from F)
#pragma unroll
        for (int to = 0; to < NTO; ++to) {
            f32x4 Fo;
            const int c = 16 * to + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) Fo[i] = (c < C) ? tF[(4 * g + i) * PITCH + c] : 0.0f;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) Fo = OP::mma(Ao[kc], sfrag[SH::OFF_O + kc * NTO + to][lane], Fo);
            if (c < C)
#pragma unroll
                for (int i = 0; i < 4; ++i) tF[(4 * g + i) * PITCH + c] = Fo[i];
        }

        // ---- F' back to the A layout: store it and decode it
        f32x4 X = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int k0 = 32 * kc + 8 * g;
            float t8[8];
            if (k0 < C) {
                const float4 a = *reinterpret_cast<const float4 *>(&tF[r * PITCH + k0]);
                const float4 b = *reinterpret_cast<const float4 *>(&tF[r * PITCH + k0 + 4]);
                t8[0] = a.x; t8[1] = a.y; t8[2] = a.z; t8[3] = a.w;
                t8[4] = b.x; t8[5] = b.y; t8[6] = b.z; t8[7] = b.w;
                if (Fout != nullptr && px_ok) OP::store8(Fout + pix * C + k0, t8);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) t8[i] = 0.0f;
            }
            X = OP::mma(OP::make(t8), sfrag[SH::OFF_D + kc][lane], X);
        }
        if (r < 5)
#pragma unroll
            for (int i = 0; i < 4; ++i) tX[(4 * g + i) * 8 + r] = X[i];

        // ---- decode depth / alpha / colour of pixel r, composite front to back
        if (px_ok) {
            const float xs = tX[r * 8 + 0], xd = tX[r * 8 + 1];
            const float xc0 = tX[r * 8 + 2], xc1 = tX[r * 8 + 3], xc2 = tX[r * 8 + 4];
            const float a_in = p.alpha_in[pix];
            const float band = p.inv_near - p.inv_far;
            const float half_l = 0.5f / (float)p.L;
            float an, dn;
            if (p.mode == 0) {
                const float a = fminf(fmaxf(a_in, 1e-6f), 1.0f - 1e-6f);
                an = sigmoidf_(logf(a / (1.0f - a)) + xs);
                float disp = invd + half_l * band * tanhf(xd);
                disp = fminf(fmaxf(disp, p.inv_far), p.inv_near);
                dn = 1.0f / disp;
            } else {
                an = sigmoidf_(xs);
                const float delta = ((float)(p.L - li) - 0.5f) / (float)p.L;
                dn = 1.0f / (fmaf(delta + half_l * tanhf(xd), band, p.inv_far));
            }
            if (g == 0) {
                p.depth_out[pix] = dn;
                p.alpha_out[pix] = an;
            }
            if (do_comp) {
                const float w = Tr * an;
                cr0 = fmaf(w, sigmoidf_(xc0), cr0);
                cr1 = fmaf(w, sigmoidf_(xc1), cr1);
                cr2 = fmaf(w, sigmoidf_(xc2), cr2);
                Tr *= (1.0f - an);
            }
        }
    }

    if (do_comp && px_ok && g == 0) {
        const size_t q = (size_t)y * p.W + x;
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
template <int C, bool BF16>
static hipError_t launch_uf(const UFParams &p, hipStream_t s) {
    hipLaunchKernelGGL((k_update_fuse<C, BF16>), dim3(p.n_tiles), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_update_fuse(const UFParams &p, int C, bool bf16, hipStream_t s) {
    switch (C) {
        case 8: return bf16 ? launch_uf<8, true>(p, s) : launch_uf<8, false>(p, s);
        case 16: return bf16 ? launch_uf<16, true>(p, s) : launch_uf<16, false>(p, s);
        case 32: return bf16 ? launch_uf<32, true>(p, s) : launch_uf<32, false>(p, s);
        case 64: return bf16 ? launch_uf<64, true>(p, s) : launch_uf<64, false>(p, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_composite(const CompParams &p, hipStream_t s) {
    const int64_t blocks = (p.npix + 255) / 256;
    hipLaunchKernelGGL(k_composite, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace qk
