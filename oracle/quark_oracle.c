/*
 * quark_oracle.c -- plain FP64 CPU reference ("oracle") for one Update & Fuse
 * step of a layered depth map (LDM) and its front-to-back composite, after
 * Quark: Real-time, High-resolution, and General Neural View Synthesis
 * (Flynn et al., ACM TOG 43(6), 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU library: every formula below is written out here from the paper.
 *
 * Style: slow, plain loops in double precision, one function per step of the
 * method, each citing the passage it follows.  No blocking, fusion or
 * reordering beyond what the definitions state.  OpenMP only splits the
 * independent layer-pixels across threads.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *   - pixel (x, y) has its centre at (x + 0.5, y + 0.5) in the continuous
 *     coordinates that K maps rays to; rescaling a camera to another grid is
 *     K' = diag(W'/W, H'/H, 1) K;
 *   - "depth" is z-depth along the novel camera's optical axis;
 *   - E is the world-to-camera transform, OpenCV axes;
 *   - bilinear sampling uses zero padding outside the feature map, and a
 *     sample whose point lies behind view m (Z_m <= 1e-6 d) is the zero
 *     vector; such samples stay in the softmax (no mask);
 *   - attention scale 1/sqrt(d_h) (per-head width), RMSNorm with unit gain
 *     and eps = 1e-6 inside the square root, applied to the query input only;
 *     no biases anywhere;
 *   - layer index 0 is the nearest layer; the paper's layer index l (whose
 *     l = 1 is the farthest band) is L - index;
 *   - colour of a layer is sigmoid(F' W_c); depth and alpha are updated
 *     residually by default (mode 0) or decoded absolutely as in the paper's
 *     depth activation (mode 1).
 *
 * Parity status: every function has a pin in the CPU tests (closed forms,
 * library routines, invariants, brute force).
 */

#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra                                               */
/* ------------------------------------------------------------------------ */

/* 4x4 inverse by Gauss-Jordan elimination with partial pivoting. */
static int inv4(const double *A, double *Ainv)
{
    double M[4][8];
    for (int r = 0; r < 4; ++r) {
        for (int c = 0; c < 4; ++c) {
            M[r][c] = A[4 * r + c];
            M[r][4 + c] = (r == c) ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (fabs(M[piv][col]) < 1e-300) return -1;
        if (piv != col)
            for (int c = 0; c < 8; ++c) {
                double t = M[col][c]; M[col][c] = M[piv][c]; M[piv][c] = t;
            }
        double p = M[col][col];
        for (int c = 0; c < 8; ++c) M[col][c] /= p;
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            double f = M[r][col];
            for (int c = 0; c < 8; ++c) M[r][c] -= f * M[col][c];
        }
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) Ainv[4 * r + c] = M[r][4 + c];
    return 0;
}

static void mul4(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[4 * r + k] * B[4 * k + c];
            C[4 * r + c] = s;
        }
}

/* Embed a 3x3 intrinsic matrix in a 4x4 homogeneous one. */
static void k_to_4x4(const double *K, double *K4)
{
    memset(K4, 0, 16 * sizeof(double));
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) K4[4 * r + c] = K[3 * r + c];
    K4[15] = 1.0;
}

/* Rescale intrinsics from a (w0, h0) grid to a (w1, h1) grid with half-pixel
 * centres: continuous pixel coordinates scale by w1/w0 and h1/h0. */
OR_EXPORT void or_scale_intrinsics(const double *K, int w0, int h0, int w1, int h1,
                                   double *Ks)
{
    double sx = (double)w1 / (double)w0, sy = (double)h1 / (double)h0;
    for (int c = 0; c < 3; ++c) {
        Ks[c] = sx * K[c];
        Ks[3 + c] = sy * K[3 + c];
        Ks[6 + c] = K[6 + c];
    }
}

/* ------------------------------------------------------------------------ */
/* Back-projection operator P^T_theta, first half: reprojection             */
/* (Sec. 3.1, the operator that carries input images onto the depth layers;  */
/*  Sec. 3.2.2, back-projection of update features through decoded depth).  */
/* ------------------------------------------------------------------------ */

/* Full 4x4 chain from the novel camera's pixel space (scaled by depth) to
 * view m's pixel space:  T = K4_m * E_m * inv(E_n) * inv(K4_n). */
OR_EXPORT int or_reprojection_matrix(const double *Kn, const double *En,
                                     const double *Km, const double *Em, double *T)
{
    double Kn4[16], Km4[16], Kn4i[16], Eni[16], A[16], B[16];
    k_to_4x4(Kn, Kn4);
    k_to_4x4(Km, Km4);
    if (inv4(Kn4, Kn4i) != 0) return -1;
    if (inv4(En, Eni) != 0) return -1;
    mul4(Eni, Kn4i, A);     /* novel pixel*depth -> world */
    mul4(Em, A, B);         /* -> camera m                */
    mul4(Km4, B, T);        /* -> view m pixel*depth      */
    return 0;
}

/* Reproject the centre of novel-grid pixel coordinate (u, v) lifted to
 * z-depth d into view m.  Returns 1 and writes (u_m, v_m) if the point lies
 * in front of view m (Z_m > 1e-6 d), else returns 0. */
OR_EXPORT int or_reproject_T(const double *T, double u, double v, double d, double *uv_out)
{
    double X[4] = {u * d, v * d, d, 1.0};
    double P[4];
    for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        for (int c = 0; c < 4; ++c) s += T[4 * r + c] * X[c];
        P[r] = s;
    }
    /* P = (Km X_m, 1) with X_m the point in camera m: P[2] = Z_m. */
    if (!(P[2] > 1e-6 * d)) return 0;
    uv_out[0] = P[0] / P[2];
    uv_out[1] = P[1] / P[2];
    return 1;
}

OR_EXPORT int or_reproject(const double *Kn, const double *En, const double *Km,
                           const double *Em, double u, double v, double d, double *uv_out)
{
    double T[16];
    if (or_reprojection_matrix(Kn, En, Km, Em, T) != 0) return -1;
    return or_reproject_T(T, u, v, d, uv_out);
}

/* ------------------------------------------------------------------------ */
/* Back-projection operator, second half: bilinear sampling of a feature map */
/* I[Hf][Wf][C] at continuous coordinate (u, v), zero padding.              */
/* ------------------------------------------------------------------------ */

OR_EXPORT void or_bilinear(const double *I, int Hf, int Wf, int C, double u, double v,
                           double *s)
{
    double x = u - 0.5, y = v - 0.5;        /* pixel centres at integer + 0.5 */
    double xf = floor(x), yf = floor(y);
    double fx = x - xf, fy = y - yf;
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    if (!(fabs(x) < 1e9 && fabs(y) < 1e9)) return;   /* far outside: all taps padded */
    long x0 = (long)xf, y0 = (long)yf;
    const long tx[4] = {x0, x0 + 1, x0, x0 + 1};
    const long ty[4] = {y0, y0, y0 + 1, y0 + 1};
    const double w[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
    for (int t = 0; t < 4; ++t) {
        if (tx[t] < 0 || tx[t] >= Wf || ty[t] < 0 || ty[t] >= Hf) continue;
        const double *p = I + ((size_t)ty[t] * Wf + (size_t)tx[t]) * C;
        for (int c = 0; c < C; ++c) s[c] += w[t] * p[c];
    }
}

/* ------------------------------------------------------------------------ */
/* Fusion-block attention (Sec. 3.3): V' = V + MultiHead(N(V), Delta), with  */
/* MultiHead(Q, K, Val) = concat(head_1..head_h) W^O and                     */
/* head_i = Attention(Q W_i^q, K W_i^k, Val W_i^val),                        */
/* Attention(Q, K, Val) = softmax(Q K^T / sqrt(d_h)) Val.                    */
/* Here the query is one layer-pixel's feature F (C values) and the keys and */
/* values come from its V samples S (V x Cf).  Weights row-major [in][out].  */
/* ------------------------------------------------------------------------ */

/* RMSNorm with unit gain: x / sqrt(mean(x^2) + 1e-6). */
OR_EXPORT void or_rmsnorm(const double *x, int C, double *y)
{
    double ss = 0.0;
    for (int c = 0; c < C; ++c) ss += x[c] * x[c];
    double r = sqrt(ss / C + 1e-6);
    for (int c = 0; c < C; ++c) y[c] = x[c] / r;
}

/* y[n_out] = x[n_in] @ W[n_in][n_out] */
static void vecmat(const double *x, const double *W, int n_in, int n_out, double *y)
{
    for (int j = 0; j < n_out; ++j) {
        double s = 0.0;
        for (int i = 0; i < n_in; ++i) s += x[i] * W[(size_t)i * n_out + j];
        y[j] = s;
    }
}

/* Standard cross-attention from one query to V samples; writes
 * F_out = F + concat_i(o_i) W_o, and (optionally) the softmax weights
 * p[h][V] used by each head. */
OR_EXPORT void or_attention(const double *F, int C, const double *S, int V, int Cf,
                            int heads, int dh, const double *Wq, const double *Wk,
                            const double *Wv, const double *Wo, double *F_out, double *p_out)
{
    int hd = heads * dh;
    double *xn = malloc(sizeof(double) * C);
    double *q = malloc(sizeof(double) * hd);
    double *k = malloc(sizeof(double) * (size_t)V * hd);
    double *v = malloc(sizeof(double) * (size_t)V * hd);
    double *o = malloc(sizeof(double) * hd);
    double *a = malloc(sizeof(double) * V);

    or_rmsnorm(F, C, xn);
    vecmat(xn, Wq, C, hd, q);
    for (int m = 0; m < V; ++m) {
        vecmat(S + (size_t)m * Cf, Wk, Cf, hd, k + (size_t)m * hd);
        vecmat(S + (size_t)m * Cf, Wv, Cf, hd, v + (size_t)m * hd);
    }
    double scale = 1.0 / sqrt((double)dh);
    for (int h = 0; h < heads; ++h) {
        double amax = -INFINITY;
        for (int m = 0; m < V; ++m) {
            double s = 0.0;
            for (int j = 0; j < dh; ++j) s += q[h * dh + j] * k[(size_t)m * hd + h * dh + j];
            a[m] = s * scale;
            if (a[m] > amax) amax = a[m];
        }
        double z = 0.0;
        for (int m = 0; m < V; ++m) { a[m] = exp(a[m] - amax); z += a[m]; }
        for (int m = 0; m < V; ++m) a[m] /= z;
        if (p_out) for (int m = 0; m < V; ++m) p_out[h * V + m] = a[m];
        for (int j = 0; j < dh; ++j) {
            double s = 0.0;
            for (int m = 0; m < V; ++m) s += a[m] * v[(size_t)m * hd + h * dh + j];
            o[h * dh + j] = s;
        }
    }
    vecmat(o, Wo, hd, C, F_out);
    for (int c = 0; c < C; ++c) F_out[c] += F[c];
    free(xn); free(q); free(k); free(v); free(o); free(a);
}

/* Blend-weight logits (Sec. 3.2.3, the blend weights): the pre-softmax
 * attention logits of the first head of the final fusion block,
 * a_m = (N(F) W_q)_0 . (s_m W_k)_0 / sqrt(d_h) for each view m; the softmax
 * over the views is applied by the render, after upsampling. */
OR_EXPORT void or_blend_logits(const double *F, int C, const double *S, int V, int Cf,
                               int heads, int dh, const double *Wq, const double *Wk,
                               double *logits)
{
    int hd = heads * dh;
    double *xn = malloc(sizeof(double) * C);
    double *q = malloc(sizeof(double) * hd);
    double *k = malloc(sizeof(double) * hd);
    or_rmsnorm(F, C, xn);
    vecmat(xn, Wq, C, hd, q);
    double scale = 1.0 / sqrt((double)dh);
    for (int m = 0; m < V; ++m) {
        vecmat(S + (size_t)m * Cf, Wk, Cf, hd, k);
        double s = 0.0;
        for (int j = 0; j < dh; ++j) s += q[j] * k[j];
        logits[m] = s * scale;
    }
    free(xn); free(q); free(k);
}

/* One-to-many (folded) attention (Sec. 3.3, "Optimized Attention", and the
 * appendix on its complexity): the key projection is folded into the query,
 * q~_i = N(F) W_i^q (W_i^k)^T / sqrt(d_h), and the value projection into the
 * output, F' = F + sum_i (sum_m p_im s_m) (W_i^val W^O_i), where W^O_i is the
 * i-th row block of W^O.  Exactly equal to or_attention in real arithmetic. */
OR_EXPORT void or_attention_folded(const double *F, int C, const double *S, int V, int Cf,
                                   int heads, int dh, const double *Wq, const double *Wk,
                                   const double *Wv, const double *Wo, double *F_out)
{
    int hd = heads * dh;
    double *xn = malloc(sizeof(double) * C);
    double *q = malloc(sizeof(double) * hd);
    double *qt = malloc(sizeof(double) * Cf);
    double *a = malloc(sizeof(double) * V);
    double *ob = malloc(sizeof(double) * Cf);
    double *ov = malloc(sizeof(double) * dh);

    or_rmsnorm(F, C, xn);
    vecmat(xn, Wq, C, hd, q);
    for (int c = 0; c < C; ++c) F_out[c] = F[c];
    double scale = 1.0 / sqrt((double)dh);
    for (int h = 0; h < heads; ++h) {
        /* q~ = q_h W_k,h^T / sqrt(dh)   (Cf values) */
        for (int i = 0; i < Cf; ++i) {
            double s = 0.0;
            for (int j = 0; j < dh; ++j) s += q[h * dh + j] * Wk[(size_t)i * hd + h * dh + j];
            qt[i] = s * scale;
        }
        double amax = -INFINITY;
        for (int m = 0; m < V; ++m) {
            double s = 0.0;
            for (int i = 0; i < Cf; ++i) s += qt[i] * S[(size_t)m * Cf + i];
            a[m] = s;
            if (s > amax) amax = s;
        }
        double z = 0.0;
        for (int m = 0; m < V; ++m) { a[m] = exp(a[m] - amax); z += a[m]; }
        for (int i = 0; i < Cf; ++i) {
            double s = 0.0;
            for (int m = 0; m < V; ++m) s += a[m] * S[(size_t)m * Cf + i];
            ob[i] = s / z;
        }
        /* (ob W_v,h) W_o,h : the folded output projection */
        for (int j = 0; j < dh; ++j) {
            double s = 0.0;
            for (int i = 0; i < Cf; ++i) s += ob[i] * Wv[(size_t)i * hd + h * dh + j];
            ov[j] = s;
        }
        for (int c = 0; c < C; ++c) {
            double s = 0.0;
            for (int j = 0; j < dh; ++j) s += ov[j] * Wo[(size_t)(h * dh + j) * C + c];
            F_out[c] += s;
        }
    }
    free(xn); free(q); free(qt); free(a); free(ob); free(ov);
}

/* ------------------------------------------------------------------------ */
/* Decode of the intermediate LDM (Sec. 3.2.2 "Decoding and rendering the    */
/* intermediate LDM", Sec. 3.2.3 depth anchors and depth activation).        */
/* ------------------------------------------------------------------------ */

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Bounds of the alpha clamp in the residual update: the float32 values
 * nearest 1e-6 and 1 - 1e-6.  Alphas arrive as float32, so the decision
 * "clamped or not" is taken against the bounds the float32 kernels apply. */
#define OR_ALPHA_LO 9.999999974752427e-07
#define OR_ALPHA_HI 0.9999989867210388

/* Given the updated feature F' of layer `li` (0 = nearest) of an L-layer LDM,
 * the layer-pixel's incoming alpha and depth, produce alpha', depth' and the
 * layer colour c' = sigmoid(F' W_c).
 *   mode 0 (residual update): alpha' = sigmoid(logit(clamp(alpha)) + F'.w_sigma)
 *          (clamp to [OR_ALPHA_LO, OR_ALPHA_HI]),
 *          disparity' = clamp(1/d + (0.5/L)(1/near - 1/far) tanh(F'.w_depth),
 *                             1/far, 1/near), d' = 1/disparity'.
 *   mode 1 (the paper's absolute decode): alpha' = sigmoid(F'.w_sigma),
 *          d' = 1 / ((delta + (0.5/L) tanh(F'.w_depth)) (1/near - 1/far) + 1/far)
 *          with the anchor delta = (l - 0.5)/L of paper layer l = L - li. */
OR_EXPORT void or_decode(const double *Fp, int C, const double *w_sigma, const double *w_depth,
                         const double *W_color, double alpha, double depth, int li, int L,
                         double near_, double far_, int mode, double *alpha_out,
                         double *depth_out, double *color_out)
{
    double xs = 0.0, xd = 0.0, xc[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < C; ++c) {
        xs += Fp[c] * w_sigma[c];
        xd += Fp[c] * w_depth[c];
        for (int j = 0; j < 3; ++j) xc[j] += Fp[c] * W_color[c * 3 + j];
    }
    for (int j = 0; j < 3; ++j) color_out[j] = sigmoid(xc[j]);
    double band = (1.0 / near_ - 1.0 / far_);
    if (mode == 0) {
        double a = alpha;
        if (a < OR_ALPHA_LO) a = OR_ALPHA_LO;
        if (a > OR_ALPHA_HI) a = OR_ALPHA_HI;
        *alpha_out = sigmoid(log(a / (1.0 - a)) + xs);
        double disp = 1.0 / depth + (0.5 / L) * band * tanh(xd);
        if (disp < 1.0 / far_) disp = 1.0 / far_;
        if (disp > 1.0 / near_) disp = 1.0 / near_;
        *depth_out = 1.0 / disp;
    } else {
        *alpha_out = sigmoid(xs);
        int l_paper = L - li;
        double delta = (l_paper - 0.5) / L;
        *depth_out = 1.0 / ((delta + (0.5 / L) * tanh(xd)) * band + 1.0 / far_);
    }
}

/* ------------------------------------------------------------------------ */
/* Over composite O (Sec. 3.1): layers composited with "over".  Written here */
/* front to back (layer 0 nearest), which equals the paper's back-to-front    */
/* order by associativity of "over"; black background, accumulated alpha     */
/* A = 1 - prod(1 - alpha) returned alongside.                               */
/* color [L][npix][3], alpha [L][npix] -> rgb [npix][3], acc [npix]          */
/* ------------------------------------------------------------------------ */

OR_EXPORT void or_composite(int L, long npix, const double *color, const double *alpha,
                            double *rgb, double *acc)
{
    for (long p = 0; p < npix; ++p) {
        double T = 1.0, r[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < L; ++l) {
            double a = alpha[(size_t)l * npix + p];
            for (int j = 0; j < 3; ++j) r[j] += T * a * color[((size_t)l * npix + p) * 3 + j];
            T *= (1.0 - a);
        }
        for (int j = 0; j < 3; ++j) rgb[p * 3 + j] = r[j];
        if (acc) acc[p] = 1.0 - T;
    }
}

/* Back-to-front form of the same operator, kept separately for the
 * order-equivalence check. */
OR_EXPORT void or_composite_back_to_front(int L, long npix, const double *color,
                                          const double *alpha, double *rgb)
{
    for (long p = 0; p < npix; ++p) {
        double r[3] = {0.0, 0.0, 0.0};
        for (int l = L - 1; l >= 0; --l) {
            double a = alpha[(size_t)l * npix + p];
            for (int j = 0; j < 3; ++j)
                r[j] = a * color[((size_t)l * npix + p) * 3 + j] + (1.0 - a) * r[j];
        }
        for (int j = 0; j < 3; ++j) rgb[p * 3 + j] = r[j];
    }
}

/* Adjoint of the over composite (Sec. 3.1, operator O), by the chain rule   */
/* through rgb = sum_l T_l alpha_l c_l with T_l = prod_{j<l} (1 - alpha_j)   */
/* and acc = 1 - T_L.  With B_l the composite of layers l..L-1 on their own  */
/* (B_L = 0, B_l = alpha_l c_l + (1 - alpha_l) B_{l+1}) and P_l the product  */
/* of (1 - alpha_j) over j >= l (P_L = 1):                                   */
/*   d rgb / d c_l     = T_l alpha_l                                         */
/*   d rgb / d alpha_l = T_l (c_l - B_{l+1})                                 */
/*   d acc / d alpha_l = T_l P_{l+1}                                         */
/* Inputs color [L][npix][3], alpha [L][npix], d_rgb [npix][3], d_acc [npix] */
/* (NULL = 0); outputs d_color [L][npix][3], d_alpha [L][npix].             */
/* ------------------------------------------------------------------------ */

OR_EXPORT void or_composite_backward(int L, long npix, const double *color, const double *alpha,
                                     const double *d_rgb, const double *d_acc, double *d_color,
                                     double *d_alpha)
{
    for (long p = 0; p < npix; ++p) {
        double *T = (double *)malloc(sizeof(double) * (size_t)(L + 1));
        double *B = (double *)malloc(sizeof(double) * (size_t)(L + 1) * 3);
        double *P = (double *)malloc(sizeof(double) * (size_t)(L + 1));
        T[0] = 1.0;
        for (int l = 0; l < L; ++l) T[l + 1] = T[l] * (1.0 - alpha[(size_t)l * npix + p]);
        for (int j = 0; j < 3; ++j) B[(size_t)L * 3 + j] = 0.0;
        P[L] = 1.0;
        for (int l = L - 1; l >= 0; --l) {
            double a = alpha[(size_t)l * npix + p];
            for (int j = 0; j < 3; ++j)
                B[(size_t)l * 3 + j] = a * color[((size_t)l * npix + p) * 3 + j] +
                                       (1.0 - a) * B[(size_t)(l + 1) * 3 + j];
            P[l] = P[l + 1] * (1.0 - a);
        }
        double gA = d_acc ? d_acc[p] : 0.0;
        for (int l = 0; l < L; ++l) {
            size_t e = (size_t)l * npix + p;
            double a = alpha[e], da = gA * T[l] * P[l + 1];
            for (int j = 0; j < 3; ++j) {
                double g = d_rgb[p * 3 + j];
                d_color[e * 3 + j] = g * T[l] * a;
                da += g * T[l] * (color[e * 3 + j] - B[(size_t)(l + 1) * 3 + j]);
            }
            d_alpha[e] = da;
        }
        free(T);
        free(B);
        free(P);
    }
}

/* ------------------------------------------------------------------------ */
/* One Update & Fuse step over a set of LDM rows (every layer of each row).  */
/* For each layer li, row y in rows[], column x and view m: reproject the    */
/* layer-pixel through its depth into view m, sample view m's feature map,   */
/* then attend across the V samples, then decode.  Layer-pixels are          */
/* independent, so any subset of rows gives the exact values of those rows.  */
/*                                                                           */
/* Inputs (all double, row-major):                                           */
/*   V views: Kin[V][9], Ein[V][16], cam_wh[V][2] (grid of Kin),             */
/*            feats[V] -> [Hf][Wf][Cf], feat_hw[V][2] = (Hf, Wf)             */
/*   novel:   Kn[9], En[16], nov_wh[2] (grid of Kn)                          */
/*   LDM:     L, H, W, C; F[L][H][W][C], depth[L][H][W], alpha[L][H][W]      */
/*   weights: Wq[C][hd], Wk[Cf][hd], Wv[Cf][hd], Wo[hd][C], w_sigma[C],      */
/*            w_depth[C], W_color[C][3]                                      */
/* Outputs, packed over the selected rows (R = nrows):                       */
/*   F_out[L][R][W][C], depth_out[L][R][W], alpha_out[L][R][W],              */
/*   color_out[L][R][W][3]; samples_out[L][R][W][V][Cf] if non-NULL;        */
/*   logits_out[L][R][W][V] if non-NULL: the blend-weight logits of the      */
/*   step's attention (or_blend_logits).                                     */
/* attn_form: 0 standard, 1 one-to-many (folded).                            */
/* ------------------------------------------------------------------------ */

OR_EXPORT int or_update_fuse(int V, const double *Kin, const double *Ein, const int *cam_wh,
                             const double *const *feats, const int *feat_hw, int Cf,
                             const double *Kn, const double *En, const int *nov_wh,
                             double near_, double far_, int L, int H, int W, int C,
                             const double *F, const double *depth, const double *alpha,
                             int heads, int dh, const double *Wq, const double *Wk,
                             const double *Wv, const double *Wo, const double *w_sigma,
                             const double *w_depth, const double *W_color, int mode,
                             int attn_form, const int *rows, int nrows, double *F_out,
                             double *depth_out, double *alpha_out, double *color_out,
                             double *samples_out, double *logits_out)
{
    double Kns[9];
    or_scale_intrinsics(Kn, nov_wh[0], nov_wh[1], W, H, Kns);
    double *T = malloc(sizeof(double) * 16 * (size_t)V);
    for (int m = 0; m < V; ++m) {
        double Kms[9];
        or_scale_intrinsics(Kin + 9 * m, cam_wh[2 * m], cam_wh[2 * m + 1], feat_hw[2 * m + 1],
                            feat_hw[2 * m], Kms);
        if (or_reprojection_matrix(Kns, En, Kms, Ein + 16 * m, T + 16 * m) != 0) {
            free(T);
            return -1;
        }
    }
    long total = (long)L * nrows * W;
    int err = 0;
#pragma omp parallel
    {
        double *S = malloc(sizeof(double) * (size_t)V * Cf);
        double *Fp = malloc(sizeof(double) * C);
#pragma omp for schedule(dynamic, 64)
        for (long idx = 0; idx < total; ++idx) {
            int x = (int)(idx % W);
            long t = idx / W;
            int r = (int)(t % nrows);
            int li = (int)(t / nrows);
            int y = rows[r];
            size_t src = ((size_t)li * H + y) * W + x;      /* layer-pixel in full arrays */
            size_t dst = ((size_t)li * nrows + r) * W + x;  /* packed output position     */
            double d = depth[src];
            double u = x + 0.5, v = y + 0.5;
            for (int m = 0; m < V; ++m) {
                double uv[2];
                double *s = S + (size_t)m * Cf;
                if (or_reproject_T(T + 16 * m, u, v, d, uv) == 1) {
                    or_bilinear(feats[m], feat_hw[2 * m], feat_hw[2 * m + 1], Cf, uv[0], uv[1], s);
                } else {
                    for (int c = 0; c < Cf; ++c) s[c] = 0.0;
                }
            }
            if (samples_out)
                memcpy(samples_out + dst * (size_t)V * Cf, S, sizeof(double) * (size_t)V * Cf);
            if (logits_out)
                or_blend_logits(F + src * C, C, S, V, Cf, heads, dh, Wq, Wk,
                                logits_out + dst * (size_t)V);
            if (attn_form == 0)
                or_attention(F + src * C, C, S, V, Cf, heads, dh, Wq, Wk, Wv, Wo, Fp, NULL);
            else
                or_attention_folded(F + src * C, C, S, V, Cf, heads, dh, Wq, Wk, Wv, Wo, Fp);
            memcpy(F_out + dst * C, Fp, sizeof(double) * C);
            or_decode(Fp, C, w_sigma, w_depth, W_color, alpha[src], d, li, L, near_, far_, mode,
                      alpha_out + dst, depth_out + dst, color_out + dst * 3);
        }
        free(S);
        free(Fp);
    }
    free(T);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Final render (Sec. 3.1, Eq. 1; Sec. 3.2.3 "Upsampling & Activation").     */
/* The final LDM arrives as unactivated attributes at a reduced grid (h, w):  */
/* depth logits x_d and density logits x_sigma [L][h][w] and blend-weight     */
/* logits [L][h][w][V] over the V input images.  They are bilinearly          */
/* upsampled to the output grid (H, W) and only then activated: density      */
/* sigma = sigmoid(x_sigma), depth through the anchored disparity-band        */
/* activation (the paper's depth activation, anchor of paper layer           */
/* l = L - index), blend weights beta = softmax over the views (delayed until */
/* after the upsampling).  Each input image is carried onto every layer by    */
/* the back-projection operator through the decoded depth (reprojection and  */
/* bilinear sampling with zero padding, a point behind a view samples zero),  */
/* the V images are mixed per layer with beta, and the layers are            */
/* over-composited with alpha = sigma (front to back, black background).     */
/* ------------------------------------------------------------------------ */

/* Bilinear resampling of src[h][w][C] at output pixel (x, y) of an (H, W)
 * grid, half-pixel centres: source coordinate (x + 0.5) w / W - 0.5, clamped
 * below at 0; taps floor and floor + 1, the latter clamped to the last
 * row/column (the border value extends outward). */
static void upsample_at(const double *src, int h, int w, int C, int H, int W, int x, int y,
                        double *out)
{
    double sy = (y + 0.5) * (double)h / (double)H - 0.5;
    double sx = (x + 0.5) * (double)w / (double)W - 0.5;
    if (sy < 0.0) sy = 0.0;
    if (sx < 0.0) sx = 0.0;
    int y0 = (int)floor(sy), x0 = (int)floor(sx);
    if (y0 > h - 1) y0 = h - 1;
    if (x0 > w - 1) x0 = w - 1;
    int y1 = (y0 + 1 < h) ? y0 + 1 : h - 1;
    int x1 = (x0 + 1 < w) ? x0 + 1 : w - 1;
    double ly = sy - y0, lx = sx - x0;
    const double *s00 = src + ((size_t)y0 * w + x0) * C, *s10 = src + ((size_t)y0 * w + x1) * C;
    const double *s01 = src + ((size_t)y1 * w + x0) * C, *s11 = src + ((size_t)y1 * w + x1) * C;
    for (int c = 0; c < C; ++c)
        out[c] = (1.0 - ly) * ((1.0 - lx) * s00[c] + lx * s10[c]) +
                 ly * ((1.0 - lx) * s01[c] + lx * s11[c]);
}

OR_EXPORT void or_upsample_bilinear(const double *src, int h, int w, int C, int H, int W,
                                    double *dst)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) upsample_at(src, h, w, C, H, W, x, y, dst + ((size_t)y * W + x) * C);
}

/* Activation of one layer-pixel's upsampled logits (layer index li, 0 =
 * nearest): sigma = sigmoid(xs); depth = 1 / ((delta + (0.5/L) tanh(xd))
 * (1/near - 1/far) + 1/far) with delta = (l - 0.5)/L, l = L - li; beta =
 * softmax of xb over the V views (maximum subtracted). */
OR_EXPORT void or_ibr_activate(double xd, double xs, const double *xb, int V, int li, int L,
                               double near_, double far_, double *depth, double *sigma,
                               double *beta)
{
    *sigma = sigmoid(xs);
    double delta = ((L - li) - 0.5) / L;
    *depth = 1.0 / ((delta + (0.5 / L) * tanh(xd)) * (1.0 / near_ - 1.0 / far_) + 1.0 / far_);
    double mx = -INFINITY;
    for (int m = 0; m < V; ++m)
        if (xb[m] > mx) mx = xb[m];
    double z = 0.0;
    for (int m = 0; m < V; ++m) { beta[m] = exp(xb[m] - mx); z += beta[m]; }
    for (int m = 0; m < V; ++m) beta[m] /= z;
}

/* The render over the listed output rows.
 * Inputs (double, row-major):
 *   V views: Kin[V][9], Ein[V][16], cam_wh[V][2] (grid of Kin),
 *            images[V] -> [Hi][Wi][3] (RGB in [0, 1]), img_hw[V][2] = (Hi, Wi)
 *   novel:   Kn[9], En[16], nov_wh[2] (grid of Kn)
 *   LDM:     L, h, w; depth_logit[L][h][w], sigma_logit[L][h][w],
 *            blend_logit[L][h][w][V]
 *   output grid H, W; rows[nrows]
 * Outputs, packed over the rows: rgb[R][W][3], acc[R][W] (1 - prod(1 - sigma)),
 * depth_map[R][W] (the decoded depth over-composited the same way), and, if
 * non-NULL, layer_color[L][R][W][3] (the blended image of each layer). */
OR_EXPORT int or_render_ibr(int V, const double *Kin, const double *Ein, const int *cam_wh,
                            const double *const *images, const int *img_hw, const double *Kn,
                            const double *En, const int *nov_wh, double near_, double far_, int L,
                            int h, int w, const double *depth_logit, const double *sigma_logit,
                            const double *blend_logit, int H, int W, const int *rows, int nrows,
                            double *rgb, double *acc, double *depth_map, double *layer_color)
{
    double Kns[9];
    or_scale_intrinsics(Kn, nov_wh[0], nov_wh[1], W, H, Kns);
    double *T = malloc(sizeof(double) * 16 * (size_t)V);
    for (int m = 0; m < V; ++m) {
        double Kms[9];
        or_scale_intrinsics(Kin + 9 * m, cam_wh[2 * m], cam_wh[2 * m + 1], img_hw[2 * m + 1],
                            img_hw[2 * m], Kms);
        if (or_reprojection_matrix(Kns, En, Kms, Ein + 16 * m, T + 16 * m) != 0) {
            free(T);
            return -1;
        }
    }
    long total = (long)nrows * W;
#pragma omp parallel
    {
        double *xb = malloc(sizeof(double) * V);
        double *beta = malloc(sizeof(double) * V);
#pragma omp for schedule(dynamic, 64)
        for (long idx = 0; idx < total; ++idx) {
            int x = (int)(idx % W);
            int r = (int)(idx / W);
            int y = rows[r];
            double u = x + 0.5, v = y + 0.5;
            double Tr = 1.0, out[3] = {0.0, 0.0, 0.0}, dm = 0.0;
            for (int li = 0; li < L; ++li) {
                double xd, xs, d, sg;
                upsample_at(depth_logit + (size_t)li * h * w, h, w, 1, H, W, x, y, &xd);
                upsample_at(sigma_logit + (size_t)li * h * w, h, w, 1, H, W, x, y, &xs);
                upsample_at(blend_logit + (size_t)li * h * w * V, h, w, V, H, W, x, y, xb);
                or_ibr_activate(xd, xs, xb, V, li, L, near_, far_, &d, &sg, beta);
                double c[3] = {0.0, 0.0, 0.0};
                for (int m = 0; m < V; ++m) {
                    double uv[2], s[3];
                    if (or_reproject_T(T + 16 * m, u, v, d, uv) == 1)
                        or_bilinear(images[m], img_hw[2 * m], img_hw[2 * m + 1], 3, uv[0], uv[1], s);
                    else
                        s[0] = s[1] = s[2] = 0.0;
                    for (int j = 0; j < 3; ++j) c[j] += beta[m] * s[j];
                }
                if (layer_color)
                    for (int j = 0; j < 3; ++j)
                        layer_color[(((size_t)li * nrows + r) * W + x) * 3 + j] = c[j];
                for (int j = 0; j < 3; ++j) out[j] += Tr * sg * c[j];
                dm += Tr * sg * d;
                Tr *= (1.0 - sg);
            }
            size_t o = (size_t)r * W + x;
            for (int j = 0; j < 3; ++j) rgb[o * 3 + j] = out[j];
            if (acc) acc[o] = 1.0 - Tr;
            if (depth_map) depth_map[o] = dm;
        }
        free(xb);
        free(beta);
    }
    free(T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Render to input views (Sec. 3.2.2 "Decoding and rendering the            */
/* intermediate LDM", Eq. 2): the decoded intermediate LDM -- per layer-     */
/* pixel depth d, density sigma and appearance a (RGB) -- is carried into    */
/* each input view by the projection operator P_theta and over-composited    */
/* there.  P_theta is the operator whose adjoint is the back-projection      */
/* P^T_theta used for sampling (Sec. 3.1): a layer-pixel reprojected through */
/* its depth to view m's continuous coordinate adds its value to the four   */
/* view pixels around that point, with the bilinear weights that sampling    */
/* at that point would give them (taps outside the view grid dropped, a      */
/* point behind the view adds nothing; no normalisation).  Each layer is     */
/* projected separately; the projected layers are composited front to back  */
/* (layer 0 nearest the novel camera) with the projected density as alpha.  */
/* ------------------------------------------------------------------------ */

/* Project one layer's values val[H][W][C] (novel grid, depth[H][W]) into a
 * view grid (Hm, Wm) through the 4x4 chain T (as for sampling), adding into
 * out[Hm][Wm][C]. */
OR_EXPORT void or_splat_layer(const double *T, int H, int W, const double *depth,
                              const double *val, int C, int Hm, int Wm, double *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double uv[2];
            size_t q = (size_t)y * W + x;
            if (or_reproject_T(T, x + 0.5, y + 0.5, depth[q], uv) != 1) continue;
            double fx_ = uv[0] - 0.5, fy_ = uv[1] - 0.5;
            if (!(fabs(fx_) < 1e9 && fabs(fy_) < 1e9)) continue;
            double xf = floor(fx_), yf = floor(fy_);
            double fx = fx_ - xf, fy = fy_ - yf;
            long x0 = (long)xf, y0 = (long)yf;
            const long tx[4] = {x0, x0 + 1, x0, x0 + 1};
            const long ty[4] = {y0, y0, y0 + 1, y0 + 1};
            const double w[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
            for (int t = 0; t < 4; ++t) {
                if (tx[t] < 0 || tx[t] >= Wm || ty[t] < 0 || ty[t] >= Hm) continue;
                double *o = out + ((size_t)ty[t] * Wm + (size_t)tx[t]) * C;
                for (int c = 0; c < C; ++c) o[c] += w[t] * val[q * C + c];
            }
        }
}

/* The whole render to the V views.
 * Inputs: Kin[V][9], Ein[V][16], cam_wh[V][2] (grid of Kin), view_hw[V][2]
 * (Hm, Wm: the grid each view is rendered on); novel Kn[9], En[16],
 * nov_wh[2]; LDM L, H, W with depth, alpha [L][H][W] and color [L][H][W][3].
 * Outputs: img[V] -> [Hm][Wm][3], acc[V] -> [Hm][Wm] (1 - prod(1 - alpha))
 * or NULL. */
OR_EXPORT int or_render_to_views(int V, const double *Kin, const double *Ein, const int *cam_wh,
                                 const int *view_hw, const double *Kn, const double *En,
                                 const int *nov_wh, int L, int H, int W, const double *depth,
                                 const double *alpha, const double *color, double *const *img,
                                 double *const *acc)
{
    double Kns[9];
    or_scale_intrinsics(Kn, nov_wh[0], nov_wh[1], W, H, Kns);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int m = 0; m < V; ++m) {
        int Hm = view_hw[2 * m], Wm = view_hw[2 * m + 1];
        double Kms[9], T[16];
        or_scale_intrinsics(Kin + 9 * m, cam_wh[2 * m], cam_wh[2 * m + 1], Wm, Hm, Kms);
        if (or_reprojection_matrix(Kns, En, Kms, Ein + 16 * m, T) != 0) { err = -1; continue; }
        size_t np = (size_t)Hm * Wm;
        double *pc = calloc(np * 3, sizeof(double));   /* P(a) of one layer     */
        double *ps = calloc(np, sizeof(double));       /* P(sigma) of one layer */
        double *Tr = malloc(np * sizeof(double));
        for (size_t p = 0; p < np; ++p) Tr[p] = 1.0;
        for (size_t p = 0; p < np * 3; ++p) img[m][p] = 0.0;
        for (int l = 0; l < L; ++l) {
            memset(pc, 0, np * 3 * sizeof(double));
            memset(ps, 0, np * sizeof(double));
            size_t off = (size_t)l * H * W;
            or_splat_layer(T, H, W, depth + off, color + off * 3, 3, Hm, Wm, pc);
            or_splat_layer(T, H, W, depth + off, alpha + off, 1, Hm, Wm, ps);
            for (size_t p = 0; p < np; ++p) {
                for (int j = 0; j < 3; ++j) img[m][p * 3 + j] += Tr[p] * ps[p] * pc[p * 3 + j];
                Tr[p] *= (1.0 - ps[p]);
            }
        }
        if (acc && acc[m])
            for (size_t p = 0; p < np; ++p) acc[m][p] = 1.0 - Tr[p];
        free(pc);
        free(ps);
        free(Tr);
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* Residual CNN block of a fusion block (Sec. 3.3: the one-to-many attention */
/* is interleaved with residual 3x3 convolutional blocks, mirroring a        */
/* Transformer's MLP block; the network tables of the appendix list them).  */
/* Per LDM layer, over the layer's (H, W) grid: the RMS normalisation N of  */
/* the attention's pre-norm, per pixel over the channels, then two 3x3       */
/* convolutions C -> C with zero padding and a GELU between them, added to   */
/* the input:                                                                */
/*   V' = V + W2 * gelu(W1 * N(V)),  gelu(x) = x Phi(x) = x (1 + erf(x/sqrt 2))/2, */
/* out(y, x)[co] = sum_{ky, kx, ci} in(y + ky - 1, x + kx - 1)[ci] W[ky][kx][ci][co]. */
/* No biases.                                                                */
/* ------------------------------------------------------------------------ */

static void conv3x3(const double *in, int H, int W, int C, const double *Wt, double *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double *o = out + ((size_t)y * W + x) * C;
            for (int co = 0; co < C; ++co) o[co] = 0.0;
            for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                    int yy = y + ky - 1, xx = x + kx - 1;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;   /* zero padding */
                    const double *i = in + ((size_t)yy * W + xx) * C;
                    const double *w = Wt + (size_t)(ky * 3 + kx) * C * C;
                    for (int ci = 0; ci < C; ++ci)
                        for (int co = 0; co < C; ++co) o[co] += i[ci] * w[(size_t)ci * C + co];
                }
        }
}

/* F, out [L][H][W][C]; W1, W2 [3][3][C][C]. */
OR_EXPORT void or_residual_conv(int L, int H, int W, int C, const double *F, const double *W1,
                                const double *W2, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < L; ++l) {
        size_t n = (size_t)H * W * C, off = (size_t)l * n;
        double *h = malloc(sizeof(double) * n);
        double *g = malloc(sizeof(double) * n);
        for (size_t p = 0; p < (size_t)H * W; ++p) or_rmsnorm(F + off + p * C, C, g + p * C);
        conv3x3(g, H, W, C, W1, h);
        for (size_t i = 0; i < n; ++i) h[i] = 0.5 * h[i] * (1.0 + erf(h[i] / sqrt(2.0)));
        conv3x3(h, H, W, C, W2, g);
        for (size_t i = 0; i < n; ++i) out[off + i] = F[off + i] + g[i];
        free(h);
        free(g);
    }
}

/* ------------------------------------------------------------------------ */
/* Layer collapse (Sec. 3.2.2, "Layer Collapse"; the Lc blocks of the        */
/* network tables): before the last two update steps the number of layers   */
/* halves; each new layer is the mean of a pair of adjacent layers plus a    */
/* residual MLP of their concatenation:                                      */
/*   out[j] = (F[2j] + F[2j+1]) / 2 + relu([F[2j], F[2j+1]] W1) W2,          */
/* W1 [2C][C], W2 [C][C], per pixel, no biases.                              */
/* ------------------------------------------------------------------------ */

/* F [L][H][W][C] with L even -> out [L/2][H][W][C]. */
OR_EXPORT void or_layer_collapse(int L, int H, int W, int C, const double *F, const double *W1,
                                 const double *W2, double *out)
{
    long npix = (long)H * W;
#pragma omp parallel
    {
        double *x = malloc(sizeof(double) * 2 * C);
        double *h = malloc(sizeof(double) * C);
#pragma omp for schedule(static)
        for (long idx = 0; idx < (long)(L / 2) * npix; ++idx) {
            long j = idx / npix, p = idx % npix;
            const double *a = F + ((size_t)(2 * j) * npix + p) * C;
            const double *b = F + ((size_t)(2 * j + 1) * npix + p) * C;
            for (int c = 0; c < C; ++c) { x[c] = a[c]; x[C + c] = b[c]; }
            for (int o = 0; o < C; ++o) {
                double s = 0.0;
                for (int i = 0; i < 2 * C; ++i) s += x[i] * W1[(size_t)i * C + o];
                h[o] = s > 0.0 ? s : 0.0;
            }
            double *y = out + ((size_t)j * npix + p) * C;
            for (int o = 0; o < C; ++o) {
                double s = 0.0;
                for (int i = 0; i < C; ++i) s += h[i] * W2[(size_t)i * C + o];
                y[o] = 0.5 * (a[o] + b[o]) + s;
            }
        }
        free(x);
        free(h);
    }
}

/* ------------------------------------------------------------------------ */
/* Ray-direction encoding of an input view's pixels (Sec. 3.2.2, "Encode     */
/* Input Images"): the ray of pixel (x, y) of view m is intersected with the */
/* planes z = near and z = far of the novel camera's frustum (its own frame),*/
/* both points are projected by the novel camera, and the difference (far    */
/* minus near) is taken in normalised device coordinates (2 u / W_n,         */
/* 2 v / H_n of the novel grid); it is squashed by tanh, encoded with 8      */
/* octaves of sinusoids -- e[4k + 0..3] = sin(2^k pi t_x), cos(2^k pi t_x),  */
/* sin(2^k pi t_y), cos(2^k pi t_y) -- and projected by W [32][C].          */
/* ------------------------------------------------------------------------ */

static void mat3_of_4x4(const double *E, double *R) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[3 * r + c] = E[4 * r + c];
}

/* Km, Em, cam_wh: view m's camera on its own grid; the view is encoded on
 * an (Hf, Wf) grid.  out [Hf][Wf][C]; delta_out [Hf][Wf][2] (the NDC
 * difference, before tanh) if non-NULL. */
OR_EXPORT int or_ray_encoding(const double *Km, const double *Em, const int *cam_wh, int Hf,
                              int Wf, const double *Kn, const double *En, const int *nov_wh,
                              double near_, double far_, const double *Wr, int C, double *out,
                              double *delta_out)
{
    double Ks[9], Ksi[16], Ks4[16], Emi[16];
    or_scale_intrinsics(Km, cam_wh[0], cam_wh[1], Wf, Hf, Ks);
    k_to_4x4(Ks, Ks4);
    if (inv4(Ks4, Ksi) != 0 || inv4(Em, Emi) != 0) return -1;
    double Rn[9];
    mat3_of_4x4(En, Rn);
    /* camera m's centre in the novel frame: En * inv(Em) * (0, 0, 0, 1) */
    double cw[4] = {Emi[3], Emi[7], Emi[11], Emi[15]}, o[3];
    for (int r = 0; r < 3; ++r)
        o[r] = En[4 * r] * cw[0] + En[4 * r + 1] * cw[1] + En[4 * r + 2] * cw[2] + En[4 * r + 3] * cw[3];
    for (int y = 0; y < Hf; ++y)
        for (int x = 0; x < Wf; ++x) {
            double pc[3] = {x + 0.5, y + 0.5, 1.0}, dc[3], dw[3], dn[3];
            for (int r = 0; r < 3; ++r)            /* ray in camera m: K^-1 (u, v, 1) */
                dc[r] = Ksi[4 * r] * pc[0] + Ksi[4 * r + 1] * pc[1] + Ksi[4 * r + 2] * pc[2];
            for (int r = 0; r < 3; ++r)            /* to world: inverse rotation of Em */
                dw[r] = Emi[4 * r] * dc[0] + Emi[4 * r + 1] * dc[1] + Emi[4 * r + 2] * dc[2];
            for (int r = 0; r < 3; ++r)            /* to the novel frame */
                dn[r] = Rn[3 * r] * dw[0] + Rn[3 * r + 1] * dw[1] + Rn[3 * r + 2] * dw[2];
            double ndc[2][2];
            const double planes[2] = {near_, far_};
            for (int k = 0; k < 2; ++k) {
                double sp = (planes[k] - o[2]) / dn[2];
                double P[3] = {o[0] + sp * dn[0], o[1] + sp * dn[1], o[2] + sp * dn[2]};
                double u = (Kn[0] * P[0] + Kn[1] * P[1] + Kn[2] * P[2]) / P[2];
                double v = (Kn[3] * P[0] + Kn[4] * P[1] + Kn[5] * P[2]) / P[2];
                ndc[k][0] = 2.0 * u / nov_wh[0];
                ndc[k][1] = 2.0 * v / nov_wh[1];
            }
            double dlt[2] = {ndc[1][0] - ndc[0][0], ndc[1][1] - ndc[0][1]};
            size_t q = (size_t)y * Wf + x;
            if (delta_out) { delta_out[2 * q] = dlt[0]; delta_out[2 * q + 1] = dlt[1]; }
            double t[2] = {tanh(dlt[0]), tanh(dlt[1])}, e[32];
            for (int k = 0; k < 8; ++k) {
                double f = M_PI * (double)(1 << k);
                e[4 * k + 0] = sin(f * t[0]);
                e[4 * k + 1] = cos(f * t[0]);
                e[4 * k + 2] = sin(f * t[1]);
                e[4 * k + 3] = cos(f * t[1]);
            }
            for (int c = 0; c < C; ++c) {
                double sacc = 0.0;
                for (int i = 0; i < 32; ++i) sacc += e[i] * Wr[(size_t)i * C + c];
                out[q * C + c] = sacc;
            }
        }
    return 0;
}

OR_EXPORT int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel regions started after this call from the
   calling thread; n <= 0 leaves it unchanged. */
OR_EXPORT void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Adjoint of one Update & Fuse step and its composite.                      */
/*                                                                          */
/* Written from the forward definitions above by the chain rule, in the     */
/* standard (unfolded) form: keys and values are formed per sample and      */
/* differentiated as such.  Gradients are ACCUMULATED into the outputs,     */
/* which the caller zero-fills.  Only the listed rows are processed: the    */
/* upstream gradients of every other row are taken as zero, so the results  */
/* are the exact gradients of a loss restricted to those rows.              */
/*                                                                          */
/* Upstream (any may be NULL = zero), full-size arrays:                     */
/*   d_rgb[H][W][3], dF_out[L][H][W][C], d_depth_out[L][H][W],              */
/*   d_alpha_out[L][H][W]                                                   */
/* Gradients (full-size, accumulated): dF, d_depth, d_alpha [like inputs],  */
/*   dI[V] -> [Hf][Wf][Cf], dWq, dWk, dWv, dWo, dw_sigma, dw_depth,          */
/*   dW_color (shapes of the weights).                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int valid;
    double um, vm;          /* sample coordinate in view m's feature grid */
    double dum_dd, dvm_dd;  /* its derivative w.r.t. the layer depth      */
} or_proj;

static void reproject_with_derivative(const double *T, double u, double v, double d, or_proj *pr)
{
    double X[4] = {u * d, v * d, d, 1.0}, dX[4] = {u, v, 1.0, 0.0};
    double P[4], dP[4];
    for (int r = 0; r < 4; ++r) {
        double s = 0.0, ds = 0.0;
        for (int c = 0; c < 4; ++c) {
            s += T[4 * r + c] * X[c];
            ds += T[4 * r + c] * dX[c];
        }
        P[r] = s;
        dP[r] = ds;
    }
    pr->valid = P[2] > 1e-6 * d;
    if (!pr->valid) return;
    pr->um = P[0] / P[2];
    pr->vm = P[1] / P[2];
    pr->dum_dd = (dP[0] * P[2] - P[0] * dP[2]) / (P[2] * P[2]);
    pr->dvm_dd = (dP[1] * P[2] - P[1] * dP[2]) / (P[2] * P[2]);
}

/* Tap value (zero outside the map). */
static const double *tap_ptr(const double *I, int Hf, int Wf, int C, long tx, long ty)
{
    if (tx < 0 || tx >= Wf || ty < 0 || ty >= Hf) return NULL;
    return I + ((size_t)ty * Wf + (size_t)tx) * C;
}

OR_EXPORT int or_update_fuse_backward(
    int V, const double *Kin, const double *Ein, const int *cam_wh, const double *const *feats,
    const int *feat_hw, int Cf, const double *Kn, const double *En, const int *nov_wh,
    double near_, double far_, int L, int H, int W, int C, const double *F, const double *depth,
    const double *alpha, int heads, int dh, const double *Wq, const double *Wk, const double *Wv,
    const double *Wo, const double *w_sigma, const double *w_depth, const double *W_color, int mode,
    const int *rows, int nrows, const double *d_rgb, const double *dF_out,
    const double *d_depth_out, const double *d_alpha_out, double *dF, double *d_depth,
    double *d_alpha, double *const *dI, double *dWq, double *dWk, double *dWv, double *dWo,
    double *dw_sigma, double *dw_depth, double *dW_color)
{
    int hd = heads * dh;
    double Kns[9];
    or_scale_intrinsics(Kn, nov_wh[0], nov_wh[1], W, H, Kns);
    double *T = malloc(sizeof(double) * 16 * (size_t)V);
    for (int m = 0; m < V; ++m) {
        double Kms[9];
        or_scale_intrinsics(Kin + 9 * m, cam_wh[2 * m], cam_wh[2 * m + 1], feat_hw[2 * m + 1],
                            feat_hw[2 * m], Kms);
        if (or_reprojection_matrix(Kns, En, Kms, Ein + 16 * m, T + 16 * m) != 0) {
            free(T);
            return -1;
        }
    }
    const double band = 1.0 / near_ - 1.0 / far_;
    const double kap = (0.5 / L) * band;
    const double isq = 1.0 / sqrt((double)dh);
    const size_t nW = (size_t)C * hd;
    long npix = (long)nrows * W;

#pragma omp parallel
    {
        /* per-thread weight-gradient accumulators */
        double *gWq = calloc((size_t)C * hd, sizeof(double));
        double *gWk = calloc((size_t)Cf * hd, sizeof(double));
        double *gWv = calloc((size_t)Cf * hd, sizeof(double));
        double *gWo = calloc((size_t)hd * C, sizeof(double));
        double *gws = calloc((size_t)C, sizeof(double));
        double *gwd = calloc((size_t)C, sizeof(double));
        double *gWc = calloc((size_t)C * 3, sizeof(double));
        /* per-layer forward state of one pixel */
        double *S = malloc(sizeof(double) * (size_t)L * V * Cf);
        or_proj *PR = malloc(sizeof(or_proj) * (size_t)L * V);
        double *XN = malloc(sizeof(double) * (size_t)L * C);
        double *RR = malloc(sizeof(double) * L);
        double *Q = malloc(sizeof(double) * (size_t)L * hd);
        double *Kk = malloc(sizeof(double) * (size_t)L * V * hd);
        double *Vv = malloc(sizeof(double) * (size_t)L * V * hd);
        double *Pp = malloc(sizeof(double) * (size_t)L * heads * V);
        double *O = malloc(sizeof(double) * (size_t)L * hd);
        double *FP = malloc(sizeof(double) * (size_t)L * C);
        double *XS = malloc(sizeof(double) * L), *XD = malloc(sizeof(double) * L);
        double *XC = malloc(sizeof(double) * (size_t)L * 3);
        double *AL = malloc(sizeof(double) * L), *DN = malloc(sizeof(double) * L);
        double *CO = malloc(sizeof(double) * (size_t)L * 3);
        double *Tt = malloc(sizeof(double) * (L + 1)), *Bb = malloc(sizeof(double) * (size_t)(L + 1) * 3);
        double *dFp = malloc(sizeof(double) * C), *dO = malloc(sizeof(double) * hd);
        double *dQ = malloc(sizeof(double) * hd), *dXN = malloc(sizeof(double) * C);
        double *dK = malloc(sizeof(double) * (size_t)V * hd), *dV = malloc(sizeof(double) * (size_t)V * hd);
        double *dS = malloc(sizeof(double) * Cf);
        double *dpv = malloc(sizeof(double) * V);

#pragma omp for schedule(dynamic, 16)
        for (long idx = 0; idx < npix; ++idx) {
            int x = (int)(idx % W);
            int y = rows[idx / W];
            double u = x + 0.5, v = y + 0.5;
            /* ---- forward recompute of every layer of this pixel */
            for (int li = 0; li < L; ++li) {
                size_t src = ((size_t)li * H + y) * W + x;
                double d = depth[src];
                for (int m = 0; m < V; ++m) {
                    or_proj *pr = &PR[li * V + m];
                    double *s = S + ((size_t)li * V + m) * Cf;
                    reproject_with_derivative(T + 16 * m, u, v, d, pr);
                    if (pr->valid)
                        or_bilinear(feats[m], feat_hw[2 * m], feat_hw[2 * m + 1], Cf, pr->um, pr->vm, s);
                    else
                        for (int c = 0; c < Cf; ++c) s[c] = 0.0;
                }
                const double *f = F + src * C;
                double ss = 0.0;
                for (int c = 0; c < C; ++c) ss += f[c] * f[c];
                RR[li] = sqrt(ss / C + 1e-6);
                for (int c = 0; c < C; ++c) XN[li * C + c] = f[c] / RR[li];
                vecmat(XN + li * C, Wq, C, hd, Q + li * hd);
                for (int m = 0; m < V; ++m) {
                    const double *s = S + ((size_t)li * V + m) * Cf;
                    vecmat(s, Wk, Cf, hd, Kk + ((size_t)li * V + m) * hd);
                    vecmat(s, Wv, Cf, hd, Vv + ((size_t)li * V + m) * hd);
                }
                for (int j = 0; j < hd; ++j) O[li * hd + j] = 0.0;
                for (int hh = 0; hh < heads; ++hh) {
                    double amax = -INFINITY, z = 0.0;
                    double *pp = Pp + ((size_t)li * heads + hh) * V;
                    for (int m = 0; m < V; ++m) {
                        double a = 0.0;
                        for (int j = 0; j < dh; ++j)
                            a += Q[li * hd + hh * dh + j] * Kk[((size_t)li * V + m) * hd + hh * dh + j];
                        pp[m] = a * isq;
                        if (pp[m] > amax) amax = pp[m];
                    }
                    for (int m = 0; m < V; ++m) { pp[m] = exp(pp[m] - amax); z += pp[m]; }
                    for (int m = 0; m < V; ++m) pp[m] /= z;
                    for (int j = 0; j < dh; ++j) {
                        double o = 0.0;
                        for (int m = 0; m < V; ++m) o += pp[m] * Vv[((size_t)li * V + m) * hd + hh * dh + j];
                        O[li * hd + hh * dh + j] = o;
                    }
                }
                vecmat(O + li * hd, Wo, hd, C, FP + li * C);
                for (int c = 0; c < C; ++c) FP[li * C + c] += f[c];
                double xs = 0.0, xd = 0.0, xc[3] = {0, 0, 0};
                for (int c = 0; c < C; ++c) {
                    xs += FP[li * C + c] * w_sigma[c];
                    xd += FP[li * C + c] * w_depth[c];
                    for (int j = 0; j < 3; ++j) xc[j] += FP[li * C + c] * W_color[c * 3 + j];
                }
                XS[li] = xs;
                XD[li] = xd;
                for (int j = 0; j < 3; ++j) { XC[li * 3 + j] = xc[j]; CO[li * 3 + j] = sigmoid(xc[j]); }
                or_decode(FP + li * C, C, w_sigma, w_depth, W_color, alpha[src], d, li, L, near_, far_,
                          mode, &AL[li], &DN[li], CO + li * 3);
            }
            /* ---- composite adjoint: T_l prefix, B_l = back-to-front remainder */
            Tt[0] = 1.0;
            for (int li = 0; li < L; ++li) Tt[li + 1] = Tt[li] * (1.0 - AL[li]);
            for (int j = 0; j < 3; ++j) Bb[(size_t)L * 3 + j] = 0.0;
            for (int li = L - 1; li >= 0; --li)
                for (int j = 0; j < 3; ++j)
                    Bb[li * 3 + j] = AL[li] * CO[li * 3 + j] + (1.0 - AL[li]) * Bb[(li + 1) * 3 + j];
            const double *g = d_rgb ? d_rgb + ((size_t)y * W + x) * 3 : NULL;

            /* ---- per-layer adjoint */
            for (int li = 0; li < L; ++li) {
                size_t src = ((size_t)li * H + y) * W + x;
                double d = depth[src];
                double dal = d_alpha_out ? d_alpha_out[src] : 0.0;
                double ddn = d_depth_out ? d_depth_out[src] : 0.0;
                double dco[3] = {0, 0, 0};
                if (g) {
                    for (int j = 0; j < 3; ++j) {
                        dco[j] = g[j] * Tt[li] * AL[li];
                        dal += g[j] * Tt[li] * (CO[li * 3 + j] - Bb[(li + 1) * 3 + j]);
                    }
                }
                /* decode adjoint */
                double dxc[3], dxs, dxd = 0.0, dd_in = 0.0, da_in = 0.0;
                for (int j = 0; j < 3; ++j) dxc[j] = dco[j] * CO[li * 3 + j] * (1.0 - CO[li * 3 + j]);
                dxs = dal * AL[li] * (1.0 - AL[li]);
                double th = tanh(XD[li]);
                if (mode == 0) {
                    double a = alpha[src];
                    if (a > OR_ALPHA_LO && a < OR_ALPHA_HI) da_in = dxs / (a * (1.0 - a));
                    double disp = 1.0 / d + kap * th;
                    if (disp > 1.0 / far_ && disp < 1.0 / near_) {
                        double ddisp = -ddn * DN[li] * DN[li];
                        dd_in += -ddisp / (d * d);
                        dxd = ddisp * kap * (1.0 - th * th);
                    }
                } else {
                    double ddisp = -ddn * DN[li] * DN[li];
                    dxd = ddisp * kap * (1.0 - th * th);
                }
                for (int c = 0; c < C; ++c) {
                    double fp = FP[li * C + c];
                    dFp[c] = (dF_out ? dF_out[src * C + c] : 0.0) + w_sigma[c] * dxs + w_depth[c] * dxd;
                    for (int j = 0; j < 3; ++j) dFp[c] += W_color[c * 3 + j] * dxc[j];
                    gws[c] += fp * dxs;
                    gwd[c] += fp * dxd;
                    for (int j = 0; j < 3; ++j) gWc[c * 3 + j] += fp * dxc[j];
                }
                /* residual and output projection: F' = F + o W_o */
                for (int c = 0; c < C; ++c) dF[src * C + c] += dFp[c];
                for (int j = 0; j < hd; ++j) {
                    double s = 0.0;
                    for (int c = 0; c < C; ++c) {
                        s += Wo[(size_t)j * C + c] * dFp[c];
                        gWo[(size_t)j * C + c] += O[li * hd + j] * dFp[c];
                    }
                    dO[j] = s;
                }
                /* attention adjoint, per head */
                for (int j = 0; j < hd; ++j) dQ[j] = 0.0;
                for (int hh = 0; hh < heads; ++hh) {
                    const double *pp = Pp + ((size_t)li * heads + hh) * V;
                    double sum_pdp = 0.0;
                    for (int m = 0; m < V; ++m) {
                        double dp = 0.0;
                        for (int j = 0; j < dh; ++j) {
                            dp += dO[hh * dh + j] * Vv[((size_t)li * V + m) * hd + hh * dh + j];
                            dV[(size_t)m * hd + hh * dh + j] = pp[m] * dO[hh * dh + j];
                        }
                        dpv[m] = dp;
                        sum_pdp += pp[m] * dp;
                    }
                    for (int m = 0; m < V; ++m) {
                        double da = pp[m] * (dpv[m] - sum_pdp);
                        for (int j = 0; j < dh; ++j) {
                            dQ[hh * dh + j] += da * Kk[((size_t)li * V + m) * hd + hh * dh + j] * isq;
                            dK[(size_t)m * hd + hh * dh + j] = da * Q[li * hd + hh * dh + j] * isq;
                        }
                    }
                }
                /* query projection and RMSNorm */
                for (int c = 0; c < C; ++c) {
                    double s = 0.0;
                    for (int j = 0; j < hd; ++j) {
                        s += Wq[(size_t)c * hd + j] * dQ[j];
                        gWq[(size_t)c * hd + j] += XN[li * C + c] * dQ[j];
                    }
                    dXN[c] = s;
                }
                double xdx = 0.0;
                for (int c = 0; c < C; ++c) xdx += XN[li * C + c] * dXN[c];
                for (int c = 0; c < C; ++c)
                    dF[src * C + c] += (dXN[c] - XN[li * C + c] * xdx / C) / RR[li];
                /* key / value projections and the gather */
                for (int m = 0; m < V; ++m) {
                    const or_proj *pr = &PR[li * V + m];
                    const double *s = S + ((size_t)li * V + m) * Cf;
                    for (int c = 0; c < Cf; ++c) {
                        double acc = 0.0;
                        for (int j = 0; j < hd; ++j) {
                            acc += Wk[(size_t)c * hd + j] * dK[(size_t)m * hd + j] +
                                   Wv[(size_t)c * hd + j] * dV[(size_t)m * hd + j];
                            gWk[(size_t)c * hd + j] += s[c] * dK[(size_t)m * hd + j];
                            gWv[(size_t)c * hd + j] += s[c] * dV[(size_t)m * hd + j];
                        }
                        dS[c] = acc;
                    }
                    if (!pr->valid) continue;
                    int Hf = feat_hw[2 * m], Wf = feat_hw[2 * m + 1];
                    double X = pr->um - 0.5, Y = pr->vm - 0.5;
                    if (!(fabs(X) < 1e9 && fabs(Y) < 1e9)) continue;
                    double xf = floor(X), yf = floor(Y), fx = X - xf, fy = Y - yf;
                    long x0 = (long)xf, y0 = (long)yf;
                    const double *I00 = tap_ptr(feats[m], Hf, Wf, Cf, x0, y0);
                    const double *I10 = tap_ptr(feats[m], Hf, Wf, Cf, x0 + 1, y0);
                    const double *I01 = tap_ptr(feats[m], Hf, Wf, Cf, x0, y0 + 1);
                    const double *I11 = tap_ptr(feats[m], Hf, Wf, Cf, x0 + 1, y0 + 1);
                    double dX = 0.0, dY = 0.0;
                    for (int c = 0; c < Cf; ++c) {
                        double i00 = I00 ? I00[c] : 0.0, i10 = I10 ? I10[c] : 0.0;
                        double i01 = I01 ? I01[c] : 0.0, i11 = I11 ? I11[c] : 0.0;
                        dX += dS[c] * ((1 - fy) * (i10 - i00) + fy * (i11 - i01));
                        dY += dS[c] * ((1 - fx) * (i01 - i00) + fx * (i11 - i10));
                    }
                    dd_in += dX * pr->dum_dd + dY * pr->dvm_dd;
                    /* scatter into the feature map */
                    const long tx[4] = {x0, x0 + 1, x0, x0 + 1}, ty[4] = {y0, y0, y0 + 1, y0 + 1};
                    const double wt[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
                    for (int t = 0; t < 4; ++t) {
                        if (tx[t] < 0 || tx[t] >= Wf || ty[t] < 0 || ty[t] >= Hf) continue;
                        double *dst = dI[m] + ((size_t)ty[t] * Wf + (size_t)tx[t]) * Cf;
                        for (int c = 0; c < Cf; ++c) {
#pragma omp atomic
                            dst[c] += wt[t] * dS[c];
                        }
                    }
                }
                d_depth[src] += dd_in;
                d_alpha[src] += da_in;
            }
        }
#pragma omp critical
        {
            for (size_t i = 0; i < (size_t)C * hd; ++i) dWq[i] += gWq[i];
            for (size_t i = 0; i < (size_t)Cf * hd; ++i) { dWk[i] += gWk[i]; dWv[i] += gWv[i]; }
            for (size_t i = 0; i < (size_t)hd * C; ++i) dWo[i] += gWo[i];
            for (int c = 0; c < C; ++c) { dw_sigma[c] += gws[c]; dw_depth[c] += gwd[c]; }
            for (int i = 0; i < C * 3; ++i) dW_color[i] += gWc[i];
        }
        free(gWq); free(gWk); free(gWv); free(gWo); free(gws); free(gwd); free(gWc);
        free(S); free(PR); free(XN); free(RR); free(Q); free(Kk); free(Vv); free(Pp); free(O);
        free(FP); free(XS); free(XD); free(XC); free(AL); free(DN); free(CO); free(Tt); free(Bb);
        free(dFp); free(dO); free(dQ); free(dXN); free(dK); free(dV); free(dS); free(dpv);
    }
    (void)nW;
    free(T);
    return 0;
}
