// capi.cpp -- host side of libquark: argument checks, the float64 camera
// composition, launch planning, error reporting.  Declarations and the
// contract of every entry point are in include/quark.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "quark.h"
#include "uf_params.h"

namespace qk {
hipError_t launch_update_fuse(const UFParams &p, int C, int hd, int prec, bool fold, hipStream_t s);
hipError_t launch_update_fuse_batch(const UFParams *reqs, const UFBatch &b, int C, int hd,
                                    int prec, bool fold, hipStream_t s);
hipError_t launch_fp8_scales(const F8Params &p, hipStream_t s);
hipError_t launch_fold_weights(const FoldParams &f, hipStream_t s);
hipError_t launch_composite(const CompParams &p, hipStream_t s);
hipError_t launch_composite_backward(const CompBwdParams &p, hipStream_t s);
hipError_t launch_update_fuse_backward(const BwdParams &p, hipStream_t s);
hipError_t launch_ldm_init(const InitParams &p, bool bf16, hipStream_t s);
hipError_t launch_render_ibr(const RenderParams &p, hipStream_t s);
hipError_t launch_render_to_views(const ViewsParams &p, hipStream_t s);
hipError_t launch_residual_conv(const ConvParams &p, int num_cu, bool frag_ready, hipStream_t s);
hipError_t launch_layer_collapse(const CollapseParams &p, int num_cu, hipStream_t s);
hipError_t launch_ray_encoding(const RayParams &p, hipStream_t s);
hipError_t launch_upsample2x(const Up2Params &p, hipStream_t s);
hipError_t launch_ldm_decode(const DecodeParams &p, hipStream_t s);
hipError_t scratch_address(int device, float **out);
}  // namespace qk

struct qk_context {
    int device;
    int num_cu = 0;
    size_t ws_cap = 0;           // cap on the device workspaces' total bytes (0: none)
    size_t ws_bytes = 0;         // their current total
    float *wfold = nullptr;      // folded-weight workspace (one-to-many form)
    size_t wfold_elems = 0;
    float *bws = nullptr;        // backward workspace: composite adjoint + partials
    size_t bws_elems = 0;
    float *f8 = nullptr;         // e4m3 scales [7] + running maximum [1]
    size_t f8_elems = 0;
    float *vws = nullptr;        // projected planes of the render to input views
    size_t vws_elems = 0;
    float *cfrag = nullptr;      // bfloat16 fragments of the residual block's kernels
    size_t cfrag_elems = 0;
    float *rws = nullptr;        // low-resolution projected ray encodings
    size_t rws_elems = 0;
    float *scratch = nullptr;    // this device's fixed scratch (allocation-free entry point)
    float *bdesc = nullptr;      // batched requests' launch parameters (device)
    size_t bdesc_elems = 0;
    void *bhost = nullptr;       // their pinned host staging
    size_t bhost_bytes = 0;
    hipEvent_t bevent = nullptr; // recorded after the staging copy
    bool bevent_live = false;
    // low-precision copies derived from float32 masters, kept while the
    // caller declares its weights static (qk_context_weights_static)
    struct Derived {
        int kind;                    // kDerivedFold or kDerivedConv
        const void *key[4];          // the masters' device pointers
        int32_t dims[4];
        float *buf;
        size_t elems;
    };
    bool weights_static = false;
    std::vector<Derived> derived;
};

namespace {

thread_local std::string g_err;

qk_status fail(qk_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
qk_status fail(qk_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

// ---- 3x3 helpers (double)
void mat3_mul(const double *A, const double *B, double *Cm) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * r + k] * B[3 * k + c];
            Cm[3 * r + c] = s;
        }
}

// Inverse by the adjugate; returns false when singular.
bool mat3_inv(const double *A, double *Ai) {
    const double a = A[0], b = A[1], c = A[2], d = A[3], e = A[4], f = A[5], g = A[6], h = A[7],
                 i = A[8];
    const double c00 = e * i - f * h, c01 = -(d * i - f * g), c02 = d * h - e * g;
    const double det = a * c00 + b * c01 + c * c02;
    if (!(std::fabs(det) > 1e-300) || !std::isfinite(det)) return false;
    const double id = 1.0 / det;
    Ai[0] = c00 * id;
    Ai[1] = -(b * i - c * h) * id;
    Ai[2] = (b * f - c * e) * id;
    Ai[3] = c01 * id;
    Ai[4] = (a * i - c * g) * id;
    Ai[5] = -(a * f - c * d) * id;
    Ai[6] = c02 * id;
    Ai[7] = -(a * h - b * g) * id;
    Ai[8] = (a * e - b * d) * id;
    return true;
}

qk_status check_camera(const qk_camera *cam, const char *what) {
    if (cam->width <= 0 || cam->height <= 0)
        return fail(QK_ESHAPE, "%s: grid %dx%d must be positive", what, cam->width, cam->height);
    const double *K = cam->K, *E = cam->E;
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(K[k])) return fail(QK_EINVAL, "%s: K not finite", what);
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(E[k])) return fail(QK_EINVAL, "%s: E not finite", what);
    if (K[6] != 0.0 || K[7] != 0.0 || K[8] != 1.0)
        return fail(QK_EINVAL, "%s: K's last row must be (0, 0, 1)", what);
    if (E[12] != 0.0 || E[13] != 0.0 || E[14] != 0.0 || E[15] != 1.0)
        return fail(QK_EINVAL, "%s: E's last row must be (0, 0, 0, 1)", what);
    double Ki[9], M[9], Mi[9];
    if (!mat3_inv(K, Ki)) return fail(QK_EINVAL, "%s: K is singular", what);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = E[4 * r + c];
    if (!mat3_inv(M, Mi)) return fail(QK_EINVAL, "%s: E's 3x3 block is singular", what);
    return QK_OK;
}

// K rescaled from the camera's own grid to a (w1, h1) grid (half-pixel centres).
void scaled_K(const qk_camera *cam, int w1, int h1, double *Ks) {
    const double sx = (double)w1 / cam->width, sy = (double)h1 / cam->height;
    for (int c = 0; c < 3; ++c) {
        Ks[c] = sx * cam->K[c];
        Ks[3 + c] = sy * cam->K[3 + c];
        Ks[6 + c] = cam->K[6 + c];
    }
}

// A = K_m M_m M_n^-1 K_n^-1 and b = K_m (t_m - M_m M_n^-1 t_n), where E = [M | t]
// (M is the rotation R for rigid cameras).  Composed in double.
void compose_table(const qk_camera *nov, int W, int H, const qk_camera *cam, int fw, int fh,
                   double *out12) {
    double Kn[9], Km[9], Kni[9], Mn[9], Mni[9], Mm[9], tn[3], tm[3];
    scaled_K(nov, W, H, Kn);
    scaled_K(cam, fw, fh, Km);
    mat3_inv(Kn, Kni);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            Mn[3 * r + c] = nov->E[4 * r + c];
            Mm[3 * r + c] = cam->E[4 * r + c];
        }
        tn[r] = nov->E[4 * r + 3];
        tm[r] = cam->E[4 * r + 3];
    }
    mat3_inv(Mn, Mni);
    double R[9], KR[9], A[9];
    mat3_mul(Mm, Mni, R);      // novel camera frame -> camera m frame (rotation part)
    mat3_mul(Km, R, KR);
    mat3_mul(KR, Kni, A);
    double tr[3];
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += R[3 * r + k] * tn[k];
        tr[r] = tm[r] - s;
    }
    for (int k = 0; k < 9; ++k) out12[k] = A[k];
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += Km[3 * r + k] * tr[k];
        out12[9 + r] = s;
    }
}

bool supported_c(int C) { return C == 8 || C == 16 || C == 32 || C == 64; }

qk_status check_update_fuse(int32_t V, const qk_camera *in_cams, const qk_feature_map *feats,
                            const qk_camera *novel, float near_, float far_, const qk_weights *w,
                            qk_precision precision, qk_attn_form attn_form,
                            qk_update_mode update_mode, const qk_ldm *in, const qk_ldm *out,
                            float *rgb_out, float *acc_out, float *blend_out) {
    if (!in_cams || !feats || !novel || !w || !in || !out)
        return fail(QK_EINVAL, "NULL argument");
    if (V < 1 || V > qk::kMaxViews)
        return fail(QK_ESHAPE, "V = %d outside 1..%d", V, qk::kMaxViews);
    if (precision != QK_PREC_FP32 && precision != QK_PREC_BF16 && precision != QK_PREC_BF16_FP8PROJ)
        return fail(QK_EINVAL, "unknown precision %d", (int)precision);
    if (attn_form != QK_ATTN_STANDARD && attn_form != QK_ATTN_FOLDED)
        return fail(QK_EINVAL, "unknown attention form %d", (int)attn_form);
    if (update_mode != QK_UPDATE_RESIDUAL && update_mode != QK_UPDATE_PAPER_DECODE)
        return fail(QK_EINVAL, "unknown update mode %d", (int)update_mode);
    if (!(near_ > 0.0f) || !(far_ > near_) || !std::isfinite(far_))
        return fail(QK_EINVAL, "need 0 < near < far (got %g, %g)", near_, far_);
    if (in->L < 1 || in->H < 1 || in->W < 1 || in->C < 1)
        return fail(QK_ESHAPE, "LDM dims must be positive (L=%d H=%d W=%d C=%d)", in->L, in->H,
                    in->W, in->C);
    if (out->L != in->L || out->H != in->H || out->W != in->W ||
        (out->F != nullptr && out->C != in->C))
        return fail(QK_ESHAPE, "ldm_out dims differ from ldm_in");
    if (in->dtype != QK_F32 && in->dtype != QK_BF16)
        return fail(QK_EDTYPE, "unknown LDM dtype %d", (int)in->dtype);
    if (out->F != nullptr && out->dtype != in->dtype)
        return fail(QK_EDTYPE, "ldm_out dtype differs from ldm_in");
    const qk_dtype need = precision == QK_PREC_FP32 ? QK_F32 : QK_BF16;
    if (in->dtype != need)
        return fail(QK_EDTYPE, "precision %d needs LDM/feature dtype %d", (int)precision, (int)need);
    if (!in->F || !in->depth || !in->alpha || !out->depth || !out->alpha)
        return fail(QK_EINVAL, "NULL LDM buffer");
    if (!w->Wq || !w->Wk || !w->Wv || !w->Wo || !w->w_sigma || !w->w_depth || !w->W_color)
        return fail(QK_EINVAL, "NULL weight buffer");
    if (w->C != in->C) return fail(QK_ESHAPE, "weights.C %d != LDM C %d", w->C, in->C);
    if (w->C_feat < 1 || w->heads < 1 || w->head_dim < 1)
        return fail(QK_ESHAPE, "weights dims must be positive");
    if (!aligned16(in->F) || (out->F && !aligned16(out->F)))
        return fail(QK_EINVAL, "LDM feature buffers must be 16-byte aligned");
    if (!aligned4(in->depth) || !aligned4(in->alpha) || !aligned4(out->depth) ||
        !aligned4(out->alpha) || (rgb_out && !aligned4(rgb_out)) || (acc_out && !aligned4(acc_out)))
        return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    if (acc_out && !rgb_out) return fail(QK_EINVAL, "acc_alpha_out needs rgb_out");
    if (blend_out && !aligned4(blend_out)) return fail(QK_EINVAL, "blend_logit_out must be 4-byte aligned");
    if (blend_out && (w->heads != 1 || w->head_dim != in->C))
        return fail(QK_EUNSUPPORTED, "blend_logit_out needs one attention head (got %d)", w->heads);
    if (blend_out && (int64_t)in->L * in->H * in->W * V >= ((int64_t)1 << 40))
        return fail(QK_EUNSUPPORTED, "blend logits too large");
    const int64_t elems = (int64_t)in->L * in->H * in->W * in->C;
    if (elems >= (int64_t)1 << 31)
        return fail(QK_EUNSUPPORTED, "LDM of %lld elements exceeds 2^31", (long long)elems);
    qk_status st = check_camera(novel, "novel camera");
    if (st != QK_OK) return st;
    for (int m = 0; m < V; ++m) {
        char what[32];
        snprintf(what, sizeof(what), "camera %d", m);
        st = check_camera(&in_cams[m], what);
        if (st != QK_OK) return st;
        if (!feats[m].data) return fail(QK_EINVAL, "feature map %d is NULL", m);
        if (!aligned16(feats[m].data))
            return fail(QK_EINVAL, "feature map %d must be 16-byte aligned", m);
        if (feats[m].H < 1 || feats[m].W < 1)
            return fail(QK_ESHAPE, "feature map %d has grid %dx%d", m, feats[m].W, feats[m].H);
        if (feats[m].dtype != need)
            return fail(QK_EDTYPE, "feature map %d has dtype %d, precision %d needs %d", m,
                        (int)feats[m].dtype, (int)precision, (int)need);
        if (feats[m].C != w->C_feat)
            return fail(QK_ESHAPE, "feature map %d has C = %d, the weights' C_feat is %d", m,
                        feats[m].C, w->C_feat);
        // the gather addresses a map as one buffer with 32-bit byte offsets
        const int64_t fbytes = (int64_t)feats[m].H * feats[m].W * w->C_feat *
                               (precision == QK_PREC_FP32 ? 4 : 2);
        if (fbytes >= (int64_t)1 << 30)
            return fail(QK_EUNSUPPORTED, "feature map %d is %lld bytes; maps must be under 1 GiB", m,
                        (long long)fbytes);
    }
    if (w->C_feat != in->C || !supported_c(in->C))
        return fail(QK_EUNSUPPORTED, "kernels support C == C_feat in {8,16,32,64} (got C=%d C_feat=%d)",
                    in->C, w->C_feat);
    if (w->heads != 1 || w->head_dim != in->C) {
        // several heads: C >= 32, heads x head_dim == C, head_dim 8 (C = 32)
        // or 16 or 32; the folded form not with e4m3 projections
        const bool ok = in->C >= 32 && w->heads * w->head_dim == in->C &&
                        ((w->head_dim == 8 && in->C == 32) || w->head_dim == 16 || w->head_dim == 32) &&
                        !(attn_form == QK_ATTN_FOLDED &&
                          (precision == QK_PREC_BF16_FP8PROJ || in->C != 32));
        if (!ok)
            return fail(QK_EUNSUPPORTED,
                        "kernels support one head of C channels, or for C >= 32 heads x head_dim "
                        "== C with head_dim 16, 32 (or 8 at C = 32), the folded form of several "
                        "heads at C = 32 without e4m3 projections "
                        "(got heads=%d head_dim=%d C=%d, %s form)",
                        w->heads, w->head_dim, in->C,
                        attn_form == QK_ATTN_FOLDED ? "folded" : "standard");
    }
    return QK_OK;
}


bool supported_backward_c(int C) { return C == 8 || C == 16; }

bool same_grid(const qk_ldm *a, const qk_ldm *b) {
    return a->L == b->L && a->H == b->H && a->W == b->W;
}

qk_status check_backward(int32_t V, const qk_camera *in_cams, const qk_feature_map *feats,
                         const qk_camera *novel, float near_, float far_, const qk_weights *w,
                         qk_update_mode update_mode, const qk_ldm *in, const qk_ldm *out,
                         const float *d_rgb, const qk_ldm *d_out, const qk_ldm *d_in,
                         float *const *d_feats, const qk_weight_grads *dw) {
    if (!in_cams || !feats || !novel || !w || !in || !d_in || !d_feats || !dw)
        return fail(QK_EINVAL, "NULL argument");
    if (d_rgb && !out) return fail(QK_EINVAL, "d_rgb needs ldm_out (F' and alpha')");
    if (V < 1 || V > qk::kMaxViews)
        return fail(QK_ESHAPE, "V = %d outside 1..%d", V, qk::kMaxViews);
    if (update_mode != QK_UPDATE_RESIDUAL && update_mode != QK_UPDATE_PAPER_DECODE)
        return fail(QK_EINVAL, "unknown update mode %d", (int)update_mode);
    if (!(near_ > 0.0f) || !(far_ > near_) || !std::isfinite(far_))
        return fail(QK_EINVAL, "need 0 < near < far (got %g, %g)", near_, far_);
    if (in->L < 1 || in->H < 1 || in->W < 1 || in->C < 1)
        return fail(QK_ESHAPE, "LDM dims must be positive (L=%d H=%d W=%d C=%d)", in->L, in->H,
                    in->W, in->C);
    if (in->dtype != QK_F32) return fail(QK_EDTYPE, "the backward pass takes float32 LDMs");
    if (!in->F || !in->depth || !in->alpha) return fail(QK_EINVAL, "NULL LDM buffer");
    if (d_rgb) {
        if (!same_grid(out, in) || out->C != in->C) return fail(QK_ESHAPE, "ldm_out dims differ from ldm_in");
        if (out->dtype != QK_F32) return fail(QK_EDTYPE, "ldm_out must be float32");
        if (!out->F || !out->alpha) return fail(QK_EINVAL, "d_rgb needs ldm_out F' and alpha'");
        if (!aligned16(out->F) || !aligned4(out->alpha) || !aligned4(d_rgb))
            return fail(QK_EINVAL, "ldm_out / d_rgb misaligned");
    }
    if (d_out) {
        if (!same_grid(d_out, in)) return fail(QK_ESHAPE, "d_out dims differ from ldm_in");
        if (d_out->F && (d_out->C != in->C || d_out->dtype != QK_F32))
            return fail(QK_ESHAPE, "d_out F must be float32 with C channels");
        if ((d_out->F && !aligned16(d_out->F)) || (d_out->depth && !aligned4(d_out->depth)) ||
            (d_out->alpha && !aligned4(d_out->alpha)))
            return fail(QK_EINVAL, "d_out misaligned");
    }
    if (!same_grid(d_in, in) || d_in->C != in->C) return fail(QK_ESHAPE, "d_in dims differ from ldm_in");
    if (d_in->dtype != QK_F32) return fail(QK_EDTYPE, "d_in must be float32");
    if (!d_in->F || !d_in->depth || !d_in->alpha) return fail(QK_EINVAL, "NULL d_in buffer");
    if (!aligned16(in->F) || !aligned16(d_in->F))
        return fail(QK_EINVAL, "LDM feature buffers must be 16-byte aligned");
    if (!aligned4(in->depth) || !aligned4(in->alpha) || !aligned4(d_in->depth) ||
        !aligned4(d_in->alpha))
        return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    if (!w->Wq || !w->Wk || !w->Wv || !w->Wo || !w->w_sigma || !w->w_depth || !w->W_color)
        return fail(QK_EINVAL, "NULL weight buffer");
    if (!dw->Wq || !dw->Wk || !dw->Wv || !dw->Wo || !dw->w_sigma || !dw->w_depth || !dw->W_color)
        return fail(QK_EINVAL, "NULL weight-gradient buffer");
    if (w->C != in->C) return fail(QK_ESHAPE, "weights.C %d != LDM C %d", w->C, in->C);
    const int64_t elems = (int64_t)in->L * in->H * in->W * in->C;
    if (elems >= (int64_t)1 << 31)
        return fail(QK_EUNSUPPORTED, "LDM of %lld elements exceeds 2^31", (long long)elems);
    qk_status st = check_camera(novel, "novel camera");
    if (st != QK_OK) return st;
    for (int m = 0; m < V; ++m) {
        char what[32];
        snprintf(what, sizeof(what), "camera %d", m);
        st = check_camera(&in_cams[m], what);
        if (st != QK_OK) return st;
        if (!feats[m].data || !d_feats[m]) return fail(QK_EINVAL, "feature map %d is NULL", m);
        if (!aligned16(feats[m].data) || !aligned16(d_feats[m]))
            return fail(QK_EINVAL, "feature map %d must be 16-byte aligned", m);
        if (feats[m].H < 1 || feats[m].W < 1)
            return fail(QK_ESHAPE, "feature map %d has grid %dx%d", m, feats[m].W, feats[m].H);
        if (feats[m].dtype != QK_F32)
            return fail(QK_EDTYPE, "feature map %d has dtype %d; the backward takes float32", m,
                        (int)feats[m].dtype);
        if (feats[m].C != w->C_feat)
            return fail(QK_ESHAPE, "feature map %d has C = %d, the weights' C_feat is %d", m,
                        feats[m].C, w->C_feat);
        if ((int64_t)feats[m].H * feats[m].W * w->C_feat >= (int64_t)1 << 31)
            return fail(QK_EUNSUPPORTED, "feature map %d exceeds 2^31 elements", m);
    }
    if (w->heads != 1 || w->head_dim != in->C || w->C_feat != in->C || !supported_backward_c(in->C))
        return fail(QK_EUNSUPPORTED,
                    "the backward kernels support heads == 1 and C == C_feat == head_dim in "
                    "{8,16} (got heads=%d head_dim=%d C=%d C_feat=%d)",
                    w->heads, w->head_dim, in->C, w->C_feat);
    return QK_OK;
}

// Grow a context buffer to at least `need` floats (synchronising the stream
// before a buffer in use is replaced).
// Grow one of the context's device workspaces to `need` floats (never
// shrinks), within the context's cap on their total.
qk_status grow(qk_context *ctx, float **buf, size_t *have, size_t need, hipStream_t stream) {
    if (*have >= need) return QK_OK;
    const size_t total = ctx->ws_bytes - *have * sizeof(float) + need * sizeof(float);
    if (ctx->ws_cap != 0 && total > ctx->ws_cap)
        return fail(QK_ENOMEM, "workspace of %zu bytes in all would pass the context's cap of %zu",
                    total, ctx->ws_cap);
    if (*buf) {
        hipError_t se = hipStreamSynchronize(stream);
        if (se != hipSuccess) return fail(QK_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(se));
        (void)hipFree(*buf);
        *buf = nullptr;
        ctx->ws_bytes -= *have * sizeof(float);
        *have = 0;
    }
    if (hipMalloc(buf, need * sizeof(float)) != hipSuccess) {
        *buf = nullptr;
        return fail(QK_ENOMEM, "workspace of %zu floats", need);
    }
    *have = need;
    ctx->ws_bytes += need * sizeof(float);
    return QK_OK;
}

// Derived weights (qk_context_weights_static): the folded attention weights
// of the one-to-many form and the residual block's bfloat16 fragments.
constexpr int kDerivedFold = 0, kDerivedConv = 1;
constexpr size_t kDerivedMax = 64;     // entries a context keeps; beyond, derived per call

// The cached copy for these masters, or NULL.
float *derived_find(qk_context *ctx, int kind, const void *const key[4], const int32_t dims[4]) {
    for (const auto &d : ctx->derived)
        if (d.kind == kind && std::equal(d.key, d.key + 4, key) && std::equal(d.dims, d.dims + 4, dims))
            return d.buf;
    return nullptr;
}

// A new entry of `elems` floats, counted against the workspace cap; *out is
// NULL (and the status QK_OK) when the context keeps no more entries.
qk_status derived_add(qk_context *ctx, int kind, const void *const key[4], const int32_t dims[4],
                      size_t elems, float **out) {
    *out = nullptr;
    if (ctx->derived.size() >= kDerivedMax) return QK_OK;
    const size_t total = ctx->ws_bytes + elems * sizeof(float);
    if (ctx->ws_cap != 0 && total > ctx->ws_cap)
        return fail(QK_ENOMEM, "workspace of %zu bytes in all would pass the context's cap of %zu",
                    total, ctx->ws_cap);
    float *buf = nullptr;
    if (hipMalloc(&buf, elems * sizeof(float)) != hipSuccess)
        return fail(QK_ENOMEM, "derived weights of %zu floats", elems);
    qk_context::Derived d;
    d.kind = kind;
    std::copy(key, key + 4, d.key);
    std::copy(dims, dims + 4, d.dims);
    d.buf = buf;
    d.elems = elems;
    ctx->derived.push_back(d);
    ctx->ws_bytes += elems * sizeof(float);
    *out = buf;
    return QK_OK;
}

// Frees every cached copy; the device is synchronised first (enqueued work
// may still read them).
qk_status derived_clear(qk_context *ctx) {
    if (ctx->derived.empty()) return QK_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(QK_EHIP, "hipDeviceSynchronize: %s", hipGetErrorString(e));
    for (const auto &d : ctx->derived) {
        (void)hipFree(d.buf);
        ctx->ws_bytes -= d.elems * sizeof(float);
    }
    ctx->derived.clear();
    return QK_OK;
}

// The folded weights W_qk, W_vo of w: from the cache when the context's
// weights are static (derived on first use, the stream then synchronised
// so every later call, on any stream, reads a complete copy), else into
// `dst` (2 per floats) on the caller's stream.
qk_status fold_weights(qk_context *ctx, const qk_weights *w, float *dst, hipStream_t stream,
                       float **wqk, float **wvo) {
    const size_t per = (size_t)w->heads * w->C * w->C_feat;
    float *wf = nullptr;
    bool fresh = true;
    if (ctx->weights_static) {
        const void *key[4] = {w->Wq, w->Wk, w->Wv, w->Wo};
        const int32_t dims[4] = {w->C, w->C_feat, w->heads, w->head_dim};
        wf = derived_find(ctx, kDerivedFold, key, dims);
        fresh = wf == nullptr;
        if (fresh) {
            qk_status st = derived_add(ctx, kDerivedFold, key, dims, 2 * per, &wf);
            if (st != QK_OK) return st;
        }
    }
    const bool cached = wf != nullptr;
    if (!cached) wf = dst;
    if (fresh) {
        qk::FoldParams fp{w->Wq, w->Wk, w->Wv, w->Wo, wf, wf + per, w->C, w->C_feat,
                          w->head_dim, w->heads, 1.0f / std::sqrt((float)w->head_dim)};
        hipError_t fe = qk::launch_fold_weights(fp, stream);
        if (fe != hipSuccess) return fail(QK_EHIP, "fold launch: %s", hipGetErrorString(fe));
        if (cached) {
            fe = hipStreamSynchronize(stream);
            if (fe != hipSuccess) return fail(QK_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(fe));
        }
    }
    *wqk = wf;
    *wvo = wf + per;
    return QK_OK;
}

qk_status check_render(int32_t V, const qk_camera *in_cams, const qk_image *images,
                       const qk_camera *novel, float near_, float far_, const qk_ldm_logits *lg,
                       int32_t H, int32_t W, const float *rgb_out, const float *acc_out,
                       const float *depth_out) {
    if (!in_cams || !images || !novel || !lg) return fail(QK_EINVAL, "NULL argument");
    if (V < 1 || V > qk::kMaxViews)
        return fail(QK_ESHAPE, "V = %d outside 1..%d", V, qk::kMaxViews);
    if (!(near_ > 0.0f) || !(far_ > near_) || !std::isfinite(far_))
        return fail(QK_EINVAL, "need 0 < near < far (got %g, %g)", near_, far_);
    if (lg->L < 1 || lg->H < 1 || lg->W < 1 || H < 1 || W < 1)
        return fail(QK_ESHAPE, "dims must be positive (L=%d h=%d w=%d H=%d W=%d)", lg->L, lg->H,
                    lg->W, H, W);
    if (lg->V != V) return fail(QK_ESHAPE, "blend logits have %d views, V = %d", lg->V, V);
    if ((int64_t)lg->L * lg->H * lg->W * V >= ((int64_t)1 << 31) ||
        (int64_t)H * W * 3 >= ((int64_t)1 << 31))
        return fail(QK_EUNSUPPORTED, "logit volume or output of 2^31 elements or more");
    if (!lg->depth_logit || !lg->sigma_logit || !lg->blend_logit || !rgb_out)
        return fail(QK_EINVAL, "NULL buffer");
    if (!aligned4(lg->depth_logit) || !aligned4(lg->sigma_logit) || !aligned4(lg->blend_logit) ||
        !aligned4(rgb_out) || (acc_out && !aligned4(acc_out)) ||
        (depth_out && !aligned4(depth_out)))
        return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    qk_status st = check_camera(novel, "novel camera");
    if (st != QK_OK) return st;
    for (int m = 0; m < V; ++m) {
        char what[32];
        snprintf(what, sizeof(what), "camera %d", m);
        st = check_camera(&in_cams[m], what);
        if (st != QK_OK) return st;
        if (!images[m].data) return fail(QK_EINVAL, "image %d is NULL", m);
        if (!aligned4(images[m].data)) return fail(QK_EINVAL, "image %d must be 4-byte aligned", m);
        if (images[m].H < 1 || images[m].W < 1)
            return fail(QK_ESHAPE, "image %d has grid %dx%d", m, images[m].W, images[m].H);
        if ((int64_t)images[m].H * images[m].W * 4 >= ((int64_t)1 << 30))
            return fail(QK_EUNSUPPORTED, "image %d is 1 GiB or more", m);
    }
    return QK_OK;
}

qk_status check_views(int32_t V, const qk_camera *in_cams, const qk_camera *novel,
                      const qk_ldm_decoded *ldm, const qk_view_image *views, int64_t *ws_floats) {
    if (!in_cams || !novel || !ldm || !views) return fail(QK_EINVAL, "NULL argument");
    if (V < 1 || V > qk::kMaxViews)
        return fail(QK_ESHAPE, "V = %d outside 1..%d", V, qk::kMaxViews);
    if (ldm->L < 1 || ldm->H < 1 || ldm->W < 1)
        return fail(QK_ESHAPE, "LDM dims must be positive (L=%d H=%d W=%d)", ldm->L, ldm->H,
                    ldm->W);
    if ((int64_t)ldm->L * ldm->H * ldm->W * 3 >= ((int64_t)1 << 31))
        return fail(QK_EUNSUPPORTED, "LDM of 2^31 elements or more");
    if (!ldm->depth || !ldm->alpha || !ldm->color) return fail(QK_EINVAL, "NULL LDM buffer");
    if (!aligned4(ldm->depth) || !aligned4(ldm->alpha) || !aligned4(ldm->color))
        return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    qk_status st = check_camera(novel, "novel camera");
    if (st != QK_OK) return st;
    int64_t total = 0;
    for (int m = 0; m < V; ++m) {
        char what[32];
        snprintf(what, sizeof(what), "camera %d", m);
        st = check_camera(&in_cams[m], what);
        if (st != QK_OK) return st;
        if (views[m].H < 1 || views[m].W < 1)
            return fail(QK_ESHAPE, "view %d has grid %dx%d", m, views[m].W, views[m].H);
        if (!views[m].rgb) return fail(QK_EINVAL, "view %d rgb is NULL", m);
        if (!aligned4(views[m].rgb) || (views[m].acc && !aligned4(views[m].acc)))
            return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
        total += (int64_t)ldm->L * views[m].H * views[m].W * 4;
        if (total >= ((int64_t)1 << 31))
            return fail(QK_EUNSUPPORTED, "projected planes of 2^31 floats or more");
    }
    if (ws_floats) *ws_floats = total;
    return QK_OK;
}

qk_status check_conv(const qk_ldm *in, const float *W1, const float *W2, const qk_ldm *out) {
    if (!in || !out || !W1 || !W2) return fail(QK_EINVAL, "NULL argument");
    if (in->L < 1 || in->H < 1 || in->W < 1)
        return fail(QK_ESHAPE, "LDM dims must be positive (L=%d H=%d W=%d)", in->L, in->H, in->W);
    if (in->C != 32) return fail(QK_EUNSUPPORTED, "the residual block supports C = 32 (got %d)", in->C);
    if (in->dtype != QK_BF16 || out->dtype != QK_BF16)
        return fail(QK_EDTYPE, "the residual block takes bfloat16 feature volumes");
    if (out->L != in->L || out->H != in->H || out->W != in->W || out->C != in->C)
        return fail(QK_ESHAPE, "ldm_out dims differ from ldm_in");
    if (!in->F || !out->F) return fail(QK_EINVAL, "NULL feature volume");
    if (!aligned16(in->F) || !aligned16(out->F))
        return fail(QK_EINVAL, "feature volumes must be 16-byte aligned");
    if (!aligned4(W1) || !aligned4(W2)) return fail(QK_EINVAL, "weights must be 4-byte aligned");
    const int64_t elems = (int64_t)in->L * in->H * in->W * in->C;
    if (elems >= ((int64_t)1 << 40)) return fail(QK_EUNSUPPORTED, "feature volume too large");
    const char *a = static_cast<const char *>(in->F), *b = static_cast<const char *>(out->F);
    const int64_t bytes = elems * 2;
    if (a < b + bytes && b < a + bytes)
        return fail(QK_EINVAL, "ldm_out must not overlap ldm_in (tiles read their neighbours)");
    return QK_OK;
}

qk_status check_ray(int32_t V, const qk_camera *in_cams, const qk_camera *novel, float near_,
                    float far_, const float *Wr, int32_t C, qk_dtype dtype, int32_t low_H,
                    int32_t low_W, const qk_feature_map_inout *feats) {
    if (!in_cams || !novel || !Wr || !feats) return fail(QK_EINVAL, "NULL argument");
    if (V < 1 || V > qk::kMaxViews)
        return fail(QK_ESHAPE, "V = %d outside 1..%d", V, qk::kMaxViews);
    if (!(near_ > 0.0f) || !(far_ > near_) || !std::isfinite(far_))
        return fail(QK_EINVAL, "need 0 < near < far (got %g, %g)", near_, far_);
    if (!supported_c(C)) return fail(QK_EUNSUPPORTED, "C = %d not in {8, 16, 32, 64}", C);
    if (dtype != QK_F32 && dtype != QK_BF16) return fail(QK_EDTYPE, "unknown dtype %d", (int)dtype);
    if (!aligned16(Wr)) return fail(QK_EINVAL, "Wr must be 16-byte aligned");
    if (low_H < 0 || low_W < 0 || (low_H == 0) != (low_W == 0))
        return fail(QK_ESHAPE, "low-resolution grid %dx%d: both positive, or both 0", low_W, low_H);
    if ((int64_t)V * low_H * low_W * C >= ((int64_t)1 << 31))
        return fail(QK_EUNSUPPORTED, "low-resolution encodings of 2^31 floats or more");
    qk_status st = check_camera(novel, "novel camera");
    if (st != QK_OK) return st;
    const int64_t esize = dtype == QK_BF16 ? 2 : 4;
    for (int m = 0; m < V; ++m) {
        char what[32];
        snprintf(what, sizeof(what), "camera %d", m);
        st = check_camera(&in_cams[m], what);
        if (st != QK_OK) return st;
        if (feats[m].H < 1 || feats[m].W < 1)
            return fail(QK_ESHAPE, "feature map %d has grid %dx%d", m, feats[m].W, feats[m].H);
        if (!feats[m].data) return fail(QK_EINVAL, "feature map %d is NULL", m);
        if (!aligned16(feats[m].data))
            return fail(QK_EINVAL, "feature map %d must be 16-byte aligned", m);
        if ((int64_t)feats[m].H * feats[m].W * C >= ((int64_t)1 << 40))
            return fail(QK_EUNSUPPORTED, "feature map %d too large", m);
        if (feats[m].src && !aligned16(feats[m].src))
            return fail(QK_EINVAL, "source map %d must be 16-byte aligned", m);
    }
    // each map is written by its own threads: two views sharing memory would
    // race, and so would a source map that overlaps a map being written
    // (other than its own, read and written in place)
    for (int a = 0; a < V; ++a) {
        const int64_t na = (int64_t)feats[a].H * feats[a].W * C * esize;
        const char *pa = static_cast<const char *>(feats[a].data);
        for (int b = a + 1; b < V; ++b) {
            const char *pb = static_cast<const char *>(feats[b].data);
            const int64_t nb = (int64_t)feats[b].H * feats[b].W * C * esize;
            if (pa < pb + nb && pb < pa + na)
                return fail(QK_EINVAL, "feature maps %d and %d overlap", a, b);
        }
        const char *sa = static_cast<const char *>(feats[a].src);
        if (!sa || sa == pa) continue;
        for (int b = 0; b < V; ++b) {
            const char *pb = static_cast<const char *>(feats[b].data);
            const int64_t nb = (int64_t)feats[b].H * feats[b].W * C * esize;
            if (sa < pb + nb && pb < sa + na)
                return fail(QK_EINVAL, "source map %d overlaps feature map %d", a, b);
        }
    }
    return QK_OK;
}

qk_status check_upsample2x(const void *src, void *dst, int32_t N, int32_t H, int32_t W, int32_t C,
                           qk_dtype dtype) {
    if (!src || !dst) return fail(QK_EINVAL, "NULL argument");
    if (N < 1 || H < 1 || W < 1 || C < 1)
        return fail(QK_ESHAPE, "dims must be positive (N=%d H=%d W=%d C=%d)", N, H, W, C);
    if (dtype != QK_F32 && dtype != QK_BF16) return fail(QK_EDTYPE, "unknown dtype %d", (int)dtype);
    const int64_t e = dtype == QK_BF16 ? 2 : 4;
    const int64_t n_in = (int64_t)N * H * W * C;
    if (n_in >= ((int64_t)1 << 38)) return fail(QK_EUNSUPPORTED, "volume too large");
    const uintptr_t need = C % 8 == 0 ? 16 : (uintptr_t)e;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & (need - 1))
        return fail(QK_EINVAL, "buffers must be %d-byte aligned", (int)need);
    const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
    if (a < b + 4 * n_in * e && b < a + n_in * e)
        return fail(QK_EINVAL, "dst must not overlap src");
    return QK_OK;
}

qk_status check_decode(const qk_ldm *ldm, const float *w_sigma, const float *w_depth,
                       const float *W_color, float near_, float far_, const float *color_out) {
    if (!ldm || !w_sigma || !w_depth || !W_color) return fail(QK_EINVAL, "NULL argument");
    if (ldm->L < 1 || ldm->H < 1 || ldm->W < 1)
        return fail(QK_ESHAPE, "LDM dims must be positive (L=%d H=%d W=%d)", ldm->L, ldm->H, ldm->W);
    if (!supported_c(ldm->C)) return fail(QK_EUNSUPPORTED, "C = %d not in {8, 16, 32, 64}", ldm->C);
    if (ldm->dtype != QK_F32 && ldm->dtype != QK_BF16)
        return fail(QK_EDTYPE, "unknown dtype %d", (int)ldm->dtype);
    if (!(near_ > 0.0f) || !(far_ > near_) || !std::isfinite(far_))
        return fail(QK_EINVAL, "need 0 < near < far (got %g, %g)", near_, far_);
    if (!ldm->F || !ldm->depth || !ldm->alpha) return fail(QK_EINVAL, "NULL LDM buffer");
    if (!aligned16(ldm->F)) return fail(QK_EINVAL, "the feature volume must be 16-byte aligned");
    if (!aligned4(ldm->depth) || !aligned4(ldm->alpha) || (color_out && !aligned4(color_out)) ||
        !aligned4(w_sigma) || !aligned4(w_depth) || !aligned4(W_color))
        return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    if ((int64_t)ldm->L * ldm->H * ldm->W * ldm->C >= ((int64_t)1 << 38))
        return fail(QK_EUNSUPPORTED, "LDM too large");
    return QK_OK;
}

qk_status check_collapse(const qk_ldm *in, const float *W1, const float *W2, const qk_ldm *out) {
    if (!in || !out || !W1 || !W2) return fail(QK_EINVAL, "NULL argument");
    if (in->L < 2 || in->H < 1 || in->W < 1)
        return fail(QK_ESHAPE, "need L >= 2 and positive H, W (L=%d H=%d W=%d)", in->L, in->H, in->W);
    if (in->L % 2 != 0) return fail(QK_ESHAPE, "layer collapse needs an even L (got %d)", in->L);
    if (in->C != 32) return fail(QK_EUNSUPPORTED, "layer collapse supports C = 32 (got %d)", in->C);
    if (in->dtype != QK_BF16 || out->dtype != QK_BF16)
        return fail(QK_EDTYPE, "layer collapse takes bfloat16 feature volumes");
    if (out->L != in->L / 2 || out->H != in->H || out->W != in->W || out->C != in->C)
        return fail(QK_ESHAPE, "ldm_out must be [L/2][H][W][C] of ldm_in");
    if (!in->F || !out->F) return fail(QK_EINVAL, "NULL feature volume");
    if (!aligned16(in->F) || !aligned16(out->F))
        return fail(QK_EINVAL, "feature volumes must be 16-byte aligned");
    if (!aligned4(W1) || !aligned4(W2)) return fail(QK_EINVAL, "weights must be 4-byte aligned");
    const int64_t bin = (int64_t)in->L * in->H * in->W * in->C * 2;
    const char *a = static_cast<const char *>(in->F), *b = static_cast<const char *>(out->F);
    if (a < b + bin / 2 && b < a + bin)
        return fail(QK_EINVAL, "ldm_out must not overlap ldm_in");
    return QK_OK;
}

}  // namespace

extern "C" {

const char *qk_last_error(void) { return g_err.c_str(); }

const char *qk_version(void) { return "libquark 0.1.0 gfx950"; }

qk_status qk_context_create(int device, size_t workspace_bytes, qk_context **out) {
    if (!out) return fail(QK_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(QK_EHIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(QK_EINVAL, "device %d of %d", device, n);
    int cu = 0;
    e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return fail(QK_EHIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    // the device's fixed scratch (a static device array), looked up once
    float *scr = nullptr;
    e = qk::scratch_address(device, &scr);
    if (e != hipSuccess) return fail(QK_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    qk_context *ctx = new qk_context{device};
    ctx->num_cu = cu > 0 ? cu : 1;
    ctx->ws_cap = workspace_bytes;
    ctx->scratch = scr;
    *out = ctx;
    return QK_OK;
}

qk_status qk_context_destroy(qk_context *ctx) {
    if (ctx && (ctx->wfold || ctx->bws || ctx->f8 || ctx->vws || ctx->cfrag || ctx->rws ||
                ctx->bdesc || ctx->bhost || ctx->bevent || !ctx->derived.empty())) {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != ctx->device) (void)hipSetDevice(ctx->device);
        (void)derived_clear(ctx);
        if (ctx->wfold) (void)hipFree(ctx->wfold);
        if (ctx->bws) (void)hipFree(ctx->bws);
        if (ctx->f8) (void)hipFree(ctx->f8);
        if (ctx->vws) (void)hipFree(ctx->vws);
        if (ctx->cfrag) (void)hipFree(ctx->cfrag);
        if (ctx->rws) (void)hipFree(ctx->rws);
        if (ctx->bevent) (void)hipEventSynchronize(ctx->bevent);
        if (ctx->bdesc) (void)hipFree(ctx->bdesc);
        if (ctx->bhost) (void)hipHostFree(ctx->bhost);
        if (ctx->bevent) (void)hipEventDestroy(ctx->bevent);
        if (cur >= 0 && cur != ctx->device) (void)hipSetDevice(cur);
    }
    delete ctx;
    return QK_OK;
}

qk_status qk_context_weights_static(qk_context *ctx, int enable) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    qk_status st = derived_clear(ctx);
    if (cur != ctx->device) (void)hipSetDevice(cur);
    if (st != QK_OK) return st;
    ctx->weights_static = enable != 0;
    return QK_OK;
}

qk_status qk_camera_tables(int32_t V, const qk_camera *in_cams, const int32_t *feat_hw,
                           const qk_camera *novel, int32_t H, int32_t W, double *out) {
    if (!in_cams || !feat_hw || !novel || !out) return fail(QK_EINVAL, "NULL argument");
    if (V < 1 || V > qk::kMaxViews) return fail(QK_ESHAPE, "V = %d outside 1..%d", V, qk::kMaxViews);
    if (H < 1 || W < 1) return fail(QK_ESHAPE, "grid must be positive");
    qk_status st = check_camera(novel, "novel camera");
    if (st != QK_OK) return st;
    for (int m = 0; m < V; ++m) {
        st = check_camera(&in_cams[m], "input camera");
        if (st != QK_OK) return st;
        if (feat_hw[2 * m] < 1 || feat_hw[2 * m + 1] < 1) return fail(QK_ESHAPE, "feature grid");
        compose_table(novel, W, H, &in_cams[m], feat_hw[2 * m + 1], feat_hw[2 * m], out + 12 * m);
    }
    return QK_OK;
}

qk_status qk_update_fuse_check(int32_t V, const qk_camera *in_cams, const qk_feature_map *feats,
                               const qk_camera *novel, float near_, float far_,
                               const qk_weights *weights, qk_precision precision,
                               qk_attn_form attn_form, qk_update_mode update_mode,
                               const qk_ldm *ldm_in, const qk_ldm *ldm_out, float *rgb_out,
                               float *acc_alpha_out, float *blend_logit_out) {
    return check_update_fuse(V, in_cams, feats, novel, near_, far_, weights, precision, attn_form,
                             update_mode, ldm_in, ldm_out, rgb_out, acc_alpha_out, blend_logit_out);
}

}  // extern "C"

namespace {

// The launch parameters of one checked Update & Fuse request: camera
// tables (composed in double), pointers, and the tiling of its grid.
qk_status fill_uf_params(int32_t V, const qk_camera *in_cams, const qk_feature_map *feats,
                         const qk_camera *novel, float near_, float far_, const qk_weights *w,
                         qk_update_mode update_mode, const qk_ldm *in, const qk_ldm *out,
                         float *rgb_out, float *acc_out, float *blend_out, qk::UFParams &p) {
    std::memset(&p, 0, sizeof(p));
    for (int m = 0; m < V; ++m) {
        p.feat[m] = feats[m].data;
        p.fH[m] = feats[m].H;
        p.fW[m] = feats[m].W;
        double t12[12];
        compose_table(novel, in->W, in->H, &in_cams[m], feats[m].W, feats[m].H, t12);
        for (int k = 0; k < 12; ++k) {
            p.cam[m][k] = (float)t12[k];
            p.camd[m][k] = t12[k];
        }
    }
    p.F_in = in->F;
    p.depth_in = in->depth;
    p.alpha_in = in->alpha;
    p.F_out = out->F;
    p.depth_out = out->depth;
    p.alpha_out = out->alpha;
    p.rgb = rgb_out;
    p.acc = acc_out;
    p.blend_logit = blend_out;
    p.Wq = w->Wq;
    p.Wk = w->Wk;
    p.Wv = w->Wv;
    p.Wo = w->Wo;
    p.w_sigma = w->w_sigma;
    p.w_depth = w->w_depth;
    p.W_color = w->W_color;
    p.V = V;
    p.L = in->L;
    p.H = in->H;
    p.W = in->W;
    p.inv_near = 1.0f / near_;
    p.inv_far = 1.0f / far_;
    p.mode = (int)update_mode;
    // a workgroup covers 64 G pixels of a row, G = 32 / C sub-tiles for C < 32
    const int sub_tiles = in->C >= 32 ? 1 : 32 / in->C;
    const int wg_pixels = 64 * sub_tiles;
    p.x_blocks = (in->W + wg_pixels - 1) / wg_pixels;
    // Layer chunks: the composite needs every layer of a pixel in one wave;
    // otherwise split layers until the grid has enough workgroups.
    const int64_t xy = (int64_t)p.x_blocks * in->H;
    int chunks = 1;
    if (!rgb_out) {
        const int64_t want = 4096;
        chunks = (int)std::min<int64_t>(in->L, std::max<int64_t>(1, (want + xy - 1) / xy));
    }
    p.layers_per_chunk = (in->L + chunks - 1) / chunks;
    p.chunks = (in->L + p.layers_per_chunk - 1) / p.layers_per_chunk;
    const int64_t tiles = xy * p.chunks;
    if (tiles >= ((int64_t)1 << 31)) return fail(QK_EUNSUPPORTED, "grid too large");
    p.n_tiles = (int32_t)tiles;
    return QK_OK;
}

// qk_update_fuse and its allocation-free variant.  fixed == NULL: the folded
// weights and the e4m3 scales go to the context's workspaces (grown on
// demand); otherwise to `fixed` (kScratchFloats floats; nothing allocated).
qk_status update_fuse_impl(qk_context *ctx, void *hip_stream, int32_t V, const qk_camera *in_cams,
                           const qk_feature_map *feats, const qk_camera *novel, float near_,
                           float far_, const qk_weights *w, qk_precision precision,
                           qk_attn_form attn_form, qk_update_mode update_mode, const qk_ldm *in,
                           const qk_ldm *out, float *rgb_out, float *acc_out, float *blend_out,
                           float *fixed) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_update_fuse(V, in_cams, feats, novel, near_, far_, w, precision,
                                     attn_form, update_mode, in, out, rgb_out, acc_out, blend_out);
    if (st != QK_OK) return st;

    qk::UFParams p;
    st = fill_uf_params(V, in_cams, feats, novel, near_, far_, w, update_mode, in, out, rgb_out,
                        acc_out, blend_out, p);
    if (st != QK_OK) return st;

    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    const bool fold = attn_form == QK_ATTN_FOLDED;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (fold) {
        // fold W_k into the query and W_v into the output projection, on the
        // caller's stream, into the context's workspace
        const size_t per = (size_t)w->heads * w->C * w->C_feat;     // per folded matrix set
        const size_t need = 2 * per;
        if (fixed != nullptr) {
            // the allocation-free entry point derives them every call
            if (need > (size_t)qk::kScratchFold)
                return fail(QK_EUNSUPPORTED, "folded weights of %zu floats exceed the fixed scratch "
                            "of %d", need, qk::kScratchFold);
            qk::FoldParams fp{w->Wq, w->Wk, w->Wv, w->Wo, fixed, fixed + per,
                              w->C, w->C_feat, w->head_dim, w->heads,
                              1.0f / std::sqrt((float)w->head_dim)};
            hipError_t fe = qk::launch_fold_weights(fp, stream);
            if (fe != hipSuccess) return fail(QK_EHIP, "fold launch: %s", hipGetErrorString(fe));
            p.Wqk = fp.Wqk;
            p.Wvo = fp.Wvo;
        } else {
            // the per-call workspace (also the fallback of a full cache)
            st = grow(ctx, &ctx->wfold, &ctx->wfold_elems, need, stream);
            if (st != QK_OK) return st;
            float *wqk = nullptr, *wvo = nullptr;
            st = fold_weights(ctx, w, ctx->wfold, stream, &wqk, &wvo);
            if (st != QK_OK) return st;
            p.Wqk = wqk;
            p.Wvo = wvo;
        }
    }
    if (precision == QK_PREC_BF16_FP8PROJ) {
        float *f8 = fixed != nullptr ? fixed + qk::kScratchFold : nullptr;
        if (f8 == nullptr) {
            st = grow(ctx, &ctx->f8, &ctx->f8_elems, 8, stream);
            if (st != QK_OK) return st;
            f8 = ctx->f8;
        }
        qk::F8Params fp8;
        std::memset(&fp8, 0, sizeof(fp8));
        for (int m = 0; m < V; ++m) {
            fp8.feat[m] = static_cast<const uint16_t *>(feats[m].data);
            fp8.feat_elems[m] = (int64_t)feats[m].H * feats[m].W * w->C_feat;
        }
        fp8.V = V;
        fp8.Wq = fold ? p.Wqk : w->Wq;
        fp8.Wk = w->Wk;
        fp8.Wv = w->Wv;
        fp8.Wo = fold ? p.Wvo : w->Wo;
        fp8.C = w->C;
        fp8.Cf = w->C_feat;
        fp8.hd = fold ? w->C_feat : w->heads * w->head_dim;
        fp8.fold = fold ? 1 : 0;
        fp8.amax_bits = reinterpret_cast<unsigned *>(f8 + 7);
        fp8.scales = f8;
        hipError_t e8 = qk::launch_fp8_scales(fp8, stream);
        if (e8 != hipSuccess) return fail(QK_EHIP, "fp8 scale launch: %s", hipGetErrorString(e8));
        p.f8_scales = f8;
    }
    hipError_t e = qk::launch_update_fuse(p, in->C, w->head_dim, (int)precision, fold, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "update_fuse launch: %s", hipGetErrorString(e));
    return QK_OK;
}

}  // namespace

extern "C" {

qk_status qk_update_fuse(qk_context *ctx, void *hip_stream, int32_t V, const qk_camera *in_cams,
                         const qk_feature_map *feats, const qk_camera *novel, float near_,
                         float far_, const qk_weights *w, qk_precision precision,
                         qk_attn_form attn_form, qk_update_mode update_mode, const qk_ldm *in,
                         const qk_ldm *out, float *rgb_out, float *acc_out, float *blend_out) {
    return update_fuse_impl(ctx, hip_stream, V, in_cams, feats, novel, near_, far_, w, precision,
                            attn_form, update_mode, in, out, rgb_out, acc_out, blend_out, nullptr);
}

qk_status qk_update_fuse_noalloc(qk_context *ctx, void *hip_stream, int32_t V,
                                 const qk_camera *in_cams, const qk_feature_map *feats,
                                 const qk_camera *novel, float near_, float far_,
                                 const qk_weights *w, qk_precision precision,
                                 qk_attn_form attn_form, qk_update_mode update_mode,
                                 const qk_ldm *in, const qk_ldm *out, float *rgb_out,
                                 float *acc_out, float *blend_out) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    if (ctx->scratch == nullptr) return fail(QK_EHIP, "the device's fixed scratch is unknown");
    return update_fuse_impl(ctx, hip_stream, V, in_cams, feats, novel, near_, far_, w, precision,
                            attn_form, update_mode, in, out, rgb_out, acc_out, blend_out,
                            ctx->scratch);
}

qk_status qk_batch_update_fuse_check(int32_t n_req, const qk_request_desc *reqs,
                                     qk_precision precision, qk_attn_form attn_form) {
    if (!reqs) return fail(QK_EINVAL, "reqs is NULL");
    if (n_req < 1 || n_req > qk::kMaxBatch)
        return fail(QK_ESHAPE, "n_req = %d outside 1..%d", n_req, qk::kMaxBatch);
    if (precision != QK_PREC_BF16)
        return fail(QK_EUNSUPPORTED, "batches run the bfloat16 form (QK_PREC_BF16)");
    int64_t tiles = 0;
    for (int r = 0; r < n_req; ++r) {
        const qk_request_desc &q = reqs[r];
        qk_status st = check_update_fuse(q.V, q.in_cams, q.feats, q.novel, q.near_, q.far_,
                                         q.weights, precision, attn_form, q.update_mode,
                                         q.ldm_in, q.ldm_out, q.rgb_out, q.acc_alpha_out,
                                         q.blend_logit_out);
        if (st != QK_OK) {
            const std::string msg = g_err;
            return fail(st, "request %d: %s", r, msg.c_str());
        }
        const qk_weights *w0 = reqs[0].weights;
        if (q.weights->C != w0->C || q.weights->heads != w0->heads ||
            q.weights->head_dim != w0->head_dim)
            return fail(QK_EUNSUPPORTED, "request %d: every request needs C, heads and head_dim "
                        "of request 0", r);
        qk::UFParams p;
        st = fill_uf_params(q.V, q.in_cams, q.feats, q.novel, q.near_, q.far_, q.weights,
                            q.update_mode, q.ldm_in, q.ldm_out, q.rgb_out, q.acc_alpha_out,
                            q.blend_logit_out, p);
        if (st != QK_OK) return st;
        tiles += p.n_tiles;
    }
    if (tiles >= ((int64_t)1 << 31)) return fail(QK_EUNSUPPORTED, "batch grid too large");
    return QK_OK;
}

qk_status qk_batch_update_fuse(qk_context *ctx, void *hip_stream, int32_t n_req,
                               const qk_request_desc *reqs, qk_precision precision,
                               qk_attn_form attn_form) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = qk_batch_update_fuse_check(n_req, reqs, precision, attn_form);
    if (st != QK_OK) return st;
    std::vector<qk::UFParams> ps((size_t)n_req);
    qk::UFBatch b;
    std::memset(&b, 0, sizeof(b));
    b.n_req = n_req;
    int64_t tiles = 0;
    for (int r = 0; r < n_req; ++r) {
        const qk_request_desc &q = reqs[r];
        st = fill_uf_params(q.V, q.in_cams, q.feats, q.novel, q.near_, q.far_, q.weights,
                            q.update_mode, q.ldm_in, q.ldm_out, q.rgb_out, q.acc_alpha_out,
                            q.blend_logit_out, ps[r]);
        if (st != QK_OK) return st;
        b.tile_start[r] = (int32_t)tiles;
        tiles += ps[r].n_tiles;
    }
    b.tile_start[n_req] = (int32_t)tiles;
    b.total_tiles = (int32_t)tiles;

    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const qk_weights *w0 = reqs[0].weights;
    const bool fold = attn_form == QK_ATTN_FOLDED;
    if (fold) {
        // each request's folded weights in its own slice of the workspace
        const size_t per = (size_t)w0->heads * w0->C * w0->C_feat;
        st = grow(ctx, &ctx->wfold, &ctx->wfold_elems, 2 * per * (size_t)n_req, stream);
        if (st != QK_OK) return st;
        for (int r = 0; r < n_req; ++r) {
            float *wqk = nullptr, *wvo = nullptr;
            st = fold_weights(ctx, reqs[r].weights, ctx->wfold + 2 * per * (size_t)r, stream, &wqk, &wvo);
            if (st != QK_OK) return st;
            ps[r].Wqk = wqk;
            ps[r].Wvo = wvo;
        }
    }
    // the requests' parameters to the device: pinned staging, reused once
    // the previous call's copy has completed
    const size_t bytes = sizeof(qk::UFParams) * (size_t)n_req;
    st = grow(ctx, &ctx->bdesc, &ctx->bdesc_elems, (bytes + 3) / 4, stream);
    if (st != QK_OK) return st;
    hipError_t e;
    if (ctx->bevent == nullptr) {
        e = hipEventCreateWithFlags(&ctx->bevent, hipEventDisableTiming);
        if (e != hipSuccess) return fail(QK_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    if (ctx->bevent_live) {
        e = hipEventSynchronize(ctx->bevent);
        if (e != hipSuccess) return fail(QK_EHIP, "hipEventSynchronize: %s", hipGetErrorString(e));
        ctx->bevent_live = false;
    }
    if (ctx->bhost_bytes < bytes) {
        if (ctx->bhost) (void)hipHostFree(ctx->bhost);
        ctx->bhost = nullptr;
        ctx->bhost_bytes = 0;
        e = hipHostMalloc(&ctx->bhost, bytes, hipHostMallocDefault);
        if (e != hipSuccess) return fail(QK_ENOMEM, "pinned staging of %zu bytes", bytes);
        ctx->bhost_bytes = bytes;
    }
    std::memcpy(ctx->bhost, ps.data(), bytes);
    e = hipMemcpyAsync(ctx->bdesc, ctx->bhost, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "parameter upload: %s", hipGetErrorString(e));
    e = hipEventRecord(ctx->bevent, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
    ctx->bevent_live = true;
    e = qk::launch_update_fuse_batch(reinterpret_cast<const qk::UFParams *>(ctx->bdesc), b, w0->C,
                                     w0->head_dim, (int)precision, fold, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "batched update_fuse launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_composite(qk_context *ctx, void *hip_stream, int32_t L, int32_t H, int32_t W,
                       const float *color, const float *alpha, float *rgb_out, float *acc_out) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    if (!color || !alpha || !rgb_out) return fail(QK_EINVAL, "NULL buffer");
    if (L < 1 || H < 1 || W < 1) return fail(QK_ESHAPE, "dims must be positive");
    if (!aligned4(color) || !aligned4(alpha) || !aligned4(rgb_out) || (acc_out && !aligned4(acc_out)))
        return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    const int64_t npix = (int64_t)H * W;
    if (npix * L * 3 >= ((int64_t)1 << 40)) return fail(QK_EUNSUPPORTED, "too large");
    qk::CompParams p{color, alpha, rgb_out, acc_out, L, npix};
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipError_t e = qk::launch_composite(p, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "composite launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_composite_backward_check(int32_t L, int32_t H, int32_t W, const float *color,
                                      const float *alpha, const float *d_rgb, const float *d_acc,
                                      const float *d_color, const float *d_alpha) {
    if (!color || !alpha || !d_rgb || !d_alpha) return fail(QK_EINVAL, "NULL buffer");
    if (L < 1 || H < 1 || W < 1) return fail(QK_ESHAPE, "dims must be positive");
    const void *bufs[6] = {color, alpha, d_rgb, d_acc, d_color, d_alpha};
    for (const void *b : bufs)
        if (b && !aligned4(b)) return fail(QK_EINVAL, "float buffers must be 4-byte aligned");
    const int64_t npix = (int64_t)H * W;
    if (npix * L * 3 >= ((int64_t)1 << 40)) return fail(QK_EUNSUPPORTED, "too large");
    // outputs must not overlap the inputs they are computed from
    const int64_t n1 = npix * L, n3 = 3 * n1;
    auto overlap = [](const float *a, int64_t na, const float *b, int64_t nb) {
        return a && b && a < b + nb && b < a + na;
    };
    const float *outs[2] = {d_color, d_alpha};
    const int64_t nouts[2] = {n3, n1};
    for (int i = 0; i < 2; ++i) {
        if (overlap(outs[i], nouts[i], color, n3) || overlap(outs[i], nouts[i], alpha, n1) ||
            overlap(outs[i], nouts[i], d_rgb, 3 * npix) || overlap(outs[i], nouts[i], d_acc, npix))
            return fail(QK_EINVAL, "an output overlaps an input");
    }
    if (overlap(d_color, n3, d_alpha, n1)) return fail(QK_EINVAL, "d_color overlaps d_alpha");
    return QK_OK;
}

qk_status qk_composite_backward(qk_context *ctx, void *hip_stream, int32_t L, int32_t H,
                                int32_t W, const float *color, const float *alpha,
                                const float *d_rgb, const float *d_acc, float *d_color,
                                float *d_alpha) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = qk_composite_backward_check(L, H, W, color, alpha, d_rgb, d_acc, d_color,
                                               d_alpha);
    if (st != QK_OK) return st;
    qk::CompBwdParams p{color, alpha, d_rgb, d_acc, d_color, d_alpha, L, (int64_t)H * W};
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipError_t e = qk::launch_composite_backward(p, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "composite backward launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_update_fuse_backward_check(int32_t V, const qk_camera *in_cams,
                                        const qk_feature_map *feats, const qk_camera *novel,
                                        float near_, float far_, const qk_weights *weights,
                                        qk_update_mode update_mode, const qk_ldm *ldm_in,
                                        const qk_ldm *ldm_out, const float *d_rgb,
                                        const qk_ldm *d_out, const qk_ldm *d_in,
                                        float *const *d_feats, const qk_weight_grads *d_weights) {
    return check_backward(V, in_cams, feats, novel, near_, far_, weights, update_mode, ldm_in,
                          ldm_out, d_rgb, d_out, d_in, d_feats, d_weights);
}

qk_status qk_update_fuse_backward(qk_context *ctx, void *hip_stream, int32_t V,
                                  const qk_camera *in_cams, const qk_feature_map *feats,
                                  const qk_camera *novel, float near_, float far_,
                                  const qk_weights *w, qk_update_mode update_mode,
                                  const qk_ldm *in, const qk_ldm *out, const float *d_rgb,
                                  const qk_ldm *d_out, const qk_ldm *d_in, float *const *d_feats,
                                  const qk_weight_grads *dw) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_backward(V, in_cams, feats, novel, near_, far_, w, update_mode, in, out,
                                  d_rgb, d_out, d_in, d_feats, dw);
    if (st != QK_OK) return st;

    qk::BwdParams p;
    std::memset(&p, 0, sizeof(p));
    for (int m = 0; m < V; ++m) {
        p.feat[m] = static_cast<const float *>(feats[m].data);
        p.dfeat[m] = d_feats[m];
        p.fH[m] = feats[m].H;
        p.fW[m] = feats[m].W;
        compose_table(novel, in->W, in->H, &in_cams[m], feats[m].W, feats[m].H, p.camd[m]);
    }
    p.F_in = static_cast<const float *>(in->F);
    p.depth_in = in->depth;
    p.alpha_in = in->alpha;
    if (d_rgb) {
        p.F_out = static_cast<const float *>(out->F);
        p.alpha_out = out->alpha;
        p.d_rgb = d_rgb;
    }
    if (d_out) {
        p.dF_out = static_cast<const float *>(d_out->F);
        p.d_depth_out = d_out->depth;
        p.d_alpha_out = d_out->alpha;
    }
    p.dF = static_cast<float *>(d_in->F);
    p.d_depth = d_in->depth;
    p.d_alpha = d_in->alpha;
    p.Wq = w->Wq;
    p.Wk = w->Wk;
    p.Wv = w->Wv;
    p.Wo = w->Wo;
    p.w_sigma = w->w_sigma;
    p.w_depth = w->w_depth;
    p.W_color = w->W_color;
    p.dWq = dw->Wq;
    p.dWk = dw->Wk;
    p.dWv = dw->Wv;
    p.dWo = dw->Wo;
    p.dw_sigma = dw->w_sigma;
    p.dw_depth = dw->w_depth;
    p.dW_color = dw->W_color;
    p.V = V;
    p.L = in->L;
    p.H = in->H;
    p.W = in->W;
    p.C = in->C;
    p.N = (int64_t)in->L * in->H * in->W;
    p.inv_near = 1.0f / near_;
    p.inv_far = 1.0f / far_;
    p.scale = 1.0f / std::sqrt((float)w->head_dim);
    p.mode = (int)update_mode;
    // persistent workgroups: four per compute unit, or fewer for small LDMs
    const int64_t tiles = (p.N + 255) / 256;
    p.blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(tiles, 4 * (int64_t)ctx->num_cu));

    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t n_comp = d_rgb ? 4 * (size_t)p.N : 0;
    const size_t n_part = (size_t)p.blocks * qk::kGradTiles * qk::kGradTileElems;
    st = grow(ctx, &ctx->bws, &ctx->bws_elems, n_comp + n_part, stream);
    if (st != QK_OK) return st;
    p.partials = ctx->bws;
    p.comp = d_rgb ? ctx->bws + n_part : nullptr;
    hipError_t e = qk::launch_update_fuse_backward(p, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "backward launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_ldm_init(qk_context *ctx, void *hip_stream, const float *f0, float near_, float far_,
                      const qk_ldm *ldm) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    if (!f0 || !ldm || !ldm->F || !ldm->depth || !ldm->alpha) return fail(QK_EINVAL, "NULL buffer");
    if (!(near_ > 0.0f) || !(far_ > near_) || !std::isfinite(far_))
        return fail(QK_EINVAL, "need 0 < near < far (got %g, %g)", near_, far_);
    if (ldm->L < 1 || ldm->H < 1 || ldm->W < 1 || ldm->C < 8 || ldm->C % 8 != 0)
        return fail(QK_ESHAPE, "need positive L, H, W and C a multiple of 8 (L=%d H=%d W=%d C=%d)",
                    ldm->L, ldm->H, ldm->W, ldm->C);
    if (ldm->dtype != QK_F32 && ldm->dtype != QK_BF16)
        return fail(QK_EDTYPE, "unknown LDM dtype %d", (int)ldm->dtype);
    if (!aligned16(f0) || !aligned16(ldm->F) || !aligned4(ldm->depth) || !aligned4(ldm->alpha))
        return fail(QK_EINVAL, "misaligned buffer");
    qk::InitParams p;
    p.f0 = f0;
    p.F = ldm->F;
    p.depth = ldm->depth;
    p.alpha = ldm->alpha;
    p.npix = (int64_t)ldm->H * ldm->W;
    p.N = p.npix * ldm->L;
    p.L = ldm->L;
    p.C = ldm->C;
    p.inv_near = 1.0f / near_;
    p.inv_far = 1.0f / far_;
    if (p.N * p.C >= ((int64_t)1 << 40)) return fail(QK_EUNSUPPORTED, "LDM too large");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipError_t e = qk::launch_ldm_init(p, ldm->dtype == QK_BF16, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "ldm_init launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_render_ibr_check(int32_t V, const qk_camera *in_cams, const qk_image *images,
                              const qk_camera *novel, float near_, float far_,
                              const qk_ldm_logits *logits, int32_t H, int32_t W,
                              const float *rgb_out, const float *acc_out, const float *depth_out) {
    return check_render(V, in_cams, images, novel, near_, far_, logits, H, W, rgb_out, acc_out,
                        depth_out);
}

qk_status qk_render_ibr(qk_context *ctx, void *hip_stream, int32_t V, const qk_camera *in_cams,
                        const qk_image *images, const qk_camera *novel, float near_, float far_,
                        const qk_ldm_logits *lg, int32_t H, int32_t W, float *rgb_out,
                        float *acc_out, float *depth_out) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_render(V, in_cams, images, novel, near_, far_, lg, H, W, rgb_out,
                                acc_out, depth_out);
    if (st != QK_OK) return st;
    qk::RenderParams p;
    std::memset(&p, 0, sizeof(p));
    for (int m = 0; m < V; ++m) {
        p.img[m] = images[m].data;
        p.iH[m] = images[m].H;
        p.iW[m] = images[m].W;
        compose_table(novel, W, H, &in_cams[m], images[m].W, images[m].H, p.cam[m]);
    }
    p.depth_logit = lg->depth_logit;
    p.sigma_logit = lg->sigma_logit;
    p.blend_logit = lg->blend_logit;
    p.rgb = rgb_out;
    p.acc = acc_out;
    p.depth = depth_out;
    p.V = V;
    p.L = lg->L;
    p.h = lg->H;
    p.w = lg->W;
    p.H = H;
    p.W = W;
    p.rx = (double)lg->W / (double)W;
    p.ry = (double)lg->H / (double)H;
    p.band = 1.0 / (double)near_ - 1.0 / (double)far_;
    p.inv_far = 1.0 / (double)far_;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipError_t e = qk::launch_render_ibr(p, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "render launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_render_to_views_check(int32_t V, const qk_camera *in_cams, const qk_camera *novel,
                                   const qk_ldm_decoded *ldm, const qk_view_image *views) {
    return check_views(V, in_cams, novel, ldm, views, nullptr);
}

qk_status qk_render_to_views(qk_context *ctx, void *hip_stream, int32_t V,
                             const qk_camera *in_cams, const qk_camera *novel,
                             const qk_ldm_decoded *ldm, const qk_view_image *views) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    int64_t total = 0;
    qk_status st = check_views(V, in_cams, novel, ldm, views, &total);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    qk::ViewsParams p;
    std::memset(&p, 0, sizeof(p));
    // The binned form holds all layers of a tile in 64 KiB of LDS (tiles of
    // 32 x th pixels, 32 bytes per pixel and layer: th = 16 for L <= 4,
    // halved as L doubles) and indexes records and view coordinates in 32
    // and 16 bits; other calls take the planes form.
    const int64_t nrec = (int64_t)V * ldm->L * ldm->H * ldm->W;
    bool small_views = true;
    for (int m = 0; m < V; ++m) small_views = small_views && views[m].W < 65535 && views[m].H < 65535;
    p.binned = ldm->L <= 128 && nrec < ((int64_t)1 << 31) && small_views;
    size_t ws_floats = (size_t)total;
    size_t rec_off = 0;
    if (p.binned) {
        p.tw = 32;
        p.th = 32;
        while (p.th > 1 && (int64_t)ldm->L * p.th * p.tw * 32 > 65536) p.th /= 2;
        int32_t tiles = 0;
        for (int m = 0; m < V; ++m) {
            p.ntx[m] = (views[m].W + p.tw - 1) / p.tw;
            p.nty[m] = (views[m].H + p.th - 1) / p.th;
            p.tbase[m] = tiles;
            tiles += p.ntx[m] * p.nty[m];
        }
        p.tbase[V] = tiles;
        p.nbins = 4 * tiles;
        // count [nbins], start [nbins + 1, padded to nbins + 4], cursor
        // [nbins], then the records (one 32-bit layer-pixel index each);
        // nbins is a multiple of 4, so every array starts on a 16-byte
        // boundary
        rec_off = (size_t)3 * p.nbins + 4;
        ws_floats = rec_off + (size_t)nrec;
    }
    st = grow(ctx, &ctx->vws, &ctx->vws_elems, ws_floats, stream);
    if (st != QK_OK) return st;
    if (p.binned) {
        uint32_t *u = reinterpret_cast<uint32_t *>(ctx->vws);
        p.count = u;
        p.start = u + p.nbins;
        p.cursor = u + 2 * (size_t)p.nbins + 4;
        p.rec = reinterpret_cast<int32_t *>(ctx->vws + rec_off);
    }
    int64_t base = 0, maxpix = 0;
    for (int m = 0; m < V; ++m) {
        compose_table(novel, ldm->W, ldm->H, &in_cams[m], views[m].W, views[m].H, p.cam[m]);
        p.vH[m] = views[m].H;
        p.vW[m] = views[m].W;
        p.sbase[m] = base;
        p.rgb[m] = views[m].rgb;
        p.acc[m] = views[m].acc;
        const int64_t np = (int64_t)views[m].H * views[m].W;
        base += (int64_t)ldm->L * np * 4;
        maxpix = std::max(maxpix, np);
    }
    p.ws = ctx->vws;
    p.ws_floats = total;
    p.depth = ldm->depth;
    p.alpha = ldm->alpha;
    p.color = ldm->color;
    p.V = V;
    p.L = ldm->L;
    p.H = ldm->H;
    p.W = ldm->W;
    p.N = (int64_t)ldm->L * ldm->H * ldm->W;
    p.max_view_pixels = maxpix;
    hipError_t e = qk::launch_render_to_views(p, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "render to views launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_residual_conv_check(const qk_ldm *ldm_in, const float *W1, const float *W2,
                                 const qk_ldm *ldm_out) {
    return check_conv(ldm_in, W1, W2, ldm_out);
}

qk_status qk_residual_conv(qk_context *ctx, void *hip_stream, const qk_ldm *in, const float *W1,
                           const float *W2, const qk_ldm *out) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_conv(in, W1, W2, out);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    constexpr size_t kFragFloats = 2 * 9 * 2 * 64 * 4;
    // the kernels' bfloat16 fragments: cached while the weights are static
    // (derived on first use, the stream then synchronised), else per call
    float *frag = nullptr;
    bool fresh = true;
    if (ctx->weights_static) {
        const void *key[4] = {W1, W2, nullptr, nullptr};
        const int32_t dims[4] = {0, 0, 0, 0};
        frag = derived_find(ctx, kDerivedConv, key, dims);
        fresh = frag == nullptr;
        if (fresh) {
            st = derived_add(ctx, kDerivedConv, key, dims, kFragFloats, &frag);
            if (st != QK_OK) return st;
        }
    }
    const bool cached = frag != nullptr;
    if (!cached) {
        st = grow(ctx, &ctx->cfrag, &ctx->cfrag_elems, kFragFloats, stream);
        if (st != QK_OK) return st;
        frag = ctx->cfrag;
    }
    qk::ConvParams p;
    std::memset(&p, 0, sizeof(p));
    p.F = static_cast<const uint16_t *>(in->F);
    p.F_out = static_cast<uint16_t *>(out->F);
    p.W1 = W1;
    p.W2 = W2;
    p.frag = reinterpret_cast<uint4 *>(frag);
    p.L = in->L;
    p.H = in->H;
    p.W = in->W;
    hipError_t e = qk::launch_residual_conv(p, ctx->num_cu, !fresh, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "residual block launch: %s", hipGetErrorString(e));
    if (cached && fresh) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(QK_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    return QK_OK;
}

qk_status qk_layer_collapse_check(const qk_ldm *ldm_in, const float *W1, const float *W2,
                                  const qk_ldm *ldm_out) {
    return check_collapse(ldm_in, W1, W2, ldm_out);
}

qk_status qk_layer_collapse(qk_context *ctx, void *hip_stream, const qk_ldm *in, const float *W1,
                            const float *W2, const qk_ldm *out) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_collapse(in, W1, W2, out);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    qk::CollapseParams p;
    std::memset(&p, 0, sizeof(p));
    p.F = static_cast<const uint16_t *>(in->F);
    p.F_out = static_cast<uint16_t *>(out->F);
    p.W1 = W1;
    p.W2 = W2;
    p.L = in->L;
    p.npix = (int64_t)in->H * in->W;
    p.n_blocks = (int64_t)(in->L / 2) * ((p.npix + 15) / 16);
    hipError_t e = qk::launch_layer_collapse(p, ctx->num_cu, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "layer collapse launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_ray_encoding_check(int32_t V, const qk_camera *in_cams, const qk_camera *novel,
                                float near_, float far_, const float *Wr, int32_t C,
                                qk_dtype dtype, int32_t low_H, int32_t low_W,
                                const qk_feature_map_inout *feats) {
    return check_ray(V, in_cams, novel, near_, far_, Wr, C, dtype, low_H, low_W, feats);
}

qk_status qk_ray_encoding(qk_context *ctx, void *hip_stream, int32_t V, const qk_camera *in_cams,
                          const qk_camera *novel, float near_, float far_, const float *Wr,
                          int32_t C, qk_dtype dtype, int32_t low_H, int32_t low_W,
                          const qk_feature_map_inout *feats) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_ray(V, in_cams, novel, near_, far_, Wr, C, dtype, low_H, low_W, feats);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (low_H > 0) {
        st = grow(ctx, &ctx->rws, &ctx->rws_elems, (size_t)V * low_H * low_W * C, stream);
        if (st != QK_OK) return st;
    }
    qk::RayParams p;
    std::memset(&p, 0, sizeof(p));
    double Mn[9], tn[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) Mn[3 * r + c] = novel->E[4 * r + c];
        tn[r] = novel->E[4 * r + 3];
    }
    int64_t maxpix = 0;
    for (int m = 0; m < V; ++m) {
        // ray direction in the novel frame: M_n M_m^-1 K_m^-1 (u, v, 1), K_m
        // rescaled to the grid the encoding is evaluated on (the map's, or
        // the low-resolution one); view m's centre there: M_n (-M_m^-1 t_m) + t_n
        const qk_camera *cam = &in_cams[m];
        double Ks[9], Ksi[9], Mm[9], Mmi[9], R[9], tm[3];
        if (low_H > 0)
            scaled_K(cam, low_W, low_H, Ks);
        else
            scaled_K(cam, feats[m].W, feats[m].H, Ks);
        mat3_inv(Ks, Ksi);
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) Mm[3 * r + c] = cam->E[4 * r + c];
            tm[r] = cam->E[4 * r + 3];
        }
        mat3_inv(Mm, Mmi);
        mat3_mul(Mn, Mmi, R);
        mat3_mul(R, Ksi, p.D[m]);
        for (int r = 0; r < 3; ++r) {
            double s = tn[r];
            for (int k = 0; k < 3; ++k) s -= R[3 * r + k] * tm[k];
            p.o[m][r] = s;
        }
        p.feat[m] = feats[m].data;
        p.src[m] = feats[m].src ? feats[m].src : feats[m].data;
        p.fH[m] = feats[m].H;
        p.fW[m] = feats[m].W;
        maxpix = std::max(maxpix, (int64_t)feats[m].H * feats[m].W);
    }
    p.kx0 = 2.0 * novel->K[0] / novel->width;
    p.kx1 = 2.0 * novel->K[1] / novel->width;
    p.ky0 = 2.0 * novel->K[3] / novel->height;
    p.ky1 = 2.0 * novel->K[4] / novel->height;
    p.inv_band = 1.0 / (double)far_ - 1.0 / (double)near_;
    p.Wr = Wr;
    p.P = low_H > 0 ? ctx->rws : nullptr;
    p.lH = low_H;
    p.lW = low_W;
    p.V = V;
    p.C = C;
    p.bf16 = dtype == QK_BF16;
    p.max_pixels = maxpix;
    hipError_t e = qk::launch_ray_encoding(p, stream);
    if (e != hipSuccess) return fail(QK_EHIP, "ray encoding launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_upsample2x_check(const void *src, void *dst, int32_t N, int32_t H, int32_t W,
                              int32_t C, qk_dtype dtype) {
    return check_upsample2x(src, dst, N, H, W, C, dtype);
}

qk_status qk_upsample2x(qk_context *ctx, void *hip_stream, const void *src, void *dst, int32_t N,
                        int32_t H, int32_t W, int32_t C, qk_dtype dtype) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_upsample2x(src, dst, N, H, W, C, dtype);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    qk::Up2Params p{src, dst, N, H, W, C, dtype == QK_BF16 ? 1 : 0};
    hipError_t e = qk::launch_upsample2x(p, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "upsample launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_ldm_decode_check(const qk_ldm *ldm, const float *w_sigma, const float *w_depth,
                              const float *W_color, float near_, float far_,
                              const float *color_out) {
    return check_decode(ldm, w_sigma, w_depth, W_color, near_, far_, color_out);
}

qk_status qk_ldm_decode(qk_context *ctx, void *hip_stream, const qk_ldm *ldm,
                        const float *w_sigma, const float *w_depth, const float *W_color,
                        float near_, float far_, float *color_out) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = check_decode(ldm, w_sigma, w_depth, W_color, near_, far_, color_out);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    qk::DecodeParams p{ldm->F, w_sigma, w_depth, W_color, ldm->depth, ldm->alpha, color_out,
                       ldm->L, ldm->H, ldm->W, ldm->C, ldm->dtype == QK_BF16 ? 1 : 0,
                       (float)(1.0 / (double)near_), (float)(1.0 / (double)far_), 0};
    hipError_t e = qk::launch_ldm_decode(p, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "decode launch: %s", hipGetErrorString(e));
    return QK_OK;
}

qk_status qk_ldm_decode_logits_check(const qk_ldm *ldm, const float *w_sigma, const float *w_depth,
                              const float *depth_logit, const float *sigma_logit) {
    if (!ldm || !depth_logit || !sigma_logit) return fail(QK_EINVAL, "NULL argument");
    qk_ldm v = *ldm;                 // the decode's checks, on the logit outputs
    v.depth = const_cast<float *>(depth_logit);
    v.alpha = const_cast<float *>(sigma_logit);
    qk_status st = check_decode(&v, w_sigma, w_depth, w_sigma, 0.5f, 1.0f, nullptr);
    if (st != QK_OK) return st;
    const int64_t n = (int64_t)ldm->L * ldm->H * ldm->W;
    const float *a = depth_logit, *b = sigma_logit;
    if (a < b + n && b < a + n) return fail(QK_EINVAL, "depth_logit overlaps sigma_logit");
    return QK_OK;
}

qk_status qk_ldm_decode_logits(qk_context *ctx, void *hip_stream, const qk_ldm *ldm,
                        const float *w_sigma, const float *w_depth, float *depth_logit,
                        float *sigma_logit) {
    if (!ctx) return fail(QK_EINVAL, "context is NULL");
    qk_status st = qk_ldm_decode_logits_check(ldm, w_sigma, w_depth, depth_logit, sigma_logit);
    if (st != QK_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(QK_EHIP, "hipGetDevice failed");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return fail(QK_EHIP, "hipSetDevice(%d) failed", ctx->device);
    qk::DecodeParams p{ldm->F, w_sigma, w_depth, w_sigma, depth_logit, sigma_logit, nullptr,
                       ldm->L, ldm->H, ldm->W, ldm->C, ldm->dtype == QK_BF16 ? 1 : 0,
                       1.0f, 1.0f, 1};
    hipError_t e = qk::launch_ldm_decode(p, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(QK_EHIP, "logits launch: %s", hipGetErrorString(e));
    return QK_OK;
}

}  // extern "C"
