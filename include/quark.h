/*
 * quark.h -- C-ABI of libquark, the MI355X (gfx950) library for one
 * Update & Fuse step of a layered depth map (LDM) and the LDM's
 * front-to-back composite, after Quark: Real-time, High-resolution, and
 * General Neural View Synthesis (Flynn et al., ACM TOG 43(6), 2024).
 *
 * The problem statement follows the paper's Sec. 3.1-3.3: M input views with
 * cameras theta and encoded feature maps I_k, a target (novel) camera, an LDM
 * of L layers x [H, W] in the novel frustum (depth d, alpha sigma, features
 * V), and an output image.
 *
 * Entry points (all but qk_ldm_init, qk_composite and qk_camera_tables with
 * a dry-run `_check` of their arguments):
 *   qk_update_fuse           one Update & Fuse step (+ composite), Sec. 3.2.2-3.3
 *   qk_update_fuse_noalloc   the same with a fixed scratch, no device allocation
 *   qk_batch_update_fuse     several requests' steps in one launch (serving)
 *   qk_update_fuse_backward  its adjoint into features, LDM and weights
 *   qk_ldm_init              learned initialisation of an LDM, Sec. 3.2
 *   qk_composite             front-to-back over composite, Sec. 3.1
 *   qk_composite_backward    its adjoint, Sec. 3.1
 *   qk_render_ibr            final render (upsample, activate, blend), Eq. 1
 *   qk_render_to_views       render of an intermediate LDM into the views, Eq. 2
 *   qk_residual_conv         residual CNN block of a fusion block, Sec. 3.3
 *   qk_layer_collapse        layer collapse, Sec. 3.2.2
 *   qk_ray_encoding          ray-direction encoding of the views, Sec. 3.2.1-3.2.2
 *   qk_upsample2x            2x resolution transition, Sec. 3.2.2
 *   qk_ldm_decode            absolute decode of an encoded LDM, Sec. 3.2.2-3.2.3
 *   qk_ldm_decode_logits     unactivated decode of the final volume, Sec. 3.2.3
 *   qk_camera_tables         the composed reprojection tables (host only)
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Every call returns a qk_status; nothing throws across the ABI.  On a
 *    non-OK status qk_last_error() returns a thread-local message.
 *  - Pointers marked "device" are HIP device pointers owned by the caller; the
 *    library keeps none of them after the call returns.  Work is enqueued
 *    asynchronously on the caller's `hip_stream` (a hipStream_t; NULL = the
 *    default stream), so device buffers must stay valid until that stream
 *    reaches the point of the call.  Pointers marked "host" are read before
 *    the call returns.
 *  - Shapes, dtypes, NULLs and 16-byte alignment of device buffers are
 *    checked before anything is enqueued; a failed check returns
 *    QK_ESHAPE / QK_EDTYPE / QK_EINVAL / QK_EUNSUPPORTED and enqueues nothing.
 *    Launch failures return QK_EHIP.  Device faults surface at the caller's
 *    next synchronisation.  Values (depth > 0, alpha in [0, 1]) are not
 *    checked.
 *  - Layouts are row-major, channel-last and layer-major:
 *       LDM features  F[L][H][W][C]     (QK_F32 float or QK_BF16 bfloat16)
 *       depth, alpha  [L][H][W]         float
 *       feature map   I[Hf][Wf][Cf]     (same dtype as F), one per view
 *       rgb           [H][W][3] float,  acc_alpha [H][W] float
 *    Layer 0 is the nearest layer.
 *  - Cameras (host, double): K is 3x3 row-major in pixel units of the
 *    camera's own (width, height) grid, pixel (x, y) centred at
 *    (x + 0.5, y + 0.5).  The library rescales K to whichever grid it is used
 *    on: K' = diag(W'/width, H'/height, 1) K.  E is the 4x4 row-major
 *    world-to-camera transform, OpenCV axes (+x right, +y down, +z forward).
 *    Depth is z-depth along the novel camera's optical axis.
 */
#ifndef QUARK_H
#define QUARK_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define QK_API __attribute__((visibility("default")))
#else
#define QK_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QK_OK = 0,
    QK_EINVAL = -1,       /* NULL pointer, bad enum, misaligned buffer      */
    QK_ESHAPE = -2,       /* inconsistent or out-of-range sizes             */
    QK_EDTYPE = -3,       /* dtype not allowed for this precision           */
    QK_ENOMEM = -4,       /* workspace allocation failed                    */
    QK_EHIP = -5,         /* a HIP runtime call or launch failed            */
    QK_EUNSUPPORTED = -6  /* valid request outside what the kernels support */
} qk_status;

typedef enum { QK_F32 = 0, QK_BF16 = 1 } qk_dtype;

/* Arithmetic form of the step.  QK_PREC_FP32: features, samples and
 * projections in float32.  QK_PREC_BF16: features, samples and the Q/K/V/O
 * and decode projections in bfloat16 on the matrix cores with float32
 * accumulation.  QK_PREC_BF16_FP8PROJ: bfloat16 storage as QK_PREC_BF16, but
 * the Q/K/V/O projections take OCP e4m3 operands (per-tensor scales: query
 * input sqrt(C)/224, samples max|I|/224 over the level's feature maps --
 * measured on the device each call, one extra read of the maps --, weights
 * max|W|/224, attention output from its convex-combination bound), float32
 * accumulation; the decode stays bfloat16.  Reprojection, RMSNorm, softmax,
 * decode activations and compositing stay float32 in every form. */
typedef enum { QK_PREC_FP32 = 0, QK_PREC_BF16 = 1, QK_PREC_BF16_FP8PROJ = 2 } qk_precision;

/* How the decoded heads update depth and alpha (Sec. 3.2.2-3.2.3):
 * RESIDUAL  alpha' = sigmoid(logit(clamp(alpha, 1e-6, 1-1e-6)) + F'.w_sigma)
 *           (the clamp bounds are the float32 values nearest 1e-6 and 1-1e-6),
 *           disp'  = clamp(1/d + (0.5/L)(1/near - 1/far) tanh(F'.w_depth),
 *                          1/far, 1/near),  d' = 1/disp';
 * PAPER_DECODE  the paper's absolute decode: alpha' = sigmoid(F'.w_sigma),
 *           d' = 1/((delta + (0.5/L) tanh(F'.w_depth))(1/near - 1/far) + 1/far)
 *           with anchor delta = (l - 0.5)/L for the paper's layer l = L - index.
 * Both: colour c' = sigmoid(F' W_color). */
typedef enum { QK_UPDATE_RESIDUAL = 0, QK_UPDATE_PAPER_DECODE = 1 } qk_update_mode;

/* Attention form (Sec. 3.3).  STANDARD: per-sample key and value
 * projections, q = N(F) W_q, k_m = s_m W_k, v_m = s_m W_v,
 * F' = F + softmax_m(q.k_m / sqrt(d_h)) v_m W_o.  FOLDED ("one-to-many"): the
 * same result with W_k folded into the query and W_v into the output
 * projection, so no per-sample matrix multiply is done. */
typedef enum { QK_ATTN_STANDARD = 0, QK_ATTN_FOLDED = 1 } qk_attn_form;

typedef struct {
    double K[9];          /* host, row-major intrinsics on (width, height)  */
    double E[16];         /* host, row-major world-to-camera                */
    int32_t width, height;
} qk_camera;

/* One view's encoded feature map.  dtype: QK_F32 under QK_PREC_FP32,
 * QK_BF16 under the bfloat16 precisions (the LDM's dtype); C: the weights'
 * C_feat.  A map whose dtype or C disagrees is rejected (QK_EDTYPE,
 * QK_ESHAPE). */
typedef struct {
    const void *data;     /* device, [H][W][C] contiguous */
    qk_dtype dtype;
    int32_t H, W, C;
} qk_feature_map;

typedef struct {
    void *F;              /* device [L][H][W][C], dtype `dtype`; may be NULL
                             in an output LDM to skip writing F'           */
    float *depth;         /* device [L][H][W]                              */
    float *alpha;         /* device [L][H][W]                              */
    int32_t L, H, W, C;
    qk_dtype dtype;
} qk_ldm;

/* Projection weights, device float32 masters, row-major [in][out], no biases.
 *   Wq [C][heads*head_dim]      Wk, Wv [C_feat][heads*head_dim]
 *   Wo [heads*head_dim][C]      w_sigma, w_depth [C]     W_color [C][3]   */
typedef struct {
    const float *Wq, *Wk, *Wv, *Wo, *w_sigma, *w_depth, *W_color;
    int32_t C, C_feat, heads, head_dim;
} qk_weights;

/* Weight gradients: device float32, the shapes and layouts of qk_weights. */
typedef struct {
    float *Wq, *Wk, *Wv, *Wo, *w_sigma, *w_depth, *W_color;
} qk_weight_grads;

typedef struct qk_context qk_context;

/* Create a context bound to HIP device `device`.  The context owns device
 * workspaces that grow on demand and live until qk_context_destroy: the
 * folded weights of the one-to-many form (2 C C_feat floats per request),
 * the e4m3 scales (8 floats), the backward pass's scratch (16 bytes per
 * layer-pixel when d_rgb is given, plus 5 KiB per backward workgroup), the
 * render to input views' records (4 bytes per layer-pixel-view) or
 * projected planes, the low-resolution ray encodings, the residual block's
 * weight fragments and the batched launch's parameter table.  Growing one
 * synchronises the caller's stream and allocates.  `workspace_bytes` caps
 * their total (0: no cap): a call whose workspace would pass the cap
 * returns QK_ENOMEM, the message naming the bytes it needed (launches of
 * the same call before the failing growth may have been enqueued; they
 * write only the context's workspace).  A context may be used from one host
 * thread at a time; calls that share it on different streams race on its
 * workspaces.  Errors: QK_EINVAL (out == NULL, no such device), QK_EHIP. */
QK_API qk_status qk_context_create(int device, size_t workspace_bytes, qk_context **out);
QK_API qk_status qk_context_destroy(qk_context *ctx);

/* Declare the float32 weight masters the calls pass as static (enable != 0)
 * or not (0, the default).  Sec. 3.3 folds the key projection into the
 * query and the value projection into the output once, ahead of rendering;
 * while the weights are static the context likewise keeps the low-precision
 * copies it derives from masters -- the one-to-many form's folded weights
 * (qk_update_fuse, qk_batch_update_fuse) and the residual block's bfloat16
 * fragments (qk_residual_conv) -- keyed by the masters' device pointers
 * (and, for the folded weights, C, C_feat, heads, head_dim), and reuses them
 * on later calls instead of deriving them again on each.  A copy is made on
 * first use (it allocates, counts against the workspace cap and
 * synchronises that call's stream, so every later call on any stream reads
 * a complete copy); a context keeps at most 64, and derives the rest per
 * call.  The caller must not change static masters in place: to change
 * them, call this again (either value), which synchronises the device and
 * drops every kept copy.  qk_update_fuse_noalloc always derives per call.
 * Errors: QK_EINVAL (ctx == NULL), QK_EHIP. */
QK_API qk_status qk_context_weights_static(qk_context *ctx, int enable);

/* One Update & Fuse step of one LDM level (Sec. 3.2.2 "Iterative Updates",
 * Sec. 3.3 fusion block).  For every layer l, pixel p and view m: reproject
 * the layer-pixel through its depth into view m (the back-projection
 * operator of Sec. 3.1), bilinearly sample view m's feature map there (zero
 * padding; a point behind view m samples zero), attend from the
 * layer-pixel's RMS-normalised feature across its V samples, add the result
 * to F, and decode depth, alpha and colour from the updated feature.  If
 * `rgb_out` is non-NULL the updated layers are composited front to back
 * (Sec. 3.1, the over operator) into rgb_out [H][W][3] and, if non-NULL,
 * acc_alpha_out [H][W] = 1 - prod(1 - alpha').
 *
 *   V           number of views, 1..16
 *   in_cams     host [V];  feats device maps [V], each [Hf][Wf][C_feat]
 *   novel       host; its K is rescaled to the LDM grid (H, W)
 *   near_, far_ LDM frustum planes, 0 < near_ < far_
 *   ldm_in      current state; ldm_out receives F', depth', alpha'
 *               (ldm_out may alias ldm_in: each layer-pixel is read before
 *               it is written, by the same wave)
 * Attention has `heads` heads of `head_dim` channels (Sec. 3.3, the
 * MultiHead equation): head h takes channels h head_dim .. (h + 1)
 * head_dim - 1 of the Q, K and V projections, its own softmax over the
 * views with logits scaled by 1/sqrt(head_dim), and the heads' outputs,
 * concatenated, go through Wo.
 * Supported by the kernels: C == C_feat in {8, 16, 32, 64}, each feature
 * map under 1 GiB, and one head of C channels, or for C >= 32 in the
 * standard form heads x head_dim == C with head_dim 16 or 32 (or 8 at
 * C = 32: the paper's four heads of its 32 channels); otherwise
 * QK_EUNSUPPORTED.  QK_PREC_FP32 needs dtype
 * QK_F32, QK_PREC_BF16 and QK_PREC_BF16_FP8PROJ need QK_BF16 (else
 * QK_EDTYPE).
 * blend_logit_out, device [L][H][W][V] float or NULL: the blend-weight
 * logits of Sec. 3.2.3 -- the step's pre-softmax attention logits
 * a_m = q . k_m / sqrt(head_dim) (one-to-many form: q~ . s_m, the same
 * value), for the final fusion block whose softmax the render applies after
 * its upsampling.  One head only (else QK_EUNSUPPORTED). */
QK_API qk_status qk_update_fuse(qk_context *ctx, void *hip_stream, int32_t V,
                         const qk_camera *in_cams, const qk_feature_map *feats,
                         const qk_camera *novel, float near_, float far_,
                         const qk_weights *weights, qk_precision precision,
                         qk_attn_form attn_form, qk_update_mode update_mode,
                         const qk_ldm *ldm_in, const qk_ldm *ldm_out,
                         float *rgb_out, float *acc_alpha_out, float *blend_logit_out);

/* qk_update_fuse without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, checks, kernels and results as
 * qk_update_fuse.  Where qk_update_fuse keeps intermediate data in the
 * context's workspaces (grown with hipMalloc on first use) -- the folded
 * weights of QK_ATTN_FOLDED and the e4m3 scales of QK_PREC_BF16_FP8PROJ --
 * this entry point uses a fixed scratch array of 8256 floats (33 KiB) in
 * device memory instead, one per GPU, held until the process ends.  Limit:
 * the folded weights, 2 heads C C_feat floats, must fit 8192 floats (every
 * shape the folded kernels support does); larger returns QK_EUNSUPPORTED.
 * Every call on a GPU shares that GPU's scratch and overwrites what it
 * needs (the running maximum of the e4m3 scales is cleared by a kernel, not
 * a memset): calls that overlap on one GPU, on different streams or from
 * different threads, race on it. */
QK_API qk_status qk_update_fuse_noalloc(qk_context *ctx, void *hip_stream, int32_t V,
                                        const qk_camera *in_cams, const qk_feature_map *feats,
                                        const qk_camera *novel, float near_, float far_,
                                        const qk_weights *weights, qk_precision precision,
                                        qk_attn_form attn_form, qk_update_mode update_mode,
                                        const qk_ldm *ldm_in, const qk_ldm *ldm_out,
                                        float *rgb_out, float *acc_alpha_out,
                                        float *blend_logit_out);

/* ---- Batched Update & Fuse (serving: several requests in one launch) ----
 * One request of a batch: the arguments of qk_update_fuse for one LDM level
 * of one request (precision and attention form are the batch's). */
typedef struct {
    int32_t V;
    const qk_camera *in_cams;       /* host [V] */
    const qk_feature_map *feats;    /* host [V] of device maps */
    const qk_camera *novel;         /* host */
    float near_, far_;
    const qk_weights *weights;      /* host struct of device pointers */
    qk_update_mode update_mode;
    const qk_ldm *ldm_in;           /* host struct of device pointers */
    const qk_ldm *ldm_out;
    float *rgb_out;                 /* device [H][W][3] or NULL */
    float *acc_alpha_out;           /* device [H][W] or NULL */
    float *blend_logit_out;         /* device [L][H][W][V] or NULL (one head) */
} qk_request_desc;

/* Update & Fuse of n_req requests (1..64) in one kernel launch (Sec. 3.2.2
 * step, as qk_update_fuse, per request): requests may differ in LDM grid
 * (L, H, W), view count, cameras, feature maps, frustum, weights, update
 * mode and whether they composite or write blend-weight logits (as
 * qk_update_fuse's blend_logit_out); they share the feature width C, the
 * heads and head width, the precision (QK_PREC_BF16 only) and the attention
 * form.  Each request's outputs equal those of qk_update_fuse on its own,
 * bit for bit (the same per-tile kernel body).  Requests must not share
 * output buffers.  The requests' launch parameters (about 2.7 KiB each) go
 * to the device through pinned host staging in the context; the folded
 * weights of QK_ATTN_FOLDED take 2 heads C C_feat floats per request of the
 * context's workspace (both grown on demand, which synchronises the stream).
 * Errors (nothing enqueued): any request's qk_update_fuse error, prefixed
 * with its index; QK_ESHAPE (n_req); QK_EUNSUPPORTED (another precision,
 * requests of different C / heads, a grid of 2^31 tiles or more). */
QK_API qk_status qk_batch_update_fuse(qk_context *ctx, void *hip_stream, int32_t n_req,
                                      const qk_request_desc *reqs, qk_precision precision,
                                      qk_attn_form attn_form);

/* Dry run of qk_batch_update_fuse's argument checks (no device use). */
QK_API qk_status qk_batch_update_fuse_check(int32_t n_req, const qk_request_desc *reqs,
                                            qk_precision precision, qk_attn_form attn_form);

/* Dry run of qk_update_fuse's argument checks: returns the status the call
 * would return before enqueuing anything, without touching a device.  Takes
 * the same arguments minus the context and stream. */
QK_API qk_status qk_update_fuse_check(int32_t V, const qk_camera *in_cams,
                               const qk_feature_map *feats, const qk_camera *novel,
                               float near_, float far_, const qk_weights *weights,
                               qk_precision precision, qk_attn_form attn_form,
                               qk_update_mode update_mode, const qk_ldm *ldm_in,
                               const qk_ldm *ldm_out, float *rgb_out,
                               float *acc_alpha_out, float *blend_logit_out);

/* Learned initialisation of an LDM (Sec. 3.2, "Initialization"): one
 * C-channel feature f0 broadcast over every layer-pixel, each layer flat at
 * its depth anchor and alpha one half (the paper leaves the initial alpha
 * unstated; one half is this library's reading).  Storage layer i (0 =
 * nearest) is the paper's layer l = L - i, anchored at disparity fraction
 * delta = (l - 1/2)/L: depth = 1 / (delta (1/near - 1/far) + 1/far).
 *   f0    device [C] float32; a QK_BF16 LDM gets it rounded to nearest even
 *   ldm   device, written: F [L][H][W][C] of ldm->dtype, depth and alpha
 * C must be a positive multiple of 8 (QK_ESHAPE otherwise). */
QK_API qk_status qk_ldm_init(qk_context *ctx, void *hip_stream, const float *f0, float near_,
                             float far_, const qk_ldm *ldm);

/* Front-to-back over composite of L layers (Sec. 3.1): for each pixel,
 * T = 1; for l = 0..L-1: rgb += T alpha_l color_l; T *= 1 - alpha_l.
 *   color device [L][H][W][3] float, alpha device [L][H][W] float,
 *   rgb_out device [H][W][3], acc_alpha_out device [H][W] or NULL. */
QK_API qk_status qk_composite(qk_context *ctx, void *hip_stream, int32_t L, int32_t H, int32_t W,
                       const float *color, const float *alpha, float *rgb_out,
                       float *acc_alpha_out);

/* Adjoint of qk_composite (Sec. 3.1, the over operator O, differentiated by
 * the chain rule; the paper prints no adjoint).  With T_l = prod_{j<l}
 * (1 - alpha_j), B_{l+1} the composite of layers l+1..L-1 on their own and
 * P_{l+1} = prod_{j>l} (1 - alpha_j):
 *   d_color_l = d_rgb T_l alpha_l,
 *   d_alpha_l = T_l (d_rgb . (color_l - B_{l+1}) + d_acc P_{l+1}).
 * Float32 arithmetic, one thread per pixel, two passes over its layers.
 *   color   device [L][H][W][3] float, alpha device [L][H][W] float: the
 *           composite's inputs
 *   d_rgb   device [H][W][3] float, dLoss/drgb
 *   d_acc   device [H][W] float, dLoss/dacc_alpha, or NULL (zero)
 *   d_color device [L][H][W][3] float, written, or NULL (not computed)
 *   d_alpha device [L][H][W] float, written (also the pass's scratch)
 * Errors (nothing enqueued): QK_EINVAL (NULL where not allowed, a buffer
 * not 4-byte aligned, an output overlapping an input or the other output),
 * QK_ESHAPE (non-positive dims), QK_EUNSUPPORTED (2^40 elements or more). */
QK_API qk_status qk_composite_backward(qk_context *ctx, void *hip_stream, int32_t L, int32_t H,
                                       int32_t W, const float *color, const float *alpha,
                                       const float *d_rgb, const float *d_acc, float *d_color,
                                       float *d_alpha);

/* Dry run of qk_composite_backward's argument checks (no device use). */
QK_API qk_status qk_composite_backward_check(int32_t L, int32_t H, int32_t W, const float *color,
                                             const float *alpha, const float *d_rgb,
                                             const float *d_acc, const float *d_color,
                                             const float *d_alpha);

/* Per-view reprojection tables the kernels use: for view m on the level
 * grid, p = A_m (u, v, 1)^T + b_m / d with A_m = K_m R_m R_n^T K_n^-1 and
 * b_m = K_m (t_m - R_m R_n^T t_n), composed in double on the host and
 * rounded to float.  out [V][12] host = A row-major then b.  Exposed so the
 * host composition can be checked without a GPU. */
QK_API qk_status qk_camera_tables(int32_t V, const qk_camera *in_cams, const int32_t *feat_hw,
                           const qk_camera *novel, int32_t H, int32_t W, double *out);

/* Adjoint of one QK_PREC_FP32 Update & Fuse step and of the composite that
 * followed it.  The paper trains through generic differentiable rendering
 * and prints no adjoint; this is the chain rule through the forward of
 * Sec. 3.1-3.3 as qk_update_fuse defines it (reprojection, bilinear
 * back-projection, attention, decode, over composite).  The loss is any
 * function of the step's outputs; its gradients with respect to them come
 * in, the gradients with respect to every input go out.  The samples and
 * the attention are recomputed, not stored by the forward.
 *
 *   V, in_cams, feats, novel, near_, far_, weights, update_mode
 *               as given to the forward (feature maps QK_F32)
 *   ldm_in      the forward's input state (QK_F32)
 *   ldm_out     the forward's output: F' and alpha' are read to
 *               differentiate the composite; used only when d_rgb != NULL
 *   d_rgb       device [H][W][3] float, dLoss/drgb, or NULL (the step was
 *               not composited or rgb does not enter the loss)
 *   d_out       upstream dLoss/dF', dLoss/ddepth', dLoss/dalpha' as an LDM of
 *               the same shape (QK_F32); d_out or any of its three buffers
 *               may be NULL, meaning zero
 *   d_in        receives dLoss/dF, dLoss/ddepth, dLoss/dalpha (overwritten)
 *   d_feats     host array [V] of device pointers, each [Hf][Wf][C_feat]
 *               float: receives dLoss/dI_m (overwritten: cleared, then
 *               scatter-added with float atomics, so its last bits vary
 *               from run to run)
 *   d_weights   receives every weight gradient (overwritten, summed in a
 *               fixed order: bitwise reproducible)
 * Through a clamp (alpha outside (1e-6, 1 - 1e-6), disparity outside
 * (1/far, 1/near)) the gradient is zero; at a bilinear tap boundary the
 * one-sided derivative of the cell the sample falls in is taken.
 * Supported: heads == 1, C == C_feat == head_dim in {8, 16}; otherwise
 * QK_EUNSUPPORTED.  Buffers must not alias one another. */
QK_API qk_status qk_update_fuse_backward(qk_context *ctx, void *hip_stream, int32_t V,
                                  const qk_camera *in_cams, const qk_feature_map *feats,
                                  const qk_camera *novel, float near_, float far_,
                                  const qk_weights *weights, qk_update_mode update_mode,
                                  const qk_ldm *ldm_in, const qk_ldm *ldm_out,
                                  const float *d_rgb, const qk_ldm *d_out, const qk_ldm *d_in,
                                  float *const *d_feats, const qk_weight_grads *d_weights);

/* Dry run of qk_update_fuse_backward's argument checks (no device use). */
QK_API qk_status qk_update_fuse_backward_check(int32_t V, const qk_camera *in_cams,
                                        const qk_feature_map *feats, const qk_camera *novel,
                                        float near_, float far_, const qk_weights *weights,
                                        qk_update_mode update_mode, const qk_ldm *ldm_in,
                                        const qk_ldm *ldm_out, const float *d_rgb,
                                        const qk_ldm *d_out, const qk_ldm *d_in,
                                        float *const *d_feats,
                                        const qk_weight_grads *d_weights);

/* ---- Final render: Upsample & Activate, blend-weight image-based render ----
 * (Sec. 3.1, Eq. 1; Sec. 3.2.3 "Upsampling & Activation".)  The final LDM is
 * given as unactivated attributes on its own reduced grid (L, h, w); the
 * render produces the output image on an (H, W) grid, usually h = H/s,
 * w = W/s for the paper's scale factor s of 2 to 4.  For each layer l (0 =
 * nearest) and output pixel:
 *   1. bilinear upsampling of the depth logit x_d, the density logit x_s and
 *      the V blend-weight logits (half-pixel centres: output pixel x reads
 *      source coordinate (x + 0.5) w / W - 0.5, clamped below at 0; the tap
 *      x0 + 1 is clamped to the last column, i.e. the border extends);
 *   2. activation after the upsampling: alpha = sigmoid(x_s); disparity
 *      ((l_p - 0.5)/L + (0.5/L) tanh(x_d)) (1/near - 1/far) + 1/far with
 *      l_p = L - l (the paper's depth activation, its layer 1 the farthest),
 *      depth = 1/disparity; beta = softmax of the V blend logits;
 *   3. the back-projection of each input image onto the layer through that
 *      depth: the pixel centre is reprojected into image m (as in
 *      qk_update_fuse, cameras composed in double) and the image sampled
 *      bilinearly with zero padding; a point behind image m samples zero;
 *   4. layer colour c = sum_m beta_m sample_m;
 *   5. front-to-back over composite: rgb += T alpha c, depth_out += T alpha
 *      depth, T *= 1 - alpha; acc_out = 1 - T (black background).
 * All arithmetic is float32 except the reprojection (double: absolute
 * coordinates on 1080p images need more than a float's 24 bits).
 *
 *   V          number of input images, 1..16
 *   in_cams    host [V]; images device [V], RGBA8 [Hi][Wi][4] (alpha byte
 *              ignored, value v reads as v/255), rows packed, 4-byte aligned,
 *              each under 1 GiB
 *   novel      host; its K is rescaled to the output grid (H, W)
 *   near_, far_ the frustum planes of the depth activation, 0 < near_ < far_
 *   logits     device float32: depth_logit and sigma_logit [L][h][w],
 *              blend_logit [L][h][w][V] (V == the call's V)
 *   rgb_out    device [H][W][3] float32; acc_out and depth_out device
 *              [H][W] float32 or NULL
 * Errors (nothing enqueued): QK_EINVAL (NULL or misaligned buffer, bad
 * camera, near/far), QK_ESHAPE (non-positive dims, logits.V != V, V out of
 * range), QK_EUNSUPPORTED (an image of 1 GiB or more, an output or logit
 * volume of 2^31 elements or more). */
typedef struct {
    const void *data;     /* device RGBA8 [H][W][4] */
    int32_t H, W;
} qk_image;

typedef struct {
    const float *depth_logit;   /* device [L][H][W] */
    const float *sigma_logit;   /* device [L][H][W] */
    const float *blend_logit;   /* device [L][H][W][V] */
    int32_t L, H, W, V;
} qk_ldm_logits;

QK_API qk_status qk_render_ibr(qk_context *ctx, void *hip_stream, int32_t V,
                               const qk_camera *in_cams, const qk_image *images,
                               const qk_camera *novel, float near_, float far_,
                               const qk_ldm_logits *logits, int32_t H, int32_t W, float *rgb_out,
                               float *acc_out, float *depth_out);

/* Dry run of qk_render_ibr's argument checks (no device use). */
QK_API qk_status qk_render_ibr_check(int32_t V, const qk_camera *in_cams, const qk_image *images,
                                     const qk_camera *novel, float near_, float far_,
                                     const qk_ldm_logits *logits, int32_t H, int32_t W,
                                     const float *rgb_out, const float *acc_out,
                                     const float *depth_out);

/* ---- Render to input views (Sec. 3.2.2 "Decoding and rendering the
 * intermediate LDM", Eq. 2) ----
 * The decoded intermediate LDM -- per layer-pixel depth d, density sigma and
 * appearance a (RGB, already activated) on the LDM grid (L, H, W) -- is
 * rendered into each input view m on that view's grid (Hm, Wm):
 *   1. projection P_theta, the transpose of the bilinear back-projection of
 *      qk_update_fuse: each layer-pixel, reprojected through its depth to
 *      view m's continuous coordinate (cameras composed in double, the
 *      novel K rescaled to (W, H), view m's K to (Wm, Hm)), adds
 *      w * (a, sigma) to the four view pixels around that point with the
 *      bilinear weights w sampling there would use (half-pixel centres;
 *      taps outside the view are dropped, a point behind it adds nothing;
 *      no normalisation), each layer into its own plane;
 *   2. over composite of the projected planes, front to back (layer 0
 *      nearest the novel camera): rgb += T P(sigma) P(a),
 *      T *= 1 - P(sigma); acc = 1 - T.
 * Float32 arithmetic (reprojection in double).  Up to 128 layers (and view
 * sides below 65535, at most 2^31 layer-pixel-views) the sums of step 1 are
 * taken in 64-bit fixed point (each contribution w * (a, sigma), a float32
 * product, rounded to the nearest 2^-32) and the result is bitwise
 * reproducible; beyond that the planes are summed with float atomics, so
 * the order of the additions into a view pixel, and its last bits, vary
 * from run to run.
 *
 *   V          number of views, 1..16; in_cams host [V]
 *   novel      host; its K is rescaled to the LDM grid
 *   ldm        device float32 depth, alpha [L][H][W], color [L][H][W][3];
 *              depth > 0
 *   views      host [V]: device rgb [Hm][Wm][3] float32 and acc [Hm][Wm]
 *              float32 or NULL, with the view's grid
 * Workspace, in the context (grown on demand like the others): up to 128
 * layers, one 4-byte record (the layer-pixel's index) per layer-pixel-view
 * whose footprint meets the view (at most V L H W words) plus 3 counters per
 * tile of 32 x th view pixels (th = 16 for L <= 4, halved as L doubles);
 * beyond, the projected planes, sum over views of L Hm Wm 4 floats.
 * Errors (nothing enqueued): QK_EINVAL (NULL or misaligned buffer, bad
 * camera), QK_ESHAPE (non-positive dims, V out of range), QK_EUNSUPPORTED
 * (an LDM or a workspace of 2^31 elements or more). */
typedef struct {
    const float *depth;   /* device [L][H][W] */
    const float *alpha;   /* device [L][H][W] */
    const float *color;   /* device [L][H][W][3] */
    int32_t L, H, W;
} qk_ldm_decoded;

typedef struct {
    float *rgb;           /* device [H][W][3] */
    float *acc;           /* device [H][W] or NULL */
    int32_t H, W;
} qk_view_image;

QK_API qk_status qk_render_to_views(qk_context *ctx, void *hip_stream, int32_t V,
                                    const qk_camera *in_cams, const qk_camera *novel,
                                    const qk_ldm_decoded *ldm, const qk_view_image *views);

/* Dry run of qk_render_to_views's argument checks (no device use). */
QK_API qk_status qk_render_to_views_check(int32_t V, const qk_camera *in_cams,
                                          const qk_camera *novel, const qk_ldm_decoded *ldm,
                                          const qk_view_image *views);

/* ---- Residual CNN block of a fusion block (Sec. 3.3: the one-to-many
 * attention is interleaved with residual 3x3 convolutional blocks; each
 * fusion block of Sec. 3.2.2 is attention plus such blocks) ----
 * Per layer l, over the layer's (H, W) grid, with zero padding:
 *   F_out = F + W2 * gelu(W1 * N(F)),
 *   N(F) = F / sqrt(mean_c F^2 + 1e-6) per pixel (the attention's pre-norm),
 *   gelu(x) = x Phi(x) (the exact form),
 *   (W * X)(y, x)[co] = sum_{ky, kx, ci} X(y + ky - 1, x + kx - 1)[ci] W[ky][kx][ci][co].
 * bfloat16 feature volumes, MFMA bfloat16 operands with float32
 * accumulation; the normalised input and the GELU output are rounded to
 * bfloat16 as the convolutions' operands; the sum is rounded once.
 *   ldm_in, ldm_out  F [L][H][W][32] bfloat16 (depth, alpha unused; may be
 *                    NULL); ldm_out must not overlap ldm_in
 *   W1, W2           device float32 [3][3][32][32]
 * Workspace: the kernels' bfloat16 fragments (36 KiB) in the context.
 * Errors (nothing enqueued): QK_EINVAL (NULL, misaligned or overlapping
 * buffers), QK_ESHAPE (dims), QK_EDTYPE (not bfloat16), QK_EUNSUPPORTED
 * (C != 32). */
QK_API qk_status qk_residual_conv(qk_context *ctx, void *hip_stream, const qk_ldm *ldm_in,
                                  const float *W1, const float *W2, const qk_ldm *ldm_out);

/* Dry run of qk_residual_conv's argument checks (no device use). */
QK_API qk_status qk_residual_conv_check(const qk_ldm *ldm_in, const float *W1, const float *W2,
                                        const qk_ldm *ldm_out);

/* ---- Layer collapse (Sec. 3.2.2, "Layer Collapse"; the Lc blocks of the
 * network tables) ----
 * Halves the number of layers: for j = 0 .. L/2 - 1 and every pixel,
 *   out[j] = (F[2j] + F[2j+1]) / 2 + relu([F[2j], F[2j+1]] W1) W2,
 * [a, b] the 2C-channel concatenation, no biases.  bfloat16 volumes, MFMA
 * bfloat16 operands, float32 accumulation; the ReLU output is rounded to
 * bfloat16 as the second product's operand, the result once at the store.
 * Only the encoded features are collapsed: depth and alpha are decoded from
 * them afresh by the next step (QK_UPDATE_PAPER_DECODE).
 *   ldm_in   F [L][H][W][32] bfloat16, L even
 *   ldm_out  F [L/2][H][W][32] bfloat16, not overlapping ldm_in
 *   W1, W2   device float32 [64][32], [32][32]
 * Errors (nothing enqueued): QK_EINVAL (NULL, misaligned or overlapping),
 * QK_ESHAPE (odd L, dims), QK_EDTYPE (not bfloat16), QK_EUNSUPPORTED
 * (C != 32). */
QK_API qk_status qk_layer_collapse(qk_context *ctx, void *hip_stream, const qk_ldm *ldm_in,
                                   const float *W1, const float *W2, const qk_ldm *ldm_out);

/* Dry run of qk_layer_collapse's argument checks (no device use). */
QK_API qk_status qk_layer_collapse_check(const qk_ldm *ldm_in, const float *W1, const float *W2,
                                         const qk_ldm *ldm_out);

/* ---- Ray-direction encoding of the input views (Sec. 3.2.1: the encoded
 * input features of every pyramid level receive an encoding of their
 * pixels' ray directions; its form, "Encode Input Images" of Sec. 3.2.2)
 * ----
 * For a pixel (u, v) (half-pixel centres) of view m on a grid, the ray
 * through it (view m's K rescaled to the grid) is cut by the planes
 * z = near and z = far of the novel camera; both points are projected by
 * the novel camera (its K on its own grid, NDC = 2 (u, v) / (width,
 * height)) and their difference, far minus near, delta = (dx, dy), is
 * encoded as
 *   t = tanh(delta),
 *   e[4k + 0..3] = sin(2^k pi t_x), cos(2^k pi t_x), sin(2^k pi t_y), cos(2^k pi t_y),
 *   k = 0..7, and e Wr is ADDED to the feature map in place.
 * Two forms, by (low_H, low_W):
 *   (0, 0)   per pixel: every pixel of the map evaluates its own encoding;
 *   (h, w)   the paper's: the encoding is evaluated on the (h, w) grid and
 *            bilinearly upsampled to each map's grid (half-pixel centres,
 *            border extended) before it is added; one low-resolution grid
 *            serves every level (each with its own Wr).
 * The geometry and tanh in double, the sinusoids in double from one
 * quarter-period series and the double-angle identities, rounded to float;
 * the projection and the upsampling in float32 onto the feature, which is
 * rounded once to its dtype.  A ray parallel to the novel image plane
 * (d_z = 0 in the novel frame) gives non-finite values.
 *   V        number of views, 1..16; in_cams host [V]
 *   novel    host camera
 *   near, far  0 < near < far, in the novel frame's depth units
 *   Wr       device float32 [32][C], 16-byte aligned
 *   C        8, 16, 32 or 64
 *   dtype    of the feature maps (QK_F32 or QK_BF16)
 *   low_H, low_W  the low-resolution grid, or both 0
 *   feats    host [V]: device [H][W][C] maps, 16-byte aligned, written;
 *            no two may overlap.  Each map's `src` is NULL (the map is read
 *            and written in place) or a device [H][W][C] map of the same
 *            grid and dtype, 16-byte aligned, that is read instead, the
 *            encoded result going to `data` (src may equal data; otherwise
 *            it may not overlap any map's data).  The out-of-place form
 *            spares a caller that keeps the encoder's maps a copy per call.
 * Workspace (low-resolution form): V h w C floats in the context.
 * Errors (nothing enqueued): QK_EINVAL (NULL, misaligned or overlapping
 * buffers, bad camera, near/far), QK_ESHAPE (dims, V out of range, a
 * low-resolution grid with one side 0), QK_EDTYPE (dtype), QK_EUNSUPPORTED
 * (C, a map of 2^40 elements or more, a workspace of 2^31 floats or
 * more). */
typedef struct {
    void *data;           /* device [H][W][C], written (and read when src is NULL) */
    int32_t H, W;
    const void *src;      /* NULL, or device [H][W][C] read instead of data */
} qk_feature_map_inout;

QK_API qk_status qk_ray_encoding(qk_context *ctx, void *hip_stream, int32_t V,
                                 const qk_camera *in_cams, const qk_camera *novel, float near_,
                                 float far_, const float *Wr, int32_t C, qk_dtype dtype,
                                 int32_t low_H, int32_t low_W,
                                 const qk_feature_map_inout *feats);

/* Dry run of qk_ray_encoding's argument checks (no device use). */
QK_API qk_status qk_ray_encoding_check(int32_t V, const qk_camera *in_cams,
                                       const qk_camera *novel, float near_, float far_,
                                       const float *Wr, int32_t C, qk_dtype dtype,
                                       int32_t low_H, int32_t low_W,
                                       const qk_feature_map_inout *feats);

/* ---- Resolution transition (Sec. 3.2.2: the steps that grow the LDM
 * upsample the feature volume and the rendered views by two in each
 * spatial dimension; the appendix network tables give the grids) ----
 * Bilinear upsampling by exactly two, half-pixel centres, border extended:
 * dst[n][Y][X] samples src[n] at ((X + 0.5)/2 - 0.5, (Y + 0.5)/2 - 0.5),
 * i.e. blends of two rows and two columns with weights 1/4 and 3/4.
 * Float32 arithmetic, one rounding to the dtype at the store.
 *   src   device [N][H][W][C], dst device [N][2H][2W][C], one dtype
 *         (QK_F32 or QK_BF16), not overlapping; 16-byte aligned when C is
 *         a multiple of 8, else aligned to the element
 * Errors (nothing enqueued): QK_EINVAL (NULL, misaligned or overlapping),
 * QK_ESHAPE (dims), QK_EDTYPE, QK_EUNSUPPORTED (2^38 elements or more). */
QK_API qk_status qk_upsample2x(qk_context *ctx, void *hip_stream, const void *src, void *dst,
                               int32_t N, int32_t H, int32_t W, int32_t C, qk_dtype dtype);

/* Dry run of qk_upsample2x's argument checks (no device use). */
QK_API qk_status qk_upsample2x_check(const void *src, void *dst, int32_t N, int32_t H,
                                     int32_t W, int32_t C, qk_dtype dtype);

/* ---- Decode of an encoded LDM (Sec. 3.2.2: each step first decodes the
 * feature volume into an LDM; the absolute decode with the depth anchors
 * of Sec. 3.2.3, as QK_UPDATE_PAPER_DECODE) ----
 * For layer l (0 nearest) of L and every pixel, with F the C-channel
 * feature:
 *   alpha = sigmoid(F . w_sigma),  colour = sigmoid(F W_color),
 *   depth = 1 / ((delta_l + (0.5/L) tanh(F . w_depth)) (1/near - 1/far) + 1/far),
 *   delta_l = (L - l - 0.5) / L.
 * Float32 arithmetic.
 *   ldm        F [L][H][W][C] (QK_F32 or QK_BF16, C in {8, 16, 32, 64})
 *              read; depth, alpha [L][H][W] written
 *   w_sigma, w_depth  device float32 [C];  W_color device float32 [C][3]
 *   color_out  device float32 [L][H][W][3] or NULL
 * Errors (nothing enqueued): QK_EINVAL (NULL or misaligned, near/far),
 * QK_ESHAPE, QK_EDTYPE, QK_EUNSUPPORTED (C, 2^38 elements or more). */
QK_API qk_status qk_ldm_decode(qk_context *ctx, void *hip_stream, const qk_ldm *ldm,
                               const float *w_sigma, const float *w_depth,
                               const float *W_color, float near_, float far_,
                               float *color_out);

/* Dry run of qk_ldm_decode's argument checks (no device use). */
QK_API qk_status qk_ldm_decode_check(const qk_ldm *ldm, const float *w_sigma,
                                     const float *w_depth, const float *W_color, float near_,
                                     float far_, const float *color_out);

/* Unactivated decode of the final feature volume (Sec. 3.2.3: the final
 * LDM's depth and density are linear projections of V, activated only after
 * the render's bilinear upsampling): for every layer-pixel
 *   depth_logit = F . w_depth,  sigma_logit = F . w_sigma,
 * the inputs qk_render_ibr takes.  Float32 arithmetic.
 *   ldm          F [L][H][W][C] (QK_F32 or QK_BF16, C in {8, 16, 32, 64})
 *                read; its depth and alpha are not used
 *   w_sigma, w_depth  device float32 [C]
 *   depth_logit, sigma_logit  device float32 [L][H][W], written, not
 *                overlapping
 * Errors (nothing enqueued): QK_EINVAL (NULL, misaligned, overlapping),
 * QK_ESHAPE, QK_EDTYPE, QK_EUNSUPPORTED (C, 2^38 elements or more). */
QK_API qk_status qk_ldm_decode_logits(qk_context *ctx, void *hip_stream, const qk_ldm *ldm,
                               const float *w_sigma, const float *w_depth, float *depth_logit,
                               float *sigma_logit);

/* Dry run of qk_ldm_decode_logits's argument checks (no device use). */
QK_API qk_status qk_ldm_decode_logits_check(const qk_ldm *ldm, const float *w_sigma,
                                     const float *w_depth, const float *depth_logit,
                                     const float *sigma_logit);

QK_API const char *qk_last_error(void);
QK_API const char *qk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QUARK_H */
