/* Drives every argument check of the C-ABI, the camera composition and the
 * entry points' early error returns (no device), for a build under the
 * address and undefined-behaviour sanitizers.  Exit status 0 when every
 * status is the expected one. */
#include <stdio.h>
#include <stdint.h>
#include <string.h>

#include "quark.h"

static int fails = 0;

static void expect(const char *what, qk_status got, qk_status want) {
    if (got != want) {
        printf("FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want, qk_last_error());
        ++fails;
    }
}

#define P(a) ((void *)(uintptr_t)(a))

static void camera(qk_camera *c, double tx, int w, int h) {
    memset(c, 0, sizeof(*c));
    c->K[0] = 50.0; c->K[2] = 0.5 * w; c->K[4] = 50.0; c->K[5] = 0.5 * h; c->K[8] = 1.0;
    for (int i = 0; i < 4; ++i) c->E[5 * i] = 1.0;
    c->E[3] = -tx;
    c->width = w;
    c->height = h;
}

int main(void) {
    enum { V = 3, L = 4, H = 6, W = 10, C = 32 };
    qk_camera cams[V], nov;
    qk_feature_map fm[V];
    for (int m = 0; m < V; ++m) {
        camera(&cams[m], 0.1 * m, W, H);
        fm[m].data = P(0x100000 + 0x10000 * m);
        fm[m].dtype = QK_BF16;
        fm[m].H = H;
        fm[m].W = W;
        fm[m].C = C;
    }
    camera(&nov, 0.05, W, H);
    qk_weights w = {P(0x600000), P(0x610000), P(0x620000), P(0x630000), P(0x640000),
                    P(0x650000), P(0x660000), C, C, 1, C};
    qk_ldm in = {P(0x300000), P(0x400000), P(0x500000), L, H, W, C, QK_BF16};
    qk_ldm out = {P(0x310000), P(0x410000), P(0x510000), L, H, W, C, QK_BF16};
    float *rgb = P(0x700000), *acc = P(0x710000), *bl = P(0x720000);

    expect("update_fuse ok", qk_update_fuse_check(V, cams, fm, &nov, 0.5f, 20.0f, &w, QK_PREC_BF16,
                                                   QK_ATTN_STANDARD, QK_UPDATE_RESIDUAL, &in, &out,
                                                   rgb, acc, bl), QK_OK);
    fm[1].dtype = QK_F32;
    expect("update_fuse map dtype", qk_update_fuse_check(V, cams, fm, &nov, 0.5f, 20.0f, &w, QK_PREC_BF16,
                                                   QK_ATTN_STANDARD, QK_UPDATE_RESIDUAL, &in, &out,
                                                   rgb, acc, bl), QK_EDTYPE);
    fm[1].dtype = QK_BF16;
    fm[1].C = 16;
    expect("update_fuse map C", qk_update_fuse_check(V, cams, fm, &nov, 0.5f, 20.0f, &w, QK_PREC_BF16,
                                                   QK_ATTN_STANDARD, QK_UPDATE_RESIDUAL, &in, &out,
                                                   rgb, acc, bl), QK_ESHAPE);
    fm[1].C = C;
    expect("update_fuse dtype", qk_update_fuse_check(V, cams, fm, &nov, 0.5f, 20.0f, &w, QK_PREC_FP32,
                                                      QK_ATTN_STANDARD, QK_UPDATE_RESIDUAL, &in,
                                                      &out, rgb, acc, NULL), QK_EDTYPE);
    expect("update_fuse near/far", qk_update_fuse_check(V, cams, fm, &nov, 5.0f, 5.0f, &w,
                                                         QK_PREC_BF16, QK_ATTN_FOLDED,
                                                         QK_UPDATE_PAPER_DECODE, &in, &out, NULL,
                                                         NULL, NULL), QK_EINVAL);
    expect("update_fuse views", qk_update_fuse_check(0, cams, fm, &nov, 0.5f, 20.0f, &w, QK_PREC_BF16,
                                                      QK_ATTN_STANDARD, QK_UPDATE_RESIDUAL, &in,
                                                      &out, NULL, NULL, NULL), QK_ESHAPE);
    qk_weights w4 = w;
    w4.heads = 4;
    w4.head_dim = 8;
    expect("update_fuse heads+blend", qk_update_fuse_check(V, cams, fm, &nov, 0.5f, 20.0f, &w4,
                                                            QK_PREC_BF16, QK_ATTN_STANDARD,
                                                            QK_UPDATE_RESIDUAL, &in, &out, NULL,
                                                            NULL, bl), QK_EUNSUPPORTED);
    qk_camera bad = nov;
    bad.K[8] = 2.0;
    expect("update_fuse camera", qk_update_fuse_check(V, cams, fm, &bad, 0.5f, 20.0f, &w,
                                                       QK_PREC_BF16, QK_ATTN_STANDARD,
                                                       QK_UPDATE_RESIDUAL, &in, &out, NULL, NULL,
                                                       NULL), QK_EINVAL);
    expect("update_fuse null ctx", qk_update_fuse(NULL, NULL, V, cams, fm, &nov, 0.5f, 20.0f, &w,
                                                  QK_PREC_BF16, QK_ATTN_STANDARD,
                                                  QK_UPDATE_RESIDUAL, &in, &out, NULL, NULL, NULL),
           QK_EINVAL);
    expect("noalloc null ctx", qk_update_fuse_noalloc(NULL, NULL, V, cams, fm, &nov, 0.5f, 20.0f,
                                                      &w, QK_PREC_BF16, QK_ATTN_STANDARD,
                                                      QK_UPDATE_RESIDUAL, &in, &out, NULL, NULL,
                                                      NULL), QK_EINVAL);

    qk_request_desc rq[2];
    for (int r = 0; r < 2; ++r) {
        rq[r].V = V; rq[r].in_cams = cams; rq[r].feats = fm; rq[r].novel = &nov;
        rq[r].near_ = 0.5f; rq[r].far_ = 20.0f; rq[r].weights = &w;
        rq[r].update_mode = QK_UPDATE_PAPER_DECODE; rq[r].ldm_in = &in; rq[r].ldm_out = &out;
        rq[r].rgb_out = NULL; rq[r].acc_alpha_out = NULL; rq[r].blend_logit_out = NULL;
    }
    expect("batch ok", qk_batch_update_fuse_check(2, rq, QK_PREC_BF16, QK_ATTN_FOLDED), QK_OK);
    expect("batch precision", qk_batch_update_fuse_check(2, rq, QK_PREC_FP32, QK_ATTN_FOLDED),
           QK_EUNSUPPORTED);
    expect("batch count", qk_batch_update_fuse_check(65, rq, QK_PREC_BF16, QK_ATTN_FOLDED),
           QK_ESHAPE);
    rq[1].near_ = 30.0f;
    expect("batch request", qk_batch_update_fuse_check(2, rq, QK_PREC_BF16, QK_ATTN_FOLDED),
           QK_EINVAL);

    /* backward: float32, one head of 16 */
    qk_weights w16 = {P(0x600000), P(0x610000), P(0x620000), P(0x630000), P(0x640000),
                      P(0x650000), P(0x660000), 16, 16, 1, 16};
    qk_feature_map fm32[V];
    for (int m = 0; m < V; ++m) {
        fm32[m] = fm[m];
        fm32[m].dtype = QK_F32;
        fm32[m].C = 16;
    }
    qk_ldm in32 = {P(0x300000), P(0x400000), P(0x500000), L, H, W, 16, QK_F32};
    qk_ldm out32 = {P(0x310000), P(0x410000), P(0x510000), L, H, W, 16, QK_F32};
    qk_ldm din = {P(0x320000), P(0x420000), P(0x520000), L, H, W, 16, QK_F32};
    float *dfe[V] = {P(0x800000), P(0x810000), P(0x820000)};
    qk_weight_grads dw = {P(0x900000), P(0x910000), P(0x920000), P(0x930000), P(0x940000),
                          P(0x950000), P(0x960000)};
    expect("backward ok", qk_update_fuse_backward_check(V, cams, fm32, &nov, 0.5f, 20.0f, &w16,
                                                        QK_UPDATE_RESIDUAL, &in32, &out32, rgb,
                                                        NULL, &din, dfe, &dw), QK_OK);
    expect("backward width", qk_update_fuse_backward_check(V, cams, fm32, &nov, 0.5f, 20.0f, &w,
                                                           QK_UPDATE_RESIDUAL, &in, &out, rgb,
                                                           NULL, &din, dfe, &dw),
           QK_EDTYPE);

    /* composite and its adjoint */
    expect("composite null ctx", qk_composite(NULL, NULL, L, H, W, rgb, acc, rgb, NULL), QK_EINVAL);
    expect("composite bwd ok", qk_composite_backward_check(L, H, W, P(0x100000), P(0x200000),
                                                           P(0x300000), NULL, P(0x400000),
                                                           P(0x500000)), QK_OK);
    expect("composite bwd overlap", qk_composite_backward_check(L, H, W, P(0x100000), P(0x200000),
                                                                P(0x300000), NULL, P(0x100040),
                                                                P(0x500000)), QK_EINVAL);

    /* final render, render to views, residual block, collapse, ray
     * encoding, resampling, decode */
    qk_image im[V];
    for (int m = 0; m < V; ++m) { im[m].data = P(0x100000 + 0x10000 * m); im[m].H = H; im[m].W = W; }
    qk_ldm_logits lg = {P(0x200000), P(0x210000), P(0x220000), L, 3, 5, V};
    expect("render ok", qk_render_ibr_check(V, cams, im, &nov, 0.5f, 20.0f, &lg, H, W, rgb, acc,
                                            NULL), QK_OK);
    lg.V = V + 1;
    expect("render views", qk_render_ibr_check(V, cams, im, &nov, 0.5f, 20.0f, &lg, H, W, rgb, acc,
                                               NULL), QK_ESHAPE);
    qk_ldm_decoded dec = {P(0x200000), P(0x210000), P(0x220000), L, H, W};
    qk_view_image vi[V];
    for (int m = 0; m < V; ++m) { vi[m].rgb = P(0x300000 + 0x10000 * m); vi[m].acc = NULL; vi[m].H = H; vi[m].W = W; }
    expect("views ok", qk_render_to_views_check(V, cams, &nov, &dec, vi), QK_OK);
    qk_ldm vin = {P(0x300000), NULL, NULL, L, H, W, 32, QK_BF16};
    qk_ldm vout = {P(0x380000), NULL, NULL, L, H, W, 32, QK_BF16};
    expect("conv ok", qk_residual_conv_check(&vin, P(0x500000), P(0x510000), &vout), QK_OK);
    expect("conv overlap", qk_residual_conv_check(&vin, P(0x500000), P(0x510000), &vin), QK_EINVAL);
    qk_ldm cout_ = {P(0x380000), NULL, NULL, L / 2, H, W, 32, QK_BF16};
    expect("collapse ok", qk_layer_collapse_check(&vin, P(0x500000), P(0x510000), &cout_), QK_OK);
    qk_feature_map_inout fio[V];
    for (int m = 0; m < V; ++m) {
        fio[m].data = P(0x100000 + 0x10000 * m); fio[m].H = H; fio[m].W = W; fio[m].src = NULL;
    }
    expect("ray ok", qk_ray_encoding_check(V, cams, &nov, 0.5f, 20.0f, P(0x500000), 32, QK_BF16, 3, 5,
                                           fio), QK_OK);
    fio[1].src = P(0x900000);
    expect("ray src ok", qk_ray_encoding_check(V, cams, &nov, 0.5f, 20.0f, P(0x500000), 32, QK_BF16,
                                               3, 5, fio), QK_OK);
    fio[1].src = fio[0].data;
    expect("ray src overlap", qk_ray_encoding_check(V, cams, &nov, 0.5f, 20.0f, P(0x500000), 32,
                                                    QK_BF16, 3, 5, fio), QK_EINVAL);
    fio[1].src = NULL;
    expect("ray grid", qk_ray_encoding_check(V, cams, &nov, 0.5f, 20.0f, P(0x500000), 32, QK_BF16, 0,
                                             5, fio), QK_ESHAPE);
    expect("upsample ok", qk_upsample2x_check(P(0x100000), P(0x200000), 2, H, W, 8, QK_F32), QK_OK);
    qk_ldm dl = {P(0x300000), P(0x400000), P(0x500000), L, H, W, 32, QK_BF16};
    expect("decode ok", qk_ldm_decode_check(&dl, P(0x600000), P(0x610000), P(0x620000), 0.5f, 20.0f,
                                            NULL), QK_OK);
    expect("logits ok", qk_ldm_decode_logits_check(&dl, P(0x600000), P(0x610000), P(0x700000),
                                                   P(0x710000)), QK_OK);

    /* host camera composition */
    int32_t fhw[2 * V];
    double tab[12 * V];
    for (int m = 0; m < V; ++m) { fhw[2 * m] = H; fhw[2 * m + 1] = W; }
    expect("camera tables", qk_camera_tables(V, cams, fhw, &nov, H, W, tab), QK_OK);
    if (!(tab[0] > 0.99 && tab[0] < 1.01)) { printf("FAIL camera table A00 %g\n", tab[0]); ++fails; }

    /* without a GPU, creating a context reports an error */
    qk_context *ctx = NULL;
    qk_status st = qk_context_create(0, 0, &ctx);
    if (st == QK_OK) qk_context_destroy(ctx);
    expect("context (NULL out)", qk_context_create(0, 0, NULL), QK_EINVAL);
    expect("weights static (NULL context)", qk_context_weights_static(NULL, 1), QK_EINVAL);
    printf("%s: %d failures (%s)\n", qk_version(), fails, st == QK_OK ? "a device" : "no device");
    return fails ? 1 : 0;
}
