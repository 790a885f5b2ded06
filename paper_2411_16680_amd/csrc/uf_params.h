// uf_params.h -- launch parameters shared by the host C-ABI and the kernels.
#pragma once
#include <stdint.h>

namespace qk {

constexpr int kMaxViews = 16;

// Fixed scratch of the allocation-free Update & Fuse entry point (floats):
// the folded weights W_qk, W_vo (2 heads C C_feat <= kScratchFold) and, after
// them, the e4m3 scales (7) and running maximum (1).
constexpr int kScratchFold = 8192;
constexpr int kScratchFloats = kScratchFold + 64;
constexpr int kMaxDevices = 64;

// One Update & Fuse launch over one LDM level.  Per view m, cam[m] holds the
// reprojection table p = A (u, v, 1)^T + b / d: A row-major (9 floats), then
// b (3 floats), composed in double on the host.
struct UFParams {
    const void *feat[kMaxViews];
    int32_t fH[kMaxViews];
    int32_t fW[kMaxViews];
    float cam[kMaxViews][12];
    double camd[kMaxViews][12];   // same tables in double (float32 form)

    const void *F_in;
    const float *depth_in;
    const float *alpha_in;
    void *F_out;           // may be NULL (skip F' store)
    float *depth_out;
    float *alpha_out;
    float *rgb;            // may be NULL (no composite)
    float *acc;            // may be NULL
    float *blend_logit;    // [L][H][W][V] attention logits (one head), or NULL

    const float *Wq, *Wk, *Wv, *Wo, *w_sigma, *w_depth, *W_color;
    const float *Wqk, *Wvo;    // folded weights (one-to-many form), C x C
    const float *f8_scales;    // [7] e4m3 scales (e4m3 projection form), device

    int32_t V, L, H, W;
    int32_t layers_per_chunk;  // layers handled by one workgroup
    int32_t x_blocks;          // ceil(W / pixels per workgroup)
    int32_t n_tiles;           // x_blocks * H * chunks (workgroups in the grid)
    int32_t chunks;
    float inv_near, inv_far;
    int32_t mode;              // 0 residual, 1 paper decode
};

// A batch of Update & Fuse requests in one launch (the requests' UFParams
// are in device memory): request r owns global tiles
// [tile_start[r], tile_start[r + 1]).
constexpr int kMaxBatch = 64;
struct UFBatch {
    int32_t tile_start[kMaxBatch + 1];
    int32_t n_req;
    int32_t total_tiles;
};

struct FoldParams {
    const float *Wq, *Wk, *Wv, *Wo;
    float *Wqk, *Wvo;              // [heads][C][Cf], [heads][Cf][C]
    int32_t C, Cf, hd, heads;      // hd: the width of one head
    float scale;                   // 1 / sqrt(hd)
};

struct CompParams {
    const float *color;    // [L][H][W][3]
    const float *alpha;    // [L][H][W]
    float *rgb;            // [H][W][3]
    float *acc;            // [H][W] or NULL
    int32_t L;
    int64_t npix;
};

// Adjoint of the standalone composite.
struct CompBwdParams {
    const float *color;    // [L][H][W][3]
    const float *alpha;    // [L][H][W]
    const float *d_rgb;    // [H][W][3]
    const float *d_acc;    // [H][W] or NULL (zero)
    float *d_color;        // [L][H][W][3] or NULL (not written)
    float *d_alpha;        // [L][H][W]
    int32_t L;
    int64_t npix;
};

}  // namespace qk

namespace qk {

// Weight-gradient tiles of the backward pass: 16 x 16 each, in this order:
// W_q, W_k, W_v, W_o, then the decode heads (columns sigma, depth, r, g, b).
constexpr int kGradTiles = 5;
constexpr int kGradTileElems = 256;

// Adjoint of one float32 Update & Fuse step (and of the composite).
struct BwdParams {
    const float *feat[kMaxViews];
    float *dfeat[kMaxViews];
    int32_t fH[kMaxViews];
    int32_t fW[kMaxViews];
    double camd[kMaxViews][12];

    const float *F_in, *depth_in, *alpha_in;
    const float *F_out, *alpha_out;     // forward outputs (read when d_rgb != NULL)
    const float *d_rgb;                 // [H][W][3] or NULL
    const float *dF_out, *d_depth_out, *d_alpha_out;   // upstream, each may be NULL
    float *dF, *d_depth, *d_alpha;

    const float *Wq, *Wk, *Wv, *Wo, *w_sigma, *w_depth, *W_color;
    float *dWq, *dWk, *dWv, *dWo, *dw_sigma, *dw_depth, *dW_color;

    float *comp;        // [L][H][W][4] composite adjoint (dc_r, dc_g, dc_b, dalpha)
    float *partials;    // [blocks][kGradTiles][256]

    int32_t V, L, H, W, C;
    int64_t N;          // L * H * W
    int32_t blocks;     // workgroups of the per-layer-pixel kernel
    float inv_near, inv_far, scale;
    int32_t mode;
};

}  // namespace qk

namespace qk {

// Learned initialisation of an LDM.
struct InitParams {
    const float *f0;        // [C] broadcast feature (device, float32)
    void *F;                // [L][H][W][C]
    float *depth, *alpha;   // [L][H][W]
    int64_t N, npix;        // L*H*W, H*W
    int32_t L, C;
    float inv_near, inv_far;
};

}  // namespace qk

namespace qk {

// Scales of the e4m3 projection form (see k_fp8.hip).
struct F8Params {
    const uint16_t *feat[kMaxViews];   // bfloat16 feature maps
    int64_t feat_elems[kMaxViews];
    int32_t V;
    const float *Wq, *Wk, *Wv, *Wo;    // folded form: Wq = W_qk, Wo = W_vo
    int32_t C, Cf, hd;
    int32_t fold;
    unsigned *amax_bits;               // workspace [1]
    float *scales;                     // out [7]
};

}  // namespace qk

namespace qk {

// Final render (upsample & activate, blend-weight image-based render).
struct RenderParams {
    const void *img[kMaxViews];     // RGBA8 [iH][iW][4]
    int32_t iH[kMaxViews], iW[kMaxViews];
    double cam[kMaxViews][12];      // output grid -> image m: A (9), b (3)
    const float *depth_logit;       // [L][h][w]
    const float *sigma_logit;       // [L][h][w]
    const float *blend_logit;       // [L][h][w][V]
    float *rgb;                     // [H][W][3]
    float *acc;                     // [H][W] or NULL
    float *depth;                   // [H][W] or NULL
    int32_t V, L, h, w, H, W;
    double rx, ry;                  // w / W, h / H (source step per output pixel)
    double band, inv_far;           // 1/near - 1/far, 1/far
};

}  // namespace qk

namespace qk {

// Render of a decoded intermediate LDM into the input views.
struct ViewsParams {
    double cam[kMaxViews][12];      // LDM grid -> view m's grid: A (9), b (3)
    int32_t vH[kMaxViews], vW[kMaxViews];
    int64_t sbase[kMaxViews];       // float offset of view m's [L][Hm][Wm][4] block in ws
    float *rgb[kMaxViews];          // [Hm][Wm][3]
    float *acc[kMaxViews];          // [Hm][Wm] or NULL
    float *ws;                      // projected layers, all views
    int64_t ws_floats;
    const float *depth, *alpha;     // [L][H][W]
    const float *color;             // [L][H][W][3]
    int32_t V, L, H, W;
    int64_t N;                      // L * H * W
    int64_t max_view_pixels;
    // binned form (no projected layers in memory): tiles of tw x th view
    // pixels, four bins per tile (the record classes), a bin's records
    // contiguous in rec
    int32_t binned;
    int32_t tw, th;
    int32_t ntx[kMaxViews], nty[kMaxViews];
    int32_t tbase[kMaxViews + 1];   // first tile of view m in the list of all views' tiles
    int32_t nbins;                  // 4 x tiles
    uint32_t *count;                // [nbins] records per bin
    uint32_t *start;                // [nbins + 1] exclusive prefix sums of count
    uint32_t *cursor;               // [nbins] next free record of a bin
    int32_t *rec;                   // [V N]: the layer-pixel index of each record
};

}  // namespace qk

namespace qk {

// Residual CNN block of a fusion block: F_out = F + W2 * relu(W1 * F), 3x3
// kernels, per layer, bfloat16 storage, C = 32.
struct ConvParams {
    const uint16_t *F;              // [L][H][W][32] bfloat16
    uint16_t *F_out;                // [L][H][W][32] bfloat16
    const float *W1, *W2;           // [3][3][32][32] float32 masters
    uint4 *frag;                    // workspace: bf16 weight fragments [2][9][2][64]
    int32_t L, H, W;
    int32_t tiles_x, tiles_y;       // output tiles per layer (set by the launcher)
    int64_t n_tiles;
};

}  // namespace qk

namespace qk {

// Layer collapse: out[j] = (F[2j] + F[2j+1]) / 2 + relu([F[2j], F[2j+1]] W1) W2,
// bfloat16 storage, C = 32.
struct CollapseParams {
    const uint16_t *F;              // [L][H][W][32]
    uint16_t *F_out;                // [L/2][H][W][32]
    const float *W1, *W2;           // [64][32], [32][32] float32 masters
    int32_t L;
    int64_t npix;                   // H * W
    int64_t n_blocks;               // 16-pixel blocks of the output
};

}  // namespace qk

namespace qk {

// Ray-direction encoding added to the input views' feature maps.
struct RayParams {
    double D[kMaxViews][9];         // (u, v, 1) on view m's grid -> ray direction, novel frame
    double o[kMaxViews][3];         // view m's centre in the novel frame
    void *feat[kMaxViews];          // [Hf][Wf][C], float32 or bfloat16, written
    const void *src[kMaxViews];     // the map read (feat[m] itself when in place)
    int32_t fH[kMaxViews], fW[kMaxViews];
    double kx0, kx1, ky0, ky1;      // (2/W_n) K_n[0][0..1], (2/H_n) K_n[1][0..1]
    double inv_band;                // 1/far - 1/near
    const float *Wr;                // [32][C]
    float *P;                       // low-resolution form: [V][lH][lW][C] workspace
    int32_t lH, lW;                 // low-resolution grid, 0 = per-pixel form
    int32_t V, C, bf16;
    int64_t max_pixels;
};

}  // namespace qk

namespace qk {

// Exact 2x bilinear upsampling of channel-last volumes [N][H][W][C].
struct Up2Params {
    const void *src;                // [N][H][W][C]
    void *dst;                      // [N][2H][2W][C]
    int32_t N, H, W, C, bf16;
};

// Decode of an encoded LDM (the paper's absolute decode).
struct DecodeParams {
    const void *F;                  // [L][H][W][C]
    const float *w_sigma, *w_depth, *W_color;   // [C], [C], [C][3]
    float *depth, *alpha, *color;   // [L][H][W], [L][H][W], [L][H][W][3] or null
    int32_t L, H, W, C, bf16;
    float inv_near, inv_far;
    int32_t logits;                 // 1: write F.w_depth, F.w_sigma unactivated
};

}  // namespace qk
