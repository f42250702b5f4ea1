/*
 * wsr.h — C-ABI of the sort-free Weighted Sum Rendering (WSR) rasterizer for
 * AMD Instinct MI355X (gfx950).
 *
 * The library renders 3D Gaussian scenes with the weighted sum of Sec. 4.2,
 * Eq. 7 of "Sort-free Gaussian Splatting via Weighted Sum Rendering":
 *
 *     C = (c_B w_B + sum_i c_i a_i) / (w_B + sum_i a_i),
 *     a_i = u_i w(d_i) exp(-q_i / 2)   for q_i <= tau, else 0,
 *
 * where q_i is the Mahalanobis form of pixel centre and projected Gaussian
 * (Sec. 3, Eqs. 3 and 5), c_i the SH colour (Eq. 4), u_i the maximum opacity
 * (sigmoid of a logit, Sec. 3; or the unclamped SH opacity of Sec. 4.3,
 * Eq. 11) and w the depth weight (Eqs. 8-10: DIR, EXP, LC).  No depth sort
 * happens anywhere: per-tile lists carry Gaussian ids only (Sec. 4.1).
 *
 * Conventions shared by every entry point
 *  - Pointers named *_dev, and every scene/gradient/image/workspace pointer,
 *    are DEVICE pointers owned by the caller.  Camera and parameter structs
 *    are HOST memory, read during the call only.
 *  - All work is enqueued on `stream` (a hipStream_t passed as void*; NULL
 *    means the default stream) and is asynchronous; no entry point
 *    allocates or frees device memory.  Only wsr_pair_count and wsr_check
 *    synchronise the stream.
 *  - Inputs are never modified.  Outputs are fully overwritten.
 *  - Host-detectable errors (null pointers, SH degree > 3, unsupported tile,
 *    workspace too small, more than WSR_MAX_VIEWS views) return an error
 *    status before anything is enqueued.  A per-tile list overflow is
 *    detected on the device: wsr_bin then records a flag in the workspace
 *    (read by wsr_check) and every later stage reads only in-bounds entries,
 *    so the images are incomplete but memory stays safe.
 *  - NaN / Inf inputs are not checked; they propagate.
 *  - Calls on one workspace must not overlap; different workspaces are
 *    independent.
 *
 * Multi-view images are concatenated: view v's image starts at pixel
 * sum_{v'<v} width_v' * height_v'; colours are [H][W][3] float32 and the
 * denominator [H][W] float32 per view.
 */
#ifndef WSR_H_
#define WSR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WSR_ABI_VERSION 6
#define WSR_MAX_VIEWS 256

typedef enum {
    WSR_OK = 0,
    WSR_ERR_INVALID = 1,     /* bad argument; nothing enqueued */
    WSR_ERR_WORKSPACE = 2,   /* workspace smaller than wsr_workspace_bytes */
    WSR_ERR_CAPACITY = 3,    /* per-tile list overflow (device flag) */
    WSR_ERR_HIP = 4,         /* a HIP runtime call failed */
    WSR_ERR_TILE_LIST = 5,   /* a tile list longer than wsr_sort_tiles takes (device flag) */
    WSR_ERR_STATIC = 6       /* larger than an allocation-free entry point's static workspace */
} wsr_status;

/* Depth weight w(d) of Sec. 4.2: Eq. 8 (DIR, w = 1), Eq. 9 (EXP,
 * w = exp(-sigma d^beta)), Eq. 10 (LC, w = max(0, 1 - d/sigma) v_i). */
typedef enum { WSR_WEIGHT_DIR = 0, WSR_WEIGHT_EXP = 1, WSR_WEIGHT_LC = 2 } wsr_weight_kind;

/* Maximum opacity: sigmoid(logit) in [0, 1] (Sec. 3), or the view-dependent
 * SH opacity u = SH_alpha(dir) + opacity_offset, unclamped (Sec. 4.3, Eq. 11). */
typedef enum { WSR_OPACITY_LOGIT = 0, WSR_OPACITY_SH = 1 } wsr_opacity_mode;

/* Storage type of means, log_scales, quats and sh.  Arithmetic is FP32 or
 * wider whatever the storage. */
typedef enum { WSR_STORE_F32 = 0, WSR_STORE_F16 = 1, WSR_STORE_BF16 = 2 } wsr_storage;

/* The scene model of Sec. 3 in planar structure-of-arrays layout.
 * K = (sh_degree + 1)^2.  Element type of the four `void` arrays is given
 * by `storage`; opacity_logit and lc_v are float32. */
typedef struct {
    int64_t n;                 /* number of Gaussians, >= 0 */
    int32_t sh_degree;         /* 0..3 */
    int32_t storage;           /* wsr_storage */
    int32_t opacity_mode;      /* wsr_opacity_mode */
    int32_t reserved_;
    const void* means;         /* [3][n]  centre p */
    const void* log_scales;    /* [3][n]  s = exp(log_scales) */
    const void* quats;         /* [4][n]  (w, x, y, z); normalised on load */
    const void* sh;            /* [K][n][4] RGBA per coefficient; A = opacity SH */
    const float* opacity_logit;/* [n]  used iff opacity_mode == LOGIT */
    const float* lc_v;         /* [n]  used iff weight kind == LC */
} wsr_scene;

/* Pinhole camera: world -> camera [R | T] row-major (+z forward, +y down),
 * focal lengths and principal point in pixels.  Pixel (px, py) is sampled at
 * (px + 0.5, py + 0.5). */
typedef struct {
    float viewmat[12];
    float fx, fy, cx, cy;
    int32_t width, height;
} wsr_camera;

/* Renderer settings.  tau is the support cutoff on q (a pair contributes iff
 * q <= tau); dilation is added to the diagonal of Sigma2D (px^2); near culls
 * Gaussians with camera-space z <= near; tile is 8, 16 or 32.
 * alpha_cut > 0 enables the opacity early-out that App. D proposes: a pair
 * also needs u exp(-q/2) >= alpha_cut (so q <= 2 ln(u / alpha_cut)), and a
 * Gaussian with u <= alpha_cut is culled.  It changes the image (opt-in);
 * 0 turns it off.  The sorted-blending entry points require 0.
 * batch is the number of splat records the raster stages in LDS per batch
 * (a tuning choice; the sums are the same): 0 for the default (64 for tile
 * 8, 256 otherwise), or 64 (tiles 8 and 16), 128 or 256 (tiles 16 and 32);
 * other values are WSR_ERR_INVALID. */
typedef struct {
    int32_t weight_kind;       /* wsr_weight_kind */
    int32_t tile;              /* 8 | 16 | 32 */
    float tau;                 /* 9 = 3-sigma ellipse */
    float dilation;            /* 0.3 */
    float near_z;              /* 0.2 */
    float opacity_offset;      /* 0.5; SH opacity mode only */
    int32_t flags;             /* WSR_FLAG_* */
    float alpha_cut;           /* opacity early-out threshold, >= 0; 0 = off */
    int32_t batch;             /* raster records staged per LDS batch; 0 = default */
} wsr_params;

/* wsr_render_fwd writes the raw sums instead of the image: out_rgb receives
 * sum_i c_i a_i and out_den sum_i a_i, without the background term.  Eq. 7
 * is a sum over Gaussians, so renders of disjoint subsets of a scene add up:
 * C = (c_B w_B + sum_shards N) / (w_B + sum_shards D).  This is how the path
 * shards Gaussians across devices. */
#define WSR_FLAG_UNNORMALISED 1

/* Weighted-blended order-independent transparency (Eq. 2, the operator the
 * method starts from) instead of Eq. 7, forward and backward:
 *     C = P c_B + (1 - P) (sum_i c_i a_i) / (sum_i a_i),  P = prod_i (1 - alpha_i),
 * with a_i = u_i w(d_i) exp(-q/2) as in Eq. 7 and alpha_i = u_i exp(-q/2)
 * clamped to [0, 1]; w_B is not used (its gradient is 0) and the weighted
 * average is 0 where its denominator vanishes.  wsr_render_fwd's out_den then
 * receives sum_i a_i.  Not combinable with WSR_FLAG_UNNORMALISED or
 * alpha_cut > 0, nor with the sorted-blending entry points. */
#define WSR_FLAG_OIT 2

/* Launch the raster stages as persistent grids: as many workgroups as the
 * device holds at once, each looping over the (view, tile) work items of all
 * views, instead of one workgroup per work item.  A scheduling choice: the
 * results are the same bit for bit. */
#define WSR_FLAG_PERSISTENT 4

/* Learnable global parameters, a DEVICE array of 6 floats:
 * [0] sigma, [1] beta (EXP only), [2] w_B, [3..5] c_B (RGB). */
#define WSR_GLOBALS 6

/* Gradient outputs (DEVICE, float32, same planar layouts as wsr_scene). */
typedef struct {
    float* means;              /* [3][n] */
    float* log_scales;         /* [3][n] */
    float* quats;              /* [4][n] */
    float* sh;                 /* [K][n][4]; A column zero in LOGIT mode */
    float* opacity_logit;      /* [n]; may be NULL in SH mode */
    float* lc_v;               /* [n]; may be NULL unless LC */
    float* globals;            /* [6], see WSR_GLOBALS */
} wsr_grads;

/* WSR_ABI_VERSION of the built library: a binding compares it with the
 * header it was written against before making any other call. */
int32_t wsr_abi_version(void);
/* A static, NUL-terminated description of a wsr_status value (the caller
 * does not free it); "unknown status" for any other value. */
const char* wsr_status_string(int32_t status);

/* Bytes of the workspace needed for n Gaussians over the given views and
 * tile size (does not include the per-pair buffer, see wsr_bin).
 * Returns -1 on invalid arguments. */
int64_t wsr_workspace_bytes(int64_t n, const wsr_camera* cams, int32_t n_views, int32_t tile);

/* Steps a1-a5 for every (view, Gaussian) pair (Sec. 3 Eqs. 3-5; Eq. 4;
 * Eqs. 8-11): view transform and near-plane cull, EWA projection with
 * dilation, conic, SH colour, opacity, depth weight, and the tile
 * rectangle of each splat's support ellipse.  Writes the workspace.
 * out_proj (nullable, DEVICE [n_views][n][16] float32) receives, per pair:
 * visible, mu_x, mu_y, conic A, B, C, r, g, b, u, w, depth, and four zeros. */
int32_t wsr_project(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views,
                    const wsr_params* params, const float* globals, void* ws, int64_t ws_bytes,
                    float* out_proj, void* stream);

/* Bytes per entry of the pair buffer (see wsr_bin). */
int64_t wsr_pair_bytes(void);

/* Step a6 (Sec. 4.1): build per-tile lists of Gaussian ids for every view,
 * with no depth key (Eq. 7 is a commutative sum, so no order is needed).
 * Each list holds its ids in increasing order, so the lists, and with them
 * every float sum of the later steps, are the same from run to run.
 * `pairs` is a DEVICE buffer of capacity * wsr_pair_bytes() bytes, aligned
 * to 256 bytes, that holds one entry per (tile, Gaussian) pair: the id lists
 * and per-pair scratch (the forward's split-tile partial sums and culling
 * masks, which the backward reuses, and the backward's partial gradients).
 * It is owned by the caller and must be passed unchanged to the later steps
 * of the same frame.  If the
 * number of pairs exceeds capacity the overflow flag is set (wsr_check,
 * wsr_pair_count give the needed capacity). */
int32_t wsr_bin(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                void* ws, int64_t ws_bytes, void* pairs, int64_t capacity, void* stream);

/* Step a7 (Eq. 7): per-pixel FP32 sums and normalisation with the weighted
 * background.  out_rgb: concatenated [H][W][3]; out_den: concatenated
 * [H][W] (w_B + sum a_i); out_count (nullable, int32 [H][W]): the number of
 * in-support pairs per pixel. */
int32_t wsr_render_fwd(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                       const float* globals, void* ws, int64_t ws_bytes, void* pairs,
                       int64_t capacity, float* out_rgb, float* out_den, int32_t* out_count,
                       void* stream);

/* Steps a8-a9: Eq. 7 differentiated per pixel and pair, then chained
 * through Eqs. 3-5 (EWA), Eq. 4 and Eq. 11 (SH colour and opacity) and
 * Eqs. 8-10 (depth weights) to the scene: the gradient of a loss L given
 * dL/dC (concatenated [H][W][3]), the forward's colour and denominator.  Recomputes every pair's amplitude
 * (nothing per pair is stored by the forward) and writes every field of
 * grads (they are overwritten, not accumulated).  out_grad2d (nullable,
 * DEVICE [n_views][n][9]) receives the per-(view, Gaussian) gradient with
 * respect to (mu_x, mu_y, A, B, C, r, g, b, a) where (A, B, C) is the conic
 * (q = A dx^2 + 2B dx dy + C dy^2) and a = u w the amplitude.  No atomics:
 * every sum is formed in a fixed order, so for given inputs the result does
 * not vary from run to run (nor does that of the forward or the binning). */
int32_t wsr_render_bwd(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views,
                       const wsr_params* params, const float* globals, void* ws, int64_t ws_bytes,
                       void* pairs, int64_t capacity, const float* dL_drgb, const float* rgb,
                       const float* den, const wsr_grads* grads, float* out_grad2d, void* stream);

/* The two halves of wsr_render_bwd, for callers that schedule or time them
 * separately; wsr_render_bwd is exactly wsr_raster_bwd then wsr_project_bwd.
 * wsr_raster_bwd (step a8, Eq. 7 differentiated) leaves one partial 2D
 * gradient per (tile, Gaussian) pair in `pairs` and per-tile background
 * partial sums in the workspace; wsr_project_bwd (step a9) sums each
 * Gaussian's partials and chains them to the scene parameters (Eqs. 3-11
 * differentiated), writing `grads`. */
int32_t wsr_raster_bwd(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                       const float* globals, void* ws, int64_t ws_bytes, void* pairs,
                       int64_t capacity, const float* dL_drgb, const float* rgb, const float* den,
                       void* stream);
int32_t wsr_project_bwd(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views,
                        const wsr_params* params, const float* globals, void* ws, int64_t ws_bytes,
                        const void* pairs, int64_t capacity, const wsr_grads* grads,
                        float* out_grad2d, void* stream);

/* Adam settings of wsr_project_bwd_adam: one learning rate per attribute
 * group, the decay rates, eps and the step number (from 1) of the bias
 * correction, as in wsr_adam. */
typedef struct {
    float lr_means, lr_log_scales, lr_quats;
    float lr_sh0;              /* SH coefficient 0 (RGBA) */
    float lr_shN;              /* SH coefficients 1..K-1 */
    float lr_opacity_logit, lr_lc_v;
    float beta1, beta2, eps;
    int32_t step;
    int32_t reserved_;
} wsr_adam_params;

/* wsr_project_bwd and one Adam step (wsr_adam's update) of the per-Gaussian
 * parameters in a single pass, for the training step of Sec. 5: every
 * gradient is applied where it is formed instead of being written to memory
 * and read back.  The result is bit for bit that of wsr_project_bwd followed
 * by wsr_adam on each array with the same settings.  The scene must use
 * FP32 storage and its arrays must be writable DEVICE memory: means,
 * log_scales, quats and sh are updated in place, and opacity_logit and lc_v
 * too where they, m's and v's fields are all non-NULL.  m and v (DEVICE,
 * the layouts of wsr_grads, `globals` fields unused) are the first and
 * second moments, read and written.  grad_globals (DEVICE [6]) receives the
 * gradient of the global parameters (WSR_GLOBALS), which this call does not
 * update (wsr_adam does, on the caller's side).  Returns WSR_ERR_INVALID for
 * 16-bit storage, missing arrays, step < 1 or a beta outside [0, 1),
 * before anything is enqueued. */
int32_t wsr_project_bwd_adam(const wsr_scene* scene, const wsr_camera* cams, int32_t n_views,
                             const wsr_params* params, const float* globals, void* ws, int64_t ws_bytes,
                             const void* pairs, int64_t capacity, const wsr_grads* m, const wsr_grads* v,
                             const wsr_adam_params* adam, float* grad_globals, float* out_grad2d,
                             void* stream);

/* Synchronises `stream` and returns, in *out_total, the number of
 * (tile, Gaussian) pairs the last wsr_bin on this workspace produced (the
 * size the id list needs). */
int32_t wsr_pair_count(const void* ws, int64_t ws_bytes, int64_t* out_total, void* stream);

/* Synchronises `stream`; returns WSR_ERR_CAPACITY if the last wsr_bin on
 * this workspace overflowed its id list, WSR_ERR_TILE_LIST if a wsr_sort_tiles
 * since then met a list longer than WSR_SORT_MAX, else WSR_OK. */
int32_t wsr_check(const void* ws, int64_t ws_bytes, void* stream);

/* ---- Sorted alpha blending (Eq. 6): the baseline the method removes the
 * sort from (Sec. 1, Sec. 4.1) -----------------------------------------
 *
 * Renders the same splats front to back: project with weight_kind
 * WSR_WEIGHT_DIR (so a splat's amplitude is its opacity u), bin, sort each
 * tile's list by camera depth, then composite
 *     C = sum_i c_i alpha_i T_i + T c_B,  alpha_i = min(alpha_max, u_i exp(-q_i / 2)),
 *     T_i = prod_{j<i} (1 - alpha_j),
 * skipping layers with alpha_i < alpha_min and stopping a pixel once its
 * transmittance falls below t_min (0 and 0 give Eq. 6 exactly; 1/255 and
 * 1e-4 are the usual 3D Gaussian Splatting settings).  Forward only. */
#define WSR_SORT_MAX 16384

typedef struct {
    float alpha_max;   /* opacity clamp, (0, 1] */
    float alpha_min;   /* layers below this are skipped, >= 0 */
    float t_min;       /* a pixel stops below this transmittance, >= 0 */
    int32_t reserved_;
} wsr_blend;

/* Sorts every tile's id list (as left by wsr_bin on the same workspace and
 * pair buffer) by (camera depth, Gaussian id), in place, one workgroup per
 * tile in LDS.  The lists stay valid input for wsr_render_fwd and the
 * backward (Eq. 7 does not depend on their order).  A list longer than
 * WSR_SORT_MAX is left unsorted and raises a flag that wsr_check reports as
 * WSR_ERR_TILE_LIST.  Asynchronous. */
int32_t wsr_sort_tiles(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                       void* ws, int64_t ws_bytes, void* pairs, int64_t capacity, void* stream);

/* Front-to-back composition of the sorted lists.  params->weight_kind must
 * be WSR_WEIGHT_DIR (else WSR_ERR_INVALID).  globals as for wsr_project
 * (c_B = globals[3..5]).  out_rgb: DEVICE concatenated [H][W][3]; out_T:
 * DEVICE concatenated [H][W], the final transmittance.  Asynchronous. */
int32_t wsr_render_sorted(const wsr_camera* cams, int32_t n_views, const wsr_params* params, int64_t n,
                          const float* globals, const wsr_blend* blend, void* ws, int64_t ws_bytes,
                          const void* pairs, int64_t capacity, float* out_rgb, float* out_T, void* stream);

/* ---- Training step around the renderer (Sec. 5, implementation details) ----
 *
 * The paper trains with the rendering loss of 3D Gaussian Splatting: an l1
 * term plus a D-SSIM term weighted 0.2.  Per view v with P_v = 3 H W entries
 *   L_v = (1 - lambda) mean|x - y| + lambda (1 - mean SSIM(x, y)),
 * and L = mean over views.  SSIM is computed per colour channel under an
 * 11 x 11 Gaussian window (sigma 1.5) with zero padding, C1 = 0.01^2 and
 * C2 = 0.03^2 (Wang et al. 2004, dynamic range 1).
 *
 * Size in bytes of the workspace wsr_loss needs for these cameras (only width
 * and height are read), or -1 for invalid input. */
int64_t wsr_loss_workspace_bytes(const wsr_camera* cams, int32_t n_views);

/* Loss and its gradient.  img, target: DEVICE float [P][3], views
 * concatenated in camera order (the layout wsr_render_fwd writes).  Writes
 * the DEVICE scalar *loss and DEVICE dL_dimg [P][3] (overwritten).  The
 * workspace (DEVICE, caller-owned, 256-byte aligned) holds the derivative maps
 * and per-tile loss shares; the shares are summed in FP64 in a fixed order,
 * so the result does not vary from run to run.  Asynchronous on `stream`.
 * Returns WSR_ERR_INVALID for null pointers, n_views outside
 * [1, WSR_MAX_VIEWS], an empty or oversized view or lambda outside [0, 1];
 * WSR_ERR_WORKSPACE if ws_bytes is too small. */
int32_t wsr_loss(const wsr_camera* cams, int32_t n_views, const float* img, const float* target, float lambda,
                 void* ws, int64_t ws_bytes, float* loss, float* dL_dimg, void* stream);

/* Size in bytes of the static workspace of wsr_loss_noalloc, per device:
 * 72 MiB, enough for one 1920 x 1080 view (wsr_loss_workspace_bytes of
 * such a camera is 74,845,440 bytes). */
#define WSR_LOSS_STATIC_BYTES (72ll << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc: wsr_loss without a workspace argument.  Same arguments,
 * results and errors as wsr_loss (the same kernels), but the workspace is a
 * static device array of WSR_LOSS_STATIC_BYTES bytes that the library holds
 * on every device it runs on until the process ends.  Calls on the current
 * device (`stream` must belong to it); nothing is allocated or freed.
 * Returns WSR_ERR_STATIC, before anything is enqueued, when
 * wsr_loss_workspace_bytes(cams, n_views) exceeds WSR_LOSS_STATIC_BYTES
 * (about 2.09 M pixels in all).  Every call on a device shares that
 * device's array, which keeps the last call's contents (each call writes
 * every byte it reads first, so nothing needs clearing): calls that overlap
 * on one device, on any streams, race and must be ordered by the caller. */
int32_t wsr_loss_noalloc(const wsr_camera* cams, int32_t n_views, const float* img, const float* target,
                         float lambda, float* loss, float* dL_dimg, void* stream);

/* One Adam update (Kingma and Ba 2015, with bias correction) of n DEVICE
 * floats in place: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  step counts
 * from 1.  param, m and v are read and written, grad is read.  Asynchronous
 * on `stream`.  Returns WSR_ERR_INVALID for null pointers with n > 0,
 * n < 0, step < 1 or beta outside [0, 1). */
int32_t wsr_adam(float* param, const float* grad, float* m, float* v, int64_t n, int32_t step, float lr,
                 float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WSR_H_ */
