/*
 * asgs.h - C ABI of libasgs, the MI355X (gfx950) anchor-Gaussian render hot path.
 *
 * The library computes, for one or more camera views:
 *   decode          anchors -> k neural Gaussians each through five two-layer
 *                   head MLPs (UP-SLAM Sec. 3.3, Eq. 8 and Eq. 9; MLP details
 *                   in the appendix);
 *   render_forward  EWA projection of the Gaussians (Sec. 3.1, Eq. 2), tile
 *                   binning (a counting sort on the tile, then every tile list
 *                   sorted on (depth, index) on its own), and
 *                   front-to-back alpha compositing of colour, depth, the opacity
 *                   sum (Eq. 3) and the low-dimensional feature (Eq. 10);
 *   render_backward the vector-Jacobian product of render_forward w.r.t. the
 *                   Gaussian parameters and the SE(3) camera pose;
 *   decode_backward the vector-Jacobian product of decode w.r.t. anchors, the
 *                   head-MLP parameters and (through the view direction) the
 *                   camera pose.
 *
 * Conventions (shared by every call):
 *  - Every array argument is a DEVICE pointer owned by the caller, except the
 *    structs themselves, which live in host memory and are read before the
 *    call returns. The library never allocates or frees device memory: scratch
 *    and the forward->backward context are caller buffers sized by the
 *    *_size queries.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL = the null stream) except asgs_render_count and asgs_ctx_status,
 *    which synchronise that stream to read a device counter.
 *  - Status: every call returns an asgs_status. Arguments are validated on
 *    the host before anything is launched, so a failing call launches
 *    nothing. asgs_last_error() gives a thread-local message for the last
 *    failing call on the calling thread.
 *  - Layouts: per-Gaussian attributes are planes [c][n] (structure of
 *    arrays, n contiguous). Images are planes [c][H][W] per view, views
 *    packed back to back: view v starts at element (sum of H*W over views
 *    before v) * c of each output array.
 *  - Pixel (px, py) is evaluated at the integer point (px, py). Quaternions
 *    are (w, x, y, z), normalised inside the projection. T_wc is the 3x4
 *    row-major camera-to-world pose; the world-to-camera rotation is taken as
 *    the transpose of its rotation block.
 *  - Pose gradients are w.r.t. the twist xi = (rho, phi) of the left
 *    perturbation T_cw <- Exp(xi) T_cw, T_cw = T_wc^-1, evaluated at xi = 0.
 */
#ifndef ASGS_H
#define ASGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASGS_ABI_VERSION 1
#define ASGS_MAX_VIEWS 64      /* views per call */
#define ASGS_MAX_K 16          /* Gaussians per anchor */

typedef enum asgs_status {
  ASGS_OK = 0,
  ASGS_E_INVALID = 1,      /* null pointer, bad size, misaligned (< 16 B) array, non-finite pose */
  ASGS_E_WORKSPACE = 2,    /* caller buffer too small; the message states the bytes needed */
  ASGS_E_CAPACITY = 3,     /* more tile/Gaussian intersections than the context holds */
  ASGS_E_DEVICE = 4,       /* a HIP runtime error; the message holds hipGetErrorString */
  ASGS_E_UNSUPPORTED = 5   /* valid but not built: n_feat not 0/16, tile != 16, k > 16 ... */
} asgs_status;

int asgs_abi_version(void);
const char* asgs_status_string(int status);
/* Thread-local message of the last failing call on this thread (never NULL). */
const char* asgs_last_error(void);

/* Pinhole camera, one per view. */
typedef struct asgs_camera {
  int32_t width, height;   /* pixels, 1..16384 each */
  float fx, fy, cx, cy;    /* focal lengths and principal point, pixels */
  float T_wc[12];          /* row-major 3x4 camera-to-world pose (Sec. 3.1) */
  float t;                 /* frame time of the view (finite); read only by decoders with the
                              temporal input (in_dim 38, Sec. 3.3 Temporal Encoding) */
} asgs_camera;

/* Rasteriser constants. asgs_render_opts_default fills the values the paper's
 * vanilla-3DGS framework uses (Sec. 3.1). */
typedef struct asgs_render_opts {
  int32_t tile;            /* screen tile side in pixels; must be 16 */
  int32_t n_feat;          /* low-dimensional feature channels N_l: 0 or 16 */
  float alpha_min;         /* 1/255: alpha below this is skipped */
  float alpha_max;         /* 0.99: alpha is clamped to this */
  float T_min;             /* 1e-4: stop before transmittance falls below this */
  float dilation;          /* 0.3 px^2 added to the 2D covariance diagonal */
  float znear;             /* 0.2: cull Gaussians with camera depth <= znear */
  float fov_clamp;         /* 1.3: Jacobian x/z clamp, in units of W/(2 fx); 0 = off */
  float bg[3];             /* background colour (colour channels only) */
  int32_t extent_mode;     /* footprint listed in the tiles: 0 = the tight box of the alpha >= alpha_min
                              ellipse (default; compositing then equals per-pixel evaluation), 1 = the
                              square of half side ceil(3 sqrt(lambda_max(Sigma'))) of vanilla 3DGS */
} asgs_render_opts;

void asgs_render_opts_default(asgs_render_opts* opts);

/* Gaussians of every view of a call. Field f of view v is at
 * ptr_f + v * view_stride[f] (elements); stride 0 shares one array across
 * views (e.g. the means, which do not depend on the view). Field order of
 * view_stride: mean, scale, rot, opacity, rgb, feat. */
typedef struct asgs_gaussians {
  int64_t n;               /* Gaussians per view, 1 .. 2^26 */
  float* mean;             /* [3][n] world position */
  float* scale;            /* [3][n] linear scale (s of Sigma = R S S^T R^T) */
  float* rot;              /* [4][n] quaternion (w,x,y,z), any norm > 0 */
  float* opacity;          /* [n]    opacity in (0, 1) */
  float* rgb;              /* [3][n] colour */
  float* feat;             /* [n_feat][n] low-dimensional feature, NULL if n_feat == 0 */
  int64_t view_stride[6];
} asgs_gaussians;

/* Rendered maps of all views, packed (see Layouts above). */
typedef struct asgs_images {
  float* rgb;              /* [3][H][W] colour + T_final * bg */
  float* depth;            /* [H][W] sum of w_i z_i, z = camera depth (not normalised) */
  float* feat;             /* [n_feat][H][W], NULL if n_feat == 0 */
  float* alpha;            /* [H][W] opacity sum of Eq. 3 = 1 - T_final */
} asgs_images;

/* ---------------------------------------------------------------------------
 * Rendering
 * ------------------------------------------------------------------------- */

/* Bytes of a render context for n_views cameras, n_gauss Gaussians per view
 * and at most `capacity` tile/Gaussian intersections (all views together).
 * Pure host arithmetic. */
int asgs_render_ctx_size(const asgs_camera* cams, int32_t n_views, int64_t n_gauss,
                         const asgs_render_opts* opts, int64_t capacity, size_t* bytes);

/* Runs the projection of all views into `ctx` and returns the exact number of
 * tile/Gaussian intersections in *n_isect (the value to size a context for).
 * Synchronises `stream`. The context needs capacity >= 0 for this call. */
int asgs_render_count(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                      const asgs_render_opts* opts, void* ctx, size_t ctx_bytes,
                      int64_t* n_isect, void* stream);

/* Forward render of n_views views (Eq. 2, Eq. 3, Eq. 10) into `out`.
 * `ctx` (asgs_render_ctx_size bytes, 256-byte aligned) receives everything
 * render_backward needs and stays valid until the caller reuses it. If the
 * intersections exceed the context's capacity, the excess is dropped, the
 * context records the overflow (asgs_ctx_status) and the images are
 * incomplete; the call itself cannot see this without a synchronisation. */
int asgs_render_forward(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                        const asgs_render_opts* opts, const asgs_images* out,
                        void* ctx, size_t ctx_bytes, void* stream);

/* Backward of render_forward for the same cams, g, opts and ctx. d_out holds
 * dL/d(outputs) in the output layout (d_out->alpha may be NULL = zero; feat
 * must be given when n_feat > 0). d_g receives dL/d(every field of g),
 * overwritten, with the same view strides as g except that a stride of 0 is
 * not allowed (each view gets its own gradient). d_pose, if not NULL,
 * receives [n_views][6] dL/d(rho, phi), overwritten. */
int asgs_render_backward(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                         const asgs_render_opts* opts, const asgs_images* d_out,
                         const asgs_gaussians* d_g, float* d_pose, void* ctx,
                         size_t ctx_bytes, void* stream);

/* Reads the context header: intersections of the last forward/count, number
 * of visible (view, Gaussian) pairs, and a non-zero overflow flag if the
 * capacity was exceeded. Synchronises `stream`. */
int asgs_ctx_status(const void* ctx, void* stream, int64_t* n_isect, int64_t* n_visible,
                    int32_t* overflow);

/* Internal arrays of a context after render_forward, for inspection:
 *  ASGS_CTX_PAIR_TILE   uint32[I]   tile key of each sorted intersection
 *                                   (view tile offset + ty * tiles_x + tx)
 *  ASGS_CTX_PAIR_GAUSS  uint32[I]   view * n + gaussian of each sorted intersection
 *  ASGS_CTX_TILE_RANGE  uint32[T][2] [start, end) of each tile key
 *  ASGS_CTX_RECT        int16[V*n][4] tx0, tx1, ty0, ty1 (empty rect: tx0 > tx1)
 *  ASGS_CTX_NCONTRIB    uint32[P]   per pixel: list position + 1 of the last
 *                                   composited Gaussian of its tile
 *  ASGS_CTX_TFINAL      float[P]    per pixel final transmittance
 *  ASGS_CTX_GEOM        float[V*n][8] u, v, conic A, B, C, opacity, ln(alpha_min / o), 0;
 *                                   written for the (view, Gaussian) pairs whose radius
 *                                   entry is >= 0, undefined for the others
 *  ASGS_CTX_RADIUS      float[V*n][2] footprint half-widths r_x, r_y in whole pixels
 *                                   (ceil of sqrt(2 ln(o / alpha_min) Sigma'), Eq. 2),
 *                                   -1 for pairs culled before the footprint
 *  ASGS_CTX_DEPTH_KEY   uint32[V*n] float32 bits of the camera depth that orders the
 *                                   tile lists; 0xFFFFFFFF for pairs that touch no tile
 *  ASGS_CTX_NTILES      uint32[V*n] tiles of the pair's rectangle, 0 when not listed
 * Tile rectangle of a listed pair from its geometry and radii (integer
 * arithmetic, T = tile side): tx0 = max(0, floor((floor(u) - r_x) / T)),
 * tx1 = min(tiles_x - 1, floor((floor(u) + r_x) / T)), ty likewise with v, r_y.
 * cams/n_views/n_gauss/opts/ctx_bytes must be those of the forward call.
 * `*ptr` is a device pointer inside ctx and `*count` its element count
 * (for the pair arrays: the capacity; read I from asgs_ctx_status). */
enum {
  ASGS_CTX_PAIR_TILE = 1,
  ASGS_CTX_PAIR_GAUSS = 2,
  ASGS_CTX_TILE_RANGE = 3,
  ASGS_CTX_RECT = 4,
  ASGS_CTX_NCONTRIB = 5,
  ASGS_CTX_TFINAL = 6,
  ASGS_CTX_GEOM = 7,
  ASGS_CTX_RADIUS = 8,
  ASGS_CTX_DEPTH_KEY = 9,
  ASGS_CTX_NTILES = 10
};
int asgs_ctx_array(const asgs_camera* cams, int32_t n_views, int64_t n_gauss,
                   const asgs_render_opts* opts, void* ctx, size_t ctx_bytes, int32_t which,
                   void** ptr, int64_t* count);

/* ---------------------------------------------------------------------------
 * Anchor decoding (Sec. 3.3, Eq. 8 and Eq. 9)
 *
 * Each anchor v has a position x_v, a 32-d feature f_v and k offsets O_vi.
 * Input X_v = [f_v (32), delta_v (3)], delta_v = (x_v - c)/|x_v - c|, c the
 * camera centre of the view (in_dim 35); the scene-variant decoders append
 * the distance |x_v - c| (in_dim 36) and then the temporal embedding
 * (sin pi t, cos pi t) of the camera's frame time t (in_dim 38; Sec. 3.3,
 * Temporal Encoding). Five heads h in the order opacity(m=1), rgb(3),
 * scale(3), rot(4), feat(n_feat): Y_h = W2_h act_h(W1_h X + b1_h) + b2_h,
 * act = ReLU for the first four, SoftPlus for feat; W1_h is [32][in_dim],
 * W2_h is [k*m_h][32]. Gaussian n = v*k + i gets opacity sigmoid(Y[i]), rgb
 * sigmoid(Y[3i..]), scale l_s * sigmoid(Y[3i..]), rot Y[4i..], feat
 * Y[16i..], mean x_v + l_o * O_vi.
 *
 * Parameters of all heads live in one float array, per head in the order
 * above: W1's first 35 columns (32*35, row-major), b1 (32), W2 (k*m*32,
 * row-major), b2 (k*m), then W1's remaining in_dim - 35 columns (32 rows of
 * in_dim - 35, row-major; nothing for in_dim 35). The 35-input parameters
 * are thus a prefix of each head's block.
 * ------------------------------------------------------------------------- */

typedef struct asgs_decoder {
  int64_t n_anchors;       /* A >= 1 */
  int32_t k;               /* Gaussians per anchor, 1..16 */
  int32_t n_feat;          /* 0 or 16 (feature head present when 16) */
  int32_t precision;       /* 0 = FP32; 1 = forward with BF16 operands on the matrix cores and FP32
                              accumulation (n_anchors * k <= 2^27, else ASGS_E_UNSUPPORTED). The
                              backward always recomputes and differentiates in FP32. */
  float l_o;               /* offset scale (metres) */
  float l_s;               /* scale bound (metres) */
  int32_t in_dim;          /* head input width: 35 (or 0, the same), 36 (+ distance) or 38 (+ distance
                              and temporal embedding); others ASGS_E_UNSUPPORTED */
} asgs_decoder;

/* Number of floats of the packed head parameters. */
int asgs_decode_param_count(const asgs_decoder* d, int64_t* count);

/* Decode anchors for n_views cameras. anchor_xyz [3][A], anchor_feat [A][32],
 * anchor_off [3][A*k]; out->n must be A*k. out view strides apply per view;
 * the mean field is written for view 0 only (it does not depend on the view)
 * and must be non-NULL there. */
int asgs_decode(const asgs_decoder* d, const float* anchor_xyz, const float* anchor_feat,
                const float* anchor_off, const float* params, const asgs_camera* cams,
                int32_t n_views, const asgs_gaussians* out, void* stream);

/* Bytes of scratch asgs_decode_backward needs. */
int asgs_decode_workspace_size(const asgs_decoder* d, int32_t n_views, size_t* bytes);

/* Backward of asgs_decode: d_g holds dL/d(decoded Gaussians) per view (the
 * mean gradient is summed over views). Writes (overwrites) d_xyz [3][A],
 * d_feat [A][32], d_off [3][A*k], d_params (packed like params); ADDS the
 * camera-centre term of the pose gradient to d_pose [n_views][6] if not
 * NULL (render_backward writes the rest of it). Pose-only mode: with
 * d_xyz, d_feat, d_off and d_params all NULL only the camera-centre term is
 * computed (d_pose required); the parameter-gradient kernels are skipped.
 * Any other mix of NULL outputs is ASGS_E_INVALID. */
int asgs_decode_backward(const asgs_decoder* d, const float* anchor_xyz, const float* anchor_feat,
                         const float* anchor_off, const float* params, const asgs_camera* cams,
                         int32_t n_views, const asgs_gaussians* d_g, float* d_xyz, float* d_feat,
                         float* d_off, float* d_params, float* d_pose, void* work,
                         size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Weighted L1 residual of rendered maps (the photometric, depth and feature
 * residual of the tracking and mapping losses, UP-SLAM Eq. 4 and Sec. 3.4)
 * and its gradient, in one pass. For view v, pixel p, channel group g (rgb,
 * depth, feat, alpha) with a target:
 *   loss[v] += scale[g] * w_p * |x - x*|,   grad = scale[g] * w_p * sign(x - x*)
 * with sign(0) = 0 and w_p = weight[p] (1 when weight is NULL). Maps,
 * targets and gradients are packed like asgs_images for n_views views of
 * width x height; a group whose target is NULL contributes nothing and its
 * gradient plane (if not NULL) is zeroed; NULL gradient planes are not
 * written. loss (NULL or device [n_views]) needs work of
 * asgs_l1_loss_work_size bytes; without loss, work may be NULL. Every map,
 * target, gradient and weight pointer must be 16-byte aligned (ASGS_E_INVALID
 * otherwise). The loss is a fixed-order sum (deterministic run to run).
 * ------------------------------------------------------------------------- */
typedef struct asgs_l1_targets {
  const float* rgb;     /* [n_views][3][H][W] or NULL */
  const float* depth;   /* [n_views][H][W] or NULL */
  const float* feat;    /* [n_views][n_feat][H][W] or NULL */
  const float* alpha;   /* [n_views][H][W] or NULL */
  const float* weight;  /* [H][W] per-pixel weight shared by the views, or NULL */
  float scale[4];       /* multipliers of the rgb, depth, feat and alpha terms */
} asgs_l1_targets;

int asgs_l1_loss_work_size(int32_t n_views, size_t* bytes);
int asgs_l1_loss(int32_t n_views, int32_t width, int32_t height, int32_t n_feat, const asgs_images* maps,
                 const asgs_l1_targets* targets, const asgs_images* grad, float* loss, void* work,
                 size_t work_bytes, void* stream);

/* Allocation-free asgs_l1_loss, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, results and status codes without
 * work/work_bytes. The loss partials live in a library-owned device array of
 * ASGS_L1_NOALLOC_MAX_VIEWS * 512 floats (128 KiB) that each GPU the library
 * runs on holds until the process ends; its address is looked up on the
 * first call on a device (the device current at the call must be the
 * stream's). Nothing in it needs clearing: every call writes all the
 * partials it reads. Calls that overlap on one GPU share the array and race:
 * serialise them (one stream, or events). n_views above
 * ASGS_L1_NOALLOC_MAX_VIEWS is ASGS_E_UNSUPPORTED. Allocates nothing. */
#define ASGS_L1_NOALLOC_MAX_VIEWS 64
int asgs_l1_loss_noalloc(int32_t n_views, int32_t width, int32_t height, int32_t n_feat,
                         const asgs_images* maps, const asgs_l1_targets* targets, const asgs_images* grad,
                         float* loss, void* stream);

/* Forward render fused with the weighted L1 residual: the same images as
 * asgs_render_forward, plus, in the forward's output stage, exactly the
 * gradient planes asgs_l1_loss(out, targets, grad) would write (same
 * arithmetic, bitwise equal) and, if loss is not NULL (device [n_views]),
 * the per-view loss as a fixed-order sum over tiles (equal to asgs_l1_loss's
 * value up to the order of the FP32 sum). Saves the separate pass over the
 * maps (the tracking loss of Sec. 3.4 in one kernel). targets and grad are
 * packed like the images (weight [H][W] shared by the views); a group
 * without target gets a zeroed gradient plane, NULL gradient planes are not
 * written; with n_feat = 0 the feature group is ignored. ctx and the
 * capacity rules are those of asgs_render_forward; after an overflow the
 * residual is that of the incomplete images. */
int asgs_render_forward_l1(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                           const asgs_render_opts* opts, const asgs_images* out,
                           const asgs_l1_targets* targets, const asgs_images* grad, float* loss,
                           void* ctx, size_t ctx_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Multi-modal tracking residual and per-pixel uncertainty (UP-SLAM Sec. 3.2,
 * Eq. 6; Sec. 3.4, Eq. 15)
 *
 * Per pixel of view v, from the rendered colour C~, depth D~ and opacity sum
 * alpha (Eq. 3), the cosine of the DINO feature F and the rendered
 * high-dimensional feature F^ (Eq. 11), and the observed colour C and depth D:
 *   R     = vis (w_rgb sum_c |C~_c - C_c| + w_depth |D~ - box3(D)| + w_feat min(1, 1 - cos)),
 *           vis = (1 - alpha < vis_T), box3 = mean of D over the pixel's in-image 3x3 neighbourhood;
 *   sigma = max(sigma_min, sqrt(2 R)), the minimiser over sigma >= sigma_min of the
 *           pixel's term 1/2 (R / sigma^2 + log sigma) of Eq. 15;
 *   dynamic = 2 sigma^2 > dyn_thresh (evaluated as 2 max(sigma_min^2, 2R) > dyn_thresh):
 *           the motion mask (1 = dynamic);
 *   xi[v] = the mean over the view's pixels of that term at sigma (Eq. 15's value).
 * ------------------------------------------------------------------------- */
typedef struct asgs_residual_opts {
  float w_rgb, w_depth, w_feat;  /* residual weights lambda_1^t..3^t: 0.25, 0.7, 0.1 (appendix) */
  float vis_T;                   /* 0.1: pixels with remaining transmittance below this contribute */
  float sigma_min;               /* 1e-3: lower bound of sigma (> 0) */
  float dyn_thresh;              /* 1: motion mask threshold on 2 sigma^2 (Eq. 14's criterion) */
  int32_t reserved;              /* must be 0 */
} asgs_residual_opts;

typedef struct asgs_residual_maps {
  const float* rgb;        /* [V][3][H][W] rendered colour */
  const float* depth;      /* [V][H][W] rendered depth */
  const float* alpha;      /* [V][H][W] rendered opacity sum */
  const float* cosine;     /* [V][H][W] cos(F, F^) (asgs_feature_lift) */
  const float* obs_rgb;    /* [V][3][H][W] observed colour */
  const float* obs_depth;  /* [V][H][W] observed depth */
} asgs_residual_maps;

void asgs_residual_opts_default(asgs_residual_opts* opts);
/* Bytes of work asgs_tracking_residual needs to produce xi. */
int asgs_residual_work_size(int32_t n_views, int32_t width, int32_t height, size_t* bytes);
/* Writes the outputs that are not NULL: R, sigma ([V][H][W] float), dynamic
 * ([V][H][W] uint8), xi ([V] float, needs work). Device pointers, no
 * alignment requirement. At least one output must be given. Asynchronous
 * on stream; xi is a fixed-order sum (deterministic). */
int asgs_tracking_residual(int32_t n_views, int32_t width, int32_t height, const asgs_residual_opts* opts,
                           const asgs_residual_maps* in, float* R, float* sigma, uint8_t* dynamic, float* xi,
                           void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Feature lift F_m and cosine distillation (UP-SLAM Sec. 3.3, Eq. 11, Eq. 12)
 *
 * Per pixel p of view v, the rendered low-dimensional feature x = F~_p (16
 * channels, Eq. 10) is lifted by the per-pixel MLP F_m (1x1 convolutions):
 *   h = relu(W1 x + b1) (128),  F^_p = W2 h + b2 (N_h),
 * and compared with the DINO feature F_p, the patch grid dino upsampled
 * bilinearly to the image (sample centres at half-integers, clamped):
 *   cos_p = F_p . F^_p / max(|F_p| |F^_p|, 1e-12),   loss[v] = mean_p (1 - cos_p).
 * The per-pixel cosine is also the feature term of the tracking residual.
 * Parameters, packed float: W1 [128][16], b1 [128], W2 [N_h][128], b2 [N_h].
 * F^ is never formed: F . F^ and |F^|^2 are evaluated through W2^T F (per
 * patch) and the Gram matrix W2^T W2 (FP32 sums of products taken on the
 * matrix cores with high and low bfloat16 parts, three products per pair).
 * ------------------------------------------------------------------------- */
typedef struct asgs_feature_lift {
  int32_t n_high;          /* N_h, channels of the DINO features: 1..1024 */
  int32_t grid_h, grid_w;  /* patch grid of the DINO features; at most 3 patches per 16 pixels */
  int32_t reserved;        /* must be 0 */
} asgs_feature_lift;

int asgs_feature_param_count(const asgs_feature_lift* f, int64_t* count);
/* Bytes of work both calls need for n_views views of width x height. */
int asgs_feature_workspace_size(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height,
                                size_t* bytes);
/* feat [V][16][H][W] rendered features, params (packed), dino [V][N_h][grid_h][grid_w];
 * writes cosine [V][H][W] and, if not NULL, loss [V] (fixed-order sums). */
int asgs_feature_forward(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height,
                         const float* feat, const float* params, const float* dino, float* cosine, float* loss,
                         void* work, size_t work_bytes, void* stream);
/* Backward of the cosine map: d_cos [V][H][W] = dL/dcos. Writes (overwrites)
 * d_feat [V][16][H][W] = dL/dF~ and d_params (packed like params, summed over
 * views). Recomputes the forward; deterministic. The DINO features get no
 * gradient. */
int asgs_feature_backward(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height,
                          const float* feat, const float* params, const float* dino, const float* d_cos,
                          float* d_feat, float* d_params, void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Probabilistic anchor update (UP-SLAM Sec. 3.3, Eq. 7)
 *
 * Per anchor, the occupancy probability p is updated with the observation
 * probability p_obs = P(n | z_t) by Bayes' rule in odds form with the prior
 * P(n) (Eq. 7's P(n)/P(n) factor read as the prior odds P(n)/(1 - P(n))):
 *   p <- 1 / (1 + (1 - p_obs)/p_obs * (1 - p)/p * prior/(1 - prior)),
 * then clamped to [p_min, p_max]. keep[i] = (p >= prune_below) marks the
 * anchors that stay; *n_keep (device int64, may be NULL) receives their
 * number. p is updated in place ([n] float, device); p_obs [n] float
 * (device); keep [n] uint8 (device) or NULL. Probabilities outside (0, 1)
 * give the IEEE result of the formula. Asynchronous; the count is exact.
 * ------------------------------------------------------------------------- */
typedef struct asgs_anchor_update_opts {
  float prior;        /* P(n), in (0, 1) */
  float p_min, p_max; /* clamp of the result, 0 <= p_min <= p_max <= 1 (0, 1: none) */
  float prune_below;  /* keep anchors with p >= this (0: keep all) */
  int32_t reserved;   /* must be 0 */
} asgs_anchor_update_opts;

int asgs_anchor_update(int64_t n_anchors, const asgs_anchor_update_opts* opts, const float* p_obs, float* p,
                       uint8_t* keep, int64_t* n_keep, void* stream);

/* ---------------------------------------------------------------------------
 * Mapping loss (UP-SLAM Sec. 3.1 Eq. 4, Sec. 3.3 Eq. 14) and its gradient
 * w.r.t. the rendered maps, in one call. Per view of width x height pixels:
 *   l_p = (1 - M_p) [ lam1 (lam |C~_p - C_p|^2 + (1 - lam)(1 - SSIM_p))
 *                     + lam2 (D~_p - D_p)^2 + lam4 (1 - cos_p) ]
 *   loss[v] = sum_p l_p / (width * height)
 * |.|^2 sums the three colour channels; SSIM_p is the mean over the channels
 * of the structural-similarity map (11 x 11 Gaussian window, sigma 1.5, zero
 * padding, C1 = 0.01^2, C2 = 0.03^2); cos_p is the distillation cosine of
 * Eq. 12 (asgs_feature_forward); M_p = dynamic[p] != 0 (the motion mask,
 * e.g. from asgs_uncertainty). The mean-scale term of Eq. 14 is
 * asgs_mean_scale. Maps are packed per view like asgs_images: rgb and
 * obs_rgb [V][3][H][W], the others [V][H][W] (device). Outputs (device,
 * overwritten, each may be NULL): loss [V], d_rgb [V][3][H][W], d_depth and
 * d_cos [V][H][W]; a NULL cosine drops the lam4 term (d_cos must then be
 * NULL). work holds asgs_mapping_work_size bytes (the SSIM backward maps and
 * the loss partials). Deterministic: fixed-order sums.
 * ------------------------------------------------------------------------- */
typedef struct asgs_mapping_opts {
  float lam;          /* 0.8: share of the squared colour error against 1 - SSIM */
  float lam1;         /* 0.6: colour weight */
  float lam2;         /* 1.0: depth weight */
  float lam4;         /* 0.01: distillation weight */
  int32_t reserved;   /* must be 0 */
} asgs_mapping_opts;

typedef struct asgs_mapping_maps {
  const float* rgb;        /* rendered colour */
  const float* depth;      /* rendered depth */
  const float* obs_rgb;    /* observed colour */
  const float* obs_depth;  /* observed depth */
  const float* cosine;     /* cos(F, F^) per pixel, or NULL */
  const uint8_t* dynamic;  /* motion mask (nonzero: dynamic, excluded), or NULL (all static) */
} asgs_mapping_maps;

void asgs_mapping_opts_default(asgs_mapping_opts* opts);
int asgs_mapping_work_size(int32_t n_views, int32_t width, int32_t height, size_t* bytes);
int asgs_mapping_loss(int32_t n_views, int32_t width, int32_t height, const asgs_mapping_opts* opts,
                      const asgs_mapping_maps* maps, float* loss, float* d_rgb, float* d_depth, float* d_cos,
                      void* work, size_t work_bytes, void* stream);

/* Mean-scale term s_bar of Eq. 14: *value = mean of scale[0 .. count) (device
 * float, may be NULL) and, if d_scale is not NULL, d_scale[i] += lam5 / count
 * (the gradient of lam5 s_bar; call after the render backward that writes
 * d_scale). scale is the flat [3][n] (or all views') linear scale array.
 * work holds asgs_mean_scale_work_size bytes. */
int asgs_mean_scale_work_size(size_t* bytes);
int asgs_mean_scale(int64_t count, const float* scale, float lam5, float* value, float* d_scale, void* work,
                    size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Uncertainty MLP F_u, its loss L_u and the motion mask (UP-SLAM Sec. 3.2
 * Eq. 5, Sec. 3.3 Eq. 13). Per pixel p of a view, with F_p the DINO feature
 * upsampled bilinearly from the patch grid as for the feature lift:
 *   sigma_p = sigma_min + softplus(w2 . relu(W1 F_p + b1) + b2)
 *   dynamic_p = (2 sigma_p^2 > 1)                       (the motion mask M)
 *   loss[v] = mean_p R_p / (2 sigma_p^2) + lam3 log sigma_p   (L_u)
 * R is the residual of Eq. 6 (asgs_tracking_residual) and is held constant:
 * d_params receives dL_u/d(F_u parameters) summed over the views, and no
 * gradient flows to the rendered maps (the mapping loss trains the Gaussians
 * with the mask as a constant; the two gradient flows stay separate).
 *
 * params (device, packed): W1 [128][n_high] row-major, b1 [128], w2 [128],
 * b2 [1] (asgs_uncertainty_param_count floats). dino [V][n_high][grid_h]
 * [grid_w]; R, sigma [V][H][W] float; dynamic [V][H][W] uint8; loss [V];
 * every output may be NULL; R is required for loss and d_params. Grids as
 * for the feature lift (a 16 x 16 pixel tile reaches at most 4 x 4 patches,
 * else ASGS_E_UNSUPPORTED); n_high a multiple of 16 in 16..2048.
 * ------------------------------------------------------------------------- */
typedef struct asgs_uncertainty_mlp {
  int32_t n_high;      /* N_h, DINO feature channels */
  int32_t grid_h;      /* patch rows */
  int32_t grid_w;      /* patch columns */
  float sigma_min;     /* floor added to the SoftPlus output: 1e-3 */
  float lam3;          /* weight of log sigma in L_u: 0.4 */
  int32_t reserved;    /* must be 0 */
} asgs_uncertainty_mlp;

int asgs_uncertainty_param_count(const asgs_uncertainty_mlp* u, int64_t* count);
int asgs_uncertainty_workspace_size(const asgs_uncertainty_mlp* u, int32_t n_views, int32_t width, int32_t height,
                                    size_t* bytes);
int asgs_uncertainty(const asgs_uncertainty_mlp* u, int32_t n_views, int32_t width, int32_t height,
                     const float* params, const float* dino, const float* R, float* sigma, uint8_t* dynamic,
                     float* loss, float* d_params, void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Timing hook (for measurement tools; off by default)
 *
 * While a kernel class is enabled, each launch of it made by this library is
 * bracketed by two hipEvents recorded on the launch stream. asgs_profile_read
 * waits for those events and returns the summed elapsed time and the number of
 * launches since the class was last enabled. Process-wide, thread-safe.
 * ------------------------------------------------------------------------- */
enum {
  ASGS_K_PROJECT = 0,      /* projection (one kernel) */
  ASGS_K_SORT = 1,         /* binning: tile scan, duplication, per-tile list sort (several kernels) */
  ASGS_K_BLEND_FWD = 2,    /* forward compositing (one kernel) */
  ASGS_K_BLEND_BWD = 3,    /* backward compositing (one kernel) */
  ASGS_K_PROJECT_BWD = 4,  /* projection backward + pose reduction (one kernel) */
  ASGS_K_DECODE = 5,       /* decoder forward (one kernel) */
  ASGS_K_DECODE_BWD = 6,   /* decoder backward + parameter reduction (several kernels) */
  ASGS_K_RESIDUAL = 7,     /* tracking residual and uncertainty (one kernel + the per-view mean) */
  ASGS_K_FEATURE = 8,      /* feature lift forward (weight and patch preparation + per-pixel kernel) */
  ASGS_K_FEATURE_BWD = 9,  /* feature lift backward (preparation, per-pixel kernel, reductions) */
  ASGS_K_MAPPING = 10,     /* mapping loss with SSIM and its gradient (two stencil kernels + the mean) */
  ASGS_K_UNCERTAINTY = 11, /* uncertainty MLP, its loss and parameter gradient */
  ASGS_K_NUM = 12
};
/* Enable the classes whose bit (1 << class) is set in mask; 0 disables all.
 * Clears earlier measurements. */
int asgs_profile_enable(uint32_t mask);
int asgs_profile_read(int32_t kernel_class, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* ASGS_H */
