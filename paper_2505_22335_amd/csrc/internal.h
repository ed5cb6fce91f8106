// Internal declarations shared by the libasgs translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "asgs.h"

namespace asgs {

constexpr int kTile = 16;            // screen tile side (pixels)
constexpr int kTilePix = kTile * kTile;
constexpr int kGeomStride = 8;       // floats per 2D geometry record: u v A B | C o - -
constexpr int kScanThreads = 256;    // (view, Gaussian) pairs per binning block, all of one view

// Binning blocks: ceil(n / kScanThreads) per view, in (view, Gaussian) order.
__host__ __device__ inline int64_t scan_blocks(int64_t n, int n_views) { return (n + kScanThreads - 1) / kScanThreads * n_views; }

// Device view table entry (128 bytes).
struct ViewDev {
  float R[9];        // world->camera rotation (transpose of the T_wc rotation block), row-major
  float t[3];        // world->camera translation
  float fx, fy, cx, cy;
  float limx, limy;  // Jacobian clamp limits on x/z and y/z (huge when off)
  float cc[3];       // camera centre in world coordinates
  int32_t W, H, TX, TY;
  int32_t tile_base; // first global tile key of this view
  int32_t pix_base;  // first pixel of this view in the packed image planes
  float lt[2];       // temporal embedding (sin pi t, cos pi t) of the frame time
  int32_t pad[3];
};
static_assert(sizeof(ViewDev) == 128, "ViewDev size");

// Scalars every render kernel needs.
struct RenderConst {
  float alpha_min, alpha_max, T_min, dilation, znear;
  float bg[3];
  int32_t n_views;
  int32_t nf;          // feature channels (0 or 16)
  int64_t n;           // Gaussians per view
  int64_t nv;          // n * n_views
  int32_t total_tiles;
  int32_t total_pix;
  int64_t cap;         // intersection capacity
  int32_t n_cu;        // compute units of the device (issue-priority bands of the blend kernels)
  int32_t extent_mode; // 0: tight alpha_min box; 1: 3-sigma square
};

// Header at the start of every render context (device memory).
// Record an error message for asgs_last_error (calling thread) and return status.
int fail(int status, const char* fmt, ...);

struct CtxHeader {
  unsigned long long n_isect;     // intersections of the last forward/count (may exceed cap)
  unsigned long long n_visible;   // visible (view, Gaussian) pairs
  uint32_t overflow;
  uint32_t counters[15];          // last-block-done counters of the multi-block kernels
  uint32_t magic;
  uint32_t pad[31];
};

// Byte layout of a render context; every array 256-byte aligned.
//  rad                 per (view, Gaussian): footprint radii (r_x, r_y), -1 when culled before
//                      the footprint
//  ntiles, dkey, toff  per (view, Gaussian): tile count, depth bits, first gradient slot
//  bsum, vsum          per scan block: tile-count sum, visible count
//  bpre, vpre          per scan block: exclusive prefixes of bsum and vsum over all blocks
//  vlist, vcount       per view: its visible Gaussians in index order (region of n), their number
//  tcur                per tile: intersection count, then the emission cursor
//  ukey, tkey          per intersection: (depth << 32 | gid) in emission order; merge scratch
//  pairgid, pslot, ptile  per sorted intersection: Gaussian, gradient slot, tile key
//  binfo               per blend position (longest list first): tile, start, end, and the
//                      list length the backward walks (largest last contributor + 1)
//  lpart               per tile and 8x8 quarter: L1 loss partial of the fused forward
//  bslot               per tile: 1 + its split-record slot, 0 when the list is not split
//  sinfo               per split-record slot: tile, start, end, walked length (tile ~0u: unused)
//  split               per split-record slot (kSplitPerView per view): per pixel the
//                      transmittance and channels at each segment boundary, and the
//                      final channels
struct CtxLayout {
  size_t hdr, views, geom, chan, rad, rect, ntiles, dkey, toff, bsum, vsum, bpre, vpre, vlist, vcount, tcur, ukey, tkey,
      pairgid, pslot,
      ptile, pmask, ranges, binfo, lpart, bslot, sinfo, split, tfinal, ncontrib, gslot, posepart;
  size_t total;
  int64_t nv, cap;
  int32_t total_tiles, total_pix, cs, gs, pose_blocks;
};

int chan_stride(int nf);   // floats per channel record: rgb, depth, feat
int gslot_stride(int nf);  // floats per per-pair gradient slot (6 + 4 + nf, padded to whole float4)
CtxLayout ctx_layout(int64_t n, int n_views, int total_tiles, int total_pix, int nf, int64_t cap);

// ---------------------------------------------------------------------------
// Kernel launchers (each defined next to its kernels). All asynchronous.
// ---------------------------------------------------------------------------
void launch_set_views(const ViewDev* host_views, int n_views, ViewDev* dev_views,
                      CtxHeader* hdr, uint32_t* tcount, int total_tiles, hipStream_t s);
void launch_project(const RenderConst& rc, const asgs_gaussians& g, const CtxLayout& L,
                    char* ctx, hipStream_t s);
void launch_bin(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s);
void launch_tile_sort(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s);
// The longest lists are walked by several backward workgroups, one per
// segment of kSeg entries (the last segment takes the rest):
// min(kSegMax, ceil(len / kSeg)) segments. The forward stages such lists kSeg
// entries at a time and records the state at every segment boundary. Which
// lists are split depends only on the lengths of the lists of their own
// view (so that results do not depend on the batch or on the order of equal
// lengths): those longer than the smallest threshold kSplitLen + j kSplitStep
// that at most kSplitPerView lists of the view exceed.
constexpr int kSeg = 128;
constexpr int kSegMax = 4;
constexpr int kSplitLen = 160;
constexpr int kSplitStep = 32;
constexpr int kSplitThresholds = 28;  // kSplitLen + j kSplitStep, j < 28 (up to 1024)
constexpr int kSplitPerView = 64;
__host__ __device__ inline int split_segments(uint32_t len) {
  const uint32_t n = (len + kSeg - 1) / kSeg;
  return n < (uint32_t)kSegMax ? (int)n : kSegMax;
}
// Floats per pixel of a boundary record (T and the channels, padded to whole
// float4) and of the final channels (padded).
__host__ __device__ constexpr int split_first(int cs) { return (1 + cs + 3) & ~3; }
__host__ __device__ constexpr int split_final(int cs) { return (cs + 3) & ~3; }
// Floats of the split records of one list.
__host__ __device__ constexpr int split_floats(int cs) {
  return ((kSegMax - 1) * split_first(cs) + split_final(cs)) * 256;
}

// Weighted L1 residual fused into the forward's output stage (same terms as
// launch_l1_loss, targets and gradients packed like the images).
struct BlendL1 {
  const float* t[4];  // targets per group (rgb, depth, feat, opacity sum), NULL = no term
  const float* w;     // per-pixel weight [H][W] shared by the views, NULL = 1
  float* g[4];        // gradient planes per group, NULL = not written
  float s[4];         // scale of each group's term
};
void launch_blend_forward(const RenderConst& rc, const CtxLayout& L, char* ctx,
                          const asgs_images& out, const BlendL1* l1, hipStream_t s);
void launch_l1_tile_loss(const RenderConst& rc, const CtxLayout& L, char* ctx, float* loss, hipStream_t s);
void launch_blend_backward(const RenderConst& rc, const CtxLayout& L, char* ctx,
                           const asgs_images& dout, hipStream_t s);
void launch_project_backward(const RenderConst& rc, const asgs_gaussians& g,
                             const asgs_gaussians& dg, float* d_pose, const CtxLayout& L,
                             char* ctx, hipStream_t s);

// Weighted L1 residual of packed maps (loss.hip). Groups: 0 rgb (3), 1 depth
// (1), 2 feature (nf), 3 opacity sum (1).
constexpr int kL1Blocks = 512;  // blocks per view of the loss kernel
struct L1Views {
  const float* t[4][ASGS_MAX_VIEWS];  // targets per group and view ([C][H][W]); NULL = no term
  const float* w[ASGS_MAX_VIEWS];     // per-pixel weights per view; NULL = 1
};
struct L1Args {
  const float* x[4];  // rendered maps per group, packed [V][C][HW]
  float* g[4];        // gradient maps per group (packed like x), NULL = not written
  float* partial;     // [V][kL1Blocks] partial sums, or NULL (no loss value)
  float* loss;        // [V] or NULL
  int64_t HW;
  int32_t nf, n_views;
  float s[4];         // scale of each group's term
};
void launch_l1_loss(const L1Args& a, const L1Views& tv, hipStream_t s);
// Validates the arguments of the L1 residual calls and fills a and tv (the
// loss outputs, a.partial and a.loss, are left NULL). Launches nothing.
int l1_setup(int32_t n_views, int32_t width, int32_t height, int32_t n_feat, const asgs_images* maps,
             const asgs_l1_targets* targets, const asgs_images* grad, L1Args& a, L1Views& tv);

// Tracking residual and uncertainty (residual.hip). Maps packed [V][C][H][W].
struct ResidualArgs {
  const float *rgb, *depth, *alpha, *cosine, *obs_rgb, *obs_depth;
  float* R;            // [V][H][W] or NULL
  float* sigma;        // [V][H][W] or NULL
  uint8_t* dynamic;    // [V][H][W] or NULL
  float* partial;      // [V][residual_partials] objective partials, or NULL (no xi)
  int32_t W, H;
  float w[3];          // residual weights: colour, depth, feature
  float vis_T, sigma_min, dyn_thresh;
};
int64_t residual_partials(int width, int height);  // per view
void launch_residual(const ResidualArgs& a, int n_views, float* xi, hipStream_t s);

// Feature lift and cosine distillation (feature.hip).
struct FeatLayout {
  size_t mfrag, mvec, cells, tile_loss, part, dqt, red, dqc, dqpix, gpart, gout, ppart, pout, total;
};
struct FeatCall {
  int32_t n_views, width, height, nh, Hp, Wp;
  const float *feat, *params, *dino, *dcos;
  float *cosine, *loss, *dfeat, *dparams;
};
FeatLayout feature_layout(int nh, int n_views, int width, int height, int Hp, int Wp);
// patch rows or columns one 16x16 pixel tile can reach (bound)
int feature_max_patch_span(int width, int height, int Hp, int Wp);
void launch_feature_forward(const FeatCall& c, const FeatLayout& L, char* work, hipStream_t s);
void launch_feature_backward(const FeatCall& c, const FeatLayout& L, char* work, hipStream_t s);

// Split-K products over (view, patch) rows (colgemm.hip):
//   out[col][k] = sum_r D[r * dstride + col] F_k(r),  r = v * rows + c,
//   F_k(r) = F[v * fview + k * fk + c * fr] (k < nk), tail[c] (k = nk, if tail),
//   1 (the last k, if ones); out is [ncol][nk (+1) (+1)].
struct ColGemm {
  const float* D;
  int64_t dstride;
  int32_t ncol;
  const float* F;
  int64_t fk, fr, fview;
  int32_t nk;
  const float* tail;
  int32_t ones;
  int32_t V, rows;
  int32_t nsplit;
  float* part;  // work: colgemm_part_floats
};
int colgemm_splits(int64_t rows, int ncol, int nkt);
size_t colgemm_part_floats(const ColGemm& g);
void launch_colgemm(const ColGemm& g, float* out, hipStream_t s);

// Mapping loss with SSIM and the mean-scale term (mapping.hip).
struct MappingArgs {
  const float *rgb, *depth, *obs_rgb, *obs_depth, *cosine;
  const uint8_t* dynamic;  // motion mask or NULL
  float *d_rgb, *d_depth, *d_cos;
  float* abc;              // work: [V][9][H][W] SSIM backward maps (NULL without d_rgb)
  double* partial;         // work: [V][mapping_tiles] loss partials
  int32_t W, H;
  float lam, lam1, lam2, lam4;
  double taps[11];         // normalised Gaussian window (sigma 1.5)
  float ftaps[11];
};
int64_t mapping_tiles(int width, int height);  // per view
void mapping_window(double* taps, float* ftaps);
void launch_mapping_loss(const MappingArgs& a, int n_views, float* loss, hipStream_t s);
size_t mean_scale_work_bytes();
void launch_mean_scale(int64_t count, const float* scale, float lam5, float* value, float* d_scale, double* work,
                       hipStream_t s);

// Uncertainty MLP F_u, its loss and the motion mask (uncertainty.hip).
struct UncArgs {
  int32_t V, W, H, nh, Hp, Wp;
  int32_t tiles_x, tiles_y, tiles;  // 16 x 16 pixel tiles per view
  float sx, sy;                     // Wp / W, Hp / H
  float sigma_min, lam3, inv_hw;
  const float* params;              // W1 [128][nh], b1 [128], w2 [128], b2
  const float* dino;                // [V][nh][Hp][Wp]
  const float* R;                   // [V][H][W] or NULL
  float* sigma;                     // [V][H][W] or NULL
  uint8_t* dynamic;                 // [V][H][W] or NULL
  float* zg;                        // work: [V][Hp * Wp][128] first layer per patch
  double* partial;                  // work: [V * tiles] loss partials, or NULL
  float* dzt;                       // work: [V * tiles][16][128], or NULL (no gradient)
  float* w2t;                       // work: [V * tiles][129] dw2 and db2 partials
  float* dzc;                       // work: [V][Hp * Wp][128] dZ per patch
};
struct UncLayout {
  size_t zg, partial, dzt, w2t, dzc, gpart, gout, total;
};
UncLayout uncertainty_layout(int n_views, int width, int height, int Hp, int Wp, int nh);
void launch_uncertainty(UncArgs a, const UncLayout& L, char* work, float* loss, float* d_params, hipStream_t s);

// Probabilistic anchor update (anchor.hip); n_keep (device, may be NULL) is zeroed first.
void launch_anchor_update(int64_t n, const float* p_obs, float* p, uint8_t* keep, unsigned long long* n_keep,
                          float prior, float p_min, float p_max, float prune_below, hipStream_t s);

struct DecodeConst {
  int64_t A;
  int32_t k, nf, n_views, precision;
  float l_o, l_s;
  int64_t head_off[5];   // float offset of each head's W1 in the packed params
  int64_t head_xoff[5];  // float offset of each head's extra first-layer columns [32][n_x]
  int32_t head_m[5];     // values per Gaussian of each head (0 = absent)
  int32_t n_x;           // input columns past the first 35: 0, 1 (distance) or 3 (+ time)
  int64_t n_params;
};
DecodeConst decode_const(const asgs_decoder& d, int n_views);
size_t decode_workspace_bytes(const DecodeConst& dc);
void launch_decode(const DecodeConst& dc, const float* xyz, const float* feat, const float* off,
                   const float* params, const ViewDev* host_views, const asgs_gaussians& out,
                   hipStream_t s);
void launch_decode_backward(const DecodeConst& dc, const float* xyz, const float* feat,
                            const float* off, const float* params, const ViewDev* host_views,
                            const asgs_gaussians& dg, float* d_xyz, float* d_feat, float* d_off,
                            float* d_params, float* d_pose, void* work, hipStream_t s);

}  // namespace asgs

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
#define ASGS_DEV __device__ __forceinline__

namespace asgs {

template <typename T>
ASGS_DEV T* ctx_ptr(char* ctx, size_t off) { return reinterpret_cast<T*>(ctx + off); }

// Bilinear source of output index p along one axis when n_in samples are
// upsampled with scale = n_in / n_out (sample centres at half-integers,
// clamped at both ends): value = (1 - w1) v[i0] + w1 v[i1].
ASGS_DEV void bilin(int p, int n_in, float scale, int& i0, int& i1, float& w1) {
  const float s = fmaxf(((float)p + 0.5f) * scale - 0.5f, 0.f);
  i0 = min((int)s, n_in - 1);
  i1 = min(i0 + 1, n_in - 1);
  w1 = s - (float)i0;
}

// ---------------------------------------------------------------------------
// Binning blocks: kScanThreads consecutive (view, Gaussian) pairs of one view,
// one per thread. A block's intersections reach the per-tile counters through
// an LDS grid over the bounding box of its Gaussians' rectangles (Gaussians of
// one block are mostly neighbours in space), so a hot tile takes one global
// atomic per block instead of one per Gaussian. Gaussians with a rectangle
// of more than kBoxRect tiles, and every Gaussian of a block whose box has
// more than kBoxCells tiles, use the global counters directly.
// ---------------------------------------------------------------------------
constexpr int kBoxCells = 4096;
constexpr int kBoxRect = 64;

struct TileBox {
  int x0, y0, w, area;  // LDS cell of tile (tx, ty): (ty - y0) * w + tx - x0
  bool lds;             // block-uniform: the box fits kBoxCells
};

template <typename T>
ASGS_DEV T wave_min(T v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// Bounding box of the rects of the lanes with small set; clears its cells.
ASGS_DEV TileBox tile_box(short4 r, bool small, int* red, uint32_t* cell) {
  const int t = threadIdx.x;
  if (t < 4) red[t] = 0x7FFFFFFF;
  __syncthreads();
  const int big = 0x7FFFFFFF;
  const int x0 = wave_min(small ? (int)r.x : big), nx1 = wave_min(small ? -(int)r.y : big);
  const int y0 = wave_min(small ? (int)r.z : big), ny1 = wave_min(small ? -(int)r.w : big);
  if ((t & 63) == 0) {
    atomicMin(&red[0], x0);
    atomicMin(&red[1], nx1);
    atomicMin(&red[2], y0);
    atomicMin(&red[3], ny1);
  }
  __syncthreads();
  TileBox b;
  b.x0 = red[0];
  b.y0 = red[2];
  b.lds = b.x0 != big;
  b.w = b.lds ? -red[1] - b.x0 + 1 : 0;
  const int h = b.lds ? -red[3] - b.y0 + 1 : 0;
  b.area = b.w * h;
  b.lds = b.lds && b.area <= kBoxCells;
  if (b.lds)
    for (int c = t; c < b.area; c += kScanThreads) cell[c] = 0u;
  __syncthreads();
  return b;
}

// View of a global tile key (views are stored in tile_base order).
ASGS_DEV int find_view(const ViewDev* views, int n_views, int tile) {
  int v = 0;
  for (int k = 1; k < n_views; ++k)
    if (tile >= views[k].tile_base) v = k;
  return v;
}

// Alpha of a Gaussian at a pixel. The same instruction sequence is used by
// the forward and the backward so both take identical skip/stop decisions.
ASGS_DEV float eval_power(float u, float v, float A, float B, float C, float px, float py,
                          float& dx, float& dy) {
  dx = u - px;
  dy = v - py;
  const float q = fmaf(C * dy, dy, A * dx * dx);
  return fmaf(-0.5f, q, -(B * dx) * dy);
}

}  // namespace asgs
