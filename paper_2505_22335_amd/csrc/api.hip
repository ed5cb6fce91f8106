// Host side of the libasgs C ABI: argument validation, context layout,
// launch sequencing and error reporting. Nothing here allocates device memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace asgs {

namespace {
thread_local std::string g_err = "no error";
}  // namespace

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

namespace {

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ASGS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return ASGS_OK;
}

// ---- timing hook -----------------------------------------------------------
struct ProfEvent {
  int cls;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
uint32_t g_prof_mask = 0;
std::vector<ProfEvent> g_prof;

// Brackets one launch sequence of class `cls` with events when enabled.
struct ProfScope {
  hipEvent_t b = nullptr;
  hipStream_t s;
  ProfScope(int cls, hipStream_t st) : s(st) {
    if (!(__atomic_load_n(&g_prof_mask, __ATOMIC_RELAXED) & (1u << cls))) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      b = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back({cls, a, b});
  }
  ~ProfScope() {
    if (b) (void)hipEventRecord(b, s);
  }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_opts(const asgs_render_opts* o) {
  if (!o) return fail(ASGS_E_INVALID, "opts is NULL");
  if (o->tile != kTile) return fail(ASGS_E_UNSUPPORTED, "tile must be %d (got %d)", kTile, o->tile);
  if (o->n_feat != 0 && o->n_feat != 16)
    return fail(ASGS_E_UNSUPPORTED, "n_feat must be 0 or 16 (got %d)", o->n_feat);
  if (!(o->alpha_min > 0.f && o->alpha_min < 1.f) || !(o->alpha_max > o->alpha_min && o->alpha_max < 1.f) ||
      !(o->T_min > 0.f && o->T_min < 1.f) || !(o->dilation >= 0.f) || !(o->znear > 0.f) ||
      !(o->fov_clamp >= 0.f) || !isfinite(o->bg[0]) || !isfinite(o->bg[1]) || !isfinite(o->bg[2]))
    return fail(ASGS_E_INVALID, "render options out of range");
  if (o->extent_mode != 0 && o->extent_mode != 1) return fail(ASGS_E_INVALID, "opts.extent_mode must be 0 or 1");
  return ASGS_OK;
}

// Validates the cameras and fills the device view table (host copy).
int make_views(const asgs_camera* cams, int32_t n_views, float fov_clamp, ViewDev* out, int* total_tiles,
               int* total_pix) {
  if (!cams) return fail(ASGS_E_INVALID, "cams is NULL");
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS)
    return fail(ASGS_E_INVALID, "n_views must be in 1..%d (got %d)", ASGS_MAX_VIEWS, n_views);
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const asgs_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
      return fail(ASGS_E_INVALID, "view %d: size %dx%d out of range", v, c.width, c.height);
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !isfinite(c.fx) || !isfinite(c.fy) || !isfinite(c.cx) ||
        !isfinite(c.cy))
      return fail(ASGS_E_INVALID, "view %d: bad intrinsics", v);
    for (int k = 0; k < 12; ++k)
      if (!isfinite(c.T_wc[k])) return fail(ASGS_E_INVALID, "view %d: non-finite T_wc", v);
    if (!isfinite(c.t)) return fail(ASGS_E_INVALID, "view %d: non-finite frame time", v);
    ViewDev& V = out[v];
    memset(&V, 0, sizeof(V));
    double Rwc[9], ctr[3];
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) Rwc[r * 3 + k] = c.T_wc[r * 4 + k];
      ctr[r] = c.T_wc[r * 4 + 3];
    }
    for (int r = 0; r < 3; ++r) {
      double tr = 0.0;
      for (int k = 0; k < 3; ++k) {
        V.R[r * 3 + k] = (float)Rwc[k * 3 + r];  // R_cw = R_wc^T
        tr -= Rwc[k * 3 + r] * ctr[k];
      }
      V.t[r] = (float)tr;
      V.cc[r] = (float)ctr[r];
    }
    V.lt[0] = (float)sin(M_PI * (double)c.t);
    V.lt[1] = (float)cos(M_PI * (double)c.t);
    V.fx = c.fx;
    V.fy = c.fy;
    V.cx = c.cx;
    V.cy = c.cy;
    V.limx = fov_clamp > 0.f ? (float)((double)fov_clamp * c.width / (2.0 * c.fx)) : 3.0e38f;
    V.limy = fov_clamp > 0.f ? (float)((double)fov_clamp * c.height / (2.0 * c.fy)) : 3.0e38f;
    V.W = c.width;
    V.H = c.height;
    V.TX = (c.width + kTile - 1) / kTile;
    V.TY = (c.height + kTile - 1) / kTile;
    V.tile_base = (int32_t)tiles;
    V.pix_base = (int32_t)pix;
    tiles += (int64_t)V.TX * V.TY;
    pix += (int64_t)c.width * c.height;
  }
  if (pix > (int64_t)1 << 30) return fail(ASGS_E_INVALID, "too many pixels in one call");
  *total_tiles = (int)tiles;
  *total_pix = (int)pix;
  return ASGS_OK;
}

int check_gauss(const asgs_gaussians* g, int nf, int n_views, bool allow_shared, const char* name) {
  if (!g) return fail(ASGS_E_INVALID, "%s is NULL", name);
  if (g->n < 1 || g->n > ((int64_t)1 << 26)) return fail(ASGS_E_INVALID, "%s: n out of range", name);
  float* const ptrs[6] = {g->mean, g->scale, g->rot, g->opacity, g->rgb, g->feat};
  const char* names[6] = {"mean", "scale", "rot", "opacity", "rgb", "feat"};
  for (int f = 0; f < 6; ++f) {
    if (f == 5 && nf == 0) continue;
    if (!ptrs[f]) return fail(ASGS_E_INVALID, "%s.%s is NULL", name, names[f]);
    if (!aligned16(ptrs[f])) return fail(ASGS_E_INVALID, "%s.%s not 16-byte aligned", name, names[f]);
    if (g->view_stride[f] < 0) return fail(ASGS_E_INVALID, "%s.%s: negative view stride", name, names[f]);
    if (n_views > 1 && g->view_stride[f] == 0 && !allow_shared)
      return fail(ASGS_E_INVALID, "%s.%s: views may not share a gradient array", name, names[f]);
  }
  return ASGS_OK;
}

// Compute units of the current device (cached per device; 0 if unknown).
int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
    cached[dev] = n;
  }
  return cached[dev];
}

struct Prep {
  ViewDev views[ASGS_MAX_VIEWS];
  int total_tiles = 0, total_pix = 0;
  RenderConst rc;
  CtxLayout L;
};

int prepare(const asgs_camera* cams, int32_t n_views, int64_t n, const asgs_render_opts* opts,
            int64_t capacity, Prep& P) {
  int st = check_opts(opts);
  if (st) return st;
  st = make_views(cams, n_views, opts->fov_clamp, P.views, &P.total_tiles, &P.total_pix);
  if (st) return st;
  if (n < 1 || n > ((int64_t)1 << 26)) return fail(ASGS_E_INVALID, "n_gauss out of range");
  if (n * n_views > ((int64_t)1 << 31)) return fail(ASGS_E_INVALID, "too many Gaussians in one call");
  if (capacity < 0 || capacity > ((int64_t)1 << 31)) return fail(ASGS_E_INVALID, "capacity out of range");
  RenderConst& rc = P.rc;
  rc.alpha_min = opts->alpha_min;
  rc.alpha_max = opts->alpha_max;
  rc.T_min = opts->T_min;
  rc.dilation = opts->dilation;
  rc.extent_mode = opts->extent_mode;
  rc.znear = opts->znear;
  for (int c = 0; c < 3; ++c) rc.bg[c] = opts->bg[c];
  rc.n_views = n_views;
  rc.nf = opts->n_feat;
  rc.n = n;
  rc.nv = n * n_views;
  rc.total_tiles = P.total_tiles;
  rc.total_pix = P.total_pix;
  rc.cap = capacity;
  rc.n_cu = device_cu_count();
  P.L = ctx_layout(n, n_views, P.total_tiles, P.total_pix, opts->n_feat, capacity);
  return ASGS_OK;
}

int check_ctx(const Prep& P, const void* ctx, size_t ctx_bytes) {
  if (!ctx) return fail(ASGS_E_INVALID, "ctx is NULL");
  if ((reinterpret_cast<uintptr_t>(ctx) & 255u) != 0) return fail(ASGS_E_INVALID, "ctx not 256-byte aligned");
  if (ctx_bytes < P.L.total)
    return fail(ASGS_E_WORKSPACE, "render context needs %zu bytes (got %zu)", P.L.total, ctx_bytes);
  return ASGS_OK;
}

// Projection, tile counting, ranges and duplication (shared by count and forward).
int run_front(const Prep& P, const asgs_gaussians* g, char* ctx, hipStream_t s) {
  launch_set_views(P.views, P.rc.n_views, reinterpret_cast<ViewDev*>(ctx + P.L.views),
                   reinterpret_cast<CtxHeader*>(ctx + P.L.hdr), reinterpret_cast<uint32_t*>(ctx + P.L.tcur),
                   P.rc.total_tiles, s);
  {
    ProfScope ps(ASGS_K_PROJECT, s);
    launch_project(P.rc, *g, P.L, ctx, s);
  }
  {
    ProfScope ps(ASGS_K_SORT, s);
    launch_bin(P.rc, P.L, ctx, s);
  }
  return check_launch("projection/binning launch");
}

}  // namespace

int chan_stride(int nf) { return 4 + nf; }
int gslot_stride(int nf) { return (6 + 4 + nf + 3) & ~3; }  // padded to whole float4

CtxLayout ctx_layout(int64_t n, int n_views, int total_tiles, int total_pix, int nf, int64_t cap) {
  CtxLayout L;
  memset(&L, 0, sizeof(L));
  const int64_t nv = n * n_views;
  const int64_t capc = cap > 0 ? cap : 1;
  L.nv = nv;
  L.cap = cap;
  L.total_tiles = total_tiles;
  L.total_pix = total_pix;
  L.cs = chan_stride(nf);
  L.gs = gslot_stride(nf);
  L.pose_blocks = (int32_t)((n + 255) / 256);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + (bytes > 0 ? bytes : 1));
    return at;
  };
  L.hdr = take(sizeof(CtxHeader));
  L.views = take(sizeof(ViewDev) * ASGS_MAX_VIEWS);
  L.geom = take((size_t)nv * kGeomStride * sizeof(float));
  L.chan = take((size_t)nv * L.cs * sizeof(float));
  L.rad = take((size_t)nv * 8);
  L.rect = take((size_t)nv * 8);
  L.ntiles = take((size_t)nv * 4);
  L.dkey = take((size_t)nv * 4);
  L.toff = take((size_t)nv * 4);
  L.bsum = take((size_t)scan_blocks(n, n_views) * 4);
  L.vsum = take((size_t)scan_blocks(n, n_views) * 4);
  L.bpre = take((size_t)scan_blocks(n, n_views) * 4);
  L.vpre = take((size_t)scan_blocks(n, n_views) * 4);
  L.vlist = take((size_t)nv * 4);
  L.vcount = take((size_t)n_views * 4);
  L.tcur = take((size_t)total_tiles * 4);
  L.ukey = take((size_t)capc * 8);
  L.tkey = take((size_t)capc * 8);
  L.pairgid = take((size_t)capc * 4);
  L.pslot = take((size_t)capc * 4);
  L.ptile = take((size_t)capc * 4);
  L.pmask = take((size_t)capc);
  L.ranges = take((size_t)total_tiles * 8);
  L.binfo = take((size_t)total_tiles * 16);
  L.lpart = take((size_t)total_tiles * 4 * sizeof(float));
  L.bslot = take((size_t)total_tiles * 4);
  L.sinfo = take((size_t)n_views * kSplitPerView * 16);
  L.split = take((size_t)n_views * kSplitPerView * split_floats(L.cs) * sizeof(float));
  L.tfinal = take((size_t)total_pix * 4);
  L.ncontrib = take((size_t)total_pix * 4);
  L.gslot = take((size_t)capc * L.gs * sizeof(float));
  L.posepart = take((size_t)n_views * L.pose_blocks * 6 * sizeof(float));
  L.total = o;
  return L;
}

int l1_setup(int32_t n_views, int32_t width, int32_t height, int32_t n_feat, const asgs_images* maps,
             const asgs_l1_targets* targets, const asgs_images* grad, L1Args& a, L1Views& tv) {
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  if (width < 1 || height < 1 || width > 8192 || height > 8192) return fail(ASGS_E_INVALID, "bad resolution");
  if (n_feat != 0 && n_feat != 16) return fail(ASGS_E_UNSUPPORTED, "n_feat must be 0 or 16");
  if (!maps || !targets || !grad) return fail(ASGS_E_INVALID, "l1_loss: NULL argument");
  const float* x[4] = {maps->rgb, maps->depth, maps->feat, maps->alpha};
  const float* tg[4] = {targets->rgb, targets->depth, targets->feat, targets->alpha};
  float* g[4] = {grad->rgb, grad->depth, grad->feat, grad->alpha};
  for (int q = 0; q < 4; ++q) {
    if (q == 2 && n_feat == 0) continue;
    if ((tg[q] || g[q]) && !x[q]) return fail(ASGS_E_INVALID, "l1_loss: map %d missing", q);
    for (const void* ptr : {(const void*)x[q], (const void*)tg[q], (const void*)g[q]})
      if (ptr && !aligned16(ptr)) return fail(ASGS_E_INVALID, "l1_loss: pointer not 16-byte aligned");
    if (!isfinite(targets->scale[q])) return fail(ASGS_E_INVALID, "l1_loss: scale not finite");
  }
  if (targets->weight && !aligned16(targets->weight))
    return fail(ASGS_E_INVALID, "l1_loss: weight pointer not 16-byte aligned");
  const int64_t HW = (int64_t)width * height;
  a = L1Args{};
  tv = L1Views{};
  const int nc[4] = {3, 1, n_feat, 1};
  for (int q = 0; q < 4; ++q) {
    a.x[q] = (q == 2 && n_feat == 0) ? nullptr : x[q];
    a.g[q] = (q == 2 && n_feat == 0) ? nullptr : g[q];
    a.s[q] = targets->scale[q];
    for (int v = 0; v < n_views; ++v) tv.t[q][v] = tg[q] ? tg[q] + (int64_t)v * nc[q] * HW : nullptr;
  }
  for (int v = 0; v < n_views; ++v) tv.w[v] = targets->weight;
  a.HW = HW;
  a.nf = n_feat;
  a.n_views = n_views;
  return ASGS_OK;
}

}  // namespace asgs

using namespace asgs;

extern "C" {

int asgs_abi_version(void) { return ASGS_ABI_VERSION; }

const char* asgs_status_string(int status) {
  switch (status) {
    case ASGS_OK: return "ok";
    case ASGS_E_INVALID: return "invalid argument";
    case ASGS_E_WORKSPACE: return "workspace too small";
    case ASGS_E_CAPACITY: return "intersection capacity exceeded";
    case ASGS_E_DEVICE: return "device error";
    case ASGS_E_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* asgs_last_error(void) { return g_err.c_str(); }

void asgs_render_opts_default(asgs_render_opts* o) {
  if (!o) return;
  o->tile = 16;
  o->n_feat = 16;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->T_min = 1e-4f;
  o->dilation = 0.3f;
  o->znear = 0.2f;
  o->fov_clamp = 1.3f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.f;
  o->extent_mode = 0;
}

int asgs_render_ctx_size(const asgs_camera* cams, int32_t n_views, int64_t n_gauss, const asgs_render_opts* opts,
                         int64_t capacity, size_t* bytes) {
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  Prep P;
  const int st = prepare(cams, n_views, n_gauss, opts, capacity, P);
  if (st) return st;
  *bytes = P.L.total;
  return ASGS_OK;
}

int asgs_render_count(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                      const asgs_render_opts* opts, void* ctx, size_t ctx_bytes, int64_t* n_isect, void* stream) {
  if (!n_isect) return fail(ASGS_E_INVALID, "n_isect is NULL");
  if (!g) return fail(ASGS_E_INVALID, "g is NULL");
  Prep P;
  int st = prepare(cams, n_views, g->n, opts, 0, P);
  if (st) return st;
  if ((st = check_gauss(g, opts->n_feat, n_views, true, "g"))) return st;
  if ((st = check_ctx(P, ctx, ctx_bytes))) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* c = static_cast<char*>(ctx);
  if ((st = run_front(P, g, c, s))) return st;
  CtxHeader h;
  hipError_t e = hipMemcpyAsync(&h, c + P.L.hdr, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ASGS_E_DEVICE, "count readback: %s", hipGetErrorString(e));
  *n_isect = (int64_t)h.n_isect;
  return ASGS_OK;
}

static int render_forward_impl(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                        const asgs_render_opts* opts, const asgs_images* out, const asgs_l1_targets* targets,
                        const asgs_images* grad, float* loss, void* ctx, size_t ctx_bytes, void* stream) {
  if (!g) return fail(ASGS_E_INVALID, "g is NULL");
  if (!out || !out->rgb || !out->depth || !out->alpha || (opts && opts->n_feat > 0 && !out->feat))
    return fail(ASGS_E_INVALID, "output images missing");
  Prep P;
  int st = prepare(cams, n_views, g->n, opts, 0, P);
  if (st) return st;
  if ((st = check_gauss(g, opts->n_feat, n_views, true, "g"))) return st;
  if (!ctx) return fail(ASGS_E_INVALID, "ctx is NULL");
  // the capacity is whatever the given context bytes hold
  {
    const CtxLayout L0 = ctx_layout(g->n, n_views, P.total_tiles, P.total_pix, opts->n_feat, 0);
    if (ctx_bytes < L0.total)
      return fail(ASGS_E_WORKSPACE, "render context needs at least %zu bytes (got %zu)", L0.total, ctx_bytes);
    int64_t lo = 0, hi = (int64_t)1 << 31;
    while (lo < hi) {  // largest capacity whose layout fits
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (ctx_layout(g->n, n_views, P.total_tiles, P.total_pix, opts->n_feat, mid).total <= ctx_bytes)
        lo = mid;
      else
        hi = mid - 1;
    }
    P.rc.cap = lo;
    P.L = ctx_layout(g->n, n_views, P.total_tiles, P.total_pix, opts->n_feat, lo);
  }
  if ((st = check_ctx(P, ctx, ctx_bytes))) return st;
  BlendL1 l1{};
  if (targets) {
    if (!grad) return fail(ASGS_E_INVALID, "render_forward_l1: grad is NULL");
    const float* tg[4] = {targets->rgb, targets->depth, targets->feat, targets->alpha};
    float* gr[4] = {grad->rgb, grad->depth, grad->feat, grad->alpha};
    for (int q = 0; q < 4; ++q) {
      const bool used = !(q == 2 && opts->n_feat == 0);
      l1.t[q] = used ? tg[q] : nullptr;
      l1.g[q] = used ? gr[q] : nullptr;
      l1.s[q] = targets->scale[q];
      if (!isfinite(targets->scale[q])) return fail(ASGS_E_INVALID, "render_forward_l1: scale not finite");
    }
    l1.w = targets->weight;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* c = static_cast<char*>(ctx);
  if ((st = run_front(P, g, c, s))) return st;
  {
    ProfScope ps(ASGS_K_SORT, s);
    launch_tile_sort(P.rc, P.L, c, s);
  }
  {
    ProfScope ps(ASGS_K_BLEND_FWD, s);
    launch_blend_forward(P.rc, P.L, c, *out, targets ? &l1 : nullptr, s);
  }
  if (targets && loss) launch_l1_tile_loss(P.rc, P.L, c, loss, s);
  return check_launch("render_forward launch");
}

int asgs_render_forward(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                        const asgs_render_opts* opts, const asgs_images* out, void* ctx, size_t ctx_bytes,
                        void* stream) {
  return render_forward_impl(cams, n_views, g, opts, out, nullptr, nullptr, nullptr, ctx, ctx_bytes, stream);
}

int asgs_render_forward_l1(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                           const asgs_render_opts* opts, const asgs_images* out, const asgs_l1_targets* targets,
                           const asgs_images* grad, float* loss, void* ctx, size_t ctx_bytes, void* stream) {
  if (!targets || !grad) return fail(ASGS_E_INVALID, "render_forward_l1: targets or grad is NULL");
  return render_forward_impl(cams, n_views, g, opts, out, targets, grad, loss, ctx, ctx_bytes, stream);
}

int asgs_render_backward(const asgs_camera* cams, int32_t n_views, const asgs_gaussians* g,
                         const asgs_render_opts* opts, const asgs_images* d_out, const asgs_gaussians* d_g,
                         float* d_pose, void* ctx, size_t ctx_bytes, void* stream) {
  if (!g) return fail(ASGS_E_INVALID, "g is NULL");
  if (!d_out || !d_out->rgb || !d_out->depth || (opts && opts->n_feat > 0 && !d_out->feat))
    return fail(ASGS_E_INVALID, "upstream gradients missing");
  Prep P;
  int st = prepare(cams, n_views, g->n, opts, 0, P);
  if (st) return st;
  if ((st = check_gauss(g, opts->n_feat, n_views, true, "g"))) return st;
  if ((st = check_gauss(d_g, opts->n_feat, n_views, false, "d_g"))) return st;
  if (d_g->n != g->n) return fail(ASGS_E_INVALID, "d_g.n != g.n");
  if (!ctx) return fail(ASGS_E_INVALID, "ctx is NULL");
  {
    int64_t lo = 0, hi = (int64_t)1 << 31;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (ctx_layout(g->n, n_views, P.total_tiles, P.total_pix, opts->n_feat, mid).total <= ctx_bytes)
        lo = mid;
      else
        hi = mid - 1;
    }
    P.rc.cap = lo;
    P.L = ctx_layout(g->n, n_views, P.total_tiles, P.total_pix, opts->n_feat, lo);
  }
  if ((st = check_ctx(P, ctx, ctx_bytes))) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* c = static_cast<char*>(ctx);
  {
    ProfScope ps(ASGS_K_BLEND_BWD, s);
    launch_blend_backward(P.rc, P.L, c, *d_out, s);
  }
  {
    ProfScope ps(ASGS_K_PROJECT_BWD, s);
    launch_project_backward(P.rc, *g, *d_g, d_pose, P.L, c, s);
  }
  return check_launch("render_backward launch");
}

int asgs_ctx_status(const void* ctx, void* stream, int64_t* n_isect, int64_t* n_visible, int32_t* overflow) {
  if (!ctx) return fail(ASGS_E_INVALID, "ctx is NULL");
  CtxHeader h;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&h, ctx, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ASGS_E_DEVICE, "ctx readback: %s", hipGetErrorString(e));
  if (n_isect) *n_isect = (int64_t)h.n_isect;
  if (n_visible) *n_visible = (int64_t)h.n_visible;
  if (overflow) *overflow = (int32_t)h.overflow;
  return ASGS_OK;
}

int asgs_ctx_array(const asgs_camera* cams, int32_t n_views, int64_t n_gauss, const asgs_render_opts* opts,
                   void* ctx, size_t ctx_bytes, int32_t which, void** ptr, int64_t* count) {
  if (!ptr || !count) return fail(ASGS_E_INVALID, "ptr/count is NULL");
  Prep P;
  int st = prepare(cams, n_views, n_gauss, opts, 0, P);
  if (st) return st;
  if (!ctx) return fail(ASGS_E_INVALID, "ctx is NULL");
  int64_t lo = 0, hi = (int64_t)1 << 31;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (ctx_layout(n_gauss, n_views, P.total_tiles, P.total_pix, opts->n_feat, mid).total <= ctx_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  const CtxLayout L = ctx_layout(n_gauss, n_views, P.total_tiles, P.total_pix, opts->n_feat, lo);
  if (L.total > ctx_bytes) return fail(ASGS_E_WORKSPACE, "ctx too small");
  char* c = static_cast<char*>(ctx);
  switch (which) {
    case ASGS_CTX_PAIR_TILE: *ptr = c + L.ptile; *count = lo; break;
    case ASGS_CTX_PAIR_GAUSS: *ptr = c + L.pairgid; *count = lo; break;
    case ASGS_CTX_TILE_RANGE: *ptr = c + L.ranges; *count = L.total_tiles; break;
    case ASGS_CTX_RECT: *ptr = c + L.rect; *count = L.nv; break;
    case ASGS_CTX_NCONTRIB: *ptr = c + L.ncontrib; *count = L.total_pix; break;
    case ASGS_CTX_TFINAL: *ptr = c + L.tfinal; *count = L.total_pix; break;
    case ASGS_CTX_GEOM: *ptr = c + L.geom; *count = L.nv; break;
    case ASGS_CTX_RADIUS: *ptr = c + L.rad; *count = L.nv; break;
    case ASGS_CTX_DEPTH_KEY: *ptr = c + L.dkey; *count = L.nv; break;
    case ASGS_CTX_NTILES: *ptr = c + L.ntiles; *count = L.nv; break;
    default: return fail(ASGS_E_INVALID, "unknown context array %d", which);
  }
  return ASGS_OK;
}

/* ------------------------------------------------------------------------- */

static int check_maps_size(int32_t n_views, int32_t width, int32_t height, const char* what) {
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "%s: n_views out of range", what);
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(ASGS_E_INVALID, "%s: bad resolution", what);
  if ((int64_t)width * height * n_views > ((int64_t)1 << 31)) return fail(ASGS_E_INVALID, "%s: too many pixels", what);
  return ASGS_OK;
}

static size_t mapping_work_bytes(int32_t n_views, int32_t width, int32_t height) {
  const size_t abc = (size_t)n_views * 9 * (size_t)width * (size_t)height * sizeof(float);
  const size_t part = (size_t)n_views * (size_t)mapping_tiles(width, height) * sizeof(double);
  return ((abc + 255) & ~(size_t)255) + part;
}

void asgs_mapping_opts_default(asgs_mapping_opts* o) {
  if (!o) return;
  o->lam = 0.8f;
  o->lam1 = 0.6f;
  o->lam2 = 1.0f;
  o->lam4 = 0.01f;
  o->reserved = 0;
}

int asgs_mapping_work_size(int32_t n_views, int32_t width, int32_t height, size_t* bytes) {
  int st = check_maps_size(n_views, width, height, "mapping_work_size");
  if (st) return st;
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  *bytes = mapping_work_bytes(n_views, width, height);
  return ASGS_OK;
}

int asgs_mapping_loss(int32_t n_views, int32_t width, int32_t height, const asgs_mapping_opts* opts,
                      const asgs_mapping_maps* m, float* loss, float* d_rgb, float* d_depth, float* d_cos, void* work,
                      size_t work_bytes, void* stream) {
  int st = check_maps_size(n_views, width, height, "mapping_loss");
  if (st) return st;
  if (!opts || !m) return fail(ASGS_E_INVALID, "mapping_loss: NULL argument");
  for (float f : {opts->lam, opts->lam1, opts->lam2, opts->lam4})
    if (!isfinite(f)) return fail(ASGS_E_INVALID, "mapping_loss: non-finite weight");
  if (opts->reserved != 0) return fail(ASGS_E_INVALID, "mapping_loss: reserved must be 0");
  for (const float* ptr : {m->rgb, m->depth, m->obs_rgb, m->obs_depth})
    if (!ptr) return fail(ASGS_E_INVALID, "mapping_loss: input map missing");
  if (d_cos && !m->cosine) return fail(ASGS_E_INVALID, "mapping_loss: d_cos needs the cosine map");
  if (!loss && !d_rgb && !d_depth && !d_cos) return fail(ASGS_E_INVALID, "mapping_loss: no output requested");
  const size_t need = mapping_work_bytes(n_views, width, height);
  if (!work || work_bytes < need) return fail(ASGS_E_WORKSPACE, "mapping_loss needs %zu bytes of work", need);
  const size_t abc = (size_t)n_views * 9 * (size_t)width * (size_t)height * sizeof(float);
  MappingArgs a{};
  a.rgb = m->rgb;
  a.depth = m->depth;
  a.obs_rgb = m->obs_rgb;
  a.obs_depth = m->obs_depth;
  a.cosine = m->cosine;
  a.dynamic = m->dynamic;
  a.d_rgb = d_rgb;
  a.d_depth = d_depth;
  a.d_cos = d_cos;
  a.abc = d_rgb ? static_cast<float*>(work) : nullptr;
  a.partial = reinterpret_cast<double*>(static_cast<char*>(work) + ((abc + 255) & ~(size_t)255));
  a.W = width;
  a.H = height;
  a.lam = opts->lam;
  a.lam1 = opts->lam1;
  a.lam2 = opts->lam2;
  a.lam4 = opts->lam4;
  mapping_window(a.taps, a.ftaps);
  {
    ProfScope ps(ASGS_K_MAPPING, reinterpret_cast<hipStream_t>(stream));
    launch_mapping_loss(a, n_views, loss, reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("mapping_loss launch");
}

int asgs_mean_scale_work_size(size_t* bytes) {
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  *bytes = mean_scale_work_bytes();
  return ASGS_OK;
}

int asgs_mean_scale(int64_t count, const float* scale, float lam5, float* value, float* d_scale, void* work,
                    size_t work_bytes, void* stream) {
  if (count < 1 || count > ((int64_t)1 << 34)) return fail(ASGS_E_INVALID, "mean_scale: count out of range");
  if (!scale) return fail(ASGS_E_INVALID, "mean_scale: scale is NULL");
  if (!isfinite(lam5)) return fail(ASGS_E_INVALID, "mean_scale: non-finite lam5");
  if (!value && !d_scale) return fail(ASGS_E_INVALID, "mean_scale: no output requested");
  if (!work || work_bytes < mean_scale_work_bytes())
    return fail(ASGS_E_WORKSPACE, "mean_scale needs %zu bytes of work", mean_scale_work_bytes());
  {
    ProfScope ps(ASGS_K_MAPPING, reinterpret_cast<hipStream_t>(stream));
    launch_mean_scale(count, scale, lam5, value, d_scale, static_cast<double*>(work),
                      reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("mean_scale launch");
}

static int check_uncertainty(const asgs_uncertainty_mlp* u) {
  if (!u) return fail(ASGS_E_INVALID, "uncertainty: descriptor is NULL");
  if (u->n_high < 16 || u->n_high > 2048 || u->n_high % 16 != 0)
    return fail(ASGS_E_UNSUPPORTED, "uncertainty: n_high must be a multiple of 16 in 16..2048");
  if (u->grid_h < 1 || u->grid_w < 1 || u->grid_h > 4096 || u->grid_w > 4096)
    return fail(ASGS_E_INVALID, "uncertainty: bad patch grid");
  if (!(u->sigma_min > 0.f) || !isfinite(u->sigma_min) || !isfinite(u->lam3))
    return fail(ASGS_E_INVALID, "uncertainty: sigma_min must be > 0 and lam3 finite");
  if (u->reserved != 0) return fail(ASGS_E_INVALID, "uncertainty: reserved must be 0");
  return ASGS_OK;
}

int asgs_uncertainty_param_count(const asgs_uncertainty_mlp* u, int64_t* count) {
  int st = check_uncertainty(u);
  if (st) return st;
  if (!count) return fail(ASGS_E_INVALID, "count is NULL");
  *count = (int64_t)128 * u->n_high + 128 + 128 + 1;
  return ASGS_OK;
}

int asgs_uncertainty_workspace_size(const asgs_uncertainty_mlp* u, int32_t n_views, int32_t width, int32_t height,
                                    size_t* bytes) {
  int st = check_uncertainty(u);
  if (st) return st;
  if ((st = check_maps_size(n_views, width, height, "uncertainty_workspace_size"))) return st;
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  *bytes = uncertainty_layout(n_views, width, height, u->grid_h, u->grid_w, u->n_high).total;
  return ASGS_OK;
}

int asgs_uncertainty(const asgs_uncertainty_mlp* u, int32_t n_views, int32_t width, int32_t height,
                     const float* params, const float* dino, const float* R, float* sigma, uint8_t* dynamic,
                     float* loss, float* d_params, void* work, size_t work_bytes, void* stream) {
  int st = check_uncertainty(u);
  if (st) return st;
  if ((st = check_maps_size(n_views, width, height, "uncertainty"))) return st;
  if (feature_max_patch_span(width, height, u->grid_h, u->grid_w) > 4)
    return fail(ASGS_E_UNSUPPORTED, "uncertainty: patch grid %dx%d too fine for %dx%d pixels", u->grid_w, u->grid_h,
                width, height);
  if (!params || !dino) return fail(ASGS_E_INVALID, "uncertainty: params and dino are required");
  if ((loss || d_params) && !R) return fail(ASGS_E_INVALID, "uncertainty: loss and d_params need R");
  if (!sigma && !dynamic && !loss && !d_params) return fail(ASGS_E_INVALID, "uncertainty: no output requested");
  const UncLayout L = uncertainty_layout(n_views, width, height, u->grid_h, u->grid_w, u->n_high);
  if (!work || work_bytes < L.total) return fail(ASGS_E_WORKSPACE, "uncertainty needs %zu bytes of work", L.total);
  UncArgs a{};
  a.V = n_views;
  a.W = width;
  a.H = height;
  a.nh = u->n_high;
  a.Hp = u->grid_h;
  a.Wp = u->grid_w;
  a.sx = (float)((double)u->grid_w / width);
  a.sy = (float)((double)u->grid_h / height);
  a.sigma_min = u->sigma_min;
  a.lam3 = u->lam3;
  a.inv_hw = (float)(1.0 / ((double)width * height));
  a.params = params;
  a.dino = dino;
  a.R = R;
  a.sigma = sigma;
  a.dynamic = dynamic;
  {
    ProfScope ps(ASGS_K_UNCERTAINTY, reinterpret_cast<hipStream_t>(stream));
    launch_uncertainty(a, L, static_cast<char*>(work), loss, d_params, reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("uncertainty launch");
}

static int check_decoder(const asgs_decoder* d) {
  if (!d) return fail(ASGS_E_INVALID, "decoder is NULL");
  if (d->n_anchors < 1 || d->n_anchors > ((int64_t)1 << 24)) return fail(ASGS_E_INVALID, "n_anchors out of range");
  if (d->k < 1 || d->k > ASGS_MAX_K) return fail(ASGS_E_UNSUPPORTED, "k must be in 1..%d", ASGS_MAX_K);
  if (d->n_feat != 0 && d->n_feat != 16) return fail(ASGS_E_UNSUPPORTED, "n_feat must be 0 or 16");
  if (d->precision != 0 && d->precision != 1) return fail(ASGS_E_INVALID, "precision must be 0 or 1");
  if (d->precision == 1 && d->n_anchors * d->k > ((int64_t)1 << 27))
    return fail(ASGS_E_UNSUPPORTED, "BF16 decode supports at most 2^27 Gaussians (n_anchors * k)");
  if (!isfinite(d->l_o) || !(d->l_s > 0.f) || !isfinite(d->l_s)) return fail(ASGS_E_INVALID, "bad l_o/l_s");
  if (d->in_dim != 0 && d->in_dim != 35 && d->in_dim != 36 && d->in_dim != 38)
    return fail(ASGS_E_UNSUPPORTED, "decoder.in_dim must be 35, 36 or 38 (got %d)", d->in_dim);
  return ASGS_OK;
}

static int check_ptrs(std::initializer_list<const void*> ps, const char* what) {
  for (const void* p : ps) {
    if (!p) return fail(ASGS_E_INVALID, "%s: NULL pointer", what);
    if (!aligned16(p)) return fail(ASGS_E_INVALID, "%s: pointer not 16-byte aligned", what);
  }
  return ASGS_OK;
}

int asgs_decode_param_count(const asgs_decoder* d, int64_t* count) {
  int st = check_decoder(d);
  if (st) return st;
  if (!count) return fail(ASGS_E_INVALID, "count is NULL");
  *count = decode_const(*d, 1).n_params;
  return ASGS_OK;
}

int asgs_decode_workspace_size(const asgs_decoder* d, int32_t n_views, size_t* bytes) {
  int st = check_decoder(d);
  if (st) return st;
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  *bytes = decode_workspace_bytes(decode_const(*d, n_views));
  return ASGS_OK;
}

static int decode_common(const asgs_decoder* d, const float* xyz, const float* feat, const float* off,
                         const float* params, const asgs_camera* cams, int32_t n_views, ViewDev* views) {
  int st = check_decoder(d);
  if (st) return st;
  if ((st = check_ptrs({xyz, feat, off, params}, "decode inputs"))) return st;
  int tt, tp;
  return make_views(cams, n_views, 0.f, views, &tt, &tp);
}

int asgs_decode(const asgs_decoder* d, const float* anchor_xyz, const float* anchor_feat, const float* anchor_off,
                const float* params, const asgs_camera* cams, int32_t n_views, const asgs_gaussians* out,
                void* stream) {
  ViewDev views[ASGS_MAX_VIEWS];
  int st = decode_common(d, anchor_xyz, anchor_feat, anchor_off, params, cams, n_views, views);
  if (st) return st;
  if ((st = check_gauss(out, d->n_feat, n_views, true, "out"))) return st;
  if (out->n != d->n_anchors * d->k) return fail(ASGS_E_INVALID, "out.n must be n_anchors * k");
  const DecodeConst dc = decode_const(*d, n_views);
  {
    ProfScope ps(ASGS_K_DECODE, reinterpret_cast<hipStream_t>(stream));
    launch_decode(dc, anchor_xyz, anchor_feat, anchor_off, params, views, *out,
                  reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("decode launch");
}

int asgs_decode_backward(const asgs_decoder* d, const float* anchor_xyz, const float* anchor_feat,
                         const float* anchor_off, const float* params, const asgs_camera* cams, int32_t n_views,
                         const asgs_gaussians* d_g, float* d_xyz, float* d_feat, float* d_off, float* d_params,
                         float* d_pose, void* work, size_t work_bytes, void* stream) {
  ViewDev views[ASGS_MAX_VIEWS];
  int st = decode_common(d, anchor_xyz, anchor_feat, anchor_off, params, cams, n_views, views);
  if (st) return st;
  if ((st = check_gauss(d_g, d->n_feat, n_views, true, "d_g"))) return st;
  if (d_g->n != d->n_anchors * d->k) return fail(ASGS_E_INVALID, "d_g.n must be n_anchors * k");
  const bool pose_only = !d_xyz && !d_feat && !d_off && !d_params;
  if (pose_only) {
    if (!d_pose) return fail(ASGS_E_INVALID, "decode_backward: pose-only mode (no anchor outputs) needs d_pose");
    if ((st = check_ptrs({work}, "decode_backward workspace"))) return st;
  } else if ((st = check_ptrs({d_xyz, d_feat, d_off, d_params, work}, "decode_backward outputs"))) {
    return st;
  }
  const DecodeConst dc = decode_const(*d, n_views);
  const size_t need = decode_workspace_bytes(dc);
  if (work_bytes < need) return fail(ASGS_E_WORKSPACE, "decode workspace needs %zu bytes (got %zu)", need, work_bytes);
  {
    ProfScope ps(ASGS_K_DECODE_BWD, reinterpret_cast<hipStream_t>(stream));
    launch_decode_backward(dc, anchor_xyz, anchor_feat, anchor_off, params, views, *d_g, d_xyz, d_feat, d_off,
                           d_params, d_pose, work, reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("decode_backward launch");
}

int asgs_l1_loss_work_size(int32_t n_views, size_t* bytes) {
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  *bytes = (size_t)n_views * kL1Blocks * sizeof(float);
  return ASGS_OK;
}

int asgs_l1_loss(int32_t n_views, int32_t width, int32_t height, int32_t n_feat, const asgs_images* maps,
                 const asgs_l1_targets* targets, const asgs_images* grad, float* loss, void* work,
                 size_t work_bytes, void* stream) {
  L1Args a{};
  L1Views tv{};
  int st = l1_setup(n_views, width, height, n_feat, maps, targets, grad, a, tv);
  if (st) return st;
  if (loss && (!work || work_bytes < (size_t)n_views * kL1Blocks * sizeof(float)))
    return fail(ASGS_E_WORKSPACE, "l1_loss: loss needs %zu bytes of work", (size_t)n_views * kL1Blocks * sizeof(float));
  a.partial = loss ? static_cast<float*>(work) : nullptr;
  a.loss = loss;
  launch_l1_loss(a, tv, reinterpret_cast<hipStream_t>(stream));
  return check_launch("l1_loss launch");
}

void asgs_residual_opts_default(asgs_residual_opts* o) {
  if (!o) return;
  o->w_rgb = 0.25f;
  o->w_depth = 0.7f;
  o->w_feat = 0.1f;
  o->vis_T = 0.1f;
  o->sigma_min = 1e-3f;
  o->dyn_thresh = 1.f;
  o->reserved = 0;
}

int asgs_residual_work_size(int32_t n_views, int32_t width, int32_t height, size_t* bytes) {
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(ASGS_E_INVALID, "bad resolution");
  *bytes = (size_t)n_views * (size_t)residual_partials(width, height) * sizeof(float);
  return ASGS_OK;
}

int asgs_tracking_residual(int32_t n_views, int32_t width, int32_t height, const asgs_residual_opts* opts,
                           const asgs_residual_maps* in, float* R, float* sigma, uint8_t* dynamic, float* xi,
                           void* work, size_t work_bytes, void* stream) {
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(ASGS_E_INVALID, "bad resolution");
  if ((int64_t)width * height * n_views > ((int64_t)1 << 31)) return fail(ASGS_E_INVALID, "too many pixels");
  if (!opts || !in) return fail(ASGS_E_INVALID, "tracking_residual: NULL argument");
  const float wts[6] = {opts->w_rgb, opts->w_depth, opts->w_feat, opts->vis_T, opts->sigma_min, opts->dyn_thresh};
  for (float f : wts)
    if (!isfinite(f)) return fail(ASGS_E_INVALID, "tracking_residual: non-finite option");
  if (!(opts->sigma_min > 0.f)) return fail(ASGS_E_INVALID, "tracking_residual: sigma_min must be > 0");
  if (opts->reserved != 0) return fail(ASGS_E_INVALID, "tracking_residual: reserved must be 0");
  for (const float* ptr : {in->rgb, in->depth, in->alpha, in->cosine, in->obs_rgb, in->obs_depth})
    if (!ptr) return fail(ASGS_E_INVALID, "tracking_residual: input map missing");
  if (!R && !sigma && !dynamic && !xi) return fail(ASGS_E_INVALID, "tracking_residual: no output requested");
  const size_t need = (size_t)n_views * (size_t)residual_partials(width, height) * sizeof(float);
  if (xi && (!work || work_bytes < need))
    return fail(ASGS_E_WORKSPACE, "tracking_residual: xi needs %zu bytes of work", need);
  ResidualArgs a{};
  a.rgb = in->rgb;
  a.depth = in->depth;
  a.alpha = in->alpha;
  a.cosine = in->cosine;
  a.obs_rgb = in->obs_rgb;
  a.obs_depth = in->obs_depth;
  a.R = R;
  a.sigma = sigma;
  a.dynamic = dynamic;
  a.partial = xi ? static_cast<float*>(work) : nullptr;
  a.W = width;
  a.H = height;
  a.w[0] = opts->w_rgb;
  a.w[1] = opts->w_depth;
  a.w[2] = opts->w_feat;
  a.vis_T = opts->vis_T;
  a.sigma_min = opts->sigma_min;
  a.dyn_thresh = opts->dyn_thresh;
  {
    ProfScope ps(ASGS_K_RESIDUAL, reinterpret_cast<hipStream_t>(stream));
    launch_residual(a, n_views, xi, reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("tracking_residual launch");
}

static int feature_check(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height) {
  if (!f) return fail(ASGS_E_INVALID, "feature lift descriptor is NULL");
  if (f->reserved != 0) return fail(ASGS_E_INVALID, "feature lift: reserved must be 0");
  if (f->n_high < 1 || f->n_high > 1024) return fail(ASGS_E_UNSUPPORTED, "feature lift: n_high must be in 1..1024");
  if (n_views < 1 || n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(ASGS_E_INVALID, "bad resolution");
  if (f->grid_h < 1 || f->grid_w < 1 || f->grid_h > height || f->grid_w > width)
    return fail(ASGS_E_INVALID, "feature lift: patch grid must be 1..height x 1..width");
  if (feature_max_patch_span(width, height, f->grid_h, f->grid_w) > 4)
    return fail(ASGS_E_UNSUPPORTED, "feature lift: a 16x16 pixel tile reaches more than 4x4 patches (grid too fine)");
  return ASGS_OK;
}

int asgs_feature_param_count(const asgs_feature_lift* f, int64_t* count) {
  if (!f || !count) return fail(ASGS_E_INVALID, "NULL argument");
  if (f->n_high < 1 || f->n_high > 1024) return fail(ASGS_E_UNSUPPORTED, "feature lift: n_high must be in 1..1024");
  *count = 128 * 16 + 128 + (int64_t)f->n_high * 128 + f->n_high;
  return ASGS_OK;
}

int asgs_feature_workspace_size(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height,
                                size_t* bytes) {
  if (!bytes) return fail(ASGS_E_INVALID, "bytes is NULL");
  int st = feature_check(f, n_views, width, height);
  if (st) return st;
  *bytes = feature_layout(f->n_high, n_views, width, height, f->grid_h, f->grid_w).total;
  return ASGS_OK;
}

static int feature_call(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height, const float* feat,
                        const float* params, const float* dino, void* work, size_t work_bytes, FeatCall& c,
                        FeatLayout& L) {
  int st = feature_check(f, n_views, width, height);
  if (st) return st;
  if (!feat || !params || !dino || !work) return fail(ASGS_E_INVALID, "feature lift: NULL input or work");
  if (!aligned16(feat) || !aligned16(params) || !aligned16(dino) || (reinterpret_cast<uintptr_t>(work) & 255u))
    return fail(ASGS_E_INVALID, "feature lift: inputs must be 16-byte and work 256-byte aligned");
  L = feature_layout(f->n_high, n_views, width, height, f->grid_h, f->grid_w);
  if (work_bytes < L.total) return fail(ASGS_E_WORKSPACE, "feature lift needs %zu bytes of work", L.total);
  c = FeatCall{};
  c.n_views = n_views;
  c.width = width;
  c.height = height;
  c.nh = f->n_high;
  c.Hp = f->grid_h;
  c.Wp = f->grid_w;
  c.feat = feat;
  c.params = params;
  c.dino = dino;
  return ASGS_OK;
}

int asgs_feature_forward(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height,
                         const float* feat, const float* params, const float* dino, float* cosine, float* loss,
                         void* work, size_t work_bytes, void* stream) {
  FeatCall c;
  FeatLayout L;
  int st = feature_call(f, n_views, width, height, feat, params, dino, work, work_bytes, c, L);
  if (st) return st;
  if (!cosine) return fail(ASGS_E_INVALID, "feature_forward: cosine is NULL");
  c.cosine = cosine;
  c.loss = loss;
  {
    ProfScope ps(ASGS_K_FEATURE, reinterpret_cast<hipStream_t>(stream));
    launch_feature_forward(c, L, static_cast<char*>(work), reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("feature_forward launch");
}

int asgs_feature_backward(const asgs_feature_lift* f, int32_t n_views, int32_t width, int32_t height,
                          const float* feat, const float* params, const float* dino, const float* d_cos,
                          float* d_feat, float* d_params, void* work, size_t work_bytes, void* stream) {
  FeatCall c;
  FeatLayout L;
  int st = feature_call(f, n_views, width, height, feat, params, dino, work, work_bytes, c, L);
  if (st) return st;
  if (!d_cos || !d_feat || !d_params) return fail(ASGS_E_INVALID, "feature_backward: NULL gradient argument");
  c.dcos = d_cos;
  c.dfeat = d_feat;
  c.dparams = d_params;
  {
    ProfScope ps(ASGS_K_FEATURE_BWD, reinterpret_cast<hipStream_t>(stream));
    launch_feature_backward(c, L, static_cast<char*>(work), reinterpret_cast<hipStream_t>(stream));
  }
  return check_launch("feature_backward launch");
}

int asgs_anchor_update(int64_t n_anchors, const asgs_anchor_update_opts* opts, const float* p_obs, float* p,
                       uint8_t* keep, int64_t* n_keep, void* stream) {
  if (!opts) return fail(ASGS_E_INVALID, "anchor_update: opts is NULL");
  if (n_anchors < 1 || n_anchors > ((int64_t)1 << 31)) return fail(ASGS_E_INVALID, "anchor_update: n_anchors out of range");
  if (!p_obs || !p) return fail(ASGS_E_INVALID, "anchor_update: NULL probabilities");
  if (!(opts->prior > 0.f && opts->prior < 1.f)) return fail(ASGS_E_INVALID, "anchor_update: prior must be in (0, 1)");
  if (!(opts->p_min >= 0.f && opts->p_max <= 1.f && opts->p_min <= opts->p_max) || !isfinite(opts->prune_below))
    return fail(ASGS_E_INVALID, "anchor_update: need 0 <= p_min <= p_max <= 1 and a finite prune level");
  if (opts->reserved != 0) return fail(ASGS_E_INVALID, "anchor_update: reserved must be 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  launch_anchor_update(n_anchors, p_obs, p, keep, reinterpret_cast<unsigned long long*>(n_keep), opts->prior,
                       opts->p_min, opts->p_max, opts->prune_below, s);
  return check_launch("anchor_update launch");
}

int asgs_profile_enable(uint32_t mask) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& e : g_prof) {
    (void)hipEventSynchronize(e.b);
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  g_prof.clear();
  __atomic_store_n(&g_prof_mask, mask & ((1u << ASGS_K_NUM) - 1u), __ATOMIC_RELAXED);
  return ASGS_OK;
}

int asgs_profile_read(int32_t kernel_class, double* total_ms, int64_t* launches) {
  if (kernel_class < 0 || kernel_class >= ASGS_K_NUM) return fail(ASGS_E_INVALID, "bad kernel class");
  if (!total_ms || !launches) return fail(ASGS_E_INVALID, "NULL output");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& e : g_prof) {
    if (e.cls != kernel_class) continue;
    hipError_t err = hipEventSynchronize(e.b);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e.a, e.b);
    if (err != hipSuccess) return fail(ASGS_E_DEVICE, "profile read: %s", hipGetErrorString(err));
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return ASGS_OK;
}

}  // extern "C"
