// Weighted L1 residual of rendered maps (the photometric / depth / feature
// residual the tracking and mapping losses are built from, UP-SLAM Eq. 4 and
// Sec. 3.4) and its gradient with respect to the maps, fused into one pass:
// per pixel p of view v and channel group (rgb, depth, feature, opacity sum),
//   L_v += s_g w_p |x - x*|,   dL/dx = s_g w_p sign(x - x*)   (sign(0) = 0).
// A group without targets contributes nothing and gets zero gradient. The
// per-view loss is a fixed-order sum of per-block partial sums.
#include <mutex>

#include "internal.h"

namespace asgs {

namespace {

constexpr int kLossThreads = 256;

ASGS_DEV float sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

template <int VW> struct Vec;
template <> struct Vec<1> { using T = float; };
template <> struct Vec<4> { using T = float4; };

ASGS_DEV float lane(float v, int) { return v; }
ASGS_DEV float lane(float4 v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
ASGS_DEV void set_lane(float& v, int, float f) { v = f; }
ASGS_DEV void set_lane(float4& v, int i, float f) {
  if (i == 0) v.x = f; else if (i == 1) v.y = f; else if (i == 2) v.z = f; else v.w = f;
}

// One channel group of VW consecutive pixels starting at p: every load of the
// group is issued before any store, so the loads are in flight together.
template <int C, int VW>
ASGS_DEV float group_l1(const float* __restrict__ x, const float* __restrict__ t, float* __restrict__ g,
                        int64_t HW, int64_t p, const typename Vec<VW>::T& w, float s) {
  using V = typename Vec<VW>::T;
  V xv[C], tv[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    xv[c] = *reinterpret_cast<const V*>(x + c * HW + p);
    tv[c] = *reinterpret_cast<const V*>(t + c * HW + p);
  }
  float l[VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) l[i] = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    V gv;
#pragma unroll
    for (int i = 0; i < VW; ++i) {
      const float d = lane(xv[c], i) - lane(tv[c], i);
      l[i] += fabsf(d);
      set_lane(gv, i, lane(w, i) * sgn(d) * s);
    }
    if (g) *reinterpret_cast<V*>(g + c * HW + p) = gv;
  }
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < VW; ++i) acc += lane(w, i) * l[i] * s;
  return acc;
}

// Zero gradient for a group without targets.
template <int C, int VW>
ASGS_DEV void group_zero(float* __restrict__ g, int64_t HW, int64_t p) {
  using V = typename Vec<VW>::T;
  V z;
#pragma unroll
  for (int i = 0; i < VW; ++i) set_lane(z, i, 0.f);
#pragma unroll
  for (int c = 0; c < C; ++c) *reinterpret_cast<V*>(g + c * HW + p) = z;
}

template <int C, int VW>
ASGS_DEV float group(const L1Args& a, const L1Views& tv, int q, int v, int64_t p, const typename Vec<VW>::T& w) {
  if (!a.x[q]) return 0.f;
  const int64_t off = (int64_t)v * C * a.HW;
  float* g = a.g[q] ? a.g[q] + off : nullptr;
  const float* t = tv.t[q][v];
  if (!t) {
    if (g) group_zero<C, VW>(g, a.HW, p);
    return 0.f;
  }
  return group_l1<C, VW>(a.x[q] + off, t, g, a.HW, p, w, a.s[q]);
}

// Each thread takes VW consecutive pixels per step (VW = 4 when the plane
// size is a multiple of 4, so every plane start is 16-byte aligned).
template <int VW>
__global__ void __launch_bounds__(kLossThreads) k_l1_loss(L1Args a, L1Views tv) {
  using V = typename Vec<VW>::T;
  __shared__ float red[kLossThreads / 64];
  const int v = blockIdx.y;
  const int64_t HW = a.HW;
  const float* w = tv.w[v];
  float acc = 0.f;
  for (int64_t p = ((int64_t)blockIdx.x * kLossThreads + threadIdx.x) * VW; p < HW;
       p += (int64_t)gridDim.x * kLossThreads * VW) {
    V wv;
    if (w) {
      wv = *reinterpret_cast<const V*>(w + p);
    } else {
#pragma unroll
      for (int i = 0; i < VW; ++i) set_lane(wv, i, 1.f);
    }
    acc += group<3, VW>(a, tv, 0, v, p, wv);
    acc += group<1, VW>(a, tv, 1, v, p, wv);
    if (a.nf == 16) acc += group<16, VW>(a, tv, 2, v, p, wv);
    acc += group<1, VW>(a, tv, 3, v, p, wv);
  }
  if (!a.partial) return;
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int q = 0; q < kLossThreads / 64; ++q) s += red[q];
    a.partial[v * kL1Blocks + blockIdx.x] = s;
  }
}

__global__ void k_l1_loss_sum(const float* partial, float* loss, int n_views) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  float s = 0.f;
  for (int b = 0; b < kL1Blocks; ++b) s += partial[v * kL1Blocks + b];
  loss[v] = s;
}

}  // namespace

void launch_l1_loss(const L1Args& a, const L1Views& tv, hipStream_t s) {
  if (a.HW % 4 == 0)
    hipLaunchKernelGGL(k_l1_loss<4>, dim3(kL1Blocks, a.n_views), dim3(kLossThreads), 0, s, a, tv);
  else
    hipLaunchKernelGGL(k_l1_loss<1>, dim3(kL1Blocks, a.n_views), dim3(kLossThreads), 0, s, a, tv);
  if (a.partial && a.loss)
    hipLaunchKernelGGL(k_l1_loss_sum, dim3(1), dim3(64), 0, s, a.partial, a.loss, a.n_views);
}

}  // namespace asgs

// ---------------------------------------------------------------------------
// Allocation-free variant of asgs_l1_loss. Its per-(view, block) loss partials
// live in a file-scope device array instead of a caller workspace. Every block
// of k_l1_loss writes its own partial on every call, so nothing has to be
// cleared between calls; calls that overlap on one GPU share the array and
// race.
// ---------------------------------------------------------------------------
static_assert(ASGS_L1_NOALLOC_MAX_VIEWS <= ASGS_MAX_VIEWS, "scratch sized per view");
static __device__ __align__(256) float scratch[(size_t)ASGS_L1_NOALLOC_MAX_VIEWS * asgs::kL1Blocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};  // device address of scratch per device (host-side name is not one)

// Device address of scratch on the current device, looked up once per device.
int scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return asgs::fail(ASGS_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return asgs::fail(ASGS_E_UNSUPPORTED, "device ordinal %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return asgs::fail(ASGS_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_dev[dev];
  return ASGS_OK;
}

}  // namespace

extern "C" int asgs_l1_loss_noalloc(int32_t n_views, int32_t width, int32_t height, int32_t n_feat,
                                    const asgs_images* maps, const asgs_l1_targets* targets,
                                    const asgs_images* grad, float* loss, void* stream) {
  if (n_views > ASGS_L1_NOALLOC_MAX_VIEWS)
    return asgs::fail(ASGS_E_UNSUPPORTED, "l1_loss_noalloc: at most %d views (its scratch holds %d loss partials)",
                      ASGS_L1_NOALLOC_MAX_VIEWS, ASGS_L1_NOALLOC_MAX_VIEWS * asgs::kL1Blocks);
  asgs::L1Args a{};
  asgs::L1Views tv{};
  int st = asgs::l1_setup(n_views, width, height, n_feat, maps, targets, grad, a, tv);
  if (st) return st;
  if (loss) {
    float* part = nullptr;
    if ((st = scratch_address(&part))) return st;
    a.partial = part;
    a.loss = loss;
  }
  asgs::launch_l1_loss(a, tv, reinterpret_cast<hipStream_t>(stream));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return asgs::fail(ASGS_E_DEVICE, "l1_loss_noalloc launch: %s", hipGetErrorString(e));
  return ASGS_OK;
}
