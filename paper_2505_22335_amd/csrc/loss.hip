// Weighted L1 residual of rendered maps (the photometric / depth / feature
// residual the tracking and mapping losses are built from, UP-SLAM Eq. 4 and
// Sec. 3.4) and its gradient with respect to the maps, fused into one pass:
// per pixel p of view v and channel group (rgb, depth, feature, opacity sum),
//   L_v += s_g w_p |x - x*|,   dL/dx = s_g w_p sign(x - x*)   (sign(0) = 0).
// A group without targets contributes nothing and gets zero gradient. The
// per-view loss is a fixed-order sum of per-block partial sums.
#include "internal.h"

namespace asgs {

namespace {

constexpr int kLossThreads = 256;

ASGS_DEV float sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__global__ void __launch_bounds__(kLossThreads) k_l1_loss(L1Args a, L1Views tv) {
  __shared__ float red[kLossThreads / 64];
  const int v = blockIdx.y;
  const int64_t HW = a.HW;
  const float* w = tv.w[v];
  const int nc[4] = {3, 1, a.nf, 1};
  float acc = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; p < HW; p += (int64_t)gridDim.x * kLossThreads) {
    const float wp = w ? w[p] : 1.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int C = nc[g];
      if (C == 0 || !a.x[g]) continue;
      const float* x = a.x[g] + (int64_t)v * C * HW;
      const float* t = tv.t[g][v];
      float* gr = a.g[g] ? a.g[g] + (int64_t)v * C * HW : nullptr;
      float l = 0.f;
      for (int c = 0; c < C; ++c) {
        float gv = 0.f;
        if (t) {
          const float d = x[c * HW + p] - t[c * HW + p];
          gv = wp * sgn(d) * a.s[g];
          l += fabsf(d);
        }
        if (gr) gr[c * HW + p] = gv;
      }
      acc += wp * l * a.s[g];
    }
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
  hipLaunchKernelGGL(k_l1_loss, dim3(kL1Blocks, a.n_views), dim3(kLossThreads), 0, s, a, tv);
  if (a.partial && a.loss)
    hipLaunchKernelGGL(k_l1_loss_sum, dim3(1), dim3(64), 0, s, a.partial, a.loss, a.n_views);
}

}  // namespace asgs
