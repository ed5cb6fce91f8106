// Multi-modal tracking residual (UP-SLAM Sec. 3.2, Eq. 6) and the per-pixel
// uncertainty of the training-free estimator with its motion mask (Sec. 3.4,
// Eq. 15), in one pass over the rendered and observed maps:
//   R     = vis * (w_rgb sum_c |C~_c - C_c| + w_depth |D~ - box3(D)| + w_feat min(1, 1 - cos))
//   vis   = (1 - alpha) < vis_T          (alpha = rendered opacity sum, Eq. 3)
//   sigma = max(sigma_min, sqrt(2 R))    (the exact minimiser of 1/2 (R/s^2 + log s), s >= sigma_min)
//   dyn   = 2 max(sigma_min^2, 2 R) > dyn_thresh   (= 2 sigma^2 > dyn_thresh)
//   xi    = mean over the view of 1/2 (R / sigma^2 + log sigma)
// box3 is the mean of the observed depth over the pixel and its in-image
// neighbours. HBM-bound: one workgroup per 64x4 pixel tile stages the tile's
// observed depth with a one-pixel halo in LDS; every other map is read once.
#include "internal.h"

namespace asgs {

namespace {

constexpr int kResTX = 64, kResTY = 4;  // pixels of one workgroup (one row of 64 per wave)
constexpr int kResThreads = kResTX * kResTY;

__global__ void __launch_bounds__(kResThreads) k_residual(ResidualArgs a) {
  __shared__ float sd[kResTY + 2][kResTX + 2];
  __shared__ float red[kResThreads / 64];
  const int v = blockIdx.z;
  const int W = a.W, H = a.H;
  const int64_t HW = (int64_t)W * H;
  const int x0 = blockIdx.x * kResTX, y0 = blockIdx.y * kResTY;
  const float* od = a.obs_depth + v * HW;
  for (int q = threadIdx.x; q < (kResTY + 2) * (kResTX + 2); q += kResThreads) {
    const int yy = q / (kResTX + 2), xx = q - yy * (kResTX + 2);
    const int gy = y0 + yy - 1, gx = x0 + xx - 1;
    sd[yy][xx] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? od[(int64_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  const int tx = threadIdx.x % kResTX, ty = threadIdx.x / kResTX;
  const int x = x0 + tx, y = y0 + ty;
  float obj = 0.f;
  if (x < W && y < H) {
    const int64_t p = (int64_t)y * W + x;
    const float* rgb = a.rgb + v * 3 * HW;
    const float* orgb = a.obs_rgb + v * 3 * HW;
    const float r0 = rgb[p], r1 = rgb[HW + p], r2 = rgb[2 * HW + p];
    const float o0 = orgb[p], o1 = orgb[HW + p], o2 = orgb[2 * HW + p];
    const float dep = a.depth[v * HW + p];
    const float alpha = a.alpha[v * HW + p];
    const float cs = a.cosine[v * HW + p];
    // box mean over the in-image part of the 3x3 neighbourhood (row by row)
    float s = 0.f;
    int cnt = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const bool in = (unsigned)(y + dy) < (unsigned)H && (unsigned)(x + dx) < (unsigned)W;
        s += in ? sd[ty + 1 + dy][tx + 1 + dx] : 0.f;
        cnt += in ? 1 : 0;
      }
    float R = 0.f;
    if (1.f - alpha < a.vis_T) {
      const float rc = fabsf(r0 - o0) + fabsf(r1 - o1) + fabsf(r2 - o2);
      const float rd = fabsf(dep - s / (float)cnt);
      const float rf = fminf(1.f, 1.f - cs);
      R = a.w[0] * rc + a.w[1] * rd + a.w[2] * rf;
    }
    const float sig = fmaxf(a.sigma_min, sqrtf(2.f * R));
    obj = 0.5f * (R / (sig * sig) + logf(sig));
    const bool dyn = 2.f * fmaxf(a.sigma_min * a.sigma_min, 2.f * R) > a.dyn_thresh;
    if (a.R) a.R[v * HW + p] = R;
    if (a.sigma) a.sigma[v * HW + p] = sig;
    if (a.dynamic) a.dynamic[v * HW + p] = dyn ? 1u : 0u;
  }
  if (!a.partial) return;
  for (int o = 32; o > 0; o >>= 1) obj += __shfl_xor(obj, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = obj;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int q = 0; q < kResThreads / 64; ++q) t += red[q];
    a.partial[(int64_t)v * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

// xi of each view: fixed-order sum of its tile partials over its pixels.
__global__ void __launch_bounds__(256) k_residual_mean(const float* __restrict__ partial, int per_view,
                                                       float inv_hw, float* xi) {
  __shared__ float red[4];
  const int v = blockIdx.x;
  float t = 0.f;
  for (int b = threadIdx.x; b < per_view; b += 256) t += partial[(int64_t)v * per_view + b];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) xi[v] = ((red[0] + red[1]) + (red[2] + red[3])) * inv_hw;
}

}  // namespace

int64_t residual_partials(int width, int height) {
  return (int64_t)((width + kResTX - 1) / kResTX) * ((height + kResTY - 1) / kResTY);
}

void launch_residual(const ResidualArgs& a, int n_views, float* xi, hipStream_t s) {
  dim3 grid((unsigned)((a.W + kResTX - 1) / kResTX), (unsigned)((a.H + kResTY - 1) / kResTY), (unsigned)n_views);
  hipLaunchKernelGGL(k_residual, grid, dim3(kResThreads), 0, s, a);
  if (xi && a.partial)
    hipLaunchKernelGGL(k_residual_mean, dim3(n_views), dim3(256), 0, s, a.partial,
                       (int)residual_partials(a.W, a.H), 1.f / ((float)a.W * (float)a.H), xi);
}

}  // namespace asgs
