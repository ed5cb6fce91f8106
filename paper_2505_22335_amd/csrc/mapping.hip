// Mapping loss of one iteration and its gradient w.r.t. the rendered maps
// (UP-SLAM Sec. 3.1 Eq. 4 and Sec. 3.3 Eq. 14), and the mean-scale term.
//
// Per pixel p of a view (HW pixels), with the motion mask M (dynamic pixels
// drop out):
//   l_p = (1 - M_p) [ lam1 (lam sum_c (C~ - C)^2 + (1 - lam)(1 - SSIM_p))
//                     + lam2 (D~ - D)^2 + lam4 (1 - cos_p) ],   L = sum_p l_p / HW
// SSIM_p averages the three colour channels' structural-similarity maps over
// an 11 x 11 Gaussian window (sigma 1.5) with zero padding. Per channel the
// window sums mu_x, mu_y, E[x^2], E[y^2], E[xy] give
//   S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)),
// s_xx = E[x^2] - mu_x^2 etc., and its gradient w.r.t. the rendered x at q is
//   G * A (q) + 2 x_q (G * B)(q) + y_q (G * Cc)(q)
// with g_p = dL/dS_p and, at p, A = g dS/dmu_x, B = g dS/dE[x^2] = -g S / m2,
// Cc = g dS/dE[xy] = 2 g S / l2 (the Gaussian window is symmetric, so the
// transposed filter is the filter).
//
// Two stencil passes over 32 x 16 pixel tiles with a 5-pixel halo staged in
// LDS, the 2D window applied as a horizontal then a vertical 11-tap pass:
//   k_map_fwd: per channel the five window sums (in FP64: the variances are
//              differences of nearly equal sums, compared with C2 = 9e-4),
//              SSIM, and A, B, Cc into the workspace; the depth and cosine
//              gradients and the loss partial of the tile (pointwise);
//   k_map_bwd: the three maps filtered again (FP32), combined with x and y
//              into the colour gradient, plus the L2 colour term.
// HBM-bound: colour, depth, cosine and mask read once, 9 floats per pixel
// written and read back, the gradients written once.
#include <math.h>

#include "internal.h"

namespace asgs {

namespace {

constexpr int kTW = 32, kTH = 16;  // output pixels of one workgroup
constexpr int kR = 5;              // window radius
constexpr int kXW = kTW + 2 * kR, kXH = kTH + 2 * kR;
constexpr int kThreads = 256;      // pixel (tx, ty) and (tx, ty + 8) per thread
constexpr int kStage = (kXH * kXW + kThreads - 1) / kThreads;  // halo values per thread
constexpr double kC1 = 0.01 * 0.01, kC2 = 0.03 * 0.03;

__global__ void __launch_bounds__(kThreads) k_map_fwd(MappingArgs a) {
  __shared__ float sx[kXH][kXW + 1], sy[kXH][kXW + 1];
  __shared__ double hs[5][kXH][kTW + 1];
  __shared__ double red[kThreads / 64];
  const int v = blockIdx.z;
  const int W = a.W, H = a.H;
  const int64_t HW = (int64_t)W * H;
  const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
  const int t = threadIdx.x;
  const int tx = t & (kTW - 1), ty = t / kTW;
  const double inv_hw = 1.0 / (double)HW;
  bool in[2];
  int64_t p[2];
  double wgt[2], ssum[2] = {0.0, 0.0}, col[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int xx = x0 + tx, yy = y0 + ty + 8 * i;
    in[i] = xx < W && yy < H;
    p[i] = in[i] ? (int64_t)yy * W + xx : 0;
    wgt[i] = in[i] && !(a.dynamic && a.dynamic[v * HW + p[i]]) ? 1.0 : 0.0;
  }
  // dL/dS of one channel's SSIM at a pixel of weight 1
  const double gS = -(double)a.lam1 * (1.0 - (double)a.lam) / 3.0 * inv_hw;
  // a channel's halo tile (zero outside the image), every load of a thread
  // issued before any store; the next channel's loads are in flight while the
  // current one is filtered
  float vx[kStage], vy[kStage];
  auto fetch = [&](int c) {
    const float* X = a.rgb + ((int64_t)v * 3 + c) * HW;
    const float* Y = a.obs_rgb + ((int64_t)v * 3 + c) * HW;
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int q = t + kThreads * k, r = q / kXW, j = q - r * kXW;
      const int gy = y0 + r - kR, gx = x0 + j - kR;
      const bool ok = q < kXH * kXW && gy >= 0 && gy < H && gx >= 0 && gx < W;
      const int64_t o = ok ? (int64_t)gy * W + gx : 0;
      vx[k] = ok ? X[o] : 0.f;
      vy[k] = ok ? Y[o] : 0.f;
    }
  };
  fetch(0);
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int q = t + kThreads * k;
      if (q < kXH * kXW) {
        sx[q / kXW][q % kXW] = vx[k];
        sy[q / kXW][q % kXW] = vy[k];
      }
    }
    __syncthreads();
    fetch(c < 2 ? c + 1 : 2);
    for (int q = t; q < kXH * kTW; q += kThreads) {
      const int r = q / kTW, j = q - r * kTW;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; ++k) {
        const double g = a.taps[k];
        const double xv = sx[r][j + k], yv = sy[r][j + k];
        const double gx = g * xv, gy = g * yv;
        m0 += gx;
        m1 += gy;
        m2 += gx * xv;
        m3 += gy * yv;
        m4 += gx * yv;
      }
      hs[0][r][j] = m0;
      hs[1][r][j] = m1;
      hs[2][r][j] = m2;
      hs[3][r][j] = m3;
      hs[4][r][j] = m4;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = ty + 8 * i;
      double mx = 0.0, my = 0.0, exx = 0.0, eyy = 0.0, exy = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; ++k) {
        const double g = a.taps[k];
        mx += g * hs[0][r + k][tx];
        my += g * hs[1][r + k][tx];
        exx += g * hs[2][r + k][tx];
        eyy += g * hs[3][r + k][tx];
        exy += g * hs[4][r + k][tx];
      }
      if (!in[i]) continue;
      const double sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
      const double l1 = 2.0 * mx * my + kC1, m1 = mx * mx + my * my + kC1;
      const double l2 = 2.0 * sxy + kC2, m2 = sxx + syy + kC2;
      // four reciprocals instead of seven divisions
      const double il1 = 1.0 / l1, im1 = 1.0 / m1, il2 = 1.0 / l2, im2 = 1.0 / m2;
      const double S = (l1 * l2) * (im1 * im2);
      ssum[i] += S;
      const double g = gS * wgt[i];
      const double dmx = S * (2.0 * my * il1 - 2.0 * mx * im1 - 2.0 * my * il2 + 2.0 * mx * im2);
      if (a.abc) {
        float* abc = a.abc + ((int64_t)v * 9 + 3 * c) * HW + p[i];
        abc[0] = (float)(g * dmx);
        abc[HW] = (float)(g * (-S * im2));
        abc[2 * HW] = (float)(g * (2.0 * S * il2));
      }
      const double dc = (double)sx[r + kR][tx + kR] - (double)sy[r + kR][tx + kR];
      col[i] += dc * dc;
    }
    __syncthreads();  // the next channel overwrites the staged rows
  }
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!in[i]) continue;
    const int64_t q = v * HW + p[i];
    double l = (double)a.lam1 * ((double)a.lam * col[i] + (1.0 - (double)a.lam) * (1.0 - ssum[i] / 3.0));
    const double dz = (double)a.depth[q] - (double)a.obs_depth[q];
    l += (double)a.lam2 * dz * dz;
    if (a.d_depth) a.d_depth[q] = (float)(wgt[i] * 2.0 * (double)a.lam2 * dz * inv_hw);
    if (a.cosine) {
      l += (double)a.lam4 * (1.0 - (double)a.cosine[q]);
      if (a.d_cos) a.d_cos[q] = (float)(-wgt[i] * (double)a.lam4 * inv_hw);
    }
    lsum += wgt[i] * l;
  }
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
  if ((t & 63) == 0) red[t >> 6] = lsum;
  __syncthreads();
  if (t == 0)
    a.partial[(int64_t)v * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] =
        (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(kThreads) k_map_bwd(MappingArgs a) {
  __shared__ float sa[3][kXH][kXW + 1];
  __shared__ float hb[3][kXH][kTW + 1];
  const int v = blockIdx.z;
  const int W = a.W, H = a.H;
  const int64_t HW = (int64_t)W * H;
  const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
  const int t = threadIdx.x;
  const int tx = t & (kTW - 1), ty = t / kTW;
  const float l2c = (float)(2.0 * (double)a.lam1 * (double)a.lam / ((double)HW));
  // a channel's three halo tiles, loaded as in the forward (next channel in flight)
  float va[3][kStage];
  auto fetch = [&](int c) {
    const float* A = a.abc + ((int64_t)v * 9 + 3 * c) * HW;
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int q = t + kThreads * k, r = q / kXW, j = q - r * kXW;
      const int gy = y0 + r - kR, gx = x0 + j - kR;
      const bool ok = q < kXH * kXW && gy >= 0 && gy < H && gx >= 0 && gx < W;
      const int64_t o = ok ? (int64_t)gy * W + gx : 0;
#pragma unroll
      for (int m = 0; m < 3; ++m) va[m][k] = ok ? A[m * HW + o] : 0.f;
    }
  };
  fetch(0);
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int k = 0; k < kStage; ++k) {
      const int q = t + kThreads * k;
      if (q < kXH * kXW) {
#pragma unroll
        for (int m = 0; m < 3; ++m) sa[m][q / kXW][q % kXW] = va[m][k];
      }
    }
    __syncthreads();
    fetch(c < 2 ? c + 1 : 2);
    for (int q = t; q < kXH * kTW; q += kThreads) {
      const int r = q / kTW, j = q - r * kTW;
      float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; ++k) {
        const float g = a.ftaps[k];
        m0 = fmaf(g, sa[0][r][j + k], m0);
        m1 = fmaf(g, sa[1][r][j + k], m1);
        m2 = fmaf(g, sa[2][r][j + k], m2);
      }
      hb[0][r][j] = m0;
      hb[1][r][j] = m1;
      hb[2][r][j] = m2;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = ty + 8 * i;
      float ga = 0.f, gb = 0.f, gc = 0.f;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; ++k) {
        const float g = a.ftaps[k];
        ga = fmaf(g, hb[0][r + k][tx], ga);
        gb = fmaf(g, hb[1][r + k][tx], gb);
        gc = fmaf(g, hb[2][r + k][tx], gc);
      }
      const int xx = x0 + tx, yy = y0 + r;
      if (xx >= W || yy >= H) continue;
      const int64_t q = ((int64_t)v * 3 + c) * HW + (int64_t)yy * W + xx;
      const float x = a.rgb[q], y = a.obs_rgb[q];
      const bool dyn = a.dynamic && a.dynamic[v * HW + (int64_t)yy * W + xx];
      a.d_rgb[q] = ga + 2.f * x * gb + y * gc + (dyn ? 0.f : l2c * (x - y));
    }
    __syncthreads();
  }
}

// Loss of each view: fixed-order sum of its tile partials over its pixels.
__global__ void __launch_bounds__(256) k_map_mean(const double* __restrict__ partial, int per_view, double inv_hw,
                                                  float* loss) {
  __shared__ double red[4];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < per_view; b += 256) s += partial[(int64_t)v * per_view + b];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[v] = (float)(((red[0] + red[1]) + (red[2] + red[3])) * inv_hw);
}

// Mean scale: block partials of a grid-stride sum (and the constant gradient
// lam5 / count added to d_scale), then their fixed-order sum.
constexpr int kScaleBlocks = 256;
__global__ void __launch_bounds__(256) k_scale_partial(int64_t count, const float* __restrict__ scale, float dval,
                                                       float* d_scale, double* partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256) {
    s += (double)scale[i];
    if (d_scale) d_scale[i] += dval;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_scale_final(const double* __restrict__ partial, int n, double inv_count,
                                                     float* value) {
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) s += partial[b];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) value[0] = (float)(((red[0] + red[1]) + (red[2] + red[3])) * inv_count);
}

}  // namespace

int64_t mapping_tiles(int width, int height) {
  return (int64_t)((width + kTW - 1) / kTW) * ((height + kTH - 1) / kTH);
}

void mapping_window(double* taps, float* ftaps) {
  double s = 0.0;
  for (int k = 0; k <= 2 * kR; ++k) {
    const double d = (double)(k - kR);
    taps[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    s += taps[k];
  }
  for (int k = 0; k <= 2 * kR; ++k) {
    taps[k] /= s;
    ftaps[k] = (float)taps[k];
  }
}

void launch_mapping_loss(const MappingArgs& a, int n_views, float* loss, hipStream_t s) {
  dim3 grid((unsigned)((a.W + kTW - 1) / kTW), (unsigned)((a.H + kTH - 1) / kTH), (unsigned)n_views);
  hipLaunchKernelGGL(k_map_fwd, grid, dim3(kThreads), 0, s, a);
  if (a.d_rgb) hipLaunchKernelGGL(k_map_bwd, grid, dim3(kThreads), 0, s, a);
  if (loss)
    hipLaunchKernelGGL(k_map_mean, dim3(n_views), dim3(256), 0, s, a.partial, (int)mapping_tiles(a.W, a.H),
                       1.0 / ((double)a.W * (double)a.H), loss);
}

size_t mean_scale_work_bytes() { return kScaleBlocks * sizeof(double); }

void launch_mean_scale(int64_t count, const float* scale, float lam5, float* value, float* d_scale, double* work,
                       hipStream_t s) {
  const int64_t need = (count + 255) / 256;
  const unsigned nb = (unsigned)(need < kScaleBlocks ? need : kScaleBlocks);
  hipLaunchKernelGGL(k_scale_partial, dim3(nb), dim3(256), 0, s, count, scale, (float)((double)lam5 / (double)count),
                     d_scale, work);
  if (value) hipLaunchKernelGGL(k_scale_final, dim3(1), dim3(256), 0, s, work, (int)nb, 1.0 / (double)count, value);
}

}  // namespace asgs
