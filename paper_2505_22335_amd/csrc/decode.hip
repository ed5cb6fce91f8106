// Anchor -> neural Gaussian decoding and its backward (UP-SLAM Sec. 3.3,
// Eq. 8 and Eq. 9; head MLP details in the appendix).
//
// Per anchor v and view with camera centre c: X = [f_v (32), delta (3)],
// delta = (x_v - c)/|x_v - c|, optionally followed by |x_v - c| and the
// temporal embedding (sin pi t, cos pi t) of the view. Five heads (opacity,
// rgb, scale, rot, feat), each Y_h = W2_h act_h(W1_h X + b1_h) + b2_h with a
// 32-wide hidden layer
// (ReLU for the first four, SoftPlus for the feature head), then the output
// activations: sigmoid (opacity, rgb), l_s * sigmoid (scale), raw (rot, feat).
//
// Forward and backward run on the matrix cores with FP32 16x16x4 MFMAs, one
// 16-anchor tile at a time (forward: decode_fwd.hip, backward:
// decode_bwd.hip); the BF16 variant of the forward rounds the operands of
// the feature columns and of the second layer to bfloat16. The backward
// recomputes the forward, forms dL/dH from the second-layer weights, dL/dZ
// through the activations, dL/dX from the first layer and from it the anchor
// gradients, and the weight gradients as per-workgroup sums reduced here in
// a fixed order (deterministic, no atomics). This file holds the reductions
// around them.
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

// Mean gradients summed over views: d_off = l_o dmu, d_xyz += sum_i dmu
// (element e of the 3 A anchor coordinates).
ASGS_DEV void dec_bwd_mean(const DecodeConst& dc, const asgs_gaussians& dg, float* d_xyz, float* d_off,
                           int64_t e) {
  const int64_t A = dc.A;
  const int k = dc.k;
  const int64_t n = A * k;
  if (e >= A * 3) return;
  const int c = (int)(e / A);
  const int64_t a = e - c * A;
  float sx = 0.f;
  for (int i = 0; i < k; ++i) {
    const int64_t gn = a * k + i;
    float s = 0.f;
    for (int view = 0; view < dc.n_views; ++view) s += dg.mean[view * dg.view_stride[0] + c * n + gn];
    d_off[c * n + gn] = dc.l_o * s;
    sx += s;
  }
  d_xyz[c * A + a] += sx;
}

// Fixed-order reduction of the workgroup partials: 64 parameters per
// workgroup, four threads per parameter (each a strided quarter of the
// partials), combined in LDS. The extra workgroup
// adds -R_cw dL/dc to the translation part of the pose gradient. Workgroups
// from mean_first on take the mean gradients instead (one launch for both).
__global__ void __launch_bounds__(256) k_decode_reduce(DecodeConst dc, DecodeViews dv, DecWork w, float* d_params,
                                                       float* d_pose, int mean_first, asgs_gaussians dg,
                                                       float* d_xyz, float* d_off) {
  if ((int)blockIdx.x >= mean_first) {
    dec_bwd_mean(dc, dg, d_xyz, d_off, (int64_t)(blockIdx.x - mean_first) * blockDim.x + threadIdx.x);
    return;
  }
  // without d_params only the camera-centre term is reduced (one block)
  __shared__ float red[4][64];
  const int t = threadIdx.x;
  const int pl = t & 63, q = t >> 6;
  const int64_t p = (int64_t)blockIdx.x * 64 + pl;
  const int64_t nparam_blocks = d_params ? (dc.n_params + 63) / 64 : 0;
  if ((int64_t)blockIdx.x < nparam_blocks) {
    // sixteen loads in flight per thread and round, summed in a fixed tree
    float acc = 0.f;
    if (p < dc.n_params) {
      const float* src = w.part + part_index(p, 0, w.nblk_w);  // workgroup b at src[64 b]
      for (int b0 = q; b0 < w.nblk_w; b0 += 64) {
        float v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int b = b0 + 4 * i;
          v[i] = b < w.nblk_w ? src[(int64_t)b * 64] : 0.f;
        }
#pragma unroll
        for (int st = 8; st > 0; st >>= 1)
#pragma unroll
          for (int i = 0; i < st; ++i) v[i] += v[i + st];
        acc += v[0];
      }
    }
    red[q][pl] = acc;
    __syncthreads();
    if (q == 0 && p < dc.n_params) d_params[p] = (red[0][pl] + red[1][pl]) + (red[2][pl] + red[3][pl]);
    return;
  }
  if (!d_pose) return;
  // camera-centre gradient: every thread sums a strided share of the
  // per-workgroup partials, then a block reduction per (view, component)
  for (int view = 0; view < dc.n_views; ++view) {
    float g[3];
    for (int c = 0; c < 3; ++c) {
      float acc = 0.f;
      for (int b = t; b < w.nblk_w; b += blockDim.x) acc += w.dcpart[((int64_t)b * dc.n_views + view) * 3 + c];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      __syncthreads();
      if ((t & 63) == 0) red[t >> 6][0] = acc;
      __syncthreads();
      g[c] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    }
    if (t < 3) {
      const float* R = dv.R[view];
      d_pose[view * 6 + t] += -(R[t * 3 + 0] * g[0] + R[t * 3 + 1] * g[1] + R[t * 3 + 2] * g[2]);
    }
  }
}

HeadTable head_table(const DecodeConst& dc) {
  HeadTable ht;
  int units = 0, rows = 0;
  ht.nx = dc.n_x;
  for (int h = 0; h < kHeads; ++h) {
    ht.off[h] = (int32_t)dc.head_off[h];
    ht.xoff[h] = (int32_t)dc.head_xoff[h];
    ht.m[h] = dc.head_m[h];
    ht.row0[h] = rows;
    rows += dc.k * dc.head_m[h];
    if (dc.head_m[h] > 0) units += kHid;
  }
  ht.row0[kHeads] = rows;
  ht.nunits = units;
  ht.nrows = rows;
  return ht;
}

DecodeViews decode_views(const ViewDev* hv, int n_views) {
  DecodeViews dv;
  for (int v = 0; v < n_views; ++v) {
    for (int c = 0; c < 3; ++c) dv.c[v][c] = hv[v].cc[c];
    for (int c = 0; c < 9; ++c) dv.R[v][c] = hv[v].R[c];
    dv.lt[v][0] = hv[v].lt[0];
    dv.lt[v][1] = hv[v].lt[1];
  }
  return dv;
}

struct WorkSizes {
  int64_t nblk_w;
  size_t part, dcpart, total;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

WorkSizes work_sizes(const DecodeConst& dc) {
  WorkSizes z;
  z.nblk_w = dec_bwd_blocks(dc.A);
  size_t o = 0;
  z.part = o; o = a256(o + (size_t)z.nblk_w * ((dc.n_params + 63) / 64 * 64) * 4);
  z.dcpart = o; o = a256(o + (size_t)z.nblk_w * dc.n_views * 3 * 4);
  z.total = o;
  return z;
}

}  // namespace

DecodeConst decode_const(const asgs_decoder& d, int n_views) {
  DecodeConst dc;
  dc.A = d.n_anchors;
  dc.k = d.k;
  dc.nf = d.n_feat;
  dc.n_views = n_views;
  dc.precision = d.precision;
  dc.l_o = d.l_o;
  dc.l_s = d.l_s;
  const int ms[kHeads] = {1, 3, 3, 4, d.n_feat};
  dc.n_x = d.in_dim > kIn ? d.in_dim - kIn : 0;
  int64_t o = 0;
  for (int h = 0; h < kHeads; ++h) {
    dc.head_off[h] = o;
    dc.head_m[h] = ms[h];
    if (ms[h] > 0) o += (int64_t)kHid * kIn + kHid + (int64_t)d.k * ms[h] * kHid + (int64_t)d.k * ms[h];
    dc.head_xoff[h] = o;
    if (ms[h] > 0) o += (int64_t)kHid * dc.n_x;
  }
  dc.n_params = o;
  return dc;
}

size_t decode_workspace_bytes(const DecodeConst& dc) { return work_sizes(dc).total; }

void launch_decode(const DecodeConst& dc, const float* xyz, const float* feat, const float* off,
                   const float* params, const ViewDev* host_views, const asgs_gaussians& out, hipStream_t s) {
  const HeadTable ht = head_table(dc);
  const DecodeViews dv = decode_views(host_views, dc.n_views);
  launch_dec_fwd(dc, ht, dv, xyz, feat, off, params, out, s);  // FP32 or BF16 by dc.precision
}

void launch_decode_backward(const DecodeConst& dc, const float* xyz, const float* feat, const float* off,
                            const float* params, const ViewDev* host_views, const asgs_gaussians& dg,
                            float* d_xyz, float* d_feat, float* d_off, float* d_params, float* d_pose,
                            void* work, hipStream_t s) {
  (void)off;
  const HeadTable ht = head_table(dc);
  const DecodeViews dv = decode_views(host_views, dc.n_views);
  const WorkSizes z = work_sizes(dc);
  char* wb = reinterpret_cast<char*>(work);
  DecWork w;
  w.part = reinterpret_cast<float*>(wb + z.part);
  w.dcpart = reinterpret_cast<float*>(wb + z.dcpart);
  w.nblk_w = (int32_t)z.nblk_w;
  for (int view = 0; view < dc.n_views; ++view)
    launch_dec_bwd(dc, ht, dv, xyz, feat, params, dg, view, w, d_xyz, d_feat, d_params != nullptr, s);
  const unsigned nrb = d_params ? (unsigned)((dc.n_params + 63) / 64) + 1 : 1u;
  const unsigned nmean = d_xyz ? (unsigned)((dc.A * 3 + 255) / 256) : 0u;
  hipLaunchKernelGGL(k_decode_reduce, dim3(nrb + nmean), dim3(256), 0, s, dc, dv, w, d_params, d_pose, (int)nrb, dg,
                     d_xyz, d_off);
}

}  // namespace asgs
