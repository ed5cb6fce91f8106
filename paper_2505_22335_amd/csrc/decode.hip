// Anchor -> neural Gaussian decoding and its backward (UP-SLAM Sec. 3.3,
// Eq. 8 and Eq. 9; head MLP details in the appendix).
//
// Per anchor v and view with camera centre c: X = [f_v (32), delta (3)],
// delta = (x_v - c)/|x_v - c|. Five heads (opacity, rgb, scale, rot, feat),
// each Y_h = W2_h act_h(W1_h X + b1_h) + b2_h with a 32-wide hidden layer
// (ReLU for the first four, SoftPlus for the feature head), then the output
// activations: sigmoid (opacity, rgb), l_s * sigmoid (scale), raw (rot, feat).
//
// FP32 path: a workgroup decodes 32 anchors of one view. The first layer of
// all heads (160 hidden units) runs with one hidden unit per thread and its
// weight row in registers, broadcasting anchor inputs from LDS; the second
// layer runs with one output row per thread over the 32 hidden activations
// held in LDS. The backward recomputes the forward per anchor batch, keeps
// per-thread weight-gradient accumulators across the batches of a
// workgroup, writes one partial per workgroup and reduces the partials in a
// fixed order (deterministic, no atomics).
#include <math.h>

#include "internal.h"

namespace asgs {

namespace {

constexpr int kDecThreads = 320;
constexpr int kFwdAnchors = 32;     // anchors per forward workgroup
constexpr int kBwdAnchors = 16;     // anchors per backward batch
constexpr int kDecBatches = 8;      // batches per workgroup in the backward
constexpr int kIn = 35;
constexpr int kHid = 32;
constexpr int kHeads = 5;
constexpr int kMaxRows = ASGS_MAX_K * 27;  // second-layer rows (k * (1+3+3+4+16))

struct DecodeViews {
  float c[ASGS_MAX_VIEWS][3];
  float R[ASGS_MAX_VIEWS][9];
};

struct HeadTable {
  int32_t off[kHeads];      // packed offset of W1 of head h
  int32_t m[kHeads];        // values per Gaussian (0 = absent)
  int32_t row0[kHeads + 1]; // first second-layer row of head h (prefix over k*m)
  int32_t nunits;           // 32 * number of present heads
  int32_t nrows;
};

ASGS_DEV float sigm(float y) { return 1.f / (1.f + expf(-y)); }
ASGS_DEV float softplus(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// Which head a hidden unit j / output row o belongs to (heads present are a
// prefix of the fixed order since only the feature head is optional).
ASGS_DEV int row_head(const HeadTable& ht, int o) {
  int h = 0;
  while (h + 1 < kHeads && o >= ht.row0[h + 1]) ++h;
  return h;
}

// Output plane pointer and element for head h, Gaussian n, component comp.
ASGS_DEV float* out_plane(const asgs_gaussians& g, int view, int h, int comp, int64_t n) {
  switch (h) {
    case 0: return g.opacity + view * g.view_stride[3];
    case 1: return g.rgb + view * g.view_stride[4] + comp * n;
    case 2: return g.scale + view * g.view_stride[1] + comp * n;
    case 3: return g.rot + view * g.view_stride[2] + comp * n;
    default: return g.feat + view * g.view_stride[5] + comp * n;
  }
}

ASGS_DEV float out_act(int h, float y, float l_s) {
  switch (h) {
    case 0:
    case 1: return sigm(y);
    case 2: return l_s * sigm(y);
    default: return y;
  }
}

// Load the 32 features and the view direction of anchors a0.. into X.
template <int kDecAnchors>
ASGS_DEV void load_inputs(const float* xyz, const float* feat, int64_t A, int64_t a0, const float cc[3],
                          float (*X)[kIn + 1], float* dist) {
  const int t = threadIdx.x;
  for (int e = t; e < kDecAnchors * 32; e += blockDim.x) {
    const int a = e / 32, c = e % 32;
    X[a][c] = (a0 + a < A) ? feat[(a0 + a) * 32 + c] : 0.f;
  }
  if (t < kDecAnchors) {
    const int64_t a = a0 + t;
    float D[3] = {0.f, 0.f, 1.f};
    if (a < A)
      for (int c = 0; c < 3; ++c) D[c] = xyz[c * A + a] - cc[c];
    const float d = sqrtf(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    for (int c = 0; c < 3; ++c) X[t][32 + c] = D[c] / d;
    X[t][35] = 0.f;
    dist[t] = d;
  }
}

// First layer: Z[a][j] = b1 + W1[j] . X[a] for hidden unit j of this thread,
// anchors of half `half`. Stores act(Z) into H (and Z itself if Zs given).
template <int kDecAnchors>
ASGS_DEV void layer1(const float* params, const HeadTable& ht, float (*X)[kIn + 1],
                     float (*H)[kHid + 1], float (*Zs)[kHid + 1]) {
  const int t = threadIdx.x;
  const int j = t % 160, half = t / 160;
  if (j >= ht.nunits || half > 1) return;
  const int h = j / kHid, jj = j % kHid;
  const float* W1 = params + ht.off[h] + jj * kIn;
  float w[kIn];
#pragma unroll
  for (int c = 0; c < kIn; ++c) w[c] = W1[c];
  const float b = params[ht.off[h] + kHid * kIn + jj];
  for (int a = half * (kDecAnchors / 2); a < (half + 1) * (kDecAnchors / 2); ++a) {
    float z = b;
#pragma unroll
    for (int c = 0; c < kIn; ++c) z = fmaf(w[c], X[a][c], z);
    H[a * kHeads + h][jj] = (h == 4) ? softplus(z) : fmaxf(z, 0.f);
    if (Zs) Zs[a * kHeads + h][jj] = z;
  }
}

__global__ void __launch_bounds__(kDecThreads) k_decode_fwd(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                            const float* __restrict__ xyz,
                                                            const float* __restrict__ feat,
                                                            const float* __restrict__ off,
                                                            const float* __restrict__ params,
                                                            asgs_gaussians out) {
  constexpr int kDecAnchors = kFwdAnchors;
  __shared__ float X[kDecAnchors][kIn + 1];
  __shared__ float H[kDecAnchors * kHeads][kHid + 1];
  __shared__ float dist[kDecAnchors];
  const int view = blockIdx.y;
  const int64_t a0 = (int64_t)blockIdx.x * kDecAnchors;
  const int64_t A = dc.A;
  const int k = dc.k;
  const int64_t n = A * k;
  load_inputs<kDecAnchors>(xyz, feat, A, a0, dv.c[view], X, dist);
  __syncthreads();
  layer1<kDecAnchors>(params, ht, X, H, nullptr);
  __syncthreads();
  const int t = threadIdx.x;
  for (int o = t; o < ht.nrows; o += kDecThreads) {
    const int h = row_head(ht, o);
    const int oh = o - ht.row0[h];
    const int m = ht.m[h];
    const int i = oh / m, comp = oh - i * m;
    const float* W2 = params + ht.off[h] + kHid * kIn + kHid + oh * kHid;
    const float b2 = params[ht.off[h] + kHid * kIn + kHid + k * m * kHid + oh];
    float w[kHid];
#pragma unroll
    for (int c = 0; c < kHid; ++c) w[c] = W2[c];
    float* plane = out_plane(out, view, h, comp, n);
    for (int a = 0; a < kDecAnchors; ++a) {
      if (a0 + a >= A) break;
      float y = b2;
#pragma unroll
      for (int c = 0; c < kHid; ++c) y = fmaf(w[c], H[a * kHeads + h][c], y);
      plane[(a0 + a) * k + i] = out_act(h, y, dc.l_s);
    }
  }
  if (view == 0) {
    for (int e = t; e < kDecAnchors * k * 3; e += kDecThreads) {
      const int c = e / (kDecAnchors * k);
      const int r = e - c * kDecAnchors * k;
      const int64_t gn = a0 * k + r;
      if (gn >= n) continue;
      const int64_t a = gn / k;
      out.mean[c * n + gn] = xyz[c * A + a] + dc.l_o * off[c * n + gn];
    }
  }
}

// Gradient of the decoded value of head h w.r.t. its pre-activation y.
ASGS_DEV float act_grad(int h, float y, float l_s) {
  switch (h) {
    case 0:
    case 1: { const float s = sigm(y); return s * (1.f - s); }
    case 2: { const float s = sigm(y); return l_s * s * (1.f - s); }
    default: return 1.f;
  }
}

__global__ void __launch_bounds__(kDecThreads) k_decode_bwd(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                            const float* __restrict__ xyz,
                                                            const float* __restrict__ feat,
                                                            const float* __restrict__ off,
                                                            const float* __restrict__ params,
                                                            asgs_gaussians dg, float* d_xyz, float* d_feat,
                                                            float* d_off, float* part, float* dcpart) {
  constexpr int kDecAnchors = kBwdAnchors;
  __shared__ float X[kDecAnchors][kIn + 1];
  __shared__ float H[kDecAnchors * kHeads][kHid + 1];
  __shared__ float Zs[kDecAnchors * kHeads][kHid + 1];
  __shared__ float dZ[kDecAnchors * kHeads][kHid + 1];
  __shared__ float dY[kDecAnchors][kMaxRows + 1];
  __shared__ float dist[kDecAnchors];
  __shared__ float dXs[kDecAnchors][kIn + 1];
  __shared__ float dcs[3][kDecThreads / 64];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int64_t A = dc.A;
  const int k = dc.k;
  const int64_t n = A * k;
  const int nrows = ht.nrows;
  // per-thread weight-gradient accumulators: second-layer rows o0 = t, o1 = t + 320
  float gW2a[kHid], gW2b[kHid], gb2a = 0.f, gb2b = 0.f;
#pragma unroll
  for (int c = 0; c < kHid; ++c) { gW2a[c] = 0.f; gW2b[c] = 0.f; }
  // first-layer unit j = t % 160 over the anchors of half t / 160
  float gW1[kIn], gb1 = 0.f;
#pragma unroll
  for (int c = 0; c < kIn; ++c) gW1[c] = 0.f;
  const int j = t % 160, half = t / 160;
  const bool has_unit = j < ht.nunits && half < 2;
  const int uh = j / kHid, ujj = j % kHid;

  for (int bt = 0; bt < kDecBatches; ++bt) {
    const int64_t a0 = ((int64_t)blockIdx.x * kDecBatches + bt) * kDecAnchors;
    if (a0 >= A) break;
    for (int view = 0; view < dc.n_views; ++view) {
      __syncthreads();
      load_inputs<kDecAnchors>(xyz, feat, A, a0, dv.c[view], X, dist);
      __syncthreads();
      layer1<kDecAnchors>(params, ht, X, H, Zs);
      __syncthreads();
      // second layer: recompute y, form dL/dy, accumulate dW2, db2
      for (int r = 0; r < 2; ++r) {
        const int o = t + r * kDecThreads;
        if (o >= nrows) break;
        const int h = row_head(ht, o);
        const int oh = o - ht.row0[h];
        const int m = ht.m[h];
        const int i = oh / m, comp = oh - i * m;
        const float* W2 = params + ht.off[h] + kHid * kIn + kHid + oh * kHid;
        const float b2 = params[ht.off[h] + kHid * kIn + kHid + k * m * kHid + oh];
        const float* plane = out_plane(dg, view, h, comp, n);
        for (int a = 0; a < kDecAnchors; ++a) {
          float g = 0.f;
          if (a0 + a < A) {
            float y = b2;
#pragma unroll
            for (int c = 0; c < kHid; ++c) y = fmaf(W2[c], H[a * kHeads + h][c], y);
            g = plane[(a0 + a) * k + i] * act_grad(h, y, dc.l_s);
          }
          dY[a][o] = g;
          if (r == 0) {
            gb2a += g;
#pragma unroll
            for (int c = 0; c < kHid; ++c) gW2a[c] = fmaf(g, H[a * kHeads + h][c], gW2a[c]);
          } else {
            gb2b += g;
#pragma unroll
            for (int c = 0; c < kHid; ++c) gW2b[c] = fmaf(g, H[a * kHeads + h][c], gW2b[c]);
          }
        }
      }
      __syncthreads();
      // dH = W2^T dY, dZ = dH * act'(Z); accumulate dW1, db1
      if (has_unit) {
        const int m = ht.m[uh];
        const int rows = k * m;
        const float* W2c = params + ht.off[uh] + kHid * kIn + kHid + ujj;  // column ujj, stride 32
        for (int a = half * (kDecAnchors / 2); a < (half + 1) * (kDecAnchors / 2); ++a) {
          float dh = 0.f;
          const int r0 = ht.row0[uh];
          for (int oh = 0; oh < rows; ++oh) dh = fmaf(W2c[oh * kHid], dY[a][r0 + oh], dh);
          const float z = Zs[a * kHeads + uh][ujj];
          const float dz = (uh == 4) ? dh * sigm(z) : (z > 0.f ? dh : 0.f);
          dZ[a * kHeads + uh][ujj] = dz;
          if (a0 + a < A) {
            gb1 += dz;
#pragma unroll
            for (int c = 0; c < kIn; ++c) gW1[c] = fmaf(dz, X[a][c], gW1[c]);
          }
        }
      }
      __syncthreads();
      // dX = W1^T dZ over the present heads
      for (int e = t; e < kDecAnchors * kIn; e += kDecThreads) {
        const int a = e / kIn, c = e - a * kIn;
        float s = 0.f;
        for (int h = 0; h < kHeads; ++h) {
          if (ht.m[h] == 0) continue;
          const float* W1 = params + ht.off[h] + c;
          for (int jj = 0; jj < kHid; ++jj) s = fmaf(W1[jj * kIn], dZ[a * kHeads + h][jj], s);
        }
        dXs[a][c] = s;
      }
      __syncthreads();
      // anchor feature / position gradients and the camera-centre term
      float dcl[3] = {0.f, 0.f, 0.f};
      for (int e = t; e < kDecAnchors * 32; e += kDecThreads) {
        const int a = e / 32, c = e % 32;
        if (a0 + a < A) {
          float* p = &d_feat[(a0 + a) * 32 + c];
          *p = (view == 0 ? 0.f : *p) + dXs[a][c];
        }
      }
      if (t < kDecAnchors && a0 + t < A) {
        const int a = t;
        const float d = dist[a];
        const float* del = &X[a][32];
        const float* gd = &dXs[a][32];
        const float pr = del[0] * gd[0] + del[1] * gd[1] + del[2] * gd[2];
        for (int c = 0; c < 3; ++c) {
          const float dD = (gd[c] - del[c] * pr) / d;
          float* p = &d_xyz[c * A + a0 + a];
          *p = (view == 0 ? 0.f : *p) + dD;
          dcl[c] = -dD;
        }
      }
      for (int c = 0; c < 3; ++c) {
        float x = dcl[c];
        for (int o2 = 32; o2 > 0; o2 >>= 1) x += __shfl_xor(x, o2);
        if (lane == 0) dcs[c][wv] = x;
      }
      __syncthreads();
      if (t < 3) {
        float s = 0.f;
        for (int w = 0; w < kDecThreads / 64; ++w) s += dcs[t][w];
        float* p = &dcpart[((int64_t)blockIdx.x * dc.n_views + view) * 3 + t];
        *p = (bt == 0 ? 0.f : *p) + s;
      }
    }
    // mean gradients (summed over views): d_off = l_o dmu, d_xyz += sum_i dmu
    __syncthreads();
    for (int e = t; e < kDecAnchors * 3; e += kDecThreads) {
      const int a = e / 3, c = e % 3;
      if (a0 + a >= A) continue;
      float sx = 0.f;
      for (int i = 0; i < k; ++i) {
        const int64_t gn = (a0 + a) * k + i;
        float s = 0.f;
        for (int view = 0; view < dc.n_views; ++view) s += dg.mean[view * dg.view_stride[0] + c * n + gn];
        d_off[c * n + gn] = dc.l_o * s;
        sx += s;
      }
      d_xyz[c * A + a0 + a] += sx;
    }
  }
  // workgroup partials of the weight gradients, packed like the parameters
  float* P = part + (int64_t)blockIdx.x * dc.n_params;
  for (int r = 0; r < 2; ++r) {
    const int o = t + r * kDecThreads;
    if (o >= nrows) break;
    const int h = row_head(ht, o);
    const int oh = o - ht.row0[h];
    const int m = ht.m[h];
    float* W2p = P + ht.off[h] + kHid * kIn + kHid + oh * kHid;
#pragma unroll
    for (int c = 0; c < kHid; ++c) W2p[c] = r == 0 ? gW2a[c] : gW2b[c];
    P[ht.off[h] + kHid * kIn + kHid + k * m * kHid + oh] = r == 0 ? gb2a : gb2b;
  }
  // two threads share each first-layer unit: combine through LDS
  __syncthreads();
  static_assert(kBwdAnchors * (kMaxRows + 1) >= 160 * (kIn + 1), "dY too small for reuse");
  float* comb = &dY[0][0];  // reuse: 160 x 36 floats
  if (has_unit && half == 1) {
#pragma unroll
    for (int c = 0; c < kIn; ++c) comb[j * (kIn + 1) + c] = gW1[c];
    comb[j * (kIn + 1) + kIn] = gb1;
  }
  __syncthreads();
  if (has_unit && half == 0) {
    float* W1p = P + ht.off[uh] + ujj * kIn;
#pragma unroll
    for (int c = 0; c < kIn; ++c) W1p[c] = gW1[c] + comb[j * (kIn + 1) + c];
    P[ht.off[uh] + kHid * kIn + ujj] = gb1 + comb[j * (kIn + 1) + kIn];
  }
}

// Fixed-order reduction of the workgroup partials; adds -R_cw dL/dc to the
// translation part of the pose gradient.
__global__ void k_decode_reduce(DecodeConst dc, DecodeViews dv, const float* part, const float* dcpart,
                                int nblk, float* d_params, float* d_pose) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < dc.n_params) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * dc.n_params + p];
    d_params[p] = s;
  } else if (d_pose && p < dc.n_params + dc.n_views * 3) {
    const int e = (int)(p - dc.n_params);
    const int view = e / 3, r = e % 3;
    float g[3] = {0.f, 0.f, 0.f};
    for (int b = 0; b < nblk; ++b)
      for (int c = 0; c < 3; ++c) g[c] += dcpart[((int64_t)b * dc.n_views + view) * 3 + c];
    const float* R = dv.R[view];
    d_pose[view * 6 + r] += -(R[r * 3 + 0] * g[0] + R[r * 3 + 1] * g[1] + R[r * 3 + 2] * g[2]);
  }
}

HeadTable head_table(const DecodeConst& dc) {
  HeadTable ht;
  int units = 0, rows = 0;
  for (int h = 0; h < kHeads; ++h) {
    ht.off[h] = (int32_t)dc.head_off[h];
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
  }
  return dv;
}

int64_t bwd_blocks(const DecodeConst& dc) {
  const int64_t per = (int64_t)kBwdAnchors * kDecBatches;
  return (dc.A + per - 1) / per;
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
  int64_t o = 0;
  for (int h = 0; h < kHeads; ++h) {
    dc.head_off[h] = o;
    dc.head_m[h] = ms[h];
    if (ms[h] > 0) o += (int64_t)kHid * kIn + kHid + (int64_t)d.k * ms[h] * kHid + (int64_t)d.k * ms[h];
  }
  dc.n_params = o;
  return dc;
}

size_t decode_workspace_bytes(const DecodeConst& dc) {
  const int64_t nb = bwd_blocks(dc);
  return (size_t)(nb * dc.n_params + nb * dc.n_views * 3) * sizeof(float) + 256;
}

void launch_decode(const DecodeConst& dc, const float* xyz, const float* feat, const float* off,
                   const float* params, const ViewDev* host_views, const asgs_gaussians& out, hipStream_t s) {
  const HeadTable ht = head_table(dc);
  const DecodeViews dv = decode_views(host_views, dc.n_views);
  dim3 grid((unsigned)((dc.A + kFwdAnchors - 1) / kFwdAnchors), (unsigned)dc.n_views);
  hipLaunchKernelGGL(k_decode_fwd, grid, dim3(kDecThreads), 0, s, dc, ht, dv, xyz, feat, off, params, out);
}

void launch_decode_backward(const DecodeConst& dc, const float* xyz, const float* feat, const float* off,
                            const float* params, const ViewDev* host_views, const asgs_gaussians& dg,
                            float* d_xyz, float* d_feat, float* d_off, float* d_params, float* d_pose,
                            void* work, hipStream_t s) {
  const HeadTable ht = head_table(dc);
  const DecodeViews dv = decode_views(host_views, dc.n_views);
  const int64_t nb = bwd_blocks(dc);
  float* part = reinterpret_cast<float*>(work);
  float* dcpart = part + nb * dc.n_params;
  hipLaunchKernelGGL(k_decode_bwd, dim3((unsigned)nb), dim3(kDecThreads), 0, s, dc, ht, dv, xyz, feat, off,
                     params, dg, d_xyz, d_feat, d_off, part, dcpart);
  const int64_t tot = dc.n_params + dc.n_views * 3;
  hipLaunchKernelGGL(k_decode_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dc, dv, part,
                     dcpart, (int)nb, d_params, d_pose);
}

}  // namespace asgs
