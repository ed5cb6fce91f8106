// Decoder backward, first part, on the matrix cores (VJP of UP-SLAM Eq. 8 and
// Eq. 9): per 16-anchor tile one wave recomputes the forward and forms every
// per-anchor gradient with FP32 16x16x4 MFMAs:
//   Z  = X W1^T + b1            (M = anchors, N = 160 hidden units, K = 36)
//   H  = act(Z)                 (ReLU; SoftPlus for the feature head)
//   Y  = H_h W2_h^T + b2        (per head, N = k*m output rows in tiles of 16)
//   dY = dL/d(decoded) * act'(Y)
//   dH = dY W2_h                (K = the head's output rows)
//   dZ = dH * act'(Z)           (from H: H > 0, or 1 - exp(-H))
//   dX = dZ W1                  (K = 160, N = 35)
// then the anchor feature and view-direction gradients and the camera-centre
// partial sums. X, H, dY and dZ are also written for the weight gradients.
// Values are FP32 throughout (products exact in FP32 MFMA, sums in FP32).
//
// Persistent workgroups (one per CU) stage both layers' weights and biases
// in LDS once and loop over groups of 64 anchors (four waves x 16).
//
// Operand layouts of v_mfma_f32_16x16x4f32 (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D rows 4 (l / 16) + r,
// column l % 16, r = 0..3. Row-major transposes between a D tile and the next
// product's A operand go through a per-wave LDS tile.
#include <math.h>

#include "decode_shared.h"

namespace asgs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kHS = 161;  // padded LDS row of the 160 hidden values
constexpr int kXS = 37;   // padded LDS row of the 36 inputs
constexpr int kW1S = 37;  // padded LDS row of a first-layer weight row (35 + zero pad)
constexpr int kW2S = 36;  // padded LDS row of a second-layer weight row (32)
constexpr int kMaxWG = 256;

ASGS_DEV f4v mfma(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

ASGS_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(64 * kWaves) k_dec_bwd_tile(DecodeConst dc, HeadTable ht, DecodeViews dv,
                                                             const float* __restrict__ xyz,
                                                             const float* __restrict__ feat,
                                                             const float* __restrict__ params, asgs_gaussians dg,
                                                             int view, DecWork w, float* d_xyz, float* d_feat) {
  __shared__ float W1s[160 * kW1S];
  __shared__ float W2s[kMaxRows * kW2S];
  __shared__ float b1s[160];
  __shared__ float b2s[kMaxRows];
  __shared__ float sX[kWaves][16][kXS];
  __shared__ float sH[kWaves][16][kHS];   // H, then dZ head by head
  __shared__ float sT[kWaves][16][17];    // one 16x16 dY tile
  __shared__ float sG[kWaves][16][4];     // view-direction gradients
  __shared__ float red[kWaves][3];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index, uniform across the wave
  const int fl = lane & 15, fg = lane >> 4;
  const int A = (int)dc.A;
  const int k = dc.k;
  const int n = A * k;
  const int nunits = ht.nunits;
  // ---- stage the weights (batches of independent loads per thread) ----
  constexpr int kNT = 64 * kWaves;
  constexpr int kB = 8;
  for (int e0 = t; e0 < nunits * kW1S; e0 += kB * kNT) {
    float v[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int e = e0 + q * kNT;
      const int u = e / kW1S, c = e - u * kW1S;
      v[q] = (e < nunits * kW1S && c < kIn) ? params[ht.off[u >> 5] + (u & 31) * kIn + c] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kB; ++q)
      if (e0 + q * kNT < nunits * kW1S) W1s[e0 + q * kNT] = v[q];
  }
  for (int u = t; u < nunits; u += kNT) b1s[u] = params[ht.off[u >> 5] + kHid * kIn + (u & 31)];
  for (int h = 0; h < kHeads; ++h) {
    if (ht.m[h] == 0) continue;
    const int rows = k * ht.m[h];
    const float* W2 = params + ht.off[h] + kHid * kIn + kHid;
    for (int e0 = t; e0 < rows * kHid; e0 += kB * kNT) {
      float v[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int e = e0 + q * kNT;
        v[q] = e < rows * kHid ? W2[e] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int e = e0 + q * kNT;
        if (e < rows * kHid) W2s[(ht.row0[h] + (e >> 5)) * kW2S + (e & 31)] = v[q];
      }
    }
    for (int r = t; r < rows; r += kNT) b2s[ht.row0[h] + r] = W2[rows * kHid + r];
  }
  __syncthreads();
  float (*X)[kXS] = sX[wv];
  float (*Hs)[kHS] = sH[wv];
  float (*Ts)[17] = sT[wv];
  const int ngrp = (A + kBwdTileAnchors - 1) / kBwdTileAnchors;
  for (int grp = blockIdx.x; grp < ngrp; grp += gridDim.x) {
  const int a0 = grp * kBwdTileAnchors + wv * 16;
  // ---- inputs: 32 features and the unit view direction of 16 anchors ----
  {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = lane + 64 * q;
      const int a = e >> 5, c = e & 31;
      v[q] = a0 + a < A ? feat[(size_t)(a0 + a) * 32 + c] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = lane + 64 * q;
      X[e >> 5][e & 31] = v[q];
    }
  }
  float dist = 1.f, del[3] = {0.f, 0.f, 0.f};
  if (lane < 16) {
    if (a0 + lane < A) {
      float D[3];
      for (int c = 0; c < 3; ++c) D[c] = xyz[(size_t)c * A + a0 + lane] - dv.c[view][c];
      dist = sqrtf(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
      for (int c = 0; c < 3; ++c) del[c] = D[c] / dist;
    }
    for (int c = 0; c < 3; ++c) X[lane][32 + c] = del[c];
    X[lane][35] = 0.f;
  }
  wave_sync();
  for (int e = lane; e < 16 * 36; e += 64) {
    const int a = e / 36, c = e - a * 36;
    if (a0 + a < A) w.X[(size_t)(a0 + a) * 36 + c] = X[a][c];
  }
  // ---- Z = X W1^T: ten 16-unit column tiles, K = 36 ----
  f4v z[10];
#pragma unroll
  for (int nt = 0; nt < 10; ++nt) z[nt] = f4v{0.f, 0.f, 0.f, 0.f};
  const int ntiles = nunits / 16;
  for (int ks = 0; ks < 9; ++ks) {
    const int kk = 4 * ks + fg;
    const float av = X[fl][kk];
#pragma unroll
    for (int nt = 0; nt < 10; ++nt) {
      if (nt < ntiles) {
        const int u = 16 * nt + fl;
        z[nt] = mfma(av, W1s[u * kW1S + kk], z[nt]);
      }
    }
  }
#pragma unroll
  for (int nt = 0; nt < 10; ++nt) {
    if (nt < ntiles) {
      const int u = 16 * nt + fl;
      const int h = u >> 5;
      const float b1 = b1s[u];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 4 * fg + r;
        const float zz = z[nt][r] + b1;
        const float hv = h == 4 ? softplus(zz) : fmaxf(zz, 0.f);
        Hs[a][u] = hv;
        if (a0 + a < A) w.H[(size_t)(a0 + a) * 160 + u] = hv;
      }
    }
  }
  wave_sync();
  // ---- per head: Y, dY, dH, dZ ----
  for (int h = 0; h < kHeads; ++h) {
    const int m = ht.m[h];
    if (m == 0) continue;
    const int rows = k * m;
    const float* W2 = &W2s[ht.row0[h] * kW2S];
    const float* b2 = &b2s[ht.row0[h]];
    const float* plane0 = out_plane(dg, view, h, 0, n);
    f4v dh0 = {0.f, 0.f, 0.f, 0.f}, dh1 = dh0;
    // upstream gradients of the decoded values, fetched one row tile ahead
    auto fetch_g = [&](int rr0, float* g) {
      const int orr = rr0 + fl;
      const int ii = orr / m, cc = orr - ii * m;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 4 * fg + r;
        g[r] = (orr < rows && a0 + a < A) ? plane0[(size_t)cc * n + (size_t)(a0 + a) * k + ii] : 0.f;
      }
    };
    float gcur[4], gnxt[4];
    fetch_g(0, gcur);
    for (int r0 = 0; r0 < rows; r0 += 16) {
      if (r0 + 16 < rows) fetch_g(r0 + 16, gnxt);
      // Y tile: 16 anchors x output rows r0..r0+15
      f4v y = {0.f, 0.f, 0.f, 0.f};
      const int orow = r0 + fl;
      const bool rok = orow < rows;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const int kk = 4 * ks + fg;
        const float av = Hs[fl][32 * h + kk];
        const float bv = rok ? W2[orow * kW2S + kk] : 0.f;
        y = mfma(av, bv, y);
      }
      const float bias = rok ? b2[orow] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 4 * fg + r;
        float gy = 0.f;
        if (rok && a0 + a < A) {
          gy = gcur[r] * act_grad(h, y[r] + bias, dc.l_s);
          w.dY[(size_t)(a0 + a) * w.RP + ht.row0[h] + orow] = gy;
        }
        Ts[a][fl] = gy;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) gcur[r] = gnxt[r];
      wave_sync();
      // dH += dY_tile W2_tile (K = the 16 rows of the tile)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kr = r0 + 4 * ks + fg;
        const float av = Ts[fl][4 * ks + fg];
        const bool kok = kr < rows;
        const float b0 = kok ? W2[kr * kW2S + fl] : 0.f;
        const float b1 = kok ? W2[kr * kW2S + 16 + fl] : 0.f;
        dh0 = mfma(av, b0, dh0);
        dh1 = mfma(av, b1, dh1);
      }
      wave_sync();
    }
    // dZ of this head (overwrites its H columns, read here for act')
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int u = 32 * h + 16 * half + fl;
      const f4v dh = half ? dh1 : dh0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 4 * fg + r;
        const float hv = Hs[a][u];
        const float dz = h == 4 ? dh[r] * (1.f - expf(-hv)) : (hv > 0.f ? dh[r] : 0.f);
        Hs[a][u] = dz;
        if (a0 + a < A) w.dZ[(size_t)(a0 + a) * 160 + u] = dz;
      }
    }
  }
  wave_sync();
  // ---- dX = dZ W1: three 16-wide column tiles (35 inputs), K = hidden units ----
  f4v dx[3];
#pragma unroll
  for (int ct = 0; ct < 3; ++ct) dx[ct] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < nunits / 4; ++ks) {
    const int u = 4 * ks + fg;
    const float av = Hs[fl][u];
    const float* W1r = &W1s[u * kW1S];
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) {
      const int c = 16 * ct + fl;
      dx[ct] = mfma(av, c < kW1S ? W1r[c] : 0.f, dx[ct]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = 4 * fg + r;
    if (d_feat && a0 + a < A) {
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        float* p = &d_feat[(size_t)(a0 + a) * 32 + 16 * ct + fl];
        *p = (view == 0 ? 0.f : *p) + dx[ct][r];
      }
    }
    if (fl < 3) sG[wv][a][fl] = dx[2][r];
  }
  wave_sync();
  // ---- view direction -> anchor position and camera centre ----
  float dcl[3] = {0.f, 0.f, 0.f};
  if (lane < 16 && a0 + lane < A) {
    const float* gd = sG[wv][lane];
    const float pr = del[0] * gd[0] + del[1] * gd[1] + del[2] * gd[2];
    for (int c = 0; c < 3; ++c) {
      const float dD = (gd[c] - del[c] * pr) / dist;
      if (d_xyz) {
        float* p = &d_xyz[(size_t)c * A + a0 + lane];
        *p = (view == 0 ? 0.f : *p) + dD;
      }
      dcl[c] = -dD;
    }
  }
  for (int c = 0; c < 3; ++c) {
    float x = dcl[c];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) red[wv][c] = x;
  }
  __syncthreads();
  if (t < 3) {
    w.dcpart[((int64_t)grp * dc.n_views + view) * 3 + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
  }
  __syncthreads();  // red is reused by the next group
  }
}

}  // namespace

void launch_dec_bwd_tile(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                         const float* feat, const float* params, const asgs_gaussians& dg, int view,
                         const DecWork& w, float* d_xyz, float* d_feat, hipStream_t s) {
  const int64_t ngrp = (dc.A + kBwdTileAnchors - 1) / kBwdTileAnchors;
  const unsigned grid = (unsigned)(ngrp < kMaxWG ? ngrp : kMaxWG);
  hipLaunchKernelGGL(k_dec_bwd_tile, dim3(grid), dim3(64 * kWaves), 0, s, dc, ht, dv, xyz, feat, params, dg, view,
                     w, d_xyz, d_feat);
}

}  // namespace asgs
