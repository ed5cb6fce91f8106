// Uncertainty MLP F_u of the mapping thread, its loss L_u and the motion mask
// (UP-SLAM Sec. 3.2 Eq. 5, Sec. 3.3 Eq. 13).
//
// Per pixel p of a view, with F_p the DINO feature bilinearly upsampled from
// the patch grid:
//   z_p = W1 F_p + b1 (128),  sigma_p = sigma_min + softplus(w2 . relu(z_p) + b2)
//   M_p = [2 sigma_p^2 > 1],  L_u = mean_p R_p / (2 sigma_p^2) + lam3 log sigma_p
// with R held constant (the gradient reaches F_u's parameters only).
//
// The first layer is linear and bilinear weights sum to one, so z_p is the
// bilinear interpolation of the per-patch Z_c = W1 F_c + b1: the N_h-wide
// contraction runs once per patch (k_fu_grid), and each pixel interpolates
// 128 values (k_fu_pix). The backward uses the same identity in reverse:
//   dZ_c = sum_p w_pc dy_p w2 o [z_p > 0]   (w_pc the bilinear weight)
//   dW1 = sum_c dZ_c F_c^T,  db1 = sum_c dZ_c,
//   dw2 = sum_p dy_p relu(z_p),  db2 = sum_p dy_p
// with dy_p = dL_u/dsigma_p * sigmoid(y_p). k_fu_pix handles one 16 x 16
// pixel tile per workgroup: a first phase, one pixel per thread, forms y_p,
// sigma, the mask and dy_p; a second phase, one hidden unit (and half of the
// pixels) per thread, recomputes z_p[u] and accumulates the tile's dZ for the
// (at most 4 x 4) patches the tile reaches and its dw2 partial. Patch and
// parameter sums follow in fixed order (deterministic, no atomics).
#include <math.h>

#include "internal.h"

namespace asgs {

namespace {

constexpr int kHid = 128;     // hidden units of F_u
constexpr int kT = 16;        // pixel tile side
constexpr int kSlots = 16;    // patches one tile reaches (4 x 4 at most)
constexpr int kZS = kHid + 1; // LDS row of one patch's 128 values (padded)
constexpr int kGC = 16;       // patches per workgroup of the grid contraction
constexpr int kGU = 16;       // hidden units per workgroup of the grid contraction
constexpr int kKC = 64;       // input channels per staged block

struct TileCells {
  int cy0, ncy, cx0, ncx;
};

ASGS_DEV TileCells tile_cells(const UncArgs& a, int tx, int ty) {
  TileCells t;
  int i0, i1;
  float w;
  const int xa = tx * kT, xe = min(xa + kT - 1, a.W - 1);
  const int ya = ty * kT, ye = min(ya + kT - 1, a.H - 1);
  bilin(xa, a.Wp, a.sx, i0, i1, w);
  t.cx0 = i0;
  bilin(xe, a.Wp, a.sx, i0, i1, w);
  t.ncx = i1 - t.cx0 + 1;
  bilin(ya, a.Hp, a.sy, i0, i1, w);
  t.cy0 = i0;
  bilin(ye, a.Hp, a.sy, i0, i1, w);
  t.ncy = i1 - t.cy0 + 1;
  return t;
}

// Z_c = W1 F_c + b1: one workgroup per 16 patches x 16 hidden units of a
// view, one (patch, unit) per thread; weight and feature blocks of kKC input
// channels staged in LDS, the next block's loads issued before the current
// block is used.
__global__ void __launch_bounds__(256) k_fu_grid(UncArgs a) {
  __shared__ float ws[kGU][kKC + 1];
  __shared__ float fs[kKC][kGC];
  const int v = blockIdx.z;
  const int plane = a.Hp * a.Wp;
  const int c0 = blockIdx.x * kGC, u0 = blockIdx.y * kGU;
  const int t = threadIdx.x;
  const int pc = t & (kGC - 1), uu = t / kGC;
  const float* F = a.dino + (int64_t)v * a.nh * plane;
  constexpr int kPer = kGU * kKC / 256;  // staged values of each block per thread
  float wn[kPer], fn[kPer];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = t + 256 * i;
      const int r = q / kKC, c = q - r * kKC;  // weight block: unit r, channel c
      wn[i] = k0 + c < a.nh ? a.params[(int64_t)(u0 + r) * a.nh + k0 + c] : 0.f;
      const int kk = q / kGC, pp = q - kk * kGC;  // feature block: channel kk, patch pp
      fn[i] = k0 + kk < a.nh && c0 + pp < plane ? F[(int64_t)(k0 + kk) * plane + c0 + pp] : 0.f;
    }
  };
  float acc = 0.f;
  load(0);
  for (int k0 = 0; k0 < a.nh; k0 += kKC) {
    __syncthreads();  // the previous block has been read
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = t + 256 * i;
      ws[q / kKC][q % kKC] = wn[i];
      fs[q / kGC][q % kGC] = fn[i];
    }
    __syncthreads();
    if (k0 + kKC < a.nh) load(k0 + kKC);
#pragma unroll 8
    for (int k = 0; k < kKC; ++k) acc = fmaf(ws[uu][k], fs[k][pc], acc);
  }
  if (c0 + pc < plane) a.zg[((int64_t)v * plane + c0 + pc) * kHid + u0 + uu] = acc + a.params[(int64_t)kHid * a.nh + u0 + uu];
}

struct PixShared {
  float z[kSlots][kZS];       // Z of the tile's patches
  float w2[kHid];
  float cw[kT * kT][4];       // bilinear corner weights of each pixel
  int cs[kT * kT][4];         // corner slots
  float dy[kT * kT];          // dL_u/dy per pixel (0 outside the image)
  float dz[2][kSlots][kZS];   // the tile's dZ, one copy per pixel half
  float red[2][kHid];
  double lred[4];
  float bred[4];
};

__global__ void __launch_bounds__(256) k_fu_pix(UncArgs a) {
  __shared__ PixShared S;
  const int tx = blockIdx.x, ty = blockIdx.y, v = blockIdx.z;
  const int t = threadIdx.x;
  const int64_t HW = (int64_t)a.W * a.H;
  const int plane = a.Hp * a.Wp;
  const TileCells tc = tile_cells(a, tx, ty);
  const int nslots = tc.ncy * tc.ncx;
  // ---- stage the patches' Z and w2 ----
  for (int q = t; q < nslots * kHid; q += 256) {
    const int sl = q / kHid, u = q - sl * kHid;
    const int cy = tc.cy0 + sl / tc.ncx, cx = tc.cx0 + sl % tc.ncx;
    S.z[sl][u] = a.zg[((int64_t)v * plane + cy * a.Wp + cx) * kHid + u];
  }
  if (t < kHid) S.w2[t] = a.params[(int64_t)kHid * a.nh + kHid + t];
  const float b2 = a.params[(int64_t)kHid * a.nh + 2 * kHid];
  // ---- phase 1: one pixel per thread ----
  const int px = tx * kT + (t & (kT - 1)), py = ty * kT + (t >> 4);
  const bool in = px < a.W && py < a.H;
  {
    int x0, x1, y0, y1;
    float wx, wy;
    bilin(in ? px : 0, a.Wp, a.sx, x0, x1, wx);
    bilin(in ? py : 0, a.Hp, a.sy, y0, y1, wy);
    const int r0 = (y0 - tc.cy0) * tc.ncx, r1 = (y1 - tc.cy0) * tc.ncx;
    S.cs[t][0] = in ? r0 + x0 - tc.cx0 : 0;
    S.cs[t][1] = in ? r0 + x1 - tc.cx0 : 0;
    S.cs[t][2] = in ? r1 + x0 - tc.cx0 : 0;
    S.cs[t][3] = in ? r1 + x1 - tc.cx0 : 0;
    S.cw[t][0] = (1.f - wy) * (1.f - wx);
    S.cw[t][1] = (1.f - wy) * wx;
    S.cw[t][2] = wy * (1.f - wx);
    S.cw[t][3] = wy * wx;
  }
  __syncthreads();
  float y = b2;
  {
    const int s0 = S.cs[t][0], s1 = S.cs[t][1], s2 = S.cs[t][2], s3 = S.cs[t][3];
    const float w0 = S.cw[t][0], w1 = S.cw[t][1], w2 = S.cw[t][2], w3 = S.cw[t][3];
#pragma unroll 8
    for (int u = 0; u < kHid; ++u) {
      const float z = w0 * S.z[s0][u] + w1 * S.z[s1][u] + w2 * S.z[s2][u] + w3 * S.z[s3][u];
      y = fmaf(S.w2[u], fmaxf(z, 0.f), y);
    }
  }
  const float sp = fmaxf(y, 0.f) + log1pf(expf(-fabsf(y)));
  const float sig = a.sigma_min + sp;
  const int64_t q = v * HW + (int64_t)py * a.W + px;
  if (in) {
    if (a.sigma) a.sigma[q] = sig;
    if (a.dynamic) a.dynamic[q] = 2.f * sig * sig > 1.f ? 1u : 0u;
  }
  double l = 0.0;
  float dy = 0.f;
  if (a.R && in) {
    const float R = a.R[q];
    const double sd = (double)sig;
    l = (double)R / (2.0 * sd * sd) + (double)a.lam3 * log(sd);
    // dL_u/dsigma = (-R / sigma^3 + lam3 / sigma) / HW, dsigma/dy = sigmoid(y)
    const float dsig = (-R / (sig * sig * sig) + a.lam3 / sig) * a.inv_hw;
    dy = dsig / (1.f + expf(-y));
  }
  if (a.partial) {
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
    if ((t & 63) == 0) S.lred[t >> 6] = l;
  }
  if (!a.dzt) {
    if (a.partial) {
      __syncthreads();
      if (t == 0)
        a.partial[(int64_t)v * a.tiles + ty * a.tiles_x + tx] = (S.lred[0] + S.lred[1]) + (S.lred[2] + S.lred[3]);
    }
    return;
  }
  S.dy[t] = dy;
  float db = dy;
  for (int o = 32; o > 0; o >>= 1) db += __shfl_xor(db, o);
  if ((t & 63) == 0) S.bred[t >> 6] = db;
  for (int e = t; e < 2 * kSlots * kZS; e += 256) (&S.dz[0][0][0])[e] = 0.f;
  __syncthreads();
  // ---- phase 2: one hidden unit and half of the pixels per thread ----
  const int u = t & (kHid - 1), ph = t >> 7;
  const float w2u = S.w2[u];
  float aw2 = 0.f;
  for (int p = ph * 128; p < ph * 128 + 128; ++p) {
    const float d = S.dy[p];  // uniform over the wave
    if (d == 0.f) continue;
    const int s0 = S.cs[p][0], s1 = S.cs[p][1], s2 = S.cs[p][2], s3 = S.cs[p][3];
    const float w0 = S.cw[p][0], w1 = S.cw[p][1], w2 = S.cw[p][2], w3 = S.cw[p][3];
    const float z = w0 * S.z[s0][u] + w1 * S.z[s1][u] + w2 * S.z[s2][u] + w3 * S.z[s3][u];
    aw2 = fmaf(d, fmaxf(z, 0.f), aw2);
    if (z > 0.f) {
      const float g = d * w2u;
      S.dz[ph][s0][u] += g * w0;
      S.dz[ph][s1][u] += g * w1;
      S.dz[ph][s2][u] += g * w2;
      S.dz[ph][s3][u] += g * w3;
    }
  }
  S.red[ph][u] = aw2;
  __syncthreads();
  const int64_t tile = (int64_t)v * a.tiles + ty * a.tiles_x + tx;
  for (int e = t; e < nslots * kHid; e += 256) {
    const int sl = e / kHid, uu = e - sl * kHid;
    a.dzt[(tile * kSlots + sl) * kHid + uu] = S.dz[0][sl][uu] + S.dz[1][sl][uu];
  }
  if (t < kHid) a.w2t[tile * (kHid + 1) + t] = S.red[0][t] + S.red[1][t];
  if (t == 0) {
    a.w2t[tile * (kHid + 1) + kHid] = (S.bred[0] + S.bred[1]) + (S.bred[2] + S.bred[3]);
    if (a.partial) a.partial[tile] = (S.lred[0] + S.lred[1]) + (S.lred[2] + S.lred[3]);
  }
}

// Per patch: dZ summed over the tiles that reach it (fixed order).
__global__ void __launch_bounds__(kHid) k_fu_cell_reduce(UncArgs a) {
  const int cell = blockIdx.x, v = blockIdx.y, u = threadIdx.x;
  const int cy = cell / a.Wp, cx = cell - cy * a.Wp;
  // the tile rows and the tile columns that reach the patch (a tile's patch
  // rows depend on its row only, its patch columns on its column only)
  int ty0 = a.tiles_y, ty1 = -1, tx0 = a.tiles_x, tx1 = -1;
  for (int ty = 0; ty < a.tiles_y; ++ty) {
    const TileCells r = tile_cells(a, 0, ty);
    if (cy >= r.cy0 && cy < r.cy0 + r.ncy) {
      ty0 = min(ty0, ty);
      ty1 = ty;
    }
  }
  for (int tx = 0; tx < a.tiles_x; ++tx) {
    const TileCells r = tile_cells(a, tx, 0);
    if (cx >= r.cx0 && cx < r.cx0 + r.ncx) {
      tx0 = min(tx0, tx);
      tx1 = tx;
    }
  }
  float s = 0.f;
  for (int ty = ty0; ty <= ty1; ++ty) {
    for (int tx = tx0; tx <= tx1; ++tx) {
      const TileCells tc = tile_cells(a, tx, ty);
      const int64_t tile = (int64_t)v * a.tiles + ty * a.tiles_x + tx;
      s += a.dzt[(tile * kSlots + (cy - tc.cy0) * tc.ncx + (cx - tc.cx0)) * kHid + u];
    }
  }
  a.dzc[((int64_t)v * a.Hp * a.Wp + cell) * kHid + u] = s;
}

// Parameter gradients from the patch sums out = [128][nh + 1] (dW1 | db1,
// from the split-K product of dZ with the DINO grid and a row of ones) and the
// tile partials of dw2, db2: thread e < 128 nh copies dW1, the next 128 db1;
// workgroups past those sum one column of the tile partials (fixed order).
__global__ void __launch_bounds__(256) k_fu_params(UncArgs a, const float* __restrict__ out, float* d_params) {
  const int64_t n1 = (int64_t)kHid * a.nh + kHid;
  const int64_t nb1 = (n1 + 255) / 256;
  if ((int64_t)blockIdx.x < nb1) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < (int64_t)kHid * a.nh) {
      const int64_t u = e / a.nh, k = e - u * a.nh;
      d_params[e] = out[u * (a.nh + 1) + k];
    } else if (e < n1) {
      const int64_t u = e - (int64_t)kHid * a.nh;
      d_params[e] = out[u * (a.nh + 1) + a.nh];
    }
    return;
  }
  __shared__ float red[4];
  const int j = (int)(blockIdx.x - nb1);  // column of w2t: dw2[j] (j < 128) or db2 (j = 128)
  const int64_t ntiles = (int64_t)a.V * a.tiles;
  float s = 0.f;
  for (int64_t tile = threadIdx.x; tile < ntiles; tile += 256) s += a.w2t[tile * (kHid + 1) + j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) d_params[n1 + j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// L_u of each view: fixed-order sum of its tile partials, over its pixels.
__global__ void __launch_bounds__(256) k_fu_mean(const double* __restrict__ partial, int per_view, double inv_hw,
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

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }


ColGemm dw1_gemm(const UncArgs& a) {
  ColGemm g{};
  g.D = a.dzc;
  g.dstride = kHid;
  g.ncol = kHid;
  g.F = a.dino;
  g.fk = (int64_t)a.Hp * a.Wp;
  g.fr = 1;
  g.fview = (int64_t)a.nh * a.Hp * a.Wp;
  g.nk = a.nh;
  g.ones = 1;
  g.V = a.V;
  g.rows = a.Hp * a.Wp;
  g.nsplit = colgemm_splits((int64_t)a.V * a.Hp * a.Wp);
  return g;
}

}  // namespace

UncLayout uncertainty_layout(int n_views, int width, int height, int Hp, int Wp, int nh) {
  UncLayout L{};
  const int64_t tiles = (int64_t)((width + kT - 1) / kT) * ((height + kT - 1) / kT) * n_views;
  const int64_t cells = (int64_t)Hp * Wp * n_views;
  size_t o = 0;
  L.zg = o;
  o = a256(o + (size_t)cells * kHid * 4);
  L.partial = o;
  o = a256(o + (size_t)tiles * 8);
  L.dzt = o;
  o = a256(o + (size_t)tiles * kSlots * kHid * 4);
  L.w2t = o;
  o = a256(o + (size_t)tiles * (kHid + 1) * 4);
  L.dzc = o;
  o = a256(o + (size_t)cells * kHid * 4);
  UncArgs ga{};
  ga.V = n_views;
  ga.Hp = Hp;
  ga.Wp = Wp;
  ga.nh = nh;
  L.gpart = o;
  o = a256(o + colgemm_part_floats(dw1_gemm(ga)) * 4);
  L.gout = o;
  o = a256(o + (size_t)kHid * (nh + 1) * 4);
  L.total = o;
  return L;
}

void launch_uncertainty(UncArgs a, const UncLayout& L, char* work, float* loss, float* d_params, hipStream_t s) {
  a.zg = reinterpret_cast<float*>(work + L.zg);
  a.partial = (loss || d_params) && a.R ? reinterpret_cast<double*>(work + L.partial) : nullptr;
  a.dzt = d_params ? reinterpret_cast<float*>(work + L.dzt) : nullptr;
  a.w2t = reinterpret_cast<float*>(work + L.w2t);
  a.dzc = reinterpret_cast<float*>(work + L.dzc);
  a.tiles_x = (a.W + kT - 1) / kT;
  a.tiles_y = (a.H + kT - 1) / kT;
  a.tiles = a.tiles_x * a.tiles_y;
  const int plane = a.Hp * a.Wp;
  hipLaunchKernelGGL(k_fu_grid, dim3((unsigned)((plane + kGC - 1) / kGC), kHid / kGU, (unsigned)a.V), dim3(256), 0, s,
                     a);
  hipLaunchKernelGGL(k_fu_pix, dim3((unsigned)a.tiles_x, (unsigned)a.tiles_y, (unsigned)a.V), dim3(256), 0, s, a);
  if (loss && a.partial)
    hipLaunchKernelGGL(k_fu_mean, dim3((unsigned)a.V), dim3(256), 0, s, (const double*)a.partial, a.tiles,
                       1.0 / ((double)a.W * (double)a.H), loss);
  if (d_params) {
    hipLaunchKernelGGL(k_fu_cell_reduce, dim3((unsigned)plane, (unsigned)a.V), dim3(kHid), 0, s, a);
    ColGemm g = dw1_gemm(a);
    g.part = reinterpret_cast<float*>(work + L.gpart);
    float* out = reinterpret_cast<float*>(work + L.gout);
    launch_colgemm(g, out, s);
    const int64_t nb1 = ((int64_t)kHid * a.nh + kHid + 255) / 256;
    hipLaunchKernelGGL(k_fu_params, dim3((unsigned)(nb1 + kHid + 1)), dim3(256), 0, s, a, (const float*)out, d_params);
  }
}

}  // namespace asgs
