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
// pixel tile per workgroup: the interpolation z = Wbil Z over the (at most
// 4 x 4) patches the tile reaches and the tile's dZ = Wbil^T G are products
// on the matrix cores (FP32); y_p, sigma, the mask and dy_p are formed in
// between, and the tile's dw2 partial alongside. Patch and parameter sums
// follow in fixed order (deterministic, no atomics).
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

typedef float f4v __attribute__((ext_vector_type(4)));

// sum over the four lanes of one column (lanes l, l ^ 16, l ^ 32, l ^ 48)
ASGS_DEV float col_sum4(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

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

// One 16 x 16 tile per workgroup; wave w takes the pixel rows 4 w .. 4 w + 3,
// one row of 16 pixels at a time, on the matrix cores (v_mfma_f32_16x16x4f32,
// FP32 products and sums):
//   z (16 pixels x 16 units) = Wbil (16 pixels x 16 patch slots) Z_slots,
// A = the bilinear weights (K = slots, four steps of four), B = the staged
// patch values; lane (g, n) receives pixels 4 g + r of unit 16 b + n. y sums
// w2 relu(z) over the units (the lanes of a row group). With dy known,
//   dZ (16 slots x 16 units) += Wbil^T G,  G = dy w2 [z > 0],
// takes the row's pixels as K: the accumulator rows 4 g + r are directly the
// B operand of step r, A = the weight of slot n at pixel 4 g + r. The four
// waves' dZ are added in a fixed order.
struct PixShared {
  float z[kSlots][kZS];          // Z of the tile's patches (zero past the last)
  float w2[kHid];
  float dzw[4][kSlots][kHid];    // each wave's dZ
  float red[4][kHid];
  double lred[4];
  float bred[4];
};

// weight of patch slot sl at a pixel whose corners are (cs, cw)
ASGS_DEV float slot_weight(const int (&cs)[4], const float (&cw)[4], int sl) {
  float w = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) w += cs[c] == sl ? cw[c] : 0.f;
  return w;
}

// corners (cs, cw) of pixel column px in a row whose patch rows are r0, r1
// (slot offsets) with weight wy
ASGS_DEV void col_corners(const UncArgs& a, const TileCells& tc, int px, int r0, int r1, float wy, int (&cs)[4],
                          float (&cw)[4]) {
  int x0, x1;
  float wx;
  bilin(px, a.Wp, a.sx, x0, x1, wx);
  cs[0] = r0 + x0 - tc.cx0;
  cs[1] = r0 + x1 - tc.cx0;
  cs[2] = r1 + x0 - tc.cx0;
  cs[3] = r1 + x1 - tc.cx0;
  cw[0] = (1.f - wy) * (1.f - wx);
  cw[1] = (1.f - wy) * wx;
  cw[2] = wy * (1.f - wx);
  cw[3] = wy * wx;
}

template <int kCtrl>
ASGS_DEV float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), kCtrl, 0xf, 0xf, false));
}
// sum over the 16 lanes of a row (rotations by 8 and 4, then within quads);
// every lane of the row gets the same bits (each step adds the same two
// partial sums, in either order)
ASGS_DEV float row_sum16(float v) {
  v += dpp<0x128>(v);
  v += dpp<0x124>(v);
  v += dpp<0x4E>(v);
  v += dpp<0xB1>(v);
  return v;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_fu_pix(UncArgs a) {
  __shared__ PixShared S;
  const int tx = blockIdx.x, ty = blockIdx.y, v = blockIdx.z;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, g = lane >> 4, n = lane & 15;
  const int64_t HW = (int64_t)a.W * a.H;
  const int plane = a.Hp * a.Wp;
  const TileCells tc = tile_cells(a, tx, ty);
  const int nslots = tc.ncy * tc.ncx;
  // R at the lane's pixel (column 4 g + n % 4) of the wave's four rows,
  // requested first (clamped into the view; pixels outside it are masked
  // where used)
  const int rr = n & 3;
  float Rq[4];
  if (a.R) {
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
      const int px = min(tx * kT + 4 * g + rr, a.W - 1), py = min(ty * kT + 4 * wv + pb, a.H - 1);
      Rq[pb] = a.R[v * HW + (int64_t)py * a.W + px];
    }
  }
  // ---- stage the patches' Z (zero past the tile's patches) and w2 ----
  for (int q = t; q < kSlots * kHid; q += 256) {
    const int sl = q / kHid, u = q - sl * kHid;
    const int cy = tc.cy0 + sl / tc.ncx, cx = tc.cx0 + sl % tc.ncx;
    S.z[sl][u] = sl < nslots ? a.zg[((int64_t)v * plane + cy * a.Wp + cx) * kHid + u] : 0.f;
  }
  if (t < kHid) S.w2[t] = a.params[(int64_t)kHid * a.nh + kHid + t];
  const float b2 = a.params[(int64_t)kHid * a.nh + 2 * kHid];
  __syncthreads();
  // B operands of z: slot 4 s + g, unit 16 b + n
  float zb[4][8], w2n[8];
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int b = 0; b < 8; ++b) zb[st][b] = S.z[4 * st + g][16 * b + n];
#pragma unroll
  for (int b = 0; b < 8; ++b) w2n[b] = S.w2[16 * b + n];
  const bool grad = a.dzt != nullptr;
  f4v dz[8];
  float aw2[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    dz[b] = f4v{0.f, 0.f, 0.f, 0.f};
    aw2[b] = 0.f;
  }
  double lsum = 0.0;
  float dbs = 0.f;
#pragma unroll
  for (int pb = 0; pb < 4; ++pb) {
    const int py = ty * kT + 4 * wv + pb;
    int y0, y1;
    float wy;
    bilin(py < a.H ? py : 0, a.Hp, a.sy, y0, y1, wy);
    const int r0 = (y0 - tc.cy0) * tc.ncx, r1 = (y1 - tc.cy0) * tc.ncx;
    // A of z: the weights of slots 4 s + g at pixel n of the row
    f4v z[8];
    {
      int cs[4];
      float cw[4];
      const int pxa = tx * kT + n;
      col_corners(a, tc, pxa < a.W ? pxa : 0, r0, r1, wy, cs, cw);
      float wA[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) wA[st] = slot_weight(cs, cw, 4 * st + g);
#pragma unroll
      for (int b = 0; b < 8; ++b) z[b] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int b = 0; b < 8; ++b) z[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(wA[st], zb[st][b], z[b], 0, 0, 0);
    }
    // y at pixels 4 g + r: w2 . relu(z) over the units, summed over the row group's lanes
    float yr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float acc = 0.f;
#pragma unroll
      for (int b = 0; b < 8; ++b) acc = fmaf(w2n[b], fmaxf(z[b][r], 0.f), acc);
      yr[r] = b2 + row_sum16(acc);
    }
    // sigma, the mask, the loss term and dy of the lane's pixel, column
    // 4 g + n % 4 (four lanes per pixel; lanes n < 4 write)
    const float y = rr == 0 ? yr[0] : rr == 1 ? yr[1] : rr == 2 ? yr[2] : yr[3];
    const int px = tx * kT + 4 * g + rr;
    const bool in = px < a.W && py < a.H;
    const float sp = fmaxf(y, 0.f) + log1pf(expf(-fabsf(y)));
    const float sig = a.sigma_min + sp;
    float dy = 0.f;
    if (a.R && in) {
      const float R = Rq[pb];
      // dL_u/dsigma = (-R / sigma^3 + lam3 / sigma) / HW, dsigma/dy = sigmoid(y)
      const float dsig = (-R / (sig * sig * sig) + a.lam3 / sig) * a.inv_hw;
      dy = dsig / (1.f + expf(-y));
    }
    if (n < 4 && in) {
      const int64_t q = v * HW + (int64_t)py * a.W + px;
      if (a.sigma) a.sigma[q] = sig;
      if (a.dynamic) a.dynamic[q] = 2.f * sig * sig > 1.f ? 1u : 0u;
      if (a.R) {
        const double sd = (double)sig;
        lsum += (double)Rq[pb] / (2.0 * sd * sd) + (double)a.lam3 * log(sd);
      }
    }
    if (grad) {
      // dy of pixels 4 g + r in every lane of the quad
      float dyr[4];
      dyr[0] = dpp<0x00>(dy);
      dyr[1] = dpp<0x55>(dy);
      dyr[2] = dpp<0xAA>(dy);
      dyr[3] = dpp<0xFF>(dy);
      // A of dZ, step r: the weight of slot n at pixel 4 g + r
      float wB[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int cs[4];
        float cw[4];
        const int pxr = tx * kT + 4 * g + r;
        col_corners(a, tc, pxr < a.W ? pxr : 0, r0, r1, wy, cs, cw);
        wB[r] = slot_weight(cs, cw, n);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const float zz = z[b][r];
          aw2[b] = fmaf(dyr[r], fmaxf(zz, 0.f), aw2[b]);
          const float G = zz > 0.f ? dyr[r] * w2n[b] : 0.f;
          dz[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(wB[r], G, dz[b], 0, 0, 0);
        }
      if (n < 4) dbs += dy;
    }
  }
  if (a.partial) {
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
    if (lane == 0) S.lred[wv] = lsum;
  }
  if (grad) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const float s = col_sum4(aw2[b]);
      if (g == 0) S.red[wv][16 * b + n] = s;
#pragma unroll
      for (int r = 0; r < 4; ++r) S.dzw[wv][4 * g + r][16 * b + n] = dz[b][r];
    }
    for (int o = 32; o > 0; o >>= 1) dbs += __shfl_xor(dbs, o);
    if (lane == 0) S.bred[wv] = dbs;
  }
  __syncthreads();
  const int64_t tile = (int64_t)v * a.tiles + ty * a.tiles_x + tx;
  if (!grad) {
    if (a.partial && t == 0) a.partial[tile] = (S.lred[0] + S.lred[1]) + (S.lred[2] + S.lred[3]);
    return;
  }
  for (int e = t; e < nslots * kHid; e += 256) {
    const int sl = e / kHid, uu = e - sl * kHid;
    a.dzt[(tile * kSlots + sl) * kHid + uu] =
        (S.dzw[0][sl][uu] + S.dzw[1][sl][uu]) + (S.dzw[2][sl][uu] + S.dzw[3][sl][uu]);
  }
  if (t < kHid) a.w2t[tile * (kHid + 1) + t] = (S.red[0][t] + S.red[1][t]) + (S.red[2][t] + S.red[3][t]);
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
  // (the first wave: one tile row or column per lane, 64 at a time, then a
  // ballot; the bounds reach the other threads through LDS)
  __shared__ int bounds[4];
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int ty0 = a.tiles_y, ty1 = -1, tx0 = a.tiles_x, tx1 = -1;
    for (int base = 0; base < a.tiles_y; base += 64) {
      const int ty = base + lane;
      bool reach = false;
      if (ty < a.tiles_y) {
        const TileCells r = tile_cells(a, 0, ty);
        reach = cy >= r.cy0 && cy < r.cy0 + r.ncy;
      }
      const uint64_t m = __ballot(reach);
      if (m) {
        ty0 = min(ty0, base + __builtin_ctzll(m));
        ty1 = base + 63 - __builtin_clzll(m);
      }
    }
    for (int base = 0; base < a.tiles_x; base += 64) {
      const int tx = base + lane;
      bool reach = false;
      if (tx < a.tiles_x) {
        const TileCells r = tile_cells(a, tx, 0);
        reach = cx >= r.cx0 && cx < r.cx0 + r.ncx;
      }
      const uint64_t m = __ballot(reach);
      if (m) {
        tx0 = min(tx0, base + __builtin_ctzll(m));
        tx1 = base + 63 - __builtin_clzll(m);
      }
    }
    if (lane == 0) {
      bounds[0] = ty0;
      bounds[1] = ty1;
      bounds[2] = tx0;
      bounds[3] = tx1;
    }
  }
  __syncthreads();
  const int ty0 = bounds[0], ty1 = bounds[1], tx0 = bounds[2], tx1 = bounds[3];
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
  g.nsplit = colgemm_splits((int64_t)a.V * a.Hp * a.Wp, kHid, a.nh + 1);
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
