// EWA projection of 3D Gaussians to 2D conics and its backward (UP-SLAM
// Sec. 3.1, Eq. 2), plus the per-Gaussian SE(3) pose partials.
//
// One thread per (view, Gaussian). The forward writes, per visible Gaussian,
// a 32-byte geometry record (u, v, conic A B C, opacity) and a channel record
// (rgb, camera depth, feature) in array-of-structures form so the blend
// kernels fetch one contiguous record per list entry; plus the tile rectangle,
// the tile count and the 32-bit depth key (float bits of camera depth, which
// order like the floats since depth > znear > 0). Each workgroup is also a
// binning block: it adds its Gaussians to the per-tile intersection counters
// and writes its tile-count sum and visible count.
#include "internal.h"

namespace asgs {

namespace {

struct ViewChunk {
  ViewDev v[16];
  int32_t first, count;
};

// Writes one chunk of the view table; the first chunk also resets the header
// and the per-tile intersection counters.
__global__ void k_set_views(ViewChunk chunk, ViewDev* views, CtxHeader* hdr, uint32_t* tcount,
                            int total_tiles) {
  const int i = threadIdx.x;
  if (chunk.first == 0)
    for (int t = blockIdx.x * blockDim.x + i; t < total_tiles; t += gridDim.x * blockDim.x) tcount[t] = 0u;
  if (blockIdx.x != 0) return;
  if (i < chunk.count) views[chunk.first + i] = chunk.v[i];
  if (chunk.first == 0 && i == 0) {
    hdr->n_isect = 0;
    hdr->n_visible = 0;
    hdr->overflow = 0;
    for (int c = 0; c < 15; ++c) hdr->counters[c] = 0;
    hdr->magic = 0x41534753u;
  }
}

ASGS_DEV void quat_rot(float w, float x, float y, float z, float R[9]) {
  R[0] = 1.f - 2.f * (y * y + z * z);
  R[1] = 2.f * (x * y - w * z);
  R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);
  R[4] = 1.f - 2.f * (x * x + z * z);
  R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);
  R[7] = 2.f * (y * z + w * x);
  R[8] = 1.f - 2.f * (x * x + y * y);
}

// Everything the forward and the backward share for one Gaussian.
struct Proj {
  float t[3];          // camera-space mean
  float qn[4], qinv;   // normalised quaternion and 1/|q|
  float R[9];          // rotation of the normalised quaternion
  float s[3];
  float M[9];          // R diag(s)
  float S[6];          // Sigma = M M^T: xx xy xz yy yz zz
  float xr, yr;        // clamped x/z, y/z
  bool clx, cly;       // clamp active
  float J00, J02, J11, J12;
  float T0[3], T1[3];  // rows of J W
  float a, b, c, det;  // 2D covariance (with dilation) and determinant
};

ASGS_DEV void load_gauss(const asgs_gaussians& g, int view, int64_t i, int64_t n, float m[3],
                         float s[3], float q[4], float& o) {
  const float* mp = g.mean + view * g.view_stride[0];
  const float* sp = g.scale + view * g.view_stride[1];
  const float* qp = g.rot + view * g.view_stride[2];
  const float* op = g.opacity + view * g.view_stride[3];
  m[0] = mp[i]; m[1] = mp[n + i]; m[2] = mp[2 * n + i];
  s[0] = sp[i]; s[1] = sp[n + i]; s[2] = sp[2 * n + i];
  q[0] = qp[i]; q[1] = qp[n + i]; q[2] = qp[2 * n + i]; q[3] = qp[3 * n + i];
  o = op[i];
}

ASGS_DEV void sym_mul(const float S[6], const float v[3], float out[3]) {
  out[0] = S[0] * v[0] + S[1] * v[1] + S[2] * v[2];
  out[1] = S[1] * v[0] + S[3] * v[1] + S[4] * v[2];
  out[2] = S[2] * v[0] + S[4] * v[1] + S[5] * v[2];
}

ASGS_DEV float dot3(const float a[3], const float b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Forward math up to the 2D covariance. Returns false if culled by depth.
ASGS_DEV bool proj_core(const ViewDev& V, const float m[3], const float s[3], const float q[4],
                        float dilation, float znear, Proj& P) {
  const float* W = V.R;
  // t = R_cw mu + t_cw = R_cw (mu - c), evaluated in FP64 from the float32
  // rotation and camera centre (exact copies of the pose) and rounded once:
  // the camera-space mean, and with it the depth key that orders the tile
  // lists, is the correctly rounded float32 of its exact value
  {
    const double d0 = (double)m[0] - (double)V.cc[0];
    const double d1 = (double)m[1] - (double)V.cc[1];
    const double d2 = (double)m[2] - (double)V.cc[2];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      P.t[r] = (float)fma((double)W[r * 3 + 0], d0, fma((double)W[r * 3 + 1], d1, (double)W[r * 3 + 2] * d2));
  }
  if (!(P.t[2] > znear)) return false;
  const float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  P.qinv = 1.0f / sqrtf(qq);
  for (int k = 0; k < 4; ++k) P.qn[k] = q[k] * P.qinv;
  quat_rot(P.qn[0], P.qn[1], P.qn[2], P.qn[3], P.R);
  for (int k = 0; k < 3; ++k) P.s[k] = s[k];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) P.M[r * 3 + c] = P.R[r * 3 + c] * s[c];
  const float* M = P.M;
  P.S[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  P.S[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  P.S[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  P.S[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  P.S[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  P.S[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  const float tz = P.t[2];
  float xr = P.t[0] / tz, yr = P.t[1] / tz;
  P.clx = (xr < -V.limx) || (xr > V.limx);
  P.cly = (yr < -V.limy) || (yr > V.limy);
  xr = fminf(fmaxf(xr, -V.limx), V.limx);
  yr = fminf(fmaxf(yr, -V.limy), V.limy);
  P.xr = xr;
  P.yr = yr;
  P.J00 = V.fx / tz;
  P.J02 = -V.fx * xr / tz;
  P.J11 = V.fy / tz;
  P.J12 = -V.fy * yr / tz;
  for (int k = 0; k < 3; ++k) {
    P.T0[k] = P.J00 * W[k] + P.J02 * W[6 + k];
    P.T1[k] = P.J11 * W[3 + k] + P.J12 * W[6 + k];
  }
  float ST0[3], ST1[3];
  sym_mul(P.S, P.T0, ST0);
  sym_mul(P.S, P.T1, ST1);
  P.a = dot3(P.T0, ST0) + dilation;
  P.b = dot3(P.T0, ST1);
  P.c = dot3(P.T1, ST1) + dilation;
  P.det = P.a * P.c - P.b * P.b;
  return true;
}

template <int NF>
__global__ void __launch_bounds__(256) k_project(RenderConst rc, asgs_gaussians g,
                                                 const ViewDev* __restrict__ views, char* ctx,
                                                 CtxLayout L) {
  constexpr int CS = 4 + NF;
  const int view = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i0 < rc.n;  // every thread reaches the block's tile counting below
  const int64_t i = valid ? i0 : 0;
  const ViewDev& V = views[view];
  const int64_t gid = (int64_t)view * rc.n + i;
  float m[3], s[3], q[4], o;
  load_gauss(g, view, i, rc.n, m, s, q, o);
  Proj P;
  bool vis = proj_core(V, m, s, q, rc.dilation, rc.znear, P);
  vis = valid && vis && (P.det > 0.f) && (o > rc.alpha_min);
  float u = 0.f, v = 0.f, A = 0.f, B = 0.f, C = 0.f;
  float rx = -1.f, ry = -1.f;
  bool staged = false;  // the footprint was computed (u, v, radii finite and in range)
  int tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;
  if (vis) {
    const float tz = P.t[2];
    u = V.fx * P.t[0] / tz + V.cx;
    v = V.fy * P.t[1] / tz + V.cy;
    A = P.c / P.det;
    B = -P.b / P.det;
    C = P.a / P.det;
    if (rc.extent_mode == 0) {
      // tight box of the ellipse alpha = alpha_min: half-widths sqrt(kappa^2 Sigma'_xx), ...
      const float kap2 = 2.f * logf(o / rc.alpha_min);
      rx = ceilf(sqrtf(kap2 * P.a));
      ry = ceilf(sqrtf(kap2 * P.c));
    } else {
      // square of half side three standard deviations along the major axis
      const float mid = 0.5f * (P.a + P.c);
      const float lmax = mid + sqrtf(fmaxf(0.1f, mid * mid - P.det));
      rx = ry = ceilf(3.f * sqrtf(lmax));
    }
    const float lim = 8388608.f;  // 2^23: beyond this the box arithmetic is not exact
    staged = isfinite(u) && isfinite(v) && fabsf(u) < lim && fabsf(v) < lim && rx < lim && ry < lim;
    vis = staged;
    if (vis) {
      const float iu = floorf(u), iv = floorf(v);
      tx0 = (int)fmaxf(0.f, floorf((iu - rx) * (1.f / kTile)));
      tx1 = (int)fminf((float)(V.TX - 1), floorf((iu + rx) * (1.f / kTile)));
      ty0 = (int)fmaxf(0.f, floorf((iv - ry) * (1.f / kTile)));
      ty1 = (int)fminf((float)(V.TY - 1), floorf((iv + ry) * (1.f / kTile)));
      vis = (tx0 <= tx1) && (ty0 <= ty1);
    }
  }
  float4* geom = ctx_ptr<float4>(ctx, L.geom);
  float* chan = ctx_ptr<float>(ctx, L.chan);
  short4* rect = ctx_ptr<short4>(ctx, L.rect);
  uint32_t* ntiles = ctx_ptr<uint32_t>(ctx, L.ntiles);
  uint32_t* dkey = ctx_ptr<uint32_t>(ctx, L.dkey);
  // footprint radii of every Gaussian that reached the tile rectangle (-1
  // otherwise), with its geometry record: what the tile lists follow from
  if (valid) ctx_ptr<float2>(ctx, L.rad)[gid] = staged ? make_float2(rx, ry) : make_float2(-1.f, -1.f);
  if (staged) {
    geom[2 * gid] = make_float4(u, v, A, B);
    // slot 6: the power at which o exp(power) reaches alpha_min, so that the
    // blend kernels test alpha >= alpha_min without an exponential
    geom[2 * gid + 1] = make_float4(C, o, logf(rc.alpha_min / o), 0.f);
  }
  if (!vis) {
    if (valid) {
      rect[gid] = make_short4(1, 0, 1, 0);
      ntiles[gid] = 0u;
      dkey[gid] = 0xFFFFFFFFu;
    }
  } else {
  const float* rgb = g.rgb + view * g.view_stride[4];
  // the channel record (80 or 16 bytes, 16-byte aligned) as float4 stores
  float4* ch = reinterpret_cast<float4*>(chan + gid * CS);
  ch[0] = make_float4(rgb[i], rgb[rc.n + i], rgb[2 * rc.n + i], P.t[2]);
  if (NF > 0) {
    const float* fp = g.feat + view * g.view_stride[5];
    float f[NF > 0 ? NF : 1];
#pragma unroll
    for (int c = 0; c < NF; ++c) f[c] = fp[(int64_t)c * rc.n + i];
#pragma unroll
    for (int c4 = 0; c4 < NF / 4; ++c4)
      ch[1 + c4] = make_float4(f[4 * c4], f[4 * c4 + 1], f[4 * c4 + 2], f[4 * c4 + 3]);
  }
  rect[gid] = make_short4((short)tx0, (short)tx1, (short)ty0, (short)ty1);
  ntiles[gid] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
  dkey[gid] = __float_as_uint(P.t[2]);
  }
  // Binning block (the workgroup's pairs): its intersections into the per-tile
  // counters, its tile-count sum and number of visible pairs.
  __shared__ unsigned long long red[256 / 64];
  __shared__ uint32_t vred[256 / 64];
  __shared__ int bred[4];
  __shared__ uint32_t cell[kBoxCells];
  const uint32_t cnt = vis ? (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1)) : 0u;
  const short4 r = vis ? make_short4((short)tx0, (short)tx1, (short)ty0, (short)ty1) : make_short4(1, 0, 1, 0);
  uint32_t* tcount = ctx_ptr<uint32_t>(ctx, L.tcur);
  const bool small = cnt > 0u && cnt <= (uint32_t)kBoxRect;
  const TileBox bx = tile_box(r, small, bred, cell);
  const bool via_lds = bx.lds && small;
  for (int ty = r.z; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.y; ++tx) {
      if (via_lds) atomicAdd(&cell[(ty - bx.y0) * bx.w + tx - bx.x0], 1u);
      else __hip_atomic_fetch_add(&tcount[V.tile_base + ty * V.TX + tx], 1u, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
  __syncthreads();
  if (bx.lds)
    for (int c = threadIdx.x; c < bx.area; c += blockDim.x) {
      const uint32_t k = cell[c];
      if (k) {
        const int cy = c / bx.w;
        __hip_atomic_fetch_add(&tcount[V.tile_base + (bx.y0 + cy) * V.TX + bx.x0 + c - cy * bx.w], k,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  unsigned long long sum = cnt;
  uint32_t nvis = cnt > 0u ? 1u : 0u;
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off);
    nvis += __shfl_xor(nvis, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = sum;
    vred[threadIdx.x >> 6] = nvis;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;  // binning block
    ctx_ptr<uint32_t>(ctx, L.bsum)[b] = (uint32_t)((red[0] + red[1]) + (red[2] + red[3]));
    ctx_ptr<uint32_t>(ctx, L.vsum)[b] = (vred[0] + vred[1]) + (vred[2] + vred[3]);
  }
}

// ---------------------------------------------------------------------------
// Backward: per Gaussian, sum the per-(tile, Gaussian) gradient slots written
// by the blend backward, then chain through conic -> 2D covariance -> J, W ->
// Sigma -> (scale, rotation) and through (u, v, depth) -> camera-space mean ->
// world mean, plus the pose partials dL/drho = dL/dt, dL/dphi = t x dL/dt +
// the rotation term of W = R_cw.
// ---------------------------------------------------------------------------
template <int NF>
__global__ void __launch_bounds__(256) k_project_backward(RenderConst rc, asgs_gaussians g,
                                                          asgs_gaussians dg, float* d_pose,
                                                          const ViewDev* __restrict__ views,
                                                          char* ctx, CtxLayout L) {
  constexpr int CS = 4 + NF;
  constexpr int GS = 6 + CS;
  const int view = blockIdx.y;
  const int64_t n = rc.n;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float* dm = dg.mean + view * dg.view_stride[0];
  float* ds = dg.scale + view * dg.view_stride[1];
  float* dq = dg.rot + view * dg.view_stride[2];
  float* dop = dg.opacity + view * dg.view_stride[3];
  float* drgb = dg.rgb + view * dg.view_stride[4];
  float* dft = NF > 0 ? dg.feat + view * dg.view_stride[5] : nullptr;
  // after an overflowed forward no list was blended and every gradient is zero
  const bool ovf = ctx_ptr<const CtxHeader>(ctx, L.hdr)->overflow != 0u;
  // Gaussian e of the view gets zero gradients when it was not visible
  if (e < n && (ovf || ctx_ptr<const uint32_t>(ctx, L.ntiles)[(int64_t)view * n + e] == 0u)) {
    for (int k = 0; k < 3; ++k) { dm[k * n + e] = 0.f; ds[k * n + e] = 0.f; drgb[k * n + e] = 0.f; }
    for (int k = 0; k < 4; ++k) dq[k * n + e] = 0.f;
    dop[e] = 0.f;
    for (int k = 0; k < NF; ++k) dft[k * n + e] = 0.f;
  }
  // and the e-th visible Gaussian of the view (index order) the full chain,
  // so that the waves on this path carry no invisible lanes
  const int64_t nvis = ovf ? 0 : (int64_t)ctx_ptr<const uint32_t>(ctx, L.vcount)[view];
  if (e < nvis) {
    const ViewDev& V = views[view];
    const int64_t gid = (int64_t)ctx_ptr<const uint32_t>(ctx, L.vlist)[(int64_t)view * n + e];
    const int64_t i = gid - (int64_t)view * n;
    // visible pairs own ntiles consecutive gradient slots from toff
    const uint32_t cnt = ctx_ptr<const uint32_t>(ctx, L.ntiles)[gid];
    {
      const uint32_t start = ctx_ptr<const uint32_t>(ctx, L.toff)[gid];
      const float* slot = ctx_ptr<const float>(ctx, L.gslot);
      float G[GS];
#pragma unroll
      for (int k = 0; k < GS; ++k) G[k] = 0.f;
      constexpr int GSP = (GS + 3) & ~3;  // slot stride (whole float4)
      const uint64_t end = min((uint64_t)start + cnt, (uint64_t)rc.cap);
      for (uint64_t p = start; p < end; ++p) {
        const float4* sp = reinterpret_cast<const float4*>(slot + p * GSP);
#pragma unroll
        for (int k4 = 0; k4 < GSP / 4; ++k4) {
          const float4 v = sp[k4];
          if (4 * k4 + 0 < GS) G[4 * k4 + 0] += v.x;
          if (4 * k4 + 1 < GS) G[4 * k4 + 1] += v.y;
          if (4 * k4 + 2 < GS) G[4 * k4 + 2] += v.z;
          if (4 * k4 + 3 < GS) G[4 * k4 + 3] += v.w;
        }
      }
      const float du = G[0], dv = G[1], dA = G[2], dB = G[3], dC = G[4];
      dop[i] = G[5];
      drgb[i] = G[6];
      drgb[n + i] = G[7];
      drgb[2 * n + i] = G[8];
      const float dzc = G[9];
#pragma unroll
      for (int k = 0; k < NF; ++k) dft[k * n + i] = G[10 + k];

      float m[3], s[3], q[4], o;
      load_gauss(g, view, i, n, m, s, q, o);
      Proj P;
      proj_core(V, m, s, q, rc.dilation, rc.znear, P);
      const float a = P.a, b = P.b, c = P.c, det = P.det;
      // conic (A,B,C) = (c, -b, a)/det  ->  2D covariance (a, b, c)
      const float id2 = 1.f / (det * det);
      const float da = (-c * c * dA + b * c * dB - b * b * dC) * id2;
      const float db = (2.f * b * c * dA + (-det - 2.f * b * b) * dB + 2.f * a * b * dC) * id2;
      const float dc = (-b * b * dA + a * b * dB - a * a * dC) * id2;
      // covariance -> T = J W and Sigma
      float ST0[3], ST1[3];
      sym_mul(P.S, P.T0, ST0);
      sym_mul(P.S, P.T1, ST1);
      float dT0[3], dT1[3];
      for (int k = 0; k < 3; ++k) {
        dT0[k] = 2.f * da * ST0[k] + db * ST1[k];
        dT1[k] = db * ST0[k] + 2.f * dc * ST1[k];
      }
      // symmetric dL/dSigma: da T0 T0^T + db (T0 T1^T + T1 T0^T)/2 + dc T1 T1^T
      float GS_[9];
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          GS_[r * 3 + cc] = da * P.T0[r] * P.T0[cc] + 0.5f * db * (P.T0[r] * P.T1[cc] + P.T1[r] * P.T0[cc]) +
                            dc * P.T1[r] * P.T1[cc];
      // Sigma = M M^T -> dM = 2 G M
      float dM[9];
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          dM[r * 3 + cc] = 2.f * (GS_[r * 3 + 0] * P.M[0 * 3 + cc] + GS_[r * 3 + 1] * P.M[1 * 3 + cc] +
                                  GS_[r * 3 + 2] * P.M[2 * 3 + cc]);
      // M = R diag(s)
      float dRm[9];
      for (int cc = 0; cc < 3; ++cc) {
        ds[cc * n + i] = dM[0 * 3 + cc] * P.R[0 * 3 + cc] + dM[1 * 3 + cc] * P.R[1 * 3 + cc] +
                         dM[2 * 3 + cc] * P.R[2 * 3 + cc];
        for (int r = 0; r < 3; ++r) dRm[r * 3 + cc] = dM[r * 3 + cc] * P.s[cc];
      }
      // rotation matrix -> normalised quaternion -> raw quaternion
      {
        const float w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
        const float* G = dRm;
        const float gw = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
        const float gx = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] +
                                w * G[7] - 2.f * x * G[8]);
        const float gy = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] +
                                z * G[7] - 2.f * y * G[8]);
        const float gz = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] +
                                y * G[5] + x * G[6] + y * G[7]);
        const float pr = w * gw + x * gx + y * gy + z * gz;
        dq[i] = (gw - w * pr) * P.qinv;
        dq[n + i] = (gx - x * pr) * P.qinv;
        dq[2 * n + i] = (gy - y * pr) * P.qinv;
        dq[3 * n + i] = (gz - z * pr) * P.qinv;
      }
      // T = J W
      const float* W = V.R;
      const float dJ00 = dot3(dT0, &W[0]);
      const float dJ02 = dot3(dT0, &W[6]);
      const float dJ11 = dot3(dT1, &W[3]);
      const float dJ12 = dot3(dT1, &W[6]);
      float dW[9];
      for (int k = 0; k < 3; ++k) {
        dW[0 + k] = P.J00 * dT0[k];
        dW[3 + k] = P.J11 * dT1[k];
        dW[6 + k] = P.J02 * dT0[k] + P.J12 * dT1[k];
      }
      // J and (u, v, depth) -> camera-space mean
      const float tx = P.t[0], ty = P.t[1], tz = P.t[2];
      const float itz = 1.f / tz, itz2 = itz * itz;
      float dt0 = 0.f, dt1 = 0.f, dt2 = 0.f;
      dt2 += -V.fx * itz2 * dJ00 - V.fy * itz2 * dJ11;
      const float dxr = -V.fx * itz * dJ02;
      const float dyr = -V.fy * itz * dJ12;
      dt2 += V.fx * P.xr * itz2 * dJ02 + V.fy * P.yr * itz2 * dJ12;
      if (!P.clx) { dt0 += dxr * itz; dt2 -= dxr * tx * itz2; }
      if (!P.cly) { dt1 += dyr * itz; dt2 -= dyr * ty * itz2; }
      dt0 += V.fx * itz * du;
      dt1 += V.fy * itz * dv;
      dt2 -= (V.fx * tx * du + V.fy * ty * dv) * itz2;
      dt2 += dzc;
      // t = W mu + t_cw
      dm[i] = W[0] * dt0 + W[3] * dt1 + W[6] * dt2;
      dm[n + i] = W[1] * dt0 + W[4] * dt1 + W[7] * dt2;
      dm[2 * n + i] = W[2] * dt0 + W[5] * dt1 + W[8] * dt2;
      // pose partials: rho, then phi = t x dt + rotation term from W
      pose[0] = dt0;
      pose[1] = dt1;
      pose[2] = dt2;
      float Q[9];  // W dW^T
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          Q[r * 3 + cc] = W[r * 3 + 0] * dW[cc * 3 + 0] + W[r * 3 + 1] * dW[cc * 3 + 1] + W[r * 3 + 2] * dW[cc * 3 + 2];
      pose[3] = ty * dt2 - tz * dt1 + (Q[5] - Q[7]);
      pose[4] = tz * dt0 - tx * dt2 + (Q[6] - Q[2]);
      pose[5] = tx * dt1 - ty * dt0 + (Q[1] - Q[3]);
    }
  }
  // block reduction of the pose partials; k_pose_reduce then sums the
  // per-block partials of every view in a fixed order
  __shared__ float red[6][256 / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float x = pose[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (lane == 0) red[k][wv] = x;
  }
  __syncthreads();
  float* part = ctx_ptr<float>(ctx, L.posepart);
  const int nbx = gridDim.x;
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    part[((int64_t)view * nbx + blockIdx.x) * 6 + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
  }
}

// Fixed-order sum of the per-block pose partials of each view: every thread
// adds the six partials of its blocks, then six wave and workgroup sums.
__global__ void __launch_bounds__(256) k_pose_reduce(int n_views, int nbx, const float* __restrict__ part,
                                                     float* d_pose) {
  __shared__ float fin[6][256 / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int vv = 0; vv < n_views; ++vv) {
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int bx = threadIdx.x; bx < nbx; bx += blockDim.x) {
      const float* p = part + ((int64_t)vv * nbx + bx) * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] += p[k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
      if (lane == 0) fin[k][wv] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      const int k = threadIdx.x;
      d_pose[vv * 6 + k] = (fin[k][0] + fin[k][1]) + (fin[k][2] + fin[k][3]);
    }
    __syncthreads();
  }
}

}  // namespace

void launch_set_views(const ViewDev* host_views, int n_views, ViewDev* dev_views, CtxHeader* hdr,
                      uint32_t* tcount, int total_tiles, hipStream_t s) {
  for (int first = 0; first < n_views; first += 16) {
    ViewChunk ch;
    ch.first = first;
    ch.count = n_views - first < 16 ? n_views - first : 16;
    for (int k = 0; k < ch.count; ++k) ch.v[k] = host_views[first + k];
    const int blocks = first == 0 ? (total_tiles + 255) / 256 : 1;
    hipLaunchKernelGGL(k_set_views, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, ch, dev_views, hdr,
                       tcount, total_tiles);
  }
}

void launch_project(const RenderConst& rc, const asgs_gaussians& g, const CtxLayout& L, char* ctx,
                    hipStream_t s) {
  static_assert(kScanThreads == 256, "a projection workgroup is one binning block");
  dim3 grid((unsigned)((rc.n + 255) / 256), (unsigned)rc.n_views);
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  if (rc.nf == 16)
    hipLaunchKernelGGL(k_project<16>, grid, dim3(256), 0, s, rc, g, views, ctx, L);
  else
    hipLaunchKernelGGL(k_project<0>, grid, dim3(256), 0, s, rc, g, views, ctx, L);
}

void launch_project_backward(const RenderConst& rc, const asgs_gaussians& g, const asgs_gaussians& dg,
                             float* d_pose, const CtxLayout& L, char* ctx, hipStream_t s) {
  dim3 grid((unsigned)((rc.n + 255) / 256), (unsigned)rc.n_views);
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  if (rc.nf == 16)
    hipLaunchKernelGGL(k_project_backward<16>, grid, dim3(256), 0, s, rc, g, dg, d_pose, views, ctx, L);
  else
    hipLaunchKernelGGL(k_project_backward<0>, grid, dim3(256), 0, s, rc, g, dg, d_pose, views, ctx, L);
  if (d_pose)
    hipLaunchKernelGGL(k_pose_reduce, dim3(1), dim3(256), 0, s, rc.n_views, (int)grid.x,
                       reinterpret_cast<const float*>(ctx + L.posepart), d_pose);
}

}  // namespace asgs
