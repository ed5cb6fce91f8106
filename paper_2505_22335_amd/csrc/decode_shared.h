// Definitions shared by the decoder translation units (not part of the ABI).
#pragma once

#include <math.h>

#include "internal.h"

namespace asgs {

constexpr int kIn = 35;      // decoder input: 32-d anchor feature + 3-d view direction (the
                             // distance and time columns of wider inputs are packed apart)
constexpr int kHid = 32;     // hidden width of every head
constexpr int kHeads = 5;    // opacity, rgb, scale, rot, feat
constexpr int kMaxRows = ASGS_MAX_K * 27;  // second-layer rows (k * (1+3+3+4+16))

struct DecodeViews {
  float c[ASGS_MAX_VIEWS][3];
  float R[ASGS_MAX_VIEWS][9];
  float lt[ASGS_MAX_VIEWS][2];  // temporal embedding (sin pi t, cos pi t) of each view
};

struct HeadTable {
  int32_t off[kHeads];      // packed offset of W1 of head h
  int32_t xoff[kHeads];     // packed offset of head h's extra first-layer columns [32][nx]
  int32_t nx;               // extra input columns: 0, 1 (distance) or 3 (distance, sin, cos)
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

// Gradient of the decoded value of head h w.r.t. its pre-activation y.
ASGS_DEV float act_grad(int h, float y, float l_s) {
  switch (h) {
    case 0:
    case 1: { const float s = sigm(y); return s * (1.f - s); }
    case 2: { const float s = sigm(y); return l_s * s * (1.f - s); }
    default: return 1.f;
  }
}

// Activations with the hardware exp2 / log2 / reciprocal (relative error of a
// few ulp, far inside the FP32 decoder's 1e-5 budget).
ASGS_DEV float fexp(float x) { return __expf(x); }
ASGS_DEV float fsigm(float y) { return __builtin_amdgcn_rcpf(1.f + fexp(-y)); }
// log(1 + e^-|z|) with the hardware log2 (argument in (1, 2], absolute error ~1e-7)
ASGS_DEV float fsoftplus(float z) {
  return fmaxf(z, 0.f) + 0.69314718f * __builtin_amdgcn_logf(1.f + fexp(-fabsf(z)));
}
ASGS_DEV float fout_act(int h, float y, float l_s) {
  switch (h) {
    case 0:
    case 1: return fsigm(y);
    case 2: return l_s * fsigm(y);
    default: return y;
  }
}
ASGS_DEV float fact_grad(int h, float y, float l_s) {
  switch (h) {
    case 0:
    case 1: { const float s = fsigm(y); return s * (1.f - s); }
    case 2: { const float s = fsigm(y); return l_s * s * (1.f - s); }
    default: return 1.f;
  }
}

struct DecWork {
  float* part;    // per-workgroup parameter-gradient partials (chunk-major, see part_index)
  float* dcpart;  // [nblk_w][n_views][3]: camera-centre gradient partial of each workgroup
  int32_t nblk_w;
};


// Workgroup partials of the parameter gradients are stored chunk-major: for
// every run of 64 parameters, the 64-float segments of all workgroups are
// contiguous, so the reduction of one run reads one contiguous region.
ASGS_DEV int64_t part_index(int64_t p, int64_t b, int64_t nblk) { return (p >> 6) * (nblk << 6) + (b << 6) + (p & 63); }

int64_t dec_bwd_blocks(int64_t n_anchors);
void launch_dec_fwd(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                    const float* feat, const float* off, const float* params, const asgs_gaussians& out,
                    hipStream_t s);
void launch_dec_bwd(const DecodeConst& dc, const HeadTable& ht, const DecodeViews& dv, const float* xyz,
                    const float* feat, const float* params, const asgs_gaussians& dg, int view, const DecWork& w,
                    float* d_xyz, float* d_feat, bool want_params, hipStream_t s);




}  // namespace asgs
