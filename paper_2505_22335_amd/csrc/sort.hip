// Tile binning: the per-tile lists of (tile, Gaussian) intersections, each
// ordered front to back by (float32 camera depth, index).
//
// The lists are built as a counting sort on the tile followed by a sort of
// every list on its own:
//  - each visible Gaussian is counted into the counter of every tile its
//    rectangle covers, so the list lengths are known;
//  - one workgroup scans the lengths into the tile ranges (and orders the
//    tiles longest list first, the order the blend kernels start them in);
//  - every visible Gaussian takes its places in its tiles' ranges through the
//    tiles' cursors, writing the 64-bit key (depth bits << 32 | index). The
//    order inside a range is arbitrary at this point;
//  - one workgroup per tile sorts its range on the key. The keys are unique,
//    so the final lists do not depend on the emission order.
// Every intersection also owns a gradient slot: the Gaussian-major position
// toff[Gaussian] + (its tile's position in the Gaussian's rectangle), from an
// exclusive scan of the tile counts in (view, Gaussian) order. The blend
// backward writes a list entry's gradient into its slot, and the projection
// backward sums a Gaussian's slots, which are contiguous.
#include "internal.h"

namespace asgs {

namespace {

template <typename T>
ASGS_DEV T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  return v;
}

// The block's (view, Gaussian) pair of this thread.
struct ScanBlock {
  int view;
  int64_t j;     // this thread's pair
  bool valid;    // j is a pair of the block
};

ASGS_DEV ScanBlock scan_block(const RenderConst& rc) {
  const int64_t nbx = (rc.n + kScanThreads - 1) / kScanThreads;
  ScanBlock sb;
  sb.view = (int)(blockIdx.x / nbx);
  const int64_t i = (int64_t)(blockIdx.x - sb.view * nbx) * kScanThreads + threadIdx.x;
  sb.valid = i < rc.n;
  sb.j = (int64_t)sb.view * rc.n + i;
  return sb;
}

// ---------------------------------------------------------------------------
// One workgroup: the tile ranges [start, end) from the list lengths, the
// emission cursors (= starts), the totals and the blend order of the tiles
// (per position: tile, start, end; the forward adds the walked length),
// longest list first (a counting sort on the length; lengths of 1023 and more
// share one bucket, and the order within a bucket is arbitrary, which changes
// no result). When the intersections exceed the capacity every range is left
// empty: nothing is blended and the overflow is recorded.
// ---------------------------------------------------------------------------
constexpr int kOrderBins = 1024;
constexpr int kTileScanThreads = 1024;

ASGS_DEV int order_bin(uint32_t c) { return kOrderBins - 1 - (int)(c < kOrderBins - 1 ? c : kOrderBins - 1); }

__global__ void __launch_bounds__(kTileScanThreads) k_tile_scan(RenderConst rc, const ViewDev* __restrict__ views,
                                                               char* ctx, CtxLayout L) {
  __shared__ uint32_t bins[kOrderBins];
  __shared__ uint32_t scount[ASGS_MAX_VIEWS][kSplitThresholds];  // per view: lists per length band, then above each threshold
  __shared__ uint32_t sused[ASGS_MAX_VIEWS];
  __shared__ uint32_t vcnt[ASGS_MAX_VIEWS];
  __shared__ unsigned long long wtot[kTileScanThreads / 64];
  __shared__ uint32_t wbin[kTileScanThreads / 64];
  __shared__ unsigned long long wvis[kTileScanThreads / 64];
  __shared__ unsigned long long wpb[kTileScanThreads / 64], wpv[kTileScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  constexpr int NW = kTileScanThreads / 64;
  const int T = rc.total_tiles;
  uint32_t* tcur = ctx_ptr<uint32_t>(ctx, L.tcur);
  uint2* ranges = ctx_ptr<uint2>(ctx, L.ranges);
  uint4* binfo = ctx_ptr<uint4>(ctx, L.binfo);
  CtxHeader* hdr = ctx_ptr<CtxHeader>(ctx, L.hdr);
  // thread t owns the consecutive tiles [a0, a1)
  const int per = (T + kTileScanThreads - 1) / kTileScanThreads;
  const int a0 = min(T, t * per), a1 = min(T, a0 + per);
  bins[t] = 0u;
  for (int q = t; q < ASGS_MAX_VIEWS * kSplitThresholds; q += kTileScanThreads) (&scount[0][0])[q] = 0u;
  if (t < ASGS_MAX_VIEWS) {
    sused[t] = 0u;
    vcnt[t] = 0u;
  }
  __syncthreads();
  unsigned long long mine = 0;
  for (int i = a0; i < a1; ++i) {
    const uint32_t c = tcur[i];
    mine += c;
    atomicAdd(&bins[order_bin(c)], 1u);
    if (c > (uint32_t)kSplitLen) {
      // band j: kSplitLen + j kSplitStep < c <= kSplitLen + (j + 1) kSplitStep (the last open)
      const uint32_t j = (c - kSplitLen - 1) / kSplitStep;
      atomicAdd(&scount[find_view(views, rc.n_views, i)][j < kSplitThresholds ? j : kSplitThresholds - 1], 1u);
    }
  }
  unsigned long long vis = 0;
  // per-block exclusive prefixes for the emission: of the tile-count sums and
  // of the visible counts, over all blocks (a view's own visible prefix is the
  // difference to its first block's); thread t takes consecutive blocks
  {
    const int64_t nbk = scan_blocks(rc.n, rc.n_views);
    const int64_t perb = (nbk + kTileScanThreads - 1) / kTileScanThreads;
    const int64_t b0 = min(nbk, (int64_t)t * perb), b1 = min(nbk, b0 + perb);
    const uint32_t* bs = ctx_ptr<const uint32_t>(ctx, L.bsum);
    const uint32_t* vs = ctx_ptr<const uint32_t>(ctx, L.vsum);
    uint32_t* bp = ctx_ptr<uint32_t>(ctx, L.bpre);
    uint32_t* vp = ctx_ptr<uint32_t>(ctx, L.vpre);
    const int64_t nbx = (rc.n + kScanThreads - 1) / kScanThreads;
    unsigned long long sb = 0, sv = 0;
    for (int64_t b = b0; b < b1; ++b) {
      sb += bs[b];
      sv += vs[b];
      atomicAdd(&vcnt[b / nbx], vs[b]);  // visible Gaussians per view
    }
    // visible pairs of the whole batch
    vis = sv;
    for (int o = 32; o > 0; o >>= 1) vis += __shfl_xor(vis, o);
    const unsigned long long ib = wave_incl_scan(sb, lane), iv = wave_incl_scan(sv, lane);
    if (lane == 63) {
      wpb[wv] = ib;
      wpv[wv] = iv;
    }
    __syncthreads();
    unsigned long long eb = ib - sb, ev = iv - sv;
    for (int w = 0; w < wv; ++w) {
      eb += wpb[w];
      ev += wpv[w];
    }
    for (int64_t b = b0; b < b1; ++b) {
      bp[b] = (uint32_t)eb;
      vp[b] = (uint32_t)ev;
      eb += bs[b];
      ev += vs[b];
    }
  }
  const unsigned long long incl = wave_incl_scan(mine, lane);
  if (lane == 63) wtot[wv] = incl;
  if (lane == 0) wvis[wv] = vis;
  __syncthreads();
  // lists above each threshold: suffix sums of the bands, one view per thread
  if (t < rc.n_views) {
    uint32_t above = 0u;
    for (int j = kSplitThresholds - 1; j >= 0; --j) {
      above += scount[t][j];
      scount[t][j] = above;
    }
  }
  const uint32_t bv = bins[t];
  const uint32_t bincl = wave_incl_scan(bv, lane);
  if (lane == 63) wbin[wv] = bincl;
  unsigned long long before = 0, total = 0, vtot = 0;
  for (int w = 0; w < NW; ++w) {
    before += w < wv ? wtot[w] : 0ull;
    total += wtot[w];
    vtot += wvis[w];
  }
  __syncthreads();
  uint32_t bbefore = 0;
  for (int w = 0; w < wv; ++w) bbefore += wbin[w];
  bins[t] = bbefore + bincl - bv;
  const bool ovf = total > (unsigned long long)rc.cap;
  if (t == 0) {
    hdr->n_isect = total;
    hdr->n_visible = vtot;
    hdr->overflow = ovf ? 1u : 0u;
  }
  __syncthreads();
  if (t < rc.n_views) ctx_ptr<uint32_t>(ctx, L.vcount)[t] = vcnt[t];
  uint4* sinfo = ctx_ptr<uint4>(ctx, L.sinfo);
  for (int q = t; q < rc.n_views * kSplitPerView; q += kTileScanThreads) sinfo[q] = make_uint4(~0u, 0u, 0u, 0u);
  __syncthreads();  // the slot table is cleared before any slot is taken
  uint32_t* bslot = ctx_ptr<uint32_t>(ctx, L.bslot);
  unsigned long long run = before + incl - mine;
  for (int i = a0; i < a1; ++i) {
    const uint32_t c = tcur[i];
    const uint2 r = ovf ? make_uint2(0u, 0u) : make_uint2((uint32_t)run, (uint32_t)(run + c));
    ranges[i] = r;
    tcur[i] = (uint32_t)run;
    binfo[atomicAdd(&bins[order_bin(c)], 1u)] = make_uint4((uint32_t)i, r.x, r.y, 0u);
    // split when longer than the view's threshold (the slot order is arbitrary)
    uint32_t sl = 0u;
    if (!ovf && c > (uint32_t)kSplitLen) {
      const int v = find_view(views, rc.n_views, i);
      int j = 0;
      while (j < kSplitThresholds && scount[v][j] > (uint32_t)kSplitPerView) ++j;
      if (j < kSplitThresholds && c > (uint32_t)(kSplitLen + j * kSplitStep)) {
        const uint32_t slot = (uint32_t)v * kSplitPerView + atomicAdd(&sused[v], 1u);
        sinfo[slot] = make_uint4((uint32_t)i, r.x, r.y, 0u);
        sl = slot + 1u;
      }
    }
    bslot[i] = sl;
    run += c;
  }
}

// ---------------------------------------------------------------------------
// Emission: the exclusive scan of the tile counts in (view, Gaussian) order
// gives every visible Gaussian its first gradient slot; the Gaussian then
// takes one place in the range of every tile of its rectangle. Places are
// reserved per block and tile through the same LDS box as the counting.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kScanThreads) k_dup_emit(RenderConst rc, const ViewDev* __restrict__ views,
                                                           char* ctx, CtxLayout L) {
  __shared__ unsigned long long wred[kScanThreads / 64];
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ uint32_t wvp[kScanThreads / 64], wvc[kScanThreads / 64];
  __shared__ int bred[4];
  __shared__ uint32_t cell[kBoxCells];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const ScanBlock sb = scan_block(rc);
  const ViewDev& V = views[sb.view];
  const uint32_t cnt = sb.valid ? ctx_ptr<const uint32_t>(ctx, L.ntiles)[sb.j] : 0u;
  const short4 r = cnt > 0u ? ctx_ptr<const short4>(ctx, L.rect)[sb.j] : make_short4(1, 0, 1, 0);
  uint32_t* tcur = ctx_ptr<uint32_t>(ctx, L.tcur);
  unsigned long long* ukey = ctx_ptr<unsigned long long>(ctx, L.ukey);
  // first gradient slot: sum of the blocks before this one (the scan's
  // prefix) + the prefix in it
  const unsigned long long pre = ctx_ptr<const uint32_t>(ctx, L.bpre)[blockIdx.x];
  const uint32_t incl = wave_incl_scan(cnt, lane);
  if (lane == 0) wred[wv] = wv == 0 ? pre : 0ull;
  if (lane == 63) wsum[wv] = incl;
  // place in the view's visible list: visible Gaussians of the view's earlier
  // blocks, of the earlier waves, of the earlier lanes
  const int64_t nbx = (rc.n + kScanThreads - 1) / kScanThreads;
  const uint32_t* vpg = ctx_ptr<const uint32_t>(ctx, L.vpre);
  const uint32_t vpre = vpg[blockIdx.x] - vpg[(int64_t)sb.view * nbx];
  const uint64_t vbits = __ballot(cnt > 0u);
  if (lane == 0) {
    wvp[wv] = wv == 0 ? vpre : 0u;
    wvc[wv] = (uint32_t)__popcll(vbits);
  }
  const bool small = cnt > 0u && cnt <= (uint32_t)kBoxRect;
  const TileBox bx = tile_box(r, small, bred, cell);  // synchronises: wred, wsum are complete
  unsigned long long off = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) off += wred[w] + (w < wv ? wsum[w] : 0u);
  off += incl - cnt;
  if (sb.valid) ctx_ptr<uint32_t>(ctx, L.toff)[sb.j] = (uint32_t)off;
  if (cnt > 0u) {
    uint32_t vp = __builtin_amdgcn_mbcnt_hi((uint32_t)(vbits >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)vbits, 0u));
    for (int w = 0; w < kScanThreads / 64; ++w) vp += wvp[w] + (w < wv ? wvc[w] : 0u);
    ctx_ptr<uint32_t>(ctx, L.vlist)[(int64_t)sb.view * rc.n + vp] = (uint32_t)sb.j;
  }
  const bool via_lds = bx.lds && small;
  // count the block's places per tile, reserve them, then hand them out
  if (via_lds)
    for (int ty = r.z; ty <= r.w; ++ty)
      for (int tx = r.x; tx <= r.y; ++tx) atomicAdd(&cell[(ty - bx.y0) * bx.w + tx - bx.x0], 1u);
  __syncthreads();
  if (bx.lds)
    for (int c = t; c < bx.area; c += kScanThreads) {
      const uint32_t k = cell[c];
      if (k) {
        const int cy = c / bx.w;
        cell[c] = atomicAdd(&tcur[V.tile_base + (bx.y0 + cy) * V.TX + bx.x0 + c - cy * bx.w], k);
      }
    }
  __syncthreads();
  if (cnt == 0u) return;
  const unsigned long long key = ((unsigned long long)ctx_ptr<const uint32_t>(ctx, L.dkey)[sb.j] << 32) |
                                 (uint32_t)sb.j;
  const uint64_t cap = (uint64_t)rc.cap;
  for (int ty = r.z; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.y; ++tx) {
      const uint32_t pos = via_lds ? atomicAdd(&cell[(ty - bx.y0) * bx.w + tx - bx.x0], 1u)
                                   : atomicAdd(&tcur[V.tile_base + ty * V.TX + tx], 1u);
      if (pos < cap) ukey[pos] = key;
    }
}

// ---------------------------------------------------------------------------
// Per tile: sort the range on the key and write the sorted Gaussian, gradient
// slot and tile key of every list entry. Ranges up to kListSort entries are
// sorted in LDS by one bitonic network; longer ranges are cut into runs of
// kListSort entries that are sorted the same way, which the workgroup then
// merges pairwise (merge-path split of the output among the threads)
// through a scratch array until one run is left.
// ---------------------------------------------------------------------------
constexpr int kListThreads = 256;
constexpr int kListSort = 2048;
constexpr unsigned long long kKeyMax = ~0ull;  // above every real key (depth bits < 0x7F800000)

// Ascending bitonic sort of sk[0, P), P a power of two; the caller has
// synchronised the workgroup after filling sk.
ASGS_DEV void bitonic_lds(unsigned long long* sk, int P, int t) {
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = t; q < (P >> 1); q += kListThreads) {
        const int lo = 2 * q - (q & (j - 1));  // q with a zero bit inserted at j
        const int hi = lo + j;
        const unsigned long long a = sk[lo], b = sk[hi];
        const bool up = (lo & k) == 0;
        if ((a > b) == up) {
          sk[lo] = b;
          sk[hi] = a;
        }
      }
      __syncthreads();
    }
}

struct ListOut {
  const short4* rect;
  const uint32_t* toff;
  uint32_t* pairgid;
  uint32_t* pslot;
  uint32_t* ptile;
  uint32_t tile;
  int tx, ty;

  // Gaussian, gradient slot and tile of list position pos.
  ASGS_DEV void put(uint64_t pos, unsigned long long key) const {
    const uint32_t gid = (uint32_t)key;
    const short4 r = rect[gid];
    pairgid[pos] = gid;
    pslot[pos] = toff[gid] + (uint32_t)((ty - r.z) * (r.y - r.x + 1) + (tx - r.x));
    ptile[pos] = tile;
  }
};

__global__ void __launch_bounds__(kListThreads) k_list_sort(RenderConst rc, const ViewDev* __restrict__ views,
                                                           char* ctx, CtxLayout L) {
  __shared__ unsigned long long sk[kListSort];
  const uint4 bi = ctx_ptr<const uint4>(ctx, L.binfo)[blockIdx.x];
  const uint32_t tile = bi.x;
  const uint2 rg = make_uint2(bi.y, bi.z);
  const uint32_t n = rg.y - rg.x;
  if (n == 0u) return;
  const int t = threadIdx.x;
  ListOut out;
  {
    const ViewDev& V = views[find_view(views, rc.n_views, (int)tile)];
    const int lt = (int)tile - V.tile_base;
    out.ty = lt / V.TX;
    out.tx = lt - out.ty * V.TX;
  }
  out.rect = ctx_ptr<const short4>(ctx, L.rect);
  out.toff = ctx_ptr<const uint32_t>(ctx, L.toff);
  out.pairgid = ctx_ptr<uint32_t>(ctx, L.pairgid);
  out.pslot = ctx_ptr<uint32_t>(ctx, L.pslot);
  out.ptile = ctx_ptr<uint32_t>(ctx, L.ptile);
  out.tile = tile;
  unsigned long long* a = ctx_ptr<unsigned long long>(ctx, L.ukey) + rg.x;
  if (n <= (uint32_t)kListSort) {
    int P = 1;
    while ((uint32_t)P < n) P <<= 1;
    for (int i = t; i < P; i += kListThreads) sk[i] = (uint32_t)i < n ? a[i] : kKeyMax;
    __syncthreads();
    bitonic_lds(sk, P, t);
    for (uint32_t i = t; i < n; i += kListThreads) out.put(rg.x + i, sk[i]);
    return;
  }
  // sorted runs of kListSort entries, in place
  for (uint32_t c0 = 0; c0 < n; c0 += kListSort) {
    const uint32_t m = min((uint32_t)kListSort, n - c0);
    for (int i = t; i < kListSort; i += kListThreads) sk[i] = (uint32_t)i < m ? a[c0 + i] : kKeyMax;
    __syncthreads();
    bitonic_lds(sk, kListSort, t);
    for (uint32_t i = t; i < m; i += kListThreads) a[c0 + i] = sk[i];
    __syncthreads();
  }
  // pairwise merges of runs of width w, a -> b, until one run is left
  unsigned long long* b = ctx_ptr<unsigned long long>(ctx, L.tkey) + rg.x;
  const uint64_t per = ((uint64_t)n + kListThreads - 1) / kListThreads;
  for (uint64_t w = kListSort; w < n; w <<= 1) {
    uint64_t o = min((uint64_t)n, (uint64_t)t * per);
    const uint64_t oend = min((uint64_t)n, o + per);
    while (o < oend) {
      const uint64_t lo = o - o % (2 * w);
      const uint64_t wa = min(w, (uint64_t)n - lo);
      const uint64_t wb = min(w, (uint64_t)n - lo - wa);
      const unsigned long long* A = a + lo;
      const unsigned long long* B = A + wa;
      const uint64_t diag = o - lo;
      // entries of A among the first diag outputs of this merge
      uint64_t i0 = diag > wb ? diag - wb : 0, i1 = min(diag, wa);
      while (i0 < i1) {
        const uint64_t mid = (i0 + i1) >> 1;
        if (A[mid] < B[diag - 1 - mid]) i0 = mid + 1;
        else i1 = mid;
      }
      uint64_t i = i0, j = diag - i0;
      const uint64_t stop = min(oend, lo + wa + wb);
      unsigned long long ka = i < wa ? A[i] : kKeyMax, kb = j < wb ? B[j] : kKeyMax;
      for (; o < stop; ++o) {
        if (ka < kb) {
          b[o] = ka;
          ++i;
          ka = i < wa ? A[i] : kKeyMax;
        } else {
          b[o] = kb;
          ++j;
          kb = j < wb ? B[j] : kKeyMax;
        }
      }
    }
    __syncthreads();
    unsigned long long* tmp = a;
    a = b;
    b = tmp;
  }
  for (uint32_t i = t; i < n; i += kListThreads) out.put(rg.x + i, a[i]);
}

}  // namespace

void launch_bin(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s) {
  const unsigned nblk = (unsigned)scan_blocks(rc.n, rc.n_views);
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kTileScanThreads), 0, s, rc, views, ctx, L);
  if (nblk > 0) hipLaunchKernelGGL(k_dup_emit, dim3(nblk), dim3(kScanThreads), 0, s, rc, views, ctx, L);
}

void launch_tile_sort(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s) {
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  hipLaunchKernelGGL(k_list_sort, dim3(rc.total_tiles), dim3(kListThreads), 0, s, rc, views, ctx, L);
}

}  // namespace asgs
