// Tile binning and the device radix sort on (tile, depth) keys.
//
// The per-tile lists must be ordered by (tile, float32 depth, index). This is
// an LSD radix sort of the 64-bit key (tile << 32 | depth bits) over the
// Gaussian-major list of intersections, done in an order that touches fewer
// items: every intersection of one Gaussian shares its depth bits, so the
// four depth digits are sorted on the (compacted) visible Gaussians before
// duplication, the list is then emitted Gaussian by Gaussian in depth order,
// and the remaining tile digits are sorted stably on the intersections. The
// result equals a stable LSD sort of the full keys of the Gaussian-major
// list.
//
// Each pass is three kernels: an upsweep (per-block 256-bin digit histogram,
// stored digit-major), a scan with one wave per digit that turns a digit's
// counts over the blocks into each block's offset within the digit and the
// digit's total, and a stable scatter that adds the digit starts (a scan of
// the 256 totals, repeated by every block). Within a block, wave ballots find
// lanes with equal digits; ranks follow item order within a wave, across the
// block's waves and across its rounds.
#include "internal.h"

namespace asgs {

namespace {

struct RadixArgs {
  const uint32_t* keys_in;
  const uint32_t* vals_in;                 // nullptr: the value is the item index
  uint32_t* keys_out;
  uint32_t* vals_out;
  const unsigned long long* count_dev;     // nullptr: use count_host
  uint64_t count_host;
  uint64_t count_cap;
  int32_t shift;
  int32_t filter;                          // drop keys equal to kInvalidKey
  uint32_t* hist;                          // [256][nb] digit-major histograms, then offsets; [256] totals after
  unsigned int* counter;                   // last-block counter (0 between uses)
  unsigned long long* total_out;           // nullptr or: number of kept items
};

ASGS_DEV uint64_t item_count(const RadixArgs& a) {
  uint64_t n = a.count_dev ? (uint64_t)__hip_atomic_load(a.count_dev, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                           : a.count_host;
  return n < a.count_cap ? n : a.count_cap;
}

ASGS_DEV uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ void __launch_bounds__(kSortThreads) k_radix_upsweep(RadixArgs a) {
  __shared__ uint32_t lh[kRadixBins];
  const uint64_t n = item_count(a);
  const uint64_t nb = (n + kSortItems - 1) / kSortItems;
  const uint64_t b = blockIdx.x;
  if (b >= nb) return;
  lh[threadIdx.x] = 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortIPT; ++r) {
    const uint64_t idx = b * kSortItems + (uint64_t)r * kSortThreads + threadIdx.x;
    if (idx < n) {
      const uint32_t k = a.keys_in[idx];
      if (!a.filter || k != kInvalidKey) atomicAdd(&lh[(k >> a.shift) & (kRadixBins - 1)], 1u);
    }
  }
  __syncthreads();
  a.hist[(uint64_t)threadIdx.x * nb + b] = lh[threadIdx.x];
}

constexpr int kScanPer = 8;  // block counts per lane in one step of the digit scan

// One wave per digit: exclusive prefix of the digit's counts over the
// blocks, in place, and the digit total after the histograms. Each lane takes
// kScanPer consecutive blocks; every load of a step is issued before the sums.
__global__ void __launch_bounds__(256) k_radix_scan(RadixArgs a) {
  const uint64_t n = item_count(a);
  const int nb = (int)((n + kSortItems - 1) / kSortItems);
  const int lane = threadIdx.x & 63;
  const int d = blockIdx.x * 4 + (threadIdx.x >> 6);
  uint32_t* h = a.hist + (uint64_t)d * nb;
  uint32_t carry = 0u;
  for (int b0 = 0; b0 < nb; b0 += 64 * kScanPer) {
    uint32_t v[kScanPer];
    uint32_t sum = 0u;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      const int b = b0 + lane * kScanPer + q;
      v[q] = b < nb ? h[b] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) sum += v[q];
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    uint32_t run = carry + incl - sum;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      const int b = b0 + lane * kScanPer + q;
      if (b < nb) h[b] = run;
      run += v[q];
    }
    carry += __shfl(incl, 63);
  }
  if (lane == 0) a.hist[(uint64_t)kRadixBins * nb + d] = carry;
}

__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(RadixArgs a) {
  __shared__ uint32_t base[kRadixBins];
  __shared__ uint32_t run[kRadixBins];
  __shared__ uint32_t wcnt[kSortThreads / 64][kRadixBins];
  const uint64_t n = item_count(a);
  const uint64_t nb = (n + kSortItems - 1) / kSortItems;
  const uint64_t b = blockIdx.x;
  if (b >= nb) return;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  // digit starts: exclusive scan of the digit totals (every block repeats it)
  {
    const uint32_t tot = a.hist[(uint64_t)kRadixBins * nb + t];
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    if (lane == 63) run[wv] = incl;  // wave totals (run is reset below)
    __syncthreads();
    uint32_t before = 0u;
    for (int w = 0; w < wv; ++w) before += run[w];
    base[t] = before + incl - tot + a.hist[(uint64_t)t * nb + b];  // + this block's offset in the digit
    if (b == 0 && t == kRadixBins - 1 && a.total_out) *a.total_out = before + incl;
    __syncthreads();
  }
  run[t] = 0u;
  for (int r = 0; r < kSortIPT; ++r) {
    const uint64_t idx = b * kSortItems + (uint64_t)r * kSortThreads + t;
    uint32_t key = 0u, val = 0u;
    bool valid = idx < n;
    if (valid) {
      key = a.keys_in[idx];
      val = a.vals_in ? a.vals_in[idx] : (uint32_t)idx;
      if (a.filter && key == kInvalidKey) valid = false;
    }
    const uint32_t d = (key >> a.shift) & (kRadixBins - 1);
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][t] = 0u;
    __syncthreads();
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    const uint32_t below = lanes_below(m);
    if (valid && below == 0) wcnt[wv][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + run[d] + below;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
      a.keys_out[pos] = key;
      a.vals_out[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0u;
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) add += wcnt[w][t];
    run[t] += add;
  }
}

void radix_pass(const RadixArgs& a, uint64_t max_items, hipStream_t s) {
  const unsigned nblk = (unsigned)((max_items + kSortItems - 1) / kSortItems);
  const unsigned g = nblk > 0 ? nblk : 1;
  hipLaunchKernelGGL(k_radix_upsweep, dim3(g), dim3(kSortThreads), 0, s, a);
  hipLaunchKernelGGL(k_radix_scan, dim3(kRadixBins / 4), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_radix_scatter, dim3(g), dim3(kSortThreads), 0, s, a);
}

// ---------------------------------------------------------------------------
// Duplication: exclusive scan of the tile counts in depth order, then each
// visible Gaussian emits one (tile key, index) pair per tile of its rect.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kScanThreads) k_dup_upsweep(RenderConst rc, char* ctx, CtxLayout L) {
  __shared__ unsigned long long red[kScanThreads / 64];
  (void)rc;
  CtxHeader* hdr = ctx_ptr<CtxHeader>(ctx, L.hdr);
  const uint64_t m = __hip_atomic_load(&hdr->n_visible, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t nb = (m + kScanItems - 1) / kScanItems;
  const uint64_t b = blockIdx.x;
  const uint32_t* ids = ctx_ptr<const uint32_t>(ctx, L.dvalB);
  const uint32_t* ntiles = ctx_ptr<const uint32_t>(ctx, L.ntiles);
  uint32_t* bsum = ctx_ptr<uint32_t>(ctx, L.bsum);
  unsigned long long s = 0;
  if (b < nb) {
    for (int r = 0; r < kScanIPT; ++r) {
      const uint64_t j = b * kScanItems + (uint64_t)r * kScanThreads + threadIdx.x;
      if (j < m) s += ntiles[ids[j]];
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (b < nb && threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) tot += red[w];
    bsum[b] = (uint32_t)tot;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_dup_emit(RenderConst rc, const ViewDev* __restrict__ views,
                                                           char* ctx, CtxLayout L) {
  __shared__ uint32_t tsum[kScanThreads];
  CtxHeader* hdr = ctx_ptr<CtxHeader>(ctx, L.hdr);
  const uint64_t m = __hip_atomic_load(&hdr->n_visible, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t nb = (m + kScanItems - 1) / kScanItems;
  const uint64_t b = blockIdx.x;
  if (b >= nb) return;
  const uint32_t* ids = ctx_ptr<const uint32_t>(ctx, L.dvalB);
  const uint32_t* ntiles = ctx_ptr<const uint32_t>(ctx, L.ntiles);
  const short4* rect = ctx_ptr<const short4>(ctx, L.rect);
  const uint32_t* bsum = ctx_ptr<const uint32_t>(ctx, L.bsum);
  uint32_t* toff = ctx_ptr<uint32_t>(ctx, L.toff);
  int32_t* rank = ctx_ptr<int32_t>(ctx, L.rank);
  uint32_t* pkey = ctx_ptr<uint32_t>(ctx, L.pkeyA);
  uint32_t* dupgid = ctx_ptr<uint32_t>(ctx, L.dupgid);
  // blocked arrangement: thread t owns items t*IPT .. t*IPT+IPT-1 of the block
  const uint64_t j0 = b * kScanItems + (uint64_t)threadIdx.x * kScanIPT;
  uint32_t cnt[kScanIPT];
  uint32_t mine = 0;
#pragma unroll
  for (int r = 0; r < kScanIPT; ++r) {
    const uint64_t j = j0 + r;
    cnt[r] = j < m ? ntiles[ids[j]] : 0u;
    mine += cnt[r];
  }
  // sums of the blocks before this one (and, in block 0, of all blocks)
  __shared__ unsigned long long bred[kScanThreads / 64];
  __shared__ unsigned long long bbase, btotal;
  {
    unsigned long long pre = 0, tot = 0;
    for (uint64_t bb = threadIdx.x; bb < nb; bb += kScanThreads) {
      const uint32_t v = bsum[bb];
      tot += v;
      pre += bb < b ? v : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o);
    if ((threadIdx.x & 63) == 0) bred[threadIdx.x >> 6] = pre;
    __syncthreads();
    if (threadIdx.x == 0) bbase = bred[0] + bred[1] + bred[2] + bred[3];
    __syncthreads();
    if (b == 0) {
      for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
      if ((threadIdx.x & 63) == 0) bred[threadIdx.x >> 6] = tot;
      __syncthreads();
      if (threadIdx.x == 0) {
        btotal = bred[0] + bred[1] + bred[2] + bred[3];
        hdr->n_isect = btotal;
        hdr->overflow = btotal > (uint64_t)rc.cap ? 1u : 0u;
      }
    }
  }
  tsum[threadIdx.x] = mine;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)off ? tsum[threadIdx.x - off] : 0u;
    __syncthreads();
    tsum[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t off = bbase + (threadIdx.x > 0 ? tsum[threadIdx.x - 1] : 0u);
  const uint64_t cap = (uint64_t)rc.cap;
  for (int r = 0; r < kScanIPT; ++r) {
    const uint64_t j = j0 + r;
    if (j >= m) break;
    const uint32_t gid = ids[j];
    toff[j] = (uint32_t)off;
    rank[gid] = (int32_t)j;
    const int view = (int)(gid / (uint64_t)rc.n);
    const ViewDev& V = views[view];
    const short4 rc4 = rect[gid];
    uint64_t p = off;
    for (int ty = rc4.z; ty <= rc4.w; ++ty) {
      for (int tx = rc4.x; tx <= rc4.y; ++tx, ++p) {
        if (p < cap) {
          pkey[p] = (uint32_t)(V.tile_base + ty * V.TX + tx);
          dupgid[p] = gid;
        }
      }
    }
    off += cnt[r];
  }
}

// Tile ranges [start, end) from the sorted keys, and the Gaussian of every
// sorted intersection.
__global__ void __launch_bounds__(256) k_ranges(RenderConst rc, char* ctx, CtxLayout L, size_t key_off,
                                                size_t val_off) {
  CtxHeader* hdr = ctx_ptr<CtxHeader>(ctx, L.hdr);
  uint64_t I = __hip_atomic_load(&hdr->n_isect, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (I > (uint64_t)rc.cap) I = rc.cap;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= I) return;
  const uint32_t* key = ctx_ptr<const uint32_t>(ctx, key_off);
  const uint32_t* val = ctx_ptr<const uint32_t>(ctx, val_off);
  uint2* ranges = ctx_ptr<uint2>(ctx, L.ranges);
  const uint32_t k = key[i];
  if (i == 0 || key[i - 1] != k) ranges[k].x = (uint32_t)i;
  if (i + 1 == I || key[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
  ctx_ptr<uint32_t>(ctx, L.pairgid)[i] = ctx_ptr<const uint32_t>(ctx, L.dupgid)[val[i]];
}

// Blend order of the tiles: longest list first, so that the longest-running
// workgroups start first and short tiles fill in behind them. A counting sort
// on the list length (lengths of 1023 and more share one bucket); the order
// within a bucket is arbitrary, which changes no result.
constexpr int kOrderBins = 1024;
__global__ void __launch_bounds__(kOrderBins) k_tile_order(RenderConst rc, char* ctx, CtxLayout L) {
  __shared__ uint32_t bins[kOrderBins];
  __shared__ uint32_t wsum[kOrderBins / 64];
  const int t = threadIdx.x;
  const uint2* ranges = ctx_ptr<const uint2>(ctx, L.ranges);
  uint32_t* order = ctx_ptr<uint32_t>(ctx, L.torder);
  const int T = rc.total_tiles;
  bins[t] = 0u;
  __syncthreads();
  for (int i = t; i < T; i += kOrderBins) {
    const uint2 r = ranges[i];
    const uint32_t c = r.y - r.x;
    atomicAdd(&bins[kOrderBins - 1 - (c < kOrderBins - 1 ? c : kOrderBins - 1)], 1u);
  }
  __syncthreads();
  // exclusive scan of the bins: within each wave, then over the wave sums
  const uint32_t v = bins[t];
  uint32_t incl = v;
  const int lane = t & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[t >> 6] = incl;
  __syncthreads();
  uint32_t before = 0u;
  for (int w = 0; w < (t >> 6); ++w) before += wsum[w];
  __syncthreads();
  bins[t] = before + incl - v;
  __syncthreads();
  for (int i = t; i < T; i += kOrderBins) {
    const uint2 r = ranges[i];
    const uint32_t c = r.y - r.x;
    const uint32_t pos = atomicAdd(&bins[kOrderBins - 1 - (c < kOrderBins - 1 ? c : kOrderBins - 1)], 1u);
    order[pos] = (uint32_t)i;
  }
}

}  // namespace

void launch_depth_sort(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s) {
  CtxHeader* hdr = reinterpret_cast<CtxHeader*>(ctx + L.hdr);
  const size_t kin[4] = {L.dkey0, L.dkeyA, L.dkeyB, L.dkeyA};
  const size_t vin[4] = {0, L.dvalA, L.dvalB, L.dvalA};
  const size_t kout[4] = {L.dkeyA, L.dkeyB, L.dkeyA, L.dkeyB};
  const size_t vout[4] = {L.dvalA, L.dvalB, L.dvalA, L.dvalB};
  for (int p = 0; p < 4; ++p) {
    RadixArgs a;
    a.keys_in = reinterpret_cast<const uint32_t*>(ctx + kin[p]);
    a.vals_in = p == 0 ? nullptr : reinterpret_cast<const uint32_t*>(ctx + vin[p]);
    a.keys_out = reinterpret_cast<uint32_t*>(ctx + kout[p]);
    a.vals_out = reinterpret_cast<uint32_t*>(ctx + vout[p]);
    a.count_dev = p == 0 ? nullptr : &hdr->n_visible;
    a.count_host = (uint64_t)rc.nv;
    a.count_cap = (uint64_t)rc.nv;
    a.shift = 8 * p;
    a.filter = p == 0;
    a.hist = reinterpret_cast<uint32_t*>(ctx + L.hist);
      a.counter = nullptr;
    a.total_out = p == 0 ? &hdr->n_visible : nullptr;
    radix_pass(a, (uint64_t)rc.nv, s);
  }
}

void launch_duplicate(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s) {
  const unsigned nblk = (unsigned)((rc.nv + kScanItems - 1) / kScanItems);
  const ViewDev* views = reinterpret_cast<const ViewDev*>(ctx + L.views);
  hipLaunchKernelGGL(k_dup_upsweep, dim3(nblk), dim3(kScanThreads), 0, s, rc, ctx, L);
  hipLaunchKernelGGL(k_dup_emit, dim3(nblk), dim3(kScanThreads), 0, s, rc, views, ctx, L);
}

void launch_tile_sort(const RenderConst& rc, const CtxLayout& L, char* ctx, hipStream_t s) {
  CtxHeader* hdr = reinterpret_cast<CtxHeader*>(ctx + L.hdr);
  for (int p = 0; p < L.tile_passes; ++p) {
    const bool even = (p % 2) == 0;
    RadixArgs a;
    a.keys_in = reinterpret_cast<const uint32_t*>(ctx + (even ? L.pkeyA : L.pkeyB));
    a.vals_in = p == 0 ? nullptr : reinterpret_cast<const uint32_t*>(ctx + (even ? L.pvalA : L.pvalB));
    a.keys_out = reinterpret_cast<uint32_t*>(ctx + (even ? L.pkeyB : L.pkeyA));
    a.vals_out = reinterpret_cast<uint32_t*>(ctx + (even ? L.pvalB : L.pvalA));
    a.count_dev = &hdr->n_isect;
    a.count_host = 0;
    a.count_cap = (uint64_t)rc.cap;
    a.shift = 8 * p;
    a.filter = 0;
    a.hist = reinterpret_cast<uint32_t*>(ctx + L.hist);
    a.counter = nullptr;
    a.total_out = nullptr;
    radix_pass(a, (uint64_t)rc.cap, s);
  }
  const unsigned nblk = (unsigned)((rc.cap + 255) / 256);
  hipLaunchKernelGGL(k_ranges, dim3(nblk > 0 ? nblk : 1), dim3(256), 0, s, rc, ctx, L, L.pkey_fin,
                     L.pval_fin);
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderBins), 0, s, rc, ctx, L);
}

}  // namespace asgs
