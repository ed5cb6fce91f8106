// Request loop over a resident anchor scene: continuous batching of tracking
// and mapping renders (UP-SLAM Sec. 3.4 tracking, Sec. 3.3 mapping), with
// admission by device memory and overlap of batches on several HIP streams.
// Semantics and ABI: asgs_serve.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "asgs.h"
#include "asgs_serve.h"
#include "internal.h"

namespace {

using asgs::fail;
using asgs::L1Args;
using asgs::L1Views;
using asgs::launch_l1_loss;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

void sleep_until_s(double t) {
  for (;;) {
    const double d = t - now_s();
    if (d <= 0) return;
    if (d > 3e-4) std::this_thread::sleep_for(std::chrono::duration<double>(d - 2e-4));
  }
}

// First-fit allocator over [0, cap) with coalescing, 256-byte granules.
class Arena {
 public:
  explicit Arena(uint64_t cap = 0) : cap_(cap) {
    if (cap) free_[0] = cap;
  }
  uint64_t capacity() const { return cap_; }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  static uint64_t round(uint64_t b) { return (b + 255) & ~uint64_t(255); }
  // offset of a block of b bytes, or UINT64_MAX
  uint64_t alloc(uint64_t b) {
    b = round(b);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= b) {
        const uint64_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > b) free_[off + b] = sz - b;
        used_ += b;
        peak_ = std::max(peak_, used_);
        return off;
      }
    }
    return UINT64_MAX;
  }
  void release(uint64_t off, uint64_t b) {
    b = round(b);
    used_ -= b;
    auto it = free_.emplace(off, b).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  uint64_t cap_;
  uint64_t used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Req {
  asgs_request r{};
  uint64_t ticket = 0;
  std::vector<asgs_camera> cams;
  std::vector<const float*> trgb, tdepth, tfeat;
  std::vector<float*> orgb, odepth;
  int attempts = 0;
  bool exact = false;  // count intersections exactly (after a capacity overflow)
};

struct Batch {
  int kind = 0;
  int V = 0;
  std::vector<Req*> reqs;
  std::vector<asgs_camera> cams;
  int stream = -1;
  uint64_t off = 0, bytes = 0;
  int64_t capacity = 0;
  bool exact = false;
  hipEvent_t ev = nullptr;
  double start = 0, sim_done = 0;
  int status = ASGS_OK;
  asgs::CtxHeader* hdr = nullptr;  // pinned host copy of the context header
};

// Byte layout of one batch's arena block.
struct BatchLayout {
  uint64_t mean, views_g, img, dimg, dg, dpose, loss, partial, work, ctx, total;
  uint64_t g_stride;     // bytes of one view's decoded attributes (scale..feat)
  uint64_t dg_stride;    // bytes of one view's Gaussian gradients
  size_t work_bytes, ctx_bytes;
};

struct Server {
  asgs_server_config cfg{};
  asgs_decoder dec{};
  asgs_render_opts opts{};
  const float *xyz = nullptr, *feat = nullptr, *off = nullptr, *params = nullptr;
  int device = 0;
  int64_t N = 0, n_params = 0;
  char* base = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;             // per stream (one batch in flight per stream)
  std::vector<asgs::CtxHeader*> headers;      // per stream, pinned host
  std::vector<std::deque<Batch*>> inflight;  // per stream, launch order
  std::vector<bool> busy;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_comp;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, asgs_result> results;
  std::unordered_map<uint64_t, Req*> live;
  uint64_t next_ticket = 1;
  bool stop = false;
  int in_flight = 0;
  std::map<std::pair<int, int>, int64_t> isect_per_view;  // resolution -> largest count per view seen
  asgs_server_stats_t st{};
  double sim_busy_until = 0;
  std::thread sched;
  std::vector<std::thread> comp;
};

BatchLayout layout(const Server& S, const Batch& b, int64_t capacity) {
  BatchLayout L{};
  const int nf = S.dec.n_feat;
  const int64_t N = S.N, V = b.V;
  const int64_t HW = (int64_t)b.cams[0].width * b.cams[0].height;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = Arena::round(o + bytes);
    return at;
  };
  L.g_stride = (uint64_t)N * 4 * (3 + 4 + 1 + 3 + nf);
  L.dg_stride = (uint64_t)N * 4 * (3 + 3 + 4 + 1 + 3 + nf);
  L.mean = take((uint64_t)N * 3 * 4);
  L.views_g = take(L.g_stride * V);
  L.img = take((uint64_t)V * HW * 4 * (3 + 1 + nf + 1));
  L.dimg = take((uint64_t)V * HW * 4 * (3 + 1 + nf));
  L.dg = take(L.dg_stride * V);
  L.dpose = take((uint64_t)V * 6 * 4);
  L.loss = take((uint64_t)V * 4);
  L.partial = take((uint64_t)V * asgs::kL1Blocks * 4);
  asgs_decoder d = S.dec;
  (void)asgs_decode_workspace_size(&d, (int32_t)V, &L.work_bytes);
  L.work = take(L.work_bytes);
  (void)asgs_render_ctx_size(b.cams.data(), (int32_t)V, N, &S.opts, capacity, &L.ctx_bytes);
  L.ctx = take(L.ctx_bytes);
  L.total = o;
  return L;
}

// Decoded Gaussians of a batch: shared means, per-view planes.
asgs_gaussians gauss_view(const Server& S, const BatchLayout& L, char* p, bool grads) {
  const int nf = S.dec.n_feat;
  const int64_t N = S.N;
  asgs_gaussians g{};
  g.n = N;
  if (!grads) {
    float* v0 = reinterpret_cast<float*>(p + L.views_g);
    g.mean = reinterpret_cast<float*>(p + L.mean);
    g.scale = v0;
    g.rot = v0 + 3 * N;
    g.opacity = v0 + 7 * N;
    g.rgb = v0 + 8 * N;
    g.feat = nf ? v0 + 11 * N : nullptr;
    const int64_t vs = (int64_t)(L.g_stride / 4);
    const int64_t st[6] = {0, vs, vs, vs, vs, vs};
    memcpy(g.view_stride, st, sizeof st);
  } else {
    float* v0 = reinterpret_cast<float*>(p + L.dg);
    g.mean = v0;
    g.scale = v0 + 3 * N;
    g.rot = v0 + 6 * N;
    g.opacity = v0 + 10 * N;
    g.rgb = v0 + 11 * N;
    g.feat = nf ? v0 + 14 * N : nullptr;
    const int64_t vs = (int64_t)(L.dg_stride / 4);
    const int64_t st[6] = {vs, vs, vs, vs, vs, vs};
    memcpy(g.view_stride, st, sizeof st);
  }
  return g;
}

int hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(ASGS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return ASGS_OK;
}

// Issue every step of a batch on its stream (device mode).
int run_batch(Server& S, Batch& b, const BatchLayout& L) {
  hipStream_t s = S.streams[b.stream];
  void* sv = reinterpret_cast<void*>(s);
  char* p = S.base + b.off;
  const int nf = S.dec.n_feat;
  const int V = b.V;
  const int64_t HW = (int64_t)b.cams[0].width * b.cams[0].height;
  asgs_decoder d = S.dec;
  asgs_gaussians g = gauss_view(S, L, p, false);
  int st;
  if ((st = asgs_decode(&d, S.xyz, S.feat, S.off, S.params, b.cams.data(), V, &g, sv))) return st;
  void* ctx = p + L.ctx;
  asgs_images img{};
  float* ib = reinterpret_cast<float*>(p + L.img);
  img.rgb = ib;
  img.depth = ib + (int64_t)V * 3 * HW;
  img.feat = nf ? ib + (int64_t)V * 4 * HW : nullptr;
  img.alpha = ib + (int64_t)V * (4 + nf) * HW;
  if ((st = asgs_render_forward(b.cams.data(), V, &g, &S.opts, &img, ctx, L.ctx_bytes, sv))) return st;
  asgs_images dimg{};
  float* db = reinterpret_cast<float*>(p + L.dimg);
  dimg.rgb = db;
  dimg.depth = db + (int64_t)V * 3 * HW;
  dimg.feat = nf ? db + (int64_t)V * 4 * HW : nullptr;
  dimg.alpha = nullptr;
  L1Args la{};
  L1Views tv{};
  {
    int v = 0;
    for (Req* r : b.reqs) {
      for (int j = 0; j < r->r.n_views; ++j, ++v) {
        tv.t[0][v] = r->trgb[j];
        tv.t[1][v] = r->tdepth[j];
        tv.t[2][v] = r->tfeat.empty() ? nullptr : r->tfeat[j];
        tv.t[3][v] = nullptr;
        tv.w[v] = r->r.weight;
      }
    }
  }
  la.x[0] = img.rgb;
  la.x[1] = img.depth;
  la.x[2] = img.feat;
  la.x[3] = nullptr;
  la.g[0] = dimg.rgb;
  la.g[1] = dimg.depth;
  la.g[2] = dimg.feat;
  la.g[3] = nullptr;
  float* loss = reinterpret_cast<float*>(p + L.loss);
  la.partial = reinterpret_cast<float*>(p + L.partial);
  la.loss = loss;
  la.HW = HW;
  la.nf = nf;
  la.n_views = V;
  la.s[0] = (float)(1.0 / (3.0 * (double)HW));
  la.s[1] = (float)(1.0 / (double)HW);
  la.s[2] = nf ? (float)(1.0 / ((double)nf * (double)HW)) : 0.f;
  la.s[3] = 0.f;
  launch_l1_loss(la, tv, s);
  if ((st = hip_check(hipGetLastError(), "loss kernels"))) return st;
  asgs_gaussians dg = gauss_view(S, L, p, true);
  float* dpose = reinterpret_cast<float*>(p + L.dpose);
  if ((st = asgs_render_backward(b.cams.data(), V, &g, &S.opts, &dimg, &dg, dpose, ctx, L.ctx_bytes, sv)))
    return st;
  const bool map = b.kind == ASGS_REQ_MAP;
  Req* r0 = b.reqs[0];
  if ((st = asgs_decode_backward(&d, S.xyz, S.feat, S.off, S.params, b.cams.data(), V, &dg,
                                 map ? r0->r.d_xyz : nullptr, map ? r0->r.d_feat : nullptr,
                                 map ? r0->r.d_off : nullptr, map ? r0->r.d_params : nullptr, dpose, p + L.work,
                                 L.work_bytes, sv)))
    return st;
  int v = 0;
  for (Req* r : b.reqs) {
    const int nv = r->r.n_views;
    if ((st = hip_check(hipMemcpyAsync(r->r.d_pose, dpose + 6 * v, sizeof(float) * 6 * nv, hipMemcpyDeviceToDevice, s),
                        "copy d_pose")))
      return st;
    if (r->r.loss &&
        (st = hip_check(hipMemcpyAsync(r->r.loss, loss + v, sizeof(float) * nv, hipMemcpyDeviceToDevice, s),
                        "copy loss")))
      return st;
    for (int j = 0; j < nv && !r->orgb.empty(); ++j) {
      if ((st = hip_check(hipMemcpyAsync(r->orgb[j], img.rgb + (int64_t)(v + j) * 3 * HW, sizeof(float) * 3 * HW,
                                         hipMemcpyDeviceToDevice, s),
                          "copy rgb")))
        return st;
      if (!r->odepth.empty() &&
          (st = hip_check(hipMemcpyAsync(r->odepth[j], img.depth + (int64_t)(v + j) * HW, sizeof(float) * HW,
                                         hipMemcpyDeviceToDevice, s),
                          "copy depth")))
        return st;
    }
    v += nv;
  }
  if ((st = hip_check(hipMemcpyAsync(b.hdr, ctx, sizeof(asgs::CtxHeader), hipMemcpyDeviceToHost, s), "copy header")))
    return st;
  return hip_check(hipEventRecord(b.ev, s), "event record");
}

double sim_service_s(const Server& S, const Batch& b) {
  const double mpix = (double)b.V * b.cams[0].width * b.cams[0].height / 1e6;
  return (S.cfg.sim_us_fixed + S.cfg.sim_us_per_mpix * mpix) * 1e-6;
}

void finish_requests(Server& S, Batch& b, double done, int status) {
  for (Req* r : b.reqs) {
    asgs_result res{};
    res.status = status;
    res.batch_views = b.V;
    res.stream = b.stream;
    res.attempts = r->attempts;
    res.arrival = r->r.arrival;
    res.start = b.start;
    res.done = done;
    S.results[r->ticket] = res;
    S.live.erase(r->ticket);
    if (status == ASGS_OK) ++S.st.completed;
    else ++S.st.failed;
    delete r;
  }
}

// Form the next batch from the queue head (lock held).
Batch* form_batch(Server& S) {
  Req* r0 = S.queue.front();
  S.queue.pop_front();
  Batch* b = new Batch();
  b->kind = r0->r.kind;
  b->reqs.push_back(r0);
  b->exact = r0->exact;
  if (b->kind == ASGS_REQ_TRACK && !r0->exact) {
    const int W = r0->cams[0].width, H = r0->cams[0].height;
    for (auto it = S.queue.begin(); it != S.queue.end() && (int)b->reqs.size() < S.cfg.max_batch_views;) {
      Req* r = *it;
      if (r->r.kind == ASGS_REQ_TRACK && !r->exact && r->cams[0].width == W && r->cams[0].height == H) {
        b->reqs.push_back(r);
        it = S.queue.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (Req* r : b->reqs) {
    r->attempts += 1;
    for (auto& c : r->cams) b->cams.push_back(c);
  }
  b->V = (int)b->cams.size();
  return b;
}

void scheduler(Server* Sp) {
  Server& S = *Sp;
  if (!S.cfg.simulate) (void)hipSetDevice(S.device);
  std::unique_lock<std::mutex> lk(S.mu);
  for (;;) {
    S.cv_sched.wait(lk, [&] {
      if (S.queue.empty()) return S.stop && S.in_flight == 0;
      if (S.cfg.fifo && S.in_flight > 0) return false;
      return std::find(S.busy.begin(), S.busy.end(), false) != S.busy.end();
    });
    if (S.queue.empty()) break;
    Batch* b = form_batch(S);
    const std::pair<int, int> res_key(b->cams[0].width, b->cams[0].height);
    auto known = S.isect_per_view.find(res_key);
    const bool count_first = b->exact || known == S.isect_per_view.end();
    int64_t cap = count_first ? 1 : (int64_t)((double)known->second * b->V * 1.25) + 4096;
    BatchLayout L = layout(S, *b, cap);
    // admission: wait for memory; split a fused batch that can never fit
    uint64_t off = UINT64_MAX;
    for (;;) {
      off = S.arena.alloc(L.total);
      if (off != UINT64_MAX) break;
      if (S.in_flight == 0) {
        if (b->reqs.size() > 1) {  // give back all but the first request
          for (size_t i = b->reqs.size(); i-- > 1;) {
            b->reqs[i]->attempts -= 1;
            S.queue.push_front(b->reqs[i]);
          }
          b->reqs.resize(1);
          b->cams = b->reqs[0]->cams;
          b->V = (int)b->cams.size();
          cap = count_first ? 1 : (int64_t)((double)known->second * b->V * 1.25) + 4096;
          L = layout(S, *b, cap);
          continue;
        }
        break;
      }
      S.cv_sched.wait(lk);
    }
    if (off == UINT64_MAX) {
      fail(ASGS_E_CAPACITY, "request needs %llu bytes, arena has %llu", (unsigned long long)L.total,
           (unsigned long long)S.arena.capacity());
      finish_requests(S, *b, now_s(), ASGS_E_CAPACITY);
      delete b;
      S.cv_done.notify_all();
      continue;
    }
    const int si = (int)(std::find(S.busy.begin(), S.busy.end(), false) - S.busy.begin());
    S.busy[si] = true;
    b->stream = si;
    if (!S.cfg.simulate) {
      b->ev = S.events[si];
      b->hdr = S.headers[si];
    }
    b->off = off;
    b->bytes = L.total;
    b->capacity = cap;
    ++S.in_flight;
    S.st.max_in_flight = std::max(S.st.max_in_flight, S.in_flight);
    ++S.st.batches;
    S.st.batch_views += b->V;
    lk.unlock();
    b->start = now_s();
    int status = ASGS_OK;
    if (S.cfg.simulate) {
      // one device shared by all streams: batches execute one after another
      const double t0 = std::max(b->start, S.sim_busy_until);
      b->sim_done = t0 + sim_service_s(S, *b);
      S.sim_busy_until = b->sim_done;
    } else {
      if (count_first) {
        // exact count on this batch's stream, then the real layout
        asgs_decoder d = S.dec;
        char* p = S.base + b->off;
        asgs_gaussians g = gauss_view(S, L, p, false);
        void* sv = reinterpret_cast<void*>(S.streams[si]);
        int64_t need = 0;
        status = asgs_decode(&d, S.xyz, S.feat, S.off, S.params, b->cams.data(), b->V, &g, sv);
        if (!status)
          status = asgs_render_count(b->cams.data(), b->V, &g, &S.opts, p + L.ctx, L.ctx_bytes, &need, sv);
        if (!status) {
          const int64_t cap2 = need + need / 16 + 1024;
          BatchLayout L2 = layout(S, *b, cap2);
          lk.lock();
          S.arena.release(b->off, b->bytes);
          uint64_t off2 = S.arena.alloc(L2.total);
          while (off2 == UINT64_MAX && S.in_flight > 1) {
            S.cv_sched.wait(lk);
            off2 = S.arena.alloc(L2.total);
          }
          auto& m = S.isect_per_view[res_key];
          m = std::max(m, (need + b->V - 1) / b->V);
          lk.unlock();
          if (off2 == UINT64_MAX) {
            status = fail(ASGS_E_CAPACITY, "batch needs %llu bytes after counting", (unsigned long long)L2.total);
            b->bytes = 0;
          } else {
            b->off = off2;
            b->bytes = L2.total;
            b->capacity = cap2;
            L = L2;
          }
        }
      }
      if (!status) status = run_batch(S, *b, L);
    }
    b->status = status;
    lk.lock();
    S.inflight[si].push_back(b);
    S.cv_comp.notify_all();
  }
}

void completer(Server* Sp, int si) {
  Server& S = *Sp;
  if (!S.cfg.simulate) (void)hipSetDevice(S.device);
  std::unique_lock<std::mutex> lk(S.mu);
  for (;;) {
    S.cv_comp.wait(lk, [&] { return !S.inflight[si].empty() || (S.stop && S.queue.empty() && S.in_flight == 0); });
    if (S.inflight[si].empty()) break;
    Batch* b = S.inflight[si].front();
    lk.unlock();
    int status = b->status;
    if (S.cfg.simulate) {
      sleep_until_s(b->sim_done);
    } else if (status == ASGS_OK) {
      const hipError_t e = hipEventSynchronize(b->ev);
      if (e != hipSuccess) status = fail(ASGS_E_DEVICE, "batch: %s", hipGetErrorString(e));
    } else {
      (void)hipStreamSynchronize(S.streams[si]);
    }
    const double done = now_s();
    bool rerun = false;
    if (!S.cfg.simulate && status == ASGS_OK && b->hdr->overflow) rerun = true;
    lk.lock();
    S.inflight[si].pop_front();
    if (b->bytes) S.arena.release(b->off, b->bytes);
    S.busy[si] = false;
    --S.in_flight;
    if (!S.cfg.simulate && status == ASGS_OK) {
      const std::pair<int, int> key(b->cams[0].width, b->cams[0].height);
      auto& m = S.isect_per_view[key];
      m = std::max(m, (int64_t)((b->hdr->n_isect + b->V - 1) / b->V));
    }
    if (rerun) {
      ++S.st.reruns;
      for (size_t i = b->reqs.size(); i-- > 0;) {
        b->reqs[i]->exact = true;
        S.queue.push_front(b->reqs[i]);
      }
    } else {
      finish_requests(S, *b, done, status);
    }
    S.cv_done.notify_all();
    S.cv_sched.notify_all();
    delete b;
  }
}

int validate(const Server& S, const asgs_request* r) {
  if (!r) return fail(ASGS_E_INVALID, "request is NULL");
  if (r->kind != ASGS_REQ_TRACK && r->kind != ASGS_REQ_MAP) return fail(ASGS_E_INVALID, "unknown request kind");
  if (r->kind == ASGS_REQ_TRACK && r->n_views != 1) return fail(ASGS_E_INVALID, "tracking requests have one view");
  if (r->n_views < 1 || r->n_views > ASGS_MAX_VIEWS) return fail(ASGS_E_INVALID, "n_views out of range");
  if (!r->cams || !r->target_rgb || !r->target_depth || !r->d_pose)
    return fail(ASGS_E_INVALID, "cams, targets and d_pose are required");
  for (int v = 0; v < r->n_views; ++v) {
    if (r->cams[v].width != r->cams[0].width || r->cams[v].height != r->cams[0].height)
      return fail(ASGS_E_INVALID, "views of one request share a resolution");
    if (r->cams[v].width < 1 || r->cams[v].height < 1 || r->cams[v].width > 8192 || r->cams[v].height > 8192)
      return fail(ASGS_E_INVALID, "bad resolution");
    if (!r->target_rgb[v] || !r->target_depth[v]) return fail(ASGS_E_INVALID, "missing target of view %d", v);
    if (r->target_feat && !r->target_feat[v]) return fail(ASGS_E_INVALID, "missing feature target of view %d", v);
    if (r->out_rgb && !r->out_rgb[v]) return fail(ASGS_E_INVALID, "missing out_rgb of view %d", v);
    if (r->out_depth && !r->out_depth[v]) return fail(ASGS_E_INVALID, "missing out_depth of view %d", v);
  }
  if (r->out_depth && !r->out_rgb) return fail(ASGS_E_INVALID, "out_depth needs out_rgb");
  if (r->target_feat && S.dec.n_feat == 0) return fail(ASGS_E_INVALID, "feature targets without a feature head");
  if (r->kind == ASGS_REQ_MAP && (!r->d_xyz || !r->d_feat || !r->d_off || !r->d_params))
    return fail(ASGS_E_INVALID, "mapping requests need d_xyz, d_feat, d_off and d_params");
  return ASGS_OK;
}

}  // namespace

extern "C" {

double asgs_server_clock(void) { return now_s(); }

int asgs_server_create(const asgs_server_config* cfg, const asgs_decoder* d, const float* anchor_xyz,
                       const float* anchor_feat, const float* anchor_off, const float* params,
                       const asgs_render_opts* opts, void** server) {
  if (!cfg || !d || !opts || !server) return fail(ASGS_E_INVALID, "server_create: NULL argument");
  if (cfg->n_streams < 1 || cfg->n_streams > 8) return fail(ASGS_E_INVALID, "n_streams must be 1..8");
  if (cfg->max_batch_views < 1 || cfg->max_batch_views > ASGS_MAX_VIEWS)
    return fail(ASGS_E_INVALID, "max_batch_views must be 1..%d", ASGS_MAX_VIEWS);
  if (cfg->arena_bytes < (1u << 20)) return fail(ASGS_E_INVALID, "arena_bytes below 1 MiB");
  if (d->n_feat != opts->n_feat) return fail(ASGS_E_INVALID, "decoder and render options disagree on n_feat");
  int64_t np = 0;
  int st = asgs_decode_param_count(d, &np);
  if (st) return st;
  if (!cfg->simulate && (!anchor_xyz || !anchor_feat || !anchor_off || !params))
    return fail(ASGS_E_INVALID, "server_create: scene pointers are required");
  auto S = std::make_unique<Server>();
  S->cfg = *cfg;
  S->dec = *d;
  S->opts = *opts;
  S->xyz = anchor_xyz;
  S->feat = anchor_feat;
  S->off = anchor_off;
  S->params = params;
  S->N = d->n_anchors * d->k;
  S->n_params = np;
  S->arena = Arena(Arena::round(cfg->arena_bytes) == cfg->arena_bytes ? cfg->arena_bytes
                                                                       : cfg->arena_bytes & ~uint64_t(255));
  S->st.arena_bytes = S->arena.capacity();
  S->inflight.resize(cfg->n_streams);
  S->busy.assign(cfg->n_streams, false);
  if (!cfg->simulate) {
    if ((st = hip_check(hipGetDevice(&S->device), "hipGetDevice"))) return st;
    void* mem = nullptr;
    if ((st = hip_check(hipMalloc(&mem, S->arena.capacity()), "arena allocation"))) return st;
    S->base = static_cast<char*>(mem);
    for (int i = 0; i < cfg->n_streams && !st; ++i) {
      hipStream_t s = nullptr;
      hipEvent_t e = nullptr;
      void* h = nullptr;
      st = hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream create");
      if (!st) S->streams.push_back(s);
      if (!st) st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event create");
      if (!st) S->events.push_back(e);
      if (!st) st = hip_check(hipHostMalloc(&h, sizeof(asgs::CtxHeader), hipHostMallocDefault), "pinned header");
      if (!st) S->headers.push_back(static_cast<asgs::CtxHeader*>(h));
    }
    if (st) {
      for (auto x : S->streams) (void)hipStreamDestroy(x);
      for (auto e : S->events) (void)hipEventDestroy(e);
      for (auto h : S->headers) (void)hipHostFree(h);
      (void)hipFree(S->base);
      return st;
    }
  }
  Server* raw = S.release();
  raw->sched = std::thread(scheduler, raw);
  for (int i = 0; i < cfg->n_streams; ++i) raw->comp.emplace_back(completer, raw, i);
  *server = raw;
  return ASGS_OK;
}

int asgs_server_submit(void* server, const asgs_request* req, uint64_t* ticket) {
  Server* S = static_cast<Server*>(server);
  if (!S || !ticket) return fail(ASGS_E_INVALID, "server_submit: NULL argument");
  int st = validate(*S, req);
  if (st) return st;
  Req* r = new Req();
  r->r = *req;
  r->cams.assign(req->cams, req->cams + req->n_views);
  r->trgb.assign(req->target_rgb, req->target_rgb + req->n_views);
  r->tdepth.assign(req->target_depth, req->target_depth + req->n_views);
  if (req->target_feat) r->tfeat.assign(req->target_feat, req->target_feat + req->n_views);
  if (req->out_rgb) r->orgb.assign(req->out_rgb, req->out_rgb + req->n_views);
  if (req->out_depth) r->odepth.assign(req->out_depth, req->out_depth + req->n_views);
  if (r->r.arrival < 0) r->r.arrival = now_s();
  // pointers into caller arrays are not kept
  r->r.cams = nullptr;
  r->r.target_rgb = r->r.target_depth = r->r.target_feat = nullptr;
  r->r.out_rgb = r->r.out_depth = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete r;
      return fail(ASGS_E_INVALID, "server is stopping");
    }
    r->ticket = S->next_ticket++;
    S->live[r->ticket] = r;
    S->queue.push_back(r);
    ++S->st.submitted;
    *ticket = r->ticket;
  }
  S->cv_sched.notify_all();
  return ASGS_OK;
}

int asgs_server_wait(void* server, uint64_t ticket, asgs_result* result) {
  Server* S = static_cast<Server*>(server);
  if (!S || !result) return fail(ASGS_E_INVALID, "server_wait: NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  if (!S->results.count(ticket) && !S->live.count(ticket)) return fail(ASGS_E_INVALID, "unknown ticket %llu",
                                                                       (unsigned long long)ticket);
  S->cv_done.wait(lk, [&] { return S->results.count(ticket) > 0; });
  *result = S->results[ticket];
  S->results.erase(ticket);
  return ASGS_OK;
}

int asgs_server_replay(void* server, const asgs_request* reqs, int64_t n, asgs_result* results) {
  Server* S = static_cast<Server*>(server);
  if (!S || (n > 0 && (!reqs || !results))) return fail(ASGS_E_INVALID, "server_replay: NULL argument");
  for (int64_t i = 0; i < n; ++i) {
    int st = validate(*S, &reqs[i]);
    if (st) return st;
    if (i && reqs[i].arrival < reqs[i - 1].arrival) return fail(ASGS_E_INVALID, "arrivals must be ascending");
  }
  std::vector<uint64_t> tickets((size_t)n);
  const double t0 = now_s();
  for (int64_t i = 0; i < n; ++i) {
    asgs_request r = reqs[i];
    r.arrival = t0 + reqs[i].arrival;
    sleep_until_s(r.arrival);
    int st = asgs_server_submit(server, &r, &tickets[(size_t)i]);
    if (st) return st;
  }
  for (int64_t i = 0; i < n; ++i) {
    int st = asgs_server_wait(server, tickets[(size_t)i], &results[i]);
    if (st) return st;
  }
  return ASGS_OK;
}

int asgs_server_stats(void* server, asgs_server_stats_t* stats) {
  Server* S = static_cast<Server*>(server);
  if (!S || !stats) return fail(ASGS_E_INVALID, "server_stats: NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *stats = S->st;
  stats->arena_peak = S->arena.peak();
  return ASGS_OK;
}

int asgs_server_destroy(void* server) {
  Server* S = static_cast<Server*>(server);
  if (!S) return fail(ASGS_E_INVALID, "server_destroy: NULL");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_sched.notify_all();
  S->cv_comp.notify_all();
  S->sched.join();
  S->cv_comp.notify_all();
  for (auto& t : S->comp) t.join();
  for (auto& kv : S->live) delete kv.second;
  int st = ASGS_OK;
  if (!S->cfg.simulate) {
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    for (auto e : S->events) (void)hipEventDestroy(e);
    for (auto h : S->headers) (void)hipHostFree(h);
    if (S->base) st = hip_check(hipFree(S->base), "arena free");
  }
  delete S;
  return st;
}

}  // extern "C"
