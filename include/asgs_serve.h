/* libasgs request loop: continuous batching of tracking and mapping renders
 * over one device-resident anchor scene.
 *
 * The method alternates a tracking thread (per frame: render the map at the
 * current pose estimate and follow the pose gradient of the photometric,
 * depth and feature residuals, UP-SLAM Sec. 3.4) and a mapping thread (per
 * keyframe window: render several keyframes and follow the gradients of the
 * anchors and decoder MLPs, Sec. 3.3). This server runs both kinds of work as
 * requests against one scene that stays resident in HBM:
 *
 *  - ASGS_REQ_TRACK: one view; returns the SE(3) pose gradient (and loss) of
 *    the weighted L1 residual of rgb, depth and (when targets are given)
 *    features against the request's target maps.
 *  - ASGS_REQ_MAP: 1..ASGS_MAX_VIEWS keyframe views of one resolution;
 *    returns the same loss summed over its views, per-view pose gradients and
 *    the gradients of the anchors (xyz, feature, offsets) and of the packed
 *    head parameters.
 *
 * Loss of one view (H x W pixels, weight w_p, 1 when no weight map is given):
 *   L = sum_{c,p} w_p |rgb - rgb*| / (3HW) + sum_p w_p |D - D*| / (HW)
 *     [+ sum_{c,p} w_p |F - F*| / (16HW) with feature targets].
 *
 * Scheduling. A scheduler thread takes the oldest queued request; a tracking
 * request is fused with the other queued tracking requests of the same
 * resolution (arrival order, at most max_batch_views views) into one
 * multi-view batch: one decode launch, one sort and one blend launch per
 * kernel class for the whole batch. A mapping request is its own batch. A
 * batch is admitted when one of the n_streams HIP streams is free and its
 * device memory fits in the free part of the server's arena (first fit);
 * otherwise it waits for completions. Batches on different streams overlap
 * on the device. Intersection capacity is reserved from the largest
 * per-view count seen so far for that resolution (with 25% slack; the first
 * batch of a resolution counts exactly); a batch whose count exceeds its
 * reservation is detected at completion and run again with the exact size.
 *
 * Every result is independent of the batch it ran in: the kernels treat the
 * views of a batch independently and sum in an order fixed by the view alone,
 * so a request's outputs are bitwise the same alone and in the mix.
 *
 * Memory: the arena is one device allocation made by asgs_server_create;
 * requests allocate nothing. Request inputs and outputs are caller-owned
 * device buffers that must stay valid until the request completes.
 *
 * Threads: submit and wait may be called from any thread. Times are seconds
 * of the server's monotonic clock (asgs_server_clock).
 * ------------------------------------------------------------------------- */
#ifndef ASGS_SERVE_H
#define ASGS_SERVE_H

#include "asgs.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { ASGS_REQ_TRACK = 0, ASGS_REQ_MAP = 1 };

typedef struct asgs_server_config {
  int32_t n_streams;        /* batches in flight (HIP streams, default priority), 1..8 */
  int32_t max_batch_views;  /* views per fused tracking batch, 1..ASGS_MAX_VIEWS (1 = no fusion) */
  int32_t fifo;             /* 1: admit a batch only when no other is in flight */
  int32_t simulate;         /* 1: no device work; a batch takes sim_us_per_mpix per megapixel
                               plus sim_us_fixed (scheduler tests without a GPU) */
  uint64_t arena_bytes;     /* device memory for in-flight batches (the admission budget) */
  float sim_us_per_mpix;
  float sim_us_fixed;
} asgs_server_config;

typedef struct asgs_request {
  int32_t kind;                        /* ASGS_REQ_TRACK or ASGS_REQ_MAP */
  int32_t n_views;                     /* 1 for TRACK; 1..ASGS_MAX_VIEWS for MAP */
  const asgs_camera* cams;             /* host [n_views], one resolution (copied at submit) */
  const float* const* target_rgb;      /* host [n_views] of device [3][H][W] */
  const float* const* target_depth;    /* host [n_views] of device [H][W] */
  const float* const* target_feat;     /* host [n_views] of device [16][H][W], or NULL (no feature term) */
  const float* weight;                 /* device [H][W] per-pixel weight shared by the views, or NULL */
  float* d_pose;                       /* device [n_views][6] out: dL/dxi (left perturbation), required */
  float* loss;                         /* device [n_views] out, or NULL */
  float* d_xyz;                        /* MAP: device [3][A] out (required for MAP) */
  float* d_feat;                       /* MAP: device [A][32] out */
  float* d_off;                        /* MAP: device [3][A*k] out */
  float* d_params;                     /* MAP: device packed head parameters out */
  float* const* out_rgb;               /* optional host [n_views] of device [3][H][W] (rendered maps), or NULL */
  float* const* out_depth;             /* optional, with out_rgb */
  double arrival;                      /* server clock seconds; < 0 = time of submit */
} asgs_request;

typedef struct asgs_result {
  int32_t status;       /* ASGS_OK or the error of the batch */
  int32_t batch_views;  /* views of the batch that served the request */
  int32_t stream;       /* stream index it ran on */
  int32_t attempts;     /* 1, or 2 after a capacity re-run */
  double arrival, start, done;  /* server clock seconds: arrival, batch launch, completion seen */
} asgs_result;

typedef struct asgs_server_stats {
  int64_t submitted, completed, failed;
  int64_t batches, batch_views, reruns;
  uint64_t arena_bytes, arena_peak;   /* budget and the largest amount in use at once */
  int32_t max_in_flight;              /* most batches in flight at once */
  int32_t reserved;
} asgs_server_stats_t;

/* Create a server over a resident scene: decoder d (n_anchors, k, n_feat,
 * precision), anchor tensors and packed parameters on the device (owned by
 * the caller, read-only while the server lives), render options opts. Makes
 * the arena allocation and starts the scheduler and completion threads. */
int asgs_server_create(const asgs_server_config* cfg, const asgs_decoder* d, const float* anchor_xyz,
                       const float* anchor_feat, const float* anchor_off, const float* params,
                       const asgs_render_opts* opts, void** server);

/* Monotonic clock in seconds (the time base of arrival/start/done). */
double asgs_server_clock(void);

/* Queue a request; returns at once with a ticket. Validation errors are
 * returned here and queue nothing. */
int asgs_server_submit(void* server, const asgs_request* req, uint64_t* ticket);

/* Wait for a ticket (blocking) and return its result; each ticket is waited
 * for at most once. */
int asgs_server_wait(void* server, uint64_t ticket, asgs_result* result);

/* Replay an arrival trace: request i is submitted at time t0 + reqs[i].arrival
 * (t0 = the call's start, arrivals ascending), then all are waited for;
 * results[i] gets request i's result with absolute times. */
int asgs_server_replay(void* server, const asgs_request* reqs, int64_t n, asgs_result* results);

int asgs_server_stats(void* server, asgs_server_stats_t* stats);

/* Drain (wait for every queued request), stop the threads, free the arena. */
int asgs_server_destroy(void* server);

#ifdef __cplusplus
}
#endif

#endif /* ASGS_SERVE_H */
