/*
 * sk_server.h - continuous-batching server for spectral-kurtosis streams.
 *
 * Arrays of different sizes (each a plan description: N, F, frame length T,
 * M, window, estimator, flags; Sec. 2.2.1, Sec. 3.2) submit frames as they
 * arrive. A dispatcher thread admits queued frames whenever a slot and
 * device memory are free: a frame's footprint (input bytes, plus its staging
 * copy for host frames, plus output bytes) must fit the budget beside the
 * frames already in flight. Frames of one array run in submission order
 * (the running normaliser of that array depends on it) on that array's HIP
 * stream; frames of different arrays run on different streams and overlap on
 * the device. Each array's normaliser state stays in device memory between
 * frames. Completion is observed through HIP events and timestamped.
 *
 * All entry points are thread-safe. Errors as in sk.h.
 */
#ifndef SK_SERVER_H
#define SK_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "sk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sk_server_s* sk_server_t;
typedef uint64_t sk_ticket_t;

typedef struct {
  size_t hbm_budget_bytes;   /* device bytes for frames in flight (inputs, staging, outputs) */
  int32_t max_inflight;      /* frames on the device at once (slots) */
  int32_t n_streams;         /* HIP streams; array a uses stream a % n_streams */
  int32_t queue_capacity;    /* queued (not yet admitted) frames before submit returns SK_ERR_AGAIN */
} sk_server_desc;

typedef struct {
  uint64_t tag;              /* caller's tag from submit */
  int32_t array_id;
  int32_t status;            /* SK_OK or the error of the frame's launch */
  double t_submit;           /* monotonic host seconds at submit */
  double t_admit;            /* when the frame's work was enqueued on the device */
  double t_done;             /* when completion was observed */
} sk_result;

typedef struct {
  uint64_t submitted, completed, rejected_full;
  int32_t peak_inflight;
  size_t peak_bytes;
  double busy_seconds;       /* time with at least one frame in flight */
} sk_server_stats;

/* Monotonic host clock used for all timestamps (seconds). */
double sk_server_now(void);

int sk_server_create(const sk_server_desc* desc, sk_server_t* server);

/* Register an array; desc->n_samples is its frame length. Allocates the
 * array's scratch and normaliser state on the server's device. */
int sk_server_add_array(sk_server_t server, const sk_plan_desc* desc, int32_t* array_id);

/* Non-blocking submit of one frame [T][F][N]. frame_on_host = 0: device
 * memory, valid until the ticket completes; 1: host memory (pinned for an
 * asynchronous copy), copied into a staging buffer the server allocates
 * within its budget. outs: device buffers for this frame's results.
 * ready_stream (a hipStream_t, or NULL): work enqueued on it before this call
 * (writing the frame, or still using the output buffers) completes before
 * the frame's work starts; NULL means the frame and outputs are ready now.
 * SK_ERR_AGAIN when the queue is full. */
int sk_stream_submit(sk_server_t server, int32_t array_id, const uint8_t* frame, int32_t frame_on_host,
                     const sk_outputs* outs, uint64_t tag, void* ready_stream, sk_ticket_t* ticket);

/* SK_OK and *result once the ticket completed (the ticket is then
 * released); SK_ERR_AGAIN before that; SK_ERR_INVALID_ARG for unknown tickets. */
int sk_stream_poll(sk_server_t server, sk_ticket_t ticket, sk_result* result);

/* Block until every submitted frame has completed. */
int sk_server_drain(sk_server_t server);

int sk_server_get_stats(sk_server_t server, sk_server_stats* stats);

/* Drains, stops the dispatcher and frees everything. */
int sk_server_destroy(sk_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* SK_SERVER_H */
