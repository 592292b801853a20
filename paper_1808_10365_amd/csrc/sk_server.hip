// Continuous-batching server: admission by device-memory footprint, per-array
// ordering on per-array streams, overlap across arrays, event-driven completion.
#include <hip/hip_runtime.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "sk_internal.h"
#include "sk_server.h"

using namespace sk;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

struct Frame {
  sk_ticket_t ticket = 0;
  int32_t array_id = 0;
  const uint8_t* src = nullptr;
  int32_t on_host = 0;
  sk_outputs outs{};
  uint64_t tag = 0;
  size_t bytes = 0;          // footprint while in flight
  uint8_t* staging = nullptr;
  hipEvent_t ready_ev = nullptr;   // recorded on the submitter's stream: the frame is ready
  hipEvent_t done_ev = nullptr;
  sk_result res{};
};

struct Array {
  sk_plan_desc desc{};
  sk_plan_t plan = nullptr;
  int stream = 0;
  size_t in_bytes = 0, out_bytes = 0;
  int queued = 0;            // frames of this array waiting for admission
};

}  // namespace

struct sk_server_s {
  sk_server_desc d{};
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<Array> arrays;
  std::deque<std::unique_ptr<Frame>> queue;           // waiting, in arrival order
  std::vector<std::unique_ptr<Frame>> inflight;
  std::map<sk_ticket_t, sk_result> done;
  std::multimap<size_t, uint8_t*> staging_free;        // reusable staging buffers by size
  std::vector<uint8_t*> staging_all;
  std::vector<hipEvent_t> event_free;
  size_t bytes_inflight = 0;
  sk_ticket_t next_ticket = 1;
  sk_server_stats stats{};
  double busy_since = -1.0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  int fatal = 0;
};

static size_t output_bytes(const sk_plan_desc& d, const sk_outputs& o) {
  const size_t B = (size_t)(d.n_samples / d.block_len), F = d.n_channels, N = d.n_inputs;
  size_t b = 0;
  if (o.s1) b += F * B * N * 4;
  if (o.s2) b += F * B * N * 4;
  if (o.r1) b += F * B * 8;
  if (o.r2) b += F * B * 8;
  if (o.v) b += F * B * 4;
  if (o.flags) b += F * B;
  if (o.n_eff) b += F * B * 4;
  if (o.sk_i) b += F * B * N * 4;
  if (o.significance) b += F * B * 4;
  return b;
}

// Called with the lock held: move completed frames to `done`.
static void reap(sk_server_s* s) {
  for (size_t k = 0; k < s->inflight.size();) {
    Frame* f = s->inflight[k].get();
    hipError_t q = hipEventQuery(f->done_ev);
    if (q == hipErrorNotReady) { ++k; continue; }
    f->res.t_done = now_s();
    if (q != hipSuccess && f->res.status == SK_OK) f->res.status = SK_ERR_DEVICE;
    s->done[f->ticket] = f->res;
    s->bytes_inflight -= f->bytes;
    if (f->staging) s->staging_free.emplace(s->arrays[f->array_id].in_bytes, f->staging);
    s->event_free.push_back(f->done_ev);
    if (f->ready_ev) s->event_free.push_back(f->ready_ev);
    s->stats.completed += 1;
    s->inflight[k] = std::move(s->inflight.back());
    s->inflight.pop_back();
  }
  if (s->inflight.empty() && s->busy_since >= 0) {
    s->stats.busy_seconds += now_s() - s->busy_since;
    s->busy_since = -1.0;
  }
}

// Called with the lock held: admit queued frames in arrival order. A frame
// may pass an earlier frame of another array that does not fit, never one of
// its own array.
static void admit(sk_server_s* s) {
  std::vector<char> blocked(s->arrays.size(), 0);
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if ((int)s->inflight.size() >= s->d.max_inflight) break;
    Frame* f = it->get();
    Array& a = s->arrays[f->array_id];
    if (blocked[f->array_id] || s->bytes_inflight + f->bytes > s->d.hbm_budget_bytes) {
      blocked[f->array_id] = 1;
      ++it;
      continue;
    }
    hipStream_t st = s->streams[a.stream];
    int rc = SK_OK;
    if (f->ready_ev && hipStreamWaitEvent(st, f->ready_ev, 0) != hipSuccess) rc = SK_ERR_DEVICE;
    const uint8_t* x = f->src;
    if (f->on_host) {
      auto fb = s->staging_free.find(a.in_bytes);
      if (fb != s->staging_free.end()) {
        f->staging = fb->second;
        s->staging_free.erase(fb);
      } else if (hipMalloc((void**)&f->staging, a.in_bytes) == hipSuccess) {
        s->staging_all.push_back(f->staging);
      } else {
        f->staging = nullptr;
        blocked[f->array_id] = 1;     // no device memory now: retry after completions
        ++it;
        continue;
      }
      if (rc == SK_OK && hipMemcpyAsync(f->staging, f->src, a.in_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = SK_ERR_DEVICE;
      x = f->staging;
    }
    if (rc == SK_OK) rc = sk_compute(a.plan, x, nullptr, &f->outs, st);
    if (s->event_free.empty()) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) { s->fatal = SK_ERR_DEVICE; return; }
      s->event_free.push_back(e);
    }
    f->done_ev = s->event_free.back();
    s->event_free.pop_back();
    (void)hipEventRecord(f->done_ev, st);
    f->res.status = rc;
    f->res.t_admit = now_s();
    s->bytes_inflight += f->bytes;
    if (s->bytes_inflight > s->stats.peak_bytes) s->stats.peak_bytes = s->bytes_inflight;
    if (s->busy_since < 0) s->busy_since = f->res.t_admit;
    a.queued -= 1;
    s->inflight.push_back(std::move(*it));
    if ((int)s->inflight.size() > s->stats.peak_inflight) s->stats.peak_inflight = (int)s->inflight.size();
    it = s->queue.erase(it);
  }
}

static void worker_main(sk_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    reap(s);
    admit(s);
    s->cv_done.notify_all();
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    if (s->fatal) break;
    if (s->inflight.empty())
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    else
      s->cv_work.wait_for(lk, std::chrono::microseconds(10));
  }
  s->cv_done.notify_all();
}

extern "C" {

double sk_server_now(void) { return now_s(); }

int sk_server_create(const sk_server_desc* desc, sk_server_t* out) {
  clear_error();
  if (!desc || !out || desc->max_inflight < 1 || desc->n_streams < 1 || desc->n_streams > 64 ||
      desc->queue_capacity < 1 || desc->hbm_budget_bytes == 0) {
    set_error("bad server description");
    return SK_ERR_INVALID_ARG;
  }
  *out = nullptr;
  sk_server_s* s = new sk_server_s();
  s->d = *desc;
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; set_error("no HIP device"); return SK_ERR_DEVICE; }
  for (int k = 0; k < desc->n_streams; ++k) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      set_error("stream create failed");
      return SK_ERR_DEVICE;
    }
    s->streams.push_back(st);
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return SK_OK;
}

int sk_server_add_array(sk_server_t s, const sk_plan_desc* desc, int32_t* array_id) {
  clear_error();
  if (!s || !desc || !array_id) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(s->mu);
  Array a;
  a.desc = *desc;
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != s->device) (void)hipSetDevice(s->device);
  int rc = sk_plan_create(desc, &a.plan);
  if (dev != s->device && dev >= 0) (void)hipSetDevice(dev);
  if (rc) return rc;
  a.stream = (int)(s->arrays.size() % s->streams.size());
  a.in_bytes = (size_t)desc->n_samples * desc->n_channels * desc->n_inputs;
  *array_id = (int32_t)s->arrays.size();
  s->arrays.push_back(a);
  return SK_OK;
}

static hipEvent_t take_event(sk_server_s* s) {
  if (s->event_free.empty()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = s->event_free.back();
  s->event_free.pop_back();
  return e;
}

int sk_stream_submit(sk_server_t s, int32_t array_id, const uint8_t* frame, int32_t frame_on_host,
                     const sk_outputs* outs, uint64_t tag, void* ready_stream, sk_ticket_t* ticket) {
  clear_error();
  if (!s || !frame || !outs || !ticket) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  const double t = now_s();
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->fatal) { set_error("server stopped after a device error"); return s->fatal; }
  if (array_id < 0 || array_id >= (int32_t)s->arrays.size()) { set_error("unknown array %d", array_id); return SK_ERR_INVALID_ARG; }
  if ((int)s->queue.size() >= s->d.queue_capacity) { s->stats.rejected_full += 1; set_error("queue full"); return SK_ERR_AGAIN; }
  Array& a = s->arrays[array_id];
  auto f = std::make_unique<Frame>();
  f->ticket = s->next_ticket++;
  f->array_id = array_id;
  f->src = frame;
  f->on_host = frame_on_host;
  f->outs = *outs;
  f->tag = tag;
  f->bytes = a.in_bytes + output_bytes(a.desc, *outs);
  if (f->bytes > s->d.hbm_budget_bytes) { set_error("frame footprint %zu exceeds the budget", f->bytes); return SK_ERR_NOMEM; }
  f->res.tag = tag;
  f->res.array_id = array_id;
  f->res.status = SK_OK;
  f->res.t_submit = t;
  if (ready_stream) {
    // Work already enqueued on the submitter's stream (the producer of the
    // frame or of its output buffers) completes before the frame's work runs.
    f->ready_ev = take_event(s);
    if (!f->ready_ev || hipEventRecord(f->ready_ev, (hipStream_t)ready_stream) != hipSuccess) {
      if (f->ready_ev) s->event_free.push_back(f->ready_ev);
      set_error("event record on the ready stream failed");
      return SK_ERR_DEVICE;
    }
  }
  *ticket = f->ticket;
  a.queued += 1;
  s->queue.push_back(std::move(f));
  s->stats.submitted += 1;
  lk.unlock();
  s->cv_work.notify_one();
  return SK_OK;
}

int sk_stream_poll(sk_server_t s, sk_ticket_t ticket, sk_result* res) {
  if (!s || !res) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    *res = it->second;
    s->done.erase(it);
    return SK_OK;
  }
  if (ticket == 0 || ticket >= s->next_ticket) { set_error("unknown ticket"); return SK_ERR_INVALID_ARG; }
  for (const auto& f : s->queue) if (f->ticket == ticket) return SK_ERR_AGAIN;
  for (const auto& f : s->inflight) if (f->ticket == ticket) return SK_ERR_AGAIN;
  set_error("ticket already collected");
  return SK_ERR_INVALID_ARG;
}

int sk_server_drain(sk_server_t s) {
  if (!s) { set_error("NULL server"); return SK_ERR_INVALID_ARG; }
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [&] { return (s->queue.empty() && s->inflight.empty()) || s->fatal; });
  return s->fatal ? s->fatal : SK_OK;
}

int sk_server_get_stats(sk_server_t s, sk_server_stats* st) {
  if (!s || !st) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  if (s->busy_since >= 0) st->busy_seconds += now_s() - s->busy_since;
  return SK_OK;
}

int sk_server_destroy(sk_server_t s) {
  if (!s) return SK_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& a : s->arrays) sk_plan_destroy(a.plan);
  for (uint8_t* p : s->staging_all) (void)hipFree(p);
  for (hipEvent_t e : s->event_free) (void)hipEventDestroy(e);
  for (auto& f : s->inflight) {
    if (f->done_ev) (void)hipEventDestroy(f->done_ev);
    if (f->ready_ev) (void)hipEventDestroy(f->ready_ev);
  }
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return SK_OK;
}

}  // extern "C"
