// C ABI: plans, validation, device memory ownership, normaliser state.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "sk_internal.h"
#include "sk_profile.h"
#include <vector>

namespace sk {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

void clear_error() { g_err.clear(); }

}  // namespace sk

using namespace sk;

struct sk_plan_s {
  sk_plan_desc d;
  int device;
  int64_t n_blocks;        // B = T / M
  int32_t hist_cap;        // max(L - 1, 0)
  int32_t hist_len;        // history blocks currently held (<= hist_cap)
  int32_t chunk;           // R
  int32_t n_chunks_max;    // chunks of the sequence when the history is full
  int32_t s1_s2_owned;
  int32_t* s1;             // [F][B][N] scratch
  int32_t* s2;
  int32_t* chunk_sum;      // [F][n_chunks_max][N]
  double* part_a;          // [F][n_groups_max][B] per-group partial sums of pass B
  double* part_q;
  int64_t* part_r1;
  int64_t* part_r2;
  int32_t* part_n;
  int32_t* hist[2];        // [F][hist_cap][N], ping-pong
  int32_t* seg_sum = nullptr;   // single-launch path: [n_cu][F*N] segment sums
  int32_t* seg_pre = nullptr;   //   [n_cu][F*N] exclusive prefixes over segments
  int32_t* hist_suf = nullptr;  //   [hist_cap][F*N] history suffix sums
  int fused_mode = 0;      // 1: single launch wherever the shape allows
  int last_fused = 0;      // whether the last call ran the single-launch path
  int fused_max_wg = 0;    // co-resident workgroups of the single-launch kernel
  int32_t cur;             // index of the live history buffer
  size_t bytes;
  int pass_a_lpr;          // 0 = heuristic
  int pass_a_variant = -1; // row batching variant of pass A; -1 = heuristic
  int pass_a_grid;         // 0 = one workgroup per task
  int pass_b_vec;          // 0 = library choice, else 1 or 4 inputs per lane
  int segments = 0;        // block segments per call (0 = library choice, 1 = none)
  int pass_b_depth = 0;    // blocks a partial wavefront loads together (0 = library choice)
  int pass_a_blocks = 0;   // consecutive blocks per pass A task (packed variants; 0 = library choice)
  int n_cu = 256;          // compute units of the plan's device
  int last_segments = 0;   // segments the last call used
  hipStream_t side = nullptr;          // pass B of segmented calls
  std::vector<hipEvent_t> seg_ev;      // pass A segment k done (on the caller's stream); last: join
  std::vector<hipEvent_t> prof;   // 3 events per recorded call
  double* thresholds;             // [N + 1][2] false-alarm thresholds by N_eff, or null
  double fap;
  int32_t prof_max, prof_n;
  int32_t prof_stride = 1, prof_calls = 0;   // record every prof_stride-th call
};

static const uint32_t kStateMagic = 0x534B5354u;  // "SKST"

struct StateHeader {
  uint32_t magic;
  uint32_t version;
  int32_t n_inputs, n_channels, block_len, window, hist_len, pad;
};

namespace sk {
int validate_desc(const sk_plan_desc* d) {
  if (!d) { set_error("desc is NULL"); return SK_ERR_INVALID_ARG; }
  if (d->n_inputs < 1 || d->n_inputs > 16384) { set_error("n_inputs %d outside [1, 16384]", d->n_inputs); return SK_ERR_SHAPE; }
  if (d->n_channels < 1) { set_error("n_channels %d < 1", d->n_channels); return SK_ERR_SHAPE; }
  if (d->block_len < 2 || d->block_len > 131071) { set_error("block_len %d outside [2, 131071]", d->block_len); return SK_ERR_SHAPE; }
  if (d->n_samples < 0 || d->n_samples % d->block_len != 0) { set_error("n_samples %lld is not a non-negative multiple of block_len %d", (long long)d->n_samples, d->block_len); return SK_ERR_SHAPE; }
  if (d->norm_window_blocks < 0 || (int64_t)d->norm_window_blocks * d->block_len * 128 >= (1LL << 31)) { set_error("norm_window_blocks %d: window power sum must fit int32", d->norm_window_blocks); return SK_ERR_SHAPE; }
  if (d->estimator != SK_EST_HAT && d->estimator != SK_EST_TILDE) { set_error("unknown estimator %d", d->estimator); return SK_ERR_INVALID_ARG; }
  if (d->estimator == SK_EST_TILDE && d->norm_window_blocks != 1) { set_error("the rescaled estimator needs norm_window_blocks == 1"); return SK_ERR_INVALID_ARG; }
  if (!(d->k_sigma >= 0.0)) { set_error("k_sigma must be >= 0"); return SK_ERR_INVALID_ARG; }
  const int64_t cells = (int64_t)d->n_channels * d->n_samples * d->n_inputs;
  if (cells < 0 || (double)d->n_channels * (double)d->n_samples * (double)d->n_inputs > 9.0e18) { set_error("input too large"); return SK_ERR_SHAPE; }
  return SK_OK;
}
}  // namespace sk

static int32_t pow2_floor(int64_t v) {
  int32_t r = 1;
  while ((int64_t)r * 2 <= v && r < (1 << 30)) r *= 2;
  return r;
}

static void free_profile(sk_plan_s* p) {
  for (hipEvent_t e : p->prof) (void)hipEventDestroy(e);
  p->prof.clear();
  p->prof_max = p->prof_n = 0;
}

static void free_plan_memory(sk_plan_s* p) {
  free_profile(p);
  for (hipEvent_t e : p->seg_ev) (void)hipEventDestroy(e);
  p->seg_ev.clear();
  if (p->side) (void)hipStreamDestroy(p->side);
  p->side = nullptr;
  if (p->thresholds) (void)hipFree(p->thresholds);
  if (p->s1_s2_owned) {
    if (p->s1) (void)hipFree(p->s1);
    if (p->s2) (void)hipFree(p->s2);
  }
  if (p->chunk_sum) (void)hipFree(p->chunk_sum);
  if (p->part_a) (void)hipFree(p->part_a);
  if (p->part_q) (void)hipFree(p->part_q);
  if (p->part_r1) (void)hipFree(p->part_r1);
  if (p->part_r2) (void)hipFree(p->part_r2);
  if (p->part_n) (void)hipFree(p->part_n);
  if (p->hist[0]) (void)hipFree(p->hist[0]);
  if (p->hist[1]) (void)hipFree(p->hist[1]);
  if (p->seg_sum) (void)hipFree(p->seg_sum);
  if (p->seg_pre) (void)hipFree(p->seg_pre);
  if (p->hist_suf) (void)hipFree(p->hist_suf);
}

#define SK_ALLOC(ptr, nbytes)                                                     \
  do {                                                                            \
    size_t nb_ = (nbytes);                                                        \
    if (nb_ > 0) {                                                                \
      hipError_t e_ = hipMalloc((void**)&(ptr), nb_);                             \
      if (e_ != hipSuccess) {                                                     \
        set_error("hipMalloc(%zu) failed: %s", nb_, hipGetErrorString(e_));       \
        free_plan_memory(p);                                                      \
        delete p;                                                                 \
        return SK_ERR_NOMEM;                                                      \
      }                                                                           \
      p->bytes += nb_;                                                            \
    }                                                                             \
  } while (0)

extern "C" {

const char* sk_last_error(void) { return g_err.c_str(); }

int sk_plan_create(const sk_plan_desc* desc, sk_plan_t* out) {
  clear_error();
  if (!out) { set_error("out is NULL"); return SK_ERR_INVALID_ARG; }
  *out = nullptr;
  int rc = validate_desc(desc);
  if (rc) return rc;
  sk_plan_s* p = new (std::nothrow) sk_plan_s();
  if (!p) { set_error("host allocation failed"); return SK_ERR_NOMEM; }
  p->d = *desc;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; set_error("no HIP device"); return SK_ERR_DEVICE; }
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && ncu > 0)
      p->n_cu = ncu;
  }
  const int64_t N = desc->n_inputs, F = desc->n_channels;
  p->n_blocks = desc->n_samples / desc->block_len;
  const int L = desc->norm_window_blocks;
  p->hist_cap = L >= 2 ? L - 1 : 0;
  p->hist_len = 0;
  // Chunk length R: a wavefront of the partial kernel reads about L/R chunk
  // sums to start its window and 3R rows in its main loop, so R near
  // sqrt(L) keeps the start-up cost small; R shrinks while there are too few
  // wavefronts to fill the device.
  const int64_t seq = p->hist_cap + p->n_blocks;
  const int64_t groups = (N + 63) / 64;   // upper bound (1 input per lane)
  int32_t R = 1, R_min = 1;
  if (L >= 2) {
    while (R < 64 && (int64_t)R * R * 2 < L) R *= 2;          // L/R <= 2R
    while (R_min < R && (int64_t)R_min * R_min * 8 < L) R_min *= 2;   // L/R <= 8R
  } else {
    R = 16;
  }
  while (R > R_min && ((seq + R - 1) / R) * F * ((N + 255) / 256) < 2048) R /= 2;
  p->chunk = R;
  p->n_chunks_max = (int32_t)((seq + R - 1) / R);
  p->s1_s2_owned = 1;
  const size_t fbn = (size_t)F * p->n_blocks * N;
  SK_ALLOC(p->s1, fbn * sizeof(int32_t));
  SK_ALLOC(p->s2, fbn * sizeof(int32_t));
  const size_t fgb = (size_t)F * groups * p->n_blocks;
  SK_ALLOC(p->part_a, fgb * sizeof(double));
  SK_ALLOC(p->part_q, fgb * sizeof(double));
  SK_ALLOC(p->part_r1, fgb * sizeof(int64_t));
  SK_ALLOC(p->part_r2, fgb * sizeof(int64_t));
  SK_ALLOC(p->part_n, fgb * sizeof(int32_t));
  if (L >= 2) {
    SK_ALLOC(p->chunk_sum, (size_t)F * p->n_chunks_max * N * sizeof(int32_t));
    SK_ALLOC(p->hist[0], (size_t)F * p->hist_cap * N * sizeof(int32_t));
    SK_ALLOC(p->hist[1], (size_t)F * p->hist_cap * N * sizeof(int32_t));
  }
  p->cur = 0;
  *out = p;
  return SK_OK;
}

int sk_plan_destroy(sk_plan_t p) {
  clear_error();
  if (!p) return SK_OK;
  (void)hipDeviceSynchronize();
  free_plan_memory(p);
  delete p;
  return SK_OK;
}

int sk_plan_device_bytes(sk_plan_t p, size_t* bytes) {
  if (!p || !bytes) { set_error("NULL argument"); return SK_ERR_INVALID_ARG; }
  *bytes = p->bytes;
  return SK_OK;
}

// Internal: force pass A lanes-per-row (autotuner and tests); 0 = heuristic.
int sk_plan_set_pass_a_tile(sk_plan_t p, int32_t lpr) {
  if (!p || (lpr != 0 && (lpr < 1 || lpr > 1024 || (lpr & (lpr - 1))))) { set_error("bad tile"); return SK_ERR_INVALID_ARG; }
  p->pass_a_lpr = lpr;
  return SK_OK;
}

static PassAConfig plan_pass_a_config(const sk_plan_s* p, const uint8_t* d_packed, PassATask* t) {
  const int64_t N = p->d.n_inputs, F = p->d.n_channels, B = p->n_blocks;
  const int vec = pick_vec(d_packed, (int32_t)N);
  t->row_bytes = F * N;
  t->n_inputs = (int32_t)N;
  t->block0 = 0;
  t->block_end = (int32_t)B;
  t->blocks_per_task = 1;
  t->block_len = p->d.block_len;
  t->n_blocks = (int32_t)B;
  PassAConfig c = default_pass_a_config(vec, t->row_bytes, B, p->d.block_len, p->pass_a_lpr == 0 && p->pass_a_variant < 0,
                                        p->n_cu);
  if (p->pass_a_lpr) c.lpr = p->pass_a_lpr;
  if (p->pass_a_variant >= 0) c.variant = p->pass_a_variant;
  {
    int lo, hi;
    pass_a_lane_range(vec, c.variant, &lo, &hi);
    if (c.lpr < lo) c.lpr = lo;
    if (c.lpr > hi) c.lpr = hi;
  }
  const int gpl = pass_a_groups_per_lane(vec, c.variant);
  t->col_groups = (int32_t)(t->row_bytes / vec);
  t->chunks = (t->col_groups + c.lpr * gpl - 1) / (c.lpr * gpl);
  if (pass_a_packed(vec, c.variant) && p->pass_a_blocks > 1) t->blocks_per_task = p->pass_a_blocks;
  if (pass_a_deferred(vec, c.variant)) {
    c.lpr = 512;
    t->chunks = (t->col_groups + 511) / 512;
    t->blocks_per_task = p->pass_a_blocks >= 1 && p->pass_a_blocks <= 4
                             ? p->pass_a_blocks : pass_a_deferred_blocks(B, t->col_groups, p->n_cu);
  }
  if (pass_a_side_by_side(vec, c.variant)) {
    c.lpr = pass_a_side_by_side_lanes(t->col_groups);
    t->blocks_per_task = c.lpr >= 256 ? 1 : 256 / c.lpr;
    t->chunks = c.lpr >= 256 ? (t->col_groups + 255) / 256 : 1;
  }
  t->n_tasks = ((B + t->blocks_per_task - 1) / t->blocks_per_task) * t->chunks;
  c.grid = (int)(t->n_tasks < (1 << 30) ? t->n_tasks : (1 << 30));
  if (p->pass_a_grid > 0 && p->pass_a_grid < c.grid) c.grid = p->pass_a_grid;
  return c;
}

int sk_plan_set_pass_a_variant(sk_plan_t p, int32_t variant, int32_t grid) {
  if (!p || variant < -1 || variant > 17 || grid < 0) { set_error("bad variant"); return SK_ERR_INVALID_ARG; }
  p->pass_a_variant = variant;
  p->pass_a_grid = grid;
  return SK_OK;
}

int sk_plan_set_segments(sk_plan_t p, int32_t segments) {
  clear_error();
  if (!p || segments < 0 || segments > 64) { set_error("segments must be in 0..64"); return SK_ERR_INVALID_ARG; }
  p->segments = segments;
  return SK_OK;
}

int sk_plan_set_pass_a_blocks(sk_plan_t p, int32_t blocks) {
  clear_error();
  if (!p || blocks < 0 || blocks > 4096) { set_error("blocks per task must be in 0..4096"); return SK_ERR_INVALID_ARG; }
  p->pass_a_blocks = blocks;
  return SK_OK;
}

int sk_plan_set_pass_b_depth(sk_plan_t p, int32_t depth) {
  clear_error();
  if (!p || (depth != 0 && depth != 2 && depth != 4 && depth != 8)) { set_error("depth must be 0, 2, 4 or 8"); return SK_ERR_INVALID_ARG; }
  p->pass_b_depth = depth;
  return SK_OK;
}

int sk_plan_set_fused(sk_plan_t p, int32_t mode) {
  clear_error();
  if (!p || mode < 0 || mode > 1) { set_error("mode must be 0 or 1"); return SK_ERR_INVALID_ARG; }
  if (mode == 1) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
      set_error("plan was created on device %d, current device is %d", p->device, dev);
      return SK_ERR_INVALID_ARG;
    }
  }
  p->fused_mode = mode;
  const int64_t F = p->d.n_channels, N = p->d.n_inputs;
  // Scratch of the single-launch path, allocated the first time it is
  // switched on for a shape it serves: wide rows covered by one 512-lane
  // workgroup, whole channels per wavefront, at most 4 blocks per workgroup
  // in one round of the CUs, a window of at least 2 blocks.
  if (mode == 1 && !p->seg_sum && p->d.norm_window_blocks >= 2 && N % 1024 == 0 && (F * N) / 16 <= 512 &&
      p->n_blocks <= 4 * (int64_t)p->n_cu) {
    const size_t seg = (size_t)p->n_cu * F * N * sizeof(int32_t);
    const size_t suf = (size_t)p->hist_cap * F * N * sizeof(int32_t);
    int32_t *a = nullptr, *b = nullptr, *c = nullptr;
    hipError_t e = hipMalloc((void**)&a, seg);
    if (e == hipSuccess) e = hipMalloc((void**)&b, seg);
    if (e == hipSuccess) e = hipMalloc((void**)&c, suf);
    if (e != hipSuccess) {
      if (a) (void)hipFree(a);
      if (b) (void)hipFree(b);
      if (c) (void)hipFree(c);
      p->fused_mode = 0;
      set_error("hipMalloc for the single-launch path failed: %s", hipGetErrorString(e));
      return SK_ERR_NOMEM;
    }
    p->seg_sum = a;
    p->seg_pre = b;
    p->hist_suf = c;
    p->bytes += 2 * seg + suf;
  }
  if (mode == 1 && p->fused_max_wg == 0) p->fused_max_wg = fused_max_workgroups();
  return SK_OK;
}

int sk_plan_get_last_fused(sk_plan_t p, int32_t* fused) {
  clear_error();
  if (!p || !fused) { set_error("NULL argument"); return SK_ERR_INVALID_ARG; }
  *fused = p->last_fused;
  return SK_OK;
}

int sk_plan_get_last_segments(sk_plan_t p, int32_t* segments) {
  clear_error();
  if (!p || !segments) { set_error("NULL argument"); return SK_ERR_INVALID_ARG; }
  *segments = p->last_segments;
  return SK_OK;
}

int sk_plan_set_pass_b_tile(sk_plan_t p, int32_t chunk, int32_t vec) {
  clear_error();
  if (!p || chunk < 0 || chunk > 1024 || (chunk & (chunk - 1)) || (vec != 0 && vec != 1 && vec != 4 && vec != 8)) {
    set_error("bad pass B tile");
    return SK_ERR_INVALID_ARG;
  }
  if (chunk > 0 && chunk != p->chunk) {
    const int64_t seq = p->hist_cap + p->n_blocks;
    const int32_t n_max = (int32_t)((seq + chunk - 1) / chunk);
    if (p->d.norm_window_blocks >= 2 && n_max > p->n_chunks_max) {
      int32_t* cs = nullptr;
      SK_HIP_TRY(hipDeviceSynchronize());
      SK_HIP_TRY(hipMalloc((void**)&cs, (size_t)p->d.n_channels * n_max * p->d.n_inputs * sizeof(int32_t)));
      if (p->chunk_sum) (void)hipFree(p->chunk_sum);
      p->chunk_sum = cs;
      p->n_chunks_max = n_max;
    }
    p->chunk = chunk;
  }
  p->pass_b_vec = vec;
  return SK_OK;
}

int sk_plan_get_pass_a_tile(sk_plan_t p, const uint8_t* d_packed, int32_t* vec, int32_t* lpr, int64_t* wgs) {
  if (!p || !vec || !lpr || !wgs) { set_error("NULL argument"); return SK_ERR_INVALID_ARG; }
  PassATask t;
  PassAConfig c = plan_pass_a_config(p, d_packed, &t);
  *vec = c.vec;
  *lpr = c.lpr;
  *wgs = c.grid;
  return SK_OK;
}

int sk_profile_enable(sk_plan_t p, int32_t max_records) {
  clear_error();
  if (!p || max_records < 0) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  free_profile(p);
  if (max_records == 0) return SK_OK;
  p->prof.resize((size_t)max_records * 3);
  for (auto& e : p->prof) SK_HIP_TRY(hipEventCreate(&e));
  p->prof_max = max_records;
  p->prof_n = 0;
  p->prof_stride = 1;
  p->prof_calls = 0;
  return SK_OK;
}

int sk_profile_set_stride(sk_plan_t p, int32_t stride) {
  clear_error();
  if (!p || stride < 1) { set_error("stride must be at least 1"); return SK_ERR_INVALID_ARG; }
  p->prof_stride = stride;
  p->prof_calls = 0;
  return SK_OK;
}

int sk_profile_read(sk_plan_t p, float* ms_a, float* ms_b, int32_t cap, int32_t* n) {
  clear_error();
  if (!p || !n || (cap > 0 && (!ms_a || !ms_b))) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  const int32_t m = p->prof_n < cap ? p->prof_n : cap;
  for (int32_t j = 0; j < m; ++j) {
    SK_HIP_TRY(hipEventSynchronize(p->prof[3 * j + 2]));
    SK_HIP_TRY(hipEventElapsedTime(&ms_a[j], p->prof[3 * j], p->prof[3 * j + 1]));
    SK_HIP_TRY(hipEventElapsedTime(&ms_b[j], p->prof[3 * j + 1], p->prof[3 * j + 2]));
  }
  *n = m;
  p->prof_n = 0;
  return SK_OK;
}

int sk_compute(sk_plan_t p, const uint8_t* d_packed, const uint8_t* d_mask, const sk_outputs* outs,
               void* stream) {
  clear_error();
  if (!p || !outs) { set_error("NULL plan or outputs"); return SK_ERR_INVALID_ARG; }
  if (!d_packed && p->d.n_samples > 0) { set_error("NULL input"); return SK_ERR_INVALID_ARG; }
  int dev = -1;
  SK_HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) { set_error("plan was created on device %d, current device is %d", p->device, dev); return SK_ERR_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  const sk_plan_desc& d = p->d;
  const int64_t N = d.n_inputs, F = d.n_channels, B = p->n_blocks;
  if (B == 0) return SK_OK;

  int32_t* s1 = outs->s1 ? outs->s1 : p->s1;
  int32_t* s2 = outs->s2 ? outs->s2 : p->s2;

  PassATask t;
  PassAConfig c = plan_pass_a_config(p, d_packed, &t);
  t.x = d_packed;
  t.s1 = s1;
  t.s2 = s2;

  PassBArgs a;
  memset(&a, 0, sizeof a);
  a.s1 = s1;
  a.s2 = s2;
  a.hist = p->hist[p->cur];
  a.hist_next = p->hist[1 - p->cur];
  a.chunk_sum = p->chunk_sum;
  a.part_a = p->part_a;
  a.part_q = p->part_q;
  a.part_r1 = p->part_r1;
  a.part_r2 = p->part_r2;
  a.part_n = p->part_n;
  a.mask = d_mask;
  a.r1 = outs->r1;
  a.r2 = outs->r2;
  a.v = outs->v;
  a.flags = outs->flags;
  a.n_eff = outs->n_eff;
  a.sk_i = outs->sk_i;
  a.significance = outs->significance;
  a.thresholds = p->thresholds;
  a.n_inputs = (int32_t)N;
  a.n_channels = (int32_t)F;
  a.n_blocks = (int32_t)B;
  a.block_len = d.block_len;
  a.window = d.norm_window_blocks;
  a.hist_len = p->hist_len;
  a.hist_cap = p->hist_cap;
  {
    const int64_t total = p->hist_len + B;
    a.hist_next_len = (int32_t)(total < p->hist_cap ? total : p->hist_cap);
  }
  a.chunk = p->chunk;
  a.n_chunks = (int32_t)((p->hist_len + B + p->chunk - 1) / p->chunk);
  // Four inputs per lane need 16-byte aligned rows of the sums.
  a.vec = pass_b_vec((int32_t)N);
  if (((uintptr_t)s1 | (uintptr_t)s2 | (uintptr_t)outs->sk_i) % 16 != 0) a.vec = 1;
  if (p->pass_b_vec == 1) a.vec = 1;
  if (p->pass_b_vec == 8 && a.vec == 4 && N % 8 == 0 && ((uintptr_t)s1 | (uintptr_t)s2 | (uintptr_t)outs->sk_i) % 32 == 0)
    a.vec = 8;
  a.n_groups = (int32_t)((N + 64 * a.vec - 1) / (64 * a.vec));
  a.depth = p->pass_b_depth ? p->pass_b_depth : 4;
  a.estimator = d.estimator;
  a.k_sigma = d.k_sigma;
  a.expect_offset = d.expect_offset;
  a.sigma_override = d.sigma_override;

  // Segments: pass B of blocks [b_k, b_k+1) needs S1 of those blocks and of
  // earlier ones only, so it can run on a second stream while pass A streams
  // the next segment. Boundaries sit on chunk boundaries of the sequence
  // (history + this call), so each segment's chunk sums read finished rows.
  int K = p->segments;
  // Library choice: one segment. Measured on MI355X (CHIME shapes), every
  // extra pass A launch adds a drain of its last workgroups (each streams
  // about 1 MiB, tens of microseconds) while pass B, latency-bound, takes
  // nearly as long for a quarter of the blocks as for all of them.
  if (K == 0) K = 1;
  if (K > a.n_chunks) K = a.n_chunks;
  if (K > 1 && !p->side) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SK_HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) {
      K = 1;   // no stream creation under capture; later calls segment
    } else {
      SK_HIP_TRY(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    }
  }
  if (K > 1 && (int)p->seg_ev.size() < K + 1) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SK_HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) {
      K = 1;
    } else {
      while ((int)p->seg_ev.size() < K + 1) {
        hipEvent_t e;
        SK_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->seg_ev.push_back(e);
      }
    }
  }

  p->last_segments = K < 1 ? 1 : K;
  const bool rec = p->prof_n < p->prof_max && (p->prof_calls++ % p->prof_stride) == 0;
  if (rec) SK_HIP_TRY(hipEventRecord(p->prof[3 * p->prof_n], s));
  int rc = SK_OK;

  // Single launch when it is switched on and the shape allows it. Off by
  // default: the two grid-wide barriers it needs cost more than the launches
  // and the S1/S2 re-read that it saves.
  const int fq = (int)((B + p->n_cu - 1) / p->n_cu);
  bool fused = p->fused_mode != 0 && K <= 1 && p->seg_sum && c.vec == 16 && d.norm_window_blocks >= 2 &&
               fq >= 1 && fq <= 4;
  if (fused) {
    const int grid = (int)((B + fq - 1) / fq);
    if (grid > p->fused_max_wg) fused = false;
  }
  p->last_fused = fused ? 1 : 0;
  if (fused) {
    FusedArgs fa;
    memset(&fa, 0, sizeof fa);
    fa.a = t;
    fa.a.s2 = outs->s2;           // S2 in memory only when requested
    fa.b = a;
    fa.b.chunk0 = 0;
    fa.b.fin_b0 = 0;
    fa.b.fin_nb = (int32_t)B;
    fa.segsum = p->seg_sum;
    fa.segpre = p->seg_pre;
    fa.hsuf = p->hist_suf;
    rc = launch_fused(fa, fq, s);
    if (rc) return rc;
    if (rec) SK_HIP_TRY(hipEventRecord(p->prof[3 * p->prof_n + 1], s));
  } else if (K <= 1) {
    rc = launch_pass_a(t, c, s);
    if (rc) return rc;
    if (rec) SK_HIP_TRY(hipEventRecord(p->prof[3 * p->prof_n + 1], s));
    rc = launch_pass_b(a, s);
    if (rc) return rc;
  } else {
    const int64_t H = p->hist_len, R = p->chunk;
    int32_t c_prev = 0;
    int32_t b_prev = 0;
    for (int k = 0; k < K; ++k) {
      int32_t c_next = a.n_chunks;
      if (k + 1 < K) {
        const int64_t target = H + (int64_t)B * (k + 1) / K;     // sequence position
        int64_t cn = (target + R / 2) / R;
        if (cn < c_prev) cn = c_prev;
        if (cn > a.n_chunks) cn = a.n_chunks;
        c_next = (int32_t)cn;
      }
      int64_t bn = (int64_t)c_next * R - H;
      if (k + 1 == K || bn > B) bn = B;
      if (bn < b_prev) bn = b_prev;
      const int32_t b_next = (int32_t)bn;
      if (b_next > b_prev) {
        PassATask ts = t;
        ts.block0 = b_prev;
        ts.block_end = b_next;
        ts.n_tasks = (int64_t)((b_next - b_prev + t.blocks_per_task - 1) / t.blocks_per_task) * t.chunks;
        rc = launch_pass_a(ts, c, s);
        if (rc) return rc;
      }
      SK_HIP_TRY(hipEventRecord(p->seg_ev[k], s));
      SK_HIP_TRY(hipStreamWaitEvent(p->side, p->seg_ev[k], 0));
      rc = launch_pass_b_range(a, c_prev, c_next, b_prev, b_next, k == 0, p->side);
      if (rc) return rc;
      c_prev = c_next;
      b_prev = b_next;
    }
    if (rec) SK_HIP_TRY(hipEventRecord(p->prof[3 * p->prof_n + 1], s));
    SK_HIP_TRY(hipEventRecord(p->seg_ev[K], p->side));
    SK_HIP_TRY(hipStreamWaitEvent(s, p->seg_ev[K], 0));
  }
  if (rec) {
    SK_HIP_TRY(hipEventRecord(p->prof[3 * p->prof_n + 2], s));
    p->prof_n += 1;
  }
  if (p->hist_cap > 0) {
    const int64_t total = p->hist_len + B;
    p->hist_len = (int32_t)(total < p->hist_cap ? total : p->hist_cap);
    p->cur = 1 - p->cur;
  }
  return SK_OK;
}

int sk_flags(sk_plan_t p, const float* d_v, const int32_t* d_n_eff, uint8_t* d_flags, int64_t n,
             void* stream) {
  clear_error();
  if (!p || (n > 0 && (!d_v || !d_n_eff || !d_flags)) || n < 0) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  FlagArgs a;
  a.thresholds = p->thresholds;
  a.n_max = p->d.n_inputs;
  a.v = d_v;
  a.n_eff = d_n_eff;
  a.flags = d_flags;
  a.n = n;
  a.block_len = p->d.block_len;
  a.window = p->d.norm_window_blocks;
  a.estimator = p->d.estimator;
  a.k_sigma = p->d.k_sigma;
  a.expect_offset = p->d.expect_offset;
  a.sigma_override = p->d.sigma_override;
  return launch_flags(a, (hipStream_t)stream);
}

int sk_plan_set_false_alarm(sk_plan_t p, double fap) {
  clear_error();
  if (!p || !(fap >= 0.0) || fap >= 0.5) { set_error("false-alarm probability must be in [0, 0.5)"); return SK_ERR_INVALID_ARG; }
  if (fap == 0.0) {
    if (p->thresholds) (void)hipFree(p->thresholds);
    p->thresholds = nullptr;
    p->fap = 0.0;
    return SK_OK;
  }
  const sk_plan_desc& d = p->d;
  std::vector<double> t(2 * ((size_t)d.n_inputs + 1));
  for (int n = 0; n <= d.n_inputs; ++n) {
    const double K = (double)n * d.block_len, Md = d.block_len;
    if (n == 0 || K < 2) { t[2 * n] = -INFINITY; t[2 * n + 1] = INFINITY; continue; }
    double e0 = 1.0;
    if (d.estimator == SK_EST_HAT && d.norm_window_blocks == 1) e0 = ((K + 1.0) * (Md - 1.0)) / ((K - 1.0) * (Md + 1.0));
    const double E = e0 + d.expect_offset;
    const double s = d.sigma_override > 0.0 ? d.sigma_override : sqrt(4.0 / K);
    const double g = 10.0 / sqrt(K);
    t[2 * n] = pearson3_quantile(E, s, g, fap);
    t[2 * n + 1] = pearson3_quantile(E, s, g, 1.0 - fap);
  }
  if (!p->thresholds) SK_HIP_TRY(hipMalloc((void**)&p->thresholds, sizeof(double) * t.size()));
  SK_HIP_TRY(hipMemcpy(p->thresholds, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
  p->fap = fap;
  return SK_OK;
}

int sk_plan_get_thresholds(sk_plan_t p, int32_t n_eff, double* lo, double* hi) {
  if (!p || !lo || !hi || n_eff < 0 || n_eff > p->d.n_inputs) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  const sk_plan_desc& d = p->d;
  const double K = (double)n_eff * d.block_len, Md = d.block_len;
  if (n_eff == 0 || K < 2) { *lo = -INFINITY; *hi = INFINITY; return SK_OK; }
  if (p->fap > 0.0) {
    const double g = 10.0 / sqrt(K);
    double e0 = 1.0;
    if (d.estimator == SK_EST_HAT && d.norm_window_blocks == 1) e0 = ((K + 1.0) * (Md - 1.0)) / ((K - 1.0) * (Md + 1.0));
    const double E = e0 + d.expect_offset;
    const double s = d.sigma_override > 0.0 ? d.sigma_override : sqrt(4.0 / K);
    *lo = pearson3_quantile(E, s, g, p->fap);
    *hi = pearson3_quantile(E, s, g, 1.0 - p->fap);
    return SK_OK;
  }
  double e0 = 1.0;
  if (d.estimator == SK_EST_HAT && d.norm_window_blocks == 1) e0 = ((K + 1.0) * (Md - 1.0)) / ((K - 1.0) * (Md + 1.0));
  const double E = e0 + d.expect_offset;
  const double s = d.sigma_override > 0.0 ? d.sigma_override : sqrt(4.0 / K);
  *lo = E - d.k_sigma * s;
  *hi = E + d.k_sigma * s;
  return SK_OK;
}

int sk_state_reset(sk_plan_t p) {
  clear_error();
  if (!p) { set_error("NULL plan"); return SK_ERR_INVALID_ARG; }
  p->hist_len = 0;
  return SK_OK;
}

int sk_state_size(sk_plan_t p, size_t* bytes) {
  if (!p || !bytes) { set_error("NULL argument"); return SK_ERR_INVALID_ARG; }
  *bytes = sizeof(StateHeader) + (size_t)p->d.n_channels * p->hist_len * p->d.n_inputs * sizeof(int32_t);
  return SK_OK;
}

int sk_state_export(sk_plan_t p, void* host_buf, size_t cap, void* stream) {
  clear_error();
  size_t need = 0;
  if (sk_state_size(p, &need)) return SK_ERR_INVALID_ARG;
  if (!host_buf || cap < need) { set_error("buffer too small: need %zu", need); return SK_ERR_INVALID_ARG; }
  StateHeader h = {kStateMagic, 1, p->d.n_inputs, p->d.n_channels, p->d.block_len, p->d.norm_window_blocks, p->hist_len, 0};
  memcpy(host_buf, &h, sizeof h);
  if (p->hist_len > 0) {
    hipStream_t s = (hipStream_t)stream;
    const size_t row = (size_t)p->hist_len * p->d.n_inputs * sizeof(int32_t);
    for (int f = 0; f < p->d.n_channels; ++f) {
      const int32_t* src = p->hist[p->cur] + (size_t)f * p->hist_cap * p->d.n_inputs;
      SK_HIP_TRY(hipMemcpyAsync((char*)host_buf + sizeof h + f * row, src, row, hipMemcpyDeviceToHost, s));
    }
    SK_HIP_TRY(hipStreamSynchronize(s));
  }
  return SK_OK;
}

int sk_state_import(sk_plan_t p, const void* host_buf, size_t size, void* stream) {
  clear_error();
  if (!p || !host_buf || size < sizeof(StateHeader)) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  StateHeader h;
  memcpy(&h, host_buf, sizeof h);
  if (h.magic != kStateMagic || h.version != 1 || h.n_inputs != p->d.n_inputs || h.n_channels != p->d.n_channels ||
      h.block_len != p->d.block_len || h.window != p->d.norm_window_blocks || h.hist_len < 0 || h.hist_len > p->hist_cap) {
    set_error("state blob does not match this plan");
    return SK_ERR_STATE;
  }
  const size_t row = (size_t)h.hist_len * p->d.n_inputs * sizeof(int32_t);
  if (size < sizeof h + row * p->d.n_channels) { set_error("state blob truncated"); return SK_ERR_STATE; }
  hipStream_t s = (hipStream_t)stream;
  if (h.hist_len > 0) {
    for (int f = 0; f < p->d.n_channels; ++f) {
      int32_t* dst = p->hist[p->cur] + (size_t)f * p->hist_cap * p->d.n_inputs;
      SK_HIP_TRY(hipMemcpyAsync(dst, (const char*)host_buf + sizeof h + f * row, row, hipMemcpyHostToDevice, s));
    }
    SK_HIP_TRY(hipStreamSynchronize(s));
  }
  p->hist_len = h.hist_len;
  return SK_OK;
}

}  // extern "C"
