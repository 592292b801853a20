// C ABI: plans, validation, device memory ownership, normaliser state.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
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
  int32_t chunk;           // R of pass B
  int32_t s1_s2_owned;
  int32_t* s1;             // [F][B][N] scratch (when the caller does not take the sums)
  int32_t* s2;
  uint32_t* pc;            // [F][ceil(B / R) + 1][N] prefix sums of pass B
  size_t pc_bytes;
  int32_t* cs;             // [F][ceil(B / R)][N] chunk sums written by pass A (variant 4 with Q == R)
  size_t cs_bytes;
  int32_t* hs[2];          // [F][hist_cap][N] history suffix sums, ping-pong
  int32_t cur;             // index of the live history buffer
  size_t bytes;
  int pass_a_lpr;          // 0 = heuristic
  int pass_a_variant = -1; // pass A variant; -1 = heuristic
  int pass_a_grid;         // 0 = one workgroup per task
  int pass_a_blocks = 0;   // consecutive blocks per pass A task (packed variants; 0 = library choice)
  int chunk_sums = 1;      // pass A hands the scan chunk sums when its tasks are the chunks (autotuner may clear)
  int pass_b_vec;          // 0 = library choice, else 1 or 4 inputs per lane
  int n_cu = 256;          // compute units of the plan's device
  std::vector<hipEvent_t> prof;   // 4 events per recorded call
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

static void free_profile(sk_plan_s* p) {
  for (hipEvent_t e : p->prof) (void)hipEventDestroy(e);
  p->prof.clear();
  p->prof_max = p->prof_n = 0;
}

static void free_plan_memory(sk_plan_s* p) {
  free_profile(p);
  if (p->thresholds) (void)hipFree(p->thresholds);
  if (p->s1_s2_owned) {
    if (p->s1) (void)hipFree(p->s1);
    if (p->s2) (void)hipFree(p->s2);
  }
  if (p->pc) (void)hipFree(p->pc);
  if (p->cs) (void)hipFree(p->cs);
  if (p->hs[0]) (void)hipFree(p->hs[0]);
  if (p->hs[1]) (void)hipFree(p->hs[1]);
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
  p->chunk = pass_b_chunk((int32_t)N, (int32_t)F, p->n_blocks, L);
  p->s1_s2_owned = 1;
  const size_t fbn = (size_t)F * p->n_blocks * N;
  SK_ALLOC(p->s1, fbn * sizeof(int32_t));
  SK_ALLOC(p->s2, fbn * sizeof(int32_t));
  if (L >= 2) {
    p->pc_bytes = pass_b_prefix_bytes((int32_t)N, (int32_t)F, p->n_blocks, p->chunk);
    SK_ALLOC(p->pc, p->pc_bytes);
    // Chunk sums from pass A when its tasks are the plan's pass B chunks
    // (sized for the shortest such chunk, R = 2, which a tuner may pick).
    if (p->n_blocks >= 2) {
      p->cs_bytes = (size_t)F * (size_t)((p->n_blocks + 1) / 2) * (size_t)N * sizeof(int32_t);
      SK_ALLOC(p->cs, p->cs_bytes);
    }
    SK_ALLOC(p->hs[0], (size_t)F * p->hist_cap * N * sizeof(int32_t));
    SK_ALLOC(p->hs[1], (size_t)F * p->hist_cap * N * sizeof(int32_t));
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

namespace {
// Pass A tuning controls of a plan (library choices when 0 / -1).
struct PassATuning {
  int lpr = 0, variant = -1, blocks = 0, grid = 0, n_cu = 256;
};
}  // namespace

static PassAConfig pass_a_config(const sk_plan_desc& d, int64_t B, const PassATuning& u, const uint8_t* d_packed,
                                 PassATask* t) {
  const int64_t N = d.n_inputs, F = d.n_channels;
  const int vec = pick_vec(d_packed, (int32_t)N);
  t->row_bytes = F * N;
  t->n_inputs = (int32_t)N;
  t->block0 = 0;
  t->block_end = (int32_t)B;
  t->blocks_per_task = 1;
  t->block_len = d.block_len;
  t->n_blocks = (int32_t)B;
  t->cs = nullptr;
  t->timeline = nullptr;
  t->simd_balance = 1;
  PassAConfig c = default_pass_a_config(vec, t->row_bytes, B, d.block_len, u.lpr == 0 && u.variant < 0, u.n_cu);
  if (u.lpr) c.lpr = u.lpr;
  if (u.variant >= 0) c.variant = u.variant;
  {
    int lo, hi;
    pass_a_lane_range(vec, c.variant, &lo, &hi);
    if (c.lpr < lo) c.lpr = lo;
    if (c.lpr > hi) c.lpr = hi;
  }
  t->col_groups = (int32_t)(t->row_bytes / vec);
  t->chunks = (t->col_groups + c.lpr - 1) / c.lpr;
  if (pass_a_packed(vec, c.variant) && u.blocks > 1) t->blocks_per_task = u.blocks;
  if (pass_a_deferred(vec, c.variant)) {
    c.lpr = 512;
    t->chunks = (t->col_groups + 511) / 512;
    t->blocks_per_task = u.blocks >= 1 && u.blocks <= 4 ? u.blocks : pass_a_deferred_blocks(B, t->col_groups, u.n_cu);
  }
  if (pass_a_side_by_side(vec, c.variant)) {
    c.lpr = pass_a_side_by_side_lanes(t->col_groups);
    t->blocks_per_task = c.lpr >= 256 ? 1 : 256 / c.lpr;
    t->chunks = c.lpr >= 256 ? (t->col_groups + 255) / 256 : 1;
  }
  t->n_tasks = ((B + t->blocks_per_task - 1) / t->blocks_per_task) * t->chunks;
  c.grid = (int)(t->n_tasks < (1 << 30) ? t->n_tasks : (1 << 30));
  if (u.grid > 0 && u.grid < c.grid) c.grid = u.grid;
  return c;
}

static PassAConfig plan_pass_a_config(const sk_plan_s* p, const uint8_t* d_packed, PassATask* t) {
  PassATuning u;
  u.lpr = p->pass_a_lpr;
  u.variant = p->pass_a_variant;
  u.blocks = p->pass_a_blocks;
  u.grid = p->pass_a_grid;
  u.n_cu = p->n_cu;
  return pass_a_config(p->d, p->n_blocks, u, d_packed, t);
}

int sk_plan_set_pass_a_variant(sk_plan_t p, int32_t variant, int32_t grid) {
  if (!p || variant < -1 || variant > 4 || grid < 0) { set_error("pass A variant must be -1..4 and grid >= 0"); return SK_ERR_INVALID_ARG; }
  p->pass_a_variant = variant;
  p->pass_a_grid = grid;
  return SK_OK;
}

int sk_plan_set_pass_a_blocks(sk_plan_t p, int32_t blocks) {
  clear_error();
  if (!p || blocks < 0 || blocks > 4096) { set_error("blocks per task must be in 0..4096"); return SK_ERR_INVALID_ARG; }
  p->pass_a_blocks = blocks;
  return SK_OK;
}

int sk_plan_set_pass_b_tile(sk_plan_t p, int32_t chunk, int32_t vec) {
  clear_error();
  if (!p || (chunk != 0 && chunk != 1 && chunk != 2 && chunk != 4) || (vec != 0 && vec != 1 && vec != 4)) {
    set_error("pass B tile: chunk must be 0, 1, 2 or 4 and inputs per lane 0, 1 or 4");
    return SK_ERR_INVALID_ARG;
  }
  const int32_t R = chunk ? chunk
                          : pass_b_chunk(p->d.n_inputs, p->d.n_channels, p->n_blocks, p->d.norm_window_blocks);
  if (p->d.norm_window_blocks >= 2) {
    const size_t need = pass_b_prefix_bytes(p->d.n_inputs, p->d.n_channels, p->n_blocks, R);
    if (need > p->pc_bytes) {
      uint32_t* pc = nullptr;
      SK_HIP_TRY(hipDeviceSynchronize());
      SK_HIP_TRY(hipMalloc((void**)&pc, need));
      if (p->pc) (void)hipFree(p->pc);
      p->bytes += need - p->pc_bytes;
      p->pc = pc;
      p->pc_bytes = need;
    }
  }
  p->chunk = R;
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
  p->prof.resize((size_t)max_records * 4);
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
    SK_HIP_TRY(hipEventSynchronize(p->prof[4 * j + 3]));
    SK_HIP_TRY(hipEventElapsedTime(&ms_a[j], p->prof[4 * j], p->prof[4 * j + 1]));
    SK_HIP_TRY(hipEventElapsedTime(&ms_b[j], p->prof[4 * j + 2], p->prof[4 * j + 3]));
  }
  *n = m;
  p->prof_n = 0;
  return SK_OK;
}

}  // extern "C"

namespace sk {

// Buffers of one call beyond the caller's input and outputs.
struct CallBuffers {
  int32_t* s1;           // [F][B][N] (the caller's output or scratch)
  int32_t* s2;
  uint32_t* pc;          // pass B prefix sums (L >= 2)
  const int32_t* hs;     // history suffix sums of this call (L >= 2; hist_len slots valid)
  int32_t* hs_next;      // the next call's
  int32_t hist_len;
};

// Pass B arguments of one call.
static PassBArgs make_pass_b_args(const sk_plan_desc& d, int64_t B, int32_t hist_cap, int32_t chunk, int32_t vec_pref,
                                  const uint8_t* mask, const sk_outputs* outs, const CallBuffers& cb,
                                  const double* thresholds) {
  PassBArgs a;
  memset(&a, 0, sizeof a);
  const int64_t N = d.n_inputs;
  a.s1 = cb.s1;
  a.s2 = cb.s2;
  a.cs = nullptr;
  a.hs = cb.hs;
  a.hs_next = cb.hs_next;
  a.pc = cb.pc;
  a.mask = mask;
  a.r1 = outs->r1;
  a.r2 = outs->r2;
  a.v = outs->v;
  a.flags = outs->flags;
  a.n_eff = outs->n_eff;
  a.sk_i = outs->sk_i;
  a.significance = outs->significance;
  a.thresholds = thresholds;
  a.n_inputs = (int32_t)N;
  a.n_channels = d.n_channels;
  a.n_blocks = (int32_t)B;
  a.block_len = d.block_len;
  a.window = d.norm_window_blocks;
  a.hist_len = cb.hist_len;
  a.hist_cap = hist_cap;
  const int64_t total = cb.hist_len + B;
  a.hist_next_len = (int32_t)(total < hist_cap ? total : hist_cap);
  a.chunk = chunk;
  a.n_chunks = (int32_t)((B + chunk - 1) / chunk);
  // Four inputs per lane need 16-byte aligned rows of the sums.
  a.vec = pass_b_vec((int32_t)N);
  if (((uintptr_t)cb.s1 | (uintptr_t)cb.s2 | (uintptr_t)outs->sk_i) % 16 != 0) a.vec = 1;
  if (vec_pref == 1) a.vec = 1;
  a.estimator = d.estimator;
  a.k_sigma = d.k_sigma;
  a.expect_offset = d.expect_offset;
  a.sigma_override = d.sigma_override;
  return a;
}

}  // namespace sk

extern "C" {

}  // extern "C"

// One call of a plan (the body of sk_compute, arguments checked): pass A,
// then pass B, with the given dispatch timing events (null: untimed).
// *chunk_sums (if given) tells whether pass A handed the scan its chunk sums.
static int plan_call(sk_plan_s* p, const uint8_t* d_packed, const uint8_t* d_mask, const sk_outputs* outs,
                     hipStream_t s, PassEvents ea, PassEvents eb, bool* chunk_sums = nullptr) {
  const int64_t B = p->n_blocks;
  CallBuffers cb;
  cb.s1 = outs->s1 ? outs->s1 : p->s1;
  cb.s2 = outs->s2 ? outs->s2 : p->s2;
  cb.pc = p->pc;
  cb.hs = p->hs[p->cur];
  cb.hs_next = p->hs[1 - p->cur];
  cb.hist_len = p->hist_len;

  PassATask t;
  PassAConfig c = plan_pass_a_config(p, d_packed, &t);
  t.x = d_packed;
  t.s1 = cb.s1;
  t.s2 = cb.s2;
  t.cs = nullptr;
  PassBArgs a = make_pass_b_args(p->d, B, p->hist_cap, p->chunk, p->pass_b_vec, d_mask, outs, cb, p->thresholds);
  // Pass A tasks of Q = R consecutive blocks hand the scan its chunk sums.
  if (a.window >= 2 && p->cs && p->chunk_sums && pass_a_deferred(c.vec, c.variant) && t.blocks_per_task == a.chunk &&
      (size_t)a.n_channels * a.n_chunks * a.n_inputs * sizeof(int32_t) <= p->cs_bytes) {
    t.cs = p->cs;
    a.cs = p->cs;
  }
  if (chunk_sums) *chunk_sums = t.cs != nullptr;

  int rc = launch_pass_a(t, c, s, ea);
  if (rc) return rc;
  rc = launch_pass_b(a, s, eb);
  if (rc) return rc;
  if (p->hist_cap > 0) {
    p->hist_len = a.hist_next_len;
    p->cur = 1 - p->cur;
  }
  return SK_OK;
}

extern "C" {

int sk_compute(sk_plan_t p, const uint8_t* d_packed, const uint8_t* d_mask, const sk_outputs* outs,
               void* stream) {
  clear_error();
  if (!p || !outs) { set_error("NULL plan or outputs"); return SK_ERR_INVALID_ARG; }
  if (!d_packed && p->d.n_samples > 0) { set_error("NULL input"); return SK_ERR_INVALID_ARG; }
  int dev = -1;
  SK_HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) { set_error("plan was created on device %d, current device is %d", p->device, dev); return SK_ERR_INVALID_ARG; }
  if (p->n_blocks == 0) return SK_OK;
  // A recorded call's four timestamps come with its kernels' dispatches:
  // pass A's kernel start and end, pass B's first start and last end.
  const bool rec = p->prof_n < p->prof_max && (p->prof_calls++ % p->prof_stride) == 0;
  PassEvents ea, eb;
  if (rec) {
    hipEvent_t* e = &p->prof[4 * p->prof_n];
    ea = PassEvents{e[0], e[1]};
    eb = PassEvents{e[2], e[3]};
  }
  const int rc = plan_call(p, d_packed, d_mask, outs, (hipStream_t)stream, ea, eb);
  if (rc == SK_OK && rec) p->prof_n += 1;
  return rc;
}

// Autotuner of one plan: every candidate (pass A variant and its lanes or
// blocks per task, pass B chunk length) runs one
// untimed and `reps` timed calls on d_x; the least pooled estimate of pass A
// plus pass B kernel time (dispatch timestamps) wins, and is kept if it also
// beats the library's choice in alternating calls. The normaliser state is
// saved before and restored after, so a stream in progress continues as if
// the tuning calls had not run.
int sk_plan_autotune(sk_plan_t p, const uint8_t* d_x, int32_t reps, void* stream, sk_plan_tuning* out) {
  clear_error();
  if (!p || !d_x || reps < 1 || reps > 100) { set_error("autotune: NULL plan or input, or reps outside 1..100"); return SK_ERR_INVALID_ARG; }
  int dev = -1;
  SK_HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) { set_error("plan was created on device %d, current device is %d", p->device, dev); return SK_ERR_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  if (p->n_blocks == 0) return SK_OK;
  // Saved state and settings.
  size_t sbytes = 0;
  int rc = sk_state_size(p, &sbytes);
  if (rc) return rc;
  std::vector<uint8_t> saved(sbytes);
  if ((rc = sk_state_export(p, saved.data(), sbytes, stream))) return rc;
  const int keep_lpr = p->pass_a_lpr, keep_var = p->pass_a_variant, keep_blocks = p->pass_a_blocks;
  const int keep_cs = p->chunk_sums;
  const int32_t keep_chunk = p->chunk, keep_vec = p->pass_b_vec;

  // cs: whether pass A may hand the scan its chunk sums.
  struct Cand { int variant, lpr, blocks, chunk, vec, cs; };
  std::vector<Cand> cands;
  const int vec = pick_vec(d_x, p->d.n_inputs);
  const int64_t cg = (int64_t)p->d.n_channels * p->d.n_inputs / vec;
  std::vector<Cand> a_opts = {{-1, 0, 0, 0, 0, 1}};
  if (vec == 16) {
    if (cg >= 512) {
      for (int q : {1, 2, 4}) a_opts.push_back({4, 0, q, 0, 0, 1});
      // The same tasks without the chunk sums where they would be written.
      if (p->cs)
        for (int q : {2, 4}) a_opts.push_back({4, 0, q, 0, 0, 0});
    }
    if (cg >= 512) a_opts.push_back({2, 1024, 1, 0, 0, 1});
    if (cg >= 256) {
      a_opts.push_back({2, 256, 1, 0, 0, 1});
      a_opts.push_back({1, 256, 1, 0, 0, 1});
    }
    if (cg < 256) a_opts.push_back({3, 0, 0, 0, 0, 1});
  }
  // Pass B inputs per lane stay as set: they fix which inputs a lane sums
  // first, so they change the combine's rounding; the chunk length does not.
  for (const Cand& a : a_opts)
    for (int R : {1, 2, 4})
      if (a.cs || R == a.blocks) cands.push_back({a.variant, a.lpr, a.blocks, R, keep_vec, a.cs});

  std::vector<hipEvent_t> ev(4 * (size_t)reps, nullptr);
  for (auto& e : ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& x : ev) if (x) (void)hipEventDestroy(x);
      set_error("autotune: event create failed");
      return SK_ERR_DEVICE;
    }
  }
  sk_outputs none;
  memset(&none, 0, sizeof none);
  // Per candidate: summed pass A and pass B times of its timed calls, and
  // whether pass A wrote the chunk sums (which changes both passes' work).
  std::vector<double> sum_a(cands.size(), 0.0), sum_b(cands.size(), 0.0);
  std::vector<char> with_cs(cands.size(), 0);
  std::vector<Cand> resolved(cands.size());   // pass A as launched (the library's choice made concrete)
  for (size_t ci = 0; ci < cands.size() && rc == SK_OK; ++ci) {
    const Cand& c = cands[ci];
    p->pass_a_lpr = c.lpr;
    p->pass_a_variant = c.variant;
    p->pass_a_blocks = c.blocks;
    p->chunk_sums = c.cs;
    if ((rc = sk_plan_set_pass_b_tile(p, c.chunk, c.vec))) break;
    {
      PassATask t;
      const PassAConfig pc = plan_pass_a_config(p, d_x, &t);
      resolved[ci] = Cand{pc.variant, pc.lpr, t.blocks_per_task, c.chunk, c.vec, c.cs};
    }
    if ((rc = plan_call(p, d_x, nullptr, &none, s, PassEvents(), PassEvents()))) break;
    bool cs = false;
    for (int r = 0; r < reps && rc == SK_OK; ++r)
      rc = plan_call(p, d_x, nullptr, &none, s, PassEvents{ev[4 * r], ev[4 * r + 1]},
                     PassEvents{ev[4 * r + 2], ev[4 * r + 3]}, &cs);
    if (rc) break;
    with_cs[ci] = cs;
    if (hipStreamSynchronize(s) != hipSuccess) { rc = SK_ERR_DEVICE; set_error("autotune: synchronize failed"); break; }
    for (int r = 0; r < reps; ++r) {
      float x = 0.f, y = 0.f;
      if (hipEventElapsedTime(&x, ev[4 * r], ev[4 * r + 1]) != hipSuccess ||
          hipEventElapsedTime(&y, ev[4 * r + 2], ev[4 * r + 3]) != hipSuccess) {
        rc = SK_ERR_DEVICE;
        set_error("autotune: event timing failed");
        break;
      }
      sum_a[ci] += x;
      sum_b[ci] += y;
    }
  }
  // Pooled estimates: pass A's time depends on its own settings (and on
  // whether it writes chunk sums), pass B's on the chunk length (and on
  // whether it reads them). Each pass is estimated from every candidate that
  // shares its settings, so one noisy pass A trial does not decide pass B.
  float best = 1e30f, best_a = 0.f, best_b = 0.f, lib_a = 0.f, lib_b = 0.f;
  size_t best_i = 0, lib_i = cands.size();
  if (rc == SK_OK) {
    auto same_a = [&](size_t i, size_t j) {
      return resolved[i].variant == resolved[j].variant && resolved[i].lpr == resolved[j].lpr &&
             resolved[i].blocks == resolved[j].blocks && with_cs[i] == with_cs[j];
    };
    auto same_b = [&](size_t i, size_t j) { return cands[i].chunk == cands[j].chunk && with_cs[i] == with_cs[j]; };
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      double ta = 0.0, tb = 0.0;
      int na = 0, nb = 0;
      for (size_t cj = 0; cj < cands.size(); ++cj) {
        if (same_a(ci, cj)) { ta += sum_a[cj]; ++na; }
        if (same_b(ci, cj)) { tb += sum_b[cj]; ++nb; }
      }
      const float ea_ms = (float)(ta / ((double)na * reps)), eb_ms = (float)(tb / ((double)nb * reps));
      const Cand& c = cands[ci];
      if (c.variant == -1 && c.lpr == 0 && c.blocks == 0 && c.chunk == keep_chunk && c.cs) {
        lib_a = ea_ms;
        lib_b = eb_ms;
        lib_i = ci;
      }
      if (ea_ms + eb_ms < best) { best = ea_ms + eb_ms; best_i = ci; best_a = ea_ms; best_b = eb_ms; }
    }
  }
  // A pick other than the library's choice is confirmed against it in
  // alternating calls (library, pick, library, pick, ...), so a drift of the
  // device's speed during the trials cannot favour either; the pick is kept
  // only if it is still faster.
  const bool differs = rc == SK_OK && lib_i != best_i && lib_i < cands.size() &&
                       !(resolved[lib_i].variant == resolved[best_i].variant &&
                         resolved[lib_i].lpr == resolved[best_i].lpr &&
                         resolved[lib_i].blocks == resolved[best_i].blocks && with_cs[lib_i] == with_cs[best_i] &&
                         cands[lib_i].chunk == cands[best_i].chunk);
  if (differs) {
    constexpr int ROUNDS = 4;
    double conf_a[2] = {0.0, 0.0}, conf_b[2] = {0.0, 0.0};
    for (int r = 0; r < ROUNDS && rc == SK_OK; ++r) {
      for (int side = 0; side < 2 && rc == SK_OK; ++side) {
        const Cand& c = cands[side ? best_i : lib_i];
        p->pass_a_lpr = c.lpr;
        p->pass_a_variant = c.variant;
        p->pass_a_blocks = c.blocks;
        p->chunk_sums = c.cs;
        if ((rc = sk_plan_set_pass_b_tile(p, c.chunk, c.vec))) break;
        if ((rc = plan_call(p, d_x, nullptr, &none, s, PassEvents{ev[0], ev[1]}, PassEvents{ev[2], ev[3]}))) break;
        float x = 0.f, y = 0.f;
        if (hipEventSynchronize(ev[3]) != hipSuccess || hipEventElapsedTime(&x, ev[0], ev[1]) != hipSuccess ||
            hipEventElapsedTime(&y, ev[2], ev[3]) != hipSuccess) {
          rc = SK_ERR_DEVICE;
          set_error("autotune: event timing failed");
          break;
        }
        conf_a[side] += x;
        conf_b[side] += y;
      }
    }
    if (rc == SK_OK) {
      lib_a = (float)(conf_a[0] / ROUNDS);
      lib_b = (float)(conf_b[0] / ROUNDS);
      if (conf_a[1] + conf_b[1] < conf_a[0] + conf_b[0]) {
        best_a = (float)(conf_a[1] / ROUNDS);
        best_b = (float)(conf_b[1] / ROUNDS);
      } else {
        best_i = lib_i;
        best_a = lib_a;
        best_b = lib_b;
      }
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) {
    p->pass_a_lpr = keep_lpr;
    p->pass_a_variant = keep_var;
    p->pass_a_blocks = keep_blocks;
    p->chunk_sums = keep_cs;
    (void)sk_plan_set_pass_b_tile(p, keep_chunk, keep_vec);
    (void)sk_state_import(p, saved.data(), sbytes, stream);
    return rc;
  }
  const Cand& c = cands[best_i];
  p->pass_a_lpr = c.lpr;
  p->pass_a_variant = c.variant;
  p->pass_a_blocks = c.blocks;
  p->chunk_sums = c.cs;
  if ((rc = sk_plan_set_pass_b_tile(p, c.chunk, c.vec))) return rc;
  if ((rc = sk_state_import(p, saved.data(), sbytes, stream))) return rc;
  if (out) {
    PassATask t;
    const PassAConfig pc = plan_pass_a_config(p, d_x, &t);
    out->pass_a_variant = pc.variant;
    out->pass_a_lanes = pc.lpr;
    out->pass_a_blocks = t.blocks_per_task;
    out->pass_b_chunk = p->chunk;
    bool cs = false;
    {
      // Whether the kept combination hands the scan chunk sums (the same
      // test as a call's).
      PassBArgs pb = make_pass_b_args(p->d, p->n_blocks, p->hist_cap, p->chunk, p->pass_b_vec, nullptr, &none,
                                      CallBuffers{p->s1, p->s2, p->pc, nullptr, nullptr, 0}, nullptr);
      cs = pb.window >= 2 && p->cs && p->chunk_sums && pass_a_deferred(pc.vec, pc.variant) &&
           t.blocks_per_task == pb.chunk &&
           (size_t)pb.n_channels * pb.n_chunks * pb.n_inputs * sizeof(int32_t) <= p->cs_bytes;
    }
    out->pass_a_chunk_sums = cs ? 1 : 0;
    out->pass_b_vec = make_pass_b_args(p->d, p->n_blocks, p->hist_cap, p->chunk, p->pass_b_vec, nullptr, &none,
                                       CallBuffers{p->s1, p->s2, p->pc, nullptr, nullptr, 0}, nullptr).vec;
    out->candidates = (int32_t)cands.size();
    out->ms_pass_a = best_a;
    out->ms_pass_b = best_b;
    out->ms_library_pass_a = lib_a;
    out->ms_library_pass_b = lib_b;
  }
  return SK_OK;
}

}  // extern "C"

extern "C" {

int sk_plan_pass_a_timeline(sk_plan_t p, const uint8_t* d_x, int32_t simd_balance, uint64_t* d_out, int64_t cap,
                            int64_t* n_waves, void* stream) {
  clear_error();
  if (!p || !d_x || !d_out || !n_waves || cap < 0 || (simd_balance != 0 && simd_balance != 1)) {
    set_error("timeline: NULL argument, negative capacity, or simd_balance not 0 or 1");
    return SK_ERR_INVALID_ARG;
  }
  *n_waves = 0;
  int dev = -1;
  SK_HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) { set_error("plan was created on device %d, current device is %d", p->device, dev); return SK_ERR_INVALID_ARG; }
  if (p->n_blocks == 0) return SK_OK;
  PassATask t;
  const PassAConfig c = plan_pass_a_config(p, d_x, &t);
  if (!pass_a_deferred(c.vec, c.variant)) {
    set_error("timeline: the plan's pass A is variant %d, not the deferred-store variant 4", c.variant);
    return SK_ERR_INVALID_ARG;
  }
  if ((int64_t)c.grid != t.n_tasks || (!simd_balance && t.blocks_per_task != 4)) {
    set_error("timeline: needs one workgroup per task (%d for %lld), and 4 blocks per task without the SIMD balance",
              c.grid, (long long)t.n_tasks);
    return SK_ERR_INVALID_ARG;
  }
  const int64_t waves = (int64_t)c.grid * 8;
  if (waves > cap) {
    set_error("timeline: %lld wavefronts, room for %lld", (long long)waves, (long long)cap);
    return SK_ERR_INVALID_ARG;
  }
  t.x = d_x;
  t.s1 = p->s1;
  t.s2 = p->s2;
  t.timeline = d_out;
  t.simd_balance = simd_balance;
  const int rc = launch_pass_a(t, c, (hipStream_t)stream);
  if (rc == SK_OK) *n_waves = waves;
  return rc;
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation call
//
// sk_compute_noalloc's scratch: pass B's prefix sums live in this
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never passes `scratch` itself to a kernel: its device address is
// taken once per device with hipGetSymbolAddress and kept below.
static constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of that device's scratch
}  // namespace

// Address of the current device's scratch (looked up on the first call on
// each device, with that device current).
static int noalloc_scratch(int dev, void** ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *ptr = it->second;
    return SK_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    return SK_ERR_DEVICE;
  }
  g_scratch_ptr[dev] = p;
  *ptr = p;
  return SK_OK;
}

extern "C" {

size_t sk_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int sk_compute_noalloc(const sk_plan_desc* desc, const uint8_t* d_packed, const uint8_t* d_mask,
                       const sk_outputs* outs, void* stream) {
  clear_error();
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (!outs || !outs->s1 || !outs->s2) {
    set_error("sk_compute_noalloc needs the caller's s1 and s2 output buffers");
    return SK_ERR_INVALID_ARG;
  }
  const sk_plan_desc& d = *desc;
  const int64_t B = d.n_samples / d.block_len;
  if (B == 0) return SK_OK;
  if (!d_packed) { set_error("NULL input"); return SK_ERR_INVALID_ARG; }
  const int L = d.norm_window_blocks;
  const int32_t R = pass_b_chunk(d.n_inputs, d.n_channels, B, L);
  const size_t need = L >= 2 ? pass_b_prefix_bytes(d.n_inputs, d.n_channels, B, R) : 0;
  if (need > kNoallocScratchBytes) {
    set_error("call needs %zu bytes of scratch; sk_compute_noalloc holds %zu (F (ceil(B / %d) + 1) N int32)", need,
              kNoallocScratchBytes, R);
    return SK_ERR_SHAPE;
  }
  int dev = -1;
  SK_HIP_TRY(hipGetDevice(&dev));
  void* sp = nullptr;
  rc = noalloc_scratch(dev, &sp);
  if (rc) return rc;
  PassATuning u;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) u.n_cu = ncu;
  hipStream_t s = (hipStream_t)stream;
  CallBuffers cb;
  cb.s1 = outs->s1;
  cb.s2 = outs->s2;
  cb.pc = (uint32_t*)sp;
  cb.hs = nullptr;
  cb.hs_next = nullptr;   // no state: nothing is carried to a next call
  cb.hist_len = 0;
  PassATask t;
  PassAConfig c = pass_a_config(d, B, u, d_packed, &t);
  t.x = d_packed;
  t.s1 = cb.s1;
  t.s2 = cb.s2;
  PassBArgs a = make_pass_b_args(d, B, L >= 2 ? L - 1 : 0, R, 0, d_mask, outs, cb, nullptr);
  rc = launch_pass_a(t, c, s);
  if (rc) return rc;
  return launch_pass_b(a, s);
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
  const int64_t H = p->hist_len, N = p->d.n_inputs, Hc = p->hist_cap;
  if (H > 0) {
    // The device keeps suffix sums HS over the history; the blob holds the
    // blocks themselves (oldest first): block y = HS(y) - HS(y + 1).
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> hs((size_t)H * N);
    int32_t* rows = (int32_t*)((char*)host_buf + sizeof h);
    for (int f = 0; f < p->d.n_channels; ++f) {
      const int32_t* src = p->hs[p->cur] + ((size_t)f * Hc + (Hc - H)) * N;
      SK_HIP_TRY(hipMemcpyAsync(hs.data(), src, hs.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      SK_HIP_TRY(hipStreamSynchronize(s));
      int32_t* dst = rows + (size_t)f * H * N;
      for (int64_t y = 0; y < H; ++y)
        for (int64_t i = 0; i < N; ++i) {
          const uint32_t next = y + 1 < H ? (uint32_t)hs[(y + 1) * N + i] : 0u;
          dst[y * N + i] = (int32_t)((uint32_t)hs[y * N + i] - next);
        }
    }
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
  const int64_t H = h.hist_len, N = p->d.n_inputs, Hc = p->hist_cap;
  const size_t row = (size_t)H * N * sizeof(int32_t);
  if (size < sizeof h + row * p->d.n_channels) { set_error("state blob truncated"); return SK_ERR_STATE; }
  hipStream_t s = (hipStream_t)stream;
  if (H > 0) {
    const int32_t* rows = (const int32_t*)((const char*)host_buf + sizeof h);
    std::vector<int32_t> hs((size_t)H * N);
    for (int f = 0; f < p->d.n_channels; ++f) {
      const int32_t* src = rows + (size_t)f * H * N;
      for (int64_t i = 0; i < N; ++i) {
        uint32_t acc = 0;
        for (int64_t y = H - 1; y >= 0; --y) {
          acc += (uint32_t)src[y * N + i];
          hs[y * N + i] = (int32_t)acc;
        }
      }
      int32_t* dst = p->hs[p->cur] + ((size_t)f * Hc + (Hc - H)) * N;
      SK_HIP_TRY(hipMemcpyAsync(dst, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
      SK_HIP_TRY(hipStreamSynchronize(s));
    }
  }
  p->hist_len = h.hist_len;
  return SK_OK;
}

}  // extern "C"
