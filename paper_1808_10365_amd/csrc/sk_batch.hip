// Batched form: many independent problems per launch (persistent kernels,
// device work queue, HIP graph) and the pass A autotuner.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "sk_batch.h"
#include "sk_internal.h"
#include "sk_pass_a_dev.h"
#include "sk_pass_b_dev.h"

namespace sk {

int validate_desc(const sk_plan_desc* d);

// One problem as the batched kernels see it (device table entry).
struct BatchProb {
  PassATask a;                 // pass A task geometry (x, s1, s2, shapes, chunks, n_tasks)
  int32_t lpr;                 // pass A lanes per block row: 512 (rows of >= 512 column groups,
                               // 512-group tasks run by a whole workgroup with deferred stores),
                               // 256 (wide rows in 256-group chunks), else 256 / lpr blocks side
                               // by side in half a workgroup
  int32_t rows;                // pass A rows per load, 8 or 16 (tuned per problem class)
  int32_t window, hist_cap, chunk, n_chunks, estimator;
  int32_t waves;               // combine waves per chunk (inputs / 256, at most 8)
  int32_t scan_waves;          // scan waves per 64-input slice (power of two, at most 8)
  int32_t wide_sums;           // 1: the combine's R1/R2 sums need 64 bits
  double k_sigma, expect_offset, sigma_override;
  uint32_t* pc;                // pass B prefix sums
  int32_t* cs_buf;             // chunk sums (wide rows, window >= 2; sized for chunks of 2 blocks), or null
  int32_t* hs[2];              // history suffix sums, ping-pong
  const uint8_t* mask;
  int64_t* r1;
  int64_t* r2;
  float* v;
  uint8_t* flags;
  int32_t* n_eff;
  float* sk_i;
  float* significance;
  // Task ranges of each kernel over the whole batch: pass A tasks, scan
  // workgroups (channel, group of 64-input slices), combine workgroups
  // (channel, group of chunks; counted within the problem's combine class).
  int64_t a_begin, sc_begin, sc_count, cb_begin, cb_count;
};

// Per-problem normaliser state kept on the device between calls.
struct BatchState {
  int32_t hist_len;
  int32_t parity;
};

__device__ __forceinline__ PassBArgs make_args(const BatchProb& P, const BatchState& S) {
  PassBArgs a;
  a.s1 = P.a.s1;
  a.s2 = P.a.s2;
  a.cs = P.a.cs;
  a.hs = P.hs[S.parity];
  a.hs_next = P.hs[S.parity ^ 1];
  a.pc = P.pc;
  a.mask = P.mask;
  a.r1 = P.r1;
  a.r2 = P.r2;
  a.v = P.v;
  a.flags = P.flags;
  a.n_eff = P.n_eff;
  a.sk_i = P.sk_i;
  a.significance = P.significance;
  a.thresholds = nullptr;
  a.n_inputs = P.a.n_inputs;
  a.n_channels = (int32_t)(P.a.row_bytes / P.a.n_inputs);
  a.n_blocks = P.a.n_blocks;
  a.block_len = P.a.block_len;
  a.window = P.window;
  a.hist_len = S.hist_len;
  a.hist_cap = P.hist_cap;
  const int64_t total = (int64_t)S.hist_len + P.a.n_blocks;
  a.hist_next_len = (int32_t)(total < P.hist_cap ? total : P.hist_cap);
  a.chunk = P.chunk;
  a.n_chunks = P.n_chunks;
  a.vec = 4;
  a.estimator = P.estimator;
  a.k_sigma = P.k_sigma;
  a.expect_offset = P.expect_offset;
  a.sigma_override = P.sigma_override;
  return a;
}

// Index of the last entry of a sorted sequence (begin(0) = 0) at or before
// `task`, found by the whole wavefront: each lane compares one entry, and the
// lanes at or before `task` are a prefix, so the highest set bit of their
// ballot is the answer (one load per 64 entries, rather than a chain of
// dependent loads). Called by every lane of the wavefront.
template <typename Begin>
__device__ __forceinline__ int last_at_or_before(int n, int64_t task, Begin begin) {
  const int lane = threadIdx.x & 63;
  int last = 0;
  for (int base = 0; base < n; base += 64) {
    const int j = base + lane;
    const uint64_t m = __ballot(j < n && begin(j) <= task);
    if (m == 0) break;
    last = base + 63 - __builtin_clzll(m);
    if (m != ~0ull) break;
  }
  return __builtin_amdgcn_readfirstlane(last);
}

// Index of the last problem whose range starts at or before `task`.
template <int64_t BatchProb::*BEGIN>
__device__ __forceinline__ int find_prob(const BatchProb* probs, int n, int64_t task) {
  return last_at_or_before(n, task, [&](int j) { return probs[j].*BEGIN; });
}

// Persistent pass A over the whole batch: every workgroup fills its table
// once, then takes two queue units at a time from one device counter until
// the queue is empty (every wavefront then exits). A task of a problem with
// rows of >= 512 column groups is two units and runs on the whole
// workgroup, its blocks' sums held until its last block (as the plan's
// deferred-store pass A); a task of any other problem is one unit and runs
// on one 256-lane half. Every problem starts on an even unit, so a claim is
// one whole task of the first kind or up to two of one problem of the
// second. The halves share each SIMD (wavefronts w and w + 4) and
// SimdBalance keeps them level. Each problem has its own rows per load.
__global__ __launch_bounds__(512) void batch_pass_a_kernel(const BatchProb* __restrict__ probs, int n,
                                                           int64_t total, uint32_t* counter) {
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  __shared__ uint32_t simd_of[8], progress[8];
  __shared__ int64_t s_unit;
  const int tid = threadIdx.x, half = tid >> 8;
  fill_lane_packed_lut<512>(lut32, tid);
  simd_balance_post(simd_of, progress, tid);
  __syncthreads();
  SimdBalance bal = simd_balance_pair(simd_of, progress, 8);
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  for (;;) {
    if (tid == 0) s_unit = (int64_t)atomicAdd(counter, 2u);
    __syncthreads();
    const int64_t u0 = s_unit;
    __syncthreads();
    if (u0 >= total) break;
    const int p = find_prob<&BatchProb::a_begin>(probs, n, u0);
    const BatchProb& P = probs[p];
    if (P.lpr == 512) {
      const int64_t task = (u0 - P.a_begin) >> 1;
      if (task < P.a.n_tasks) {
        const int q = P.a.blocks_per_task;
        if (P.rows == 8) {
          if (q == 4) pass_a_task_deferred<4, 8>(P.a, task, lut, bal);
          else if (q == 2) pass_a_task_deferred<2, 8>(P.a, task, lut, bal);
          else pass_a_task_deferred<1, 8>(P.a, task, lut, bal);
        } else {
          if (q == 4) pass_a_task_deferred<4, 16>(P.a, task, lut, bal);
          else if (q == 2) pass_a_task_deferred<2, 16>(P.a, task, lut, bal);
          else pass_a_task_deferred<1, 16>(P.a, task, lut, bal);
        }
      }
    } else {
      const int64_t task = u0 + half - P.a_begin;   // past the problem's tasks: its padding unit
      if (task < P.a.n_tasks) {
        if (P.rows == 8) pass_a_task_side_by_side<8>(P.a, P.lpr, task, lut, tid & 255, bal);
        else pass_a_task_side_by_side<16>(P.a, P.lpr, task, lut, tid & 255, bal);
      }
    }
  }
}

// Wavefronts of a batched scan workgroup. Eight rather than sixteen: the
// kernel's registers allow three such workgroups per CU against one of
// sixteen wavefronts, so more rows are in flight.
constexpr int BATCH_SCAN_WAVES = 8;

// Scan workgroups of the whole batch: (problem, channel, group of 64-input
// slices), BATCH_SCAN_WAVES wavefronts, Ws per slice (the problem's
// scan_waves) and BATCH_SCAN_WAVES / Ws slices per workgroup. The chunk
// length is read at run time (scan_body_rows); the prefix sums are exact
// integers, so they equal the single-plan kernel's.
__global__ __launch_bounds__(64 * BATCH_SCAN_WAVES) void batch_scan_kernel(const BatchProb* __restrict__ probs,
                                                                        const BatchState* __restrict__ st, int n) {
  __shared__ uint32_t lds[BATCH_SCAN_WAVES * 64];
  const int64_t task = blockIdx.x;
  const int p = find_prob<&BatchProb::sc_begin>(probs, n, task);
  const BatchProb& P = probs[p];
  const int64_t lt = task - P.sc_begin;
  if (lt >= P.sc_count) return;                       // whole workgroup
  const PassBArgs a = make_args(P, st[p]);
  const int Ws = P.scan_waves, spw = BATCH_SCAN_WAVES / Ws;
  const int slices = (a.n_inputs + 63) / 64;
  const int groups = (slices + spw - 1) / spw;
  const int f = (int)(lt / groups);
  const int w = wave_id(), sub = w / Ws;
  const int slice = (int)(lt % groups) * spw + sub;   // >= slices: every lane idle, barriers kept
  scan_body_rows(a, f, slice, w % Ws, Ws, lds + sub * Ws * 64);
}

// What a call does after its last kernel: advance every problem's history
// length and ping-pong parity, and re-arm the pass A queue.
__device__ __forceinline__ void advance_state(const BatchProb* __restrict__ probs, BatchState* st, int n,
                                              uint32_t* counter, int tid, int threads) {
  for (int p = tid; p < n; p += threads) {
    if (probs[p].window >= 2) {
      const int64_t total = (int64_t)st[p].hist_len + probs[p].a.n_blocks;
      st[p].hist_len = (int32_t)(total < probs[p].hist_cap ? total : probs[p].hist_cap);
      st[p].parity ^= 1;
    }
  }
  if (tid == 0) *counter = 0u;
}

// The last combine launch of a call also advances the state: its last
// workgroup to finish (a count in done[0], cleared again by that workgroup)
// runs advance_state once every workgroup has read the state it needs. The
// count is a relaxed atomic: each workgroup adds to it after its last read.
struct BatchFinal {
  BatchState* st;        // null: not the last launch (or a tuning run)
  uint32_t* counter;     // pass A queue counter
  uint32_t* done;        // workgroups of this launch that have finished
  int n;
};

// Combine workgroups of one class of problems (chunk length R, 32- or 64-bit
// R1/R2 sums):
// (problem, channel, group of 8 / W chunks), 8 wavefronts, W per chunk as in
// the single-plan kernel (so results equal the plan's bit for bit); a problem
// of narrow rows (W < 8) puts 8 / W chunks into one workgroup instead of
// leaving wavefronts idle. members[0 .. count) are the class's table
// positions, begins[] their first workgroups.
template <int R, typename RI, bool OFF32>
__global__ __launch_bounds__(64 * COMBINE_MAX_WAVES) void batch_combine_kernel(
    const BatchProb* __restrict__ probs, const BatchState* st, const int32_t* __restrict__ members,
    const int64_t* __restrict__ begins, int count, BatchFinal fin) {
  __shared__ CombineShared sh[COMBINE_MAX_WAVES];
  __shared__ uint32_t last_out;
  const int64_t task = blockIdx.x;
  const int p = members[last_at_or_before(count, task, [&](int j) { return begins[j]; })];
  const BatchProb& P = probs[p];
  const int64_t lt = task - P.cb_begin;
  if (lt < P.cb_count) {                              // else the whole workgroup is idle
    const PassBArgs a = make_args(P, st[p]);
    const int W = P.waves, cpw = COMBINE_MAX_WAVES / W;
    const int groups = (a.n_chunks + cpw - 1) / cpw;
    const int f = (int)(lt / groups);
    const int w = wave_id(), sub = w / W;
    const int k = (int)(lt % groups) * cpw + sub;
    const bool live = sub < cpw && k < a.n_chunks;
    combine_body<4, R, RI, OFF32>(a, k, f, w % W, W, sh[sub < cpw ? sub : 0], live);
  }
  if (fin.st) {
    __syncthreads();   // every wavefront of this workgroup has read the state
    if (threadIdx.x == 0) last_out = atomicAdd(fin.done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (last_out) {
      advance_state(probs, fin.st, fin.n, fin.counter, threadIdx.x, blockDim.x);
      if (threadIdx.x == 0) *fin.done = 0u;
    }
  }
}

// Last node: advance every problem's history and rearm the work queue.
__global__ __launch_bounds__(256) void batch_state_kernel(const BatchProb* __restrict__ probs,
                                                          BatchState* st, int n, uint32_t* counter) {
  advance_state(probs, st, n, counter, threadIdx.x, 256);
}

}  // namespace sk

using namespace sk;

// ------------------------------------------------------------------ tuning cache

namespace {

std::string cache_path(const sk_batch_opts* o) {
  if (o && o->tune_cache) return o->tune_cache;
  const char* e = getenv("SK_TUNE_CACHE");
  return e ? e : "";
}

// Flat JSON object of "key": integer pairs (any layout; keys hold no
// escaped quotes). Anything else in the file is skipped.
std::map<std::string, int> load_cache(const std::string& path) {
  std::map<std::string, int> m;
  if (path.empty()) return m;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return m;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  fclose(f);
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    size_t q = end + 1;
    while (q < text.size() && (text[q] == ' ' || text[q] == '\t' || text[q] == '\n' || text[q] == '\r')) ++q;
    if (q < text.size() && text[q] == ':') {
      char* stop = nullptr;
      const long v = strtol(text.c_str() + q + 1, &stop, 10);
      if (stop != text.c_str() + q + 1) m[key] = (int)v;
      pos = stop ? (size_t)(stop - text.c_str()) : q + 1;
    } else {
      pos = end + 1;
    }
  }
  return m;
}

void save_cache(const std::string& path, const std::map<std::string, int>& m) {
  if (path.empty()) return;
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++k < m.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path.c_str());
}

}  // namespace

// Task ranges of every kernel over a table of problems. Combine classes:
// chunk length R in {1, 2, 4} (class R / 2 = 0, 1, 2) plus 3 when the R1/R2
// sums need 64 bits.
constexpr int N_COMBINE_CLASSES = 6;

__host__ __device__ __forceinline__ int combine_class(int chunk, int wide_sums) {
  return (chunk == 1 ? 0 : chunk == 2 ? 1 : 2) + 3 * wide_sums;
}

struct Layout {
  int64_t ta = 0, tsc = 0;
  int64_t tcb[N_COMBINE_CLASSES] = {};
  int cls_off[N_COMBINE_CLASSES] = {}, cls_cnt[N_COMBINE_CLASSES] = {};
  std::vector<int32_t> members;
  std::vector<int64_t> begins;
  bool off32 = true;
};

struct sk_batch_s {
  int n = 0;
  int device = 0;
  std::string arch;
  std::vector<sk_plan_desc> desc;
  std::vector<BatchProb> host;     // host copy of the table
  std::vector<int> order;          // table position -> caller's problem index
  BatchProb* d_probs = nullptr;
  BatchState* d_state = nullptr;
  uint32_t* d_counter = nullptr;
  int32_t* d_members = nullptr;    // combine classes: table positions, class by class
  int64_t* d_begins = nullptr;     // and their first combine workgroups
  std::vector<void*> owned;
  int grid_a = 0;
  Layout lay;                      // task ranges of the table as it is on the device
  std::vector<int> tuned_from_cache;   // per table position: 1 if its class's pick came from the cache
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(sk_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (void* p : b->owned) (void)hipFree(p);
  if (b->d_probs) (void)hipFree(b->d_probs);
  if (b->d_state) (void)hipFree(b->d_state);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->d_members) (void)hipFree(b->d_members);
  if (b->d_begins) (void)hipFree(b->d_begins);
  delete b;
}

static int batch_alloc(sk_batch_s* b, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return SK_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return SK_ERR_NOMEM;
  }
  b->owned.push_back(*p);
  return SK_OK;
}

// Pass A settings of one problem: rows per load (8, 16) and, for wide rows,
// consecutive blocks per task.
static void set_pass_a(BatchProb& P, int rows, int q) {
  P.a.cs = nullptr;             // set by set_pass_b, which follows
  P.a.timeline = nullptr;
  P.a.simd_balance = 1;
  P.rows = rows;
  P.a.block0 = 0;
  P.a.block_end = P.a.n_blocks;
  P.a.blocks_per_task = P.lpr >= 256 ? q : 256 / P.lpr;
  P.a.chunks = P.lpr >= 256 ? (P.a.col_groups + P.lpr - 1) / P.lpr : 1;
  P.a.n_tasks = (((int64_t)P.a.n_blocks + P.a.blocks_per_task - 1) / P.a.blocks_per_task) * P.a.chunks;
}

// Pass B chunk length of one problem. When pass A's wide-row tasks walk
// exactly one chunk, they write its S1 total and the scan reads those chunk
// sums instead of the rows.
static void set_pass_b(BatchProb& P, int R) {
  P.chunk = R;
  P.n_chunks = (int32_t)((P.a.n_blocks + R - 1) / R);
  const bool cs = P.cs_buf && P.lpr >= 256 && R >= 2 && P.a.blocks_per_task == R;
  P.a.cs = cs ? P.cs_buf : nullptr;
  // Waves per slice: enough for the units in SCAN_ROWS-unit lanes, and for
  // the history rows moved once the history is full (a call shorter than the
  // window), a power of two.
  int w = scan_rows_waves(cs ? P.n_chunks : P.a.n_blocks, BATCH_SCAN_WAVES);
  const int64_t sg = shift_groups(P.hist_cap, P.a.n_blocks);
  while (w < BATCH_SCAN_WAVES && w < sg) w *= 2;
  P.scan_waves = w;
}

static Layout layout(std::vector<BatchProb>& tab) {
  Layout l;
  for (BatchProb& P : tab) {
    const int64_t F = P.a.row_bytes / P.a.n_inputs;
    // Queue units: two per task of 512-group rows, one otherwise; every
    // problem starts on an even unit.
    P.a_begin = (l.ta + 1) & ~(int64_t)1;
    l.ta = P.a_begin + P.a.n_tasks * (P.lpr == 512 ? 2 : 1);
    P.sc_begin = l.tsc;
    const int slices = (P.a.n_inputs + 63) / 64, spw = BATCH_SCAN_WAVES / P.scan_waves;
    P.sc_count = (P.a.n_blocks > 0 && pass_b_needs_scan(P.window, P.chunk, P.a.n_blocks))
                     ? F * ((slices + spw - 1) / spw) : 0;
    l.tsc += P.sc_count;
    if (!combine_offsets_fit_32(P.a.n_inputs, P.a.n_blocks, P.n_chunks, P.hist_cap)) l.off32 = false;
  }
  for (int c = 0; c < N_COMBINE_CLASSES; ++c) {
    l.cls_off[c] = (int)l.members.size();
    for (size_t q = 0; q < tab.size(); ++q) {
      BatchProb& P = tab[q];
      if (combine_class(P.chunk, P.wide_sums) != c) continue;
      const int64_t F = P.a.row_bytes / P.a.n_inputs;
      const int cpw = COMBINE_MAX_WAVES / P.waves;
      P.cb_begin = l.tcb[c];
      P.cb_count = F * ((P.n_chunks + cpw - 1) / cpw);
      l.tcb[c] += P.cb_count;
      l.members.push_back((int32_t)q);
      l.begins.push_back(P.cb_begin);
    }
    l.cls_cnt[c] = (int)l.members.size() - l.cls_off[c];
  }
  return l;
}

// Device copies of a table and its combine class lists (capacity n).
struct DeviceTable {
  BatchProb* probs;
  int32_t* members;
  int64_t* begins;
};

static hipError_t upload_table(const DeviceTable& d, const std::vector<BatchProb>& tab, const Layout& l,
                               hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d.probs, tab.data(), sizeof(BatchProb) * tab.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d.members, l.members.data(), sizeof(int32_t) * l.members.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d.begins, l.begins.data(), sizeof(int64_t) * l.begins.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

static void launch_pass_a_table(const BatchProb* d_tab, int n, int64_t total, int grid, uint32_t* counter,
                                hipStream_t s) {
  batch_pass_a_kernel<<<dim3(grid), dim3(512), 0, s>>>(d_tab, n, total, counter);
}

template <int R, typename RI>
static void launch_combine_class(const DeviceTable& d, BatchState* st, const Layout& l, hipStream_t s,
                                 const BatchFinal& fin, int last_class) {
  const int c = combine_class(R, sizeof(RI) == 8 ? 1 : 0);
  if (l.tcb[c] <= 0) return;
  const dim3 grid((unsigned)l.tcb[c]), wg(64 * COMBINE_MAX_WAVES);
  const int32_t* m = d.members + l.cls_off[c];
  const int64_t* bg = d.begins + l.cls_off[c];
  const BatchFinal f = c == last_class ? fin : BatchFinal{nullptr, nullptr, nullptr, 0};
  if (l.off32) batch_combine_kernel<R, RI, true><<<grid, wg, 0, s>>>(d.probs, st, m, bg, l.cls_cnt[c], f);
  else batch_combine_kernel<R, RI, false><<<grid, wg, 0, s>>>(d.probs, st, m, bg, l.cls_cnt[c], f);
}

// Combine classes in launch order.
static const int kCombineOrder[N_COMBINE_CLASSES][2] = {{4, 0}, {2, 0}, {1, 0}, {4, 1}, {2, 1}, {1, 1}};

// The class whose combine launch comes last in a call, or -1 without one.
static int last_combine_class(const Layout& l) {
  int last = -1;
  for (const auto& rc : kCombineOrder) {
    const int c = combine_class(rc[0], rc[1]);
    if (l.tcb[c] > 0) last = c;
  }
  return last;
}

// Scan, then one combine launch per nonempty class, the longest first. With
// fin.st set, the last combine launch also advances the state (the caller
// launches batch_state_kernel instead when there is no combine launch).
static void launch_pass_b_table(const DeviceTable& d, BatchState* st, int n, const Layout& l, hipStream_t s,
                                const BatchFinal& fin = BatchFinal{nullptr, nullptr, nullptr, 0}) {
  if (l.tsc > 0) batch_scan_kernel<<<dim3((unsigned)l.tsc), dim3(64 * BATCH_SCAN_WAVES), 0, s>>>(d.probs, st, n);
  const int last = fin.st ? last_combine_class(l) : -1;
  launch_combine_class<4, int32_t>(d, st, l, s, fin, last);
  launch_combine_class<2, int32_t>(d, st, l, s, fin, last);
  launch_combine_class<1, int32_t>(d, st, l, s, fin, last);
  launch_combine_class<4, int64_t>(d, st, l, s, fin, last);
  launch_combine_class<2, int64_t>(d, st, l, s, fin, last);
  launch_combine_class<1, int64_t>(d, st, l, s, fin, last);
}

static DeviceTable device_table(const sk_batch_s* b) { return DeviceTable{b->d_probs, b->d_members, b->d_begins}; }

static int launch_sequence(sk_batch_s* b, hipStream_t s) {
  launch_pass_a_table(b->d_probs, b->n, b->lay.ta, b->grid_a, b->d_counter, s);
  SK_HIP_TRY(hipGetLastError());
  const BatchFinal fin{b->d_state, b->d_counter, b->d_counter + 1, b->n};
  launch_pass_b_table(device_table(b), b->d_state, b->n, b->lay, s, fin);
  SK_HIP_TRY(hipGetLastError());
  if (last_combine_class(b->lay) < 0) {
    batch_state_kernel<<<dim3(1), dim3(256), 0, s>>>(b->d_probs, b->d_state, b->n, b->d_counter);
    SK_HIP_TRY(hipGetLastError());
  }
  return SK_OK;
}

// Best of `reps` timed runs of `run` (after one untimed run), in ms; the
// queue counter is cleared before every pass A run. Runs before any graph
// capture.
template <typename Fn>
static float best_time(hipStream_t s, uint32_t* counter, int reps, Fn run) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e30f;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return 1e30f; }
  float best = 1e30f;
  for (int rep = 0; rep <= reps; ++rep) {
    (void)hipMemsetAsync(counter, 0, sizeof(uint32_t), s);
    (void)hipEventRecord(e0, s);
    run();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && ms < best) best = ms;     // the first run warms up
  }
  (void)hipMemsetAsync(counter, 0, sizeof(uint32_t), s);
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Pass A of the whole batch alone (profiling), best of three.
static float time_pass_a_batch(sk_batch_s* b, hipStream_t s) {
  return best_time(s, b->d_counter, 3,
                   [&] { launch_pass_a_table(b->d_probs, b->n, b->lay.ta, b->grid_a, b->d_counter, s); });
}

// Autotuner. Problems are grouped by class (N, M, F). For each class not in
// the cache, the class's problems alone (a sub-table) are timed with every
// candidate, best of kTuneReps launches after one untimed: first pass A alone
// over rows per load {8, 16} x blocks per task {1, 2, 4} (wide rows; 1 for
// narrow rows), then whole calls (pass A and pass B) with the best rows and
// blocks over pass B chunk length {1, 2, 4}, and, for wide rows with a
// window, with blocks per task equal to the chunk {2, 4} (pass A then hands
// the scan its chunk sums). The least whole-call time is kept. Every
// candidate's time (ns) and the pick go into the cache, keyed by the device
// arch and the class; a class found in the cache takes its pick without
// timing.
// Timed launches per tuning candidate (the least is kept): candidates of one
// class often differ by a few microseconds, about the spread of single runs.
constexpr int kTuneReps = 5;

static int tune_batch(sk_batch_s* b, const std::string& path, hipStream_t s) {
  std::map<std::string, int> cache = load_cache(path);
  std::map<std::string, std::vector<int>> classes;
  for (int q = 0; q < b->n; ++q) {
    const BatchProb& P = b->host[q];
    char key[256];
    snprintf(key, sizeof key, "%s|batch|N=%d|M=%d|F=%d", b->arch.c_str(), P.a.n_inputs, P.a.block_len,
             (int)(P.a.row_bytes / P.a.n_inputs));
    classes[key].push_back(q);
  }
  DeviceTable d{nullptr, nullptr, nullptr};
  if (hipMalloc((void**)&d.probs, sizeof(BatchProb) * b->n) != hipSuccess ||
      hipMalloc((void**)&d.members, sizeof(int32_t) * b->n) != hipSuccess ||
      hipMalloc((void**)&d.begins, sizeof(int64_t) * b->n) != hipSuccess) {
    if (d.probs) (void)hipFree(d.probs);
    if (d.members) (void)hipFree(d.members);
    set_error("hipMalloc of the tuning table failed");
    return SK_ERR_NOMEM;
  }
  bool dirty = false;
  int rc = SK_OK;
  for (auto& kv : classes) {
    const std::string& key = kv.first;
    const std::vector<int>& members = kv.second;
    auto it = cache.find(key + "|pick");
    int rows = 16, q = 1, R = 4;
    if (it != cache.end()) {
      rows = it->second / 100;
      q = it->second / 10 % 10;
      R = it->second % 10;
      for (int m : members) b->tuned_from_cache[m] = 1;
    } else {
      std::vector<BatchProb> sub;
      for (int m : members) sub.push_back(b->host[m]);
      const bool wide = sub[0].lpr >= 256;
      // Step 1: pass A alone over rows per load x blocks per task.
      float best = 1e30f;
      for (int rr : {8, 16}) {
        for (int qq : {1, 2, 4}) {
          if (qq > 1 && !wide) continue;
          for (BatchProb& P : sub) { set_pass_a(P, rr, qq); set_pass_b(P, P.chunk); }
          const Layout l = layout(sub);
          if (upload_table(d, sub, l, s) != hipSuccess) {
            rc = SK_ERR_DEVICE;
            break;
          }
          const float t = best_time(s, b->d_counter, kTuneReps, [&] {
            launch_pass_a_table(d.probs, (int)sub.size(), l.ta, b->grid_a, b->d_counter, s);
          });
          char ck[320];
          snprintf(ck, sizeof ck, "%s|A|rows=%d|blocks=%d", key.c_str(), rr, qq);
          cache[ck] = (int)(t * 1e6f);
          if (t < best) { best = t; rows = rr; q = qq; }
        }
        if (rc) break;
      }
      // Step 2: whole calls (pass A, then pass B) over the chunk length,
      // with step 1's pass A, and for wide rows also with tasks of one chunk
      // (pass A then writes the chunk sums the scan reads).
      std::vector<std::pair<int, int>> ab;   // (blocks per task, chunk)
      for (int RR : {1, 2, 4}) ab.push_back({q, RR});
      if (wide && sub[0].window >= 2)
        for (int RR : {2, 4})
          if (RR != q) ab.push_back({RR, RR});
      best = 1e30f;
      for (const auto& c : ab) {
        if (rc) break;
        for (BatchProb& P : sub) { set_pass_a(P, rows, c.first); set_pass_b(P, c.second); }
        const Layout l = layout(sub);
        if (upload_table(d, sub, l, s) != hipSuccess) {
          rc = SK_ERR_DEVICE;
          break;
        }
        const float t = best_time(s, b->d_counter, kTuneReps, [&] {
          launch_pass_a_table(d.probs, (int)sub.size(), l.ta, b->grid_a, b->d_counter, s);
          launch_pass_b_table(d, b->d_state, (int)sub.size(), l, s);
        });
        char ck[320];
        snprintf(ck, sizeof ck, "%s|AB|rows=%d|blocks=%d|chunk=%d", key.c_str(), rows, c.first, c.second);
        cache[ck] = (int)(t * 1e6f);
        if (t < best) { best = t; q = c.first; R = c.second; }
      }
      cache[key + "|pick"] = rows * 100 + q * 10 + R;
      dirty = true;
    }
    for (int m : members) {
      set_pass_a(b->host[m], rows, q);
      set_pass_b(b->host[m], R);
    }
    if (rc) break;
  }
  (void)hipFree(d.probs);
  (void)hipFree(d.members);
  (void)hipFree(d.begins);
  if (rc == SK_OK && hipGetLastError() != hipSuccess) rc = SK_ERR_DEVICE;
  if (rc) { set_error("autotuning launch failed"); return rc; }
  if (dirty) save_cache(path, cache);
  return SK_OK;
}

extern "C" {

int sk_batch_create(const sk_plan_desc* descs, int32_t n, const sk_batch_opts* opts,
                    const uint8_t* const* d_inputs, const sk_outputs* outs, sk_batch_t* out) {
  clear_error();
  if (!out || !descs || !d_inputs || !outs || n < 1) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  *out = nullptr;
  for (int j = 0; j < n; ++j) {
    int rc = validate_desc(&descs[j]);
    if (rc) { std::string m = sk_last_error(); set_error("problem %d: %s", j, m.c_str()); return rc; }
    if (descs[j].n_inputs % 16 != 0 || ((uintptr_t)d_inputs[j] % 16) != 0) {
      set_error("problem %d: batched problems need N %% 16 == 0 and 16-byte aligned inputs", j);
      return SK_ERR_SHAPE;
    }
  }
  sk_batch_s* b = new sk_batch_s();
  b->n = n;
  b->desc.assign(descs, descs + n);
  if (hipGetDevice(&b->device) != hipSuccess) { batch_free(b); set_error("no HIP device"); return SK_ERR_DEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) { batch_free(b); set_error("device query failed"); return SK_ERR_DEVICE; }
  b->arch = prop.gcnArchName;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_pass_a_kernel, 512, 0) != hipSuccess || occ < 1) occ = 1;
  b->grid_a = occ * prop.multiProcessorCount;
  b->use_graph = !opts || opts->use_graph;

  // Table order while tuning: largest problems first (the queue order is
  // set after tuning, below).
  b->order.resize(n);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
    return (int64_t)descs[x].block_len * descs[x].n_inputs * descs[x].n_channels >
           (int64_t)descs[y].block_len * descs[y].n_inputs * descs[y].n_channels;
  });

  b->host.resize(n);
  int rc = SK_OK;
  for (int q = 0; q < n && rc == SK_OK; ++q) {
    const int j = b->order[q];
    const sk_plan_desc& d = descs[j];
    BatchProb& P = b->host[q];
    memset(&P, 0, sizeof P);
    const int64_t N = d.n_inputs, F = d.n_channels, B = d.n_samples / d.block_len;
    const int L = d.norm_window_blocks;
    P.a.x = d_inputs[j];
    P.a.row_bytes = F * N;
    P.a.n_inputs = (int32_t)N;
    P.a.block_len = d.block_len;
    P.a.n_blocks = (int32_t)B;
    P.a.col_groups = (int32_t)(F * N / 16);
    {
      int lpb = 1;
      while (lpb < 256 && lpb < P.a.col_groups) lpb *= 2;
      P.lpr = P.a.col_groups >= 512 ? 512 : lpb;
    }
    P.window = L;
    P.hist_cap = L >= 2 ? L - 1 : 0;
    P.estimator = d.estimator;
    P.k_sigma = d.k_sigma;
    P.expect_offset = d.expect_offset;
    P.sigma_override = d.sigma_override;
    P.waves = combine_waves((int32_t)N, 4);
    P.wide_sums = combine_sums_fit_32((int32_t)N, 4, d.block_len) ? 0 : 1;
    P.mask = nullptr;
    const sk_outputs& o = outs[j];
    const size_t fbn = (size_t)F * B * N;
    void* p = nullptr;
    if (o.s1) P.a.s1 = o.s1; else { rc = batch_alloc(b, &p, fbn * 4); P.a.s1 = (int32_t*)p; }
    if (rc) break;
    if (o.s2) P.a.s2 = o.s2; else { rc = batch_alloc(b, &p, fbn * 4); P.a.s2 = (int32_t*)p; }
    if (rc) break;
    if (((uintptr_t)P.a.s1 | (uintptr_t)P.a.s2) % 16) { set_error("problem %d: outputs s1/s2 must be 16-byte aligned", j); rc = SK_ERR_INVALID_ARG; break; }
    if (L >= 2) {
      // Prefix sums for the shortest chunk the autotuner may pick (R = 1).
      if ((rc = batch_alloc(b, &p, pass_b_prefix_bytes((int32_t)N, (int32_t)F, B, 1)))) break;
      P.pc = (uint32_t*)p;
      if (P.lpr >= 256 && B >= 2) {
        if ((rc = batch_alloc(b, &p, (size_t)F * (size_t)((B + 1) / 2) * N * 4))) break;
        P.cs_buf = (int32_t*)p;
      }
      if ((rc = batch_alloc(b, &p, (size_t)F * P.hist_cap * N * 4))) break;
      P.hs[0] = (int32_t*)p;
      if ((rc = batch_alloc(b, &p, (size_t)F * P.hist_cap * N * 4))) break;
      P.hs[1] = (int32_t*)p;
    }
    set_pass_a(P, 16, 1);
    set_pass_b(P, pass_b_chunk((int32_t)N, (int32_t)F, B, L));
    P.r1 = o.r1;
    P.r2 = o.r2;
    P.v = o.v;
    P.flags = o.flags;
    P.n_eff = o.n_eff;
    P.sk_i = o.sk_i;
    P.significance = o.significance;
    if ((uintptr_t)P.sk_i % 16) { set_error("problem %d: output sk_i must be 16-byte aligned", j); rc = SK_ERR_INVALID_ARG; break; }
  }
  if (rc) { batch_free(b); return rc; }

  hipStream_t s = nullptr;
  if (hipStreamCreate(&b->cap_stream) != hipSuccess) { batch_free(b); set_error("stream create failed"); return SK_ERR_DEVICE; }
  s = b->cap_stream;

  void* p = nullptr;
  if ((rc = batch_alloc(b, &p, sizeof(BatchProb) * n))) { batch_free(b); return rc; }
  b->owned.pop_back();
  b->d_probs = (BatchProb*)p;
  if ((rc = batch_alloc(b, &p, sizeof(BatchState) * n))) { batch_free(b); return rc; }
  b->owned.pop_back();
  b->d_state = (BatchState*)p;
  // [0] pass A queue, [1] finished workgroups of the last combine launch.
  if ((rc = batch_alloc(b, &p, 2 * sizeof(uint32_t)))) { batch_free(b); return rc; }
  b->owned.pop_back();
  b->d_counter = (uint32_t*)p;
  if ((rc = batch_alloc(b, &p, sizeof(int32_t) * n))) { batch_free(b); return rc; }
  b->owned.pop_back();
  b->d_members = (int32_t*)p;
  if ((rc = batch_alloc(b, &p, sizeof(int64_t) * n))) { batch_free(b); return rc; }
  b->owned.pop_back();
  b->d_begins = (int64_t*)p;
  std::vector<BatchState> st(n, BatchState{0, 0});
  (void)layout(b->host);
  if (hipMemcpyAsync(b->d_probs, b->host.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b->d_state, st.data(), sizeof(BatchState) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(b->d_counter, 0, 2 * sizeof(uint32_t), s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    batch_free(b);
    set_error("batch table upload failed");
    return SK_ERR_DEVICE;
  }

  // Per-class tile choices: timed on this batch's problems, or from the
  // cache keyed by (arch, N, M, F).
  b->tuned_from_cache.assign(n, 0);
  const bool tune = !opts || opts->autotune;
  if (tune) {
    rc = tune_batch(b, cache_path(opts), s);
    if (rc) { batch_free(b); return rc; }
  }
  // Longest tasks first. A task's duration is set by the rows each lane
  // walks one after the other (M per block, times the blocks a wide-row task
  // walks), not by its bytes: those lead the queue and the short tasks fill
  // in behind them, so no long task starts when the queue is nearly empty.
  // Ties go to the larger problem.
  {
    auto walk = [](const BatchProb& P) {
      return (int64_t)P.a.block_len * (P.lpr >= 256 ? P.a.blocks_per_task : 1);
    };
    auto bytes = [](const BatchProb& P) { return (int64_t)P.a.n_blocks * P.a.block_len * P.a.row_bytes; };
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
      const int64_t wx = walk(b->host[x]), wy = walk(b->host[y]);
      if (wx != wy) return wx > wy;
      return bytes(b->host[x]) > bytes(b->host[y]);
    });
    std::vector<BatchProb> host(n);
    std::vector<int> order(n), cached(n);
    for (int q = 0; q < n; ++q) {
      host[q] = b->host[perm[q]];
      order[q] = b->order[perm[q]];
      cached[q] = b->tuned_from_cache[perm[q]];
    }
    b->host.swap(host);
    b->order.swap(order);
    b->tuned_from_cache.swap(cached);
  }
  {
    b->lay = layout(b->host);
    const Layout& l = b->lay;
    // The work-queue counter runs past the last task by one claim per
    // workgroup; it must not wrap. Grids stay within 2^31 workgroups.
    bool big = l.ta + (1LL << 24) >= (int64_t)UINT32_MAX || l.tsc >= (1LL << 31);
    for (int c = 0; c < N_COMBINE_CLASSES; ++c) big = big || l.tcb[c] >= (1LL << 31);
    if (big) {
      batch_free(b);
      set_error("batch too large");
      return SK_ERR_SHAPE;
    }
    if (upload_table(device_table(b), b->host, l, s) != hipSuccess ||
        hipMemsetAsync(b->d_counter, 0, 2 * sizeof(uint32_t), s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      batch_free(b);
      set_error("batch table upload failed");
      return SK_ERR_DEVICE;
    }
  }

  if (b->use_graph) {
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) { batch_free(b); set_error("graph capture failed"); return SK_ERR_DEVICE; }
    rc = launch_sequence(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc || e != hipSuccess) { if (g) (void)hipGraphDestroy(g); batch_free(b); if (!rc) set_error("graph capture failed"); return rc ? rc : SK_ERR_DEVICE; }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) { batch_free(b); set_error("graph instantiate failed"); return SK_ERR_DEVICE; }
  }
  *out = b;
  return SK_OK;
}

int sk_batch_compute(sk_batch_t b, const uint8_t* const* d_inputs, void* stream) {
  clear_error();
  if (!b) { set_error("NULL batch"); return SK_ERR_INVALID_ARG; }
  hipStream_t s = (hipStream_t)stream;
  if (d_inputs) {
    bool changed = false;
    for (int q = 0; q < b->n; ++q) {
      const uint8_t* x = d_inputs[b->order[q]];
      if (!x || (uintptr_t)x % 16) { set_error("input %d is NULL or not 16-byte aligned", b->order[q]); return SK_ERR_INVALID_ARG; }
      if (x != b->host[q].a.x) { b->host[q].a.x = x; changed = true; }
    }
    if (changed) SK_HIP_TRY(hipMemcpyAsync(b->d_probs, b->host.data(), sizeof(BatchProb) * b->n, hipMemcpyHostToDevice, s));
  }
  if (b->exec) {
    SK_HIP_TRY(hipGraphLaunch(b->exec, s));
    return SK_OK;
  }
  return launch_sequence(b, s);
}

int sk_batch_state_reset(sk_batch_t b, void* stream) {
  clear_error();
  if (!b) { set_error("NULL batch"); return SK_ERR_INVALID_ARG; }
  std::vector<BatchState> st(b->n, BatchState{0, 0});
  hipStream_t s = (hipStream_t)stream;
  SK_HIP_TRY(hipMemcpyAsync(b->d_state, st.data(), sizeof(BatchState) * b->n, hipMemcpyHostToDevice, s));
  SK_HIP_TRY(hipStreamSynchronize(s));
  return SK_OK;
}

int sk_batch_get_tiles(sk_batch_t b, int32_t j, int32_t* lpr, int32_t* grid) {
  if (!b || j < 0 || j >= b->n || !lpr || !grid) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  for (int q = 0; q < b->n; ++q)
    if (b->order[q] == j) *lpr = b->host[q].lpr;
  *grid = b->grid_a;
  return SK_OK;
}

int sk_batch_get_tuning(sk_batch_t b, int32_t j, int32_t* rows, int32_t* blocks, int32_t* chunk,
                        int32_t* from_cache) {
  clear_error();
  if (!b || j < 0 || j >= b->n || !rows || !blocks || !chunk || !from_cache) {
    set_error("bad arguments");
    return SK_ERR_INVALID_ARG;
  }
  for (int q = 0; q < b->n; ++q) {
    if (b->order[q] != j) continue;
    const BatchProb& P = b->host[q];
    *rows = P.rows;
    *blocks = P.a.blocks_per_task;
    *chunk = P.chunk;
    *from_cache = b->tuned_from_cache.empty() ? 0 : b->tuned_from_cache[q];
  }
  return SK_OK;
}

int sk_batch_time_pass_a(sk_batch_t b, void* stream, float* ms) {
  clear_error();
  if (!b || !ms) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) {
    set_error("batch was created on device %d, current device is %d", b->device, dev);
    return SK_ERR_INVALID_ARG;
  }
  const float t = time_pass_a_batch(b, (hipStream_t)stream);
  SK_HIP_TRY(hipGetLastError());
  if (!(t < 1e29f)) { set_error("pass A timing failed"); return SK_ERR_DEVICE; }
  *ms = t;
  return SK_OK;
}

int sk_batch_get_state(sk_batch_t b, int32_t j, int32_t* hist_len) {
  clear_error();
  if (!b || j < 0 || j >= b->n || !hist_len) { set_error("bad arguments"); return SK_ERR_INVALID_ARG; }
  SK_HIP_TRY(hipDeviceSynchronize());
  for (int q = 0; q < b->n; ++q) {
    if (b->order[q] != j) continue;
    BatchState st;
    SK_HIP_TRY(hipMemcpy(&st, b->d_state + q, sizeof st, hipMemcpyDeviceToHost));
    *hist_len = st.hist_len;
  }
  return SK_OK;
}

int sk_batch_destroy(sk_batch_t b) {
  clear_error();
  if (!b) return SK_OK;
  (void)hipDeviceSynchronize();
  batch_free(b);
  return SK_OK;
}

}  // extern "C"
