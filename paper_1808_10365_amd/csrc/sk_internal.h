// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <string>

#include "sk.h"

namespace sk {

// Thread-local error message behind sk_last_error().
void set_error(const char* fmt, ...);
void clear_error();

#define SK_HIP_TRY(expr)                                                          \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::sk::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                      __FILE__, __LINE__);                                        \
      return SK_ERR_DEVICE;                                                       \
    }                                                                             \
  } while (0)

// ---------------------------------------------------------------- pass A
// Per-input block sums S1 = sum p, S2 = sum p^2 over the M samples of a block
// (Eq. singlesums), for every (channel, block, input), from bytes [T][F][N].
//
// A row of the input is the G = F*N bytes of one time sample. A lane owns VEC
// consecutive columns (inputs of one channel: N % VEC == 0) and walks rows.
// A workgroup of 256 lanes covers LPR column groups times RP = 256/LPR row
// phases of one block; partial sums of the row phases meet in LDS.
struct PassATask {
  const uint8_t* x;     // [T][F][N] bytes of this call
  int32_t* s1;          // [F][B][N]
  int32_t* s2;          // [F][B][N]
  int64_t row_bytes;    // G = F * N
  int32_t n_inputs;     // N
  int32_t block_len;    // M
  int32_t n_blocks;     // B
  int32_t col_groups;   // G / VEC
  int32_t chunks;       // ceil(col_groups / (LPR * groups per lane))
  int64_t n_tasks;      // blocks of this launch * chunks
  int32_t block0;       // first block of this launch (tasks cover blocks block0 ..)
  int32_t block_end;    // one past the last block of this launch
  int32_t blocks_per_task;  // consecutive blocks one task walks (packed-table variants; else 1)
  int32_t* cs;          // variant 4 only, or null: [F][ceil(B / Q)][N] S1 summed over each
                        // task's Q blocks (the chunk sums of pass B's scan when its R == Q)
  uint64_t* timeline;   // variant 4 only, or null: 6 words per wavefront (see
                        // sk_plan_pass_a_timeline), one task per workgroup
  int32_t simd_balance; // variant 4: 1 = wavefronts of a SIMD kept level (the library's
                        // setting), 0 = left to the arbiter (timeline comparisons only)
};

struct PassAConfig {
  int vec;     // 16, 4 or 1 bytes per lane per row
  int lpr;     // lanes per row: power of two, 1..256
  int variant; // 0 shared table; 16-byte path: 1, 2 packed, 3 side by side, 4 deferred stores
  int grid;    // workgroups launched (<= tasks; grid-stride beyond)
};

// Timing of a pass, recorded by the kernel dispatches themselves (either
// event may be null): `start` when the pass's first kernel starts, `stop`
// when its last one ends. The timestamps come with the dispatch packets
// (hipExtLaunchKernel), so a timed call has no extra packets between its
// kernels.
struct PassEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

template <typename... P, typename... A>
inline void launch_kernel(void (*k)(P...), dim3 grid, dim3 wg, uint32_t lds, hipStream_t s, hipEvent_t start,
                          hipEvent_t stop, A... args) {
  if (start || stop) hipExtLaunchKernelGGL(k, grid, wg, lds, s, start, stop, 0u, static_cast<P>(args)...);
  else k<<<grid, wg, lds, s>>>(static_cast<P>(args)...);
}

int launch_pass_a(const PassATask& t, const PassAConfig& c, hipStream_t s, PassEvents ev = PassEvents());
int pick_vec(const uint8_t* x, int32_t n_inputs);
// Lanes per row the variant supports; the planner clamps into [lo, hi].
void pass_a_lane_range(int vec, int variant, int* lo, int* hi);
// Whether the variant uses the packed lane table (tasks may span several blocks).
bool pass_a_packed(int vec, int variant);
// Variant 3: 256-lane tasks, blocks side by side for narrow rows.
bool pass_a_side_by_side(int vec, int variant);
int pass_a_side_by_side_lanes(int64_t col_groups);
// Variant 4: blocks held per task (stores deferred to the task's end).
bool pass_a_deferred(int vec, int variant);
int pass_a_deferred_blocks(int64_t n_blocks, int64_t col_groups, int n_cu);
// lane_table: the packed lane-table variants may be chosen.
PassAConfig default_pass_a_config(int vec, int64_t row_bytes, int64_t n_blocks, int block_len, bool lane_table,
                                  int n_cu);

// ---------------------------------------------------------------- pass B
// Normaliser window, array combine, estimator and flags (Eq. discreteMean,
// normedSum1/2, avgSK, final; Sec. 3.2). Kernels and positions: see
// sk_pass_b_dev.h. A call runs the scan kernel (L >= 2), then the combine
// kernel.
struct PassBArgs {
  const int32_t* s1;      // [F][B][N]
  const int32_t* s2;      // [F][B][N]
  const int32_t* cs;      // [F][n_chunks][N] S1 summed over each chunk (pass A), or null: from s1
  const int32_t* hs;      // [F][hist_cap][N] history suffix sums (slots >= hist_cap - hist_len valid)
  int32_t* hs_next;       // [F][hist_cap][N] the same for the next call (null: not kept)
  uint32_t* pc;           // [F][n_chunks + 1][N] exclusive prefix sums of S1 at chunk boundaries
  const uint8_t* mask;    // [F][N] or null
  int64_t* r1;            // [F][B] or null
  int64_t* r2;
  float* v;
  uint8_t* flags;
  int32_t* n_eff;
  float* sk_i;            // [F][B][N] or null
  float* significance;    // [F][B] or null
  const double* thresholds;  // [N + 1][2] (lo, hi) by N_eff, or null: E -+ k sigma
  int32_t n_inputs, n_channels, n_blocks, block_len, window, hist_len, hist_cap, hist_next_len;
  int32_t chunk;          // R: blocks per combine workgroup and per prefix step (1, 2 or 4)
  int32_t n_chunks;       // ceil(B / R)
  int32_t vec;            // inputs per combine lane: 4 (16-byte aligned sums, N % 4 == 0) or 1
  int32_t estimator;
  double k_sigma, expect_offset, sigma_override;
};

// Library choice of R for a call of B blocks (F channels, N inputs).
int pass_b_chunk(int32_t n_inputs, int32_t n_channels, int64_t n_blocks, int32_t window);
int pass_b_vec(int32_t n_inputs);
// Device bytes of the prefix buffer: F (ceil(B / R) + 1) N uint32.
size_t pass_b_prefix_bytes(int32_t n_inputs, int32_t n_channels, int64_t n_blocks, int32_t chunk);
int launch_pass_b(const PassBArgs& a, hipStream_t s, PassEvents ev = PassEvents());

double pearson3_quantile(double mean, double sd, double skew, double p);

struct FlagArgs {
  const double* thresholds;
  const float* v;
  const int32_t* n_eff;
  uint8_t* flags;
  int64_t n;
  int32_t n_max;          // N of the plan: n_eff above it has no threshold entry
  int32_t block_len, window, estimator;
  double k_sigma, expect_offset, sigma_override;
};
int launch_flags(const FlagArgs& a, hipStream_t s);

}  // namespace sk
