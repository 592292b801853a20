// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
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
};

struct PassAConfig {
  int vec;     // 16, 4 or 1 bytes per lane per row
  int lpr;     // lanes per row: power of two, 1..256
  int variant; // row batching variant (0..17, 16-byte path; see pass_a_groups_per_lane)
  int grid;    // workgroups launched (<= tasks; grid-stride beyond)
};

int launch_pass_a(const PassATask& t, const PassAConfig& c, hipStream_t s);
int pick_vec(const uint8_t* x, int32_t n_inputs);
// Column groups each lane owns in pass A for this vector width and variant.
int pass_a_groups_per_lane(int vec, int variant);
// Whether this variant uses the lane-replicated power table (needs >= 256
// lanes per row: one row phase).
bool pass_a_lane_table(int vec, int variant);
// Lanes per row the variant supports; the planner clamps into [lo, hi].
void pass_a_lane_range(int vec, int variant, int* lo, int* hi);
// Whether the variant uses the packed lane table (tasks may span several blocks).
bool pass_a_packed(int vec, int variant);
// Variant 16: 256-lane tasks, blocks side by side for narrow rows.
bool pass_a_side_by_side(int vec, int variant);
int pass_a_side_by_side_lanes(int64_t col_groups);
// Variant 17: blocks held per task (stores deferred to the task's end).
bool pass_a_deferred(int vec, int variant);
int pass_a_deferred_blocks(int64_t n_blocks, int64_t col_groups, int n_cu);
// lane_table: the lane-replicated table variants may be chosen (single-plan
// kernel only; the batched kernel has its own table).
PassAConfig default_pass_a_config(int vec, int64_t row_bytes, int64_t n_blocks, int block_len, bool lane_table,
                                  int n_cu);

// ---------------------------------------------------------------- pass B
// Normaliser window, array combine, estimator and flags (Eq. discreteMean,
// normedSum1/2, avgSK, final; Sec. 3.2).
//
// Extended block sequence per (channel, input): e = 0..H-1 are the H history
// blocks (oldest first), e = H..H+B-1 the blocks of this call. Chunks of R
// consecutive e carry exclusive prefix sums so any window sum is two lookups
// plus fewer than R reads.
struct PassBArgs {
  const int32_t* s1;      // [F][B][N]
  const int32_t* s2;      // [F][B][N]
  const int32_t* hist;    // [F][Hcap][N], entries 0..H-1 valid (oldest first)
  int32_t* hist_next;     // [F][Hcap][N] history for the next call
  int32_t* chunk_sum;     // [F][n_chunks][N] sums of S1 over chunks of the sequence
  double* part_a;         // [F][n_groups][B] per-group partial sums
  double* part_q;
  int64_t* part_r1;
  int64_t* part_r2;
  int32_t* part_n;
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
  int32_t chunk, n_chunks, n_groups, vec, estimator;
  // Range of one launch sequence: chunks [chunk0, chunk0 + grid) of the
  // chunk-sum and partial kernels, blocks [fin_b0, fin_b0 + fin_nb) of the
  // finalize kernel (a whole call: 0, n_chunks, 0, n_blocks).
  int32_t chunk0, fin_b0, fin_nb;
  int32_t depth;          // blocks a partial-kernel wavefront loads together (2, 4 or 8)
  double k_sigma, expect_offset, sigma_override;
};

int pass_b_vec(int32_t n_inputs);
int launch_pass_b(const PassBArgs& a, hipStream_t s);
// Pass B kernels for chunks [c_begin, c_end) and blocks [b_begin, b_end) of
// one call; the history carry (when a call is shorter than the window) runs
// with the range that has with_hist_copy set.
int launch_pass_b_range(PassBArgs a, int32_t c_begin, int32_t c_end, int32_t b_begin, int32_t b_end,
                        bool with_hist_copy, hipStream_t s);

// ---------------------------------------------------------------- single launch
// One cooperative kernel for wide rows filling one round of CUs (see
// sk_fused.hip): pass A, the window scans and pass B of a call.
struct FusedArgs {
  PassATask a;          // x, s1 (always written), s2 (null: not stored), geometry
  PassBArgs b;          // window, history, outputs, flag parameters
  int32_t* segsum;      // [segments][F*N] S1 sums of each workgroup's blocks
  int32_t* segpre;      // [segments][F*N] exclusive prefix over segments
  int32_t* hsuf;        // [hist_cap][F*N] suffix sums of the history rows
};
int launch_fused(const FusedArgs& fa, int blocks_per_workgroup, hipStream_t s);
int fused_max_workgroups();

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
