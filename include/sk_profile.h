/*
 * sk_profile.h - per-phase timing and tile control for sk_plan_t.
 *
 * For measurement tools and the autotuner: HIP events that the kernel
 * dispatches of sk_compute record themselves (hipExtLaunchKernel) for its two
 * phases (pass A: the per-input block sums of Eq. singlesums, from its
 * kernel's start to its end; pass B: normaliser window, array combine,
 * estimator and flags of Eq. discreteMean .. final, from its first kernel's
 * start to its last kernel's end).
 */
#ifndef SK_PROFILE_H
#define SK_PROFILE_H

#include <stdint.h>

#include "sk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Record the phase durations of the next max_records sk_compute calls on
 * this plan (0 turns recording off and frees the events). Host-side only. */
int sk_profile_enable(sk_plan_t plan, int32_t max_records);

/* Record only every stride-th call from now on (1, the default after
 * sk_profile_enable: every call). The timestamps travel with the dispatches,
 * so a recorded call adds no packets between its kernels; a stride still
 * bounds the number of events a long run needs. */
int sk_profile_set_stride(sk_plan_t plan, int32_t stride);

/* Wait for the recorded calls and return their phase durations in
 * milliseconds (ms_pass_a[j], ms_pass_b[j], j < *n, n <= cap); then start a
 * new recording. */
int sk_profile_read(sk_plan_t plan, float* ms_pass_a, float* ms_pass_b, int32_t cap, int32_t* n);

/* Force pass A's lanes per row (power of two, 1..1024; 0 = library choice).
 * Up to 256 a workgroup has 256 lanes split into 256 / lanes row phases;
 * 512 and 1024 use workgroups of that many lanes with one row phase. */
int sk_plan_set_pass_a_tile(sk_plan_t plan, int32_t lanes_per_row);

/* Pass A variants (sk_plan_set_pass_a_variant). */
#define SK_PASS_A_AUTO (-1)       /* library choice */
#define SK_PASS_A_SHARED 0        /* shared 256-entry power table, 256-lane workgroups of
                                   * 256 / lanes_per_row row phases reduced in LDS; any
                                   * vector width */
#define SK_PASS_A_PACKED8 1       /* power table replicated per lane (64 KiB of LDS, free of
                                   * bank conflicts) with packed entries p | p^2 << 12 (one
                                   * 32-bit add per sample for both sums), one row phase of
                                   * 256..1024 lanes, 8 rows per load */
#define SK_PASS_A_PACKED16 2      /* as PACKED8, 16 rows per load */
#define SK_PASS_A_SIDE 3          /* packed table in 256-lane workgroups whose lanes each sum
                                   * whole rows: narrow rows put 256 / L blocks side by side,
                                   * L = the power of two covering the row's column groups
                                   * (replaces the lanes-per-row setting) */
#define SK_PASS_A_DEFERRED 4      /* packed table in 512-lane workgroups, each task walking
                                   * 1..4 consecutive blocks with every block's sums held in
                                   * registers until its last block, then stored (about one
                                   * task per CU unless sk_plan_set_pass_a_blocks gives 1..4) */

/* Pass A's variant (SK_PASS_A_*) and workgroup count (0: one per task; fewer:
 * workgroups loop over tasks). Variants 1..4 apply to the 16-byte path
 * (N % 16 == 0, aligned input); other inputs use variant 0. Lanes per row
 * are clamped to 256..1024 for variants 1 and 2. SK_ERR_INVALID_ARG outside
 * -1..4. */
int sk_plan_set_pass_a_variant(sk_plan_t plan, int32_t variant, int32_t grid);

/* Consecutive blocks one pass A task walks with the packed-table variants
 * (1, 2: 1..4096; 4: 1..4), 0 = library choice. Longer tasks stream longer
 * contiguous runs of rows per workgroup. */
int sk_plan_set_pass_a_blocks(sk_plan_t plan, int32_t blocks);

/* Pass B's chunk length R (blocks per combine workgroup and per prefix step:
 * 1, 2 or 4; 0 = library choice) and inputs per lane (1 or 4; 0 = library
 * choice, 4 when N % 4 == 0 and the sums are 16-byte aligned). Results do not
 * depend on R. */
int sk_plan_set_pass_b_tile(sk_plan_t plan, int32_t chunk, int32_t inputs_per_lane);

/* Pass A's lanes per row and workgroup count for the next call (after
 * sk_plan_set_pass_a_tile or the library's choice), for reporting. */
int sk_plan_get_pass_a_tile(sk_plan_t plan, const uint8_t* d_packed, int32_t* vec_bytes,
                            int32_t* lanes_per_row, int64_t* workgroups);

/* Read-only stream probe, the practical HBM read ceiling for streaming
 * kernels such as pass A: reads the `bytes` bytes at device pointer d_x once
 * (16-byte nontemporal loads, one contiguous slab per workgroup of 256
 * lanes) and writes one XOR word per lane to d_sink, which must hold
 * workgroups * 256 uint32 words. Needs a 16-byte aligned d_x and
 * bytes % 16 == 0, else SK_ERR_INVALID_ARG. Asynchronous on `stream`; the
 * caller times it. The sink's contents carry no meaning. */
int sk_read_probe(const uint8_t* d_x, int64_t bytes, int32_t workgroups, uint32_t* d_sink, void* stream);

/* Result of sk_plan_autotune: the settings kept and their times. */
typedef struct {
  int32_t pass_a_variant;      /* 0..4, as SK_PASS_A_* */
  int32_t pass_a_lanes;        /* lanes per row */
  int32_t pass_a_blocks;       /* consecutive blocks per task */
  int32_t pass_a_chunk_sums;   /* 1: pass A writes the chunk sums the scan reads */
  int32_t pass_b_chunk;        /* blocks per combine workgroup (1, 2, 4) */
  int32_t pass_b_vec;          /* inputs per combine lane (1 or 4) */
  int32_t candidates;          /* combinations timed */
  float ms_pass_a, ms_pass_b;  /* pooled kernel-time estimates of the kept combination */
  float ms_library_pass_a, ms_library_pass_b;  /* the library's own choice, same measurement */
} sk_plan_tuning;

/* Time every candidate tile combination of this plan on the device input
 * d_x ([T][F][N] bytes) and keep the fastest: pass A variant (the library's
 * choice; the deferred-store variant at 1, 2 and 4 blocks per task, and
 * at 2 and 4 without writing the chunk sums for a scan of that chunk; the
 * packed-table variants at 1024 and 256 lanes; blocks side by side for
 * narrow rows), crossed with pass B chunk length {1, 2, 4}. Pass B inputs
 * per lane stay as set (they order the FP64 combine). Each combination runs
 * one untimed and `reps` (1..100) timed calls on `stream` without outputs.
 * Each pass's time is estimated from every combination that runs that pass
 * the same way (pass A: its launched variant, lanes, blocks per task and
 * whether it writes chunk sums; pass B: its chunk length and whether it
 * reads them), and the combination with the least sum of the two estimates
 * is kept if, timed again in 4 calls alternating with the library's choice,
 * it is still faster (else the library's choice is kept). The
 * normaliser state is exported before and imported after, so a stream in
 * progress continues unchanged; results of later calls do not depend on the
 * choice (integer sums are exact, and the combine's order does not depend on
 * the chunk length). Synchronises `stream`; must not overlap other calls of
 * the plan. `out` may be NULL. */
int sk_plan_autotune(sk_plan_t plan, const uint8_t* d_x, int32_t reps, void* stream, sk_plan_tuning* out);

/* Per-wavefront timeline of pass A (diagnostic). Runs the plan's pass A once
 * on d_x ([T][F][N] bytes), writing the sums into the plan's own S1/S2
 * buffers (pass B does not run; the normaliser state is untouched). The
 * plan's pass A must be the deferred-store variant (SK_PASS_A_DEFERRED, as
 * the library picks for CHIME-like rows) with one workgroup per task. Lane 0
 * of every wavefront writes 6 uint64 at d_out[6 (8 workgroup + wavefront)]:
 * the GPU real-time clock (100 MHz) at its start, after its last read and
 * after its stores completed, then its XCD id, its HW_ID register and its
 * SIMD. simd_balance: 1 as the library runs (the wavefronts of each SIMD
 * kept level by priority), 0 left to the instruction arbiter (needs 4 blocks
 * per task), for comparison. d_out holds cap records (device memory); *n_waves
 * receives the number written. Asynchronous on `stream`. SK_ERR_INVALID_ARG
 * for another variant, too small a cap, or bad arguments. */
int sk_plan_pass_a_timeline(sk_plan_t plan, const uint8_t* d_x, int32_t simd_balance, uint64_t* d_out, int64_t cap,
                            int64_t* n_waves, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SK_PROFILE_H */
