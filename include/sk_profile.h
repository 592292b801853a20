/*
 * sk_profile.h - per-phase timing and tile control for sk_plan_t.
 *
 * For measurement tools and the autotuner: HIP events recorded on the
 * caller's stream around the two kernel phases of sk_compute (pass A: the
 * per-input block sums of Eq. singlesums; pass B: normaliser window, array
 * combine, estimator and flags of Eq. discreteMean .. final).
 */
#ifndef SK_PROFILE_H
#define SK_PROFILE_H

#include <stdint.h>

#include "sk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Record events around the phases of the next max_records sk_compute calls
 * on this plan (0 turns recording off and frees the events). Host-side only. */
int sk_profile_enable(sk_plan_t plan, int32_t max_records);

/* Record only every stride-th call from now on (1, the default after
 * sk_profile_enable: every call). The events sit between dependent kernels
 * and cost a few microseconds per recorded call; a stride samples the phase
 * durations of a long run of calls while the others run unperturbed. */
int sk_profile_set_stride(sk_plan_t plan, int32_t stride);

/* Wait for the recorded calls and return their phase durations in
 * milliseconds (ms_pass_a[j], ms_pass_b[j], j < *n, n <= cap); then start a
 * new recording. */
int sk_profile_read(sk_plan_t plan, float* ms_pass_a, float* ms_pass_b, int32_t cap, int32_t* n);

/* Force pass A's lanes per row (power of two, 1..1024; 0 = library choice).
 * Up to 256 a workgroup has 256 lanes split into 256 / lanes row phases;
 * 512 and 1024 use workgroups of that many lanes with one row phase. */
int sk_plan_set_pass_a_tile(sk_plan_t plan, int32_t lanes_per_row);

/* Pass A's row batching variant (-1: library choice; 0: 8 rows per batch;
 * 1: 8 rows with the next batch's loads issued before the current batch is
 * reduced; 2: 4 rows with that prefetch; 3: 16 rows; 4: two column groups of
 * 16 inputs per lane, lanes_per_row apart, 4 rows per batch; 5: two groups,
 * 8 rows; 6: four groups, 2 rows; 7: power table replicated per lane (64 KiB
 * of LDS, free of bank conflicts), 8 rows; 8: replicated table, two groups,
 * 4 rows; 9: replicated table, 8 rows with prefetch; 10: replicated table,
 * 16 rows; 11: replicated table, 16 rows with prefetch; 12: replicated table
 * shared by 512-lane workgroups of 512 / lanes_per_row row phases, 8 rows;
 * 13: as 12 with two groups, 4 rows; 14: replicated table of packed entries
 * p | p^2 << 12, one 32-bit add per sample for both sums, 8 rows; 15: as 14,
 * 16 rows; 16: packed table in 256-lane workgroups whose lanes each sum whole
 * rows: narrow rows put 256 / L blocks side by side, L = the power of two
 * covering the row's column groups, which replaces the lanes-per-row
 * setting; 17: packed table in 512-lane workgroups, each task walking 1..4
 * consecutive blocks with every block's sums held until its last block, then
 * stored, sized for about one task per CU unless sk_plan_set_pass_a_blocks
 * gives 1..4) and workgroup count (0: one per task; fewer: workgroups loop
 * over tasks). Variants 1..17 apply to the 16-byte path (N % 16 == 0,
 * aligned input); the others use variant 0. Lanes per row are clamped to 256..1024
 * for variants 7..11, 14 and 15 (one row phase) and to 64..512 for variants
 * 12 and 13. */
int sk_plan_set_pass_a_variant(sk_plan_t plan, int32_t variant, int32_t grid);

/* Block segments per call (1..64; 0 = library choice, currently 1: on
 * MI355X the extra pass A launches cost more than the overlap gains for the
 * CHIME shapes). With K > 1 a call
 * runs pass A over K consecutive block ranges on the caller's stream and
 * pass B of each range on a plan-owned stream as soon as that range's pass A
 * is done, so pass B overlaps the next range's pass A; the caller's stream
 * then waits for the last pass B. Results are identical for every K. The
 * plan stream is created on the first segmented call made outside stream
 * capture (a call under capture before that runs unsegmented). */
int sk_plan_set_segments(sk_plan_t plan, int32_t segments);

/* Segments (pass A launches) the plan's last sk_compute used; 0 before the
 * first call. */
int sk_plan_get_last_segments(sk_plan_t plan, int32_t* segments);

/* Single-launch path: one cooperative kernel per call (pass A, the window
 * prefix scans across workgroups, then the combine, V and flags of each
 * workgroup's blocks), for 16-byte lanes, N % 1024 == 0, F N / 16 <= 512
 * column groups, a window of L >= 2 blocks, one segment, and at most 4
 * blocks per workgroup with one workgroup per CU. mode 0 (the default):
 * never; 1: whenever the shape allows (its scratch, 2 n_cu F N + (L-1) F N
 * int32, is allocated by this call; SK_ERR_NOMEM if that fails). Calls of
 * other shapes run the two-pass path. Results equal the two-pass path's
 * integer outputs and flags; V differs only by the order of its FP64 sums.
 * Off by default because each of its two grid-wide barriers costs more
 * than the separate launches and the S1/S2 re-read that it saves. */
int sk_plan_set_fused(sk_plan_t plan, int32_t mode);

/* 1 if the plan's last sk_compute ran the single-launch path. */
int sk_plan_get_last_fused(sk_plan_t plan, int32_t* fused);

/* Consecutive blocks one pass A task walks with the packed-table variants
 * (14, 15): 1..4096, 0 = library choice. Longer tasks stream longer
 * contiguous runs of rows per workgroup. */
int sk_plan_set_pass_a_blocks(sk_plan_t plan, int32_t blocks);

/* Blocks whose sums a pass B partial-kernel wavefront loads together (2, 4
 * or 8; 0 = library choice, 4). Applies to 4 inputs per lane. */
int sk_plan_set_pass_b_depth(sk_plan_t plan, int32_t depth);

/* Pass B's chunk length (blocks per wavefront, power of two; 0 keeps the
 * library's choice) and inputs per lane (1, 4 or 8; 0 = library choice; 8
 * needs N % 8 == 0 and 32-byte aligned sums, else the library's choice). */
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

#ifdef __cplusplus
}
#endif

#endif /* SK_PROFILE_H */
