/*
 * sk_batch.h - many independent spectral-kurtosis problems in one launch.
 *
 * Each problem is a full plan description (its own N, F, T, M, window,
 * estimator and flag parameters, Sec. 2.2.1 and Sec. 3.2) with its own input,
 * outputs and normaliser state. sk_batch_compute runs one call of every
 * problem: pass A for all problems is one persistent kernel whose workgroups
 * take tasks from a device work queue, the tasks whose lanes walk the most
 * rows first (a task's duration follows its rows, not its bytes). Its
 * workgroups have 512 lanes. For rows of >= 512 column groups a task is 1, 2
 * or 4 consecutive blocks of a chunk of 512 column groups, run by the whole
 * workgroup with its blocks' sums stored after its last block; otherwise a
 * task runs on half a workgroup and is consecutive blocks of a chunk of 256
 * column groups (rows of 256..511 groups), or 256 / L consecutive blocks
 * side by side for rows of L <= 128 column groups (L a power of two). Every
 * lane sums whole rows with the lane-replicated packed power table, and the
 * two wavefronts of each SIMD are kept level. Pass B for all problems follows
 * in a few more kernels; the
 * whole sequence is captured once into a HIP graph, so one call is one graph
 * launch. Tile choices are made per problem class (N, M, F) by the library's
 * autotuner: the class's problems alone are launched with every candidate
 * and timed on the device (pass A rows per load {8, 16} x consecutive blocks
 * per task {1, 2, 4} for wide rows, then pass B chunk length {1, 2, 4}); each
 * candidate's time and the pick are cached in a JSON file keyed by the
 * device arch and the class, and a class found there is not timed again.
 *
 * Requirements: every problem has N % 16 == 0 and a 16-byte aligned input.
 * Errors as in sk.h.
 */
#ifndef SK_BATCH_H
#define SK_BATCH_H

#include <stdint.h>

#include "sk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sk_batch_s* sk_batch_t;

typedef struct {
  int32_t autotune;        /* 1: time the tile candidates of each class on the device (cached);
                              0: 16 rows per load, 1 block per task, the plan's pass B chunk */
  int32_t use_graph;       /* 1: capture the launch sequence into a HIP graph */
  const char* tune_cache;  /* JSON tuning cache path; NULL: env SK_TUNE_CACHE, or none */
} sk_batch_opts;

/* descs[j], d_inputs[j] ([T][F][N] device bytes) and outs[j] (device output
 * pointers, any may be NULL) for j < n. Allocates per-problem scratch and
 * state on the current device, tunes, and captures the graph on `stream`'s
 * device. The inputs and outputs must stay valid while the batch is used. */
int sk_batch_create(const sk_plan_desc* descs, int32_t n, const sk_batch_opts* opts,
                    const uint8_t* const* d_inputs, const sk_outputs* outs, sk_batch_t* batch);

/* One call of every problem, enqueued on `stream`. d_inputs may be NULL (use
 * the pointers given at creation) or a new set of n input pointers of the
 * same shapes; new pointers are written into the device problem table before
 * the graph runs. */
int sk_batch_compute(sk_batch_t batch, const uint8_t* const* d_inputs, void* stream);

/* Forget every problem's normaliser history. Synchronises `stream`. */
int sk_batch_state_reset(sk_batch_t batch, void* stream);

/* Lanes per block row of problem j's pass A tasks (512 for rows of >= 512
 * column groups, 256 for 256..511, else the power of two covering its column
 * groups) and the persistent workgroup count of pass A. */
int sk_batch_get_tiles(sk_batch_t batch, int32_t j, int32_t* lanes_per_row, int32_t* pass_a_grid);

/* Tile choices of problem j: pass A rows per load, blocks per task, pass B
 * chunk length, and whether they came from the tuning cache (1) or from
 * timing or the defaults (0). */
int sk_batch_get_tuning(sk_batch_t batch, int32_t j, int32_t* rows_per_load, int32_t* blocks_per_task,
                        int32_t* pass_b_chunk, int32_t* from_cache);

/* History length (blocks) problem j's normaliser holds on the device now.
 * Synchronises the device. */
int sk_batch_get_state(sk_batch_t batch, int32_t j, int32_t* hist_len);

/* Profiling: runs pass A of the whole batch alone (the persistent kernel,
 * with the batch's tile choices) 4 times on `stream`, the first as a
 * warm-up, and returns the best time in milliseconds. Synchronises `stream`.
 * It rewrites every problem's S1/S2 from the current inputs (the values a
 * call would write) and leaves the normaliser state alone. It resets the
 * work-queue counter with hipMemsetAsync, so it must not run under graph
 * capture or overlap a call of the same batch. */
int sk_batch_time_pass_a(sk_batch_t batch, void* stream, float* ms);

int sk_batch_destroy(sk_batch_t batch);

#ifdef __cplusplus
}
#endif

#endif /* SK_BATCH_H */
