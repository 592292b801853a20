/*
 * sk_diag.h - per-channel diagnostics of the estimator stream.
 *
 * App. A: a common-mode signal shared by the receivers correlates them and
 * raises the variance of the multi-receiver estimator from 4/(nN) toward the
 * single-receiver 4/n; re-expressed, the effective number of independent
 * receivers is N_eff = 4 / (n var). This entry point measures that from the
 * values of one or more calls.
 */
#ifndef SK_DIAG_H
#define SK_DIAG_H

#include <stdint.h>

#include "sk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* For each channel f < n_channels of d_v [F][B] (device float, NaN = invalid
 * block): the mean and the unbiased variance of the valid values, N_eff =
 * 4 / (block_len * var) (NaN when fewer than two valid blocks or var = 0),
 * and the number of valid blocks. Outputs are device arrays of n_channels
 * entries. Enqueued on `stream`. */
int sk_channel_stats(const float* d_v, int32_t n_channels, int64_t n_blocks, int32_t block_len,
                     double* d_mean, double* d_var, double* d_n_eff, int64_t* d_count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SK_DIAG_H */
