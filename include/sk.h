/*
 * sk.h - C ABI of the MI355X (gfx950) multi-receiver spectral-kurtosis library.
 *
 * Method: Taylor et al., "Spectral Kurtosis Based RFI Mitigation for CHIME",
 * arXiv:1808.10365, Sec. 2.1-2.2.1 (estimator) and Sec. 3.2 (flags).
 *
 * For every frequency channel f and every block b of M time samples the
 * library
 *   1. decodes 4+4-bit offset-encoded complex samples (high nibble = Re + 8,
 *      low nibble = Im + 8; App. B bounds the components to [-7, 7]);
 *   2. forms power p = Re^2 + Im^2 (Sec. 2.2.3, "Calculating Power");
 *   3. sums per input i over the block: S1_i = sum p, S2_i = sum p^2
 *      (Eq. singlesums), exactly, in int32;
 *   4. forms the normaliser P_i[b] = sum of S1_i over the L blocks ending at b
 *      (L = 1 is Eq. discreteMean; the running form carries history across
 *      calls; L = 0 disables normalisation);
 *   5. combines across inputs: A = sum_i S1_i / P_i and Bq = sum_i S2_i / P_i^2
 *      in FP64 (Eq. normedSum1, normedSum2, up to factors that cancel), and the
 *      raw sums R1 = sum_i S1_i, R2 = sum_i S2_i in int64;
 *   6. evaluates V = (K+1)/(K-1) * (K Bq / A^2 - 1), K = N_eff M (Eq. avgSK),
 *      or the rescaled form (M+1)/(M-1) * (M Bq / N_eff - 1) (Eq. final, L = 1);
 *   7. flags V outside E +- k sigma (Sec. 3.2), E = E0 + expect_offset.
 *
 * Layouts (all row-major, C order):
 *   packed input   uint8  [T][F][N]   time-major, inputs innermost
 *   mask           uint8  [F][N]      nonzero = input used; NULL = all used
 *   s1, s2         int32  [F][B][N]   per-input block sums, B = T / M
 *   r1, r2         int64  [F][B]
 *   v              float  [F][B]      NaN where invalid
 *   flags          uint8  [F][B]      bit0 low, bit1 high, bit2 invalid
 *   n_eff          int32  [F][B]      inputs used (mask set and P_i > 0)
 *   sk_i           float  [F][B][N]   per-input estimate SK_i (Eq. originalSK), NaN if S1_i = 0
 *   significance   float  [F][B]      detection significance (V - E) / sigma (Sec. 3.2)
 *
 * Ownership: the caller owns every input and output buffer (device memory,
 * e.g. torch tensors). A plan owns its scratch and its normaliser state
 * (device memory allocated at creation, released by destroy). No pointer is
 * retained past the completion of the work enqueued on the given stream.
 *
 * Errors: every entry point returns 0 on success or a negative SK_ERR_*
 * code; sk_last_error() gives a message for the calling thread. Nothing
 * throws across the ABI. Work is enqueued asynchronously on the caller's
 * HIP stream (hipStream_t passed as void*; NULL = the null stream).
 * A plan is not thread-safe; a server is.
 */
#ifndef SK_H
#define SK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SK_OK 0
#define SK_ERR_INVALID_ARG (-1)   /* NULL handle, bad enum, bad pointer alignment */
#define SK_ERR_SHAPE (-2)         /* sizes violate the limits stated below */
#define SK_ERR_NOMEM (-3)         /* device or host allocation failed */
#define SK_ERR_DEVICE (-4)        /* a HIP call failed */
#define SK_ERR_AGAIN (-5)         /* server queue full / result not ready */
#define SK_ERR_STATE (-6)         /* state blob does not match the plan */

#define SK_EST_HAT 0              /* Eq. avgSK, first line */
#define SK_EST_TILDE 1            /* Eq. final (only with norm_window_blocks == 1) */

#define SK_FLAG_LOW 1
#define SK_FLAG_HIGH 2
#define SK_FLAG_INVALID 4

/* Limits checked by sk_plan_create (SK_ERR_SHAPE otherwise):
 *   1 <= N <= 16384, 1 <= F, 2 <= M <= 131071 (M * 128^2 < 2^31: S2 fits int32),
 *   n_samples >= 0 and a multiple of M,
 *   0 <= L and L * M * 128 < 2^31 (the window sum P fits int32),
 *   SK_EST_TILDE requires L == 1, k_sigma >= 0. */
typedef struct {
  int32_t n_inputs;            /* N: receivers of the compact array */
  int32_t n_channels;          /* F: frequency channels in this stream */
  int64_t n_samples;           /* T: samples per channel per call */
  int32_t block_len;           /* M: samples per input per estimate (paper's n) */
  int32_t norm_window_blocks;  /* L: 0 none, 1 the block's own mean, >1 running window */
  int32_t estimator;           /* SK_EST_HAT or SK_EST_TILDE */
  double k_sigma;              /* half-width of the accepted interval in sigmas (paper: 5) */
  double expect_offset;        /* delta added to the expectation (App. B digitisation offset) */
  double sigma_override;       /* > 0: sigma to use; <= 0: sqrt(4 / K) (Eq. final variance) */
} sk_plan_desc;

/* Device output pointers; any may be NULL (not produced). */
typedef struct {
  int32_t* s1;
  int32_t* s2;
  int64_t* r1;
  int64_t* r2;
  float* v;
  uint8_t* flags;
  int32_t* n_eff;
  float* sk_i;
  float* significance;
} sk_outputs;

typedef struct sk_plan_s* sk_plan_t;

/* Message for the last error on the calling thread ("" if none). */
const char* sk_last_error(void);

/* Validate desc, allocate scratch and the normaliser state on the current
 * device, and select kernel tile shapes. *plan is NULL on failure. */
int sk_plan_create(const sk_plan_desc* desc, sk_plan_t* plan);

/* Release the plan's device memory. Waits for the device first. */
int sk_plan_destroy(sk_plan_t plan);

/* Bytes of device memory the plan holds. */
int sk_plan_device_bytes(sk_plan_t plan, size_t* bytes);

/* One call of the whole path on d_packed [T][F][N] (device, caller-owned).
 * Enqueued on `stream`; continues the normaliser from the previous call on
 * this plan (stream semantics) and advances it. d_mask may be NULL.
 * d_packed must stay valid until the stream reaches this work. */
int sk_compute(sk_plan_t plan, const uint8_t* d_packed, const uint8_t* d_mask,
               const sk_outputs* outs, void* stream);

/* The call of sk_compute with a fresh normaliser (no history, as on a new
 * plan's first call) and no plan, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc. It allocates nothing. desc as for sk_plan_create;
 * outs->s1 and outs->s2 are required (the per-input sums live in the
 * caller's buffers); the other outputs as for sk_compute. Pass B's prefix
 * sums use a static device array of sk_noalloc_scratch_bytes() bytes per
 * GPU (32 MiB, held until the process ends): a call whose window (L >= 2)
 * needs more, F (ceil(B / R) + 1) N 4 bytes with R the library's chunk
 * length, returns SK_ERR_SHAPE. False-alarm thresholds are not available
 * (k sigma flags). Calls that overlap on one GPU share the array and race:
 * order them on one stream. */
int sk_compute_noalloc(const sk_plan_desc* desc, const uint8_t* d_packed, const uint8_t* d_mask,
                       const sk_outputs* outs, void* stream);

/* Bytes of sk_compute_noalloc's static scratch on each GPU. */
size_t sk_noalloc_scratch_bytes(void);

/* Flags from precomputed values (Sec. 3.2), with the plan's k_sigma,
 * expect_offset, sigma_override, M, L and estimator: flags[j] from v[j]
 * (promoted to FP64) and n_eff[j], j < n. Device pointers. */
int sk_flags(sk_plan_t plan, const float* d_v, const int32_t* d_n_eff, uint8_t* d_flags,
             int64_t n, void* stream);

/* Flag thresholds from a false-alarm probability instead of E -+ k sigma
 * (Sec. 3.2: for small nN the skewness of the estimator makes a symmetric
 * interval inaccurate). For each N_eff the thresholds are the p and 1 - p
 * quantiles of a Pearson type III law with mean E (as for the symmetric
 * cut), standard deviation sigma (sqrt(4/K) or sigma_override) and skewness
 * 10 / sqrt(K) (Sec. 2.1), K = N_eff M. fap in (0, 0.5); 0 restores the
 * symmetric cut. Applies to sk_compute and sk_flags of this plan. */
int sk_plan_set_false_alarm(sk_plan_t plan, double fap);

/* The (lo, hi) thresholds the plan applies for a given N_eff (host). */
int sk_plan_get_thresholds(sk_plan_t plan, int32_t n_eff, double* lo, double* hi);

/* Forget the normaliser history (the next call starts a fresh warm-up). */
int sk_state_reset(sk_plan_t plan);

/* Size in bytes of the state blob of this plan (history of up to L-1 blocks). */
int sk_state_size(sk_plan_t plan, size_t* bytes);

/* Copy the normaliser state into host memory (synchronises `stream`).
 * cap must be >= sk_state_size. */
int sk_state_export(sk_plan_t plan, void* host_buf, size_t cap, void* stream);

/* Restore a state blob written by sk_state_export for a plan with the same
 * N, F, M and L (SK_ERR_STATE otherwise). Synchronises `stream`. */
int sk_state_import(sk_plan_t plan, const void* host_buf, size_t size, void* stream);

/* App. B digitisation model for expectation and spread (host, FP64).
 * Components are round(sigma_i z) clipped to [-clip, clip]. For n inputs of
 * RMS sigma[i] and block length M, returns the offset delta of the mean of V
 * from 1 (kappa_bar - 2, kappa = E[p^2] / E[p]^2) and the delta-method
 * standard deviation of V for K = n M samples. */
int sk_digitised_expectation(const double* sigma, int32_t n, int32_t block_len, int32_t clip,
                             double* delta, double* sigma_v);

#ifdef __cplusplus
}
#endif

#endif /* SK_H */
