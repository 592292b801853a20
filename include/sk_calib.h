/*
 * sk_calib.h - Monte-Carlo calibration of the flag thresholds (App. B).
 *
 * The paper sets its thresholds from simulations of its correlator's 4+4-bit
 * data: Gaussian components of a given RMS, rounded and bounded to [-7, 7];
 * the mean of the estimator under digitisation is offset from 1 and that
 * offset is added to the threshold. sk_calibrate_mc runs such a simulation on
 * the GPU: every simulated estimate draws N inputs x M samples, forms the
 * per-input sums and the multi-receiver estimator with each input normalised
 * by its own block mean (Eq. discreteMean, L = 1), and the moments of the
 * estimates are returned.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014); the n-th
 * draw for key k is the SplitMix64 output function of k + (n + 1) *
 * 0x9E3779B97F4A7C15, with k = SplitMix64 output of the seed. Sample j of
 * input i of estimate s uses draw n = (s * N + i) * M + j: the high 32 bits
 * give the real part, the low 32 bits the imaginary part, each quantised by
 * inverse CDF against the 2*clip integer thresholds
 * floor(2^32 * Phi((v + 1/2) / sigma)), v = -clip .. clip-1.
 */
#ifndef SK_CALIB_H
#define SK_CALIB_H

#include <stdint.h>

#include "sk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_inputs;       /* N receivers per simulated estimate */
  int32_t block_len;      /* M samples per receiver */
  int32_t estimator;      /* SK_EST_HAT or SK_EST_TILDE */
  int32_t clip;           /* component bound, 7 for 4+4-bit data */
  double sigma;           /* component RMS in counts (all inputs) */
  int64_t n_sim;          /* simulated estimates */
  uint64_t seed;
} sk_mc_desc;

/* Simulate; moments[0..3] = mean, unbiased variance, skewness, excess
 * kurtosis of the valid estimates (host array). d_values, if not NULL, is a
 * device array of n_sim doubles that receives every simulated estimate.
 * Synchronises `stream`. */
int sk_calibrate_mc(const sk_mc_desc* desc, double* moments, double* d_values, void* stream);

/* Quantile at lower-tail probability p of the Pearson type III law with the
 * given mean, standard deviation and skewness (>= 0; 0 is the normal law):
 * the model behind sk_plan_set_false_alarm (host, FP64). */
int sk_pearson3_quantile(double mean, double sd, double skew, double p, double* out);

#ifdef __cplusplus
}
#endif

#endif /* SK_CALIB_H */
