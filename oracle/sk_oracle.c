/*
 * CPU ORACLE for the multi-receiver spectral-kurtosis estimator.
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the bench's
 * CPU-baseline leg are the only callers. The GPU library never calls, links
 * or includes this file, and this file includes nothing of the GPU library.
 *
 * Plain loops, int64 for integer sums, FP64 for everything that is not an
 * integer, summation in input order i = 0..N-1. No blocking, no fusion.
 *
 * Paper: Taylor et al., "Spectral Kurtosis Based RFI Mitigation for CHIME"
 * (arXiv:1808.10365).
 *   Sec. 2.1, Eq. (1)-(2)        single-receiver S1, S2 and SK
 *   Sec. 2.2.1 Eq. singlesums    per-receiver (S1)_i, (S2)_i over n samples
 *   Sec. 2.2.1 Eq. originalSK    per-receiver SK_i
 *   Sec. 2.2.1 Eq. discreteMean  mean power mu_i = (S1)_i / n
 *   Sec. 2.2.1 Eq. normedSum1/2  normalised array cumulants
 *   Sec. 2.2.1 Eq. avgSK         multi-receiver estimator, effective count nN
 *   Sec. 2.2.1 Eq. final         rescaled estimator = Avg(SK_i)
 *   Sec. 3.2                     detection significance, symmetric a-sigma cut
 *   App. B                       4+4-bit data bounded to [-7, 7]
 *
 * Names: N inputs (receivers), F channels, T samples per channel, M samples
 * per input per estimate (the paper's n), B = T / M blocks, K = N_eff * M the
 * effective sample count (the paper's nN), L the normaliser window in blocks.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes):
 *   - Byte encoding: high nibble = Re + 8, low nibble = Im + 8. Code 0 decodes
 *     literally to -8, so one sample's power is at most 128.
 *   - Normaliser: mu_i is proportional to P_i[b], the sum of S1_i over the L
 *     blocks ending at and including b (blocks before the stream's start are
 *     absent, so a warm-up window holds fewer blocks). L = 1 is exactly
 *     Eq. discreteMean; L = 0 means no normalisation (unit weights). The
 *     factor count*M that turns P_i into a mean is the same for every input of
 *     a (channel, block) and cancels in the estimator, so weights are 1/P_i.
 *   - Inputs with P_i = 0, or masked out, are dropped and not counted in N_eff.
 *   - V is invalid (NaN, flag bit 2) when N_eff * M < 2 or A = 0.
 *   - Expectation: E = E0 + delta, where E0 = 1, except the unrescaled
 *     estimator with L = 1, whose mean is (K+1)(M-1) / ((K-1)(M+1)) by
 *     Eq. avgSK (last line) with mean(SK_i) = 1. delta is the caller's
 *     digitisation offset (App. B adds it to the threshold).
 *   - sigma = sqrt(4 / K) (Eq. final variance) unless the caller overrides it.
 *   - Flags: bit 0 when V < E - k sigma, bit 1 when V > E + k sigma (strict).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_EST_HAT = 0, ORC_EST_TILDE = 1 };
enum { ORC_FLAG_LOW = 1, ORC_FLAG_HIGH = 2, ORC_FLAG_INVALID = 4 };

/* Power of one offset-encoded complex sample: re(x)^2 + im(x)^2
 * (Sec. 2.2.3, "Calculating Power"). */
int orc_power(uint8_t byte) {
  int re = (int)(byte >> 4) - 8;
  int im = (int)(byte & 15) - 8;
  return re * re + im * im;
}

/* Eq. singlesums: (S1)_i = sum_j |x_j|^2, (S2)_i = sum_j |x_j|^4 over the M
 * samples of block b, for every (channel f, block b, input i).
 * x is [T][F][N]; S1, S2 are [F][B][N]. */
void orc_block_sums(const uint8_t* x, int64_t N, int64_t F, int64_t T, int64_t M,
                    int64_t* S1, int64_t* S2) {
  int64_t B = T / M;
  memset(S1, 0, sizeof(int64_t) * (size_t)(F * B * N));
  memset(S2, 0, sizeof(int64_t) * (size_t)(F * B * N));
  for (int64_t f = 0; f < F; ++f)
    for (int64_t b = 0; b < B; ++b)
      for (int64_t j = 0; j < M; ++j) {
        int64_t t = b * M + j;
        for (int64_t i = 0; i < N; ++i) {
          int64_t p = orc_power(x[(t * F + f) * N + i]);
          S1[(f * B + b) * N + i] += p;
          S2[(f * B + b) * N + i] += p * p;
        }
      }
}

/* Same sums for real-valued power p[T][F][N] (FP64), for statistics tests on
 * continuous chi-squared power. */
void orc_block_sums_f64(const double* p, int64_t N, int64_t F, int64_t T, int64_t M,
                        double* S1, double* S2) {
  int64_t B = T / M;
  for (int64_t q = 0; q < F * B * N; ++q) S1[q] = S2[q] = 0.0;
  for (int64_t f = 0; f < F; ++f)
    for (int64_t b = 0; b < B; ++b)
      for (int64_t j = 0; j < M; ++j)
        for (int64_t i = 0; i < N; ++i) {
          double v = p[((b * M + j) * F + f) * N + i];
          S1[(f * B + b) * N + i] += v;
          S2[(f * B + b) * N + i] += v * v;
        }
}

/* Normaliser window: P[f][b][i] = sum of S1_i over blocks b-L+1 .. b.
 * Blocks before this call come from hist[f][H + b'][i] for -H <= b' < 0
 * (oldest first); blocks before that do not exist. L = 0 gives P = S1. */
void orc_window(const int64_t* S1, const int64_t* hist, int64_t H, int64_t N, int64_t F,
                int64_t B, int64_t L, int64_t* P) {
  for (int64_t f = 0; f < F; ++f)
    for (int64_t b = 0; b < B; ++b) {
      int64_t* out = P + (f * B + b) * N;
      if (L == 0) {
        for (int64_t i = 0; i < N; ++i) out[i] = S1[(f * B + b) * N + i];
        continue;
      }
      for (int64_t i = 0; i < N; ++i) out[i] = 0;
      for (int64_t bb = b - L + 1; bb <= b; ++bb) {
        const int64_t* src = NULL;
        if (bb >= 0)
          src = S1 + (f * B + bb) * N;
        else if (bb >= -H)
          src = hist + (f * H + (H + bb)) * N;
        if (src)
          for (int64_t i = 0; i < N; ++i) out[i] += src[i];
      }
    }
}

void orc_window_f64(const double* S1, int64_t N, int64_t F, int64_t B, int64_t L, double* P) {
  for (int64_t f = 0; f < F; ++f)
    for (int64_t b = 0; b < B; ++b) {
      double* out = P + (f * B + b) * N;
      if (L == 0) {
        for (int64_t i = 0; i < N; ++i) out[i] = S1[(f * B + b) * N + i];
        continue;
      }
      for (int64_t i = 0; i < N; ++i) out[i] = 0.0;
      for (int64_t bb = b - L + 1; bb <= b; ++bb)
        if (bb >= 0)
          for (int64_t i = 0; i < N; ++i) out[i] += S1[(f * B + bb) * N + i];
    }
}

/* Expectation and spread used by the symmetric cut (Sec. 3.2). */
static void orc_expectation(int64_t K, int64_t M, int64_t L, int est, double delta,
                            double sigma_override, double* E, double* sigma) {
  double Kd = (double)K, Md = (double)M;
  double e0 = 1.0;
  if (est == ORC_EST_HAT && L == 1) e0 = ((Kd + 1.0) * (Md - 1.0)) / ((Kd - 1.0) * (Md + 1.0));
  *E = e0 + delta;
  *sigma = sigma_override > 0.0 ? sigma_override : sqrt(4.0 / Kd);
}

/* Symmetric a-sigma cut on one value (Sec. 3.2). */
uint8_t orc_flag_one(double V, int64_t n_eff, int64_t M, int64_t L, int est, double k,
                     double delta, double sigma_override) {
  int64_t K = n_eff * M;
  if (K < 2 || isnan(V)) return ORC_FLAG_INVALID;
  double E, s;
  orc_expectation(K, M, L, est, delta, sigma_override, &E, &s);
  double lo = E - k * s, hi = E + k * s;
  uint8_t fl = 0;
  if (V < lo) fl |= ORC_FLAG_LOW;
  if (V > hi) fl |= ORC_FLAG_HIGH;
  return fl;
}

/* Detection significance (Sec. 3.2): (V - E) / sigma, NaN where invalid. */
double orc_significance_one(double V, int64_t n_eff, int64_t M, int64_t L, int est, double delta,
                            double sigma_override) {
  int64_t K = n_eff * M;
  if (K < 2 || isnan(V)) return NAN;
  double E, s;
  orc_expectation(K, M, L, est, delta, sigma_override, &E, &s);
  return (V - E) / s;
}

void orc_significance(const double* V, const int32_t* n_eff, int64_t n, int64_t M, int64_t L, int est,
                      double delta, double sigma_override, double* out) {
  for (int64_t j = 0; j < n; ++j)
    out[j] = orc_significance_one(V[j], n_eff[j], M, L, est, delta, sigma_override);
}

void orc_flags(const double* V, const int32_t* n_eff, int64_t n, int64_t M, int64_t L, int est,
               double k, double delta, double sigma_override, uint8_t* flags) {
  for (int64_t j = 0; j < n; ++j)
    flags[j] = orc_flag_one(V[j], n_eff[j], M, L, est, k, delta, sigma_override);
}

/* Array combine, estimator and flags for every (f, b).
 * Eq. normedSum1: A = sum_i S1_i / P_i;  Eq. normedSum2: Bq = sum_i S2_i / P_i^2
 * (both up to the common factors M*count and (M*count)^2, which cancel).
 * Eq. avgSK, first form: V = (K+1)/(K-1) * (K * Bq / A^2 - 1), K = N_eff * M.
 * Eq. final, second form (L = 1 only): V = (M+1)/(M-1) * (M * Bq / N_eff - 1).
 * L = 0: Eq. (2) over all K samples: V = (K+1)/(K-1) * (K R2 - R1^2) / R1^2,
 * with the numerator formed exactly in 128-bit integers.
 * R1, R2 are the raw integer sums over the included inputs. */
void orc_combine(const int64_t* S1, const int64_t* S2, const int64_t* P, const uint8_t* mask,
                 int64_t N, int64_t F, int64_t B, int64_t M, int64_t L, int est, double k,
                 double delta, double sigma_override, double* A_out, double* Bq_out,
                 int64_t* R1_out, int64_t* R2_out, int32_t* n_eff_out, double* V_out,
                 uint8_t* flags_out) {
  for (int64_t f = 0; f < F; ++f)
    for (int64_t b = 0; b < B; ++b) {
      double A = 0.0, Bq = 0.0;
      int64_t R1 = 0, R2 = 0, n = 0;
      for (int64_t i = 0; i < N; ++i) {
        if (mask && mask[f * N + i] == 0) continue;
        int64_t idx = (f * B + b) * N + i;
        int64_t p = P[idx];
        if (p <= 0) continue;
        n += 1;
        R1 += S1[idx];
        R2 += S2[idx];
        if (L >= 1) {
          double pd = (double)p;
          A += (double)S1[idx] / pd;
          Bq += (double)S2[idx] / (pd * pd);
        }
      }
      int64_t K = n * M;
      double Kd = (double)K, Md = (double)M;
      double V;
      int invalid = (K < 2);
      if (L == 0) {
        A = (double)R1;
        Bq = (double)R2;
        invalid = invalid || (R1 == 0);
        if (!invalid) {
          __int128 num = (__int128)K * (__int128)R2 - (__int128)R1 * (__int128)R1;
          __int128 den = (__int128)R1 * (__int128)R1;
          V = (Kd + 1.0) / (Kd - 1.0) * ((double)num / (double)den);
        }
      } else {
        invalid = invalid || (A == 0.0);
        if (!invalid) {
          if (est == ORC_EST_TILDE)
            V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)n - 1.0);
          else
            V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);
        }
      }
      if (invalid) V = NAN;
      int64_t o = f * B + b;
      if (A_out) A_out[o] = A;
      if (Bq_out) Bq_out[o] = Bq;
      if (R1_out) R1_out[o] = R1;
      if (R2_out) R2_out[o] = R2;
      if (n_eff_out) n_eff_out[o] = (int32_t)n;
      if (V_out) V_out[o] = V;
      if (flags_out) flags_out[o] = orc_flag_one(V, n, M, L, est, k, delta, sigma_override);
    }
}

/* The same combine on real-valued sums (continuous chi-squared power). */
void orc_combine_f64(const double* S1, const double* S2, const double* P, int64_t N, int64_t F,
                     int64_t B, int64_t M, int64_t L, int est, double* V_out) {
  for (int64_t f = 0; f < F; ++f)
    for (int64_t b = 0; b < B; ++b) {
      double A = 0.0, Bq = 0.0, R1 = 0.0, R2 = 0.0;
      int64_t n = 0;
      for (int64_t i = 0; i < N; ++i) {
        int64_t idx = (f * B + b) * N + i;
        double p = P[idx];
        if (!(p > 0.0)) continue;
        n += 1;
        R1 += S1[idx];
        R2 += S2[idx];
        A += S1[idx] / p;
        Bq += S2[idx] / (p * p);
      }
      double Kd = (double)(n * M), Md = (double)M, V;
      if (n * M < 2) V = NAN;
      else if (L == 0) V = (Kd + 1.0) / (Kd - 1.0) * (Kd * R2 / (R1 * R1) - 1.0);
      else if (est == ORC_EST_TILDE) V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)n - 1.0);
      else V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);
      V_out[f * B + b] = V;
    }
}

/* Eq. originalSK: per-receiver estimate SK_i = (M+1)/(M-1) (M S2_i / S1_i^2 - 1).
 * NaN where S1_i = 0. */
void orc_sk_per_input(const int64_t* S1, const int64_t* S2, int64_t count, int64_t M, double* out) {
  double Md = (double)M;
  for (int64_t j = 0; j < count; ++j) {
    if (S1[j] == 0) { out[j] = NAN; continue; }
    double s1 = (double)S1[j];
    out[j] = (Md + 1.0) / (Md - 1.0) * (Md * (double)S2[j] / (s1 * s1) - 1.0);
  }
}

/* Whole path on one call: decode, sums, window, combine, flags.
 * hist (may be NULL when H = 0) is [F][H][N] S1 of the blocks just before
 * this call, oldest first. Outputs are [F][B][N] (S1, S2, P) and [F][B]. */
int orc_sk(const uint8_t* x, const uint8_t* mask, int64_t N, int64_t F, int64_t T, int64_t M,
           int64_t L, int est, double k, double delta, double sigma_override,
           const int64_t* hist, int64_t H, int64_t* S1, int64_t* S2, int64_t* P,
           int64_t* R1, int64_t* R2, int32_t* n_eff, double* V, uint8_t* flags) {
  if (M < 2 || T % M != 0 || N < 1 || F < 1 || L < 0) return -1;
  if (est == ORC_EST_TILDE && L != 1) return -1;
  int64_t B = T / M;
  orc_block_sums(x, N, F, T, M, S1, S2);
  orc_window(S1, hist, H, N, F, B, L, P);
  orc_combine(S1, S2, P, mask, N, F, B, M, L, est, k, delta, sigma_override, NULL, NULL, R1, R2,
              n_eff, V, flags);
  return 0;
}

/* ------------------------------------------------------------------ App. B
 * Digitised Gaussian model. A component is round(sigma z) clipped to
 * [-clip, clip]: Pr(v) = Phi((v+1/2)/sigma) - Phi((v-1/2)/sigma) for |v| <
 * clip, with both tails lumped into +-clip. The complex sample has
 * independent components, so p = re^2 + im^2 has the 2-D lattice PMF.
 * Output: m[0] = E[p], m[1] = E[p^2], m[2] = E[p^3], m[3] = E[p^4]. */
static double orc_phi(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

void orc_quantised_power_moments(double sigma, int clip, double* m) {
  double pr[64];
  for (int v = -clip; v <= clip; ++v) {
    double lo = (v == -clip) ? 0.0 : orc_phi(((double)v - 0.5) / sigma);
    double hi = (v == clip) ? 1.0 : orc_phi(((double)v + 0.5) / sigma);
    pr[v + clip] = hi - lo;
  }
  m[0] = m[1] = m[2] = m[3] = 0.0;
  for (int a = -clip; a <= clip; ++a)
    for (int c = -clip; c <= clip; ++c) {
      double w = pr[a + clip] * pr[c + clip];
      double p = (double)(a * a + c * c);
      m[0] += w * p;
      m[1] += w * p * p;
      m[2] += w * p * p * p;
      m[3] += w * p * p * p * p;
    }
}

/* ------------------------------------------------------------------ App. A
 * Per-channel statistics of the estimator over the blocks of a call: mean,
 * unbiased variance over the valid (non-NaN) blocks, and the effective number
 * of independent receivers N_eff = 4 / (M var) (the variance of the
 * estimator is 4/(nN) for N independent receivers, Eq. final). */
void orc_channel_stats(const double* V, int64_t F, int64_t B, int64_t M, double* mean, double* var,
                       double* n_eff_est, int64_t* count) {
  for (int64_t f = 0; f < F; ++f) {
    int64_t n = 0;
    double s = 0.0;
    for (int64_t b = 0; b < B; ++b)
      if (!isnan(V[f * B + b])) { s += V[f * B + b]; n += 1; }
    double m = n > 0 ? s / (double)n : NAN;
    double q = 0.0;
    for (int64_t b = 0; b < B; ++b)
      if (!isnan(V[f * B + b])) { double d = V[f * B + b] - m; q += d * d; }
    double v = n > 1 ? q / (double)(n - 1) : NAN;
    mean[f] = m;
    var[f] = v;
    n_eff_est[f] = (n > 1 && v > 0.0) ? 4.0 / ((double)M * v) : NAN;
    count[f] = n;
  }
}

/* ------------------------------------------------------------------ App. B
 * Monte-Carlo simulation of digitised data and the estimator (the paper's
 * way of setting thresholds). SplitMix64 (Steele, Lea and Flood 2014): key =
 * output function of the seed; draw n = output function of key + (n+1) *
 * 0x9E3779B97F4A7C15. Sample j of input i of estimate s uses draw
 * (s N + i) M + j; high 32 bits -> real part, low 32 bits -> imaginary part,
 * each = -clip + #{k : thr[k] <= u}, thr[k] = floor(2^32 Phi((k - clip + 1/2)/sigma)).
 * Each input is normalised by its own block mean (L = 1). */
static uint64_t orc_splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void orc_mc_thresholds(double sigma, int clip, uint32_t* thr) {
  for (int k = 0; k < 2 * clip; ++k) {
    double s = floor(orc_phi(((double)(k - clip) + 0.5) / sigma) * 4294967296.0);
    if (s < 0) s = 0;
    if (s > 4294967295.0) s = 4294967295.0;
    thr[k] = (uint32_t)s;
  }
}

/* Codes of input i, estimate s (for tests of the generator): re, im [M]. */
void orc_mc_codes(int64_t N, int64_t M, int clip, double sigma, uint64_t seed, int64_t s, int64_t i,
                  int32_t* re, int32_t* im) {
  uint32_t thr[16];
  orc_mc_thresholds(sigma, clip, thr);
  uint64_t key = orc_splitmix_out(seed);
  for (int64_t j = 0; j < M; ++j) {
    uint64_t n = ((uint64_t)s * N + i) * (uint64_t)M + j;
    uint64_t r = orc_splitmix_out(key + (n + 1) * 0x9E3779B97F4A7C15ULL);
    uint32_t ur = (uint32_t)(r >> 32), ui = (uint32_t)r;
    int a = -clip, c = -clip;
    for (int k = 0; k < 2 * clip; ++k) { a += (thr[k] <= ur); c += (thr[k] <= ui); }
    re[j] = a;
    im[j] = c;
  }
}

void orc_mc_calibrate(int64_t N, int64_t M, int est, int clip, double sigma, int64_t n_sim, uint64_t seed,
                      double* values) {
  int32_t* re = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  int32_t* im = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  for (int64_t s = 0; s < n_sim; ++s) {
    double Bq = 0.0;
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
      orc_mc_codes(N, M, clip, sigma, seed, s, i, re, im);
      int64_t s1 = 0, s2 = 0;
      for (int64_t j = 0; j < M; ++j) {
        int64_t p = (int64_t)re[j] * re[j] + (int64_t)im[j] * im[j];
        s1 += p;
        s2 += p * p;
      }
      if (s1 > 0) {
        Bq += (double)s2 / ((double)s1 * (double)s1);
        n += 1;
      }
    }
    double Md = (double)M, Kd = (double)(n * M), V = NAN;
    if (n > 0 && n * M >= 2) {
      if (est == ORC_EST_TILDE)
        V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)n - 1.0);
      else
        V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / ((double)n * (double)n) - 1.0);
    }
    values[s] = V;
  }
  free(re);
  free(im);
}

/* ------------------------------------------------------------------ Sec. 3.2
 * False-alarm thresholds for small K: quantiles of a Pearson type III law
 * with mean E, standard deviation s and skewness g = 10 / sqrt(K) (Sec. 2.1,
 * divided by sqrt(N) for the average of N receivers, Eq. final). The gamma
 * CDF is integrated numerically (composite Simpson); for shape a < 1 the
 * substitution u = t^a removes the singularity at 0. */
static double orc_gamma_cdf(double a, double x) {
  /* P(a, x) = int_0^x t^(a-1) e^-t dt / Gamma(a). With t = v^m the integrand
   * becomes m v^(m a - 1) exp(-v^m); m = ceil(6 / a) makes it smooth at 0, so
   * composite Simpson converges at its full order. For large a the mass sits
   * within a few sqrt(a) of a, and the integral starts below it. */
  if (x <= 0.0) return 0.0;
  int m = (int)ceil(6.0 / a);
  if (m < 1) m = 1;
  double tlo = 0.0;
  if (m == 1) {
    tlo = a - 60.0 * sqrt(a) - 60.0;
    if (tlo < 0.0) tlo = 0.0;
  }
  if (x <= tlo) return 0.0;
  const int n = 40000;
  double vlo = pow(tlo, 1.0 / m), vhi = pow(x, 1.0 / m);
  double h = (vhi - vlo) / n, s = 0.0;
  for (int k = 0; k <= n; ++k) {
    double v = vlo + k * h;
    double f = v > 0.0 ? (double)m * exp(((double)m * a - 1.0) * log(v) - pow(v, (double)m) - lgamma(a)) : 0.0;
    s += f * ((k == 0 || k == n) ? 1.0 : (k % 2 ? 4.0 : 2.0));
  }
  return s * h / 3.0;
}

double orc_pearson3_quantile(double mean, double sd, double skew, double p) {
  if (skew < 1e-6) {
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (lo + hi);
      if (0.5 * erfc(-mid / sqrt(2.0)) < p) lo = mid; else hi = mid;
    }
    return mean + sd * 0.5 * (lo + hi);
  }
  double a = 4.0 / (skew * skew);
  double lo = 0.0, hi = a + 20.0 * sqrt(a) + 20.0;
  while (orc_gamma_cdf(a, hi) < p) hi *= 2.0;
  for (int it = 0; it < 64; ++it) {
    double mid = 0.5 * (lo + hi);
    if (orc_gamma_cdf(a, mid) < p) lo = mid; else hi = mid;
  }
  return mean - 2.0 * sd / skew + sd * skew / 2.0 * 0.5 * (lo + hi);
}

/* Flags with false-alarm thresholds (fap per tail); the thresholds depend
 * only on N_eff, so they are computed once per distinct value. */
void orc_flags_fap(const double* V, const int32_t* n_eff, int64_t n, int64_t M, int64_t L, int est,
                   double fap, double delta, double sigma_override, double* lo_out, double* hi_out,
                   uint8_t* flags) {
  int32_t nmax = 0;
  for (int64_t j = 0; j < n; ++j)
    if (n_eff[j] > nmax) nmax = n_eff[j];
  double* tlo = (double*)malloc(sizeof(double) * ((size_t)nmax + 1));
  double* thi = (double*)malloc(sizeof(double) * ((size_t)nmax + 1));
  char* have = (char*)calloc((size_t)nmax + 1, 1);
  for (int64_t j = 0; j < n; ++j) {
    int64_t K = (int64_t)n_eff[j] * M;
    if (K < 2 || isnan(V[j])) {
      flags[j] = ORC_FLAG_INVALID;
      if (lo_out) lo_out[j] = NAN;
      if (hi_out) hi_out[j] = NAN;
      continue;
    }
    int32_t ne = n_eff[j];
    if (!have[ne]) {
      double E, s;
      orc_expectation(K, M, L, est, delta, sigma_override, &E, &s);
      double g = 10.0 / sqrt((double)K);
      tlo[ne] = orc_pearson3_quantile(E, s, g, fap);
      thi[ne] = orc_pearson3_quantile(E, s, g, 1.0 - fap);
      have[ne] = 1;
    }
    double lo = tlo[ne], hi = thi[ne];
    if (lo_out) lo_out[j] = lo;
    if (hi_out) hi_out[j] = hi;
    flags[j] = (uint8_t)((V[j] < lo ? ORC_FLAG_LOW : 0) | (V[j] > hi ? ORC_FLAG_HIGH : 0));
  }
  free(tlo);
  free(thi);
  free(have);
}
