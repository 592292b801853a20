// Digitisation model for the flag thresholds (App. B).
//
// The paper sets its excision thresholds from simulations of the correlator's
// 4+4-bit data: under digitisation the mean of the estimator converges to a
// value offset from 1, and that offset is added to the threshold, while the
// variance converges to the undigitised value for large arrays. Here the
// simulation is replaced by the exact distribution: a component is
// round(sigma z) clipped to [-clip, clip], so p = Re^2 + Im^2 has a PMF over
// the (2 clip + 1)^2 lattice points, and its moments follow by summation.
//
// With q = p / E[p] per input (what the running normaliser approximates),
//   mean(V) -> kappa_bar - 1,  kappa = E[q^2]   (2 for chi-squared power)
//   var(V)  ~ (M / K^2) sum_i [Var(q^2) - 4 kappa_bar Cov(q, q^2) + 4 kappa_bar^2 Var(q)]
// (first-order delta method on V + 1 = K sum q^2 / (sum q)^2); for
// chi-squared power this is 4/K, the paper's variance (Eq. final).
#include <math.h>
#include <stdint.h>

#include <vector>

#include "sk.h"

namespace {

double normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

// E[p^k], k = 1..4, for one input.
void lattice_moments(double sigma, int clip, double m[4]) {
  std::vector<double> pr(2 * clip + 1);
  for (int v = -clip; v <= clip; ++v) {
    const double lo = v == -clip ? 0.0 : normal_cdf((v - 0.5) / sigma);
    const double hi = v == clip ? 1.0 : normal_cdf((v + 0.5) / sigma);
    pr[v + clip] = hi - lo;
  }
  m[0] = m[1] = m[2] = m[3] = 0.0;
  for (int re = -clip; re <= clip; ++re) {
    for (int im = -clip; im <= clip; ++im) {
      const double w = pr[re + clip] * pr[im + clip];
      const double p = (double)(re * re + im * im);
      double pk = p;
      for (int k = 0; k < 4; ++k) {
        m[k] += w * pk;
        pk *= p;
      }
    }
  }
}

}  // namespace

extern "C" int sk_digitised_expectation(const double* sigma, int32_t n, int32_t block_len,
                                        int32_t clip, double* delta, double* sigma_v) {
  if (!sigma || n < 1 || block_len < 2 || clip < 1 || clip > 7 || !delta || !sigma_v) return SK_ERR_INVALID_ARG;
  std::vector<double> k2(n), k3(n), k4(n);
  double kbar = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!(sigma[i] > 0.0)) return SK_ERR_INVALID_ARG;
    double m[4];
    lattice_moments(sigma[i], clip, m);
    const double mu = m[0];
    k2[i] = m[1] / (mu * mu);
    k3[i] = m[2] / (mu * mu * mu);
    k4[i] = m[3] / (mu * mu * mu * mu);
    kbar += k2[i];
  }
  kbar /= n;
  double acc = 0.0;
  for (int i = 0; i < n; ++i) {
    const double var_q = k2[i] - 1.0;
    const double var_q2 = k4[i] - k2[i] * k2[i];
    const double cov = k3[i] - k2[i];
    acc += var_q2 - 4.0 * kbar * cov + 4.0 * kbar * kbar * var_q;
  }
  const double M = block_len;
  const double K = (double)n * M;
  const double c = (K + 1.0) / (K - 1.0);
  *delta = kbar - 2.0;
  *sigma_v = c * sqrt(M / (K * K) * acc);
  return SK_OK;
}
