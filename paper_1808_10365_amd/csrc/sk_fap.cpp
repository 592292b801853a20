// False-alarm thresholds for small effective sample counts (Sec. 3.2 notes
// that a symmetric cut relies on large nN, and that thresholds from the
// predicted false-alarm probability suit smaller nN where the skewness of the
// estimator matters).
//
// The estimator's distribution is approximated by a Pearson type III (shifted
// gamma) law with its first three moments: mean E, standard deviation s and
// skewness g = 10 / sqrt(K) (Sec. 2.1 gives 10 / sqrt(M) for one receiver; the
// multi-receiver estimator averages N of them, Eq. final, dividing the
// skewness by sqrt(N)). With shape a = 4 / g^2 and scale s g / 2, the value
// at lower-tail probability p is E - 2 s / g + (s g / 2) G_a^{-1}(p), where G_a
// is the regularised lower incomplete gamma function. The thresholds are the
// values at p and 1 - p.
#include <math.h>

#include "sk_internal.h"

namespace sk {
namespace {

// Regularised lower incomplete gamma P(a, x): power series for x < a + 1,
// otherwise 1 - Q(a, x) with Q from its continued fraction (modified Lentz).
double reg_gamma_p(double a, double x) {
  if (x <= 0.0) return 0.0;
  const double lead = a * log(x) - x - lgamma(a);
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (term < sum * 1e-17) break;
    }
    return sum * exp(lead);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int n = 1; n < 100000; ++n) {
    const double an = -n * (n - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return 1.0 - exp(lead) * h;
}

// x with P(a, x) = p, by bisection on a bracket that doubles until it holds.
double gamma_quantile(double a, double p) {
  double lo = 0.0, hi = a + 10.0 * sqrt(a) + 10.0;
  while (reg_gamma_p(a, hi) < p) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (reg_gamma_p(a, mid) < p) lo = mid; else hi = mid;
    if (hi - lo <= 1e-15 * hi) break;
  }
  return 0.5 * (lo + hi);
}

double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (0.5 * erfc(-mid / sqrt(2.0)) < p) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

double pearson3_quantile(double mean, double sd, double skew, double p) {
  if (skew < 1e-6) return mean + sd * normal_quantile(p);
  const double a = 4.0 / (skew * skew);
  const double scale = sd * skew / 2.0;
  return mean - 2.0 * sd / skew + scale * gamma_quantile(a, p);
}

}  // namespace sk

extern "C" int sk_pearson3_quantile(double mean, double sd, double skew, double p, double* out) {
  if (!out || !(sd > 0.0) || !(skew >= 0.0) || !(p > 0.0) || !(p < 1.0)) return SK_ERR_INVALID_ARG;
  *out = sk::pearson3_quantile(mean, sd, skew, p);
  return SK_OK;
}
