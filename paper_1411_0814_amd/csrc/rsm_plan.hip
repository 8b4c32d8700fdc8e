// Step 1 of the algorithm (Section IV-A): how many sub-matrices to draw, from Theorem 3's
// bound on the trial count and Lemma 1's normal-approximation bracket of the binomial
// distribution function.  Host code only: no device call, nothing allocated.
//
// Theorem 3 is stated for row-first sampling (k rows per trial; the columns known on all of
// them, about n rho^k, form the sub-matrix).  Column-first sampling (method M1: l columns,
// the rows known on all of them) is the same sampling of Y^T, so its bound is the row-first
// one with m and n exchanged and l in place of k.
//
// Lemma 1's sum for P(X < k) runs to i = k; it is read as P(X <= k) for X ~ B(n, rho), i.e.
// C_{n,rho}(k) <= P(X <= k) <= C_{n,rho}(k + 1), the reading under which the lemma's end
// cases (k = 0 and k = n - 1 hold with equality) are consistent.
#include <cmath>
#include <cstdint>

#include "rsm.h"

namespace {

// phi(x, rho) of Lemma 1: the Kullback-Leibler divergence of Bernoulli(x) from
// Bernoulli(rho), with 0 log 0 = 0.
double kl_bernoulli(double x, double rho) {
  const double a = x <= 0.0 ? 0.0 : x * std::log(x / rho);
  const double b = x >= 1.0 ? 0.0 : (1.0 - x) * std::log((1.0 - x) / (1.0 - rho));
  return a + b;
}

bool lemma1_args_ok(int64_t n, double rho, int64_t k) {
  return n >= 1 && k >= 0 && k <= n && rho > 0.0 && rho < 1.0;
}

// C_{n,rho}(k): (1 - rho)^n at k = 0, 1 - rho^n at k = n, otherwise the standard normal
// distribution function at sgn(k/n - rho) sqrt(2 n phi(k/n, rho)).
double lemma1(int64_t n, double rho, int64_t k) {
  const double nd = static_cast<double>(n);
  if (k == 0) return std::pow(1.0 - rho, nd);
  if (k == n) return 1.0 - std::pow(rho, nd);
  const double x = static_cast<double>(k) / nd;
  const double z = std::copysign(1.0, x - rho) * std::sqrt(2.0 * nd * kl_bernoulli(x, rho));
  return 0.5 * std::erfc(-z / std::sqrt(2.0));
}

// Theorem 3 as stated: rows m, columns n, k rows per trial.  Returns RSM_OK and the bound
// (+inf when no trial is likely to keep more than r columns).
int32_t bound_rows_first(int64_t m, int64_t n, double rho, int32_t r, int32_t k, double eps,
                         double* out) {
  if (m < 1 || n < 1 || r < 1 || k <= r || !(eps > 0.0 && eps < 1.0) ||
      !(rho > 0.0 && rho < 1.0) || static_cast<int64_t>(r) + 2 > n)
    return RSM_E_ARG;
  const double p = std::pow(rho, static_cast<double>(k));
  if (!(p > 0.0)) {  // rho^k underflows: no trial keeps a column
    *out = INFINITY;
    return RSM_OK;
  }
  const double tail = 1.0 - lemma1(n, p, static_cast<int64_t>(r) + 2);
  if (!(tail > 0.0)) {
    *out = INFINITY;
    return RSM_OK;
  }
  *out = static_cast<double>(m) * static_cast<double>(n) * rho /
         (static_cast<double>(k) * static_cast<double>(r + 1) * tail) * std::log(1.0 / (1.0 - eps));
  return RSM_OK;
}

}  // namespace

extern "C" {

int32_t rsm_lemma1_c(int64_t n, double rho, int64_t k, double* value) {
  if (!value || !lemma1_args_ok(n, rho, k)) return RSM_E_ARG;
  *value = lemma1(n, rho, k);
  return RSM_OK;
}

int32_t rsm_trials_bound(int64_t m, int64_t n, double rho, int32_t r, int32_t l, double eps,
                         int32_t rows_first, double* bound) {
  if (!bound) return RSM_E_ARG;
  const int32_t k = l == 0 ? r + 1 : l;
  return rows_first ? bound_rows_first(m, n, rho, r, k, eps, bound)
                    : bound_rows_first(n, m, rho, r, k, eps, bound);
}

int32_t rsm_plan_trials(int64_t m, int64_t n, double rho, int32_t r, int32_t l, double eps,
                        int32_t rows_first, int64_t* trials) {
  if (!trials) return RSM_E_ARG;
  double b = 0.0;
  const int32_t st = rsm_trials_bound(m, n, rho, r, l, eps, rows_first, &b);
  if (st != RSM_OK) return st;
  // an infinite (or unrepresentable) bound: no useful trial count exists at this density
  if (!std::isfinite(b) || b >= 9.2e18) return RSM_E_ARG;
  *trials = static_cast<int64_t>(std::ceil(b));
  return RSM_OK;
}

}  // extern "C"
