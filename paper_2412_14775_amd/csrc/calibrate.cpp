// calibrate.cpp -- host-side hyperparameter helpers (Section 2.3): thresholds from a
// desired false-alarm probability, and calibration of d and the thresholds on the
// kernel's own statistics of RFI-free data.  No device code.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/rfi.h"
#include "internal.h"

namespace {

// E[prod w_i^{a_i}] for w ~ Dirichlet(k, ..., k) with W components:
// Gamma(Wk) / Gamma(Wk + sum a) * prod Gamma(k + a_i) / Gamma(k).
double dirichlet_moment(int W, double k, std::initializer_list<int> a) {
  double s = 0.0, lg = 0.0;
  for (int e : a) {
    s += e;
    lg += std::lgamma(k + e) - std::lgamma(k);
  }
  return std::exp(std::lgamma(W * k) - std::lgamma(W * k + s) + lg);
}

// Standard normal quantile by bisection on the CDF (robust, 1e-12 absolute).
double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int i = 0; i < 200; ++i) {
    const double mid = 0.5 * (lo + hi);
    (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p ? lo : hi) = mid;
  }
  return 0.5 * (lo + hi);
}

// Quantile of chi-square with 3 degrees of freedom: CDF(x) = erf(sqrt(x/2)) - sqrt(2x/pi) exp(-x/2).
double chi2_3_quantile(double p) {
  double lo = 0.0, hi = 400.0;
  for (int i = 0; i < 200; ++i) {
    const double x = 0.5 * (lo + hi);
    const double cdf = std::erf(std::sqrt(0.5 * x)) - std::sqrt(2.0 * x / M_PI) * std::exp(-0.5 * x);
    (cdf < p ? lo : hi) = x;
  }
  return 0.5 * (lo + hi);
}

// Empirical quantile (linear interpolation between order statistics).
double quantile(std::vector<float> &v, double p) {
  if (v.empty()) return NAN;
  const double pos = p * (double)(v.size() - 1);
  const size_t i = (size_t)std::floor(pos);
  std::nth_element(v.begin(), v.begin() + i, v.end());
  const double a = v[i];
  if (i + 1 >= v.size()) return a;
  const double b = *std::min_element(v.begin() + i + 1, v.end());
  return a + (pos - (double)i) * (b - a);
}

}  // namespace

extern "C" {

int rfi_sk_null_moments(int32_t W, float d, double *mean, double *var, double *skew) {
  if (W < 2 || !(d > 0.0f) || !std::isfinite(d) || mean == nullptr || var == nullptr || skew == nullptr)
    return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "need W >= 2, finite d > 0 and non-NULL outputs");
  const double k = d;
  // X = sum_i w_i^2 with w = x / sum x, x_i ~ Gamma(k) i.i.d.: w is Dirichlet(k, ..., k)
  const double m1 = W * dirichlet_moment(W, k, {2});
  const double m2 = W * dirichlet_moment(W, k, {4}) + (double)W * (W - 1) * dirichlet_moment(W, k, {2, 2});
  const double m3 = W * dirichlet_moment(W, k, {6}) + 3.0 * W * (W - 1) * dirichlet_moment(W, k, {4, 2}) +
                    (double)W * (W - 1) * (W - 2) * dirichlet_moment(W, k, {2, 2, 2});
  const double pre = (W * k + 1.0) / (W - 1.0);
  const double a = pre * W;  // tau = a X - pre
  *mean = a * m1 - pre;
  *var = a * a * (m2 - m1 * m1);
  *skew = a * a * a * (m3 - 3.0 * m1 * m2 + 2.0 * m1 * m1 * m1) / std::pow(*var, 1.5);
  return RFI_OK;
}

int rfi_thresholds_from_pfa(int32_t W, float d, double pfa_sk, double pfa_ds, float *sk_low, float *sk_high,
                            float *ds_gamma) {
  if (!(pfa_sk > 0.0 && pfa_sk < 1.0 && pfa_ds > 0.0 && pfa_ds < 1.0))
    return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "false-alarm probabilities must be in (0, 1)");
  if (sk_low == nullptr || sk_high == nullptr || ds_gamma == nullptr)
    return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "outputs must not be NULL");
  double mean, var, skew;
  if (int rc = rfi_sk_null_moments(W, d, &mean, &var, &skew)) return rc;
  const double sd = std::sqrt(var);
  auto cornish_fisher = [&](double p) {
    const double z = normal_quantile(p);
    return mean + sd * (z + (z * z - 1.0) * skew / 6.0);
  };
  *sk_low = (float)cornish_fisher(0.5 * pfa_sk);
  *sk_high = (float)cornish_fisher(1.0 - 0.5 * pfa_sk);
  *ds_gamma = (float)std::min(1.0, std::sqrt(chi2_3_quantile(1.0 - pfa_ds) / (3.0 * W)));
  return RFI_OK;
}

int rfi_calibrate_from_stats(const float *stats, size_t n_windows, int32_t W, float d_used, double pfa_sk,
                             double pfa_ds, float *d_cal, float *sk_low, float *sk_high, float *ds_gamma) {
  if (stats == nullptr || d_cal == nullptr || sk_low == nullptr || sk_high == nullptr || ds_gamma == nullptr)
    return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "pointers must not be NULL");
  if (W < 2 || !(d_used > 0.0f) || !(pfa_sk > 0.0 && pfa_sk < 1.0 && pfa_ds > 0.0 && pfa_ds < 1.0))
    return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "need W >= 2, d_used > 0, probabilities in (0, 1)");
  const double pre_used = (W * (double)d_used + 1.0) / (W - 1.0);
  std::vector<float> ratio;  // R - 1 = W S2 / S1^2 - 1, recovered from tau
  std::vector<float> r;
  ratio.reserve(n_windows);
  r.reserve(2 * n_windows);
  double sum = 0.0;
  for (size_t i = 0; i < n_windows; ++i) {
    const float tau = stats[3 * i], rre = stats[3 * i + 1], rim = stats[3 * i + 2];
    if (std::isfinite(tau)) {
      const double x = tau / pre_used;
      ratio.push_back((float)x);
      sum += x;
    }
    if (std::isfinite(rre)) r.push_back(rre);
    if (std::isfinite(rim) && rim != 0.0f) r.push_back(rim);  // autocorrelations have r_im = 0
  }
  if (ratio.size() < 2 || r.empty()) return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "too few finite statistics");
  const double er1 = sum / (double)ratio.size();  // E[R] - 1
  if (!(er1 > 0.0)) return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "degenerate statistics (E[W S2/S1^2] <= 1)");
  // E[tau] = 1  <=>  (W d + 1) / (W - 1) * E[R - 1] = 1
  const double d = ((W - 1.0) / er1 - 1.0) / W;
  if (!(d > 0.0)) return rfi::set_error(RFI_ERR_INVALID_ARGUMENT, "calibrated d is not positive");
  const double pre = (W * d + 1.0) / (W - 1.0);
  *d_cal = (float)d;
  *sk_low = (float)(pre * quantile(ratio, 0.5 * pfa_sk));
  *sk_high = (float)(pre * quantile(ratio, 1.0 - 0.5 * pfa_sk));
  *ds_gamma = (float)std::min(1.0, quantile(r, 1.0 - pfa_ds));
  return RFI_OK;
}

}  // extern "C"
