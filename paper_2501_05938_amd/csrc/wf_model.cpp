// wf_model.cpp -- the launch-concurrency model of arXiv 2501.05938 (Sections 2.3,
// 2.4 and 3), applied to choosing how many streams the per-grid path spreads its
// launches over.
//
// The paper splits the run time of a job on s streams into a part the streams
// overlap, `sum` (Eq. 3), which ideally shrinks to sum/s, and an overhead that
// grows with s (Eq. 5):
//     T_overhead = (T_str - T_non_str) + (s - 1)/s * sum.
// It models sum as a straight line in the problem size (Eq. 4) and the overhead
// with two logarithmic forms, one per size regime (Eq. 7):
//     small (size <= split): a*size + b*log10(s) + c
//     big   (size >  split): (a*size + b)*log2(s^(4/3)) + c,
// both linear in (a, b, c), each fitted by least squares on a shuffled 3:1
// train/test split.  A stream count pays when its overhead stays below the time
// it saves, (s - 1)/s * sum (Eq. 6); the count with the largest positive gap is
// chosen, one stream when none has one (Section 3, where s = 1 is scored like
// the other candidates with gap -T_overhead(size, 1)).
#include "../../include/wf.h"
#include "wf_host.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

namespace {

// Least squares for a tall n x p system (p <= 3) by Householder QR on column-scaled
// data.  Returns false when the columns are (numerically) dependent.
bool lstsq(std::vector<double> X, std::vector<double> y, int n, int p, double* b) {
  if (n < p) return false;
  double scale[3] = {1, 1, 1};
  for (int j = 0; j < p; ++j) {
    double mx = 0;
    for (int i = 0; i < n; ++i) mx = std::max(mx, std::fabs(X[i * p + j]));
    if (mx == 0) return false;
    scale[j] = mx;
    for (int i = 0; i < n; ++i) X[i * p + j] /= mx;
  }
  double diag[3] = {0, 0, 0};
  for (int k = 0; k < p; ++k) {
    double norm = 0;
    for (int i = k; i < n; ++i) norm += X[i * p + k] * X[i * p + k];
    norm = std::sqrt(norm);
    if (norm < 1e-12 * std::sqrt((double)n)) return false;
    const double alpha = X[k * p + k] > 0 ? -norm : norm;
    // v = x - alpha e_k, stored in place; H = I - 2 v v^T / (v^T v)
    X[k * p + k] -= alpha;
    double vv = 0;
    for (int i = k; i < n; ++i) vv += X[i * p + k] * X[i * p + k];
    for (int j = k + 1; j < p; ++j) {
      double d = 0;
      for (int i = k; i < n; ++i) d += X[i * p + k] * X[i * p + j];
      const double f = 2 * d / vv;
      for (int i = k; i < n; ++i) X[i * p + j] -= f * X[i * p + k];
    }
    double d = 0;
    for (int i = k; i < n; ++i) d += X[i * p + k] * y[i];
    const double f = 2 * d / vv;
    for (int i = k; i < n; ++i) y[i] -= f * X[i * p + k];
    diag[k] = alpha;
  }
  // Back substitution on R (diagonal in diag[], above it in X).
  for (int k = p - 1; k >= 0; --k) {
    double s = y[k];
    for (int j = k + 1; j < p; ++j) s -= X[k * p + j] * b[j];
    b[k] = s / diag[k];
  }
  for (int j = 0; j < p; ++j) b[j] /= scale[j];
  return true;
}

void report(const std::vector<double>& X, const std::vector<double>& y, int p, const std::vector<int64_t>& idx,
            const double* b, double* r2, double* mse, int64_t* count) {
  double mean = 0;
  for (int64_t i : idx) mean += y[i];
  mean = idx.empty() ? 0 : mean / (double)idx.size();
  double ss_res = 0, ss_tot = 0;
  for (int64_t i : idx) {
    double yh = 0;
    for (int j = 0; j < p; ++j) yh += X[i * p + j] * b[j];
    ss_res += (y[i] - yh) * (y[i] - yh);
    ss_tot += (y[i] - mean) * (y[i] - mean);
  }
  *r2 = ss_tot > 0 ? 1.0 - ss_res / ss_tot : NAN;
  *mse = idx.empty() ? NAN : ss_res / (double)idx.size();
  *count = (int64_t)idx.size();
}

// Fit y ~ X on a 3:1 split given by `perm` (the first ceil(n/4) entries are the test set).
wf_status fit_split(const std::vector<double>& X, const std::vector<double>& y, int p, const int64_t* perm,
                    const char* what, double* b, wf_fit_report* rep) {
  const int64_t n = (int64_t)y.size();
  std::vector<char> seen((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (perm[i] < 0 || perm[i] >= n || seen[(size_t)perm[i]])
      return wfh::fail(WF_EINVAL, std::string(what) + ": permutation is not a permutation of its samples");
    seen[(size_t)perm[i]] = 1;
  }
  const int64_t n_test = (n + 3) / 4;
  std::vector<int64_t> tr(perm + n_test, perm + n), te(perm, perm + n_test);
  std::vector<double> Xt, yt;
  for (int64_t i : tr) {
    for (int j = 0; j < p; ++j) Xt.push_back(X[i * p + j]);
    yt.push_back(y[i]);
  }
  if (!lstsq(Xt, yt, (int)tr.size(), p, b))
    return wfh::fail(WF_EINVAL, std::string(what) + ": too few or degenerate training samples");
  if (rep) {
    report(X, y, p, tr, b, &rep->r2_train, &rep->mse_train, &rep->n_train);
    report(X, y, p, te, b, &rep->r2_test, &rep->mse_test, &rep->n_test);
  }
  return WF_OK;
}

double log2_s43(double s) { return std::log2(std::pow(s, 4.0 / 3.0)); }

}  // namespace

extern "C" wf_status wf_stream_model_fit(const wf_stream_sample* x, int64_t count, double split_size,
                                         const int64_t* perm_sum, const int64_t* perm_small,
                                         const int64_t* perm_big, wf_stream_model* out, wf_fit_report* rep) {
  if (!x || count <= 0 || !out || !perm_sum || !perm_small || !perm_big)
    return wfh::fail(WF_EINVAL, "samples, permutations and out must not be NULL");
  for (int64_t i = 0; i < count; ++i) {
    const wf_stream_sample& s = x[i];
    if (s.streams < 1 || !(s.size >= 0) || !std::isfinite(s.t_str) || !std::isfinite(s.t_non_str) ||
        !std::isfinite(s.sum) || !std::isfinite(s.size))
      return wfh::fail(WF_EINVAL, "sample " + std::to_string(i) + " is invalid");
  }
  // Eq. 4: one (size, sum) pair per distinct size, in order of first appearance; the
  // sum of a size is the mean over its samples.
  std::vector<double> sizes, sums;
  std::vector<int> nsum;
  std::map<double, size_t> at;
  for (int64_t i = 0; i < count; ++i) {
    auto it = at.find(x[i].size);
    if (it == at.end()) {
      at[x[i].size] = sizes.size();
      sizes.push_back(x[i].size);
      sums.push_back(x[i].sum);
      nsum.push_back(1);
    } else {
      sums[it->second] += x[i].sum;
      nsum[it->second] += 1;
    }
  }
  std::vector<double> Xs, ys;
  for (size_t k = 0; k < sizes.size(); ++k) {
    Xs.push_back(sizes[k]);
    Xs.push_back(1.0);
    ys.push_back(sums[k] / nsum[k]);
  }
  wf_stream_model m;
  double b2[2] = {0, 0};
  wf_status st = fit_split(Xs, ys, 2, perm_sum, "sum model (Eq. 4)", b2, rep ? &rep[0] : nullptr);
  if (st != WF_OK) return st;
  m.sum_slope = b2[0];
  m.sum_intercept = b2[1];
  m.split_size = split_size;
  // Eq. 5 on every sample with s >= 2, then Eq. 7 per regime, in input order.
  std::vector<double> Xsm, ysm, Xbg, ybg;
  for (int64_t i = 0; i < count; ++i) {
    const wf_stream_sample& s = x[i];
    if (s.streams < 2) continue;
    const double sv = (double)s.streams;
    const double ov = (s.t_str - s.t_non_str) + (sv - 1) / sv * s.sum;
    if (s.size <= split_size) {
      Xsm.insert(Xsm.end(), {s.size, std::log10(sv), 1.0});
      ysm.push_back(ov);
    } else {
      const double L = log2_s43(sv);
      Xbg.insert(Xbg.end(), {s.size * L, L, 1.0});
      ybg.push_back(ov);
    }
  }
  double b3[3] = {0, 0, 0};
  if (!ysm.empty()) {
    st = fit_split(Xsm, ysm, 3, perm_small, "small-size overhead model (Eq. 7)", b3, rep ? &rep[1] : nullptr);
    if (st != WF_OK) return st;
  } else if (rep) {
    rep[1] = wf_fit_report{NAN, NAN, NAN, NAN, 0, 0};
  }
  for (int j = 0; j < 3; ++j) m.small[j] = b3[j];
  double c3[3] = {0, 0, 0};
  if (!ybg.empty()) {
    st = fit_split(Xbg, ybg, 3, perm_big, "big-size overhead model (Eq. 7)", c3, rep ? &rep[2] : nullptr);
    if (st != WF_OK) return st;
  } else if (rep) {
    rep[2] = wf_fit_report{NAN, NAN, NAN, NAN, 0, 0};
  }
  for (int j = 0; j < 3; ++j) m.big[j] = c3[j];
  *out = m;
  return WF_OK;
}

extern "C" double wf_stream_model_overhead(const wf_stream_model* m, double size, int32_t s) {
  if (!m || s < 1) return NAN;
  const double sv = (double)s;
  if (size <= m->split_size) return m->small[0] * size + m->small[1] * std::log10(sv) + m->small[2];
  return (m->big[0] * size + m->big[1]) * log2_s43(sv) + m->big[2];
}

extern "C" wf_status wf_stream_model_choose(const wf_stream_model* m, double size, const int32_t* candidates,
                                            int32_t ncand, int32_t* best, double* gaps) {
  static const int32_t kDefault[6] = {1, 2, 4, 8, 16, 32};
  if (!m || !best) return wfh::fail(WF_EINVAL, "model and best must not be NULL");
  if (!candidates) {
    candidates = kDefault;
    ncand = 6;
  }
  if (ncand <= 0) return wfh::fail(WF_EINVAL, "no candidate stream counts");
  const double sum = m->sum_slope * size + m->sum_intercept;
  int32_t b = 1;
  double bg = 0;
  bool have = false;
  for (int32_t k = 0; k < ncand; ++k) {
    const int32_t s = candidates[k];
    if (s < 1) return wfh::fail(WF_EINVAL, "stream counts must be >= 1");
    const double g = (double)(s - 1) / (double)s * sum - wf_stream_model_overhead(m, size, s);
    if (gaps) gaps[k] = g;
    if (g > 0 && (!have || g > bg)) {
      have = true;
      bg = g;
      b = s;
    }
  }
  *best = b;
  return WF_OK;
}
