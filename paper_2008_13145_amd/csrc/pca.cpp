// Pruning in a reduced space and the cluster -> kernel rules.
//
// Section 4.1 of the paper transforms the normalized performance vectors with
// principal component analysis before k-means; section 4.2 turns a cluster
// into the kernel to deploy, either from a representative point (the
// configuration best for the k-means centroid) or, from the labels alone,
// from the geometric mean of the cluster's members.  Section 4.3 scores a
// kernel set by the geometric mean over problems of the fraction of the
// optimal performance it keeps; the same score picks the normalization the
// deployed pruning uses.
//
// Host code in FP64: the table is at most a few thousand rows by a few
// hundred configurations, so the covariance (n d^2) and the symmetric eigen-
// decomposition (a few sweeps of d^3) take milliseconds on one core, far
// below a kernel launch's worth of any GPU work they would replace, and FP64
// keeps the quantized coordinates identical to any other FP64 evaluation of
// the same definition.  The normalization and the integer k-means run on the
// GPU (prune.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "kt_internal.hpp"

namespace kt {

namespace {

constexpr int32_t PCA_MAX_D = 1024;
constexpr int32_t PCA_MAX_ROWS = 1 << 20;

// Cyclic Jacobi method for a symmetric d x d matrix A (row-major, FP64):
// every sweep visits the pairs (p, q), p < q, in order and applies the plane
// rotation that zeroes A[p][q] (rotation tangent t = sign(tau) /
// (|tau| + sqrt(1 + tau^2)), tau = (A[q][q] - A[p][p]) / (2 A[p][q]), the
// smaller of the two angles); sweeps repeat until the off-diagonal mass is
// negligible against the diagonal.  On return A's diagonal holds the
// eigenvalues and the columns of V the unit eigenvectors.
void jacobi_eigen(std::vector<double>& A, int d, std::vector<double>& V) {
  V.assign((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) V[(size_t)i * d + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * d + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < d; ++i) {
      diag += a(i, i) * a(i, i);
      for (int j = i + 1; j < d; ++j) off += a(i, j) * a(i, j);
    }
    if (off == 0.0 || off <= 1e-36 * diag) break;
    for (int p = 0; p < d - 1; ++p) {
      for (int q = p + 1; q < d; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double tau = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < d; ++r) {
          if (r == p || r == q) continue;
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = a(p, r) = c * arp - s * arq;
          a(r, q) = a(q, r) = s * arp + c * arq;
        }
        a(p, p) -= t * apq;
        a(q, q) += t * apq;
        a(p, q) = a(q, p) = 0.0;
        for (int r = 0; r < d; ++r) {
          const double vrp = V[(size_t)r * d + p], vrq = V[(size_t)r * d + q];
          V[(size_t)r * d + p] = c * vrp - s * vrq;
          V[(size_t)r * d + q] = s * vrp + c * vrq;
        }
      }
    }
  }
}

struct Pca {
  std::vector<double> mean;        // d
  std::vector<double> comps;       // d x d, row c = component c (decreasing variance)
  std::vector<double> var;         // d eigenvalues, decreasing
  std::vector<double> Z;           // n x m projections
  double explained = 1.0;
};

// Principal components of the rows x = q / 65535 of a Q16 table: centred at
// the column means, covariance Xc^T Xc / (n - 1), unit eigenvectors by
// decreasing eigenvalue (stable on the original index), each signed so that
// its first entry within a factor 1 - 1e-9 of the largest magnitude is
// positive; Z = Xc V_m.
void pca_fit(const uint16_t* Xq, int32_t n, int32_t d, int32_t m, Pca& P) {
  std::vector<double> Xc((size_t)n * d);
  P.mean.assign(d, 0.0);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = 0; j < d; ++j) P.mean[j] += Xq[(size_t)i * d + j] / 65535.0;
  for (int32_t j = 0; j < d; ++j) P.mean[j] /= n;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = 0; j < d; ++j) Xc[(size_t)i * d + j] = Xq[(size_t)i * d + j] / 65535.0 - P.mean[j];
  std::vector<double> C((size_t)d * d, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    const double* x = &Xc[(size_t)i * d];
    for (int32_t p = 0; p < d; ++p) {
      if (x[p] == 0.0) continue;
      double* row = &C[(size_t)p * d];
      for (int32_t q = p; q < d; ++q) row[q] += x[p] * x[q];
    }
  }
  double trace = 0.0;
  for (int32_t p = 0; p < d; ++p) {
    for (int32_t q = p; q < d; ++q) {
      C[(size_t)p * d + q] /= (n - 1);
      C[(size_t)q * d + p] = C[(size_t)p * d + q];
    }
    trace += C[(size_t)p * d + p];
  }
  std::vector<double> V;
  jacobi_eigen(C, d, V);
  std::vector<int32_t> order(d);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return C[(size_t)a * d + a] > C[(size_t)b * d + b];
  });
  P.var.resize(d);
  P.comps.assign((size_t)d * d, 0.0);
  for (int32_t c = 0; c < d; ++c) {
    const int32_t src = order[c];
    P.var[c] = C[(size_t)src * d + src];
    double* v = &P.comps[(size_t)c * d];
    double big = 0.0;
    for (int32_t j = 0; j < d; ++j) {
      v[j] = V[(size_t)j * d + src];
      big = std::max(big, fabs(v[j]));
    }
    int32_t first = 0;
    while (first < d && !(fabs(v[first]) >= (1.0 - 1e-9) * big)) ++first;
    if (first < d && v[first] < 0.0)
      for (int32_t j = 0; j < d; ++j) v[j] = -v[j];
  }
  double lead = 0.0;
  for (int32_t c = 0; c < m; ++c) lead += P.var[c];
  P.explained = trace > 0.0 ? lead / trace : 1.0;
  P.Z.assign((size_t)n * m, 0.0);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t c = 0; c < m; ++c) {
      const double* v = &P.comps[(size_t)c * d];
      const double* x = &Xc[(size_t)i * d];
      double s = 0.0;
      for (int32_t j = 0; j < d; ++j) s += x[j] * v[j];
      P.Z[(size_t)i * m + c] = s;
    }
}

// One offset and one scale for every coordinate: U = rint((Z - lo) / span * 65535).
void quantize(const std::vector<double>& Z, std::vector<uint16_t>& U, double* lo, double* span) {
  double mn = Z.empty() ? 0.0 : Z[0], mx = mn;
  for (double z : Z) { mn = std::min(mn, z); mx = std::max(mx, z); }
  *lo = mn;
  *span = mx - mn;
  U.assign(Z.size(), 0);
  if (*span == 0.0) return;
  for (size_t e = 0; e < Z.size(); ++e) U[e] = (uint16_t)nearbyint((Z[e] - mn) / *span * 65535.0);
}

// Fixed-point logarithm of a Q16 value: round(2^32 log2(max(q, 1) / 65535)).
const std::vector<int64_t>& log2_q16_table() {
  static const std::vector<int64_t> table = [] {
    std::vector<int64_t> t(65536);
    for (int q = 0; q < 65536; ++q)
      t[q] = (int64_t)nearbyint(4294967296.0 * log2((double)std::max(q, 1) / 65535.0));
    return t;
  }();
  return table;
}

// Distinct picks: each score vector in order takes its largest unpicked
// entry (lowest index on ties); empty clusters are skipped; a short list is
// completed from `fill` the same way.
void pick_distinct(const std::vector<std::vector<int64_t>>& scores, const std::vector<int64_t>& fill,
                   int32_t d, int32_t k, int32_t* chosen) {
  std::vector<char> used(d, 0);
  int32_t got = 0;
  auto take = [&](const std::vector<int64_t>& sc) {
    int32_t best = -1;
    for (int32_t j = 0; j < d; ++j)
      if (!used[j] && (best < 0 || sc[j] > sc[best])) best = j;
    used[best] = 1;
    chosen[got++] = best;
  };
  for (const auto& sc : scores) {
    if (got == k) break;
    if (!sc.empty()) take(sc);
  }
  while (got < k) take(fill);
}

kt_status representatives(Ctx* h, const uint16_t* Xq, int32_t n, int32_t d, const int32_t* labels,
                          int32_t n_clusters, int32_t k, kt_rep rep, int32_t* chosen) {
  std::vector<int64_t> count(n_clusters, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (labels[i] < 0 || labels[i] >= n_clusters) return fail(h, KT_EINVAL, "label out of range");
    count[labels[i]]++;
  }
  std::vector<std::vector<int64_t>> sums(n_clusters);
  std::vector<int64_t> fill(d, 0);
  const std::vector<int64_t>* L = rep == KT_REP_GEOMEAN ? &log2_q16_table() : nullptr;
  for (int32_t c = 0; c < n_clusters; ++c)
    if (count[c]) sums[c].assign(d, 0);
  for (int32_t i = 0; i < n; ++i) {
    std::vector<int64_t>& s = sums[labels[i]];
    const uint16_t* x = Xq + (size_t)i * d;
    for (int32_t j = 0; j < d; ++j) {
      const int64_t v = L ? (*L)[x[j]] : (int64_t)x[j];
      s[j] += v;
      fill[j] += v;
    }
  }
  if (rep == KT_REP_MEAN)   // rounded member means floor((2 s + n) / (2 n))
    for (int32_t c = 0; c < n_clusters; ++c)
      for (int64_t& v : sums[c]) v = (2 * v + count[c]) / (2 * count[c]);
  pick_distinct(sums, fill, d, k, chosen);
  return KT_OK;
}

// Fraction-of-optimal summary of one table (section 4.3).
kt_status evaluate(Ctx* h, const int64_t* T, int32_t n, int32_t d, const int32_t* rows,
                   int32_t n_eval, const int32_t* picks, const int32_t* chosen, int32_t k,
                   kt_eval* out) {
  double log_sum = 0.0, sum = 0.0, mn = 0.0, tb_sum = 0.0, tu_sum = 0.0;
  int64_t ge = 0;
  for (int32_t e = 0; e < n_eval; ++e) {
    const int32_t r = rows ? rows[e] : e;
    if (r < 0 || r >= n) return fail(h, KT_EINVAL, "evaluation row out of range");
    const int64_t* t = T + (size_t)r * d;
    int64_t tb = 0;
    for (int32_t j = 0; j < d; ++j)
      if (t[j] > 0 && (tb == 0 || t[j] < tb)) tb = t[j];
    int64_t tu = 0;
    if (picks) {
      if (picks[e] < 0 || picks[e] >= d) return fail(h, KT_EINVAL, "pick out of range");
      tu = t[picks[e]];
    } else {
      for (int32_t j = 0; j < k; ++j) {
        const int64_t v = t[chosen[j]];
        if (v > 0 && (tu == 0 || v < tu)) tu = v;
      }
    }
    if (tb <= 0 || tu <= 0)
      return fail(h, KT_EINVAL, "row " + std::to_string(r) + " has no measured time to evaluate");
    const double ratio = (double)tb / (double)tu;
    log_sum += log(ratio);
    sum += ratio;
    mn = e == 0 ? ratio : std::min(mn, ratio);
    ge += ratio >= 0.9;
    tb_sum += (double)tb;
    tu_sum += (double)tu;
  }
  out->n = n_eval;
  out->geomean = exp(log_sum / n_eval);
  out->mean = sum / n_eval;
  out->min = mn;
  out->frac_ge_0_9 = (double)ge / n_eval;
  out->time_weighted = tb_sum / tu_sum;
  return KT_OK;
}

}  // namespace

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_pca(kt_handle hh, const uint16_t* Xq, int32_t n, int32_t d, int32_t m, double* mean,
                 double* components, double* variances, uint16_t* U, double* lo_span,
                 double* explained) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!Xq) return fail(h, KT_EINVAL, "NULL table");
  if (n < 2 || d < 1 || m < 1 || m > d) return fail(h, KT_EINVAL, "need n >= 2 and 1 <= m <= d");
  if (d > PCA_MAX_D || n > PCA_MAX_ROWS)
    return fail(h, KT_EUNSUPPORTED, "PCA limits: d <= 1024 and n <= 2^20");
  Pca P;
  pca_fit(Xq, n, d, m, P);
  if (mean) memcpy(mean, P.mean.data(), (size_t)d * 8);
  if (components) memcpy(components, P.comps.data(), (size_t)m * d * 8);
  if (variances) memcpy(variances, P.var.data(), (size_t)d * 8);
  if (explained) *explained = P.explained;
  if (U || lo_span) {
    std::vector<uint16_t> Uq;
    double lo, span;
    quantize(P.Z, Uq, &lo, &span);
    if (U) memcpy(U, Uq.data(), Uq.size() * 2);
    if (lo_span) { lo_span[0] = lo; lo_span[1] = span; }
  }
  return KT_OK;
}

kt_status kt_representatives(kt_handle hh, const uint16_t* Xq, int32_t n, int32_t d,
                             const int32_t* labels, int32_t n_clusters, int32_t k, kt_rep rep,
                             int32_t* chosen) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!Xq || !labels || !chosen) return fail(h, KT_EINVAL, "NULL argument");
  if (n < 1 || d < 1 || n_clusters < 1 || k < 1 || k > d)
    return fail(h, KT_EINVAL, "need n, d, n_clusters >= 1 and 1 <= k <= d");
  if (rep != KT_REP_MEAN && rep != KT_REP_GEOMEAN)
    return fail(h, KT_EINVAL, "labels-only representatives are KT_REP_MEAN or KT_REP_GEOMEAN");
  if (n > (1 << 26))   // keeps every sum of fixed-point logarithms above -2^62
    return fail(h, KT_EUNSUPPORTED, "representatives limit: n <= 2^26");
  return representatives(h, Xq, n, d, labels, n_clusters, k, rep, chosen);
}

kt_status kt_log2_q16_table(int64_t* table) {
  if (!table) return fail(nullptr, KT_EINVAL, "NULL table");
  memcpy(table, log2_q16_table().data(), 65536 * 8);
  return KT_OK;
}

kt_status kt_evaluate(kt_handle hh, const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                      const int32_t* rows, int32_t n_eval, const int32_t* picks,
                      const int32_t* chosen, int32_t k, kt_eval* out) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!time_ns || !out) return fail(h, KT_EINVAL, "NULL argument");
  if (n_rows < 1 || n_configs < 1) return fail(h, KT_EINVAL, "empty table");
  if (!rows) n_eval = n_rows;
  if (n_eval < 1) return fail(h, KT_EINVAL, "nothing to evaluate");
  if (!picks) {
    if (!chosen || k < 1) return fail(h, KT_EINVAL, "a ceiling needs the chosen configurations");
    for (int32_t j = 0; j < k; ++j)
      if (chosen[j] < 0 || chosen[j] >= n_configs) return fail(h, KT_EINVAL, "chosen id out of range");
  }
  return evaluate(h, time_ns, n_rows, n_configs, rows, n_eval, picks, chosen, k, out);
}

kt_status kt_prune_pca(kt_handle hh, const int64_t* time_ns, int32_t n, int32_t d, int32_t k,
                       kt_norm norm, int32_t m, kt_rep rep, uint64_t seed, int32_t n_init,
                       int32_t max_iter, void* workspace, size_t ws_bytes, void* stream,
                       int32_t* chosen, int64_t* inertia_out, int32_t* labels, double* explained) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (!time_ns || !chosen || !inertia_out) return fail(h, KT_EINVAL, "NULL argument");
  if (n < 2 || d < 1 || m < 1 || m > d) return fail(h, KT_EINVAL, "need n >= 2 and 1 <= m <= d");
  if (k < 1 || k > n || k > d) return fail(h, KT_EINVAL, "need 1 <= k <= min(n_rows, n_configs)");
  if (rep != KT_REP_CENTROID && rep != KT_REP_GEOMEAN)
    return fail(h, KT_EINVAL, "PCA pruning takes KT_REP_CENTROID or KT_REP_GEOMEAN");
  if (d > PCA_MAX_D) return fail(h, KT_EUNSUPPORTED, "PCA limit: d <= 1024");
  std::vector<uint16_t> Xq((size_t)n * d);
  kt_status st = normalize_table_host(h, time_ns, n, d, norm, workspace, ws_bytes,
                                      (hipStream_t)stream, Xq.data());
  if (st != KT_OK) return st;
  Pca P;
  pca_fit(Xq.data(), n, d, m, P);
  std::vector<uint16_t> U;
  double lo, span;
  quantize(P.Z, U, &lo, &span);
  std::vector<int32_t> lab(n);
  std::vector<int64_t> cent((size_t)k * m);
  st = kt_kmeans_u16(hh, U.data(), n, m, k, seed, n_init, max_iter, workspace, ws_bytes, stream,
                     lab.data(), cent.data(), inertia_out);
  if (st != KT_OK) return st;
  if (rep == KT_REP_GEOMEAN) {
    st = representatives(h, Xq.data(), n, d, lab.data(), k, k, KT_REP_GEOMEAN, chosen);
    if (st != KT_OK) return st;
  } else {
    // each centroid read back in the original coordinates as Q16 values
    std::vector<std::vector<int64_t>> scores(k, std::vector<int64_t>(d));
    for (int32_t c = 0; c < k; ++c) {
      std::vector<double> z(m);
      for (int32_t q = 0; q < m; ++q) z[q] = lo + (double)cent[(size_t)c * m + q] * span / 65535.0;
      for (int32_t j = 0; j < d; ++j) {
        double x = P.mean[j];
        for (int32_t q = 0; q < m; ++q) x += P.comps[(size_t)q * d + j] * z[q];
        scores[c][j] = (int64_t)nearbyint(65535.0 * x);
      }
    }
    pick_distinct(scores, scores[0], d, k, chosen);
  }
  if (labels) memcpy(labels, lab.data(), (size_t)n * 4);
  if (explained) *explained = P.explained;
  return KT_OK;
}

kt_status kt_prune_auto(kt_handle hh, const int64_t* time_ns, int32_t n, int32_t d, int32_t k,
                        uint64_t seed, int32_t n_init, int32_t max_iter, void* workspace,
                        size_t ws_bytes, void* stream, int32_t* chosen, int32_t* norm_out,
                        double* scores) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!chosen || !norm_out) return fail(h, KT_EINVAL, "NULL argument");
  double best = -1.0;
  std::vector<int32_t> ch(k > 0 ? k : 1);
  for (int norm = 0; norm < 4; ++norm) {
    int64_t inertia = 0;
    kt_status st = kt_prune(hh, time_ns, n, d, k, (kt_norm)norm, seed, n_init, max_iter, workspace,
                            ws_bytes, stream, ch.data(), &inertia, nullptr, nullptr);
    if (st != KT_OK) return st;
    kt_eval ev;
    st = evaluate(h, time_ns, n, d, nullptr, n, nullptr, ch.data(), k, &ev);
    if (st != KT_OK) return st;
    if (scores) scores[norm] = ev.geomean;
    if (ev.geomean > best) {
      best = ev.geomean;
      *norm_out = norm;
      memcpy(chosen, ch.data(), (size_t)k * 4);
    }
  }
  return KT_OK;
}

}  // extern "C"
