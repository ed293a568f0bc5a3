// Decision-tree pruning (section 4.1, "Decision tree"): a regression tree
// from the matrix sizes (M, N, K, batch, transA, transB) to the normalized
// performance vector, grown best first to k leaves; every leaf's rounded
// mean vector picks one configuration.  Host code: the tree has at most k
// leaves over at most a few thousand rows, far below a kernel launch's cost.
//
// Exactness: per node, column sums are int64; squared norms, split scores
// A / n_L + B / n_R and gains are compared as fractions in 128-bit integers
// (bounded by n <= 4096 rows and d <= 256 configurations).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "kt_internal.hpp"

namespace kt {

namespace {

typedef __int128 i128;

constexpr int NF = 6;
constexpr int32_t TREE_MAX_ROWS = 4096;
constexpr int32_t TREE_MAX_D = 256;

uint64_t isqrt_prod(uint64_t a, uint64_t b) {   // floor(sqrt(a * b)), a, b < 2^40
  const unsigned __int128 p = (unsigned __int128)a * b;
  uint64_t r = (uint64_t)std::sqrt((long double)p);
  while ((unsigned __int128)r * r > p) --r;
  while ((unsigned __int128)(r + 1) * (r + 1) <= p) ++r;
  return r;
}

struct Frac {   // num / den with den > 0
  i128 num, den;
};
bool greater(const Frac& a, const Frac& b) { return a.num * b.den > b.num * a.den; }

struct Split {
  bool ok = false;
  Frac gain{0, 1};
  int f = -1;
  int64_t t = 0;
};

struct Node {
  std::vector<int32_t> rows;
  int f = -1;
  int64_t t = 0;
  int left = -1, right = -1;
};

struct RegTree {
  const int64_t* F;      // n x NF features
  const uint16_t* X;     // n x d
  int32_t d;

  i128 sqnorm(const std::vector<int64_t>& s) const {
    i128 a = 0;
    for (int32_t j = 0; j < d; ++j) a += (i128)s[j] * s[j];
    return a;
  }

  Split best_split(const std::vector<int32_t>& rows) const {
    Split best;
    const int64_t n = (int64_t)rows.size();
    std::vector<int64_t> tot(d, 0), left(d), right(d);
    for (int32_t i : rows)
      for (int32_t j = 0; j < d; ++j) tot[j] += X[(size_t)i * d + j];
    const i128 P = sqnorm(tot);
    Frac best_score{0, 1};
    std::vector<int32_t> order(rows);
    for (int f = 0; f < NF; ++f) {
      std::stable_sort(order.begin(), order.end(),
                       [&](int32_t a, int32_t b) { return F[(size_t)a * NF + f] < F[(size_t)b * NF + f]; });
      std::fill(left.begin(), left.end(), 0);
      int64_t pos = 0;
      while (pos < n) {
        const int64_t v = F[(size_t)order[pos] * NF + f];
        while (pos < n && F[(size_t)order[pos] * NF + f] == v) {
          const uint16_t* x = X + (size_t)order[pos] * d;
          for (int32_t j = 0; j < d; ++j) left[j] += x[j];
          ++pos;
        }
        if (pos == n) break;
        const int64_t b = F[(size_t)order[pos] * NF + f];
        for (int32_t j = 0; j < d; ++j) right[j] = tot[j] - left[j];
        const i128 A = sqnorm(left), B = sqnorm(right);
        const int64_t nl = pos, nr = n - pos;
        const Frac score{A * nr + B * nl, (i128)nl * nr};
        if (!best.ok || greater(score, best_score)) {
          best.ok = true;
          best_score = score;
          best.f = f;
          best.t = (int64_t)isqrt_prod((uint64_t)v, (uint64_t)b);
        }
      }
    }
    if (best.ok)   // gain = score - P / n
      best.gain = Frac{best_score.num * n - P * best_score.den, best_score.den * n};
    return best;
  }
};

// Grow the regression tree best first to at most k leaves; returns the
// nodes and the leaves in pre-order (left child first).
kt_status grow_tree(Ctx* h, const kt_shape* shapes, const uint16_t* Xq, int32_t n, int32_t d,
                    int32_t k, std::vector<Node>& nodes, std::vector<int>& pre) {
  if (!shapes || !Xq) return fail(h, KT_EINVAL, "NULL argument");
  if (n < 1 || d < 1 || k < 1 || k > d) return fail(h, KT_EINVAL, "need n, d >= 1 and 1 <= k <= d");
  if (n > TREE_MAX_ROWS || d > TREE_MAX_D)
    return fail(h, KT_EUNSUPPORTED, "decision-tree pruning limits: n <= 4096, d <= 256");
  std::vector<int64_t> F((size_t)n * NF);
  for (int32_t i = 0; i < n; ++i) {
    const kt_shape& s = shapes[i];
    const int64_t v[NF] = {s.M, s.N, s.K, s.batch, s.transA, s.transB};
    for (int f = 0; f < NF; ++f) {
      if (v[f] < 0 || v[f] >= ((int64_t)1 << 40)) return fail(h, KT_EINVAL, "shape feature out of range");
      F[(size_t)i * NF + f] = v[f];
    }
  }
  RegTree tr{F.data(), Xq, d};
  nodes.assign(1, Node());
  nodes[0].rows.resize(n);
  std::iota(nodes[0].rows.begin(), nodes[0].rows.end(), 0);
  std::vector<Split> cand(1, tr.best_split(nodes[0].rows));
  std::vector<int> leaves(1, 0);   // ascending node id = creation order
  const Frac zero{0, 1};
  while ((int32_t)leaves.size() < k) {
    int pick = -1;
    for (int leaf : leaves) {
      const Split& c = cand[leaf];
      if (!c.ok || !greater(c.gain, zero)) continue;
      if (pick < 0 || greater(c.gain, cand[pick].gain)) pick = leaf;
    }
    if (pick < 0) break;
    const int f = cand[pick].f;
    const int64_t t = cand[pick].t;
    Node l, r;
    for (int32_t i : nodes[pick].rows) (F[(size_t)i * NF + f] <= t ? l.rows : r.rows).push_back(i);
    nodes[pick].f = f;
    nodes[pick].t = t;
    nodes[pick].left = (int)nodes.size();
    nodes[pick].right = (int)nodes.size() + 1;
    nodes.push_back(std::move(l));
    nodes.push_back(std::move(r));
    cand.push_back(tr.best_split(nodes[nodes.size() - 2].rows));
    cand.push_back(tr.best_split(nodes[nodes.size() - 1].rows));
    leaves.erase(std::find(leaves.begin(), leaves.end(), pick));
    leaves.push_back((int)nodes.size() - 2);
    leaves.push_back((int)nodes.size() - 1);
  }
  pre.clear();
  std::vector<int> stack(1, 0);
  while (!stack.empty()) {
    const int i = stack.back();
    stack.pop_back();
    if (nodes[i].f < 0) { pre.push_back(i); continue; }
    stack.push_back(nodes[i].right);
    stack.push_back(nodes[i].left);
  }
  return KT_OK;
}

}  // namespace

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_prune_tree_leaves(kt_handle hh, const kt_shape* shapes, const uint16_t* Xq, int32_t n,
                               int32_t d, int32_t k, int32_t* labels, int32_t* n_leaves) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!labels || !n_leaves) return fail(h, KT_EINVAL, "NULL argument");
  std::vector<Node> nodes;
  std::vector<int> pre;
  kt_status st = grow_tree(h, shapes, Xq, n, d, k, nodes, pre);
  if (st != KT_OK) return st;
  for (size_t pos = 0; pos < pre.size(); ++pos)
    for (int32_t i : nodes[pre[pos]].rows) labels[i] = (int32_t)pos;
  *n_leaves = (int32_t)pre.size();
  return KT_OK;
}

kt_status kt_prune_tree(kt_handle hh, const kt_shape* shapes, const uint16_t* Xq, int32_t n,
                        int32_t d, int32_t k, int32_t* chosen) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!chosen) return fail(h, KT_EINVAL, "NULL argument");
  std::vector<Node> nodes;
  std::vector<int> pre;
  kt_status st = grow_tree(h, shapes, Xq, n, d, k, nodes, pre);
  if (st != KT_OK) return st;
  // leaves in pre-order, each picks its rounded-mean argmax (distinct)
  std::vector<char> used(d, 0);
  int32_t m = 0;
  std::vector<int64_t> s(d);
  for (int leaf : pre) {
    const std::vector<int32_t>& rows = nodes[leaf].rows;
    const int64_t nr = (int64_t)rows.size();
    std::fill(s.begin(), s.end(), 0);
    for (int32_t i : rows)
      for (int32_t j = 0; j < d; ++j) s[j] += Xq[(size_t)i * d + j];
    int best = -1;
    int64_t bv = 0;
    for (int32_t j = 0; j < d; ++j) {
      if (used[j]) continue;
      const int64_t mj = (2 * s[j] + nr) / (2 * nr);
      if (best < 0 || mj > bv) { best = j; bv = mj; }
    }
    used[best] = 1;
    chosen[m++] = best;
  }
  if (m < k) {   // too few leaves: the largest column sums over all rows
    std::fill(s.begin(), s.end(), 0);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = 0; j < d; ++j) s[j] += Xq[(size_t)i * d + j];
    while (m < k) {
      int best = -1;
      for (int32_t j = 0; j < d; ++j)
        if (!used[j] && (best < 0 || s[j] > s[best])) best = j;
      used[best] = 1;
      chosen[m++] = best;
    }
  }
  return KT_OK;
}

}  // extern "C"
