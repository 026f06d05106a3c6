// Host-side cluster tree, admissibility lists and sampling (compiled with
// -ffp-contract=off so the geometry follows the stated operation order).
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace h2 {

int num_levels(int64_t n, int leaf) {
  int L = 0;
  while ((n + (int64_t(1) << L) - 1) / (int64_t(1) << L) > leaf) ++L;
  return L;
}

void build_tree(const double* X, int64_t n, int dim, int leaf, double eta, Tree& t) {
  t.n = n;
  t.dim = dim;
  t.L = num_levels(n, leaf);
  t.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) t.perm[i] = i;
  t.start.assign(t.L + 1, {});
  t.start[0] = {0, n};
  std::vector<int64_t> tmp;
  for (int l = 0; l < t.L; ++l) {
    const auto& st = t.start[l];
    std::vector<int64_t> nx;
    nx.reserve(((size_t)1 << (l + 1)) + 1);
    nx.push_back(0);
    for (size_t b = 0; b + 1 < st.size(); ++b) {
      const int64_t s = st[b], e = st[b + 1];
      double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int64_t q = s; q < e; ++q)
        for (int a = 0; a < dim; ++a) {
          const double v = X[t.perm[q] * dim + a];
          mn[a] = std::min(mn[a], v);
          mx[a] = std::max(mx[a], v);
        }
      int axis = 0;
      double best = mx[0] - mn[0];
      for (int a = 1; a < dim; ++a)
        if (mx[a] - mn[a] > best) { best = mx[a] - mn[a]; axis = a; }
      std::stable_sort(t.perm.begin() + s, t.perm.begin() + e, [&](int64_t p, int64_t q) {
        return X[p * dim + axis] < X[q * dim + axis];
      });
      const int64_t h = (e - s) / 2;
      nx.push_back(s + h);
      nx.push_back(e);
    }
    t.start[l + 1] = std::move(nx);
  }
  // geometry of every box from all of its points
  t.center.assign(t.L + 1, {});
  t.extent.assign(t.L + 1, {});
  t.radius.assign(t.L + 1, {});
  for (int l = 0; l <= t.L; ++l) {
    const int nb = 1 << l;
    t.center[l].assign((size_t)nb * dim, 0.0);
    t.extent[l].assign((size_t)nb * dim, 0.0);
    t.radius[l].assign(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
      double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int64_t q = t.start[l][b]; q < t.start[l][b + 1]; ++q)
        for (int a = 0; a < dim; ++a) {
          const double v = X[t.perm[q] * dim + a];
          mn[a] = std::min(mn[a], v);
          mx[a] = std::max(mx[a], v);
        }
      double s2 = 0.0;
      for (int a = 0; a < dim; ++a) {
        t.center[l][(size_t)b * dim + a] = 0.5 * (mx[a] + mn[a]);
        const double dg = mx[a] - mn[a];
        t.extent[l][(size_t)b * dim + a] = dg;
        s2 += dg * dg;
      }
      t.radius[l][b] = 0.5 * std::sqrt(s2);
    }
  }
  // near / far lists
  t.near.assign(t.L + 1, {});
  t.far.assign(t.L + 1, {});
  t.near[0] = {{0, 0}};
  for (int l = 1; l <= t.L; ++l) {
    auto& nr = t.near[l];
    auto& fr = t.far[l];
    const auto& c = t.center[l];
    const auto& r = t.radius[l];
    for (const auto& IJ : t.near[l - 1]) {
      for (int a = 2 * IJ.first; a <= 2 * IJ.first + 1; ++a)
        for (int b = 2 * IJ.second; b <= 2 * IJ.second + 1; ++b) {
          if (a == b) { nr.push_back({a, b}); continue; }
          double s2 = 0.0;
          for (int q = 0; q < dim; ++q) {
            const double df = c[(size_t)a * dim + q] - c[(size_t)b * dim + q];
            s2 += df * df;
          }
          const double dist = std::sqrt(s2);
          if (dist > eta * (r[a] + r[b])) fr.push_back({a, b});
          else nr.push_back({a, b});
        }
    }
    std::sort(nr.begin(), nr.end());
    std::sort(fr.begin(), fr.end());
  }
}

void sample_level(const std::vector<std::vector<int64_t>>& B,
                  const std::vector<std::vector<int>>& near_of, const int64_t* rank,
                  int64_t id_base, int s_far, int s_near, std::vector<std::vector<int64_t>>& SF,
                  std::vector<std::vector<int64_t>>& SC, int nthreads) {
  const int nb = (int)B.size();
  SF.assign(nb, {});
  SC.assign(nb, {});
  // all active points of the level in pi order, with their box
  std::vector<std::pair<int64_t, int>> order;  // (rank, box) with id recoverable below
  std::vector<int64_t> ids;
  size_t tot = 0;
  for (int i = 0; i < nb; ++i) tot += B[i].size();
  std::vector<std::pair<int64_t, int64_t>> rk;  // (rank, id)
  std::vector<int> owner_of;
  rk.reserve(tot);
  std::vector<int> box_of;
  box_of.reserve(tot);
  for (int i = 0; i < nb; ++i)
    for (int64_t id : B[i]) rk.push_back({rank[id - id_base], id});
  // owner box per id through a parallel array sorted alongside
  std::vector<size_t> idx(tot);
  {
    size_t q = 0;
    for (int i = 0; i < nb; ++i)
      for (size_t u = 0; u < B[i].size(); ++u) { box_of.push_back(i); idx[q] = q; ++q; }
  }
  std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return rk[a].first < rk[b].first; });
  std::vector<int64_t> sorted_id(tot);
  std::vector<int> sorted_box(tot);
  for (size_t q = 0; q < tot; ++q) {
    sorted_id[q] = rk[idx[q]].second;
    sorted_box[q] = box_of[idx[q]];
  }
  auto work = [&](int i0, int i1) {
    std::vector<char> isnear(nb, 0);
    for (int i = i0; i < i1; ++i) {
      for (int j : near_of[i]) isnear[j] = 1;
      // far: walk pi order
      auto& sf = SF[i];
      for (size_t q = 0; q < tot; ++q) {
        if (s_far >= 0 && (int)sf.size() >= s_far) break;
        if (!isnear[sorted_box[q]]) sf.push_back(sorted_id[q]);
      }
      // near: candidates of near boxes j != i, ordered by rank
      std::vector<std::pair<int64_t, int64_t>> cand;
      for (int j : near_of[i])
        if (j != i)
          for (int64_t id : B[j]) cand.push_back({rank[id - id_base], id});
      std::sort(cand.begin(), cand.end());
      auto& sc = SC[i];
      const size_t take = s_near < 0 ? cand.size() : std::min(cand.size(), (size_t)s_near);
      for (size_t q = 0; q < take; ++q) sc.push_back(cand[q].second);
      for (int j : near_of[i]) isnear[j] = 0;
    }
  };
  if (nthreads < 1) nthreads = 1;
  if (nthreads > nb) nthreads = nb;
  std::vector<std::thread> th;
  const int per = (nb + nthreads - 1) / nthreads;
  for (int w = 0; w < nthreads; ++w) {
    const int a = w * per, b = std::min(nb, a + per);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto& x : th) x.join();
}

}  // namespace h2
