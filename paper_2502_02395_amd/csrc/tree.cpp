// Host-side cluster tree, admissibility lists and sampling (compiled with
// -ffp-contract=off so the geometry follows the stated operation order).
#include "tree.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

namespace h2 {

int num_levels(int64_t n, int leaf) {
  int L = 0;
  while ((n + (int64_t(1) << L) - 1) / (int64_t(1) << L) > leaf) ++L;
  return L;
}

namespace {

// fn(i, w) for i in [0, count) on up to nthreads threads (w: the thread's index)
template <class F>
void parallel_for(int count, int nthreads, F fn) {
  const int nt = std::max(1, std::min(nthreads, count));
  if (nt == 1) {
    for (int i = 0; i < count; ++i) fn(i, 0);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w]() {
      for (int i; (i = next.fetch_add(1)) < count;) fn(i, w);
    });
  for (auto& x : th) x.join();
}

// Sorts distinct keys on up to nthreads threads: runs sorted in parallel,
// then merged pairwise (distinct keys have one sorted order).
template <class K>
void sort_distinct(std::vector<K>& k, int nthreads) {
  const int T = std::max(1, std::min(nthreads, (int)(k.size() / 32768)));
  if (T == 1) {
    std::sort(k.begin(), k.end());
    return;
  }
  std::vector<size_t> bnd(T + 1);
  for (int i = 0; i <= T; ++i) bnd[i] = k.size() * i / T;
  parallel_for(T, T, [&](int i, int) { std::sort(k.begin() + bnd[i], k.begin() + bnd[i + 1]); });
  for (int w = 1; w < T; w *= 2) {
    const int jobs = (T + 2 * w - 1) / (2 * w);
    parallel_for(jobs, T, [&](int j, int) {
      const int a = 2 * w * j, m = std::min(a + w, T), e = std::min(a + 2 * w, T);
      if (m < e) std::inplace_merge(k.begin() + bnd[a], k.begin() + bnd[m], k.begin() + bnd[e]);
    });
  }
}

}  // namespace

// Every level sorts each box's points along the longest axis of its bounding
// box.  The points travel with their coordinates (a copy in tree order, so
// every scan is contiguous); a box sorts (coordinate, position) keys, whose
// order is the one a stable sort by coordinate gives, since positions are
// unique; the boxes of a level are spread over threads (a level with fewer
// boxes than threads sorts each box on its share of them).  Geometry: a leaf's
// bounding box from its points, a parent's from its children's (min and max
// are exact, so each is the bounding box of the box's points).
void build_tree(const double* X, int64_t n, int dim, int leaf, double eta, Tree& t,
                int nthreads) {
  t.n = n;
  t.dim = dim;
  t.L = num_levels(n, leaf);
  t.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) t.perm[i] = i;
  std::vector<double> Xp(X, X + n * dim);
  t.start.assign(t.L + 1, {});
  t.start[0] = {0, n};
  struct Scratch {
    std::vector<std::pair<double, int64_t>> key;
    std::vector<double> x;
    std::vector<int64_t> p;
  };
  std::vector<Scratch> scr(std::max(1, nthreads));
  for (int l = 0; l < t.L; ++l) {
    const std::vector<int64_t>& st = t.start[l];
    const int nb = 1 << l;
    std::vector<int64_t> nx((size_t)2 * nb + 1, 0);
    const int inner = std::max(1, nthreads / nb);  // threads per box for its sort
    parallel_for(nb, nthreads, [&](int b, int w) {
      Scratch& sc = scr[w];
      const int64_t s = st[b], e = st[b + 1], m = e - s;
      double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int64_t q = s; q < e; ++q)
        for (int a = 0; a < dim; ++a) {
          const double v = Xp[q * dim + a];
          mn[a] = std::min(mn[a], v);
          mx[a] = std::max(mx[a], v);
        }
      int axis = 0;
      double best = mx[0] - mn[0];
      for (int a = 1; a < dim; ++a)
        if (mx[a] - mn[a] > best) { best = mx[a] - mn[a]; axis = a; }
      sc.key.resize(m);
      for (int64_t q = 0; q < m; ++q) sc.key[q] = {Xp[(s + q) * dim + axis], q};
      sort_distinct(sc.key, inner);
      sc.x.resize(m * dim);
      sc.p.resize(m);
      for (int64_t q = 0; q < m; ++q) {
        const int64_t src = s + sc.key[q].second;
        sc.p[q] = t.perm[src];
        for (int a = 0; a < dim; ++a) sc.x[q * dim + a] = Xp[src * dim + a];
      }
      std::copy(sc.p.begin(), sc.p.end(), t.perm.begin() + s);
      std::copy(sc.x.begin(), sc.x.end(), Xp.begin() + s * dim);
      nx[2 * b + 1] = s + m / 2;  // the left child takes floor(m / 2)
      nx[2 * b + 2] = e;
    });
    t.start[l + 1] = std::move(nx);
  }
  // geometry of every box
  t.center.assign(t.L + 1, {});
  t.extent.assign(t.L + 1, {});
  t.radius.assign(t.L + 1, {});
  std::vector<double> bmn((size_t)dim << t.L), bmx((size_t)dim << t.L);
  parallel_for(1 << t.L, nthreads, [&](int b, int) {
    for (int a = 0; a < dim; ++a) {
      bmn[(size_t)b * dim + a] = INFINITY;
      bmx[(size_t)b * dim + a] = -INFINITY;
    }
    for (int64_t q = t.start[t.L][b]; q < t.start[t.L][b + 1]; ++q)
      for (int a = 0; a < dim; ++a) {
        const double v = Xp[q * dim + a];
        bmn[(size_t)b * dim + a] = std::min(bmn[(size_t)b * dim + a], v);
        bmx[(size_t)b * dim + a] = std::max(bmx[(size_t)b * dim + a], v);
      }
  });
  for (int l = t.L; l >= 0; --l) {
    const int nb = 1 << l;
    if (l < t.L)  // children 2b, 2b + 1 of level l + 1 into box b
      for (int b = 0; b < nb; ++b)
        for (int a = 0; a < dim; ++a) {
          bmn[(size_t)b * dim + a] =
              std::min(bmn[(size_t)(2 * b) * dim + a], bmn[(size_t)(2 * b + 1) * dim + a]);
          bmx[(size_t)b * dim + a] =
              std::max(bmx[(size_t)(2 * b) * dim + a], bmx[(size_t)(2 * b + 1) * dim + a]);
        }
    t.center[l].assign((size_t)nb * dim, 0.0);
    t.extent[l].assign((size_t)nb * dim, 0.0);
    t.radius[l].assign(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
      double s2 = 0.0;
      for (int a = 0; a < dim; ++a) {
        const double mx = bmx[(size_t)b * dim + a], mn = bmn[(size_t)b * dim + a];
        t.center[l][(size_t)b * dim + a] = 0.5 * (mx + mn);
        const double dg = mx - mn;
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
  // all active points of the level in pi order, with their box: one slot
  // per position in pi (positions of distinct points are distinct)
  size_t tot = 0;
  int64_t rmax = -1;
  for (int i = 0; i < nb; ++i) {
    tot += B[i].size();
    for (int64_t id : B[i]) rmax = std::max(rmax, rank[id - id_base]);
  }
  std::vector<int> slot_box((size_t)(rmax + 1), -1);
  std::vector<int64_t> slot_id((size_t)(rmax + 1));
  for (int i = 0; i < nb; ++i)
    for (int64_t id : B[i]) {
      const int64_t r = rank[id - id_base];
      slot_box[r] = i;
      slot_id[r] = id;
    }
  std::vector<int64_t> sorted_id;
  std::vector<int> sorted_box;
  sorted_id.reserve(tot);
  sorted_box.reserve(tot);
  for (int64_t r = 0; r <= rmax; ++r)
    if (slot_box[r] >= 0) {
      sorted_id.push_back(slot_id[r]);
      sorted_box.push_back(slot_box[r]);
    }
  tot = sorted_id.size();
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
      // the first `take` in pi order (ranks are unique: the prefix of the
      // full sort)
      auto& sc = SC[i];
      const size_t take = s_near < 0 ? cand.size() : std::min(cand.size(), (size_t)s_near);
      std::partial_sort(cand.begin(), cand.begin() + take, cand.end());
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
