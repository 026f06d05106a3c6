// Host-side cluster tree and block lists (plain C++, no HIP).
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

namespace h2 {

// Binary cluster tree of one point set: level l has 2^l boxes, box i covers
// the contiguous tree positions [start[l][i], start[l][i+1]).  Children of box
// i are 2i and 2i+1.  Points are split at the median of the longest axis of
// the box's bounding box (left child takes floor(n/2)).
struct Tree {
  int64_t n = 0;
  int dim = 3;
  int L = 0;
  std::vector<int64_t> perm;                    // tree position -> local point index
  std::vector<std::vector<int64_t>> start;      // per level, 2^l + 1 entries
  std::vector<std::vector<double>> center;      // per level, 2^l * dim
  std::vector<std::vector<double>> extent;      // per level, 2^l * dim (bbox sides)
  std::vector<std::vector<double>> radius;      // per level, 2^l
  // ordered pairs per level, both orientations, sorted lexicographically
  std::vector<std::vector<std::pair<int, int>>> near, far;
};

int num_levels(int64_t n, int leaf);

// Far iff ||c_a - c_b||_2 > eta (rho_a + rho_b), evaluated in this order in
// double precision; only children of near pairs are tested.  X must be finite
// (dim <= 3).  nthreads: threads for the boxes of a level (the result does
// not depend on it).
void build_tree(const double* X, int64_t n, int dim, int leaf, double eta, Tree& t,
                int nthreads = 1);

// Sample selection of one level of one instance (Algorithm 1, Sample()):
// for each box i, S_F = the s_far active points of non-near boxes that come
// first in pi order, S_C = the s_near active points of near boxes j != i that
// come first in pi order (negative size: all of them).  Active points are
// given per box as ids; rank[id - id_base] is the position of a point in pi
// (distinct points, distinct positions).
void sample_level(const std::vector<std::vector<int64_t>>& B,
                  const std::vector<std::vector<int>>& near_of,
                  const int64_t* rank, int64_t id_base, int s_far, int s_near,
                  std::vector<std::vector<int64_t>>& SF,
                  std::vector<std::vector<int64_t>>& SC, int nthreads);

}  // namespace h2
