// C entry points over the library's host-side cluster tree and sampling
// (csrc/tree.cpp), for comparing them with the oracle's on the CPU through
// ctypes.  One tree and one sample selection are kept between calls; the
// accessors copy them out.  Not thread-safe (a test helper).
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../paper_2502_02395_amd/csrc/tree.hpp"

namespace {
h2::Tree g_tree;
std::vector<std::vector<int64_t>> g_sf, g_sc;
}  // namespace

extern "C" {

// Builds the tree of X (n x dim, row-major) on nthreads threads; returns its
// number of levels L.
int tc_build(const double* X, int64_t n, int dim, int leaf, double eta, int nthreads) {
  g_tree = h2::Tree();
  h2::build_tree(X, n, dim, leaf, eta, g_tree, nthreads);
  return g_tree.L;
}

void tc_perm(int64_t* out) { std::memcpy(out, g_tree.perm.data(), g_tree.perm.size() * 8); }

// start: 2^l + 1 entries; center, extent: 2^l x dim; radius: 2^l
void tc_level(int l, int64_t* start, double* center, double* extent, double* radius) {
  std::memcpy(start, g_tree.start[l].data(), g_tree.start[l].size() * 8);
  std::memcpy(center, g_tree.center[l].data(), g_tree.center[l].size() * 8);
  std::memcpy(extent, g_tree.extent[l].data(), g_tree.extent[l].size() * 8);
  std::memcpy(radius, g_tree.radius[l].data(), g_tree.radius[l].size() * 8);
}

int64_t tc_npairs(int l, int far) {
  return (int64_t)(far ? g_tree.far[l] : g_tree.near[l]).size();
}

// pairs as (i, j) rows
void tc_pairs(int l, int far, int32_t* out) {
  const auto& v = far ? g_tree.far[l] : g_tree.near[l];
  for (size_t q = 0; q < v.size(); ++q) {
    out[2 * q] = v[q].first;
    out[2 * q + 1] = v[q].second;
  }
}

// sample_level on flattened inputs: box i's active ids are
// ids[ids_off[i] .. ids_off[i + 1]), its near boxes near[near_off[i] ..
// near_off[i + 1]); rank[id - id_base] is the id's position in pi.
void tc_sample(int nb, const int64_t* ids, const int64_t* ids_off, const int32_t* near,
               const int64_t* near_off, const int64_t* rank, int64_t id_base, int s_far,
               int s_near, int nthreads) {
  std::vector<std::vector<int64_t>> B(nb);
  std::vector<std::vector<int>> near_of(nb);
  for (int i = 0; i < nb; ++i) {
    B[i].assign(ids + ids_off[i], ids + ids_off[i + 1]);
    near_of[i].assign(near + near_off[i], near + near_off[i + 1]);
  }
  h2::sample_level(B, near_of, rank, id_base, s_far, s_near, g_sf, g_sc, nthreads);
}

int64_t tc_sample_size(int box, int near) {
  return (int64_t)(near ? g_sc[box] : g_sf[box]).size();
}

void tc_sample_get(int box, int near, int64_t* out) {
  const auto& v = near ? g_sc[box] : g_sf[box];
  std::memcpy(out, v.data(), v.size() * 8);
}

}  // extern "C"
