// Device kd-tree layout and builder interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace gs {

// Node arrays in breadth-first numbering; boxes and centres are [node][D].
struct DevTree {
  int64_t capacity = 0, n_nodes = 0, n_points = 0;
  int D = 0;
  int32_t *begin = nullptr, *count = nullptr, *left = nullptr, *depth = nullptr;
  int32_t* parent = nullptr;       // -1 at the root
  int32_t *perm = nullptr;         // [n_points] original index at each position
  int32_t *leaf_of_pos = nullptr;  // [n_points] leaf containing each position
  double *lo = nullptr, *hi = nullptr, *ctr = nullptr;
  double *rinf = nullptr, *W = nullptr, *wmin = nullptr;
  double* rad = nullptr;           // Euclidean radius about ctr (sphere-rectangle bounds)
  const int32_t* perm_list = nullptr;
  std::vector<int> level_begin;    // host: first node of each level, then n_nodes
  std::vector<int> level_max;      // host: most points in a node of each level
};

struct TreeBuildArgs {
  int64_t n = 0;
  int D = 0;
  int leaf_size = 64;
  const double* xs = nullptr;  // [D][n]
  const double* w = nullptr;   // [n] or nullptr (unit weights)
  int32_t *ids = nullptr, *lists = nullptr, *lists_alt = nullptr;  // ids [n], lists [(D+1) n]
  int32_t *pos_node = nullptr, *pos_node_alt = nullptr, *isleft = nullptr;  // [n]
  int32_t *flags = nullptr, *scan = nullptr;                             // [(D+1) n]
  int32_t *splitdim = nullptr;                                           // [capacity]
  double* sort_keys = nullptr;                                           // [n]
  int32_t* host_topo = nullptr;  // pinned host memory, 5 * capacity: the node topology
  void* temp = nullptr;
  size_t temp_bytes = 0;
};

int64_t tree_node_capacity(int64_t n, int leaf_size);
// Node counts follow from n and leaf_size alone (the split rule takes whole
// leaves), so the topology -- begin, count, left, depth of every node and the
// level boundaries -- is computed on the host; the device only sorts points.
size_t tree_sort_temp_bytes(int64_t n, int D);
// rad[i] = sqrt(max over node i's points of sum_d (x_d - ctr_d)^2), the
// squares summed in d order; x_perm: [n_points][D] in tree order.
hipError_t launch_node_radius(const DevTree& t, int64_t n_nodes, const double* x_perm, int D,
                              hipStream_t s);

hipError_t build_tree_device(const TreeBuildArgs& a, DevTree& t, std::vector<int>& level_begin,
                             hipStream_t s);

}  // namespace gs
