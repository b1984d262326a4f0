// rn_partition.h -- host-side heuristic recursive bisection (Section 3).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace rn {

// Recursive bisection of the graph (arcs taken as undirected edges) by
// Algorithm 1 with the smoothing of Equations (1)-(2).  part[x] receives the
// leaf id of x (leaves numbered in a left-to-right walk of the recursion) and
// order lists the vertices leaf by leaf (ascending ids inside a leaf).
// Returns false (with msg) only when memory runs out.
bool partition_graph(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                     float alpha, int32_t max_leaf, std::vector<int32_t> &part,
                     std::vector<int32_t> &order, std::string &msg);

}  // namespace rn
