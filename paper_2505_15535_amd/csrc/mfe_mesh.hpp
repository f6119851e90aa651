// Host-side numbering of the Q_p nodes of a general hexahedral mesh.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace mfe {

// Canonical node numbering of a degree-p mesh of ne hexahedra over nv
// vertices, cell e listing its vertices ev[8e..8e+7] in lexicographic local
// order (local vertex bx + 2 by + 4 bz at reference corner (bx, by, bz)):
// vertices first (node v = vertex v), then p-1 nodes per edge (edges sorted
// by their (lower, higher) vertex ids, nodes counted from the lower end), then
// (p-1)^2 per face (faces sorted by their ascending vertex ids, node
// (s-1) + (p-1)(t-1) with s counted from the face's lowest vertex towards the
// lower-id of its two edge neighbours on the face, t towards the other), then
// (p-1)^3 interior nodes per cell in local lexicographic order.
// On success fills conn[e*(p+1)^3 + a] (a = i + (p+1)(j + (p+1)k)) and
// n_nodes and returns ""; otherwise returns what is wrong with the mesh (ids
// out of range, a repeated vertex, a face shared by more than two cells or by
// two cells that disagree on its edges).
std::string number_hex_nodes(int64_t nv, int64_t ne, const int32_t* ev, int p, std::vector<int32_t>& conn,
                             int64_t& n_nodes);

// perm[k] = the cell processed k-th: cells sorted (stably) by the Morton
// code of their centroids (21 bits per axis over the vertices' bounding
// box), so that consecutive cells are close in space.
void morton_order(int64_t nv, const double* xyz, int64_t ne, const int32_t* ev, std::vector<int32_t>& perm);

}  // namespace mfe
