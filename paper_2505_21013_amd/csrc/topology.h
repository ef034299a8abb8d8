// Host-side sparsity and scatter-map construction for the tetrahedral mesh.
//
// The global Hessian H = sum_e H^e (Sec. 3) has one 3x3 block per vertex
// pair that shares an element; its sparsity never changes (Sec. 4.1).  The
// element kernel writes each element's blocks into "slots" ordered by the
// block they belong to, so that assembly is a contiguous segmented sum per
// block with no atomics and a fixed summation order:
//
//  * vertex slots: one per (element, corner), grouped by vertex and, within a
//    vertex, ascending by element.  A slot holds the corner's gradient (3) and
//    its diagonal Hessian block (6, symmetric upper).
//  * edge slots: one per (element, vertex pair), grouped by the edge (lo, hi)
//    with lo < hi, ascending by element.  A slot holds the 3x3 off-diagonal
//    block H_(lo,hi) in global orientation (row = lo vertex).
//
// The block-sparse matrix is stored full (both triangles) with columns
// ascending in each row and the diagonal block included.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ppn {

// Local vertex pairs of a tetrahedron, in the order used for edge slots.
constexpr int kPairA[6] = {0, 0, 0, 1, 1, 2};
constexpr int kPairC[6] = {1, 2, 3, 2, 3, 3};

struct Topology {
  int32_t n_verts = 0, n_tets = 0, n_edges = 0;
  int64_t n_blocks = 0;
  // element -> slot maps, SoA: [corner or pair][element]
  std::vector<int32_t> vslot;      // [4][T]
  std::vector<int32_t> eslot;      // [6][T]
  std::vector<int32_t> elem_edge;  // [6][T] edge id of each pair
  // slot ranges
  std::vector<int32_t> vptr;       // [N+1]
  std::vector<int32_t> vslot_elem; // [4T] element owning each vertex slot
  std::vector<int32_t> eptr;       // [E+1]
  std::vector<int32_t> edge_lo, edge_hi;  // [E]
  // block-sparse rows
  std::vector<int32_t> row_ptr;    // [N+1]
  std::vector<int32_t> col;        // [NB]
  std::vector<int32_t> diag_blk;   // [N]
  std::vector<int32_t> eblk_up;    // [E] block (lo, hi)
  std::vector<int32_t> eblk_lo;    // [E] block (hi, lo)

  // Sliced-ELL copy of the pattern used by the device: rows in groups of 64
  // (kSell), group g using gslots[g] = its longest row.  Storage is slot-major:
  // slot s of group g is block row (s * n_groups + g), s < smax (the longest row
  // of the mesh), so that wavefronts walking their groups' slots in step read
  // neighbouring memory.  The block in (slot s, group g, lane l) has position
  // (s * n_groups + g) * 64 + l: its column is stored there and its values at
  // value_index(position, entry) (device.h).  Slots past a row's end hold column = the row
  // itself and zero values; slots past a group's end are never read.
  int32_t n_groups = 0;
  int32_t smax = 0;
  int64_t n_slots = 0;              // smax * n_groups block rows of 64
  std::vector<int32_t> gslots;      // [n_groups]
  std::vector<int32_t> sell_col;    // [n_slots * 64]
  // Block positions slot * 64 + lane (the block's values are addressed in
  // 64-bit arithmetic from the position: value_index() in device.h).
  std::vector<int32_t> csr_base;    // [NB] position of each CSR block
  std::vector<int32_t> diag_base;   // [N]
  std::vector<int32_t> eup_base;    // [E]
  std::vector<int32_t> elo_base;    // [E]
};

constexpr int kSell = 64;  // rows per sliced-ELL group (one wavefront)

// Builds the topology from tets [T][4] (AoS, 0-based).  Returns false and sets
// err when an index is out of range, an element repeats a vertex, a vertex
// belongs to no element, or the mesh exceeds the 32-bit index limits.
bool build_topology(int32_t n_verts, int32_t n_tets, const int32_t* tets, Topology& out,
                    std::string& err);

// Vertex orders of locality_order.
constexpr int32_t kOrderPencil = 0;  // banded sweep across the longest axis
constexpr int32_t kOrderMorton = 1;  // Z-order curve of the rest positions

// A numbering of the mesh with spatial locality: vertex_order[n_verts] and
// tet_order[n_tets] list the input ids in their new order (new -> old), the
// vertices in the order `kind` names, the elements by their new vertex ids.
// Returns false and sets err for an empty mesh, an unknown kind, a
// non-finite position or an index out of range.
bool locality_order(int32_t n_verts, const double* X, int32_t n_tets, const int32_t* tets,
                    int32_t kind, int32_t* vertex_order, int32_t* tet_order, std::string& err);

}  // namespace ppn
