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
// The block-sparse pattern is described full (both triangles, CSR with columns
// ascending in each row and the diagonal block included), while the device
// stores the values of the symmetric matrix once: the diagonal block of every
// vertex and one block per edge (see the half storage below).
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

  // Sliced-ELL form of the full pattern walked by the matrix product: rows in
  // groups of 64 (kSell), group g using gslots[g] = its longest row.  Storage is
  // slot-major: slot s of group g is block row (s * n_groups + g), s < smax (the
  // longest row of the mesh), so that wavefronts walking their groups' slots in
  // step read neighbouring memory.  The order of a row's slots fixes the
  // product's accumulation order.  Matrices whose stored values exceed
  // kDistanceOrderBytes hold each row's blocks by distance |j - i| (the
  // diagonal first; j = i - d before j = i + d): the two reads of a stored
  // block, by its owner row and transposed by its partner row, then fall at
  // about the same slot of the concurrently running rows and meet in the L2.
  // Smaller matrices, which stay in the cache anyway, keep the CSR order
  // (columns ascending).  Per (slot s,
  // group g, lane l), at (s * n_groups + g) * 64 + l: the column (sell_col) and
  // the reference of the block's values (sell_ref).  Slots past a row's end
  // hold column = the row itself and refer to a block of zeros; slots past a
  // group's end are never read.
  int32_t n_groups = 0;
  int32_t smax = 0;
  int64_t n_slots = 0;              // smax * n_groups block rows of 64
  std::vector<int32_t> gslots;      // [n_groups]
  std::vector<int32_t> sell_col;    // [n_slots * 64]
  std::vector<int32_t> sell_ref;    // [n_slots * 64]

  // Half storage of the values.  Row i owns its diagonal block and its upper
  // blocks (i, j), j > i: 1 + (upper count) blocks, kept in a sliced-ELL layout
  // of their own, slot-major over "half slots" (hslots per group = its longest
  // owned list, hsmax over the mesh); owned block k of row i = 64 g + l sits at
  // position (k * n_groups + g) * 64 + l, and its values at value_index(position,
  // entry) (device.h): a wavefront's lanes at the same slot read neighbouring
  // positions wherever their rows share a neighbour pattern (the interior of
  // a grid).  A lower
  // block (i, j), j < i, refers to the position of (j, i) in row j with
  // kRefTranspose set: its values are read transposed.  One extra half row of
  // 64 zero blocks (position zero_pos) serves the padding slots.
  bool by_distance = false;         // slot order: by distance, else CSR
  int32_t hsmax = 0;
  int64_t n_hslots = 0;             // hsmax * n_groups half rows of 64, plus the zero row
  int32_t zero_pos = 0;             // position of a zero block
  // References: a half position, with kRefTranspose set for a lower block.
  std::vector<int32_t> csr_ref;     // [NB] reference of each CSR block
  std::vector<int32_t> diag_pos;    // [N] half position of each diagonal block
  std::vector<int32_t> edge_pos;    // [E] half position of each edge block (lo, hi)
};

// Set in a reference when the block is read transposed (it is stored as the
// upper block of the column's row).
constexpr int32_t kRefTranspose = int32_t(0x80000000u);
constexpr int32_t kRefPosMask = 0x7fffffff;

constexpr int kSell = 64;  // rows per sliced-ELL group (one wavefront)

// Stored FP64 matrix values above which the slots are ordered by distance
// (measured on the 1.57M-tet cube, 158 MB: 55.5 against 62.0 us per FP64
// product with the CSR order).
constexpr int64_t kDistanceOrderBytes = int64_t(64) << 20;

// Slot order requested from build_topology: chosen from the size, or forced.
constexpr int kSlotOrderAuto = -1, kSlotOrderCsr = 0, kSlotOrderDistance = 1;

// Builds the topology from tets [T][4] (AoS, 0-based).  Returns false and sets
// err when an index is out of range, an element repeats a vertex, a vertex
// belongs to no element, or the mesh exceeds the 32-bit index limits.
bool build_topology(int32_t n_verts, int32_t n_tets, const int32_t* tets, Topology& out,
                    std::string& err, int slot_order = kSlotOrderAuto);

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
