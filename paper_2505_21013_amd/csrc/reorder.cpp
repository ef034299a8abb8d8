// Locality orderings of a tetrahedral mesh (see topology.h).
//
// Two vertex orders, both deterministic functions of the mesh (ties keep the
// input order):
//  * pencil: the axes ranked by the mesh's extent along them, longest first
//    (ties by axis index); rest coordinates along the first two rounded to
//    multiples of the mesh spacing h (the 10th percentile of the edge
//    lengths, over a fixed-stride sample of at most 2^20 elements); vertices sorted by those two and then by the exact coordinate
//    along the shortest axis.  Neighbours then lie within one slab across the
//    longest axis, the narrowest band a sweep can give, in runs of ids along
//    the shortest one, which keeps the column gathers of the matrix product
//    on whole cache lines.  On a regular grid with spacing h this is a
//    lexicographic numbering, shortest axis fastest.
//  * Morton: the Z-order curve of the rest positions, each coordinate
//    quantised to 21 bits over the bounding box and the bit strings
//    interleaved into one 63-bit key (Morton, IBM technical report, 1966).
//    It adapts to graded meshes, at the cost of longer jumps between runs.
// Elements follow their vertices: sorted by their four new vertex ids in
// ascending order, compared lexicographically.
#include "topology.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

namespace ppn {
namespace {

// Spreads the low 21 bits of v so that bit i lands on bit 3i.
uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x001f00000000ffffULL;
  v = (v | (v << 16)) & 0x001f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

struct Quantiser {
  double lo[3], scale[3];
  uint64_t key(const double p[3]) const {
    uint64_t k = 0;
    for (int c = 0; c < 3; ++c) {
      double q = std::floor((p[c] - lo[c]) * scale[c]);
      q = std::min(std::max(q, 0.0), double((1 << 21) - 1));
      k |= spread3(uint64_t(q)) << c;
    }
    return k;
  }
};

}  // namespace

bool locality_order(int32_t N, const double* X, int32_t T, const int32_t* tets, int32_t kind,
                    int32_t* vertex_order, int32_t* tet_order, std::string& err) {
  if (N <= 0 || T <= 0) {
    err = "empty mesh";
    return false;
  }
  if (kind != kOrderPencil && kind != kOrderMorton) {
    err = "unknown ordering kind " + std::to_string(kind);
    return false;
  }
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) {
    lo[c] = INFINITY;
    hi[c] = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
      double x = X[3 * i + c];
      if (!std::isfinite(x)) {
        err = "rest position of vertex " + std::to_string(i) + " is not finite";
        return false;
      }
      lo[c] = std::min(lo[c], x);
      hi[c] = std::max(hi[c], x);
    }
  }
  for (int64_t e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a) {
      int32_t v = tets[4 * e + a];
      if (v < 0 || v >= N) {
        err = "tet " + std::to_string(e) + " has vertex index " + std::to_string(v) +
              " outside [0, " + std::to_string(N) + ")";
        return false;
      }
    }

  std::iota(vertex_order, vertex_order + N, 0);
  if (kind == kOrderMorton) {
    Quantiser qz;
    for (int c = 0; c < 3; ++c) {
      qz.lo[c] = lo[c];
      // A flat extent (all coordinates equal) quantises to 0.
      qz.scale[c] = hi[c] > lo[c] ? double(1 << 21) / (hi[c] - lo[c]) : 0.0;
    }
    std::vector<uint64_t> key(N);
    for (int64_t i = 0; i < N; ++i) key[i] = qz.key(X + 3 * i);
    std::stable_sort(vertex_order, vertex_order + N,
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  } else {
    // Mesh spacing: the 10th percentile of the element edge lengths (every
    // edge counted once per element that holds it), over at most 2^20
    // elements taken at a fixed stride.
    const int64_t ns = std::min<int64_t>(T, int64_t(1) << 20);
    std::vector<double> len(ns * 6);
    for (int64_t k = 0; k < ns; ++k) {
      const int64_t e = k * T / ns;
      for (int p = 0; p < 6; ++p) {
        const double* a = X + 3 * int64_t(tets[4 * e + kPairA[p]]);
        const double* b = X + 3 * int64_t(tets[4 * e + kPairC[p]]);
        len[6 * k + p] = std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                                   (a[2] - b[2]) * (a[2] - b[2]));
      }
    }
    auto nth = len.begin() + len.size() / 10;
    std::nth_element(len.begin(), nth, len.end());
    double h = *nth;
    double extent = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    if (!(h > 0.0)) h = extent > 0.0 ? extent / std::cbrt(double(N)) : 1.0;
    // Rounded coordinates stay below 2^40 (far inside int64) whatever the edges.
    h = std::max(h, extent * 0x1p-40);
    int ax[3] = {0, 1, 2};
    std::stable_sort(ax, ax + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    std::vector<int64_t> q0(N), q1(N);
    for (int64_t i = 0; i < N; ++i) {
      q0[i] = std::llround((X[3 * i + ax[0]] - lo[ax[0]]) / h);
      q1[i] = std::llround((X[3 * i + ax[1]] - lo[ax[1]]) / h);
    }
    std::stable_sort(vertex_order, vertex_order + N, [&](int32_t a, int32_t b) {
      if (q0[a] != q0[b]) return q0[a] < q0[b];
      if (q1[a] != q1[b]) return q1[a] < q1[b];
      return X[3 * int64_t(a) + ax[2]] < X[3 * int64_t(b) + ax[2]];
    });
  }

  std::vector<int32_t> new_of_old(N);
  for (int32_t i = 0; i < N; ++i) new_of_old[vertex_order[i]] = i;
  std::vector<std::array<int32_t, 4>> key(T);
  for (int64_t e = 0; e < T; ++e) {
    for (int a = 0; a < 4; ++a) key[e][a] = new_of_old[tets[4 * e + a]];
    std::sort(key[e].begin(), key[e].end());
  }
  std::iota(tet_order, tet_order + T, 0);
  std::stable_sort(tet_order, tet_order + T, [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  return true;
}

}  // namespace ppn
