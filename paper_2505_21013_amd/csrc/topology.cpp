// Host-side sparsity and scatter-map construction (see topology.h).
#include "topology.h"

#include <algorithm>
#include <cstdlib>
#include <numeric>

namespace ppn {

bool build_topology(int32_t N, int32_t T, const int32_t* tets, Topology& t, std::string& err,
                    int slot_order) {
  if (N <= 0 || T <= 0) {
    err = "empty mesh";
    return false;
  }
  for (int64_t e = 0; e < T; ++e) {
    for (int a = 0; a < 4; ++a) {
      int32_t v = tets[4 * e + a];
      if (v < 0 || v >= N) {
        err = "tet " + std::to_string(e) + " has vertex index " + std::to_string(v) +
              " outside [0, " + std::to_string(N) + ")";
        return false;
      }
      for (int b = 0; b < a; ++b)
        if (tets[4 * e + b] == v) {
          err = "tet " + std::to_string(e) + " repeats vertex " + std::to_string(v);
          return false;
        }
    }
  }
  // Per-element arrays are indexed [k][T] with k < 9 in 32-bit arithmetic.
  if (int64_t(T) * 9 >= (int64_t(1) << 31)) {
    err = "too many elements for 32-bit element indices (at most 238,609,294)";
    return false;
  }
  t.n_verts = N;
  t.n_tets = T;

  // ---- vertex slots: counting sort of (element, corner) by vertex, stable in element order
  t.vptr.assign(N + 1, 0);
  for (int64_t e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a) t.vptr[tets[4 * e + a] + 1]++;
  // A vertex outside every element has no mass and no stiffness: its diagonal
  // block is singular and would leave every Newton system indefinite.
  for (int32_t i = 0; i < N; ++i)
    if (t.vptr[i + 1] == 0) {
      err = "vertex " + std::to_string(i) + " belongs to no tetrahedron";
      return false;
    }
  for (int32_t i = 0; i < N; ++i) t.vptr[i + 1] += t.vptr[i];
  std::vector<int32_t> fill(t.vptr.begin(), t.vptr.end() - 1);
  t.vslot.resize(4 * size_t(T));
  t.vslot_elem.resize(4 * size_t(T));
  for (int64_t e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a) {
      int32_t s = fill[tets[4 * e + a]]++;
      t.vslot[size_t(a) * T + e] = s;
      t.vslot_elem[s] = int32_t(e);
    }

  // ---- edge records (lo, hi, element, pair) bucketed by lo, then sorted by (hi, element)
  std::vector<int32_t> lo_ptr(N + 1, 0);
  for (int64_t e = 0; e < T; ++e)
    for (int p = 0; p < 6; ++p) {
      int32_t va = tets[4 * e + kPairA[p]], vc = tets[4 * e + kPairC[p]];
      lo_ptr[std::min(va, vc) + 1]++;
    }
  for (int32_t i = 0; i < N; ++i) lo_ptr[i + 1] += lo_ptr[i];
  const int64_t R = int64_t(6) * T;
  std::vector<int64_t> rec(R);  // key: hi << 32 | (element*6 + pair); element-major inside hi
  std::vector<int32_t> rfill(lo_ptr.begin(), lo_ptr.end() - 1);
  for (int64_t e = 0; e < T; ++e)
    for (int p = 0; p < 6; ++p) {
      int32_t va = tets[4 * e + kPairA[p]], vc = tets[4 * e + kPairC[p]];
      int32_t lo = std::min(va, vc), hi = std::max(va, vc);
      rec[rfill[lo]++] = (int64_t(hi) << 32) | int64_t(e * 6 + p);
    }
  t.eptr.clear();
  t.eptr.reserve(size_t(R / 4));
  t.edge_lo.clear();
  t.edge_hi.clear();
  t.eslot.resize(6 * size_t(T));
  t.elem_edge.resize(6 * size_t(T));
  for (int32_t lo = 0; lo < N; ++lo) {
    auto b = rec.begin() + lo_ptr[lo], en = rec.begin() + lo_ptr[lo + 1];
    std::sort(b, en);
    int32_t prev_hi = -1;
    for (int64_t r = lo_ptr[lo]; r < lo_ptr[lo + 1]; ++r) {
      int32_t hi = int32_t(rec[r] >> 32);
      int32_t ep = int32_t(rec[r] & 0xffffffff);
      if (hi != prev_hi) {
        t.eptr.push_back(int32_t(r));
        t.edge_lo.push_back(lo);
        t.edge_hi.push_back(hi);
        prev_hi = hi;
      }
      int32_t e = ep / 6, p = ep % 6;
      t.eslot[size_t(p) * T + e] = int32_t(r);
      t.elem_edge[size_t(p) * T + e] = int32_t(t.edge_lo.size() - 1);
    }
  }
  t.n_edges = int32_t(t.edge_lo.size());
  t.eptr.push_back(int32_t(R));

  // ---- full block-sparse rows: [lower neighbours ascending] [diagonal] [upper ascending]
  const int32_t E = t.n_edges;
  std::vector<int32_t> up_cnt(N, 0), low_cnt(N, 0);
  for (int32_t k = 0; k < E; ++k) {
    up_cnt[t.edge_lo[k]]++;
    low_cnt[t.edge_hi[k]]++;
  }
  t.row_ptr.assign(N + 1, 0);
  for (int32_t i = 0; i < N; ++i) t.row_ptr[i + 1] = t.row_ptr[i] + low_cnt[i] + 1 + up_cnt[i];
  t.n_blocks = t.row_ptr[N];
  t.col.resize(size_t(t.n_blocks));
  t.diag_blk.resize(N);
  t.eblk_up.resize(E);
  t.eblk_lo.resize(E);
  // Upper part: edges are ordered by (lo, hi), so each row's upper neighbours come in order.
  std::vector<int32_t> upos(N), lpos(N);
  for (int32_t i = 0; i < N; ++i) {
    t.diag_blk[i] = t.row_ptr[i] + low_cnt[i];
    t.col[t.diag_blk[i]] = i;
    upos[i] = t.diag_blk[i] + 1;
    lpos[i] = t.row_ptr[i];
  }
  for (int32_t k = 0; k < E; ++k) {
    int32_t lo = t.edge_lo[k], hi = t.edge_hi[k];
    int32_t bu = upos[lo]++;
    t.col[bu] = hi;
    t.eblk_up[k] = bu;
    // Lower part of row hi: edges with this hi arrive in ascending lo because k runs in (lo, hi) order.
    int32_t bl = lpos[hi]++;
    t.col[bl] = lo;
    t.eblk_lo[k] = bl;
  }

  // ---- half storage: each row owns [diagonal][upper blocks ascending]
  t.n_groups = (N + kSell - 1) / kSell;
  std::vector<int32_t> hslots(t.n_groups, 0);
  for (int32_t i = 0; i < N; ++i) hslots[i / kSell] = std::max(hslots[i / kSell], 1 + up_cnt[i]);
  t.hsmax = *std::max_element(hslots.begin(), hslots.end());
  t.n_hslots = int64_t(t.hsmax) * t.n_groups + 1;  // + one row of zero blocks
  if (t.n_hslots * kSell >= (int64_t(1) << 31)) {
    err = "matrix too large for 31-bit block positions";
    return false;
  }
  t.zero_pos = int32_t((t.n_hslots - 1) * kSell);
  auto hpos = [&](int32_t i, int32_t k) {  // half position of owned block k of row i
    return int32_t((int64_t(k) * t.n_groups + i / kSell) * kSell + i % kSell);
  };
  t.diag_pos.resize(N);
  for (int32_t i = 0; i < N; ++i) t.diag_pos[i] = hpos(i, 0);
  t.edge_pos.resize(E);
  t.csr_ref.resize(size_t(t.n_blocks));
  for (int32_t i = 0; i < N; ++i) t.csr_ref[t.diag_blk[i]] = t.diag_pos[i];
  for (int32_t k = 0; k < E; ++k) {
    const int32_t lo = t.edge_lo[k];
    // owned block index: 1 + rank of this edge among lo's upper edges (column order)
    const int32_t kk = 1 + (t.eblk_up[k] - t.diag_blk[lo] - 1);
    t.edge_pos[k] = hpos(lo, kk);
    t.csr_ref[t.eblk_up[k]] = t.edge_pos[k];
    t.csr_ref[t.eblk_lo[k]] = t.edge_pos[k] | kRefTranspose;
  }

  // ---- sliced-ELL form of the full pattern, slot-major, each row's blocks in
  // CSR order or by distance |j - i| (see topology.h)
  t.by_distance = slot_order == kSlotOrderAuto
                      ? t.n_hslots * kSell * 9 * int64_t(sizeof(double)) > kDistanceOrderBytes
                      : slot_order == kSlotOrderDistance;
  t.gslots.assign(t.n_groups, 0);
  for (int32_t i = 0; i < N; ++i)
    t.gslots[i / kSell] = std::max(t.gslots[i / kSell], t.row_ptr[i + 1] - t.row_ptr[i]);
  t.smax = *std::max_element(t.gslots.begin(), t.gslots.end());
  t.n_slots = int64_t(t.smax) * t.n_groups;
  if (t.n_slots * kSell >= (int64_t(1) << 31)) {
    err = "matrix too large for 32-bit sliced-ELL block positions";
    return false;
  }
  t.sell_col.assign(size_t(t.n_slots) * kSell, 0);
  t.sell_ref.assign(size_t(t.n_slots) * kSell, t.zero_pos);
  std::vector<int32_t> ord;
  for (int32_t g = 0; g < t.n_groups; ++g)
    for (int32_t l = 0; l < kSell; ++l) {
      const int32_t i = g * kSell + l;
      if (i >= N) continue;
      const int32_t len = t.row_ptr[i + 1] - t.row_ptr[i];
      ord.resize(len);
      for (int32_t q = 0; q < len; ++q) ord[q] = t.row_ptr[i] + q;
      if (t.by_distance)
        std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
          const int64_t da = std::abs(int64_t(t.col[a]) - i), db = std::abs(int64_t(t.col[b]) - i);
          return da < db || (da == db && t.col[a] < t.col[b]);
        });
      for (int32_t s = 0; s < t.smax; ++s) {
        const int64_t at = (int64_t(s) * t.n_groups + g) * kSell + l;
        int32_t c = i, ref = t.zero_pos;
        if (s < len) {
          const int32_t k = ord[s];
          c = t.col[k];
          ref = t.csr_ref[k];
        }
        t.sell_col[size_t(at)] = c;
        t.sell_ref[size_t(at)] = ref;
      }
    }
  return true;
}

}  // namespace ppn
