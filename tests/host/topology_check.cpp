// Host-side check of the sparsity and scatter-map construction (build_topology):
// random meshes and degenerate inputs, the block pattern, slot maps and
// sliced-ELL positions against brute force.  Built and run by
// tests/test_host_topology.py, with AddressSanitizer where available.
#include <cstdio>
#include <random>
#include <set>
#include <algorithm>
#include <cstdlib>
#include "topology.h"
#include "wg_order.h"
using namespace ppn;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)
static void check_mesh(int N, const std::vector<int32_t>& tets, int order = kSlotOrderAuto) {
  Topology t; std::string err;
  const int T = int(tets.size() / 4);
  bool ok = build_topology(N, T, tets.data(), t, err, order);
  if (ok && order != kSlotOrderAuto) CHECK(t.by_distance == (order == kSlotOrderDistance));
  if (ok && order == kSlotOrderAuto) CHECK(!t.by_distance);  // small meshes keep the CSR order
  // brute force
  std::vector<int> used(N, 0);
  bool valid = T > 0 && N > 0;
  for (int e = 0; e < T && valid; ++e)
    for (int a = 0; a < 4; ++a) {
      int v = tets[4 * e + a];
      if (v < 0 || v >= N) { valid = false; break; }
      for (int b = 0; b < a; ++b) if (tets[4 * e + b] == v) valid = false;
      used[v] = 1;
    }
  if (valid) for (int i = 0; i < N; ++i) if (!used[i]) valid = false;
  CHECK(ok == valid);
  if (!ok) return;
  std::set<std::pair<int, int>> blocks;
  for (int e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) blocks.insert({tets[4 * e + a], tets[4 * e + b]});
  CHECK(t.n_blocks == int64_t(blocks.size()));
  for (int i = 0; i < N; ++i)
    for (int k = t.row_ptr[i]; k < t.row_ptr[i + 1]; ++k) {
      CHECK(blocks.count({i, t.col[k]}));
      if (k > t.row_ptr[i]) CHECK(t.col[k] > t.col[k - 1]);
    }
  for (int i = 0; i < N; ++i) CHECK(t.col[t.diag_blk[i]] == i);
  // Half storage: a symmetric matrix with distinct entries, block (i, j) =
  // B(i, j), B(j, i) = B(i, j)^T, written once through diag_pos / edge_pos
  // (the positions the assembly writes) and read back through every
  // reference, full sliced-ELL slots and CSR blocks alike.
  auto entry = [](int i, int j, int r, int c) {  // entry (r, c) of B(i, j), symmetric overall
    const int a = 3 * i + r, b = 3 * j + c;
    return double(std::min(a, b)) * 100003.0 + double(std::max(a, b)) + 1.0;
  };
  const int64_t npos = t.n_hslots * kSell;
  CHECK(t.zero_pos == int32_t(npos - kSell));
  std::vector<double> half(size_t(npos) * 9, 0.0);
  std::vector<int> owner(size_t(npos), 0);
  for (int i = 0; i < N; ++i) {
    const int32_t p = t.diag_pos[i];
    CHECK(p >= 0 && p < t.zero_pos && owner[p]++ == 0);
    for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) half[size_t(p) * 9 + 3 * r + c] = entry(i, i, r, c);
  }
  for (int k = 0; k < t.n_edges; ++k) {
    const int32_t p = t.edge_pos[k];
    CHECK(p >= 0 && p < t.zero_pos && owner[p]++ == 0);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) half[size_t(p) * 9 + 3 * r + c] = entry(t.edge_lo[k], t.edge_hi[k], r, c);
  }
  auto read = [&](int32_t ref, int r, int c) {
    const int32_t p = ref & kRefPosMask;
    return ref < 0 ? half[size_t(p) * 9 + 3 * c + r] : half[size_t(p) * 9 + 3 * r + c];
  };
  for (int i = 0; i < N; ++i)
    for (int k = t.row_ptr[i]; k < t.row_ptr[i + 1]; ++k) {
      const int j = t.col[k];
      CHECK((t.csr_ref[k] < 0) == (j < i));
      for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) CHECK(read(t.csr_ref[k], r, c) == entry(i, j, r, c));
    }
  CHECK(t.n_slots == int64_t(t.smax) * t.n_groups);
  for (int i = 0; i < N; ++i) {
    const int g = i / kSell, l = i % kSell, len = t.row_ptr[i + 1] - t.row_ptr[i];
    CHECK(len <= t.gslots[g]);
    std::set<int> seen;
    for (int s = 0; s < t.smax; ++s) {
      const size_t at = (size_t(s) * t.n_groups + g) * kSell + l;
      const int j = t.sell_col[at];
      const int32_t ref = t.sell_ref[at];
      if (s >= len) {  // padding: the row itself and the zero block
        CHECK(j == i && ref == t.zero_pos);
        continue;
      }
      CHECK(blocks.count({i, j}) && seen.insert(j).second);
      for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) CHECK(read(ref, r, c) == entry(i, j, r, c));
      if (t.by_distance) {
        // blocks by distance |j - i|, the lower one first at equal distance
        if (s > 0) {
          const int jp = t.sell_col[(size_t(s - 1) * t.n_groups + g) * kSell + l];
          const int d = std::abs(j - i), dp = std::abs(jp - i);
          CHECK(dp < d || (dp == d && jp < j));
        }
      } else {
        CHECK(j == t.col[t.row_ptr[i] + s]);  // CSR order
      }
    }
    CHECK(int(seen.size()) == len);
  }
  for (size_t k = size_t(t.zero_pos) * 9; k < half.size(); ++k) CHECK(half[k] == 0.0);
  // every slot maps back to its element
  for (int e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a) CHECK(t.vslot_elem[t.vslot[size_t(a) * T + e]] == e);
  for (int e = 0; e < T; ++e)
    for (int p = 0; p < 6; ++p) {
      const int k = t.elem_edge[size_t(p) * T + e];
      int va = tets[4 * e + kPairA[p]], vc = tets[4 * e + kPairC[p]];
      CHECK(t.edge_lo[k] == std::min(va, vc) && t.edge_hi[k] == std::max(va, vc));
      const int s = t.eslot[size_t(p) * T + e];
      CHECK(s >= t.eptr[k] && s < t.eptr[k + 1]);
    }
}
int main() {
  std::mt19937 rng(1);
  for (int trial = 0; trial < 300; ++trial) {
    const int N = 4 + int(rng() % 200), T = 1 + int(rng() % 400);
    std::vector<int32_t> tets(4 * size_t(T));
    for (int e = 0; e < T; ++e) {
      std::vector<int> v(N); for (int i = 0; i < N; ++i) v[i] = i;
      for (int a = 0; a < 4; ++a) { std::swap(v[a], v[a + rng() % (N - a)]); tets[4 * e + a] = v[a]; }
    }
    if (trial % 7 == 1) tets[rng() % tets.size()] = N + int(rng() % 5);          // out of range
    if (trial % 7 == 2) tets[rng() % tets.size()] = -1;
    if (trial % 7 == 3) { size_t e = rng() % T; tets[4 * e + 1] = tets[4 * e]; }  // repeated vertex
    // ensure coverage of all vertices in most trials
    if (trial % 7 != 4) {
      std::vector<int> used(N, 0);
      for (int32_t v : tets) if (v >= 0 && v < N) used[v] = 1;
      for (int i = 0; i < N; ++i) if (!used[i]) { tets.push_back(i); tets.push_back((i + 1) % N); tets.push_back((i + 2) % N); tets.push_back((i + 3) % N); }
    }
    check_mesh(N, tets, trial % 3 == 0 ? kSlotOrderAuto : trial % 3 == 1 ? kSlotOrderCsr : kSlotOrderDistance);
  }
  // the product's panel order is a bijection of every XCD chunk
  for (int C = 1; C <= 300; ++C)
    for (int P = -1; P <= C + 2; ++P) {
      std::vector<int> hit(C, 0);
      for (int k = 0; k < C; ++k) {
        const int w = panel_order(k, C, P);
        if (w >= 0 && w < C) ++hit[w];
        else CHECK(w >= 0 && w < C);
      }
      for (int w = 0; w < C; ++w) CHECK(hit[w] == 1);
    }
  Topology t; std::string err;
  CHECK(!build_topology(0, 1, nullptr, t, err));
  int32_t one[4] = {0, 1, 2, 3};
  check_mesh(4, std::vector<int32_t>(one, one + 4));
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
