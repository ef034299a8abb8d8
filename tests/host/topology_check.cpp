// Host-side check of the sparsity and scatter-map construction (build_topology):
// random meshes and degenerate inputs, the block pattern, slot maps and
// sliced-ELL positions against brute force.  Built and run by
// tests/test_host_topology.py, with AddressSanitizer where available.
#include <cstdio>
#include <random>
#include <set>
#include <algorithm>
#include "topology.h"
using namespace ppn;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)
static void check_mesh(int N, const std::vector<int32_t>& tets) {
  Topology t; std::string err;
  const int T = int(tets.size() / 4);
  bool ok = build_topology(N, T, tets.data(), t, err);
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
      // sliced-ELL position holds the same column
      const int32_t pos = t.csr_base[k];
      CHECK(t.sell_col[size_t(pos)] == t.col[k]);
    }
  for (int i = 0; i < N; ++i) CHECK(t.col[t.diag_blk[i]] == i);
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
    check_mesh(N, tets);
  }
  Topology t; std::string err;
  CHECK(!build_topology(0, 1, nullptr, t, err));
  int32_t one[4] = {0, 1, 2, 3};
  check_mesh(4, std::vector<int32_t>(one, one + 4));
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
