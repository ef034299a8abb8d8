// Atomic-free block-sparse assembly, incremental re-gather, residual-based
// selection with ballot/prefix-sum compaction, and small reductions.
//
// Assembly (Sec. 3): every block of H and every vertex entry of g is the sum
// of its contiguous slot range, in ascending element order, plus the per-vertex
// inertia m_i/h^2 and Dirichlet-penalty k_D terms.  Projecting an element
// overwrites its slots with Hhat^e, and re-summing the touched blocks applies
// Delta H^e = Hhat^e - H^e in place without changing the sparsity (Sec. 4.1,
// Eq. (5)); the result does not depend on the order of the updates.
//
// Selection (Algorithm 1): element e is projected when
// |S^e g|_inf = max over its 4 vertices of max_c |g_(i,c)| exceeds delta, or
// when delta <= eps_delta (fallback to PN).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "k_common.h"
#include "topology.h"

namespace ppn {

// Diagonal block of vertex i from the summed element part hd (upper 6) plus
// (m_i/h^2 + k_D [i in D]) I; also its inverse for block-Jacobi and the
// Sylvester test (leading principal minors > 0).
__device__ inline void store_diag(const Dev& D, int i, const double hd[6]) {
  const double di = D.mass[i] / (D.h * D.h) + (D.dir_idx[i] >= 0 ? D.k_dir : 0.0);
  const double a00 = hd[0] + di, a01 = hd[1], a02 = hd[2];
  const double a11 = hd[3] + di, a12 = hd[4], a22 = hd[5] + di;
  const int32_t pb = D.diag_blk[i];
  const double a[9] = {a00, a01, a02, a01, a11, a12, a02, a12, a22};
#pragma unroll
  for (int e = 0; e < 9; ++e) D.vals[value_index(pb, e)] = a[e];
  const double c00 = a11 * a22 - a12 * a12;
  const double c01 = a02 * a12 - a01 * a22;
  const double c02 = a01 * a12 - a02 * a11;
  const double c11 = a00 * a22 - a02 * a02;
  const double c12 = a01 * a02 - a00 * a12;
  const double c22 = a00 * a11 - a01 * a01;
  const double det = a00 * c00 + a01 * c01 + a02 * c02;
  const bool ok = (a00 > 0.0) && (c22 > 0.0) && (det > 0.0);
  const double id = ok ? 1.0 / det : 0.0;
  const int N = D.N;
  D.pinv[0 * N + i] = c00 * id;
  D.pinv[1 * N + i] = c01 * id;
  D.pinv[2 * N + i] = c02 * id;
  D.pinv[3 * N + i] = c11 * id;
  D.pinv[4 * N + i] = c12 * id;
  D.pinv[5 * N + i] = c22 * id;
  D.spd_ok[i] = ok ? 1 : 0;
}

// One edge block (lo, hi) from the edge's slots (the matrix stores it once;
// the product reads it transposed for row hi).
__device__ inline void gather_edge(const Dev& D, int k) {
  double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = D.eptr[k]; t < D.eptr[k + 1]; ++t) {
    const double* sl = D.eslots + size_t(t) * 9;
#pragma unroll
    for (int c = 0; c < 9; ++c) s[c] += sl[c];
  }
  const int32_t pu = D.eblk_up[k];
#pragma unroll
  for (int c = 0; c < 9; ++c) D.vals[value_index(pu, c)] = s[c];
}

// Vertex pass of the full assembly: gradient, |g_i|_inf, diagonal block,
// block-Jacobi inverse, and partial |g|_2^2 and |g|_inf per workgroup.
//
// The slot sums are component-parallel: thread (v, c) of a chunk of
// kVChunk vertices sums component c of vertex v's slots, so the threads of a
// wavefront read consecutive doubles of the contiguous slot range of their
// vertices (instead of one lane streaming a vertex's ~1.7 KB range alone);
// each component is summed in ascending slot order as before.  The sums meet
// in LDS and one thread per vertex finishes it.
constexpr int kVChunk = kBlock / 9;  // 28 vertices (252 threads) per chunk

__device__ __forceinline__ void assemble_vertex_body(const Dev& D, int b) {
  __shared__ double lds[16];
  __shared__ double sv[kVChunk][9];
  const int G = D.G;
  const int w = xcd_chunk(b, G);
  const int i0 = w * D.rows_per_wg, i1 = min(D.N, i0 + D.rows_per_wg);
  const double ih2 = 1.0 / (D.h * D.h);
  const int t = threadIdx.x, vl = t / 9, c = t % 9;
  double g2 = 0.0, gm = 0.0;
  for (int base = i0; base < i1; base += kVChunk) {
    const int i = base + vl;
    if (vl < kVChunk && i < i1) {
      double s = 0.0;
#pragma unroll 8
      for (int k = D.vptr[i]; k < D.vptr[i + 1]; ++k) s += D.vslots[size_t(k) * 9 + c];
      sv[vl][c] = s;
    }
    __syncthreads();
    if (t < kVChunk && base + t < i1) {
      const int iv = base + t;
      const double* sl = sv[t];
      const int di = D.dir_idx[iv];
      double gi[3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const double xi = D.x[3 * iv + cc];
        double tt = sl[cc] + D.mass[iv] * ih2 * (xi - D.xhat[3 * iv + cc]);
        if (di >= 0) tt += D.k_dir * (xi - D.xbar[3 * di + cc]);
        gi[cc] = tt;
        D.g[3 * iv + cc] = tt;
      }
      const double r = fmax(fabs(gi[0]), fmax(fabs(gi[1]), fabs(gi[2])));
      D.rinf[iv] = r;
      g2 += gi[0] * gi[0] + gi[1] * gi[1] + gi[2] * gi[2];
      gm = fmax(gm, r);
      double hd[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) hd[q] = sl[3 + q];
      store_diag(D, iv, hd);
    }
    __syncthreads();
  }
  g2 = block_sum(g2, lds);
  gm = block_max(gm, lds);
  if (threadIdx.x == 0) {
    D.part[kPartG2 * G + w] = g2;
    D.part[kPartGmax * G + w] = gm;
  }
}

// Edge pass: off-diagonal block (lo, hi), stored once.  Like
// the vertex pass it is component-parallel: thread (k, c) of a workgroup's
// kEChunk edges sums entry c of edge k's slots in ascending slot order (the
// order of gather_edge, so the same bits) and stores it.  The
// threads of a wavefront read consecutive doubles of their edges' contiguous
// slot range, where one lane per edge would walk its own 72-byte records and
// fetch each cache line several times.  One chunk per workgroup, mapped so
// that each XCD owns a contiguous range of edges: the chunks in flight on an
// XCD are one narrow window, whose scattered block writes fill whole lines
// while they are in that XCD's L2.
constexpr int kEBlock = 1024;
constexpr int kEChunk = kEBlock / 9;  // 113 edges (1017 threads) per workgroup
// Edge-pass workgroups of a scene: a multiple of 8 (the extra ones exit at once).
__host__ __device__ inline int eval_wgs_edge_dev(const Dev& D) {
  return D.E > 0 ? int(((int64_t(D.E) + kEChunk - 1) / kEChunk + 7) / 8 * 8) : 0;
}
__device__ __forceinline__ void assemble_edge_body(const Dev& D, int b, int n_wg) {
  const int vl = threadIdx.x / 9, c = threadIdx.x % 9;
  const int64_t k = int64_t(xcd_chunk(b, n_wg)) * kEChunk + vl;
  if (vl >= kEChunk || k >= D.E) return;
  double s = 0.0;
#pragma unroll 4
  for (int t = D.eptr[k]; t < D.eptr[k + 1]; ++t) s += D.eslots[size_t(t) * 9 + c];
  D.vals[value_index(D.eblk_up[k], c)] = s;
}

__global__ __launch_bounds__(kBlock) void k_assemble_vertex(const EvalJob* __restrict__ jobs, int n) {
  int w;
  const EvalJob& J = eval_job<1>(jobs, n, w);
  assemble_vertex_body(J.D, w);
}

__global__ __launch_bounds__(kEBlock) void k_assemble_edge(const EvalJob* __restrict__ jobs, int n) {
  int w;
  const EvalJob& J = eval_job<2>(jobs, n, w);
  assemble_edge_body(J.D, w, eval_wgs_edge_dev(J.D));
}

// Re-gather the 10 blocks of each listed (just projected) element.  Blocks
// shared by several listed elements are recomputed by each of them from the
// same slots in the same order, so the duplicate stores write identical bits.
__global__ __launch_bounds__(kBlock) void k_regather(Dev D, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= 10 * n) return;
  const int e = D.list[t / 10];
  const int j = t % 10;
  if (j < 4) {
    const int i = D.tets[j * D.T + e];
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int k = D.vptr[i]; k < D.vptr[i + 1]; ++k) {
      const double* sl = D.vslots + size_t(k) * 9 + 3;
#pragma unroll
      for (int c = 0; c < 6; ++c) s[c] += sl[c];
    }
    store_diag(D, i, s);
  } else {
    gather_edge(D, D.elem_edge[(j - 4) * D.T + e]);
  }
}

void launch_regather_list(const Dev& D, int32_t n, hipStream_t st) {
  if (n <= 0) return;
  k_regather<<<(10 * n + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, n);
}

// ---------------------------------------------------------------- selection + compaction
__device__ inline bool selected(const Dev& D, int e, double delta, int fallback) {
  if (D.proj[e]) return false;
  if (fallback) return true;
  const int T = D.T;
  double s = D.rinf[D.tets[e]];
  s = fmax(s, D.rinf[D.tets[T + e]]);
  s = fmax(s, D.rinf[D.tets[2 * T + e]]);
  s = fmax(s, D.rinf[D.tets[3 * T + e]]);
  return s > delta;
}

__global__ __launch_bounds__(kBlock) void k_select_count(Dev D, double delta, int fallback) {
  static_assert(kBlock == 4 * 64, "k_select_count adds the counts of exactly four wavefronts");
  __shared__ int cnt[kBlock / 64];
  const int e = blockIdx.x * kBlock + threadIdx.x;
  const bool p = (e < D.T) && selected(D, e, delta, fallback);
  if (e < D.T) D.sel[e] = p ? 1 : 0;
  const unsigned long long m = __ballot(p);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) D.sel_cnt[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// Exclusive scan of the per-workgroup counts in one workgroup of 1024 threads;
// the total lands in sel_cnt[n].
__global__ __launch_bounds__(1024) void k_select_scan(Dev D) {
  __shared__ int part[1024];
  const int n = D.n_sel_wg;
  const int per = (n + 1023) / 1024;
  const int b0 = threadIdx.x * per, b1 = min(n, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += D.sel_cnt[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;  // exclusive prefix of this thread's range
  for (int b = b0; b < b1; ++b) {
    const int c = D.sel_cnt[b];
    D.sel_cnt[b] = run;
    run += c;
  }
  if (threadIdx.x == 1023) D.sel_cnt[n] = part[1023];
}

__global__ __launch_bounds__(kBlock) void k_select_write(Dev D) {
  __shared__ int woff[kBlock / 64];
  const int e = blockIdx.x * kBlock + threadIdx.x;
  const bool p = (e < D.T) && D.sel[e];
  const unsigned long long m = __ballot(p);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) woff[wv] = __popcll(m);
  __syncthreads();
  int base = D.sel_cnt[blockIdx.x];
  for (int k = 0; k < wv; ++k) base += woff[k];
  if (p) {
    const unsigned long long below = lane ? (m & ((~0ull) >> (64 - lane))) : 0ull;
    D.list[base + __popcll(below)] = e;
    D.proj[e] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_rinf_from(Dev D, const double* g) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= D.N) return;
  D.rinf[i] = fmax(fabs(g[3 * i]), fmax(fabs(g[3 * i + 1]), fabs(g[3 * i + 2])));
}

void launch_rinf_from(const Dev& D, const double* g, hipStream_t st) {
  k_rinf_from<<<(D.N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, g);
}

void launch_select_count(const Dev& D, double delta, int fallback, hipStream_t st) {
  k_select_count<<<D.n_sel_wg, kBlock, 0, st>>>(D, delta, fallback);
  k_select_scan<<<1, 1024, 0, st>>>(D);
}

void launch_select_write(const Dev& D, hipStream_t st) {
  k_select_write<<<D.n_sel_wg, kBlock, 0, st>>>(D);
}

// ---------------------------------------------------------------- reductions and fills
// Reduce partial slots [first, first + n_sum) as sums and the next n_max as
// maxima into scal[0 .. n_sum + n_max).
__global__ __launch_bounds__(kBlock) void k_reduce(Dev D, int first, int n_sum, int n_max, int G) {
  __shared__ double lds[16];
  for (int k = 0; k < n_sum + n_max; ++k) {
    const double* p = D.part + size_t(first + k) * G;
    double v;
    if (k < n_sum) {
      double s = 0.0;
      for (int i = threadIdx.x; i < G; i += kBlock) s += p[i];
      v = block_sum(s, lds);
    } else {
      double s = 0.0;
      for (int i = threadIdx.x; i < G; i += kBlock) s = fmax(s, p[i]);
      v = block_max(s, lds);
    }
    if (threadIdx.x == 0) D.scal[k] = v;
  }
}

void launch_reduce(const Dev& D, int first_slot, int n_sum, int n_max, hipStream_t st) {
  k_reduce<<<1, kBlock, 0, st>>>(D, first_slot, n_sum, n_max, D.G);
}

// k_reduce for every job of a table: workgroup k reduces job k's partials
// (written with its G workgroups) into its scal.
__global__ __launch_bounds__(kBlock) void k_reduce_jobs(const EvalJob* __restrict__ jobs, int first,
                                                        int n_sum, int n_max) {
  __shared__ double lds[16];
  const Dev& D = jobs[blockIdx.x].D;
  const int G = D.G;
  for (int k = 0; k < n_sum + n_max; ++k) {
    const double* p = D.part + size_t(first + k) * G;
    double v;
    if (k < n_sum) {
      double s = 0.0;
      for (int i = threadIdx.x; i < G; i += kBlock) s += p[i];
      v = block_sum(s, lds);
    } else {
      double s = 0.0;
      for (int i = threadIdx.x; i < G; i += kBlock) s = fmax(s, p[i]);
      v = block_max(s, lds);
    }
    if (threadIdx.x == 0) D.scal[k] = v;
  }
}

void launch_reduce_jobs(const EvalJob* jobs, int n, int first_slot, int n_sum, int n_max, hipStream_t st) {
  if (n > 0) k_reduce_jobs<<<n, kBlock, 0, st>>>(jobs, first_slot, n_sum, n_max);
}

int eval_wgs_vert(const Dev& D) { return D.G; }
int eval_wgs_edge(const Dev& D) { return eval_wgs_edge_dev(D); }

EvalGrid layout_eval_jobs(EvalJob* jobs, int n) {
  EvalGrid g;
  for (int k = 0; k < n; ++k) {
    EvalJob& j = jobs[k];
    j.wg_elem = g.elem;
    j.wg_vert = g.vert;
    j.wg_edge = g.edge;
    j.wg_ls = g.ls;
    g.elem += eval_wgs_elem(j.D);
    g.vert += eval_wgs_vert(j.D);
    g.edge += eval_wgs_edge(j.D);
    g.ls += eval_wgs_ls(j.D);
  }
  return g;
}

void launch_assemble_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st) {
  if (n <= 0) return;
  k_assemble_vertex<<<gr.vert, kBlock, 0, st>>>(jobs, n);
  if (gr.edge > 0) k_assemble_edge<<<gr.edge, kEBlock, 0, st>>>(jobs, n);
}

void launch_evaluate_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st) {
  if (n <= 0) return;
  launch_elem_jobs(jobs, n, gr, st);
  launch_assemble_jobs(jobs, n, gr, st);
  launch_reduce_jobs(jobs, n, kPartG2, 1, 1, st);
}

void launch_reduce_pcg(const Dev& D, int first_slot, int n_sum, hipStream_t st) {
  k_reduce<<<1, kBlock, 0, st>>>(D, first_slot, n_sum, 0, D.Gp);
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < n) p[k] = v;
}

void launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_u8<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(p, v, n);
}

// |dx|_inf and g.dx -> scal[0] (sum g.dx), scal[1] (max |dx|)
__global__ __launch_bounds__(kBlock) void k_dx_stats(Dev D) {
  __shared__ double lds[16];
  const int G = D.G;
  const int w = logical_wg(G);
  const int i0 = w * D.rows_per_wg, i1 = min(D.N, i0 + D.rows_per_wg);
  double gd = 0.0, mx = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double d = D.dx[3 * i + c];
      gd += D.g[3 * i + c] * d;
      mx = fmax(mx, fabs(d));
    }
  }
  gd = block_sum(gd, lds);
  mx = block_max(mx, lds);
  if (threadIdx.x == 0) {
    D.part[kPartA * G + w] = gd;
    D.part[(kPartA + 1) * G + w] = mx;
  }
}

void launch_dx_stats(const Dev& D, hipStream_t st) {
  k_dx_stats<<<D.G, kBlock, 0, st>>>(D);
  launch_reduce(D, kPartA, 1, 1, st);
}

// dx = -P^-1 g (block-Jacobi direction), used when a solve stays indefinite
// with every element projected and the last PCG iterate is zero.
__global__ __launch_bounds__(kBlock) void k_safety_dir(Dev D) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= D.N) return;
  const int N = D.N;
  const double g0 = D.g[3 * i], g1 = D.g[3 * i + 1], g2 = D.g[3 * i + 2];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    D.dx[3 * i + r] = -(D.pinv[kSym3[r][0] * N + i] * g0 + D.pinv[kSym3[r][1] * N + i] * g1 +
                        D.pinv[kSym3[r][2] * N + i] * g2);
}

void launch_safety_dir(const Dev& D, hipStream_t st) {
  k_safety_dir<<<(D.N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D);
}

}  // namespace ppn
