// Device helpers shared by the kernels: deterministic workgroup reductions and
// the XCD-aware mapping from workgroup index to a contiguous chunk of rows.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"
#include "wg_order.h"

namespace ppn {

#define PPN_HOST_DEVICE __host__ __device__

// Sum over the 64 lanes of a wavefront; the xor butterfly fixes the order.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the workgroup (up to 16 wavefronts), returned to every thread; the
// order is fixed by the workgroup size.  lds: 16 doubles.
__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = lds[0];
  for (int k = 1; k < nw; ++k) s += lds[k];
  return s;
}

// Sums of two values over the workgroup, each in block_sum's order (so with
// the same bits), for one barrier round instead of two; lds: 16 doubles (up
// to 8 wavefronts).
__device__ inline void block_sum2(double& a, double& b, double* lds) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    lds[w] = a;
    lds[8 + w] = b;
  }
  __syncthreads();
  double sa = lds[0], sb = lds[8];
  for (int k = 1; k < nw; ++k) {
    sa += lds[k];
    sb += lds[8 + k];
  }
  a = sa;
  b = sb;
}

__device__ inline double block_max(double v, double* lds) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = lds[0];
  for (int k = 1; k < nw; ++k) s = fmax(s, lds[k]);
  return s;
}

// Reduce G per-workgroup partials in a fixed order (every workgroup that calls
// this gets bit-identical results).
__device__ inline double reduce_partials(const double* p, int G, double* lds) {
  double s = 0.0;
  for (int i = threadIdx.x; i < G; i += blockDim.x) s += p[i];
  return block_sum(s, lds);
}

// The block-Jacobi inverse of a symmetric 3x3 block is symmetric and stored as
// its upper triangle, entries (00, 01, 02, 11, 12, 22) in planes [6][N];
// kSym3[r][c] is the plane of entry (r, c).
constexpr int kSym3[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

// Workgroups are dispatched round-robin over the 8 XCDs.  Map the hardware
// index so that XCD x owns the contiguous logical chunks [x*G/8, (x+1)*G/8):
// neighbouring rows then share an L2.  Requires G % 8 == 0.
__device__ inline int xcd_chunk(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }
__device__ inline int logical_wg(int G) { return xcd_chunk(blockIdx.x, G); }

__device__ inline int logical_wg_panels(int G, int P) {
  const int b = blockIdx.x, C = G >> 3;
  return (b & 7) * C + panel_order(b >> 3, C, P);
}

// The job of a shared launch that owns this workgroup (largest range start <=
// blockIdx.x, by binary search over the table) and the workgroup's index
// within that job's range.  kField picks the kernel's range: 0 element, 1
// vertex, 2 edge, 3 line search.
template <int kField>
__device__ inline int eval_range_start(const EvalJob& j) {
  return kField == 0 ? j.wg_elem : kField == 1 ? j.wg_vert : kField == 2 ? j.wg_edge : j.wg_ls;
}
template <int kField>
__device__ inline const EvalJob& eval_job(const EvalJob* __restrict__ jobs, int n, int& w) {
  const int b = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (eval_range_start<kField>(jobs[mid]) <= b) lo = mid; else hi = mid - 1;
  }
  w = b - eval_range_start<kField>(jobs[lo]);
  return jobs[lo];
}

}  // namespace ppn
