// Block-Jacobi preconditioned CG on the 3x3 block-sparse Hessian, with the
// early exit on non-positive curvature d^T H d <= 0 that proves H indefinite
// (Sec. 4.1, Linear Solvers), zero initial guess, and |r| <= rtol |r0|.
//
// One iteration is two kernels whose control scalars stay on the device:
//   spmv   : beta from the r^T z partials, the new direction d = z + beta d_old
//            (formed on the fly for every gathered column), q = H d and
//            partials of d^T q;
//   update : alpha = r^T z / d^T q, x += alpha d, r -= alpha q, z = P^-1 r and
//            partials of r^T r and r^T z.
// Every workgroup reduces the same partials in the same order, so all of them
// take the same stop decision; workgroup 0 records it in PcgState and later
// launches return at once.  The host only polls PcgState every few iterations.
//
// SpMV mapping: 16 lanes per block row (rows have at most 15 blocks in a
// Kuhn-split grid; longer rows loop), 16 rows per 256-thread workgroup step;
// the SoA value layout makes each of the 9 value loads of a lane group one
// contiguous run.  Workgroups own contiguous row chunks, grouped per XCD.
#include <hip/hip_runtime.h>

#include "k_common.h"

namespace ppn {

__device__ inline void pcg_finish(const Dev& D, int ind, int iters) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D.pcg->ind = ind;
    D.pcg->iters = iters;
    D.pcg->done = 1;
  }
}

// r = -g, x = 0, z = P^-1 r; partials of r^T r, r^T z and the count of
// diagonal blocks failing Sylvester's criterion.
__global__ __launch_bounds__(kBlock) void k_pcg_init(Dev D) {
  __shared__ double lds[4];
  const int G = D.G, N = D.N;
  const int w = logical_wg(G);
  const int i0 = w * D.rows_per_wg, i1 = min(N, i0 + D.rows_per_wg);
  double rr = 0.0, rz = 0.0, bad = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = -D.g[3 * i + c];
      D.r[3 * i + c] = r[c];
      D.dx[3 * i + c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double zc = D.pinv[(3 * c) * N + i] * r[0] + D.pinv[(3 * c + 1) * N + i] * r[1] +
                        D.pinv[(3 * c + 2) * N + i] * r[2];
      D.z[3 * i + c] = zc;
      rz += r[c] * zc;
      rr += r[c] * r[c];
    }
    bad += D.spd_ok[i] ? 0.0 : 1.0;
  }
  rr = block_sum(rr, lds);
  rz = block_sum(rz, lds);
  bad = block_sum(bad, lds);
  if (threadIdx.x == 0) {
    D.part[kPartRR * G + w] = rr;
    D.part[kPartRZ0 * G + w] = rz;
    D.part[kPartSpd * G + w] = bad;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    D.pcg->done = 0;
    D.pcg->ind = 0;
    D.pcg->iters = 0;
  }
}

template <bool kFirst>
__global__ __launch_bounds__(kBlock) void k_pcg_spmv(Dev D, int j, double tol2, int maxit) {
  __shared__ double lds[4];
  if (D.pcg->done) return;
  const int G = D.G;
  const double* dold = (j & 1) ? D.d0 : D.d1;
  double* dnew = (j & 1) ? D.d1 : D.d0;
  double beta = 0.0;
  if (kFirst) {
    const double rr0 = reduce_partials(D.part + kPartRR * G, G, lds);
    const double rz0 = reduce_partials(D.part + kPartRZ0 * G, G, lds);
    const double bad = reduce_partials(D.part + kPartSpd * G, G, lds);
    if (bad > 0.0) { pcg_finish(D, 1, 0); return; }
    if (rr0 == 0.0) { pcg_finish(D, 0, 0); return; }
    if (rz0 <= 0.0) { pcg_finish(D, 1, 0); return; }
    if (blockIdx.x == 0 && threadIdx.x == 0) D.pcg->rr0 = rr0;
  } else {
    const double rr = reduce_partials(D.part + kPartRR * G, G, lds);
    const double rz = reduce_partials(D.part + ((j & 1) ? kPartRZ1 : kPartRZ0) * G, G, lds);
    if (rr <= tol2 * D.pcg->rr0) { pcg_finish(D, 0, j); return; }
    if (rz <= 0.0) { pcg_finish(D, 1, j); return; }
    if (j >= maxit) { pcg_finish(D, 0, j); return; }
    const double rzo = reduce_partials(D.part + ((j & 1) ? kPartRZ0 : kPartRZ1) * G, G, lds);
    beta = rz / rzo;
  }
  const int w = logical_wg(G);
  const int i0 = w * D.rows_per_wg, i1 = min(D.N, i0 + D.rows_per_wg);
  const int lane = threadIdx.x & 15;
  const int64_t NB = D.NB;
  double kap = 0.0;
  for (int ib = i0; ib < i1; ib += kBlock / 16) {
    const int i = ib + (threadIdx.x >> 4);
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    if (i < i1) {
      const int k0 = D.row_ptr[i], k1 = D.row_ptr[i + 1];
      for (int k = k0 + lane; k < k1; k += 16) {
        const int c = D.col[k];
        double d0, d1, d2;
        if (kFirst) {
          d0 = D.z[3 * c];
          d1 = D.z[3 * c + 1];
          d2 = D.z[3 * c + 2];
        } else {
          d0 = D.z[3 * c] + beta * dold[3 * c];
          d1 = D.z[3 * c + 1] + beta * dold[3 * c + 1];
          d2 = D.z[3 * c + 2] + beta * dold[3 * c + 2];
        }
        q0 += D.vals[0 * NB + k] * d0 + D.vals[1 * NB + k] * d1 + D.vals[2 * NB + k] * d2;
        q1 += D.vals[3 * NB + k] * d0 + D.vals[4 * NB + k] * d1 + D.vals[5 * NB + k] * d2;
        q2 += D.vals[6 * NB + k] * d0 + D.vals[7 * NB + k] * d1 + D.vals[8 * NB + k] * d2;
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      q0 += __shfl_xor(q0, o, 16);
      q1 += __shfl_xor(q1, o, 16);
      q2 += __shfl_xor(q2, o, 16);
    }
    if (i < i1 && lane == 0) {
      double dn0, dn1, dn2;
      if (kFirst) {
        dn0 = D.z[3 * i];
        dn1 = D.z[3 * i + 1];
        dn2 = D.z[3 * i + 2];
      } else {
        dn0 = D.z[3 * i] + beta * dold[3 * i];
        dn1 = D.z[3 * i + 1] + beta * dold[3 * i + 1];
        dn2 = D.z[3 * i + 2] + beta * dold[3 * i + 2];
      }
      dnew[3 * i] = dn0;
      dnew[3 * i + 1] = dn1;
      dnew[3 * i + 2] = dn2;
      D.q[3 * i] = q0;
      D.q[3 * i + 1] = q1;
      D.q[3 * i + 2] = q2;
      kap += dn0 * q0 + dn1 * q1 + dn2 * q2;
    }
  }
  kap = block_sum(kap, lds);
  if (threadIdx.x == 0) D.part[kPartKappa * G + w] = kap;
}

__global__ __launch_bounds__(kBlock) void k_pcg_update(Dev D, int j) {
  __shared__ double lds[4];
  if (D.pcg->done) return;
  const int G = D.G, N = D.N;
  const double kap = reduce_partials(D.part + kPartKappa * G, G, lds);
  if (kap <= 0.0) { pcg_finish(D, 1, j + 1); return; }
  const double rz = reduce_partials(D.part + ((j & 1) ? kPartRZ1 : kPartRZ0) * G, G, lds);
  const double alpha = rz / kap;
  const double* d = (j & 1) ? D.d1 : D.d0;
  const int w = logical_wg(G);
  const int i0 = w * D.rows_per_wg, i1 = min(N, i0 + D.rows_per_wg);
  double rr = 0.0, rzn = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D.dx[3 * i + c] += alpha * d[3 * i + c];
      r[c] = D.r[3 * i + c] - alpha * D.q[3 * i + c];
      D.r[3 * i + c] = r[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double zc = D.pinv[(3 * c) * N + i] * r[0] + D.pinv[(3 * c + 1) * N + i] * r[1] +
                        D.pinv[(3 * c + 2) * N + i] * r[2];
      D.z[3 * i + c] = zc;
      rzn += r[c] * zc;
      rr += r[c] * r[c];
    }
  }
  rr = block_sum(rr, lds);
  rzn = block_sum(rzn, lds);
  if (threadIdx.x == 0) {
    D.part[kPartRR * G + w] = rr;
    D.part[((j & 1) ? kPartRZ0 : kPartRZ1) * G + w] = rzn;
  }
}

void launch_pcg_init(const Dev& D, hipStream_t st) { k_pcg_init<<<D.G, kBlock, 0, st>>>(D); }

void launch_pcg_iter(const Dev& D, int j, double tol2, int maxit, hipStream_t st) {
  if (j == 0)
    k_pcg_spmv<true><<<D.G, kBlock, 0, st>>>(D, j, tol2, maxit);
  else
    k_pcg_spmv<false><<<D.G, kBlock, 0, st>>>(D, j, tol2, maxit);
  k_pcg_update<<<D.G, kBlock, 0, st>>>(D, j);
}

// Plain q = H d (parity tests and benchmarks).
__global__ __launch_bounds__(kBlock) void k_spmv_plain(Dev D, const double* d, double* q) {
  const int G = D.G;
  const int w = logical_wg(G);
  const int i0 = w * D.rows_per_wg, i1 = min(D.N, i0 + D.rows_per_wg);
  const int lane = threadIdx.x & 15;
  const int64_t NB = D.NB;
  for (int ib = i0; ib < i1; ib += kBlock / 16) {
    const int i = ib + (threadIdx.x >> 4);
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    if (i < i1) {
      for (int k = D.row_ptr[i] + lane; k < D.row_ptr[i + 1]; k += 16) {
        const int c = D.col[k];
        const double d0 = d[3 * c], d1 = d[3 * c + 1], d2 = d[3 * c + 2];
        q0 += D.vals[0 * NB + k] * d0 + D.vals[1 * NB + k] * d1 + D.vals[2 * NB + k] * d2;
        q1 += D.vals[3 * NB + k] * d0 + D.vals[4 * NB + k] * d1 + D.vals[5 * NB + k] * d2;
        q2 += D.vals[6 * NB + k] * d0 + D.vals[7 * NB + k] * d1 + D.vals[8 * NB + k] * d2;
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      q0 += __shfl_xor(q0, o, 16);
      q1 += __shfl_xor(q1, o, 16);
      q2 += __shfl_xor(q2, o, 16);
    }
    if (i < i1 && lane == 0) {
      q[3 * i] = q0;
      q[3 * i + 1] = q1;
      q[3 * i + 2] = q2;
    }
  }
}

void launch_spmv_plain(const Dev& D, const double* d, double* q, hipStream_t st) {
  k_spmv_plain<<<D.G, kBlock, 0, st>>>(D, d, q);
}

}  // namespace ppn
