// Block-Jacobi preconditioned CG on the 3x3 block-sparse Hessian, with the
// early exit on non-positive curvature d^T H d <= 0 that proves H indefinite
// (Sec. 4.1, Linear Solvers), zero initial guess, and |r| <= rtol |r0|.
//
// One iteration is two kernels whose control scalars stay on the device:
//   spmv   : beta = r_j^T z_j / r_{j-1}^T z_{j-1}, the new direction
//            d_j = z_j + beta d_{j-1}, q = H d_j and partials of d_j^T q;
//   update : alpha = r_j^T z_j / d_j^T q, x += alpha d_j, r -= alpha q,
//            z = P^-1 r and partials of r^T r and r^T z.
// Every workgroup reduces the same partials in the same order, so all of them
// take the same stop decision; workgroup 0 records it in PcgState and later
// launches return at once.  The host only polls PcgState every few iterations.
// No fences or grid barriers are used: on a multi-XCD part a device-scope
// fence writes back the whole L2, while the kernel boundary does it once.
//
// Data: zd[N][6] holds (z_j, d_{j-1}) per vertex in 48-byte records, which the
// product gathers with three 16-byte loads per column; it writes its row's new
// direction d_j to dn[N][3].  The update then rewrites the whole record as
// (z_{j+1}, d_j): every store of both kernels covers whole cache lines (a
// record half written alone would leave each line partly written, twice per
// iteration), and no kernel writes the records while the product reads them,
// so one copy suffices.  The mixed form gathers FP32 roundings of the records
// instead (zd32) and keeps z alone, in FP64, as [N][3] for the rows' own use.
//
// The kernels are templates on the matrix type M.  FP64 is the plain path.
// With M = FP32 (the mixed-precision path) the sliced-ELL values and the
// block-Jacobi inverse are stored in FP32 and the matrix product is formed and
// accumulated in FP32, which halves the bytes of the dominant stream; the CG
// vectors, their recurrences and all dot products stay FP64, so the Krylov
// iteration itself loses nothing to FP32 rounding.  Each such solve is refined
// against the FP64 system (r = -g - H dx with the FP64 matrix, then another
// solve on r) until the FP64 residual meets the tolerance.
//
// The product is formed as H z + beta H d_old so that the streaming loop does
// not wait for this iteration's reductions.
//
// Matrix product: one row per lane, one 64-row sliced-ELL group per wavefront
// (uniform slot loop; every column-index and block-entry load is one contiguous
// 256 / 512-byte run), 4 groups per 256-thread workgroup, workgroups mapped to
// contiguous row ranges per XCD.  Slot-major storage keeps the wavefronts that
// walk their groups' slots at the same pace inside a narrow window of memory.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "k_common.h"
#include "topology.h"

namespace ppn {

constexpr int kPcgBlock = 256;  // threads per PCG workgroup: 4 groups of 64 rows

// The decision is recorded by the scene's logical workgroup 0.
__device__ inline void pcg_finish(const Dev& D, int w, int ind, int iters) {
  if (w == 0 && threadIdx.x == 0) {
    D.pcg->ind = ind;
    D.pcg->iters = iters;
    D.pcg->done = 1;
  }
}

// Whether the solve has ended.  Workgroup 0 of a launch may record the end
// while other workgroups of the same launch start, so the flag is read once per
// workgroup and shared through LDS: all waves of a workgroup take the same
// branch (a wave that returned alone would leave the others summing stale LDS
// partials after the next barrier).
__device__ __forceinline__ bool solve_done(const PcgState* pcg) {
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = *reinterpret_cast<const volatile int32_t*>(&pcg->done);
  __syncthreads();
  return s_done != 0;
}

// r = sign * src, x = 0, records (z, 0) with z = P^-1 r; partials of r^T r, r^T z and
// the count of diagonal blocks failing Sylvester's criterion.
// The bodies below take the scene's logical workgroup index w (0 .. Gp-1):
// the single-scene kernels derive it from the hardware index, the batched
// kernels from the job table.
template <typename M>
__device__ __forceinline__ void pcg_init_body(const Dev& D, const PcgVec<M>& V, const double* src,
                                              double sign, int w) {
  __shared__ double lds[16];
  const int Gp = D.Gp, N = D.N;
  const int i = w * kPcgBlock + threadIdx.x;
  double rr = 0.0, rz = 0.0, bad = 0.0;
  if (i < N) {
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = sign * src[3 * i + c];
      V.r[3 * i + c] = r[c];
      V.x[3 * i + c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double zc = double(V.pinv[kSym3[c][0] * N + i]) * r[0] +
                        double(V.pinv[kSym3[c][1] * N + i]) * r[1] +
                        double(V.pinv[kSym3[c][2] * N + i]) * r[2];
      if constexpr (sizeof(M) == 4) {
        V.zd[3 * size_t(i) + c] = zc;
        V.zd32[6 * size_t(i) + c] = float(zc);
        V.zd32[6 * size_t(i) + 3 + c] = 0.0f;
      } else {
        V.zd[6 * size_t(i) + c] = zc;
        V.zd[6 * size_t(i) + 3 + c] = 0.0;
      }
      rz += r[c] * zc;
      rr += r[c] * r[c];
    }
    bad = D.spd_ok[i] ? 0.0 : 1.0;
  }
  rr = block_sum(rr, lds);
  rz = block_sum(rz, lds);
  bad = block_sum(bad, lds);
  if (threadIdx.x == 0) {
    D.part[kPartRR * Gp + w] = rr;
    D.part[kPartRZ0 * Gp + w] = rz;
    D.part[kPartSpd * Gp + w] = bad;
  }
  if (w == 0 && threadIdx.x == 0) {
    D.pcg->done = 0;
    D.pcg->ind = 0;
    D.pcg->iters = 0;
    D.pcg->j_rr = -1;
  }
}

template <typename M>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_init(Dev D, PcgVec<M> V, const double* src,
                                                         double sign) {
  pcg_init_body<M>(D, V, src, sign, logical_wg(D.Gp));
}

// The 9 entries of the block at half position pos = slot * 64 + lane of the
// value array (value_index layout).
// FP64: entries paired, pair k = (2k, 2k+1) at slot*576 + 128k + 2*lane, entry 8
// at slot*576 + 512 + lane: four 16-byte loads and one 8-byte load, contiguous
// runs over a wavefront whose lanes read neighbouring positions (owned blocks;
// lower blocks read from their column's row keep runs of up to 64 lanes).
// kLoad == kLoadStream (forced only): the matrix is streamed with
// non-temporal loads; otherwise ordinary loads, which let a block's second
// (transposed) read hit the L2 and keep a matrix of up to the last-level
// cache's size resident between iterations.  The choice changes no arithmetic.
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <int kLoad>
__device__ __forceinline__ void load_block(const double* __restrict__ vals, int32_t pos, double w[9]) {
  const double* base = vals + size_t(pos >> 6) * (9 * kSell);
  const int l = pos & 63;
  const f64x2* v2 = reinterpret_cast<const f64x2*>(base) + l;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const f64x2 p = kLoad == kLoadStream ? __builtin_nontemporal_load(v2 + k * kSell) : v2[k * kSell];
    w[2 * k] = p.x;
    w[2 * k + 1] = p.y;
  }
  w[8] = kLoad == kLoadStream ? __builtin_nontemporal_load(base + 8 * kSell + l) : base[8 * kSell + l];
}
// FP32: entries paired, pair k = (2k, 2k+1) as a float2 at slot*576 + 2*(64k + lane)
// for k < 4, entry 8 at slot*576 + 512 + lane: five loads of 512 / 256 bytes.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int kLoad>
__device__ __forceinline__ void load_block(const float* __restrict__ vals, int32_t pos, float w[9]) {
  const float* base = vals + size_t(pos >> 6) * (9 * kSell);
  const int l = pos & 63;
  const f32x2* v2 = reinterpret_cast<const f32x2*>(base) + l;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const f32x2 p = kLoad == kLoadStream ? __builtin_nontemporal_load(v2 + k * kSell) : v2[k * kSell];
    w[2 * k] = p.x;
    w[2 * k + 1] = p.y;
  }
  w[8] = kLoad == kLoadStream ? __builtin_nontemporal_load(base + 8 * kSell + l) : base[8 * kSell + l];
}

// A lower block (i, j), j < i, is stored as (j, i): read it transposed.  Selects
// rather than a branch, since the lanes of a wavefront may differ.
template <typename M>
__device__ __forceinline__ void orient_block(int32_t ref, M w[9]) {
  const bool t = ref < 0;  // kRefTranspose is the sign bit
  const M a1 = w[1], a2 = w[2], a5 = w[5];
  w[1] = t ? w[3] : a1;
  w[3] = t ? a1 : w[3];
  w[2] = t ? w[6] : a2;
  w[6] = t ? a2 : w[6];
  w[5] = t ? w[7] : a5;
  w[7] = t ? a5 : w[7];
}

// One component of a 3x3 block times a vector: b0 v0 + b1 v1 + b2 v2 with the
// roundings written out (b1 v1 rounded, then b0 v0 and b2 v2 fused in turn),
// so that the arithmetic is fixed by the source and not by which products the
// compiler chooses to fuse.
__device__ __forceinline__ double block_row(double b0, double b1, double b2, double v0, double v1,
                                            double v2) {
  return __builtin_fma(b2, v2, __builtin_fma(b0, v0, b1 * v1));
}
__device__ __forceinline__ float block_row(float b0, float b1, float b2, float v0, float v1,
                                           float v2) {
  return __builtin_fmaf(b2, v2, __builtin_fmaf(b0, v0, b1 * v1));
}

// Column and value reference of slot (slot, lane): one 8-byte load.
__device__ __forceinline__ int2 slot_colref(const Dev& D, int slot, int l) {
  return reinterpret_cast<const int2*>(D.colref)[size_t(slot) * kSell + l];
}

// q_i = sum over the row's slots of B d_col, d read from a plain [N][3] vector (FP64).
__device__ __forceinline__ void sell_row_product(const Dev& D, const double* __restrict__ src,
                                                 int g, int l, double& q0, double& q1,
                                                 double& q2) {
  const int S = D.gslots[g];
  q0 = q1 = q2 = 0.0;
#pragma unroll 4
  for (int s = 0; s < S; ++s) {
    const int2 cr = slot_colref(D, s * D.n_groups + g, l);
    const int c = cr.x;
    const double d0 = src[3 * c], d1 = src[3 * c + 1], d2 = src[3 * c + 2];
    double v[9];
    load_block<kLoadCached>(D.vals, cr.y & kRefPosMask, v);
    orient_block(cr.y, v);
    q0 += block_row(v[0], v[1], v[2], d0, d1, d2);
    q1 += block_row(v[3], v[4], v[5], d0, d1, d2);
    q2 += block_row(v[6], v[7], v[8], d0, d1, d2);
  }
}

// Split product over the gathered (z, d_old) records: qz = H z and qd = H d_old,
// so that q = H (z + beta d_old) = qz + beta qd needs beta only at the end.
// The arithmetic and the accumulation are in the matrix type M (FP32 for the
// FP32 matrix: the gathered FP64 vectors are rounded on load).
// The gathered record of column c as (z, d_old) in type M: the FP64 record,
// or for the FP32 product its FP32 rounding (24 instead of 48 bytes; the same
// values the FP64 record rounds to).
template <typename M>
struct Gathered { M z0, z1, z2, d0, d1, d2; };
template <typename M>
__device__ __forceinline__ Gathered<M> gather_record(const double* __restrict__ zd,
                                                     const float* __restrict__ zd32, int c,
                                                     bool with_d) {
  Gathered<M> r;
  if constexpr (sizeof(M) == 4) {
    const float2* p = reinterpret_cast<const float2*>(zd32 + 6 * size_t(c));
    const float2 a = p[0], b = p[1];
    r.z0 = a.x; r.z1 = a.y; r.z2 = b.x; r.d0 = b.y;
    if (with_d) { const float2 e = p[2]; r.d1 = e.x; r.d2 = e.y; } else { r.d1 = r.d2 = 0.0f; }
  } else {
    const double2* p = reinterpret_cast<const double2*>(zd + 6 * size_t(c));
    const double2 a = p[0], b = p[1];
    r.z0 = a.x; r.z1 = a.y; r.z2 = b.x; r.d0 = b.y;
    if (with_d) { const double2 e = p[2]; r.d1 = e.x; r.d2 = e.y; } else { r.d1 = r.d2 = 0.0; }
  }
  return r;
}

template <typename M, int kLoad>
__device__ __forceinline__ void sell_row_product_split(const Dev& D, const M* __restrict__ vals,
                                                       const double* __restrict__ zd,
                                                       const float* __restrict__ zd32, bool with_d,
                                                       int g, int l, M qz[3], M qd[3]) {
  const int S = D.gslots[g];
  qz[0] = qz[1] = qz[2] = qd[0] = qd[1] = qd[2] = M(0);
  if (sizeof(M) == 4 && D.f32_full) {
    // full-layout FP32 copy: the block of slot s sits at its own position
#pragma unroll 2
    for (int s = 0; s < S; ++s) {
      const int slot = s * D.n_groups + g;
      const int c = D.col32[slot * kSell + l];
      const Gathered<M> v = gather_record<M>(zd, zd32, c, with_d);
      const M z0 = v.z0, z1 = v.z1, z2 = v.z2;
      M w[9];
      load_block<kLoad>(vals, slot * kSell + l, w);
      qz[0] += block_row(w[0], w[1], w[2], z0, z1, z2);
      qz[1] += block_row(w[3], w[4], w[5], z0, z1, z2);
      qz[2] += block_row(w[6], w[7], w[8], z0, z1, z2);
      if (with_d) {
        const M d0 = v.d0, d1 = v.d1, d2 = v.d2;
        qd[0] += block_row(w[0], w[1], w[2], d0, d1, d2);
        qd[1] += block_row(w[3], w[4], w[5], d0, d1, d2);
        qd[2] += block_row(w[6], w[7], w[8], d0, d1, d2);
      }
    }
    return;
  }
  // Half storage (FP64, or its FP32 copy): the slots in batches of kSlotBatch
  // whose loads (column and reference one batch ahead, then records and
  // blocks) are all issued before the batch is accumulated, in slot order.
  // Measured on the 1.57M-tet cube (FP64, 3 / 2 resident workgroups per CU):
  // one slot at a time with its reference loaded a slot ahead 49.1 / 53.1 us,
  // batches of 2 48.9 / 48.0 us, of 4 47.5 / 46.9 us.
  constexpr int kSlotBatch = 4;
  int2 nx[kSlotBatch];
#pragma unroll
  for (int k = 0; k < kSlotBatch; ++k)
    nx[k] = k < S ? slot_colref(D, k * D.n_groups + g, l) : make_int2(0, 0);
  for (int s0 = 0; s0 < S; s0 += kSlotBatch) {
    int2 cr[kSlotBatch];
#pragma unroll
    for (int k = 0; k < kSlotBatch; ++k) {
      cr[k] = nx[k];
      if (s0 + kSlotBatch + k < S) nx[k] = slot_colref(D, (s0 + kSlotBatch + k) * D.n_groups + g, l);
    }
    M w[kSlotBatch][9];
    Gathered<M> rv[kSlotBatch];
#pragma unroll
    for (int k = 0; k < kSlotBatch; ++k) {
      if (s0 + k < S) {  // S is the group's: uniform over the wavefront
        rv[k] = gather_record<M>(zd, zd32, cr[k].x, with_d);
        load_block<kLoad>(vals, cr[k].y & kRefPosMask, w[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kSlotBatch; ++k) {
      if (s0 + k < S) {
        orient_block(cr[k].y, w[k]);
        const M z0 = rv[k].z0, z1 = rv[k].z1, z2 = rv[k].z2;
        qz[0] += block_row(w[k][0], w[k][1], w[k][2], z0, z1, z2);
        qz[1] += block_row(w[k][3], w[k][4], w[k][5], z0, z1, z2);
        qz[2] += block_row(w[k][6], w[k][7], w[k][8], z0, z1, z2);
        if (with_d) {
          const M d0 = rv[k].d0, d1 = rv[k].d1, d2 = rv[k].d2;
          qd[0] += block_row(w[k][0], w[k][1], w[k][2], d0, d1, d2);
          qd[1] += block_row(w[k][3], w[k][4], w[k][5], d0, d1, d2);
          qd[2] += block_row(w[k][6], w[k][7], w[k][8], d0, d1, d2);
        }
      }
    }
  }
}

// The streaming loop does not depend on this iteration's scalars: the partial
// sums that decide beta and the stop test are loaded first, the product runs,
// and only then are the partials combined (their load latency hides under the loop).
// kFirst: the first product of a solve.  It stays a compile-time constant in
// the batched kernels too, so that they compile to the same arithmetic as the
// single-scene kernels (a runtime flag changes which products the compiler
// fuses into FMAs, and with it the last bits).
template <typename M, bool kFirst, int kLoad>
__device__ __forceinline__ void pcg_spmv_body(const Dev& D, const PcgVec<M>& V, int j, double tol2,
                                              int maxit, int w) {
  __shared__ double lds[16];
  if (solve_done(D.pcg)) return;
  const int Gp = D.Gp;
  const double* zcur = V.zd;
  const double* pa = D.part + kPartRR * Gp;
  const double* pb = D.part + ((j & 1) ? kPartRZ1 : kPartRZ0) * Gp;
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int k = threadIdx.x; k < Gp; k += kPcgBlock) {
    sa += pa[k];
    sb += pb[k];
    if (kFirst) sc += D.part[kPartSpd * Gp + k];
  }
  const int i = w * kPcgBlock + threadIdx.x;
  const int g = i / kSell, l = i % kSell;
  M qz[3] = {0, 0, 0}, qd[3] = {0, 0, 0};
  if (g < D.n_groups) sell_row_product_split<M, kLoad>(D, V.vals, zcur, V.zd32, !kFirst, g, l, qz, qd);

  sa = wave_sum(sa);
  sb = wave_sum(sb);
  if (kFirst) sc = wave_sum(sc);
  // The combination below is written out for the four wavefronts of a workgroup.
  static_assert(kPcgBlock == 4 * 64, "pcg_spmv_body sums the partials of exactly four wavefronts");
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    lds[wv] = sa;
    lds[4 + wv] = sb;
    lds[8 + wv] = sc;
  }
  __syncthreads();
  const double rr = ((lds[0] + lds[1]) + lds[2]) + lds[3];
  const double rz = ((lds[4] + lds[5]) + lds[6]) + lds[7];
  const double bad = ((lds[8] + lds[9]) + lds[10]) + lds[11];
  double beta = 0.0;
  if (kFirst) {
    if (bad > 0.0) { pcg_finish(D, w, 1, 0); return; }
    if (rr == 0.0) { pcg_finish(D, w, 0, 0); return; }
    if (rz <= 0.0) { pcg_finish(D, w, 1, 0); return; }
    if (w == 0 && threadIdx.x == 0) {
      D.pcg->rr0 = rr;
      D.pcg->rz[0] = rz;
      D.pcg->rr = rr;
      D.pcg->j_rr = 0;
    }
  } else {
    if (rr <= tol2 * D.pcg->rr0) { pcg_finish(D, w, 0, j); return; }
    if (rz <= 0.0) { pcg_finish(D, w, 1, j); return; }
    if (j >= maxit) { pcg_finish(D, w, 0, j); return; }
    beta = rz / D.pcg->rz[(j - 1) & 1];
    if (w == 0 && threadIdx.x == 0) {
      D.pcg->rz[j & 1] = rz;
      D.pcg->rr = rr;
      D.pcg->j_rr = j;
    }
  }
  double kap = 0.0;
  if (i < D.N) {
    // the row's own z_j and d_{j-1}: from its record, or in the mixed form
    // (whose gathers read the FP32 records) from z [N][3] and this vector
    double z0, z1, z2, o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if constexpr (sizeof(M) == 4) {
      z0 = zcur[3 * i];
      z1 = zcur[3 * i + 1];
      z2 = zcur[3 * i + 2];
      if (!kFirst) {
        o0 = V.dn[3 * i];
        o1 = V.dn[3 * i + 1];
        o2 = V.dn[3 * i + 2];
      }
    } else {
      const double2* p = reinterpret_cast<const double2*>(zcur + 6 * size_t(i));
      const double2 a = p[0], b = p[1], e = p[2];
      z0 = a.x;
      z1 = a.y;
      z2 = b.x;
      o0 = b.y;
      o1 = e.x;
      o2 = e.y;
    }
    double dn0 = z0, dn1 = z1, dn2 = z2;
    double q0 = double(qz[0]), q1 = double(qz[1]), q2 = double(qz[2]);
    if (!kFirst) {
      dn0 += beta * o0;
      dn1 += beta * o1;
      dn2 += beta * o2;
      q0 += beta * double(qd[0]);
      q1 += beta * double(qd[1]);
      q2 += beta * double(qd[2]);
    }
    V.dn[3 * i] = dn0;
    V.dn[3 * i + 1] = dn1;
    V.dn[3 * i + 2] = dn2;
    V.q[3 * i] = q0;
    V.q[3 * i + 1] = q1;
    V.q[3 * i + 2] = q2;
    kap = dn0 * q0 + dn1 * q1 + dn2 * q2;
  }
  kap = block_sum(kap, lds);
  if (threadIdx.x == 0) D.part[kPartKappa * Gp + w] = kap;
}

template <typename M, bool kFirst, int kLoad>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_spmv(Dev D, PcgVec<M> V, int j, double tol2,
                                                        int maxit) {
  // FP64 products of cache-resident matrices run their workgroups in panel
  // order (wg_order.h): on the 1.57M-tet cube 7.5% fewer bytes fetched and
  // 46.7 -> 45.7 us; the FP32 copy, half the bytes per block, is better in row
  // order (31.6 against 32.0 us).
  pcg_spmv_body<M, kFirst, kLoad>(D, V, j, tol2, maxit,
                                  kLoad == kLoadCached && sizeof(M) == 8
                                      ? logical_wg_panels(D.Gp, D.spmv_panel)
                                      : logical_wg(D.Gp));
}

// The row's inputs are loaded before the d^T q partials are combined, so both
// latencies overlap.  The workgroup's 256 vertices own a contiguous run of 768
// values of each [N][3] vector and of 1536 values of the records: q, r, x and
// d are moved from HBM to LDS with unit-stride non-temporal loads (read once;
// kept out of the L2, they leave it to the next product: 47.0 -> 46.7 us per
// product on the 1.57M-tet cube; the block-Jacobi inverse likewise made the
// update slower, 13.7 -> 14.5 us, and keeps ordinary loads), and r, x and the new
// records (z_{j+1}, d_j), assembled in LDS, back with unit-stride non-temporal
// stores, instead of 24- and 48-byte-strided accesses per lane.  None of the
// outputs is read again within the kernel; kept out of the L2 as dirty lines
// they shorten its write-back at the kernel's end.  Measured on the 1.57M-tet
// cube, per FP64 update: 14.6 us with z written into half of each record,
// 15.3 us with whole records stored per lane, 13.7 us as here.
template <typename M, bool kStream>
__device__ __forceinline__ void pcg_update_body(const Dev& D, const PcgVec<M>& V, int j, int w) {
  __shared__ double lds[16];
  // q and d, then (once both are read) the new records
  __shared__ double sqd[6 * kPcgBlock], sr[3 * kPcgBlock], sx[3 * kPcgBlock];
  double* sq = sqd;
  double* sd = sqd + 3 * kPcgBlock;
  if (solve_done(D.pcg)) return;
  const int Gp = D.Gp, N = D.N;
  const int t = threadIdx.x;
  const int i = w * kPcgBlock + t;
  const int64_t f0 = int64_t(w) * (3 * kPcgBlock);  // first vector value of the workgroup
  const int64_t nf = 3 * int64_t(N);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int64_t f = f0 + k * kPcgBlock + t;
    if (f < nf) {
      sq[k * kPcgBlock + t] = __builtin_nontemporal_load(V.q + f);
      sr[k * kPcgBlock + t] = __builtin_nontemporal_load(V.r + f);
      sx[k * kPcgBlock + t] = __builtin_nontemporal_load(V.x + f);
      sd[k * kPcgBlock + t] = __builtin_nontemporal_load(V.dn + f);
    }
  }
  double P[6];
  if (i < N) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      P[k] = double(kStream ? __builtin_nontemporal_load(V.pinv + k * N + i) : V.pinv[k * N + i]);
  }
  const double kap = reduce_partials(D.part + kPartKappa * Gp, Gp, lds);  // synchronises
  if (kap <= 0.0) { pcg_finish(D, w, 1, j + 1); return; }
  const double alpha = D.pcg->rz[j & 1] / kap;
  double rr = 0.0, rzn = 0.0;
  double d[3] = {0, 0, 0}, z[3] = {0, 0, 0};
  if (i < N) {
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d[c] = sd[3 * t + c];
      sx[3 * t + c] += alpha * d[c];
      r[c] = sr[3 * t + c] - alpha * sq[3 * t + c];
      sr[3 * t + c] = r[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[c] = P[kSym3[c][0]] * r[0] + P[kSym3[c][1]] * r[1] + P[kSym3[c][2]] * r[2];
      rzn += r[c] * z[c];
      rr += r[c] * r[c];
    }
  }
  block_sum2(rr, rzn, lds);  // synchronises: sx and sr are complete, sq and sd read
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    sqd[6 * t + c] = z[c];
    sqd[6 * t + 3 + c] = d[c];
  }
  __syncthreads();
  const int64_t e0 = int64_t(w) * (6 * kPcgBlock), ne = 6 * int64_t(N);
  if constexpr (sizeof(M) == 4) {
    // mixed form: z as [N][3] for the rows' own use, and the records rounded
    // to FP32 for the next product's gathers
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int idx = k * kPcgBlock + t;
      const int64_t f = f0 + idx;
      if (f < nf) __builtin_nontemporal_store(sqd[6 * (idx / 3) + idx % 3], V.zd + f);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int64_t e = e0 + k * kPcgBlock + t;
      if (e < ne) __builtin_nontemporal_store(float(sqd[k * kPcgBlock + t]), V.zd32 + e);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int64_t e = e0 + k * kPcgBlock + t;
      if (e < ne) __builtin_nontemporal_store(sqd[k * kPcgBlock + t], V.zd + e);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int64_t f = f0 + k * kPcgBlock + t;
    if (f < nf) {
      __builtin_nontemporal_store(sr[k * kPcgBlock + t], V.r + f);
      __builtin_nontemporal_store(sx[k * kPcgBlock + t], V.x + f);
    }
  }
  if (t == 0) {
    D.part[kPartRR * Gp + w] = rr;
    D.part[((j & 1) ? kPartRZ0 : kPartRZ1) * Gp + w] = rzn;
  }
}

template <typename M, bool kStream>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_update(Dev D, PcgVec<M> V, int j) {
  pcg_update_body<M, kStream>(D, V, j, logical_wg(D.Gp));
}

template <typename T>
static void pcg_init(const Dev& D, const PcgVec<T>& V, const double* src, double sign,
                     hipStream_t st) {
  k_pcg_init<T><<<D.Gp, kPcgBlock, 0, st>>>(D, V, src, sign);
}

// A sampled product (events given) is launched with the events attached to the
// launch itself, so that their interval is the kernel's execution and not the
// dispatch gap after the preceding kernel.
// Resident product workgroups per CU when the matrix stays in the last-level
// cache.  Each stored block is read twice, by its owner row and transposed by
// its partner row one slot later; the second read hits the XCD's L2 only if
// the bytes that all workgroups in flight on that XCD read in between (about
// one slot of every row in flight) fit there.  With every workgroup of the
// 1.57M-tet cube resident at once (4.2 per CU) they do not.  Capping residency,
// so that rows run as a window moving through each XCD's range, cut the FP64
// product's L2 fetches by 15% at 3 per CU and by 25% at 2 per CU; at 2 per CU
// the batched slot loads above keep enough bytes in flight (measured, FP64 in
// row order: 54.9 us uncapped, 47.5 us at 3, 46.9 us at 2).  With the panel
// order of the FP64 product the partners' reads meet anyway, and 3 per CU is
// better again (45.2 against 45.7 us at 2); the FP32 copy, with half the
// bytes per slot, is best at 3 too (34.8 us; 37.4 at 2).  The cap is an
// otherwise unused dynamic LDS request just above 1/(cap + 1) of the CU's LDS.
template <typename T>
static size_t spmv_cap_lds() {
  constexpr int kWgPerCu = 3;
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int v = cached[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int per_cu = 0;
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess || per_cu <= 0)
      per_cu = 160 * 1024;
    v = per_cu / (kWgPerCu + 1) + 1024;
    cached[dev].store(v, std::memory_order_relaxed);
  }
  return size_t(v);
}

template <typename T, int kLoad>
static void pcg_iter_k(const Dev& D, const PcgVec<T>& V, int j, double tol2, int maxit,
                       hipStream_t st, hipEvent_t ev_spmv_start, hipEvent_t ev_spmv_stop) {
  const size_t lds = kLoad == kLoadCached ? spmv_cap_lds<T>() : 0;
  if (ev_spmv_start && ev_spmv_stop) {
    if (j == 0)
      hipExtLaunchKernelGGL(k_pcg_spmv<T, true, kLoad>, dim3(D.Gp), dim3(kPcgBlock), lds, st,
                            ev_spmv_start, ev_spmv_stop, 0, D, V, j, tol2, maxit);
    else
      hipExtLaunchKernelGGL(k_pcg_spmv<T, false, kLoad>, dim3(D.Gp), dim3(kPcgBlock), lds, st,
                            ev_spmv_start, ev_spmv_stop, 0, D, V, j, tol2, maxit);
  } else if (j == 0) {
    k_pcg_spmv<T, true, kLoad><<<D.Gp, kPcgBlock, lds, st>>>(D, V, j, tol2, maxit);
  } else {
    k_pcg_spmv<T, false, kLoad><<<D.Gp, kPcgBlock, lds, st>>>(D, V, j, tol2, maxit);
  }
  k_pcg_update<T, kLoad == kLoadStream><<<D.Gp, kPcgBlock, 0, st>>>(D, V, j);
}

// The matrix values a product of type T reads: the FP64 half storage, or the
// mixed form's full-layout FP32 copy.
template <typename T>
static int load_mode_of(const Dev& D) {
  return load_mode(sizeof(T) == 8 ? matrix_bytes(D) : matrix_bytes_f32(D));
}

template <typename T>
static void pcg_iter(const Dev& D, const PcgVec<T>& V, int j, double tol2, int maxit,
                     hipStream_t st, hipEvent_t ev_spmv_start, hipEvent_t ev_spmv_stop) {
  switch (D.pcg_load >= 0 ? D.pcg_load : load_mode_of<T>(D)) {
    case kLoadStream: pcg_iter_k<T, kLoadStream>(D, V, j, tol2, maxit, st, ev_spmv_start, ev_spmv_stop); break;
    case kLoadCached: pcg_iter_k<T, kLoadCached>(D, V, j, tol2, maxit, st, ev_spmv_start, ev_spmv_stop); break;
    default: pcg_iter_k<T, kLoadSmall>(D, V, j, tol2, maxit, st, ev_spmv_start, ev_spmv_stop);
  }
}

void launch_pcg_init(const Dev& D, const PcgVec<double>& V, const double* src, double sign,
                     hipStream_t st) {
  pcg_init(D, V, src, sign, st);
}
void launch_pcg_init(const Dev& D, const PcgVec<float>& V, const double* src, double sign,
                     hipStream_t st) {
  pcg_init(D, V, src, sign, st);
}
void launch_pcg_iter(const Dev& D, const PcgVec<double>& V, int j, double tol2, int maxit,
                     hipStream_t st, hipEvent_t ev_spmv_start, hipEvent_t ev_spmv_stop) {
  pcg_iter(D, V, j, tol2, maxit, st, ev_spmv_start, ev_spmv_stop);
}
void launch_pcg_iter(const Dev& D, const PcgVec<float>& V, int j, double tol2, int maxit,
                     hipStream_t st, hipEvent_t ev_spmv_start, hipEvent_t ev_spmv_stop) {
  pcg_iter(D, V, j, tol2, maxit, st, ev_spmv_start, ev_spmv_stop);
}

// Plain q = H d in FP64 (parity tests and benchmarks).
__global__ __launch_bounds__(kPcgBlock) void k_spmv_plain(Dev D, const double* d, double* q) {
  const int w = logical_wg(D.Gp);
  const int i = w * kPcgBlock + threadIdx.x;
  const int g = i / kSell, l = i % kSell;
  if (g >= D.n_groups) return;
  double q0, q1, q2;
  sell_row_product(D, d, g, l, q0, q1, q2);
  if (i < D.N) {
    q[3 * i] = q0;
    q[3 * i + 1] = q1;
    q[3 * i + 2] = q2;
  }
}

void launch_spmv_plain(const Dev& D, const double* d, double* q, hipStream_t st) {
  k_spmv_plain<<<D.Gp, kPcgBlock, 0, st>>>(D, d, q);
}

// ---- mixed precision: solves with the FP32 matrix refined against the FP64 system ----

// dst = float(src) over n values.
__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ src,
                                                   float* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += stride)
    dst[k] = float(__builtin_nontemporal_load(src + k));
}

// FP32 copy of the matrix in the full sliced-ELL layout (every slot's block at
// its own position slot * 64 + lane, lower blocks transposed here once per
// solve), entries paired as read by load_block: the FP32 product of a small
// (CSR-ordered) matrix then reads contiguous runs and 4-byte columns, without
// references (measured: 30.9 against 30.1 mixed steps/s on the 122,880-tet
// beam, 307 against 286 on the 64-scene batch).  Large, distance-ordered
// matrices keep an FP32 copy of the half storage (36.5 against 39.1 us per
// product on the 1.57M-tet cube).
__global__ __launch_bounds__(kBlock) void k_half_to_full_f32(Dev D, const double* __restrict__ src,
                                                             float* __restrict__ dst) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  const int64_t n = D.n_slots * kSell;
  for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += stride) {
    const int32_t ref = reinterpret_cast<const int2*>(D.colref)[k].y;
    double w[9];
    load_block<kLoadStream>(src, ref & kRefPosMask, w);
    orient_block(ref, w);
    const int64_t slot = k / kSell;
    const int l = int(k % kSell);
    float* o = dst + slot * (9 * kSell);
    float2* o2 = reinterpret_cast<float2*>(o) + l;
#pragma unroll
    for (int p = 0; p < 4; ++p) o2[p * kSell] = make_float2(float(w[2 * p]), float(w[2 * p + 1]));
    o[8 * kSell + l] = float(w[8]);
  }
}

void launch_matrix_to_f32(const Dev& D, hipStream_t st) {
  if (!D.f32_full) {
    launch_to_f32(D.vals, D.vals32, D.n_hslots * 9 * kSell, st);
    return;
  }
  const int64_t n = D.n_slots * kSell;
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
  k_half_to_full_f32<<<unsigned(blocks), kBlock, 0, st>>>(D, D.vals, D.vals32);
}

void launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
  k_to_f32<<<unsigned(blocks), kBlock, 0, st>>>(src, dst, n);
}

// Outer start: dx = 0, r = -g, partials of |r|^2 in kPartA.
__global__ __launch_bounds__(kPcgBlock) void k_refine_init(Dev D) {
  __shared__ double lds[16];
  const int w = logical_wg(D.Gp);
  const int i = w * kPcgBlock + threadIdx.x;
  double rr = 0.0;
  if (i < D.N) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double rc = -D.g[3 * i + c];
      D.r[3 * i + c] = rc;
      D.dx[3 * i + c] = 0.0;
      rr += rc * rc;
    }
  }
  rr = block_sum(rr, lds);
  if (threadIdx.x == 0) D.part[kPartA * D.Gp + w] = rr;
}

// dx += e (the correction of the last inner solve).
__global__ __launch_bounds__(kPcgBlock) void k_refine_add(Dev D, const double* e) {
  const int i = blockIdx.x * kPcgBlock + threadIdx.x;
  if (i < 3 * D.N) D.dx[i] += e[i];
}

// r = -g - H dx in FP64, partials of |r|^2 in kPartA.
__global__ __launch_bounds__(kPcgBlock) void k_refine_residual(Dev D) {
  __shared__ double lds[16];
  const int w = logical_wg(D.Gp);
  const int i = w * kPcgBlock + threadIdx.x;
  const int g = i / kSell, l = i % kSell;
  double rr = 0.0;
  if (g < D.n_groups) {
    double q0, q1, q2;
    sell_row_product(D, D.dx, g, l, q0, q1, q2);
    if (i < D.N) {
      const double r0 = -D.g[3 * i] - q0, r1 = -D.g[3 * i + 1] - q1, r2 = -D.g[3 * i + 2] - q2;
      D.r[3 * i] = r0;
      D.r[3 * i + 1] = r1;
      D.r[3 * i + 2] = r2;
      rr = r0 * r0 + r1 * r1 + r2 * r2;
    }
  }
  rr = block_sum(rr, lds);
  if (threadIdx.x == 0) D.part[kPartA * D.Gp + w] = rr;
}

void launch_refine_init(const Dev& D, hipStream_t st) {
  k_refine_init<<<D.Gp, kPcgBlock, 0, st>>>(D);
}
void launch_refine_add(const Dev& D, const double* e, hipStream_t st) {
  k_refine_add<<<(3 * D.N + kPcgBlock - 1) / kPcgBlock, kPcgBlock, 0, st>>>(D, e);
}
void launch_refine_residual(const Dev& D, hipStream_t st) {
  k_refine_residual<<<D.Gp, kPcgBlock, 0, st>>>(D);
}

// ---- batched solves: one launch over the workgroups of many scenes ----
// Job k owns the global workgroups [wg0_k, wg0_k + Gp_k); each workgroup finds
// its job by binary search and runs the scene's body with its local index and
// the job's own iteration number (jobs join a running batch), so every scene
// computes exactly what it computes alone.
template <typename M>
__device__ __forceinline__ const PcgJob<M>& find_job(const PcgJob<M>* __restrict__ jobs, int n,
                                                    int& w) {
  const int b = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg0 <= b) lo = mid; else hi = mid - 1;
  }
  w = b - jobs[lo].wg0;
  return jobs[lo];
}

template <typename M>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_init_batch(const PcgJob<M>* __restrict__ jobs, int n) {
  int w;
  const PcgJob<M>& J = find_job(jobs, n, w);
  pcg_init_body<M>(J.D, J.V, J.src, J.sign, w);
}

// Iteration jg of the batch is iteration jg - j0 of each job's own solve.  The
// kFirst instance serves the jobs at their first iteration, the other the rest.
template <typename M, bool kFirst, int kLoad>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_spmv_batch(const PcgJob<M>* __restrict__ jobs, int n,
                                                              int jg) {
  int w;
  const PcgJob<M>& J = find_job(jobs, n, w);
  const int j = jg - J.j0;
  if ((j == 0) != kFirst) return;
  pcg_spmv_body<M, kFirst, kLoad>(J.D, J.V, j, J.tol2, J.maxit, w);
}

template <typename M, bool kStream>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_update_batch(const PcgJob<M>* __restrict__ jobs, int n,
                                                                int jg) {
  int w;
  const PcgJob<M>& J = find_job(jobs, n, w);
  pcg_update_body<M, kStream>(J.D, J.V, jg - J.j0, w);
}

// out[k] = job k's PcgState (one read-back for the whole batch).
template <typename M>
__global__ void k_pcg_gather_state(const PcgJob<M>* __restrict__ jobs, int n, PcgState* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = *jobs[k].D.pcg;
}

template <typename M>
static void batch_init(const PcgJob<M>* jobs, int n, int total_wg, hipStream_t st) {
  k_pcg_init_batch<M><<<total_wg, kPcgBlock, 0, st>>>(jobs, n);
}
template <typename M, int kLoad>
static void batch_iter_k(const PcgJob<M>* jobs, int n, int total_wg, int j, bool any_first,
                         hipStream_t st) {
  if (any_first) k_pcg_spmv_batch<M, true, kLoad><<<total_wg, kPcgBlock, 0, st>>>(jobs, n, j);
  k_pcg_spmv_batch<M, false, kLoad><<<total_wg, kPcgBlock, 0, st>>>(jobs, n, j);
  k_pcg_update_batch<M, kLoad == kLoadStream><<<total_wg, kPcgBlock, 0, st>>>(jobs, n, j);
}
// matrix_bytes: the summed size of the matrix values the jobs read (they share the cache).
template <typename M>
static void batch_iter(const PcgJob<M>* jobs, int n, int total_wg, int j, bool any_first,
                       int64_t matrix_bytes, hipStream_t st) {
  switch (load_mode(matrix_bytes)) {
    case kLoadStream: batch_iter_k<M, kLoadStream>(jobs, n, total_wg, j, any_first, st); break;
    case kLoadCached: batch_iter_k<M, kLoadCached>(jobs, n, total_wg, j, any_first, st); break;
    default: batch_iter_k<M, kLoadSmall>(jobs, n, total_wg, j, any_first, st);
  }
}
template <typename M>
static void batch_gather(const PcgJob<M>* jobs, int n, PcgState* out, hipStream_t st) {
  k_pcg_gather_state<M><<<(n + 63) / 64, 64, 0, st>>>(jobs, n, out);
}

void launch_pcg_batch_init(const PcgJob<double>* jobs, int n, int total_wg, hipStream_t st) {
  batch_init(jobs, n, total_wg, st);
}
void launch_pcg_batch_init(const PcgJob<float>* jobs, int n, int total_wg, hipStream_t st) {
  batch_init(jobs, n, total_wg, st);
}
void launch_pcg_batch_iter(const PcgJob<double>* jobs, int n, int total_wg, int j, bool any_first,
                           int64_t matrix_bytes, hipStream_t st) {
  batch_iter(jobs, n, total_wg, j, any_first, matrix_bytes, st);
}
void launch_pcg_batch_iter(const PcgJob<float>* jobs, int n, int total_wg, int j, bool any_first,
                           int64_t matrix_bytes, hipStream_t st) {
  batch_iter(jobs, n, total_wg, j, any_first, matrix_bytes, st);
}
void launch_pcg_batch_gather(const PcgJob<double>* jobs, int n, PcgState* out, hipStream_t st) {
  batch_gather(jobs, n, out, st);
}
void launch_pcg_batch_gather(const PcgJob<float>* jobs, int n, PcgState* out, hipStream_t st) {
  batch_gather(jobs, n, out, st);
}

}  // namespace ppn
