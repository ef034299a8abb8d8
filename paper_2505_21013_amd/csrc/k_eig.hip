// Batched projection of 12x12 element Hessians to the SPD cone by eigenvalue
// clamping (Sec. 3, Eq. (4)): Hhat = Q max(D, eps) Q^T, written here in the
// difference form Hhat = H + sum_{lambda_i < eps} (eps - lambda_i) q_i q_i^T so
// that the untouched part of the spectrum is kept exactly.
//
// GPU design (one element per lane, everything in registers):
//  * Exact deflation of the translations.  The element gradient operator has
//    b_0 + b_1 + b_2 + b_3 = 0, so H^e annihilates the three rigid
//    translations.  With U = (1/2) Had_4 (x) I_3 (Had_4 the symmetric 4x4
//    Hadamard matrix, U = U^T = U^-1) the first 3x3 block row of U H U is the
//    translation block (zero up to rounding) and the remaining 9x9 block K
//    carries the rest of the spectrum.  The translation eigenvalues (0) are
//    clamped to eps exactly, so Delta H = U diag(eps I_3, Delta K) U.
//  * Cyclic Jacobi on K in round-robin order (9 rounds of 4 disjoint
//    rotations per sweep, fully unrolled with compile-time indices), stopping
//    when off(K) <= 1e-15 |K|_F (FP32: ~3e-7) or after 15 sweeps.  Every lane
//    of a wavefront sweeps until all 64 have converged.
//  * The element matrix is streamed block by block on the way in (into K) and
//    on the way out (H + Delta H), so only K, V and one 3x3 block are live.
#include <hip/hip_runtime.h>

#include "k_common.h"
#include "topology.h"

namespace ppn {

constexpr int kMaxSweeps = 15;

__host__ __device__ constexpr int ui12(int r, int c) {
  return r <= c ? r * 12 - r * (r - 1) / 2 + (c - r) : c * 12 - c * (c - 1) / 2 + (r - c);
}
__host__ __device__ constexpr int ui9(int r, int c) {
  return r <= c ? r * 9 - r * (r - 1) / 2 + (c - r) : c * 9 - c * (c - 1) / 2 + (r - c);
}
// Hadamard sign s[A][a]
__host__ __device__ constexpr double hs(int A, int a) {
  return ((A == 0) || (A == 1 && a < 2) || (A == 2 && (a == 0 || a == 2)) ||
          (A == 3 && (a == 0 || a == 3)))
             ? 1.0
             : -1.0;
}

// Working state of one element, held by one lane: the upper triangle of the
// 9x9 matrix and the accumulated eigenvector matrix V (row-major).
template <typename T>
struct EigLane {
  T a[45];
  T v[81];
};

// Reciprocal and reciprocal square root from the hardware estimates refined
// by Newton steps (the FP64 estimates carry about 23 correct bits, two steps
// bring them to the last bit).  Arguments are positive normal numbers.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ float rcp_nr(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
__device__ __forceinline__ float rsq_nr(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}

// Rotation annihilating a(P,Q): t = tan(theta), s = sin(theta), tau = tan(theta/2).
template <typename T>
struct Rot {
  T t, s, tau;
};

template <int P, int Q, typename T>
__device__ __forceinline__ Rot<T> angle(const EigLane<T>& L) {
  const T apq = L.a[ui9(P, Q)];
  const T d = L.a[ui9(Q, Q)] - L.a[ui9(P, P)];
  const T x = d * d + T(4) * apq * apq;
  const bool act = x > (sizeof(T) == 8 ? T(1e-280) : T(1e-30));
  const T r = x * rsq_nr(act ? x : T(1));  // sqrt(d^2 + 4 apq^2)
  const T inv = rcp_nr(act ? fabs(d) + r : T(1));
  const T t = act ? T(2) * (d >= T(0) ? apq : -apq) * inv : T(0);
  const T c = rsq_nr(T(1) + t * t);
  const T s = t * c;
  return {t, s, s * rcp_nr(T(1) + c)};
}

// Applies the rotation of (P,Q) (Rutishauser's update).  Entries of other
// disjoint pairs' 2x2 diagonal blocks are not touched, so the rotations of one
// round commute and their angles can all be taken before any is applied.
template <int P, int Q, typename T>
__device__ __forceinline__ void apply(EigLane<T>& L, const Rot<T>& R) {
  T* a = L.a;
  const T apq = a[ui9(P, Q)];
  a[ui9(P, P)] -= R.t * apq;
  a[ui9(Q, Q)] += R.t * apq;
  a[ui9(P, Q)] = T(0);
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    if (r != P && r != Q) {
      const T g = a[ui9(r, P)], h = a[ui9(r, Q)];
      a[ui9(r, P)] = g - R.s * (h + g * R.tau);
      a[ui9(r, Q)] = h + R.s * (g - h * R.tau);
    }
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const T g = L.v[9 * r + P], h = L.v[9 * r + Q];
    L.v[9 * r + P] = g - R.s * (h + g * R.tau);
    L.v[9 * r + Q] = h + R.s * (g - h * R.tau);
  }
}

// Round-robin (parallel) ordering of the 36 pairs of 9 indices: in round k the
// pairs {(k + i) mod 9, (k - i) mod 9}, i = 1..4, are disjoint, and each pair
// occurs in exactly one of the 9 rounds.  The four angles of a round are
// independent, which gives the wavefront four chains of divides and square
// roots to overlap instead of one.
__host__ __device__ constexpr int rr_p(int k, int i) {
  return ((k + i) % 9) < ((k + 9 - i) % 9) ? (k + i) % 9 : (k + 9 - i) % 9;
}
__host__ __device__ constexpr int rr_q(int k, int i) {
  return ((k + i) % 9) < ((k + 9 - i) % 9) ? (k + 9 - i) % 9 : (k + i) % 9;
}

template <int K>
struct Sweep {
  template <typename T>
  __device__ __forceinline__ static void run(EigLane<T>& L) {
    const Rot<T> r1 = angle<rr_p(K, 1), rr_q(K, 1)>(L);
    const Rot<T> r2 = angle<rr_p(K, 2), rr_q(K, 2)>(L);
    const Rot<T> r3 = angle<rr_p(K, 3), rr_q(K, 3)>(L);
    const Rot<T> r4 = angle<rr_p(K, 4), rr_q(K, 4)>(L);
    apply<rr_p(K, 1), rr_q(K, 1)>(L, r1);
    apply<rr_p(K, 2), rr_q(K, 2)>(L, r2);
    apply<rr_p(K, 3), rr_q(K, 3)>(L, r3);
    apply<rr_p(K, 4), rr_q(K, 4)>(L, r4);
    if constexpr (K + 1 < 9) Sweep<K + 1>::run(L);
  }
};

// Corners (a, c) of 3x3 block b of an element matrix: blocks 0..3 are the
// diagonal blocks of the four corners, blocks 4..9 the corner pairs a < c.
__host__ __device__ constexpr int blk_a(int b) { return b < 4 ? b : kPairA[b - 4]; }
__host__ __device__ constexpr int blk_c(int b) { return b < 4 ? b : kPairC[b - 4]; }

// Adds block b (m[3i+k] = H[3a+i][3c+k]) into the upper triangle k of
// U H U restricted to its non-translational 9x9 part, without the factor 1/4:
// K[(A,i)][(B,k)] = sum_{a,c} s_A(a) s_B(c) H[3a+i][3c+k], A, B = 1..3.  An
// off-diagonal block also stands for its transpose (c, a).
template <typename T>
__device__ __forceinline__ void add_block_to_k(int b, const double* m, T* k) {
  const int a = blk_a(b), c = blk_c(b);
#pragma unroll
  for (int R = 0; R < 9; ++R) {
#pragma unroll
    for (int C = R; C < 9; ++C) {
      const int A = 1 + R / 3, i = R % 3, B = 1 + C / 3, kk = C % 3;
      double t = hs(A, a) * hs(B, c) * m[3 * i + kk];
      if (a != c) t += hs(A, c) * hs(B, a) * m[3 * kk + i];
      k[ui9(R, C)] += T(t);
    }
  }
}

// Block b of Delta H = U diag(eps I_3, dk) U (dk: upper triangle of the 9x9 part).
template <typename T>
__device__ __forceinline__ void delta_block(int b, const T* dk, double eps, double* m) {
  const int a = blk_a(b), c = blk_c(b);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      double s = (i == kk) ? eps : 0.0;
#pragma unroll
      for (int A = 1; A < 4; ++A)
#pragma unroll
        for (int B = 1; B < 4; ++B)
          s += hs(A, a) * hs(B, c) * double(dk[ui9(3 * (A - 1) + i, 3 * (B - 1) + kk)]);
      m[3 * i + kk] = 0.25 * s;
    }
  }
}

// Projection of one element.
template <typename T, class IO>
__device__ __forceinline__ void project_one(const IO& io, double eps, bool mirror) {
  EigLane<T> L;
#pragma unroll
  for (int i = 0; i < 45; ++i) L.a[i] = T(0);
#pragma unroll
  for (int b = 0; b < 10; ++b) {
    double m[9];
    io.load(b, m);
    add_block_to_k<T>(b, m, L.a);
  }
#pragma unroll
  for (int i = 0; i < 45; ++i) L.a[i] *= T(0.25);
#pragma unroll
  for (int i = 0; i < 81; ++i) L.v[i] = (i % 10 == 0) ? T(1) : T(0);
  const T tol2 = sizeof(T) == 8 ? T(1e-30) : T(1e-13);
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    T off = T(0), dia = T(0);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      dia += L.a[ui9(r, r)] * L.a[ui9(r, r)];
#pragma unroll
      for (int c = r + 1; c < 9; ++c) off += L.a[ui9(r, c)] * L.a[ui9(r, c)];
    }
    const bool done = off <= tol2 * (dia + T(2) * off);
    if (__all(done)) break;
    Sweep<0>::run(L);
  }
  // Delta K = V W V^T with W = diag(lambda_hat_i - lambda_i): lambda_hat =
  // max(lambda, eps) when clamping, max(|lambda|, eps) when mirroring; both
  // leave every lambda >= eps exactly unchanged (w = 0).
  T w[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T l = L.a[ui9(i, i)];
    w[i] = mirror ? fmax(fabs(l), T(eps)) - l : fmax(T(eps) - l, T(0));
  }
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      T s = T(0);
#pragma unroll
      for (int i = 0; i < 9; ++i) s += w[i] * L.v[9 * r + i] * L.v[9 * c + i];
      L.a[ui9(r, c)] = s;
    }
#pragma unroll
  for (int b = 0; b < 10; ++b) {
    double m[9], d[9];
    io.load(b, m);
    delta_block<T>(b, L.a, eps, d);
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] += d[i];
    io.store(b, m);
  }
}

// Element Hessian stored in the scatter slots of element e.
struct SlotIO {
  const Dev& D;
  int vs[4], es[6];
  bool flip[6];
  __device__ SlotIO(const Dev& d, int e) : D(d) {
    const int T = D.T;
    int v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      v[a] = D.tets[a * T + e];
      vs[a] = D.vslot[a * T + e];
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      es[p] = D.eslot[p * T + e];
      flip[p] = v[kPairA[p]] > v[kPairC[p]];
    }
  }
  // m[3i+k] = H[3a+i][3c+k] for block b (diagonal blocks: the slot keeps the
  // upper triangle; edge slots keep the block of the lower-to-higher vertex).
  __device__ __forceinline__ void load(int b, double* m) const {
    if (b < 4) {
      const double* s = D.vslots + size_t(vs[b]) * 9 + 3;
      m[0] = s[0]; m[1] = s[1]; m[2] = s[2];
      m[4] = s[3]; m[5] = s[4]; m[8] = s[5];
      m[3] = m[1]; m[6] = m[2]; m[7] = m[5];
    } else {
      const int p = b - 4;
      const double* s = D.eslots + size_t(es[p]) * 9;
      double t[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) t[k] = s[k];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) m[3 * i + k] = flip[p] ? t[3 * k + i] : t[3 * i + k];
    }
  }
  __device__ __forceinline__ void store(int b, const double* m) const {
    if (b < 4) {
      double* s = D.vslots + size_t(vs[b]) * 9 + 3;
      s[0] = m[0]; s[1] = m[1]; s[2] = m[2];
      s[3] = m[4]; s[4] = m[5]; s[5] = m[8];
    } else {
      const int p = b - 4;
      double* s = D.eslots + size_t(es[p]) * 9;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) s[3 * i + k] = flip[p] ? m[3 * k + i] : m[3 * i + k];
    }
  }
};

// Row-major dense 12x12 matrix (upper-triangle blocks read, both triangles written).
struct DenseIO {
  const double* in;
  double* out;
  __device__ __forceinline__ void load(int b, double* m) const {
    const int a = blk_a(b), c = blk_c(b);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // diagonal blocks: upper triangle only
        const int r = 3 * a + i, q = 3 * c + k;
        m[3 * i + k] = (a == c && i > k) ? in[12 * q + r] : in[12 * r + q];
      }
  }
  __device__ __forceinline__ void store(int b, const double* m) const {
    const int a = blk_a(b), c = blk_c(b);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        out[12 * (3 * a + i) + 3 * c + k] = m[3 * i + k];
        if (a != c) out[12 * (3 * c + k) + 3 * a + i] = m[3 * i + k];
      }
  }
};

template <class IO>
struct Guarded {
  const IO& io;
  bool live;
  __device__ __forceinline__ void load(int b, double* m) const { io.load(b, m); }
  __device__ __forceinline__ void store(int b, const double* m) const {
    if (live) io.store(b, m);
  }
};

// Lanes past the end still take part in the wavefront's sweep vote: they work
// on the first element's data in registers and never store.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_eig_all(Dev D, double eps, int mirror) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  const bool live = e < D.T;
  SlotIO io(D, live ? e : 0);
  project_one<T>(Guarded<SlotIO>{io, live}, eps, mirror != 0);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eig_list(Dev D, int n, double eps, int mirror) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const bool live = k < n;
  SlotIO io(D, D.list[live ? k : 0]);
  project_one<T>(Guarded<SlotIO>{io, live}, eps, mirror != 0);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eig_dense(const double* in, double* out, int64_t n,
                                                       double eps) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool live = k < n;
  const int64_t m = live ? k : 0;
  DenseIO io{in + 144 * m, out + 144 * m};
  project_one<T>(Guarded<DenseIO>{io, live}, eps, false);
}

// Precondition of the dense projector, which deflates the translations
// exactly: each matrix is symmetric and annihilates the three rigid
// translations (in every row, the four vertex columns of each coordinate sum
// to zero), both up to rtol times its largest entry.  A matrix that fails (or
// holds a NaN) sets *bad = 1; every writer stores the same value.
__global__ __launch_bounds__(kBlock) void k_check_dense(const double* in, int64_t n, double rtol,
                                                        int32_t* bad) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= n) return;
  const double* H = in + 144 * k;
  // fmax drops NaN operands, so finiteness is tested on its own.
  double amax = 0.0, trans = 0.0, asym = 0.0;
  bool finite = true;
  for (int r = 0; r < 12; ++r) {
    for (int c = 0; c < 3; ++c) {
      const double t = ((H[12 * r + c] + H[12 * r + 3 + c]) + H[12 * r + 6 + c]) + H[12 * r + 9 + c];
      trans = fmax(trans, fabs(t));
    }
    for (int c = 0; c < 12; ++c) {
      const double h = H[12 * r + c];
      finite = finite && isfinite(h);
      amax = fmax(amax, fabs(h));
      if (c > r) asym = fmax(asym, fabs(h - H[12 * c + r]));
    }
  }
  if (!finite || !(trans <= rtol * amax) || !(asym <= rtol * amax)) *bad = 1;
}

// Full 12x12 element matrices gathered from the slots (debug / parity output).
__global__ __launch_bounds__(kBlock) void k_elem_dense(Dev D, const int32_t* ids, int n,
                                                        double* out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int e = ids ? ids[t] : t;
  SlotIO io(D, e);
  DenseIO o{nullptr, out + size_t(t) * 144};
#pragma unroll
  for (int b = 0; b < 10; ++b) {
    double m[9];
    io.load(b, m);
    o.store(b, m);
  }
}

void launch_eig_all(const Dev& D, double eps, int mirror, hipStream_t st) {
  k_eig_all<double><<<(D.T + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, eps, mirror);
}

void launch_eig_list(const Dev& D, int32_t n, double eps, int mirror, hipStream_t st) {
  if (n <= 0) return;
  k_eig_list<double><<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, n, eps, mirror);
}

void launch_eig_all_f32(const Dev& D, double eps, int mirror, hipStream_t st) {
  k_eig_all<float><<<(D.T + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, eps, mirror);
}

void launch_eig_list_f32(const Dev& D, int32_t n, double eps, int mirror, hipStream_t st) {
  if (n <= 0) return;
  k_eig_list<float><<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, n, eps, mirror);
}

void launch_project_batch(const double* H, double* out, int64_t n, double eps, hipStream_t st) {
  if (n <= 0) return;
  k_eig_dense<double><<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(H, out, n, eps);
}

void launch_check_dense(const double* H, int64_t n, double rtol, int32_t* bad, hipStream_t st) {
  if (n <= 0) return;
  k_check_dense<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(H, n, rtol, bad);
}

void launch_element_hessians(const Dev& D, const int32_t* ids, int32_t n, double* out,
                             hipStream_t st) {
  if (n <= 0) return;
  k_elem_dense<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, ids, n, out);
}

}  // namespace ppn
