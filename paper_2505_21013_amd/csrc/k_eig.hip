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
//  * Cyclic-by-row Jacobi on K (36 rotations per sweep, fully unrolled with
//    compile-time indices), eigenvectors accumulated in a 9x9 register
//    array, stopping when off(K) <= 1e-15 |K|_F or after 15 sweeps.  Every
//    lane of a wavefront sweeps until all 64 have converged.
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

// One Jacobi rotation annihilating a(P,Q) (Rutishauser's update with tau = tan(theta/2)).
template <int P, int Q>
__device__ __forceinline__ void jrot(double* a, double* v) {
  const double apq = a[ui9(P, Q)];
  const double app = a[ui9(P, P)], aqq = a[ui9(Q, Q)];
  const double d = aqq - app;
  const double den = fabs(d) + sqrt(d * d + 4.0 * apq * apq);
  const double t = den > 0.0 ? (d >= 0.0 ? 2.0 * apq : -2.0 * apq) / den : 0.0;
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = t * c;
  const double tau = s / (1.0 + c);
  a[ui9(P, P)] = app - t * apq;
  a[ui9(Q, Q)] = aqq + t * apq;
  a[ui9(P, Q)] = 0.0;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    if (r != P && r != Q) {
      const double g = a[ui9(r, P)], h = a[ui9(r, Q)];
      a[ui9(r, P)] = g - s * (h + g * tau);
      a[ui9(r, Q)] = h + s * (g - h * tau);
    }
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const double g = v[9 * r + P], h = v[9 * r + Q];
    v[9 * r + P] = g - s * (h + g * tau);
    v[9 * r + Q] = h + s * (g - h * tau);
  }
}

template <int P, int Q>
struct Sweep {
  __device__ __forceinline__ static void run(double* a, double* v) {
    jrot<P, Q>(a, v);
    if constexpr (Q + 1 < 9) {
      Sweep<P, Q + 1>::run(a, v);
    } else if constexpr (P + 2 < 9) {
      Sweep<P + 1, P + 2>::run(a, v);
    }
  }
};

// K = (U H U) restricted to the non-translational 9x9 block, from the upper
// triangle h[78] of H.
__device__ __forceinline__ void build_k(const double* h, double* k) {
#pragma unroll
  for (int R = 0; R < 9; ++R) {
#pragma unroll
    for (int C = R; C < 9; ++C) {
      const int A = 1 + R / 3, i = R % 3, B = 1 + C / 3, kk = C % 3;
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) s += hs(A, a) * hs(B, c) * h[ui12(3 * a + i, 3 * c + kk)];
      k[ui9(R, C)] = 0.25 * s;
    }
  }
}

// h += Delta H where Delta H = U diag(eps I_3, dk) U.
__device__ __forceinline__ void add_delta(double* h, const double* dk, double eps) {
#pragma unroll
  for (int r = 0; r < 12; ++r) {
#pragma unroll
    for (int c = r; c < 12; ++c) {
      const int a = r / 3, i = r % 3, cb = c / 3, kk = c % 3;
      double s = (i == kk) ? eps : 0.0;
#pragma unroll
      for (int A = 1; A < 4; ++A)
#pragma unroll
        for (int B = 1; B < 4; ++B) s += hs(A, a) * hs(B, cb) * dk[ui9(3 * (A - 1) + i, 3 * (B - 1) + kk)];
      h[ui12(r, c)] += 0.25 * s;
    }
  }
}

template <class IO>
__device__ __forceinline__ void project_one(IO& io, double eps) {
  double a[45];
  {
    double h[78];
    io.load(h);
    build_k(h, a);
  }
  double v[81];
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = 0; c < 9; ++c) v[9 * r + c] = (r == c) ? 1.0 : 0.0;
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      dia += a[ui9(r, r)] * a[ui9(r, r)];
#pragma unroll
      for (int c = r + 1; c < 9; ++c) off += a[ui9(r, c)] * a[ui9(r, c)];
    }
    const bool done = off <= 1e-30 * (dia + 2.0 * off);
    if (__all(done)) break;
    Sweep<0, 1>::run(a, v);
  }
  // Delta K = sum_i max(eps - lambda_i, 0) q_i q_i^T
  double w[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) w[i] = fmax(eps - a[ui9(i, i)], 0.0);
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 9; ++i) s += w[i] * v[9 * r + i] * v[9 * c + i];
      a[ui9(r, c)] = s;
    }
  {
    double h[78];
    io.load(h);
    add_delta(h, a, eps);
    io.store(h);
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
  __device__ __forceinline__ void load(double* h) const {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double* s = D.vslots + size_t(vs[a]) * 9 + 3;
      h[ui12(3 * a + 0, 3 * a + 0)] = s[0];
      h[ui12(3 * a + 0, 3 * a + 1)] = s[1];
      h[ui12(3 * a + 0, 3 * a + 2)] = s[2];
      h[ui12(3 * a + 1, 3 * a + 1)] = s[3];
      h[ui12(3 * a + 1, 3 * a + 2)] = s[4];
      h[ui12(3 * a + 2, 3 * a + 2)] = s[5];
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int a = kPairA[p], c = kPairC[p];
      const double* s = D.eslots + size_t(es[p]) * 9;
      double b[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) b[k] = s[k];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) h[ui12(3 * a + i, 3 * c + k)] = flip[p] ? b[3 * k + i] : b[3 * i + k];
    }
  }
  __device__ __forceinline__ void store(const double* h) const {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double* s = D.vslots + size_t(vs[a]) * 9 + 3;
      s[0] = h[ui12(3 * a + 0, 3 * a + 0)];
      s[1] = h[ui12(3 * a + 0, 3 * a + 1)];
      s[2] = h[ui12(3 * a + 0, 3 * a + 2)];
      s[3] = h[ui12(3 * a + 1, 3 * a + 1)];
      s[4] = h[ui12(3 * a + 1, 3 * a + 2)];
      s[5] = h[ui12(3 * a + 2, 3 * a + 2)];
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int a = kPairA[p], c = kPairC[p];
      double* s = D.eslots + size_t(es[p]) * 9;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double val = h[ui12(3 * a + i, 3 * c + k)];
          if (flip[p]) s[3 * k + i] = val; else s[3 * i + k] = val;
        }
    }
  }
};

// Row-major dense 12x12 matrix (upper triangle read, both triangles written).
struct DenseIO {
  const double* in;
  double* out;
  __device__ __forceinline__ void load(double* h) const {
#pragma unroll
    for (int r = 0; r < 12; ++r)
#pragma unroll
      for (int c = r; c < 12; ++c) h[ui12(r, c)] = in[12 * r + c];
  }
  __device__ __forceinline__ void store(const double* h) const {
#pragma unroll
    for (int r = 0; r < 12; ++r)
#pragma unroll
      for (int c = 0; c < 12; ++c) out[12 * r + c] = h[ui12(r, c)];
  }
};

__global__ __launch_bounds__(kBlock) void k_eig_all(Dev D, double eps) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  // Lanes past the end still take part in the wavefront's sweep vote; they
  // work on element 0's data in registers and never store.
  const bool live = e < D.T;
  SlotIO io(D, live ? e : 0);
  struct Guard {
    SlotIO& io;
    bool live;
    __device__ void load(double* h) const { io.load(h); }
    __device__ void store(const double* h) const {
      if (live) io.store(h);
    }
  } g{io, live};
  project_one(g, eps);
}

__global__ __launch_bounds__(kBlock) void k_eig_list(Dev D, int n, double eps) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const bool live = t < n;
  const int e = D.list[live ? t : 0];
  SlotIO io(D, e);
  struct Guard {
    SlotIO& io;
    bool live;
    __device__ void load(double* h) const { io.load(h); }
    __device__ void store(const double* h) const {
      if (live) io.store(h);
    }
  } g{io, live};
  project_one(g, eps);
}

__global__ __launch_bounds__(kBlock) void k_eig_dense(const double* in, double* out, int64_t n,
                                                       double eps) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool live = t < n;
  const int64_t m = live ? t : 0;
  struct Guard {
    DenseIO io;
    bool live;
    __device__ void load(double* h) const { io.load(h); }
    __device__ void store(const double* h) const {
      if (live) io.store(h);
    }
  } g{DenseIO{in + 144 * m, out + 144 * m}, live};
  project_one(g, eps);
}

// Full 12x12 element matrices gathered from the slots (debug / parity output).
__global__ __launch_bounds__(kBlock) void k_elem_dense(Dev D, const int32_t* ids, int n,
                                                        double* out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int e = ids ? ids[t] : t;
  SlotIO io(D, e);
  double h[78];
  io.load(h);
  double* o = out + size_t(t) * 144;
  for (int r = 0; r < 12; ++r)
    for (int c = 0; c < 12; ++c) o[12 * r + c] = h[ui12(r, c)];
}

void launch_eig_all(const Dev& D, double eps, hipStream_t st) {
  k_eig_all<<<(D.T + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, eps);
}

void launch_eig_list(const Dev& D, int32_t n, double eps, hipStream_t st) {
  if (n <= 0) return;
  k_eig_list<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, n, eps);
}

void launch_project_batch(const double* H, double* out, int64_t n, double eps, hipStream_t st) {
  if (n <= 0) return;
  k_eig_dense<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(H, out, n, eps);
}

void launch_element_hessians(const Dev& D, const int32_t* ids, int32_t n, double* out,
                             hipStream_t st) {
  if (n <= 0) return;
  k_elem_dense<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, ids, n, out);
}

}  // namespace ppn
