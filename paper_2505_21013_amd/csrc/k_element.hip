// Element kernels: rest-shape precompute, Stable Neo-Hookean energy / gradient /
// Hessian of linear tetrahedra written into the scatter slots, the line-search
// energy difference, and the per-vertex time-integration updates.
//
// Element quantities (Sec. 3: H = sum_e H^e, g = sum_e g^e), with
// F = sum_a x_a b_a^T, b_1..b_3 the rows of Dm^-1 and b_0 = -(b_1+b_2+b_3):
//   psi(F) = mu/2 (tr F^T F - 3) - mu (J - 1) + lam/2 (J - 1)^2
//   P      = mu F + s cof F,                 s = lam (J - 1) - mu
//   g^e_a  = V P b_a
//   H^e_ac = V [ mu (b_a.b_c) I + lam u_a u_c^T - s [F (b_a x b_c)]_x ],  u_a = cof F b_a
// The last term is the contraction of d^2J/dF^2 with b_a and b_c; for a = c
// it vanishes and the diagonal block is symmetric.  One element per lane.
#include <hip/hip_runtime.h>

#include "k_common.h"
#include "topology.h"

namespace ppn {

__device__ inline void load_shape(const Dev& D, int e, double b[4][3]) {
  const int T = D.T;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) b[r + 1][c] = D.Bm[(3 * r + c) * T + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) b[0][c] = -(b[1][c] + b[2][c] + b[3][c]);
}

// F = sum_{a=1..3} (x_a - x_0) b_a^T
__device__ inline void def_grad(const double xs[4][3], const double b[4][3], double F[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double e1 = xs[1][i] - xs[0][i], e2 = xs[2][i] - xs[0][i], e3 = xs[3][i] - xs[0][i];
#pragma unroll
    for (int j = 0; j < 3; ++j) F[i][j] = e1 * b[1][j] + e2 * b[2][j] + e3 * b[3][j];
  }
}

// cof F: column j is f_{j+1} x f_{j+2}; returns J = det F.
__device__ inline double cofactor(const double F[3][3], double C[3][3]) {
  // columns f0 = F[.][0], f1 = F[.][1], f2 = F[.][2]
  C[0][0] = F[1][1] * F[2][2] - F[2][1] * F[1][2];
  C[1][0] = F[2][1] * F[0][2] - F[0][1] * F[2][2];
  C[2][0] = F[0][1] * F[1][2] - F[1][1] * F[0][2];
  C[0][1] = F[1][2] * F[2][0] - F[2][2] * F[1][0];
  C[1][1] = F[2][2] * F[0][0] - F[0][2] * F[2][0];
  C[2][1] = F[0][2] * F[1][0] - F[1][2] * F[0][0];
  C[0][2] = F[1][0] * F[2][1] - F[2][0] * F[1][1];
  C[1][2] = F[2][0] * F[0][1] - F[0][0] * F[2][1];
  C[2][2] = F[0][0] * F[1][1] - F[1][0] * F[0][1];
  return F[0][0] * C[0][0] + F[1][0] * C[1][0] + F[2][0] * C[2][0];
}

__device__ inline double snh_psi(const double F[3][3], double mu, double lam) {
  double C[3][3];
  const double J = cofactor(F, C);
  double ic = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) ic += F[i][j] * F[i][j];
  const double jm = J - 1.0;
  return 0.5 * mu * (ic - 3.0) - mu * jm + 0.5 * lam * jm * jm;
}

__device__ inline void load_corners(const Dev& D, const double* __restrict__ x, int e, int v[4],
                                    double xs[4][3]) {
  const int T = D.T;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    v[a] = D.tets[a * T + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) xs[a][i] = x[3 * v[a] + i];
  }
}

// ---------------------------------------------------------------- precompute
__global__ __launch_bounds__(kBlock) void k_precompute_elem(Dev D) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= D.T) return;
  int v[4];
  double xs[4][3];
  load_corners(D, D.X, e, v, xs);
  double Dm[3][3];  // columns X_a - X_0
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) Dm[i][a] = xs[a + 1][i] - xs[0][i];
  double C[3][3];
  const double det = cofactor(Dm, C);
  if (!(det > 0.0)) {
    atomicAdd(&D.flag[0], 1);
    return;
  }
  // Dm^-1 = cof(Dm)^T / det ; row r of Dm^-1 is column r of cof(Dm) / det
  const int T = D.T;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) D.Bm[(3 * r + c) * T + e] = C[c][r] / det;
  D.vol[e] = det / 6.0;
  const double E = D.Eyoung[e], nu = D.nu[e];
  const double mu_l = E / (2.0 * (1.0 + nu));
  const double lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  D.mu[e] = mu_l;
  D.lam[e] = lam_l + mu_l;
}

__global__ __launch_bounds__(kBlock) void k_precompute_mass(Dev D, double rho) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= D.N) return;
  double m = 0.0;
  for (int s = D.vptr[i]; s < D.vptr[i + 1]; ++s) m += rho * D.vol[D.vslot_elem[s]] / 4.0;
  D.mass[i] = m;
}

void launch_precompute(const Dev& D, double rho, hipStream_t st) {
  k_precompute_elem<<<(D.T + kBlock - 1) / kBlock, kBlock, 0, st>>>(D);
  k_precompute_mass<<<(D.N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, rho);
}

// ---------------------------------------------------------------- element evaluation
// Element e = w * kBlock + thread of a scene (w: the workgroup's index in the
// scene's range); also clears the element's projected flag for the iteration.
__device__ __forceinline__ void elem_eval_body(const Dev& D, int w) {
  const int e = w * kBlock + threadIdx.x;
  if (e >= D.T) return;
  const int T = D.T;
  D.proj[e] = 0;
  int v[4];
  double xs[4][3];
  load_corners(D, D.x, e, v, xs);
  double b[4][3];
  load_shape(D, e, b);
  double F[3][3];
  def_grad(xs, b, F);
  const double mu = D.mu[e], lam = D.lam[e], V = D.vol[e];
  double C[3][3];
  const double J = cofactor(F, C);
  const double s = lam * (J - 1.0) - mu;

  double u[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double ga[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double pg = 0.0, cu = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        pg += (mu * F[i][j] + s * C[i][j]) * b[a][j];
        cu += C[i][j] * b[a][j];
      }
      ga[i] = V * pg;
      u[a][i] = cu;
    }
    const double bb = b[a][0] * b[a][0] + b[a][1] * b[a][1] + b[a][2] * b[a][2];
    const double md = mu * bb;
    double* out = D.vslots + size_t(D.vslot[a * T + e]) * 9;
    out[0] = ga[0];
    out[1] = ga[1];
    out[2] = ga[2];
    out[3] = V * (md + lam * u[a][0] * u[a][0]);
    out[4] = V * (lam * u[a][0] * u[a][1]);
    out[5] = V * (lam * u[a][0] * u[a][2]);
    out[6] = V * (md + lam * u[a][1] * u[a][1]);
    out[7] = V * (lam * u[a][1] * u[a][2]);
    out[8] = V * (md + lam * u[a][2] * u[a][2]);
  }
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const int a = kPairA[p], c = kPairC[p];
    const double w0 = b[a][1] * b[c][2] - b[a][2] * b[c][1];
    const double w1 = b[a][2] * b[c][0] - b[a][0] * b[c][2];
    const double w2 = b[a][0] * b[c][1] - b[a][1] * b[c][0];
    const double y0 = F[0][0] * w0 + F[0][1] * w1 + F[0][2] * w2;
    const double y1 = F[1][0] * w0 + F[1][1] * w1 + F[1][2] * w2;
    const double y2 = F[2][0] * w0 + F[2][1] * w1 + F[2][2] * w2;
    const double md = mu * (b[a][0] * b[c][0] + b[a][1] * b[c][1] + b[a][2] * b[c][2]);
    double H[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) H[i][k] = lam * u[a][i] * u[c][k];
    H[0][0] += md;
    H[1][1] += md;
    H[2][2] += md;
    H[0][1] += s * y2;
    H[0][2] -= s * y1;
    H[1][0] -= s * y2;
    H[1][2] += s * y0;
    H[2][0] += s * y1;
    H[2][1] -= s * y0;
    double* out = D.eslots + size_t(D.eslot[p * T + e]) * 9;
    if (v[a] < v[c]) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) out[3 * i + k] = V * H[i][k];
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) out[3 * i + k] = V * H[k][i];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_elem_eval(const EvalJob* __restrict__ jobs, int n) {
  int w;
  const EvalJob& J = eval_job<0>(jobs, n, w);
  elem_eval_body(J.D, w);
}

int eval_wgs_elem(const Dev& D) { return ((D.T + kBlock - 1) / kBlock + 7) / 8 * 8; }
int eval_wgs_ls(const Dev& D) { return D.G; }

// ---------------------------------------------------------------- time integration helpers
__global__ __launch_bounds__(kBlock) void k_predict(Dev D) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= D.N) return;
  const double h = D.h;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double xi = D.x[3 * i + c];
    D.xn[3 * i + c] = xi;
    D.xhat[3 * i + c] = xi + h * D.v[3 * i + c] + h * h * D.grav[c];
  }
}

void launch_predict(const Dev& D, hipStream_t st) {
  k_predict<<<(D.N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D);
}

__global__ __launch_bounds__(kBlock) void k_axpy_x(Dev D, double gamma) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= 3 * D.N) return;
  D.x[k] += gamma * D.dx[k];
}

void launch_axpy_x(const Dev& D, double gamma, hipStream_t st) {
  k_axpy_x<<<(3 * D.N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D, gamma);
}

__global__ __launch_bounds__(kBlock) void k_finish_step(Dev D) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= 3 * D.N) return;
  D.v[k] = (D.x[k] - D.xn[k]) / D.h;
}

void launch_finish_step(const Dev& D, hipStream_t st) {
  k_finish_step<<<(3 * D.N + kBlock - 1) / kBlock, kBlock, 0, st>>>(D);
}

// ---------------------------------------------------------------- line-search energy difference
// Psi(x + gamma_k dx) - Psi(x), summed per term: per element V (psi(F_k) - psi(F_0)),
// per vertex m/(2h^2) s.(2(x - xhat) + s) and the penalty analogue, s = gamma_k dx.
// Workgroup wg of the scene's G: a contiguous share of its elements and vertices.
__device__ __forceinline__ void energy_diff_body(const Dev& D, int ng, const double* __restrict__ gam,
                                                 int wg) {
  __shared__ double lds[16];
  const int G = D.G;
  double g4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) g4[k] = k < ng ? gam[k] : 0.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int epw = (D.T + G - 1) / G;
  const int e0 = wg * epw, e1 = min(D.T, e0 + epw);
  for (int e = e0 + threadIdx.x; e < e1; e += kBlock) {
    int v[4];
    double xs[4][3], ds[4][3];
    load_corners(D, D.x, e, v, xs);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) ds[a][i] = D.dx[3 * v[a] + i];
    double b[4][3];
    load_shape(D, e, b);
    const double mu = D.mu[e], lam = D.lam[e], V = D.vol[e];
    double F[3][3];
    def_grad(xs, b, F);
    const double p0 = snh_psi(F, mu, lam);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < ng) {
        double xk[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i) xk[a][i] = xs[a][i] + g4[k] * ds[a][i];
        def_grad(xk, b, F);
        acc[k] += V * (snh_psi(F, mu, lam) - p0);
      }
    }
  }
  const int vpw = (D.N + G - 1) / G;
  const int i0 = wg * vpw, i1 = min(D.N, i0 + vpw);
  const double ih2 = 1.0 / (D.h * D.h);
  for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const double m = 0.5 * D.mass[i] * ih2;
    const int di = D.dir_idx[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < ng) {
        double t = 0.0, p = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double s = g4[k] * D.dx[3 * i + c];
          const double xi = D.x[3 * i + c];
          t += s * (2.0 * (xi - D.xhat[3 * i + c]) + s);
          if (di >= 0) p += s * (2.0 * (xi - D.xbar[3 * di + c]) + s);
        }
        acc[k] += m * t + 0.5 * D.k_dir * p;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double s = block_sum(acc[k], lds);
    if (threadIdx.x == 0) D.part[(kPartA + k) * G + wg] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_energy_diff(const EvalJob* __restrict__ jobs, int n) {
  int w;
  const EvalJob& J = eval_job<3>(jobs, n, w);
  energy_diff_body(J.D, J.n_gamma, J.gamma, w);
}

void launch_energy_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st) {
  if (n <= 0) return;
  k_energy_diff<<<gr.ls, kBlock, 0, st>>>(jobs, n);
  launch_reduce_jobs(jobs, n, kPartA, 4, 0, st);
}

void launch_elem_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st) {
  if (n <= 0) return;
  k_elem_eval<<<gr.elem, kBlock, 0, st>>>(jobs, n);
}

}  // namespace ppn
