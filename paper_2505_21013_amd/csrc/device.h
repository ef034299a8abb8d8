// Device-side data of one scene and the launchers of the hot-path kernels.
//
// Layout in HBM (all FP64 unless noted):
//   element data   SoA [k][T]: tets (int32, 4), Dm^-1 rows (9), V, mu, lam
//   vertex vectors AoS [N][3]: x, x^n, v, xhat, g, dx, r, q; PCG (z, d) records [2][N][6]
//   vertex slots   AoS [4T][9]: corner gradient (3) + diagonal block (6)
//   edge slots     AoS [6T][9]: off-diagonal block, row-major, global orientation
//   matrix         the symmetric 3x3 block matrix stored once (half storage,
//                  topology.h): each row owns its diagonal and upper blocks, in
//                  sliced ELL (rows in groups of 64, one wavefront; slot-major,
//                  half slot k of group g is block row k*n_groups + g); per block
//                  row the 64 rows' blocks as four entry pairs [4][64][2] and
//                  entry 8 [64] (value_index).  The product walks the full
//                  pattern (column and value reference per slot, lower blocks
//                  read transposed from their column's row)
//   block-Jacobi   SoA [6][N]: inverse of each diagonal block (symmetric: upper triangle)
//   mixed precision (only when requested): FP32 copies of the sliced-ELL
//                  values and of the block-Jacobi inverse, three more [N][3]
//                  vectors for the inner solve (correction, residual, H d)
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ppn {

constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels

// Partial-sum slots (each G doubles long) in Dev::part.
enum PartSlot : int {
  kPartKappa = 0,  // d^T H d
  kPartRR = 1,     // r^T r
  kPartRZ0 = 2,    // r^T z, even iterations
  kPartRZ1 = 3,    // r^T z, odd iterations
  kPartSpd = 4,    // count of diagonal blocks failing Sylvester's criterion
  kPartG2 = 5,     // |g|^2
  kPartGmax = 6,   // max |g_i|
  kPartA = 7,      // generic scratch sums (line search uses 7..7+4)
  kPartCount = 12
};

struct PcgState {
  int32_t done;
  int32_t ind;
  int32_t iters;
  int32_t j_rr;    // iteration of the last product that went on (-1 before the first)
  double rr0;      // r0^T r0
  double rz[2];    // r_j^T z_j by iteration parity (beta of the next direction, alpha)
  double rr;       // r^T r at iteration j_rr (the host sizes its launch chunks from it)
};

// Matrix (type M: FP64, or FP32 in the mixed-precision path) and FP64
// vectors of one PCG solve.
template <typename M>
struct PcgVec {
  const M* vals = nullptr;    // sliced-ELL values
  const M* pinv = nullptr;    // [6][N] block-Jacobi inverse (symmetric, upper triangle)
  double* zd = nullptr;       // [N][6] (z, previous d) records; for M = float, z alone as [N][3]
  float* zd32 = nullptr;      // [N][6] (M = float only) the records rounded to FP32, which the
                              // FP32 product gathers
  double* dn = nullptr;       // [N][3] new direction
  double* r = nullptr;        // [N][3] residual
  double* q = nullptr;        // [N][3] H d
  double* x = nullptr;        // [N][3] solution
};

struct EvalJob;

struct Dev {
  int32_t N = 0, T = 0, E = 0;
  int64_t NB = 0;
  int32_t G = 0;          // workgroups of the assembly / reduction kernels (fixed per scene)
  int32_t rows_per_wg = 0;  // vertex chunk per workgroup of those kernels
  int32_t Gp = 0;         // workgroups of the PCG kernels (multiple of 8; 256 rows each)
  int32_t spmv_panel = 0; // panel length of the cache-resident product's workgroup order (0: none)
  int32_t pcg_load = -1;  // load mode of the PCG product (kLoad*), -1: chosen from the size
  int32_t n_groups = 0;   // 64-row groups of the sliced-ELL matrix
  int64_t n_slots = 0;    // smax * n_groups (slot-major block rows of the full pattern)
  int64_t n_hslots = 0;   // block rows of the half storage (hsmax * n_groups + 1)
  int32_t by_distance = 0;  // slots ordered by distance (large matrices), else CSR order
  int32_t f32_full = 0;     // the mixed form's FP32 copy is in the full layout (CSR-ordered
                            // matrices), read with col32; else it mirrors the half storage
  int32_t nD = 0;         // Dirichlet vertices
  double h = 1.0 / 30.0;
  double k_dir = 1e8;
  double grav[3] = {0, 0, -9.81};

  // mesh
  int32_t* tets = nullptr;  // [4][T]
  double* Bm = nullptr;     // [9][T]
  double* vol = nullptr;    // [T]
  double* mu = nullptr;     // [T]
  double* lam = nullptr;    // [T]
  double* Eyoung = nullptr; // [T]
  double* nu = nullptr;     // [T]
  double* mass = nullptr;   // [N]
  double* X = nullptr;      // [N][3]
  // maps
  int32_t* vslot = nullptr;      // [4][T]
  int32_t* eslot = nullptr;      // [6][T]
  int32_t* elem_edge = nullptr;  // [6][T]
  int32_t* vptr = nullptr;       // [N+1]
  int32_t* vslot_elem = nullptr; // [4T]
  int32_t* eptr = nullptr;       // [E+1]
  int32_t* gslots = nullptr;     // [n_groups] slots of each 64-row group
  int32_t* colref = nullptr;     // [n_slots * 64][2] per (slot, lane): column, and value
                                 // reference (half position | kRefTranspose for a lower block)
  int32_t* diag_blk = nullptr;   // [N] half position of the diagonal block
  int32_t* eblk_up = nullptr;    // [E] half position of the edge block (lo, hi)
  // slots and matrix
  double* vslots = nullptr;  // [4T][9]
  double* eslots = nullptr;  // [6T][9]
  double* vals = nullptr;    // [n_hslots * 9 * 64] half storage, entries at value_index()
  double* pinv = nullptr;    // [6][N] upper triangle of the symmetric inverse
  uint8_t* spd_ok = nullptr; // [N]
  // Dirichlet
  int32_t* dir_idx = nullptr;  // [N], -1 if free
  double* xbar = nullptr;      // [nD][3]
  // vectors [N][3]
  double *x = nullptr, *xn = nullptr, *v = nullptr, *xhat = nullptr, *g = nullptr, *dx = nullptr;
  double *r = nullptr, *q = nullptr, *xt = nullptr;
  double* zd = nullptr;    // [N][6]: (z, previous d) records of the PCG
  float* zd32 = nullptr;   // [N][6]: the same rounded to FP32 (mixed form)
  double* dn = nullptr;    // [N][3]: the PCG's new direction
  double* rinf = nullptr;  // [N]
  // mixed precision (null in FP64 scenes)
  float* vals32 = nullptr;  // FP32 matrix: full layout [n_slots * 9 * 64] (f32_full) or the half
                            // storage's [n_hslots * 9 * 64]; per block row four [64] float2 entry
                            // pairs (0,1) (2,3) (4,5) (6,7), then entry 8 as [64] float
  int32_t* col32 = nullptr; // [n_slots * 64] columns of the full-layout FP32 product (f32_full)
                            // (0,1) (2,3) (4,5) (6,7), then entry 8 as [64] float
  float* pinv32 = nullptr;  // [6][N]
  double* e = nullptr;      // [N][3] correction of one refinement round
  double* ri = nullptr;     // [N][3] residual of the inner solve
  double* qi = nullptr;     // [N][3] H d of the inner solve
  // selection
  uint8_t* proj = nullptr;  // [T]
  uint8_t* sel = nullptr;   // [T]
  int32_t* list = nullptr;  // [T]
  int32_t* sel_cnt = nullptr;  // [n_sel_wg + 1]
  int32_t n_sel_wg = 0;
  // reductions and control
  double* part = nullptr;   // [kPartCount][G]
  double* scal = nullptr;   // [16] final reduced values
  PcgState* pcg = nullptr;
  int32_t* flag = nullptr;  // [4] misc device flags (bad element count, ...)
  EvalJob* job = nullptr;   // [1] this scene's own table for the evaluation kernels
};

// One scene's share of a shared launch of the evaluation kernels (element
// quantities, assembly, norm reduction) or of the line-search energy kernel.
// Every kernel of these phases takes a table of jobs: workgroup b finds the job
// whose range [wg, wg + count) holds it and runs that scene's code with the
// local index b - wg.  The ranges start at multiples of 8, so that a scene's
// workgroups meet the same XCDs as when it runs alone.  A single scene runs the
// same kernels with a table of one job, so its results are the same bit for
// bit whether or not it shares a launch.
struct EvalJob {
  Dev D;
  int32_t wg_elem, wg_vert, wg_edge, wg_ls;  // first workgroup in each kernel's grid
  int32_t n_gamma, pad;
  double gamma[4];                           // line-search step sizes
};
// Workgroups of one scene in each kernel (multiples of 8).
int eval_wgs_elem(const Dev& D);
int eval_wgs_vert(const Dev& D);
int eval_wgs_edge(const Dev& D);
int eval_wgs_ls(const Dev& D);
// Sums of the above over a table (host side), and the table offsets set in place.
struct EvalGrid {
  int elem = 0, vert = 0, edge = 0, ls = 0;
};
EvalGrid layout_eval_jobs(EvalJob* jobs, int n);

// Index of entry e (row-major 3x3) of the sliced-ELL block at position
// pos = slot * 64 + lane, in 64-bit arithmetic.  Per slot the 64 lanes'
// blocks take 9 * 64 values: entries (0,1) (2,3) (4,5) (6,7) as pairs,
// [4][64][2], then entry 8 as [64]; a lane reads its block with four 16-byte
// loads and one 8-byte load, each one contiguous run over the wavefront.
__host__ __device__ inline size_t value_index(int32_t pos, int e) {
  const size_t base = size_t(pos >> 6) * (9 * 64);
  const size_t lane = size_t(pos & 63);
  return e < 8 ? base + size_t(e >> 1) * 128 + 2 * lane + size_t(e & 1) : base + 512 + lane;
}

// Bytes of the FP64 matrix values (half storage: 9 entries of 64 rows per half slot).
inline int64_t matrix_bytes(const Dev& D) { return D.n_hslots * 9 * 64 * int64_t(sizeof(double)); }
// Bytes of the mixed form's FP32 copy (9 entries of 64 rows per block row).
inline int64_t matrix_bytes_f32(const Dev& D) {
  return (D.f32_full ? D.n_slots : D.n_hslots) * 9 * 64 * int64_t(sizeof(float));
}

// Load modes of the PCG product, chosen per launch from the size of the matrix
// values (FP64, or the FP32 copy; summed over the jobs of a batched launch).
// None changes the arithmetic or its order.
//  * kLoadSmall, up to 64 MB: ordinary loads; few workgroups, all resident.
//  * kLoadCached, above 64 MB: ordinary loads, and a single scene's product
//    keeps at most 3 workgroups resident per CU (the FP64 product runs its
//    workgroups in panel order, wg_order.h), so that the transposed read of a
//    stored block meets its owner's read in the L2 (k_pcg.hip).  It is the
//    mode at every size above 64 MB, also far beyond the 256 MB last-level
//    cache: on the 128^3 cube (FP64 values 1.07 GB) the FP64 product took
//    532.7 us this way against 620.9 us with non-temporal loads (469 us with
//    the panel order), the FP32 one 375.8 against 427.4 us.
//  * kLoadStream, only when forced (ppn_params.pcg_load_mode = 2): non-temporal
//    loads, no cap.  With the matrix stored whole it was the better mode above
//    224 MB (101 against 91 us per FP64 iteration on the 64^3 cube, 297 MB of
//    values); with half storage a streamed block is fetched from HBM twice,
//    by its owner row and by its partner row.
constexpr int kLoadSmall = 0, kLoadCached = 1, kLoadStream = 2;
constexpr int64_t kSmallMatrixBytes = int64_t(64) << 20;
inline int load_mode(int64_t bytes) { return bytes > kSmallMatrixBytes ? kLoadCached : kLoadSmall; }

// ---- launchers (all asynchronous on `st`) --------------------------------
void launch_precompute(const Dev& D, double rho, hipStream_t st);
void launch_predict(const Dev& D, hipStream_t st);
// Evaluation at the current x for the jobs of a table (device memory): the
// element kernel (which also clears the projected flags), the vertex and edge
// assembly passes and the reduction of |g|_2^2 and |g|_inf into each scene's
// scal[0..1].
void launch_evaluate_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st);
// Re-assembly only (vertex and edge passes) of the jobs' matrices and gradients.
void launch_assemble_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st);
// Psi(x + gamma_k dx) - Psi(x) for each job's n_gamma step sizes into its scal[0..3].
void launch_energy_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st);
void launch_elem_jobs(const EvalJob* jobs, int n, const EvalGrid& gr, hipStream_t st);
// k_reduce of every job's partial slots into its scal (one workgroup per job).
void launch_reduce_jobs(const EvalJob* jobs, int n, int first_slot, int n_sum, int n_max, hipStream_t st);
void launch_reduce(const Dev& D, int first_slot, int n_sum, int n_max, hipStream_t st);
// The same over partials written with the PCG grid's stride (Gp).
void launch_reduce_pcg(const Dev& D, int first_slot, int n_sum, hipStream_t st);
void launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st);
void launch_select_count(const Dev& D, double delta, int fallback, hipStream_t st);
void launch_select_write(const Dev& D, hipStream_t st);
// mirror = 0: eigenvalues clamped to max(lambda, eps); 1: max(|lambda|, eps).
void launch_eig_all(const Dev& D, double eps, int mirror, hipStream_t st);
void launch_eig_list(const Dev& D, int32_t n, double eps, int mirror, hipStream_t st);
// FP32 eigensolves (mixed precision); the slots stay FP64.
void launch_eig_all_f32(const Dev& D, double eps, int mirror, hipStream_t st);
void launch_eig_list_f32(const Dev& D, int32_t n, double eps, int mirror, hipStream_t st);
void launch_regather_list(const Dev& D, int32_t n, hipStream_t st);
void launch_project_batch(const double* H, double* out, int64_t n, double eps, hipStream_t st);
// Sets *bad (device memory) if a dense 12x12 matrix is not symmetric or
// does not annihilate the rigid translations, up to rtol of its largest entry.
void launch_check_dense(const double* H, int64_t n, double rtol, int32_t* bad, hipStream_t st);
// r = sign * src (FP64 source), x = 0, first preconditioned residual.
void launch_pcg_init(const Dev& D, const PcgVec<double>& V, const double* src, double sign,
                     hipStream_t st);
void launch_pcg_init(const Dev& D, const PcgVec<float>& V, const double* src, double sign,
                     hipStream_t st);
void launch_pcg_iter(const Dev& D, const PcgVec<double>& V, int j, double tol2, int maxit,
                     hipStream_t st, hipEvent_t ev_spmv_start = nullptr,
                     hipEvent_t ev_spmv_stop = nullptr);
void launch_pcg_iter(const Dev& D, const PcgVec<float>& V, int j, double tol2, int maxit,
                     hipStream_t st, hipEvent_t ev_spmv_start = nullptr,
                     hipEvent_t ev_spmv_stop = nullptr);
// One PCG solve of a batch (see the batched launchers below).
template <typename M>
struct PcgJob {
  Dev D;
  PcgVec<M> V;
  const double* src;  // right-hand side = sign * src
  double sign;
  double tol2;        // rtol^2
  int32_t maxit;
  int32_t wg0;        // first global workgroup of this job; jobs sorted by wg0
  int32_t j0;         // batch iteration at which this job's solve started
  int32_t pad;
};
// Batched solves: n jobs, total_wg = sum of their Gp; every launch covers all
// jobs and a finished job's workgroups return at once.  Iteration j of the
// batch is iteration j - j0 of each job.
void launch_pcg_batch_init(const PcgJob<double>* jobs, int n, int total_wg, hipStream_t st);
void launch_pcg_batch_init(const PcgJob<float>* jobs, int n, int total_wg, hipStream_t st);
// any_first: some job starts at this iteration (its first product is a
// separate instance, launched only then).  matrix_bytes: the summed size of
// the matrix values the jobs read (matrix_bytes, or matrix_bytes_f32 for the
// FP32 copies; selects the load mode).
void launch_pcg_batch_iter(const PcgJob<double>* jobs, int n, int total_wg, int j, bool any_first,
                           int64_t matrix_bytes, hipStream_t st);
void launch_pcg_batch_iter(const PcgJob<float>* jobs, int n, int total_wg, int j, bool any_first,
                           int64_t matrix_bytes, hipStream_t st);
void launch_pcg_batch_gather(const PcgJob<double>* jobs, int n, PcgState* out, hipStream_t st);
void launch_pcg_batch_gather(const PcgJob<float>* jobs, int n, PcgState* out, hipStream_t st);
void launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st);
// The mixed form's FP32 copy of the matrix: in the full sliced-ELL layout
// (each slot's block at its own position, lower blocks transposed) when
// D.f32_full, else entry by entry in the half storage's layout.
void launch_matrix_to_f32(const Dev& D, hipStream_t st);
void launch_refine_init(const Dev& D, hipStream_t st);      // dx = 0, r = -g, |r|^2 partials
void launch_refine_add(const Dev& D, const double* e, hipStream_t st);  // dx += e
void launch_refine_residual(const Dev& D, hipStream_t st);  // r = -g - H dx, |r|^2 partials
void launch_dx_stats(const Dev& D, hipStream_t st);  // |dx|_inf, g.dx -> scal[0..1]
void launch_safety_dir(const Dev& D, hipStream_t st);
void launch_rinf_from(const Dev& D, const double* g, hipStream_t st);  // rinf_i = max_c |g_(i,c)|
void launch_axpy_x(const Dev& D, double gamma, hipStream_t st);
void launch_finish_step(const Dev& D, hipStream_t st);
void launch_spmv_plain(const Dev& D, const double* d, double* q, hipStream_t st);
void launch_element_hessians(const Dev& D, const int32_t* ids, int32_t n, double* out,
                             hipStream_t st);

}  // namespace ppn
