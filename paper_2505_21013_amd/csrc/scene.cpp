// Host orchestration of one time step: PN, PDN and PPN (Algorithm 1) over the
// device kernels.  The host only reads back the scalars that decide the
// control flow (gradient norms, solve status, selection count, line-search
// energies); every vector and matrix operation runs in the kernels.
#include "scene.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>

namespace ppn {

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess)                                                                      \
      throw HipError{std::string(#x) + ": " + hipGetErrorString(e_),                           \
                     e_ == hipErrorOutOfMemory ? PPN_ERR_OOM : PPN_ERR_DEVICE};                \
  } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

static void fail(const std::string& m, ppn_status c = PPN_ERR_ARG) { throw HipError{m, c}; }

// Every kProfileEvery-th PCG matrix product is bracketed by timing events when
// profiling is on (sampling keeps the events from perturbing the launch stream).
constexpr int kProfileEvery = 16;

// Size of the next chunk of PCG iterations to enqueue (from iteration jend on)
// after reading the state of the chunk before the one in flight.  The device
// takes every stop decision; launches past it return at once, so the chunk
// size only trades such empty launches against host round trips.  Once two
// residuals are known (r0 and the last one read), the decay per iteration
// between them predicts where |r| meets the tolerance; the chunk ends there
// plus kChunkMargin iterations (at least kChunkMin, at most kChunkMax).
// Without a prediction (the residual grew, or none yet) chunks double.
constexpr int kChunkMin = 4, kChunkMax = 32, kChunkMargin = 2;
static int next_chunk(const PcgState& S, double tol2, int jend, int chunk, int& j_prev,
                      double& rr_prev) {
  int next = std::min(2 * chunk, kChunkMax);
  if (S.j_rr < 0 || !(S.rr > 0.0) || !(S.rr0 > 0.0)) return next;
  if (j_prev < 0) {
    j_prev = 0;
    rr_prev = S.rr0;
  }
  if (S.j_rr > j_prev && S.rr < rr_prev) {
    const double lr = std::log(S.rr / rr_prev) / double(S.j_rr - j_prev);
    const double rem = std::log(tol2 * S.rr0 / S.rr) / lr;  // iterations after j_rr
    if (std::isfinite(rem)) {
      const double target = double(S.j_rr) + std::max(rem, 0.0) + kChunkMargin;
      next = int(std::min<double>(kChunkMax, std::max<double>(kChunkMin, std::ceil(target) - jend)));
    }
  }
  if (S.j_rr > j_prev) {
    j_prev = S.j_rr;
    rr_prev = S.rr;
  }
  return next;
}

void params_defaults(ppn_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->alpha = 0.5;
  p->beta = 2.0;
  p->eps_delta = 1e-12;
  p->eps_clamp = 1e-8;
  p->pcg_rtol = 1e-4;
  p->pcg_maxit = 10000;
  p->pdn_countdown = 4;
  p->stop_mode = PPN_STOP_VEL;
  p->newton_maxit = 100;
  p->stop_tol = 1e-3;
  p->armijo_c = 1e-4;
  p->ls_maxit = 30;
  p->k_dirichlet = 1e8;
  p->pcg_load_mode = -1;
  p->use_graphs = 1;
}

Scene::Scene(hipStream_t stream, bool own, int precision)
    : st_(stream), own_stream_(own), precision_(precision) {
  params_defaults(&prm_);
  HIPCHK(hipGetDevice(&device_));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hscal_), 64 * sizeof(double)));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hpcg_), 4 * sizeof(PcgState)));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hint_), 16 * sizeof(int32_t)));
  HIPCHK(hipEventCreateWithFlags(&ev_[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev_[1], hipEventDisableTiming));
  HIPCHK(hipEventCreate(&ev_[2]));
  HIPCHK(hipEventCreate(&ev_[3]));
}

Scene::~Scene() {
  if (st_) (void)hipStreamSynchronize(st_);
  free_all();
  if (hscal_) (void)hipHostFree(hscal_);
  if (hpcg_) (void)hipHostFree(hpcg_);
  if (hint_) (void)hipHostFree(hint_);
  for (auto& e : ev_)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : prof_ev_) (void)hipEventDestroy(e);
  if (own_stream_ && st_) (void)hipStreamDestroy(st_);
}

template <class T>
T* Scene::alloc(size_t n) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) fail("hipMalloc of " + std::to_string(bytes) + " bytes failed", PPN_ERR_OOM);
  allocs_.push_back(p);
  dev_bytes_ += int64_t(bytes);
  return static_cast<T*>(p);
}

void Scene::free_all() {
  if (eval_graph_) (void)hipGraphExecDestroy(eval_graph_);
  eval_graph_ = nullptr;
  job_valid_ = false;
  for (void* p : allocs_) (void)hipFree(p);
  allocs_.clear();
  dev_bytes_ = 0;
  D_ = Dev{};
}

void Scene::sync() { HIPCHK(hipStreamSynchronize(st_)); }

void Scene::read_scal(int n, double* out) {
  HIPCHK(hipMemcpyAsync(out, D_.scal, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
}

// ---------------------------------------------------------------- set-up
// Launch geometry of a scene from its topology.
static void geometry(Dev& D, const Topology& t) {
  const int N = t.n_verts, T = t.n_tets;
  D.N = N;
  D.T = T;
  D.E = t.n_edges;
  D.NB = t.n_blocks;
  int G = (N + 127) / 128;
  G = std::min(2048, std::max(8, ((G + 7) / 8) * 8));
  D.G = G;
  D.rows_per_wg = (((N + G - 1) / G) + 15) / 16 * 16;
  D.n_sel_wg = (T + kBlock - 1) / kBlock;
  // PCG kernels: one row per thread, one 64-row group per wavefront, four
  // groups per 256-thread workgroup, a multiple of 8 workgroups (one per XCD).
  D.n_groups = t.n_groups;
  D.n_slots = t.n_slots;
  D.n_hslots = t.n_hslots;
  D.by_distance = t.by_distance ? 1 : 0;
  D.f32_full = t.by_distance ? 0 : 1;
  D.Gp = ((D.n_groups + 3) / 4 + 7) / 8 * 8;
  // Panel length of the product's workgroup order (k_common.h panel_order):
  // the median over rows of the distance to the farthest lower column, in
  // 256-row workgroups, so that a row and its farthest partners run together.
  std::vector<int32_t> far;
  far.reserve(size_t(N));
  for (int32_t i = 0; i < N; ++i)
    if (t.row_ptr[i + 1] > t.row_ptr[i] && t.col[t.row_ptr[i]] < i) far.push_back(i - t.col[t.row_ptr[i]]);
  D.spmv_panel = 0;
  if (!far.empty()) {
    std::nth_element(far.begin(), far.begin() + far.size() / 2, far.end());
    const int32_t p = (far[far.size() / 2] + 128) / 256;
    D.spmv_panel = p >= 2 ? p : 0;
  }
}

// Every device buffer of a scene, in one place.  A::get<T>(count) either
// allocates or only counts the bytes (footprint()).
template <class A>
static void plan_buffers(Dev& D, int precision, A& alloc) {
  const size_t n = size_t(D.N), m = size_t(D.T);
  D.tets = alloc.template get<int32_t>(4 * m);
  D.Bm = alloc.template get<double>(9 * m);
  D.vol = alloc.template get<double>(m);
  D.mu = alloc.template get<double>(m);
  D.lam = alloc.template get<double>(m);
  D.Eyoung = alloc.template get<double>(m);
  D.nu = alloc.template get<double>(m);
  D.mass = alloc.template get<double>(n);
  D.X = alloc.template get<double>(3 * n);
  D.vslot = alloc.template get<int32_t>(4 * m);
  D.eslot = alloc.template get<int32_t>(6 * m);
  D.elem_edge = alloc.template get<int32_t>(6 * m);
  D.vptr = alloc.template get<int32_t>(n + 1);
  D.vslot_elem = alloc.template get<int32_t>(4 * m);
  D.eptr = alloc.template get<int32_t>(size_t(D.E) + 1);
  D.gslots = alloc.template get<int32_t>(size_t(D.n_groups));
  D.colref = alloc.template get<int32_t>(size_t(D.n_slots) * kSell * 2);
  D.diag_blk = alloc.template get<int32_t>(n);
  D.eblk_up = alloc.template get<int32_t>(size_t(D.E));
  D.vslots = alloc.template get<double>(4 * m * 9);
  D.eslots = alloc.template get<double>(6 * m * 9);
  D.vals = alloc.template get<double>(size_t(D.n_hslots) * 9 * kSell);
  D.pinv = alloc.template get<double>(6 * n);
  D.spd_ok = alloc.template get<uint8_t>(n);
  D.dir_idx = alloc.template get<int32_t>(n);
  D.xbar = alloc.template get<double>(3 * n);
  double** vecs[] = {&D.x, &D.xn, &D.v, &D.xhat, &D.g, &D.dx, &D.r, &D.q, &D.xt};
  for (double** p : vecs) *p = alloc.template get<double>(3 * n);
  D.zd = alloc.template get<double>(6 * n);
  D.dn = alloc.template get<double>(3 * n);
  D.rinf = alloc.template get<double>(n);
  if (precision == PPN_MIXED) {
    D.vals32 = alloc.template get<float>(size_t(D.f32_full ? D.n_slots : D.n_hslots) * 9 * kSell);
    if (D.f32_full) D.col32 = alloc.template get<int32_t>(size_t(D.n_slots) * kSell);
    D.pinv32 = alloc.template get<float>(6 * n);
    D.zd32 = alloc.template get<float>(6 * n);
    D.e = alloc.template get<double>(3 * n);
    D.ri = alloc.template get<double>(3 * n);
    D.qi = alloc.template get<double>(3 * n);
  }
  D.proj = alloc.template get<uint8_t>(m);
  D.sel = alloc.template get<uint8_t>(m);
  D.list = alloc.template get<int32_t>(m);
  D.sel_cnt = alloc.template get<int32_t>(size_t(D.n_sel_wg) + 1);
  D.part = alloc.template get<double>(size_t(kPartCount) * std::max(D.G, D.Gp));
  D.scal = alloc.template get<double>(16);
  D.pcg = alloc.template get<PcgState>(1);
  D.job = alloc.template get<EvalJob>(1);
  D.flag = alloc.template get<int32_t>(4);
}

struct CountBytes {
  int64_t bytes = 0;
  template <class T>
  T* get(size_t n) {
    bytes += int64_t(std::max<size_t>(n, 1) * sizeof(T));
    return nullptr;
  }
};

struct DeviceAlloc {
  Scene* s;
  template <class T>
  T* get(size_t n) { return s->alloc<T>(n); }
};

int64_t Scene::footprint(const Topology& t, int precision) {
  Dev D;
  geometry(D, t);
  CountBytes c;
  plan_buffers(D, precision, c);
  return c.bytes;
}

void Scene::load_mesh(int32_t N, const double* rest, int32_t T, const int32_t* tets,
                      const double* init) {
  if (!rest || !tets) fail("rest_xyz and tets must not be NULL");
  Topology t;
  std::string err;
  if (!build_topology(N, T, tets, t, err)) fail(err, PPN_ERR_MESH);
  load_mesh(std::move(t), rest, tets, init);
}

void Scene::load_mesh(Topology&& t, const double* rest, const int32_t* tets, const double* init) {
  if (!rest || !tets) fail("rest_xyz and tets must not be NULL");
  if (loaded()) {
    sync();
    free_all();
  }
  topo_ = std::move(t);
  const int32_t N = topo_.n_verts, T = topo_.n_tets;
  try {
    Dev D;
    geometry(D, topo_);
    D.h = D_.h;
    D.k_dir = prm_.k_dirichlet;
    D.pcg_load = prm_.pcg_load_mode;
    std::memcpy(D.grav, D_.grav, sizeof(D.grav));
    D_ = D;
    const size_t n = size_t(N), m = size_t(T);
    DeviceAlloc da{this};
    plan_buffers(D_, precision_, da);
    if (dev_bytes_ != footprint(topo_, precision_)) fail("internal: footprint mismatch", PPN_ERR_DEVICE);
    {
      EvalJob e;
      std::memset(static_cast<void*>(&e), 0, sizeof(e));
      e.D = D_;
      grid_ = layout_eval_jobs(&e, 1);
    }

    std::vector<int32_t> soa(4 * m);
    for (size_t e = 0; e < m; ++e)
      for (int a = 0; a < 4; ++a) soa[a * m + e] = tets[4 * e + a];
    auto up = [&](void* dst, const void* src, size_t bytes) {
      HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_));
    };
    up(D_.tets, soa.data(), 4 * m * 4);
    up(D_.X, rest, 3 * n * 8);
    up(D_.x, init ? init : rest, 3 * n * 8);
    HIPCHK(hipMemsetAsync(D_.v, 0, 3 * n * 8, st_));
    up(D_.vslot, topo_.vslot.data(), 4 * m * 4);
    up(D_.eslot, topo_.eslot.data(), 6 * m * 4);
    up(D_.elem_edge, topo_.elem_edge.data(), 6 * m * 4);
    up(D_.vptr, topo_.vptr.data(), (n + 1) * 4);
    up(D_.vslot_elem, topo_.vslot_elem.data(), 4 * m * 4);
    up(D_.eptr, topo_.eptr.data(), (size_t(D_.E) + 1) * 4);
    up(D_.gslots, topo_.gslots.data(), size_t(D_.n_groups) * 4);
    std::vector<int32_t> colref(2 * size_t(D_.n_slots) * kSell);
    for (size_t k = 0; k < size_t(D_.n_slots) * kSell; ++k) {
      colref[2 * k] = topo_.sell_col[k];
      colref[2 * k + 1] = topo_.sell_ref[k];
    }
    up(D_.colref, colref.data(), colref.size() * 4);
    if (D_.col32) up(D_.col32, topo_.sell_col.data(), size_t(D_.n_slots) * kSell * 4);
    up(D_.diag_blk, topo_.diag_pos.data(), n * 4);
    up(D_.eblk_up, topo_.edge_pos.data(), size_t(D_.E) * 4);
    // padding blocks and the zero row of the half storage stay zero for the life of the scene
    HIPCHK(hipMemsetAsync(D_.vals, 0, size_t(D_.n_hslots) * 9 * kSell * 8, st_));
    X_.assign(rest, rest + 3 * n);
    if (E_.size() != m) {
      const double e0 = E_.empty() ? 1e5 : E_[0], n0 = nu_.empty() ? 0.45 : nu_[0];
      E_.assign(m, e0);
      nu_.assign(m, n0);
    }
    dir_ids_.clear();
    dir_tgt_.clear();
    dirichlet_dirty_ = true;
    upload_dirichlet();
    material_dirty_ = true;
    upload_material();
    sync();
  } catch (...) {
    (void)hipStreamSynchronize(st_);
    free_all();
    throw;
  }
}

void Scene::upload_material() {
  if (!loaded() || !material_dirty_) return;
  const size_t m = size_t(D_.T);
  HIPCHK(hipMemcpyAsync(D_.Eyoung, E_.data(), m * 8, hipMemcpyHostToDevice, st_));
  HIPCHK(hipMemcpyAsync(D_.nu, nu_.data(), m * 8, hipMemcpyHostToDevice, st_));
  HIPCHK(hipMemsetAsync(D_.flag, 0, 4 * sizeof(int32_t), st_));
  launch_precompute(D_, rho_, st_);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(hint_, D_.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
  sync();
  if (hint_[0] != 0)
    fail(std::to_string(hint_[0]) + " rest tetrahedra have det(Dm) <= 0", PPN_ERR_MESH);
  material_dirty_ = false;
}

void Scene::set_material(double rho, const double* E, const double* nu, bool per_element) {
  if (!(rho > 0.0) || !E || !nu) fail("rho must be > 0 and E, nu non-NULL");
  if (per_element && !loaded()) fail("per-element material needs a loaded mesh");
  const size_t m = per_element ? size_t(D_.T) : 1;
  for (size_t k = 0; k < m; ++k)
    if (!(E[k] >= 0.0) || !(nu[k] >= 0.0 && nu[k] < 0.5)) fail("need E >= 0 and 0 <= nu < 0.5");
  rho_ = rho;
  const size_t T = loaded() ? size_t(D_.T) : 1;
  E_.resize(T);
  nu_.resize(T);
  for (size_t e = 0; e < T; ++e) {
    E_[e] = per_element ? E[e] : E[0];
    nu_[e] = per_element ? nu[e] : nu[0];
  }
  material_dirty_ = true;
  if (loaded()) upload_material();
}

void Scene::set_time_step(double dt, const double* gravity) {
  if (!(dt > 0.0) || !std::isfinite(dt)) fail("dt must be finite and > 0");
  D_.h = dt;
  if (gravity)
    for (int c = 0; c < 3; ++c) D_.grav[c] = gravity[c];
}

void Scene::upload_dirichlet() {
  if (!loaded() || !dirichlet_dirty_) return;
  const int32_t N = D_.N;
  std::vector<int32_t> idx(N, -1);
  for (size_t k = 0; k < dir_ids_.size(); ++k) idx[dir_ids_[k]] = int32_t(k);
  HIPCHK(hipMemcpyAsync(D_.dir_idx, idx.data(), size_t(N) * 4, hipMemcpyHostToDevice, st_));
  if (!dir_tgt_.empty())
    HIPCHK(hipMemcpyAsync(D_.xbar, dir_tgt_.data(), dir_tgt_.size() * 8, hipMemcpyHostToDevice, st_));
  D_.nD = int32_t(dir_ids_.size());
  sync();
  dirichlet_dirty_ = false;
}

void Scene::set_dirichlet(int32_t n, const int32_t* ids, const double* targets) {
  if (!loaded()) fail("load the mesh before setting Dirichlet constraints");
  if (n < 0 || (n > 0 && (!ids || !targets))) fail("bad Dirichlet arguments");
  std::vector<uint8_t> seen(D_.N, 0);
  for (int32_t k = 0; k < n; ++k) {
    if (ids[k] < 0 || ids[k] >= D_.N) fail("Dirichlet vertex id out of range");
    if (seen[ids[k]]++) fail("duplicate Dirichlet vertex id");
  }
  for (int64_t k = 0; k < 3 * int64_t(n); ++k)
    if (!std::isfinite(targets[k])) fail("non-finite Dirichlet target");
  const bool same_ids = int32_t(dir_ids_.size()) == n && std::equal(ids, ids + n, dir_ids_.begin());
  dir_tgt_.assign(targets, targets + 3 * size_t(n));
  if (same_ids && !dirichlet_dirty_) {
    if (n > 0)
      HIPCHK(hipMemcpyAsync(D_.xbar, dir_tgt_.data(), dir_tgt_.size() * 8, hipMemcpyHostToDevice, st_));
    sync();
    return;
  }
  dir_ids_.assign(ids, ids + n);
  dirichlet_dirty_ = true;
  upload_dirichlet();
}

void Scene::set_params(const ppn_params& p) {
  if (!(p.alpha > 0.0 && p.alpha < 1.0)) fail("alpha must be in (0, 1)");
  if (!(p.beta >= 1.0)) fail("beta must be >= 1");
  if (!(p.eps_clamp > 0.0) || !(p.eps_delta >= 0.0)) fail("eps_clamp > 0 and eps_delta >= 0 required");
  if (!(p.pcg_rtol > 0.0 && p.pcg_rtol < 1.0) || p.pcg_maxit < 1) fail("bad PCG tolerance or cap");
  if (p.stop_mode != PPN_STOP_VEL && p.stop_mode != PPN_STOP_GRAD_REL) fail("bad stop_mode");
  if (!(p.stop_tol >= 0.0) || p.newton_maxit < 1 || p.ls_maxit < 0 || p.pdn_countdown < 0)
    fail("bad Newton / line-search parameters");
  if (!(p.armijo_c > 0.0 && p.armijo_c < 1.0)) fail("armijo_c must be in (0, 1)");
  if (!(p.k_dirichlet >= 0.0)) fail("k_dirichlet must be >= 0");
  if (p.eig_mirror != 0 && p.eig_mirror != 1) fail("eig_mirror must be 0 or 1");
  if (p.pcg_load_mode < -1 || p.pcg_load_mode > 2) fail("pcg_load_mode must be -1, 0, 1 or 2");
  if (p.use_graphs != 0 && p.use_graphs != 1) fail("use_graphs must be 0 or 1");
  prm_ = p;
  D_.k_dir = p.k_dirichlet;
  D_.pcg_load = p.pcg_load_mode;
}

// ---------------------------------------------------------------- building blocks
// The scene's one-entry table of the evaluation kernels holds a copy of D_
// (and the line search's step sizes); it is rewritten when that changes.
void Scene::upload_job(int n_gamma, const double* gam) {
  EvalJob e;
  std::memset(static_cast<void*>(&e), 0, sizeof(e));
  e.D = D_;
  e.n_gamma = n_gamma;
  for (int k = 0; k < 4; ++k) e.gamma[k] = k < n_gamma ? gam[k] : 0.0;
  layout_eval_jobs(&e, 1);
  if (job_valid_ && std::memcmp(&e, &job_host_, sizeof(e)) == 0) return;
  job_host_ = e;
  job_valid_ = true;
  // from pageable memory: the copy is staged before the call returns
  HIPCHK(hipMemcpyAsync(D_.job, &job_host_, sizeof(e), hipMemcpyHostToDevice, st_));
}

// Psi(x + gamma_k dx) - Psi(x) for up to four step sizes into scal[0..n).
void Scene::energy_diff(int n, const double* gam) {
  upload_job(n, gam);
  if (batcher_ && batch_eval_) {
    sync();
    batcher_->energy(job_host_);
  } else {
    launch_energy_jobs(D_.job, 1, grid_, st_);
  }
  LAUNCHCHK();
}

void Scene::launch_assemble() {
  upload_job();
  launch_assemble_jobs(D_.job, 1, grid_, st_);
}

// Element quantities, assembly and the gradient norms into scal[0..1].  Alone,
// the launches run as one HIP graph captured at the first call (kernel
// arguments are the scene's fixed table and grid sizes; what changes lives in
// the table); handed to the batcher, they share launches with other scenes.
void Scene::evaluate_at_current_x() {
  upload_job();
  if (batcher_ && batch_eval_) {
    sync();  // the batcher's stream reads what this stream wrote
    batcher_->evaluate(job_host_);
  } else if (prm_.use_graphs) {
    if (!eval_graph_) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
      launch_evaluate_jobs(D_.job, 1, grid_, st_);
      const hipError_t e = hipStreamEndCapture(st_, &g);
      if (e == hipSuccess) {
        const hipError_t ei = hipGraphInstantiate(&eval_graph_, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ei);
      }
      HIPCHK(e);
    }
    HIPCHK(hipGraphLaunch(eval_graph_, st_));
  } else {
    launch_evaluate_jobs(D_.job, 1, grid_, st_);
  }
  LAUNCHCHK();
  n_projected_ = 0;
  all_projected_ = false;
}

void Scene::eig_all() {
  if (precision_ == PPN_MIXED)
    launch_eig_all_f32(D_, prm_.eps_clamp, prm_.eig_mirror, st_);
  else
    launch_eig_all(D_, prm_.eps_clamp, prm_.eig_mirror, st_);
}

void Scene::eig_list(int32_t n) {
  if (precision_ == PPN_MIXED)
    launch_eig_list_f32(D_, n, prm_.eps_clamp, prm_.eig_mirror, st_);
  else
    launch_eig_list(D_, n, prm_.eps_clamp, prm_.eig_mirror, st_);
}

void Scene::project_all() {
  HIPCHK(hipEventRecord(ev_[2], st_));
  eig_all();
  hipEvent_t stop = ev_[3];
  HIPCHK(hipEventRecord(stop, st_));
  launch_fill_u8(D_.proj, 1, D_.T, st_);
  launch_assemble();
  LAUNCHCHK();
  HIPCHK(hipEventSynchronize(stop));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ev_[2], stop));
  last_stats.ms_eig += ms;
  last_stats.projected += D_.T - n_projected_;
  n_projected_ = D_.T;
  all_projected_ = true;
}

int32_t Scene::select_and_project(double delta, bool fallback) {
  launch_select_count(D_, delta, fallback ? 1 : 0, st_);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(hint_, D_.sel_cnt + D_.n_sel_wg, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
  sync();
  const int32_t n = hint_[0];
  if (n <= 0) return 0;
  launch_select_write(D_, st_);
  HIPCHK(hipEventRecord(ev_[2], st_));
  eig_list(n);
  hipEvent_t stop = ev_[3];
  HIPCHK(hipEventRecord(stop, st_));
  if (int64_t(n) * 8 > D_.T)
    launch_assemble();
  else
    launch_regather_list(D_, n, st_);
  LAUNCHCHK();
  HIPCHK(hipEventSynchronize(stop));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ev_[2], stop));
  last_stats.ms_eig += ms;
  last_stats.projected += n;
  n_projected_ += n;
  all_projected_ = n_projected_ >= D_.T;
  return n;
}

void Scene::project_mask(const uint8_t* mask) {
  if (!mask) return;
  std::vector<int32_t> ids;
  for (int32_t e = 0; e < D_.T; ++e)
    if (mask[e]) ids.push_back(e);
  HIPCHK(hipMemcpyAsync(D_.proj, mask, size_t(D_.T), hipMemcpyHostToDevice, st_));
  if (ids.empty()) return;
  HIPCHK(hipMemcpyAsync(D_.list, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, st_));
  eig_list(int32_t(ids.size()));
  launch_regather_list(D_, int32_t(ids.size()), st_);
  LAUNCHCHK();
  sync();
}

template <typename T>
void Scene::run_pcg(const PcgVec<T>& V, const double* src, double sign, double rtol, int maxit,
                    int32_t& ind, int32_t& iters) {
  if (batcher_) {
    sync();  // the batcher's stream reads what this stream wrote
    batcher_->solve(D_, V, src, sign, rtol, maxit, ind, iters);
    return;
  }
  launch_pcg_init(D_, V, src, sign, st_);
  LAUNCHCHK();
  const double tol2 = rtol * rtol;
  // Iterations are enqueued in chunks; the status of chunk c-1 is read while
  // chunk c runs, so launches past convergence (which return at once) are at
  // most two chunks, whose sizes next_chunk() fits to the predicted end.
  int j = 0, chunk = 8, slot = 0, j_prev = -1;
  double rr_prev = 0.0;
  bool pending = false;
  while (j <= maxit) {
    const int jend = std::min(j + chunk, maxit + 1);
    if (profile_on)
      while (prof_ev_.size() < 2 * size_t(jend / kProfileEvery + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        prof_ev_.push_back(e);
      }
    for (; j < jend; ++j) {
      if (profile_on && j % kProfileEvery == 0)
        launch_pcg_iter(D_, V, j, tol2, maxit, st_, prof_ev_[2 * (j / kProfileEvery)],
                        prof_ev_[2 * (j / kProfileEvery) + 1]);
      else
        launch_pcg_iter(D_, V, j, tol2, maxit, st_);
    }
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(&hpcg_[slot], D_.pcg, sizeof(PcgState), hipMemcpyDeviceToHost, st_));
    HIPCHK(hipEventRecord(ev_[slot], st_));
    if (pending) {
      HIPCHK(hipEventSynchronize(ev_[slot ^ 1]));
      if (hpcg_[slot ^ 1].done) break;
      chunk = next_chunk(hpcg_[slot ^ 1], tol2, jend, chunk, j_prev, rr_prev);
    } else {
      chunk = std::min(chunk * 2, kChunkMax);
    }
    pending = true;
    slot ^= 1;
  }
  HIPCHK(hipMemcpyAsync(&hpcg_[2], D_.pcg, sizeof(PcgState), hipMemcpyDeviceToHost, st_));
  sync();
  if (!hpcg_[2].done) fail("PCG ended without a decision", PPN_ERR_DEVICE);
  ind = hpcg_[2].ind;
  iters = hpcg_[2].iters;
  if (profile_on) {
    // Sampled launches j = 0, 16, 32, ... < iters carried out a full product
    // (launches at j >= iters returned at once).  j = 0 is the first-direction
    // variant and is skipped.
    for (int k = kProfileEvery; k < iters; k += kProfileEvery) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, prof_ev_[2 * (k / kProfileEvery)],
                                 prof_ev_[2 * (k / kProfileEvery) + 1]));
      last_stats.ms_spmv += ms;
      last_stats.n_spmv++;
    }
  }
}

void Scene::solve(int32_t& ind, int32_t& iters) {
  const auto t0 = std::chrono::steady_clock::now();
  if (precision_ == PPN_MIXED) {
    solve_mixed(ind, iters);
  } else {
    PcgVec<double> V;
    V.vals = D_.vals;
    V.pinv = D_.pinv;
    V.zd = D_.zd;
    V.dn = D_.dn;
    V.r = D_.r;
    V.q = D_.q;
    V.x = D_.dx;
    run_pcg(V, D_.g, -1.0, prm_.pcg_rtol, prm_.pcg_maxit, ind, iters);
  }
  last_stats.ms_pcg +=
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Mixed precision: PCG with the FP32 rounding of H (FP32 matrix product, FP64
// vectors), refined against the FP64 system.  Round k solves H e = r_k (zero
// start, curvature exit as in the FP64 solve), adds e to dx and forms
// r_{k+1} = -g - H dx with the FP64 matrix; the solve ends once |r|_2 <= rtol |g|_2, the same
// criterion as the FP64 solve's, now on the true FP64 residual.  A round's
// own tolerance asks for the remaining reduction (at most rtol, at least
// kMinInner).  Iterations over all rounds count against pcg_maxit.
void Scene::solve_mixed(int32_t& ind, int32_t& iters) {
  constexpr int kMaxRounds = 8;
  constexpr double kMinInner = 1e-6;
  launch_matrix_to_f32(D_, st_);
  launch_to_f32(D_.pinv, D_.pinv32, int64_t(6) * D_.N, st_);
  launch_refine_init(D_, st_);
  launch_reduce_pcg(D_, kPartA, 1, st_);
  LAUNCHCHK();
  read_scal(1, hscal_);
  const double rr0 = hscal_[0];
  PcgVec<float> V;
  V.vals = D_.vals32;
  V.pinv = D_.pinv32;
  V.zd = D_.zd;
  V.zd32 = D_.zd32;
  V.dn = D_.dn;
  V.r = D_.ri;  // D_.r holds the refinement residual, the inner solve's right-hand side
  V.q = D_.qi;
  V.x = D_.e;
  ind = 0;
  iters = 0;
  if (rr0 == 0.0) return;
  const double goal2 = prm_.pcg_rtol * prm_.pcg_rtol * rr0;
  double rr = rr0;
  for (int round = 0; round < kMaxRounds && iters < prm_.pcg_maxit; ++round) {
    const double rtol_in = std::max(kMinInner, std::min(prm_.pcg_rtol, std::sqrt(goal2 / rr)));
    int32_t ind_k = 0, it_k = 0;
    run_pcg(V, D_.r, 1.0, rtol_in, prm_.pcg_maxit - iters, ind_k, it_k);
    iters += it_k;
    last_stats.refine_rounds++;
    if (ind_k) {
      ind = 1;
      return;
    }
    launch_refine_add(D_, D_.e, st_);
    launch_refine_residual(D_, st_);
    launch_reduce_pcg(D_, kPartA, 1, st_);
    LAUNCHCHK();
    read_scal(1, hscal_);
    rr = hscal_[0];
    if (rr <= goal2) return;
  }
}

// ---------------------------------------------------------------- one time step
// The projections and solves of one Newton iteration at the evaluated iterate
// (element Hessians assembled, nothing projected yet): PN projects every
// element; PDN projects every element while its countdown runs and, when a
// solve reports indefiniteness, projects every element, solves again and
// restarts the countdown; PPN runs the inner loop of Algorithm 1 (delta
// initialised to alpha |g|_inf, tightened by alpha after each indefinite
// solve, relaxed by beta at the end).  Returns the final solve's
// indefiniteness and updates delta and countdown.
int32_t Scene::project_and_solve(int mode, double g_inf, double& delta, int& countdown,
                                 ppn_step_stats& S, ppn_iter_record& rec) {
  if (mode == PPN_PN || (mode == PPN_PDN && countdown > 0)) {
    project_all();
    if (mode == PPN_PDN) countdown--;
  }
  int32_t ind = 0, it = 0;
  solve(ind, it);
  S.solves++;
  S.pcg_iters += it;
  S.indefinite_solves += ind;
  rec.first_ind = ind;
  rec.first_iters = it;
  if (mode == PPN_PDN && ind && !all_projected_) {
    project_all();
    solve(ind, it);
    S.solves++;
    S.pcg_iters += it;
    S.indefinite_solves += ind;
    countdown = prm_.pdn_countdown;
  }
  if (mode == PPN_PPN) {
    while (ind) {
      if (std::isinf(delta)) delta = prm_.alpha * g_inf;
      const int32_t n_new = select_and_project(delta, delta <= prm_.eps_delta);
      S.inner_rounds++;
      rec.rounds++;
      if (n_new > 0) {
        solve(ind, it);
        S.solves++;
        S.pcg_iters += it;
        S.indefinite_solves += ind;
      } else {
        // Nothing new was projected: H is unchanged and the solve would
        // repeat the previous one exactly (still indefinite).
        S.skipped_solves++;
      }
      if (ind) delta = prm_.alpha * delta;
      if (ind && all_projected_) break;
    }
    delta = prm_.beta * delta;
  }
  return ind;
}

ppn_status Scene::newton_step(int mode, ppn_step_stats* out) {
  if (!loaded()) fail("no mesh loaded");
  if (mode != PPN_PN && mode != PPN_PDN && mode != PPN_PPN) fail("unknown mode");
  upload_material();
  upload_dirichlet();
  const auto t0 = std::chrono::steady_clock::now();
  last_stats = ppn_step_stats{};
  ppn_step_stats& S = last_stats;
  trace.clear();
  trace_ids.clear();
  const double h = D_.h;
  launch_predict(D_, st_);
  LAUNCHCHK();
  double delta = std::numeric_limits<double>::infinity();
  int countdown = 0;
  double g0 = 0.0;
  bool converged = false;
  ppn_status status = PPN_OK;

  for (int k = 0; k < prm_.newton_maxit; ++k) {
    S.newton_iters++;
    ppn_iter_record rec{};
    rec.k = k;
    rec.delta_in = delta;
    evaluate_at_current_x();
    read_scal(2, hscal_);
    const double g_l2 = std::sqrt(hscal_[0]), g_inf = hscal_[1];
    if (!std::isfinite(g_l2)) fail("non-finite gradient", PPN_ERR_STATE);
    S.res_l2 = g_l2;
    S.res_inf = g_inf;
    rec.g_l2 = g_l2;
    rec.g_inf = g_inf;
    if (k == 0) {
      g0 = g_l2;
      S.res0_l2 = g_l2;
    }
    if (prm_.stop_mode == PPN_STOP_GRAD_REL && g_l2 <= prm_.stop_tol * g0) {
      converged = true;
      rec.delta_out = delta;
      if (trace_on) {
        trace.push_back(rec);
        trace_ids.emplace_back();
      }
      break;
    }
    const int32_t ind = project_and_solve(mode, g_inf, delta, countdown, S, rec);
    rec.last_ind = ind;
    rec.delta_out = delta;
    rec.n_projected = n_projected_;
    if (ind) {
      S.safety_events++;
      launch_dx_stats(D_, st_);
      read_scal(2, hscal_);
      if (hscal_[1] == 0.0) launch_safety_dir(D_, st_);
    }
    launch_dx_stats(D_, st_);
    LAUNCHCHK();
    read_scal(2, hscal_);
    const double gdx = hscal_[0], dx_inf = hscal_[1];
    rec.dx_inf = dx_inf;
    if (trace_on) {
      std::vector<uint8_t> pm(size_t(D_.T));
      HIPCHK(hipMemcpyAsync(pm.data(), D_.proj, pm.size(), hipMemcpyDeviceToHost, st_));
      sync();
      std::vector<int32_t> ids;
      for (int32_t e = 0; e < D_.T; ++e)
        if (pm[e]) ids.push_back(e);
      trace_ids.push_back(std::move(ids));
    }
    if (prm_.stop_mode == PPN_STOP_VEL && dx_inf / h < prm_.stop_tol) {
      converged = true;
      if (trace_on) trace.push_back(rec);
      break;
    }
    // Armijo backtracking, four trial steps per kernel launch.
    bool accepted = false;
    double gamma = 0.0;
    int trial = 0;
    while (trial <= prm_.ls_maxit && !accepted) {
      const int nb = std::min(4, prm_.ls_maxit + 1 - trial);
      double gam[4];
      for (int q = 0; q < nb; ++q) gam[q] = std::ldexp(1.0, -(trial + q));
      energy_diff(nb, gam);
      read_scal(nb, hscal_);
      int q = 0;
      for (; q < nb; ++q)
        if (hscal_[q] <= prm_.armijo_c * gam[q] * gdx) {
          accepted = true;
          gamma = gam[q];
          break;
        }
      trial += q;
    }
    S.ls_backtracks += trial;
    rec.gamma = accepted ? gamma : 0.0;
    if (trace_on) trace.push_back(rec);
    if (!accepted) {
      S.ls_fail = 1;
      status = PPN_WARN_LS_FAIL;
      break;
    }
    launch_axpy_x(D_, gamma, st_);
    LAUNCHCHK();
  }
  if (!converged && status == PPN_OK) status = PPN_WARN_NOT_CONVERGED;
  launch_finish_step(D_, st_);
  LAUNCHCHK();
  sync();
  S.converged = converged ? 1 : 0;
  S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = S;
  return status;
}

// ---------------------------------------------------------------- stage entry points
// xhat comes from the scene state (x^n, v^n); the caller's x replaces the
// iterate for the duration of the call and the state is restored afterwards.
void Scene::stage_state(const double* x) {
  if (!loaded()) fail("no mesh loaded");
  if (!x) fail("x must not be NULL");
  upload_material();
  upload_dirichlet();
  launch_predict(D_, st_);
  HIPCHK(hipMemcpyAsync(D_.x, x, size_t(D_.N) * 24, hipMemcpyHostToDevice, st_));
}

struct RestoreX {
  Scene* s;
  const Dev& D;
  hipStream_t st;
  ~RestoreX() {
    (void)hipMemcpyAsync(D.x, D.xn, size_t(D.N) * 24, hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
  }
};

void Scene::eval_gradient(const double* x, double* g) {
  stage_state(x);
  RestoreX r{this, D_, st_};
  evaluate_at_current_x();
  HIPCHK(hipMemcpyAsync(g, D_.g, size_t(D_.N) * 24, hipMemcpyDeviceToHost, st_));
  sync();
}

int32_t Scene::element_hessians_count(int32_t n, const int32_t* ids) const {
  if (!loaded()) fail("no mesh loaded");
  if (!ids) return D_.T;
  if (n < 0) fail("n must be >= 0");
  for (int32_t k = 0; k < n; ++k)
    if (ids[k] < 0 || ids[k] >= D_.T) fail("element id out of range");
  return n;
}

// The evaluation itself, with the device staging given: dids (n ids, used when
// ids is not NULL) and dout (n 12x12 matrices).
void Scene::eval_element_hessians_staged(const double* x, const uint8_t* mask, int32_t n,
                                         const int32_t* ids, int32_t* dids, double* dout,
                                         double* out) {
  stage_state(x);
  RestoreX r{this, D_, st_};
  evaluate_at_current_x();
  project_mask(mask);
  if (ids && n > 0) HIPCHK(hipMemcpyAsync(dids, ids, size_t(n) * 4, hipMemcpyHostToDevice, st_));
  launch_element_hessians(D_, ids ? dids : nullptr, n, dout, st_);
  LAUNCHCHK();
  if (n > 0) HIPCHK(hipMemcpyAsync(out, dout, size_t(n) * 144 * 8, hipMemcpyDeviceToHost, st_));
  sync();
}

void Scene::eval_element_hessians(const double* x, const uint8_t* mask, int32_t n,
                                  const int32_t* ids, double* out) {
  if (!out) fail("H_out must not be NULL");
  n = element_hessians_count(n, ids);
  int32_t* dids = nullptr;
  double* dout = nullptr;
  hipError_t e = hipSuccess;
  if (ids) e = hipMalloc(&dids, std::max<size_t>(1, size_t(n)) * 4);
  if (e == hipSuccess) e = hipMalloc(&dout, std::max<size_t>(1, size_t(n)) * 144 * 8);
  if (e != hipSuccess) {
    if (dids) (void)hipFree(dids);
    fail("hipMalloc of the element-Hessian staging failed", PPN_ERR_OOM);
  }
  struct Free {
    void* a;
    void* b;
    ~Free() {
      if (a) (void)hipFree(a);
      if (b) (void)hipFree(b);
    }
  } release{dids, dout};
  eval_element_hessians_staged(x, mask, n, ids, dids, dout, out);
}

void Scene::eval_hessian(const double* x, const uint8_t* mask, int32_t* row_ptr, int32_t* col,
                         double* vals) {
  stage_state(x);
  RestoreX r{this, D_, st_};
  evaluate_at_current_x();
  project_mask(mask);
  if (vals) {
    const size_t NB = size_t(D_.NB);
    std::vector<double> half(size_t(D_.n_hslots) * 9 * kSell);
    HIPCHK(hipMemcpyAsync(half.data(), D_.vals, half.size() * 8, hipMemcpyDeviceToHost, st_));
    sync();
    for (size_t b = 0; b < NB; ++b) {
      const int32_t ref = topo_.csr_ref[b];
      const int32_t pos = ref & kRefPosMask;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          vals[9 * b + 3 * r + c] = half[value_index(pos, ref < 0 ? 3 * c + r : 3 * r + c)];
    }
  }
  if (row_ptr) std::copy(topo_.row_ptr.begin(), topo_.row_ptr.end(), row_ptr);
  if (col) std::copy(topo_.col.begin(), topo_.col.end(), col);
}

void Scene::select(const double* g, double delta, const uint8_t* proj_in, uint8_t* mask,
                   int32_t* cnt) {
  if (!loaded()) fail("no mesh loaded");
  if (!g) fail("g must not be NULL");
  HIPCHK(hipMemcpyAsync(D_.xt, g, size_t(D_.N) * 24, hipMemcpyHostToDevice, st_));
  launch_rinf_from(D_, D_.xt, st_);
  if (proj_in)
    HIPCHK(hipMemcpyAsync(D_.proj, proj_in, size_t(D_.T), hipMemcpyHostToDevice, st_));
  else
    launch_fill_u8(D_.proj, 0, D_.T, st_);
  launch_select_count(D_, delta, delta <= prm_.eps_delta ? 1 : 0, st_);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(hint_, D_.sel_cnt + D_.n_sel_wg, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
  if (mask) HIPCHK(hipMemcpyAsync(mask, D_.sel, size_t(D_.T), hipMemcpyDeviceToHost, st_));
  sync();
  if (cnt) *cnt = hint_[0];
}

void Scene::solve_at(const double* x, const uint8_t* mask, double* dx, int32_t* ind,
                     int32_t* iters) {
  stage_state(x);
  RestoreX r{this, D_, st_};
  evaluate_at_current_x();
  project_mask(mask);
  int32_t i1 = 0, i2 = 0;
  solve(i1, i2);
  if (dx) HIPCHK(hipMemcpyAsync(dx, D_.dx, size_t(D_.N) * 24, hipMemcpyDeviceToHost, st_));
  sync();
  if (ind) *ind = i1;
  if (iters) *iters = i2;
}

void Scene::debug_iterate(int mode, const double* x, double delta_in, uint8_t* mask_out,
                          double* delta_out, int32_t* ind_out) {
  if (mode != PPN_PN && mode != PPN_PDN && mode != PPN_PPN) fail("unknown mode");
  if (!(delta_in > 0.0)) fail("delta_in must be > 0 (INFINITY: not set yet)");
  stage_state(x);
  RestoreX r{this, D_, st_};
  const ppn_step_stats saved = last_stats;
  evaluate_at_current_x();
  read_scal(2, hscal_);
  const double g_inf = hscal_[1];
  if (!std::isfinite(g_inf)) fail("non-finite gradient", PPN_ERR_STATE);
  double delta = delta_in;
  int countdown = 0;
  ppn_step_stats S{};
  ppn_iter_record rec{};
  const int32_t ind = project_and_solve(mode, g_inf, delta, countdown, S, rec);
  last_stats = saved;
  if (mask_out) HIPCHK(hipMemcpyAsync(mask_out, D_.proj, size_t(D_.T), hipMemcpyDeviceToHost, st_));
  sync();
  if (delta_out) *delta_out = delta;
  if (ind_out) *ind_out = ind;
}

void Scene::hessian_product(const double* x, const uint8_t* mask, const double* d, double* q) {
  if (!d || !q) fail("d and q must not be NULL");
  stage_state(x);
  RestoreX r{this, D_, st_};
  evaluate_at_current_x();
  project_mask(mask);
  HIPCHK(hipMemcpyAsync(D_.xt, d, size_t(D_.N) * 24, hipMemcpyHostToDevice, st_));
  launch_spmv_plain(D_, D_.xt, D_.q, st_);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(q, D_.q, size_t(D_.N) * 24, hipMemcpyDeviceToHost, st_));
  sync();
}

void Scene::energy_difference(const double* x, const double* dx, int32_t n, const double* gam,
                              double* out) {
  if (!dx || !gam || !out || n < 0) fail("bad energy_difference arguments");
  stage_state(x);
  RestoreX r{this, D_, st_};
  HIPCHK(hipMemcpyAsync(D_.dx, dx, size_t(D_.N) * 24, hipMemcpyHostToDevice, st_));
  for (int32_t k = 0; k < n; k += 4) {
    const int nb = std::min(4, n - k);
    energy_diff(nb, gam + k);
    read_scal(nb, hscal_);
    for (int q = 0; q < nb; ++q) out[k + q] = hscal_[q];
  }
}

void Scene::get_positions(double* out) {
  if (!loaded()) fail("no mesh loaded");
  HIPCHK(hipMemcpyAsync(out, D_.x, size_t(D_.N) * 24, hipMemcpyDeviceToHost, st_));
  sync();
}

void Scene::get_positions_dev(void* out, hipStream_t st) {
  if (!loaded()) fail("no mesh loaded");
  sync();
  HIPCHK(hipMemcpyAsync(out, D_.x, size_t(D_.N) * 24, hipMemcpyDeviceToDevice, st ? st : st_));
  if (!st) sync();
}

void Scene::get_state(double* x, double* v) {
  if (!loaded()) fail("no mesh loaded");
  if (x) HIPCHK(hipMemcpyAsync(x, D_.x, size_t(D_.N) * 24, hipMemcpyDeviceToHost, st_));
  if (v) HIPCHK(hipMemcpyAsync(v, D_.v, size_t(D_.N) * 24, hipMemcpyDeviceToHost, st_));
  sync();
}

void Scene::set_state(const double* x, const double* v) {
  if (!loaded()) fail("no mesh loaded");
  const size_t n = size_t(D_.N) * 3;
  for (size_t k = 0; k < n; ++k)
    if ((x && !std::isfinite(x[k])) || (v && !std::isfinite(v[k])))
      fail("non-finite state", PPN_ERR_STATE);
  if (x) HIPCHK(hipMemcpyAsync(D_.x, x, n * 8, hipMemcpyHostToDevice, st_));
  if (v) HIPCHK(hipMemcpyAsync(D_.v, v, n * 8, hipMemcpyHostToDevice, st_));
  sync();
}

}  // namespace ppn
