// Scene: owns the device buffers of one simulation and runs its time steps.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/ppn.h"
#include "device.h"
#include "pcg_batch.h"
#include "topology.h"

namespace ppn {

// Most element Hessians one ppn_eval_element_hessians_noalloc call evaluates.
constexpr int32_t kNoAllocMaxElements = PPN_NOALLOC_MAX_ELEMENTS;

// Defaults of every parameter (the paper's values).
void params_defaults(ppn_params* p);

struct HipError {
  std::string msg;
  ppn_status code;
};

class Scene {
 public:
  Scene(hipStream_t stream, bool own_stream, int precision);
  ~Scene();

  void load_mesh(int32_t n_verts, const double* rest, int32_t n_tets, const int32_t* tets,
                 const double* init);
  // Same with a topology built beforehand (build_topology on the same tets).
  void load_mesh(Topology&& t, const double* rest, const int32_t* tets, const double* init);
  // Device bytes a scene of this topology allocates (exactly what load_mesh takes).
  static int64_t footprint(const Topology& t, int precision);
  template <class T>
  T* alloc(size_t n);
  void set_material(double rho, const double* E, const double* nu, bool per_element);
  void set_time_step(double dt, const double* gravity);
  void set_dirichlet(int32_t n, const int32_t* ids, const double* targets);
  void set_params(const ppn_params& p);
  ppn_status newton_step(int mode, ppn_step_stats* out);

  // stage entry points
  void eval_gradient(const double* x, double* g);
  void eval_element_hessians(const double* x, const uint8_t* mask, int32_t n, const int32_t* ids,
                             double* out);
  // The same without device allocation: the staging sits in the library's
  // fixed per-device array (at most kNoAllocMaxElements elements per call).
  void eval_element_hessians_noalloc(const double* x, const uint8_t* mask, int32_t n,
                                     const int32_t* ids, double* out);
  void eval_hessian(const double* x, const uint8_t* mask, int32_t* row_ptr, int32_t* col,
                    double* vals);
  void select(const double* g, double delta, const uint8_t* proj_in, uint8_t* mask, int32_t* cnt);
  void solve_at(const double* x, const uint8_t* mask, double* dx, int32_t* ind, int32_t* iters);
  void debug_iterate(int mode, const double* x, double delta_in, uint8_t* mask_out, double* delta_out,
                     int32_t* ind_out);
  void hessian_product(const double* x, const uint8_t* mask, const double* d, double* q);
  void energy_difference(const double* x, const double* dx, int32_t n, const double* gam,
                         double* out);

  void get_positions(double* out);
  void get_positions_dev(void* out, hipStream_t st);
  void get_state(double* x, double* v);
  void set_state(const double* x, const double* v);

  // Hand PCG solves (and, with eval, the evaluation and line-search launches)
  // to a batcher shared with other scenes (nullptr: everything alone).
  void set_batcher(PcgBatcher* b, bool eval = false) {
    batcher_ = b;
    batch_eval_ = b && eval;
  }
  bool loaded() const { return D_.N > 0; }
  const Dev& dev() const { return D_; }
  const Topology& topo() const { return topo_; }
  int64_t device_bytes() const { return dev_bytes_; }

  ppn_step_stats last_stats{};
  std::string last_error;
  bool trace_on = false;
  bool profile_on = false;
  std::vector<ppn_iter_record> trace;
  std::vector<std::vector<int32_t>> trace_ids;

 private:
  void free_all();
  // Number of matrices a call evaluates (n_tets without ids); checks the ids.
  int32_t element_hessians_count(int32_t n, const int32_t* ids) const;
  void eval_element_hessians_staged(const double* x, const uint8_t* mask, int32_t n,
                                    const int32_t* ids, int32_t* dids, double* dout, double* out);
  void upload_material();
  void upload_dirichlet();
  void sync();
  void stage_state(const double* x);
  void evaluate_at_current_x();
  void project_mask(const uint8_t* mask);
  void project_all();
  int32_t select_and_project(double delta, bool fallback);
  int32_t project_and_solve(int mode, double g_inf, double& delta, int& countdown, ppn_step_stats& S,
                            ppn_iter_record& rec);
  void solve(int32_t& ind, int32_t& iters);
  // One PCG run of the given arithmetic on the system whose right-hand side is
  // sign * src; returns its indefiniteness flag and iteration count.
  template <typename T>
  void run_pcg(const PcgVec<T>& V, const double* src, double sign, double rtol, int maxit,
               int32_t& ind, int32_t& iters);
  void solve_mixed(int32_t& ind, int32_t& iters);
  void eig_all();
  void eig_list(int32_t n);
  void upload_job(int n_gamma = 0, const double* gam = nullptr);
  void launch_assemble();
  void energy_diff(int n, const double* gam);
  void read_scal(int n, double* out);

  hipStream_t st_;
  int device_ = 0;  // the HIP device current at creation
  bool own_stream_;
  int precision_;
  PcgBatcher* batcher_ = nullptr;
  bool batch_eval_ = false;
  Dev D_;
  EvalJob job_host_{};          // the table entry last written to D_.job
  bool job_valid_ = false;
  EvalGrid grid_;               // this scene's grids of the evaluation kernels
  hipGraphExec_t eval_graph_ = nullptr;
  Topology topo_;
  std::vector<void*> allocs_;
  int64_t dev_bytes_ = 0;
  ppn_params prm_{};
  // host copies
  std::vector<double> X_, E_, nu_;
  double rho_ = 1000.0;
  std::vector<int32_t> dir_ids_;
  std::vector<double> dir_tgt_;
  bool material_dirty_ = true;
  bool dirichlet_dirty_ = true;
  // pinned host scratch
  double* hscal_ = nullptr;
  PcgState* hpcg_ = nullptr;
  int32_t* hint_ = nullptr;
  hipEvent_t ev_[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> prof_ev_;  // start/stop pairs of profiled matrix-product launches
  bool all_projected_ = false;
  int32_t n_projected_ = 0;
};

}  // namespace ppn
