// extern "C" boundary of libppn: argument checks, exception capture, status codes.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <new>
#include <string>

#include "../../include/ppn.h"
#include "engine.h"
#include "scene.h"
#include "topology.h"

struct ppn_scene {
  ppn::Scene* impl = nullptr;
};

struct ppn_engine {
  ppn::Engine* impl = nullptr;
};

namespace {

thread_local std::string g_error;

// Relative tolerance of the dense projector's precondition (symmetry and the
// translation null space), far above the rounding of FP64 element Hessians.
constexpr double kDenseCheckRtol = 1e-9;

template <class F>
ppn_status guarded(ppn_scene* s, F&& f) {
  try {
    return f();
  } catch (const ppn::HipError& e) {
    if (s && s->impl) s->impl->last_error = e.msg;
    g_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    const char* m = "host allocation failed";
    if (s && s->impl) s->impl->last_error = m;
    g_error = m;
    return PPN_ERR_OOM;
  } catch (const std::exception& e) {
    if (s && s->impl) s->impl->last_error = e.what();
    g_error = e.what();
    return PPN_ERR_ARG;
  }
}

ppn_status bad_handle() {
  g_error = "NULL scene handle";
  return PPN_ERR_ARG;
}

// A NULL pointer argument of a call on a valid scene.
ppn_status null_arg(ppn_scene* s, const char* name) {
  g_error = std::string(name) + " must not be NULL";
  if (s && s->impl) s->impl->last_error = g_error;
  return PPN_ERR_ARG;
}

}  // namespace

#define IMPL(s)                     \
  if (!(s) || !(s)->impl) return bad_handle(); \
  ppn::Scene& S = *(s)->impl

extern "C" {

ppn_status ppn_params_default(ppn_params* out) {
  if (!out) {
    g_error = "out must not be NULL";
    return PPN_ERR_ARG;
  }
  ppn::params_defaults(out);
  return PPN_OK;
}

ppn_status ppn_scene_create(ppn_scene** out, void* hip_stream, int32_t precision) {
  if (!out) {
    g_error = "out must not be NULL";
    return PPN_ERR_ARG;
  }
  *out = nullptr;
  if (precision != PPN_FP64 && precision != PPN_MIXED) {
    g_error = "precision must be PPN_FP64 or PPN_MIXED";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    bool own = false;
    if (!st) {
      hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e != hipSuccess) throw ppn::HipError{std::string("hipStreamCreate: ") + hipGetErrorString(e), PPN_ERR_DEVICE};
      own = true;
    }
    auto* h = new ppn_scene;
    try {
      h->impl = new ppn::Scene(st, own, precision);
    } catch (...) {
      delete h;
      if (own) (void)hipStreamDestroy(st);
      throw;
    }
    *out = h;
    return PPN_OK;
  });
}

ppn_status ppn_scene_destroy(ppn_scene* s) {
  if (!s) return PPN_OK;
  delete s->impl;
  delete s;
  return PPN_OK;
}

ppn_status ppn_load_mesh(ppn_scene* s, int32_t n_verts, const double* rest_xyz, int32_t n_tets,
                         const int32_t* tets, const double* init_xyz) {
  IMPL(s);
  return guarded(s, [&] {
    S.load_mesh(n_verts, rest_xyz, n_tets, tets, init_xyz);
    return PPN_OK;
  });
}

ppn_status ppn_set_material(ppn_scene* s, double rho, const double* E, const double* nu,
                            int32_t per_element) {
  IMPL(s);
  return guarded(s, [&] {
    S.set_material(rho, E, nu, per_element != 0);
    return PPN_OK;
  });
}

ppn_status ppn_set_time_step(ppn_scene* s, double dt, const double* gravity) {
  IMPL(s);
  return guarded(s, [&] {
    S.set_time_step(dt, gravity);
    return PPN_OK;
  });
}

ppn_status ppn_set_dirichlet(ppn_scene* s, int32_t n, const int32_t* ids, const double* tgt) {
  IMPL(s);
  return guarded(s, [&] {
    S.set_dirichlet(n, ids, tgt);
    return PPN_OK;
  });
}

ppn_status ppn_set_params(ppn_scene* s, const ppn_params* p) {
  IMPL(s);
  if (!p) return null_arg(s, "p");
  return guarded(s, [&] {
    S.set_params(*p);
    return PPN_OK;
  });
}

ppn_status ppn_newton_step(ppn_scene* s, int32_t mode, ppn_step_stats* out) {
  IMPL(s);
  return guarded(s, [&] { return S.newton_step(mode, out); });
}

ppn_status ppn_get_positions(ppn_scene* s, double* out) {
  IMPL(s);
  if (!out) return null_arg(s, "out");
  return guarded(s, [&] {
    S.get_positions(out);
    return PPN_OK;
  });
}

ppn_status ppn_get_positions_dev(ppn_scene* s, void* out_dev, void* hip_stream) {
  IMPL(s);
  if (!out_dev) return null_arg(s, "out_dev");
  return guarded(s, [&] {
    S.get_positions_dev(out_dev, static_cast<hipStream_t>(hip_stream));
    return PPN_OK;
  });
}

ppn_status ppn_get_state(ppn_scene* s, double* x, double* v) {
  IMPL(s);
  return guarded(s, [&] {
    S.get_state(x, v);
    return PPN_OK;
  });
}

ppn_status ppn_set_state(ppn_scene* s, const double* x, const double* v) {
  IMPL(s);
  return guarded(s, [&] {
    S.set_state(x, v);
    return PPN_OK;
  });
}

ppn_status ppn_get_last_stats(ppn_scene* s, ppn_step_stats* out) {
  IMPL(s);
  if (!out) return null_arg(s, "out");
  *out = S.last_stats;
  return PPN_OK;
}

ppn_status ppn_scene_info(ppn_scene* s, int32_t* n_verts, int32_t* n_tets, int32_t* n_edges,
                          int64_t* n_blocks, int64_t* device_bytes) {
  IMPL(s);
  const auto& D = S.dev();
  if (n_verts) *n_verts = D.N;
  if (n_tets) *n_tets = D.T;
  if (n_edges) *n_edges = D.E;
  if (n_blocks) *n_blocks = D.NB;
  if (device_bytes) *device_bytes = S.device_bytes();
  return PPN_OK;
}

const char* ppn_last_error(const ppn_scene* s) {
  if (s && s->impl) return s->impl->last_error.c_str();
  return g_error.c_str();
}

ppn_status ppn_set_trace(ppn_scene* s, int32_t enable) {
  IMPL(s);
  S.trace_on = enable != 0;
  return PPN_OK;
}

ppn_status ppn_set_profiling(ppn_scene* s, int32_t enable) {
  IMPL(s);
  S.profile_on = enable != 0;
  return PPN_OK;
}

ppn_status ppn_trace_count(ppn_scene* s, int32_t* count) {
  IMPL(s);
  if (!count) return null_arg(s, "count");
  *count = int32_t(S.trace.size());
  return PPN_OK;
}

ppn_status ppn_trace_get(ppn_scene* s, int32_t i, ppn_iter_record* rec, int32_t* proj_ids) {
  IMPL(s);
  if (i < 0 || i >= int32_t(S.trace.size()) || !rec) {
    S.last_error = "trace index out of range";
    return PPN_ERR_ARG;
  }
  *rec = S.trace[i];
  if (proj_ids && i < int32_t(S.trace_ids.size())) {
    const auto& v = S.trace_ids[i];
    for (size_t k = 0; k < v.size(); ++k) proj_ids[k] = v[k];
  }
  return PPN_OK;
}

ppn_status ppn_eval_gradient(ppn_scene* s, const double* x, double* g_out) {
  IMPL(s);
  if (!g_out) return null_arg(s, "g_out");
  return guarded(s, [&] {
    S.eval_gradient(x, g_out);
    return PPN_OK;
  });
}

ppn_status ppn_eval_element_hessians(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                                     int32_t n, const int32_t* ids, double* H_out) {
  IMPL(s);
  return guarded(s, [&] {
    S.eval_element_hessians(x, proj_mask, n, ids, H_out);
    return PPN_OK;
  });
}

ppn_status ppn_eval_element_hessians_noalloc(ppn_scene* s, const double* x,
                                             const uint8_t* proj_mask, int32_t n,
                                             const int32_t* ids, double* H_out) {
  IMPL(s);
  return guarded(s, [&] {
    S.eval_element_hessians_noalloc(x, proj_mask, n, ids, H_out);
    return PPN_OK;
  });
}

ppn_status ppn_eval_hessian(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                            int32_t* row_ptr, int32_t* col, double* vals) {
  IMPL(s);
  return guarded(s, [&] {
    S.eval_hessian(x, proj_mask, row_ptr, col, vals);
    return PPN_OK;
  });
}

ppn_status ppn_select(ppn_scene* s, const double* g, double delta, const uint8_t* proj_in,
                      uint8_t* mask_out, int32_t* count_out) {
  IMPL(s);
  return guarded(s, [&] {
    S.select(g, delta, proj_in, mask_out, count_out);
    return PPN_OK;
  });
}

ppn_status ppn_solve(ppn_scene* s, const double* x, const uint8_t* proj_mask, double* dx_out,
                     int32_t* ind_out, int32_t* iters_out) {
  IMPL(s);
  return guarded(s, [&] {
    S.solve_at(x, proj_mask, dx_out, ind_out, iters_out);
    return PPN_OK;
  });
}

ppn_status ppn_debug_iterate(ppn_scene* s, int32_t mode, const double* x, double delta_in,
                             uint8_t* mask_out, double* delta_out, int32_t* ind_out) {
  IMPL(s);
  return guarded(s, [&] {
    S.debug_iterate(mode, x, delta_in, mask_out, delta_out, ind_out);
    return PPN_OK;
  });
}

ppn_status ppn_hessian_product(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                               const double* d, double* q_out) {
  IMPL(s);
  return guarded(s, [&] {
    S.hessian_product(x, proj_mask, d, q_out);
    return PPN_OK;
  });
}

ppn_status ppn_energy_difference(ppn_scene* s, const double* x, const double* dx, int32_t n_gamma,
                                 const double* gammas, double* out) {
  IMPL(s);
  return guarded(s, [&] {
    S.energy_difference(x, dx, n_gamma, gammas, out);
    return PPN_OK;
  });
}

ppn_status ppn_project_batch_dev(const double* H_dev, double* Hhat_dev, int64_t n, double eps,
                                 void* hip_stream) {
  if (n < 0 || (n > 0 && (!H_dev || !Hhat_dev)) || !(eps > 0.0)) {
    g_error = "bad ppn_project_batch_dev arguments";
    return PPN_ERR_ARG;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // The precondition is checked before anything is written (the output may
  // alias the input).  The check kernel raises a flag in a small device buffer
  // (one per device, allocated at the first call) that is copied back; calls
  // are serialised around it.
  static std::mutex mu;
  static std::map<int, int32_t*> flags;
  std::lock_guard<std::mutex> lk(mu);
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  int32_t*& bad = flags[device];
  if (e == hipSuccess && !bad) e = hipMalloc(reinterpret_cast<void**>(&bad), 256);
  int32_t bad_host = 0;
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int32_t), st);
  if (e == hipSuccess) {
    ppn::launch_check_dense(H_dev, n, kDenseCheckRtol, bad, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad_host, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && bad_host) {
    g_error = "ppn_project_batch_dev: an input matrix is not symmetric or does not annihilate the "
              "rigid translations (tolerance 1e-9 of its largest entry); nothing was written";
    return PPN_ERR_ARG;
  }
  if (e == hipSuccess) {
    ppn::launch_project_batch(H_dev, Hhat_dev, n, eps, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    g_error = std::string("ppn_project_batch_dev: ") + hipGetErrorString(e);
    return PPN_ERR_DEVICE;
  }
  return PPN_OK;
}

ppn_status ppn_locality_order(int32_t n_verts, const double* rest_xyz, int32_t n_tets,
                              const int32_t* tets, int32_t kind, int32_t* vertex_order,
                              int32_t* tet_order) {
  const char* null_name = !rest_xyz ? "rest_xyz" : !tets ? "tets" : !vertex_order ? "vertex_order"
                          : !tet_order ? "tet_order" : nullptr;
  if (null_name) return null_arg(nullptr, null_name);
  try {
    std::string err;
    if (!ppn::locality_order(n_verts, rest_xyz, n_tets, tets, kind, vertex_order, tet_order, err)) {
      g_error = err;
      return PPN_ERR_MESH;
    }
  } catch (const std::bad_alloc&) {
    g_error = "host allocation failed";
    return PPN_ERR_OOM;
  }
  return PPN_OK;
}

// ---- serving engine
#define ENGINE(e)                                  \
  if (!(e) || !(e)->impl) {                        \
    g_error = "NULL engine handle";                \
    return PPN_ERR_ARG;                            \
  }                                                \
  ppn::Engine& EG = *(e)->impl

ppn_status ppn_engine_create(ppn_engine** out, int32_t n_workers, int64_t mem_budget_bytes) {
  if (!out) {
    g_error = "out must not be NULL";
    return PPN_ERR_ARG;
  }
  *out = nullptr;
  if (n_workers < 1 || n_workers > 256) {
    g_error = "n_workers must be in [1, 256]";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) throw ppn::HipError{std::string("hipGetDevice: ") + hipGetErrorString(e), PPN_ERR_DEVICE};
    auto* h = new ppn_engine;
    try {
      h->impl = new ppn::Engine(dev, n_workers, mem_budget_bytes);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return PPN_OK;
  });
}

ppn_status ppn_engine_destroy(ppn_engine* e) {
  if (!e) return PPN_OK;
  delete e->impl;
  delete e;
  return PPN_OK;
}

ppn_status ppn_engine_add_scene(ppn_engine* e, const ppn_scene_desc* d, int32_t* scene_id_out) {
  ENGINE(e);
  if (!d || !scene_id_out) {
    g_error = "desc and scene_id_out must not be NULL";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    *scene_id_out = EG.add_scene(*d);
    return PPN_OK;
  });
}

ppn_status ppn_engine_scene_footprint(ppn_engine* e, int32_t scene_id, int64_t* bytes_out) {
  ENGINE(e);
  if (!bytes_out) {
    g_error = "bytes_out must not be NULL";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    *bytes_out = EG.footprint(scene_id);
    return PPN_OK;
  });
}

ppn_status ppn_engine_submit(ppn_engine* e, int32_t scene_id, int32_t mode, const double* targets,
                             int64_t* request_id_out) {
  ENGINE(e);
  if (!request_id_out) {
    g_error = "request_id_out must not be NULL";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    *request_id_out = EG.submit(scene_id, mode, targets);
    return PPN_OK;
  });
}

ppn_status ppn_engine_wait(ppn_engine* e, int64_t request_id, ppn_status* step_status_out,
                           ppn_step_stats* stats_out, double* latency_ms_out, double* queue_ms_out) {
  ENGINE(e);
  return guarded(nullptr, [&]() -> ppn_status {
    std::string err;
    const ppn_status st = EG.wait(request_id, stats_out, latency_ms_out, queue_ms_out, &err);
    if (!err.empty()) g_error = err;
    if (step_status_out) *step_status_out = st;
    return PPN_OK;
  });
}

ppn_status ppn_engine_get_state(ppn_engine* e, int32_t scene_id, double* x_out, double* v_out) {
  ENGINE(e);
  return guarded(nullptr, [&]() -> ppn_status {
    EG.get_state(scene_id, x_out, v_out);
    return PPN_OK;
  });
}

ppn_status ppn_engine_set_pcg_batching(ppn_engine* e, int32_t enable) {
  ENGINE(e);
  return guarded(nullptr, [&]() -> ppn_status {
    EG.set_batching(enable != 0 ? PPN_BATCH_PCG : 0);
    return PPN_OK;
  });
}

ppn_status ppn_engine_set_batching(ppn_engine* e, int32_t flags) {
  ENGINE(e);
  if (flags < 0 || flags > (PPN_BATCH_PCG | PPN_BATCH_EVAL) || (flags == PPN_BATCH_EVAL)) {
    g_error = "batching flags: 0, PPN_BATCH_PCG, or PPN_BATCH_PCG | PPN_BATCH_EVAL";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    EG.set_batching(flags);
    return PPN_OK;
  });
}

ppn_status ppn_engine_get_info(ppn_engine* e, ppn_engine_info* out) {
  ENGINE(e);
  if (!out) {
    g_error = "out must not be NULL";
    return PPN_ERR_ARG;
  }
  return guarded(nullptr, [&]() -> ppn_status {
    EG.info(out);
    return PPN_OK;
  });
}

}  // extern "C"
