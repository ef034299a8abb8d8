#include "engine.h"

#include <algorithm>
#include <cmath>

namespace ppn {

static void fail_arg(const std::string& m) { throw HipError{m, PPN_ERR_ARG}; }

Engine::Engine(int device, int n_workers, int64_t mem_budget) : device_(device) {
  if (n_workers < 1 || n_workers > 256) fail_arg("n_workers must be in [1, 256]");
  if (mem_budget <= 0) {
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) throw HipError{std::string("hipMemGetInfo: ") + hipGetErrorString(e), PPN_ERR_DEVICE};
    mem_budget = int64_t(0.9 * double(free_b));
  }
  budget_ = mem_budget;
  for (int k = 0; k < n_workers; ++k) workers_.emplace_back([this] { worker(); });
}

Engine::~Engine() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  for (auto& t : workers_) t.join();
  slots_.clear();  // frees the resident scenes
}

int32_t Engine::n_scenes() {
  std::lock_guard<std::mutex> lk(mu_);
  return int32_t(slots_.size());
}

void Engine::set_batching(int flags) {
  std::lock_guard<std::mutex> lk(mu_);
  for (auto& s : slots_)
    if (s->busy) throw HipError{"set_batching needs an idle engine", PPN_ERR_STATE};
  if (!pending_.empty()) throw HipError{"set_batching needs an idle engine", PPN_ERR_STATE};
  const bool on = (flags & PPN_BATCH_PCG) != 0;
  batch_eval_ = on && (flags & PPN_BATCH_EVAL) != 0;
  if (on && !batcher_) batcher_ = std::make_unique<PcgBatcher>(device_);
  for (auto& s : slots_)
    if (s->dev) s->dev->set_batcher(on ? batcher_.get() : nullptr, batch_eval_);
  if (!on) batcher_.reset();
}

int64_t Engine::footprint(int32_t scene) {
  std::lock_guard<std::mutex> lk(mu_);
  if (scene < 0 || scene >= int32_t(slots_.size())) fail_arg("unknown scene id");
  return slots_[size_t(scene)]->footprint;
}

int32_t Engine::add_scene(const ppn_scene_desc& d) {
  if (d.n_verts <= 0 || d.n_tets <= 0 || !d.rest_xyz || !d.tets) fail_arg("empty or NULL mesh");
  if (!(d.rho > 0.0) || !(d.dt > 0.0) || !std::isfinite(d.dt)) fail_arg("rho and dt must be > 0");
  if (!d.E || !d.nu) fail_arg("E and nu must not be NULL");
  if (d.precision != PPN_FP64 && d.precision != PPN_MIXED) fail_arg("bad precision");
  if (d.n_dirichlet < 0 || (d.n_dirichlet > 0 && !d.dirichlet_ids)) fail_arg("bad Dirichlet ids");
  auto s = std::make_unique<Slot>();
  s->N = d.n_verts;
  s->T = d.n_tets;
  const size_t n3 = 3 * size_t(d.n_verts), m = size_t(d.n_tets);
  s->X.assign(d.rest_xyz, d.rest_xyz + n3);
  s->x = d.init_xyz ? std::vector<double>(d.init_xyz, d.init_xyz + n3) : s->X;
  s->v = d.init_vel ? std::vector<double>(d.init_vel, d.init_vel + n3) : std::vector<double>(n3, 0.0);
  s->tets.assign(d.tets, d.tets + 4 * m);
  const size_t nm = d.per_element ? m : 1;
  s->E.assign(d.E, d.E + nm);
  s->nu.assign(d.nu, d.nu + nm);
  for (size_t k = 0; k < nm; ++k)
    if (!(s->E[k] >= 0.0) || !(s->nu[k] >= 0.0 && s->nu[k] < 0.5)) fail_arg("need E >= 0 and 0 <= nu < 0.5");
  s->rho = d.rho;
  s->dt = d.dt;
  for (int c = 0; c < 3; ++c) s->grav[c] = d.gravity[c];
  std::vector<uint8_t> seen(size_t(d.n_verts), 0);
  for (int32_t k = 0; k < d.n_dirichlet; ++k) {
    const int32_t i = d.dirichlet_ids[k];
    if (i < 0 || i >= d.n_verts || seen[size_t(i)]++) fail_arg("Dirichlet id out of range or repeated");
  }
  s->dir_ids.assign(d.dirichlet_ids, d.dirichlet_ids + d.n_dirichlet);
  s->precision = d.precision;
  if (d.params)
    s->params = *d.params;
  else
    params_defaults(&s->params);
  std::string err;
  if (!build_topology(d.n_verts, d.n_tets, d.tets, s->topo, err)) throw HipError{err, PPN_ERR_MESH};
  s->footprint = Scene::footprint(s->topo, s->precision);
  std::lock_guard<std::mutex> lk(mu_);
  slots_.push_back(std::move(s));
  return int32_t(slots_.size()) - 1;
}

int64_t Engine::submit(int32_t scene, int32_t mode, const double* targets) {
  if (mode != PPN_PN && mode != PPN_PDN && mode != PPN_PPN) fail_arg("unknown mode");
  std::unique_lock<std::mutex> lk(mu_);
  if (scene < 0 || scene >= int32_t(slots_.size())) fail_arg("unknown scene id");
  const Slot& s = *slots_[size_t(scene)];
  const size_t nt = 3 * s.dir_ids.size();
  if (nt > 0 && !targets) fail_arg("targets must not be NULL");
  for (size_t k = 0; k < nt; ++k)
    if (!std::isfinite(targets[k])) fail_arg("non-finite Dirichlet target");
  auto r = std::make_unique<Request>();
  r->id = next_id_++;
  r->scene = scene;
  r->mode = mode;
  r->targets.assign(targets, targets + nt);
  r->t_submit = Clock::now();
  pending_.push_back(r.get());
  const int64_t id = r->id;
  requests_.emplace(id, std::move(r));
  lk.unlock();
  cv_work_.notify_one();
  return id;
}

Engine::Request* Engine::pick(bool& load, std::vector<std::unique_ptr<Scene>>& evicted) {
  for (auto it = pending_.begin(); it != pending_.end();) {
    Request* r = *it;
    Slot& s = *slots_[size_t(r->scene)];
    if (s.busy) {  // an earlier request of this scene is running
      ++it;
      continue;
    }
    if (s.dev) {
      pending_.erase(it);
      load = false;
      return r;
    }
    if (s.footprint > budget_) {  // can never be admitted
      r->status = PPN_ERR_OOM;
      r->error = "scene footprint " + std::to_string(s.footprint) + " B exceeds the engine budget";
      r->t_start = r->t_done = Clock::now();
      r->done = true;
      it = pending_.erase(it);
      cv_done_.notify_all();
      continue;
    }
    // admission: evict idle resident scenes, least recently used first
    while (resident_bytes_ + s.footprint > budget_) {
      Slot* lru = nullptr;
      for (auto& o : slots_)
        if (o->dev && !o->busy && o.get() != &s && (!lru || o->last_used < lru->last_used)) lru = o.get();
      if (!lru) break;
      lru->dev->get_state(lru->x.data(), lru->v.data());
      evicted.push_back(std::move(lru->dev));
      resident_bytes_ -= lru->footprint;
      evictions_++;
    }
    if (resident_bytes_ + s.footprint > budget_) {  // wait for a busy scene to finish
      ++it;
      continue;
    }
    resident_bytes_ += s.footprint;
    admissions_++;
    pending_.erase(it);
    load = true;
    return r;
  }
  return nullptr;
}

std::unique_ptr<Scene> Engine::build(Slot& s) {
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) throw HipError{std::string("hipStreamCreate: ") + hipGetErrorString(e), PPN_ERR_DEVICE};
  std::unique_ptr<Scene> sc;
  try {
    sc = std::make_unique<Scene>(st, true, s.precision);
  } catch (...) {
    (void)hipStreamDestroy(st);
    throw;
  }
  sc->set_params(s.params);
  sc->set_time_step(s.dt, s.grav);
  Topology t = s.topo;
  sc->load_mesh(std::move(t), s.X.data(), s.tets.data(), nullptr);
  sc->set_material(s.rho, s.E.data(), s.nu.data(), s.E.size() > 1);
  sc->set_state(s.x.data(), s.v.data());
  sc->set_batcher(batcher_.get(), batch_eval_);
  return sc;
}

void Engine::worker() {
  (void)hipSetDevice(device_);
  std::unique_lock<std::mutex> lk(mu_);
  for (;;) {
    bool load = false;
    std::vector<std::unique_ptr<Scene>> evicted;
    Request* r = nullptr;
    while (!stop_) {
      r = pick(load, evicted);
      if (r) break;
      if (!evicted.empty()) {
        lk.unlock();
        evicted.clear();
        lk.lock();
        continue;
      }
      cv_work_.wait(lk);
    }
    if (!r) return;
    Slot& s = *slots_[size_t(r->scene)];
    s.busy = true;
    r->t_start = Clock::now();
    lk.unlock();
    evicted.clear();  // frees evicted scenes' device memory outside the lock
    ppn_status st = PPN_OK;
    std::string err;
    std::unique_ptr<Scene> fresh;
    try {
      if (load) fresh = build(s);
      Scene* sc = load ? fresh.get() : s.dev.get();
      sc->set_dirichlet(int32_t(s.dir_ids.size()), s.dir_ids.data(), r->targets.data());
      st = sc->newton_step(r->mode, &r->stats);
    } catch (const HipError& e) {
      st = e.code;
      err = e.msg;
    } catch (const std::exception& e) {
      st = PPN_ERR_DEVICE;
      err = e.what();
    }
    lk.lock();
    if (load) {
      if (fresh) {
        s.dev = std::move(fresh);
      } else {
        resident_bytes_ -= s.footprint;  // admission failed
      }
    }
    s.busy = false;
    s.last_used = ++tick_;
    r->status = st;
    r->error = err;
    r->t_done = Clock::now();
    r->done = true;
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
}

ppn_status Engine::wait(int64_t id, ppn_step_stats* stats, double* latency_ms, double* queue_ms,
                        std::string* error) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = requests_.find(id);
  if (it == requests_.end()) fail_arg("unknown request id (or already waited on)");
  Request& r = *it->second;
  ++r.waiters;
  cv_done_.wait(lk, [&] { return r.done; });
  if (stats) *stats = r.stats;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
  if (queue_ms) *queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count();
  if (error) *error = r.error;
  const ppn_status st = r.status;
  if (--r.waiters == 0) requests_.erase(id);  // the record is freed once waited on
  return st;
}

void Engine::get_state(int32_t scene, double* x, double* v) {
  std::unique_lock<std::mutex> lk(mu_);
  if (scene < 0 || scene >= int32_t(slots_.size())) fail_arg("unknown scene id");
  Slot& s = *slots_[size_t(scene)];
  // wait until no request of this scene is pending or running
  cv_done_.wait(lk, [&] {
    if (s.busy) return false;
    for (const Request* r : pending_)
      if (r->scene == scene) return false;
    return true;
  });
  if (s.dev) s.dev->get_state(s.x.data(), s.v.data());
  const size_t n3 = 3 * size_t(s.N);
  if (x) std::copy(s.x.begin(), s.x.begin() + n3, x);
  if (v) std::copy(s.v.begin(), s.v.begin() + n3, v);
}

void Engine::info(ppn_engine_info* out) {
  std::lock_guard<std::mutex> lk(mu_);
  out->budget_bytes = budget_;
  out->resident_bytes = resident_bytes_;
  out->admissions = admissions_;
  out->evictions = evictions_;
  int32_t res = 0;
  for (auto& s : slots_) res += s->dev ? 1 : 0;
  out->resident_scenes = res;
  out->n_scenes = int32_t(slots_.size());
  out->n_workers = int32_t(workers_.size());
  out->pending = int32_t(pending_.size());
  out->pcg_batches = batcher_ ? batcher_->batches() : 0;
  out->pcg_batched_solves = batcher_ ? batcher_->solves() : 0;
  out->eval_launches = batcher_ ? batcher_->eval_batcher().launches() : 0;
  out->eval_batched_phases = batcher_ ? batcher_->eval_batcher().jobs() : 0;
}

}  // namespace ppn
