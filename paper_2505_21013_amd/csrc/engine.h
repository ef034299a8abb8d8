// Serving engine: many resident scenes stepped on request.
//
// Each registered scene keeps its description (mesh, material, time step,
// constraints, parameters) and its state on the host; while resident it also
// owns a Scene (device buffers, pattern, scatter maps, its own HIP stream).
// Worker threads take requests in arrival order, skipping requests whose
// scene is busy, so requests of different scenes run concurrently and their
// kernels overlap on the device (one stream per scene); requests of one scene
// run in submission order.  A scene is admitted to device memory when its
// footprint fits the budget, evicting idle resident scenes least recently
// used first (their state is copied back to the host).  A scene's arithmetic
// does not depend on what else runs, so every result is the same alone and in
// the mix.
#pragma once
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ppn.h"
#include "pcg_batch.h"
#include "scene.h"
#include "topology.h"

namespace ppn {

class Engine {
 public:
  Engine(int device, int n_workers, int64_t mem_budget);
  ~Engine();
  int32_t add_scene(const ppn_scene_desc& d);
  int64_t submit(int32_t scene, int32_t mode, const double* targets);
  // Blocks until the request is done; returns its step status.
  ppn_status wait(int64_t id, ppn_step_stats* stats, double* latency_ms, double* queue_ms,
                  std::string* error);
  void get_state(int32_t scene, double* x, double* v);
  void info(ppn_engine_info* out);
  int32_t n_scenes();
  int64_t footprint(int32_t scene);
  // Shared launches across scenes (PPN_BATCH_* flags: PCG solves, and with them
  // the evaluation and line-search phases); only while no request is pending or running.
  void set_batching(int flags);

 private:
  using Clock = std::chrono::steady_clock;
  struct Slot {
    // description (host copies)
    int32_t N = 0, T = 0;
    std::vector<double> X, x, v;  // rest shape, current state
    std::vector<int32_t> tets;
    std::vector<double> E, nu;
    double rho = 1000.0, dt = 1.0 / 30.0;
    double grav[3] = {0, 0, -9.81};
    std::vector<int32_t> dir_ids;
    int32_t precision = PPN_FP64;
    ppn_params params{};
    Topology topo;  // kept so that re-admission skips the host pattern build
    int64_t footprint = 0;
    // residency
    std::unique_ptr<Scene> dev;
    bool busy = false;
    bool loading = false;
    uint64_t last_used = 0;
  };
  struct Request {
    int64_t id = 0;
    int32_t scene = 0, mode = 0;
    std::vector<double> targets;
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    ppn_status status = PPN_OK;
    ppn_step_stats stats{};
    std::string error;
    int waiters = 0;  // threads inside wait() for this request
  };

  void worker();
  // Under the lock: the first runnable pending request and whether its scene
  // must be loaded; evicts idle scenes to make room.  nullptr if none.
  Request* pick(bool& load, std::vector<std::unique_ptr<Scene>>& evicted);
  std::unique_ptr<Scene> build(Slot& s);

  int device_;
  std::unique_ptr<PcgBatcher> batcher_;  // declared before the slots: outlives their scenes
  bool batch_eval_ = false;
  int64_t budget_;
  int64_t resident_bytes_ = 0;
  int64_t admissions_ = 0, evictions_ = 0;
  uint64_t tick_ = 0;
  int64_t next_id_ = 1;
  bool stop_ = false;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::vector<std::unique_ptr<Slot>> slots_;
  std::deque<Request*> pending_;
  // Requests not waited on yet; a record is freed when a wait on it returns.
  std::unordered_map<int64_t, std::unique_ptr<Request>> requests_;
  std::vector<std::thread> workers_;
};

}  // namespace ppn
