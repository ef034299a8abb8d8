// Batched PCG solves across scenes.
//
// Scenes stepped by different host threads hand their solves to one batcher
// thread, which runs all of them in shared launches: one product and one
// update launch per iteration for every solve in flight instead of two per
// scene, so many small scenes stop paying one launch latency each.  The batch
// is continuous: the batcher advances in chunks of kChunk iterations; a solve
// that arrives joins at the next chunk (starting its own iteration count
// there) and a finished solve is handed back at the first chunk boundary
// after it finished, while the others go on.  Each workgroup runs its own
// scene's code with its own scene-local index and iteration number, so every
// scene's result is bit-identical to its unbatched solve.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "device.h"

namespace ppn {

// Shared launches of the per-iteration evaluation kernels (element quantities,
// assembly, gradient norms) and of the line-search energy kernel: scenes that
// reach one of these phases hand it over (their stream drained) and wait; a
// thread with its own stream takes every request present, lays the scenes out
// in one job table and runs each kernel of the phase once for all of them.
class EvalBatcher {
 public:
  explicit EvalBatcher(int device);
  ~EvalBatcher();
  void run(const EvalJob& job, int kind);  // kind 0: evaluation, 1: line search; blocks
  int64_t launches() const { return launches_.load(); }  // shared phase launches
  int64_t jobs() const { return jobs_.load(); }          // scene phases carried by them

 private:
  struct Req {
    EvalJob job;
    int kind = 0;
    bool done = false;
    std::string err;
  };
  void loop();
  void launch(std::vector<Req*>& reqs, int kind);
  int device_;
  hipStream_t st_ = nullptr;
  hipEvent_t ev_ = nullptr;
  EvalJob* d_tab_ = nullptr;
  EvalJob* h_tab_ = nullptr;
  size_t cap_ = 0;
  // written by the batcher thread, read by any (engine statistics)
  std::atomic<int64_t> launches_{0}, jobs_{0};
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  std::deque<Req*> q_;
  bool stop_ = false;
  std::thread th_;
};

class PcgBatcher {
 public:
  explicit PcgBatcher(int device);
  ~PcgBatcher();
  // The evaluation and line-search phases of the scenes that share this batcher.
  void evaluate(const EvalJob& j) { eval_.run(j, 0); }
  void energy(const EvalJob& j) { eval_.run(j, 1); }
  const EvalBatcher& eval_batcher() const { return eval_; }
  // Solve on the batcher's stream; blocks until done.  The caller's stream
  // must have completed the work the solve reads.
  void solve(const Dev& D, const PcgVec<double>& V, const double* src, double sign, double rtol,
             int maxit, int32_t& ind, int32_t& iters);
  void solve(const Dev& D, const PcgVec<float>& V, const double* src, double sign, double rtol,
             int maxit, int32_t& ind, int32_t& iters);
  int64_t batches() const { return batches_.load(); }  // chunks launched
  int64_t solves() const { return solves_.load(); }     // solves handed back

 private:
  struct Job {
    bool fp32 = false;
    Dev D;
    PcgVec<double> V64;
    PcgVec<float> V32;
    const double* src = nullptr;
    double sign = 1.0, tol2 = 0.0;
    int32_t maxit = 0;
    int32_t j0 = 0;       // batch iteration at which the solve started
    int32_t ind = 0, iters = 0;
    uint64_t id = 0;      // unique per solve (table entries refer to solves by id)
    bool done = false;    // handed back to the caller
    std::string err;
  };
  // Solves of one arithmetic in flight, and the device tables of the chunks.
  struct Lane {
    bool fp32 = false;
    std::vector<Job*> members;  // in table order
    int32_t jg = 0;             // batch iteration counter
    // per chunk parity: device and pinned host tables, gathered states
    void* d_tab[2] = {nullptr, nullptr};
    void* h_tab[2] = {nullptr, nullptr};
    size_t tab_cap = 0;         // entries
    void* d_new = nullptr;      // table of the solves joining this chunk
    void* h_new[2] = {nullptr, nullptr};
    size_t new_cap = 0;
    PcgState* d_state[2] = {nullptr, nullptr};
    PcgState* h_state[2] = {nullptr, nullptr};
    std::vector<uint64_t> polled[2];  // solves of the chunk whose states are in h_state[k]
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    int parity = 0;
  };
  // Iterations per chunk: a finished solve waits for the chunk boundary, so
  // short chunks return solves sooner (64-scene batch: 16 -> 294, 8 -> 314,
  // 6 -> 321, 4 -> 320 steps/s; each chunk costs a state read-back).
  static constexpr int kChunk = 6;
  void submit(Job& j, int32_t& ind, int32_t& iters);
  void loop();
  // One chunk of lane L (with the solves joining now); hands back, into
  // finished, the solves whose end the previous chunk's states show.
  // Returns false when the lane had nothing to run.
  template <typename M>
  bool step(Lane& L, std::vector<Job*>& joining, std::vector<Job*>& finished);
  void retire(Lane& L, int parity, std::vector<Job*>& finished);
  template <typename M>
  void reserve(Lane& L, size_t n_tab, size_t n_new, std::vector<Job*>& finished);
  void free_lane(Lane& L);

  int device_;
  EvalBatcher eval_;
  hipStream_t st_ = nullptr;
  Lane lanes_[2];  // FP64 matrix, FP32 matrix
  std::atomic<int64_t> batches_{0}, solves_{0};  // as EvalBatcher's counters
  uint64_t next_id_ = 1;
  std::unordered_map<uint64_t, Job*> live_;  // batcher thread only
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  std::deque<Job*> q_;
  bool stop_ = false;
  std::thread th_;
};

}  // namespace ppn
