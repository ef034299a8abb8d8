#include "pcg_batch.h"

#include <algorithm>
#include <cstring>

#include "scene.h"

namespace ppn {

#define BCHK(x)                                                                                \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess)                                                                      \
      throw HipError{std::string(#x) + ": " + hipGetErrorString(e_),                           \
                     e_ == hipErrorOutOfMemory ? PPN_ERR_OOM : PPN_ERR_DEVICE};                \
  } while (0)

EvalBatcher::EvalBatcher(int device) : device_(device) {
  BCHK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
  BCHK(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
  th_ = std::thread([this] { loop(); });
}

EvalBatcher::~EvalBatcher() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  th_.join();
  (void)hipStreamSynchronize(st_);
  if (d_tab_) (void)hipFree(d_tab_);
  if (h_tab_) (void)hipHostFree(h_tab_);
  (void)hipEventDestroy(ev_);
  (void)hipStreamDestroy(st_);
}

void EvalBatcher::run(const EvalJob& job, int kind) {
  Req r;
  r.job = job;
  r.kind = kind;
  std::unique_lock<std::mutex> lk(mu_);
  q_.push_back(&r);
  cv_.notify_one();
  cv_done_.wait(lk, [&] { return r.done; });
  if (!r.err.empty()) throw HipError{r.err, PPN_ERR_DEVICE};
}

// One launch of each kernel of the phase for every request in reqs; the
// requests' own step sizes (line search) travel in their table entries.
void EvalBatcher::launch(std::vector<Req*>& reqs, int kind) {
  const size_t n = reqs.size();
  if (n > cap_) {
    BCHK(hipStreamSynchronize(st_));
    if (d_tab_) (void)hipFree(d_tab_);
    if (h_tab_) (void)hipHostFree(h_tab_);
    d_tab_ = nullptr;
    h_tab_ = nullptr;
    cap_ = std::max<size_t>(2 * cap_, std::max<size_t>(n, 64));
    BCHK(hipMalloc(reinterpret_cast<void**>(&d_tab_), cap_ * sizeof(EvalJob)));
    BCHK(hipHostMalloc(reinterpret_cast<void**>(&h_tab_), cap_ * sizeof(EvalJob)));
  }
  for (size_t k = 0; k < n; ++k) h_tab_[k] = reqs[k]->job;
  const EvalGrid gr = layout_eval_jobs(h_tab_, int(n));
  BCHK(hipMemcpyAsync(d_tab_, h_tab_, n * sizeof(EvalJob), hipMemcpyHostToDevice, st_));
  if (kind == 0)
    launch_evaluate_jobs(d_tab_, int(n), gr, st_);
  else
    launch_energy_jobs(d_tab_, int(n), gr, st_);
  BCHK(hipGetLastError());
  BCHK(hipEventRecord(ev_, st_));
  BCHK(hipEventSynchronize(ev_));  // also keeps h_tab_ until its copy is done
}

void EvalBatcher::loop() {
  (void)hipSetDevice(device_);
  std::unique_lock<std::mutex> lk(mu_);
  std::vector<Req*> by_kind[2];
  for (;;) {
    cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
    if (stop_ && q_.empty()) return;
    while (!q_.empty()) {
      Req* r = q_.front();
      q_.pop_front();
      by_kind[r->kind].push_back(r);
    }
    lk.unlock();
    std::string err;
    int64_t nl = 0, nj = 0;
    for (int kind = 0; kind < 2; ++kind) {
      if (by_kind[kind].empty()) continue;
      try {
        launch(by_kind[kind], kind);
        nl++;
        nj += int64_t(by_kind[kind].size());
      } catch (const HipError& e) {
        err = e.msg;
        for (Req* r : by_kind[kind]) r->err = err;
      }
    }
    lk.lock();
    launches_ += nl;
    jobs_ += nj;
    for (auto& v : by_kind) {
      for (Req* r : v) r->done = true;
      v.clear();
    }
    cv_done_.notify_all();
  }
}

PcgBatcher::PcgBatcher(int device) : device_(device), eval_(device) {
  BCHK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
  lanes_[1].fp32 = true;
  for (Lane& L : lanes_)
    for (auto& e : L.ev) BCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  th_ = std::thread([this] { loop(); });
}

void PcgBatcher::free_lane(Lane& L) {
  for (int k = 0; k < 2; ++k) {
    if (L.d_tab[k]) (void)hipFree(L.d_tab[k]);
    if (L.h_tab[k]) (void)hipHostFree(L.h_tab[k]);
    if (L.h_new[k]) (void)hipHostFree(L.h_new[k]);
    if (L.d_state[k]) (void)hipFree(L.d_state[k]);
    if (L.h_state[k]) (void)hipHostFree(L.h_state[k]);
    L.d_tab[k] = L.h_tab[k] = L.h_new[k] = nullptr;
    L.d_state[k] = L.h_state[k] = nullptr;
  }
  if (L.d_new) (void)hipFree(L.d_new);
  L.d_new = nullptr;
  L.tab_cap = L.new_cap = 0;
}

PcgBatcher::~PcgBatcher() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  th_.join();
  (void)hipStreamSynchronize(st_);
  for (Lane& L : lanes_) {
    free_lane(L);
    for (auto& e : L.ev)
      if (e) (void)hipEventDestroy(e);
  }
  (void)hipStreamDestroy(st_);
}

void PcgBatcher::submit(Job& j, int32_t& ind, int32_t& iters) {
  std::unique_lock<std::mutex> lk(mu_);
  j.id = next_id_++;
  q_.push_back(&j);
  cv_.notify_one();
  cv_done_.wait(lk, [&] { return j.done; });
  if (!j.err.empty()) throw HipError{j.err, PPN_ERR_DEVICE};
  ind = j.ind;
  iters = j.iters;
}

void PcgBatcher::solve(const Dev& D, const PcgVec<double>& V, const double* src, double sign,
                       double rtol, int maxit, int32_t& ind, int32_t& iters) {
  Job j;
  j.D = D;
  j.V64 = V;
  j.src = src;
  j.sign = sign;
  j.tol2 = rtol * rtol;
  j.maxit = maxit;
  submit(j, ind, iters);
}

void PcgBatcher::solve(const Dev& D, const PcgVec<float>& V, const double* src, double sign,
                       double rtol, int maxit, int32_t& ind, int32_t& iters) {
  Job j;
  j.fp32 = true;
  j.D = D;
  j.V32 = V;
  j.src = src;
  j.sign = sign;
  j.tol2 = rtol * rtol;
  j.maxit = maxit;
  submit(j, ind, iters);
}

void PcgBatcher::loop() {
  (void)hipSetDevice(device_);
  std::unique_lock<std::mutex> lk(mu_);
  std::vector<Job*> joining[2], finished;
  for (;;) {
    auto busy = [&] {
      for (const Lane& L : lanes_)
        if (!L.members.empty() || L.pending[0] || L.pending[1]) return true;
      return false;
    };
    cv_.wait(lk, [&] { return stop_ || !q_.empty() || busy(); });
    if (stop_ && q_.empty() && !busy()) return;
    while (!q_.empty()) {
      Job* j = q_.front();
      q_.pop_front();
      joining[j->fp32 ? 1 : 0].push_back(j);
    }
    lk.unlock();
    std::string err;
    int chunks = 0;
    try {
      chunks += step<double>(lanes_[0], joining[0], finished) ? 1 : 0;
      chunks += step<float>(lanes_[1], joining[1], finished) ? 1 : 0;
    } catch (const HipError& e) {
      err = e.msg;
    }
    lk.lock();
    batches_ += chunks;
    if (!err.empty()) {
      // a device error ends every solve in flight
      (void)hipStreamSynchronize(st_);
      for (Lane& L : lanes_) {
        for (Job* j : L.members) finished.push_back(j);
        L.members.clear();
        L.pending[0] = L.pending[1] = false;
      }
      for (auto& jl : joining)
        for (Job* j : jl) finished.push_back(j);
      for (Job* j : finished) j->err = err;
    }
    joining[0].clear();
    joining[1].clear();
    for (Job* j : finished) {
      live_.erase(j->id);
      j->done = true;
      solves_++;
    }
    if (!finished.empty()) cv_done_.notify_all();
    finished.clear();
  }
}

// Hands back the solves whose end the states gathered by chunk `parity` show.
void PcgBatcher::retire(Lane& L, int parity, std::vector<Job*>& finished) {
  if (!L.pending[parity]) return;
  BCHK(hipEventSynchronize(L.ev[parity]));
  L.pending[parity] = false;
  const PcgState* st = L.h_state[parity];
  const std::vector<uint64_t>& ids = L.polled[parity];
  for (size_t k = 0; k < ids.size(); ++k) {
    auto it = live_.find(ids[k]);
    if (it == live_.end() || !st[k].done) continue;  // already handed back, or still running
    Job* j = it->second;
    j->ind = st[k].ind;
    j->iters = st[k].iters;
    live_.erase(it);
    auto m = std::find(L.members.begin(), L.members.end(), j);
    if (m != L.members.end()) L.members.erase(m);
    finished.push_back(j);
  }
}

template <typename M>
void PcgBatcher::reserve(Lane& L, size_t n_tab, size_t n_new, std::vector<Job*>& finished) {
  if (n_tab <= L.tab_cap && n_new <= L.new_cap) return;
  // buffers of chunks in flight may be replaced: let them finish first
  retire(L, L.parity ^ 1, finished);
  retire(L, L.parity, finished);
  BCHK(hipStreamSynchronize(st_));
  const size_t tab = std::max<size_t>({n_tab, 2 * L.tab_cap, 32});
  const size_t nw = std::max<size_t>({n_new, 2 * L.new_cap, 32});
  free_lane(L);
  for (int k = 0; k < 2; ++k) {
    BCHK(hipMalloc(&L.d_tab[k], tab * sizeof(PcgJob<M>)));
    BCHK(hipHostMalloc(&L.h_tab[k], tab * sizeof(PcgJob<M>)));
    BCHK(hipHostMalloc(&L.h_new[k], nw * sizeof(PcgJob<M>)));
    BCHK(hipMalloc(reinterpret_cast<void**>(&L.d_state[k]), tab * sizeof(PcgState)));
    BCHK(hipHostMalloc(reinterpret_cast<void**>(&L.h_state[k]), tab * sizeof(PcgState)));
  }
  BCHK(hipMalloc(&L.d_new, nw * sizeof(PcgJob<M>)));
  L.tab_cap = tab;
  L.new_cap = nw;
}

template <typename M>
static const PcgVec<M>& vec_of(const PcgVec<double>& a, const PcgVec<float>& b);
template <>
const PcgVec<double>& vec_of<double>(const PcgVec<double>& a, const PcgVec<float>&) { return a; }
template <>
const PcgVec<float>& vec_of<float>(const PcgVec<double>&, const PcgVec<float>& b) { return b; }

template <typename M>
static PcgJob<M> entry(const Dev& D, const PcgVec<M>& V, const double* src, double sign, double tol2,
                       int maxit, int wg0, int j0) {
  PcgJob<M> e;
  std::memset(static_cast<void*>(&e), 0, sizeof(e));
  e.D = D;
  e.V = V;
  e.src = src;
  e.sign = sign;
  e.tol2 = tol2;
  e.maxit = maxit;
  e.wg0 = wg0;
  e.j0 = j0;
  return e;
}

template <typename M>
bool PcgBatcher::step(Lane& L, std::vector<Job*>& joining, std::vector<Job*>& finished) {
  if (L.members.empty() && joining.empty()) {
    // nothing to launch; hand back what the last chunks show
    retire(L, L.parity ^ 1, finished);
    retire(L, L.parity, finished);
    return false;
  }
  reserve<M>(L, L.members.size() + joining.size(), joining.size(), finished);
  const int p = L.parity;
  for (Job* j : joining) {
    j->j0 = L.jg;
    live_[j->id] = j;
    L.members.push_back(j);
  }
  const int n = int(L.members.size());
  auto* tab = static_cast<PcgJob<M>*>(L.h_tab[p]);
  int total = 0;
  int64_t mbytes = 0;
  L.polled[p].clear();
  for (int k = 0; k < n; ++k) {
    const Job& j = *L.members[size_t(k)];
    tab[k] = entry<M>(j.D, vec_of<M>(j.V64, j.V32), j.src, j.sign, j.tol2, j.maxit, total, j.j0);
    total += j.D.Gp;
    mbytes += sizeof(M) == 8 ? matrix_bytes(j.D) : matrix_bytes_f32(j.D);
    L.polled[p].push_back(j.id);
  }
  const auto* dtab = static_cast<const PcgJob<M>*>(L.d_tab[p]);
  BCHK(hipMemcpyAsync(L.d_tab[p], L.h_tab[p], size_t(n) * sizeof(PcgJob<M>), hipMemcpyHostToDevice, st_));
  if (!joining.empty()) {
    auto* nt = static_cast<PcgJob<M>*>(L.h_new[p]);
    int tn = 0;
    for (size_t k = 0; k < joining.size(); ++k) {
      const Job& j = *joining[k];
      nt[k] = entry<M>(j.D, vec_of<M>(j.V64, j.V32), j.src, j.sign, j.tol2, j.maxit, tn, j.j0);
      tn += j.D.Gp;
    }
    BCHK(hipMemcpyAsync(L.d_new, L.h_new[p], joining.size() * sizeof(PcgJob<M>), hipMemcpyHostToDevice, st_));
    launch_pcg_batch_init(static_cast<const PcgJob<M>*>(L.d_new), int(joining.size()), tn, st_);
  }
  for (int k = 0; k < kChunk; ++k)
    launch_pcg_batch_iter(dtab, n, total, L.jg + k, k == 0 && !joining.empty(), mbytes, st_);
  L.jg += kChunk;
  launch_pcg_batch_gather(dtab, n, L.d_state[p], st_);
  BCHK(hipGetLastError());
  BCHK(hipMemcpyAsync(L.h_state[p], L.d_state[p], size_t(n) * sizeof(PcgState), hipMemcpyDeviceToHost, st_));
  BCHK(hipEventRecord(L.ev[p], st_));
  L.pending[p] = true;
  // while this chunk runs, hand back what the previous one shows
  retire(L, p ^ 1, finished);
  L.parity ^= 1;
  return true;
}

}  // namespace ppn
