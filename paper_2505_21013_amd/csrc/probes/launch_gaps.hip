// Launch cost of a chain of dependent kernels: plain stream launches against
// a HIP graph of the same launches, replayed.
//
// One "iteration" is two dependent kernels that hold the GPU for t1 and t2
// microseconds (the two PCG kernels of an iteration: the product and the
// update), over the grid of a scene's PCG launches.  The host enqueues
// `iters` iterations (a) as plain launches on one stream, (b) as replays of a
// graph captured from g iterations of the same launches, and (c) as plain
// launches with an event recorded every 8 iterations and the one before it
// waited on (the solve loop's chunked status reads).  Prints one JSON line per
// (grid, form) with the wall time per iteration; the excess over t1 + t2 is
// what the launches cost.
//
// Each workgroup writes one int to out[blockIdx.x]; grids are checked against
// the buffer's size on the host.  The spin ends by time or by count.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s: %s (line %d)\n", #x, hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

constexpr int kMaxGrid = 4096;

__global__ void hold(int* out, long long ticks) {
  const long long t0 = wall_clock64();
  long long n = 0;
  while (wall_clock64() - t0 < ticks && n < 100000000LL) ++n;
  if (threadIdx.x == 0) out[blockIdx.x] = int(n);
}

template <typename F>
static double per_iteration_us(hipStream_t st, int iters, F enqueue) {
  double us = 0.0;
  for (int rep = 0; rep < 2; ++rep) {  // the first repetition warms up
    CHECK(hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    enqueue();
    CHECK(hipStreamSynchronize(st));
    us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }
  return us / iters;
}

int main(int argc, char** argv) {
  const double t1 = argc > 1 ? std::atof(argv[1]) : 12.0;
  const double t2 = argc > 2 ? std::atof(argv[2]) : 5.0;
  const int iters = 2000;
  const int grids[] = {96, 1080};
  const int graph_iters[] = {2, 4, 8};
  int* out = nullptr;
  CHECK(hipMalloc(&out, kMaxGrid * sizeof(int)));
  hipStream_t st;
  CHECK(hipStreamCreate(&st));
  int khz = 0;
  CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0));
  const long long k1 = (long long)(t1 * khz / 1000.0), k2 = (long long)(t2 * khz / 1000.0);
  hipEvent_t ev[2];
  for (auto& e : ev) CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (int grid : grids) {
    if (grid > kMaxGrid) return 1;
    auto one = [&] {
      hold<<<grid, 256, 0, st>>>(out, k1);
      hold<<<grid, 256, 0, st>>>(out, k2);
    };
    const double plain = per_iteration_us(st, iters, [&] { for (int i = 0; i < iters; ++i) one(); });
    std::printf("{\"grid\": %d, \"form\": \"stream\", \"us_per_iteration\": %.3f, \"held_us\": %.1f}\n",
                grid, plain, t1 + t2);
    const double polled = per_iteration_us(st, iters, [&] {
      for (int c = 0; c < iters / 8; ++c) {
        for (int i = 0; i < 8; ++i) one();
        CHECK(hipEventRecord(ev[c & 1], st));
        if (c > 0) CHECK(hipEventSynchronize(ev[(c & 1) ^ 1]));
      }
    });
    std::printf("{\"grid\": %d, \"form\": \"stream, status read every 8\", \"us_per_iteration\": %.3f, "
                "\"held_us\": %.1f}\n", grid, polled, t1 + t2);
    for (int g : graph_iters) {
      hipGraph_t graph;
      hipGraphExec_t exec;
      CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < g; ++i) one();
      CHECK(hipStreamEndCapture(st, &graph));
      CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      const double gr = per_iteration_us(st, iters, [&] {
        for (int i = 0; i < iters / g; ++i) CHECK(hipGraphLaunch(exec, st));
      });
      std::printf("{\"grid\": %d, \"form\": \"graph of %d iterations\", \"us_per_iteration\": %.3f, "
                  "\"held_us\": %.1f}\n", grid, g, gr, t1 + t2);
      CHECK(hipGraphExecDestroy(exec));
      CHECK(hipGraphDestroy(graph));
    }
  }
  for (auto& e : ev) CHECK(hipEventDestroy(e));
  CHECK(hipStreamDestroy(st));
  CHECK(hipFree(out));
  return 0;
}
