// HBM read rate of a plain streaming kernel: the reference the matrix
// product's achieved bandwidth is read against.
//
// Sums a resident FP64 buffer of `mib` MiB with 16-byte loads, non-temporal or
// ordinary, 4 or 8 loads in flight per thread, over grids of 4, 8 or 16
// workgroups of 256 threads per CU in a grid-stride loop, each workgroup
// writing its partial sum to out[blockIdx.x].  Timed with HIP events over
// `reps` launches after two warm-up launches; prints one JSON line per
// configuration.  Grids are checked against the partials buffer on the host.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s: %s (line %d)\n", #x, hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

typedef double f64x2 __attribute__((ext_vector_type(2)));
constexpr int kBlock = 256;
constexpr int kMaxGrid = 1 << 14;

template <bool kNt, int kU>
__global__ __launch_bounds__(kBlock) void read_sum(const f64x2* __restrict__ v, long long n2, double* out) {
  __shared__ double part[kBlock / 64];
  const long long stride = (long long)gridDim.x * kBlock;
  double s = 0.0;
  long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  for (; i + (kU - 1) * stride < n2; i += kU * stride) {
    f64x2 a[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) a[k] = kNt ? __builtin_nontemporal_load(v + i + k * stride) : v[i + k * stride];
#pragma unroll
    for (int k = 0; k < kU; ++k) s += a[k].x + a[k].y;
  }
  for (; i < n2; i += stride) {
    const f64x2 a = kNt ? __builtin_nontemporal_load(v + i) : v[i];
    s += a.x + a.y;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ void fill(f64x2* v, long long n2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long long)gridDim.x * blockDim.x)
    v[i] = f64x2{1.0, 1.0};
}

template <bool kNt, int kU>
static void run(const f64x2* v, long long n2, double* out, int grid, int reps, long long bytes) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  for (int r = 0; r < 2; ++r) read_sum<kNt, kU><<<grid, kBlock>>>(v, n2, out);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < reps; ++r) read_sum<kNt, kU><<<grid, kBlock>>>(v, n2, out);
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  double host[1];
  CHECK(hipMemcpy(host, out, sizeof(double), hipMemcpyDeviceToHost));
  const double s = ms * 1e-3 / reps;
  std::printf("{\"metric\": \"plain read of a resident FP64 buffer\", \"loads\": \"%s\", \"in_flight\": %d, "
              "\"bytes\": %lld, \"us\": %.2f, \"GB_per_s\": %.1f, \"frac_of_8TBps\": %.4f, \"grid\": %d}\n",
              kNt ? "non-temporal 16-byte" : "ordinary 16-byte", kU, bytes, s * 1e6, bytes / s / 1e9,
              bytes / s / 8e12, grid);
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
}

int main(int argc, char** argv) {
  const long long mib = argc > 1 ? std::atoll(argv[1]) : 1024;
  const int reps = argc > 2 ? std::atoi(argv[2]) : 20;
  if (mib < 1 || mib > 65536 || reps < 1) {
    std::fprintf(stderr, "usage: read_bw [MiB 1..65536] [reps >= 1]\n");
    return 2;
  }
  const long long bytes = mib << 20;
  const long long n2 = bytes / 16;
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  if (cus < 1 || cus * 16 > kMaxGrid) {
    std::fprintf(stderr, "grid %d outside 1..%d\n", cus * 16, kMaxGrid);
    return 1;
  }
  f64x2* v = nullptr;
  double* out = nullptr;
  CHECK(hipMalloc(&v, bytes));
  CHECK(hipMalloc(&out, kMaxGrid * sizeof(double)));
  fill<<<1024, 256>>>(v, n2);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  for (int per_cu : {4, 8, 16}) {
    const int grid = cus * per_cu;
    run<true, 4>(v, n2, out, grid, reps, bytes);
    run<true, 8>(v, n2, out, grid, reps, bytes);
    run<false, 4>(v, n2, out, grid, reps, bytes);
    run<false, 8>(v, n2, out, grid, reps, bytes);
  }
  CHECK(hipFree(v));
  CHECK(hipFree(out));
  return 0;
}
