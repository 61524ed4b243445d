// LDS read throughput of this GPU, the ceiling against which the on-the-fly
// local sum's LDS operand rate is reported.  Two patterns, each in workgroups
// of 256 threads that stage 16 KB in LDS (eight workgroups, 32 wavefronts, to
// a compute unit) and then read it at fixed offsets from the lane's own index:
//   * 16-byte reads (ds_read_b128): thread t reads pair t + 256 k (k < 4) of
//     1024 double pairs;
//   * 8-byte reads two at a time (ds_read2st64_b64, the instruction the local
//     sum's source stencils use): thread t reads element t + 256 k (k < 8) of
//     2048 doubles.
// Every index stays inside its array.  Prints one JSON line with the lane
// bytes read per second of each pattern (the best of five timings of twenty
// launches, after twenty warm-up launches that bring the clocks to their
// loaded state) and the larger as the ceiling.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kElems = 2048;
constexpr int kOuter = 128;
constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) lds_read_b64x2(double* out, int salt) {
  __shared__ double s[kElems];
  for (int i = threadIdx.x; i < kElems; i += kThreads) s[i] = i * 1e-3 + salt;
  __syncthreads();
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const double* p = s + threadIdx.x;   // threadIdx.x + 7 * 256 < 2048
  for (int o = 0; o < kOuter; ++o) {
#pragma unroll
    for (int k = 0; k < 32; k += 4) {
      a0 += p[((k + 0) & 7) * 256];
      a1 += p[((k + 1) & 7) * 256];
      a2 += p[((k + 2) & 7) * 256];
      a3 += p[((k + 3) & 7) * 256];
      if ((k & 7) == 4) asm volatile("" ::: "memory");   // keep every read (no reuse across groups)
    }
    asm volatile("" ::: "memory");
  }
  out[blockIdx.x * kThreads + threadIdx.x] = a0 + a1 + a2 + a3;
}

__global__ void __launch_bounds__(kThreads) lds_read_b128(double* out, int salt) {
  __shared__ double2 s[kElems / 2];
  for (int i = threadIdx.x; i < kElems / 2; i += kThreads) s[i] = make_double2(i * 1e-3 + salt, i * 2e-3);
  __syncthreads();
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const double2* p = s + threadIdx.x;   // threadIdx.x + 3 * 256 < 1024
  for (int o = 0; o < kOuter; ++o) {
#pragma unroll
    for (int k = 0; k < 16; k += 4) {
      const double2 v0 = p[((k + 0) & 3) * 256], v1 = p[((k + 1) & 3) * 256];
      const double2 v2 = p[((k + 2) & 3) * 256], v3 = p[((k + 3) & 3) * 256];
      a0 += v0.x + v0.y;
      a1 += v1.x + v1.y;
      a2 += v2.x + v2.y;
      a3 += v3.x + v3.y;
      asm volatile("" ::: "memory");   // keep every read (no reuse across groups)
    }
    asm volatile("" ::: "memory");
  }
  out[blockIdx.x * kThreads + threadIdx.x] = a0 + a1 + a2 + a3;
}

// Best rate of five timings of twenty launches (bytes: kOuter * 32 doubles a
// lane in both patterns), or a negative value on a HIP error.
double best_rate(void (*kern)(double*, int), int blocks, double* out, hipEvent_t e0, hipEvent_t e1) {
  for (int r = 0; r < 20; ++r) hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, 0, out, r);
  const int launches = 20;
  const double bytes = 8.0 * blocks * kThreads * (double)kOuter * 32.0 * launches;
  double best = 0.0;
  for (int rep = 0; rep < 5; ++rep) {
    if (hipEventRecord(e0) != hipSuccess) return -1.0;
    for (int r = 0; r < launches; ++r) hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, 0, out, r);
    if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess) return -1.0;
    const double rate = bytes / (ms * 1e-3);
    if (rate > best) best = rate;
  }
  return best;
}

}  // namespace

int main() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  const int blocks = ncu * 32;   // four rounds of eight workgroups per compute unit
  double* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * blocks * kThreads) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  const double r64 = best_rate(lds_read_b64x2, blocks, out, e0, e1);
  const double r128 = best_rate(lds_read_b128, blocks, out, e0, e1);
  if (r64 < 0.0 || r128 < 0.0) return 1;
  std::printf("{\"lds_read_bytes_per_s\": %.6e, \"ds_read_b128_bytes_per_s\": %.6e, "
              "\"ds_read2st64_b64_bytes_per_s\": %.6e, \"compute_units\": %d, \"pattern\": \"8 workgroups of 256 "
              "threads per compute unit, best of 5 x 20 launches; the ceiling is the larger rate\"}\n",
              r128 > r64 ? r128 : r64, r128, r64, ncu);
  (void)hipFree(out);
  return 0;
}
