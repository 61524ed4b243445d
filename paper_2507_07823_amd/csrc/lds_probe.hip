// LDS read throughput of this GPU, the ceiling against which the on-the-fly
// local sum's LDS operand rate is reported.  Every workgroup stages 16 KB
// (2048 doubles) in LDS, so eight workgroups (32 wavefronts) share a compute
// unit, and each lane then reads 4096 doubles at fixed offsets from its own
// index: thread t reads element t + 256 k (k < 8), each read pair issued as
// one ds_read2st64_b64 (the instruction the local sum's source stencils use).
// Every index stays inside the 2048-element array.  Prints one JSON line with
// the lane bytes read per second (the best of five timings of twenty launches,
// after twenty warm-up launches).
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kElems = 2048;
constexpr int kOuter = 128;
constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) lds_read(double* out, int salt) {
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
  // warm-up launches bring the clocks to their loaded state; then the best of
  // five measurements of twenty launches each (about 20 ms each)
  for (int r = 0; r < 20; ++r) hipLaunchKernelGGL(lds_read, dim3(blocks), dim3(kThreads), 0, 0, out, r);
  const int launches = 20;
  const double bytes = 8.0 * blocks * kThreads * (double)kOuter * 32.0 * launches;
  double best = 0.0;
  for (int rep = 0; rep < 5; ++rep) {
    if (hipEventRecord(e0) != hipSuccess) return 1;
    for (int r = 0; r < launches; ++r) hipLaunchKernelGGL(lds_read, dim3(blocks), dim3(kThreads), 0, 0, out, r);
    if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess) return 1;
    const double rate = bytes / (ms * 1e-3);
    if (rate > best) best = rate;
  }
  std::printf("{\"lds_read_bytes_per_s\": %.6e, \"compute_units\": %d, \"pattern\": \"ds_read2st64_b64, "
              "8 workgroups of 256 threads per compute unit, best of 5 x 20 launches\"}\n",
              best, ncu);
  (void)hipFree(out);
  return 0;
}
