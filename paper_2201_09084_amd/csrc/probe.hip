// Throughput of the float atomic additions that deposit_current can accumulate with, on the
// current device (a measurement aid, not a step of the method).  The 3D push sums a chunk's
// current in an LDS box and adds the box to J with global atomics: which precision the box
// holds, and how many entries a flush can afford, follow from these rates.
//
// Each kernel runs AR_BLOCKS workgroups of AR_TPB threads (many per compute unit, so that the
// chip is full); every lane adds 1 AR_ITERS times.  LDS: into a box of AR_NODES words per
// workgroup, the 64 lanes of a wavefront on 64 consecutive words (distinct banks in FP32, bank
// pairs in FP64), the wavefronts of a workgroup on different words.  Global: the lanes of the
// grid on consecutive words of an array, each pass on the next stretch (the flush's pattern:
// distinct consecutive addresses).  Rates are lane additions per second, timed with HIP
// events around one launch after a warm-up launch.
#include <string>

#include "common.h"
#include "pml_pic.h"

namespace pmlpic {

constexpr int AR_TPB = 256;
constexpr int AR_BLOCKS = 4096;
constexpr int AR_NODES = 2048;
constexpr int AR_ITERS = 256;
constexpr long AR_GLOBAL = 1L << 23;   // words of the global target

template <typename T>
__global__ void __launch_bounds__(AR_TPB) k_lds_atomic_rate(T *out) {
  __shared__ T box[AR_NODES];
  for (int q = threadIdx.x; q < AR_NODES; q += AR_TPB) box[q] = T(0);
  __syncthreads();
#pragma unroll 8
  for (int i = 0; i < AR_ITERS; ++i) atomicAdd(&box[(threadIdx.x + i * AR_TPB) & (AR_NODES - 1)], T(1));
  __syncthreads();
  // every box word was hit AR_ITERS * AR_TPB / AR_NODES times: written out so that the adds
  // are not dropped
  out[(size_t)blockIdx.x * AR_TPB + threadIdx.x] = box[threadIdx.x];
}

template <typename T>
__global__ void __launch_bounds__(AR_TPB) k_global_atomic_rate(T *dst) {
  const long lane = (long)blockIdx.x * AR_TPB + threadIdx.x, span = (long)gridDim.x * AR_TPB;
#pragma unroll 8
  for (int i = 0; i < AR_ITERS; ++i) atomic_add(dst + ((lane + i * span) & (AR_GLOBAL - 1)), T(1));
}

namespace {
struct ProbeBuffers {
  void *out = nullptr, *dst = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~ProbeBuffers() {
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    if (dst) (void)hipFree(dst);
    if (out) (void)hipFree(out);
  }
};

bool hip_ok(hipError_t e, const char *what, std::string *err) {
  if (e == hipSuccess) return true;
  if (err) *err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

// one warm-up launch, then one timed launch: lane additions per second
template <class Launch>
bool time_launch(ProbeBuffers &b, Launch launch, double lanes, double *rate, std::string *err) {
  launch();
  if (!hip_ok(hipGetLastError(), "probe launch", err)) return false;
  if (!hip_ok(hipEventRecord(b.e0, b.s), "hipEventRecord", err)) return false;
  launch();
  if (!hip_ok(hipEventRecord(b.e1, b.s), "hipEventRecord", err)) return false;
  if (!hip_ok(hipEventSynchronize(b.e1), "hipEventSynchronize", err)) return false;
  float ms = 0.f;
  if (!hip_ok(hipEventElapsedTime(&ms, b.e0, b.e1), "hipEventElapsedTime", err)) return false;
  *rate = ms > 0.f ? lanes / (1e-3 * ms) : 0.0;
  return true;
}
}  // namespace

int atomic_rates(double rates[4], std::string *err) {
  ProbeBuffers b;
  const size_t out_bytes = sizeof(double) * (size_t)AR_BLOCKS * AR_TPB;
  if (!hip_ok(hipMalloc(&b.out, out_bytes), "hipMalloc", err)) return PML_PIC_E_HIP;
  if (!hip_ok(hipMalloc(&b.dst, sizeof(double) * (size_t)AR_GLOBAL), "hipMalloc", err)) return PML_PIC_E_HIP;
  if (!hip_ok(hipStreamCreate(&b.s), "hipStreamCreate", err)) return PML_PIC_E_HIP;
  if (!hip_ok(hipEventCreate(&b.e0), "hipEventCreate", err)) return PML_PIC_E_HIP;
  if (!hip_ok(hipEventCreate(&b.e1), "hipEventCreate", err)) return PML_PIC_E_HIP;
  if (!hip_ok(hipMemsetAsync(b.dst, 0, sizeof(double) * (size_t)AR_GLOBAL, b.s), "hipMemsetAsync", err)) return PML_PIC_E_HIP;
  const double lanes = (double)AR_BLOCKS * AR_TPB * AR_ITERS;
  const dim3 grid(AR_BLOCKS), block(AR_TPB);
  bool ok = time_launch(b, [&] { hipLaunchKernelGGL(k_lds_atomic_rate<double>, grid, block, 0, b.s, (double *)b.out); },
                        lanes, &rates[0], err) &&
            time_launch(b, [&] { hipLaunchKernelGGL(k_lds_atomic_rate<float>, grid, block, 0, b.s, (float *)b.out); },
                        lanes, &rates[1], err) &&
            time_launch(b, [&] { hipLaunchKernelGGL(k_global_atomic_rate<float>, grid, block, 0, b.s, (float *)b.dst); },
                        lanes, &rates[2], err) &&
            hip_ok(hipMemsetAsync(b.dst, 0, sizeof(double) * (size_t)AR_GLOBAL, b.s), "hipMemsetAsync", err) &&
            time_launch(b, [&] { hipLaunchKernelGGL(k_global_atomic_rate<double>, grid, block, 0, b.s, (double *)b.dst); },
                        lanes, &rates[3], err);
  if (!ok) return PML_PIC_E_HIP;
  return hip_ok(hipStreamSynchronize(b.s), "hipStreamSynchronize", err) ? PML_PIC_OK : PML_PIC_E_HIP;
}

}  // namespace pmlpic
