// Random-access rates of the device: the reference rates for the solve
// engine's roofline. The engine's work is random accesses -- a vertex's state
// word, its row bounds, a neighbour's distance, an atomicMin -- each moving a
// few bytes, so its ceiling is the rate at which the chip serves independent
// random accesses, not HBM bandwidth. These kernels measure that rate for the
// access kinds the engine is made of.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "runtime.h"

namespace sssp {
namespace {

constexpr long long kRows = 1ll << 26;        // 64-byte rows: 4 GiB
constexpr long long kSmallWords = 1ll << 24;  // 8-byte words: 128 MiB
constexpr long long kLargeWords = 1ll << 29;  // 8-byte words: 4 GiB
constexpr long long kAccesses = 1ll << 24;    // per timed launch
constexpr int kProbeWgPerCu = 16;

// SplitMix64's output function (Steele, Lea and Flood, 2014): the position of
// access i, uniform over a power-of-two range.
__device__ __forceinline__ unsigned long long position(unsigned long long i, unsigned long long mask) {
  unsigned long long z = i * 0x9e3779b97f4a7c15ull + 0x632be59bd9b4e019ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return (z ^ (z >> 31)) & mask;
}

__global__ void __launch_bounds__(kBlock) k_probe_rows(const uint4* __restrict__ tab, uint32_t* __restrict__ out) {
  uint32_t acc = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < kAccesses; i += stride) {
    const uint4* r = tab + position((unsigned long long)i, kRows - 1) * 4;
    const uint4 a = r[0], b = r[1], c = r[2], d = r[3];
    acc ^= a.x ^ b.y ^ c.z ^ d.w;
  }
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void __launch_bounds__(kBlock) k_probe_words(const unsigned long long* __restrict__ arr,
                                                        unsigned long long mask, uint32_t* __restrict__ out) {
  unsigned long long acc = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < kAccesses; i += stride)
    acc ^= arr[position((unsigned long long)i, mask)];
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)acc;
}

__global__ void __launch_bounds__(kBlock) k_probe_atomics(unsigned long long* arr, unsigned long long mask) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < kAccesses; i += stride)
    atomicMin(arr + position((unsigned long long)i, mask), (unsigned long long)i);
}

}  // namespace
}  // namespace sssp

using namespace sssp;

extern "C" sssp_status sssp_device_random_rates(sssp_random_rates* out, hipStream_t stream) {
  if (!out) return fail(SSSP_E_INVAL, "out is NULL");
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = std::max(1, cus) * kProbeWgPerCu;
  void* tab = nullptr;
  void* small = nullptr;
  void* large = nullptr;
  void* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (tab) (void)hipFree(tab);
    if (small) (void)hipFree(small);
    if (large) (void)hipFree(large);
    if (sink) (void)hipFree(sink);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&tab, (size_t)kRows * 64) != hipSuccess || hipMalloc(&small, (size_t)kSmallWords * 8) != hipSuccess ||
      hipMalloc(&large, (size_t)kLargeWords * 8) != hipSuccess ||
      hipMalloc(&sink, (size_t)grid * kBlock * sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(SSSP_E_NOMEM, "the random-access probe needs about 8.4 GB of device memory");
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemsetAsync(tab, 1, (size_t)kRows * 64, stream);
  if (e == hipSuccess) e = hipMemsetAsync(small, 0xff, (size_t)kSmallWords * 8, stream);
  if (e == hipSuccess) e = hipMemsetAsync(large, 1, (size_t)kLargeWords * 8, stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4 && e == hipSuccess; ++k) {
    float fastest = 0.0f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, stream);
      if (e != hipSuccess) break;
      if (k == 0)
        hipLaunchKernelGGL(k_probe_rows, dim3(grid), dim3(kBlock), 0, stream, (const uint4*)tab, (uint32_t*)sink);
      else if (k == 1)
        hipLaunchKernelGGL(k_probe_words, dim3(grid), dim3(kBlock), 0, stream, (const unsigned long long*)small,
                           (unsigned long long)(kSmallWords - 1), (uint32_t*)sink);
      else if (k == 2)
        hipLaunchKernelGGL(k_probe_words, dim3(grid), dim3(kBlock), 0, stream, (const unsigned long long*)large,
                           (unsigned long long)(kLargeWords - 1), (uint32_t*)sink);
      else
        hipLaunchKernelGGL(k_probe_atomics, dim3(grid), dim3(kBlock), 0, stream, (unsigned long long*)small,
                           (unsigned long long)(kSmallWords - 1));
      e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      // the first launch of each kind is untimed
      if (e == hipSuccess && rep > 0 && (fastest == 0.0f || ms < fastest)) fastest = ms;
    }
    if (fastest > 0.0f) best[k] = (double)kAccesses / (fastest * 1e-3);
  }
  release();
  if (e != hipSuccess) return fail(SSSP_E_DEVICE, std::string("random-access probe: ") + hipGetErrorString(e));
  *out = sssp_random_rates{};
  out->rows64_per_s = best[0];
  out->words8_small_per_s = best[1];
  out->words8_large_per_s = best[2];
  out->atomics8_small_per_s = best[3];
  out->accesses = kAccesses;
  return ok();
}
