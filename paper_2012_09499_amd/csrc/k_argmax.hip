// Per-frame argmax of an SRP map (Section 2.2), lowest candidate index on ties.
//
// While a map kernel runs, the first 8 bytes of each srp_peak hold a 64-bit
// key (see peak_key) that workgroups combine with atomicMax; peaks_finalize
// turns the key back into (index, value) in place.
#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

__global__ void peaks_init_kernel(unsigned long long* keys, int F) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < F) keys[2 * f] = 0ull;
}

__global__ void peaks_finalize_kernel(srp_peak* peaks, int F) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const unsigned long long key = *reinterpret_cast<const unsigned long long*>(peaks + f);
  srp_peak out;
  out.index = key ? static_cast<int64_t>(key_index(key)) : 0;
  out.value = key ? key_value(key) : __int_as_float(0x7fc00000);
  out.reserved = 0;
  peaks[f] = out;
}

constexpr int kArgmaxPerThread = 8;

__global__ __launch_bounds__(256) void argmax_kernel(const float* __restrict__ map, int64_t J,
                                                      unsigned long long* __restrict__ keys) {
  __shared__ unsigned long long part[4];
  const int f = blockIdx.y;
  const float* row = map + (size_t)f * J;
  const int64_t base = (int64_t)blockIdx.x * 256 * kArgmaxPerThread + threadIdx.x;
  unsigned long long best = 0ull;
#pragma unroll
  for (int e = 0; e < kArgmaxPerThread; ++e) {
    const int64_t i = base + (int64_t)e * 256;
    if (i < J) {
      const unsigned long long k = peak_key(row[i], static_cast<unsigned>(i));
      best = k > best ? k : best;
    }
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) best = part[w] > best ? part[w] : best;
    atomicMax(keys + 2 * (size_t)f, best);
  }
}

}  // namespace

hipError_t launch_peaks_init(srp_peak* peaks, int F, hipStream_t s) {
  hipLaunchKernelGGL(peaks_init_kernel, dim3((F + 255) / 256), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long*>(peaks), F);
  return hipGetLastError();
}

hipError_t launch_peaks_finalize(srp_peak* peaks, int F, hipStream_t s) {
  hipLaunchKernelGGL(peaks_finalize_kernel, dim3((F + 255) / 256), dim3(256), 0, s, peaks, F);
  return hipGetLastError();
}

hipError_t launch_argmax(const float* map, int F, int64_t J, unsigned long long* keys,
                         hipStream_t s) {
  const int64_t per_block = 256 * kArgmaxPerThread;
  dim3 grid(static_cast<unsigned>((J + per_block - 1) / per_block), static_cast<unsigned>(F));
  hipLaunchKernelGGL(argmax_kernel, grid, dim3(256), 0, s, map, J, keys);
  return hipGetLastError();
}

}  // namespace srp
