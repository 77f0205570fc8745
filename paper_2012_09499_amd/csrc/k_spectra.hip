// Frequency-domain GCC (Eq. corrmatrix with the PHAT weight).
//
// Step 1 (fft_phat): one workgroup per (frame, microphone) applies the window,
// runs a radix-2 decimation-in-time FFT of length L in LDS, and keeps the
// phase of every one-sided bin: ytil = Y / |Y| (0 where Y = 0). Because
// |Y_m Y_m'^*| = |Y_m| |Y_m'|, the PHAT-weighted cross-spectrum of a pair is
// the product of the two unit phasors, so each microphone is normalised once
// instead of once per pair.
//
// Step 2 (cross): psi_p(k) = ytil_m(k) conj(ytil_m'(k)) for every pair,
// written as interleaved complex float32 [F][P][K].
#include <mutex>

#include "srp_internal.h"

namespace srp {
namespace {

__device__ __forceinline__ float2 unit_phase(float2 v) {
  const float mx = fmaxf(fabsf(v.x), fabsf(v.y));
  if (!(mx > 0.0f)) return make_float2(0.0f, 0.0f);
  const float x = v.x / mx;
  const float y = v.y / mx;
  const float n = sqrtf(x * x + y * y);
  return make_float2(x / n, y / n);
}

__global__ __launch_bounds__(256) void fft_phat_kernel(const float* __restrict__ frames,
                                                        const float* __restrict__ win,
                                                        const float2* __restrict__ tw, int L,
                                                        int log2L, int K,
                                                        float2* __restrict__ ytil) {
  extern __shared__ float2 buf[];
  const size_t row = blockIdx.x;  // f * M + m
  const float* y = frames + row * (size_t)L;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    const unsigned r = __brev(static_cast<unsigned>(t)) >> (32 - log2L);
    buf[r] = make_float2(y[t] * win[t], 0.0f);
  }
  __syncthreads();
  const int half = L >> 1;
  for (int s = 0; s < log2L; ++s) {
    const int span = 1 << s;
    for (int b = threadIdx.x; b < half; b += blockDim.x) {
      const int pos = b & (span - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos;
      const int i1 = i0 + span;
      const float2 w = tw[pos << (log2L - 1 - s)];
      const float2 a = buf[i0];
      const float2 c = buf[i1];
      const float2 t = make_float2(w.x * c.x - w.y * c.y, w.x * c.y + w.y * c.x);
      buf[i0] = make_float2(a.x + t.x, a.y + t.y);
      buf[i1] = make_float2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
  float2* out = ytil + row * (size_t)K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) out[k] = unit_phase(buf[k]);
}

__global__ __launch_bounds__(256) void cross_kernel(const float2* __restrict__ ytil,
                                                     const PairDesc* __restrict__ pairs, int M,
                                                     int P, int K, float2* __restrict__ psi) {
  const size_t fp = blockIdx.x;  // f * P + p
  const int f = static_cast<int>(fp / P);
  const int p = static_cast<int>(fp - (size_t)f * P);
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const PairDesc pd = pairs[p];
  const float2 a = ytil[((size_t)f * M + pd.m) * K + k];
  const float2 b = ytil[((size_t)f * M + pd.mp) * K + k];
  psi[fp * K + k] = make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// Weighted cross-spectra for the BF16/FP16 conventional map: row (f, p) of
// Kp bins, value k = w_k psi_p(k) for k < K and 0 above, (re, im) rounded once
// to T. One thread per bin.
template <typename T>
__global__ __launch_bounds__(256) void spectra_lowp_kernel(const float2* __restrict__ psi,
                                                           const float* __restrict__ binw, int K,
                                                           int Kp, T* __restrict__ out) {
  const size_t row = blockIdx.x;  // f * P + p
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k >= Kp) return;
  float2 v = make_float2(0.0f, 0.0f);
  if (k < K) {
    const float2 z = psi[row * K + k];
    const float w = binw[k];
    v = make_float2(w * z.x, w * z.y);
  }
  T* o = out + (row * Kp + k) * 2;
  o[0] = static_cast<T>(v.x);
  o[1] = static_cast<T>(v.y);
}

}  // namespace

hipError_t launch_spectra_lowp(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                               void* out, hipStream_t s) {
  const size_t rows = (size_t)F * g->info.P;
  const dim3 grid(static_cast<unsigned>(rows), (g->Kp + 255) / 256);
  if (dtype == SRP_BF16)
    hipLaunchKernelGGL(spectra_lowp_kernel<__bf16>, grid, dim3(256), 0, s, psi, g->d_binw,
                       g->info.K, g->Kp, static_cast<__bf16*>(out));
  else
    hipLaunchKernelGGL(spectra_lowp_kernel<_Float16>, grid, dim3(256), 0, s, psi, g->d_binw,
                       g->info.K, g->Kp, static_cast<_Float16*>(out));
  return hipGetLastError();
}

hipError_t launch_fft_phat(const srp_geometry_s* g, const float* frames, int F, float2* ytil,
                           hipStream_t s) {
  const int L = g->info.L;
  const size_t rows = (size_t)F * g->info.M;
  const int threads = L >= 512 ? 256 : (L / 2 >= 64 ? L / 2 : 64);
  hipLaunchKernelGGL(fft_phat_kernel, dim3(static_cast<unsigned>(rows)), dim3(threads),
                     L * sizeof(float2), s, frames, g->d_window, g->d_twiddle, L, g->log2L,
                     g->info.K, ytil);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Library-owned staging of the per-microphone unit phasors for callers that
// cannot allocate device memory (srp_cross_spectra_noalloc). One array per
// GPU, held until the process ends. Every call on a GPU reuses it: fft_phat
// writes every element that cross then reads, so nothing needs clearing, and
// calls that overlap on one GPU race on it.
static __device__ __align__(256) float2 scratch[kCrossStaticElems];

namespace {
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t cross_static_scratch(int device, float2** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device] == nullptr) {
    // the caller has made `device` current: the symbol's address on that GPU
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<float2*>(g_scratch_ptr[device]);
  return hipSuccess;
}

hipError_t launch_cross(const srp_geometry_s* g, const float2* ytil, int F, float2* psi,
                        hipStream_t s) {
  const int K = g->info.K;
  const size_t rows = (size_t)F * g->info.P;
  dim3 grid(static_cast<unsigned>(rows), (K + 255) / 256);
  hipLaunchKernelGGL(cross_kernel, grid, dim3(256), 0, s, ytil, g->d_pairs, g->info.M,
                     g->info.P, K, psi);
  return hipGetLastError();
}

}  // namespace srp
