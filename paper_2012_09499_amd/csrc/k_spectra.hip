// Frequency-domain GCC (Eq. corrmatrix with the PHAT weight).
//
// Step 1 (fft_phat): one workgroup per (frame, two microphones) applies the
// window and runs ONE complex FFT of length L on z = y_a + j y_b in LDS
// (Stockham passes of radix 4, a last radix-2 pass when log2 L is odd, one
// barrier per pass). Because y_a and y_b are real, their spectra separate as
// Y_a(k) = (Z(k) + Z(L-k)^*) / 2 and Y_b(k) = (Z(k) - Z(L-k)^*) / (2j). Every
// one-sided bin keeps only its phase, ytil = Y / |Y| (0 where Y = 0, and for a
// microphone whose windowed frame is all zeros): since |Y_m Y_m'^*| =
// |Y_m| |Y_m'|, the PHAT-weighted cross-spectrum of a pair is the product of
// the two unit phasors, so each microphone is normalised once instead of once
// per pair. Rows of ytil hold Kr = K rounded up to 16 bins (zeros past K).
//
// Step 2 (cross): psi_p(k) = ytil_m(k) conj(ytil_m'(k)) for every pair,
// written as interleaved complex float32 [F][P][K].
#include <mutex>

#include "srp_internal.h"

namespace srp {
namespace {

// v / |v| (0 for v = 0). v is first scaled by the hardware reciprocal of
// m = max(|x|, |y|) (1 ulp; below 2^-100, v and m are multiplied by 2^100
// first, exactly, so the reciprocal stays finite), so the squared norm lies
// in [1, 2] and the hardware reciprocal square root (1 ulp) needs no range
// handling: a few ulp in all, far below the float32 FFT's own rounding.
__device__ __forceinline__ float2 unit_phase(float2 v) {
  const float mx = fmaxf(fabsf(v.x), fabsf(v.y));
  if (!(mx > 0.0f)) return make_float2(0.0f, 0.0f);
  const float sc = mx < 0x1p-100f ? 0x1p100f : 1.0f;
  const float r = __builtin_amdgcn_rcpf(mx * sc);
  const float x = (v.x * sc) * r;
  const float y = (v.y * sc) * r;
  const float n = __builtin_amdgcn_rsqf(x * x + y * y);
  return make_float2(x * n, y * n);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int LOG2L>
constexpr int fft_threads() {
  return (1 << LOG2L) / 4 >= 256 ? 256 : ((1 << LOG2L) / 4 >= 64 ? (1 << LOG2L) / 4 : 64);
}

// tw[t] = exp(-j 2 pi t / L), t < L.
template <int LOG2L>
__global__ __launch_bounds__(fft_threads<LOG2L>()) void fft_phat_kernel(
    const float* __restrict__ frames, const float* __restrict__ win,
    const float2* __restrict__ tw, int M, int K, int Kr, float2* __restrict__ ytil) {
  constexpr int L = 1 << LOG2L;
  constexpr int T = fft_threads<LOG2L>();
  __shared__ __attribute__((aligned(16))) float2 buf[2][L];
  const int tid = threadIdx.x;
  const int halves = (M + 1) / 2;
  const int f = static_cast<int>(blockIdx.x) / halves;
  const int ma = 2 * (static_cast<int>(blockIdx.x) - f * halves);
  const bool has_b = ma + 1 < M;
  const float4* ya = reinterpret_cast<const float4*>(frames + ((size_t)f * M + ma) * L);
  const float4* yb = ya + L / 4;
  const float4* w4 = reinterpret_cast<const float4*>(win);

  int nza = 0, nzb = 0;
  for (int t4 = tid; t4 < L / 4; t4 += T) {
    const float4 w = w4[t4];
    const float4 a = ya[t4];
    const float4 b = has_b ? yb[t4] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float4 za = make_float4(w.x * a.x, w.y * a.y, w.z * a.z, w.w * a.w);
    const float4 zb = make_float4(w.x * b.x, w.y * b.y, w.z * b.z, w.w * b.w);
    nza |= (za.x != 0.0f) | (za.y != 0.0f) | (za.z != 0.0f) | (za.w != 0.0f);
    nzb |= (zb.x != 0.0f) | (zb.y != 0.0f) | (zb.z != 0.0f) | (zb.w != 0.0f);
    float4* d = reinterpret_cast<float4*>(&buf[0][4 * t4]);
    d[0] = make_float4(za.x, zb.x, za.y, zb.y);
    d[1] = make_float4(za.z, zb.z, za.w, zb.w);
  }
  nza = __syncthreads_or(nza);
  nzb = __syncthreads_or(nzb);

  // Stockham autosort passes: natural order in, natural order out
  int cur = 0;
#pragma unroll
  for (int Ns = 1; Ns * 4 <= L; Ns *= 4) {
    const float2* src = buf[cur];
    float2* dst = buf[cur ^ 1];
    constexpr int q = L / 4;
    const int step = L / (4 * Ns);
    for (int j = tid; j < q; j += T) {
      const int k = j & (Ns - 1);
      float2 v0 = src[j], v1 = src[j + q], v2 = src[j + 2 * q], v3 = src[j + 3 * q];
      if (Ns > 1) {
        v1 = cmul(v1, tw[k * step]);
        v2 = cmul(v2, tw[2 * k * step]);
        v3 = cmul(v3, tw[3 * k * step]);
      }
      const float2 a0 = make_float2(v0.x + v2.x, v0.y + v2.y);
      const float2 a1 = make_float2(v0.x - v2.x, v0.y - v2.y);
      const float2 a2 = make_float2(v1.x + v3.x, v1.y + v3.y);
      const float2 a3 = make_float2(v1.y - v3.y, v3.x - v1.x);  // -j (v1 - v3)
      const int base = (j - k) * 4 + k;
      dst[base] = make_float2(a0.x + a2.x, a0.y + a2.y);
      dst[base + Ns] = make_float2(a1.x + a3.x, a1.y + a3.y);
      dst[base + 2 * Ns] = make_float2(a0.x - a2.x, a0.y - a2.y);
      dst[base + 3 * Ns] = make_float2(a1.x - a3.x, a1.y - a3.y);
    }
    __syncthreads();
    cur ^= 1;
  }
  if constexpr (LOG2L % 2 == 1) {
    constexpr int Ns = L / 2;
    const float2* src = buf[cur];
    float2* dst = buf[cur ^ 1];
    for (int j = tid; j < L / 2; j += T) {
      const float2 v0 = src[j];
      const float2 v1 = cmul(src[j + L / 2], tw[j]);
      dst[j] = make_float2(v0.x + v1.x, v0.y + v1.y);
      dst[j + Ns] = make_float2(v0.x - v1.x, v0.y - v1.y);
    }
    __syncthreads();
    cur ^= 1;
  }

  // separate the two real spectra, keep the phases, two bins per thread
  const float2* Z = buf[cur];
  float4* oa = reinterpret_cast<float4*>(ytil + ((size_t)f * M + ma) * Kr);
  float4* ob = oa + Kr / 2;
  for (int kp = tid; kp < Kr / 2; kp += T) {
    float2 ra[2], rb[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = 2 * kp + e;
      ra[e] = rb[e] = make_float2(0.0f, 0.0f);
      if (k < K) {
        const float2 z = Z[k];
        const float2 zc = Z[(L - k) & (L - 1)];
        if (nza) ra[e] = unit_phase(make_float2(z.x + zc.x, z.y - zc.y));
        if (nzb) rb[e] = unit_phase(make_float2(z.y + zc.y, zc.x - z.x));
      }
    }
    oa[kp] = make_float4(ra[0].x, ra[0].y, ra[1].x, ra[1].y);
    if (has_b) ob[kp] = make_float4(rb[0].x, rb[0].y, rb[1].x, rb[1].y);
  }
}

__global__ __launch_bounds__(256) void cross_kernel(const float2* __restrict__ ytil,
                                                     const PairDesc* __restrict__ pairs, int M,
                                                     int P, int K, int Kr,
                                                     float2* __restrict__ psi) {
  const size_t fp = blockIdx.x;  // f * P + p
  const int f = static_cast<int>(fp / P);
  const int p = static_cast<int>(fp - (size_t)f * P);
  const int k = blockIdx.y * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const PairDesc pd = pairs[p];
  const float2 a = ytil[((size_t)f * M + pd.m) * Kr + k];
  const float2 b = ytil[((size_t)f * M + pd.mp) * Kr + k];
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

template <int LOG2L>
void launch_fft_phat_l(const srp_geometry_s* g, const float* frames, int F, float2* ytil,
                       hipStream_t s) {
  const size_t blocks = (size_t)F * ((g->info.M + 1) / 2);
  hipLaunchKernelGGL((fft_phat_kernel<LOG2L>), dim3(static_cast<unsigned>(blocks)),
                     dim3(fft_threads<LOG2L>()), 0, s, frames, g->d_window, g->d_twiddle,
                     g->info.M, g->info.K, g->Kr, ytil);
}

hipError_t launch_fft_phat(const srp_geometry_s* g, const float* frames, int F, float2* ytil,
                           hipStream_t s) {
  switch (g->log2L) {
    case 4: launch_fft_phat_l<4>(g, frames, F, ytil, s); break;
    case 5: launch_fft_phat_l<5>(g, frames, F, ytil, s); break;
    case 6: launch_fft_phat_l<6>(g, frames, F, ytil, s); break;
    case 7: launch_fft_phat_l<7>(g, frames, F, ytil, s); break;
    case 8: launch_fft_phat_l<8>(g, frames, F, ytil, s); break;
    case 9: launch_fft_phat_l<9>(g, frames, F, ytil, s); break;
    case 10: launch_fft_phat_l<10>(g, frames, F, ytil, s); break;
    case 11: launch_fft_phat_l<11>(g, frames, F, ytil, s); break;
    case 12: launch_fft_phat_l<12>(g, frames, F, ytil, s); break;
    case 13: launch_fft_phat_l<13>(g, frames, F, ytil, s); break;
    default: return hipErrorInvalidValue;
  }
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
                     g->info.P, K, g->Kr, psi);
  return hipGetLastError();
}

}  // namespace srp
