// Conventional SRP map (Eq. SRP_T_IFT with one discrete IFT evaluation per
// candidate, pair and bin; cost Eq. SRPomp):
//   map[f][i] = 2 sum_p sum_k w_k (Re psi_p(k) cos theta - Im psi_p(k) sin theta),
//   theta = 2 pi f_k dt_p(i) = 2 pi k x_s / L,  x_s = dt_p(i) fs.
//
// Same skeleton as the Nyquist kernel: per pair, a product of a phase matrix
// [candidates x 2K] with the weighted spectra [2K x frames]. Each matrix-core
// step consumes two bins (k = 2s + g for lane half g) as two instructions:
// A = w_k Re psi with B = cos theta, and A = -w_k Im psi with B = sin theta.
// The phasor of each lane is advanced by a rotation through 2 bins; it is
// re-anchored at every 32-bin chunk from the float64 phase k x_s / L reduced
// mod 1, so rounding drift spans at most 16 rotations.
#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

constexpr int kKC = 32;          // bins per LDS chunk (16 steps)
constexpr int kCStride = kKC + 1;

struct ConvArgs {
  const double* cand;
  const double* mic;
  const PairDesc* pairs;
  int P;
  const float2* psi;   // [F][P][K]
  const float* binw;   // [K]
  int F;
  int K;
  int L;
  int64_t J;
  double fs_over_c;    // metres -> samples
  int far_field;
  float* map;
  unsigned long long* keys;
};

__device__ __forceinline__ double pair_xs(const ConvArgs& a, const PairDesc& pd, double qx,
                                          double qy, double qz) {
  const double* pm = a.mic + 3 * pd.m;
  const double* pn = a.mic + 3 * pd.mp;
  if (a.far_field) {
    return ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * a.fs_over_c;
  }
  const double ax = qx - pm[0], ay = qy - pm[1], az = qz - pm[2];
  const double bx = qx - pn[0], by = qy - pn[1], bz = qz - pn[2];
  return (sqrt(ax * ax + ay * ay + az * az) - sqrt(bx * bx + by * by + bz * bz)) * a.fs_over_c;
}

// (cos, sin) of 2 pi v for v given in float64 turns, reduced mod 1 in float64.
__device__ __forceinline__ void phasor_turns(double v, float* c, float* s) {
  const float t = static_cast<float>(v - rint(v));  // [-1/2, 1/2]
  sincospif(2.0f * t, s, c);
}

template <int CT, int FT>
__global__ __launch_bounds__(256) void conventional_f32_kernel(ConvArgs a) {
  constexpr int FB = 32 * FT;
  constexpr int JW = 32 * CT;
  constexpr int JB = 4 * JW;
  __shared__ float re_s[FB * kCStride];
  __shared__ float im_s[FB * kCStride];
  __shared__ unsigned long long kbest[FB];

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int cl = lane & 31;
  const int g = lane >> 5;
  const int64_t jb = (int64_t)blockIdx.x * JB + wave * JW;
  const int f0 = blockIdx.y * FB;
  const double invL = 1.0 / a.L;

  double qx[CT], qy[CT], qz[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    int64_t ci = jb + ct * 32 + cl;
    ci = ci < a.J ? ci : a.J - 1;
    qx[ct] = a.cand[ci];
    qy[ct] = a.cand[a.J + ci];
    qz[ct] = a.cand[2 * a.J + ci];
  }
  for (int i = tid; i < FB; i += 256) kbest[i] = 0ull;

  floatx16 acc[CT][FT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[ct][ft][r] = 0.0f;

  for (int p = 0; p < a.P; ++p) {
    const PairDesc pd = a.pairs[p];
    double xs[CT];
    float rc[CT], rs[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      xs[ct] = pair_xs(a, pd, qx[ct], qy[ct], qz[ct]);
      phasor_turns(2.0 * xs[ct] * invL, &rc[ct], &rs[ct]);  // rotation by two bins
    }
    const float2* prow = a.psi + (size_t)p * a.K;
    for (int k0 = 0; k0 < a.K; k0 += kKC) {
      __syncthreads();
      // stage w_k Re psi and -w_k Im psi as [frame][bin]
      for (int row = 2 * wave + g; row < FB; row += 8) {
        const int fg = f0 + row;
        const int k = k0 + cl;
        float vr = 0.0f, vi = 0.0f;
        if (fg < a.F && k < a.K) {
          const float2 v = prow[(size_t)fg * a.P * a.K + k];
          const float w = a.binw[k];
          vr = w * v.x;
          vi = -w * v.y;
        }
        re_s[row * kCStride + cl] = vr;
        im_s[row * kCStride + cl] = vi;
      }
      __syncthreads();
      float cs[CT], sn[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        phasor_turns(static_cast<double>(k0 + g) * xs[ct] * invL, &cs[ct], &sn[ct]);
      const int remain = a.K - k0;
      const int steps = remain >= kKC ? kKC / 2 : (remain + 1) / 2;
      const float* rrow = re_s + cl * kCStride + g;
      const float* irow = im_s + cl * kCStride + g;
      for (int s = 0; s < steps; ++s) {
        float ar[FT], ai[FT];
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) {
          ar[ft] = rrow[ft * 32 * kCStride + 2 * s];
          ai[ft] = irow[ft * 32 * kCStride + 2 * s];
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int ft = 0; ft < FT; ++ft) {
            acc[ct][ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[ft], cs[ct], acc[ct][ft], 0, 0, 0);
            acc[ct][ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[ft], sn[ct], acc[ct][ft], 0, 0, 0);
          }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const float c2 = cs[ct] * rc[ct] - sn[ct] * rs[ct];
          const float s2 = cs[ct] * rs[ct] + sn[ct] * rc[ct];
          cs[ct] = c2;
          sn[ct] = s2;
        }
      }
    }
  }

#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int fl = ft * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
      const int fg = f0 + fl;
      unsigned long long best = 0ull;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int64_t ci = jb + ct * 32 + cl;
        const float v = 2.0f * acc[ct][ft][r];
        if (ci < a.J && fg < a.F) {
          if (a.map) a.map[(size_t)fg * a.J + ci] = v;
          const unsigned long long k = peak_key(v, static_cast<unsigned>(ci));
          best = k > best ? k : best;
        }
      }
      if (a.keys) {
        best = half_wave_max(best);
        if (cl == 0 && best) atomicMax(&kbest[fl], best);
      }
    }
  }
  if (a.keys) {
    __syncthreads();
    for (int i = tid; i < FB; i += 256) {
      const unsigned long long k = kbest[i];
      if (k && f0 + i < a.F) atomicMax(a.keys + 2 * (size_t)(f0 + i), k);
    }
  }
}

// Float64 instance (vector units), one thread per candidate, 8 frames per
// block, phases from the float64 turn count reduced mod 1.
constexpr int kFB64 = 8;

__global__ __launch_bounds__(256) void conventional_f64_kernel(ConvArgs a) {
  __shared__ float2 ps[kFB64 * kKC];
  __shared__ unsigned long long kbest[kFB64];
  const int tid = threadIdx.x;
  const int64_t ci0 = (int64_t)blockIdx.x * 256 + tid;
  const int64_t ci = ci0 < a.J ? ci0 : a.J - 1;
  const int f0 = blockIdx.y * kFB64;
  const double qx = a.cand[ci], qy = a.cand[a.J + ci], qz = a.cand[2 * a.J + ci];
  if (tid < kFB64) kbest[tid] = 0ull;
  double acc[kFB64];
#pragma unroll
  for (int f = 0; f < kFB64; ++f) acc[f] = 0.0;
  for (int p = 0; p < a.P; ++p) {
    const PairDesc pd = a.pairs[p];
    const double xsv = pair_xs(a, pd, qx, qy, qz);
    for (int k0 = 0; k0 < a.K; k0 += kKC) {
      __syncthreads();
      for (int e = tid; e < kFB64 * kKC; e += 256) {
        const int f = e / kKC, k = k0 + (e - f * kKC);
        const int fg = f0 + f;
        float2 v = make_float2(0.0f, 0.0f);
        if (fg < a.F && k < a.K) {
          v = a.psi[((size_t)fg * a.P + p) * a.K + k];
          v.x *= a.binw[k];
          v.y *= a.binw[k];
        }
        ps[e] = v;
      }
      __syncthreads();
      const int kn = a.K - k0 < kKC ? a.K - k0 : kKC;
      for (int kk = 0; kk < kn; ++kk) {
        const double v = static_cast<double>(k0 + kk) * xsv / a.L;
        double sn, cs;
        sincospi(2.0 * (v - rint(v)), &sn, &cs);
#pragma unroll
        for (int f = 0; f < kFB64; ++f) {
          const float2 z = ps[f * kKC + kk];
          acc[f] += static_cast<double>(z.x) * cs - static_cast<double>(z.y) * sn;
        }
      }
    }
  }
  for (int f = 0; f < kFB64; ++f) {
    const int fg = f0 + f;
    const float v = static_cast<float>(2.0 * acc[f]);
    unsigned long long k = 0ull;
    if (ci0 < a.J && fg < a.F) {
      if (a.map) a.map[(size_t)fg * a.J + ci0] = v;
      k = peak_key(v, static_cast<unsigned>(ci0));
    }
    if (a.keys) {
      k = wave_max(k);
      if ((tid & 63) == 0 && k) atomicMax(&kbest[f], k);
    }
  }
  if (a.keys) {
    __syncthreads();
    if (tid < kFB64 && f0 + tid < a.F && kbest[tid]) atomicMax(a.keys + 2 * (size_t)(f0 + tid), kbest[tid]);
  }
}

}  // namespace

hipError_t launch_conventional(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                               float* map, unsigned long long* keys, hipStream_t s) {
  ConvArgs a;
  a.cand = g->d_cand;
  a.mic = g->d_mic;
  a.pairs = g->d_pairs;
  a.P = g->info.P;
  a.psi = psi;
  a.binw = g->d_binw;
  a.F = F;
  a.K = g->info.K;
  a.L = g->info.L;
  a.J = g->info.J;
  a.fs_over_c = g->fs_over_c;
  a.far_field = g->info.field == SRP_FAR_FIELD;
  a.map = map;
  a.keys = keys;
  if (dtype == SRP_FP32) {
    constexpr int CT = 2, FT = 2;
    constexpr int JB = 4 * 32 * CT, FB = 32 * FT;
    dim3 grid(static_cast<unsigned>((a.J + JB - 1) / JB), (F + FB - 1) / FB);
    hipLaunchKernelGGL((conventional_f32_kernel<CT, FT>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (dtype == SRP_FP64) {
    dim3 grid(static_cast<unsigned>((a.J + 255) / 256), (F + kFB64 - 1) / kFB64);
    hipLaunchKernelGGL(conventional_f64_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return hipErrorNotSupported;
}

}  // namespace srp
