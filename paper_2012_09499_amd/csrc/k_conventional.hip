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

constexpr int kKC = 32;          // bins per staged run (16 steps)
// Above this many terms (2 K P) per map value the FP32 kernel sums in two levels.
constexpr int64_t kConvPlainSumMax = 262144;
constexpr int kCStride = 2 * kKC + 1;  // LDS row stride (odd): interleaved re, im

struct ConvArgs {
  const double* cand;
  const double* mic;
  const PairDesc* pairs;
  const LagRun* runs;  // bin runs (p, k0, len), an even number of them
  int n_runs;
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

// x_s = dt fs for the candidate (qx, qy, qz), float64. `exact` selects the
// correctly rounded square root (the float64 exactness kernel) over norm3.
template <bool exact = false>
__device__ __forceinline__ double pair_xs(const ConvArgs& a, const double* __restrict__ mic,
                                          const PairDesc& pd, double qx, double qy, double qz) {
  const double* pm = mic + 3 * pd.m;
  const double* pn = mic + 3 * pd.mp;
  if (a.far_field) {
    return ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * a.fs_over_c;
  }
  const double ax = qx - pm[0], ay = qy - pm[1], az = qz - pm[2];
  const double bx = qx - pn[0], by = qy - pn[1], bz = qz - pn[2];
  if (exact)
    return (sqrt(ax * ax + ay * ay + az * az) - sqrt(bx * bx + by * by + bz * bz)) * a.fs_over_c;
  return (norm3(ax, ay, az) - norm3(bx, by, bz)) * a.fs_over_c;
}

// (cos, sin) of 2 pi v for v given in float64 turns, reduced mod 1 in float64.
__device__ __forceinline__ void phasor_turns(double v, float* c, float* s) {
  const float t = static_cast<float>(v - rint(v));  // [-1/2, 1/2]
  sincospif(2.0f * t, s, c);
}

// Asynchronous copy of one bin run of pair p (interleaved re, im; 2 len
// floats per frame row) into the LDS tile [frame][2 * kKC]; wave w copies rows
// w, w + 4, ... below nrows. Lanes past the run copy its last float.
__device__ __forceinline__ void stage_bins(const ConvArgs& a, const LagRun& run, float* tile,
                                           int f0, int nrows, int wave, int lane) {
  typedef __attribute__((address_space(3))) void* lds_ptr;
  if (run.len <= 0) return;
  const int n = 2 * run.len;
  const int t = lane < n ? lane : n - 1;
  const float* src = reinterpret_cast<const float*>(a.psi) +
                     2 * (((size_t)(f0 + wave) * a.P + run.p) * a.K + run.t0) + t;
  const size_t step = 8 * (size_t)a.P * a.K;  // 4 frames of 2 K floats per pair
  float* dst = tile + wave * kCStride;
  for (int f = wave; f < nrows; f += 4) {
    __builtin_amdgcn_global_load_lds(src, (lds_ptr)dst, 4, 0, 0);
    src += step;
    dst += 4 * kCStride;
  }
}

template <int CT>
struct ConvLane {
  double qx[CT], qy[CT], qz[CT];
  double xs[CT];     // dt fs (samples) for the current pair
  float rc[CT], rs[CT];  // rotation through two bins
  int cur_p;
};

// Contracts one staged bin run into acc: A = (re, im) of psi from LDS,
// B = (w'_k cos theta, -w'_k sin theta) with w'_k = w_k / 2 (the factor 2 of
// the interior bins is applied in the epilogue).
template <int CT, int FT>
__device__ __forceinline__ void conv_run(const ConvArgs& a, const double* __restrict__ mic,
                                         const PairDesc* __restrict__ pairs,
                                         const LagRun& run, ConvLane<CT>& st,
                                         const float* tile, int cl, int g,
                                         floatx16 (&acc)[CT][FT]) {
  if (run.len <= 0) return;
  if (run.p != st.cur_p) {
    st.cur_p = run.p;
    const PairDesc pd = pairs[run.p];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      st.xs[ct] = pair_xs(a, mic, pd, st.qx[ct], st.qy[ct], st.qz[ct]);
      phasor_turns(2.0 * st.xs[ct] / a.L, &st.rc[ct], &st.rs[ct]);
    }
  }
  float cs[CT], sn_[CT];
  int k = run.t0 + g;  // this lane's bin at step 0
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
    phasor_turns(static_cast<double>(k) * st.xs[ct] / a.L, &cs[ct], &sn_[ct]);
  const float* rrow = tile + cl * kCStride + 2 * g;
  const int steps = (run.len + 1) >> 1;
  const int kend = run.t0 + run.len < a.K ? run.t0 + run.len : a.K;
  // software pipeline, two steps per iteration with ping-pong operand sets:
  // the LDS operands of the next step are read while the matrix cores work on
  // the current one
  float ar0[FT], ai0[FT], ar1[FT], ai1[FT];
  auto fetch = [&](int s, float (&ar)[FT], float (&ai)[FT]) {
    const int sc = s < steps ? s : steps - 1;
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      ar[ft] = rrow[ft * 32 * kCStride + 4 * sc];
      ai[ft] = rrow[ft * 32 * kCStride + 4 * sc + 1];
    }
  };
  auto contract = [&](const float (&ar)[FT], const float (&ai)[FT]) {
    const float wk = k >= kend ? 0.0f : (k == 0 || 2 * k == a.L) ? 0.5f : 1.0f;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float bc = wk * cs[ct];
      const float bs = -wk * sn_[ct];
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) {
        acc[ct][ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[ft], bc, acc[ct][ft], 0, 0, 0);
        acc[ct][ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[ft], bs, acc[ct][ft], 0, 0, 0);
      }
      const float c2 = cs[ct] * st.rc[ct] - sn_[ct] * st.rs[ct];
      const float s2 = cs[ct] * st.rs[ct] + sn_[ct] * st.rc[ct];
      cs[ct] = c2;
      sn_[ct] = s2;
    }
    k += 2;
  };
  auto order = [&]() {
    // one matrix-core instruction (operands read a half-iteration earlier),
    // then the next step's LDS reads, then the rest with VALU work between
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * FT, 0);
#pragma unroll
    for (int i = 1; i < 2 * CT * FT; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
  };
  fetch(0, ar0, ai0);
  int s = 0;
  for (; s + 1 < steps; s += 2) {
    fetch(s + 1, ar1, ai1);
    contract(ar0, ai0);
    order();
    fetch(s + 2, ar0, ai0);
    contract(ar1, ai1);
    order();
  }
  if (s < steps) contract(ar0, ai0);
}

// mic, pairs and runs arrive as __restrict__ const kernel parameters so that
// their uniform reads are scalar loads (they then never wait on the
// asynchronous LDS copies in flight).
// COMP: two-level summation (the matrix-core accumulator holds one pair's
// 2K terms and is added into a second float32 accumulator when the pair
// changes), for geometries where one float32 sum over all 2KP terms would
// lose the 1e-5 map accuracy.
template <int CT, int FT, bool COMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void conventional_f32_kernel(ConvArgs a, const double* __restrict__ mic,
                             const PairDesc* __restrict__ pairs,
                             const LagRun* __restrict__ runs) {
  constexpr int FB = 32 * FT;
  constexpr int JW = 32 * CT;
  constexpr int JB = 4 * JW;
  __shared__ float ps0[FB * kCStride];
  __shared__ float ps1[FB * kCStride];
  __shared__ unsigned long long kbest[FB];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int cl = lane & 31;
  const int g = lane >> 5;
  const int64_t jb = (int64_t)blockIdx.x * JB + wave * JW;
  const int f0 = blockIdx.y * FB;
  const int nrows = a.F - f0 < FB ? a.F - f0 : FB;

  ConvLane<CT> st;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    int64_t ci = jb + ct * 32 + cl;
    ci = ci < a.J ? ci : a.J - 1;
    st.qx[ct] = a.cand[ci];
    st.qy[ct] = a.cand[a.J + ci];
    st.qz[ct] = a.cand[2 * a.J + ci];
    st.xs[ct] = 0.0;
    st.rc[ct] = 1.0f;
    st.rs[ct] = 0.0f;
  }
  st.cur_p = -1;
  for (int i = tid; i < FB; i += 256) kbest[i] = 0ull;

  floatx16 acc[CT][FT];
  floatx16 hi[COMP ? CT : 1][COMP ? FT : 1];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[ct][ft][r] = 0.0f;
  if (COMP) {
#pragma unroll
    for (int ct = 0; ct < (COMP ? CT : 1); ++ct)
#pragma unroll
      for (int ft = 0; ft < (COMP ? FT : 1); ++ft)
#pragma unroll
        for (int r = 0; r < 16; ++r) hi[ct][ft][r] = 0.0f;
  }
  auto fold = [&](const LagRun& run) {
    if (COMP && run.len > 0 && run.p != st.cur_p && st.cur_p >= 0) {
#pragma unroll
      for (int ct = 0; ct < (COMP ? CT : 1); ++ct)
#pragma unroll
        for (int ft = 0; ft < (COMP ? FT : 1); ++ft) {
          hi[ct][ft] += acc[ct][ft];
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[ct][ft][r] = 0.0f;
        }
    }
  };

  stage_bins(a, runs[0], ps0, f0, nrows, wave, lane);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int ri = 0; ri < a.n_runs; ri += 2) {
    const LagRun r0 = runs[ri];
    const LagRun r1 = runs[ri + 1];
    stage_bins(a, r1, ps1, f0, nrows, wave, lane);
    fold(r0);
    conv_run<CT, FT>(a, mic, pairs, r0, st, ps0, cl, g, acc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (ri + 2 < a.n_runs) stage_bins(a, runs[ri + 2], ps0, f0, nrows, wave, lane);
    fold(r1);
    conv_run<CT, FT>(a, mic, pairs, r1, st, ps1, cl, g, acc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  if (COMP) {
#pragma unroll
    for (int ct = 0; ct < (COMP ? CT : 1); ++ct)
#pragma unroll
      for (int ft = 0; ft < (COMP ? FT : 1); ++ft) acc[ct][ft] += hi[ct][ft];
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
        const float v = 4.0f * acc[ct][ft][r];
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
    const double xsv = pair_xs<true>(a, a.mic, pd, qx, qy, qz);
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

bool conventional_supports(int dtype) {
  return dtype == SRP_FP32 || dtype == SRP_FP64 || dtype == SRP_BF16 || dtype == SRP_FP16;
}

hipError_t launch_conventional(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                               float* map, unsigned long long* keys, hipStream_t s) {
  ConvArgs a;
  a.cand = g->d_cand;
  a.mic = g->d_mic;
  a.pairs = g->d_pairs;
  a.runs = g->d_conv_runs;
  a.n_runs = static_cast<int>(g->conv_runs.size());
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
    constexpr int FT = 4, FB = 32 * FT;
    if (2 * (int64_t)a.K * a.P <= kConvPlainSumMax) {
      constexpr int CT = 2, JB = 4 * 32 * CT;
      dim3 grid(static_cast<unsigned>((a.J + JB - 1) / JB), (F + FB - 1) / FB);
      hipLaunchKernelGGL((conventional_f32_kernel<CT, FT, false>), grid, dim3(256), 0, s, a,
                         a.mic, a.pairs, a.runs);
    } else {
      constexpr int CT = 1, JB = 4 * 32 * CT;
      dim3 grid(static_cast<unsigned>((a.J + JB - 1) / JB), (F + FB - 1) / FB);
      hipLaunchKernelGGL((conventional_f32_kernel<CT, FT, true>), grid, dim3(256), 0, s, a,
                         a.mic, a.pairs, a.runs);
    }
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
