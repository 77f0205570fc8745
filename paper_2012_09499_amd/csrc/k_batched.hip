// Ragged batched Nyquist maps for serving: one launch covers many arrays
// (different microphone counts, pair windows and candidate grids), each with
// a few frames (Eq. SRPapprox summed over pairs, Eq. SRP_T_IFT).
//
// With one to a few frames per array a matrix-core tile would be mostly
// empty, so this kernel runs on the vector units: one thread per candidate,
// one workgroup per 256 candidates of one array. For every lag the thread
// forms its sinc weight (two weights per reciprocal, as in the BF16 kernel)
// and multiplies it into the <= kBatchMaxF frames of the batch; the samples
// are the same for all threads of a workgroup and come from one read-only
// (__restrict__) sample arena, so they arrive through scalar loads (no LDS,
// no barriers). Each pair's contribution is summed separately
// and then added to the total (two-level float32 sum).
//
// BF16 / FP16 samples: the same sum on matrix cores (v_mfma_f32_16x16x32),
// with up to 16 frames per item. A = samples [16 frames x 32 lags] read
// straight from the arena (a 16-byte load per lane, shared by the wave's four
// candidate tiles), B = weights [32 lags x 16 candidates] formed in registers
// from the float64 TDOA split exactly as in the single-array BF16 kernel. Each
// lane computes the split once for its own candidate; the lanes that need it
// for a tile fetch it with a lane shuffle, so no float64 work is repeated.
// Windows are padded with zero samples to multiples of 8 lags, so a lane's
// 8-lag chunk either lies in its pair's padded window or is skipped (zero
// operand); the weights stay finite everywhere and need no mask.
//
// Workgroup b belongs to the item whose [block_begin, block_begin + blocks)
// range contains b (binary search over the item table).
#include <type_traits>

#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

// Two consecutive samples (an even lag and the next) as floats. For 16-bit
// samples both come from one aligned 32-bit word: windows start at multiples
// of 8 samples, so an even lag of the window is 4-byte aligned, and the word
// stays inside the window's zero-padded span.
__device__ __forceinline__ void load_pair(const float* p, float& a, float& b) {
  a = p[0];
  b = p[1];
}
__device__ __forceinline__ void load_pair(const __bf16* p, float& a, float& b) {
  const unsigned u = *reinterpret_cast<const unsigned*>(p);
  a = __uint_as_float(u << 16);
  b = __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ void load_pair(const _Float16* p, float& a, float& b) {
  const unsigned u = *reinterpret_cast<const unsigned*>(p);
  a = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(u & 0xffffu)));
  b = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(u >> 16)));
}

// Eight consecutive samples (starting at a multiple of 8 within a window,
// so 16-bit chunks are 16-byte aligned) as floats; one scalar load when the
// address is uniform.
struct F8 {
  float v[8];
};
struct U4 {
  unsigned u[4];
};
__device__ __forceinline__ void load8(const float* p, float (&x)[8]) {
  const F8 c = *reinterpret_cast<const F8*>(p);
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = c.v[j];
}
__device__ __forceinline__ void load8(const __bf16* p, float (&x)[8]) {
  const U4 c = *reinterpret_cast<const U4*>(p);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[2 * j] = __uint_as_float(c.u[j] << 16);
    x[2 * j + 1] = __uint_as_float(c.u[j] & 0xffff0000u);
  }
}
__device__ __forceinline__ void load8(const _Float16* p, float (&x)[8]) {
  const U4 c = *reinterpret_cast<const U4*>(p);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[2 * j] = static_cast<float>(
        __builtin_bit_cast(_Float16, static_cast<unsigned short>(c.u[j] & 0xffffu)));
    x[2 * j + 1] = static_cast<float>(
        __builtin_bit_cast(_Float16, static_cast<unsigned short>(c.u[j] >> 16)));
  }
}

template <int FMAX, typename T>
__global__ __launch_bounds__(256) void nyquist_batched_kernel(const BatchItemDev* __restrict__ items,
                                                               int n_items,
                                                               const T* __restrict__ xi) {
  // locate this workgroup's item (uniform)
  int lo = 0, hi = n_items - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  const BatchItemDev it = items[lo];
  const int64_t ci0 = (int64_t)(b - it.block_begin) * 256 + threadIdx.x;
  const int64_t ci = ci0 < it.J ? ci0 : it.J - 1;
  const double qx = it.cand[ci], qy = it.cand[it.J + ci], qz = it.cand[2 * it.J + ci];
  constexpr bool kExact = !std::is_same<T, float>::value;
  const double xq_scale = ldexp(1.0, it.xq_exp);

  float tot[FMAX];
#pragma unroll
  for (int f = 0; f < FMAX; ++f) tot[f] = 0.0f;
  int cur_m = -1;
  double rm = 0.0;
  for (int p = 0; p < it.P; ++p) {
    // the pair record is the same for the whole workgroup: keep it in scalar
    // registers so the lag loop is uniform and its sample reads are scalar loads
    const PairDesc pdv = it.pairs[p];
    PairDesc pd;
    pd.m = __builtin_amdgcn_readfirstlane(pdv.m);
    pd.mp = __builtin_amdgcn_readfirstlane(pdv.mp);
    pd.h = __builtin_amdgcn_readfirstlane(pdv.h);
    pd.off = __builtin_amdgcn_readfirstlane(pdv.off);
    const double* pm = it.mic + 3 * pd.m;
    const double* pn = it.mic + 3 * pd.mp;
    double x;
    if (it.far_field) {
      x = ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * it.inv_cT;
    } else {
      if (pd.m != cur_m) {
        rm = norm3(qx - pm[0], qy - pm[1], qz - pm[2]);
        cur_m = pd.m;
      }
      x = (rm - norm3(qx - pn[0], qy - pn[1], qz - pn[2])) * it.inv_cT;
    }
    const double r = rint(x);
    double fd = x - r;
    if (kExact) {
      // BF16/FP16 items: the fraction on the grid 2^-xq_exp (a nonzero grid
      // point), so that every sinc denominator below is an exact float32
      // number (see nyquist_batched_mx_kernel)
      double q = rint(fd * xq_scale);
      q = q != 0.0 ? q : (fd < 0.0 ? -1.0 : 1.0);
      fd = q / xq_scale;
    } else {
      fd = fabs(fd) < 1e-30 ? 1e-30 : fd;
    }
    const float xf = static_cast<float>(fd);
    const float sp = sinpi_over_pi(fd);
    // lag t = 0 .. 2h: n = t - h, x - n = (xr + h - t) + xf
    const int ia = static_cast<int>(r) + pd.h;
    const float q0 = (ia & 1) ? -sp : sp;  // (-1)^(xr - n) sin(pi xf)/pi at t = 0
    float acc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f) acc[f] = 0.0f;
    // rows of frames past the item's F repeat its last frame (branch-free;
    // their sums are discarded)
    const T* row[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f)
      row[f] = xi + it.xi_off + (size_t)(f < it.F ? f : it.F - 1) * it.S + pd.off;
    const int W = 2 * pd.h + 1;
    // the weights of lags t and t + 1 from one reciprocal: d0 = base + xf,
    // d1 = d0 - 1 (base = ia - t), r = q0 / (d0 d1), w0 = d1 r, w1 = -d0 r;
    // FP32 items form each denominator as (exact integer) + xf, BF16/FP16
    // items hold the exact sum base + xf in `base`
    auto pair_weights = [&](float b, float& w0, float& w1) {
      if (kExact) {
        const float qr = q0 * __builtin_amdgcn_rcpf(fmaf(b, b, -b));
        w0 = fmaf(qr, b, -qr);
        w1 = -qr * b;
      } else {
        const float d0 = b + xf;
        const float d1 = (b - 1.0f) + xf;
        const float qr = q0 * __builtin_amdgcn_rcpf(d0 * d1);
        w0 = qr * d1;
        w1 = -qr * d0;
      }
    };
    float base = static_cast<float>(ia) + (kExact ? xf : 0.0f);
    int t = 0;
    // 8 lags per iteration: each frame's 8 samples arrive by one scalar load,
    // issued together before the arithmetic that uses them
    for (; t + 8 <= W; t += 8) {
      float xs[FMAX][8];
#pragma unroll
      for (int f = 0; f < FMAX; ++f) load8(row[f] + t, xs[f]);
#pragma unroll
      for (int j = 0; j < 8; j += 2, base -= 2.0f) {
        float w0, w1;
        pair_weights(base, w0, w1);
#pragma unroll
        for (int f = 0; f < FMAX; ++f) {
          acc[f] = fmaf(w0, xs[f][j], acc[f]);
          acc[f] = fmaf(w1, xs[f][j + 1], acc[f]);
        }
      }
    }
    for (; t + 1 < W; t += 2, base -= 2.0f) {
      float w0, w1;
      pair_weights(base, w0, w1);
#pragma unroll
      for (int f = 0; f < FMAX; ++f) {
        float x0, x1;
        load_pair(row[f] + t, x0, x1);
        acc[f] = fmaf(w0, x0, acc[f]);
        acc[f] = fmaf(w1, x1, acc[f]);
      }
    }
    {  // last lag (W is odd)
      const float w0 = q0 * __builtin_amdgcn_rcpf(kExact ? base : base + xf);
#pragma unroll
      for (int f = 0; f < FMAX; ++f) {
        float x0, x1;  // x1 is the first zero of the window's padding
        load_pair(row[f] + t, x0, x1);
        acc[f] = fmaf(w0, x0, acc[f]);
      }
    }
#pragma unroll
    for (int f = 0; f < FMAX; ++f) tot[f] += acc[f];
  }

  // epilogue: x2, map store, argmax (one 64-bit atomic per wave and frame)
#pragma unroll
  for (int f = 0; f < FMAX; ++f) {
    if (f >= it.F) break;
    const float v = 2.0f * tot[f];
    unsigned long long key = 0ull;
    if (ci0 < it.J) {
      if (it.map) it.map[(size_t)f * it.J + ci0] = v;
      key = peak_key(v, static_cast<unsigned>(ci0));
    }
    if (it.keys) {
      key = wave_max(key);
      if ((threadIdx.x & 63) == 0 && key) atomicMax(it.keys + 2 * (size_t)f, key);
    }
  }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mx16;
template <> struct Mx16<__bf16> {
  typedef bf16x8 type;
  typedef bf16x4 half_type;
  static __device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ floatx4 mfma16(bf16x4 a, bf16x4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
template <> struct Mx16<_Float16> {
  typedef halfx8 type;
  typedef halfx4 half_type;
  static __device__ __forceinline__ floatx4 mfma(halfx8 a, halfx8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ floatx4 mfma16(halfx4 a, halfx4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

// Weights of one lane for N consecutive lags starting at integer offset
// base = xr + h - t0 (so d_j = (base - j) + xf, sign alternating from qs).
template <typename T, typename V, int N>
__device__ __forceinline__ V lag_weights(float base, float xf, float qs) {
  float w[N];
#pragma unroll
  for (int j = 0; j < N; j += 2) {
    const float d0 = (base - static_cast<float>(j)) + xf;
    const float d1 = (base - static_cast<float>(j + 1)) + xf;
    const float qr = qs * __builtin_amdgcn_rcpf(d0 * d1);
    w[j] = qr * d1;
    w[j + 1] = -qr * d0;
  }
  V v;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = static_cast<T>(w[j]);
  return v;
}

// The same weights when the sinc denominators are exact: tb = base + xf is a
// float32 number and so is every tb - j (the fraction lies on a grid chosen
// so), hence d_j = tb - j and d_{j+1} = d_j - 1 need no separate formation:
// with u = d_j, r = qs / (u (u - 1)), w_j = (u - 1) r and w_{j+1} = -u r.
template <typename T, typename V, int N>
__device__ __forceinline__ V lag_weights_exact(float tb, float qs) {
  float w[N];
#pragma unroll
  for (int j = 0; j < N; j += 2) {
    const float u = tb - static_cast<float>(j);
    const float r = qs * __builtin_amdgcn_rcpf(fmaf(u, u, -u));
    w[j] = fmaf(r, u, -r);
    w[j + 1] = -r * u;
  }
  V v;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = static_cast<T>(w[j]);
  return v;
}

// Lane layouts (64 lanes, g = lane / 16, c = lane % 16), result register r
// holding D[4g + r][c] for both:
//   v_mfma_f32_16x16x32: A[c][8g + j], B[8g + j][c], j = 0..7;
//   v_mfma_f32_16x16x16: A[c][4g + j], B[4g + j][c], j = 0..3 (the tail step
//   of a window whose last lags fit in 16).
template <typename T>
__global__ __launch_bounds__(256) void nyquist_batched_mx_kernel(
    const BatchItemDev* __restrict__ items, int n_items, const T* __restrict__ xi) {
  typedef typename Mx16<T>::type vec8;
  typedef typename Mx16<T>::half_type vec4;
  int lo = 0, hi = n_items - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  const BatchItemDev it = items[lo];
  const int lane = threadIdx.x & 63;
  const int c16 = lane & 15;
  const int g = lane >> 4;
  const int64_t wbase = (int64_t)(b - it.block_begin) * 256 + (threadIdx.x & ~63);
  const int64_t own = wbase + lane < it.J ? wbase + lane : it.J - 1;
  const double qx = it.cand[own], qy = it.cand[it.J + own], qz = it.cand[2 * it.J + own];
  // A operand row: frame c16 (rows past the item's frames repeat its last one
  // and are never stored)
  const int fr = c16 < it.F ? c16 : it.F - 1;
  const T* xrow = xi + it.xi_off + (size_t)fr * it.S;

  floatx4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const double xq_scale = ldexp(1.0, it.xq_exp);
  int cur_m = -1;
  double rm = 0.0;
  for (int p = 0; p < it.P; ++p) {
    const PairDesc pdv = it.pairs[p];
    PairDesc pd;
    pd.m = __builtin_amdgcn_readfirstlane(pdv.m);
    pd.mp = __builtin_amdgcn_readfirstlane(pdv.mp);
    pd.h = __builtin_amdgcn_readfirstlane(pdv.h);
    pd.off = __builtin_amdgcn_readfirstlane(pdv.off);
    const double* pm = it.mic + 3 * pd.m;
    const double* pn = it.mic + 3 * pd.mp;
    double x;
    if (it.far_field) {
      x = ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * it.inv_cT;
    } else {
      if (pd.m != cur_m) {
        rm = norm3(qx - pm[0], qy - pm[1], qz - pm[2]);
        cur_m = pd.m;
      }
      x = (rm - norm3(qx - pn[0], qy - pn[1], qz - pn[2])) * it.inv_cT;
    }
    // the fraction rounded to the grid 2^-xq_exp (a nonzero grid point), so
    // that the sinc denominators below are exact float32 numbers; this moves
    // x by at most half a grid step (2^-17 for the serving arrays), a change
    // of the weights far below a BF16/FP16 unit
    const double r = rint(x);
    double fd = x - r;
    double q = rint(fd * xq_scale);
    q = q != 0.0 ? q : (fd < 0.0 ? -1.0 : 1.0);
    fd = q / xq_scale;
    const int xr_own = static_cast<int>(r);
    const float xf_own = static_cast<float>(fd);
    const float sp_own = sinpi_over_pi(fd);
    // tile t uses candidate wbase + 16 t + c16, whose split lane 16 t + c16
    // holds; ia = xr + h is the integer offset of lag 0 (d = (ia - lag) + xf)
    int ia[4];
    float xf[4], sp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int src = 16 * t + c16;
      ia[t] = __shfl(xr_own, src, 64) + pd.h;
      xf[t] = __shfl(xf_own, src, 64);
      sp[t] = __shfl(sp_own, src, 64);
    }
    const int W = 2 * pd.h + 1;
    const int W8 = (W + 7) & ~7;  // the pair's lags plus its zero-filled gap
    const int rem = W & 31;
    // 32-lag steps, then one 16-lag step if the last lags fit in 16
    const int steps = (W >> 5) + (rem > 16 ? 1 : 0);
    const T* src = xrow + pd.off;
    for (int s = 0; s < steps; ++s) {
      const int t0 = 32 * s + 8 * g;  // lane's first lag
      vec8 av;
      if (t0 < W8) {
        av = *reinterpret_cast<const vec8*>(src + t0);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) av[j] = static_cast<T>(0.0f);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int base = ia[t] - t0;
        const float qs = (base & 1) ? -sp[t] : sp[t];
        acc[t] = Mx16<T>::mfma(
            av, lag_weights_exact<T, vec8, 8>(static_cast<float>(base) + xf[t], qs), acc[t]);
      }
    }
    if (rem > 0 && rem <= 16) {
      const int t0 = 32 * steps + 4 * g;
      vec4 av;
      if (t0 < W8) {
        av = *reinterpret_cast<const vec4*>(src + t0);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) av[j] = static_cast<T>(0.0f);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int base = ia[t] - t0;
        const float qs = (base & 1) ? -sp[t] : sp[t];
        acc[t] = Mx16<T>::mfma16(
            av, lag_weights_exact<T, vec4, 4>(static_cast<float>(base) + xf[t], qs), acc[t]);
      }
    }
  }

  // epilogue: x2, map store, argmax (max over the wave's 16 candidates of a
  // 16-lane row, then one 64-bit atomic per wave and frame)
  unsigned long long kmax[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t ci = wbase + 16 * t + c16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 4 * g + r;
      const float v = 2.0f * acc[t][r];
      if (ci < it.J && f < it.F) {
        if (it.map) it.map[(size_t)f * it.J + ci] = v;
        const unsigned long long k = peak_key(v, static_cast<unsigned>(ci));
        kmax[r] = k > kmax[r] ? k : kmax[r];
      }
    }
  }
  if (it.keys) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      unsigned long long k = kmax[r];
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(k, off, 64);
        k = o > k ? o : k;
      }
      if (c16 == 0 && k && 4 * g + r < it.F) atomicMax(it.keys + 2 * (size_t)(4 * g + r), k);
    }
  }
}

__global__ void batch_peaks_kernel(const BatchItemDev* __restrict__ items, int finalize) {
  const BatchItemDev it = items[blockIdx.x];
  const int f = threadIdx.x;
  if (f >= it.F || it.keys == nullptr) return;
  unsigned long long* k = it.keys + 2 * (size_t)f;
  if (!finalize) {
    *k = 0ull;
    return;
  }
  const unsigned long long key = *k;
  srp_peak out;
  out.index = key ? static_cast<int64_t>(key_index(key)) : 0;
  out.value = key ? key_value(key) : __int_as_float(0x7fc00000);
  out.reserved = 0;
  *reinterpret_cast<srp_peak*>(k) = out;
}

}  // namespace

hipError_t launch_nyquist_batched(const BatchItemDev* d_items, int n_vec, int blocks_vec,
                                  int max_f_vec, int n_mx, int blocks_mx, int dtype,
                                  const void* xi, hipStream_t s) {
  const int n_items = n_vec + n_mx;
  hipLaunchKernelGGL(batch_peaks_kernel, dim3(n_items), dim3(kBatchMaxFMx), 0, s, d_items, 0);
  const dim3 blk(256);
  if (n_vec > 0) {
    const dim3 grid(blocks_vec);
    if (dtype == SRP_FP32) {
      const float* x = static_cast<const float*>(xi);
      if (max_f_vec <= 1)
        hipLaunchKernelGGL((nyquist_batched_kernel<1, float>), grid, blk, 0, s, d_items, n_vec, x);
      else if (max_f_vec <= 2)
        hipLaunchKernelGGL((nyquist_batched_kernel<2, float>), grid, blk, 0, s, d_items, n_vec, x);
      else if (max_f_vec <= 4)
        hipLaunchKernelGGL((nyquist_batched_kernel<4, float>), grid, blk, 0, s, d_items, n_vec, x);
      else
        hipLaunchKernelGGL((nyquist_batched_kernel<kBatchMaxF, float>), grid, blk, 0, s, d_items,
                           n_vec, x);
    } else if (dtype == SRP_BF16) {
      const __bf16* x = static_cast<const __bf16*>(xi);
      if (max_f_vec <= 1)
        hipLaunchKernelGGL((nyquist_batched_kernel<1, __bf16>), grid, blk, 0, s, d_items, n_vec, x);
      else
        hipLaunchKernelGGL((nyquist_batched_kernel<kBatchVecMaxF, __bf16>), grid, blk, 0, s,
                           d_items, n_vec, x);
    } else {
      const _Float16* x = static_cast<const _Float16*>(xi);
      if (max_f_vec <= 1)
        hipLaunchKernelGGL((nyquist_batched_kernel<1, _Float16>), grid, blk, 0, s, d_items, n_vec,
                           x);
      else
        hipLaunchKernelGGL((nyquist_batched_kernel<kBatchVecMaxF, _Float16>), grid, blk, 0, s,
                           d_items, n_vec, x);
    }
  }
  if (n_mx > 0) {
    const dim3 grid(blocks_mx);
    if (dtype == SRP_BF16)
      hipLaunchKernelGGL(nyquist_batched_mx_kernel<__bf16>, grid, blk, 0, s, d_items + n_vec, n_mx,
                         static_cast<const __bf16*>(xi));
    else
      hipLaunchKernelGGL(nyquist_batched_mx_kernel<_Float16>, grid, blk, 0, s, d_items + n_vec,
                         n_mx, static_cast<const _Float16*>(xi));
  }
  hipLaunchKernelGGL(batch_peaks_kernel, dim3(n_items), dim3(kBatchMaxFMx), 0, s, d_items, 1);
  return hipGetLastError();
}

}  // namespace srp
