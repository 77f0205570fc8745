// Device helpers shared by the libsrp kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace srp {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// ||(dx, dy, dz)|| in float64 from the hardware reciprocal square root refined
// by two Newton steps y <- y (3/2 - s y^2 / 2) (relative error ~1e-16, far
// below what a TDOA needs); 0 at the origin.
__device__ __forceinline__ double norm3(double dx, double dy, double dz) {
  const double s = dx * dx + dy * dy + dz * dz;
  const double h = 0.5 * s;
  double y = __builtin_amdgcn_rsq(s);
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return s > 0.0 ? s * y : 0.0;
}

// sin(pi x) / pi for |x| <= 1/2: Taylor series of sin in float64,
// x * sum_k (-1)^k pi^(2k) x^(2k) / (2k+1)!, truncated after x^17 (relative
// truncation error < 1e-12 on the interval), then rounded once to float32.
__device__ __forceinline__ float sinpi_over_pi(double x) {
  const double u = x * x;
  double p = 2.531217404137026e-07;  //  pi^16 / 17!
  p = fma(p, u, -6.975873661656377e-06);  // -pi^14 / 15!
  p = fma(p, u, 0.00014842879303107092);  //  pi^12 / 13!
  p = fma(p, u, -0.0023460810354558226);  // -pi^10 / 11!
  p = fma(p, u, 0.02614784781765479);  //  pi^8 / 9!
  p = fma(p, u, -0.1907518241220842);  // -pi^6 / 7!
  p = fma(p, u, 0.8117424252833535);  //  pi^4 / 5!
  p = fma(p, u, -1.6449340668482264);  // -pi^2 / 3!
  p = fma(p, u, 1.0);  // 1
  return static_cast<float>(x * p);
}

// Unsigned key whose integer order is the float order of `v` (finite or inf),
// with the candidate index in the low word so that, among equal values, the
// LOWEST index has the LARGEST key. Key 0 means "no candidate yet".
__device__ __forceinline__ unsigned long long peak_key(float v, unsigned idx) {
  unsigned u = __float_as_uint(v);
  unsigned ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return (static_cast<unsigned long long>(ord) << 32) | (0xFFFFFFFFu - idx);
}

__device__ __forceinline__ float key_value(unsigned long long key) {
  unsigned ord = static_cast<unsigned>(key >> 32);
  unsigned u = (ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord;
  return __uint_as_float(u);
}

__device__ __forceinline__ unsigned key_index(unsigned long long key) {
  return 0xFFFFFFFFu - static_cast<unsigned>(key & 0xFFFFFFFFull);
}

// Max over the 32 lanes of each half of a wave64 (halves stay separate).
__device__ __forceinline__ unsigned long long half_wave_max(unsigned long long k) {
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
    unsigned long long o = __shfl_xor(k, off, 64);
    k = o > k ? o : k;
  }
  return k;
}

// Per-frame argmax of one wave's 32-frame tile over its 32 NC candidates,
// through LDS instead of cross-lane shuffles. The wave writes the values of
// its NC matrix-core tiles (D layout of the 32x32 instructions: lane (cl, g),
// register r holds frame 8 (r / 4) + 4 g + r % 4 and candidate 32 c + cl of
// tile c) into its own block `ep` (32 rows of 32 NC + 1 floats); lane l then
// scans frame l % 32 over candidates 16 NC (l / 32) .. 16 NC (l / 32 + 1) - 1
// in order, keeping the first maximum. Returns the key (value, -index) of that
// maximum, candidate cand0 + its offset, or 0 when every value scanned is
// -inf. v[c][r]: the values, -inf for candidates past the end. Only the
// calling wave uses `ep`, whose LDS operations run in program order.
template <int NC>
__device__ __forceinline__ unsigned long long tile_argmax_key(float* ep, const float (&v)[NC][16],
                                                              int64_t cand0) {
  constexpr int RS = 32 * NC + 1;
  const int lane = threadIdx.x & 63;
  const int cl = lane & 31;
  const int g = lane >> 5;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) ep[(8 * (r >> 2) + 4 * g + (r & 3)) * RS + 32 * c + cl] = v[c][r];
  const float* row = ep + cl * RS + 16 * NC * g;
  float best = -__builtin_inff();
  int bi = 0;
#pragma unroll
  for (int i = 0; i < 16 * NC; ++i) {
    const float x = row[i];
    if (x > best) {
      best = x;
      bi = i;
    }
  }
  return best > -__builtin_inff()
             ? peak_key(best, static_cast<unsigned>(cand0 + 16 * NC * g + bi))
             : 0ull;
}

// Floats of the per-wave LDS blocks of tile_argmax_key.
template <int NC>
constexpr int argmax_block_floats() {
  return 32 * (32 * NC + 1);
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long k) {
  unsigned long long o = __shfl_xor(k, 32, 64);
  k = o > k ? o : k;
  return half_wave_max(k);
}

}  // namespace srp
