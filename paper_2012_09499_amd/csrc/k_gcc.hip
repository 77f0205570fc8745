// GCC samples at the critical lags (Section 3.2, first step; cost Eq.
// SRPapproxcompC): xi_p(n T) = sum_k w_k Re[psi_p(k) exp(j 2 pi f_k n T)]
// for |n| <= h_p.
//
// For one pair this is a dense product: rows = frames, inner = 2K (the real
// and imaginary part of each bin), columns = the pair's lags:
//   xi[f][t] = sum_k  (w_k Re psi[f][k]) cos(theta_kt) + (w_k Im psi[f][k]) (-sin(theta_kt)).
// One wave computes a 32-lag tile of one pair for 32 * FT frames with the
// float32 matrix-core instruction v_mfma_f32_32x32x2f32: each step consumes
// one bin (k2 = 0: real part, k2 = 1: imaginary part). The phase table holds
// (cos, -sin) of 2 pi f_k n T, built in float64 on the host with the phase
// reduced exactly mod 2 pi and rounded once. Samples accumulate in float32
// and are stored as OutT (float, bf16 or fp16: one rounding).
#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

// Bins are split over the KS waves of a workgroup (each wave sums a
// contiguous range of bins, so short transforms and few frames still give many
// waves); the partial tiles are added in LDS in wave order, so the result
// does not depend on timing. Each wave prefetches the next group of bins while
// the matrix cores consume the current one.
template <int FT, typename OutT, int KS>
__global__ __launch_bounds__(64 * KS) void gcc_samples_kernel(
    const float2* __restrict__ psi, const float* __restrict__ binw,
    const float2* __restrict__ table, int nw, int h_max, const LagRun* __restrict__ tiles,
    int n_tiles, const PairDesc* __restrict__ pairs, int F, int P, int K, int S,
    OutT* __restrict__ xi) {
  constexpr int U = 4;  // bins per group
  __shared__ floatx16 part[(KS > 1 ? KS - 1 : 1) * FT * 64];
  // Workgroup b runs on XCD b mod 8 (the grid's x extent is a multiple of 8):
  // each XCD takes a contiguous range of lag tiles, so the tiles of one pair
  // (which read the same spectra) share that XCD's L2 instead of each
  // fetching the pair's spectra from HBM.
  const int per_xcd = gridDim.x / 8;
  const int ti = static_cast<int>(blockIdx.x % 8) * per_xcd + static_cast<int>(blockIdx.x / 8);
  if (ti >= n_tiles) return;  // the whole workgroup (padding of the grid)
  const LagRun tl = tiles[ti];
  const PairDesc pd = pairs[tl.p];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & 31;
  const int g = lane >> 5;
  const int fbase = blockIdx.y * 32 * FT;

  // A operand: lane (cl, g) holds A[frame cl][k2 = g] = w_k (Re | Im) psi[f][p][k].
  const float* arow[FT];
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
    int f = fbase + ft * 32 + cl;
    f = f < F ? f : F - 1;
    arow[ft] = reinterpret_cast<const float*>(psi + ((size_t)f * P + tl.p) * K) + g;
  }
  // B operand: lane (cl, g) holds B[k2 = g][lag cl] = (cos | -sin)(theta_k,n).
  const float* brow = reinterpret_cast<const float*>(table + (h_max - pd.h + tl.t0 + cl)) + g;
  const size_t bstride = 2 * (size_t)nw;

  floatx16 acc[FT];
#pragma unroll
  for (int ft = 0; ft < FT; ++ft)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[ft][r] = 0.0f;

  // this wave's bins [k0, k1)
  const int per = (K + KS - 1) / KS;
  const int k0 = wave * per;
  const int k1 = k0 + per < K ? k0 + per : K;
  int k = k0;
  if (k + U <= k1) {
    float b[U], a[U][FT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      b[u] = brow[(size_t)(k + u) * bstride];
      const float wk = binw[k + u];
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) a[u][ft] = arow[ft][2 * (k + u)] * wk;
    }
    for (; k + 2 * U <= k1; k += U) {
      float nb[U], na[U][FT];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        nb[u] = brow[(size_t)(k + U + u) * bstride];
        const float wk = binw[k + U + u];
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) na[u][ft] = arow[ft][2 * (k + U + u)] * wk;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int ft = 0; ft < FT; ++ft)
          acc[ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u][ft], b[u], acc[ft], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        b[u] = nb[u];
#pragma unroll
        for (int ft = 0; ft < FT; ++ft) a[u][ft] = na[u][ft];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
        acc[ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u][ft], b[u], acc[ft], 0, 0, 0);
    k += U;
  }
  for (; k < k1; ++k) {
    const float b = brow[(size_t)k * bstride];
    const float wk = binw[k];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
      acc[ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(arow[ft][2 * k] * wk, b, acc[ft], 0, 0, 0);
  }

  if (KS > 1) {
    if (wave > 0) {
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) part[((wave - 1) * FT + ft) * 64 + lane] = acc[ft];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 1; w < KS; ++w)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) acc[ft] += part[((w - 1) * FT + ft) * 64 + lane];
  }

  // D[frame][lag]: lane (cl, g), register r holds frame 8 (r / 4) + 4 g + r % 4, lag cl.
  // lags past the window up to the next multiple of kSampleAlign are the
  // layout's gap: written as zeros (the window length 2h+1 is odd, so the gap
  // of the last tile always fits in it)
  const int W = 2 * pd.h + 1;
  const int Wpad = (W + kSampleAlign - 1) / kSampleAlign * kSampleAlign;
  const int tl_end = Wpad - tl.t0 < kGccLagTile ? Wpad - tl.t0 : kGccLagTile;
  if (cl < tl_end) {
    const bool real = cl < tl.len;
    OutT* col = xi + pd.off + tl.t0 + cl;
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = fbase + ft * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
        if (f < F) col[(size_t)f * S] = static_cast<OutT>(real ? acc[ft][r] : 0.0f);
      }
  }
}

}  // namespace

template <int FT, int KS, typename OutT>
void launch_gcc(const srp_geometry_s* g, const float2* psi, int F, OutT* xi, hipStream_t s) {
  const int n_tiles = static_cast<int>(g->gcc_tiles.size());
  const int gx = (n_tiles + 7) / 8 * 8;  // a multiple of the 8 XCDs (see the kernel)
  const dim3 grid(gx, (F + 32 * FT - 1) / (32 * FT));
  hipLaunchKernelGGL((gcc_samples_kernel<FT, OutT, KS>), grid, dim3(64 * KS), 0, s, psi,
                     g->d_binw, g->d_gcc_table, g->gcc_nw, g->info.h_max, g->d_gcc_tiles, n_tiles,
                     g->d_pairs, F, g->info.P, g->info.K, static_cast<int>(g->info.S), xi);
}

// Up to 32 frames (serving batches): one 32-frame tile per wave, bins over 8
// waves; more frames: two 32-frame tiles per wave, bins over 4 waves.
template <typename OutT>
void launch_gcc_any(const srp_geometry_s* g, const float2* psi, int F, OutT* xi, hipStream_t s) {
  if (F <= 32)
    launch_gcc<1, 8>(g, psi, F, xi, s);
  else
    launch_gcc<2, 4>(g, psi, F, xi, s);
}

hipError_t launch_gcc_samples(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                              void* xi, hipStream_t s) {
  if (dtype == SRP_FP32)
    launch_gcc_any(g, psi, F, static_cast<float*>(xi), s);
  else if (dtype == SRP_BF16)
    launch_gcc_any(g, psi, F, static_cast<__bf16*>(xi), s);
  else if (dtype == SRP_FP16)
    launch_gcc_any(g, psi, F, static_cast<_Float16*>(xi), s);
  else
    return hipErrorNotSupported;
  return hipGetLastError();
}

}  // namespace srp
