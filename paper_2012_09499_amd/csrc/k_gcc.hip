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

// GCC samples straight from the per-microphone PHAT phasors (the fused path of
// srp_gcc_samples_frames): the same sum as above with psi_p(k) =
// ytil_m(k) conj(ytil_m'(k)) formed on chip, so the cross-spectra are never
// written to memory. The bin weight w_k (1 or 2: exact in float32) is folded
// into a second phase table, wtab = w_k (cos, -sin).
//
// Work unit: one item (up to kGccItemTiles 32-lag tiles of one pair) for 64
// frames. Wave w of a workgroup takes frame tile w & 1 (32 frames) and the
// bin pairs of parity w >> 1, with every tile of the item; the two parities
// are added in LDS at the end, odd into even (a fixed order). Bins go
// through LDS in chunks of 16, double-buffered, copied by the LDS DMA path
// (no registers): the raw phasor rows of both microphones (128 rows of
// 128 bytes; in each row the 16-byte slot of bin pair s sits at position
// s ^ (row & 7), which spreads the reads of 8 consecutive rows over 8 slots)
// and the weighted table rows of the chunk for the item's lags (16 nt + 1
// slots of two lags per row, from the even column at or before the first). A wave forms psi for
// its (frame, bin) lanes from the two phasors and runs two matrix-core
// products per bin pair and tile: for k2 = g (bin 2i + g) one takes the real
// parts against w cos, the other the imaginary parts against -w sin.
//
// The grid is persistent (two workgroups per CU). Items are sorted by tile
// count, largest first. With at least 8 frame blocks, XCD x takes the frame
// blocks x, x + 8, ... (the phasors of 64 frames of every microphone then
// stay in that XCD's L2 while all pairs read them); otherwise the units are
// dealt over all workgroups. Either way a workgroup takes units q, 2n - 1 - q,
// 2n + q, ... of its cost-sorted list (n workgroups share the list), a
// serpentine deal that pairs each expensive unit with a cheap one.
typedef __attribute__((address_space(3))) void* lds_ptr;
constexpr int kPhBytes = 128 * 128;  // 128 phasor rows x 128 bytes
constexpr int kBufBytes = kPhBytes + (16 * (16 * kGccItemTiles + 1) + 63) / 64 * 1024;

struct PhasorArgs {
  const float2* ytil;
  const float2* wtab;
  const GccItem* items;
  const PairDesc* pairs;
  int M, Kr, nw, h_max, n_items, n_fb, F, S;
};

// One work unit with NT lag tiles (see gcc_phasor_kernel). b0 and b1 are two
// distinct LDS arrays: chunk c is read from b0 when c is even and from b1 when
// it is odd, while the next chunk is copied into the other one, so the
// compiler sees that the copies in flight never touch the array being read.
template <int NT, typename OutT>
__device__ __forceinline__ void gcc_phasor_unit(const PhasorArgs& a, const GccItem& it, int fb,
                                                char* b0, char* b1, OutT* __restrict__ xi) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ft = wave & 1;
  const int kh = wave >> 1;
  const int cl = lane & 31;
  const int g = lane >> 5;
  const int n_chunks = a.Kr / 16;
  const PairDesc pd = a.pairs[it.p];
  const int f0 = fb * 64;
  const int j0 = a.h_max - pd.h + it.t0 * 32;  // table column of the item's first lag

  // DMA lanes. Phasors: copy j (0-3) of wave w moves rows 8 (4 w + j) .. +7,
  // lane l -> row 8 (4 w + j) + l / 8, position l % 8 <- bin pair
  // (l % 8) ^ (row % 8); row r < 64 is microphone m, frame f0 + r, else m'.
  unsigned poff[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = 8 * (4 * wave + j) + (lane >> 3);
    int f = f0 + (row & 63);
    f = f < a.F ? f : a.F - 1;
    const int mic = row < 64 ? pd.m : pd.mp;
    // offsets from the frame block's first row: under 64 M Kr 8 bytes < 2^32
    poff[j] = static_cast<unsigned>(((f - f0) * a.M + mic) * a.Kr) * 8u +
              16u * static_cast<unsigned>((lane & 7) ^ (row & 7));
  }
  const char* yblk = reinterpret_cast<const char*>(a.ytil + (size_t)f0 * a.M * a.Kr);
  // table: each chunk row copies SR 16-byte slots from the even column at or
  // before the item's first lag (nw is even, so the slots are aligned); copy
  // ci of the chunk's [16][SR] block goes to wave ci % 4 (lanes past the block
  // repeat its last slot)
  constexpr int SR = 16 * NT + 1;
  constexpr int NTC = (16 * SR + 63) / 64;   // copies per chunk
  constexpr int NTW = (NTC + 3) / 4;         // copies per wave (at most)
  const int codd = j0 & 1;
  const char* tsrc = reinterpret_cast<const char*>(a.wtab + (j0 - codd));
  unsigned toff[NTW];  // under 16 nw 8 bytes
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    int e = 64 * (wave + 4 * j) + lane;
    e = e < 16 * SR ? e : 16 * SR - 1;
    const int r = e / SR;
    toff[j] = static_cast<unsigned>(r * a.nw + 2 * (e - r * SR)) * 8u;
  }
  auto dma = [&](int c, char* buf) __attribute__((always_inline)) {
    const char* ysrc = yblk + (size_t)c * 128;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(ysrc + poff[j]),
                                       (lds_ptr)(buf + (4 * wave + j) * 1024), 16, 0, 0);
    const char* trow = tsrc + (size_t)c * 16 * a.nw * 8;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
      const int ci = wave + 4 * j;
      if (NTC % 4 == 0 || ci < NTC)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(trow + toff[j]),
                                         (lds_ptr)(buf + kPhBytes + ci * 1024), 16, 0, 0);
    }
  };

  floatx16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;

  const int ra = 32 * ft + cl;  // phasor row of microphone m (m' is 64 rows on)
  const int rsw = ra & 7;
  // One chunk: every LDS read of the chunk first (into registers), then the
  // copy of the chunk after next into `nxt` (issued after the reads, so no read
  // waits for it), then the products.
  float2 ya[4], yb[4], bt[4][NT];
  auto chunk = [&](const char* buf, int c_next, char* nxt) __attribute__((always_inline)) {
    const float2* tb = reinterpret_cast<const float2*>(buf + kPhBytes) + codd + cl;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int i = 2 * jj + kh;  // bin pair of the chunk
      const int slot = (i ^ rsw) * 16 + 8 * g;
      ya[jj] = *reinterpret_cast<const float2*>(buf + ra * 128 + slot);
      yb[jj] = *reinterpret_cast<const float2*>(buf + (ra + 64) * 128 + slot);
#pragma unroll
      for (int t = 0; t < NT; ++t) bt[jj][t] = tb[(2 * i + g) * 2 * SR + 32 * t];
    }
    if (c_next < n_chunks) dma(c_next, nxt);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const float pr = ya[jj].x * yb[jj].x + ya[jj].y * yb[jj].y;  // psi of bin 2i + g
      const float pi = ya[jj].y * yb[jj].x - ya[jj].x * yb[jj].y;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(pr, bt[jj][t].x, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(pi, bt[jj][t].y, acc[t], 0, 0, 0);
      }
    }
    // the products stay before the wait for the copy in flight
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };

  // chunk c is read from b0 when even, from b1 when odd; the copy of chunk
  // c + 1 goes to the other array while chunk c is in use
  dma(0, b0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int c = 0; c < n_chunks; c += 2) {
    chunk(b0, c + 1, b1);
    if (c + 1 < n_chunks) chunk(b1, c + 2, b0);
  }

  // the odd bin pairs' partial tiles go to the even waves through LDS (b0 is
  // free after the last barrier)
  floatx16* part = reinterpret_cast<floatx16*>(b0);
  if (kh == 1) {
#pragma unroll
    for (int t = 0; t < NT; ++t) part[(ft * NT + t) * 64 + lane] = acc[t];
  }
  __syncthreads();
  if (kh == 0) {
    // D[frame][lag]: lane (cl, g), register r holds frame 8 (r / 4) + 4 g +
    // r % 4, lag cl of the tile; lags past the window up to the next multiple
    // of kSampleAlign are the layout's gap, written as zeros
    const int W = 2 * pd.h + 1;
    const int Wpad = (W + kSampleAlign - 1) / kSampleAlign * kSampleAlign;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const floatx16 tot = acc[t] + part[(ft * NT + t) * 64 + lane];
      const int lag = (it.t0 + t) * 32 + cl;
      if (lag < Wpad) {
        const bool real = lag < W;
        OutT* col = xi + pd.off + lag;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int f = f0 + 32 * ft + 8 * (r >> 2) + 4 * g + (r & 3);
          if (f < a.F) col[(size_t)f * a.S] = static_cast<OutT>(real ? tot[r] : 0.0f);
        }
      }
    }
  }
  __syncthreads();  // the partial tiles are read before the next unit's copies
}

template <typename OutT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void gcc_phasor_kernel(
    PhasorArgs a, OutT* __restrict__ xi) {
  __shared__ __attribute__((aligned(16))) char b0[kBufBytes];
  __shared__ __attribute__((aligned(16))) char b1[kBufBytes];
  // this workgroup's share of the unit list
  const bool by_xcd = a.n_fb >= 8 && gridDim.x % 8 == 0;
  const int n_share = by_xcd ? gridDim.x / 8 : gridDim.x;
  const int q = by_xcd ? blockIdx.x / 8 : blockIdx.x;
  const int x = blockIdx.x % 8;
  const int nfx = by_xcd ? (a.n_fb - x + 7) / 8 : a.n_fb;  // frame blocks in the list
  const int n_list = a.n_items * nfx;
  for (int k = 0;; ++k) {
    const int v = k * n_share + ((k & 1) ? n_share - 1 - q : q);
    if (v >= n_list) break;
    const GccItem it = a.items[v / nfx];
    const int fb = by_xcd ? x + 8 * (v % nfx) : v % nfx;
    switch (it.nt) {
      case 1: gcc_phasor_unit<1>(a, it, fb, b0, b1, xi); break;
      case 2: gcc_phasor_unit<2>(a, it, fb, b0, b1, xi); break;
      default: gcc_phasor_unit<3>(a, it, fb, b0, b1, xi); break;
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

template <typename OutT>
void launch_gcc_phasor_t(const srp_geometry_s* g, const float2* ytil, int F, OutT* xi,
                         hipStream_t s) {
  PhasorArgs a;
  a.ytil = ytil;
  a.wtab = g->d_gcc_wtable;
  a.items = g->d_gcc_items;
  a.pairs = g->d_pairs;
  a.M = g->info.M;
  a.Kr = g->Kr;
  a.nw = g->gcc_nw;
  a.h_max = g->info.h_max;
  a.n_items = static_cast<int>(g->gcc_items.size());
  a.n_fb = (F + 63) / 64;
  a.F = F;
  a.S = static_cast<int>(g->info.S);
  // two resident workgroups per CU (the kernel's LDS budget), a multiple of 8
  int slots = 2 * g->n_cu / 8 * 8;
  if (slots < 8) slots = 8;
  hipLaunchKernelGGL(gcc_phasor_kernel<OutT>, dim3(slots), dim3(256), 0, s, a, xi);
}

hipError_t launch_gcc_phasor(const srp_geometry_s* g, const float2* ytil, int F, int dtype,
                             void* xi, hipStream_t s) {
  if (dtype == SRP_FP32)
    launch_gcc_phasor_t(g, ytil, F, static_cast<float*>(xi), s);
  else if (dtype == SRP_BF16)
    launch_gcc_phasor_t(g, ytil, F, static_cast<__bf16*>(xi), s);
  else if (dtype == SRP_FP16)
    launch_gcc_phasor_t(g, ytil, F, static_cast<_Float16*>(xi), s);
  else
    return hipErrorNotSupported;
  return hipGetLastError();
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
