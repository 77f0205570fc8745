// Nyquist maps from cached weights (Section 3.3: the interpolation weights
// sinc(dt_p(i) / T - n) do not depend on the frames, so they can be built once
// per geometry; cost of the map Eq. SRPapproxcompR).
//
// Weight matrix W [J][Sw] in the packed lag layout of the GCC samples (the
// column of lag n of pair p is off_p + n + h_p; the zero-filled gap columns
// and the columns up to Sw = S rounded up to 128 hold 0):
//   W[i][off_p + t] = sinc(x_p(i) - (t - h_p)),  x_p(i) = dt_p(i) / T,
// every entry computed in float64 (TDOA with sqrt, sin(pi f) by sinpi,
// correctly rounded division) and rounded once to bfloat16 or half.
//
// The map is then the plain product map[f][i] = 2 sum_k W[i][k] xi[f][k]
// over the packed columns: no TDOA and no weight arithmetic per frame batch.
// It runs on v_mfma_f32_32x32x16_{bf16,f16}: workgroup = 256 candidates x
// 256 frames, each of its 8 waves 64 candidates x 128 frames (both operands
// come from LDS here, and this square-ish wave tile reads 6 operand chunks per
// 8 matrix-core instructions, against 9 for 32 candidates x 256 frames);
// samples staged in 64-column tiles through LDS with a conflict-free swizzle;
// the weights of the workgroup's 256 candidates are staged the same way (rows
// of W are 16-byte chunks apart in the operand layout, so direct loads would
// fetch each cache line several times); copies run one tile ahead. The frame
// blocks of a candidate tile are placed on the same XCD at the same time
// (workgroup b runs on XCD b mod 8), so W is read from HBM about once per
// launch.
#include <type_traits>

#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <typename T> struct Mx32;
template <> struct Mx32<__bf16> {
  typedef bf16x8 type;
  static __device__ __forceinline__ floatx16 mfma(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mx32<_Float16> {
  typedef halfx8 type;
  static __device__ __forceinline__ floatx16 mfma(halfx8 a, halfx8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// ---------------------------------------------------------------- weights
// One thread per (candidate, 8-column chunk): the chunk's pair comes from a
// per-chunk table (-1 past the last window), the thread forms x_p(i) once
// and writes the chunk's 8 weights as one 16-byte store (consecutive threads
// write consecutive chunks of a row).
template <typename T>
__global__ __launch_bounds__(256) void weights_kernel(
    const double* __restrict__ cand, int64_t J, const double* __restrict__ mic,
    const PairDesc* __restrict__ pairs, const int* __restrict__ chunk_pair, int nchunk,
    int far_field, double inv_cT, T* __restrict__ w) {
  typedef typename Mx32<T>::type vec8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= J * nchunk) return;
  const int64_t i = idx / nchunk;
  const int ch = static_cast<int>(idx - i * nchunk);
  const int p = chunk_pair[ch];
  vec8 out;
#pragma unroll
  for (int j = 0; j < 8; ++j) out[j] = static_cast<T>(0.0f);
  if (p >= 0) {
    const PairDesc pd = pairs[p];
    const double qx = cand[i], qy = cand[J + i], qz = cand[2 * J + i];
    const double* pm = mic + 3 * pd.m;
    const double* pn = mic + 3 * pd.mp;
    double x;
    if (far_field) {
      x = ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * inv_cT;
    } else {
      const double ax = qx - pm[0], ay = qy - pm[1], az = qz - pm[2];
      const double bx = qx - pn[0], by = qy - pn[1], bz = qz - pn[2];
      x = (sqrt(ax * ax + ay * ay + az * az) - sqrt(bx * bx + by * by + bz * bz)) * inv_cT;
    }
    const double xr = rint(x);
    const double fd = x - xr;  // exact, |fd| <= 1/2
    const double sp = sinpi(fd) / M_PI;
    const int W = 2 * pd.h + 1;
    const int t0 = 8 * ch - pd.off;  // lag index of the chunk's first column
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int t = t0 + j;
      double v = 0.0;
      if (t < W) {
        // x - n = k + fd with the integer k = xr - (t - h)
        const int k = static_cast<int>(xr) + pd.h - t;
        if (fd == 0.0)
          v = k == 0 ? 1.0 : 0.0;
        else
          v = ((k & 1) ? -sp : sp) / (static_cast<double>(k) + fd);
      }
      out[j] = static_cast<T>(v);
    }
  }
  *reinterpret_cast<vec8*>(w + i * (int64_t)nchunk * 8 + 8 * ch) = out;
}

// ---------------------------------------------------------------- map
constexpr int kCWaves = 8;     // waves per workgroup
constexpr int kCFT = 8;        // 32-frame tiles per workgroup
constexpr int kCWC = 4;        // waves along the candidates (x kCWF along the frames)
constexpr int kCWF = kCWaves / kCWC;
constexpr int kCCT = 2;        // 32-candidate tiles per wave
constexpr int kCWT = kCFT / kCWF;  // 32-frame tiles per wave
constexpr int kCTile = 64;     // packed columns per staged tile
constexpr int kCRow = kCTile;  // LDS row length (elements, 128 bytes)
constexpr int kCSteps = kCTile / 16;  // matrix-core steps per tile

struct CachedArgs {
  int64_t J;
  int F, S, Sw;
  int n_ct, n_fb;
  const float* zero;
  float* map;
  unsigned long long* keys;
};

// Copies a [ROWS][64-column] tile into LDS, 16 bytes per lane, 8 rows of 128
// bytes per instruction, chunk c of row r stored at c ^ ((r >> 1) & 7) (the
// LDS serves 16 lanes x 16 bytes over 256 bytes of banks, i.e. two rows; this
// keeps the 16 rows one 16-lane group reads on 16 different chunk slots).
// Source row r is src + min(r, nrows - 1) * ld; columns at or past ncols come
// from the zero buffer. Straight-line code (fixed trip count, selects instead
// of branches), so the compiler can count the outstanding loads exactly.
template <typename T, int ROWS>
__device__ __forceinline__ void stage_tile(const T* __restrict__ src, int64_t ld, int nrows,
                                           int c0, int ncols, const float* zero, T* tile,
                                           int wave, int lane) {
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const int rsub = lane >> 3;
  const int cp = lane & 7;
  static_assert(ROWS % (8 * kCWaves) == 0, "whole row groups per wave");
#pragma unroll
  for (int it = 0; it < ROWS / (8 * kCWaves); ++it) {
    const int rb = 8 * wave + 8 * kCWaves * it;
    const int row = rb + rsub;
    const int c = cp ^ ((row >> 1) & 7);
    const int rr = row < nrows ? row : nrows - 1;
    const int col = c0 + 8 * c;
    const T* real = src + rr * ld + (col < ncols ? col : 0);
    const void* p = col < ncols ? static_cast<const void*>(real) : static_cast<const void*>(zero);
    __builtin_amdgcn_global_load_lds(p, (lds_ptr)(tile + rb * kCRow), 16, 0, 0);
  }
}

template <typename T>
__global__ __launch_bounds__(64 * kCWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
void cached_map_kernel(CachedArgs a, const T* __restrict__ xi, const T* __restrict__ w) {
  typedef typename Mx32<T>::type vec8;
  constexpr int FT = kCFT, FB = 32 * FT, JB = 32 * kCWaves;
  __shared__ __attribute__((aligned(16))) T xs0[FB * kCRow];
  __shared__ __attribute__((aligned(16))) T xs1[FB * kCRow];
  __shared__ __attribute__((aligned(16))) T ws0[JB * kCRow];
  __shared__ __attribute__((aligned(16))) T ws1[JB * kCRow];
  __shared__ unsigned long long kbest[FB];

  // XCD-aware placement: the n_fb frame blocks of one candidate tile are
  // workgroups b, b + 8, ... (same XCD, dispatched together)
  const int b = blockIdx.x;
  const int per = 8 * a.n_fb;
  const int grp = b / per, r = b - grp * per;
  const int ct = grp * 8 + (r & 7);
  const int fb = r >> 3;
  if (ct >= a.n_ct) return;  // whole workgroup: no barrier is skipped by part of it

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int cl = lane & 31;
  const int g = lane >> 5;
  static_assert(JB == 32 * kCCT * kCWC && FT == kCWT * kCWF, "wave tiles cover the workgroup");
  const int wc = wave % kCWC;  // the wave's candidate rows: 64 wc .. 64 wc + 63
  const int wf = wave / kCWC;  // the wave's frame rows: 128 wf .. 128 wf + 127
  const int64_t jb = (int64_t)ct * JB + wc * 32 * kCCT;
  const int f0 = fb * FB;
  const int nrows = a.F - f0 < FB ? a.F - f0 : FB;
  const int64_t j0 = (int64_t)ct * JB;           // first candidate of the workgroup
  const int jrows = a.J - j0 < JB ? static_cast<int>(a.J - j0) : JB;
  const T* wblk = w + j0 * a.Sw;
  const T* xblk = xi + (size_t)f0 * a.S;
  for (int i = tid; i < FB; i += 64 * kCWaves) kbest[i] = 0ull;

  floatx16 acc[kCCT][kCWT];
#pragma unroll
  for (int c = 0; c < kCCT; ++c)
#pragma unroll
    for (int ft = 0; ft < kCWT; ++ft)
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[c][ft][k] = 0.0f;

  // Two buffers each for the sample tile [256 frames][64 columns] and the
  // weight tile [256 candidates][64 columns], both copied with coalesced
  // 16-byte loads; the copies of tile t + 1 run while tile t is contracted.
  // Sw is a multiple of two tiles.
  const int ntiles = a.Sw / kCTile;
  const int rowsw = (cl >> 1) & 7;
  auto stage = [&](int t, T* xb, T* wb) {
    stage_tile<T, FB>(xblk, a.S, nrows, t * kCTile, a.S, a.zero, xb, wave, lane);
    stage_tile<T, JB>(wblk, a.Sw, jrows, t * kCTile, a.Sw, a.zero, wb, wave, lane);
  };
  // Contraction of one staged tile (4 matrix-core steps of 16 columns),
  // software-pipelined: the LDS operands of step s + 1 are read while the
  // matrix cores work on step s (two operand sets), so the read latency is
  // not exposed before every instruction.
  auto contract = [&](const T* xb, const T* wb) {
    const T* trow = xb + (wf * 32 * kCWT + cl) * kCRow;
    const T* wrow = wb + (wc * 32 * kCCT + cl) * kCRow;
    vec8 a0[kCWT], a1[kCWT], b0[kCCT], b1[kCCT];
    auto load = [&](int s, vec8 (&av)[kCWT], vec8 (&bw)[kCCT]) {
      const int pc = (2 * s + g) ^ rowsw;
#pragma unroll
      for (int c = 0; c < kCCT; ++c)
        bw[c] = *reinterpret_cast<const vec8*>(wrow + c * 32 * kCRow + 8 * pc);
#pragma unroll
      for (int ft = 0; ft < kCWT; ++ft)
        av[ft] = *reinterpret_cast<const vec8*>(trow + ft * 32 * kCRow + 8 * pc);
    };
    auto mm = [&](const vec8 (&av)[kCWT], const vec8 (&bw)[kCCT]) {
#pragma unroll
      for (int c = 0; c < kCCT; ++c)
#pragma unroll
        for (int ft = 0; ft < kCWT; ++ft) acc[c][ft] = Mx32<T>::mfma(av[ft], bw[c], acc[c][ft]);
    };
    auto order = [&]() {
      // one matrix-core instruction, the next step's read addresses and LDS
      // reads, then the remaining matrix-core instructions
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, kCWT + kCCT, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, kCCT * kCWT - 1, 0);
      __builtin_amdgcn_sched_barrier(0);  // one step per scheduling region
    };
    static_assert(kCSteps == 4, "the pipeline below is written for 4 steps per tile");
    load(0, a0, b0);
    load(1, a1, b1);
    mm(a0, b0);
    order();
    load(2, a0, b0);
    mm(a1, b1);
    order();
    load(3, a1, b1);
    mm(a0, b0);
    order();
    mm(a1, b1);
  };
  // hand the buffers over: every copy has landed and the LDS reads of the
  // tile just contracted are done; a plain barrier (no memory fence)
  auto handover = [&]() {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
  };

  stage(0, xs0, ws0);
  handover();
  for (int kt = 0; kt < ntiles; kt += 2) {
    stage(kt + 1, xs1, ws1);
    contract(xs0, ws0);
    handover();
    const int kn = kt + 2 < ntiles ? kt + 2 : ntiles - 1;
    stage(kn, xs0, ws0);
    contract(xs1, ws1);
    handover();
  }

  // epilogue: x2, optional map store, argmax per frame tile through the
  // wave's LDS block (the staging buffers are free: waves 0-1 use xs0, 2-3
  // xs1, 4-5 ws0, 6-7 ws1), then the block's LDS max per frame and one global
  // 64-bit atomic per frame and workgroup
  constexpr int kEp = argmax_block_floats<kCCT>();
  static_assert(kCWaves == 8 && FB * kCRow * sizeof(T) >= 2 * kEp * sizeof(float) &&
                    JB * kCRow * sizeof(T) >= 2 * kEp * sizeof(float),
                "two argmax blocks per staging buffer");
  float* ep = reinterpret_cast<float*>(wave < 2 ? xs0 : wave < 4 ? xs1 : wave < 6 ? ws0 : ws1) +
              (wave & 1) * kEp;
#pragma unroll
  for (int ft = 0; ft < kCWT; ++ft) {
    float v[kCCT][16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int fg = f0 + (wf * kCWT + ft) * 32 + 8 * (k >> 2) + 4 * g + (k & 3);
#pragma unroll
      for (int c = 0; c < kCCT; ++c) {
        const int64_t ci = jb + c * 32 + cl;
        v[c][k] = 2.0f * acc[c][ft][k];
        if (a.map && ci < a.J && fg < a.F) a.map[(size_t)fg * a.J + ci] = v[c][k];
        if (ci >= a.J) v[c][k] = -__builtin_inff();
      }
    }
    if (a.keys) {
      const unsigned long long key = tile_argmax_key<kCCT>(ep, v, jb);
      const int fl = (wf * kCWT + ft) * 32 + cl;
      if (key && f0 + fl < a.F) atomicMax(&kbest[fl], key);
    }
  }
  if (a.keys) {
    __syncthreads();
    for (int i = tid; i < FB; i += 64 * kCWaves) {
      const unsigned long long k = kbest[i];
      if (k && f0 + i < a.F) atomicMax(a.keys + 2 * (size_t)(f0 + i), k);
    }
  }
}

}  // namespace

int cached_weight_cols(const srp_geometry_s* g) {
  constexpr int group = 2 * kCTile;
  return static_cast<int>((g->info.S + group - 1) / group * group);
}

hipError_t launch_nyquist_weights(const srp_geometry_s* g, int dtype, void* w, hipStream_t s) {
  const int nchunk = cached_weight_cols(g) / 8;
  const int64_t threads = g->info.J * nchunk;
  const dim3 grid(static_cast<unsigned>((threads + 255) / 256));
  const int far = g->info.field == SRP_FAR_FIELD;
  if (dtype == SRP_BF16)
    hipLaunchKernelGGL(weights_kernel<__bf16>, grid, dim3(256), 0, s, g->d_cand, g->info.J,
                       g->d_mic, g->d_pairs, g->d_chunk_pair, nchunk, far, g->inv_cT,
                       static_cast<__bf16*>(w));
  else
    hipLaunchKernelGGL(weights_kernel<_Float16>, grid, dim3(256), 0, s, g->d_cand, g->info.J,
                       g->d_mic, g->d_pairs, g->d_chunk_pair, nchunk, far, g->inv_cT,
                       static_cast<_Float16*>(w));
  return hipGetLastError();
}

hipError_t launch_nyquist_cached(const srp_geometry_s* g, const void* w, const void* xi, int F,
                                 int dtype, float* map, unsigned long long* keys, hipStream_t s) {
  CachedArgs a;
  a.J = g->info.J;
  a.F = F;
  a.S = static_cast<int>(g->info.S);
  a.Sw = cached_weight_cols(g);
  a.n_ct = static_cast<int>((a.J + 32 * kCWaves - 1) / (32 * kCWaves));
  a.n_fb = (F + 32 * kCFT - 1) / (32 * kCFT);
  a.zero = g->d_zero;
  a.map = map;
  a.keys = keys;
  const int64_t groups = (a.n_ct + 7) / 8;
  const dim3 grid(static_cast<unsigned>(groups * 8 * a.n_fb)), blk(64 * kCWaves);
  if (dtype == SRP_BF16)
    hipLaunchKernelGGL(cached_map_kernel<__bf16>, grid, blk, 0, s, a,
                       static_cast<const __bf16*>(xi), static_cast<const __bf16*>(w));
  else
    hipLaunchKernelGGL(cached_map_kernel<_Float16>, grid, blk, 0, s, a,
                       static_cast<const _Float16*>(xi), static_cast<const _Float16*>(w));
  return hipGetLastError();
}

}  // namespace srp
