// BF16 / FP16 Nyquist-Shannon SRP map (Eq. SRPapprox summed over pairs as in
// Eq. SRP_T_IFT; cost Eq. SRPapproxcompR) on v_mfma_f32_32x32x16_{bf16,f16}
// with float32 accumulation:
//   map[f][i] = 2 sum_p sum_{|n| <= h_p} xi_p(nT) sinc(x_p(i) - n).
//
// Layout. A workgroup is 8 waves, two per SIMD, and owns 256 candidates x up
// to 256 frames. Each wave owns 32 candidates and ALL the workgroup's frames
// (FT 32-frame tiles, FT <= 8): every weight a lane forms feeds FT
// matrix-core instructions, and the FT accumulator tiles take 16 FT registers
// per lane. One step consumes 16 lags: lane (cl, g) (cl = lane % 32,
// g = lane / 32) holds lags 8g .. 8g+7 of the step for frame cl of every frame
// tile (A = samples, one 16-byte LDS read per tile) and for candidate cl
// (B = weights, formed in registers).
//
// Samples. Each lag run (<= 128 lags of one pair window, <= 256 with at most
// 4 frame tiles; lagrun records of the geometry) is copied into LDS with 16-byte global-to-LDS copies issued by all
// waves, double-buffered: the next run's copies are in flight while the
// current run is contracted. For each pair of 16-byte chunks and each group of
// 32 rows, the tile holds the rows' first chunks, then their second chunks, so
// one copy instruction lands as 1 KB of contiguous LDS and a step's fragment
// read is 1 KB read in lane order. A chunk past the run repeats the run's last
// chunk and its weights are zeroed instead (a run's last chunk ends at its
// window's end, and the columns between the window's end and the chunk's end
// are the sample layout's zero gap).
//
// Weights. x = xi + xf with xi = rint(x) and the fraction xf rounded to the
// grid 2^-e, e chosen per geometry so that every sinc denominator
// d = (xi - n) + xf (|d| < 2 h_max + 64) is an exact float32 number; a zero
// fraction becomes one grid step. This moves x by at most 2^-(e+1) (2^-17 at
// the room scale), far below a BF16/FP16 unit of the weights. With exact
// denominators a pair of weights costs one fma for d (d - 1), one reciprocal
// and three multiplies: with u = d_j, r = qs / (u (u - 1)),
// w_j = (u - 1) r and w_{j+1} = -u r, qs = (-1)^(xi - n) sin(pi xf) / pi.
// TDOAs are float32 per pair, from float32 candidate and microphone positions
// relative to the microphone centroid: their error, about 2^-23 of the largest
// candidate-to-array distance times 2 fs / c (1e-4 samples at 10 m and
// 48 kHz), stays below the BF16/FP16 rounding of the weights (the
// conventional path computes them in float64).
#include <cmath>
#include <type_traits>
#include <utility>

#include "launch_split.h"
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

// Launch shape: candidate tiles per wave and waves per workgroup (a multiple
// of the 4 SIMDs of a CU). One tile per wave and two waves per SIMD in one
// workgroup: the two waves of a SIMD overlap each other's vector work and
// waits with the matrix cores (measured at the room scale: 4.54 ms per call,
// against 5.72 ms for two tiles per wave and one wave per SIMD, and 5.17 ms
// for two 4-wave workgroups per CU, which copy every run twice per CU).
constexpr int kTiles = 1;
constexpr int kWavesPerBlock = 8;
// LDS reads of the next step's fragments issued after each of a step's first
// matrix-core instructions, and vector instructions slotted after each
// (measured at the room scale and at 32 microphones against groups of 2 and 8
// and 3 vector instructions: within 1 %, this the fastest).
constexpr int kMxReadGroup = 4;
constexpr int kMxValuPerMfma = 4;

struct MxArgs {
  const double* cand;      // [3][J]
  int F;
  int f_base;              // first frame of this launch's frame blocks
  int64_t j_base;          // first candidate of this launch's candidate blocks
  int S;
  int64_t J;
  int n_runs;
  double inv_cT;
  double xq_scale;         // 2^e: the grid of the TDOA fractions
  double xq_inv;           // 2^-e
  double inv_L;            // conventional map: 1 / L (bin k has phase k x fs / L turns)
  int far_field;
  double centre[3];        // origin of the float32 positions (the microphone centroid, near field)
  float* map;              // [F][J] or null
  unsigned long long* keys;  // peaks viewed as u64 pairs, or null
};

// sin(pi x) / pi for |x| <= 1/2 in float32: the Taylor series of sin,
// x sum_k (-1)^k pi^(2k) x^(2k) / (2k+1)!, truncated after x^13 (truncation
// error below 3e-10), a few float32 units of error. The weights of this kernel
// are rounded to BF16/FP16, so float32 suffices here (x is exact: a grid point).
__device__ __forceinline__ float sinpi_over_pi_f32(float x) {
  const float u = x * x;
  float p = 0.00014842879f;        //  pi^12 / 13!
  p = fmaf(p, u, -0.0023460810f);  // -pi^10 / 11!
  p = fmaf(p, u, 0.026147848f);    //  pi^8 / 9!
  p = fmaf(p, u, -0.19075182f);    // -pi^6 / 7!
  p = fmaf(p, u, 0.81174243f);     //  pi^4 / 5!
  p = fmaf(p, u, -1.6449341f);     // -pi^2 / 3!
  p = fmaf(p, u, 1.0f);
  return x * p;
}

// Calls f(integral_constant<int, I>) for I = 0 .. N-1, each call inlined.
template <typename F, int... I>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>()), ...);
}

// Max of v over the 32 lanes of each half-wave (halves separate): butterflies
// within each row of 16 lanes, then across the two rows of the half.
__device__ __forceinline__ float half_wave_fmax(float v) {
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// CONV selects the conventional map (B = phasors of the bins, A = the
// weighted cross-spectra) instead of the Nyquist map (B = sinc weights of the
// lags, A = the GCC samples); the rest of the kernel is shared.
template <typename T, int FT, int CT, int NW, bool CONV>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
void nyquist_mx2_kernel(MxArgs a, const T* __restrict__ xi, const RunRec* __restrict__ recs) {
  typedef typename Mx32<T>::type vec8;
  typedef __attribute__((address_space(3))) void* lds_ptr;
  static_assert(CT == 1 || CT == 2, "one or two candidate tiles per wave");
  static_assert(!CONV || CT == 1, "the conventional map uses one candidate tile per wave");
  static_assert(NW % 4 == 0, "whole waves per SIMD");
  constexpr int FB = 32 * FT;
  constexpr int JW = 32 * CT;            // candidates per wave
  constexpr int JB = JW * NW;
  // chunk pairs (16 lags or 8 bins) of a staging tile: a Nyquist lag run
  // (<= kMxRunMax lags, <= kMxRunMaxFew with at most 4 frame tiles) or a
  // conventional 32-bin run
  constexpr int kChunkPairs = CONV ? 4 : (FT <= 4 ? kMxRunMaxFew : kMxRunMax) / 16;
  constexpr int kTile = kChunkPairs * FB * 16;  // elements of a staging tile
  __shared__ __attribute__((aligned(16))) T xs0[kTile];
  __shared__ __attribute__((aligned(16))) T xs1[kTile];
  __shared__ unsigned long long kbest[FB];
  // argmax blocks of the epilogue (one candidate tile per wave): in the
  // staging buffers (free by then) when half the waves fit in each, else
  // an array of their own
  constexpr int kEp = argmax_block_floats<1>();
  constexpr bool kEpInTiles = kTile * sizeof(T) >= (NW / 2) * kEp * sizeof(float);
  __shared__ __attribute__((aligned(16))) float epi[CT == 1 && !kEpInTiles ? NW * kEp : 1];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int cl = lane & 31;
  const int g = lane >> 5;
  const int64_t jw = a.j_base + (int64_t)blockIdx.x * JB + wave * JW;  // the wave's first candidate
  const int f0 = a.f_base + blockIdx.y * FB;
  const int nrows = a.F - f0 < FB ? a.F - f0 : FB;

  // The lane's own candidate: with two tiles, jw + 32 g + cl (tile g; lanes cl
  // and cl + 32 split the TDOAs of the two tiles' candidates cl and exchange
  // them), with one tile jw + cl.
  const int64_t own = jw + (CT == 2 ? 32 * g : 0) + cl;
  const int64_t oc = own < a.J ? own : a.J - 1;
  const double qx = a.cand[oc], qy = a.cand[a.J + oc], qz = a.cand[2 * a.J + oc];
  for (int i = tid; i < FB; i += 64 * NW) kbest[i] = 0ull;

  // staging: the tile holds, for each pair j of 16-byte chunks (16 lags) and
  // each group G of 32 rows, the first chunks of the 32 rows, then their second
  // chunks: element (j FB + 32 G) 16 + (r + 32 h) 8 + e for row 32 G + r,
  // chunk 2 j + h. One copy instruction moves one chunk pair of 32 rows (lane
  // i: row 32 G + i % 32, chunk 2 j + i / 32), landing as 1 KB of contiguous
  // LDS, and a step's fragment read (lane (cl, g): row cl, chunk g) is then
  // 1 KB read in lane order, free of bank conflicts; wave w copies the row
  // groups G = w, w + NW, ... Rows at or past F repeat the last frame (their
  // outputs are discarded); a chunk past the run repeats its last chunk (its
  // weights are zero). Only the chunk pairs the run's steps read are copied.
  constexpr int kGroups = FT;                             // 32-row groups of the tile
  constexpr int kGpw = (kGroups + NW - 1) / NW;           // groups per wave
  const int sub = lane >> 5;
  unsigned roff[kGpw];
#pragma unroll
  for (int k = 0; k < kGpw; ++k) {
    const int row = 32 * (wave + NW * k) + (lane & 31);
    const int rr = row < nrows ? row : nrows - 1;
    roff[k] = static_cast<unsigned>(rr) * static_cast<unsigned>(a.S) * sizeof(T);
  }
  const T* xblk = xi + (size_t)f0 * a.S;
  // copies of a wave per chunk pair (its row groups)
  const int gw = kGroups % NW == 0 ? kGpw : (kGroups - wave + NW - 1) / NW;
  // issues a run's copies; returns how many this wave issued
  auto stage = [&](const RunRec& run, T* tile) __attribute__((always_inline)) {
    if (run.len <= 0) return 0;
    const int nch = (run.len + 7) >> 3;
    const int npairs = (nch + 1) >> 1;
    const char* base = reinterpret_cast<const char*>(xblk + run.off + run.t0);
#pragma unroll
    for (int j = 0; j < kChunkPairs; ++j) {
      if (j >= npairs) break;  // (uniform)
      const int ch = 2 * j + sub < nch ? 2 * j + sub : nch - 1;
#pragma unroll
      for (int k = 0; k < kGpw; ++k) {
        const int G = wave + NW * k;
        if (kGroups % NW != 0 && G >= kGroups) break;  // (uniform) no such group
        __builtin_amdgcn_global_load_lds(
            reinterpret_cast<const void*>(base + (roff[k] + 16u * static_cast<unsigned>(ch))),
            (lds_ptr)(tile + (j * FB + 32 * G) * 16), 16, 0, 0);
      }
    }
    return npairs * gw;
  };

  floatx16 acc[CT][FT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[ct][ft][r] = 0.0f;

  // per-pair TDOA split of the tiles' candidates cl (index = tile); for the
  // conventional map the TDOA in samples and the phasors of 1 and 8 bins
  int cur_p = -1, cur_m = -1;
  double rm = 0.0;
  float rmf = 0.0f;
  int xr[CT];
  float xf[CT], sp[CT];
  double xs = 0.0;
  float r1c = 1.0f, r1s = 0.0f, r8c = 1.0f, r8s = 0.0f;
  // Nyquist: the TDOA and its split in float32, from the candidate and the
  // microphone positions relative to the microphone centroid, rounded to
  // float32: an error of about 2^-23 of the largest candidate-to-array
  // distance, times 2 fs / c (1e-4 samples at 10 m and 48 kHz), below the
  // BF16/FP16 rounding of the weights it moves
  const float qxf = static_cast<float>(qx - a.centre[0]),
              qyf = static_cast<float>(qy - a.centre[1]),
              qzf = static_cast<float>(qz - a.centre[2]);
  const float inv_cT_f = static_cast<float>(a.inv_cT);
  const float xq_scale_f = static_cast<float>(a.xq_scale);
  const float xq_inv_f = static_cast<float>(a.xq_inv);
  auto norm3f = [](float dx, float dy, float dz) __attribute__((always_inline)) {
    return __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
  };
  auto pair_split = [&](const RunRec& run) __attribute__((always_inline)) {
    if constexpr (!CONV) {
      float x;
      if (a.far_field) {
        x = ((run.pmf[0] - run.pnf[0]) * qxf + (run.pmf[1] - run.pnf[1]) * qyf +
             (run.pmf[2] - run.pnf[2]) * qzf) * inv_cT_f;
      } else {
        if (run.m != cur_m) {
          rmf = norm3f(qxf - run.pmf[0], qyf - run.pmf[1], qzf - run.pmf[2]);
          cur_m = run.m;
        }
        x = (rmf - norm3f(qxf - run.pnf[0], qyf - run.pnf[1], qzf - run.pnf[2])) * inv_cT_f;
      }
      const float r = rintf(x);
      const float fd0 = x - r;  // exact
      float q = rintf(fd0 * xq_scale_f);
      q = q != 0.0f ? q : (fd0 < 0.0f ? -1.0f : 1.0f);
      const float fd = q * xq_inv_f;  // exact (a power of two)
      const int xr_own = static_cast<int>(r);
      const float sp_own = sinpi_over_pi_f32(fd);
      if (CT == 2) {
        const int xr_oth = __shfl_xor(xr_own, 32, 64);
        const float xf_oth = __shfl_xor(fd, 32, 64);
        const float sp_oth = __shfl_xor(sp_own, 32, 64);
        xr[0] = g ? xr_oth : xr_own;
        xr[CT - 1] = g ? xr_own : xr_oth;
        xf[0] = g ? xf_oth : fd;
        xf[CT - 1] = g ? fd : xf_oth;
        sp[0] = g ? sp_oth : sp_own;
        sp[CT - 1] = g ? sp_own : sp_oth;
      } else {
        xr[0] = xr_own;
        xf[0] = fd;
        sp[0] = sp_own;
      }
      cur_p = run.p;
      return;
    }
    double x;
    if (a.far_field) {
      x = ((run.pm[0] - run.pn[0]) * qx + (run.pm[1] - run.pn[1]) * qy +
           (run.pm[2] - run.pn[2]) * qz) * a.inv_cT;
    } else {
      if (run.m != cur_m) {
        rm = norm3(qx - run.pm[0], qy - run.pm[1], qz - run.pm[2]);
        cur_m = run.m;
      }
      x = (rm - norm3(qx - run.pn[0], qy - run.pn[1], qz - run.pn[2])) * a.inv_cT;
    }
    // conventional: x is the TDOA in samples; phase of bin k: k x / L turns,
    // reduced mod 1 in float64, then rounded to float32 for the rotations
    xs = x;
    const double t1 = x * a.inv_L, t8 = 8.0 * t1;
    sincospif(2.0f * static_cast<float>(t1 - rint(t1)), &r1s, &r1c);
    sincospif(2.0f * static_cast<float>(t8 - rint(t8)), &r8s, &r8c);
    cur_p = run.p;
  };

  // Contracts one staged run. A step's sample fragment of frame tile ft is
  // row 32 ft + cl of chunk pair s, half g: one 16-byte LDS read (the 64 lanes
  // together read 1 KB of contiguous LDS), used by the matrix-core
  // instructions of both candidate tiles.
  auto contract_run = [&](const RunRec& run, const T* tile) __attribute__((always_inline)) {
    if (run.len <= 0) return;
    if (run.p != cur_p) pair_split(run);
    const int nch = (run.len + 7) >> 3;
    const int steps = (run.len + 15) >> 4;
    // Nyquist: d of the lane's first lag in step s for tile ct,
    // (xr + h - t0 - 8g - 16 s) + xf, exact; the sign (-1)^(xi - n) is the
    // same for all of them. Conventional: the phasor of the lane's first bin
    // k0 + 4g (run.h holds k0), from the float64 phase reduced mod 1; each
    // step then takes 4 consecutive bins (rotations by one bin) and moves on
    // by 8 bins
    float qs[CT], u0[CT];
    float pc = 1.0f, ps = 0.0f;
    if (CONV) {
      const double t = static_cast<double>(run.h + 4 * g) * xs * a.inv_L;
      sincospif(2.0f * static_cast<float>(t - rint(t)), &ps, &pc);
    } else {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int ia = xr[ct] + run.h - run.t0 - 8 * g;
        qs[ct] = (ia & 1) ? -sp[ct] : sp[ct];
        u0[ct] = static_cast<float>(ia) + xf[ct];
      }
    }
    const T* tbase = tile + (cl + 32 * g) * 8;
    // (steps past the run re-read its last step and are never contracted)
    auto frag_addr = [&](int s) __attribute__((always_inline)) {
      const int sc = s < steps ? s : steps - 1;
      return tbase + sc * (FB * 16);
    };
    auto read = [&](const T* src, int ft) __attribute__((always_inline)) {
      return *reinterpret_cast<const vec8*>(src + ft * 32 * 16);
    };
    // (called for s = 0, 1, 2, ... in order: the conventional phasor advances)
    auto weights = [&](int s, vec8 (&wv)[CT]) __attribute__((always_inline)) {
      // chunks past the run carry weight 0 (their samples repeat the last chunk)
      const bool live = 2 * s + g < nch;
      if (CONV) {
        // B rows of bin k: (cos theta_k, -sin theta_k) multiply (Re, Im) of the
        // weighted spectrum: Re[psi e^{j theta}] = Re psi cos - Im psi sin
        const float z = live ? 1.0f : 0.0f;
        float c = pc, sn = ps;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          wv[0][2 * j] = static_cast<T>(z * c);
          wv[0][2 * j + 1] = static_cast<T>(-z * sn);
          const float c2 = c * r1c - sn * r1s;
          sn = c * r1s + sn * r1c;
          c = c2;
        }
        const float c8 = pc * r8c - ps * r8s;
        ps = pc * r8s + ps * r8c;
        pc = c8;
        return;
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const float q = live ? qs[ct] : 0.0f;
        const float ub = u0[ct] - static_cast<float>(16 * s);
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const float u = ub - static_cast<float>(j);
          const float r = q * __builtin_amdgcn_rcpf(fmaf(u, u, -u));
          wv[ct][j] = static_cast<T>(fmaf(r, u, -r));
          wv[ct][j + 1] = static_cast<T>(-r * u);
        }
      }
    };
    // Software pipeline: two register sets of a step's FT sample fragments.
    // A step contracts one set while the next step's fragments are read into
    // the other, those reads issued in groups of kMxReadGroup right after the
    // step's first matrix-core instructions; the next step's weights are
    // formed between the matrix-core instructions. (While a run's copies into
    // the other staging buffer are in flight, the compiler waits for all LDS
    // reads before the first matrix-core instruction of a step rather than
    // for the fragment it needs; with the reads issued early in the previous
    // step, that wait finds them done.)
    vec8 ra[FT], rb[FT];
    {
      const T* src = frag_addr(0);
#pragma unroll
      for (int i = 0; i < FT; ++i) ra[i] = read(src, i);
    }
    // (reads: whether to read the next step's fragments from nxt)
    auto step = [&](auto reads, const vec8 (&wc)[CT], const vec8 (&rc)[FT], vec8 (&rn)[FT],
                    const T* nxt) __attribute__((always_inline)) {
      constexpr bool kReads = decltype(reads)::value;
#pragma unroll
      for (int i = 0; i < FT; ++i)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          acc[ct][i] = Mx32<T>::mfma(rc[i], wc[ct], acc[ct][i]);
      if (kReads) {
#pragma unroll
        for (int i = 0; i < FT; ++i) rn[i] = read(nxt, i);
      }
      // issue order: per fragment the matrix-core instruction(s) of its
      // tiles, then (for the first fragments) a group of reads, then vector
      // instructions
      static_for(std::make_integer_sequence<int, FT>(), [&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        constexpr int left = FT - i * kMxReadGroup;  // reads not yet placed
        __builtin_amdgcn_sched_group_barrier(0x008, CT, 0);
        if constexpr (kReads && left > 0)
          __builtin_amdgcn_sched_group_barrier(0x100, left < kMxReadGroup ? left : kMxReadGroup, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, kMxValuPerMfma * CT, 0);
      });
    };
    // each step's instructions with the next step's weights slotted between
    // them (the read addresses are recomputed from the tile every iteration
    // rather than carried across iterations: a pointer that the loop carries
    // hides which staging buffer it points into, and the compiler then waits
    // for the other buffer's copies in flight before reading)
    typedef std::integral_constant<bool, true> WithReads;
    typedef std::integral_constant<bool, false> NoReads;
    vec8 w0[CT], w1[CT];
    weights(0, w0);
    int s = 0;
    for (; s + 1 < steps; s += 2) {
      const T* p1 = frag_addr(s + 1);
      const T* p2 = frag_addr(s + 2);
      __builtin_amdgcn_sched_barrier(0);
      weights(s + 1, w1);
      step(WithReads(), w0, ra, rb, p1);
      __builtin_amdgcn_sched_barrier(0);
      weights(s + 2, w0);
      step(WithReads(), w1, rb, ra, p2);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (s < steps) step(NoReads(), w0, ra, rb, frag_addr(s));
  };

  stage(recs[0], xs0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int ri = 0; ri < a.n_runs; ri += 2) {
    // even run: read xs0, copy the next run into xs1; odd run: the other way
    // round (the run count is even)
    const RunRec r0 = recs[ri];
    const RunRec r1 = recs[ri + 1];
    // Every record field this iteration reads, the next run's staging fields
    // included, is tied to a scalar register here, so their scalar loads issue
    // together and wait once, not once per first use inside the runs (a wait
    // that stalls the matrix-core stream of the wave).
    auto pin = [](const RunRec& r) __attribute__((always_inline)) {
      asm volatile("" ::"s"(r.p), "s"(r.t0), "s"(r.len), "s"(r.off), "s"(r.h), "s"(r.m));
      if constexpr (CONV) {
        asm volatile("" ::"s"(r.pm[0]), "s"(r.pm[1]), "s"(r.pm[2]));
        asm volatile("" ::"s"(r.pn[0]), "s"(r.pn[1]), "s"(r.pn[2]));
      } else {
        asm volatile("" ::"s"(r.pmf[0]), "s"(r.pmf[1]), "s"(r.pmf[2]));
        asm volatile("" ::"s"(r.pnf[0]), "s"(r.pnf[1]), "s"(r.pnf[2]));
      }
    };
    pin(r0);
    pin(r1);
    RunRec r2;
    {
      const RunRec& nx = recs[ri + 2 < a.n_runs ? ri + 2 : ri];
      r2.t0 = nx.t0;
      r2.len = nx.len;
      r2.off = nx.off;
      asm volatile("" ::"s"(r2.t0), "s"(r2.len), "s"(r2.off));
    }
    stage(r1, xs1);
    contract_run(r0, xs0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (ri + 2 < a.n_runs) stage(r2, xs0);  // (reads t0, len and off only)
    contract_run(r1, xs1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // epilogue: D[frame][cand], lane (cl, g), register r -> frame 8 (r / 4) + 4 g + r % 4,
  // candidate jw + 32 ct + cl. Per frame, the maximum over the wave's 64
  // candidates, the lowest candidate holding it (tile 0 before tile 1, lower
  // lanes first), and one LDS max per frame and wave on a (value, -index) key.
  bool valid[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) valid[ct] = jw + 32 * ct + cl < a.J;
  if constexpr (CT == 1) {
    // one candidate tile: the argmax of each frame tile through the wave's LDS
    // block, then the block's LDS max on the (value, -index) key per frame
    float* ep = kEpInTiles ? reinterpret_cast<float*>(wave < NW / 2 ? xs0 : xs1) +
                                 (wave % (NW / 2)) * kEp
                           : epi + wave * kEp;
    static_for(std::make_integer_sequence<int, FT>(), [&](auto ftc) __attribute__((always_inline)) {
      constexpr int ft = decltype(ftc)::value;
      float v[1][16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int fg = f0 + ft * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
        v[0][r] = 2.0f * acc[0][ft][r];
        if (a.map && valid[0] && fg < a.F) a.map[(size_t)fg * a.J + jw + cl] = v[0][r];
        if (!valid[0]) v[0][r] = -__builtin_inff();
      }
      if (a.keys) {
        const unsigned long long k = tile_argmax_key<1>(ep, v, jw);
        if (k && f0 + ft * 32 + cl < a.F) atomicMax(&kbest[ft * 32 + cl], k);
      }
    });
  } else {
    static_for(std::make_integer_sequence<int, FT>(), [&](auto ftc) __attribute__((always_inline)) {
      constexpr int ft = decltype(ftc)::value;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int fl = ft * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
        const int fg = f0 + fl;
        float vv[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const float v = 2.0f * acc[ct][ft][r];
          if (a.map && valid[ct] && fg < a.F) a.map[(size_t)fg * a.J + jw + 32 * ct + cl] = v;
          vv[ct] = valid[ct] ? v : -__builtin_inff();
        }
        if (a.keys) {
          const float vmax = half_wave_fmax(fmaxf(vv[0], vv[CT - 1]));
          const unsigned long long h0 = __ballot(vv[0] == vmax);
          const unsigned long long m0 = g ? (h0 >> 32) : (h0 & 0xffffffffull);
          const unsigned long long h1 = __ballot(vv[CT - 1] == vmax);
          const unsigned long long m1 = g ? (h1 >> 32) : (h1 & 0xffffffffull);
          const int first = m0 ? __builtin_ctzll(m0) : 32 + __builtin_ctzll(m1 | (1ull << 63));
          if (cl == 0 && fg < a.F && vmax > -__builtin_inff())
            atomicMax(&kbest[fl], peak_key(vmax, static_cast<unsigned>(jw + first)));
        }
      }
    });
  }
  if (a.keys) {
    __syncthreads();
    for (int i = tid; i < FB; i += 64 * NW) {
      const unsigned long long k = kbest[i];
      if (k && f0 + i < a.F) atomicMax(a.keys + 2 * (size_t)(f0 + i), k);
    }
  }
}

}  // namespace

// The grid exponent e of the TDOA fractions: every |d| < 2 h_max + 64 must be
// a float32 number on the grid 2^-e, i.e. fit 24 significant bits.
int mx_fraction_grid_exponent(int h_max) {
  int bits = 0;
  while ((int64_t(1) << bits) <= 2 * int64_t(h_max) + 64) ++bits;
  return 24 - bits;
}

bool mx2_supported(const srp_geometry_s* g) {
  // 32-bit copy offsets within a frame block of 256 rows of 2-byte samples
  // (S < 2^23)
  return (int64_t)256 * g->info.S * 2 < (int64_t(1) << 32) &&
         mx_fraction_grid_exponent(g->info.h_max) >= 8;
}

int mx2_workgroups_per_cu(int dtype) {
  int n = 0;
  const void* k = dtype == SRP_BF16
                      ? reinterpret_cast<const void*>(
                            &nyquist_mx2_kernel<__bf16, 8, kTiles, kWavesPerBlock, false>)
                      : reinterpret_cast<const void*>(
                            &nyquist_mx2_kernel<_Float16, 8, kTiles, kWavesPerBlock, false>);
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * kWavesPerBlock, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_nyquist_mx2(const srp_geometry_s* g, const void* xi, int F, int dtype,
                              float* map, unsigned long long* keys, hipStream_t s) {
  static_assert(32 * kTiles * kWavesPerBlock == 256, "256-candidate blocks (launch_in_rounds)");
  MxArgs a;
  a.cand = g->d_cand;
  a.F = F;
  a.f_base = 0;
  a.j_base = 0;
  a.S = static_cast<int>(g->info.S);
  a.J = g->info.J;
  a.n_runs = 0;  // per launch: the run list its frame-tile count takes
  a.inv_cT = g->inv_cT;
  a.xq_scale = std::ldexp(1.0, mx_fraction_grid_exponent(g->info.h_max));
  a.xq_inv = std::ldexp(1.0, -mx_fraction_grid_exponent(g->info.h_max));
  a.inv_L = 1.0 / g->info.L;
  a.far_field = g->info.field == SRP_FAR_FIELD;
  for (int d = 0; d < 3; ++d) a.centre[d] = g->mic_centre[d];
  a.map = map;
  a.keys = keys;
  const int per_cu = g->wg_per_cu[dtype == SRP_BF16 ? 1 : 2];
  launch_in_rounds(g, F, a, per_cu, [&](auto ft, const MxArgs& b, dim3 grid) {
    constexpr int FTv = decltype(ft)::value;
    constexpr bool kFew = FTv <= 4;  // the kernel's staging tile holds kMxRunMaxFew lags
    MxArgs c = b;
    c.n_runs = static_cast<int>((kFew ? g->mx_runs_few : g->mx_runs).size());
    const RunRec* recs = kFew ? g->d_mx_recs_few : g->d_mx_recs;
    const dim3 blk(64 * kWavesPerBlock);
    if (dtype == SRP_BF16)
      hipLaunchKernelGGL((nyquist_mx2_kernel<__bf16, FTv, kTiles, kWavesPerBlock, false>), grid,
                         blk, 0, s, c, static_cast<const __bf16*>(xi), recs);
    else
      hipLaunchKernelGGL((nyquist_mx2_kernel<_Float16, FTv, kTiles, kWavesPerBlock, false>),
                         grid, blk, 0, s, c, static_cast<const _Float16*>(xi), recs);
  });
  return hipGetLastError();
}

bool conv_mx_supported(const srp_geometry_s* g) {
  // 32-bit copy offsets within a frame block of 256 rows of 2 P Kp 2-byte values
  return (int64_t)256 * 2 * g->info.P * g->Kp * 2 < (int64_t(1) << 32);
}

int conv_mx_workgroups_per_cu(int dtype) {
  int n = 0;
  const void* k = dtype == SRP_BF16
                      ? reinterpret_cast<const void*>(
                            &nyquist_mx2_kernel<__bf16, 8, 1, kWavesPerBlock, true>)
                      : reinterpret_cast<const void*>(
                            &nyquist_mx2_kernel<_Float16, 8, 1, kWavesPerBlock, true>);
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * kWavesPerBlock, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

// Conventional map in BF16/FP16 on the same skeleton: the runs are 32-bin runs
// of each pair over the weighted, rounded spectra [F][P][Kp] x (re, im)
// (srp_spectra_lowp), a frame row holding 2 P Kp values.
hipError_t launch_conventional_mx(const srp_geometry_s* g, const void* spec, int F, int dtype,
                                  float* map, unsigned long long* keys, hipStream_t s) {
  static_assert(kTiles == 1, "256-candidate blocks");
  MxArgs a;
  a.cand = g->d_cand;
  a.F = F;
  a.f_base = 0;
  a.j_base = 0;
  a.S = 2 * g->info.P * g->Kp;
  a.J = g->info.J;
  a.n_runs = g->n_convmx_runs;
  a.inv_cT = g->fs_over_c;  // path difference (m) -> TDOA in samples
  a.xq_scale = 1.0;
  a.xq_inv = 1.0;
  a.inv_L = 1.0 / g->info.L;
  a.far_field = g->info.field == SRP_FAR_FIELD;
  for (int d = 0; d < 3; ++d) a.centre[d] = 0.0;  // (float64 positions only)
  a.map = map;
  a.keys = keys;
  const int per_cu = g->wg_per_cu_conv[dtype == SRP_BF16 ? 0 : 1];
  launch_in_rounds(g, F, a, per_cu, [&](auto ft, const MxArgs& b, dim3 grid) {
    constexpr int FTv = decltype(ft)::value;
    const dim3 blk(64 * kWavesPerBlock);
    if (dtype == SRP_BF16)
      hipLaunchKernelGGL((nyquist_mx2_kernel<__bf16, FTv, 1, kWavesPerBlock, true>), grid, blk,
                         0, s, b, static_cast<const __bf16*>(spec), g->d_convmx_recs);
    else
      hipLaunchKernelGGL((nyquist_mx2_kernel<_Float16, FTv, 1, kWavesPerBlock, true>), grid,
                         blk, 0, s, b, static_cast<const _Float16*>(spec), g->d_convmx_recs);
  });
  return hipGetLastError();
}

}  // namespace srp
