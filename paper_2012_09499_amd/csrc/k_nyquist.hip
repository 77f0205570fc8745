// Nyquist-Shannon SRP approximation (Eq. SRPapprox summed over pairs as in
// Eq. SRP_T_IFT; cost Eq. SRPapproxcompR):
//   map[f][i] = 2 sum_p sum_{|n| <= h_p} xi_p(nT) sinc(x_p(i) - n),  x_p(i) = dt_p(i) / T.
//
// For a block of candidates and a block of frames this is a product of a
// weight matrix [candidates x packed lags] with the samples [packed lags x
// frames]. The weights are never stored: each lane forms them in registers
// right before the matrix-core instruction that consumes them.
//
// Weight formation. With x = xi + xf (xi = rint(x) in float64, xf = x - xi
// exact in float64, then rounded once to float32, |xf| <= 1/2):
//   sinc(x - n) = (-1)^(xi - n) sin(pi xf) / (pi ((xi - n) + xf)).
// (xi - n) is an exact small integer, so the denominator carries a single
// float32 rounding; sin(pi xf) / pi is formed once per candidate and pair. At
// xf = 0 the fraction is replaced by 1e-30, which gives weight 1 at n = xi and
// 0 elsewhere (to float32 precision) without a branch per weight. |weight| <= 1.
//
// TDOAs: x = (||q - p_m|| - ||q - p_m'||) / (c T) in float64 (near field,
// Eq. Deltat_i) or (p_m - p_m') . r / (c T) (far field, Eq. Deltat_i_spher),
// recomputed per pair from the candidate held in registers, so no J x P table
// exists anywhere.
//
// FP32 kernel layout (v_mfma_f32_32x32x2f32, D[frame][cand] += A[frame][k] B[k][cand]):
//   block = NW waves (8; 4 for the two-level sum), two per SIMD; each wave owns
//   32 * CT candidates, all waves share the block's 32 * FT frames;
//   step s of a lag run covers, of its 4-lag chunk s >> 1, lags 4 (s >> 1) + (s & 1)
//   (k = 0, lanes 0-31) and 4 (s >> 1) + 2 + (s & 1) (k = 1, lanes 32-63), so a lane
//   reads the two lags it takes from a chunk with one 8-byte LDS read;
//   A = samples staged in LDS as [frame][lag]; B = weights (lane = candidate);
//   epilogue: x2, optional map store, argmax via LDS u64 max + one global atomic per frame.
#include <type_traits>

#include "launch_split.h"
#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

constexpr int kStride = kNyqRunMax + 1;  // LDS row stride (odd) of the [frame][lag] tile

// Above this many samples per frame the FP32 kernel sums in two levels. The
// relative error of one float32 accumulator over all S terms grows like
// sqrt(S): measured 1.2e-5 at S = 609,344 (above the maps' 1e-5 bound), so
// about 4e-6 at the 65,536 limit.
constexpr int64_t kNyqPlainSumMax = 65536;

struct NyqArgs {
  const double* cand;      // [3][J]
  const double* mic;       // [M][3]
  const PairDesc* pairs;
  const LagRun* runs;
  int n_runs;
  const float* xi;         // [F][S]
  int F;
  int f_base;              // first frame of this launch's frame blocks
  int64_t j_base;          // first candidate of this launch's candidate blocks
  int S;
  int64_t J;
  double inv_cT;
  int far_field;
  const float* zero;       // >= 16 zero bytes (staging source past a run's end)
  float* map;              // [F][J] or null
  unsigned long long* keys;  // peaks viewed as u64 pairs, or null
};

// x_p(i) = dt_p(i) / T for the candidate (qx, qy, qz), float64.
__device__ __forceinline__ double pair_x(const NyqArgs& a, const PairDesc& pd, double qx,
                                         double qy, double qz) {
  const double* pm = a.mic + 3 * pd.m;
  const double* pn = a.mic + 3 * pd.mp;
  if (a.far_field) {
    return ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * a.inv_cT;
  }
  const double ax = qx - pm[0], ay = qy - pm[1], az = qz - pm[2];
  const double bx = qx - pn[0], by = qy - pn[1], bz = qz - pn[2];
  return (sqrt(ax * ax + ay * ay + az * az) - sqrt(bx * bx + by * by + bz * bz)) * a.inv_cT;
}

// FP32 staging tile: frame tiles of 32 rows [frame][64 lags], 256 bytes per
// row, the tiles kBlk32 floats apart (16 bytes of padding between tiles, so
// the compiler never merges a step's reads of different tiles into one
// instruction, which would hide from it which buffer they read). Within a row,
// 16-byte chunk c (lags 4c .. 4c+3) is stored at chunk c ^ (R & 15): a step's
// read has each wave half read the same lags from 32 rows, and the swizzle
// puts 16 consecutive rows on 16 different bank groups.
constexpr int kRow32 = kNyqRunMax;   // floats per LDS row
constexpr int kBlk32 = 32 * kRow32 + 4;  // floats per 32-row frame tile

// Per-lane constants of the FP32 staging copies. One copy instruction moves
// 4 rows (64 lanes x 16 bytes, landing in lane order): lane i fills chunk
// i & 15 of row 4G + (i >> 4) of row group G. Wave w copies the groups
// G = w, w + NW, ...; with NW a multiple of 4, G & 3 = w & 3, so the logical
// chunk a lane loads is the same for all its groups and runs.
struct Stage32 {
  int jr;         // row of the lane within a group
  int lchunk;     // logical chunk this lane loads
  unsigned roff;  // jr rows, in bytes
};

template <int NW>
__device__ __forceinline__ Stage32 stage32_init(const NyqArgs& a, int wave, int lane) {
  static_assert(NW % 4 == 0, "row groups of a wave must share their swizzle");
  Stage32 sg;
  sg.jr = lane >> 4;
  sg.lchunk = (lane & 15) ^ (4 * (wave & 3) + sg.jr);
  sg.roff = static_cast<unsigned>(sg.jr) * 4u * static_cast<unsigned>(a.S);
  return sg;
}

// Issues the asynchronous copy of one lag run of the samples into a staging
// tile. The steps read lags 0 .. 2 ceil(len / 2) - 1 of the run, all in chunks
// 0 .. (len - 1) / 4; chunks past those repeat the last one (they are never
// read). A run of odd length ends at its pair window's end (runs before the
// last one of a window are multiples of 8 long), and its lag len, which the
// last step reads, is then the layout's zero-filled gap after the window (a
// window holds an odd number of lags and starts at a multiple of 8), so no
// weight needs a mask.
//
// Only the first 4 waves copy (one per SIMD, waves w and w + 4 sharing SIMD
// w): right after a barrier, each SIMD then has one wave issuing its copies
// and one issuing matrix-core instructions, instead of both stalled on a
// burst of copies.
template <int FB, int NW0>
__device__ __forceinline__ void stage_run(const NyqArgs& a, const RunRec& run, const Stage32& sg,
                                          float* tile, int f0, int nrows, int wave) {
  typedef __attribute__((address_space(3))) void* lds_ptr;
  constexpr int NW = 4;                   // copying waves
  constexpr int kGroups = FB / (4 * NW);  // row groups per copying wave
  static_assert(FB % (4 * NW) == 0, "every copying wave copies the same number of row groups");
  if (run.len <= 0 || wave >= NW) return;
  const int lc = (run.len - 1) >> 2;  // last chunk the steps read
  const unsigned cb = 16u * static_cast<unsigned>(sg.lchunk < lc ? sg.lchunk : lc);
  // group base rows advance by 4 NW rows (scalar arithmetic). The empty asm
  // keeps the compiler from hoisting the per-group addresses out of the run
  // loop into spilled registers.
  int nr = nrows, w = wave;
  asm volatile("" : "+s"(nr), "+s"(w));
  const float* col = a.xi + run.off + run.t0;
  const char* base = reinterpret_cast<const char*>(col + (size_t)(f0 + 4 * w) * a.S);
  const size_t gstep = (size_t)4 * NW * a.S * sizeof(float);
  if (nr == FB) {
    const unsigned vo = sg.roff + cb;  // per-lane 32-bit offset from a scalar base
#pragma unroll
    for (int k = 0; k < kGroups; ++k) {
      const int G = w + k * NW;
      float* dst = tile + (G >> 3) * kBlk32 + 4 * (G & 7) * kRow32;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(base + vo), (lds_ptr)dst,
                                       16, 0, 0);
      base += gstep;
    }
  } else {
    // the block's last frames: rows at or past F repeat the last frame (their
    // outputs are discarded); a group that starts past it is based at the
    // last frame, so offsets from a group's base row are never negative
    const char* lastrow = reinterpret_cast<const char*>(col + (size_t)(f0 + nr - 1) * a.S);
#pragma unroll
    for (int k = 0; k < kGroups; ++k) {
      const int G = w + k * NW;
      const int g0 = 4 * G;
      const int gb = g0 < nr ? g0 : nr - 1;
      const int r = g0 + sg.jr < nr ? g0 + sg.jr : nr - 1;
      const unsigned vo = static_cast<unsigned>(r - gb) * 4u * static_cast<unsigned>(a.S) + cb;
      float* dst = tile + (G >> 3) * kBlk32 + 4 * (G & 7) * kRow32;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>((g0 < nr ? base : lastrow) + vo),
                                       (lds_ptr)dst, 16, 0, 0);
      base += gstep;
    }
  }
}

// Per-lane state of the FP32 kernel's candidates for the current pair.
template <int CT>
struct LaneState {
  double qx[CT], qy[CT], qz[CT];  // candidate (float64)
  double rm[CT];                  // ||q - p_m|| for the current m (near field)
  int xr[CT];                     // rint(x)
  float xf[CT];                   // x - rint(x)
  float sp[CT];                   // sin(pi xf) / pi
  int cur_m, cur_p;
  // the prepared run: sinc denominator of the lane's next lag (integer part),
  // sign-carrying numerator, and the first step's weight
  float dnum[CT], qv[CT], w0[CT];
};

// x_p(i) of the lane's candidates for a new pair (float64), split into
// rint(x), the float32 fraction and sin(pi xf) / pi.
template <int CT>
__device__ __forceinline__ void pair_setup(const NyqArgs& a, const RunRec& run,
                                           LaneState<CT>& st) {
  st.cur_p = run.p;
  const double* pm = run.pm;
  const double* pn = run.pn;
  const bool new_m = run.m != st.cur_m;
  st.cur_m = run.m;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    double x;
    if (a.far_field) {
      x = ((pm[0] - pn[0]) * st.qx[ct] + (pm[1] - pn[1]) * st.qy[ct] +
           (pm[2] - pn[2]) * st.qz[ct]) * a.inv_cT;
    } else {
      if (new_m) st.rm[ct] = norm3(st.qx[ct] - pm[0], st.qy[ct] - pm[1], st.qz[ct] - pm[2]);
      x = (st.rm[ct] - norm3(st.qx[ct] - pn[0], st.qy[ct] - pn[1], st.qz[ct] - pn[2])) *
          a.inv_cT;
    }
    const double r = rint(x);
    double f = x - r;
    f = fabs(f) < 1e-30 ? 1e-30 : f;
    st.xr[ct] = static_cast<int>(r);
    st.xf[ct] = static_cast<float>(f);
    st.sp[ct] = sinpi_over_pi(f);
  }
}

// Everything of a run that does not need its staged samples: the pair's
// TDOA split (when the pair changes) and the first step's weights. Called
// before the barrier that publishes the run's samples, so this latency
// overlaps the previous run's last matrix-core instructions.
template <int CT>
__device__ __forceinline__ void nyq_prepare(const NyqArgs& a, const RunRec& run,
                                            LaneState<CT>& st, int g) {
  if (run.len <= 0) return;
  if (run.p != st.cur_p) pair_setup<CT>(a, run, st);
  // this lane's first lag in the run: n = -h + t0 + 2g (lane g takes lags
  // 4k + 2g and 4k + 2g + 1 of chunk k, at the run's even and odd steps)
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int ia = st.xr[ct] + run.h - run.t0 - 2 * g;
    st.dnum[ct] = static_cast<float>(ia);
    st.qv[ct] = (ia & 1) ? -st.sp[ct] : st.sp[ct];
    st.w0[ct] = st.qv[ct] * __builtin_amdgcn_rcpf(st.dnum[ct] + st.xf[ct]);
  }
}

// Contracts one staged lag run (tile = samples [frame][lag]) into acc; the
// run was prepared by nyq_prepare.
template <int CT, int FT>
__device__ __forceinline__ void nyq_run(const RunRec& run, LaneState<CT>& st, const float* tile,
                                        int cl, int g, floatx16 (&acc)[CT][FT]) {
  if (run.len <= 0) return;
  float dnum[CT], qv[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    dnum[ct] = st.dnum[ct];
    qv[ct] = st.qv[ct];
  }
  // Lags of row R: step s takes, from chunk k = s >> 1 (stored at chunk
  // k ^ (R & 15)), lag 4k + (s & 1) in the lanes g = 0 and lag 4k + 2 + (s & 1)
  // in the lanes g = 1, so a lane reads its two lags of a chunk (elements 2g,
  // 2g + 1) with one 8-byte LDS read for the chunk's two steps. R & 15 = cl & 15
  // in every frame tile. Over the two steps of a chunk the matrix cores sum all
  // four of its lags. The step count covers every lag of the run: a run's
  // length is a multiple of 8 or its window's end, and the lags of the last
  // chunk past that end read the sample layout's zero gap (with finite weights:
  // a denominator is never an integer).
  const float* arow = tile + cl * kRow32 + 2 * g;
  const int swz4 = (cl & 15) << 2;  // the row's chunk swizzle, in floats
  const int steps = (run.len & 3) == 2 ? ((run.len >> 2) + 1) << 1 : (run.len + 1) >> 1;
  // software pipeline over chunks with ping-pong operand sets: the next
  // chunk's samples are read while the matrix cores work on the current one
  // (a read past the run stays inside the row and is never used); each step's
  // weight is formed while the previous step's matrix-core instructions run.
  // Even steps: (-1)^n sin(pi xf) / pi / (dnum + xf); odd steps the lag one
  // further: the opposite sign and dnum - 1; the next chunk: dnum - 4.
  float2 avA[FT], avB[FT];
  float we[CT], wo[CT];
  auto chunk_src = [&](int k) { return arow + (((k & 15) << 2) ^ swz4); };
  auto load = [&](const float* src, float2 (&av)[FT]) {
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) av[ft] = *reinterpret_cast<const float2*>(src + ft * kBlk32);
  };
  auto weight_odd = [&]() {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      wo[ct] = -qv[ct] * __builtin_amdgcn_rcpf((dnum[ct] - 1.0f) + st.xf[ct]);
  };
  auto weight_even_next = [&]() {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      dnum[ct] -= 4.0f;
      we[ct] = qv[ct] * __builtin_amdgcn_rcpf(dnum[ct] + st.xf[ct]);
    }
  };
  auto contract = [&](const float2 (&av)[FT], bool odd, const float (&w)[CT]) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int ft = 0; ft < FT; ++ft)
        acc[ct][ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(odd ? av[ft].y : av[ft].x, w[ct],
                                                          acc[ct][ft], 0, 0, 0);
  };
  auto order = [&](bool reads) {
    // issue order: one matrix-core instruction (its operands were read or
    // formed earlier), then (at a chunk's even step) the next chunk's LDS
    // reads, then the other matrix-core instructions with the weight
    // arithmetic slotted between them
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
    if (reads) __builtin_amdgcn_sched_group_barrier(0x100, FT, 0);
#pragma unroll
    for (int i = 1; i < CT * FT; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
  };
  load(chunk_src(0), avA);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) we[ct] = st.w0[ct];
  // four steps (two chunks) per iteration
  int s = 0;
  for (; s + 3 < steps; s += 4) {
    const int k = s >> 1;
    load(chunk_src(k + 1), avB);
    weight_odd();
    contract(avA, false, we);
    order(true);
    weight_even_next();
    contract(avA, true, wo);
    order(false);
    load(chunk_src(k + 2), avA);
    weight_odd();
    contract(avB, false, we);
    order(true);
    weight_even_next();
    contract(avB, true, wo);
    order(false);
  }
  // the last 1 to 3 steps: a whole chunk (its successor's samples then move
  // into the first operand set), then a last even step
  if (s + 1 < steps) {
    load(chunk_src((s >> 1) + 1), avB);
    weight_odd();
    contract(avA, false, we);
    order(true);
    weight_even_next();
    contract(avA, true, wo);
    order(false);
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) avA[ft] = avB[ft];
    s += 2;
  }
  if (s < steps) contract(avA, false, we);
}

// COMP: two-level summation for long sample sets. The matrix-core
// accumulator then holds one pair's contribution and is added into a second
// float32 accumulator whenever the pair changes, so rounding grows with the
// number of pairs and the steps per pair instead of with S.
template <int CT, int FT, int NW, bool COMP>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
void nyquist_f32_kernel(NyqArgs a, const RunRec* __restrict__ recs) {
  constexpr int FB = 32 * FT;
  constexpr int JW = 32 * CT;
  constexpr int JB = NW * JW;
  // two staging tiles as distinct objects: the copy into one never aliases
  // the reads of the other, so reads wait only on their own tile's copy
  __shared__ __attribute__((aligned(16))) float xs0[FT * kBlk32];
  __shared__ __attribute__((aligned(16))) float xs1[FT * kBlk32];
  __shared__ unsigned long long kbest[FB];
  // argmax blocks of the epilogue
  constexpr int kEp = argmax_block_floats<CT>();
  constexpr bool kEpInTiles = FT * kBlk32 >= (NW / 2) * kEp;
  __shared__ __attribute__((aligned(16))) float epi[kEpInTiles ? 1 : NW * kEp];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int cl = lane & 31;
  const int g = lane >> 5;
  const int64_t jb = a.j_base + (int64_t)blockIdx.x * JB + wave * JW;
  const int f0 = a.f_base + blockIdx.y * FB;
  const int nrows = a.F - f0 < FB ? a.F - f0 : FB;

  LaneState<CT> st;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    int64_t ci = jb + ct * 32 + cl;
    ci = ci < a.J ? ci : a.J - 1;
    st.qx[ct] = a.cand[ci];
    st.qy[ct] = a.cand[a.J + ci];
    st.qz[ct] = a.cand[2 * a.J + ci];
    st.rm[ct] = 0.0;
    st.xr[ct] = 0;
    st.xf[ct] = 0.0f;
    st.sp[ct] = 0.0f;
  }
  st.cur_m = -1;
  st.cur_p = -1;
  for (int i = tid; i < FB; i += 64 * NW) kbest[i] = 0ull;

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
  int acc_p = -1;  // the pair whose terms acc holds (two-level sums)
  auto fold = [&](int p) {
    if (COMP && p != acc_p && acc_p >= 0) {
#pragma unroll
      for (int ct = 0; ct < (COMP ? CT : 1); ++ct)
#pragma unroll
        for (int ft = 0; ft < (COMP ? FT : 1); ++ft) {
          hi[ct][ft] += acc[ct][ft];
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[ct][ft][r] = 0.0f;
        }
    }
    acc_p = p;
  };

  const Stage32 sg = stage32_init<NW>(a, wave, lane);
  stage_run<FB, NW>(a, recs[0], sg, xs0, f0, nrows, wave);
  nyq_prepare<CT>(a, recs[0], st, g);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int ri = 0; ri < a.n_runs; ri += 2) {
    // even run: read xs0, copy the next run into xs1; odd run: read xs1,
    // copy the next run into xs0 (the run count is even). Each run is
    // prepared before the barrier ahead of it.
    const RunRec r0 = recs[ri];
    const RunRec r1 = recs[ri + 1];
    stage_run<FB, NW>(a, r1, sg, xs1, f0, nrows, wave);
    fold(r0.p);
    nyq_run<CT, FT>(r0, st, xs0, cl, g, acc);
    nyq_prepare<CT>(a, r1, st, g);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const bool more = ri + 2 < a.n_runs;
    const RunRec r2 = recs[more ? ri + 2 : ri];
    if (more) stage_run<FB, NW>(a, r2, sg, xs0, f0, nrows, wave);
    fold(r1.p);
    nyq_run<CT, FT>(r1, st, xs1, cl, g, acc);
    if (more) nyq_prepare<CT>(a, r2, st, g);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  if (COMP) {
#pragma unroll
    for (int ct = 0; ct < (COMP ? CT : 1); ++ct)
#pragma unroll
      for (int ft = 0; ft < (COMP ? FT : 1); ++ft) acc[ct][ft] += hi[ct][ft];
  }

  // epilogue: D[frame][cand], lane (cl, g), register r -> frame 8 (r / 4) + 4 g + r % 4.
  // x2, optional map store, the argmax of each frame tile through the wave's
  // LDS block (in the staging tiles, free after the last barrier, when half
  // the waves fit in each; else an array of its own), then the block's LDS
  // max per frame and one global 64-bit atomic per frame and workgroup
  float* ep = kEpInTiles ? (wave < NW / 2 ? xs0 : xs1) + (wave % (NW / 2)) * kEp : epi + wave * kEp;
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
    float v[CT][16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int fg = f0 + ft * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int64_t ci = jb + ct * 32 + cl;
        v[ct][r] = 2.0f * acc[ct][ft][r];
        if (a.map && ci < a.J && fg < a.F) a.map[(size_t)fg * a.J + ci] = v[ct][r];
        if (ci >= a.J) v[ct][r] = -__builtin_inff();
      }
    }
    if (a.keys) {
      const unsigned long long k = tile_argmax_key<CT>(ep, v, jb);
      if (k && f0 + ft * 32 + cl < a.F) atomicMax(&kbest[ft * 32 + cl], k);
    }
  }
  if (a.keys) {
    __syncthreads();
    for (int i = tid; i < FB; i += 64 * NW) {
      const unsigned long long k = kbest[i];
      if (k && f0 + i < a.F) atomicMax(a.keys + 2 * (size_t)(f0 + i), k);
    }
  }
}

// Float64 instance (vector units): one thread per candidate, FB64 frames per
// block. Same data flow as the FP32 kernel; exists to check indexing and
// algebra against the float64 oracle to ~1e-12.
constexpr int kFB64 = 8;

__global__ __launch_bounds__(256) void nyquist_f64_kernel(NyqArgs a) {
  __shared__ float xs[kFB64 * kStride];
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
  for (int ri = 0; ri < a.n_runs; ++ri) {
    const LagRun run = a.runs[ri];
    const PairDesc pd = a.pairs[run.p];
    __syncthreads();
    const float* src = a.xi + pd.off + run.t0;
    for (int e = tid; e < kFB64 * run.len; e += 256) {
      const int f = e / run.len, t = e - f * run.len;
      const int fg = f0 + f;
      xs[f * kStride + t] = fg < a.F ? src[(size_t)fg * a.S + t] : 0.0f;
    }
    __syncthreads();
    const double x = pair_x(a, pd, qx, qy, qz);
    const double xr = rint(x);
    const double xf = x - xr;
    const double sp = sinpi(xf);
    for (int t = 0; t < run.len; ++t) {
      const int n = -pd.h + run.t0 + t;
      const int ia = static_cast<int>(xr) - n;
      double wgt;
      if (ia == 0 && xf == 0.0) {
        wgt = 1.0;
      } else {
        wgt = ((ia & 1) ? -sp : sp) / (M_PI * (static_cast<double>(ia) + xf));
      }
#pragma unroll
      for (int f = 0; f < kFB64; ++f) acc[f] += wgt * static_cast<double>(xs[f * kStride + t]);
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

int nyquist_workgroups_per_cu(int dtype) {
  if (dtype != SRP_FP32) return mx2_workgroups_per_cu(dtype);
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &n, reinterpret_cast<const void*>(&nyquist_f32_kernel<1, 8, 8, false>), 64 * 8, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_nyquist(const srp_geometry_s* g, const void* xi, int F, int dtype, float* map,
                          unsigned long long* keys, hipStream_t s) {
  NyqArgs a;
  a.cand = g->d_cand;
  a.mic = g->d_mic;
  a.pairs = g->d_pairs;
  a.runs = g->d_nyq_runs;
  a.n_runs = static_cast<int>(g->nyq_runs.size());
  a.xi = static_cast<const float*>(xi);
  a.F = F;
  a.f_base = 0;
  a.j_base = 0;
  a.S = static_cast<int>(g->info.S);
  a.J = g->info.J;
  a.inv_cT = g->inv_cT;
  a.far_field = g->info.field == SRP_FAR_FIELD;
  a.map = map;
  a.keys = keys;
  a.zero = g->d_zero;
  if (dtype == SRP_FP32) {
    int64_t samples = 0;
    for (const PairDesc& pd : g->pairs) samples += 2 * pd.h + 1;
    if (samples <= kNyqPlainSumMax) {
      launch_in_rounds(g, F, a, g->wg_per_cu[0], [&](auto ft, const NyqArgs& b, dim3 grid) {
        hipLaunchKernelGGL((nyquist_f32_kernel<1, decltype(ft)::value, 8, false>), grid,
                           dim3(64 * 8), 0, s, b, g->d_nyq_recs);
      });
    } else {
      launch_frame_blocks<4>(F, a, [&](auto ft, const NyqArgs& b, int fblocks) {
        constexpr int CT = 1, NW = 4, JB = NW * 32 * CT;
        const dim3 grid(static_cast<unsigned>((b.J + JB - 1) / JB), fblocks);
        hipLaunchKernelGGL((nyquist_f32_kernel<CT, decltype(ft)::value, NW, true>), grid,
                           dim3(64 * NW), 0, s, b, g->d_nyq_recs);
      });
    }
    return hipGetLastError();
  }
  if (dtype == SRP_BF16 || dtype == SRP_FP16)
    return launch_nyquist_mx2(g, xi, F, dtype, map, keys, s);
  if (dtype == SRP_FP64) {
    dim3 grid(static_cast<unsigned>((a.J + 255) / 256), (F + kFB64 - 1) / kFB64);
    hipLaunchKernelGGL(nyquist_f64_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  return hipErrorNotSupported;
}

}  // namespace srp
