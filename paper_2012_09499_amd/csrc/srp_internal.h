// Internal declarations shared by the host API (srp_api.hip) and the kernel
// translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "srp.h"

namespace srp {

// One microphone pair (Section 2.1): mics m > mp, window half-width
// h = N_p + N_aux and the column of its first sample in the packed layout.
struct PairDesc {
  int32_t m, mp, h, off;
};

// A run of consecutive lags [t0, t0 + len) of pair p's window (t counts from
// the window's first lag n = -h). Long windows are cut into several runs so
// that one run fits a kernel's on-chip staging buffer.
struct LagRun {
  int32_t p, t0, len, pad;
};

// Everything the BF16/FP16 interpolation kernel needs for one lag run in one
// record, so a run costs one scalar load instead of the dependent chain
// run -> pair -> microphone positions.
struct RunRec {
  int32_t p, t0, len, off;  // the run, and its pair's window offset in the sample layout
  int32_t h, m, mp, pad;    // the pair: half window, microphones m > mp
  double pm[3], pn[3];      // positions of microphones m and mp
  float pmf[3], pnf[3];     // the same minus the microphone centroid, in float32 (the
                            // Nyquist BF16/FP16 TDOAs; far field: not shifted)
};

// Lag runs of the Nyquist interpolation kernels are at most this long (one
// lane per lag when a wave copies a run into LDS).
constexpr int kNyqRunMax = 64;
// Lag runs of the BF16/FP16 Nyquist kernel are at most this long (8 of its
// 16-lag steps): one run per pair window up to 128 lags, so fewer run
// boundaries (a copy, a barrier and a pipeline restart each) than with
// kNyqRunMax.
constexpr int kMxRunMax = 128;
// ... and at most this long in its launches of at most 4 frame tiles (128
// frames), whose staging tiles then take the same LDS.
constexpr int kMxRunMaxFew = 256;
// Pair windows of the GCC-sample layout start at multiples of this many
// samples (16 bytes of bf16/fp16), so staging copies can move 16-byte chunks.
constexpr int kSampleAlign = 8;
// Bin runs of the conventional kernel are at most this many bins.
constexpr int kConvRunBins = 32;
// Lag tiles of the GCC-sample kernel are 32 lags wide (one matrix-core tile).
constexpr int kGccLagTile = 32;
// Lag tiles per work unit of the fused GCC kernel (srp_gcc_samples_frames).
constexpr int kGccItemTiles = 3;

// Lag tiles [t0, t0 + nt) (32 lags each, counted from the window's first lag)
// of pair p: the lags of one work unit of the fused GCC kernel.
struct GccItem {
  int32_t p, t0, nt, pad;
};

// Frames per array in one batched launch (srp_map_nyquist_batched): FP32
// samples (vector units) and BF16/FP16 samples (16-frame matrix-core tile).
constexpr int kBatchMaxF = 8;
constexpr int kBatchMaxFMx = 16;
// BF16/FP16 items with at most this many frames run on the vector units (the
// matrix-core tile costs about the same for 1 and for 16 frames; measured over
// 64 serving arrays, the vector kernel is faster up to 2 frames per array).
constexpr int kBatchVecMaxF = 2;

// Device copy of one item of a batched launch.
struct BatchItemDev {
  const double* cand;        // [3][J]
  const double* mic;         // [M][3]
  const PairDesc* pairs;     // [P]
  int64_t J;
  int64_t xi_off;            // first sample of the item in the batch's sample arena
  int S, P, F, far_field;
  double inv_cT;
  float* map;                // [F][J] or null
  unsigned long long* keys;  // srp_peak[F] viewed as u64 pairs, or null
  int block_begin;           // first workgroup of the item
  int xq_exp;                // BF16/FP16 items: fractions on the grid 2^-xq_exp (see k_batched)
};

}  // namespace srp

struct srp_geometry_s {
  srp_geometry_info info;
  int device = 0;
  int n_cu = 256;          // compute units of the device (workgroup rounds)
  int wg_per_cu[3] = {1, 1, 1};  // resident Nyquist workgroups per CU: FP32, BF16, FP16
  int wg_per_cu_conv[2] = {1, 1};  // resident BF16/FP16 conventional workgroups per CU
  int Kp = 0;              // bins of a row of the BF16/FP16 conventional input (K up to a multiple of 8)
  int Kr = 0;              // bins of a row of the per-microphone phasors (K up to a multiple of 16)
  int n_convmx_runs = 0;   // 32-bin runs of the BF16/FP16 conventional map (even count)
  double inv_cT = 0.0;     // converts a path difference in metres into x = dt / T
  double fs_over_c = 0.0;  // converts a path difference in metres into samples
  double mic_centre[3] = {0.0, 0.0, 0.0};  // centroid of the microphones (near field)
  int log2L = 0;
  int gcc_nw = 0;          // row width of the GCC phase tables (2 h_max + 34, even)
  std::vector<srp::PairDesc> pairs;
  std::vector<int32_t> N_p;
  std::vector<int64_t> offsets;
  std::vector<srp::LagRun> gcc_tiles;  // lag tiles of srp_gcc_samples
  std::vector<srp::GccItem> gcc_items;  // workgroup items of srp_gcc_samples_frames
  std::vector<srp::LagRun> nyq_runs;   // lag runs of srp_map_nyquist (even count)
  std::vector<srp::LagRun> mx_runs;    // lag runs of the BF16/FP16 Nyquist map (even count)
  std::vector<srp::LagRun> mx_runs_few;  // the same up to kMxRunMaxFew lags (<= 4 frame tiles)
  std::vector<srp::LagRun> conv_runs;  // bin runs (p, k0, len) of srp_map_conventional (even count)
  // device copies
  double* d_mic = nullptr;             // [M][3]
  double* d_cand = nullptr;            // [3][J] (structure of arrays)
  srp::PairDesc* d_pairs = nullptr;    // [P]
  srp::LagRun* d_gcc_tiles = nullptr;
  srp::GccItem* d_gcc_items = nullptr;
  srp::LagRun* d_nyq_runs = nullptr;
  srp::RunRec* d_nyq_recs = nullptr;   // one record per entry of nyq_runs
  srp::RunRec* d_mx_recs = nullptr;    // one record per entry of mx_runs
  srp::RunRec* d_mx_recs_few = nullptr;  // one record per entry of mx_runs_few
  srp::RunRec* d_convmx_recs = nullptr;  // 32-bin runs of the BF16/FP16 conventional map
  srp::LagRun* d_conv_runs = nullptr;
  float* d_window = nullptr;           // [L]
  float2* d_twiddle = nullptr;         // [L] exp(-j 2 pi t / L)
  float2* d_gcc_table = nullptr;       // [Kr][gcc_nw] (cos, -sin) of 2 pi f_k n T (zeros past K)
  float2* d_gcc_wtable = nullptr;      // [Kr][gcc_nw] the same times the bin weight w_k
  float* d_binw = nullptr;             // [Kr] (zeros past K)
  float* d_zero = nullptr;             // 64 zeros (source of zero-filled staging chunks)
  int* d_chunk_pair = nullptr;         // pair of each 8-column chunk of the cached weights (-1: none)
};

namespace srp {

void set_error(const std::string& msg);

// Kernel launchers. Each returns hipSuccess or the launch error; the host API
// validates every argument before calling them.
// ytil: [F][M][Kr] unit phasors (zeros past K).
hipError_t launch_fft_phat(const srp_geometry_s* g, const float* frames, int F, float2* ytil,
                           hipStream_t s);
// GCC samples of every pair from the phasors ytil (fused cross-spectrum + GCC).
hipError_t launch_gcc_phasor(const srp_geometry_s* g, const float2* ytil, int F, int dtype,
                             void* xi, hipStream_t s);
hipError_t launch_cross(const srp_geometry_s* g, const float2* ytil, int F, float2* psi,
                        hipStream_t s);
// Per-microphone phasor staging owned by the library (srp_cross_spectra_noalloc):
// kCrossStaticElems float2 per GPU. Returns its device address on `device`,
// which must be the current device (looked up once per device).
constexpr size_t kCrossStaticElems = size_t(64) << 20 >> 3;  // 64 MiB of float2
constexpr int kMaxDevices = 64;
hipError_t cross_static_scratch(int device, float2** out);
hipError_t launch_gcc_samples(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                              void* xi, hipStream_t s);
int nyquist_workgroups_per_cu(int dtype);  // occupancy of the interpolation kernels
hipError_t launch_nyquist(const srp_geometry_s* g, const void* xi, int F, int dtype, float* map,
                          unsigned long long* keys, hipStream_t s);
// BF16/FP16 Nyquist map kernel (k_nyquist_mx.hip): the geometries it takes
// (S < 2^23 columns), its resident workgroups per CU, and its launch.
bool mx2_supported(const srp_geometry_s* g);
int mx2_workgroups_per_cu(int dtype);
// BF16/FP16 conventional map on the same kernel (k_nyquist_mx.hip): the
// geometries it takes (256 x 2 P Kp x 2 bytes < 2^32), occupancy, launch; and
// the weighted, rounded spectra it reads (k_spectra.hip).
bool conv_mx_supported(const srp_geometry_s* g);
int conv_mx_workgroups_per_cu(int dtype);
hipError_t launch_conventional_mx(const srp_geometry_s* g, const void* spec, int F, int dtype,
                                  float* map, unsigned long long* keys, hipStream_t s);
hipError_t launch_spectra_lowp(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                               void* out, hipStream_t s);
hipError_t launch_nyquist_mx2(const srp_geometry_s* g, const void* xi, int F, int dtype,
                              float* map, unsigned long long* keys, hipStream_t s);
bool conventional_supports(int dtype);  // dtypes srp_map_conventional has a kernel for
hipError_t launch_conventional(const srp_geometry_s* g, const float2* psi, int F, int dtype,
                               float* map, unsigned long long* keys, hipStream_t s);
// Items [0, n_vec) go to the vector-unit kernel, [n_vec, n_vec + n_mx) to the
// matrix-core kernel (BF16/FP16 only); block_begin counts within each group.
hipError_t launch_nyquist_batched(const BatchItemDev* d_items, int n_vec, int blocks_vec,
                                  int max_f_vec, int n_mx, int blocks_mx, int dtype,
                                  const void* xi, hipStream_t s);
hipError_t launch_points(const srp_geometry_s* g, const float* xi, int F, const double* pts,
                         int Q, float* out, hipStream_t s);
int cached_weight_cols(const srp_geometry_s* g);
hipError_t launch_nyquist_weights(const srp_geometry_s* g, int dtype, void* w, hipStream_t s);
hipError_t launch_nyquist_cached(const srp_geometry_s* g, const void* w, const void* xi, int F,
                                 int dtype, float* map, unsigned long long* keys, hipStream_t s);
hipError_t launch_peaks_init(srp_peak* peaks, int F, hipStream_t s);
hipError_t launch_peaks_finalize(srp_peak* peaks, int F, hipStream_t s);
hipError_t launch_argmax(const float* map, int F, int64_t J, unsigned long long* keys,
                         hipStream_t s);

}  // namespace srp
