// C ABI of libsrp: argument validation, host-side geometry precompute and
// kernel dispatch. Host arithmetic here is float64 and is compiled without
// floating-point contraction, so pair distances and N_p = floor(d_p / (c T))
// are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "srp_internal.h"

namespace srp {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

srp_status fail(srp_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

srp_status device_fail(hipError_t e, const char* where) {
  return fail(SRP_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Euclidean distance, summed x, y, z in that order (no contraction).
double dist3(const double* a, const double* b) {
  double dx = a[0] - b[0];
  double dy = a[1] - b[1];
  double dz = a[2] - b[2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

// Per-pair window half-widths (Section 3.2): N_p = floor(d_p / (c T)), and
// the sample layout: pair p's W_p = 2 (N_p + N_aux) + 1 samples start at
// offsets[p], a multiple of kSampleAlign.
srp_status layout(const double* mic, int M, double c, double f_max, int n_aux,
                  std::vector<int32_t>& N_p, std::vector<int64_t>& offsets) {
  if (mic == nullptr) return fail(SRP_ERR_INVALID_ARG, "mic_xyz is NULL");
  if (M < 2 || M > 256) return fail(SRP_ERR_INVALID_ARG, "M must be in [2, 256]");
  if (!(c > 0.0) || !std::isfinite(c)) return fail(SRP_ERR_INVALID_ARG, "c must be > 0");
  if (!(f_max > 0.0) || !std::isfinite(f_max))
    return fail(SRP_ERR_INVALID_ARG, "f_max must be > 0");
  if (n_aux < 0) return fail(SRP_ERR_INVALID_ARG, "n_aux must be >= 0");
  for (int i = 0; i < 3 * M; ++i)
    if (!std::isfinite(mic[i])) return fail(SRP_ERR_INVALID_ARG, "non-finite mic coordinate");
  const double T = 1.0 / (2.0 * f_max);
  const int P = M * (M - 1) / 2;
  N_p.assign(P, 0);
  offsets.assign(P + 1, 0);
  int p = 0;
  for (int m = 1; m < M; ++m) {
    for (int mp = 0; mp < m; ++mp, ++p) {
      const double d = dist3(mic + 3 * m, mic + 3 * mp);
      const double q = std::floor(d / (c * T));
      if (q > 1.0e8) return fail(SRP_ERR_INVALID_ARG, "pair window too long");
      N_p[p] = static_cast<int32_t>(q);
      // windows start at multiples of kSampleAlign samples (zero-filled gaps)
      const int64_t W = 2 * (int64_t)(N_p[p] + n_aux) + 1;
      offsets[p + 1] = offsets[p] + (W + kSampleAlign - 1) / kSampleAlign * kSampleAlign;
    }
  }
  return SRP_OK;
}

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n, hipStream_t s) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(T) > 0 ? n * sizeof(T) : 16);
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  return hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, s);
}

void free_geometry(srp_geometry_s* g) {
  if (!g) return;
  hipFree(g->d_mic);
  hipFree(g->d_cand);
  hipFree(g->d_pairs);
  hipFree(g->d_gcc_tiles);
  hipFree(g->d_gcc_items);
  hipFree(g->d_nyq_runs);
  hipFree(g->d_nyq_recs);
  hipFree(g->d_mx_recs);
  hipFree(g->d_mx_recs_few);
  hipFree(g->d_convmx_recs);
  hipFree(g->d_conv_runs);
  hipFree(g->d_window);
  hipFree(g->d_twiddle);
  hipFree(g->d_gcc_table);
  hipFree(g->d_gcc_wtable);
  hipFree(g->d_binw);
  hipFree(g->d_zero);
  hipFree(g->d_chunk_pair);
  delete g;
}

}  // namespace
}  // namespace srp

using namespace srp;

extern "C" {

const char* srp_last_error(void) { return g_last_error.c_str(); }

const char* srp_version(void) { return "libsrp 0.1.0 gfx950"; }

srp_status srp_pair_layout(const double* mic_xyz, int32_t M, double c, double f_max,
                           int32_t n_aux, int32_t* N_p, int64_t* offsets, int64_t* S) {
  std::vector<int32_t> np;
  std::vector<int64_t> off;
  srp_status st = layout(mic_xyz, M, c, f_max, n_aux, np, off);
  if (st != SRP_OK) return st;
  if (N_p) std::memcpy(N_p, np.data(), np.size() * sizeof(int32_t));
  if (offsets) std::memcpy(offsets, off.data(), off.size() * sizeof(int64_t));
  if (S) *S = off.back();
  return SRP_OK;
}

srp_status srp_geometry(const double* mic_xyz, int32_t M, const double* cand_xyz, int64_t J,
                        int32_t field, double c, double fs, int32_t L, double f_max,
                        int32_t n_aux, int32_t window, void* stream, srp_geometry_t** out) {
  if (out == nullptr) return fail(SRP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (cand_xyz == nullptr) return fail(SRP_ERR_INVALID_ARG, "cand_xyz is NULL");
  if (J < 1 || J >= (int64_t(1) << 31)) return fail(SRP_ERR_INVALID_ARG, "J must be in [1, 2^31)");
  if (field != SRP_NEAR_FIELD && field != SRP_FAR_FIELD)
    return fail(SRP_ERR_INVALID_ARG, "unknown field model");
  if (window != SRP_WIN_HANN && window != SRP_WIN_SQRT_HANN && window != SRP_WIN_RECT)
    return fail(SRP_ERR_INVALID_ARG, "unknown window");
  if (!(fs > 0.0) || !std::isfinite(fs)) return fail(SRP_ERR_INVALID_ARG, "fs must be > 0");
  if (!is_pow2(L) || L < 16 || L > 8192)
    return fail(SRP_ERR_INVALID_ARG, "L must be a power of two in [16, 8192]");
  if (!(f_max > 0.0) || f_max > fs / 2.0)
    return fail(SRP_ERR_INVALID_ARG, "f_max must be in (0, fs/2]");
  std::vector<int32_t> np;
  std::vector<int64_t> off;
  srp_status st = layout(mic_xyz, M, c, f_max, n_aux, np, off);
  if (st != SRP_OK) return st;
  const int P = M * (M - 1) / 2;
  int h_max = 0;
  for (int p = 0; p < P; ++p) {
    const int h = np[p] + n_aux;
    if (2 * (int64_t)h + 1 > L)
      return fail(SRP_ERR_INVALID_ARG,
                  "a pair window 2 (N_p + N_aux) + 1 exceeds L (the discrete GCC is L-periodic)");
    h_max = h > h_max ? h : h_max;
  }
  if (off.back() >= (int64_t(1) << 31)) return fail(SRP_ERR_INVALID_ARG, "S too large");
  for (int64_t i = 0; i < 3 * J; ++i)
    if (!std::isfinite(cand_xyz[i]))
      return fail(SRP_ERR_INVALID_ARG, "non-finite candidate coordinate");
  if (field == SRP_FAR_FIELD) {
    for (int64_t i = 0; i < J; ++i) {
      const double* r = cand_xyz + 3 * i;
      const double n = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      if (std::fabs(n - 1.0) > 1e-9)
        return fail(SRP_ERR_INVALID_ARG, "far-field candidates must be unit vectors");
    }
  }

  srp_geometry_s* g = new (std::nothrow) srp_geometry_s();
  if (!g) return fail(SRP_ERR_OUT_OF_MEMORY, "host allocation failed");
  srp_geometry_info& in = g->info;
  in.M = M;
  in.P = P;
  in.L = L;
  in.K = static_cast<int32_t>(std::floor(f_max * L / fs)) + 1;
  in.J = J;
  in.S = off.back();
  in.h_max = h_max;
  in.n_aux = n_aux;
  in.field = field;
  in.window = window;
  in.c = c;
  in.fs = fs;
  in.f_max = f_max;
  in.T = 1.0 / (2.0 * f_max);
  g->inv_cT = 1.0 / (c * in.T);
  g->fs_over_c = fs / c;
  if (field != SRP_FAR_FIELD) {
    for (int i = 0; i < M; ++i)
      for (int d = 0; d < 3; ++d) g->mic_centre[d] += mic_xyz[3 * i + d] / M;
  }
  g->log2L = 0;
  while ((1 << g->log2L) < L) ++g->log2L;
  g->N_p = np;
  g->offsets = off;
  g->pairs.resize(P);
  {
    int p = 0;
    for (int m = 1; m < M; ++m)
      for (int mp = 0; mp < m; ++mp, ++p)
        g->pairs[p] = PairDesc{m, mp, np[p] + n_aux, static_cast<int32_t>(off[p])};
  }
  for (int p = 0; p < P; ++p) {
    const int W = 2 * g->pairs[p].h + 1;
    for (int t0 = 0; t0 < W; t0 += kGccLagTile)
      g->gcc_tiles.push_back(LagRun{p, t0, W - t0 < kGccLagTile ? W - t0 : kGccLagTile, 0});
    // the fused GCC kernel: the window's ceil(W / 32) tiles (whose last one also
    // covers the layout's gap up to the next multiple of 8) in about equal
    // items of at most kGccItemTiles tiles
    {
      const int ntiles = (W + kGccLagTile - 1) / kGccLagTile;
      const int n_it = (ntiles + kGccItemTiles - 1) / kGccItemTiles;
      const int per_it = (ntiles + n_it - 1) / n_it;
      for (int t = 0; t < ntiles; t += per_it)
        g->gcc_items.push_back(GccItem{p, t, ntiles - t < per_it ? ntiles - t : per_it, 0});
    }
    // a window longer than one run is split into runs of about equal length
    // (all but the last a multiple of kSampleAlign lags, so every run starts
    // on an aligned column), not into full runs and a short remainder: each
    // run costs a fixed copy and synchronisation, which a short run does not
    // cover with work
    auto split = [&](int run_max, std::vector<LagRun>& runs) {
      const int nr = (W + run_max - 1) / run_max;
      const int per = (W + nr - 1) / nr;
      const int run_len = (per + kSampleAlign - 1) / kSampleAlign * kSampleAlign;
      for (int t0 = 0; t0 < W; t0 += run_len)
        runs.push_back(LagRun{p, t0, W - t0 < run_len ? W - t0 : run_len, 0});
    };
    split(kNyqRunMax, g->nyq_runs);
    split(kMxRunMax, g->mx_runs);
    split(kMxRunMaxFew, g->mx_runs_few);
  }
  // the FP32 interpolation kernel consumes runs two at a time, the BF16/FP16
  // one three at a time: pad to a multiple of 6 with empty runs of the last
  // pair (no lags, no copy, no pair change)
  while (g->nyq_runs.size() % 6)
    g->nyq_runs.push_back(LagRun{P - 1, 2 * (np[P - 1] + n_aux) + 1, 0, 0});
  // the BF16/FP16 kernel consumes its runs two at a time
  for (std::vector<LagRun>* runs : {&g->mx_runs, &g->mx_runs_few})
    if (runs->size() % 2) runs->push_back(LagRun{P - 1, 2 * (np[P - 1] + n_aux) + 1, 0, 0});
  // the fused GCC kernel deals its units out largest first
  std::stable_sort(g->gcc_items.begin(), g->gcc_items.end(),
                   [](const GccItem& a, const GccItem& b) { return a.nt > b.nt; });
  for (int p = 0; p < P; ++p)
    for (int k0 = 0; k0 < in.K; k0 += kConvRunBins)
      g->conv_runs.push_back(LagRun{p, k0, in.K - k0 < kConvRunBins ? in.K - k0 : kConvRunBins, 0});
  if (g->conv_runs.size() % 2) g->conv_runs.push_back(LagRun{P - 1, in.K, 0, 0});
  const int K = in.K;
  g->Kr = (K + 15) / 16 * 16;
  const int Kr = g->Kr;
  // lags -h_max .. h_max plus a tile's overhang and one more, rounded to even
  // (16-byte aligned copies of lag pairs in the fused GCC kernel)
  g->gcc_nw = 2 * h_max + 2 + kGccLagTile;

  // float64 tables, each rounded once to float32
  std::vector<float> win(L);
  for (int t = 0; t < L; ++t) {
    const double hann = 0.5 - 0.5 * std::cos(2.0 * M_PI * t / L);
    win[t] = static_cast<float>(window == SRP_WIN_HANN ? hann
                                : window == SRP_WIN_SQRT_HANN ? std::sqrt(hann)
                                                              : 1.0);
  }
  std::vector<float2> tw(L);
  for (int t = 0; t < L; ++t) {
    const double a = 2.0 * M_PI * t / L;
    tw[t] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a)));
  }
  std::vector<float> binw(Kr, 0.0f);
  for (int k = 0; k < K; ++k) binw[k] = 2.0f;
  binw[0] = 1.0f;
  if (2 * (K - 1) == L) binw[K - 1] = 1.0f;
  // GCC phase 2 pi f_k n T in turns: k n fs T / L, reduced mod 1 exactly when
  // fs T = 1/2 ... in general through the float64 fraction.
  std::vector<float2> gtab((size_t)Kr * g->gcc_nw, make_float2(0.0f, 0.0f));
  const bool integer_lags = (2.0 * f_max == fs);
  for (int k = 0; k < K; ++k) {
    for (int j = 0; j < g->gcc_nw; ++j) {
      const int64_t n = (int64_t)j - h_max;
      double turns;
      if (integer_lags) {
        int64_t r = ((int64_t)k * n) % L;
        if (r < 0) r += L;
        turns = (double)r / L;
      } else {
        const double v = (double)k * (double)n * (fs * in.T) / L;
        turns = v - std::floor(v);
      }
      const double a = 2.0 * M_PI * turns;
      gtab[(size_t)k * g->gcc_nw + j] =
          make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a)));
    }
  }
  std::vector<double> cand_soa(3 * (size_t)J);
  for (int64_t i = 0; i < J; ++i)
    for (int d = 0; d < 3; ++d) cand_soa[(size_t)d * J + i] = cand_xyz[3 * i + d];

  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&g->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, g->device);
  if (e == hipSuccess && g->n_cu < 1) g->n_cu = 1;
  if (e == hipSuccess) {
    g->wg_per_cu[0] = nyquist_workgroups_per_cu(SRP_FP32);
    g->wg_per_cu[1] = nyquist_workgroups_per_cu(SRP_BF16);
    g->wg_per_cu[2] = nyquist_workgroups_per_cu(SRP_FP16);
    g->wg_per_cu_conv[0] = conv_mx_workgroups_per_cu(SRP_BF16);
    g->wg_per_cu_conv[1] = conv_mx_workgroups_per_cu(SRP_FP16);
  }
  if (e == hipSuccess) e = upload(&g->d_mic, mic_xyz, 3 * (size_t)M, s);
  if (e == hipSuccess) e = upload(&g->d_cand, cand_soa.data(), cand_soa.size(), s);
  if (e == hipSuccess) e = upload(&g->d_pairs, g->pairs.data(), g->pairs.size(), s);
  if (e == hipSuccess) e = upload(&g->d_gcc_tiles, g->gcc_tiles.data(), g->gcc_tiles.size(), s);
  if (e == hipSuccess) e = upload(&g->d_gcc_items, g->gcc_items.data(), g->gcc_items.size(), s);
  if (e == hipSuccess) e = upload(&g->d_nyq_runs, g->nyq_runs.data(), g->nyq_runs.size(), s);
  // self-contained records of the lag runs (the run, its pair's window and
  // microphone positions) for the kernels that read one record per run
  auto run_records = [&](const std::vector<LagRun>& runs) {
    std::vector<RunRec> recs(runs.size());
    for (size_t i = 0; i < recs.size(); ++i) {
      const LagRun& r = runs[i];
      const PairDesc& pd = g->pairs[r.p];
      RunRec& q = recs[i];
      q.p = r.p;
      q.t0 = r.t0;
      q.len = r.len;
      q.off = pd.off;
      q.h = pd.h;
      q.m = pd.m;
      q.mp = pd.mp;
      q.pad = 0;
      for (int d = 0; d < 3; ++d) {
        q.pm[d] = mic_xyz[3 * pd.m + d];
        q.pn[d] = mic_xyz[3 * pd.mp + d];
        q.pmf[d] = static_cast<float>(q.pm[d] - g->mic_centre[d]);
        q.pnf[d] = static_cast<float>(q.pn[d] - g->mic_centre[d]);
      }
    }
    return recs;
  };
  const std::vector<RunRec> recs = run_records(g->nyq_runs);
  const std::vector<RunRec> mx_recs = run_records(g->mx_runs);
  const std::vector<RunRec> mx_recs_few = run_records(g->mx_runs_few);
  if (e == hipSuccess) e = upload(&g->d_nyq_recs, recs.data(), recs.size(), s);
  if (e == hipSuccess) e = upload(&g->d_mx_recs, mx_recs.data(), mx_recs.size(), s);
  if (e == hipSuccess)
    e = upload(&g->d_mx_recs_few, mx_recs_few.data(), mx_recs_few.size(), s);
  // 32-bin runs of the BF16/FP16 conventional map over the weighted spectra
  // [F][P][Kp] x (re, im): a run's values start at 2 (p Kp + k0) of a frame row
  g->Kp = (in.K + 7) / 8 * 8;
  std::vector<RunRec> crecs;
  for (int p = 0; p < P; ++p) {
    const PairDesc& pd = g->pairs[p];
    for (int k0 = 0; k0 < g->Kp; k0 += kConvRunBins) {
      RunRec q;
      q.p = p;
      q.t0 = 2 * k0;
      q.len = 2 * (g->Kp - k0 < kConvRunBins ? g->Kp - k0 : kConvRunBins);
      q.off = 2 * p * g->Kp;
      q.h = k0;
      q.m = pd.m;
      q.mp = pd.mp;
      q.pad = 0;
      for (int d = 0; d < 3; ++d) {
        q.pm[d] = mic_xyz[3 * pd.m + d];
        q.pn[d] = mic_xyz[3 * pd.mp + d];
        q.pmf[d] = static_cast<float>(q.pm[d] - g->mic_centre[d]);
        q.pnf[d] = static_cast<float>(q.pn[d] - g->mic_centre[d]);
      }
      crecs.push_back(q);
    }
  }
  if (crecs.size() % 2) {  // consumed two at a time: an empty run of the last pair
    RunRec q = crecs.back();
    q.len = 0;
    crecs.push_back(q);
  }
  g->n_convmx_runs = static_cast<int>(crecs.size());
  if (e == hipSuccess) e = upload(&g->d_convmx_recs, crecs.data(), crecs.size(), s);
  if (e == hipSuccess) e = upload(&g->d_conv_runs, g->conv_runs.data(), g->conv_runs.size(), s);
  if (e == hipSuccess) e = upload(&g->d_window, win.data(), win.size(), s);
  if (e == hipSuccess) e = upload(&g->d_twiddle, tw.data(), tw.size(), s);
  if (e == hipSuccess) e = upload(&g->d_gcc_table, gtab.data(), gtab.size(), s);
  // the fused GCC kernel's table: w_k (1 or 2, so exact) times the phase table
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < g->gcc_nw; ++j) {
      float2& v = gtab[(size_t)k * g->gcc_nw + j];
      v = make_float2(binw[k] * v.x, binw[k] * v.y);
    }
  if (e == hipSuccess) e = upload(&g->d_gcc_wtable, gtab.data(), gtab.size(), s);
  if (e == hipSuccess) e = upload(&g->d_binw, binw.data(), binw.size(), s);
  const std::vector<float> zeros(64, 0.0f);
  if (e == hipSuccess) e = upload(&g->d_zero, zeros.data(), zeros.size(), s);
  // cached-weight columns: the pair owning each 8-column chunk (window plus gap)
  std::vector<int> chunk_pair((g->info.S + 127) / 128 * 16, -1);
  for (int p = 0; p < P; ++p) {
    const int64_t W8 = (2 * (int64_t)g->pairs[p].h + 1 + kSampleAlign - 1) / kSampleAlign *
                       kSampleAlign;
    for (int64_t c = g->pairs[p].off; c < g->pairs[p].off + W8; c += 8)
      chunk_pair[c / 8] = p;
  }
  if (e == hipSuccess) e = upload(&g->d_chunk_pair, chunk_pair.data(), chunk_pair.size(), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    const bool oom = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation);
    std::string msg = std::string("srp_geometry: ") + hipGetErrorString(e);
    free_geometry(g);
    return fail(oom ? SRP_ERR_OUT_OF_MEMORY : SRP_ERR_DEVICE, msg);
  }
  *out = g;
  return SRP_OK;
}

srp_status srp_geometry_query(const srp_geometry_t* g, srp_geometry_info* info, int32_t* N_p,
                              int64_t* offsets) {
  if (g == nullptr) return fail(SRP_ERR_INVALID_ARG, "geometry is NULL");
  if (info) *info = g->info;
  if (N_p) std::memcpy(N_p, g->N_p.data(), g->N_p.size() * sizeof(int32_t));
  if (offsets) std::memcpy(offsets, g->offsets.data(), g->offsets.size() * sizeof(int64_t));
  return SRP_OK;
}

void srp_geometry_destroy(srp_geometry_t* g) {
  if (!g) return;
  DeviceGuard dg(g->device);
  free_geometry(g);
}

srp_status srp_cross_spectra_workspace(const srp_geometry_t* g, int32_t F, size_t* bytes) {
  if (g == nullptr || bytes == nullptr) return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  *bytes = (size_t)F * g->info.M * g->Kr * sizeof(float2);
  return SRP_OK;
}

srp_status srp_cross_spectra(const srp_geometry_t* g, const float* frames, int32_t F,
                             int32_t weighting, void* workspace, size_t workspace_bytes,
                             float* psi, void* stream) {
  if (g == nullptr || frames == nullptr || workspace == nullptr || psi == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "srp_cross_spectra: NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (weighting != SRP_PHAT) return fail(SRP_ERR_UNSUPPORTED, "only PHAT weighting");
  const size_t need = (size_t)F * g->info.M * g->Kr * sizeof(float2);
  if (workspace_bytes < need) return fail(SRP_ERR_INVALID_ARG, "workspace too small");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  float2* ytil = static_cast<float2*>(workspace);
  hipError_t e = launch_fft_phat(g, frames, F, ytil, s);
  if (e != hipSuccess) return device_fail(e, "fft_phat");
  e = launch_cross(g, ytil, F, reinterpret_cast<float2*>(psi), s);
  if (e != hipSuccess) return device_fail(e, "cross");
  return SRP_OK;
}

srp_status srp_cross_spectra_noalloc(const srp_geometry_t* g, const float* frames, int32_t F,
                                     int32_t weighting, float* psi, void* stream) {
  if (g == nullptr || frames == nullptr || psi == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "srp_cross_spectra_noalloc: NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (weighting != SRP_PHAT) return fail(SRP_ERR_UNSUPPORTED, "only PHAT weighting");
  const size_t need = (size_t)F * g->info.M * g->Kr;
  if (need > kCrossStaticElems)
    return fail(SRP_ERR_INVALID_ARG,
                "srp_cross_spectra_noalloc: F * M * Kr * 8 bytes exceed the 64 MiB static buffer "
                "(Kr = K rounded up to a multiple of 16)");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  float2* ytil = nullptr;
  hipError_t e = cross_static_scratch(g->device, &ytil);
  if (e != hipSuccess) return device_fail(e, "static scratch address");
  hipStream_t s = static_cast<hipStream_t>(stream);
  e = launch_fft_phat(g, frames, F, ytil, s);
  if (e != hipSuccess) return device_fail(e, "fft_phat");
  e = launch_cross(g, ytil, F, reinterpret_cast<float2*>(psi), s);
  if (e != hipSuccess) return device_fail(e, "cross");
  return SRP_OK;
}

srp_status srp_gcc_samples(const srp_geometry_t* g, const float* psi, int32_t F, int32_t dtype,
                           void* xi, void* stream) {
  if (g == nullptr || psi == nullptr || xi == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "srp_gcc_samples: NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (dtype != SRP_FP32 && dtype != SRP_BF16 && dtype != SRP_FP16)
    return fail(SRP_ERR_UNSUPPORTED, "srp_gcc_samples stores FP32, BF16 or FP16");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipError_t e = launch_gcc_samples(g, reinterpret_cast<const float2*>(psi), F, dtype, xi,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "gcc_samples");
  return SRP_OK;
}

srp_status srp_gcc_samples_frames(const srp_geometry_t* g, const float* frames, int32_t F,
                                  int32_t weighting, int32_t dtype, void* workspace,
                                  size_t workspace_bytes, void* xi, void* stream) {
  if (g == nullptr || frames == nullptr || workspace == nullptr || xi == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "srp_gcc_samples_frames: NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (weighting != SRP_PHAT) return fail(SRP_ERR_UNSUPPORTED, "only PHAT weighting");
  if (dtype != SRP_FP32 && dtype != SRP_BF16 && dtype != SRP_FP16)
    return fail(SRP_ERR_UNSUPPORTED, "srp_gcc_samples_frames stores FP32, BF16 or FP16");
  const size_t need = (size_t)F * g->info.M * g->Kr * sizeof(float2);
  if (workspace_bytes < need) return fail(SRP_ERR_INVALID_ARG, "workspace too small");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  float2* ytil = static_cast<float2*>(workspace);
  hipError_t e = launch_fft_phat(g, frames, F, ytil, s);
  if (e != hipSuccess) return device_fail(e, "fft_phat");
  e = launch_gcc_phasor(g, ytil, F, dtype, xi, s);
  if (e != hipSuccess) return device_fail(e, "gcc_phasor");
  return SRP_OK;
}

srp_status srp_spectra_lowp_bytes(const srp_geometry_t* g, int32_t F, int32_t dtype,
                                  size_t* bytes) {
  if (g == nullptr || bytes == nullptr) return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (dtype != SRP_BF16 && dtype != SRP_FP16)
    return fail(SRP_ERR_UNSUPPORTED, "low-precision spectra are BF16 or FP16");
  *bytes = (size_t)F * g->info.P * g->Kp * 2 * 2;
  return SRP_OK;
}

srp_status srp_spectra_lowp(const srp_geometry_t* g, const float* psi, int32_t F, int32_t dtype,
                            void* out, size_t out_bytes, void* stream) {
  size_t need = 0;
  srp_status st = srp_spectra_lowp_bytes(g, F, dtype, &need);
  if (st != SRP_OK) return st;
  if (psi == nullptr || out == nullptr) return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (out_bytes < need) return fail(SRP_ERR_INVALID_ARG, "output buffer too small");
  if ((reinterpret_cast<uintptr_t>(out) & 15) != 0)
    return fail(SRP_ERR_INVALID_ARG, "output must be 16-byte aligned");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipError_t e = launch_spectra_lowp(g, reinterpret_cast<const float2*>(psi), F, dtype, out,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "spectra_lowp");
  return SRP_OK;
}

static srp_status check_map_args(const srp_geometry_t* g, const void* in, int32_t F,
                                 int32_t dtype, float* map, srp_peak* peaks) {
  if (g == nullptr || in == nullptr) return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (map == nullptr && peaks == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "map and peaks are both NULL");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (dtype != SRP_FP32 && dtype != SRP_BF16 && dtype != SRP_FP16 && dtype != SRP_FP64)
    return fail(SRP_ERR_INVALID_ARG, "unknown dtype");
  return SRP_OK;
}

srp_status srp_map_nyquist(const srp_geometry_t* g, const void* xi, int32_t F, int32_t dtype,
                           float* map, srp_peak* peaks, void* stream) {
  srp_status st = check_map_args(g, xi, F, dtype, map, peaks);
  if (st != SRP_OK) return st;
  if ((dtype == SRP_BF16 || dtype == SRP_FP16) && !mx2_supported(g))
    return fail(SRP_ERR_UNSUPPORTED, "BF16/FP16 maps need fewer than 2^23 sample columns");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (peaks) e = launch_peaks_init(peaks, F, s);
  if (e == hipSuccess)
    e = launch_nyquist(g, xi, F, dtype, map, reinterpret_cast<unsigned long long*>(peaks), s);
  if (e == hipSuccess && peaks) e = launch_peaks_finalize(peaks, F, s);
  if (e != hipSuccess) return device_fail(e, "map_nyquist");
  return SRP_OK;
}

srp_status srp_nyquist_weights_bytes(const srp_geometry_t* g, int32_t dtype, size_t* bytes) {
  if (g == nullptr || bytes == nullptr) return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (dtype != SRP_BF16 && dtype != SRP_FP16)
    return fail(SRP_ERR_UNSUPPORTED, "cached weights are BF16 or FP16");
  *bytes = (size_t)g->info.J * (size_t)cached_weight_cols(g) * 2;
  return SRP_OK;
}

srp_status srp_nyquist_weights(const srp_geometry_t* g, int32_t dtype, void* weights,
                               size_t bytes, void* stream) {
  size_t need = 0;
  srp_status st = srp_nyquist_weights_bytes(g, dtype, &need);
  if (st != SRP_OK) return st;
  if (weights == nullptr) return fail(SRP_ERR_INVALID_ARG, "weights is NULL");
  if (bytes < need) return fail(SRP_ERR_INVALID_ARG, "weights buffer too small");
  if ((reinterpret_cast<uintptr_t>(weights) & 15) != 0)
    return fail(SRP_ERR_INVALID_ARG, "weights must be 16-byte aligned");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipError_t e = launch_nyquist_weights(g, dtype, weights, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "nyquist_weights");
  return SRP_OK;
}

srp_status srp_map_nyquist_cached(const srp_geometry_t* g, const void* weights, const void* xi,
                                  int32_t F, int32_t dtype, float* map, srp_peak* peaks,
                                  void* stream) {
  srp_status st = check_map_args(g, xi, F, dtype, map, peaks);
  if (st != SRP_OK) return st;
  if (dtype != SRP_BF16 && dtype != SRP_FP16)
    return fail(SRP_ERR_UNSUPPORTED, "cached weights are BF16 or FP16");
  if (weights == nullptr) return fail(SRP_ERR_INVALID_ARG, "weights is NULL");
  if ((reinterpret_cast<uintptr_t>(weights) & 15) != 0 ||
      (reinterpret_cast<uintptr_t>(xi) & 15) != 0)
    return fail(SRP_ERR_INVALID_ARG, "weights and xi must be 16-byte aligned");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (peaks) e = launch_peaks_init(peaks, F, s);
  if (e == hipSuccess)
    e = launch_nyquist_cached(g, weights, xi, F, dtype, map,
                              reinterpret_cast<unsigned long long*>(peaks), s);
  if (e == hipSuccess && peaks) e = launch_peaks_finalize(peaks, F, s);
  if (e != hipSuccess) return device_fail(e, "map_nyquist_cached");
  return SRP_OK;
}

srp_status srp_map_nyquist_points(const srp_geometry_t* g, const float* xi, int32_t F,
                                  const double* points, int32_t Q, float* values, void* stream) {
  if (g == nullptr || xi == nullptr || points == nullptr || values == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (F < 1 || F > 65535) return fail(SRP_ERR_INVALID_ARG, "F must be in [1, 65535]");
  if (Q < 1) return fail(SRP_ERR_INVALID_ARG, "Q must be >= 1");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipError_t e = launch_points(g, xi, F, points, Q, values, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "map_nyquist_points");
  return SRP_OK;
}

srp_status srp_map_conventional(const srp_geometry_t* g, const float* psi, int32_t F,
                                int32_t dtype, float* map, srp_peak* peaks, void* stream) {
  srp_status st = check_map_args(g, psi, F, dtype, map, peaks);
  if (st != SRP_OK) return st;
  // every dtype without a kernel is refused here, before the peaks are
  // initialised, so an unsupported call writes nothing
  if (!conventional_supports(dtype))
    return fail(SRP_ERR_UNSUPPORTED, "srp_map_conventional: dtype not supported");
  if ((dtype == SRP_BF16 || dtype == SRP_FP16) && !conv_mx_supported(g))
    return fail(SRP_ERR_UNSUPPORTED, "BF16/FP16 conventional maps need 256 x 4 P Kp < 2^32 bytes");
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the geometry's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (peaks) e = launch_peaks_init(peaks, F, s);
  if (e == hipSuccess) {
    if (dtype == SRP_BF16 || dtype == SRP_FP16)
      e = launch_conventional_mx(g, psi, F, dtype, map,
                                 reinterpret_cast<unsigned long long*>(peaks), s);
    else
      e = launch_conventional(g, reinterpret_cast<const float2*>(psi), F, dtype, map,
                              reinterpret_cast<unsigned long long*>(peaks), s);
  }
  if (e == hipSuccess && peaks) e = launch_peaks_finalize(peaks, F, s);
  if (e != hipSuccess) return device_fail(e, "map_conventional");
  return SRP_OK;
}

srp_status srp_map_nyquist_batched_workspace(int32_t n_items, size_t* bytes) {
  if (bytes == nullptr || n_items < 1) return fail(SRP_ERR_INVALID_ARG, "n_items must be >= 1");
  *bytes = (size_t)n_items * sizeof(BatchItemDev);
  return SRP_OK;
}

srp_status srp_map_nyquist_batched(const srp_batch_item* items, int32_t n_items, const void* xi,
                                   int64_t xi_elems, int32_t dtype, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  if (items == nullptr || xi == nullptr || workspace == nullptr)
    return fail(SRP_ERR_INVALID_ARG, "srp_map_nyquist_batched: NULL argument");
  if (n_items < 1) return fail(SRP_ERR_INVALID_ARG, "n_items must be >= 1");
  if (xi_elems < 1) return fail(SRP_ERR_INVALID_ARG, "xi_elems must be >= 1");
  if (dtype != SRP_FP32 && dtype != SRP_BF16 && dtype != SRP_FP16)
    return fail(SRP_ERR_UNSUPPORTED, "batched samples must be FP32, BF16 or FP16");
  const bool mx = dtype != SRP_FP32;
  const int max_frames = mx ? kBatchMaxFMx : kBatchMaxF;
  if (mx && (reinterpret_cast<uintptr_t>(xi) & 15) != 0)
    return fail(SRP_ERR_INVALID_ARG, "BF16/FP16 sample arena must be 16-byte aligned");
  if (workspace_bytes < (size_t)n_items * sizeof(BatchItemDev))
    return fail(SRP_ERR_INVALID_ARG, "workspace too small");
  // vector-unit items first, then matrix-core items; block_begin per group
  std::vector<BatchItemDev> dev;
  dev.reserve(n_items);
  int64_t blocks[2] = {0, 0};
  int n_group[2] = {0, 0};
  int max_f_vec = 1;
  int device = -1;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = 0; i < n_items; ++i) {
      const srp_batch_item& it = items[i];
      if (pass == 0) {
        if (it.g == nullptr) return fail(SRP_ERR_INVALID_ARG, "item geometry is NULL");
        if (it.F < 1 || it.F > max_frames)
          return fail(SRP_ERR_INVALID_ARG,
                      mx ? "item F must be in [1, 16]" : "item F must be in [1, 8]");
        if (it.map == nullptr && it.peaks == nullptr)
          return fail(SRP_ERR_INVALID_ARG, "item map and peaks are both NULL");
        if (it.xi_offset < 0) return fail(SRP_ERR_INVALID_ARG, "negative xi_offset");
        // the item's F x S samples must lie inside the arena
        if (it.xi_offset > xi_elems ||
            (int64_t)it.F * it.g->info.S > xi_elems - it.xi_offset)
          return fail(SRP_ERR_INVALID_ARG, "item samples extend past the end of xi");
        if (mx && it.xi_offset % kSampleAlign != 0)
          return fail(SRP_ERR_INVALID_ARG, "BF16/FP16 xi_offset must be a multiple of 8");
        if (device >= 0 && it.g->device != device)
          return fail(SRP_ERR_INVALID_ARG, "items on different devices");
        device = it.g->device;
      }
      const int grp = (mx && it.F > kBatchVecMaxF) ? 1 : 0;
      if (grp != pass) continue;
      BatchItemDev d;
      d.cand = it.g->d_cand;
      d.mic = it.g->d_mic;
      d.pairs = it.g->d_pairs;
      d.J = it.g->info.J;
      d.xi_off = it.xi_offset;
      d.S = static_cast<int>(it.g->info.S);
      d.P = it.g->info.P;
      d.F = it.F;
      d.far_field = it.g->info.field == SRP_FAR_FIELD;
      d.inv_cT = it.g->inv_cT;
      d.map = it.map;
      d.keys = reinterpret_cast<unsigned long long*>(it.peaks);
      d.block_begin = static_cast<int>(blocks[grp]);
      // BF16/FP16 items: the grid 2^-e of the TDOA fractions on which every
      // sinc denominator (|d| < 2 h_max + 64) is a float32 number
      d.xq_exp = 0;
      if (mx) {
        int hmax = 0;
        for (const PairDesc& pd : it.g->pairs) hmax = pd.h > hmax ? pd.h : hmax;
        int bits = 0;
        while ((int64_t(1) << bits) <= 2 * int64_t(hmax) + 64) ++bits;
        d.xq_exp = 24 - bits;
        if (d.xq_exp < 8) return fail(SRP_ERR_UNSUPPORTED, "pair windows too long for BF16/FP16 batches");
      }
      dev.push_back(d);
      blocks[grp] += (d.J + 255) / 256;
      ++n_group[grp];
      if (grp == 0) max_f_vec = it.F > max_f_vec ? it.F : max_f_vec;
    }
  }
  if (blocks[0] >= (int64_t(1) << 31) || blocks[1] >= (int64_t(1) << 31))
    return fail(SRP_ERR_INVALID_ARG, "batch too large");
  DeviceGuard dg(device);
  if (!dg.ok) return fail(SRP_ERR_DEVICE, "cannot select the items' device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // pageable source: the runtime stages it before returning, so `dev` may go
  hipError_t e = hipMemcpyAsync(workspace, dev.data(), dev.size() * sizeof(BatchItemDev),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_nyquist_batched(static_cast<const BatchItemDev*>(workspace), n_group[0],
                               static_cast<int>(blocks[0]), max_f_vec, n_group[1],
                               static_cast<int>(blocks[1]), dtype, xi, s);
  if (e != hipSuccess) return device_fail(e, "map_nyquist_batched");
  return SRP_OK;
}

srp_status srp_argmax(const float* map, int32_t F, int64_t J, srp_peak* peaks, void* stream) {
  if (map == nullptr || peaks == nullptr) return fail(SRP_ERR_INVALID_ARG, "NULL argument");
  if (F < 1) return fail(SRP_ERR_INVALID_ARG, "F must be >= 1");
  if (J < 1 || J >= (int64_t(1) << 31)) return fail(SRP_ERR_INVALID_ARG, "J must be in [1, 2^31)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_peaks_init(peaks, F, s);
  if (e == hipSuccess)
    e = launch_argmax(map, F, J, reinterpret_cast<unsigned long long*>(peaks), s);
  if (e == hipSuccess) e = launch_peaks_finalize(peaks, F, s);
  if (e != hipSuccess) return device_fail(e, "argmax");
  return SRP_OK;
}

}  // extern "C"
