/*
 * srp.h - C ABI of libsrp: steered response power (SRP) maps on one AMD
 * Instinct MI355X (gfx950), conventional and with the Nyquist-Shannon
 * approximation of Dietzen, De Sena and van Waterschoot, "Low-Complexity
 * Steered Response Power Mapping based on Nyquist-Shannon Sampling"
 * (WASPAA 2021).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers are DEVICE pointers unless marked "host". Device buffers are
 *   owned by the caller, contiguous, and 16-byte aligned; the library never
 *   frees them.
 * - `stream` is a hipStream_t (NULL = the default stream). Every call that
 *   takes a stream validates its arguments on the host, then enqueues its
 *   kernels on that stream and returns before they finish. An invalid
 *   argument returns SRP_ERR_INVALID_ARG with nothing enqueued and no output
 *   written. A failed launch returns SRP_ERR_DEVICE. No call aborts the
 *   process or throws; srp_last_error() gives the message of the last failing
 *   call on the calling thread.
 * - Microphones are 0-based. Pair p of microphones (m, m') with m > m' has
 *   index p = m(m-1)/2 + m' (the pair set of Section 2.1); P = M(M-1)/2.
 * - Frequency bins: f_k = k fs / L for k = 0 .. K-1, K = floor(f_max L / fs) + 1.
 *   Bin weights w_k = 1 at k = 0 and at f_k = fs/2, 2 elsewhere: the
 *   one-sided sum that stands for the integral over [-omega_0, omega_0]
 *   (Eq. SRP_T).
 * - Discrete GCC: xi_p(tau) = sum_k w_k Re[psi_p(k) exp(j 2 pi f_k tau)]
 *   (Eq. GCC_IFT with the integral replaced by a sum, Section 2.4).
 * - Critical period T = 1 / (2 f_max) (Section 3.1). Per-pair window
 *   half-width h_p = N_p + N_aux with N_p = floor(d_p / (c T)) evaluated in
 *   float64 exactly in that order, d_p = ||p_m - p_m'||; the window holds
 *   W_p = 2 h_p + 1 lags n = -h_p .. h_p (Eq. SRPapprox, Section 3.3).
 * - GCC-sample layout: sample (p, n) of a frame sits at column
 *   offset_p + (n + h_p); offset_0 = 0 and offset_{p+1} = offset_p + W_p
 *   rounded up to a multiple of 8 (the up to 7 columns after each window are
 *   zeros), S = offset_P. Windows start at multiples of 8 samples so that
 *   16-byte copies of bf16/fp16 samples stay aligned.
 */
#ifndef SRP_H
#define SRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SRP_OK = 0,
  SRP_ERR_INVALID_ARG = -1,
  SRP_ERR_OUT_OF_MEMORY = -2,
  SRP_ERR_DEVICE = -3,
  SRP_ERR_UNSUPPORTED = -4
} srp_status;

/* Arithmetic type of a map or sample kernel's contraction. Accumulation is
 * float32 for SRP_FP32/SRP_BF16/SRP_FP16 (matrix cores) and float64 for
 * SRP_FP64 (vector units; a slow exactness check, not a fast path). */
typedef enum { SRP_FP32 = 0, SRP_BF16 = 1, SRP_FP16 = 2, SRP_FP64 = 3 } srp_dtype;

/* Propagation model: near field (Eq. Deltat_i, candidates are points in
 * metres) or far field (Eq. Deltat_i_spher, candidates are unit incident
 * directions r pointing from the source towards the array). */
typedef enum { SRP_NEAR_FIELD = 0, SRP_FAR_FIELD = 1 } srp_field;

/* Analysis window applied to every frame before its DFT: periodic Hann
 * 0.5 - 0.5 cos(2 pi t / L), its square root, or rectangular. */
typedef enum { SRP_WIN_HANN = 0, SRP_WIN_SQRT_HANN = 1, SRP_WIN_RECT = 2 } srp_window;

/* Weighting of the GCC matrix (Eq. corrmatrix). Only the phase transform. */
typedef enum { SRP_PHAT = 0 } srp_weighting;

/* Per-frame map maximum (Section 2.2: the location estimate is the argmax).
 * Ties go to the lowest candidate index. 16 bytes. */
typedef struct {
  int64_t index;
  float value;
  int32_t reserved;
} srp_peak;

/* Opaque, immutable array description. Owns device copies of the geometry
 * and the tables derived from it. May be used from several streams at once;
 * the caller keeps it alive until all work enqueued with it has finished. */
typedef struct srp_geometry_s srp_geometry_t;

/* Layout summary of a geometry handle (all host values). */
typedef struct {
  int32_t M, P, L, K;      /* mics, pairs, frame length, one-sided bins            */
  int64_t J;               /* candidates                                            */
  int64_t S;               /* GCC-sample columns per frame (layout above)           */
  int32_t h_max;           /* max_p h_p                                             */
  int32_t n_aux;
  int32_t field, window;
  double c, fs, f_max, T;  /* speed of sound, sample rate, band limit, period      */
} srp_geometry_info;

/* Host-only pair layout (Section 3.2, 3.3): computes h_p - n_aux = N_p for
 * every pair (into N_p, P entries, may be NULL), the sample-layout offsets
 * (P + 1 entries, may be NULL) and S (may be NULL). mic_xyz: host, M x 3 float64,
 * metres, row-major. Requires M >= 2, c > 0, f_max > 0, n_aux >= 0. Touches
 * no device. */
srp_status srp_pair_layout(const double* mic_xyz, int32_t M, double c, double f_max,
                           int32_t n_aux, int32_t* N_p, int64_t* offsets, int64_t* S);

/* Creates a geometry handle (Section 2.1: microphone positions p_m, candidate
 * locations q_i or directions r_i, speed of sound c, band limit omega_0).
 *   mic_xyz   host, M x 3 float64 (metres)
 *   cand_xyz  host, J x 3 float64: points (near field) or unit vectors (far field)
 *   f_max     band limit omega_0 / (2 pi), 0 < f_max <= fs / 2
 *   L         frame length, a power of two with 16 <= L <= 8192
 *   n_aux     auxiliary samples per side, >= 0
 * Invalid: M < 2 or M > 256, J < 1 or J >= 2^31, c <= 0, fs <= 0, bad L or
 * f_max, n_aux < 0, 2 h_p + 1 > L for some pair, a far-field direction whose
 * norm differs from 1 by more than 1e-9, a NULL pointer. Copies the tables to
 * the device on `stream` and waits for the copies before returning, so the
 * host arrays may be freed at once. The handle belongs to the device current
 * at this call; its compute-unit count and the occupancy of the interpolation
 * kernels are read here to size their launches. */
srp_status srp_geometry(const double* mic_xyz, int32_t M, const double* cand_xyz, int64_t J,
                        int32_t field, double c, double fs, int32_t L, double f_max,
                        int32_t n_aux, int32_t window, void* stream, srp_geometry_t** out);

/* Layout of a handle; N_p (P entries) and offsets (P + 1) are host and may be NULL. */
srp_status srp_geometry_query(const srp_geometry_t* g, srp_geometry_info* info, int32_t* N_p,
                              int64_t* offsets);

/* Frees the handle's device memory. The caller synchronises first. NULL is a no-op. */
void srp_geometry_destroy(srp_geometry_t* g);

/* Bytes of device workspace srp_cross_spectra and srp_gcc_samples_frames need
 * for F frames: F * M * Kr * 8, Kr = K rounded up to a multiple of 16 (the
 * per-microphone unit phasors, one row of Kr bins per frame and microphone). */
srp_status srp_cross_spectra_workspace(const srp_geometry_t* g, int32_t F, size_t* bytes);

/* Frequency-domain GCC of every pair (Eq. corrmatrix with the PHAT weight):
 * windowed DFT of each frame and microphone, then
 * psi_p(k) = y_m y_m'^* / |y_m y_m'^*|, with psi_p(k) = 0 where y_m or y_m' is 0.
 *   frames     device, F x M x L float32
 *   workspace  device, >= srp_cross_spectra_workspace bytes (overwritten)
 *   psi        device, F x P x K complex (interleaved float32 re, im), written
 * F >= 1. */
srp_status srp_cross_spectra(const srp_geometry_t* g, const float* frames, int32_t F,
                             int32_t weighting, void* workspace, size_t workspace_bytes,
                             float* psi, void* stream);

/* srp_cross_spectra without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc). The
 * per-microphone unit phasors are staged in a buffer the library owns: one
 * static device array of 64 MiB per GPU, present from the library's load
 * until the process ends, its address looked up once per device at the first
 * call there. Same arguments, result and errors as srp_cross_spectra, except:
 *   F * M * Kr * 8 bytes (Kr = K rounded up to a multiple of 16) must not
 *   exceed 64 MiB, else SRP_ERR_INVALID_ARG with nothing enqueued (e.g.
 *   F <= 992 for 16 mics and K = 513, Kr = 528).
 * Every call on a GPU shares that GPU's buffer: calls that overlap on one GPU
 * (several streams or threads at once) race and must be serialised by the
 * caller. The call itself allocates nothing. */
srp_status srp_cross_spectra_noalloc(const srp_geometry_t* g, const float* frames, int32_t F,
                                     int32_t weighting, float* psi, void* stream);

/* GCC samples at the critical lags (Section 3.2, first step; cost Eq.
 * SRPapproxcompC): xi[f][offset_p + n + h_p] = xi_p(n T) for |n| <= h_p.
 *   psi    device, F x P x K complex64 as written by srp_cross_spectra
 *   dtype  storage type of xi: SRP_FP32 (float), SRP_BF16 (bfloat16) or
 *          SRP_FP16 (IEEE half). The sum is accumulated in float32 and rounded
 *          once to the storage type.
 *   xi     device, F x S elements of that type, written */
srp_status srp_gcc_samples(const srp_geometry_t* g, const float* psi, int32_t F, int32_t dtype,
                           void* xi, void* stream);

/* Frames to GCC samples in one call (Section 2.1, Eq. corrmatrix with the PHAT
 * weight, then Section 3.2, first step): the same samples as srp_cross_spectra
 * followed by srp_gcc_samples, with psi_p(k) = ytil_m(k) ytil_m'(k)^* formed
 * on chip from the per-microphone unit phasors ytil = y / |y| instead of being
 * written to memory (F P K complex values fewer in memory traffic each way).
 *   frames     device, F x M x L float32
 *   weighting  SRP_PHAT
 *   dtype      storage type of xi: SRP_FP32, SRP_BF16 or SRP_FP16 (float32
 *              accumulation, rounded once)
 *   workspace  device, >= srp_cross_spectra_workspace bytes (overwritten)
 *   xi         device, F x S elements of that type, written (layout above)
 * F >= 1. The samples equal those of the two-call path up to float32 rounding
 * (the sums run in another order). */
srp_status srp_gcc_samples_frames(const srp_geometry_t* g, const float* frames, int32_t F,
                                  int32_t weighting, int32_t dtype, void* workspace,
                                  size_t workspace_bytes, void* xi, void* stream);

/* Input of the BF16/FP16 conventional map: the cross-spectra weighted by the
 * bin weights (Eq. SRP_T) and rounded once to the 16-bit type,
 * out[f][p][k] = (Re, Im) of w_k psi_p(k) for k < K and (0, 0) for
 * K <= k < Kp, Kp = K rounded up to a multiple of 8 (row-major, 2 values per
 * bin, 4 P Kp bytes per frame).
 *   srp_spectra_lowp_bytes  size for F frames; SRP_ERR_UNSUPPORTED for any
 *                           dtype other than SRP_BF16 / SRP_FP16
 *   psi                     device, F x P x K complex64 (srp_cross_spectra)
 *   out                     device, >= srp_spectra_lowp_bytes, 16-byte aligned */
srp_status srp_spectra_lowp_bytes(const srp_geometry_t* g, int32_t F, int32_t dtype,
                                  size_t* bytes);
srp_status srp_spectra_lowp(const srp_geometry_t* g, const float* psi, int32_t F, int32_t dtype,
                            void* out, size_t out_bytes, void* stream);

/* Conventional SRP map (Eq. SRP_T_IFT with one discrete IFT per candidate,
 * pair and bin, Section 2.4; cost Eq. SRPomp): map[f][i] = 2 sum_p xi_p(dt_p(i)).
 *   psi    device: for SRP_FP32 / SRP_FP64, F x P x K complex64 (srp_cross_spectra);
 *          for SRP_BF16 / SRP_FP16, the weighted rounded spectra of
 *          srp_spectra_lowp with the same dtype (16-byte aligned)
 *   map    device, F x J float32, written; may be NULL if peaks is not
 *   peaks  device, F srp_peak, written; may be NULL if map is not
 * dtype: SRP_FP32 (float32 matrix cores), SRP_BF16 / SRP_FP16 (matrix cores on
 * the 16-bit spectra and phasors of the bins, float32 accumulation; phases
 * from the float64 TDOA reduced mod 1 at every 32-bin run, rotated in float32
 * within it; SRP_ERR_UNSUPPORTED when 1024 P Kp >= 2^32) or SRP_FP64 (see
 * srp_dtype). Every refusal happens before anything is enqueued. */
srp_status srp_map_conventional(const srp_geometry_t* g, const float* psi, int32_t F,
                                int32_t dtype, float* map, srp_peak* peaks, void* stream);

/* Nyquist-Shannon SRP approximation (Eq. SRPapprox summed over pairs as in
 * Eq. SRP_T_IFT; cost Eq. SRPapproxcompR):
 * map[f][i] = 2 sum_p sum_{|n| <= h_p} xi_p(nT) sinc(dt_p(i) / T - n),
 * sinc(x) = sin(pi x) / (pi x), sinc(0) = 1. TDOAs are formed on the fly:
 * in float64 for SRP_FP32 and SRP_FP64, whose sinc weights take the float64
 * argument split into an integer and a float32 fraction; in float32 for
 * SRP_BF16 and SRP_FP16, from positions relative to the microphone centroid
 * (an error of about 2^-23 of the largest candidate-to-array distance times
 * 2 fs / c samples, below the rounding of their weights).
 *   xi     device, F x S samples in the srp_gcc_samples layout, stored as
 *          float for SRP_FP32 and SRP_FP64, bfloat16 for SRP_BF16, half for
 *          SRP_FP16 (srp_gcc_samples with the same dtype writes them); the gap
 *          columns after each window must hold zeros, as that layout states
 *          (the interpolation reads the first one with a weight, unmasked)
 *   dtype  SRP_FP32: float32 matrix cores; SRP_BF16 / SRP_FP16: weights and
 *          samples in that type on the matrix cores, float32 accumulation,
 *          the TDOA fraction rounded to a per-geometry grid of at most 2^-8
 *          (2^-16 at the room scale) on which every sinc denominator is exact
 *          (SRP_ERR_UNSUPPORTED, nothing enqueued, when S >= 2^23);
 *          SRP_FP64: float64 vector units (an exactness check, not a fast path)
 *   map    device, F x J float32, written; may be NULL if peaks is not
 *   peaks  device, F srp_peak, written; may be NULL if map is not */
srp_status srp_map_nyquist(const srp_geometry_t* g, const void* xi, int32_t F, int32_t dtype,
                           float* map, srp_peak* peaks, void* stream);

/* Cached interpolation weights (Section 3.3: the weights sinc(dt_p(i)/T - n)
 * of Eq. SRPapprox do not depend on the frames; cost of the map with them,
 * Eq. SRPapproxcompR). The weight matrix W is J x Sw, row-major (one row per
 * candidate), Sw = S rounded up to a multiple of 128, in the column layout of
 * the GCC samples: W[i][off_p + n + h_p] = sinc(dt_p(i)/T - n) for |n| <= h_p,
 * 0 in the gap columns and past S. Every entry is computed in float64 and
 * rounded once to bfloat16 (SRP_BF16) or half (SRP_FP16). The caller owns the
 * buffer (J * Sw * 2 bytes; e.g. 8.1 GB for 576,000 candidates and S = 7,008)
 * and decides whether the geometry is worth caching.
 *   srp_nyquist_weights_bytes  size of W for dtype; SRP_ERR_UNSUPPORTED for
 *                              any dtype other than SRP_BF16 / SRP_FP16
 *   srp_nyquist_weights        writes W (device, 16-byte aligned, >= bytes) */
srp_status srp_nyquist_weights_bytes(const srp_geometry_t* g, int32_t dtype, size_t* bytes);
srp_status srp_nyquist_weights(const srp_geometry_t* g, int32_t dtype, void* weights,
                               size_t bytes, void* stream);

/* Nyquist map from cached weights: map[f][i] = 2 sum_k W[i][k] xi[f][k] over
 * the packed columns (the same sum as srp_map_nyquist, Eq. SRPapprox summed
 * over pairs as in Eq. SRP_T_IFT, with the weights read instead of formed).
 *   weights  device, written by srp_nyquist_weights for this geometry and dtype
 *   xi       device, F x S samples written by srp_gcc_samples with this dtype
 *            (16-byte aligned)
 *   dtype    SRP_BF16 or SRP_FP16 (matrix cores, float32 accumulation)
 *   map, peaks as for srp_map_nyquist */
srp_status srp_map_nyquist_cached(const srp_geometry_t* g, const void* weights, const void* xi,
                                  int32_t F, int32_t dtype, float* map, srp_peak* peaks,
                                  void* stream);

/* Nyquist SRP at arbitrary points, different for every frame (Eq. SRPapprox
 * summed over pairs as in Eq. SRP_T_IFT): the interpolation defines the map
 * off the candidate grid too, so a coarse map's peak can be refined on finer
 * local grids from the same samples (the refined spatial search that Section 1
 * and Section 3.3 name as an extension; the package's refine_peaks does this).
 *   xi      device, F x S float32 samples (srp_gcc_samples, SRP_FP32)
 *   points  device, F x Q x 3 float64: positions in metres (near field) or
 *           unit propagation directions (far field; not checked), per frame
 *   values  device, F x Q float32, written: 2 sum_p xi_p,appr(dt_p(point))
 * float32 vector arithmetic with the float64 TDOA split of srp_map_nyquist;
 * 1 <= F <= 65535, Q >= 1. */
srp_status srp_map_nyquist_points(const srp_geometry_t* g, const float* xi, int32_t F,
                                  const double* points, int32_t Q, float* values, void* stream);

/* One item of a batched Nyquist launch: an array and its frames of the batch. */
typedef struct {
  const srp_geometry_t* g;   /* the array                                            */
  int64_t xi_offset;         /* index (in elements) of the item's first sample in xi; */
                             /* the item's samples are F x S (srp_gcc_samples layout) */
  int32_t F;                 /* frames of the item: 1..8 (SRP_FP32), 1..16 (BF16/FP16) */
  int32_t reserved;
  float* map;                /* device F x J float32, written; may be NULL if peaks is not */
  srp_peak* peaks;           /* device F, written; may be NULL if map is not         */
} srp_batch_item;

/* Bytes of device workspace srp_map_nyquist_batched needs for n_items items. */
srp_status srp_map_nyquist_batched_workspace(int32_t n_items, size_t* bytes);

/* Nyquist maps of many arrays in one ragged launch (Eq. SRPapprox summed over
 * pairs, Eq. SRP_T_IFT), for serving: arrays of different microphone counts,
 * windows and grids, each with a few frames. Same result definition as
 * srp_map_nyquist.
 *   items      host, n_items entries (read before the call returns)
 *   xi         device sample arena holding every item's samples, stored as
 *              float (SRP_FP32), bfloat16 (SRP_BF16) or half (SRP_FP16)
 *   xi_elems   number of elements of the arena; an item whose samples
 *              [xi_offset, xi_offset + F S) do not lie inside it is rejected
 *              with SRP_ERR_INVALID_ARG before anything is enqueued
 *   dtype      SRP_FP32: float32 on the vector units (with one to eight
 *              frames per array the weights are formed once per candidate and
 *              lag and used by those frames only), the accuracy of
 *              srp_map_nyquist in FP32;
 *              SRP_BF16 / SRP_FP16: items of one or two frames on the vector
 *              units, longer ones on the matrix cores (16 frames x 16
 *              candidates x 32 lags per instruction); weights in that type,
 *              float32 accumulation, the TDOA fraction rounded to a grid of at
 *              most 2^-8 (2^-16 for windows of up to 191 lags) on which every
 *              sinc denominator is exact; the accuracy of srp_map_nyquist in
 *              that type; the arena must be 16-byte aligned and every
 *              xi_offset a multiple of 8
 *   workspace  device, >= srp_map_nyquist_batched_workspace bytes; holds the
 *              item table until the launch has finished (do not reuse it for
 *              another batch on another stream before then)
 * All items must live on one device. */
srp_status srp_map_nyquist_batched(const srp_batch_item* items, int32_t n_items, const void* xi,
                                   int64_t xi_elems, int32_t dtype, void* workspace,
                                   size_t workspace_bytes, void* stream);

/* Per-frame argmax of a map (Section 2.2), lowest index on ties.
 *   map    device, F x J float32;  peaks device, F srp_peak, written.
 * F >= 1, 1 <= J < 2^31. */
srp_status srp_argmax(const float* map, int32_t F, int64_t J, srp_peak* peaks, void* stream);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char* srp_last_error(void);

/* Library version string. */
const char* srp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SRP_H */
