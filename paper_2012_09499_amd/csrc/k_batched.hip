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
// Workgroup b belongs to the item whose [block_begin, block_begin + blocks)
// range contains b (binary search over the item table).
#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

template <int FMAX>
__global__ __launch_bounds__(256) void nyquist_batched_kernel(const BatchItemDev* __restrict__ items,
                                                               int n_items,
                                                               const float* __restrict__ xi) {
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
    fd = fabs(fd) < 1e-30 ? 1e-30 : fd;
    const float xf = static_cast<float>(fd);
    const float sp = sinpi_over_pi(fd);
    // lag t = 0 .. 2h: n = t - h, x - n = (xr + h - t) + xf
    const int ia = static_cast<int>(r) + pd.h;
    const float q0 = (ia & 1) ? -sp : sp;  // (-1)^(xr - n) sin(pi xf)/pi at t = 0
    float acc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; ++f) acc[f] = 0.0f;
    const float* col = xi + it.xi_off + pd.off;
    const int W = 2 * pd.h + 1;
    float base = static_cast<float>(ia);
    int t = 0;
#pragma unroll 4
    for (; t + 1 < W; t += 2, base -= 2.0f) {
      const float d0 = base + xf;
      const float d1 = (base - 1.0f) + xf;
      const float qr = q0 * __builtin_amdgcn_rcpf(d0 * d1);
      const float w0 = qr * d1;
      const float w1 = -qr * d0;
#pragma unroll
      for (int f = 0; f < FMAX; ++f) {
        if (f < it.F) {
          acc[f] = fmaf(w0, col[(size_t)f * it.S + t], acc[f]);
          acc[f] = fmaf(w1, col[(size_t)f * it.S + t + 1], acc[f]);
        }
      }
    }
    {  // last lag (W is odd)
      const float w0 = q0 * __builtin_amdgcn_rcpf(base + xf);
#pragma unroll
      for (int f = 0; f < FMAX; ++f)
        if (f < it.F) acc[f] = fmaf(w0, col[(size_t)f * it.S + t], acc[f]);
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

hipError_t launch_nyquist_batched(const BatchItemDev* d_items, int n_items, int total_blocks,
                                  int max_f, const float* xi, hipStream_t s) {
  hipLaunchKernelGGL(batch_peaks_kernel, dim3(n_items), dim3(kBatchMaxF), 0, s, d_items, 0);
  if (max_f <= 1)
    hipLaunchKernelGGL(nyquist_batched_kernel<1>, dim3(total_blocks), dim3(256), 0, s, d_items,
                       n_items, xi);
  else if (max_f <= 2)
    hipLaunchKernelGGL(nyquist_batched_kernel<2>, dim3(total_blocks), dim3(256), 0, s, d_items,
                       n_items, xi);
  else if (max_f <= 4)
    hipLaunchKernelGGL(nyquist_batched_kernel<4>, dim3(total_blocks), dim3(256), 0, s, d_items,
                       n_items, xi);
  else
    hipLaunchKernelGGL(nyquist_batched_kernel<kBatchMaxF>, dim3(total_blocks), dim3(256), 0, s,
                       d_items, n_items, xi);
  hipLaunchKernelGGL(batch_peaks_kernel, dim3(n_items), dim3(kBatchMaxF), 0, s, d_items, 1);
  return hipGetLastError();
}

}  // namespace srp
