// Nyquist SRP at arbitrary per-frame points (Eq. SRPapprox summed over pairs
// as in Eq. SRP_T_IFT). The interpolation gives the map as a continuous
// function of the candidate position, so one set of GCC samples also serves
// points off the candidate grid, e.g. a finer local grid around a coarse
// peak (the refined search the paper names as a possible extension).
//
// One thread per (frame, point): the thread forms the point's TDOA for every
// pair in float64, splits it into an integer and a float32 fraction, and sums
// the pair's window of float32 samples of its own frame with the sinc weights
// formed as in the other kernels (two weights per reciprocal); each pair's sum
// is added to the total separately (two-level float32 sum). The samples of a
// frame are read by all threads of that frame's points: a workgroup covers
// 256 points of one frame, so its sample reads are uniform (scalar loads).
#include "srp_device.h"
#include "srp_internal.h"

namespace srp {
namespace {

__global__ __launch_bounds__(256) void points_kernel(
    const float* __restrict__ xi, int S, const double* __restrict__ mic,
    const PairDesc* __restrict__ pairs, int P, const double* __restrict__ pts, int Q,
    int far_field, double inv_cT, float* __restrict__ out) {
  const int f = blockIdx.y;
  const int q0 = blockIdx.x * 256 + threadIdx.x;
  const int q = q0 < Q ? q0 : Q - 1;
  const double* pt = pts + ((size_t)f * Q + q) * 3;
  const double qx = pt[0], qy = pt[1], qz = pt[2];
  const float* row = xi + (size_t)f * S;
  float tot = 0.0f;
  int cur_m = -1;
  double rm = 0.0;
  for (int p = 0; p < P; ++p) {
    const PairDesc pdv = pairs[p];
    PairDesc pd;
    pd.m = __builtin_amdgcn_readfirstlane(pdv.m);
    pd.mp = __builtin_amdgcn_readfirstlane(pdv.mp);
    pd.h = __builtin_amdgcn_readfirstlane(pdv.h);
    pd.off = __builtin_amdgcn_readfirstlane(pdv.off);
    const double* pm = mic + 3 * pd.m;
    const double* pn = mic + 3 * pd.mp;
    double x;
    if (far_field) {
      x = ((pm[0] - pn[0]) * qx + (pm[1] - pn[1]) * qy + (pm[2] - pn[2]) * qz) * inv_cT;
    } else {
      if (pd.m != cur_m) {
        rm = norm3(qx - pm[0], qy - pm[1], qz - pm[2]);
        cur_m = pd.m;
      }
      x = (rm - norm3(qx - pn[0], qy - pn[1], qz - pn[2])) * inv_cT;
    }
    const double r = rint(x);
    double fd = x - r;
    fd = fabs(fd) < 1e-30 ? 1e-30 : fd;
    const float xf = static_cast<float>(fd);
    const float sp = sinpi_over_pi(fd);
    // lag t = 0 .. 2h: x - n = (xr + h - t) + xf
    const int ia = static_cast<int>(r) + pd.h;
    const float q0s = (ia & 1) ? -sp : sp;
    const float* col = row + pd.off;
    const int W = 2 * pd.h + 1;
    float base = static_cast<float>(ia);
    float acc = 0.0f;
    int t = 0;
#pragma unroll 4
    for (; t + 1 < W; t += 2, base -= 2.0f) {
      const float d0 = base + xf;
      const float d1 = (base - 1.0f) + xf;
      const float qr = q0s * __builtin_amdgcn_rcpf(d0 * d1);
      acc = fmaf(qr * d1, col[t], acc);
      acc = fmaf(-qr * d0, col[t + 1], acc);
    }
    acc = fmaf(q0s * __builtin_amdgcn_rcpf(base + xf), col[t], acc);  // last lag (W is odd)
    tot += acc;
  }
  if (q0 < Q) out[(size_t)f * Q + q0] = 2.0f * tot;
}

}  // namespace

hipError_t launch_points(const srp_geometry_s* g, const float* xi, int F, const double* pts,
                         int Q, float* out, hipStream_t s) {
  const dim3 grid((Q + 255) / 256, F);
  hipLaunchKernelGGL(points_kernel, grid, dim3(256), 0, s, xi, static_cast<int>(g->info.S),
                     g->d_mic, g->d_pairs, g->info.P, pts, Q,
                     g->info.field == SRP_FAR_FIELD, g->inv_cT, out);
  return hipGetLastError();
}

}  // namespace srp
