// Launch splitting shared by the Nyquist map kernels (host side). Both work
// on an argument struct with the fields F, f_base, j_base and J.
#pragma once

#include <cstdint>
#include <type_traits>

#include "srp_internal.h"

namespace srp {

// Frame blocks of FTMAX 32-frame tiles, then (if F is not a multiple of the
// block) one more launch whose single block has just enough tiles for the
// remaining frames, so no matrix-core work is spent on frames past F.
template <int FTMAX, typename Args, typename Launch>
void launch_frame_blocks(int F, const Args& a, Launch&& launch) {
  constexpr int FB = 32 * FTMAX;
  const int full = F / FB;
  const int rem = F - full * FB;
  const int tiles = (rem + 31) / 32;  // 0 .. FTMAX (FTMAX <= 8)
  // a remainder that needs every tile anyway is one more block of the launch
  const int blocks = full + (tiles == FTMAX ? 1 : 0);
  if (blocks > 0) {
    Args b = a;
    b.f_base = 0;
    launch(std::integral_constant<int, FTMAX>(), b, blocks);
  }
  if (tiles == 0 || tiles == FTMAX) return;
  Args b = a;
  b.f_base = full * FB;
  static_assert(FTMAX <= 8, "tail dispatch covers up to 8 tiles");
  switch (tiles) {
    case 1: launch(std::integral_constant<int, 1>(), b, 1); break;
    case 2: launch(std::integral_constant<int, 2>(), b, 1); break;
    case 3: launch(std::integral_constant<int, (3 < FTMAX ? 3 : FTMAX)>(), b, 1); break;
    case 4: launch(std::integral_constant<int, (4 < FTMAX ? 4 : FTMAX)>(), b, 1); break;
    case 5: launch(std::integral_constant<int, (5 < FTMAX ? 5 : FTMAX)>(), b, 1); break;
    case 6: launch(std::integral_constant<int, (6 < FTMAX ? 6 : FTMAX)>(), b, 1); break;
    case 7: launch(std::integral_constant<int, (7 < FTMAX ? 7 : FTMAX)>(), b, 1); break;
    default: launch(std::integral_constant<int, FTMAX>(), b, 1); break;
  }
}

// Launches of a kernel with 256-candidate blocks, per_cu workgroups per CU at
// a time (as their LDS and registers allow) and all of about the same
// duration. When the workgroups do not fill a whole number of rounds of the
// CUs, the last round would leave CUs idle for a whole workgroup's time. So
// the candidate blocks that fill whole rounds run first (frame blocks of up to
// 8 tiles), and the rest run in one launch with the shortest frame blocks of
// which one round holds them all, if those are shorter than the first
// launch's (their last frame block carries padding rows rather than becoming
// a launch of its own, which would be another round). launch(ft, args, grid)
// launches the kernel instance with ft 32-frame tiles per block.
template <typename Args, typename Launch>
void launch_in_rounds(const srp_geometry_s* g, int F, const Args& a, int per_cu,
                      Launch&& launch) {
  constexpr int JB = 256;
  const int64_t round = (int64_t)g->n_cu * per_cu;
  const int64_t n_cb = (a.J + JB - 1) / JB;
  const int64_t n_fb = (F + 255) / 256;
  const int64_t full_cb = (n_cb * n_fb) / round * round / n_fb;
  const int64_t rest_cb = n_cb - full_cb;
  const int ft_main = (F + 31) / 32 < 8 ? (F + 31) / 32 : 8;  // tiles of the first launch's blocks
  auto rest_fb = [&](int ft) { return (F + 32 * ft - 1) / (32 * ft); };
  int ft_rest = 0;
  for (int ft = 1; ft < ft_main && ft_rest == 0; ++ft)
    if (rest_cb * rest_fb(ft) <= round) ft_rest = ft;
  const bool split = full_cb > 0 && rest_cb > 0 && ft_rest > 0;
  const unsigned gx = static_cast<unsigned>(split ? full_cb : n_cb);
  launch_frame_blocks<8>(F, a, [&](auto ft, const Args& b, int fblocks) {
    launch(ft, b, dim3(gx, fblocks));
  });
  if (!split) return;
  Args b = a;
  b.j_base = full_cb * JB;
  const dim3 grid(static_cast<unsigned>(rest_cb), static_cast<unsigned>(rest_fb(ft_rest)));
  switch (ft_rest) {
    case 1: launch(std::integral_constant<int, 1>(), b, grid); break;
    case 2: launch(std::integral_constant<int, 2>(), b, grid); break;
    case 3: launch(std::integral_constant<int, 3>(), b, grid); break;
    case 4: launch(std::integral_constant<int, 4>(), b, grid); break;
    case 5: launch(std::integral_constant<int, 5>(), b, grid); break;
    case 6: launch(std::integral_constant<int, 6>(), b, grid); break;
    default: launch(std::integral_constant<int, 7>(), b, grid); break;
  }
}

}  // namespace srp
