// Size limit and 32-bit byte offsets of a frame's maps, shared by the host
// argument checks and the kernels (no HIP include, so that a CPU test can
// compile it with g++ and check the arithmetic at the limit).
//
// The kernels address a map with 32-bit byte offsets from its base: cell
// (y, x) of an H x W map is at 4 (y W + x).  The streaming phase-1 kernel
// also stores the values of its idle lanes to a scratch slot just past the
// map, at byte offset 4 H W.  Both fit in 32 bits iff H W < 2^30, which is
// therefore the largest frame the library accepts.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define IPB_OFF_HD __host__ __device__ __forceinline__
#else
#define IPB_OFF_HD inline
#endif

namespace ipb {

constexpr long long kMaxCells = (1LL << 30) - 1;   // largest accepted H * W

IPB_OFF_HD bool cells_ok(int H, int W) {
  return H >= 1 && W >= 1 && static_cast<long long>(H) * W <= kMaxCells;
}

// byte offset of cell (y, x) (0 <= y < H, 0 <= x < W)
IPB_OFF_HD unsigned cell_offset(int y, int x, int W) {
  return 4u * ((unsigned)y * (unsigned)W + (unsigned)x);
}

// byte offset of the scratch slot past the map (the map is followed by at
// least 256 bytes of workspace)
IPB_OFF_HD unsigned sink_offset(int H, int W) { return 4u * ((unsigned)H * (unsigned)W); }

}  // namespace ipb
