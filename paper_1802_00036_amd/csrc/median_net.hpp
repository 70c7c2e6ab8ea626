// Compile-time sorting network used for the median blur (Sec. III "Median
// and Gaussian Blur": the middle value of each window).
//
// Batcher's odd-even merge sort on the next power of two above N, with every
// comparator that touches a position >= N dropped.  Padding positions would
// hold +inf; a comparator puts its minimum at the lower index, so +inf never
// moves below N and those comparators are no-ops.  The caller reads one
// output (the middle); the compiler removes the min/max halves that do not
// feed it, which leaves a pruned selection network.
//
// Usable from host code too (the CPU test compiles it with g++).
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define IPB_HD __host__ __device__ __forceinline__
#else
#define IPB_HD inline
#endif

namespace ipb {
namespace net {

IPB_HD float fmin_(float a, float b) { return fminf(a, b); }
IPB_HD float fmax_(float a, float b) { return fmaxf(a, b); }

template <int N>
struct OddEven {
  template <int I, int J>
  static IPB_HD void cx(float* a) {
    if constexpr (J < N) {
      const float x = a[I], y = a[J];
      a[I] = fmin_(x, y);
      a[J] = fmax_(x, y);
    }
  }
  // comparators (i, i + R) for i = I, I + STEP, ... while i < END
  template <int I, int END, int STEP, int R>
  static IPB_HD void span(float* a) {
    if constexpr (I < END) {
      cx<I, I + R>(a);
      span<I + STEP, END, STEP, R>(a);
    }
  }
  // merge the sorted halves of a[LO..HI] (HI inclusive), elements R apart
  template <int LO, int HI, int R>
  static IPB_HD void merge(float* a) {
    constexpr int STEP = 2 * R;
    if constexpr (STEP < HI - LO) {
      merge<LO, HI, STEP>(a);
      merge<LO + R, HI, STEP>(a);
      span<LO + R, HI - R, STEP, R>(a);
    } else {
      cx<LO, LO + R>(a);
    }
  }
  template <int LO, int HI>
  static IPB_HD void sort(float* a) {
    if constexpr (HI - LO >= 1) {
      constexpr int MID = LO + (HI - LO) / 2;
      sort<LO, MID>(a);
      sort<MID + 1, HI>(a);
      merge<LO, HI, 1>(a);
    }
  }
};

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

// Sorts a[0..N) ascending in place (a must have pow2_at_least(N) slots; the
// slots >= N are never read or written).
template <int N>
IPB_HD void sort_network(float* a) {
  OddEven<N>::template sort<0, pow2_at_least(N) - 1>(a);
}

}  // namespace net
}  // namespace ipb
