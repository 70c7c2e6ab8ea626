// Building blocks of the streaming 5x5 median (Sec. III "Median and
// Gaussian Blur": the middle of the 25 window values) that sorts rows first:
// each row's 5-wide window is sorted across neighbouring columns, then the
// five sorted row windows of an output are merged down the rows, where
// outputs in consecutive rows share most of the work (a pair merge and the
// middle ranks of four rows).
//
// Keys are the bit patterns of non-negative floats (+0, positive finite,
// +inf) read as int32: their integer order is the float order, so the
// three-input median below may compare them as floats.  Host-compilable
// (a CPU test checks every block against a sort).
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define IPB_MR_HD __host__ __device__ __forceinline__
#else
#define IPB_MR_HD inline
#endif

namespace ipb {
namespace mr {

IPB_MR_HD int kmin(int a, int b) { return a < b ? a : b; }
IPB_MR_HD int kmax(int a, int b) { return a < b ? b : a; }
IPB_MR_HD float kf(int k) {
  union { int i; float f; } u;
  u.i = k;
  return u.f;
}
IPB_MR_HD int fk(float f) {
  union { float f; int i; } u;
  u.f = f;
  return u.i;
}
// the middle of three keys (one v_med3 on the device)
IPB_MR_HD int kmed3(int a, int b, int c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return fk(__builtin_amdgcn_fmed3f(kf(a), kf(b), kf(c)));
#else
  return kmax(kmin(a, b), kmin(kmax(a, b), c));
#endif
}

// Sorted union of two sorted pairs (p0 <= p1, q0 <= q1): 6 operations.
IPB_MR_HD void merge2_2(int p0, int p1, int q0, int q1, int* s) {
  s[0] = kmin(p0, q0);
  s[3] = kmax(p1, q1);
  s[1] = kmed3(p0, q0, kmin(p1, q1));
  s[2] = kmed3(p1, q1, kmax(p0, q0));
}

// Sorted union of a sorted 4-list and one value: 5 operations.
IPB_MR_HD void insert4(const int* s, int x, int* o) {
  o[0] = kmin(s[0], x);
  o[1] = kmed3(s[0], x, s[1]);
  o[2] = kmed3(s[1], x, s[2]);
  o[3] = kmed3(s[2], x, s[3]);
  o[4] = kmax(s[3], x);
}

// Sorted 5-wide windows of one row at two neighbouring columns a and a + 1
// from the values of columns a - 2 .. a + 3 (c[0] .. c[5]): the four middle
// columns are sorted once (two pairs, merged) and each window adds its outer
// column.
IPB_MR_HD void row_windows(const int* c, int* wa, int* wb) {
  int s[4];
  merge2_2(kmin(c[1], c[2]), kmax(c[1], c[2]), kmin(c[3], c[4]), kmax(c[3], c[4]), s);
  insert4(s, c[0], wa);
  insert4(s, c[5], wb);
}

// The median of 25 values given ranks 7..12 (c, sorted) of 20 of them and
// the other 5 (e, sorted): rank 5 of the 11, as the least over the splits
// of the largest of their two parts (5 max, then the min of six): 8
// operations with three-input mins.
IPB_MR_HD int median_of_core(const int* c, const int* e) {
  const int t0 = kmax(c[0], e[4]), t1 = kmax(c[1], e[3]), t2 = kmax(c[2], e[2]);
  const int t3 = kmax(c[3], e[1]), t4 = kmax(c[4], e[0]);
  return kmin(kmin(kmin(t0, t1), t2), kmin(kmin(t3, t4), c[5]));
}

}  // namespace mr
}  // namespace ipb
