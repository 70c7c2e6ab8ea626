// gfx950 kernels of the depth-completion chain (Ku, Harakeh & Waslander
// 2018, Sec. III "Proposed Algorithm").
//
// Border rules (fixed identically in the CPU oracle):
//   morphology (stages 2-4, 6): taps outside the image are ignored
//     (max: neutral 0, since every map value is >= +0; min: neutral +inf);
//   median (stage 7): replicated border (coordinates clamped);
//   Gaussian (stage 8): reflect-101 border.
// Arithmetic: stages 2-7 only select values; stage 1 and 9 are one rounded
// fp32 subtraction each; stage 8 sums in fp64 (exact for the binomial taps)
// and rounds once to fp32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "median_net.hpp"

#pragma clang fp contract(off)

namespace ipb {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// reflect-101 index (-1 -> 1, n -> n - 2; n == 1 -> 0)
__device__ __forceinline__ int refl101(int q, int n) {
  if (n == 1) return 0;
  const int period = 2 * n - 2;
  int m = q % period;
  if (m < 0) m += period;
  return m < n ? m : period - m;
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical tiles so that tiles sharing halos share an L2.
__device__ __forceinline__ int xcd_tile(int b, int g) {
  if ((g & 7) != 0) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

__device__ __forceinline__ const FrameDesc* plan_frames(const PlanHeader* p) {
  return reinterpret_cast<const FrameDesc*>(p + 1);
}

// Spread a rows x cols rectangle over the workgroup: each thread takes one
// column and a run of consecutive rows (lanes of a wave hold neighbouring
// columns of the same rows, so LDS reads are bank-conflict free and global
// accesses coalesce).
template <class F>
__device__ __forceinline__ void for_column_runs(int r0, int r1, int c0, int c1, F&& body) {
  const int ncols = c1 - c0, nrows = r1 - r0;
  if (ncols <= 0 || nrows <= 0) return;
  int nseg = kThreads / ncols;
  if (nseg < 1) nseg = 1;
  const int seg = (nrows + nseg - 1) / nseg;
  for (int w = threadIdx.x; w < ncols * nseg; w += kThreads) {
    const int s = w / ncols;
    const int c = c0 + (w - s * ncols);
    const int ya = r0 + s * seg;
    const int yb = min(r1, ya + seg);
    if (ya < yb) body(c, ya, yb);
  }
}

template <bool MAX>
__device__ __forceinline__ float red2(float a, float b) { return MAX ? fmaxf(a, b) : fminf(a, b); }

// reduce p[-R..R]
template <int R, bool MAX>
__device__ __forceinline__ float hred(const float* p) {
  float v = p[0];
#pragma unroll
  for (int k = 1; k <= R; ++k) v = red2<MAX>(red2<MAX>(v, p[-k]), p[k]);
  return v;
}

// ---------------------------------------------------------------------------
// Stage 2: dilation with a row-convex symmetric kernel.  Row dy of the kernel
// is the centred interval |dx| <= se_half(dy).
template <int SHAPE, int R>
__host__ __device__ constexpr int se_half(int dy) {
  const int ady = dy < 0 ? -dy : dy;
  if (SHAPE == 0) return R;                               // full
  if (SHAPE == 1) return ady == 0 ? R : 0;                // cross
  if (SHAPE == 2) return R - ady;                         // diamond
  // circle: largest e with 4 (e^2 + dy^2) <= (2R + 1)^2
  int e = 0;
  while (e < R && 4 * ((e + 1) * (e + 1) + ady * ady) <= (2 * R + 1) * (2 * R + 1)) ++e;
  return e;
}

template <int SHAPE, int R>
__device__ void dilate_se(const float* src, float* dst, int pitch, int r0, int r1, int c0, int c1,
                          int oy, int ox, int H, int W) {
  for_column_runs(r0, r1, c0, c1, [&](int c, int ya, int yb) {
    float h[2 * R + 1][R + 1];   // per window row: max over |dx| <= e, e = 0..R
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      const float* p = src + (ya - R + k) * pitch + c;
      h[k + 1][0] = p[0];
#pragma unroll
      for (int e = 1; e <= R; ++e) h[k + 1][e] = fmaxf(fmaxf(h[k + 1][e - 1], p[-e]), p[e]);
    }
    const int gx = ox + c;
    const bool colin = gx >= 0 && gx < W;
    for (int y = ya; y < yb; ++y) {
#pragma unroll
      for (int k = 0; k < 2 * R; ++k)
#pragma unroll
        for (int e = 0; e <= R; ++e) h[k][e] = h[k + 1][e];
      {
        const float* p = src + (y + R) * pitch + c;
        h[2 * R][0] = p[0];
#pragma unroll
        for (int e = 1; e <= R; ++e) h[2 * R][e] = fmaxf(fmaxf(h[2 * R][e - 1], p[-e]), p[e]);
      }
      float v = h[R][se_half<SHAPE, R>(0)];
#pragma unroll
      for (int dy = -R; dy <= R; ++dy)
        if (dy != 0) v = fmaxf(v, h[dy + R][se_half<SHAPE, R>(dy)]);
      const int gy = oy + y;
      dst[y * pitch + c] = (colin && gy >= 0 && gy < H) ? v : 0.f;
    }
  });
}

__device__ __forceinline__ void dilate_se_dispatch(int shape, int r, const float* src, float* dst, int pitch,
                                   int r0, int r1, int c0, int c1, int oy, int ox, int H, int W) {
#define IPB_SE(S, RR) \
  if (shape == S && r == RR) { dilate_se<S, RR>(src, dst, pitch, r0, r1, c0, c1, oy, ox, H, W); return; }
  IPB_SE(2, 2) IPB_SE(1, 2) IPB_SE(0, 2) IPB_SE(3, 2)
  IPB_SE(2, 1) IPB_SE(1, 1) IPB_SE(0, 1) IPB_SE(3, 1)
  IPB_SE(2, 3) IPB_SE(1, 3) IPB_SE(0, 3) IPB_SE(3, 3)
#undef IPB_SE
}

// Stages 3a/3b: full (2R+1)^2 max or min; cells outside the image get `oob`
// (the neutral element of the next stage).
template <int R, bool MAX>
__device__ void sep_full(const float* src, float* dst, int pitch, int r0, int r1, int c0, int c1,
                         int oy, int ox, int H, int W, float oob) {
  for_column_runs(r0, r1, c0, c1, [&](int c, int ya, int yb) {
    float win[2 * R + 1];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) win[k + 1] = hred<R, MAX>(src + (ya - R + k) * pitch + c);
    const int gx = ox + c;
    const bool colin = gx >= 0 && gx < W;
    for (int y = ya; y < yb; ++y) {
#pragma unroll
      for (int k = 0; k < 2 * R; ++k) win[k] = win[k + 1];
      win[2 * R] = hred<R, MAX>(src + (y + R) * pitch + c);
      float v = win[0];
#pragma unroll
      for (int k = 1; k <= 2 * R; ++k) v = red2<MAX>(v, win[k]);
      const int gy = oy + y;
      dst[y * pitch + c] = (colin && gy >= 0 && gy < H) ? v : oob;
    }
  });
}

template <bool MAX>
__device__ __forceinline__ void sep_full_dispatch(int r, const float* src, float* dst, int pitch, int r0, int r1,
                                  int c0, int c1, int oy, int ox, int H, int W, float oob) {
  if (r == 2) sep_full<2, MAX>(src, dst, pitch, r0, r1, c0, c1, oy, ox, H, W, oob);
  else if (r == 1) sep_full<1, MAX>(src, dst, pitch, r0, r1, c0, c1, oy, ox, H, W, oob);
  else if (r == 3) sep_full<3, MAX>(src, dst, pitch, r0, r1, c0, c1, oy, ox, H, W, oob);
}

// Stage 4: empty pixels take the (2R+1)^2 window max; the result goes to
// global memory, and the topmost non-empty row of each column is folded
// into the frame's column table.
template <int R>
__device__ void small_fill(const float* src, int pitch, int r0, int r1, int c0, int c1, int oy,
                           int ox, int H, int W, float thr, float* dst, int32_t* top) {
  for_column_runs(r0, r1, c0, c1, [&](int c, int ya, int yb) {
    float win[2 * R + 1];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) win[k + 1] = hred<R, true>(src + (ya - R + k) * pitch + c);
    const int gx = ox + c;
    if (gx >= W) return;
    int first = kNoTop;
    for (int y = ya; y < yb; ++y) {
#pragma unroll
      for (int k = 0; k < 2 * R; ++k) win[k] = win[k + 1];
      win[2 * R] = hred<R, true>(src + (y + R) * pitch + c);
      float m = win[0];
#pragma unroll
      for (int k = 1; k <= 2 * R; ++k) m = fmaxf(m, win[k]);
      const float ctr = src[y * pitch + c];
      const float v = ctr <= thr ? m : ctr;
      const int gy = oy + y;
      if (gy < H) {
        dst[(size_t)gy * W + gx] = v;
        if (v > thr && first == kNoTop) first = gy;
      }
    }
    if (top != nullptr && first != kNoTop) atomicMin(top + gx, first);
  });
}

__device__ __forceinline__ void small_fill_dispatch(int r, const float* src, int pitch, int r0, int r1, int c0, int c1,
                                    int oy, int ox, int H, int W, float thr, float* dst, int32_t* top) {
  if (r == 3) small_fill<3>(src, pitch, r0, r1, c0, c1, oy, ox, H, W, thr, dst, top);
  else if (r == 2) small_fill<2>(src, pitch, r0, r1, c0, c1, oy, ox, H, W, thr, dst, top);
  else if (r == 1) small_fill<1>(src, pitch, r0, r1, c0, c1, oy, ox, H, W, thr, dst, top);
}

// Copy the in-image cells of the tile window of an LDS buffer to global
// (rows below ylim and columns left of xlim only).
__device__ void store_tile(const float* buf, int pitch, int bcol0, int r0, int r1, int c0, int c1,
                           int oy, int ox, int H, int W, float* dst, int ylim = 0x7fffffff,
                           int xlim = 0x7fffffff) {
  const int nc = c1 - c0, n = (r1 - r0) * nc;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const int r = r0 + i / nc, c = c0 + i % nc;
    const int gy = oy + r, gx = ox + c;
    if (gy >= 0 && gy < H && gy < ylim && gx >= 0 && gx < W && gx < xlim)
      dst[(size_t)gy * W + gx] = buf[r * pitch + (c - bcol0)];
  }
}

// ---------------------------------------------------------------------------
// Phase 1: stages 1-4 of one TH x TW tile.
template <int TH, int TW, int HL>
__device__ void local_tile(const FrameDesc& f, const KParams& kp, int ty0, int tx0, float* A, float* B) {
  constexpr int RH = TH + 2 * HL, RW = TW + 2 * HL;
  const int oy = ty0 - HL, ox = tx0 - HL;
  const int H = f.H, W = f.W;
  const float thr = kp.thr, off = kp.off;

  // Stage 1: inversion (Sec. III "Depth Inversion").
  for (int i = threadIdx.x; i < RH * RW; i += kThreads) {
    const int r = i / RW, c = i - r * RW;
    const int gy = oy + r, gx = ox + c;
    float v = 0.f;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
      const float d = f.in[(size_t)gy * W + gx];
      const float inv = off - d;
      v = (d > thr && inv > thr) ? inv : 0.f;
    }
    A[i] = v;
  }
  __syncthreads();
  if (kp.last_stage == 1) { store_tile(A, RW, 0, HL, HL + TH, HL, HL + TW, oy, ox, H, W, f.out); return; }

  // Stage 2: kernel-shaped dilation.
  int s = kp.rd;
  dilate_se_dispatch(kp.shape, kp.rd, A, B, RW, s, RH - s, s, RW - s, oy, ox, H, W);
  __syncthreads();
  if (kp.last_stage == 2) { store_tile(B, RW, 0, HL, HL + TH, HL, HL + TW, oy, ox, H, W, f.out); return; }

  // Stage 3: closing = dilation then erosion, full kernel.
  s += kp.rc;
  sep_full_dispatch<true>(kp.rc, B, A, RW, s, RH - s, s, RW - s, oy, ox, H, W, __int_as_float(0x7f800000));
  __syncthreads();
  s += kp.rc;
  sep_full_dispatch<false>(kp.rc, A, B, RW, s, RH - s, s, RW - s, oy, ox, H, W, 0.f);
  __syncthreads();
  if (kp.last_stage == 3) { store_tile(B, RW, 0, HL, HL + TH, HL, HL + TW, oy, ox, H, W, f.out); return; }

  // Stage 4: small hole fill.
  const bool final4 = kp.last_stage == 4;
  small_fill_dispatch(kp.rf, B, RW, HL, HL + TH, HL, HL + TW, oy, ox, H, W, thr,
                      final4 ? f.out : f.v4, final4 ? nullptr : f.top);
}

template <int TH, int TW, int HL>
__global__ __launch_bounds__(kThreads) void k_local(FrameSource src, KParams kp) {
  constexpr int RH = TH + 2 * HL, RW = TW + 2 * HL;
  __shared__ float A[RH * RW];
  __shared__ float B[RH * RW];
  const int total = src.plan ? src.plan->ltiles : src.single_ltiles;
  for (int t = xcd_tile(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
    FrameDesc f;
    if (src.plan) f = plan_frames(src.plan)[src.plan->ltab[t]];
    else f = src.single;
    const int lt = t - f.ltile0;
    const int tr = lt / f.lcols;
    const int ty0 = tr * TH, tx0 = (lt - tr * f.lcols) * TW;
    local_tile<TH, TW, HL>(f, kp, ty0, tx0, A, B);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Phase 2 pieces.

// Large fill, horizontal pass: dst[r][c - bcol0] = max over src[r][c-R .. c+R].
template <int R>
__device__ void hmax_pass(const float* src, int pitch, float* dst, int dpitch, int bcol0,
                          int r0, int r1, int c0, int c1) {
  for_column_runs(r0, r1, c0, c1, [&](int c, int ya, int yb) {
    for (int y = ya; y < yb; ++y) dst[y * dpitch + (c - bcol0)] = hred<R, true>(src + y * pitch + c);
  });
}

__device__ __forceinline__ void hmax_pass_rt(int r, const float* src, int pitch, float* dst, int dpitch, int bcol0,
                             int r0, int r1, int c0, int c1) {
  if (r == 15) { hmax_pass<15>(src, pitch, dst, dpitch, bcol0, r0, r1, c0, c1); return; }
  for_column_runs(r0, r1, c0, c1, [&](int c, int ya, int yb) {
    for (int y = ya; y < yb; ++y) {
      const float* p = src + y * pitch + c;
      float v = p[0];
      for (int k = 1; k <= r; ++k) v = fmaxf(fmaxf(v, p[-k]), p[k]);
      dst[y * dpitch + (c - bcol0)] = v;
    }
  });
}

// Large fill, vertical pass and select, in place on A.
__device__ void vfill_pass(int r, float* A, int pitch, const float* Bh, int bpitch, int bcol0,
                           int r0, int r1, int c0, int c1, float thr) {
  for_column_runs(r0, r1, c0, c1, [&](int c, int ya, int yb) {
    for (int y = ya; y < yb; ++y) {
      const float ctr = A[y * pitch + c];
      if (ctr <= thr) {
        const float* q = Bh + y * bpitch + (c - bcol0);
        float v = q[0];
        for (int k = 1; k <= r; ++k) v = fmaxf(fmaxf(v, q[-k * bpitch]), q[k * bpitch]);
        A[y * pitch + c] = v;
      }
    }
  });
}

// Stage 7: median of the (2RM+1)^2 window with clamped coordinates, for
// in-image cells; writes B[r][c - bcol0].
template <int RM>
__device__ void median_pass(const float* A, int pitch, float* B, int bpitch, int bcol0,
                            int r0, int r1, int c0, int c1, int oy, int ox, int H, int W) {
  constexpr int K = 2 * RM + 1;
  constexpr int N = K * K;
  const int ra = max(r0, -oy), rb = min(r1, H - oy);
  const int ca = max(c0, -ox), cb = min(c1, W - ox);
  for_column_runs(ra, rb, ca, cb, [&](int c, int ya, int yb) {
    int cc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) cc[k] = clampi(ox + c + k - RM, 0, W - 1) - ox;
    float win[K][K];
    auto load_row = [&](int y, float* w) {
      const float* p = A + (clampi(oy + y, 0, H - 1) - oy) * pitch;
#pragma unroll
      for (int k = 0; k < K; ++k) w[k] = p[cc[k]];
    };
#pragma unroll
    for (int k = 0; k < K - 1; ++k) load_row(ya - RM + k, win[k + 1]);
    for (int y = ya; y < yb; ++y) {
#pragma unroll
      for (int k = 0; k < K - 1; ++k)
#pragma unroll
        for (int j = 0; j < K; ++j) win[k][j] = win[k + 1][j];
      load_row(y + RM, win[K - 1]);
      float a[net::pow2_at_least(N)];
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int j = 0; j < K; ++j) a[k * K + j] = win[k][j];
      net::sort_network<N>(a);
      B[y * bpitch + (c - bcol0)] = a[N / 2];
    }
  });
}

// Stage 7 off: copy the in-image cells.
__device__ void copy_pass(const float* A, int pitch, float* B, int bpitch, int bcol0,
                          int r0, int r1, int c0, int c1, int oy, int ox, int H, int W) {
  const int ra = max(r0, -oy), rb = min(r1, H - oy);
  const int ca = max(c0, -ox), cb = min(c1, W - ox);
  for_column_runs(ra, rb, ca, cb, [&](int c, int ya, int yb) {
    for (int y = ya; y < yb; ++y) B[y * bpitch + (c - bcol0)] = A[y * pitch + c];
  });
}

// Out-of-image cells within `rg` of the image take the value of their
// reflect-101 image cell (the Gaussian's border).
__device__ void reflect_fixup(float* B, int bpitch, int bcol0, int r0, int r1, int c0, int c1,
                              int oy, int ox, int H, int W, int rg) {
  const int nc = c1 - c0, n = (r1 - r0) * nc;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const int r = r0 + i / nc, c = c0 + i % nc;
    const int gy = oy + r, gx = ox + c;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) continue;
    if (gy < -rg || gy >= H + rg || gx < -rg || gx >= W + rg) continue;
    // the reflected cell lies within the tile +- rg; the clamp only keeps the
    // read inside the buffer
    const int sr = clampi(refl101(gy, H) - oy, r0, r1 - 1);
    const int sc = clampi(refl101(gx, W) - ox, c0, c1 - 1);
    B[r * bpitch + (c - bcol0)] = B[sr * bpitch + (sc - bcol0)];
  }
}

// Stages 8 and 9: Gaussian (fp64 sum, reflect-101 border already in B),
// masked by the median output, then the output inversion.
// Stages 8 (bilateral variant, Sec. IV, Table 3) and 9: the weighted mean
// of the (2 RG + 1)^2 window of the median map, each tap weighted by its
// distance and by the difference of its value from the centre value
// (float32 throughout), masked like the Gaussian.  B holds the median map
// with its reflect-101 border cells already filled.
template <int RG>
__device__ void bilat_out(const float* B, int bpitch, int bcol0, int r0, int r1, int c0, int c1,
                          int oy, int ox, int H, int W, const KParams& kp, float* dst, bool stage8,
                          int ylim, int xlim) {
  const int rb = min(r1, min(ylim, H) - oy), cb = min(c1, min(xlim, W) - ox);
  const float thr = kp.thr, off = kp.off, kc = kp.bl_kc;
  for_column_runs(r0, rb, c0, cb, [&](int c, int ya, int yb) {
    const int gx = ox + c;
    for (int y = ya; y < yb; ++y) {
      const float* p = B + y * bpitch + (c - bcol0);
      const float v7 = p[0];
      float num = 0.f, den = 0.f;
#pragma unroll
      for (int dy = -RG; dy <= RG; ++dy) {
#pragma unroll
        for (int dx = -RG; dx <= RG; ++dx) {
          const float q = p[dy * bpitch + dx];
          const float d = q - v7;
          const float w = kp.bl_ws[(dy < 0 ? -dy : dy) * 3 + (dx < 0 ? -dx : dx)] * expf(-(d * d) * kc);
          num += w * q;
          den += w;
        }
      }
      const bool m = v7 > thr;
      const float v8 = m ? num / den : 0.f;
      const float o = m ? off - v8 : 0.f;
      dst[(size_t)(oy + y) * W + gx] = stage8 ? v8 : o;
    }
  });
}

template <int RG>
__device__ void gauss_out(const float* B, int bpitch, int bcol0, int r0, int r1, int c0, int c1,
                          int oy, int ox, int H, int W, const KParams& kp, float* dst, bool stage8,
                          int ylim, int xlim) {
  const int rb = min(r1, min(ylim, H) - oy), cb = min(c1, min(xlim, W) - ox);
  const double w0 = kp.gw[0], w1 = kp.gw[1], w2 = kp.gw[2], sc = kp.gscale;
  const float thr = kp.thr, off = kp.off;
  for_column_runs(r0, rb, c0, cb, [&](int c, int ya, int yb) {
    auto hsum = [&](int y) -> double {
      const float* p = B + y * bpitch + (c - bcol0);
      double h = w0 * (double)p[0];
      if (RG >= 1) h = h + w1 * ((double)p[-1] + (double)p[1]);
      if (RG >= 2) h = h + w2 * ((double)p[-2] + (double)p[2]);
      return h;
    };
    double win[2 * RG + 1];
#pragma unroll
    for (int k = 0; k < 2 * RG; ++k) win[k + 1] = hsum(ya - RG + k);
    const int gx = ox + c;
    for (int y = ya; y < yb; ++y) {
#pragma unroll
      for (int k = 0; k < 2 * RG; ++k) win[k] = win[k + 1];
      win[2 * RG] = hsum(y + RG);
      double g = w0 * win[RG];
      if (RG >= 1) g = g + w1 * (win[RG - 1] + win[RG + 1]);
      if (RG >= 2) g = g + w2 * (win[RG - 2] + win[RG + 2]);
      g = g * sc;
      const float v7 = B[y * bpitch + (c - bcol0)];
      const bool m = v7 > thr;
      const float v8 = m ? (float)g : 0.f;
      const float o = m ? off - v8 : 0.f;
      dst[(size_t)(oy + y) * W + gx] = stage8 ? v8 : o;
    }
  });
}

// Gaussian off: output inversion of the median map.
__device__ void plain_out(const float* B, int bpitch, int bcol0, int r0, int r1, int c0, int c1,
                          int oy, int ox, int H, int W, const KParams& kp, float* dst, bool stage8,
                          int ylim, int xlim) {
  const int rb = min(r1, min(ylim, H) - oy), cb = min(c1, min(xlim, W) - ox);
  for_column_runs(r0, rb, c0, cb, [&](int c, int ya, int yb) {
    for (int y = ya; y < yb; ++y) {
      const float v7 = B[y * bpitch + (c - bcol0)];
      const bool m = v7 > kp.thr;
      const float v8 = m ? v7 : 0.f;
      dst[(size_t)(oy + y) * W + (ox + c)] = stage8 ? v8 : (m ? kp.off - v8 : 0.f);
    }
  });
}

constexpr int kHG = 19;   // phase-2 halo: 15 (31x31 fill) + 2 (median) + 2 (Gaussian)

// Phase 2: stages 5-9 of one TH x TW tile.
template <int TH, int TW>
__device__ void global_tile(const FrameDesc& f, const KParams& kp, int ty0, int tx0, float* A, float* B,
                            int* s_top, float* s_topv, int ylim = 0x7fffffff, int xlim = 0x7fffffff) {
  constexpr int RH = TH + 2 * kHG, RW = TW + 2 * kHG, BW = TW + 8, B0 = kHG - 4;
  const int oy = ty0 - kHG, ox = tx0 - kHG;
  const int H = f.H, W = f.W;
  const float thr = kp.thr;
  const int E = kp.rm + kp.rg;

  // Column table of the region: the row and value that stage 5 copies upward.
  for (int c = threadIdx.x; c < RW; c += kThreads) {
    const int gx = ox + c;
    int top = 0;
    float tv = 0.f;
    if (kp.extrapolate && gx >= 0 && gx < W) {
      const int t = f.top[gx];
      if (t < H) { top = t; tv = f.v4[(size_t)t * W + gx]; }
    }
    s_top[c] = top;
    s_topv[c] = tv;
  }
  __syncthreads();

  // Stage 5 (extension to top of frame) while loading the cells the median
  // and blur need; note whether any of them is still empty.
  const int n0 = kHG - E, n1 = kHG + TH + E;
  const int ext = kp.ext_rows;
  auto load5 = [&](int r, int c) -> float {
    const int gy = oy + r, gx = ox + c;
    if (gy < 0 || gy >= H || gx < 0 || gx >= W) return 0.f;
    return (gy < s_top[c] && (ext <= 0 || gy >= s_top[c] - ext)) ? s_topv[c] : f.v4[(size_t)gy * W + gx];
  };
  const int m0 = kHG - E, m1 = kHG + TW + E;   // needed columns
  int empty = 0;
  {
    const int ncol = m1 - m0;
    const int ncell = (n1 - n0) * ncol;
    for (int i = threadIdx.x; i < ncell; i += kThreads) {
      const int r = n0 + i / ncol, c = m0 + i % ncol;
      const float v = load5(r, c);
      A[r * RW + c] = v;
      const int gy = oy + r, gx = ox + c;
      if (v <= thr && gy >= 0 && gy < H && gx >= 0 && gx < W) empty = 1;
    }
  }
  const bool any_empty = __syncthreads_or(empty) != 0;
  if (kp.last_stage == 5) {
    store_tile(A, RW, 0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, f.out, ylim, xlim);
    return;
  }

  // Stage 6: large hole fill, only where something is left to fill.
  if (kp.extrapolate && any_empty) {
    for (int i = threadIdx.x; i < RH * RW; i += kThreads) {
      const int r = i / RW, c = i - r * RW;
      if (r >= n0 && r < n1 && c >= m0 && c < m1) continue;
      A[i] = load5(r, c);
    }
    __syncthreads();
    const int rl = kp.rl;
    hmax_pass_rt(rl, A, RW, B, BW, B0, n0 - rl, n1 + rl, m0, m1);
    __syncthreads();
    vfill_pass(rl, A, RW, B, BW, B0, n0, n1, m0, m1, thr);
    __syncthreads();
  }
  if (kp.last_stage == 6) {
    store_tile(A, RW, 0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, f.out, ylim, xlim);
    return;
  }

  // Stage 7: median blur over the tile plus the Gaussian's reach.
  const int q0 = kHG - kp.rg, q1r = kHG + TH + kp.rg, q1c = kHG + TW + kp.rg;
  if (kp.rm == 2) median_pass<2>(A, RW, B, BW, B0, q0, q1r, q0, q1c, oy, ox, H, W);
  else if (kp.rm == 1) median_pass<1>(A, RW, B, BW, B0, q0, q1r, q0, q1c, oy, ox, H, W);
  else copy_pass(A, RW, B, BW, B0, q0, q1r, q0, q1c, oy, ox, H, W);
  __syncthreads();
  if (kp.last_stage == 7) {
    store_tile(B, BW, B0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, f.out, ylim, xlim);
    return;
  }
  if (kp.rg > 0) {
    reflect_fixup(B, BW, B0, q0, q1r, q0, q1c, oy, ox, H, W, kp.rg);
    __syncthreads();
  }

  // Stages 8 and 9.
  const bool st8 = kp.last_stage == 8;
  if (kp.blur == 1 && kp.rg == 2) bilat_out<2>(B, BW, B0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, kp, f.out, st8, ylim, xlim);
  else if (kp.blur == 1 && kp.rg == 1) bilat_out<1>(B, BW, B0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, kp, f.out, st8, ylim, xlim);
  else if (kp.rg == 2) gauss_out<2>(B, BW, B0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, kp, f.out, st8, ylim, xlim);
  else if (kp.rg == 1) gauss_out<1>(B, BW, B0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, kp, f.out, st8, ylim, xlim);
  else plain_out(B, BW, B0, kHG, kHG + TH, kHG, kHG + TW, oy, ox, H, W, kp, f.out, st8, ylim, xlim);
}

template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_global(FrameSource src, KParams kp) {
  constexpr int RH = TH + 2 * kHG, RW = TW + 2 * kHG, BW = TW + 8;
  __shared__ float A[RH * RW];
  __shared__ float B[RH * BW];
  __shared__ int s_top[RW];
  __shared__ float s_topv[RW];
  const int total = src.plan ? src.plan->gtiles : src.single_gtiles;
  for (int t = xcd_tile(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
    FrameDesc f;
    if (src.plan) f = plan_frames(src.plan)[src.plan->gtab[t]];
    else f = src.single;
    const int gt = t - f.gtile0;
    const int tr = gt / f.gcols;
    const int ty0 = tr * TH, tx0 = (gt - tr * f.gcols) * TW;
    global_tile<TH, TW>(f, kp, ty0, tx0, A, B, s_top, s_topv);
    __syncthreads();
  }
}

// Phase 2, queued tiles of frames under 3 rows or columns (whose reflect-101
// border the streaming kernel does not handle): streaming tiles (srows x
// scols) recomputed with the LDS tile code, each covered by TH x TW LDS tiles
// clipped to the streaming tile.
template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_global_slow(FrameSource src, KParams kp, int srows, int scols) {
  constexpr int RH = TH + 2 * kHG, RW = TW + 2 * kHG, BW = TW + 8;
  __shared__ float A[RH * RW];
  __shared__ float B[RH * BW];
  __shared__ int s_top[RW];
  __shared__ float s_topv[RW];
  const int32_t* slow = src.plan ? src.plan->slow : src.slow;
  const int cap = src.plan ? src.plan->slow_cap : src.slow_cap;
  const int count = min(slow[1], cap);
  const int32_t* queue = slow + lds_queue_offset(cap);
  const int nsy = (srows + TH - 1) / TH, nsx = (scols + TW - 1) / TW, per = nsy * nsx;
  for (int i = blockIdx.x; i < count * per; i += gridDim.x) {
    const int t = queue[i / per], j = i % per;
    FrameDesc f;
    if (src.plan) f = plan_frames(src.plan)[src.plan->gtab[t]];
    else f = src.single;
    const int gt = t - f.gtile0;
    const int tr = gt / f.gcols;
    const int sy0 = tr * srows, sx0 = (gt - tr * f.gcols) * scols;
    const int ty0 = sy0 + (j / nsx) * TH, tx0 = sx0 + (j % nsx) * TW;
    if (ty0 < f.H && tx0 < f.W) global_tile<TH, TW>(f, kp, ty0, tx0, A, B, s_top, s_topv, sy0 + srows, sx0 + scols);
    __syncthreads();
  }
}

// Column tables of every frame of a launch: reset to "no non-empty row";
// empty the queues of the 31x31 fill.
__global__ __launch_bounds__(kThreads) void k_reset(FrameSource src) {
  int32_t* base = src.plan ? src.plan->top_base : src.single.top;
  const int n = src.plan ? src.plan->ncols : src.single.W;
  int32_t* slow = src.plan ? src.plan->slow : src.slow;
  const int gid = blockIdx.x * kThreads + threadIdx.x, stride = gridDim.x * kThreads;
  if (blockIdx.x == 0 && threadIdx.x < kQueueHead && slow != nullptr) slow[threadIdx.x] = 0;
  for (int i = gid; i < n; i += stride) base[i] = kNoTop;
  // the frame of every tile, so that a tile's wave finds its frame with one
  // load: a workgroup per frame writes its tiles' entries
  if (src.plan) {
    const PlanHeader* p = src.plan;
    const FrameDesc* fd = plan_frames(p);
    for (int f = blockIdx.x; f < p->n; f += gridDim.x) {
      const FrameDesc d = fd[f];
      const int nl = d.lcols * ((d.H + p->lt_rows - 1) / p->lt_rows);
      const int ng = d.gcols * ((d.H + p->gt_rows - 1) / p->gt_rows);
      for (int j = threadIdx.x; j < nl; j += kThreads) p->ltab[d.ltile0 + j] = f;
      for (int j = threadIdx.x; j < ng; j += kThreads) p->gtab[d.gtile0 + j] = f;
    }
  }
}

// A launch plan built on the host travels to the workspace in kernel
// arguments, a chunk per launch: the call then needs no host staging
// buffer, no copy engine and no wait, and can be captured into a graph.
struct PlanChunk {
  int32_t words[kPlanChunkWords];
};
__global__ __launch_bounds__(kThreads) void k_plan_upload(PlanChunk c, int32_t* dst, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += kThreads) dst[i] = c.words[i];
}

// ---------------------------------------------------------------------------
// Tile shapes.
struct Shape { int rows, cols; };
constexpr Shape kLocalShapes[] = {{32, 64}, {16, 64}, {32, 128}, {64, 64}};
constexpr Shape kGlobalShapes[] = {{32, 64}, {16, 64}, {48, 64}, {16, 128}};
constexpr int kNumLocal = 4, kNumGlobal = 4;

template <class K>
int occupancy(K kernel) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kThreads, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace

int local_tile_rows(int id) { return (id >= 1 && id <= kNumLocal) ? kLocalShapes[id - 1].rows : 0; }
int local_tile_cols(int id) { return (id >= 1 && id <= kNumLocal) ? kLocalShapes[id - 1].cols : 0; }
int global_tile_rows(int id) { return (id >= 1 && id <= kNumGlobal) ? kGlobalShapes[id - 1].rows : 0; }
int global_tile_cols(int id) { return (id >= 1 && id <= kNumGlobal) ? kGlobalShapes[id - 1].cols : 0; }
int num_local_tiles() { return kNumLocal; }
int num_global_tiles() { return kNumGlobal; }

#define IPB_LOCAL_CASES(X) \
  X(1, 9, 32, 64) X(2, 9, 16, 64) X(3, 9, 32, 128) X(4, 9, 64, 64) \
  X(1, 12, 32, 64) X(2, 12, 16, 64) X(3, 12, 32, 128) X(4, 12, 64, 64)
#define IPB_GLOBAL_CASES(X) X(1, 32, 64) X(2, 16, 64) X(3, 48, 64) X(4, 16, 128)

hipError_t launch_reset(const FrameSource& src, int max_items, hipStream_t s) {
  int grid = (max_items + kThreads - 1) / kThreads;
  if (grid < 1) grid = 1;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(kThreads), 0, s, src);
  return hipGetLastError();
}

hipError_t launch_plan_upload(const void* plan_host, size_t bytes, void* plan_dev, hipStream_t s) {
  const int32_t* src = static_cast<const int32_t*>(plan_host);
  int32_t* dst = static_cast<int32_t*>(plan_dev);
  const size_t words = (bytes + 3) / 4;
  for (size_t w0 = 0; w0 < words; w0 += kPlanChunkWords) {
    const int nw = (int)std::min<size_t>(kPlanChunkWords, words - w0);
    PlanChunk c;
    std::memcpy(c.words, src + w0, sizeof(int32_t) * nw);
    hipLaunchKernelGGL(k_plan_upload, dim3(1), dim3(kThreads), 0, s, c, dst + w0, nw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_local(const FrameSource& src, const KParams& kp, int tile_id, int halo, int grid,
                        hipStream_t s) {
#define X(ID, HL, TH, TW)                                                                  \
  if (tile_id == ID && halo == HL) {                                                       \
    hipLaunchKernelGGL((k_local<TH, TW, HL>), dim3(grid), dim3(kThreads), 0, s, src, kp); \
    return hipGetLastError();                                                              \
  }
  IPB_LOCAL_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_global(const FrameSource& src, const KParams& kp, int tile_id, int grid, hipStream_t s) {
#define X(ID, TH, TW)                                                                   \
  if (tile_id == ID) {                                                                  \
    hipLaunchKernelGGL((k_global<TH, TW>), dim3(grid), dim3(kThreads), 0, s, src, kp); \
    return hipGetLastError();                                                           \
  }
  IPB_GLOBAL_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_global_slow(const FrameSource& src, const KParams& kp, int stream_rows, int stream_cols,
                              int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_global_slow<32, 64>), dim3(grid), dim3(kThreads), 0, s, src, kp, stream_rows, stream_cols);
  return hipGetLastError();
}

int slow_subtiles(int stream_rows, int stream_cols) { return ((stream_rows + 31) / 32) * ((stream_cols + 63) / 64); }

int slow_resident_blocks() { return occupancy(k_global_slow<32, 64>); }

int max_resident_blocks(int phase, int tile_id, int halo) {
  if (phase == 1) {
#define X(ID, HL, TH, TW) \
  if (tile_id == ID && halo == HL) return occupancy(k_local<TH, TW, HL>);
    IPB_LOCAL_CASES(X)
#undef X
  } else {
#define X(ID, TH, TW) \
  if (tile_id == ID) return occupancy(k_global<TH, TW>);
    IPB_GLOBAL_CASES(X)
#undef X
  }
  return 1;
}

}  // namespace ipb
