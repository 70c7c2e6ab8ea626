// Streaming gfx950 kernels for the default chain (Ku, Harakeh & Waslander
// 2018, Sec. III): one wave64 per tile, two neighbouring columns per lane,
// rows streamed top to bottom through register ring buffers.  Neighbouring
// columns come from the adjacent lanes by DPP row moves (wave_shr/wave_shl),
// so the streaming kernels use no LDS and no barriers; k_local_stream and
// k_global_rows run four such waves per workgroup, one tile each.  On frames
// of even width a lane's column pair is one 8-byte access.
//
//   k_local_stream  : stages 1-4 (inversion, kernel dilation, 5x5 closing,
//                     7x7 small fill); 128 input columns -> 108 output
//                     columns; also the column tops and per tile column a
//                     record (first non-empty row, bands holding holes).
//   k_fill_scan,
//   k_fill_tiles    : stage 6 ahead of phase 2 for the default chain: the
//                     records and the final tops give the cells that are
//                     empty after the extension; their 31x31 fill goes into
//                     the stage-4 map, tagged.
//   k_global_rows   : stages 5, 7, 8, 9 of the default chain (extension on
//                     load, 5x5 median, Gaussian, output inversion) on the
//                     filled map, two rows per step, the median sorting rows
//                     first; 128 input columns -> 120 output columns.
//   k_global_stream : the same stages for other chains, one row per step,
//                     the median sorting columns first.  A tile whose
//                     needed cells still hold an
//                     empty pixel after the extension needs the 31x31 fill
//                     (stage 6): its quarters are queued, and the empty
//                     cells of quarters with few of them are queued one by
//                     one; k_fill_cells (per cell) or k_fill_dense (per
//                     quarter) computes the fill at the empty cells and
//                     k_global_patched runs those quarters again.
//
// Border rules are the ones of the LDS kernels: morphology ignores cells
// outside the image, the median replicates the border, the Gaussian reflects
// about the edge pixel (reflect-101).
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "common.hpp"
#include "median_rows.hpp"
#include "networks.hpp"
#include "offsets.hpp"

#pragma clang fp contract(off)

namespace ipb {
namespace {

constexpr int kLanes = 64;
constexpr int kInfKey = 0x7f800000;   // +inf

// Selection works on ordering keys: the bit patterns of the map values read
// as int32.  Every map value is +0, a positive finite float or +inf, and for
// those the integer order of the bit patterns is the float order, so integer
// min/max select exactly the values float min/max would (and need no NaN
// canonicalisation).
__device__ __forceinline__ int key(float v) { return __float_as_int(v); }

// Frame buffers are device (global) memory; say so, so that accesses use
// global loads/stores with a scalar row base and a 32-bit lane offset.
typedef __attribute__((address_space(1))) int gint;
typedef __attribute__((address_space(1))) const int gcint;
typedef __attribute__((address_space(1))) const float gcfloat;
__device__ __forceinline__ gcint* gc(const void* p) { return (gcint*)(const int*)p; }
__device__ __forceinline__ gcfloat* gcf(const float* p) { return (gcfloat*)p; }
__device__ __forceinline__ gint* gw(void* p) { return (gint*)(int*)p; }
typedef __attribute__((address_space(1))) const char gcchar;
typedef __attribute__((address_space(1))) char gchar;
// element at a 32-bit byte offset from a (uniform) row base
__device__ __forceinline__ int ldk(gcint* row, unsigned off) { return *(gcint*)((gcchar*)row + off); }
__device__ __forceinline__ float ldf(gcfloat* row, unsigned off) { return *(gcfloat*)((gcchar*)row + off); }
__device__ __forceinline__ void stk(gint* row, unsigned off, int v) { *(gint*)((gchar*)row + off) = v; }
__device__ __forceinline__ float val(int k) { return __int_as_float(k); }
// Device-memory atomic min as a global (not flat) atomic.  A flat operation
// still in flight makes every later wait for a vector load a wait for all
// outstanding loads, which would drain the row prefetch of the next tile.
__device__ __forceinline__ void atomic_min_g(int* p, int v) {
  __hip_atomic_fetch_min((gint*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_add_g(int* p, int v) {
  return __hip_atomic_fetch_add((gint*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// lane i receives lane i-1's value (lane 0 receives 0; its neighbours are
// outside the tile's input columns and never feed an output)
__device__ __forceinline__ int from_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
// lane i receives lane i+1's value (lane 63 receives 0)
__device__ __forceinline__ int from_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
// Max over the wave of non-negative values, as a uniform value: prefix
// maxima within rows of 16 lanes (row_shr 1, 2, 4, 8), then across rows
// (row_bcast 15 and 31); lane 63 ends with the whole wave's max.  Lanes
// without a source contribute 0.
__device__ __forceinline__ int wave_max_nonneg(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int max3i(int a, int b, int c) { return max(max(a, b), c); }
__device__ __forceinline__ int min3i(int a, int b, int c) { return min(min(a, b), c); }
__device__ __forceinline__ int clampi_s(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int xcd_tile_s(int b, int g) {
  if ((g & 7) != 0) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// The frame of a tile is the same for the whole wave: keep it in scalar
// registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A register copy the compiler cannot fold away.  Taking a prefetched row
// out of its ring slot this way lets the prefetch of row r + 4 load into the
// slot's own register; otherwise the loop carries register copies of loads
// still in flight, and every pass of the unrolled loop waits for all of them.
__device__ __forceinline__ int detach(int v) {
  int r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}
__device__ __forceinline__ float detachf(float v) { return __int_as_float(detach(__float_as_int(v))); }
template <class P>
__device__ __forceinline__ P* uni_ptr(P* p) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
  return reinterpret_cast<P*>(((unsigned long long)hi << 32) | lo);
}
// Descriptor fidx of a device plan.
__device__ __forceinline__ FrameDesc plan_frame(const FrameSource& src, int fidx) {
  return reinterpret_cast<const FrameDesc*>(src.plan + 1)[fidx];
}
__device__ __forceinline__ FrameDesc uniform_frame(const FrameDesc& f) {
  FrameDesc u;
  u.in = uni_ptr(f.in);
  u.out = uni_ptr(f.out);
  u.v4 = uni_ptr(f.v4);
  u.top = uni_ptr(f.top);
  u.H = uni(f.H);
  u.W = uni(f.W);
  u.ltile0 = uni(f.ltile0);
  u.gtile0 = uni(f.gtile0);
  u.lcols = uni(f.lcols);
  u.gcols = uni(f.gcols);
  u.v6p = uni_ptr(f.v6p);
  return u;
}


// Stage-2 kernel rows: row dy of the kernel is the centred interval
// |dx| <= se_half(dy) (full, cross, diamond, circle).
template <int SHAPE, int R>
__host__ __device__ constexpr int se_half_s(int dy) {
  const int ady = dy < 0 ? -dy : dy;
  if (SHAPE == 0) return R;
  if (SHAPE == 1) return ady == 0 ? R : 0;
  if (SHAPE == 2) return R - ady;
  int e = 0;
  while (e < R && 4 * ((e + 1) * (e + 1) + ady * ady) <= (2 * R + 1) * (2 * R + 1)) ++e;
  return e;
}

// f(integral_constant<int, 0>) .. f(integral_constant<int, 7>): the ring
// slots of one block of 8 rows as compile-time constants.
template <class F, int... Us>
__device__ __forceinline__ void for_slots_impl(F&& f, std::integer_sequence<int, Us...>) {
  (f(std::integral_constant<int, Us>{}), ...);
}
template <class F>
__device__ __forceinline__ void for_slots(F&& f) {
  for_slots_impl(f, std::make_integer_sequence<int, 8>{});
}

// Phase-1 column record of a tile column: the first non-empty row relative
// to the tile's first row (low 16 bits; kRecNone: none) and the 32-row bands
// of the tile that hold an empty row after it (high 16 bits, bit b: band b).
constexpr int kRecNone = 0xffff;

// ---------------------------------------------------------------------------
// Phase 1, streaming: stages 1-4 for 108 x TH output cells per wave.
constexpr int kLocalHalo = 10;                         // >= RD + 2 + 2 + 3 for RD <= 3
constexpr int kLocalTW = 2 * kLanes - 2 * kLocalHalo;  // 108
// Word 3 of a raw buffer resource on gfx9-family chips (32-bit data format).
constexpr int kBufferWord3 = 0x00020000;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
// 8-byte stores of column pairs (the streaming kernels' lanes own columns
// 2 l + even offset): every row of the map starts 8-byte aligned.
__device__ __forceinline__ bool pair_ok(int W, const void* map) {
  return (W & 1) == 0 && (reinterpret_cast<unsigned long long>(map) & 7u) == 0;
}

// One band of a column's record: nz holds the non-empty flags of the band's
// nb rows (the band's first row in bit nb - 1), vm those of them within the
// frame.  Sets first (the tile-relative first non-empty row, kRecNone if
// none yet) at the band's first non-empty row, and bit 16 + b of holes if
// an empty row follows the column's first non-empty row within the band.
__device__ __forceinline__ void resolve_band(unsigned nz, unsigned vm, int b, int nb, int& first, unsigned& holes) {
  const unsigned ne = nz & vm, em = ~nz & vm;
  const int p = 31 - __builtin_clz(ne | 1u);   // the band's first non-empty row is bit p
  const bool seen = first != kRecNone;
  const unsigned after = seen ? em : em & ((1u << p) - 1u);
  holes |= ((seen || ne != 0u) && after != 0u) ? 0x10000u << b : 0u;
  first = (!seen && ne != 0u) ? 32 * b + (nb - 1 - p) : first;
}

// Writes the stage-4 map into f.v4 for the later stages (the stage hooks
// 1-4 take the LDS kernel).  The per-row work keeps to few instructions and
// no branch: loads and stores take the row's byte offset in a scalar
// register and the lane's column offset in a vector one (buffer accesses),
// and with PAIR (frames of even width, where a lane's two columns are an
// 8-byte aligned pair, in or out of the frame together) one 8-byte store
// writes both columns, so that a wave's output row is one contiguous store;
// row checks are one unsigned compare; the column records are a shift
// register of non-empty flags per column, resolved once per 32-row band;
// and the stores are unconditional, the lanes with nothing to store writing
// to a scratch slot just past the map.
template <int SHAPE, int RD, int TH, bool PAIR>
__device__ void local_stream_tile(const FrameDesc& f, const KParams& kp, int ty0, int tx0, int lane) {
  const int H = f.H, W = f.W;
  const float thr = kp.thr, off = kp.off;
  const int kthr = key(thr);
  const int ca = tx0 - kLocalHalo + 2 * lane, cb = ca + 1;
  const bool ina = ca >= 0 && ca < W, inb = cb >= 0 && cb < W;
  const bool lane_out = lane >= kLocalHalo / 2 && lane < kLocalHalo / 2 + kLocalTW / 2;
  const bool outa = lane_out && ina, outb = lane_out && inb;
  const unsigned ua = 4u * (unsigned)ca, ub = ua + 4u;   // byte offsets, used only when in the image
  // load offsets: columns clamped into the image, so that every load is
  // issued unconditionally (the values of outside columns are masked where
  // they are used); loads issued on every path let the compiler wait for
  // each row alone instead of draining the prefetch
  // (PAIR: the pair's first column, clamped to 0 .. W - 2)
  const unsigned la = 4u * (unsigned)clampi_s(ca, 0, PAIR ? W - 2 : W - 1);
  const unsigned lb = 4u * (unsigned)clampi_s(cb, 0, W - 1);
  constexpr int D2 = RD, D3A = RD + 2, D3B = RD + 4, D4 = RD + 7;  // row delays of the stage outputs
  const int q0 = ty0 - D4;
  const int n = TH + 2 * D4;
  // output row q0 + r - D4 = ty0 + r - 2 D4 ends a band (or the tile) at
  // block slot (2 D4 - 1) & 7
  constexpr int kResolve = (2 * D4 + 7) & 7;

  // ring buffers (slot = relative row & 7), ordering keys
  int h[8][RD + 1][2];        // stage-2 horizontal maxima per radius
  int hd[8][2];               // stage-3a horizontal max
  int he[8][2];               // stage-3b horizontal min
  int hf[8][2];               // stage-4 horizontal max
  int v3[8][2];               // stage-3 map (centre of the fill)
#pragma unroll
  for (int s = 0; s < 8; ++s) {
#pragma unroll
    for (int e = 0; e <= RD; ++e) h[s][e][0] = h[s][e][1] = 0;
    hd[s][0] = hd[s][1] = 0;
    he[s][0] = he[s][1] = kInfKey;
    hf[s][0] = hf[s][1] = 0;
    v3[s][0] = v3[s][1] = 0;
  }
  // column records for the fill ahead of phase 2, written once at the end
  // of the tile: per column the non-empty flags of the current band's rows
  // so far (newest in bit 0), the first non-empty row of the tile (relative
  // to ty0; kRecNone: none yet) and the bands with a hole after it (bits 16..)
  unsigned nz_a = 0u, nz_b = 0u, holes_a = 0u, holes_b = 0u;
  int first_a = kRecNone, first_b = kRecNone;
  gchar* rec = (gchar*)(char*)f.v6p + 4 * (size_t)(ty0 / TH) * W;   // uniform row base; lanes add ua / ub
  // byte offsets within a map are below 2^32 (H W < 2^30)
  const __amdgpu_buffer_rsrc_t src = __builtin_amdgcn_make_buffer_rsrc((void*)f.in, (short)0, -1, kBufferWord3);
  const __amdgpu_buffer_rsrc_t dst = __builtin_amdgcn_make_buffer_rsrc((void*)f.v4, (short)0, -1, kBufferWord3);
  const unsigned W4 = 4u * (unsigned)W;
  const unsigned sink = sink_offset(H, W);               // scratch slot past the stage-4 map
  const unsigned uH = (unsigned)H;

  // input rows are fetched 4 rows ahead of their use (fewer registers keep
  // five waves per SIMD)
  float da[4], db[4];
  auto fetch = [&](int r, float& xa_, float& xb_) {
    const int rowoff = (int)((unsigned)clampi_s(q0 + r, 0, H - 1) * W4);
    if constexpr (PAIR) {
      // both cells at one column offset (a register copy made here, so that
      // the + 4 stays an immediate): the compiler issues one 8-byte load
      const int lo = detach((int)la);
      xa_ = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, lo, rowoff, 0));
      xb_ = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, lo + 4, rowoff, 0));
    } else {
      xa_ = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, (int)la, rowoff, 0));
      xb_ = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, (int)lb, rowoff, 0));
    }
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    fetch(u, da[u], db[u]);
    __builtin_amdgcn_sched_barrier(0);   // keep the prefetch in row order
  }
  // As many stores per prefetched row to the scratch slots past the map as
  // a row step makes: the row loop is entered with as many memory
  // operations in flight as in its steady state, so the waits at the top of
  // its blocks keep the full prefetch distance (vector memory operations
  // complete in order, and the compiler waits for the fewer in flight of the
  // loop's two entries).
#pragma unroll
  for (int k = 0; k < (PAIR ? 4 : 8); ++k) __builtin_amdgcn_raw_buffer_store_b32(0u, dst, 0, (int)(sink + 4u * k), 0);

  // Whole blocks of 8 rows: the steps past row n compute values no row
  // stores (their rows are past the tile), which keeps the unrolled block
  // free of exits.
  for (int rb = 0; rb < n; rb += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = rb + u;
      const int q = q0 + r;

      // Stage 1: inversion of input row q.
      int va, vb;
      {
        const bool rin = (unsigned)q < uH;
        const float d0 = detachf(da[u & 3]), d1 = detachf(db[u & 3]);
        fetch(r + 4, da[u & 3], db[u & 3]);
        __builtin_amdgcn_sched_barrier(0);   // issue the prefetch here, four rows ahead
        // cells outside the frame are empty (the loads read a clamped cell);
        // with a finite offset, min(d, off - d) > thr is d > thr and
        // off - d > thr (a NaN fails both)
        const float v0 = off - d0, v1 = off - d1;
        va = (rin && ina && d0 > thr && v0 > thr) ? key(v0) : 0;
        vb = (rin && inb && d1 > thr && v1 > thr) ? key(v1) : 0;
      }

      // Stage 2: kernel dilation; horizontal maxima of row q, then the
      // vertical combination for row q - RD.
      {
        const int La = from_prev(va), Lb = from_prev(vb), Ra = from_next(va), Rb = from_next(vb);
        h[u][0][0] = va;
        h[u][0][1] = vb;
        if constexpr (RD >= 1) { h[u][1][0] = max3i(Lb, va, vb); h[u][1][1] = max3i(va, vb, Ra); }
        if constexpr (RD >= 2) { h[u][2][0] = max3i(h[u][1][0], La, Ra); h[u][2][1] = max3i(h[u][1][1], Lb, Rb); }
        if constexpr (RD >= 3) {
          const int LLb = from_prev(Lb), RRa = from_next(Ra);
          h[u][3][0] = max3i(h[u][2][0], LLb, Rb);
          h[u][3][1] = max3i(h[u][2][1], La, RRa);
        }
      }
      const int p2 = q - D2;
      int w2a = h[(u - RD) & 7][se_half_s<SHAPE, RD>(0)][0];
      int w2b = h[(u - RD) & 7][se_half_s<SHAPE, RD>(0)][1];
#pragma unroll
      for (int dy = -RD; dy <= RD; ++dy) {
        if (dy == 0) continue;
        w2a = max(w2a, h[(u - RD + dy) & 7][se_half_s<SHAPE, RD>(dy)][0]);
        w2b = max(w2b, h[(u - RD + dy) & 7][se_half_s<SHAPE, RD>(dy)][1]);
      }
      const bool row2 = (unsigned)p2 < uH;
      w2a = (row2 && ina) ? w2a : 0;
      w2b = (row2 && inb) ? w2b : 0;

      // Stage 3a: 5x5 dilation; horizontal max of stage-2 row p2.
      {
        const int La = from_prev(w2a), Lb = from_prev(w2b), Ra = from_next(w2a), Rb = from_next(w2b);
        const int t = max3i(Lb, w2a, w2b);
        hd[u][0] = max3i(t, La, Ra);
        hd[u][1] = max3i(t, Ra, Rb);
      }
      const int p3 = q - D3A;
      int ta = max3i(max3i(hd[(u - 4) & 7][0], hd[(u - 3) & 7][0], hd[(u - 2) & 7][0]), hd[(u - 1) & 7][0], hd[u][0]);
      int tb = max3i(max3i(hd[(u - 4) & 7][1], hd[(u - 3) & 7][1], hd[(u - 2) & 7][1]), hd[(u - 1) & 7][1], hd[u][1]);
      const bool row3 = (unsigned)p3 < uH;
      ta = (row3 && ina) ? ta : kInfKey;
      tb = (row3 && inb) ? tb : kInfKey;

      // Stage 3b: 5x5 erosion; horizontal min of row p3.
      {
        const int La = from_prev(ta), Lb = from_prev(tb), Ra = from_next(ta), Rb = from_next(tb);
        const int t = min3i(Lb, ta, tb);
        he[u][0] = min3i(t, La, Ra);
        he[u][1] = min3i(t, Ra, Rb);
      }
      const int p4 = q - D3B;
      int ea = min3i(min3i(he[(u - 4) & 7][0], he[(u - 3) & 7][0], he[(u - 2) & 7][0]), he[(u - 1) & 7][0], he[u][0]);
      int eb = min3i(min3i(he[(u - 4) & 7][1], he[(u - 3) & 7][1], he[(u - 2) & 7][1]), he[(u - 1) & 7][1], he[u][1]);
      const bool row4 = (unsigned)p4 < uH;
      ea = (row4 && ina) ? ea : 0;
      eb = (row4 && inb) ? eb : 0;
      v3[u][0] = ea;
      v3[u][1] = eb;

      // Stage 4: 7x7 fill of empty pixels; horizontal max of row p4, then
      // the vertical max and the select for row p4 - 3.
      {
        const int La = from_prev(ea), Lb = from_prev(eb), Ra = from_next(ea), Rb = from_next(eb);
        const int LLb = from_prev(Lb), RRa = from_next(Ra);
        const int t = max(max3i(max3i(La, Lb, ea), eb, Ra), Rb);
        hf[u][0] = max(t, LLb);
        hf[u][1] = max(t, RRa);
      }
      const int o4 = q - D4;
      const int o4rel = o4 - ty0;
      const bool o4row = o4rel >= 0 && o4rel < TH && o4 < H;
      int oa, ob;
      {
        const int ma = max3i(max3i(hf[(u - 6) & 7][0], hf[(u - 5) & 7][0], hf[(u - 4) & 7][0]),
                             max3i(hf[(u - 3) & 7][0], hf[(u - 2) & 7][0], hf[(u - 1) & 7][0]), hf[u][0]);
        const int mb = max3i(max3i(hf[(u - 6) & 7][1], hf[(u - 5) & 7][1], hf[(u - 4) & 7][1]),
                             max3i(hf[(u - 3) & 7][1], hf[(u - 2) & 7][1], hf[(u - 1) & 7][1]), hf[u][1]);
        const int c3a = v3[(u - 3) & 7][0], c3b = v3[(u - 3) & 7][1];
        oa = c3a <= kthr ? ma : c3a;
        ob = c3b <= kthr ? mb : c3b;
        nz_a = nz_a + nz_a + (oa > kthr ? 1u : 0u);
        nz_b = nz_b + nz_b + (ob > kthr ? 1u : 0u);
      }
      {
        const unsigned row = o4row ? (unsigned)o4 * W4 : sink;
        if constexpr (PAIR) {
          u32x2 v;
          v.x = (unsigned)oa;
          v.y = (unsigned)ob;
          __builtin_amdgcn_raw_buffer_store_b64(v, dst, (int)((o4row && outa) ? ua : sink - row), (int)row, 0);
        } else {
          __builtin_amdgcn_raw_buffer_store_b32((unsigned)oa, dst, (int)((o4row && outa) ? ua : sink - row),
                                                (int)row, 0);
          __builtin_amdgcn_raw_buffer_store_b32((unsigned)ob, dst, (int)((o4row && outb) ? ub : sink - row),
                                                (int)row, 0);
        }
      }
      // the last row of a band (or of the tile): its rows within the frame
      // give the first non-empty row and whether an empty row follows it
      if (u == kResolve && o4rel >= 0 && o4rel < TH && ((o4rel & 31) == 31 || o4rel == TH - 1)) {
        const int b = o4rel >> 5;
        const int nb = o4rel - 32 * b + 1;                    // rows of the band
        const int nv = clampi_s(H - ty0 - 32 * b, 0, nb);    // of them within the frame
        const unsigned vm = nv == 0 ? 0u : (0xffffffffu >> (32 - nv)) << (nb - nv);
        resolve_band(nz_a, vm, b, nb, first_a, holes_a);
        resolve_band(nz_b, vm, b, nb, first_b, holes_b);
      }
    }
  }
  if (outa && first_a != kRecNone) atomic_min_g(f.top + ca, ty0 + first_a);
  if (outb && first_b != kRecNone) atomic_min_g(f.top + cb, ty0 + first_b);
  if (outa) stk((gint*)rec, ua, (int)(holes_a | (unsigned)first_a));
  if (outb) stk((gint*)rec, ub, (int)(holes_b | (unsigned)first_b));
}

// Four waves per workgroup, one tile each: the waves of a workgroup go to
// the four SIMDs of a compute unit, so 4 k tiles per compute unit put k
// waves on every SIMD (single-wave workgroups were placed 2 to 4 per SIMD
// for 3 on average, and the SIMDs with 4 set the launch's time).
constexpr int kLocalWaves = 4;

template <int SHAPE, int RD, int TH>
__global__ __launch_bounds__(kLanes * kLocalWaves) __attribute__((amdgpu_waves_per_eu(5))) void k_local_stream(FrameSource src, KParams kp) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = uni((int)threadIdx.x / kLanes);
  const int total = src.plan ? src.plan->ltiles : src.single_ltiles;
  for (int t = xcd_tile_s(blockIdx.x, gridDim.x) * kLocalWaves + wave; t < total; t += gridDim.x * kLocalWaves) {
    FrameDesc f;
    if (src.plan) f = plan_frame(src, gc(src.plan->ltab)[t]);
    else f = src.single;
    f = uniform_frame(f);
    const int lt = t - f.ltile0;
    const int tr = lt / f.lcols;
    if (pair_ok(f.W, f.v4)) local_stream_tile<SHAPE, RD, TH, true>(f, kp, tr * TH, (lt - tr * f.lcols) * kLocalTW, lane);
    else local_stream_tile<SHAPE, RD, TH, false>(f, kp, tr * TH, (lt - tr * f.lcols) * kLocalTW, lane);
  }
}

// ---------------------------------------------------------------------------
// Phase 2, streaming.

constexpr int kGlobalTW = 2 * kLanes - 8;   // 120

// Remove one occurrence of `out` from the sorted 5-window s and insert `in`
// (ordering keys).
__device__ __forceinline__ void window_update(int* s, int out, int in) {
  const int t0 = s[0] < out ? s[0] : s[1];
  const int t1 = s[1] < out ? s[1] : s[2];
  const int t2 = s[2] < out ? s[2] : s[3];
  const int t3 = s[3] < out ? s[3] : s[4];
  s[0] = min(t0, in);
  // clamp(in, t_{i-1}, t_i) as one v_med3 on the keys' float values (all
  // non-negative, no NaN: the same order as the keys)
  s[1] = key(__builtin_amdgcn_fmed3f(val(in), val(t0), val(t1)));
  s[2] = key(__builtin_amdgcn_fmed3f(val(in), val(t1), val(t2)));
  s[3] = key(__builtin_amdgcn_fmed3f(val(in), val(t2), val(t3)));
  s[4] = max(t3, in);
}

__device__ __forceinline__ double hsum5(double wc, double w1, double w2, int m2, int m1, int c, int p1, int p2) {
  // exact for the binomial taps (integer weights): every partial sum fits
  // in the 53-bit significand
  const double s2 = (double)val(m2) + (double)val(p2);
  const double s1 = (double)val(m1) + (double)val(p1);
  return fma(wc, (double)val(c), fma(w1, s1, w2 * s2));
}

// Stages 5-9 of one streaming tile (TH x 120 output cells) for chains other
// than the default one (which takes rows_first_tile).
// First pass (PATCHED false): the stage-6 map is taken to equal
// the stage-5 map; tiles where that does not hold are queued by quarter.
// Second pass (PATCHED true, one quarter): cells empty after stage 5 read
// their stage-6 value from f.v6p (written by k_fill_cells / k_fill_dense).
// s_cells: LDS lists of the first kCellEmpty empty cells of each quarter
// (first pass only).
template <int TH, bool PATCHED>
__device__ __forceinline__ void global_stream_tile(const FrameDesc& f, const KParams& kp, int t, int fidx, int gt,
                                                   int ty0, int tx0, int lane, int32_t* slow, int cap, int* s_cells) {
  const int H = f.H, W = f.W;
  const float thr = kp.thr, off = kp.off;
  const int kthr = key(thr);
  const int last = kp.last_stage;
  const bool median = kp.rm == 2;
  if (!PATCHED && (H < 3 || W < 3)) {   // reflect-101 on tiny frames: leave it to the LDS kernel
    if (lane == 0) {
      const int pos = atomic_add_g(slow + 1, 1);
      if (pos < cap) gw(slow)[lds_queue_offset(cap) + pos] = t;
    }
    return;
  }
  const int ca = tx0 - 4 + 2 * lane, cb = ca + 1;
  const int xa = clampi_s(ca, 0, W - 1), xb = clampi_s(cb, 0, W - 1);     // replicated border columns
  const unsigned oxa = 4u * (unsigned)xa, oxb = 4u * (unsigned)xb;
  const bool ina = ca >= 0 && ca < W, inb = cb >= 0 && cb < W;
  const bool lane_out = lane >= 2 && lane < 62;
  const bool outa = lane_out && ina, outb = lane_out && inb;
  const unsigned ua = 4u * (unsigned)ca, ub = ua + 4u;   // byte offsets, used only when in the image
  const bool edge_cols = tx0 - 4 < 0 || tx0 + kGlobalTW + 4 > W;
  gcint* v4 = gc(f.v4);
  gint* out = gw(f.out);

  // Stage 5 (extension to top of frame) on load: a row above its column's
  // top reads the top cell instead, V5[y][x] = V4[max(y, top)][x]; as byte
  // offsets, the larger of the row's and the top cell's (0 without a top).
  // Every load is issued unconditionally, so that the compiler waits for
  // each row alone instead of draining the prefetch.
  // With a limited reach (ext_rows > 0) only rows at or below top - ext_rows
  // copy the top cell: byte offsets from tlim up.
  const unsigned W4 = 4u * (unsigned)W;
  unsigned toffa = 0, toffb = 0, tlima = 0, tlimb = 0;
  if (kp.extrapolate) {
    gcint* top = gc(f.top);
    const int t_a = top[xa], t_b = top[xb];
    if (t_a < H) toffa = (unsigned)t_a * W4 + oxa;
    if (t_b < H) toffb = (unsigned)t_b * W4 + oxb;
    if (kp.ext_rows > 0) {
      if (t_a < H) tlima = (unsigned)max(t_a - kp.ext_rows, 0) * W4 + oxa;
      if (t_b < H) tlimb = (unsigned)max(t_b - kp.ext_rows, 0) * W4 + oxb;
    }
  }

  // reflect-101 source lane/slot of this lane's columns, for the Gaussian's border
  int sla = 0, slb = 0;
  bool sela = false, selb = false;
  if (edge_cols) {
    auto refl = [&](int c) {
      if (c < 0) c = -c;
      if (c >= W) c = 2 * W - 2 - c;
      return c;
    };
    const int sa = refl(ca) - (tx0 - 4), sb = refl(cb) - (tx0 - 4);
    sla = clampi_s(sa >> 1, 0, kLanes - 1);
    slb = clampi_s(sb >> 1, 0, kLanes - 1);
    sela = (sa & 1) != 0;
    selb = (sb & 1) != 0;
  }

  const double wc = kp.gw[0], w1 = kp.gw[1], w2 = kp.gw[2];
  const double gsc = kp.gscale;
  const int q0 = ty0 - 4;
  const int n = TH + 8;
  int raw[8][2];         // stage-5 keys (window of the median)
  int s7[8][2];          // median output keys
  double hs[8][2];       // Gaussian horizontal sums of the median rows
  int Sa[5], Sb[5];      // sorted 5-row windows of the lane's two columns
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    raw[s][0] = raw[s][1] = kInfKey;
    s7[s][0] = s7[s][1] = 0;
    hs[s][0] = hs[s][1] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) Sa[k] = Sb[k] = kInfKey;
  // quarters (TH/4 output rows each) whose input rows (+-4) hold an empty
  // cell, and the number of empty cells in each quarter's own rows
  unsigned qmask = 0;
  int qempty[4] = {0, 0, 0, 0};

  // Stage 5 on load: rows of the stage-4 map (border rows replicated), the
  // extension applied; fetched 4 rows ahead of their use.
  // PATCHED: the stage-6 value of the same cell, used where the stage-5
  // value is empty (such a cell is at or below its column's top).
  int pa[4], pb[4], ppa[4], ppb[4];
  gcint* v6p = gc(f.v6p);
  auto fetch = [&](int r, int u_) {
    const unsigned rowoff = (unsigned)clampi_s(q0 + r, 0, H - 1) * W4;
    unsigned oa_ = rowoff + oxa, ob_ = rowoff + oxb;
    oa_ = (oa_ < toffa && oa_ >= tlima) ? toffa : oa_;
    ob_ = (ob_ < toffb && ob_ >= tlimb) ? toffb : ob_;
    pa[u_] = ldk(v4, oa_);
    pb[u_] = ldk(v4, ob_);
    if (PATCHED) {
      ppa[u_] = ldk(v6p, rowoff + oxa);
      ppb[u_] = ldk(v6p, rowoff + oxb);
    }
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) fetch(u, u);

  // One row step: row q = q0 + r enters, the median of row q - 2 and the
  // outputs of row q - 4 leave.
  auto step = [&](auto u_tag, const int r, auto warm_tag) __attribute__((always_inline)) {
    constexpr int u = decltype(u_tag)::value;            // ring slot: a constant
    constexpr bool WARM = decltype(warm_tag)::value;     // the first block: r = u
    const int q = q0 + r;
    int va = detach(pa[u & 3]), vb = detach(pb[u & 3]);
    if (PATCHED) {
      va = va <= kthr ? detach(ppa[u & 3]) : va;
      vb = vb <= kthr ? detach(ppb[u & 3]) : vb;
    }
    fetch(r + 4, u & 3);
    if (q >= 0 && q < H) {
      if (!PATCHED && __ballot((ina && va <= kthr) || (inb && vb <= kthr)) != 0) {
        // row q is an input row of quarter k when k*QR - 4 <= q - ty0 < (k+1)*QR + 4
        const int rel = q - ty0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (rel >= k * (TH / 4) - 4 && rel < (k + 1) * (TH / 4) + 4) qmask |= 1u << k;
        if (rel >= 0 && rel < TH && q < H) {
          // empty output cells of this row: count them per quarter and
          // list the first kCellEmpty of each quarter (y * W + x)
          const bool ea = outa && va <= kthr, eb = outb && vb <= kthr;
          const unsigned long long ma = __ballot(ea), mb = __ballot(eb);
          const unsigned long long below = (1ull << lane) - 1ull;
          const int k = rel / (TH / 4);
          int base = 0;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            if (kk == k) base = qempty[kk];
          const int ja = base + __popcll(ma & below), jb = base + __popcll(ma) + __popcll(mb & below);
          if (ea && ja < kCellEmpty) s_cells[k * kCellEmpty + ja] = q * W + ca;
          if (eb && jb < kCellEmpty) s_cells[k * kCellEmpty + jb] = q * W + cb;
          const int n_e = __popcll(ma) + __popcll(mb);
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            if (kk == k) qempty[kk] += n_e;
        }
      }
      if ((last == 5 || last == 6) && q >= ty0 && q < ty0 + TH) {
        const unsigned ro = (unsigned)q * W4;
        if (outa) stk(out, ro + ua, va);
        if (outb) stk(out, ro + ub, vb);
      }
    }
    if (median) {
      window_update(Sa, raw[(u - 5) & 7][0], va);
      window_update(Sb, raw[(u - 5) & 7][1], vb);
    }
    raw[u][0] = va;
    raw[u][1] = vb;
    if (WARM && u < 4) return;

    // Stage 7: median of row m = q - 2.
    const int m = q - 2;
    int v7a, v7b;
    if (median) {
      int Lb[5], La[5], Rb[5], m1[10], m2[10], core[6];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        Lb[k] = from_prev(Sb[k]);   // column a - 1
        La[k] = from_prev(Sa[k]);   // column a - 2
        Rb[k] = from_next(Sb[k]);   // column b + 2
      }
      net::merge5_5(Lb, Sa, m1);    // columns a - 1, a
#pragma unroll
      for (int k = 0; k < 10; ++k) m2[k] = from_next(m1[k]);   // columns b, b + 1
      net::ranks7_12_of_10_10(m1, m2, core);
      net::rank5_of_6_5(core, La, &v7a);
      net::rank5_of_6_5(core, Rb, &v7b);
    } else {
      v7a = raw[(u - 2) & 7][0];
      v7b = raw[(u - 2) & 7][1];
    }
    if (edge_cols) {   // out-of-image columns take the median of their reflect-101 column
      const int fa0 = __shfl(v7a, sla), fa1 = __shfl(v7b, sla);
      const int fb0 = __shfl(v7a, slb), fb1 = __shfl(v7b, slb);
      if (!ina) v7a = sela ? fa1 : fa0;
      if (!inb) v7b = selb ? fb1 : fb0;
    }
    s7[u][0] = v7a;
    s7[u][1] = v7b;
    if (last == 7 && m >= ty0 && m < ty0 + TH && m < H && m >= 0) {
      const unsigned ro = (unsigned)m * W4;
      if (outa) stk(out, ro + ua, v7a);
      if (outb) stk(out, ro + ub, v7b);
    }

    // Stage 8: horizontal sums of row m (reflect-101 rows are copies).
    if (m >= 0 && m < H) {
      const int La = from_prev(v7a), Lb = from_prev(v7b), Ra = from_next(v7a), Rb = from_next(v7b);
      hs[u][0] = hsum5(wc, w1, w2, La, Lb, v7a, v7b, Ra);
      hs[u][1] = hsum5(wc, w1, w2, Lb, v7a, v7b, Ra, Rb);
    }
    if (m == 2 && q0 + 2 <= 0) {         // rows -1, -2 mirror rows 1, 2
      hs[(u - 3) & 7][0] = hs[(u - 1) & 7][0];
      hs[(u - 3) & 7][1] = hs[(u - 1) & 7][1];
      hs[(u - 4) & 7][0] = hs[u][0];
      hs[(u - 4) & 7][1] = hs[u][1];
    } else if (m == H) {                        // row H mirrors H - 2
      hs[u][0] = hs[(u - 2) & 7][0];
      hs[u][1] = hs[(u - 2) & 7][1];
    } else if (m == H + 1) {                    // row H + 1 mirrors H - 3
      hs[u][0] = hs[(u - 4) & 7][0];
      hs[u][1] = hs[(u - 4) & 7][1];
    }
    if (WARM) return;

    // Stages 8 and 9 for row g = q - 4.
    const int g = q - 4;
    if (g >= ty0 && g < ty0 + TH && g < H && last >= 8) {
      const int ca7 = s7[(u - 2) & 7][0], cb7 = s7[(u - 2) & 7][1];
      const bool ma = ca7 > kthr, mb = cb7 > kthr;
      float oa, ob;
      if (kp.rg > 0) {
        const double ga = fma(wc, hs[(u - 2) & 7][0],
                              fma(w1, hs[(u - 3) & 7][0] + hs[(u - 1) & 7][0],
                                  w2 * (hs[(u - 4) & 7][0] + hs[u][0])));
        const double gb = fma(wc, hs[(u - 2) & 7][1],
                              fma(w1, hs[(u - 3) & 7][1] + hs[(u - 1) & 7][1],
                                  w2 * (hs[(u - 4) & 7][1] + hs[u][1])));
        oa = ma ? (float)(ga * gsc) : 0.f;
        ob = mb ? (float)(gb * gsc) : 0.f;
      } else {
        oa = ma ? val(ca7) : 0.f;
        ob = mb ? val(cb7) : 0.f;
      }
      if (last == 9) {
        oa = ma ? off - oa : 0.f;
        ob = mb ? off - ob : 0.f;
      }
      const unsigned ro = (unsigned)g * W4;
      if (outa) stk(out, ro + ua, key(oa));
      if (outb) stk(out, ro + ub, key(ob));
    }
  };

  // The first block fills the windows (rows q0 .. q0 + 7); n is a multiple
  // of 8, so every later block is whole.
  static_assert(TH % 8 == 0, "tile rows");
  auto block = [&](const int rb, auto warm_tag) __attribute__((always_inline)) {
    for_slots([&](auto u_tag) __attribute__((always_inline)) { step(u_tag, rb + decltype(u_tag)::value, warm_tag); });
  };
  block(0, std::true_type{});
  for (int rb = 8; rb < n; rb += 8) block(rb, std::false_type{});
  // Quarters whose median and blur inputs still hold an empty pixel need the
  // 31x31 fill and a second pass: queue them (tile id in the low 27 bits,
  // quarter above), and queue the empty cells of those with few of them.
  if (!PATCHED && kp.extrapolate && qmask != 0) {
    __syncthreads();                                 // the cell lists are complete
    // One atomic per queue and tile: thousands of tiles push at once on
    // frames with large holes, and atomics on one address serialise.
    unsigned dmask = 0, smask = 0;
    int ncell = 0;
#pragma unroll
    for (int qk = 0; qk < 4; ++qk) {
      if (((qmask >> qk) & 1u) == 0) continue;
      if (qempty[qk] > kCellEmpty) {
        dmask |= 1u << qk;
      } else {
        smask |= 1u << qk;
        ncell += qempty[qk];
      }
    }
    int ps = 0, pd = 0, pc = 0;
    if (lane == 0) {
      if (smask) ps = atomic_add_g(slow + 0, __popc(smask));
      if (dmask) pd = atomic_add_g(slow + 2, __popc(dmask));
      if (ncell) pc = atomic_add_g(slow + 3, ncell);
    }
    ps = __shfl(ps, 0);
    pd = __shfl(pd, 0);
    pc = __shfl(pc, 0);
    // (the bounds hold when every tile is visited once after a reset; a
    // repeated launch without one drops entries instead of overrunning)
    if (lane < 4 && ((qmask >> lane) & 1u)) {
      const unsigned below = (1u << lane) - 1u;
      const bool dense = (dmask >> lane) & 1u;
      const int pos = dense ? pd + __popc(dmask & below) : ps + __popc(smask & below);
      if (pos < 4 * cap) {
        gint* e = gw(slow) + (dense ? dense_queue_offset(cap) : sparse_queue_offset(cap)) + 2 * pos;
        e[0] = fidx;
        e[1] = gt | (lane << 27);
      }
    }
    gint* cells = gw(slow) + cell_queue_offset(cap);
#pragma unroll
    for (int qk = 0; qk < 4; ++qk) {
      if (((smask >> qk) & 1u) == 0) continue;
      const int ne = qempty[qk];
      if (lane < ne && pc + lane < 4 * kCellEmpty * cap) {
        cells[2 * (pc + lane)] = fidx;
        cells[2 * (pc + lane) + 1] = s_cells[qk * kCellEmpty + lane];
      }
      pc += ne;
    }
  }
}


// Stages 5, 7, 8 and 9 of one streaming tile of the default chain (TH x 120
// output cells), two rows per step.  The 31x31 fill of stage 6 already ran
// ahead of this pass and left its values, tagged, in the stage-4 map.
//
// The median sorts rows first.  Each input row's 5-wide windows are sorted
// across the lane's two columns and its neighbours' (mr::row_windows); an
// output's five sorted row windows are then merged down the rows in
// registers.  A step takes input rows q and q + 1 and gives the medians of
// rows q - 2 and q - 1, which share rows q - 3 .. q: the pair merges of rows
// (q - 3, q - 2) (from the step before) and (q - 1, q), and ranks 7..12 of
// those 20 values; each median adds its fifth row (q - 4 or q + 1) to them.
// The Gaussian's horizontal sums of the two median rows go to a ring, and the
// outputs of rows q - 4 and q - 3 leave with their vertical sums.
//
// Rows outside the frame are the replicated border rows the clamped loads
// give (the median's border rule); the Gaussian's reflected rows (-1, -2
// and H, H + 1) are copies of its sums of rows 1, 2 and H - 2, H - 3, and
// its reflected columns come from the lanes that hold them.  INTERIOR tiles
// need none of these rows.
//
// Rows above the extension's reach: in a column with a top, every stage-5
// row at or above the top holds the top cell's value (Sec. III "Extension
// to Top of Frame"), and the fill leaves such non-empty cells alone.  An
// output row g whose median and blur windows (rows g - 4 .. g + 4) lie at or
// above the top of every column the wave reads therefore sees five equal
// rows: its median is the middle of the row's sorted 5-window, its blur is
// 16 times the row's horizontal sum, and every such row of the tile has the
// same outputs.  They are computed once from the top cells and stored to
// those rows; the streaming loop runs over the remaining rows (a multiple
// of 8, from the tile's end) only.
template <int TH, bool INTERIOR, bool PAIR>
__device__ __forceinline__ void rows_first_tile(const FrameDesc& f, const KParams& kp, int ty0, int tx0, int lane) {
  static_assert(TH % 8 == 0, "tile rows");
  const int H = f.H, W = f.W;
  const float off = kp.off;
  const int kthr = key(kp.thr);
  const int ca = tx0 - 4 + 2 * lane, cb = ca + 1;
  const int xa = clampi_s(ca, 0, W - 1), xb = clampi_s(cb, 0, W - 1);     // replicated border columns
  const unsigned oxa = 4u * (unsigned)xa, oxb = 4u * (unsigned)xb;
  const bool ina = ca >= 0 && ca < W, inb = cb >= 0 && cb < W;
  const bool lane_out = lane >= 2 && lane < 62;
  const bool outa = lane_out && ina, outb = lane_out && inb;
  const unsigned ua = 4u * (unsigned)ca, ub = ua + 4u;   // byte offsets, used only when in the image
  const bool edge_cols = tx0 - 4 < 0 || tx0 + kGlobalTW + 4 > W;
  gcint* v4 = gc(f.v4);
  gint* out = gw(f.out);
  const unsigned W4 = 4u * (unsigned)W;
  // output row stores: with PAIR (even W: a lane's two columns are an 8-byte
  // aligned pair, in or out of the frame together) one 8-byte store per lane
  const __amdgpu_buffer_rsrc_t orsrc = __builtin_amdgcn_make_buffer_rsrc((void*)f.out, (short)0, -1, kBufferWord3);
  auto put = [&](unsigned ro, int va, int vb) __attribute__((always_inline)) {
    if constexpr (PAIR) {
      if (outa) {
        u32x2 v;
        v.x = (unsigned)va;
        v.y = (unsigned)vb;
        __builtin_amdgcn_raw_buffer_store_b64(v, orsrc, (int)ua, (int)ro, 0);
      }
    } else {
      if (outa) stk(out, ro + ua, va);
      if (outb) stk(out, ro + ub, vb);
    }
  };
  // Stage 5 on load: a row above its column's top reads the top cell,
  // V5[y][x] = V4[max(y, top)][x]; as byte offsets, the larger of the row's
  // and the top cell's (0 without a top or without the extension).
  unsigned toffa = 0, toffb = 0;
  int sky = 0;                          // rows from 0 whose outputs are the sky row's (see above)
  if (kp.extrapolate) {
    gcint* top = gc(f.top);
    const int t_a = top[xa], t_b = top[xb];
    if (t_a < H) toffa = (unsigned)t_a * W4 + oxa;
    if (t_b < H) toffb = (unsigned)t_b * W4 + oxb;
    // the least top over the wave's columns (0 if a column has none)
    const int mine = (t_a < H && t_b < H) ? min(t_a, t_b) : 0;
    sky = 0x7fffffff - wave_max_nonneg(0x7fffffff - mine) - 3;   // rows g < least top - 3
  }
  // output rows ty0 .. r_start - 1 are sky rows; the loop covers r_start ..
  // ty0 + TH - 1, a multiple of 8 rows
  int r_start = ty0;
  if (sky > ty0) r_start = ty0 + TH - 8 * ((ty0 + TH - min(sky, ty0 + TH) + 7) / 8);
  // reflect-101 source lane/slot of this lane's columns, for the Gaussian's border
  int sla = 0, slb = 0;
  bool sela = false, selb = false;
  if (edge_cols) {
    auto refl = [&](int c) {
      if (c < 0) c = -c;
      if (c >= W) c = 2 * W - 2 - c;
      return c;
    };
    const int sa = refl(ca) - (tx0 - 4), sb = refl(cb) - (tx0 - 4);
    sla = clampi_s(sa >> 1, 0, kLanes - 1);
    slb = clampi_s(sb >> 1, 0, kLanes - 1);
    sela = (sa & 1) != 0;
    selb = (sb & 1) != 0;
  }
  if (r_start > ty0) {
    // the sky row: the top cells' values, their row medians and blur
    const int a0 = ldk(v4, toffa) & ~kFillTag, b0 = ldk(v4, toffb) & ~kFillTag;
    const int c0[6] = {from_prev(a0), from_prev(b0), a0, b0, from_next(a0), from_next(b0)};
    int Wa[5], Wb[5];
    mr::row_windows(c0, Wa, Wb);
    int ea = Wa[2], eb = Wb[2];                    // medians of five equal rows
    const bool ma = ea > kthr, mb = eb > kthr;     // (masks of the in-image columns)
    if (edge_cols) {
      const int fa = __shfl(ea, sla), fb = __shfl(eb, sla), ga = __shfl(ea, slb), gb = __shfl(eb, slb);
      if (!ina) ea = sela ? fb : fa;
      if (!inb) eb = selb ? gb : ga;
    }
    const int La = from_prev(ea), Lb = from_prev(eb), Ra = from_next(ea), Rb = from_next(eb);
    const double ha = hsum5(6.0, 4.0, 1.0, La, Lb, ea, eb, Ra), hb = hsum5(6.0, 4.0, 1.0, Lb, ea, eb, Ra, Rb);
    // the vertical taps sum to 16: (16 h) / 256 = h / 16, exactly
    const int oa = key(ma ? off - (float)(ha * (1.0 / 16.0)) : 0.f);
    const int ob = key(mb ? off - (float)(hb * (1.0 / 16.0)) : 0.f);
    for (int g = ty0; g < r_start; ++g) put((unsigned)g * W4, oa, ob);
    if (r_start == ty0 + TH) return;
  }
  const int q0 = r_start - 4;           // first input row; step s takes rows q0 + 2s, q0 + 2s + 1

  int Fw[2][2][5];      // sorted row windows of the first rows of the last two steps (by step parity)
  int Rp[2][5];         // sorted row windows of the previous step's second row
  int Pp[2][10];        // the previous step's pair merge
  int mk[2][2];         // medians of the previous step's rows: the output mask
  double hs[8][2];      // Gaussian horizontal sums of median rows, slot (row - q0) & 7
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int k = 0; k < 5; ++k) Fw[0][c][k] = Fw[1][c][k] = Rp[c][k] = 0;
#pragma unroll
    for (int k = 0; k < 10; ++k) Pp[c][k] = 0;
    mk[0][c] = mk[1][c] = 0;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) hs[k][0] = hs[k][1] = 0.0;

  // rows of the stage-4 map (border rows replicated), the extension applied,
  // fetched two steps ahead of their use
  int pa[4], pb[4];
  auto fetch = [&](int r, int slot) {
    const unsigned rowoff = (unsigned)clampi_s(q0 + r, 0, H - 1) * W4;
    pa[slot] = ldk(v4, max(rowoff + oxa, toffa));
    pb[slot] = ldk(v4, max(rowoff + oxb, toffb));
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) fetch(u, u);

  auto hsum = [&](int ma, int mb, double& ha, double& hb) __attribute__((always_inline)) {
    // binomial taps (1 4 6 4 1) as integers: exact in float64
    const int La = from_prev(ma), Lb = from_prev(mb), Ra = from_next(ma), Rb = from_next(mb);
    ha = hsum5(6.0, 4.0, 1.0, La, Lb, ma, mb, Ra);
    hb = hsum5(6.0, 4.0, 1.0, Lb, ma, mb, Ra, Rb);
  };
  auto vsum = [&](double m2, double m1, double c, double p1, double p2) __attribute__((always_inline)) {
    return fma(6.0, c, fma(4.0, m1 + p1, m2 + p2));
  };

  // Step s (slot u = s mod 4; WARM: the first four steps, which give no
  // output row): r = 2s is the step's first input row relative to q0.
  auto step = [&](auto u_tag, const int r, auto warm_tag) __attribute__((always_inline)) {
    constexpr int u = decltype(u_tag)::value;
    constexpr bool WARM = decltype(warm_tag)::value;
    constexpr int s0 = (2 * u) & 3, s1 = (2 * u + 1) & 3;
    const int q = q0 + r;
    // cells the fill ahead of this pass completed carry kFillTag
    const int a0 = detach(pa[s0]) & ~kFillTag, b0 = detach(pb[s0]) & ~kFillTag;
    const int a1 = detach(pa[s1]) & ~kFillTag, b1 = detach(pb[s1]) & ~kFillTag;
    fetch(r + 4, s0);
    fetch(r + 5, s1);
    // sorted 5-wide row windows of rows q and q + 1 at the lane's columns
    int W0[2][5], W1[2][5];
    {
      const int c0[6] = {from_prev(a0), from_prev(b0), a0, b0, from_next(a0), from_next(b0)};
      const int c1[6] = {from_prev(a1), from_prev(b1), a1, b1, from_next(a1), from_next(b1)};
      mr::row_windows(c0, W0[0], W0[1]);
      mr::row_windows(c1, W1[0], W1[1]);
    }
    if (!(WARM && u == 0)) {
      int Pn[2][10];
#pragma unroll
      for (int c = 0; c < 2; ++c) net::merge5_5(Rp[c], W0[c], Pn[c]);   // rows q - 1, q
      if (!(WARM && u == 1)) {
        // Stage 7: medians of rows q - 2 and q - 1
        int m0[2], m1[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          int K[6];
          net::ranks7_12_of_10_10(Pp[c], Pn[c], K);            // rows q - 3 .. q
          m0[c] = mr::median_of_core(K, Fw[u & 1][c]);          // + row q - 4
          m1[c] = mr::median_of_core(K, W1[c]);                 // + row q + 1
        }
        // Stage 8: horizontal sums of the two median rows (out-of-image
        // columns take their reflect-101 column's median)
        int e0a = m0[0], e0b = m0[1], e1a = m1[0], e1b = m1[1];
        if (edge_cols) {
          const int f0a = __shfl(e0a, sla), f0b = __shfl(e0b, sla), g0a = __shfl(e0a, slb), g0b = __shfl(e0b, slb);
          const int f1a = __shfl(e1a, sla), f1b = __shfl(e1b, sla), g1a = __shfl(e1a, slb), g1b = __shfl(e1b, slb);
          if (!ina) { e0a = sela ? f0b : f0a; e1a = sela ? f1b : f1a; }
          if (!inb) { e0b = selb ? g0b : g0a; e1b = selb ? g1b : g1a; }
        }
        hsum(e0a, e0b, hs[(u * 2 + 6) & 7][0], hs[(u * 2 + 6) & 7][1]);   // row q - 2: slot r - 2
        hsum(e1a, e1b, hs[(u * 2 + 7) & 7][0], hs[(u * 2 + 7) & 7][1]);   // row q - 1: slot r - 1
        if (!INTERIOR) {
          // reflected rows: H mirrors H - 2, H + 1 mirrors H - 3
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int m = q - 2 + k;
            double* h = hs[(u * 2 + 6 + k) & 7];
            if (m == H) { h[0] = hs[(u * 2 + 4 + k) & 7][0]; h[1] = hs[(u * 2 + 4 + k) & 7][1]; }
            else if (m == H + 1) { h[0] = hs[(u * 2 + 2 + k) & 7][0]; h[1] = hs[(u * 2 + 2 + k) & 7][1]; }
          }
          // rows -2 and -1 mirror rows 2 and 1 (ready once rows 2 and 3 are in)
          if (r_start == 0 && q == 4) {
            hs[(u * 2 + 2) & 7][0] = hs[(u * 2 + 6) & 7][0];
            hs[(u * 2 + 2) & 7][1] = hs[(u * 2 + 6) & 7][1];
            hs[(u * 2 + 3) & 7][0] = hs[(u * 2 + 5) & 7][0];
            hs[(u * 2 + 3) & 7][1] = hs[(u * 2 + 5) & 7][1];
          }
        }
        if (!WARM) {
          // Stages 8 and 9 for rows q - 4 and q - 3: the vertical sums, the
          // mask of the median rows, the output inversion
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int g = q - 4 + k;
            if (INTERIOR || g < H) {
              const int sl = u * 2 + 4 + k;      // slot of row g
              const double ga = vsum(hs[(sl - 2) & 7][0], hs[(sl - 1) & 7][0], hs[sl & 7][0], hs[(sl + 1) & 7][0],
                                     hs[(sl + 2) & 7][0]);
              const double gb = vsum(hs[(sl - 2) & 7][1], hs[(sl - 1) & 7][1], hs[sl & 7][1], hs[(sl + 1) & 7][1],
                                     hs[(sl + 2) & 7][1]);
              const bool ma = mk[k][0] > kthr, mb = mk[k][1] > kthr;
              const float oa = ma ? off - (float)(ga * (1.0 / 256.0)) : 0.f;
              const float ob = mb ? off - (float)(gb * (1.0 / 256.0)) : 0.f;
              put((unsigned)g * W4, key(oa), key(ob));
            }
          }
        }
        mk[0][0] = m0[0];
        mk[0][1] = m0[1];
        mk[1][0] = m1[0];
        mk[1][1] = m1[1];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < 10; ++k) Pp[c][k] = Pn[c][k];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        Fw[u & 1][c][k] = W0[c][k];
        Rp[c][k] = W1[c][k];
      }
  };

  // four steps (eight rows) per block; the first block only fills the
  // windows, the ring and the mask (TH / 2 + 4 steps in all)
  auto block = [&](const int rb, auto warm_tag) __attribute__((always_inline)) {
    step(std::integral_constant<int, 0>{}, rb, warm_tag);
    step(std::integral_constant<int, 1>{}, rb + 2, warm_tag);
    step(std::integral_constant<int, 2>{}, rb + 4, warm_tag);
    step(std::integral_constant<int, 3>{}, rb + 6, warm_tag);
  };
  block(0, std::true_type{});
  for (int rb = 8; rb < ty0 + TH - r_start + 8; rb += 8) block(rb, std::false_type{});
}

// Phase 2 of chains other than the default one (the stage hooks 5-9 among
// them): one TH x 120 tile per wave and pass.
template <int TH>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(4))) void k_global_stream(FrameSource src, KParams kp) {
  __shared__ int s_cells[4 * kCellEmpty];
  const int lane = threadIdx.x;
  const int total = src.plan ? src.plan->gtiles : src.single_gtiles;
  int32_t* slow = src.plan ? src.plan->slow : src.slow;
  const int cap = src.plan ? src.plan->slow_cap : src.slow_cap;
  for (int t = xcd_tile_s(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
    FrameDesc f;
    int fidx = 0;
    if (src.plan) {
      fidx = gc(src.plan->gtab)[t];
      f = plan_frame(src, fidx);
    } else {
      f = src.single;
    }
    f = uniform_frame(f);
    const int gt = t - f.gtile0;
    const int tr = gt / f.gcols;
    const int ty0 = tr * TH, tx0 = (gt - tr * f.gcols) * kGlobalTW;
    global_stream_tile<TH, false>(f, kp, t, fidx, gt, ty0, tx0, lane, slow, cap, s_cells);
  }
}

// Phase 2 of the default chain (rows_first_tile): tiles whose rows all lie
// away from the frame's first and last two rows take the variant without the
// Gaussian's reflected rows.  Frames under 3 rows or columns go to the LDS
// kernel.  Up to 168 registers (three waves per SIMD): the row windows,
// the pair merge and the ring of sums stay in registers.
template <int TH>
// (four waves per workgroup, one tile each, as k_local_stream)
__global__ __launch_bounds__(kLanes * kLocalWaves) __attribute__((amdgpu_waves_per_eu(3))) void k_global_rows(FrameSource src, KParams kp) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = uni((int)threadIdx.x / kLanes);
  const int total = src.plan ? src.plan->gtiles : src.single_gtiles;
  int32_t* slow = src.plan ? src.plan->slow : src.slow;
  const int cap = src.plan ? src.plan->slow_cap : src.slow_cap;
  // A batch of frames of one shape is visited bottom tile row first, over
  // all frames, its workgroups going to the XCDs in turn: the top tile rows
  // lie above the column tops, where a tile only copies the sky row's
  // outputs, so the last tiles handed out, which run while the SIMDs empty,
  // are cheap ones on every XCD.  Other launches go frame by frame, each
  // XCD taking a contiguous run of tiles.
  const int grows = src.plan ? src.plan->g_rows_same : 0;
  const int gcols = src.plan ? src.plan->g_cols_same : 0;
  const int b0 = grows ? (int)blockIdx.x : xcd_tile_s(blockIdx.x, gridDim.x);
  for (int t = b0 * kLocalWaves + wave; t < total; t += gridDim.x * kLocalWaves) {
    FrameDesc f;
    int tr, tc;
    if (grows) {
      const int per_row = src.plan->n * gcols;        // tiles of one tile row over all frames
      const int k = t / per_row, rem = t - k * per_row;
      const int fi = rem / gcols;
      f = uniform_frame(plan_frame(src, fi));
      tr = grows - 1 - k;
      tc = rem - fi * gcols;
    } else {
      f = uniform_frame(src.plan ? plan_frame(src, gc(src.plan->gtab)[t]) : src.single);
      const int gt = t - f.gtile0;
      tr = gt / f.gcols;
      tc = gt - tr * f.gcols;
    }
    const int ty0 = tr * TH, tx0 = tc * kGlobalTW;
    if (f.H < 3 || f.W < 3) {
      if (lane == 0) {
        const int pos = atomic_add_g(slow + 1, 1);
        if (pos < cap) gw(slow)[lds_queue_offset(cap) + pos] = t;
      }
    } else if (ty0 >= 4 && ty0 + TH + 2 <= f.H) {
      if (pair_ok(f.W, f.out)) rows_first_tile<TH, true, true>(f, kp, ty0, tx0, lane);
      else rows_first_tile<TH, true, false>(f, kp, ty0, tx0, lane);
    } else {
      if (pair_ok(f.W, f.out)) rows_first_tile<TH, false, true>(f, kp, ty0, tx0, lane);
      else rows_first_tile<TH, false, false>(f, kp, ty0, tx0, lane);
    }
  }
}

// Phase 2, queued cells, step 1 (Sec. III "Large Hole Fill"): a cell empty
// after stage 5 takes the largest stage-5 value of the full (2 rl + 1)^2
// window around it (cells outside the image ignored).  One wave per cell:
// lane l covers window column (l mod 32) - rl and, for l < 32, the window
// rows -rl .. -rl + 15, else the next 16, so every load instruction reads
// two short row segments; a wave-wide max reduces the lanes.  The value
// goes to f.v6p at the cell only, so the stage-5 reads of other waves are
// unaffected.
constexpr int kFillRad = 15;   // largest large-fill radius (31x31)

// The largest stage-5 key of the (2 rl + 1)^2 window around cell (y, x),
// in every lane of the wave (cells outside the image ignored; cells the
// fill ahead of phase 2 already wrote carry kFillTag, a negative key, and
// count as empty).  Lane l covers window column (l mod 32) - rl and, for
// l < 32, the window rows -rl .. -rl + 15, else the next 16.
__device__ __forceinline__ int window_max(const FrameDesc& f, const KParams& kp, int y, int x, int lane) {
  const int H = f.H, W = f.W, rl = kp.rl;
  const int dx = (lane & 31) - rl;
  const bool colw = (lane & 31) <= 2 * rl;
  const int dy0 = 16 * (lane >> 5) - rl;
  gcint* v4 = gc(f.v4);
  const int gx = x + dx;
  const bool colin = colw && gx >= 0 && gx < W;
  const int xc = clampi_s(gx, 0, W - 1);
  const int tt = kp.extrapolate ? gc(f.top)[xc] : H;   // stage 5: rows above the top read the top
  int w[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int yc = clampi_s(y + dy0 + k, 0, H - 1);
    w[k] = v4[(size_t)v5_row(yc, tt, H, kp.ext_rows) * W + xc];
  }
  int m = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int gy = y + dy0 + k;
    m = max(m, (colin && dy0 + k <= rl && gy >= 0 && gy < H) ? w[k] : 0);
  }
  return wave_max_nonneg(m);
}

__global__ __launch_bounds__(kLanes) void k_fill_cells(FrameSource src, KParams kp) {
  const int lane = threadIdx.x;
  gcint* slow = gc(src.plan ? src.plan->slow : src.slow);
  const int cap = src.plan ? src.plan->slow_cap : src.slow_cap;
  const int count = min(slow[3], 4 * kCellEmpty * cap);
  gcint* cells = slow + cell_queue_offset(cap);
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const int fidx = cells[2 * i], pos = cells[2 * i + 1];
    FrameDesc f = src.plan ? plan_frame(src, fidx) : src.single;
    f = uniform_frame(f);
    const int W = f.W;
    const int y = uni(pos / W), x = uni(pos - (pos / W) * W);
    const int m = window_max(f, kp, y, x, lane);
    if (lane == 0) gw(f.v6p)[(size_t)pos] = m;
  }
}

// Van Herk/Gil-Werman running max of width 31: out[j] = max(a[j .. j+30])
// for 32 outputs from 62 inputs (prefix maxima of one block, suffix maxima
// of the other).
__device__ __forceinline__ void vhgw31(const int* a, int* out) {
  int suf[31], pre[31];
  suf[30] = a[30];
#pragma unroll
  for (int k = 29; k >= 0; --k) suf[k] = max(a[k], suf[k + 1]);
  pre[0] = a[31];
#pragma unroll
  for (int k = 1; k < 31; ++k) pre[k] = max(pre[k - 1], a[31 + k]);
  out[0] = suf[0];
#pragma unroll
  for (int j = 1; j < 31; ++j) out[j] = max(suf[j], pre[j - 1]);
  out[31] = pre[30];
}

// The fill computed separably for a region of nr <= QR rows (from y0) and
// ncols <= 128 columns (from x0) by a workgroup of four waves.  The stage-5
// values of the region's rows +- rl and columns +- rl go to LDS (cells
// outside the image and tagged cells as 0, which no max selects over a
// non-empty value); their horizontal window maxima (van Herk/Gil-Werman for
// the 31-wide window) replace them in place; each cell of the region that is
// empty after stage 5 takes the vertical max of those (for the 31-row window:
// the rows all the region's windows share, then the prefix and suffix maxima
// at both ends) and is handed to out(y, x, value).  TOPS: the caller has
// already put the tops of the staged columns (x0 - rl + i, clamped into the
// image) in s_top and passed a barrier since, and no thread still reads S.
constexpr int kDW = kGlobalTW + 2 * kFillRad + 8;    // 158 staged columns (4 runs of 32 outputs + 30)
constexpr int kDenseThreads = 256;

template <int QR, bool TOPS, class Out>
__device__ __forceinline__ void fill_region(const FrameDesc& f, const KParams& kp, int y0, int nr, int x0, int ncols,
                                            int* S, int* s_top, int tid, Out&& out) {
  static_assert(QR + 2 * kFillRad <= kLanes, "one staged row per lane for the horizontal maxima");
  const int H = f.H, W = f.W, rl = kp.rl;
  const int kthr = key(kp.thr);
  gcint* v4 = gc(f.v4);
  const int sr = nr + 2 * rl;
  if constexpr (!TOPS) {
    __syncthreads();                                  // LDS of the previous region is no longer read
    if (tid < kDW) {                                  // column tops of the staged columns (>= H: none)
      const int x = clampi_s(x0 - rl + tid, 0, W - 1);
      s_top[tid] = kp.extrapolate ? gc(f.top)[x] : H;
    }
    __syncthreads();
  }
  {
    // Each thread stages whole runs of one column, so the column's clamped x,
    // its top and whether it lies in the image are worked out once: columns
    // 0 .. 127 by all threads (two halves of the rows), the remaining
    // kDW - 128 columns by groups of threads over slices of RB rows.
    // Rows past sr load a clamped cell and are not stored.
    constexpr int SRM = QR + 2 * kFillRad;
    constexpr int RA = (SRM + 1) / 2;
    constexpr int NB = kDW - 128, GB = kDenseThreads / NB, RB = (SRM + GB - 1) / GB;
    static_assert(kDenseThreads == 256 && NB > 0 && GB * RB >= SRM, "staging split");
    const int ext = kp.ext_rows;
    auto stage = [&](int cc, int r0, auto n_rows) {
      constexpr int N = decltype(n_rows)::value;
      const int gx = x0 - rl + cc;
      const unsigned x4 = 4u * (unsigned)clampi_s(gx, 0, W - 1), W4 = 4u * (unsigned)W;
      const bool colin = gx >= 0 && gx < W;
      // stage 5 reads the top row for rows lo .. top - 1 of the column (none
      // when the column has no top)
      const int top = s_top[cc];
      const int lo = top >= H ? H : (ext > 0 ? max(top - ext, 0) : 0);
      const unsigned span = (unsigned)(min(top, H) - lo);
      const int yb = y0 - rl + r0;
      int v[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int y = clampi_s(yb + k, 0, H - 1);
        const int row = (unsigned)(y - lo) < span ? top : y;
        v[k] = ldk(v4, (unsigned)row * W4 + x4);
      }
#pragma unroll
      for (int k = 0; k < N; ++k)
        if (r0 + k < sr) S[(r0 + k) * kDW + cc] = (colin && (unsigned)(yb + k) < (unsigned)H) ? max(v[k], 0) : 0;
    };
    // (columns from ncols + 2 rl on feed only outputs past ncols, which are
    // not used: they are not staged)
    if ((tid & 127) < ncols + 2 * rl) stage(tid & 127, (tid >> 7) * RA, std::integral_constant<int, RA>{});
    if (tid < GB * NB && 128 + tid % NB < ncols + 2 * rl)
      stage(128 + tid % NB, (tid / NB) * RB, std::integral_constant<int, RB>{});
  }
  __syncthreads();
  // the region's cells that are empty after stage 5, one column per thread
  // (bit r: row y0 + r), taken before the staged values are overwritten
  unsigned emask = 0u;
  if (tid < ncols) {
    for (int r = 0; r < nr; ++r)
      if (S[(rl + r) * kDW + rl + tid] <= kthr) emask |= 1u << r;
  }
  // horizontal window maxima of 128 (>= ncols) columns, written over the
  // staged values once every row has been read
  {
    const int rr = tid & (kLanes - 1), j0 = (tid / kLanes) * 32;   // a wave per run: lanes 158 ints apart
    const bool act = rr < sr && j0 < ncols;
    int o[32];
    if (act) {
      if (rl == kFillRad) {
        int a[62];
#pragma unroll
        for (int c = 0; c < 62; ++c) a[c] = S[rr * kDW + j0 + c];
        vhgw31(a, o);
      } else {
#pragma unroll
        for (int c = 0; c < 32; ++c) {
          const int* p = S + rr * kDW + j0 + c;
          int m = p[0];
          for (int d = 1; d <= 2 * rl; ++d) m = max(m, p[d]);
          o[c] = m;
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < 32; ++c) S[rr * kDW + j0 + c] = o[c];
    }
  }
  __syncthreads();
  // vertical max at the empty cells of the region, one column per thread.
  // Row r takes rows r .. r + 2 rl; when 2 rl >= QR - 2 they split into rows
  // r .. QR - 2 (a suffix maximum), QR - 1 .. 2 rl (shared by every row) and
  // 2 rl + 1 .. 2 rl + r (a prefix maximum).  Staged rows past sr only feed
  // rows past nr.
  static_assert(QR <= 32, "one bit per row");
  if (tid < ncols && emask != 0u) {
    const int c = tid;
    const int gx = x0 + c;
    if (2 * rl >= QR - 2) {
      int mid = 0;
      for (int d = QR - 1; d <= 2 * rl; ++d) mid = max(mid, S[d * kDW + c]);
      int lo[QR];
      int acc = 0;
      lo[QR - 1] = 0;
#pragma unroll
      for (int r = QR - 2; r >= 0; --r) {
        acc = max(acc, S[r * kDW + c]);
        lo[r] = acc;
      }
      int hi = 0;
#pragma unroll
      for (int r = 0; r < QR; ++r) {
        if (r > 0) hi = max(hi, S[(2 * rl + r) * kDW + c]);
        if ((emask >> r) & 1u) out(y0 + r, gx, max(max(mid, lo[r]), hi));
      }
    } else {
      for (int r = 0; r < nr; ++r) {
        if (((emask >> r) & 1u) == 0u) continue;
        int m = 0;
        for (int d = 0; d <= 2 * rl; ++d) m = max(m, S[(r + d) * kDW + c]);
        out(y0 + r, gx, m);
      }
    }
  }
}

// Phase 2, queued quarters with many empty cells, step 1: the same fill
// values, computed separably for the whole quarter (fill_region).
template <int TH>
__global__ __launch_bounds__(kDenseThreads) void k_fill_dense(FrameSource src, KParams kp) {
  constexpr int QR = TH / 4, SR = QR + 2 * kFillRad;
  __shared__ int S[SR * kDW];
  __shared__ int s_top[kDW];
  const int tid = threadIdx.x;
  gcint* slow = gc(src.plan ? src.plan->slow : src.slow);
  const int cap = src.plan ? src.plan->slow_cap : src.slow_cap;
  const int count = min(slow[2], 4 * cap);
  gcint* queue = slow + dense_queue_offset(cap);
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const int fidx = queue[2 * i], tq = queue[2 * i + 1];
    const int gt = tq & ((1 << 27) - 1), qk = (unsigned)tq >> 27;
    FrameDesc f = src.plan ? plan_frame(src, fidx) : src.single;
    f = uniform_frame(f);
    const int tr = gt / f.gcols;
    const int y0 = tr * TH + qk * QR, tx0 = (gt - tr * f.gcols) * kGlobalTW;
    const int nr = min(QR, f.H - y0), ncols = min(kGlobalTW, f.W - tx0);
    if (nr <= 0) continue;                      // a quarter past the last row (queued for its input rows)
    gint* v6p = gw(f.v6p);
    const int W = f.W;
    fill_region<QR, false>(f, kp, y0, nr, tx0, ncols, S, s_top, tid,
                    [&](int y, int x, int m) { v6p[(size_t)y * W + x] = m; });
  }
}

// ---------------------------------------------------------------------------
// The fill of stage 6 ahead of phase 2 (the default chain with the streaming
// phase 1).  After phase 1 every column's top is final, so the cells empty
// after stage 5 are known: in a phase-1 tile column they are
//   - the empty rows after its first non-empty row (holes: such rows lie at
//     or below the column's top), and
//   - the rows before its first non-empty row (all of them when there is
//     none) when the column's top lies in a tile above or the column has no
//     top (the extension then leaves them empty).
// Their fill values go into the stage-4 map itself, tagged (kFillTag):
// stage-5 reads of other fills take a tagged cell as empty, as it was, and
// phase 2 reads stage-6 values with the tag cleared.  Every cell belongs to
// one phase-1 tile, whose workgroup alone writes it.

// bits of the bands (kBandRows rows) that rows lo .. hi of a tile touch
__device__ __forceinline__ unsigned band_bits(int lo, int hi) {
  return (2u << (hi / kBandRows)) - (1u << (lo / kBandRows));
}

// The bands of a tile column (rows: the tile's rows in the frame) that hold
// such a cell, given its record, the column's top (>= H: none) and the
// tile's first row: those of its leading rows, and those the record marks
// as holding an empty row after its first non-empty row.
__device__ __forceinline__ unsigned record_bands(int rec, int top, int y0, int rows, int H) {
  const int first = rec & 0xffff;
  unsigned m = 0u;
  if ((top >= H || top < y0) && first != 0) m |= band_bits(0, (first == kRecNone ? rows : first) - 1);
  return m | (((unsigned)rec >> 16) & ((1u << kBandsPerTile) - 1u));
}

// Bitwise or over the wave, as a uniform value (as wave_max_nonneg).
__device__ __forceinline__ unsigned wave_or(unsigned v) {
  int x = (int)v;
  x |= __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);
  x |= __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);
  x |= __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);
  x |= __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);
  x |= __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
  x |= __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
  return (unsigned)__builtin_amdgcn_readlane(x, 63);
}

// One wave per column of phase-1 tiles and group of eight tile rows (the
// waves of the group's first tile row) reads the records of those tiles
// and queues the 32-row bands that may hold such a cell: the launch tile id,
// and the frame index with the band in bits 24..25.  Frames under 3 rows or
// columns are left to phase 2, which recomputes them whole.
__global__ __launch_bounds__(kLanes) void k_fill_scan(FrameSource src, KParams kp, int lth) {
  const int lane = threadIdx.x;
  const int total = src.plan ? src.plan->ltiles : src.single_ltiles;
  int32_t* slow = src.plan ? src.plan->slow : src.slow;
  const int gcap = src.plan ? src.plan->slow_cap : src.slow_cap;
  gint* queue = gw(slow + fill_queue_offset(gcap));
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const int fidx = src.plan ? gc(src.plan->ltab)[t] : 0;
    FrameDesc f = src.plan ? plan_frame(src, fidx) : src.single;
    f = uniform_frame(f);
    const int lt = t - f.ltile0;
    const int H = f.H, W = f.W;
    const int tr0 = lt / f.lcols, tc = lt - tr0 * f.lcols;   // tile row and column
    if ((tr0 & 7) != 0 || H < 3 || W < 3) continue;
    const int x0 = tc * kLocalTW;
    const int xa = x0 + lane, xb = x0 + kLanes + lane;
    const bool ina = xa < W, inb = kLanes + lane < kLocalTW && xb < W;
    const int xac = min(xa, W - 1), xbc = min(xb, W - 1);
    gcint* top = gc(f.top);
    gcint* rec = gc(f.v6p);
    const int ta = top[xac], tb = top[xbc];
    const int ntr = (H + lth - 1) / lth;
    int ra[8], rb[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t row = (size_t)min(tr0 + k, ntr - 1) * W;
      ra[k] = rec[row + xac];
      rb[k] = rec[row + xbc];
    }
    // bands with candidates: four bits per tile row (bit 4 k + b: tile row
    // tr0 + k, band b), or-ed over the tile columns of the wave
    unsigned m = 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int y0 = (tr0 + k) * lth, rows = min(lth, H - y0);
      if (tr0 + k < ntr) {
        const unsigned mk = (ina ? record_bands(ra[k], ta, y0, rows, H) : 0u) |
                            (inb ? record_bands(rb[k], tb, y0, rows, H) : 0u);
        m |= mk << (4 * k);
      }
    }
    const unsigned need = wave_or(m);
    if (need == 0u) continue;   // the next tile
    int pos = 0;
    if (lane == 0) pos = atomic_add_g(slow + 4, __popc(need));
    pos = __shfl(pos, 0) + __popc(need & ((1u << (lane & 31)) - 1u));
    if (lane < 32 && ((need >> lane) & 1u) && pos < kBandsPerTile * total) {
      queue[2 * pos] = f.ltile0 + (tr0 + lane / 4) * f.lcols + tc;
      queue[2 * pos + 1] = fidx | ((lane & 3) << 24);
    }
  }
}

// cells of a band filled one by one; beyond: separably (a staged band costs
// about as much as eight 31x31 windows read cell by cell)
constexpr int kFillSparse = 8;
constexpr int kFillScan = 2048;   // hole rows of a band checked one by one; beyond: separably

// The fill of a band of nr <= kBandRows rows (from y0) and ncols <= 108
// columns (from x0) for the 31x31 window, the vertical maxima first.  Each
// staged column (x0 - 15 + i for i < ncols + 30) loads its 62 rows from
// y0 - 15 into registers (stage 5 applied; cells outside the image and
// tagged cells as 0, which no max selects over a non-empty value), keeps
// the band's empty cells of its column as a bit mask and writes the maxima
// of its 31-row windows at the band's rows to LDS (van Herk/Gil-Werman).
// Each band row holding an empty cell then takes, 32 columns at a time, the
// maxima of 31 of those across and hands the empty cells' values to
// out(y, x, value).  The caller has put the staged columns' tops in s_top,
// set *s_rows to 0 and passed a barrier since; no thread still reads S.
constexpr int kDWV = 159;   // LDS row pitch: odd, so a row pass's lanes (one row each) hit distinct banks
// threads of the 31x31 window's band fill: the 138 staged columns and the
// 128 threads of the row pass fit three waves
constexpr int kVfThreads = 192;
template <class Out>
__device__ __forceinline__ void fill_band_vfirst(const FrameDesc& f, const KParams& kp, int y0, int nr, int x0,
                                                 int ncols, int* S, const int* s_top, unsigned* s_em,
                                                 unsigned* s_rows, int tid, Out&& out) {
  constexpr int R = kFillRad, SRM = kBandRows + 2 * R;
  static_assert(SRM == 62 && kBandRows == 32, "vhgw31 takes 62 values to 32 maxima");
  static_assert(4 * 32 + 2 * R <= kDWV && kLocalTW <= 128 && kLocalTW + 2 * R <= kVfThreads && kVfThreads >= 128,
                "band layout");
  const int H = f.H, W = f.W;
  const int kthr = key(kp.thr);
  gcint* v4 = gc(f.v4);
  if (tid < ncols + 2 * R) {
    const int gx = x0 - R + tid;
    const unsigned x4 = 4u * (unsigned)clampi_s(gx, 0, W - 1), W4 = 4u * (unsigned)W;
    const bool colin = gx >= 0 && gx < W;
    // stage 5 reads the top row for rows lo .. top - 1 of the column (none
    // when the column has no top)
    const int top = s_top[tid];
    const int lo = top >= H ? H : (kp.ext_rows > 0 ? max(top - kp.ext_rows, 0) : 0);
    const unsigned span = (unsigned)(min(top, H) - lo);
    const int yb = y0 - R;
    int a[SRM];
#pragma unroll
    for (int k = 0; k < SRM; ++k) {
      const int y = clampi_s(yb + k, 0, H - 1);
      const int row = (unsigned)(y - lo) < span ? top : y;
      a[k] = ldk(v4, (unsigned)row * W4 + x4);
    }
#pragma unroll
    for (int k = 0; k < SRM; ++k) a[k] = (colin && (unsigned)(yb + k) < (unsigned)H) ? max(a[k], 0) : 0;
    if (tid >= R && tid < R + ncols) {
      unsigned em = 0u;
#pragma unroll
      for (int r = 0; r < kBandRows; ++r)
        if (r < nr && a[R + r] <= kthr) em |= 1u << r;
      s_em[tid - R] = em;
      if (em != 0u) atomicOr(s_rows, em);
    }
    int o[kBandRows];
    vhgw31(a, o);
#pragma unroll
    for (int r = 0; r < kBandRows; ++r) S[r * kDWV + tid] = o[r];
  }
  __syncthreads();
  // band row rr, columns j0 .. j0 + 31: lanes 0-31 of a wave take rows 0-31
  // of one run, lanes 32-63 those of the next
  const unsigned rows = *s_rows;
  const int rr = tid & 31, j0 = (tid >> 5) * 32;
  if (j0 < ncols && ((rows >> rr) & 1u)) {
    int a[62], o[32];
#pragma unroll
    for (int c = 0; c < 62; ++c) a[c] = S[rr * kDWV + j0 + c];
    vhgw31(a, o);
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (j0 + c < ncols && ((s_em[j0 + c] >> rr) & 1u)) out(y0 + rr, x0 + j0 + c, o[c]);
  }
}

// window_max for up to NC cells of one phase-1 tile at once (pos: y * W + x,
// nc of them valid), every load issued before the first is used; the tops
// come from s_top, which holds those of columns xs0 .. xs0 + kDW - 1
// (clamped into the image).
template <int NC>
__device__ __forceinline__ void window_max_n(const FrameDesc& f, const KParams& kp, const int* pos, int nc,
                                             const int* s_top, int xs0, int lane, int* m_out) {
  const int H = f.H, W = f.W, rl = kp.rl;
  const int dx = (lane & 31) - rl;
  const bool colw = (lane & 31) <= 2 * rl;
  const int dy0 = 16 * (lane >> 5) - rl;
  gcint* v4 = gc(f.v4);
  int w[NC][16], yk[NC];
  bool colin[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int p = pos[k < nc ? k : 0];
    const int y = p / W, x = p - y * W;
    const int gx = x + dx;
    yk[k] = y;
    colin[k] = k < nc && colw && gx >= 0 && gx < W;
    const unsigned xc4 = 4u * (unsigned)clampi_s(gx, 0, W - 1);
    const int tt = kp.extrapolate ? s_top[gx - xs0] : H;   // stage 5: rows above the top read the top
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int yc = clampi_s(y + dy0 + i, 0, H - 1);
      w[k][i] = ldk(v4, (unsigned)v5_row(yc, tt, H, kp.ext_rows) * (4u * (unsigned)W) + xc4);
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    int m = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int gy = yk[k] + dy0 + i;
      m = max(m, (colin[k] && dy0 + i <= rl && gy >= 0 && gy < H) ? w[k][i] : 0);
    }
    m_out[k] = wave_max_nonneg(m);
  }
}

// One workgroup per queued band (kBandRows rows of a phase-1 tile).  The
// column records and tops give each column's leading rows and whether holes
// follow its first non-empty row; the hole rows within the band are checked
// cell by cell (all threads over the flattened list of hole-column rows).
// Up to kFillSparse cells then each take the window max (window_max_n, two
// or three per wave at a time); a band with more is filled separably: VF (the 31x31
// window) by fill_band_vfirst, other windows by fill_region.  The fill is
// bound by the latency of a band's dependent steps, so VF, whose band needs
// half the LDS, runs five waves per SIMD (96 registers) rather than four, in
// workgroups of three waves: six bands per CU.  ALL: the launch
// visits every band of every phase-1 tile rather than those k_fill_scan
// queued (small launches, whose bands all fit one round of workgroups: the
// classification above finds the same cells, and the scan would cost a
// launch and a round trip more than the bands it spares).
template <bool VF, bool ALL>
__global__ __launch_bounds__(VF ? kVfThreads : kDenseThreads) __attribute__((amdgpu_waves_per_eu(VF ? 5 : 4))) void k_fill_tiles(FrameSource src, KParams kp, int lth) {
  constexpr int NT = VF ? kVfThreads : kDenseThreads;   // threads of the workgroup
  static_assert(NT >= kDW && NT >= kLocalTW, "a thread per staged column top and per band column");
  constexpr int SR = kBandRows + 2 * kFillRad;
  __shared__ int S[VF ? kBandRows * kDWV : SR * kDW];
  __shared__ int s_top[kDW];
  __shared__ unsigned s_em[VF ? kLocalTW : 1], s_rows;
  __shared__ int s_list[kFillSparse];
  __shared__ short s_hcol[kLocalTW], s_hfirst[kLocalTW];
  __shared__ int s_n, s_lead, s_nh, s_cand;
  const int tid = threadIdx.x, lane = tid & (kLanes - 1), wv = tid / kLanes;
  gcint* slow = gc(src.plan ? src.plan->slow : src.slow);
  const int gcap = src.plan ? src.plan->slow_cap : src.slow_cap;
  const int lcap = src.plan ? src.plan->ltiles : src.single_ltiles;
  const int nbt = (lth + kBandRows - 1) / kBandRows;    // bands per phase-1 tile
  const int count = ALL ? nbt * lcap : min(slow[4], kBandsPerTile * lcap);
  gcint* queue = slow + fill_queue_offset(gcap);
  const int kthr = key(kp.thr);
  const int rl = kp.rl;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    int t, fidx, band;
    if constexpr (ALL) {
      t = i / nbt;
      band = i - t * nbt;
      fidx = src.plan ? gc(src.plan->ltab)[t] : 0;
    } else {
      t = queue[2 * i];
      const int e1 = queue[2 * i + 1];
      fidx = e1 & 0xffffff;
      band = (int)((unsigned)e1 >> 24);
    }
    FrameDesc f = src.plan ? plan_frame(src, fidx) : src.single;
    f = uniform_frame(f);
    const int H = f.H, W = f.W;
    const int lt = t - f.ltile0, tr = lt / f.lcols, tc = lt - tr * f.lcols;
    const int y0 = tr * lth, x0 = tc * kLocalTW;
    const int rows = min(lth, H - y0), cols = min(kLocalTW, W - x0);
    const int b0 = band * kBandRows, b1 = min(b0 + kBandRows, rows);   // the band's rows within the tile
    // (whole workgroup alike, ahead of the band's first barrier) frames
    // under 3 rows or columns are left to phase 2, as the scan leaves them;
    // a tile's last bands may lie past its rows
    if (ALL && (H < 3 || W < 3 || b0 >= rows)) continue;
    gcint* v4 = gc(f.v4);
    gint* v4w = gw(f.v4);
    // tops of the columns x0 - rl .. x0 - rl + kDW - 1 (clamped into the
    // image) and the band's column records, loaded before the barrier so
    // that they are in flight while the previous band's last cells go out
    const int topv = tid < kDW ? (kp.extrapolate ? gc(f.top)[clampi_s(x0 - rl + tid, 0, W - 1)] : H) : 0;
    const int x = x0 + tid;
    const int rec = tid < cols ? gc(f.v6p)[(size_t)tr * W + x] : 0;
    __syncthreads();                                   // LDS of the previous band is no longer read
    if (tid == 0) {
      s_n = 0;
      s_lead = 0;
      s_nh = 0;
      s_cand = 0;
      if constexpr (VF) s_rows = 0u;
    }
    if (tid < kDW) s_top[tid] = topv;
    __syncthreads();
    // this thread's column within the band: leading rows l0 .. l1 - 1 (tile
    // rows), and whether empty rows may follow the first non-empty one
    int l0 = 0, l1 = 0;
    if (tid < cols) {
      const int top = s_top[tid + rl];
      const int first = rec & 0xffff;
      if ((top >= H || top < y0) && first != 0) {
        l0 = b0;
        l1 = min(b1, first == kRecNone ? rows : first);
        if (l1 > l0) atomicAdd(&s_lead, l1 - l0);
      }
      if ((((unsigned)rec >> 16) >> band) & 1u) {     // empty rows after the first non-empty one, in this band
        const int h0 = max(first + 1, b0);
        if (h0 < b1) {
          const int k = atomicAdd(&s_nh, 1);
          s_hcol[k] = (short)tid;
          s_hfirst[k] = (short)h0;
          atomicAdd(&s_cand, b1 - h0);
        }
      }
    }
    __syncthreads();
    bool dense = s_lead > kFillSparse || s_lead + s_cand > kFillScan;
    if (!dense) {
      for (int r = l0; r < l1; ++r) {
        const int j = atomicAdd(&s_n, 1);
        if (j < kFillSparse) s_list[j] = (y0 + r) * W + x;
      }
      // hole rows: the band's rows of every hole column, flattened over the
      // threads, four per thread at a time; a thread stops once the band has
      // more than kFillSparse cells (it is then filled separably)
      const int nh = s_nh, nb = b1 - b0, total = nh * nb;
      for (int base = 0; base < total; base += 4 * NT) {
        if (*(volatile int*)&s_n > kFillSparse) break;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int idx = base + u * NT + tid;
          if (idx < total) {
            const int k = idx / nb, r = b0 + idx - k * nb;
            const int c = s_hcol[k];
            const int y = y0 + r, xx = x0 + c;
            const int v = v4[(size_t)y * W + xx];
            if (r >= s_hfirst[k] && v <= kthr) {
              const int j = atomicAdd(&s_n, 1);
              if (j < kFillSparse) s_list[j] = y * W + xx;
            }
          }
        }
      }
      __syncthreads();
      dense = s_n > kFillSparse;
    }
    if (!dense) {
      // three cells per wave at a time (two in the five-wave build of the
      // 31x31 window's kernel, which would otherwise spill)
      constexpr int NC = VF ? 2 : 3;
      const int n = s_n;
      for (int j0 = wv * NC; j0 < n; j0 += NC * (NT / kLanes)) {
        const int nc = min(NC, n - j0);
        int pos[NC], m[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) pos[k] = uni(s_list[k < nc ? j0 + k : j0]);
        window_max_n<NC>(f, kp, pos, nc, s_top, x0 - rl, lane, m);
        if (lane == 0) {
#pragma unroll
          for (int k = 0; k < NC; ++k)
            if (k < nc && m[k] > 0) v4w[pos[k]] = m[k] | kFillTag;
        }
      }
    } else {
      // s_top holds the staged columns' tops, and S is not read since the
      // barrier at the top of the loop
      auto put = [&](int y, int xx, int m) {
        if (m > 0) v4w[(size_t)y * W + xx] = m | kFillTag;
      };
      if constexpr (VF) fill_band_vfirst(f, kp, y0 + b0, b1 - b0, x0, cols, S, s_top, s_em, &s_rows, tid, put);
      else fill_region<kBandRows, true>(f, kp, y0 + b0, b1 - b0, x0, cols, S, s_top, tid, put);
    }
  }
}

// Phase 2, queued quarters, step 2: median, blur and output inversion of
// the quarter again, with the stage-6 values of step 1.
template <int TH>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(3))) void k_global_patched(FrameSource src, KParams kp) {
  constexpr int QR = TH / 4;
  const int lane = threadIdx.x;
  gcint* slow = gc(src.plan ? src.plan->slow : src.slow);
  const int cap = src.plan ? src.plan->slow_cap : src.slow_cap;
  const int n_sparse = min(slow[0], 4 * cap), count = n_sparse + min(slow[2], 4 * cap);
  if (kp.last_stage == 5) return;                   // the stage-5 map needs no second pass
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    gcint* e = i < n_sparse ? slow + sparse_queue_offset(cap) + 2 * i
                            : slow + dense_queue_offset(cap) + 2 * (i - n_sparse);
    const int fidx = e[0], tq = e[1];
    const int gt = tq & ((1 << 27) - 1), qk = (unsigned)tq >> 27;
    FrameDesc f = src.plan ? plan_frame(src, fidx) : src.single;
    f = uniform_frame(f);
    const int tr = gt / f.gcols;
    global_stream_tile<QR, true>(f, kp, 0, fidx, gt, tr * TH + qk * QR, (gt - tr * f.gcols) * kGlobalTW, lane,
                                       nullptr, 0, nullptr);
  }
}

constexpr int stream_local_rows(int id) {
  return id == 5 ? 64 : id == 6 ? 128 : id == 7 ? 32 : id == 8 ? 16 : id == 9 ? 8 : id == 10 ? 96 : 0;
}
constexpr int stream_global_rows(int id) {
  return id == 5 ? 64 : id == 6 ? 32 : id == 7 ? 128 : id == 8 ? 16 : id == 9 ? 8 : 0;
}


}  // namespace

int stream_local_tile_rows(int id) { return stream_local_rows(id); }
int stream_local_tile_cols(int id) { return stream_local_rows(id) ? kLocalTW : 0; }
int stream_global_tile_rows(int id) { return stream_global_rows(id); }
int stream_global_tile_cols(int id) { return stream_global_rows(id) ? kGlobalTW : 0; }

bool stream_local_supported(int shape, int rd, int rc, int rf) {
  if (rc != 2 || rf != 3) return false;
  if (rd == 2) return true;                      // all four shapes, 5x5
  return shape == 0 && (rd == 1 || rd == 3);      // full 3x3 and 7x7
}

bool stream_global_supported(int rm, int rg) { return (rm == 0 || rm == 2) && rg >= 0 && rg <= 2; }

#define IPB_STREAM_LOCAL(X)                                                          \
  X(2, 2, 5) X(1, 2, 5) X(0, 2, 5) X(3, 2, 5) X(0, 1, 5) X(0, 3, 5) X(2, 2, 6) X(2, 2, 7) \
  X(1, 2, 6) X(0, 2, 6) X(3, 2, 6) X(0, 1, 6) X(0, 3, 6) X(1, 2, 7) X(0, 2, 7) X(3, 2, 7) X(0, 1, 7) X(0, 3, 7) \
  X(2, 2, 8) X(1, 2, 8) X(0, 2, 8) X(3, 2, 8) X(0, 1, 8) X(0, 3, 8) \
  X(2, 2, 9) X(1, 2, 9) X(0, 2, 9) X(3, 2, 9) X(0, 1, 9) X(0, 3, 9) \
  X(2, 2, 10) X(1, 2, 10) X(0, 2, 10) X(3, 2, 10) X(0, 1, 10) X(0, 3, 10)

hipError_t launch_local_stream(const FrameSource& src, const KParams& kp, int tile_id, int grid, hipStream_t s) {
  // grid: one wave per tile; workgroups of kLocalWaves waves, a multiple of
  // the 8 XCDs of them
  const int wgs = ((grid + kLocalWaves - 1) / kLocalWaves + 7) / 8 * 8;
#define X(S, R, ID)                                                                                          \
  if (kp.shape == S && kp.rd == R && tile_id == ID) {                                                        \
    hipLaunchKernelGGL((k_local_stream<S, R, stream_local_rows(ID)>), dim3(wgs), dim3(kLanes * kLocalWaves), 0, \
                       s, src, kp);                                                                          \
    return hipGetLastError();                                                                                \
  }
  IPB_STREAM_LOCAL(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_global_stream(const FrameSource& src, const KParams& kp, int tile_id, bool fast, int grid,
                                hipStream_t s) {
  // k_global_rows: workgroups of kLocalWaves waves (a multiple of 8 of them)
  const int wgs = ((grid + kLocalWaves - 1) / kLocalWaves + 7) / 8 * 8;
  const dim3 rb(kLanes * kLocalWaves);
#define IPB_GS(TH)                                                                       \
  if (fast) hipLaunchKernelGGL((k_global_rows<TH>), dim3(wgs), rb, 0, s, src, kp);        \
  else hipLaunchKernelGGL((k_global_stream<TH>), dim3(grid), dim3(kLanes), 0, s, src, kp);
  if (tile_id == 5) { IPB_GS(64) }
  else if (tile_id == 6) { IPB_GS(32) }
  else if (tile_id == 7) { IPB_GS(128) }
  else if (tile_id == 8 && fast)   // 16- and 8-row tiles: the default chain only
    hipLaunchKernelGGL((k_global_rows<16>), dim3(wgs), rb, 0, s, src, kp);
  else if (tile_id == 9 && fast)
    hipLaunchKernelGGL((k_global_rows<8>), dim3(wgs), rb, 0, s, src, kp);
  else return hipErrorInvalidValue;
#undef IPB_GS
  return hipGetLastError();
}

hipError_t launch_global_repair(const FrameSource& src, const KParams& kp, int tile_id, int grid, int cell_grid,
                                hipStream_t s) {
  // the fill values of the queued cells and of the dense quarters, then the
  // second pass over both quarter queues (16- and 8-row tiles: the default
  // chain only, which has no second pass)
  if (tile_id == 8 || tile_id == 9) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fill_cells, dim3(cell_grid), dim3(kLanes), 0, s, src, kp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int dgrid = std::max(1, grid / 4);   // four waves per workgroup
  if (tile_id == 5) hipLaunchKernelGGL((k_fill_dense<64>), dim3(dgrid), dim3(kDenseThreads), 0, s, src, kp);
  else if (tile_id == 6) hipLaunchKernelGGL((k_fill_dense<32>), dim3(dgrid), dim3(kDenseThreads), 0, s, src, kp);
  else if (tile_id == 7) hipLaunchKernelGGL((k_fill_dense<128>), dim3(dgrid), dim3(kDenseThreads), 0, s, src, kp);
  else return hipErrorInvalidValue;
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (tile_id == 5) hipLaunchKernelGGL((k_global_patched<64>), dim3(grid), dim3(kLanes), 0, s, src, kp);
  else if (tile_id == 6) hipLaunchKernelGGL((k_global_patched<32>), dim3(grid), dim3(kLanes), 0, s, src, kp);
  else hipLaunchKernelGGL((k_global_patched<128>), dim3(grid), dim3(kLanes), 0, s, src, kp);
  return hipGetLastError();
}

hipError_t launch_prefill(const FrameSource& src, const KParams& kp, int local_rows, int scan_grid, int tile_grid,
                          bool all_bands, hipStream_t s) {
  if (!all_bands) {
    hipLaunchKernelGGL(k_fill_scan, dim3(scan_grid), dim3(kLanes), 0, s, src, kp, local_rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const bool vf = prefill_full_window(kp);
  if (vf && all_bands)
    hipLaunchKernelGGL((k_fill_tiles<true, true>), dim3(tile_grid), dim3(kVfThreads), 0, s, src, kp, local_rows);
  else if (vf)
    hipLaunchKernelGGL((k_fill_tiles<true, false>), dim3(tile_grid), dim3(kVfThreads), 0, s, src, kp, local_rows);
  else if (all_bands)
    hipLaunchKernelGGL((k_fill_tiles<false, true>), dim3(tile_grid), dim3(kDenseThreads), 0, s, src, kp, local_rows);
  else
    hipLaunchKernelGGL((k_fill_tiles<false, false>), dim3(tile_grid), dim3(kDenseThreads), 0, s, src, kp, local_rows);
  return hipGetLastError();
}

bool prefill_full_window(const KParams& kp) { return kp.rl == kFillRad; }

int prefill_resident_blocks(bool full_window) {
  int nb = 0;
  const hipError_t e =
      full_window ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fill_tiles<true, false>, kVfThreads, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fill_tiles<false, false>, kDenseThreads, 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

// The default chain (5x5 median, the binomial 5x5 Gaussian, every stage, the
// full extension): phase 2 then runs k_global_rows.  The host takes it only
// with the streaming phase 1, whose column records the fill ahead of phase 2
// reads.
bool fast_chain(const KParams& kp) {
  return kp.rm == 2 && kp.rg == 2 && kp.last_stage == 9 && kp.blur == 0 && kp.ext_rows == 0 && kp.gw[0] == 6.0 &&
         kp.gw[1] == 4.0 && kp.gw[2] == 1.0 && kp.gscale == 1.0 / 256.0;
}


}  // namespace ipb
