// Host side of the C ABI declared in include/ipb.h: argument checks,
// workspace layout, launch plans and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "ipb.h"
#include "offsets.hpp"

using namespace ipb;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = static_cast<int>(e);
  return IPB_ERR_HIP;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// every byte offset within a map, and the scratch slot just past it, fits
// in 32 bits (the kernels address maps with 32-bit offsets from the map's
// base): H * W < 2^30
bool size_ok(int H, int W) { return cells_ok(H, W); }

// Parameters resolved into what the kernels take.
struct Resolved {
  KParams kp;
  int ltile, gtile, halo;
  int lth, ltw, gth, gtw;
  bool lstream, gstream;   // streaming kernels (tile ids 5 and up) or LDS tile kernels (ids 1-4)
};

constexpr int kTileIdsLocal = 10;   // ids 5-10 streaming (10: 96 rows)
constexpr int kTileIdsGlobal = 9;   // ids 8, 9: 16- and 8-row streaming tiles, default chain only

bool odd_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v % 2) == 1; }

int resolve(const ipb_params* p, Resolved* r) {
  if (p == nullptr || p->struct_size != sizeof(ipb_params)) return IPB_ERR_INVALID_ARG;
  if (p->dilate_shape < IPB_SE_FULL || p->dilate_shape > IPB_SE_CIRCLE) return IPB_ERR_INVALID_ARG;
  const int sizes[] = {p->dilate_size, p->close_size, p->fill_size, p->large_fill_size};
  for (int s : sizes)
    if (s < 1 || s % 2 == 0) return IPB_ERR_INVALID_ARG;
  if (p->median_size < 0 || (p->median_size != 0 && p->median_size % 2 == 0)) return IPB_ERR_INVALID_ARG;
  if (p->gauss_size < 0 || (p->gauss_size != 0 && p->gauss_size % 2 == 0)) return IPB_ERR_INVALID_ARG;
  if (!std::isfinite(p->max_depth) || !std::isfinite(p->valid_thresh) || !std::isfinite(p->gauss_sigma))
    return IPB_ERR_INVALID_ARG;
  if (!(p->valid_thresh > 0.f) || !(p->max_depth > 2.f * p->valid_thresh)) return IPB_ERR_INVALID_ARG;
  if (p->extrapolate != 0 && p->extrapolate != 1) return IPB_ERR_INVALID_ARG;
  if (!odd_in(p->dilate_size, 3, 7) || !odd_in(p->close_size, 3, 7) || !odd_in(p->fill_size, 3, 7) ||
      !odd_in(p->large_fill_size, 3, 31))
    return IPB_ERR_UNSUPPORTED;
  if (p->median_size != 0 && !odd_in(p->median_size, 3, 5)) return IPB_ERR_UNSUPPORTED;
  if (p->gauss_size != 0 && !odd_in(p->gauss_size, 3, 5)) return IPB_ERR_UNSUPPORTED;
  if (p->tile_local < 0 || p->tile_local > kTileIdsLocal) return IPB_ERR_INVALID_ARG;
  if (p->tile_global < 0 || p->tile_global > kTileIdsGlobal) return IPB_ERR_INVALID_ARG;
  if (p->blur != IPB_BLUR_GAUSSIAN && p->blur != IPB_BLUR_BILATERAL) return IPB_ERR_INVALID_ARG;
  if (!std::isfinite(p->bilateral_sigma_space) || !(p->bilateral_sigma_space > 0.f) ||
      !std::isfinite(p->bilateral_sigma_color) || !(p->bilateral_sigma_color > 0.f))
    return IPB_ERR_INVALID_ARG;
  if (p->extend_rows < 0) return IPB_ERR_INVALID_ARG;

  KParams& k = r->kp;
  std::memset(&k, 0, sizeof(k));
  k.shape = p->dilate_shape;
  k.rd = p->dilate_size / 2;
  k.rc = p->close_size / 2;
  k.rf = p->fill_size / 2;
  k.extrapolate = p->extrapolate;
  k.rl = p->large_fill_size / 2;
  k.rm = p->median_size / 2;
  k.rg = p->gauss_size / 2;
  k.off = p->max_depth;
  k.thr = p->valid_thresh;
  k.last_stage = 9;
  k.blur = p->blur;
  k.ext_rows = p->extend_rows;
  {
    const double ss = p->bilateral_sigma_space, sc = p->bilateral_sigma_color;
    k.bl_kc = static_cast<float>(1.0 / (2.0 * sc * sc));
    for (int dy = 0; dy < 3; ++dy)
      for (int dx = 0; dx < 3; ++dx)
        k.bl_ws[dy * 3 + dx] = static_cast<float>(std::exp(-(double)(dy * dy + dx * dx) / (2.0 * ss * ss)));
  }
  if (k.rg > 0) {
    if (p->gauss_sigma <= 0.f) {
      // binomial taps, kept as integers; the sum is scaled once at the end
      if (k.rg == 2) { k.gw[0] = 6; k.gw[1] = 4; k.gw[2] = 1; k.gscale = 1.0 / 256.0; }
      else { k.gw[0] = 2; k.gw[1] = 1; k.gw[2] = 0; k.gscale = 1.0 / 16.0; }
    } else {
      const double s = static_cast<double>(p->gauss_sigma);
      double w[5] = {0, 0, 0, 0, 0};
      double sum = 0.0;
      for (int i = -k.rg; i <= k.rg; ++i) w[i + 2] = std::exp(-(double)(i * i) / (2.0 * s * s));
      for (int i = -k.rg; i <= k.rg; ++i) sum += w[i + 2];
      for (int i = 0; i <= k.rg; ++i) k.gw[i] = w[i + 2] / sum;
      k.gscale = 1.0;
    }
  }
  const int need_local = k.rd + 2 * k.rc + k.rf;
  r->halo = need_local <= 9 ? 9 : 12;
  if (need_local > 12) return IPB_ERR_UNSUPPORTED;
  if (k.rl + k.rm + k.rg > 19) return IPB_ERR_UNSUPPORTED;
  const bool ls_ok = stream_local_supported(k.shape, k.rd, k.rc, k.rf);
  const bool gs_ok = stream_global_supported(k.rm, k.rg) && !(k.blur == IPB_BLUR_BILATERAL && k.rg > 0);
  r->ltile = p->tile_local ? p->tile_local : (ls_ok ? 5 : 1);
  r->gtile = p->tile_global ? p->tile_global : (gs_ok ? 6 : 1);
  r->lstream = r->ltile >= 5;
  r->gstream = r->gtile >= 5;
  if ((r->lstream && !ls_ok) || (r->gstream && !gs_ok)) return IPB_ERR_UNSUPPORTED;
  // 16- and 8-row phase-2 tiles exist for the default chain only (its
  // phase 2 has no second pass, whose quarters would be 4 or 2 rows)
  if (r->gtile >= 8 && !(r->lstream && fast_chain(k))) return IPB_ERR_UNSUPPORTED;
  if (r->lstream) {
    r->lth = stream_local_tile_rows(r->ltile);
    r->ltw = stream_local_tile_cols(r->ltile);
  } else {
    r->lth = local_tile_rows(r->ltile);
    r->ltw = local_tile_cols(r->ltile);
  }
  if (r->gstream) {
    r->gth = stream_global_tile_rows(r->gtile);
    r->gtw = stream_global_tile_cols(r->gtile);
  } else {
    r->gth = global_tile_rows(r->gtile);
    r->gtw = global_tile_cols(r->gtile);
  }
  return IPB_OK;
}

int cdiv(int a, int b) { return (a + b - 1) / b; }

// The default tiles for calls that know their frames, so that small
// launches spread over more waves, in waves per SIMD of the GPU (1024 SIMDs
// on MI355X): phase 1 takes 32-row tiles when 64-row ones would give fewer
// than two, 16-row ones when 32-row ones would give fewer than one, 8-row
// ones when 16-row ones would give fewer than half; phase 2 of the default
// chain takes the tallest of 32, 16 and 8 rows that gives at least four.
// (Measured on MI355X on batches of 1-16 frames: below these sizes the
// shorter tiles finish sooner despite their larger halo share.)  Calls that
// only see a plan keep the defaults, as the plan was built with them.
// count(rows, cols): the launch's tiles of that shape.
constexpr long long kAutoLocal32 = 2048, kAutoLocal16 = 1024, kAutoLocal8 = 512, kAutoGlobal = 4096;
template <class Count>
void auto_tiles(const ipb_params* p, Resolved* r, Count count) {
  if (p->tile_local == 0 && r->lstream && r->ltile == 5 && count(r->lth, r->ltw) < kAutoLocal32) {
    auto local = [&](int id) { return count(stream_local_tile_rows(id), stream_local_tile_cols(id)); };
    const int id = local(7) >= kAutoLocal16 ? 7 : local(8) >= kAutoLocal8 ? 8 : 9;
    r->ltile = id;
    r->lth = stream_local_tile_rows(id);
    r->ltw = stream_local_tile_cols(id);
  }
  if (p->tile_global == 0 && r->gstream && r->gtile == 6 && count(r->gth, r->gtw) < kAutoGlobal && r->lstream &&
      fast_chain(r->kp)) {
    const int id = count(stream_global_tile_rows(8), stream_global_tile_cols(8)) >= kAutoGlobal ? 8 : 9;
    r->gtile = id;
    r->gth = stream_global_tile_rows(id);
    r->gtw = stream_global_tile_cols(id);
  }
}

int resolve_single(const ipb_params* p, int H, int W, Resolved* r) {
  const int st = resolve(p, r);
  if (st == IPB_OK && size_ok(H, W))
    auto_tiles(p, r, [&](int th, int tw) { return (long long)cdiv(W, tw) * cdiv(H, th); });
  return st;
}

int resolve_frames(const ipb_params* p, const ipb_frame* frames, int n, Resolved* r) {
  const int st = resolve(p, r);
  if (st != IPB_OK || frames == nullptr || n < 1) return st;
  auto_tiles(p, r, [&](int th, int tw) {
    long long t = 0;
    for (int i = 0; i < n; ++i)
      if (size_ok(frames[i].H, frames[i].W)) t += (long long)cdiv(frames[i].W, tw) * cdiv(frames[i].H, th);
    return t;
  });
  return st;
}

// Per-device facts: CU count and resident workgroups per kernel variant.
struct DeviceFacts {
  int cus = 0;
  int occ[3][8][2] = {};    // LDS kernels: [phase][tile id][halo 9/12]
  int prefill_occ[2] = {0, 0};   // fill ahead of phase 2 (k_fill_tiles; [1]: the 31x31 window's)
};
std::mutex g_dev_mu;
DeviceFacts g_dev[64];

int device_cus(int* out_dev) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= 64) return IPB_ERR_UNSUPPORTED;
  *out_dev = dev;
  std::lock_guard<std::mutex> g(g_dev_mu);
  if (g_dev[dev].cus == 0) {
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e);
    g_dev[dev].cus = cus > 0 ? cus : 1;
  }
  return IPB_OK;
}

int resident(int dev, int phase, int tile, int halo) {
  std::lock_guard<std::mutex> g(g_dev_mu);
  int& slot = g_dev[dev].occ[phase][tile][halo == 12 ? 1 : 0];
  if (slot == 0) slot = max_resident_blocks(phase, tile, halo);
  return slot;
}

int prefill_res(int dev, const KParams& kp) {
  const bool full = prefill_full_window(kp);
  std::lock_guard<std::mutex> g(g_dev_mu);
  int& slot = g_dev[dev].prefill_occ[full ? 1 : 0];
  if (slot == 0) slot = prefill_resident_blocks(full);
  return slot;
}

// The stage-4 map and, past its last cell, a scratch slot that the
// streaming kernel's idle lanes store to.
size_t v4_bytes(int H, int W) { return align_up(sizeof(float) * (size_t)H * W + kAlign); }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

// Host memory in which ipb_complete_batch builds a plan before its upload
// kernels take it by value; grown as needed, reused by the calling thread.
thread_local std::vector<int32_t> t_plan;

// Workspace of ipb_complete_static: a fixed device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it only stands for the symbol):
// the device address comes from hipGetSymbolAddress, once per device with
// that device current, and is kept per device.
static __device__ __align__(256) unsigned char scratch[IPB_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

int static_scratch(int dev, void** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (ptr == nullptr || (reinterpret_cast<uintptr_t>(ptr) % kAlign) != 0) return hip_fail(hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return IPB_OK;
}

// Fill a plan (host memory) for frames whose workspace is ws.
void build_plan(const ipb_frame* frames, int n, const Resolved& r, void* ws, void* plan_host) {
  auto* hdr = static_cast<PlanHeader*>(plan_host);
  auto* fd = reinterpret_cast<FrameDesc*>(hdr + 1);
  std::memset(hdr, 0, sizeof(PlanHeader));
  char* base = static_cast<char*>(ws);
  size_t off = align_up(sizeof(PlanHeader) + sizeof(FrameDesc) * (size_t)n);
  long long cols = 0;
  for (int i = 0; i < n; ++i) cols += frames[i].W;
  auto* top_base = reinterpret_cast<int32_t*>(base + off);
  off += align_up(sizeof(int32_t) * (size_t)cols);
  long long gtot = 0, ltot = 0;
  for (int i = 0; i < n; ++i) gtot += (long long)cdiv(frames[i].W, r.gtw) * cdiv(frames[i].H, r.gth);
  for (int i = 0; i < n; ++i) ltot += (long long)cdiv(frames[i].W, r.ltw) * cdiv(frames[i].H, r.lth);
  auto* slow = reinterpret_cast<int32_t*>(base + off);
  off += align_up(sizeof(int32_t) * slow_queue_ints((int)gtot, (int)ltot));
  auto* ltab = reinterpret_cast<int32_t*>(base + off);
  off += align_up(sizeof(int32_t) * (size_t)ltot);
  auto* gtab = reinterpret_cast<int32_t*>(base + off);
  off += align_up(sizeof(int32_t) * (size_t)gtot);
  int lt = 0, gt = 0, col = 0;
  for (int i = 0; i < n; ++i) {
    const int H = frames[i].H, W = frames[i].W;
    FrameDesc& d = fd[i];
    std::memset(&d, 0, sizeof(d));
    d.in = frames[i].in;
    d.out = frames[i].out;
    d.v4 = reinterpret_cast<float*>(base + off);
    off += v4_bytes(H, W);
    d.v6p = reinterpret_cast<float*>(base + off);
    off += align_up(sizeof(float) * (size_t)H * W);
    d.top = top_base + col;
    d.H = H;
    d.W = W;
    d.lcols = cdiv(W, r.ltw);
    d.gcols = cdiv(W, r.gtw);
    d.ltile0 = lt;
    d.gtile0 = gt;
    lt += d.lcols * cdiv(H, r.lth);
    gt += d.gcols * cdiv(H, r.gth);
    col += W;
  }
  hdr->n = n;
  hdr->ltiles = lt;
  hdr->gtiles = gt;
  hdr->ncols = col;
  hdr->top_base = top_base;
  hdr->lt_rows = r.lth;
  hdr->lt_cols = r.ltw;
  hdr->gt_rows = r.gth;
  hdr->gt_cols = r.gtw;
  hdr->slow = slow;
  hdr->slow_cap = (int32_t)gtot;
  hdr->ltab = ltab;
  hdr->gtab = gtab;
  bool same = frames[0].H >= 3 && frames[0].W >= 3;
  for (int i = 1; i < n && same; ++i) same = frames[i].H == frames[0].H && frames[i].W == frames[0].W;
  hdr->g_rows_same = same ? cdiv(frames[0].H, r.gth) : 0;
  hdr->g_cols_same = same ? cdiv(frames[0].W, r.gtw) : 0;
}

size_t batch_bytes(const ipb_frame* frames, int n, const Resolved& r) {
  size_t total = align_up(sizeof(PlanHeader) + sizeof(FrameDesc) * (size_t)n);
  size_t cols = 0, gtot = 0;
  for (int i = 0; i < n; ++i) cols += (size_t)frames[i].W;
  for (int i = 0; i < n; ++i) gtot += (size_t)cdiv(frames[i].W, r.gtw) * cdiv(frames[i].H, r.gth);
  size_t ltot = 0;
  for (int i = 0; i < n; ++i) ltot += (size_t)cdiv(frames[i].W, r.ltw) * cdiv(frames[i].H, r.lth);
  total += align_up(sizeof(int32_t) * cols);
  total += align_up(sizeof(int32_t) * slow_queue_ints((int)gtot, (int)ltot));
  total += align_up(sizeof(int32_t) * ltot) + align_up(sizeof(int32_t) * gtot);   // tile -> frame tables
  for (int i = 0; i < n; ++i)
    total += v4_bytes(frames[i].H, frames[i].W) + align_up(sizeof(float) * (size_t)frames[i].H * frames[i].W);
  return total;
}

// Frames valid, outputs disjoint from every other frame's buffers.
int check_frames(const ipb_frame* frames, int n) {
  if (frames == nullptr || n < 1) return IPB_ERR_INVALID_ARG;
  struct Iv { const char* lo; const char* hi; int frame; int is_out; };
  std::vector<Iv> iv;
  iv.reserve(2 * (size_t)n);
  long long cols = 0;
  for (int i = 0; i < n; ++i) {
    const ipb_frame& f = frames[i];
    if (f.in == nullptr || f.out == nullptr || !size_ok(f.H, f.W)) return IPB_ERR_INVALID_ARG;
    const size_t nb = sizeof(float) * (size_t)f.H * f.W;
    const char* in = reinterpret_cast<const char*>(f.in);
    const char* out = reinterpret_cast<const char*>(f.out);
    if (in != out && overlaps(in, nb, out, nb)) return IPB_ERR_INVALID_ARG;
    iv.push_back({in, in + nb, i, 0});
    if (out != in) iv.push_back({out, out + nb, i, 1});
    else iv.back().is_out = 1;   // in-place: the one interval is also an output
    cols += f.W;
  }
  if (cols >= (1LL << 31)) return IPB_ERR_INVALID_ARG;
  std::sort(iv.begin(), iv.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
  // Any two overlapping intervals of different frames where one is an output
  // is a conflict (inputs may be shared read-only).
  for (size_t a = 0; a < iv.size(); ++a) {
    for (size_t b = a + 1; b < iv.size() && iv[b].lo < iv[a].hi; ++b) {
      if (iv[a].frame != iv[b].frame && (iv[a].is_out || iv[b].is_out)) return IPB_ERR_INVALID_ARG;
    }
  }
  return IPB_OK;
}

FrameSource single_source(const float* in, int H, int W, float* out, void* ws, const Resolved& r) {
  FrameSource s;
  std::memset(&s, 0, sizeof(s));
  s.plan = nullptr;
  FrameDesc& d = s.single;
  d.in = in;
  d.out = out;
  d.v4 = static_cast<float*>(ws);
  const size_t map = align_up(sizeof(float) * (size_t)H * W);
  const size_t map4 = v4_bytes(H, W);
  d.v6p = reinterpret_cast<float*>(static_cast<char*>(ws) + map4);
  d.top = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + map4 + map);
  s.slow = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + map4 + map + align_up(sizeof(int32_t) * (size_t)W));
  d.H = H;
  d.W = W;
  d.lcols = cdiv(W, r.ltw);
  d.gcols = cdiv(W, r.gtw);
  d.ltile0 = 0;
  d.gtile0 = 0;
  s.single_ltiles = d.lcols * cdiv(H, r.lth);
  s.single_gtiles = d.gcols * cdiv(H, r.gth);
  s.slow_cap = s.single_gtiles;
  return s;
}

size_t frame_ws_bytes(int H, int W, const Resolved& r) {
  const size_t gtiles = (size_t)cdiv(W, r.gtw) * cdiv(H, r.gth);
  const size_t ltiles = (size_t)cdiv(W, r.ltw) * cdiv(H, r.lth);
  return v4_bytes(H, W) + align_up(sizeof(float) * (size_t)H * W) + align_up(sizeof(int32_t) * (size_t)W) +
         align_up(sizeof(int32_t) * slow_queue_ints((int)gtiles, (int)ltiles));
}

// Launch the phases of a frame source (-1: all; ipb_complete_planned lists
// them): 0 reset, 1 stages 1-4, 2 the fill of stage 6 ahead of phase 2,
// 3 stages 5-9, 4 the second pass of queued quarters, 5 tiny frames.
int launch_phases(const FrameSource& src, const Resolved& r, int phase, int last_stage, int max_lt, int max_gt,
                  int max_cols, bool persistent, bool may_tiny, hipStream_t s) {
  int dev = 0;
  int st = device_cus(&dev);
  if (st != IPB_OK) return st;
  const int cus = g_dev[dev].cus;
  KParams kp = r.kp;
  kp.last_stage = last_stage;
  // the default chain on streaming kernels: the fill runs ahead of phase 2,
  // which then needs no second pass
  const bool fast = r.lstream && r.gstream && fast_chain(kp);
  const bool prefill = fast && kp.extrapolate;
  hipError_t e;
  if ((phase == -1 || phase == 0) && last_stage >= 5) {
    e = launch_reset(src, std::max(max_cols, std::max(max_lt, max_gt)), s);
    if (e != hipSuccess) return hip_fail(e);
  }
  // Streaming kernels: one wave per tile, a grid of every tile (rounded up to
  // a multiple of the 8 XCDs); surplus blocks find no tile and exit.  LDS
  // kernels of a planned launch: a persistent grid of resident blocks.
  if (phase == -1 || phase == 1) {
    int grid = max_lt;
    if (r.lstream) grid = (grid + 7) / 8 * 8;
    else if (persistent) grid = std::min(grid, resident(dev, 1, r.ltile, r.halo) * cus);
    e = r.lstream ? launch_local_stream(src, kp, r.ltile, grid, s) : launch_local(src, kp, r.ltile, r.halo, grid, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (last_stage < 5) return IPB_OK;
  if ((phase == -1 || phase == 2) && prefill) {
    // one scanning wave per phase-1 tile (those of the first tile row work);
    // one workgroup per queued band, at most the resident ones.  When every
    // band of every tile fits one round of resident workgroups, the fill
    // visits them all and the scan is left out.
    const long long slots = (long long)prefill_res(dev, kp) * cus;
    const long long bands = (long long)cdiv(r.lth, kBandRows) * max_lt;
    const bool all_bands = bands <= slots;
    const int tgrid = std::max(1, (int)std::min<long long>(all_bands ? bands : (long long)kBandsPerTile * max_lt, slots));
    e = launch_prefill(src, kp, r.lth, max_lt, tgrid, all_bands, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (phase == -1 || phase == 3) {
    int grid = max_gt;
    if (r.gstream) grid = (grid + 7) / 8 * 8;
    else if (persistent) grid = std::min(grid, resident(dev, 2, r.gtile, 0) * cus);
    e = r.gstream ? launch_global_stream(src, kp, r.gtile, fast, grid, s)
                  : launch_global(src, kp, r.gtile, grid, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if ((phase == -1 || phase == 4) && r.gstream && !fast) {
    // queued quarters (at most four per tile) and cells (at most
    // 4 kCellEmpty per tile); grids of at most 32 waves per CU
    const int rgrid = std::max(1, std::min(4 * max_gt, 32 * cus));
    const int cgrid = std::max(1, (int)std::min<long long>(4LL * kCellEmpty * max_gt, 32LL * cus));
    e = launch_global_repair(src, kp, r.gtile, rgrid, cgrid, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  // (skipped when the caller knows no frame has under 3 rows or columns)
  if ((phase == -1 || phase == 5) && r.gstream && may_tiny) {
    const int per = slow_subtiles(r.gth, r.gtw);
    // frames under 3 rows or columns are rare and small: one workgroup per CU
    const int sgrid = std::max(1, std::min(max_gt * per, cus));
    e = launch_global_slow(src, kp, r.gth, r.gtw, sgrid, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  return IPB_OK;
}

int run_single(const float* in, int H, int W, const ipb_params* p, float* out, int last_stage, void* ws,
               size_t ws_bytes, hipStream_t s) {
  Resolved r;
  int st = resolve_single(p, H, W, &r);
  if (st != IPB_OK) return st;
  if (in == nullptr || out == nullptr || !size_ok(H, W)) return IPB_ERR_INVALID_ARG;
  if (last_stage < 1 || last_stage > 9) return IPB_ERR_INVALID_ARG;
  const size_t nb = sizeof(float) * (size_t)H * W;
  if (in != out && overlaps(in, nb, out, nb)) return IPB_ERR_INVALID_ARG;
  if (in == out && last_stage <= 4) return IPB_ERR_INVALID_ARG;   // stage 1-4 maps race with the halo reads
  if (ws == nullptr || ws_bytes < frame_ws_bytes(H, W, r) || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
    return IPB_ERR_WORKSPACE;
  if (overlaps(ws, frame_ws_bytes(H, W, r), in, nb) || overlaps(ws, frame_ws_bytes(H, W, r), out, nb))
    return IPB_ERR_INVALID_ARG;
  if (last_stage <= 4 && r.lstream) {   // the stage hooks 1-4 take the LDS kernel
    r.lstream = false;
    r.ltile = 1;
    r.lth = local_tile_rows(1);
    r.ltw = local_tile_cols(1);
  }
  if (last_stage < 9 && r.gtile >= 8) {  // stage hooks run the general phase 2, on 32-row tiles
    r.gtile = 6;                          // (fewer tiles than the workspace was sized for)
    r.gth = stream_global_tile_rows(6);
    r.gtw = stream_global_tile_cols(6);
  }
  FrameSource src = single_source(in, H, W, out, ws, r);
  return launch_phases(src, r, -1, last_stage, src.single_ltiles, src.single_gtiles, W, false, H < 3 || W < 3, s);
}

int planned(const void* plan_dev, const Resolved& r, int phase, int max_tiles_local, int max_tiles_global,
            int max_cols, bool may_tiny, void* stream) {
  if (plan_dev == nullptr || phase < -1 || phase > 5) return IPB_ERR_INVALID_ARG;
  if (max_tiles_local < 1 || max_tiles_global < 1 || max_cols < 1) return IPB_ERR_INVALID_ARG;
  FrameSource src;
  std::memset(&src, 0, sizeof(src));
  src.plan = static_cast<const PlanHeader*>(plan_dev);
  return launch_phases(src, r, phase, 9, max_tiles_local, max_tiles_global, max_cols, true, may_tiny,
                       static_cast<hipStream_t>(stream));
}

}  // namespace

extern "C" {

void ipb_params_default(ipb_params* p) {
  if (p == nullptr) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(ipb_params);
  p->dilate_shape = IPB_SE_DIAMOND;
  p->dilate_size = 5;
  p->close_size = 5;
  p->fill_size = 7;
  p->extrapolate = 1;
  p->large_fill_size = 31;
  p->median_size = 5;
  p->gauss_size = 5;
  p->gauss_sigma = 0.f;
  p->max_depth = 100.f;
  p->valid_thresh = 0.1f;
  p->tile_local = 0;
  p->tile_global = 0;
  p->blur = IPB_BLUR_GAUSSIAN;
  p->bilateral_sigma_space = 2.f;
  p->bilateral_sigma_color = 1.5f;
  p->extend_rows = 0;
}

size_t ipb_workspace_bytes(int H, int W, const ipb_params* p) {
  Resolved r;
  if (resolve_single(p, H, W, &r) != IPB_OK || !size_ok(H, W)) return 0;
  return frame_ws_bytes(H, W, r);
}

int ipb_complete_ws(const float* depth_in, int H, int W, const ipb_params* p, float* depth_out, void* ws,
                    size_t ws_bytes, void* stream) {
  return run_single(depth_in, H, W, p, depth_out, 9, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int ipb_complete_stage(const float* depth_in, int H, int W, const ipb_params* p, float* out, int last_stage,
                       void* ws, size_t ws_bytes, void* stream) {
  return run_single(depth_in, H, W, p, out, last_stage, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int ipb_complete(const float* depth_in, int H, int W, const ipb_params* p, float* depth_out, void* stream) {
  Resolved r;
  int st = resolve_single(p, H, W, &r);
  if (st != IPB_OK) return st;
  if (depth_in == nullptr || depth_out == nullptr || !size_ok(H, W)) return IPB_ERR_INVALID_ARG;
  const size_t nb = sizeof(float) * (size_t)H * W;
  if (depth_in != depth_out && overlaps(depth_in, nb, depth_out, nb)) return IPB_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = frame_ws_bytes(H, W, r);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, need, s);
  if (e != hipSuccess) return hip_fail(e);
  st = run_single(depth_in, H, W, p, depth_out, 9, ws, need, s);
  e = hipFreeAsync(ws, s);
  if (st != IPB_OK) return st;
  if (e != hipSuccess) return hip_fail(e);
  return IPB_OK;
}

int ipb_complete_static(const float* depth_in, int H, int W, const ipb_params* p, float* depth_out,
                        void* stream) {
  Resolved r;
  int st = resolve_single(p, H, W, &r);
  if (st != IPB_OK) return st;
  if (depth_in == nullptr || depth_out == nullptr || !size_ok(H, W)) return IPB_ERR_INVALID_ARG;
  if (frame_ws_bytes(H, W, r) > (size_t)IPB_STATIC_SCRATCH_BYTES) return IPB_ERR_SCRATCH;
  int dev = 0;
  st = device_cus(&dev);                 // the current device (no allocation)
  if (st != IPB_OK) return st;
  void* ws = nullptr;
  st = static_scratch(dev, &ws);
  if (st != IPB_OK) return st;
  // the reset step of the chain clears what must start at zero (column
  // tops, queue counters); everything else is written before it is read
  return run_single(depth_in, H, W, p, depth_out, 9, ws, (size_t)IPB_STATIC_SCRATCH_BYTES,
                    static_cast<hipStream_t>(stream));
}

size_t ipb_batch_plan_bytes(int n) {
  if (n < 1) return 0;
  return sizeof(PlanHeader) + sizeof(FrameDesc) * (size_t)n;
}

size_t ipb_batch_workspace_bytes(const ipb_frame* frames, int n, const ipb_params* p) {
  Resolved r, ra;
  if (resolve(p, &r) != IPB_OK || check_frames(frames, n) != IPB_OK) return 0;
  resolve_frames(p, frames, n, &ra);
  // enough for ipb_complete_batch (which may take 32-row phase-1 tiles for
  // few frames) and for a plan of ipb_batch_plan (the default tiles)
  return std::max(batch_bytes(frames, n, r), batch_bytes(frames, n, ra));
}

int ipb_batch_plan(const ipb_frame* frames, int n, const ipb_params* p, void* ws, size_t ws_bytes,
                   void* plan_host, size_t plan_bytes) {
  Resolved r;
  int st = resolve(p, &r);
  if (st != IPB_OK) return st;
  st = check_frames(frames, n);
  if (st != IPB_OK) return st;
  if (plan_host == nullptr || plan_bytes < ipb_batch_plan_bytes(n)) return IPB_ERR_INVALID_ARG;
  if (ws == nullptr || ws_bytes < batch_bytes(frames, n, r) || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
    return IPB_ERR_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    const size_t nb = sizeof(float) * (size_t)frames[i].H * frames[i].W;
    if (overlaps(ws, ws_bytes, frames[i].in, nb) || overlaps(ws, ws_bytes, frames[i].out, nb))
      return IPB_ERR_INVALID_ARG;
  }
  build_plan(frames, n, r, ws, plan_host);
  return IPB_OK;
}

int ipb_plan_totals(const void* plan_host, int* n, int* tiles_local, int* tiles_global, int* cols) {
  if (plan_host == nullptr) return IPB_ERR_INVALID_ARG;
  const auto* h = static_cast<const PlanHeader*>(plan_host);
  if (n) *n = h->n;
  if (tiles_local) *tiles_local = h->ltiles;
  if (tiles_global) *tiles_global = h->gtiles;
  if (cols) *cols = h->ncols;
  return IPB_OK;
}


int ipb_complete_planned(const void* plan_dev, const ipb_params* p, int phase, int max_tiles_local,
                         int max_tiles_global, int max_cols, void* stream) {
  // a plan may be rewritten for other frames after the launch is captured
  Resolved r;
  const int st = resolve(p, &r);
  if (st != IPB_OK) return st;
  // -2: every step but the one of frames under 3 rows or columns, which the
  // caller guarantees none of its plans holds
  if (phase == -2) return planned(plan_dev, r, -1, max_tiles_local, max_tiles_global, max_cols, false, stream);
  return planned(plan_dev, r, phase, max_tiles_local, max_tiles_global, max_cols, true, stream);
}

int ipb_complete_batch(const ipb_frame* frames, int n, const ipb_params* p, void* ws, size_t ws_bytes,
                       void* stream) {
  Resolved r;
  int st = resolve_frames(p, frames, n, &r);
  if (st != IPB_OK) return st;
  st = check_frames(frames, n);
  if (st != IPB_OK) return st;
  if (ws == nullptr || ws_bytes < batch_bytes(frames, n, r) || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
    return IPB_ERR_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    const size_t nb = sizeof(float) * (size_t)frames[i].H * frames[i].W;
    if (overlaps(ws, ws_bytes, frames[i].in, nb) || overlaps(ws, ws_bytes, frames[i].out, nb))
      return IPB_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the plan is built in host memory of this thread and reaches the
  // workspace in the arguments of upload kernels on the stream: no staging
  // buffer, no copy to wait for, so the call can be captured into a graph
  const size_t pb = ipb_batch_plan_bytes(n);
  if (t_plan.size() < pb / sizeof(int32_t)) t_plan.resize(pb / sizeof(int32_t));
  void* host = t_plan.data();
  build_plan(frames, n, r, ws, host);
  const auto* hdr = static_cast<const PlanHeader*>(host);
  const int lt = hdr->ltiles, gt = hdr->gtiles, cols = hdr->ncols;
  hipError_t e = launch_plan_upload(host, pb, ws, s);
  if (e != hipSuccess) return hip_fail(e);
  bool tiny = false;
  for (int i = 0; i < n; ++i) tiny = tiny || frames[i].H < 3 || frames[i].W < 3;
  return planned(ws, r, -1, lt, gt, cols, tiny, stream);
}

const char* ipb_status_string(int status) {
  switch (status) {
    case IPB_OK: return "ok";
    case IPB_ERR_INVALID_ARG: return "invalid argument";
    case IPB_ERR_UNSUPPORTED: return "unsupported parameter value";
    case IPB_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case IPB_ERR_HIP: return "HIP runtime error";
    case IPB_ERR_SCRATCH: return "frame needs more workspace than the static scratch holds";
    default: return "unknown status";
  }
}

int ipb_last_hip_error(void) { return g_last_hip; }

int ipb_stream_create(void** stream) {
  if (stream == nullptr) return IPB_ERR_INVALID_ARG;
  *stream = nullptr;
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e);
  if (ncu <= 0) return hip_fail(hipErrorInvalidDevice);
  // every compute unit of the device: the mask only makes the runtime give
  // the stream a hardware queue of its own, it narrows nothing
  std::vector<uint32_t> mask((ncu + 31) / 32, 0xffffffffu);
  if (ncu % 32 != 0) mask.back() = (1u << (ncu % 32)) - 1u;
  hipStream_t s = nullptr;
  e = hipExtStreamCreateWithCUMask(&s, static_cast<uint32_t>(mask.size()), mask.data());
  if (e != hipSuccess) return hip_fail(e);
  *stream = s;
  return IPB_OK;
}

int ipb_stream_destroy(void* stream) {
  if (stream == nullptr) return IPB_ERR_INVALID_ARG;
  hipError_t e = hipStreamDestroy(static_cast<hipStream_t>(stream));
  return e == hipSuccess ? IPB_OK : hip_fail(e);
}

int ipb_tile_shape(int phase, int tile_id, int* rows, int* cols) {
  if (rows == nullptr || cols == nullptr) return IPB_ERR_INVALID_ARG;
  if (tile_id == 0) tile_id = phase == 1 ? 5 : 6;   // defaults of the streaming kernels
  if (tile_id < 1 || tile_id > (phase == 2 ? kTileIdsGlobal : kTileIdsLocal)) return IPB_ERR_INVALID_ARG;
  if (phase == 1) {
    *rows = tile_id >= 5 ? stream_local_tile_rows(tile_id) : local_tile_rows(tile_id);
    *cols = tile_id >= 5 ? stream_local_tile_cols(tile_id) : local_tile_cols(tile_id);
    return IPB_OK;
  }
  if (phase == 2) {
    *rows = tile_id >= 5 ? stream_global_tile_rows(tile_id) : global_tile_rows(tile_id);
    *cols = tile_id >= 5 ? stream_global_tile_cols(tile_id) : global_tile_cols(tile_id);
    return IPB_OK;
  }
  return IPB_ERR_INVALID_ARG;
}

int ipb_tile_count(int phase) { return phase == 1 ? kTileIdsLocal : phase == 2 ? kTileIdsGlobal : 0; }

}  // extern "C"
