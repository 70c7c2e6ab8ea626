// Host logic of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
// (built for the host only; the GPU code is compiled but never launched):
// argument checks, workspace sizing, frame-overlap checks, plan building and
// the offset and size arithmetic, on random and boundary inputs.  Every call
// here returns before any HIP call is made.  Exit status 0 when every check
// holds; a sanitizer report aborts the run.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "common.hpp"
#include "ipb.h"

namespace {

int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

// placeholder device addresses: never dereferenced
char* fake(uint64_t off) { return reinterpret_cast<char*>((uint64_t)1 << 44) + off; }

std::vector<ipb_frame> random_frames(std::mt19937& rng, int n, bool in_place) {
  std::vector<ipb_frame> f(n);
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    f[i].H = 1 + (int)(rng() % 700);
    f[i].W = 1 + (int)(rng() % 2100);
    const uint64_t nb = ((uint64_t)4 * f[i].H * f[i].W + 255) / 256 * 256;
    f[i].in = reinterpret_cast<const float*>(fake(off));
    off += nb;
    if (in_place) {
      f[i].out = const_cast<float*>(f[i].in);
    } else {
      f[i].out = reinterpret_cast<float*>(fake(off));
      off += nb;
    }
  }
  return f;
}

void params_and_sizes() {
  ipb_params p;
  ipb_params_default(&p);
  CHECK(p.struct_size == sizeof(ipb_params));
  CHECK(ipb_workspace_bytes(375, 1242, &p) > (size_t)8 * 375 * 1242);
  CHECK(ipb_workspace_bytes(1, 1, &p) > 0);
  CHECK(ipb_workspace_bytes(0, 5, &p) == 0);
  CHECK(ipb_workspace_bytes(5, -1, &p) == 0);
  CHECK(ipb_workspace_bytes(1, (1 << 30) - 1, &p) > (size_t)8 * ((1 << 30) - 1));
  CHECK(ipb_workspace_bytes(1 << 15, 1 << 15, &p) == 0);
  CHECK(ipb_workspace_bytes(1 << 30, 1 << 30, &p) == 0);
  CHECK(ipb_workspace_bytes(2147483647, 2147483647, &p) == 0);
  CHECK(ipb_workspace_bytes(10, 10, nullptr) == 0);
  // every tile id, every supported size, some invalid values
  for (int tl = -1; tl <= 10; ++tl)
    for (int tg = -1; tg <= 10; ++tg) {
      ipb_params q = p;
      q.tile_local = tl;
      q.tile_global = tg;
      (void)ipb_workspace_bytes(333, 777, &q);
    }
  const int bad_sizes[] = {-3, 0, 1, 2, 3, 4, 5, 7, 9, 31, 33, 1 << 30};
  for (int a : bad_sizes)
    for (int field = 0; field < 6; ++field) {
      ipb_params q = p;
      int* fp[] = {&q.dilate_size, &q.close_size, &q.fill_size, &q.large_fill_size, &q.median_size, &q.gauss_size};
      *fp[field] = a;
      (void)ipb_workspace_bytes(64, 64, &q);
    }
  ipb_params q = p;
  q.struct_size = 4;
  CHECK(ipb_workspace_bytes(64, 64, &q) == 0);
  q = p;
  q.max_depth = 0.15f;
  CHECK(ipb_workspace_bytes(64, 64, &q) == 0);
  q = p;
  q.extend_rows = -1;
  CHECK(ipb_workspace_bytes(64, 64, &q) == 0);
  for (int id = -2; id <= 12; ++id)
    for (int ph = 0; ph <= 3; ++ph) {
      int r = -1, c = -1;
      (void)ipb_tile_shape(ph, id, &r, &c);
    }
  CHECK(ipb_tile_shape(1, 0, nullptr, nullptr) == IPB_ERR_INVALID_ARG);
  for (int st = -8; st <= 3; ++st) CHECK(ipb_status_string(st) != nullptr);
}

void argument_checks() {
  ipb_params p;
  ipb_params_default(&p);
  const float* in = reinterpret_cast<const float*>(fake(0));
  float* out = reinterpret_cast<float*>(fake(1 << 30));
  void* ws = fake((uint64_t)2 << 30);
  const size_t nb = ipb_workspace_bytes(64, 64, &p);
  CHECK(ipb_complete_ws(nullptr, 64, 64, &p, out, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_ws(in, 64, 64, &p, nullptr, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_ws(in, 0, 64, &p, out, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_ws(in, 64, 64, &p, out, nullptr, nb, nullptr) == IPB_ERR_WORKSPACE);
  CHECK(ipb_complete_ws(in, 64, 64, &p, out, ws, nb - 1, nullptr) == IPB_ERR_WORKSPACE);
  CHECK(ipb_complete_ws(in, 64, 64, &p, out, fake(((uint64_t)2 << 30) + 8), nb, nullptr) == IPB_ERR_WORKSPACE);
  CHECK(ipb_complete_ws(in, 64, 64, &p, reinterpret_cast<float*>(fake(4)), ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_ws(in, 64, 64, &p, out, fake(256), nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_ws(in, 1 << 15, 1 << 15, &p, out, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_stage(in, 64, 64, &p, out, 0, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_stage(in, 64, 64, &p, out, 10, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_stage(in, 64, 64, &p, const_cast<float*>(in), 3, ws, nb, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete(nullptr, 64, 64, &p, out, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_static(in, 4096, 4096, &p, out, nullptr) == IPB_ERR_SCRATCH);
  CHECK(ipb_complete_static(nullptr, 64, 64, &p, out, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_planned(nullptr, &p, -1, 1, 1, 1, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_planned(ws, &p, 7, 1, 1, 1, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_planned(ws, &p, -1, 0, 1, 1, nullptr) == IPB_ERR_INVALID_ARG);
  ipb_frame f[2] = {{in, out, 64, 64}, {in, out, 64, 64}};   // the same output twice
  CHECK(ipb_batch_workspace_bytes(f, 2, &p) == 0);
  CHECK(ipb_complete_batch(f, 2, &p, ws, 1 << 30, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_batch(nullptr, 1, &p, ws, 1 << 30, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_batch(f, 0, &p, ws, 1 << 30, nullptr) == IPB_ERR_INVALID_ARG);
  CHECK(ipb_complete_batch(f, 1, &p, ws, 16, nullptr) == IPB_ERR_WORKSPACE);
  f[1].in = reinterpret_cast<const float*>(fake(8));         // input overlapping another frame's
  f[1].out = reinterpret_cast<float*>(fake(8));               // ... and in place: an output over frame 0's input
  CHECK(ipb_batch_workspace_bytes(f, 2, &p) == 0);
}

void plans(std::mt19937& rng) {
  ipb_params p;
  ipb_params_default(&p);
  for (int it = 0; it < 300; ++it) {
    const int n = 1 + (int)(rng() % 70);
    const bool in_place = (it % 3) == 0;
    std::vector<ipb_frame> f = random_frames(rng, n, in_place);
    if (it % 4 == 1) {
      // a batch of one shape: the smallest height and width of the frames
      // (every buffer still holds its frame)
      int h = f[0].H, w = f[0].W;
      for (const ipb_frame& x : f) h = std::min(h, x.H), w = std::min(w, x.W);
      for (ipb_frame& x : f) x.H = h, x.W = w;
    }
    ipb_params q = p;
    q.tile_local = (int)(rng() % 10);
    q.tile_global = (int)(rng() % 8);
    const size_t need = ipb_batch_workspace_bytes(f.data(), n, &q);
    if (need == 0) continue;                      // an unsupported tile pair
    const size_t pb = ipb_batch_plan_bytes(n);
    CHECK(pb == sizeof(ipb::PlanHeader) + sizeof(ipb::FrameDesc) * (size_t)n);
    std::vector<unsigned char> host(pb + 7);
    char* ws = fake((uint64_t)1 << 42);
    CHECK(ipb_batch_plan(f.data(), n, &q, ws, 16, host.data(), pb) == IPB_ERR_WORKSPACE);
    CHECK(ipb_batch_plan(f.data(), n, &q, ws, need, host.data(), pb - 1) == IPB_ERR_INVALID_ARG);
    const int st = ipb_batch_plan(f.data(), n, &q, ws, need, host.data(), pb);
    CHECK(st == IPB_OK);
    if (st != IPB_OK) continue;
    int pn = 0, lt = 0, gt = 0, cols = 0;
    CHECK(ipb_plan_totals(host.data(), &pn, &lt, &gt, &cols) == IPB_OK);
    CHECK(pn == n);
    const auto* hdr = reinterpret_cast<const ipb::PlanHeader*>(host.data());
    const auto* d = reinterpret_cast<const ipb::FrameDesc*>(hdr + 1);
    long long sum_w = 0, lsum = 0, gsum = 0;
    const char* lo = ws;
    const char* hi = ws + need;
    for (int i = 0; i < n; ++i) {
      sum_w += f[i].W;
      CHECK(d[i].H == f[i].H && d[i].W == f[i].W);
      CHECK(d[i].ltile0 == lsum && d[i].gtile0 == gsum);
      lsum += (long long)d[i].lcols * ((d[i].H + hdr->lt_rows - 1) / hdr->lt_rows);
      gsum += (long long)d[i].gcols * ((d[i].H + hdr->gt_rows - 1) / hdr->gt_rows);
      // the frame's maps and column table lie inside the workspace, past the plan
      const char* v4 = reinterpret_cast<const char*>(d[i].v4);
      const char* v6 = reinterpret_cast<const char*>(d[i].v6p);
      const char* tp = reinterpret_cast<const char*>(d[i].top);
      const size_t map = (size_t)4 * d[i].H * d[i].W;
      CHECK(v4 >= lo + pb && v4 + map + 256 <= hi);
      CHECK(v6 >= lo + pb && v6 + map <= hi);
      CHECK(tp >= lo + pb && tp + 4 * (size_t)d[i].W <= hi);
      CHECK(((uintptr_t)v4 % 256) == 0 && ((uintptr_t)v6 % 256) == 0);
    }
    CHECK(cols == sum_w && lt == lsum && gt == gsum);
    // frames of one shape (at least 3 x 3) give phase 2's per-frame tiling
    bool same = f[0].H >= 3 && f[0].W >= 3;
    for (int i = 1; i < n; ++i) same = same && f[i].H == f[0].H && f[i].W == f[0].W;
    if (same) {
      CHECK(hdr->g_rows_same == (f[0].H + hdr->gt_rows - 1) / hdr->gt_rows && hdr->g_cols_same == d[0].gcols);
      CHECK((long long)hdr->g_rows_same * hdr->g_cols_same * n == gt);
    } else {
      CHECK(hdr->g_rows_same == 0 && hdr->g_cols_same == 0);
    }
  }
}

}  // namespace

int main() {
  std::mt19937 rng(1234);
  params_and_sizes();
  argument_checks();
  plans(rng);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host logic ok\n");
  return 0;
}
