// Shared device/host definitions of the gfx950 depth-completion library.
//
// Two phases per frame (the column extension of Sec. III "Extension to Top
// of Frame" makes row 0 of a column depend on the lowest rows, so the chain
// is split where that global dependency sits):
//   phase 1 (local):  stages 1-4 on tiles with a halo; writes the stage-4
//                     map and, per column, the topmost non-empty row (atomic
//                     integer min);
//   phase 2 (global): stages 5-9 on tiles with a halo; reads the stage-4
//                     map and the column table, writes the output.
// Each phase has streaming kernels (stream.hip, one wave per tile) and LDS
// tile kernels (kernels.hip, one workgroup per tile).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipb {

constexpr int kThreads = 256;          // 4 wave64 per workgroup
constexpr int kNoTop = 0x7fffffff;      // column without a non-empty pixel

// One frame as the kernels see it.
struct FrameDesc {
  const float* in;
  float* out;
  float* v4;          // stage-4 map, H * W floats
  int32_t* top;       // W entries
  int32_t H, W;
  int32_t ltile0;     // first phase-1 tile of this frame within the launch
  int32_t gtile0;     // first phase-2 tile
  int32_t lcols;      // phase-1 tiles per row of tiles
  int32_t gcols;      // phase-2 tiles per row of tiles
  float* v6p;         // stage-6 values of the cells that were empty after stage 5 (H * W floats;
                      // only those cells are written and read).  Its first
                      // ceil(H / phase-1 tile rows) * W ints hold the phase-1
                      // column records (first non-empty and last empty row of
                      // each tile column) that the fill ahead of phase 2 reads;
                      // the general second pass overwrites them freely.
};

// Device-resident launch plan: header followed by n FrameDesc.
struct PlanHeader {
  int32_t n;
  int32_t ltiles;     // total phase-1 tiles
  int32_t gtiles;     // total phase-2 tiles
  int32_t ncols;      // total column-table entries (sum of W)
  int32_t* top_base;  // column tables of all frames, contiguous
  int32_t lt_rows, lt_cols;   // phase-1 tile shape the plan was built for
  int32_t gt_rows, gt_cols;   // phase-2 tile shape
  int32_t* slow;              // phase-2 tile queues, see SlowQueue
  int32_t slow_cap;           // capacity of each queue (phase-2 tiles of the launch)
  int32_t pad0;
  int32_t* ltab;              // frame index of every phase-1 tile (written by k_reset)
  int32_t* gtab;              // frame index of every phase-2 tile (written by k_reset)
  // phase-2 tile rows and columns of every frame when all frames have one
  // shape of at least 3 x 3 (else 0): k_global_rows then visits the tiles
  // bottom tile row first, over all frames
  int32_t g_rows_same, g_cols_same;
  int32_t pad1[12];
};
static_assert(sizeof(PlanHeader) == 128, "plan header layout");
static_assert(sizeof(FrameDesc) == 64, "frame descriptor layout");

// Kernel parameters, passed by value.
struct KParams {
  int32_t shape;      // ipb_se
  int32_t rd;         // dilation radius
  int32_t rc;         // closing radius
  int32_t rf;         // small fill radius
  int32_t extrapolate;
  int32_t rl;         // large fill radius
  int32_t rm;         // median radius (0 = off)
  int32_t rg;         // Gaussian radius (0 = off)
  float off;          // inversion offset
  float thr;          // empty iff value <= thr
  int32_t last_stage; // 1..9
  int32_t pad;
  double gw[3];       // Gaussian taps: centre, +-1, +-2 (integers for the binomial case)
  double gscale;      // applied to the 2-D sum (1/256 for binomial 5, 1/16 for 3)
  int32_t blur;       // 0 Gaussian, 1 bilateral
  int32_t ext_rows;   // stage-5 reach above the top; 0 = unlimited
  float bl_kc;        // bilateral: 1 / (2 sigma_color^2)
  float bl_ws[9];     // bilateral spatial weights, [|dy| * 3 + |dx|]
};

// Row of the stage-4 map that stage 5 reads for row y of a column whose
// topmost non-empty row is top (top >= H: none): the top row above it,
// within ext_rows rows when that is positive.
__host__ __device__ inline int v5_row(int y, int top, int H, int ext_rows) {
  return (top < H && y < top && (ext_rows <= 0 || y >= top - ext_rows)) ? top : y;
}

// Where a launch finds its frames: a device plan, or one frame by value.
struct FrameSource {
  const PlanHeader* plan;   // nullptr: single frame
  FrameDesc single;
  int32_t single_ltiles;
  int32_t single_gtiles;
  int32_t* slow;            // single frame: phase-2 tile queues, see SlowQueue
  int32_t slow_cap;
};

// Queues of the streaming kernels, in the workspace (gcap = phase-2 tiles,
// lcap = phase-1 tiles of the launch); eight counters, then the entries:
//   slow[0]   quarters whose input rows still hold an empty cell after the
//             extension and whose own rows hold at most kCellEmpty empty
//             cells (their cells go to the cell queue);
//   slow[2]   such quarters with more empty cells: the fill is computed
//             separably for the whole quarter (k_fill_dense);
//             entries of both: two ints, the frame index and the tile index
//             within the frame with the quarter in bits 27..28; both queues
//             then run again (k_global_patched);
//   slow[3]   cells of the first kind of quarter, each filled on its own
//             (k_fill_cells): two ints, the frame index and y * W + x;
//   slow[1]   tiles of frames under 3 rows or columns (launch tile ids),
//             recomputed by the LDS kernel;
//   slow[4]   32-row bands of phase-1 tiles that may hold a cell empty
//             after the extension, for the fill ahead of phase 2
//             (k_fill_scan, k_fill_tiles): two ints, the launch tile id and
//             the frame index with the band in bits 24..25;
//   slow[8 ..)              the first queue (8 gcap ints), the dense queue
//                           (8 gcap ints), the tiny-frame queue (gcap), the
//                           cell queue (8 kCellEmpty gcap ints), then the
//                           band queue (2 kBandsPerTile lcap ints).
// The first three queues and the cell queue serve the general phase 2 (its
// second pass); the phase-1 tile queue serves the default chain, whose fill
// runs before phase 2.
constexpr int kCellEmpty = 32;
constexpr int kQueueHead = 8;
constexpr int kBandRows = 32;      // rows of a band of the fill ahead of phase 2
constexpr int kBandsPerTile = 4;   // 32-row bands of a phase-1 tile (at most 128 rows)
__host__ __device__ inline size_t slow_queue_ints(int gcap, int lcap) {
  return kQueueHead + (17 + 8 * kCellEmpty) * (size_t)gcap + 2 * kBandsPerTile * (size_t)lcap;
}
__host__ __device__ inline int sparse_queue_offset(int) { return kQueueHead; }
__host__ __device__ inline int dense_queue_offset(int cap) { return kQueueHead + 8 * cap; }
__host__ __device__ inline int lds_queue_offset(int cap) { return kQueueHead + 16 * cap; }
__host__ __device__ inline int cell_queue_offset(int cap) { return kQueueHead + 17 * cap; }
__host__ __device__ inline int fill_queue_offset(int cap) { return kQueueHead + (17 + 8 * kCellEmpty) * cap; }

// Cells that the fill ahead of phase 2 wrote into the stage-4 map carry the
// sign bit: readers of stage-5 values take them as empty, the phase-2
// kernel clears the bit.
constexpr int kFillTag = (int)0x80000000u;

// Host-side launchers (kernels.hip).
hipError_t launch_reset(const FrameSource& src, int max_items, hipStream_t s);
// Copies a host plan (bytes, a multiple of 4) to device memory through the
// arguments of small kernels on the stream, kPlanChunkWords ints per launch.
constexpr int kPlanChunkWords = 896;   // 3584 bytes of kernel arguments
hipError_t launch_plan_upload(const void* plan_host, size_t bytes, void* plan_dev, hipStream_t s);
hipError_t launch_global_slow(const FrameSource& src, const KParams& kp, int stream_rows, int stream_cols,
                              int grid, hipStream_t s);
int slow_subtiles(int stream_rows, int stream_cols);
int slow_resident_blocks();

// Streaming kernels (stream.hip).
int stream_local_tile_rows(int id);
int stream_local_tile_cols(int id);
int stream_global_tile_rows(int id);
int stream_global_tile_cols(int id);
bool stream_local_supported(int shape, int rd, int rc, int rf);
bool stream_global_supported(int rm, int rg);
hipError_t launch_local_stream(const FrameSource& src, const KParams& kp, int tile_id, int grid, hipStream_t s);
hipError_t launch_global_stream(const FrameSource& src, const KParams& kp, int tile_id, bool fast, int grid,
                                hipStream_t s);
hipError_t launch_global_repair(const FrameSource& src, const KParams& kp, int tile_id, int grid, int cell_grid,
                                hipStream_t s);
hipError_t launch_prefill(const FrameSource& src, const KParams& kp, int local_rows, int scan_grid, int tile_grid,
                          bool all_bands, hipStream_t s);
bool fast_chain(const KParams& kp);
// whether the fill ahead of phase 2 takes the 31x31 window's kernel, and
// the resident workgroups per CU of the kernel it takes
bool prefill_full_window(const KParams& kp);
int prefill_resident_blocks(bool full_window);
hipError_t launch_local(const FrameSource& src, const KParams& kp, int tile_id, int halo,
                        int grid, hipStream_t s);
hipError_t launch_global(const FrameSource& src, const KParams& kp, int tile_id,
                         int grid, hipStream_t s);
int local_tile_rows(int tile_id);
int local_tile_cols(int tile_id);
int global_tile_rows(int tile_id);
int global_tile_cols(int tile_id);
int num_local_tiles();
int num_global_tiles();
int max_resident_blocks(int phase, int tile_id, int halo);

}  // namespace ipb
