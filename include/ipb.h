/*
 * ipb.h - C ABI of the MI355X (gfx950) depth-completion library.
 *
 * The library fills a sparse float32 depth map with the eight-step classical
 * pipeline of Ku, Harakeh & Waslander, "In Defense of Classical Image
 * Processing: Fast Depth Completion on the CPU" (2018), Sec. III "Proposed
 * Algorithm".  Problem statement (Sec. II, Eq. 1): given a sparse M x N depth
 * map, return a dense map of the same size with empty pixels replaced by
 * depth estimates; the method is unguided, so no image is taken.
 *
 * Stage numbers used by ipb_complete_stage():
 *   1 depth inversion           (Sec. III "Depth Inversion")
 *   2 kernel-shaped dilation    ("Custom Kernel Dilation")
 *   3 closing                   ("Small Hole Closure")
 *   4 small-hole fill           ("Small Hole Fill")
 *   5 extension to the top      ("Extension to Top of Frame")
 *   6 large-hole fill           ("Large Hole Fill")
 *   7 median blur               ("Median and Gaussian Blur")
 *   8 Gaussian blur             ("Median and Gaussian Blur")
 *   9 output inversion          (the final "Depth Inversion")
 * Stages 1-8 are in the inverted domain (valid = max_depth - depth, empty = 0);
 * stage 9 is the output depth map (empty = 0).
 *
 * Conventions shared by every entry point:
 *   - Maps are float32, row-major, pitch = W, in DEVICE memory.  1 <= H, W and
 *     H * W < 2^30 (the kernels address a map, and a scratch slot just past
 *     it, with 32-bit byte offsets).
 *   - Ownership: the caller owns every buffer (inputs, outputs, workspace) and
 *     keeps it alive until the stream work completes.  The library keeps no
 *     pointer after a call returns.
 *   - Errors: every function returns an ipb_status and never aborts.  All
 *     argument checks run before anything is enqueued: on error nothing is
 *     enqueued and the outputs are untouched.  Faults during kernel execution
 *     surface at the caller's next stream synchronisation, as with any HIP
 *     launch.  The library never synchronises the stream.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Results are bitwise deterministic.  The kernels' atomics are integer
 *     mins (column tops) and adds that hand out queue positions; every queued
 *     item writes cells no other item writes, so no result depends on the
 *     order of a queue.
 */
#ifndef IPB_H
#define IPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IPB_OK = 0,
  IPB_ERR_INVALID_ARG = -1,   /* null pointer, bad size, bad parameter, overlap  */
  IPB_ERR_UNSUPPORTED = -2,   /* a parameter value outside what the kernels hold */
  IPB_ERR_WORKSPACE = -3,     /* workspace missing or smaller than required      */
  IPB_ERR_HIP = -4,           /* a HIP call failed; see ipb_last_hip_error()     */
  IPB_ERR_SCRATCH = -5        /* ipb_complete_static: frame too large for the
                                 static scratch                                  */
} ipb_status;

/* Kernel shapes compared in Sec. IV "Custom Kernel Design" (Table 2).  The
 * figure that draws them is not available; the shapes are read from their
 * names: FULL all k x k, CROSS the centre row and column, DIAMOND
 * |dx| + |dy| <= k/2, CIRCLE dx^2 + dy^2 <= (k/2)^2. */
typedef enum { IPB_SE_FULL = 0, IPB_SE_CROSS = 1, IPB_SE_DIAMOND = 2, IPB_SE_CIRCLE = 3 } ipb_se;

/* Stage-8 blur: the Gaussian of the final design, or the bilateral blur the
 * paper compares it with (Sec. IV "Noise Reduction through Blurring",
 * Table 3) and recommends for point clouds.  The bilateral blur weighs each
 * tap of the (gauss_size)^2 window by exp(-(dy^2 + dx^2) / (2 s^2)) *
 * exp(-(v_q - v_p)^2 / (2 c^2)) (s = bilateral_sigma_space in pixels,
 * c = bilateral_sigma_color in depth units), divides by the weights' sum,
 * reflects about the edge pixel at the border and, like the Gaussian, is
 * written only where the median output is non-empty.  It is computed in
 * float32 (within 1e-5 relative of the float64 definition). */
typedef enum { IPB_BLUR_GAUSSIAN = 0, IPB_BLUR_BILATERAL = 1 } ipb_blur;

/* Pipeline parameters.  Defaults (ipb_params_default) are the paper's final
 * design.  Supported values are listed per field; anything else returns
 * IPB_ERR_UNSUPPORTED. */
typedef struct {
  uint32_t struct_size;     /* = sizeof(ipb_params); set by ipb_params_default    */
  int32_t dilate_shape;     /* ipb_se; DIAMOND (Sec. III, Table 2)                 */
  int32_t dilate_size;      /* 3, 5 or 7; 5 (Sec. IV "Custom Kernel Design")       */
  int32_t close_size;       /* full kernel, 3, 5 or 7; 5 ("Small Hole Closure")    */
  int32_t fill_size;        /* full kernel, 3, 5 or 7; 7 ("Small Hole Fill")       */
  int32_t extrapolate;      /* 1: run stages 5 and 6; 0: skip both (the point-cloud
                               use described in Sec. IV)                           */
  int32_t large_fill_size;  /* full kernel, odd 3..31; 31 ("Large Hole Fill")      */
  int32_t median_size;      /* 0 (off), 3 or 5; 5 ("Median and Gaussian Blur")     */
  int32_t gauss_size;       /* 0 (off), 3 or 5; 5                                  */
  float gauss_sigma;        /* <= 0: binomial taps (1 4 6 4 1)/16 for size 5;
                               > 0: exp(-i^2 / 2 sigma^2), normalised              */
  float max_depth;          /* inversion offset, 100.0 (Sec. III "Depth Inversion");
                               must exceed 2 * valid_thresh                        */
  float valid_thresh;       /* a value is empty iff <= this; 0.1; > 0              */
  int32_t tile_local;       /* tile shape id for stages 1-4; 0 = automatic         */
  int32_t tile_global;      /* tile shape id for stages 5-9; 0 = automatic         */
  int32_t blur;             /* ipb_blur; GAUSSIAN                                  */
  float bilateral_sigma_space;  /* > 0; 2.0 (not given in the paper)              */
  float bilateral_sigma_color;  /* > 0; 1.5 (not given in the paper)              */
  int32_t extend_rows;      /* >= 0; rows above its top a column's value reaches in
                               stage 5; 0 = up to row 0 (Sec. III); a positive
                               limit is the point-cloud advice of Sec. IV         */
} ipb_params;

/* Fill *p with the paper's defaults (Sec. III; Tables 2 and 3: diamond 5x5
 * dilation, 5x5 closing, 7x7 fill, extension, 31x31 fill, 5x5 median, 5x5
 * Gaussian, offset 100).  p must not be NULL. */
void ipb_params_default(ipb_params* p);

/* Workspace bytes one frame of H x W needs: the stage-4 map, a map for the
 * large-fill values of cells left empty after the extension (its start also
 * holds the phase-1 column records), one int32 per column and the queues of
 * the tiles, bands and cells that need the large fill.  With tile_local 0 a
 * frame whose 64-row phase-1 tiles give the GPU fewer than two waves per
 * SIMD (2048 waves) takes 32-row ones, 16-row ones if those give fewer than
 * one (1024), 8-row ones if 16-row ones give fewer than half (512); with
 * tile_global 0 and the default chain (stages 1-4 and 5-9 on the streaming
 * kernels, 5x5 median) phase 2 takes the tallest of 32, 16 and 8 rows that
 * gives at least four (4096), here and in the calls below.
 * Returns 0 for invalid sizes or parameters. */
size_t ipb_workspace_bytes(int H, int W, const ipb_params* p);

/* Complete one frame: depth_in (H x W, device) -> depth_out (H x W, device).
 * The whole chain of Sec. III, stages 1-9.  The workspace is taken from the
 * stream-ordered allocator (hipMallocAsync) and released on the stream.
 * depth_out == depth_in (in place) is allowed; any other overlap is
 * IPB_ERR_INVALID_ARG. */
int ipb_complete(const float* depth_in, int H, int W, const ipb_params* p,
                 float* depth_out, void* stream);

/* As ipb_complete with a caller-supplied device workspace of at least
 * ipb_workspace_bytes(H, W, p) bytes (256-byte aligned).  Allocates nothing,
 * synchronises nothing. */
int ipb_complete_ws(const float* depth_in, int H, int W, const ipb_params* p,
                    float* depth_out, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * ipb_complete_ws with the library's own static device array of
 * IPB_STATIC_SCRATCH_BYTES as the workspace, one per GPU, held until the
 * process ends.  Allocates nothing (no hipMalloc, no allocating library
 * call; the array's device address is looked up once per device on the
 * first call there) and synchronises nothing.  Frames whose workspace
 * (ipb_workspace_bytes) exceeds the array return IPB_ERR_SCRATCH before
 * anything is enqueued: 1024 x 4096 fits with the default parameters.  The
 * array keeps the last call's contents; each call clears what must start
 * at zero.  Every call on a GPU shares that GPU's array: calls that overlap
 * in time on one GPU (on different streams, or from different threads with
 * no stream order between them) race and give wrong results; order them on
 * one stream. */
#define IPB_STATIC_SCRATCH_BYTES ((size_t)48 << 20)
int ipb_complete_static(const float* depth_in, int H, int W, const ipb_params* p,
                        float* depth_out, void* stream);

/* Test hook: run stages 1..last_stage (1 <= last_stage <= 9) and write the map
 * of stage last_stage to out (see the stage list above).  Same workspace rule
 * as ipb_complete_ws. */
int ipb_complete_stage(const float* depth_in, int H, int W, const ipb_params* p,
                       float* out, int last_stage, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- batches --
 * Many frames of any sizes in one launch per phase.  Frames are independent
 * (Sec. II: the map is completed from its own points only). */
typedef struct {
  const float* in;          /* device, H x W                                      */
  float* out;               /* device, H x W; may equal in; frames must not overlap
                               each other                                          */
  int32_t H, W;
} ipb_frame;

/* Workspace for a batch: the launch plan, then per frame what
 * ipb_workspace_bytes lists.  With tile id 0 it covers both layouts a batch
 * may take: ipb_complete_batch's (the smaller tiles of ipb_workspace_bytes
 * when the frames are too few to give the GPU a wave per SIMD with the
 * default ones) and ipb_batch_plan's (the default tiles).  Returns 0 if any frame is invalid,
 * two frames' outputs overlap another frame's buffers, or n < 1. */
size_t ipb_batch_workspace_bytes(const ipb_frame* frames, int n, const ipb_params* p);

/* Complete n frames (host array of descriptors with device pointers).  The
 * launch plan is built in host memory of the calling thread and written into
 * the workspace by small upload kernels on the stream that take it in their
 * arguments, so the caller's array may be reused when the call returns.
 * Allocates no device or pinned memory, synchronises nothing, reads no
 * device memory on the host: the call can be captured into a graph (whose
 * replays then complete the same frames; for new frames per replay use
 * ipb_batch_plan and ipb_complete_planned). */
int ipb_complete_batch(const ipb_frame* frames, int n, const ipb_params* p,
                       void* ws, size_t ws_bytes, void* stream);

/* Bytes of the launch plan for n frames (host side and device side alike). */
size_t ipb_batch_plan_bytes(int n);

/* Build, in host memory plan_host (ipb_batch_plan_bytes(n) bytes), the launch
 * plan of n frames whose workspace will be ws (device, ws_bytes).  The plan
 * holds device pointers into ws.  The caller copies it to device memory
 * (plan_dev) and passes that to ipb_complete_planned; with a pinned plan
 * buffer and a captured copy, a graph can be replayed for new frames (up to
 * the sizes the workspace was sized for) by rewriting the host plan. */
int ipb_batch_plan(const ipb_frame* frames, int n, const ipb_params* p,
                   void* ws, size_t ws_bytes, void* plan_host, size_t plan_bytes);

/* Run a planned batch.  plan_dev: device copy of a plan built by
 * ipb_batch_plan with the same parameters p; max_tiles_local/global and
 * max_cols bound the plans it may be replayed with (the launch grids are
 * derived from them, so the call can be captured once and replayed).
 * phase: -1 = everything; -2 = everything but step 5, for callers that
 * know no frame of the plans the call runs with has under 3 rows or columns
 * (a tiny frame in such a plan is left incomplete); else one launch step, in
 * this order:
 *   0 reset the column tables and the tile queues;
 *   1 stages 1-4;
 *   2 the default chain (Sec. III; Tables 2 and 3: 5x5 median, 5x5
 *     binomial Gaussian, the full extension) on the streaming kernels: the 31x31
 *     fill of the cells that are empty after stage 5, written into the
 *     stage-4 map ahead of phase 2 (no-op otherwise);
 *   3 stages 5-9 (other chains on the streaming kernel: every tile,
 *     assuming the 31x31 fill changes nothing; tile quarters where it does
 *     are queued);
 *   4 the queued quarters: the fill at their empty cells, then stages 7-9
 *     again (streaming kernels, chains other than the default; no-op
 *     otherwise);
 *   5 tiles of frames under 3 rows or columns (streaming kernels only).
 * The split exists for per-kernel timing.  Allocates nothing, synchronises
 * nothing, reads no device memory on the host. */
int ipb_complete_planned(const void* plan_dev, const ipb_params* p, int phase,
                         int max_tiles_local, int max_tiles_global, int max_cols,
                         void* stream);

/* Totals of a host plan: tiles per phase and columns (for max_* above). */
int ipb_plan_totals(const void* plan_host, int* n, int* tiles_local, int* tiles_global, int* cols);

/* ------------------------------------------------------------------ misc -- */

/* Static text of a status code. */
const char* ipb_status_string(int status);

/* The hipError_t behind the calling thread's last IPB_ERR_HIP (0 if none). */
int ipb_last_hip_error(void);

/* A stream of the current device with a hardware queue of its own, for
 * callers that keep several batches in flight.  The runtime maps ordinary
 * streams onto a small pool of hardware queues (GPU_MAX_HW_QUEUES, 4 by
 * default), so two of them can share one queue and run their batches one
 * after the other; a stream created with a compute-unit mask always gets a
 * queue of its own.  The mask names every compute unit, so kernels on the
 * stream still use the whole device.  The stream is at the default
 * priority and, as any stream created without flags, synchronises with the
 * legacy null stream.  On success *stream holds the hipStream_t; the caller
 * owns it and releases it with ipb_stream_destroy.  Returns
 * IPB_ERR_INVALID_ARG for a null pointer (*stream is then untouched) and
 * IPB_ERR_HIP if the runtime refuses (*stream is then null). */
int ipb_stream_create(void** stream);

/* Destroys a stream made by ipb_stream_create once its queued work has
 * finished (as hipStreamDestroy).  IPB_ERR_INVALID_ARG for a null stream. */
int ipb_stream_destroy(void* stream);

/* Tile shapes (rows, cols) of a tile id for phase 1 (local) or 2 (global);
 * returns IPB_ERR_INVALID_ARG for an unknown id.  Id 0 = automatic.  Ids
 * 1-4 are LDS tiles, 5 and up streaming tiles (phase 1: 64, 128, 32, 16, 8
 * and 96 rows of 108 columns for ids 5-10).  Phase-2 ids 8 and 9 (16- and
 * 8-row streaming tiles) serve the default chain only; with any other chain
 * they are IPB_ERR_UNSUPPORTED. */
int ipb_tile_shape(int phase, int tile_id, int* rows, int* cols);

/* Number of tile ids per phase (ids 1..count). */
int ipb_tile_count(int phase);

#ifdef __cplusplus
}
#endif
#endif /* IPB_H */
