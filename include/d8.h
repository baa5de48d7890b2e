/*
 * d8.h -- C ABI of the MI355X (gfx950) D8 flow-direction and up-slope-area library.
 *
 * Method: Barnes, Lehman & Mulla, "Distributed Parallel D8 Up-Slope Area
 * Calculation in Digital Elevation Models" (PDPTA 2011).
 *   - Sec. 2, Eq. (1): up-slope area A(p) = w(p) + sum of A(i) over the cells i
 *     that drain into p (w = 1 gives the cell count; Sec. 2 allows weights).
 *   - Sec. 1: the D8 function sends all of a cell's flow to the lowest of its
 *     eight neighbours, so flows join but never split (the field is a forest).
 *   - Sec. 3: the DEM is partitioned; each part computes its internal area with
 *     the inflows from other parts left as unknowns (Alg. 1-4), one solve over
 *     the parts' border graph resolves them (Alg. 5-6), and each part adds the
 *     resolved inflows along its downstream paths (Alg. 7-8).  Here the parts
 *     are square tiles of one GPU's DEM and the border graph is solved on the
 *     GPU in O(log depth) rounds.
 *
 * Conventions shared by every entry point
 *   Grids are row-major, `rows` x `cols`, contiguous, row 0 = north edge,
 *   column 0 = west edge.  NoData = NaN in a DEM, code 255 in a direction field.
 *   Direction codes (uint8): 0 E (0,+1), 1 NE (-1,+1), 2 N (-1,0), 3 NW (-1,-1),
 *   4 W (0,-1), 5 SW (+1,-1), 6 S (+1,0), 7 SE (+1,+1), 8 outlet, 255 NoData.
 *   A cell with code 0..7 drains into the neighbour at that offset.
 *
 * Ownership and ordering
 *   Every array argument is a DEVICE pointer owned by the caller (the library
 *   never allocates device memory), except the host arrays of
 *   d8_accum_streamed.  Scratch memory is a caller-owned device
 *   workspace of at least d8_*_workspace_bytes() bytes, 256-byte aligned.
 *   Outputs must not alias inputs.  Every call only enqueues work on `stream`
 *   (a hipStream_t; NULL = the default stream) and returns; there is no hidden
 *   synchronisation, so calls may be captured into a HIP graph (the
 *   exceptions, d8_fill_eps and d8_accum_streamed, say so).
 *
 * Errors
 *   Argument errors (NULL pointers, rows*cols == 0 or > 2^32-1, rows or cols
 *   > 2^31-1, unsupported tile, workspace too small, a HIP launch failure)
 *   are returned at once and nothing is enqueued.  Data errors found on the
 *   device (a direction code outside {0..8, 255}; a target off the grid or
 *   into NoData; a cycle) are OR-ed into a status word in the workspace; the
 *   computation still runs to completion and the outputs of affected cells
 *   are unspecified.  Read the word with d8_device_status() after the call.
 */
#ifndef D8_H_
#define D8_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  D8_OK = 0,
  D8_EINVAL = 1,        /* bad argument */
  D8_ENOMEM = 2,        /* workspace too small */
  D8_EHIP = 3,          /* a HIP runtime call or launch failed */
  D8_EBADDIR = 4,       /* device: bad direction code or target off-grid / into NoData */
  D8_ECYCLE = 5,        /* device: the direction field contains a cycle */
  D8_EUNSUPPORTED = 6   /* combination the library does not implement */
} d8_status;

enum { D8_E = 0, D8_NE, D8_N, D8_NW, D8_W, D8_SW, D8_S, D8_SE, D8_NONE = 8, D8_NODATA = 255 };

typedef enum { D8_U32 = 0, D8_F32 = 1 } d8_dtype;

/* One DEM of a batch: element offset of its first cell in the packed buffers
 * (the same offset is used for dem, dirs, weights, outputs and gradients) and
 * its shape.  Host array for d8_batched_workspace_bytes and the host_desc
 * arguments, device array for the dev_desc arguments of the batched launches. */
typedef struct {
  int64_t offset;
  int32_t rows;
  int32_t cols;
} d8_desc;

/* Tile sides accepted by `tile`: 0 (library default, 64), 32, 64, and 128
 * for counts.  Larger tiles do not fit a CU's 160 KiB of LDS. */
#define D8_TILE_DEFAULT 0

/* ------------------------------------------------------------------------ */
/* Flow directions (Sec. 1 "lowest of eight"; Sec. 3 halo of neighbour rows). */

/* dem: float32 [rows*cols]; dirs: uint8 [rows*cols] (output).
 * A NaN cell gets 255.  A valid cell on the DEM boundary or 8-adjacent to NaN
 * gets 8.  Otherwise the neighbours are scanned E,NE,N,NW,W,SW,S,SE and the
 * first one strictly lower than every earlier candidate and than the cell
 * wins; with no strictly lower neighbour the cell gets 8.  Exact (compares
 * only).  No workspace. */
d8_status d8_flowdirs(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, void* stream);

/* Steepest-slope variant (Sec. 3 states the D8 rule as the largest drop over
 * the distance to the neighbour, distance 1 for E, N, W, S and sqrt(2) for the
 * diagonals; Sec. 1 as the lowest neighbour, which d8_flowdirs follows).  Same
 * arguments, NoData and edge rules as d8_flowdirs.  The slope to neighbour d
 * is evaluated in double precision as (z_cell - z_d) * f_d, f_d = 1 or
 * 1/sqrt(2) rounded to double; the largest strictly positive slope wins, ties
 * to the first in E,NE,N,NW,W,SW,S,SE order; with no positive slope the cell
 * gets 8.  Exact for that definition.  No workspace. */
d8_status d8_flowdirs_steepest(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, void* stream);

/* ------------------------------------------------------------------------ */
/* Up-slope area (Eq. 1) over a direction field. */

/* Bytes of workspace the forward calls (d8_accum, d8_accum_dem) need for this
 * shape and tile (0 = default).  Returns 0 for an invalid shape or tile. */
size_t d8_workspace_bytes(int64_t rows, int64_t cols, int tile);

/* Bytes of workspace d8_accum_backward needs: d8_workspace_bytes plus 6 bytes
 * per cell, which hold between its two tile passes each cell's in-tile path
 * sum (low part) and the tile exit its path leaves by.  Returns 0 for an
 * invalid shape or tile. */
size_t d8_backward_workspace_bytes(int64_t rows, int64_t cols, int tile);

/* dirs: uint8 codes [rows*cols].
 * weights: float32 [rows*cols], or NULL for unit weights.
 * out_dtype: D8_U32 (counts; requires weights == NULL) or D8_F32.
 * out: uint32 or float32 [rows*cols] (output).  NoData cells get 0.
 *   Counts are exact.  Weighted sums are accumulated in fp64 (inside tiles
 *   and across tiles); out = RN32(sum).
 * out_lo: NULL, or float32 [rows*cols] receiving RN32(sum - out), so that
 *   out + out_lo carries about 48 significant bits of the fp64 sum (weighted
 *   only).
 * ws / ws_bytes: workspace.  tile: 0, 32, 64, or 128 (counts only). */
d8_status d8_accum(const uint8_t* dirs, int64_t rows, int64_t cols, const float* weights,
                   d8_dtype out_dtype, void* out, float* out_lo, void* ws, size_t ws_bytes, int tile,
                   void* stream);

/* For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same as d8_accum, with the
 * workspace taken from a static device array of the library
 * (D8_NOALLOC_SCRATCH_BYTES per GPU; each GPU the library runs on holds it
 * until the process ends) instead of a caller workspace; the call allocates
 * nothing.  Shapes whose d8_workspace_bytes exceed the array (at tile 64
 * about 1.9 bytes per cell, so up to about 5900 x 5900 cells) return
 * D8_ENOMEM and enqueue nothing.  Every call on one GPU uses that GPU's array:
 * calls that overlap in time on one GPU (concurrent streams, threads) race.
 * status: NULL, or a device uint32 that receives, on `stream` after the
 * call's kernels, its data-error word (0; bit 0: a bad direction code or a
 * target off the grid or into NoData; bit 1: a cycle). */
#define D8_NOALLOC_SCRATCH_BYTES (64u << 20)
d8_status d8_accum_noalloc(const uint8_t* dirs, int64_t rows, int64_t cols, const float* weights,
                           d8_dtype out_dtype, void* out, float* out_lo, int tile, uint32_t* status,
                           void* stream);

/* Fused flow directions and counts: dem (float32, NaN = NoData) -> dirs and
 * out, equal to d8_flowdirs followed by d8_accum with unit weights and
 * D8_U32 output.  The tile pass computes each tile's codes from the DEM
 * (with a two-cell halo) instead of reading a direction field, so one read
 * of the DEM replaces d8_flowdirs' read and write and the tile pass' read of
 * the codes.  dirs (uint8 [rows*cols], output) receives the codes.  Same
 * workspace, tile and error rules as d8_accum. */
d8_status d8_accum_dem(const float* dem, int64_t rows, int64_t cols, uint8_t* dirs, uint32_t* out, void* ws,
                       size_t ws_bytes, int tile, void* stream);

/* Adjoint of the weighted accumulation.  The map w -> A is linear,
 * A = (I - P)^-1 w with P the D8 drainage matrix, so for a loss with
 * dL/dA = grad_out the gradient is grad_weights = (I - P)^-T grad_out:
 * grad_weights(c) = sum of grad_out over the cells on c's downstream path,
 * c included.  grad_out, grad_weights: float32 [rows*cols]; NoData -> 0.
 * Path sums in fp64 (the in-tile part carried between the tile passes as a
 * float32 pair, to 2^-48 of its magnitude), rounded to float32 once, in a
 * fixed order: the result is the same on every run.  ws_bytes: at least
 * d8_backward_workspace_bytes(rows, cols, tile).  tile: 0, 32 or 64. */
d8_status d8_accum_backward(const uint8_t* dirs, int64_t rows, int64_t cols, const float* grad_out,
                            float* grad_weights, void* ws, size_t ws_bytes, int tile, void* stream);

/* Up-slope counts of a direction field that stays in host memory (Sec. 4,
 * Conclusions: on one node the method can keep intermediate results out of
 * core and so handle DEMs larger than memory; here the per-tile perimeter
 * records and the resolve stay on the device while the field and the counts
 * stream through it).
 * dirs_host: uint8 codes [rows*cols], out_host: uint32 [rows*cols] (output),
 * both HOST pointers (pinned memory lets the copies run at full PCIe rate).
 * strip_rows: rows per strip, a positive multiple of 64.  Row strips are
 * copied to the device twice: once for the tile pass with unknown inflows
 * (whose tile-local counts go back to out_host), once with those counts for
 * the finalising pass.  The kernels run on `stream`; the copies run on two
 * streams of the call's own (created and destroyed inside it, default
 * priority), so the next strip's upload and the previous strip's download
 * overlap the current strip's kernels.  ws: device workspace of
 * d8_accum_streamed_workspace_bytes(rows, cols, strip_rows) bytes (the
 * d8_workspace_bytes of the DEM at tile 64 plus two strip slots, about
 * 10 B per strip-row cell).  Same results and data-error reporting as
 * d8_accum with unit weights, tile 64.  SYNCHRONISES `stream` before
 * returning (the host buffers are in use until then). */
size_t d8_accum_streamed_workspace_bytes(int64_t rows, int64_t cols, int64_t strip_rows);
d8_status d8_accum_streamed(const uint8_t* dirs_host, int64_t rows, int64_t cols, uint32_t* out_host,
                            int64_t strip_rows, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Conditioning (Sec. 3 assumes the DEM is free of pits and flats before the
 * method runs: a pit is raised to the level it drains at, flats get small
 * elevation changes; the paper leaves the algorithm open).  Epsilon fill
 * (Planchon & Darboux 2002): seeds are the valid cells on the DEM boundary or
 * 8-adjacent to NaN and keep their elevation; every other valid cell gets the
 * unique fixed point F(c) = max(z(c), min over valid neighbours n of
 * inc(F(n))), inc(x) = fl32(x + eps) or, where that rounds back to x, the next
 * float above x.  Min and max follow the total order of the float bits (-0
 * below +0), so the result is exact and independent of evaluation order.
 * Afterwards lowest-of-eight (d8_flowdirs) gives outlets exactly at the seeds.
 *
 * dem: float32 [rows*cols] (NaN = NoData); out: float32 [rows*cols] (output,
 * NaN where dem is NaN; must not overlap dem).  eps: a positive normal float.
 * ws: workspace of d8_fill_workspace_bytes(rows, cols) bytes, 256-aligned.
 * rounds: NULL, or receives the number of tile rounds that had work.
 * Unlike every other entry point this call SYNCHRONISES `stream`: it runs
 * rounds of 64x64-tile relaxation until no tile changes, and reads the length
 * of the next round's tile queue back to the host every few rounds.  Returns
 * D8_ECYCLE if 2^24 rounds pass without convergence (not reachable for
 * finite inputs in practice). */
size_t d8_fill_workspace_bytes(int64_t rows, int64_t cols);
d8_status d8_fill_eps(const float* dem, int64_t rows, int64_t cols, float eps, float* out, void* ws,
                      size_t ws_bytes, int64_t* rounds, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched: n DEMs of uneven shapes packed in one buffer, one set of launches
 * for the whole batch.  host_desc / dev_desc describe the same n DEMs (host
 * and device copies).  A DEM may not exceed 2^31-1 cells.
 * `waves` (0 = default) picks the launch shape of the tile passes:
 *   tile 64: one tile per workgroup of 64 * waves threads; waves 2, 4, 8
 *     (default) or 16, i.e. 32, 16, 8 or 4 cells per thread of the in-LDS
 *     doubling pass; for counts (D8_U32) waves 1, 2 and 4 instead select the
 *     last-arriver walk pass (Alg. 2's queue) with that many waves per tile;
 *   tile 32: workgroups of waves = 1 (default), 2 or 4 tiles, 64 * waves
 *     threads, 16 cells per thread;
 *   tile 128 (counts only): one tile per workgroup of 1024 threads (waves 16).
 * Other values return D8_EUNSUPPORTED.  d8_autotune_batched times every
 * shape the fp64 passes accept. */

/* Workspace of the batched forward calls, and of d8_accum_backward_batched
 * (6 more bytes per packed cell, up to the largest offset + rows * cols). */
size_t d8_batched_workspace_bytes(const d8_desc* host_desc, int32_t n, int tile);
size_t d8_batched_backward_workspace_bytes(const d8_desc* host_desc, int32_t n, int tile);

/* Flow directions for every DEM of the batch (same rule as d8_flowdirs).
 * ws: workspace of d8_batched_workspace_bytes(host_desc, n, 0) bytes (only
 * its header and DEM table are used). */
d8_status d8_flowdirs_batched(const float* dem_packed, const d8_desc* host_desc, const d8_desc* dev_desc,
                              int32_t n, uint8_t* dirs_packed, void* ws, size_t ws_bytes, void* stream);

d8_status d8_accum_batched(const uint8_t* dirs_packed, const d8_desc* host_desc, const d8_desc* dev_desc,
                           int32_t n, const float* w_packed, d8_dtype out_dtype, void* out_packed,
                           float* out_lo_packed, void* ws, size_t ws_bytes, int tile, int waves,
                           void* stream);

d8_status d8_accum_backward_batched(const uint8_t* dirs_packed, const d8_desc* host_desc,
                                    const d8_desc* dev_desc, int32_t n, const float* g_packed,
                                    float* gw_packed, void* ws, size_t ws_bytes, int tile, int waves,
                                    void* stream);

/* Times the batched weighted forward+backward (d8_accum_batched with D8_F32,
 * then d8_accum_backward_batched) at every (tile, waves) pair the fp64 passes
 * accept -- tile 32 with waves 1, 2, 4 and tile 64 with waves 2, 4, 8, 16 --
 * on the given inputs (synchronising `stream`), best of two timed repeats
 * after one warm-up, and writes the fastest pair.  Outputs are scratch.  ws
 * must be sized for the backward at the largest tile side tried
 * (d8_batched_backward_workspace_bytes with tile 32). */
d8_status d8_autotune_batched(const uint8_t* dirs_packed, const d8_desc* host_desc, const d8_desc* dev_desc,
                              int32_t n, const float* w_packed, float* out_scratch, float* g_scratch,
                              void* ws, size_t ws_bytes, int* best_tile, int* best_waves, float* best_ms,
                              void* stream);

/* ------------------------------------------------------------------------ */

/* Synchronises `stream`, then reads the device status word of `ws` into
 * *status_out (D8_OK, or the first of D8_EBADDIR / D8_ECYCLE found) and
 * returns D8_OK, or D8_EHIP if the read failed. */
d8_status d8_device_status(const void* ws, void* stream, int32_t* status_out);

/* Static text for a status code. */
const char* d8_strerror(d8_status s);

/* Phase timing, for measurement tools.  d8_phase_timing(1) clears the
 * totals and makes every later call record a HIP event on its stream before
 * and after each kernel phase; d8_phase_timing(0) stops recording.
 * d8_phase_report synchronises the recorded events and returns, for phase
 * index `phase` (0 .. D8_NPHASES-1), its name, the summed milliseconds and the
 * number of timed calls.  Not thread-safe; host-side state only. */
#define D8_NPHASES 10
d8_status d8_phase_timing(int enable);
d8_status d8_phase_report(int phase, const char** name, float* total_ms, int32_t* calls);

/* Library version string. */
const char* d8_version(void);

#ifdef __cplusplus
}
#endif

#endif /* D8_H_ */
