/*
 * d8flow.h -- C ABI of the MI355X (gfx950) D8 flow-accumulation library.
 *
 * The library computes flow accumulation, Eq. (1) of Barnes, "Parallel
 * Non-divergent Flow Accumulation For Trillion Cell Digital Elevation Models
 * On Desktops Or Clusters" (arXiv:1608.04431), for non-divergent (D8) flow:
 *
 *     A(p) = w(p) + sum of A(n) over the neighbours n whose flow goes to p,
 *
 * with the paper's tile decomposition (Section "The Algorithm"; Algorithms 1-3):
 * every tile is accumulated locally, the tiles' perimeter links and partial
 * sums form one small global graph that is solved, and a second pass over each
 * tile adds the resolved inflows (the EVICT strategy).  It also provides the
 * D8 directions that feed it and the adjoint of the accumulation.
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *     owned by the caller, row-major and contiguous: cell (r, c) is element
 *     r * cols + c.  The library never frees, retains or reallocates them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls only enqueue work on it and return; they do not synchronise and do
 *     not allocate device memory.  Scratch memory is the caller's workspace
 *     `ws` of at least d8_workspace_bytes(...) bytes.
 *   - Synchronous argument errors are returned as negative codes before
 *     anything is enqueued.  Errors that depend on the data (an invalid
 *     direction code, a cycle) are recorded in a status word inside `ws` and
 *     read with d8_check_status(); outputs are then undefined.
 *   - Work sharing one workspace must be ordered (same stream or events): the
 *     workspace holds intermediate results between kernels.
 */
#ifndef D8FLOW_H
#define D8FLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One byte per cell (Section "Data Types": ten distinct values).  The paper
 * does not fix the encoding; this one is a 3x3 scan without the centre, so
 * the opposite of direction k is 7 - k. */
enum d8_code {
    D8_NW = 0, D8_N = 1, D8_NE = 2, D8_W = 3, D8_E = 4, D8_SW = 5, D8_S = 6, D8_SE = 7,
    D8_NOFLOW = 8, /* part of the DEM, no flow direction: an outlet */
    D8_NODATA = 9  /* not part of the DEM; codes 10..255 are invalid */
};

enum d8_status {
    D8_OK = 0,
    D8_EINVAL = -1,     /* bad argument: null pointer, size, tile shape, type   */
    D8_EWORKSPACE = -2, /* workspace missing, not 256-byte aligned, or too small */
    D8_EHIP = -3,       /* a HIP launch or runtime call failed                   */
    D8_EDIRCODE = -4,   /* (data) a direction code above 9 was found             */
    D8_ECYCLE = -5      /* (data) the directions contain a cycle                 */
};

enum d8_acc_type {
    D8_ACC_U32 = 0, /* unit weights, exact 32-bit counts (weights must be NULL)  */
    D8_ACC_F32 = 1  /* float32 weights (NULL = unit), float32 result             */
};

/* Largest tile side supported by the tile kernels (one wavefront per tile,
 * one lane per tile row), in cells. */
#define D8_MAX_TILE_SIDE 64

/*
 * D8 flow directions (O'Callaghan & Mark 1984; the paper's non-divergent
 * example, Introduction, and the "separate algorithm" that produces its input,
 * Section "The Algorithm").  For every cell:
 *   NoData (9)  if dem == nodata or dem is NaN;
 *   else the neighbour k (0..7) with the steepest strictly positive descent,
 *        the float32 drop d = z_c - z_n divided by 1 (cardinal) or sqrt(2)
 *        (diagonal), compared exactly (2 d^2 vs d^2 in double); equal slopes
 *        keep the lowest k; off-raster and NoData neighbours are not candidates;
 *   else NoFlow (8).
 * dem: float32 [rows*cols] (in); dirs: uint8 [rows*cols] (out).
 * rows, cols >= 0 (an empty raster is a no-op).  Returns D8_OK, D8_EINVAL
 * (null pointer with a non-empty raster, negative size) or D8_EHIP.
 */
int d8_directions(const float *dem, uint8_t *dirs, int64_t rows, int64_t cols, float nodata,
                  void *stream);

/*
 * rho8 directions (Fairfield and Leymarie, 1991), the other non-divergent
 * metric the paper's Introduction names: as d8_directions, but the distance
 * to a diagonal neighbour is t = fl32(2 - r(c)) instead of sqrt 2, with r(c)
 * one uniform draw in [0, 1) per cell supplied by the caller (rnd, float32
 * [rows*cols], the dem's layout; values outside [0, 1) are used as given).
 * The diagonal factor 1 / t lies in (1/2, 1] with mean ln 2, so straight
 * drainage lines no longer follow the grid's preferred directions.  The
 * steepest slope wins, compared exactly (drop against t times the cardinal
 * drop in double); the lowest index wins ties.  Returns as d8_directions.
 */
int d8_directions_rho8(const float *dem, const float *rnd, uint8_t *dirs, int64_t rows, int64_t cols,
                       float nodata, void *stream);

/*
 * Workspace needed by flow_accum / flow_accum_adjoint for this raster and tile
 * shape (tile_rows = tile_cols = 0 picks the default shape).  One workspace
 * serves both calls.  Returns 0 for an invalid tile shape.
 */
size_t d8_workspace_bytes(int64_t rows, int64_t cols, int tile_rows, int tile_cols);

/*
 * Flow accumulation, Eq. (1) with alpha in {0,1} (Introduction), by the tiled
 * method of Algorithms 1-3:
 *   pass 1   per tile, dependency counts and the Kahn order of Algorithm 1 in
 *            LDS, and Algorithm 2's links for every perimeter cell;
 *   resolve  the global flow graph of perimeter cells, joined across tile
 *            edges and corners (Section "Constructing a Global Solution");
 *   pass 2   per tile, Algorithm 1 again with each perimeter cell's resolved
 *            cross-tile inflow added to its own weight (EVICT, Section
 *            "Broadcasting & Finalizing").
 * A data cell whose direction leaves the raster, enters a NoData cell or is
 * NoFlow is an outlet (it keeps its accumulation).
 *
 * dirs:     uint8 [rows*cols] direction codes (in).
 * weights:  float32 [rows*cols] per-cell w (in), or NULL for w = 1.
 * acc:      out, [rows*cols]: uint32 for D8_ACC_U32, float32 for D8_ACC_F32;
 *           NoData cells are set to 0.
 * tile_rows, tile_cols: tile shape (0, 0 = default 64 x 64); each >= 1; a
 *           side longer than the raster is cut to the raster; after that
 *           each side <= D8_MAX_TILE_SIDE.
 * ws, ws_bytes: workspace (device, 256-byte aligned as every torch or hipMalloc
 *     allocation is), at least d8_workspace_bytes(...).
 * U32 counts are exact while every true count is below 2^32.
 * F32: each tile sums in float32, the cross-tile resolve in float64.
 * Returns D8_OK, D8_EINVAL, D8_EWORKSPACE or D8_EHIP (asynchronous data errors
 * via d8_check_status).
 */
int flow_accum(const uint8_t *dirs, const float *weights, void *acc, int acc_type, int64_t rows,
               int64_t cols, int tile_rows, int tile_cols, void *ws, size_t ws_bytes,
               void *stream);

/*
 * Adjoint of flow_accum.  Eq. (1) is linear in w: A = (I - P)^-1 w, with
 * P(p, n) = 1 when n's flow goes to p.  For a loss L(A) with g = dL/dA the
 * weight gradient is lambda = (I - P)^-T g, i.e.
 *     lambda(c) = g(c) + lambda(receiver of c)   (0 if c is an outlet),
 * the sum of g along c's downstream flow path.  Computed with the same tiles:
 * pass 1 sums g along each perimeter cell's in-tile path (Algorithm 2's walk),
 * the perimeter graph resolves the downstream sums across tiles, and pass 2
 * fills in every cell.  This operation is not in the paper; it follows from
 * the linearity of Eq. (1).
 *
 * dirs: uint8 [rows*cols] (in); grad_acc: float32 [rows*cols] g (in);
 * grad_weights: float32 [rows*cols] lambda (out), 0 on NoData cells.
 * Other arguments and returns as for flow_accum.
 */
int flow_accum_adjoint(const uint8_t *dirs, const float *grad_acc, float *grad_weights,
                       int64_t rows, int64_t cols, int tile_rows, int tile_cols, void *ws,
                       size_t ws_bytes, void *stream);

/*
 * Flow accumulation with absorption: Eq. (1) with alpha(n, p) = alpha(n) in
 * [0, 1] for n's single receiver p, i.e. A(p) = w(p) + sum over donors n of
 * alpha(n) A(n) -- the fraction alpha(n) of a cell's flow reaches its
 * receiver (the paper's Eq. (1) and its remark that absorption is a simple
 * extension of the tiled method).  Same three stages as flow_accum; each
 * perimeter link also carries the product of alpha along the entry's in-tile
 * path, and the cross-tile resolve multiplies by it (float64).
 *
 * dirs: uint8 codes; weights: float32 w or NULL (w = 1); alpha: float32 per
 * cell (values outside [0, 1] are used as given); acc: float32 A (out), 0 on
 * NoData cells.  ws: at least d8_absorb_workspace_bytes(...) (256-byte
 * aligned).  Other arguments and returns as for flow_accum, except that
 * tile_rows = tile_cols = 0 picks 48 x 32: the tile's LDS holds alpha besides
 * the values, so smaller tiles keep more of them resident per CU.
 */
size_t d8_absorb_workspace_bytes(int64_t rows, int64_t cols, int tile_rows, int tile_cols);
int flow_accum_absorb(const uint8_t *dirs, const float *weights, const float *alpha, float *acc,
                      int64_t rows, int64_t cols, int tile_rows, int tile_cols, void *ws, size_t ws_bytes,
                      void *stream);

/*
 * Adjoint of flow_accum_absorb with respect to the weights:
 * lambda(c) = g(c) + alpha(c) lambda(receiver(c)) (0 beyond a cell without a
 * receiver), i.e. lambda = (I - P_alpha)^-T g for the absorbing transfer
 * matrix P_alpha of Eq. (1).  Not in the paper; the same tiles as
 * flow_accum_adjoint, with each cell's in-tile alpha product carried to the
 * exit-level resolve, which composes affine maps by pointer jumping.
 *
 * dirs, alpha as for flow_accum_absorb; grad_acc: float32 g; grad_weights:
 * float32 lambda (out), 0 on NoData cells.  ws: at least
 * d8_absorb_workspace_bytes(...) (256-byte aligned; the forward and the
 * adjoint take the same size).  Returns as for flow_accum_adjoint.
 */
int flow_accum_absorb_adjoint(const uint8_t *dirs, const float *alpha, const float *grad_acc,
                              float *grad_weights, int64_t rows, int64_t cols, int tile_rows, int tile_cols,
                              void *ws, size_t ws_bytes, void *stream);

/*
 * Gradient with respect to the absorption fractions: for a loss with
 * gradient c with respect to A (the output of flow_accum_absorb), alpha(n)
 * scales only the edge from n to its receiver in Eq. (1), so
 * dL/dalpha(n) = A(n) lambda(receiver(n)), lambda = flow_accum_absorb_adjoint
 * of c (not in the paper).  0 where n has no data receiver (NoFlow, NoData,
 * off the raster, invalid codes).  One elementwise pass.
 *
 * dirs: uint8 codes; acc: float32 A from flow_accum_absorb; grad_lam: float32
 * lambda from flow_accum_absorb_adjoint; grad_alpha: float32 (out).  All
 * device, [rows*cols] row-major.  Returns D8_OK, D8_EINVAL (sizes, NULL
 * pointers for a non-empty raster) or D8_EHIP.
 */
int flow_accum_absorb_alpha_grad(const uint8_t *dirs, const float *acc, const float *grad_lam,
                                 float *grad_alpha, int64_t rows, int64_t cols, void *stream);

/*
 * Forward accumulation (unit weights, uint32 counts) of a raster that stays
 * in host memory, for rasters larger than the device's memory -- the regime
 * the paper's tiles were designed for (Introduction; the EVICT strategy of
 * Section "Broadcasting & Finalizing" recomputes each tile from its codes, so
 * only the perimeter records persist between the passes).  The raster goes
 * through the device in bands of band_rows rows (whole tile rows): pass 1 per
 * band (the band's codes plus one halo row above and below), the band's
 * perimeter-graph edges, the resolve over the whole perimeter graph, which
 * stays in the workspace, then pass 2 per band with the band's counts copied
 * back.  Host traffic: the codes twice and the counts once (6 B per cell).
 * Copies run on a stream of the library's own and overlap the kernels;
 * results equal flow_accum's with the same tile shape, bit for bit.
 *
 * dirs_host: uint8 [rows*cols] codes in host memory (in).
 * acc_host:  uint32 [rows*cols] counts in host memory (out), 0 on NoData
 *            cells; complete when `stream` reaches the end of this call.
 *            Pinned memory (hipHostMalloc, torch's pin_memory) lets the
 *            copies overlap the kernels; pageable memory works, slower.
 * band_rows: rows per band, a multiple of the tile height after the tile is
 *            cut to the raster (0 = 16 tile rows); cut to the raster.
 * ws, ws_bytes: device workspace (256-byte aligned) of at least
 *            d8_stream_workspace_bytes(...) bytes: the perimeter graph of the
 *            whole raster, three code slots, two result slots and two slots
 *            for a float input of a band.
 * Other arguments and returns as for flow_accum (data errors via
 * d8_check_status(ws, stream)).  Calls that share a workspace, or run at the
 * same time on one device, must be ordered (the library's copy stream and
 * events are one per device).
 */
size_t d8_stream_workspace_bytes(int64_t rows, int64_t cols, int tile_rows, int tile_cols,
                                 int64_t band_rows);
int flow_accum_streamed(const uint8_t *dirs_host, uint32_t *acc_host, int64_t rows, int64_t cols,
                        int tile_rows, int tile_cols, int64_t band_rows, void *ws, size_t ws_bytes,
                        void *stream);

/*
 * The same out-of-core scheme for float weights and for the adjoint, so the
 * whole path runs on rasters larger than device memory (Introduction; EVICT,
 * Section "Broadcasting & Finalizing").  Both stream one float per cell
 * (the weights or the cotangent) from host memory in each of the two passes
 * and copy one float per cell back: host traffic 14 B per cell (codes twice,
 * the float input twice, the result once).
 *
 * flow_accum_streamed_f32: A of Eq. (1) with float32 weights (weights_host
 * NULL = unit weights, then 6 B per cell), float32 result, NoData cells 0.
 * The cross-tile sums are the fixed-order float resolve of flow_accum, so the
 * result equals flow_accum(D8_ACC_F32)'s on the same tile shape bit for bit.
 *
 * flow_accum_adjoint_streamed: lambda = (I-P)^-T g (see flow_accum_adjoint),
 * float32, NoData cells 0.  Pass 1 keeps only the perimeter records; the
 * exits' edges are stored as the bands pass (the codes do not stay on the
 * device); pass 2 recomputes each tile's upstream sums with every exit seeded
 * by the resolved sum of the tile it flows into, so no per-cell state is kept
 * between the passes.  Agrees with flow_accum_adjoint within float32
 * rounding (the sums are grouped differently).
 *
 * dirs_host: uint8 codes; weights_host / grad_host: float32; acc_host /
 * grad_weights_host: float32 results -- all [rows*cols] in host memory
 * (pinned memory lets the copies overlap the kernels).  Other arguments,
 * workspace (d8_stream_workspace_bytes, which covers all three streamed
 * calls), ordering rules and returns as for flow_accum_streamed; NULL
 * grad_host is D8_EINVAL.
 */
int flow_accum_streamed_f32(const uint8_t *dirs_host, const float *weights_host, float *acc_host, int64_t rows,
                            int64_t cols, int tile_rows, int tile_cols, int64_t band_rows, void *ws,
                            size_t ws_bytes, void *stream);
int flow_accum_adjoint_streamed(const uint8_t *dirs_host, const float *grad_host, float *grad_weights_host,
                                int64_t rows, int64_t cols, int tile_rows, int tile_cols, int64_t band_rows,
                                void *ws, size_t ws_bytes, void *stream);

/*
 * Batches of rasters.  Many rasters of uneven sizes go through the same
 * three stages together: a few launches per stage for the whole batch
 * instead of several per raster.  The tile passes launch one wavefront per
 * (raster, tile) pair of the batch's tile list, one launch per requested tile
 * shape (its LDS size); within a shape, rasters are ordered by decreasing
 * cell count, so the largest rasters' tiles are dispatched first.  All
 * rasters' perimeter cells form one global flow graph (the
 * paper hands tiles to workers in turn and resolves one graph of all
 * perimeters, Sections "Constructing a Global Solution" and "Implementation
 * Details").  Forward accumulation is float32 (weights, or NULL for w = 1);
 * the results equal those of flow_accum(D8_ACC_F32) / flow_accum_adjoint per
 * raster with the same tile shapes, bit for bit.
 *
 * d8_batch_item: one raster; every pointer is a device pointer owned by the
 * caller.  rows, cols >= 0 (an empty raster is skipped); tile_rows,
 * tile_cols as for flow_accum (0, 0 = 64 x 64), per raster.
 *   dirs (in); weights (in, NULL = 1) and acc (out) for D8_BATCH_FWD;
 *   grad_acc (in) and grad_weights (out) for D8_BATCH_ADJ.
 * mode: D8_BATCH_FWD, D8_BATCH_ADJ or both (forward first, then adjoint).
 * items: host array of n items (read during the call only).
 * ws, ws_bytes: device workspace (256-byte aligned) of at least d8_batch_workspace_bytes(items,
 *   n) bytes (the same items; 0 means the items are invalid).  It holds the
 *   batch's descriptor tables and perimeter-graph arrays.
 */
typedef struct {
    const uint8_t *dirs;
    const float *weights;
    float *acc;
    const float *grad_acc;
    float *grad_weights;
    int64_t rows, cols;
    int tile_rows, tile_cols;
} d8_batch_item;

enum { D8_BATCH_FWD = 1, D8_BATCH_ADJ = 2 };

size_t d8_batch_workspace_bytes(const d8_batch_item *items, int n);

/*
 * Runs a batch on `stream`.  The descriptor tables are copied into `ws`
 * first, from a pinned host buffer of the library's own (a ring of four,
 * allocated on first use and grown when a batch needs more; the host waits
 * for a buffer only if its copy from four calls back has not run yet), then
 * the stages are enqueued; the call does not synchronise `stream`.  Returns D8_OK,
 * D8_EINVAL (bad item, mode, or a missing pointer the mode needs),
 * D8_EWORKSPACE or D8_EHIP; data errors via d8_check_status(ws, stream).
 */
int flow_accum_batched(const d8_batch_item *items, int n, int mode, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * The same batch recorded once as a HIP graph: d8_graph_create copies the
 * descriptor tables into `ws` on `stream` and waits for that copy (a setup
 * call: the graph may then be launched on any stream), records every stage on
 * a private stream and returns an executable graph in *graph_exec.
 * d8_graph_launch replays it on `stream` -- one launch for the whole batch;
 * it reads and writes the items' arrays and `ws` as they are at replay time
 * (the pointers are fixed at creation).  Replays on one workspace must not
 * overlap.  d8_graph_destroy frees the graph.  The graph allocates nothing
 * and contains no memset nodes.
 */
int d8_graph_create(const d8_batch_item *items, int n, int mode, void *ws, size_t ws_bytes,
                    void *stream, void **graph_exec);
int d8_graph_launch(void *graph_exec, void *stream);
int d8_graph_destroy(void *graph_exec);

/*
 * flow_accum for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same computation and results as flow_accum with the same arguments, but the
 * workspace is the library's own device array of D8_NOALLOC_SCRATCH_BYTES,
 * one per GPU, held from the library's load until the process ends.  The
 * caller passes inputs and outputs only.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).
 * status: NULL, or a caller-owned device uint32 that receives the call's data
 * status when its kernels have run: 0 ok, 4 an invalid direction code, 5 a
 * cycle (outputs are then undefined).
 * Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (other streams, other threads) race; calls on one stream are ordered.
 * Returns D8_EWORKSPACE when the raster needs a workspace larger than the array
 * (d8_workspace_bytes(rows, cols, tile_rows, tile_cols) >
 * D8_NOALLOC_SCRATCH_BYTES: about 2e7 cells at 64 x 64 tiles), otherwise what
 * flow_accum returns.
 */
#define D8_NOALLOC_SCRATCH_BYTES (64u << 20)
int flow_accum_noalloc(const uint8_t *dirs, const float *weights, void *acc, int acc_type, int64_t rows,
                       int64_t cols, int tile_rows, int tile_cols, uint32_t *status, void *stream);

/*
 * Waits for `stream`, then returns the data-dependent status recorded in
 * `ws` by the last flow_accum / flow_accum_adjoint / batch call on it: D8_OK,
 * D8_EDIRCODE or D8_ECYCLE (or D8_EHIP if the wait itself fails, D8_EINVAL for
 * a NULL workspace).
 */
int d8_check_status(const void *ws, void *stream);

/*
 * Kernel timing, a profiling aid.  on = 1: every kernel launched by the calls
 * above is bracketed by two HIP events recorded on its launch stream; on = 2:
 * only the per-tile passes (labels containing "pass"), which keeps the events
 * out of the small kernels between them; on = 0: off (other values:
 * D8_EINVAL).
 * d8_timing_report waits for the recorded events, writes up to max_entries
 * (kernel name, summed milliseconds, launch count) triples -- names are static
 * strings owned by the library -- forgets the records, and returns the number
 * of entries written (or D8_EHIP).  Host memory only; never captured in a graph.
 */
int d8_timing_enable(int on);
int d8_timing_report(const char **names, double *total_ms, int64_t *launches, int max_entries);

/* The HIP error behind the calling thread's last D8_EHIP (kernel name and
 * HIP message), or "" -- a diagnostic string owned by the library. */
const char *d8_last_error_message(void);

/* Static description of a status code. */
const char *d8_strerror(int code);

/* Library version, major * 10000 + minor * 100 + patch. */
int d8_version(void);

#ifdef __cplusplus
}
#endif

#endif /* D8FLOW_H */
