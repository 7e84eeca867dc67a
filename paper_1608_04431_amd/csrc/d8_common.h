// d8_common.h -- device/host helpers shared by the gfx950 kernels of libd8flow.
//
// Tile geometry.  The raster is cut into th x tw tiles in row-major tile
// order; the last tile row / column may be smaller (the paper notes equal
// tiles are a convenience, not a requirement, Section "The Algorithm").
// Every tile's perimeter cells are numbered along a ring; the global node id
// of perimeter cell p of tile (ty, tx) is node_base(ty, tx) + p, so the
// global flow graph of Section "Constructing a Global Solution" has one node
// per perimeter cell and needs no lookup table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d8 {

constexpr int kNoFlow = 8;
constexpr int kNoData = 9;

// Per-perimeter-cell link (Algorithm 2): a ring index of the exit cell, or one
// of these markers.
constexpr uint16_t kLinkTerm = 0xFFFF;    // FlowTerminates
constexpr uint16_t kLinkExt = 0xFFFE;     // FlowExternal: the cell itself exits
constexpr uint16_t kLinkNoData = 0xFFFD;  // a NoData perimeter cell (never a receiver)
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Status word values (first word of the workspace).
constexpr uint32_t kStatusOk = 0;
constexpr uint32_t kStatusDirCode = 4;
constexpr uint32_t kStatusCycle = 5;

// Direction k -> row / column offset.  0 NW, 1 N, 2 NE, 3 W, 4 E, 5 SW, 6 S, 7 SE.
__host__ __device__ inline int dir_dr(int k) { return k < 3 ? -1 : (k < 5 ? 0 : 1); }
__host__ __device__ inline int dir_dc(int k)
{
    return (k == 0 || k == 3 || k == 5) ? -1 : ((k == 1 || k == 6) ? 0 : 1);
}

struct Geo {
    int64_t rows, cols;
    int th, tw;          // nominal tile shape
    int nty, ntx;        // tile grid
    int h_last, w_last;  // shape of the last tile row / column
    int64_t row_nodes;   // perimeter nodes in one full-height tile row
    int64_t nnodes;      // all perimeter nodes
};

__host__ __device__ inline int ring_size(int h, int w)
{
    return (h <= 2 || w <= 2) ? h * w : 2 * (h + w) - 4;
}

// Ring index of tile-local cell (r, c), or -1 for an interior cell.
// Order: top row, bottom row, left column (without corners), right column.
__host__ __device__ inline int ring_index(int r, int c, int h, int w)
{
    if (h <= 2 || w <= 2) return r * w + c;
    if (r == 0) return c;
    if (r == h - 1) return w + c;
    if (c == 0) return 2 * w + (r - 1);
    if (c == w - 1) return 2 * w + (h - 2) + (r - 1);
    return -1;
}

__host__ __device__ inline void ring_cell(int p, int h, int w, int &r, int &c)
{
    if (h <= 2 || w <= 2) { r = p / w; c = p % w; return; }
    if (p < w) { r = 0; c = p; return; }
    if (p < 2 * w) { r = h - 1; c = p - w; return; }
    p -= 2 * w;
    if (p < h - 2) { r = p + 1; c = 0; return; }
    r = p - (h - 2) + 1;
    c = w - 1;
}

__host__ __device__ inline int tile_h(const Geo &g, int ty) { return ty == g.nty - 1 ? g.h_last : g.th; }
__host__ __device__ inline int tile_w(const Geo &g, int tx) { return tx == g.ntx - 1 ? g.w_last : g.tw; }

__host__ __device__ inline int64_t node_base(const Geo &g, int ty, int tx)
{
    return (int64_t)ty * g.row_nodes + (int64_t)tx * ring_size(tile_h(g, ty), g.tw);
}

// Inverse of node_base + ring index (node ids and the nodes of one tile row
// fit 32 bits: the callers check nnodes < 2^32 - 1).
__host__ __device__ inline void node_tile(const Geo &g, int64_t id, int &ty, int &tx, int &p)
{
    const uint32_t a = (uint32_t)id / (uint32_t)g.row_nodes;
    ty = (int)(a < (uint32_t)(g.nty - 1) ? a : (uint32_t)(g.nty - 1));
    const uint32_t rem = (uint32_t)id - (uint32_t)ty * (uint32_t)g.row_nodes;
    const uint32_t P = (uint32_t)ring_size(tile_h(g, ty), g.tw);
    const uint32_t b = rem / P;
    tx = (int)(b < (uint32_t)(g.ntx - 1) ? b : (uint32_t)(g.ntx - 1));
    p = (int)(rem - (uint32_t)tx * P);
}

// The tile (uty, utx) and tile-local cell (ur, uc) of the cell at local
// (r, c) of tile (ty, tx) of height h and width w, for a cell at most one
// step outside the tile (no division).
__host__ __device__ inline void step_tile(const Geo &g, int ty, int tx, int h, int w, int r, int c, int &uty,
                                          int &utx, int &ur, int &uc)
{
    uty = r < 0 ? ty - 1 : (r >= h ? ty + 1 : ty);
    utx = c < 0 ? tx - 1 : (c >= w ? tx + 1 : tx);
    ur = r < 0 ? tile_h(g, uty) - 1 : (r >= h ? 0 : r);
    uc = c < 0 ? tile_w(g, utx) - 1 : (c >= w ? 0 : c);
}

inline Geo make_geo(int64_t rows, int64_t cols, int th, int tw)
{
    Geo g;
    g.rows = rows;
    g.cols = cols;
    g.th = th;
    g.tw = tw;
    g.nty = (int)((rows + th - 1) / th);
    g.ntx = (int)((cols + tw - 1) / tw);
    g.h_last = (int)(rows - (int64_t)(g.nty - 1) * th);
    g.w_last = (int)(cols - (int64_t)(g.ntx - 1) * tw);
    g.row_nodes = (int64_t)(g.ntx - 1) * ring_size(th, tw) + ring_size(th, g.w_last);
    g.nnodes = (int64_t)(g.nty - 1) * g.row_nodes + (int64_t)(g.ntx - 1) * ring_size(g.h_last, tw) +
               ring_size(g.h_last, g.w_last);
    return g;
}

// One raster of a batch (device-side descriptor).  Node and tile numbers
// of the raster are offset by node0 / tile0 in the batch's arrays.
struct DemDesc {
    Geo g;
    int64_t node0;      // first perimeter node of this raster
    int64_t tile0;      // first tile of this raster in the batch's tile order
    const uint8_t *dirs;
    const float *w;     // forward weights (NULL = 1)
    float *acc;         // forward output
    const float *gacc;  // adjoint cotangent
    float *gw;          // adjoint output
    uint8_t *root8;     // adjoint: root label per cell (batch workspace)
};

// First error wins.
__device__ inline void set_status(uint32_t *status, uint32_t code)
{
    atomicCAS(status, kStatusOk, code);
}

}  // namespace d8
