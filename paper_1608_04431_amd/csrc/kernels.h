// kernels.h -- gfx950 kernels of libd8flow (included by d8flow.hip).
//
// Forward (Eq. (1), alpha in {0,1}), the paper's three stages on one GPU:
//   fwd_walk<1>       one wavefront per tile (walk.h): Algorithm 1's
//                     accumulation, then Algorithm 2's links of the entry
//                     cells; one record (link, A_loc) per perimeter cell.
//   graph_build       joins every FlowExternal perimeter cell to the perimeter
//                     cell it flows into in the neighbouring tile (across an
//                     edge or a corner) and to that cell's exit; counts each
//                     exit's children.
//   resolve_fwd_*     accumulates the forest of exit cells and records each
//                     perimeter cell's cross-tile inflow (float weights: in
//                     a fixed order, over children lists, csr_*).
//   fwd_walk<2>       Algorithm 1 again per tile with the inflow added to the
//                     receiving cell's own weight (EVICT), writes A; reports
//                     exits of its tile whose children never all arrived.
// Adjoint (lambda = (I-P)^-T g, not in the paper):
//   adj_walk          per tile: upstream walks give lambda_loc (the sum of g
//                     along each cell's in-tile path) and each cell's root
//                     label; records (link, S) per perimeter cell.
//   adj_compact_*     dense numbers for the exits;
//   adj_jump_*        each exit's edge (as graph_build finds it), then the
//                     downstream sums over the exit forest by pointer jumping;
//   adj_finish        lambda = lambda_loc + the sum of the cell's root exit.
// With absorption (Eq. (1) with alpha(n) in [0, 1]) the same stages carry
// the product of alpha along paths: *_absorb kernels here and in walk.h.
// D8 directions (and rho8's): d8_kernel.
#pragma once
#include "d8_common.h"
// the tile kernels for tiles up to 64 columns (namespace w64), and the same
// kernels with register rows of 44 and 32 columns for narrower tiles: less
// work in every per-row loop of the setup
#include "walk.h"
#define D8_WALK_KW 44
#define D8_WALK_NS w44
#include "walk.h"
#define D8_WALK_KW 32
#define D8_WALK_NS w32
#include "walk.h"

namespace d8 {
using namespace w64;
}

namespace d8 {

// ------------------------------------------------------------------- D8 ----
// Steepest descent (O'Callaghan and Mark, the rule the paper takes as given):
// among the in-grid data neighbours strictly lower than the cell, the one with
// the largest drop per unit distance, the lowest code on ties; none -> NoFlow.
// The drop is one float32 subtraction.  The best cardinal drop bc and the best
// diagonal drop bd come from float maxima and compares (the key is monotone in
// the drop); between them the diagonal wins when bd exceeds bc times its
// distance (sqrt 2 for D8, t = fl32(2 - r) for rho8), compared exactly in
// double (2 bc^2 against bd^2, or bc t against bd).  A float product decides
// first: bc * fl32(sqrt 2) is within 2^-23 of bc sqrt 2 and bc * t within 2^-24
// of bc t, so a margin of 2^-20 (plus the smallest normal float, which keeps
// underflowed products out) makes the float verdict the exact one; the rare
// cells inside the margin, and those with no lower neighbour or no data, take
// the exact compare.
//
// Shared drops: fl(a - b) = -fl(b - a), so the drops of a cell toward its N,
// NW, NE and W neighbours are the negated S, SE, SW and E drops of cells
// already done (the row above, the cell to the left).  A row of 4 cells needs
// 19 subtractions instead of 32; the maxima take the negation as an operand
// modifier.
//
// Layout: a block of 256 lanes covers 1024 columns (4 consecutive cells per
// lane) and walks a strip of kD8Rows rows top to bottom.  Every elevation is
// read from HBM once, plus the row above and the three rows below the strip
// (the loads run two rows ahead).  The row loop is unrolled by 6 so that the 3
// rows of elevations and the 2 load buffers and 2 sets of shared drops change
// roles without register copies.  Column neighbours come from the adjacent
// lane (a wavefront-wide DPP shift) or, at a wavefront's edge, one extra vector
// load whose address is the same in every lane.  NoData, off-grid and missing
// cells are NaN, which no maximum selects and no compare matches.  VEC: rows
// start 16-byte aligned
// (cols % 4 == 0 and an aligned dem), so a lane moves its 4 cells with one
// 16-byte load and one 4-byte store; otherwise per element.  Blocks are mapped
// XCD-contiguously so vertically and horizontally adjacent blocks share an L2.
constexpr int kD8Threads = 256;
constexpr int kD8Cols = 4 * kD8Threads;
constexpr int kD8Rows = 64;
constexpr int kDppWaveShl1 = 0x130;  // lane i reads lane i + 1
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i - 1

// A row as loaded: the lane's 4 cells and the halo cells left of lane 0 and
// right of lane 63 (the same address in every lane).
struct D8Raw {
    float4 q;
    float hl, hr;
};

// A row ready for the stencil: NoData and off-grid cells NaN; l and r the cells
// left of v[0] and right of v[3].
struct D8Row {
    float v[4];
    float l, r;
};

// The drops of a row's 4 cells toward the row below: S, SE, SW.
struct D8Down {
    float s[4], se[4], sw[4];
};

// Rows are addressed relative to the strip's first row r0 (k = r - r0 in
// -1 .. kD8Rows + 2), so that the range checks are 32-bit scalar compares.
struct D8Lane {
    int64_t rows, cols, r0, c0, cw;  // cw: first column of the lane's wavefront
    int nrem;                        // rows r0 .. r0 + nrem - 1 exist (capped)
    bool above;                      // row r0 - 1 exists
    bool rvalid;                     // the cell right of v[3] is in the raster
    __device__ bool row_in(int k) const { return (k >= 0 || above) && k < nrem; }
    __device__ int64_t row_clamped(int k) const
    {
        return k < 0 ? (above ? r0 - 1 : r0) : (k < nrem ? r0 + k : r0 + nrem - 1);
    }
};

template <bool VEC>
__device__ inline D8Raw d8_load(const float *__restrict__ dem, const D8Lane &L, int k)
{
    const float nan = __builtin_nanf("");
    const float *p = dem + L.row_clamped(k) * L.cols;  // in bounds; rows outside mapped below
    D8Raw o;
    if constexpr (VEC) {
        // lanes past the raster read its last 4 cells: nothing uses their values
        const int64_t cc = L.c0 < L.cols ? L.c0 : L.cols - 4;
        o.q = *reinterpret_cast<const float4 *>(p + cc);
    } else {
        o.q = make_float4(nan, nan, nan, nan);
        if (L.c0 < L.cols) o.q.x = p[L.c0];
        if (L.c0 + 1 < L.cols) o.q.y = p[L.c0 + 1];
        if (L.c0 + 2 < L.cols) o.q.z = p[L.c0 + 2];
        if (L.c0 + 3 < L.cols) o.q.w = p[L.c0 + 3];
    }
    o.hl = p[L.cw > 0 ? (L.cw - 1 < L.cols ? L.cw - 1 : L.cols - 1) : 0];
    o.hr = p[L.cw + 256 < L.cols ? L.cw + 256 : L.cols - 1];
    return o;
}

// NoData (and rows outside the raster) to NaN, and the neighbours across lanes.
__device__ inline D8Row d8_finish(const D8Raw &a, const D8Lane &L, int k, float nodata)
{
    const float nan = __builtin_nanf("");
    const bool rin = L.row_in(k);  // uniform
    D8Row o;
    o.v[0] = rin && a.q.x != nodata ? a.q.x : nan;
    o.v[1] = rin && a.q.y != nodata ? a.q.y : nan;
    o.v[2] = rin && a.q.z != nodata ? a.q.z : nan;
    o.v[3] = rin && a.q.w != nodata ? a.q.w : nan;
    const float hl = rin && L.cw > 0 && a.hl != nodata ? a.hl : nan;
    const float hr = rin && L.cw + 256 < L.cols && a.hr != nodata ? a.hr : nan;
    o.l = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, hl),
                                                                __builtin_bit_cast(int, o.v[3]),
                                                                kDppWaveShr1, 0xF, 0xF, false));
    const float rr = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, hr),
                                                                           __builtin_bit_cast(int, o.v[0]),
                                                                           kDppWaveShl1, 0xF, 0xF, false));
    o.r = L.rvalid ? rr : nan;
    return o;
}

// The drops of `mid` toward `dn` (S, SE, SW).
__device__ inline D8Down d8_down(const D8Row &mid, const D8Row &dn)
{
    D8Down d;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        d.s[i] = __fsub_rn(mid.v[i], dn.v[i]);
        d.se[i] = __fsub_rn(mid.v[i], i < 3 ? dn.v[i + 1] : dn.r);
        d.sw[i] = __fsub_rn(mid.v[i], i > 0 ? dn.v[i - 1] : dn.l);
    }
    return d;
}

// max(0, +-a, +-b) and max(m, a, b) on the VALU's IEEE maximum, which ignores
// a quiet NaN operand.  Every operand is a difference (so any NaN is quiet) or
// an earlier maximum; written out so that the compiler neither re-quiets the
// operands nor spends an instruction on a negation.
template <bool NA, bool NB>
__device__ inline float d8_max0(float a, float b)
{
    float m;
    if constexpr (NA && NB)
        asm("v_max3_f32 %0, 0, -%1, -%2" : "=v"(m) : "v"(a), "v"(b));
    else if constexpr (NA)
        asm("v_max3_f32 %0, 0, -%1, %2" : "=v"(m) : "v"(a), "v"(b));
    else if constexpr (NB)
        asm("v_max3_f32 %0, 0, %1, -%2" : "=v"(m) : "v"(a), "v"(b));
    else
        asm("v_max3_f32 %0, 0, %1, %2" : "=v"(m) : "v"(a), "v"(b));
    return m;
}

__device__ inline float d8_max(float m, float a, float b)
{
    float o;
    asm("v_max3_f32 %0, %1, %2, %3" : "=v"(o) : "v"(m), "v"(a), "v"(b));
    return o;
}

// The exact choice (rare): no data, no lower neighbour, or slopes within the
// float margin.  Equal slopes keep the lower code (possible for rho8 only).
template <bool RHO>
__device__ inline int d8_pick_exact(float zc, float bc, int kc, float bd, int kd, float t)
{
    if (zc != zc) return kNoData;
    if (!(bc > 0.0f) && !(bd > 0.0f)) return kNoFlow;
    const double dc = bc, dd = bd;
    const double keyc = RHO ? dc * (double)t : 2.0 * (dc * dc);
    const double keyd = RHO ? dd : dd * dd;
    return keyd > keyc ? kd : (keyc > keyd ? kc : (kc < kd ? kc : kd));
}

// Codes of the lane's 4 cells in row `mid`: `up` gives only its halo cells
// (l, r), `in` the drops of the row above toward `mid`, `out` receives mid's
// drops toward `dn`.  t: rho8's diagonal distances (RHO only).
template <bool RHO>
__device__ inline uint32_t d8_codes4(const D8Row &up, const D8Row &mid, const D8Row &dn, const D8Down &in,
                                     D8Down &out, float4 t)
{
    constexpr float kUp = 1.0f + 0x1p-20f;
    constexpr float kMin = 0x1p-126f;  // smallest normal float
    constexpr float kSqrt2 = 0x1.6a09e6p+0f;  // sqrt 2 rounded to float
    out = d8_down(mid, dn);
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = __fsub_rn(mid.v[i], i < 3 ? mid.v[i + 1] : mid.r);
    const float w0 = __fsub_rn(mid.v[0], mid.l);
    const float nw0 = __fsub_rn(mid.v[0], up.l), ne3 = __fsub_rn(mid.v[3], up.r);
    const float tt[4] = {t.x, t.y, t.z, t.w};
    uint32_t codes = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // cardinal: N = -in.s[i], W = -e[i-1] (w0 for i = 0), E, S
        const float W = i > 0 ? -e[i - 1] : w0, N = -in.s[i];
        const float mc = d8_max(i > 0 ? d8_max0<true, true>(in.s[i], e[i > 0 ? i - 1 : 0])
                                      : d8_max0<true, false>(in.s[i], w0),
                                e[i], out.s[i]);
        int kc = e[i] == mc ? 4 : 6;
        kc = W == mc ? 3 : kc;
        kc = N == mc ? 1 : kc;
        // diagonal: NW = -in.se[i-1] (nw0 for i = 0), NE = -in.sw[i+1] (ne3 for i = 3), SW, SE
        const float NW = i > 0 ? -in.se[i > 0 ? i - 1 : 0] : nw0;
        const float NE = i < 3 ? -in.sw[i < 3 ? i + 1 : 3] : ne3;
        float md;
        if (i == 0)
            md = d8_max(d8_max0<false, true>(nw0, in.sw[1]), out.sw[i], out.se[i]);
        else if (i == 3)
            md = d8_max(d8_max0<true, false>(in.se[2], ne3), out.sw[i], out.se[i]);
        else
            md = d8_max(d8_max0<true, true>(in.se[i - 1], in.sw[i + 1]), out.sw[i], out.se[i]);
        int kd = out.sw[i] == md ? 5 : 7;
        kd = NE == md ? 2 : kd;
        kd = NW == md ? 0 : kd;
        // cardinal against diagonal
        const float y = mc * (RHO ? tt[i] : kSqrt2);
        const bool no_dwin = !(md > __builtin_fmaf(y, kUp, kMin));
        const bool no_cwin = !(y > __builtin_fmaf(md, kUp, kMin));
        int code = no_cwin ? kd : kc;
        if (no_dwin && no_cwin) code = d8_pick_exact<RHO>(mid.v[i], mc, kc, md, kd, tt[i]);
        codes |= (uint32_t)code << (8 * i);
    }
    return codes;
}

// rnd (RHO only): rho8's per-cell random values, the dem's layout; returns
// t = fl32(2 - r).  Rows past the raster read its last row (unused).
template <bool VEC, bool RHO>
__device__ inline float4 d8_rnd_load(const float *__restrict__ rnd, const D8Lane &L, int k)
{
    float4 t = make_float4(2.0f, 2.0f, 2.0f, 2.0f);
    if constexpr (RHO) {
        const float *p = rnd + L.row_clamped(k) * L.cols;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (VEC) {
            v = *reinterpret_cast<const float4 *>(p + (L.c0 < L.cols ? L.c0 : L.cols - 4));
        } else {
            if (L.c0 < L.cols) v.x = p[L.c0];
            if (L.c0 + 1 < L.cols) v.y = p[L.c0 + 1];
            if (L.c0 + 2 < L.cols) v.z = p[L.c0 + 2];
            if (L.c0 + 3 < L.cols) v.w = p[L.c0 + 3];
        }
        t = make_float4(__fsub_rn(2.0f, v.x), __fsub_rn(2.0f, v.y), __fsub_rn(2.0f, v.z),
                        __fsub_rn(2.0f, v.w));
    }
    return t;
}

template <bool VEC>
__device__ inline void d8_store(uint8_t *__restrict__ dirs, const D8Lane &L, int k, uint32_t codes)
{
    uint8_t *o = dirs + (L.r0 + k) * L.cols + L.c0;
    if constexpr (VEC) {
        if (L.c0 < L.cols) *reinterpret_cast<uint32_t *>(o) = codes;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (L.c0 + i < L.cols) o[i] = (uint8_t)(codes >> (8 * i));
    }
}

template <int J>
using D8Step = std::integral_constant<int, J>;

template <bool VEC, bool RHO>
__global__ void __launch_bounds__(kD8Threads)
d8_kernel(const float *__restrict__ dem, const float *__restrict__ rnd, uint8_t *__restrict__ dirs,
          int64_t rows, int64_t cols, float nodata, int64_t ncb, int64_t strip0)
{
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t strip = strip0 + t / ncb, cb = t - (t / ncb) * ncb;
    D8Lane L;
    L.rows = rows;
    L.cols = cols;
    L.c0 = cb * kD8Cols + 4 * (int64_t)threadIdx.x;
    // the wavefront's halo cells are read by every lane with one vector load
    // (the same address): as scalar loads they each fetched their own line
    L.cw = L.c0 - 4 * (int64_t)(threadIdx.x & 63);
    L.rvalid = L.c0 + 4 < cols;
    L.r0 = strip * kD8Rows;
    L.above = L.r0 > 0;
    L.nrem = rows - L.r0 < kD8Rows + 3 ? (int)(rows - L.r0) : kD8Rows + 3;
    const int n = L.nrem < kD8Rows ? L.nrem : kD8Rows;  // rows of this strip
    // rings (k = row - r0): F[k mod 3] holds row k, R[(k - 1) mod 2] the raw row
    // k + 1 in flight, C[(k + 1) mod 2] the drops of row k - 1 toward row k,
    // T[k mod 2] rho8's distances of row k
    D8Row F[3];
    D8Raw R[2];
    D8Down C[2];
    float4 T[2];
    F[2] = d8_finish(d8_load<VEC>(dem, L, -1), L, -1, nodata);
    F[0] = d8_finish(d8_load<VEC>(dem, L, 0), L, 0, nodata);
    C[1] = d8_down(F[2], F[0]);
    R[1] = d8_load<VEC>(dem, L, 1);
    R[0] = d8_load<VEC>(dem, L, 2);
    T[0] = d8_rnd_load<VEC, RHO>(rnd, L, 0);
    T[1] = d8_rnd_load<VEC, RHO>(rnd, L, 1);
    auto step = [&](auto J, int k) {
        constexpr int j = decltype(J)::value;
        // row k: mid F[j % 3], below F[(j + 1) % 3] (finished now from R), above F[(j + 2) % 3]
        F[(j + 1) % 3] = d8_finish(R[(j + 1) % 2], L, k + 1, nodata);
        R[(j + 1) % 2] = d8_load<VEC>(dem, L, k + 3);
        const uint32_t codes =
            d8_codes4<RHO>(F[(j + 2) % 3], F[j % 3], F[(j + 1) % 3], C[(j + 1) % 2], C[j % 2], T[j % 2]);
        T[j % 2] = d8_rnd_load<VEC, RHO>(rnd, L, k + 2);
        d8_store<VEC>(dirs, L, k, codes);
    };
    for (int k = 0; k < n; k += 6) {
        step(D8Step<0>{}, k);
        if (k + 1 >= n) break;
        step(D8Step<1>{}, k + 1);
        if (k + 2 >= n) break;
        step(D8Step<2>{}, k + 2);
        if (k + 3 >= n) break;
        step(D8Step<3>{}, k + 3);
        if (k + 4 >= n) break;
        step(D8Step<4>{}, k + 4);
        if (k + 5 >= n) break;
        step(D8Step<5>{}, k + 5);
    }
}

// ------------------------------------------------------------ perimeter graph
// For every FlowExternal node e: entry(e) = the perimeter node its flow enters
// (in the tile across the edge or corner), succ(e) = that node's exit node
// (itself if it is FlowExternal, none if its path terminates).  indeg (when
// given) counts each exit node's children in the exit forest; it is not
// changed afterwards, so the resolve can tell leaves from inner nodes.
// The edge of exit `id` (link kLinkExt) of a raster whose nodes start at
// node0: e = the perimeter node its flow enters, s = that node's exit (or
// kNone; e = kNone too when the flow enters NoData).
__device__ inline void graph_edge(const uint8_t *__restrict__ dirs, const Geo &g, int64_t node0,
                                  int64_t id, const uint16_t *__restrict__ link, uint32_t &e,
                                  uint32_t &s)
{
    e = s = kNone;
    int ty, tx, p, r, c;
    node_tile(g, id, ty, tx, p);
    const int h = tile_h(g, ty), w = tile_w(g, tx);
    ring_cell(p, h, w, r, c);
    int64_t gr = (int64_t)ty * g.th + r, gc = (int64_t)tx * g.tw + c;
    int k = dirs[gr * g.cols + gc];
    // an exit's flow leaves its tile by one step (edge or corner)
    int uty, utx, lr, lc;
    step_tile(g, ty, tx, h, w, r + dir_dr(k), c + dir_dc(k), uty, utx, lr, lc);
    int64_t ub = node0 + node_base(g, uty, utx);
    int q = ring_index(lr, lc, tile_h(g, uty), tile_w(g, utx));  // >= 0: borders a tile edge
    int64_t n = ub + (q < 0 ? 0 : q);
    uint16_t L = q < 0 ? kLinkNoData : link[n];
    if (L != kLinkNoData) {
        e = (uint32_t)n;
        s = (L == kLinkExt) ? (uint32_t)n : (L == kLinkTerm ? kNone : (uint32_t)(ub + L));
    }
}

__device__ inline void graph_node(const uint8_t *__restrict__ dirs, const Geo &g, int64_t node0,
                                  int64_t id, const uint16_t *__restrict__ link,
                                  uint32_t *__restrict__ entry, uint32_t *__restrict__ succ,
                                  uint32_t *__restrict__ indeg)
{
    const int64_t gid = node0 + id;
    uint32_t e = kNone, s = kNone;
    if (link[gid] == kLinkExt) graph_edge(dirs, g, node0, id, link, e, s);
    entry[gid] = e;
    succ[gid] = s;
    if (indeg && s != kNone) atomicAdd(&indeg[s], 1u);
}

// Nodes id0 .. id1 - 1 (all of them, or one band's when streaming).
__global__ void graph_build(const uint8_t *__restrict__ dirs, Geo g,
                            const uint16_t *__restrict__ link, uint32_t *__restrict__ entry,
                            uint32_t *__restrict__ succ, uint32_t *__restrict__ indeg, int64_t id0,
                            int64_t id1)
{
    int64_t id = id0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= id1) return;
    graph_node(dirs, g, 0, id, link, entry, succ, indeg);
}

// Batch: the raster of node id starts at chunk_dem[id >> kChunkShift] and is
// found by stepping forward over the (few) rasters that start in the chunk.
constexpr int kChunkShift = 12;

__device__ inline int dem_of(const DemDesc *__restrict__ dems, int ndem,
                             const uint32_t *__restrict__ chunk_dem, int64_t id)
{
    int d = (int)chunk_dem[id >> kChunkShift];
    while (d + 1 < ndem && dems[d + 1].node0 <= id) ++d;
    return d;
}

__global__ void graph_build_batch(const DemDesc *__restrict__ dems, int ndem,
                                  const uint32_t *__restrict__ chunk_dem, int64_t nnodes,
                                  const uint16_t *__restrict__ link, uint32_t *__restrict__ entry,
                                  uint32_t *__restrict__ succ, uint32_t *__restrict__ indeg)
{
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nnodes) return;
    const DemDesc &D = dems[dem_of(dems, ndem, chunk_dem, id)];
    graph_node(D.dirs, D.g, D.node0, id - D.node0, link, entry, succ, indeg);
}

// Forest accumulation over exit nodes (the paper's modified Algorithm 1 on the
// global graph): V(e) = A_loc(e) + sum of V over exits flowing into e; every
// V(e) is also added to the inflow ext(entry(e)).  Walkers start at leaves
// (indeg 0) and continue from a node only as its last arriving child.
//
// Unit counts: one 64-bit atomic per step updates (inflow sum : arrivals)
// together -- adding (v << 32) + 1 -- so the last child reads the complete
// sum from the returned value and no fence is needed.
__global__ void resolve_fwd_u32(int64_t nnodes, const uint16_t *__restrict__ link,
                                const uint32_t *__restrict__ aloc, const uint32_t *__restrict__ entry,
                                const uint32_t *__restrict__ succ, const uint32_t *__restrict__ indeg,
                                unsigned long long *packed, uint32_t *ext)
{
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nnodes) return;
    if (link[id] != kLinkExt || indeg[id] != 0) return;
    uint32_t v = aloc[id];
    uint32_t n = entry[id], s = succ[id];
    for (;;) {
        if (n == kNone) break;
        atomicAdd(&ext[n], v);
        if (s == kNone) break;
        // the next node's fields do not depend on the arrival: fetch them
        // while the atomic is in flight
        const uint32_t as = aloc[s], is = indeg[s], ns = entry[s], ss = succ[s];
        unsigned long long old = atomicAdd(&packed[s], ((unsigned long long)v << 32) | 1ull);
        if ((uint32_t)old + 1u != is) break;
        v = as + (uint32_t)(old >> 32) + v;
        n = ns;
        s = ss;
    }
}

// Exits on or below a cycle of exits are never finished: their children
// never all arrive.  Forward pass 2 checks its tile's exits (arrivals equal
// to the child count for unit counts, a count left at zero for float
// weights) and reports a cycle; no separate pass over the nodes is needed.

// -------------------------------------------------------------- adjoint ----
// mu(e) = lambda(entry(e)) = S(entry(e)) + mu(succ(e)): a downstream path sum
// over the exit forest, by pointer jumping.  One 64-bit word per node:
// pointer in the low half, float partial sum in the high half.  A pointer
// kNone means the sum is complete; kJumpDone additionally means the word
// holds the same complete sum in both buffers, so rounds skip the node.
constexpr uint32_t kJumpDone = 0xFFFFFFFEu;

__device__ inline unsigned long long jump_word(uint32_t ptr, float v)
{
    return ((unsigned long long)__float_as_uint(v) << 32) | ptr;
}
__device__ inline float jump_val(unsigned long long w) { return __uint_as_float((uint32_t)(w >> 32)); }

// Only exits take part: they are numbered densely in node order (a stream
// compaction of the link array), so the rounds run over the exit forest
// alone (about a third of the perimeter nodes), in contiguous memory.
// Blocks of 256 lanes take 4096 consecutive nodes, 16 per lane.
constexpr int kCompactBlock = 256;
constexpr int kCompactPer = 16;
constexpr int64_t kCompactNodes = (int64_t)kCompactBlock * kCompactPer;

// Bit j: node n0 + j is an exit (n0 is a multiple of 16).
__device__ inline uint32_t exit_bits16(const uint16_t *__restrict__ link, int64_t nnodes, int64_t n0)
{
    uint32_t m = 0;
    if (n0 + kCompactPer <= nnodes && (reinterpret_cast<uintptr_t>(link + n0) & 15) == 0) {
        const uint4 *p = reinterpret_cast<const uint4 *>(link + n0);
        const uint4 a = p[0], b = p[1];
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            m |= (uint32_t)((w[i] & 0xFFFFu) == kLinkExt) << (2 * i);
            m |= (uint32_t)((w[i] >> 16) == kLinkExt) << (2 * i + 1);
        }
    } else {
        for (int j = 0; j < kCompactPer; ++j)
            if (n0 + j < nnodes && link[n0 + j] == kLinkExt) m |= 1u << j;
    }
    return m;
}

// Exclusive prefix of v over the block's lanes; *total gets the block sum.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kCompactBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kCompactBlock / 64; ++i) {
        before += i < wv ? wsum[i] : 0u;
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Exits per block of 4096 nodes.
__global__ void __launch_bounds__(kCompactBlock)
adj_compact_count(int64_t nnodes, const uint16_t *__restrict__ link, uint32_t *__restrict__ bsum)
{
    const int64_t n0 = (int64_t)blockIdx.x * kCompactNodes + (int64_t)threadIdx.x * kCompactPer;
    const uint32_t c = __popc(exit_bits16(link, nnodes, n0));
    uint32_t total;
    block_excl_scan(c, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the block counts in place (one block); the number of
// exits goes to *nexit.
__global__ void __launch_bounds__(1024)
adj_compact_scan(int64_t nblocks, uint32_t *bsum, uint32_t *nexit)
{
    __shared__ uint32_t part[16];
    __shared__ uint32_t carry_s;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    // chunks of 8192 counts: 8 consecutive per lane
    for (int64_t c0 = 0; c0 < nblocks; c0 += 8192) {
        const int64_t i0 = c0 + 8 * (int64_t)threadIdx.x;
        uint32_t v[8], s = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = i0 + k < nblocks ? bsum[i0 + k] : 0u;
            s += v[k];
        }
        uint32_t x = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) part[wv] = x;
        __syncthreads();
        uint32_t before = carry_s, all = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            before += i < wv ? part[i] : 0u;
            all += part[i];
        }
        uint32_t run = before + x - s;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (i0 + k < nblocks) bsum[i0 + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) *nexit = carry_s;
}

// cmap[n] = the dense index of exit n, kNone for other nodes; inv[c] = the
// node of dense index c.
__global__ void __launch_bounds__(kCompactBlock)
adj_compact_map(int64_t nnodes, const uint16_t *__restrict__ link, const uint32_t *__restrict__ bsum,
                uint32_t *__restrict__ cmap, uint32_t *__restrict__ inv)
{
    const int64_t n0 = (int64_t)blockIdx.x * kCompactNodes + (int64_t)threadIdx.x * kCompactPer;
    const uint32_t m = exit_bits16(link, nnodes, n0);
    uint32_t total;
    uint32_t idx = bsum[blockIdx.x] + block_excl_scan(__popc(m), &total);
    uint32_t out[kCompactPer];
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
        const bool ex = (m >> j) & 1u;
        out[j] = ex ? idx : kNone;
        if (ex) inv[idx] = (uint32_t)(n0 + j);
        idx += ex ? 1u : 0u;
    }
    if (n0 + kCompactPer <= nnodes && (reinterpret_cast<uintptr_t>(cmap + n0) & 15) == 0) {
        uint4 *p = reinterpret_cast<uint4 *>(cmap + n0);
#pragma unroll
        for (int i = 0; i < kCompactPer / 4; ++i)
            p[i] = make_uint4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
    } else {
        for (int j = 0; j < kCompactPer; ++j)
            if (n0 + j < nnodes) cmap[n0 + j] = out[j];
    }
}

// Where the adjoint's exits find their edges: one raster (dems == nullptr)
// or a batch.
struct JumpGraph {
    const uint8_t *dirs;
    Geo g;
    const DemDesc *dems;
    int ndem;
    const uint32_t *chunk_dem;
    // edges found earlier (graph_build's entry and succ, for a raster whose
    // directions are not resident): used when set
    const uint32_t *entry = nullptr, *succ = nullptr;
};

__device__ inline void jump_edge(const JumpGraph &G, const uint16_t *__restrict__ link, int64_t id, uint32_t &n,
                                 uint32_t &s)
{
    if (G.entry) {
        n = G.entry[id];
        s = G.succ[id];
    } else if (G.dems) {
        const DemDesc &D = G.dems[dem_of(G.dems, G.ndem, G.chunk_dem, id)];
        graph_edge(D.dirs, D.g, D.node0, id - D.node0, link, n, s);
    } else {
        graph_edge(G.dirs, G.g, 0, id, link, n, s);
    }
}

// Initial words of the exits (a fixed grid strides over them): each exit's
// edge (as graph_build finds it), pointer = the dense index of the
// successor (kNone at a root), val = S(entry).  Round 0 writes every word of
// the other buffer, which holds inv until then.
__global__ void __launch_bounds__(256)
adj_jump_init(const uint32_t *__restrict__ nexit, const uint32_t *__restrict__ inv, JumpGraph G,
              const uint16_t *__restrict__ link, const float *__restrict__ S,
              const uint32_t *__restrict__ cmap, unsigned long long *__restrict__ buf0)
{
    const int64_t E = *nexit;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += stride) {
        const int64_t id = inv[i];
        uint32_t n, s;
        jump_edge(G, link, id, n, s);
        buf0[i] = jump_word(s != kNone ? cmap[s] : kNone, n != kNone ? S[n] : 0.0f);
    }
}

// One synchronous round r over the exits (their count is *nexit): reads
// buffer r&1, writes buffer (r+1)&1.  Each word is composed with the next two
// along its chain, val' = val + val[ptr] + val[ptr[ptr]] and ptr' =
// ptr[ptr[ptr]], so a round triples the stretch of path a word covers and
// ceil(log3 N) rounds finish any chain (a word whose successor is complete
// becomes complete).  live[r%3] is set when any pointer is still live after
// the round; round r reads live[(r-1)%3] and, if nothing was live, records
// the final buffer in state[0] and does nothing.  live[(r+1)%3] is cleared
// here for the next round (its previous contents were read by round r-1,
// which has completed).  A fixed grid strides over the exits, so rounds after
// convergence cost one small launch.
__device__ inline bool jump_live(uint32_t p) { return p != kNone && p != kJumpDone; }

__device__ inline void jump_compose(unsigned long long *w_in, unsigned long long *__restrict__ w_out, int64_t i,
                                    unsigned long long w, unsigned long long t, unsigned long long u, bool &alive)
{
    const uint32_t p = (uint32_t)w;
    if (p == kNone) {
        // complete since the last round: the same word, done, in both
        // buffers (readers of w_in see the same sum either way)
        const unsigned long long d = jump_word(kJumpDone, jump_val(w));
        w_out[i] = d;
        w_in[i] = d;
    } else if (p != kJumpDone) {
        const float s = jump_val(w) + jump_val(t);
        if (!jump_live((uint32_t)t)) {
            w_out[i] = jump_word(kNone, s);
        } else {
            uint32_t np = (uint32_t)u;
            if (np == kJumpDone) np = kNone;
            alive |= np != kNone;
            w_out[i] = jump_word(np, s + jump_val(u));
        }
    }
}

__global__ void __launch_bounds__(256)
adj_jump_round(const uint32_t *__restrict__ nexit, unsigned long long *w_in,
               unsigned long long *__restrict__ w_out, uint32_t *state, int round)
{
    uint32_t *live = state + 1;
    if (live[(round + 2) % 3] == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (state[0] == kNone) state[0] = (uint32_t)(round & 1);
            live[(round + 1) % 3] = 0;
        }
        return;
    }
    const int64_t E = *nexit;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t id0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id0 == 0) live[(round + 1) % 3] = 0;
    bool alive = false;
    for (int64_t i = id0; i < E; i += 2 * stride) {
        // two words per lane in flight
        const int64_t j = i + stride;
        const unsigned long long w = w_in[i];
        const unsigned long long w2 = j < E ? w_in[j] : jump_word(kJumpDone, 0.0f);
        const uint32_t p = (uint32_t)w, p2 = (uint32_t)w2;
        unsigned long long t = jump_word(kNone, 0.0f), t2 = jump_word(kNone, 0.0f);
        if (jump_live(p)) t = w_in[p];
        if (jump_live(p2)) t2 = w_in[p2];
        const uint32_t q = (uint32_t)t, q2 = (uint32_t)t2;
        unsigned long long u = 0, u2 = 0;
        if (jump_live(p) && jump_live(q)) u = w_in[q];
        if (jump_live(p2) && jump_live(q2)) u2 = w_in[q2];
        jump_compose(w_in, w_out, i, w, t, u, alive);
        if (j < E) jump_compose(w_in, w_out, j, w2, t2, u2, alive);
    }
    if (__ballot(alive) != 0 && (threadIdx.x & 63) == 0) live[round % 3] = 1;
}

// With absorption, mu(e) = S(entry(e)) + P(entry(e)) mu(succ(e)): an affine
// chain.  Words of 16 bytes: pointer, sum a and product b, with
// mu(e) = a + b mu(pointer); a round composes a word with its pointer's
// word, (a, b) o (a', b') = (a + b a', b b'), here with the next two words.
// Same conventions as above (kNone: complete; kJumpDone: complete in both
// buffers).
__global__ void __launch_bounds__(256)
adj_jump_init_absorb(const uint32_t *__restrict__ nexit, const uint32_t *__restrict__ inv,
                     JumpGraph G, const uint16_t *__restrict__ link, const float *__restrict__ S,
                     const float *__restrict__ P, const uint32_t *__restrict__ cmap,
                     uint4 *__restrict__ buf0)
{
    const int64_t E = *nexit;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += stride) {
        const int64_t id = inv[i];
        uint32_t n, s;
        graph_edge(G.dirs, G.g, 0, id, link, n, s);
        const float a = n != kNone ? S[n] : 0.0f, b = n != kNone ? P[n] : 0.0f;
        buf0[i] = make_uint4(s != kNone ? cmap[s] : kNone, __float_as_uint(a), __float_as_uint(b), 0u);
    }
}

__global__ void __launch_bounds__(256)
adj_jump_round_absorb(const uint32_t *__restrict__ nexit, uint4 *w_in, uint4 *__restrict__ w_out,
                      uint32_t *state, int round)
{
    uint32_t *live = state + 1;
    if (live[(round + 2) % 3] == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (state[0] == kNone) state[0] = (uint32_t)(round & 1);
            live[(round + 1) % 3] = 0;
        }
        return;
    }
    const int64_t E = *nexit;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t id0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id0 == 0) live[(round + 1) % 3] = 0;
    bool alive = false;
    for (int64_t i = id0; i < E; i += stride) {
        // composed with the next two words, as in adj_jump_round:
        // (a, b) o (a2, b2) o (a3, b3), left to right
        const uint4 w = w_in[i];
        const uint32_t p = w.x;
        if (p == kNone) {
            const uint4 d = make_uint4(kJumpDone, w.y, w.z, 0u);
            w_out[i] = d;
            w_in[i] = d;
        } else if (p != kJumpDone) {
            const uint4 t = w_in[p];
            const bool more = jump_live(t.x);
            const uint4 u = more ? w_in[t.x] : make_uint4(kNone, 0u, 0u, 0u);
            const float a = __uint_as_float(w.y), b = __uint_as_float(w.z);
            const float a2 = __uint_as_float(t.y), b2 = __uint_as_float(t.z);
            float na = a + b * a2, nb = b * b2;
            uint32_t np = kNone;
            if (more) {
                np = u.x == kJumpDone ? kNone : u.x;
                na = na + nb * __uint_as_float(u.y);
                nb = nb * __uint_as_float(u.z);
            }
            alive |= np != kNone;
            w_out[i] = make_uint4(np, __float_as_uint(na), __float_as_uint(nb), 0u);
        }
    }
    if (__ballot(alive) != 0 && (threadIdx.x & 63) == 0) live[round % 3] = 1;
}

// Derivative of <c, A> with respect to the absorption fractions: alpha(n)
// scales only the edge n -> receiver(n) of Eq. (1), so it is
// A(n) lambda(receiver(n)) with lambda the absorbing adjoint of c; 0 where n
// has no data receiver (NoFlow, NoData, off the raster, invalid codes).  One
// lane per cell of a row, blocks stride over the rows (gridDim.y).
constexpr int kGradBlock = 256;

__global__ void __launch_bounds__(kGradBlock)
absorb_alpha_grad(const uint8_t *__restrict__ dirs, const float *__restrict__ A,
                  const float *__restrict__ lam, float *__restrict__ out, int64_t rows, int64_t cols)
{
    const int64_t c = (int64_t)blockIdx.x * kGradBlock + threadIdx.x;
    if (c >= cols) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const int64_t i = r * cols + c;
        const uint32_t k = dirs[i];
        float v = 0.0f;
        if (k < (uint32_t)kNoFlow) {
            const int64_t nr = r + dir_dr((int)k), nc = c + dir_dc((int)k);
            if (nr >= 0 && nr < rows && nc >= 0 && nc < cols) {
                const int64_t j = nr * cols + nc;
                if (dirs[j] < (uint8_t)kNoData) v = A[i] * lam[j];
            }
        }
        out[i] = v;
    }
}

// After the last round: if no round found convergence, the final buffer is
// rounds&1, and pointers still live mean a cycle.
__global__ void adj_jump_finish(uint32_t *state, int rounds, uint32_t *status)
{
    if (state[0] == kNone) {
        if (state[1 + (rounds + 2) % 3] != 0) set_status(status, kStatusCycle);
        state[0] = (uint32_t)(rounds & 1);
    }
}

// ------------------------------------------- float resolve, fixed order ----
// The modified Algorithm 1 on the exit forest for float weights, with every
// sum taken in an order fixed by the input, so the result repeats bit for
// bit run to run and equals between a batch and single-raster calls:
//   V(e) = A_loc(e) + the sum of V(u) over e's children u (exits whose flow
//          reaches e) in increasing node id, in double;
//   ext(n) = the sum of V(u) over the exits u flowing into perimeter cell n,
//          in direction order (a gather, after the resolve).
// Children lists (CSR): offsets = exclusive scan of the child counts, each
// list filled by atomics and then sorted.  Walkers start at leaves; a node
// is summed by the child that arrives last (arrival counter counted down
// from the child count), reading its children's V with atomics (they may
// have been written on another XCD).  Absorption (ABS): a child u contributes
// coef(u) V(u), coef(u) = alpha(u) times the path product of the cell it
// enters, and ext(n) sums alpha(u) V(u).

// Only nodes with two children or more get a list: the walker that reaches
// a node's only child goes on without reading it.
__device__ inline uint32_t csr_len(uint32_t k) { return k >= 2u ? k : 0u; }

// A lane's kCompactPer list lengths (16-byte loads when its run of nodes is
// whole: the node arrays start on 256-byte boundaries).
__device__ inline void csr_lens(int64_t nnodes, int64_t n0, const uint32_t *__restrict__ indeg,
                                uint32_t (&v)[kCompactPer])
{
    if (n0 + kCompactPer <= nnodes) {
        const uint4 *q = reinterpret_cast<const uint4 *>(indeg + n0);
#pragma unroll
        for (int i = 0; i < kCompactPer / 4; ++i) {
            const uint4 x = q[i];
            v[4 * i] = x.x;
            v[4 * i + 1] = x.y;
            v[4 * i + 2] = x.z;
            v[4 * i + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kCompactPer; ++j) v[j] = n0 + j < nnodes ? indeg[n0 + j] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) v[j] = csr_len(v[j]);
}

// Listed children per block of 4096 nodes.
__global__ void __launch_bounds__(kCompactBlock)
csr_count(int64_t nnodes, const uint32_t *__restrict__ indeg, uint32_t *__restrict__ bsum)
{
    const int64_t n0 = (int64_t)blockIdx.x * kCompactNodes + (int64_t)threadIdx.x * kCompactPer;
    uint32_t v[kCompactPer], c = 0;
    csr_lens(nnodes, n0, indeg, v);
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) c += v[j];
    uint32_t total;
    block_excl_scan(c, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// off[n] = first slot of n's children; cnt[n] = 0 (fill position).
__global__ void __launch_bounds__(kCompactBlock)
csr_offsets(int64_t nnodes, const uint32_t *__restrict__ indeg, const uint32_t *__restrict__ bsum,
            uint32_t *__restrict__ off, uint32_t *__restrict__ cnt)
{
    const int64_t n0 = (int64_t)blockIdx.x * kCompactNodes + (int64_t)threadIdx.x * kCompactPer;
    uint32_t v[kCompactPer], c = 0;
    csr_lens(nnodes, n0, indeg, v);
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) c += v[j];
    uint32_t total;
    uint32_t run = bsum[blockIdx.x] + block_excl_scan(c, &total);
    if (n0 + kCompactPer <= nnodes) {
        uint4 *qo = reinterpret_cast<uint4 *>(off + n0);
        uint4 *qc = reinterpret_cast<uint4 *>(cnt + n0);
#pragma unroll
        for (int i = 0; i < kCompactPer / 4; ++i) {
            uint4 o;
            o.x = run;
            run += v[4 * i];
            o.y = run;
            run += v[4 * i + 1];
            o.z = run;
            run += v[4 * i + 2];
            o.w = run;
            run += v[4 * i + 3];
            qo[i] = o;
            qc[i] = make_uint4(0u, 0u, 0u, 0u);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
        if (n0 + j < nnodes) {
            off[n0 + j] = run;
            cnt[n0 + j] = 0;
        }
        run += v[j];
    }
}

// cnt[s] ends as s's child count (the arrivals the resolve counts down).
// Absorption: coef[u] = alpha(u) times the path product of the cell u's flow
// enters, the factor of V(u) in its parent's sum (exact in double: a product
// of two floats).
template <bool ABS>
__global__ void csr_fill(int64_t nnodes, const uint16_t *__restrict__ link, const uint32_t *__restrict__ succ,
                         const uint32_t *__restrict__ indeg, const uint32_t *__restrict__ off, uint32_t *cnt,
                         uint32_t *__restrict__ kids, const uint32_t *__restrict__ entry = nullptr,
                         const float *__restrict__ anode = nullptr, const float *__restrict__ pathp = nullptr,
                         double *__restrict__ coef = nullptr)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nnodes || link[id] != kLinkExt) return;
    const uint32_t s = succ[id];
    if (s == kNone) return;
    if constexpr (ABS) coef[id] = (double)anode[id] * (double)pathp[entry[id]];
    if (indeg[s] < 2u) {
        cnt[s] = 1u;  // the only child
        return;
    }
    kids[off[s] + atomicAdd(&cnt[s], 1u)] = (uint32_t)id;
}

// Each child's place in its parent's list, in increasing node id: its rank
// among the (unordered, atomically filled) siblings in kids, written to
// sorted.  A child reads its parent's k siblings, so the work per parent is
// k^2 but spread over its k children (lists are short: a parent's children
// lie on the borders of the tiles around it, at most 2 (h + w) + 4).
__global__ void csr_rank(int64_t nnodes, const uint16_t *__restrict__ link, const uint32_t *__restrict__ succ,
                         const uint32_t *__restrict__ indeg, const uint32_t *__restrict__ off,
                         const uint32_t *__restrict__ kids, uint32_t *__restrict__ sorted)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nnodes || link[id] != kLinkExt) return;
    const uint32_t s = succ[id];
    if (s == kNone) return;
    const uint32_t k = indeg[s], o = off[s], u = (uint32_t)id;
    if (k < 2u) return;
    uint32_t r = 0;
    for (uint32_t i0 = 0; i0 < k; i0 += 8) {
        // eight siblings with their loads in flight together (indices clamped
        // to the list; the clamped copies are not counted)
        uint32_t c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = kids[o + (i0 + (uint32_t)j < k ? i0 + (uint32_t)j : k - 1u)];
#pragma unroll
        for (int j = 0; j < 8; ++j) r += (i0 + (uint32_t)j < k && c[j] < u) ? 1u : 0u;
    }
    sorted[o + r] = u;
}

// A value another lane may have written during this kernel (on any XCD).
__device__ inline double v_read(unsigned long long *vn, uint32_t u)
{
    return __longlong_as_double((long long)__hip_atomic_load(&vn[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Walkers from the leaves of the exit forest.  cnt holds each node's child
// count (left by csr_fill) and is counted down by arrivals.  At a node with
// one child the walker goes on at once (V of the child and the arrival have
// one writer: plain stores, read by later kernels).  Otherwise it publishes
// V(u) with an atomic exchange and counts its arrival only once the exchange
// has returned; the last child to arrive reads its siblings' V (its own is
// in hand), eight at a time with every load in flight together (indices
// clamped to the list, so the loads take no branches), and adds them in list
// order.  One walker from leaf id.
template <typename T, bool ABS>
__device__ inline void resolve_walk(int64_t id, const T *__restrict__ aloc, const uint32_t *__restrict__ succ,
                                        const uint32_t *__restrict__ indeg, const uint32_t *__restrict__ off,
                                        const uint32_t *__restrict__ kids, uint32_t *cnt, unsigned long long *vn,
                                        const double *__restrict__ coef)
{
    uint32_t u = (uint32_t)id;
    double v = (double)aloc[u];
    uint32_t s = succ[u];
    for (;;) {
        if (s == kNone) {
            vn[u] = (unsigned long long)__double_as_longlong(v);  // read by a later kernel only
            break;
        }
        const uint32_t k = indeg[s], o = off[s], s2 = succ[s];
        const double as = (double)aloc[s];
        if (k == 1u) {
            vn[u] = (unsigned long long)__double_as_longlong(v);
            cnt[s] = 0u;
            v = as + (ABS ? coef[u] * v : v);
            u = s;
            s = s2;
            continue;
        }
        const unsigned long long prev = atomicExch(&vn[u], (unsigned long long)__double_as_longlong(v));
        uint32_t c0[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c0[j] = kids[o + ((uint32_t)j < k ? (uint32_t)j : k - 1u)];
        uint32_t one = 1u;
        // the count waits for the store; the children's ids are fetched
        // while the exchange is in flight
        asm volatile("" : "+v"(one) : "v"(prev), "v"(c0[0]), "v"(c0[1]), "v"(c0[2]), "v"(c0[3]), "v"(c0[4]),
                     "v"(c0[5]), "v"(c0[6]), "v"(c0[7]));
        if (atomicSub(&cnt[s], one) != 1u) break;
        double sum = as;
        for (uint32_t i0 = 0; i0 < k; i0 += 8) {
            uint32_t c[8];
            double vc[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t i = i0 + (uint32_t)j < k ? i0 + (uint32_t)j : k - 1u;
                c[j] = i0 == 0 ? c0[j] : kids[o + i];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) vc[j] = v_read(vn, c[j]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                double x = c[j] == u ? v : vc[j];
                if constexpr (ABS) x = coef[c[j]] * x;
                sum += i0 + (uint32_t)j < k ? x : 0.0;
            }
        }
        u = s;
        v = sum;
        s = s2;
    }
}

// One lane per node; walkers start at the leaf exits.
template <typename T, bool ABS>
__global__ void resolve_fwd_det(int64_t nnodes, const uint16_t *__restrict__ link, const T *__restrict__ aloc,
                                const uint32_t *__restrict__ succ, const uint32_t *__restrict__ indeg,
                                const uint32_t *__restrict__ off, const uint32_t *__restrict__ kids,
                                uint32_t *cnt, unsigned long long *vn, const double *__restrict__ coef = nullptr)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nnodes || link[id] != kLinkExt || indeg[id] != 0) return;
    resolve_walk<T, ABS>(id, aloc, succ, indeg, off, kids, cnt, vn, coef);
}

// ext(n) of one perimeter node (id within a raster whose nodes start at
// node0): the V of each neighbour in another tile that flows into n, in
// direction order.
template <bool ABS>
__device__ inline double ext_gather(const uint8_t *__restrict__ dirs, const Geo &g, int64_t node0, int64_t id,
                                    const uint16_t *__restrict__ link, const double *__restrict__ vn,
                                    const float *__restrict__ anode)
{
    if (link[node0 + id] == kLinkNoData) return 0.0;
    int ty, tx, p, r, c;
    node_tile(g, id, ty, tx, p);
    const int h = tile_h(g, ty), w = tile_w(g, tx);
    ring_cell(p, h, w, r, c);
    const int64_t gr = (int64_t)ty * g.th + r, gc = (int64_t)tx * g.tw + c;
    double e = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int lr = r + dir_dr(k), lc = c + dir_dc(k);
        if (lr >= 0 && lr < h && lc >= 0 && lc < w) continue;  // same tile
        const int64_t nr = gr + dir_dr(k), nc = gc + dir_dc(k);
        if (nr < 0 || nr >= g.rows || nc < 0 || nc >= g.cols) continue;
        if (dirs[nr * g.cols + nc] != (uint8_t)(7 - k)) continue;
        int uty, utx, ur, uc;
        step_tile(g, ty, tx, h, w, lr, lc, uty, utx, ur, uc);
        const int64_t u = node0 + node_base(g, uty, utx) +
                          ring_index(ur, uc, tile_h(g, uty), tile_w(g, utx));
        double vu = vn[u];  // final: written by the resolve, an earlier kernel
        if constexpr (ABS) vu = (double)anode[u] * vu;
        e += vu;
    }
    return e;
}

// Nodes id0 .. id1 - 1 (all of them, or one band's when streaming: then
// dirs holds the band's rows and one halo row above and below).
template <bool ABS>
__global__ void resolve_ext(const uint8_t *__restrict__ dirs, Geo g, const uint16_t *__restrict__ link,
                            const double *__restrict__ vn, double *__restrict__ ext,
                            const float *__restrict__ anode, int64_t id0, int64_t id1)
{
    const int64_t id = id0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= id1) return;
    ext[id] = ext_gather<ABS>(dirs, g, 0, id, link, vn, anode);
}

__global__ void resolve_ext_batch(const DemDesc *__restrict__ dems, int ndem, const uint32_t *__restrict__ chunk_dem,
                                  int64_t nnodes, const uint16_t *__restrict__ link,
                                  const double *__restrict__ vn, double *__restrict__ ext)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nnodes) return;
    const DemDesc &D = dems[dem_of(dems, ndem, chunk_dem, id)];
    ext[id] = ext_gather<false>(D.dirs, D.g, D.node0, id - D.node0, link, vn, nullptr);
}

}  // namespace d8
