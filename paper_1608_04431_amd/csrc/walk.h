// walk.h -- one wavefront per tile: flow walkers in LDS.
//
// Tile shape: up to 64 rows x 64 columns, one 64-lane wavefront per tile.
//
// Setup.  Lane r owns tile row r: its 64 direction codes sit in 16 registers
// (4 codes per word) and the in-tile donor counts of all 64 cells come from
// byte-parallel compares against the rows above and below (lanes r-1, r+1).
//
// LDS.  One byte per cell and one 32-bit value per cell, both indexed by the
// same cell index (r + 1) * S + 1 + c with S = w + 2: the tile sits inside a
// one-cell frame, so a step in direction k is `idx + offset(k)` and leaving
// the tile shows up as a frame byte -- no bounds arithmetic on the walk path.
// Cell bytes hold the code in the low nibble and, for confluences of the
// forward pass, the number of donors still to arrive in the high nibble.
// Frame bytes hold kFrameTile (a cell of a neighbouring tile) or kFrameOut
// (outside the raster) in the low nibble.
//
// Walks.  Start cells wait in an LDS queue; idle lanes claim the next ones in
// a single step (lane rank among idle lanes by mbcnt).  Forward walks
// (Algorithm 1's Kahn order, done by walkers) start at sources; a walk adds
// each cell's seed; at a confluence it adds its total to the cell's value and
// decrements the cell's pending count with LDS atomics, and only the last
// arriving donor continues.  Link walks (Algorithm 2's FollowPath) run from
// entry cells (perimeter cells with a donor in another tile) to the end of
// their in-tile path.  Upstream walks (the adjoint) run from roots against
// the flow; side donors of a branching cell are finished on the spot and
// queued.  All walks of a tile run in one wavefront, so the order of LDS
// operations is fixed by the input.
//
// Register rows.  Lane r holds tile row r in ceil(kW / 4) words, so the row
// width kW bounds the tile width and sets the work of every per-row loop.
// This file is included once per width: without D8_WALK_KW it defines the
// general kernels (kW = 64) in namespace d8::w64; the includer may define
// D8_WALK_KW and D8_WALK_NS to compile the same kernels for narrower tiles in
// a namespace of their own.

#ifndef D8_WALK_KW
#define D8_WALK_KW 64
#define D8_WALK_NS w64
#endif

#include <type_traits>

#include "d8_common.h"

namespace d8 {
namespace D8_WALK_NS {
namespace wk {

constexpr int kW = D8_WALK_KW;  // max tile width (columns)
constexpr int kH = 64;          // max tile height (rows) = lanes
constexpr int kWords = kW / 4;  // code words per row

constexpr int kRingPerLane = 4;  // ring cells per lane: 2 (64 + 64) - 4 <= 4 x 64

constexpr uint32_t kFrameTile = 0x0Eu;  // frame cell inside the raster (another tile)
constexpr uint32_t kFrameOut = 0x0Fu;   // frame cell outside the raster

struct WTile {
    int ty, tx, h, w, P;
    int S;          // LDS row stride (cells) = w + 2
    uint32_t invS;  // ceil(2^20 / S), for dividing cell indices by S
    int64_t r0, c0, base;
};

__device__ inline WTile wtile_of(const Geo &g, int t)
{
    WTile T;
    T.ty = t / g.ntx;
    T.tx = t - T.ty * g.ntx;
    T.h = tile_h(g, T.ty);
    T.w = tile_w(g, T.tx);
    T.P = ring_size(T.h, T.w);
    T.S = T.w + 2;
    T.invS = ((1u << 20) + (uint32_t)T.S - 1u) / (uint32_t)T.S;
    T.r0 = (int64_t)T.ty * g.th;
    T.c0 = (int64_t)T.tx * g.tw;
    T.base = node_base(g, T.ty, T.tx);
    return T;
}

__device__ inline int cidx(const WTile &T, int r, int c) { return (r + 1) * T.S + 1 + c; }

// Row and column of a cell index (exact for every index of a tile up to
// 66 x 66 frame cells: the error of the scaled reciprocal is below 1/S).
__device__ inline void idx_rc(const WTile &T, int idx, int &r, int &c)
{
    int r1 = (int)(((uint32_t)idx * T.invS) >> 20);
    r = r1 - 1;
    c = idx - r1 * T.S - 1;
}

// Index offset of the neighbour in direction k (0..7).  Codes 8..15 give
// -(S + 1), a valid index for any cell of the tile, so speculative reads
// stay inside the tile's LDS.
__device__ inline int dir_off(uint32_t k, int S)
{
    uint32_t dr = (0xA940u >> (2u * k)) & 3u;  // row offset + 1 of directions 0..7
    uint32_t dc = (0x9224u >> (2u * k)) & 3u;  // column offset + 1
    return (int)(dr * (uint32_t)S + dc) - (S + 1);
}

__device__ inline int lane_id() { return __lane_id(); }

// number of set bits of m in lanes below this one
__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Values kept in LDS and the type they are summed in: local unit counts of
// a tile (at most 64 x 64) fit 16 bits.
template <typename VT> struct Acc { using type = VT; };
template <> struct Acc<uint16_t> { using type = uint32_t; };

__device__ inline void lds_add(uint8_t *, float *p, float v) { atomicAdd(p, v); }
__device__ inline void lds_add(uint8_t *, uint32_t *p, uint32_t v) { atomicAdd(p, v); }
// 16-bit slot: add to its 32-bit word (sums stay below 2^16, no carry out).
// The word is addressed from the LDS base so the add stays an LDS atomic.
__device__ inline void lds_add(uint8_t *lds8, uint16_t *p, uint32_t v)
{
    const int off = (int)(reinterpret_cast<uint8_t *>(p) - lds8);
    atomicAdd(reinterpret_cast<uint32_t *>(lds8 + (off & ~3)), v << ((off & 2) * 8));
}

// Makes the compiler produce v here: a value read next to another LDS read
// is then fetched with it instead of inside a later branch.
template <typename T>
__device__ inline void keep_read(T &v)
{
    asm volatile("" : "+v"(v));
}

__device__ inline int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ----------------------------------------------------------- byte SWAR ---

// 0x80 in every zero byte of x, 0 elsewhere (exact, no carries between bytes).
__device__ inline uint32_t zero_bytes(uint32_t x)
{
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
}
__device__ inline uint32_t eq_bytes(uint32_t x, uint32_t k) { return zero_bytes(x ^ (k * 0x01010101u)); }
// bytes [4m-1 .. 4m+2] and [4m+1 .. 4m+4] of a row given words m-1, m, m+1
__device__ inline uint32_t left1(uint32_t cur, uint32_t prev) { return __builtin_amdgcn_alignbyte(cur, prev, 3); }
__device__ inline uint32_t right1(uint32_t next, uint32_t cur) { return __builtin_amdgcn_alignbyte(next, cur, 1); }
// 0x80 in bytes holding a data code 0..8
__device__ inline uint32_t valid_markers(uint32_t x)
{
    uint32_t ge9 = (((x & 0x7F7F7F7Fu) + 0x77777777u) | x) & 0x80808080u;
    return ~ge9 & 0x80808080u;
}
// byte b (0..3) of each 0x80-marker word packed into bit b
__device__ inline uint32_t marker_bits(uint32_t z)
{
    return ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u);
}
// Set byte (col - 4m) of word m of a row to `v` when that column falls in the word.
__device__ inline uint32_t put_byte(uint32_t word, int m, int col, uint32_t v)
{
    int b = col - 4 * m;
    if (b < 0 || b > 3) return word;
    return (word & ~(0xFFu << (8 * b))) | (v << (8 * b));
}

// value of lane-1 (row above); lane 0 gets `edge`
__device__ inline uint32_t from_above(uint32_t x, uint32_t edge)
{
    uint32_t v = __shfl_up(x, 1, 64);
    return lane_id() == 0 ? edge : v;
}
// value of lane+1 (row below); lane 63 gets `edge`
__device__ inline uint32_t from_below(uint32_t x, uint32_t edge)
{
    uint32_t v = __shfl_down(x, 1, 64);
    return lane_id() == 63 ? edge : v;
}

// w codes of one raster row into 16 words (bytes beyond w unspecified):
// 16-byte loads when the row is 16-byte aligned, else words, else bytes.
__device__ inline void load_codes(const uint8_t *__restrict__ row, int w, uint32_t (&W)[kWords])
{
    if ((((uintptr_t)row) & 15) == 0 && (w & 15) == 0) {
        const uint4 *row16 = reinterpret_cast<const uint4 *>(row);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (16 * i < w) {
                uint4 v = row16[i];
                W[4 * i] = v.x;
                W[4 * i + 1] = v.y;
                W[4 * i + 2] = v.z;
                W[4 * i + 3] = v.w;
            }
    } else if ((((uintptr_t)row) & 3) == 0 && (w & 3) == 0) {
        const uint32_t *row4 = reinterpret_cast<const uint32_t *>(row);
#pragma unroll
        for (int m = 0; m < kWords; ++m)
            if (4 * m < w) W[m] = row4[m];
    } else {
        // the aligned 4-byte words that cover the row, joined with byte
        // funnel shifts: the first and the last word reach at most 3 bytes
        // outside the row, inside the aligned word of a byte of the row (so
        // on its page); bytes past the row's end are left for the caller
        const uintptr_t a = reinterpret_cast<uintptr_t>(row);
        const uint32_t *base = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a & 3);
        const int nw = (int)((sh + (uint32_t)w + 3u) >> 2);  // words over the row's bytes
        uint32_t cur = base[0];
#pragma unroll
        for (int m = 0; m < kWords; ++m) {
            if (4 * m < w) {
                const uint32_t nxt = base[m + 1 < nw ? m + 1 : nw - 1];
                W[m] = __builtin_amdgcn_alignbyte(nxt, cur, sh);
                cur = nxt;
            }
        }
    }
}

// Codes of tile row r (lane r), padded with 0xFF outside the tile; codes
// above 9 are reported and replaced by NoData.
__device__ inline void load_row(const uint8_t *__restrict__ dirs, const Geo &g, const WTile &T,
                                uint32_t (&W)[kWords], uint32_t *status)
{
    const int r = lane_id();
#pragma unroll
    for (int m = 0; m < kWords; ++m) W[m] = 0xFFFFFFFFu;
    if (r >= T.h) return;
    load_codes(dirs + (T.r0 + r) * g.cols + T.c0, T.w, W);
    // pad columns beyond the tile
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        int valid = T.w - 4 * m;  // bytes of this word inside the tile
        if (valid <= 0) W[m] = 0xFFFFFFFFu;
        else if (valid < 4) W[m] |= 0xFFFFFFFFu << (8 * valid);
    }
    // codes 10..255 inside the tile are invalid
    bool bad = false;
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        uint32_t x = W[m];
        // bytes >= 10: (x & 0x7F) + 0x76 carries into bit 7, or bit 7 already set
        uint32_t ge10 = (((x & 0x7F7F7F7Fu) + 0x76767676u) | x) & 0x80808080u;
        uint32_t pad = eq_bytes(x, 0xFFu);
        if (ge10 & ~pad) bad = true;
    }
    if (bad) {
        set_status(status, kStatusDirCode);
#pragma unroll
        for (int m = 0; m < kWords; ++m) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                uint32_t k = (W[m] >> (8 * b)) & 0xFFu;
                if (k > kNoData && k != 0xFFu) k = kNoData;
                v |= k << (8 * b);
            }
            W[m] = v;
        }
    }
}

// Codes of a row outside the tile (the halo rows above / below), for columns
// -1 .. w; bytes outside the raster are 0xFF.  Returns words for columns
// 0..63 in H and the corner bytes in left / right.
__device__ inline void load_halo_row(const uint8_t *__restrict__ dirs, const Geo &g, const WTile &T,
                                     int64_t gr, uint32_t (&H)[kWords], uint32_t &left,
                                     uint32_t &right)
{
#pragma unroll
    for (int m = 0; m < kWords; ++m) H[m] = 0xFFFFFFFFu;
    left = right = 0xFFu;
    if (gr < 0 || gr >= g.rows) return;
    const uint8_t *row = dirs + gr * g.cols + T.c0;
    load_codes(row, T.w, H);
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        int valid = T.w - 4 * m;  // bytes of this word inside the tile's columns
        if (valid <= 0) H[m] = 0xFFFFFFFFu;
        else if (valid < 4) H[m] |= 0xFFFFFFFFu << (8 * valid);
    }
    if (T.c0 > 0) left = row[-1];
    if (T.c0 + T.w < g.cols) right = row[T.w];
}

// Per-lane setup result (bit c = column c of this lane's row).
struct Setup {
    uint64_t noflow; // forward: NoFlow cells
    uint64_t src;    // forward: data cells without in-tile donors
    uint64_t entry;  // data cells with a donor in another tile
    uint64_t root;   // adjoint: data cells without an in-tile receiver
    uint64_t valid;  // data cells
};

// Writes the cell bytes of the tile and its frame.
//   MODE 0 (forward): code | pending donors of a confluence << 4;
//   MODE 1 (links only): code;
//   MODE 2 (upstream walks): bit j = the neighbour in direction j is a donor.
// Entries are found when WANT_ENTRY, roots when MODE == 2 (NoData bytes are
// then 0xFF).
template <int MODE, bool WANT_ENTRY>
__device__ inline Setup setup_tile(const uint8_t *__restrict__ dirs, const Geo &g, const WTile &Tl,
                                   uint8_t *cb8, uint32_t *status)
{
    const int r = lane_id();
    uint32_t W[kWords], A[kWords], B[kWords];
    load_row(dirs, g, Tl, W, status);
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        A[m] = from_above(W[m], 0xFFFFFFFFu);
        B[m] = from_below(W[m], 0xFFFFFFFFu);
    }
    Setup St;
    St.noflow = St.src = St.entry = St.root = St.valid = 0;
    const uint32_t G = 0xFFFFFFFFu;  // guard word outside the tile
    const bool own = r < Tl.h;
    uint8_t *rowb = cb8 + (r + 1) * Tl.S + 1;
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        uint32_t a0 = m ? A[m - 1] : G, a2 = m + 1 < kWords ? A[m + 1] : G;
        uint32_t n0 = m ? W[m - 1] : G, n2 = m + 1 < kWords ? W[m + 1] : G;
        uint32_t b0 = m ? B[m - 1] : G, b2 = m + 1 < kWords ? B[m + 1] : G;
        uint32_t vm = valid_markers(W[m]);
        St.valid |= (uint64_t)marker_bits(vm) << (4 * m);
        uint32_t bytes;
        if (MODE == 0 || MODE == 2) {
            // per direction j: 0x80 where the neighbour in direction j flows in
            uint32_t e[8];
            e[0] = eq_bytes(left1(A[m], a0), 7);
            e[1] = eq_bytes(A[m], 6);
            e[2] = eq_bytes(right1(a2, A[m]), 5);
            e[3] = eq_bytes(left1(W[m], n0), 4);
            e[4] = eq_bytes(right1(n2, W[m]), 3);
            e[5] = eq_bytes(left1(B[m], b0), 2);
            e[6] = eq_bytes(B[m], 1);
            e[7] = eq_bytes(right1(b2, B[m]), 0);
            if (MODE == 0) {
                uint32_t cnt = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) cnt += e[j] >> 7;
                // the high nibble keeps the pending-donor count of confluences
                // only; 0 marks a cell with one donor (or none)
                uint32_t single = (eq_bytes(cnt, 1) >> 7) * 0xFFu;
                bytes = W[m] | ((cnt & ~single) << 4);
                St.src |= (uint64_t)marker_bits(zero_bytes(cnt) & vm) << (4 * m);
                St.noflow |= (uint64_t)marker_bits(eq_bytes(W[m], kNoFlow)) << (4 * m);
            } else {
                uint32_t mask = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) mask |= (e[j] >> 7) << j;
                // NoData cells: 0xFF (never walked; marks them after the walks)
                bytes = mask | (~(vm >> 7) & 0x01010101u) * 0xFFu;
                // roots: NoFlow, or a direction whose target is outside the tile / NoData
                uint32_t va = valid_markers(A[m]), vw = vm, vb = valid_markers(B[m]);
                uint32_t va0 = valid_markers(a0), va2 = valid_markers(a2);
                uint32_t vn0 = valid_markers(n0), vn2 = valid_markers(n2);
                uint32_t vb0 = valid_markers(b0), vb2 = valid_markers(b2);
                uint32_t tv[8];
                tv[0] = left1(va, va0);
                tv[1] = va;
                tv[2] = right1(va2, va);
                tv[3] = left1(vw, vn0);
                tv[4] = right1(vn2, vw);
                tv[5] = left1(vb, vb0);
                tv[6] = vb;
                tv[7] = right1(vb2, vb);
                uint32_t root = eq_bytes(W[m], kNoFlow);
#pragma unroll
                for (int k = 0; k < 8; ++k) root |= eq_bytes(W[m], k) & ~tv[k];
                St.root |= (uint64_t)marker_bits(root & vm) << (4 * m);
            }
        } else {
            bytes = W[m];
        }
        if (own) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (4 * m + b < Tl.w) rowb[4 * m + b] = (uint8_t)(bytes >> (8 * b));
        }
    }
    if (MODE != 2) {
        // frame: rows -1 and h (columns -1 .. w), columns -1 and w
        const int S = Tl.S;
        for (int j = r; j < S; j += 64) {
            int64_t gc = Tl.c0 + j - 1;
            bool cin = gc >= 0 && gc < g.cols;
            cb8[j] = (uint8_t)((Tl.r0 > 0 && cin) ? kFrameTile : kFrameOut);
            cb8[(Tl.h + 1) * S + j] = (uint8_t)((Tl.r0 + Tl.h < g.rows && cin) ? kFrameTile : kFrameOut);
        }
        if (own) {
            cb8[(r + 1) * S] = (uint8_t)(Tl.c0 > 0 ? kFrameTile : kFrameOut);
            cb8[(r + 1) * S + Tl.w + 1] = (uint8_t)(Tl.c0 + Tl.w < g.cols ? kFrameTile : kFrameOut);
        }
    }
    if (WANT_ENTRY) {
        // halo: left / right neighbours of this row, rows above / below the tile
        uint32_t HL = 0xFFu, HR = 0xFFu;
        if (own) {
            const uint8_t *row = dirs + (Tl.r0 + r) * g.cols + Tl.c0;
            if (Tl.c0 > 0) HL = row[-1];
            if (Tl.c0 + Tl.w < g.cols) HR = row[Tl.w];
        }
        uint32_t H[kWords], Hl, Hr;
        int64_t hr = r == 0 ? Tl.r0 - 1 : Tl.r0 + Tl.h;
        if (r == 0 || r == Tl.h - 1) load_halo_row(dirs, g, Tl, hr, H, Hl, Hr);
        else {
#pragma unroll
            for (int m = 0; m < kWords; ++m) H[m] = G;
            Hl = Hr = 0xFFu;
        }
        // the cell at column 0 / w-1: donors among the left / right halo column
        uint32_t top_l = __shfl(Hl, 0, 64), top_r = __shfl(Hr, 0, 64);
        uint32_t bot_l = __shfl(Hl, Tl.h - 1, 64), bot_r = __shfl(Hr, Tl.h - 1, 64);
        uint32_t HLa = from_above(HL, top_l), HLb = from_below(HL, 0xFFu);
        uint32_t HRa = from_above(HR, top_r), HRb = from_below(HR, 0xFFu);
        if (r == Tl.h - 1) {
            // the halo row below; a one-row tile reads it in its own block below
            HLb = Tl.h > 1 ? bot_l : 0xFFu;
            HRb = Tl.h > 1 ? bot_r : 0xFFu;
        }
        uint64_t ent = 0;
        if ((HLa == 7u) || (HL == 4u) || (HLb == 2u)) ent |= 1ull;
        if ((HRa == 5u) || (HR == 3u) || (HRb == 0u)) ent |= 1ull << (Tl.w - 1);
        // row 0 / h-1: donors in the halo row above / below
        if (r == 0 || r == Tl.h - 1) {
            const bool top = (r == 0);
#pragma unroll
            for (int m = 0; m < kWords; ++m) {
                uint32_t h0 = m ? H[m - 1] : ((Hl << 24) | 0x00FFFFFFu);
                uint32_t h1 = put_byte(H[m], m, Tl.w, Hr);
                uint32_t h2 = m + 1 < kWords ? put_byte(H[m + 1], m + 1, Tl.w, Hr)
                                             : (Tl.w == kW ? (0xFFFFFF00u | Hr) : G);
                uint32_t e;
                if (top) e = eq_bytes(left1(h1, h0), 7) | eq_bytes(h1, 6) | eq_bytes(right1(h2, h1), 5);
                else e = eq_bytes(left1(h1, h0), 2) | eq_bytes(h1, 1) | eq_bytes(right1(h2, h1), 0);
                ent |= (uint64_t)marker_bits(e) << (4 * m);
            }
            // a one-row tile has the halo row below as well
            if (Tl.h == 1) {
                uint32_t H2[kWords], Hl2, Hr2;
                load_halo_row(dirs, g, Tl, Tl.r0 + 1, H2, Hl2, Hr2);
#pragma unroll
                for (int m = 0; m < kWords; ++m) {
                    uint32_t h0 = m ? H2[m - 1] : ((Hl2 << 24) | 0x00FFFFFFu);
                    uint32_t h1 = put_byte(H2[m], m, Tl.w, Hr2);
                    uint32_t h2 = m + 1 < kWords ? put_byte(H2[m + 1], m + 1, Tl.w, Hr2)
                                                 : (Tl.w == kW ? (0xFFFFFF00u | Hr2) : G);
                    uint32_t e = eq_bytes(left1(h1, h0), 2) | eq_bytes(h1, 1) |
                                 eq_bytes(right1(h2, h1), 0);
                    ent |= (uint64_t)marker_bits(e) << (4 * m);
                }
                if (Hl2 == 2u) ent |= 1ull;
                if (Hr2 == 0u) ent |= 1ull << (Tl.w - 1);
            }
        }
        St.entry = own ? (ent & St.valid) : 0;
    }
    return St;
}

// ---------------------------------------------------------------- queue ---
// Start cells wait in an LDS array of 32-bit entries: bits 0..12 the cell
// index, 13..20 the cell's byte (code, or donor mask for upstream walks),
// bit 21 = link walk, bits 22..29 the ring index of a link walk's start.
constexpr uint32_t kQIdx = 0x1FFFu;
constexpr int kQByte = 13;
constexpr uint32_t kQLink = 1u << 21;
constexpr int kQRing = 22;

// Link walk results kept in LDS until the records are written: the index of
// the exit cell reached, or one of these.
constexpr uint16_t kLlTerm = 0xFFFF;
constexpr uint16_t kLlCycle = 0xFFFE;

// fill_queue appends the cells of every lane's masks (lane r = tile row r,
// row-major order; m0's cells are plain walks, m1's link walks) at positions
// 0.. of the queue, at most `cap`, and clears the bits it wrote; returns how
// many it wrote (wave-uniform).
__device__ inline uint32_t fill_queue(uint32_t *q, uint32_t cap, const WTile &Tl, const uint8_t *cb8,
                                      uint32_t byte_mask, uint64_t &m0, uint64_t &m1)
{
    const int lane = lane_id();
    uint32_t n = (uint32_t)(__popcll(m0) + __popcll(m1));
    uint32_t incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    uint32_t pos = incl - n;
    const int rowbase = (lane + 1) * Tl.S + 1;
    while (m0 != 0 && pos < cap) {
        int c = __ffsll((unsigned long long)m0) - 1;
        m0 &= m0 - 1ull;
        const int idx = rowbase + c;
        q[pos++] = (uint32_t)idx | ((cb8[idx] & byte_mask) << kQByte);
    }
    while (m1 != 0 && pos < cap) {
        int c = __ffsll((unsigned long long)m1) - 1;
        m1 &= m1 - 1ull;
        const int idx = rowbase + c;
        q[pos++] = (uint32_t)idx | ((cb8[idx] & byte_mask) << kQByte) | kQLink |
                   ((uint32_t)ring_index(lane, c, Tl.h, Tl.w) << kQRing);
    }
    return total < cap ? total : cap;
}

__device__ inline int ring_of_idx(const WTile &Tl, int idx)
{
    int r, c;
    idx_rc(Tl, idx, r, c);
    return ring_index(r, c, Tl.h, Tl.w);
}

// Algorithm 2's link from a link-walk result.
__device__ inline uint16_t link_of(const WTile &Tl, uint16_t v, uint32_t *status)
{
    if (v == kLlCycle) {
        set_status(status, kStatusCycle);
        return kLinkTerm;
    }
    return v == kLlTerm ? kLinkTerm : (uint16_t)ring_of_idx(Tl, v);
}

// ---------------------------------------------------------------- walks ---

// Forward walks (Algorithm 1's accumulation in Kahn order) from every
// source.  avp[idx] holds each cell's seed and receives its accumulation.
// Returns the number of cells this lane finished.
//
// A walk ends on reaching a cell whose flow goes nowhere further inside the
// tile (NoFlow, NoData, the frame), so a walker's cell always has a code
// 0..7: its neighbour's index offset comes from a per-tile byte table with
// one v_perm (offset + 128 per code), and NoFlow sources are finished without
// a walk.  The claim and the plain step take no branches: an idle lane steps
// with selector 12 (byte 0) from index 128, i.e. to cell 0 of the frame (its
// step ends at once), and a store that does not apply goes to the value slot
// of a frame column (row lane % h, column -1), which nothing reads.  Only the
// confluence step branches.  SEED: 0 = seeds are read from avp at a claim
// (the read completes with the step's reads), 1 = every seed is 1.
// ABS (absorption, Eq. (1) with alpha(n, p) = alpha(n) in [0, 1]): a walker
// passes alpha(cur) A(cur) on; alp holds alpha per cell, laid out like avp.
template <typename VT, int SEED, bool ABS = false>
__device__ inline int fwd_walks(const WTile &Tl, uint8_t *lds8, uint8_t *cb8, uint32_t *cbw, VT *avp,
                                uint32_t *q, uint32_t qcap, uint64_t src, uint64_t noflow,
                                const float *alp = nullptr)
{
    using T = typename Acc<VT>::type;
    const int S = Tl.S;
    const int lane = lane_id();
    VT *mine = avp + (lane % Tl.h + 1) * S;
    // offset + 128 of directions 0..7: (dr, dc) = NW N NE W E SW S SE
    const uint32_t s8 = (uint32_t)S;
    const uint32_t lut_lo = (128u - s8 - 1u) | ((128u - s8) << 8) | ((128u - s8 + 1u) << 16) | (127u << 24);
    const uint32_t lut_hi = 129u | ((128u + s8 - 1u) << 8) | ((128u + s8) << 16) | ((128u + s8 + 1u) << 24);
    // NoFlow sources are complete as they are
    int visited = __popcll(src & noflow);
    src &= ~noflow;
    uint64_t none = 0;
    uint32_t ntask = __builtin_amdgcn_readfirstlane(fill_queue(q, qcap, Tl, cb8, 15u, src, none));
    uint32_t head = 0;
    bool more = __ballot(src != 0) != 0;
    int cur = -1;
    uint32_t code = 12u;
    T a = (T)0;
    for (;;) {
        const uint64_t idle = __ballot(cur < 0);
        if (head >= ntask) {
            if (more) {
                // the queue has been handed out completely: refill it
                ntask = __builtin_amdgcn_readfirstlane(fill_queue(q, qcap, Tl, cb8, 15u, src, none));
                head = 0;
                more = __ballot(src != 0) != 0;
            } else if (idle == ~0ull) {
                break;
            }
        }
        bool took = false;
        T a0 = (T)1;
        if (idle != 0 && head < ntask) {
            const uint32_t j = head + lanes_below(idle);
            const bool take = cur < 0 && j < ntask;
            const uint32_t t = q[take ? j : 0];
            const int nc = (int)(t & kQIdx);
            if constexpr (SEED == 0) a0 = (T)avp[take ? nc : S + 1];
            cur = take ? nc : cur;
            code = take ? ((t >> kQByte) & 15u) : code;
            took = take;
            visited += take ? 1 : 0;
            const uint32_t nidle = (uint32_t)__popcll(idle);
            head = (ntask - head < nidle) ? ntask : head + nidle;
        }
        const bool act = cur >= 0;
        const uint32_t sel = act ? code : 12u;
        const int base = act ? cur : 128;
        const int ni = base + (int)__builtin_amdgcn_perm(lut_hi, lut_lo, 0x0C0C0C00u | sel) - 128;
        const uint32_t nb = cb8[ni];
        T sv = (T)avp[ni];
        keep_read(sv);
        T al = (T)1;
        if constexpr (ABS) {
            al = (T)alp[base];
            keep_read(al);
        }
        keep_read(a0);
        a = took ? a0 : a;
        const T out = ABS ? al * a : a;  // what reaches the next cell
        const uint32_t nk = nb & 15u;
        const bool fw = act && nk < (uint32_t)kNoData;
        const bool plain = fw && nb < 16u;
        const T ap = out + sv;
        *(plain ? &avp[ni] : mine) = (VT)ap;
        bool last = false;
        if (fw && nb >= 16u) {
            // confluence: add this donor's total, count the arrival; the
            // last donor to arrive continues with the cell's total
            const int sh = 8 * (ni & 3) + 4;
            lds_add(lds8, &avp[ni], out);
            const uint32_t old = atomicSub(&cbw[ni >> 2], 1u << sh);
            last = ((old >> sh) & 15u) == 1u;
            if (last) a = (T)avp[ni];
        }
        a = plain ? ap : a;
        visited += (plain || last) ? 1 : 0;
        // the walk goes on from the next cell only if its flow stays in the tile
        cur = ((plain || last) && nk < (uint32_t)kNoFlow) ? ni : -1;
        code = nk;
    }
    return visited;
}

// Algorithm 2 (FollowPath) for the entries of a tile, after the forward
// walks: one walk per entry along its flow path to the cell whose flow leaves
// the tile (its exit: the cell index goes to ll[ring index of the entry]),
// or to the end of its flow inside the tile (kLlTerm), or kLlCycle after more
// steps than the tile has cells.  Only the low nibble (the code) of each
// cell byte is read.  Offsets as in fwd_walks; an idle lane steps to frame
// cell 0 (ll_dummy is the ring index of no walk).
// ABS: also the product of alpha over each entry's path up to (without) its
// exit, stored to pathp[node] (global) for the entry's node.
template <bool ABS = false>
__device__ inline void link_walks(const WTile &Tl, const uint8_t *cb8, uint32_t *q, uint32_t qcap,
                                  uint64_t ent, uint16_t *ll, int ll_dummy, const float *alp = nullptr,
                                  float *pathp = nullptr)
{
    const uint32_t s8 = (uint32_t)Tl.S;
    const uint32_t lut_lo = (128u - s8 - 1u) | ((128u - s8) << 8) | ((128u - s8 + 1u) << 16) | (127u << 24);
    const uint32_t lut_hi = 129u | ((128u + s8 - 1u) << 8) | ((128u + s8) << 16) | ((128u + s8 + 1u) << 24);
    uint64_t none = 0;
    uint32_t ntask = __builtin_amdgcn_readfirstlane(fill_queue(q, qcap, Tl, cb8, 15u, none, ent));
    uint32_t head = 0;
    bool more = __ballot(ent != 0) != 0;
    int cur = -1, steps = 0, ring = ll_dummy;
    uint32_t code = 12u;
    float p = 1.0f;
    const int max_steps = Tl.h * Tl.w;
    for (;;) {
        const uint64_t idle = __ballot(cur < 0);
        if (head >= ntask) {
            if (more) {
                ntask = __builtin_amdgcn_readfirstlane(fill_queue(q, qcap, Tl, cb8, 15u, none, ent));
                head = 0;
                more = __ballot(ent != 0) != 0;
            } else if (idle == ~0ull) {
                break;
            }
        }
        if (idle != 0 && head < ntask) {
            const uint32_t j = head + lanes_below(idle);
            const bool take = cur < 0 && j < ntask;
            const uint32_t t = q[take ? j : 0];
            cur = take ? (int)(t & kQIdx) : cur;
            code = take ? ((t >> kQByte) & 15u) : code;
            ring = take ? (int)(t >> kQRing) : ring;
            steps = take ? 0 : steps;
            p = take ? 1.0f : p;
            const uint32_t nidle = (uint32_t)__popcll(idle);
            head = (ntask - head < nidle) ? ntask : head + nidle;
        }
        const bool act = cur >= 0;
        const uint32_t sel = act ? code : 12u;
        const int base = act ? cur : 128;
        const int ni = base + (int)__builtin_amdgcn_perm(lut_hi, lut_lo, 0x0C0C0C00u | sel) - 128;
        const uint32_t nk = cb8[ni] & 15u;
        float al = 1.0f;
        if constexpr (ABS) al = alp[base];
        ++steps;
        const bool stop = nk >= (uint32_t)kNoFlow || steps > max_steps;
        const uint16_t v = steps > max_steps ? kLlCycle : (nk == kFrameTile ? (uint16_t)cur : kLlTerm);
        // only finishing walks store (the others would all hit one dummy slot)
        if (act && stop) ll[ring] = v;
        if constexpr (ABS) {
            if (act && stop) pathp[Tl.base + ring] = p;
            p *= al;
        }
        cur = (act && !stop) ? ni : -1;
        code = nk;
    }
}

// Upstream walks for the adjoint, local part: lambda_loc(d) = g(d) +
// lambda_loc(receiver) inside the tile (0 beyond a root), and for every cell
// the label of its root: the root's ring index if the root's flow leaves the
// tile into the raster (an exit), else kLabelTerm.  The adjoint of a cell is
// then lambda_loc plus the downstream sum of its root's exit.
//
// A walk starts at a root (or a queued cell) and moves to its first donor;
// the other donors of a branching cell are finished on the spot and queued.
// Cell bytes hold donor masks until a walk reaches the cell, then its label.
// Queue entries: index | donor mask << 13 | label << 22.  Roots that do not
// fit the queue wait in the lanes' masks; side donors that do not fit go to
// the pending bitmap (their label already in their byte; the donor mask is
// rebuilt from the direction raster when they are queued).  The upstream
// walks never leave the tile, so the value slots of the frame columns are
// free: row r's pending bits for columns 0..31 live in its slot of column
// -1, those for columns 32..63 in its slot of column w.
struct PendRows {
    uint32_t *v;  // the value area, as words, indexed like the cells
    WTile Tl;
    __device__ uint64_t get(int r) const
    {
        if (r >= Tl.h) return 0;
        const uint32_t lo = v[cidx(Tl, r, -1)];
        const uint32_t hi = kW > 32 ? v[cidx(Tl, r, Tl.w)] : 0u;
        return (uint64_t)lo | ((uint64_t)hi << 32);
    }
    __device__ void put(int r, uint64_t m) const
    {
        if (r >= Tl.h) return;
        v[cidx(Tl, r, -1)] = (uint32_t)m;
        if (kW > 32) v[cidx(Tl, r, Tl.w)] = (uint32_t)(m >> 32);
    }
    __device__ void add(int r, int c) const
    {
        if (kW <= 32 || c < 32) atomicOr(&v[cidx(Tl, r, -1)], 1u << (c & 31));
        else atomicOr(&v[cidx(Tl, r, Tl.w)], 1u << (c & 31));
    }
};
constexpr uint32_t kLabelTerm = 254;
constexpr uint32_t kLabelNoData = 255;

__device__ inline uint32_t donor_mask_global(const uint8_t *__restrict__ dirs, const Geo &g,
                                             const WTile &Tl, int r, int c)
{
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int nr = r + dir_dr(j), nc = c + dir_dc(j);
        if (nr < 0 || nr >= Tl.h || nc < 0 || nc >= Tl.w) continue;
        if (dirs[(Tl.r0 + nr) * g.cols + Tl.c0 + nc] == (uint8_t)(7 - j)) m |= 1u << j;
    }
    return m;
}

// Queue fill for upstream walks from lane masks (lane = tile row).  ROOTS:
// label from the exit bitmap, mask from the cell byte; otherwise (pending
// side donors): label from the cell byte, mask rebuilt from dirs.
template <bool ROOTS>
__device__ inline uint32_t fill_up(uint32_t *q, uint32_t cap, const WTile &Tl, const Geo &g,
                                   const uint8_t *__restrict__ dirs, const uint8_t *cb8,
                                   const uint32_t *exitbits, uint64_t &m)
{
    const int lane = lane_id();
    const uint32_t n = (uint32_t)__popcll(m);
    uint32_t incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    uint32_t pos = incl - n;
    const int rowbase = (lane + 1) * Tl.S + 1;
    while (m != 0 && pos < cap) {
        const int c = __ffsll((unsigned long long)m) - 1;
        m &= m - 1ull;
        const int idx = rowbase + c;
        uint32_t mask, label;
        if (ROOTS) {
            mask = cb8[idx];
            const int p = ring_index(lane, c, Tl.h, Tl.w);
            label = (p >= 0 && ((exitbits[p >> 5] >> (p & 31)) & 1u)) ? (uint32_t)p : kLabelTerm;
        } else {
            mask = donor_mask_global(dirs, g, Tl, lane, c);
            label = cb8[idx];
        }
        q[pos++] = (uint32_t)idx | (mask << kQByte) | (label << kQRing);
    }
    return total < cap ? total : cap;
}

// With absorption (ABS), lambda_loc(d) = g(d) + alpha(d) lambda_loc(receiver)
// and each cell also gets P(d), the product of alpha along its in-tile path,
// itself and its root included: alp holds alpha and is overwritten with P as
// cells are reached (a root keeps P = alpha(root)).
template <bool ABS = false>
__device__ inline int up_walks(const WTile &Tl, const Geo &g, const uint8_t *__restrict__ dirs,
                               uint8_t *cb8, float *avp, uint32_t *q, uint32_t qcap, uint64_t roots,
                               const uint32_t *exitbits, float *alp = nullptr)
{
    const PendRows pend{reinterpret_cast<uint32_t *>(avp), Tl};
    const int S = Tl.S;
    const int lane = lane_id();
    int visited = 0;
    uint32_t head = 0;
    uint32_t tail = __builtin_amdgcn_readfirstlane(
        fill_up<true>(q, qcap, Tl, g, dirs, cb8, exitbits, roots));
    bool roots_left = __ballot(roots != 0) != 0;
    bool pending = false;
    pend.put(lane, 0);
    int cur = -1;
    uint32_t mask = 0, label = 0;
    float a = 0.0f, pp = 1.0f;
    for (;;) {
        const uint64_t idle = __ballot(cur < 0);
        if (head >= tail) {
            if (roots_left) {
                head = 0;
                tail = __builtin_amdgcn_readfirstlane(
                    fill_up<true>(q, qcap, Tl, g, dirs, cb8, exitbits, roots));
                roots_left = __ballot(roots != 0) != 0;
            } else if (pending) {
                // queue empty: move pending side donors into it
                uint64_t m = pend.get(lane);
                head = 0;
                tail = __builtin_amdgcn_readfirstlane(
                    fill_up<false>(q, qcap, Tl, g, dirs, cb8, exitbits, m));
                pend.put(lane, m);
                pending = __ballot(m != 0) != 0;
            } else if (idle == ~0ull) {
                break;
            }
        }
        if (idle != 0 && head < tail) {
            const uint32_t j = head + lanes_below(idle);
            if (cur < 0 && j < tail) {
                const uint32_t t = q[j & (qcap - 1)];
                cur = (int)(t & kQIdx);
                mask = (t >> kQByte) & 0xFFu;
                label = t >> kQRing;
                a = avp[cur];
                if constexpr (ABS) pp = alp[cur];
                cb8[cur] = (uint8_t)label;
            }
            const uint32_t nidle = (uint32_t)__popcll(idle);
            head = (tail - head < nidle) ? tail : head + nidle;
        }
        uint32_t rest = 0;
        const int from = cur;
        const float af = a, pf = pp;
        if (cur >= 0) {
            if (mask == 0) {
                cur = -1;
            } else {
                const uint32_t j0 = (uint32_t)__ffs(mask) - 1u;
                rest = mask & (mask - 1u);
                const int d = cur + dir_off(j0, S);
                const uint32_t nm = cb8[d];
                float sd = avp[d];
                keep_read(sd);
                cb8[d] = (uint8_t)label;
                if constexpr (ABS) {
                    float ad = alp[d];
                    keep_read(ad);
                    a = sd + ad * a;
                    pp = ad * pp;
                    alp[d] = pp;
                } else {
                    a += sd;
                }
                avp[d] = a;
                ++visited;
                cur = d;
                mask = nm;
            }
        }
        // side donors: finish and queue them
        while (__ballot(rest != 0) != 0) {
            const bool has = rest != 0;
            int d = 0;
            uint32_t dm = 0;
            if (has) {
                const uint32_t j = (uint32_t)__ffs(rest) - 1u;
                rest &= rest - 1u;
                d = from + dir_off(j, S);
                dm = cb8[d];
                cb8[d] = (uint8_t)label;
                if constexpr (ABS) {
                    const float ad = alp[d];
                    avp[d] = avp[d] + ad * af;
                    alp[d] = ad * pf;
                } else {
                    avp[d] += af;
                }
                ++visited;
            }
            const uint64_t b = __ballot(has);
            const uint32_t slot = tail + lanes_below(b);
            const uint32_t room = qcap - (tail - head);
            if (has) {
                if (slot - tail < room) {
                    q[slot & (qcap - 1)] = (uint32_t)d | (dm << kQByte) | (label << kQRing);
                } else {
                    int rr, cc;
                    idx_rc(Tl, d, rr, cc);
                    pend.add(rr, cc);
                }
            }
            uint32_t nb = (uint32_t)__popcll(b);
            if (nb > room) {
                pending = true;
                nb = room;
            }
            tail += nb;
        }
    }
    return visited;
}

}  // namespace wk

// ------------------------------------------------------------ LDS layout --
// Per tile: cell bytes (with frame), values (one per cell, frame columns
// included, frame rows excluded), the queue, and a tail area.  Speculative
// value reads of frame rows land in the cell bytes (before) or the queue
// (after), both at least 4 (S + 1) bytes long.
struct WLayout {
    int av, al, q, tail, total;
    uint32_t qcap;
};

// LDS value type of the forward passes: local unit counts of pass 1 in 16 bits.
template <int PASS, typename T>
using FwdLds = typename std::conditional<PASS == 1 && std::is_same<T, uint32_t>::value, uint16_t, T>::type;

enum WalkKind { kWalkFwd1 = 0, kWalkFwd2 = 1, kWalkAdj1 = 2, kWalkAdj2 = 3 };

__host__ __device__ inline WLayout walk_layout(int th, int tw, int kind, int vbytes = 4,
                                               bool absorb = false)
{
    WLayout L;
    const int S = tw + 2;
    int cb = (th + 2) * S;
    if (cb < 4 * (S + 1)) cb = 4 * (S + 1);
    L.av = (cb + 15) & ~15;
    // absorption: each cell's alpha after the values, laid out like them
    L.al = L.av + ((th * S * vbytes + 15) & ~15);
    L.q = absorb ? L.al + ((th * S * 4 + 15) & ~15) : L.al;
    // queue entries: start cells (forward queues, refilled from the lanes'
    // masks when empty) or roots and side donors as walks branch (adjoint;
    // side donors that do not fit wait in the pending bitmap)
    L.qcap = 128u;
    L.tail = L.q + (int)L.qcap * 4;
    int tail = 0;
    if (kind == kWalkFwd1) tail = (ring_size(th, tw) * 2 + 2 + 15) & ~15;  // links + a spare slot
    if (kind == kWalkAdj1) tail = 32;  // exit bitmap (the pending bitmap uses the frame value slots)
    L.total = L.tail + tail;
    return L;
}

// ---------------------------------------------------------------- kernels --
// Row transfers between a global array (row-major, `cols` wide) and the
// tile's LDS values.  Vector path (16-byte aligned rows, width a multiple of
// 4): lane l moves columns 4 (l % 16) .. + 3 of rows l / 16 + 4 i, and all
// 16 loads (or LDS reads) of a lane are issued before their results are
// used, so a wavefront keeps up to 16 KiB in flight.
__device__ inline bool rows_vec(const wk::WTile &Tl, const Geo &g, const void *p)
{
    return ((g.cols & 3) == 0) && ((Tl.w & 3) == 0) && ((Tl.c0 & 3) == 0) &&
           ((reinterpret_cast<uintptr_t>(p) & 15) == 0);
}

// Vector path: the tile as h x w/4 groups of 4 cells; group k of a lane is
// lane + 64 k (row gi / (w/4) by a scaled reciprocal, exact for h <= 64 and
// w/4 <= 16), so no lane idles when w < 64.
struct RowGroups {
    int ncg, ngr;
    uint32_t inv;
};

__device__ inline RowGroups row_groups(const wk::WTile &Tl)
{
    RowGroups G;
    G.ncg = Tl.w >> 2;
    G.ngr = Tl.h * G.ncg;
    G.inv = (65536u + (uint32_t)G.ncg - 1u) / (uint32_t)(G.ncg > 0 ? G.ncg : 1);
    return G;
}

__device__ inline void group_rc(const RowGroups &G, int gi, int &r, int &c)
{
    r = (int)(((uint32_t)gi * G.inv) >> 16);
    c = 4 * (gi - r * G.ncg);
}

// (Loads by 16-column quarters of 4 rows: lane l takes columns 4 (l % 16)
// .. + 3 of rows l / 16 + 4 i, which keeps fewer addresses live than the
// group order.)
template <typename T>
__device__ inline void rows_in(const wk::WTile &Tl, const Geo &g, T *avp, const T *__restrict__ src)
{
    const int lane = wk::lane_id();
    if (rows_vec(Tl, g, src)) {
        const int c = 4 * (lane & 15), rq = lane >> 4;
        uint4 v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = rq + 4 * i;
            if (r < Tl.h && c < Tl.w)
                v[i] = *reinterpret_cast<const uint4 *>(src + (Tl.r0 + r) * g.cols + Tl.c0 + c);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = rq + 4 * i;
            if (r < Tl.h && c < Tl.w) {
                T *d = avp + wk::cidx(Tl, r, c);
                d[0] = __builtin_bit_cast(T, v[i].x);
                d[1] = __builtin_bit_cast(T, v[i].y);
                d[2] = __builtin_bit_cast(T, v[i].z);
                d[3] = __builtin_bit_cast(T, v[i].w);
            }
        }
        return;
    }
    const int c = lane;
    if (c >= Tl.w) return;
#pragma unroll 8
    for (int r = 0; r < Tl.h; ++r) avp[wk::cidx(Tl, r, c)] = src[(Tl.r0 + r) * g.cols + Tl.c0 + c];
}

// Every value slot of the tile's rows (frame columns included) to v, with
// 16-byte LDS stores over the whole value area.
template <typename T>
__device__ inline void rows_fill(const wk::WTile &Tl, T *avp, T v)
{
    uint32_t w;
    if constexpr (sizeof(T) == 2) w = (uint32_t)__builtin_bit_cast(uint16_t, v) * 0x00010001u;
    else w = __builtin_bit_cast(uint32_t, v);
    uint4 *p = reinterpret_cast<uint4 *>(avp + Tl.S);  // 16-byte aligned (layout)
    const int n16 = (Tl.h * Tl.S * (int)sizeof(T) + 15) >> 4;
    for (int i = wk::lane_id(); i < n16; i += 64) p[i] = make_uint4(w, w, w, w);
}

// out = avp for data cells, 0 for NoData (valid: this lane's row mask)
template <typename T>
__device__ inline void rows_out(const wk::WTile &Tl, const Geo &g, const T *avp, uint64_t valid, T *out)
{
    const int lane = wk::lane_id();
    const uint32_t vlo = (uint32_t)valid, vhi = (uint32_t)(valid >> 32);
    if (rows_vec(Tl, g, out)) {
        const RowGroups G = row_groups(Tl);
        uint4 v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int gi = lane + 64 * k;
            int r, c;
            group_rc(G, gi, r, c);
            const uint32_t lo = (uint32_t)__shfl((int)vlo, r & 63, 64);
            const uint32_t hi = (uint32_t)__shfl((int)vhi, r & 63, 64);
            const uint32_t bits = (c < 32 ? lo >> c : hi >> (c - 32)) & 15u;
            if (gi < G.ngr) {
                const T *s = avp + wk::cidx(Tl, r, c);
                v[k].x = (bits & 1u) ? __builtin_bit_cast(uint32_t, s[0]) : 0u;
                v[k].y = (bits & 2u) ? __builtin_bit_cast(uint32_t, s[1]) : 0u;
                v[k].z = (bits & 4u) ? __builtin_bit_cast(uint32_t, s[2]) : 0u;
                v[k].w = (bits & 8u) ? __builtin_bit_cast(uint32_t, s[3]) : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int gi = lane + 64 * k;
            if (gi < G.ngr) {
                int r, c;
                group_rc(G, gi, r, c);
                *reinterpret_cast<uint4 *>(out + (Tl.r0 + r) * g.cols + Tl.c0 + c) = v[k];
            }
        }
        return;
    }
    const int c = lane;
    for (int r = 0; r < Tl.h; ++r) {
        uint32_t lo = __builtin_amdgcn_readlane(vlo, r), hi = __builtin_amdgcn_readlane(vhi, r);
        uint64_t row_valid = ((uint64_t)hi << 32) | lo;
        if (c < Tl.w) {
            T v = ((row_valid >> c) & 1ull) ? avp[wk::cidx(Tl, r, c)] : (T)0;
            out[(Tl.r0 + r) * g.cols + Tl.c0 + c] = v;
        }
    }
}

// Cell bytes of the tile to a raster-shaped byte array (4 bytes per lane
// when the rows are 4-byte aligned).
__device__ inline void bytes_out(const wk::WTile &Tl, const Geo &g, const uint8_t *cb8,
                                 uint8_t *__restrict__ dst)
{
    const int lane = wk::lane_id();
    if (((g.cols & 3) == 0) && ((Tl.w & 3) == 0) && ((Tl.c0 & 3) == 0) &&
        ((reinterpret_cast<uintptr_t>(dst) & 3) == 0)) {
        const int c = 4 * (lane & 15), rq = lane >> 4;
        for (int r = rq; r < Tl.h; r += 4) {
            if (c >= Tl.w) continue;
            const uint8_t *s = cb8 + wk::cidx(Tl, r, c);
            const uint32_t v = (uint32_t)s[0] | ((uint32_t)s[1] << 8) | ((uint32_t)s[2] << 16) |
                               ((uint32_t)s[3] << 24);
            *reinterpret_cast<uint32_t *>(dst + (Tl.r0 + r) * g.cols + Tl.c0 + c) = v;
        }
        return;
    }
    const int c = lane;
    if (c >= Tl.w) return;
    for (int r = 0; r < Tl.h; ++r) dst[(Tl.r0 + r) * g.cols + Tl.c0 + c] = cb8[wk::cidx(Tl, r, c)];
}

// One wavefront per tile (tiles up to 64 x 64).  Forward:
//   PASS 1: A_loc and links -> one record per perimeter cell; resolve state zeroed
//   PASS 2: seeds w + cross-tile inflow -> A for every cell
// Resolve state: indeg = children in the exit forest (graph_build); unit
// counts keep (inflow sum << 32 | arrivals) in acc; float weights keep the
// double sum in acc and arrivals in cnt.
template <int PASS, typename T, typename V, typename E, bool ABS = false>
__device__ __forceinline__ void fwd_tile(const uint8_t *__restrict__ dirs, const float *__restrict__ w,
                                const Geo &g, int64_t node0, int t, uint16_t *__restrict__ link,
                                T *__restrict__ aloc, uint32_t *__restrict__ indeg,
                                uint32_t *__restrict__ cnt, V *__restrict__ acc, E *__restrict__ ext,
                                T *__restrict__ out, uint32_t *status, uint8_t *lds8,
                                const float *__restrict__ alpha = nullptr, float *anode = nullptr,
                                float *pathp = nullptr)
{
    using namespace wk;
    WTile Tl = wtile_of(g, t);
    Tl.base += node0;
    using VT = FwdLds<PASS, T>;
    const WLayout L = walk_layout(g.th, g.tw, PASS == 1 ? kWalkFwd1 : kWalkFwd2, (int)sizeof(VT), ABS);
    float *alp = reinterpret_cast<float *>(lds8 + L.al) - Tl.S;  // ABS only
    uint8_t *cb8 = lds8;
    uint32_t *cbw = reinterpret_cast<uint32_t *>(lds8);
    VT *avp = reinterpret_cast<VT *>(lds8 + L.av) - Tl.S;
    uint32_t *q = reinterpret_cast<uint32_t *>(lds8 + L.q);
    uint16_t *ll = reinterpret_cast<uint16_t *>(lds8 + L.tail);
    const int lane = lane_id();

    Setup St = setup_tile<0, PASS == 1>(dirs, g, Tl, cb8, status);

    // seeds: own weight (+ resolved inflow on the perimeter in pass 2)
    if constexpr (std::is_same<VT, float>::value) {
        if (w) rows_in(Tl, g, avp, w);
        else rows_fill(Tl, avp, 1.0f);
    } else {
        rows_fill(Tl, avp, (VT)1);
    }
    if constexpr (ABS) rows_in(Tl, g, alp, alpha);
    if constexpr (PASS == 2) {
        __syncthreads();
        // all of a lane's loads first (a ring has at most 4 x 64 cells),
        // with what tells whether the tile's exits were finished by the
        // resolve: arrivals (the low word of acc) equal to the child count
        // for unit counts, an arrival count left at zero for float weights
        constexpr bool kCounts = std::is_same<T, uint32_t>::value;
        E e[kRingPerLane];
        uint32_t lk[kRingPerLane], ar[kRingPerLane], kc[kRingPerLane];
#pragma unroll
        for (int k = 0; k < kRingPerLane; ++k) {
            const int p = lane + 64 * k;
            const int64_t id = Tl.base + (p < Tl.P ? p : 0);
            e[k] = p < Tl.P ? ext[id] : (E)0;
            lk[k] = p < Tl.P ? link[id] : 0u;
            if constexpr (kCounts) {
                ar[k] = reinterpret_cast<const uint32_t *>(acc)[2 * id];
                kc[k] = indeg[id];
            } else {
                ar[k] = cnt[id];
                kc[k] = 0u;
            }
        }
        bool open = false;
#pragma unroll
        for (int k = 0; k < kRingPerLane; ++k) {
            const int p = lane + 64 * k;
            if (p < Tl.P) {
                int qr, qc;
                ring_cell(p, Tl.h, Tl.w, qr, qc);
                avp[cidx(Tl, qr, qc)] += (VT)e[k];
                open |= lk[k] == kLinkExt && ar[k] != kc[k];
            }
        }
        if (__ballot(open) != 0 && lane == 0) set_status(status, kStatusCycle);
    } else {
        for (int p = lane; p < Tl.P; p += 64) ll[p] = kLlTerm;
    }
    __syncthreads();

    // unit weights (uint32 counts): every seed is 1 in pass 1, and 1 plus the
    // resolved inflow on the perimeter in pass 2
    constexpr int kSeed = (std::is_same<T, uint32_t>::value && PASS == 1) ? 1 : 0;
    int visited = fwd_walks<VT, kSeed, ABS>(Tl, lds8, cb8, cbw, avp, q, L.qcap, St.src, St.noflow, alp);
    if (wave_sum(visited) != wave_sum(__popcll(St.valid)) && lane == 0) set_status(status, kStatusCycle);
    __syncthreads();
    // Algorithm 2's links of the entries (NoFlow entries keep kLlTerm)
    if constexpr (PASS == 1) {
        link_walks<ABS>(Tl, cb8, q, L.qcap, St.entry & ~St.noflow, ll, Tl.P, alp, pathp);
        __syncthreads();
    }

    if constexpr (PASS == 2) {
        rows_out(Tl, g, avp, St.valid, out);
        return;
    }

    for (int p = lane; p < Tl.P; p += 64) {
        int qr, qc;
        ring_cell(p, Tl.h, Tl.w, qr, qc);
        const int idx = cidx(Tl, qr, qc);
        uint32_t k = cb8[idx] & 15u;
        uint16_t Lk;
        if (k >= (uint32_t)kNoData) Lk = kLinkNoData;
        else if (k < (uint32_t)kNoFlow && (cb8[idx + dir_off(k, Tl.S)] & 15u) == kFrameTile) Lk = kLinkExt;
        else Lk = link_of(Tl, ll[p], status);
        int64_t id = Tl.base + p;
        link[id] = Lk;
        aloc[id] = k < (uint32_t)kNoData ? (T)avp[idx] : (T)0;
        if constexpr (ABS) anode[id] = alp[idx];
        indeg[id] = 0;
        if (cnt) cnt[id] = 0;
        acc[id] = (V)0;
        ext[id] = (E)0;
    }
}

// Adjoint, one wavefront per tile.
//   PASS 1: per perimeter cell, the link and (entries) the sum of g along its in-tile path
//   PASS 2: lambda for every cell, exits seeded with the resolved downstream sum
// Adjoint pass 1, one wavefront per tile: upstream walks give lambda_loc
// (written to out) and every cell's root label (written to root8, one byte
// per cell); each perimeter cell's record is its link (from its label) and
// S = lambda_loc, the sum of g along its in-tile path.
// With absorption (ABS): alpha is read too, lambda_loc follows the absorbing
// recursion, each perimeter cell's record also holds P (the alpha product of
// its in-tile path, Pg) and every cell's P goes to pout.
template <bool ABS = false>
__device__ __forceinline__ void adj_tile(const uint8_t *__restrict__ dirs, const float *__restrict__ gin,
                                const Geo &g, int64_t node0, int t, uint16_t *__restrict__ link,
                                float *__restrict__ Sg, float *__restrict__ out,
                                uint8_t *__restrict__ root8, uint32_t *status, uint8_t *lds8,
                                const float *__restrict__ alpha = nullptr, float *__restrict__ Pg = nullptr,
                                float *__restrict__ pout = nullptr, const uint32_t *__restrict__ cmap = nullptr,
                                const unsigned long long *__restrict__ mu = nullptr)
{
    using namespace wk;
    WTile Tl = wtile_of(g, t);
    Tl.base += node0;
    const WLayout L = walk_layout(g.th, g.tw, kWalkAdj1, 4, ABS);
    uint8_t *cb8 = lds8;
    float *avp = reinterpret_cast<float *>(lds8 + L.av) - Tl.S;
    float *alp = reinterpret_cast<float *>(lds8 + L.al) - Tl.S;  // ABS only
    uint32_t *q = reinterpret_cast<uint32_t *>(lds8 + L.q);
    uint32_t *exitbits = reinterpret_cast<uint32_t *>(lds8 + L.tail);
    const int lane = lane_id();

    Setup St = setup_tile<2, false>(dirs, g, Tl, cb8, status);
    rows_in(Tl, g, avp, gin);
    if constexpr (ABS) rows_in(Tl, g, alp, alpha);
    // exits: perimeter cells whose flow leaves the tile into the raster
    if (lane < 8) exitbits[lane] = 0;
    __syncthreads();
    uint32_t codes[kRingPerLane];
#pragma unroll
    for (int k = 0; k < kRingPerLane; ++k) {
        const int p = lane + 64 * k;
        codes[k] = kNoFlow;
        if (p < Tl.P) {
            int qr, qc;
            ring_cell(p, Tl.h, Tl.w, qr, qc);
            codes[k] = dirs[(Tl.r0 + qr) * g.cols + Tl.c0 + qc];
        }
    }
#pragma unroll
    for (int k = 0; k < kRingPerLane; ++k) {
        const int p = lane + 64 * k;
        const uint32_t kc = codes[k];
        if (p >= Tl.P || kc >= (uint32_t)kNoFlow) continue;
        int qr, qc;
        ring_cell(p, Tl.h, Tl.w, qr, qc);
        const int nr = qr + dir_dr(kc), nc = qc + dir_dc(kc);
        const int64_t gr = Tl.r0 + nr, gc = Tl.c0 + nc;
        const bool out_tile = nr < 0 || nr >= Tl.h || nc < 0 || nc >= Tl.w;
        if (out_tile && gr >= 0 && gr < g.rows && gc >= 0 && gc < g.cols)
            atomicOr(&exitbits[p >> 5], 1u << (p & 31));
    }
    __syncthreads();
    if (mu) {
        // finishing without retained sums (EVICT, for rasters streamed from
        // host memory): each exit starts from g + mu, the resolved sum of the
        // tile it flows into, so the walks give lambda itself
        for (int p = lane; p < Tl.P; p += 64) {
            const uint32_t cm = cmap[Tl.base + p];
            if (cm != kNone) {
                int qr, qc;
                ring_cell(p, Tl.h, Tl.w, qr, qc);
                avp[cidx(Tl, qr, qc)] += __uint_as_float((uint32_t)(mu[cm] >> 32));
            }
        }
        __syncthreads();
    }
    int visited = up_walks<ABS>(Tl, g, dirs, cb8, avp, q, L.qcap, St.root, exitbits, alp);
    if (wave_sum(visited + __popcll(St.root)) != wave_sum(__popcll(St.valid)) && lane == 0)
        set_status(status, kStatusCycle);
    __syncthreads();
    for (int p = lane; link && p < Tl.P; p += 64) {
        int qr, qc;
        ring_cell(p, Tl.h, Tl.w, qr, qc);
        const int idx = cidx(Tl, qr, qc);
        const uint32_t lab = cb8[idx];
        uint16_t Lk;
        if (lab == kLabelNoData) Lk = kLinkNoData;
        else if (lab == (uint32_t)p) Lk = kLinkExt;
        else if (lab == kLabelTerm) Lk = kLinkTerm;
        else Lk = (uint16_t)lab;
        link[Tl.base + p] = Lk;
        Sg[Tl.base + p] = lab == kLabelNoData ? 0.0f : avp[idx];
        if constexpr (ABS) Pg[Tl.base + p] = lab == kLabelNoData ? 0.0f : alp[idx];
    }
    if (out) rows_out(Tl, g, avp, St.valid, out);
    if (root8) bytes_out(Tl, g, cb8, root8);
    if constexpr (ABS) rows_out(Tl, g, alp, St.valid, pout);
}

// Adjoint pass 2, one wavefront per tile, no walks: lambda = lambda_loc +
// the downstream sum of the cell's root exit (mu of that perimeter node),
// in place in out.
// With absorption (ABS): lambda = lambda_loc + P mu, P per cell from pcell,
// mu words of 16 bytes (pointer, sum, product, unused).
__device__ inline float mu_value(unsigned long long w) { return __uint_as_float((uint32_t)(w >> 32)); }
__device__ inline float mu_value(uint4 w) { return __uint_as_float(w.y); }

template <bool ABS = false, typename W = unsigned long long>
__device__ __forceinline__ void adj_finish_tile(const Geo &g, int64_t node0, int t,
                                       const uint8_t *__restrict__ root8,
                                       const uint32_t *__restrict__ cmap,
                                       const W *__restrict__ mu,
                                       float *__restrict__ out, float *mu_l,
                                       const float *__restrict__ pcell = nullptr)
{
    using namespace wk;
    WTile Tl = wtile_of(g, t);
    Tl.base += node0;
    const int lane = lane_id();
    const bool vec = rows_vec(Tl, g, out) && ((reinterpret_cast<uintptr_t>(root8) & 3) == 0);
    // vector path: the tile as h x w/4 groups of 4 cells, group k of a lane
    // = lane + 64 k; every load is issued before the exit sums are fetched
    const int ncg = Tl.w >> 2, ngr = Tl.h * ncg;
    const uint32_t inv = (65536u + (uint32_t)ncg - 1u) / (uint32_t)(ncg > 0 ? ncg : 1);
    float4 v[16];
    float4 pv[ABS ? 16 : 1];
    uint32_t lb[16];
    if (vec) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int gi = lane + 64 * k;
            if (gi < ngr) {
                const int r = (int)(((uint32_t)gi * inv) >> 16), cg = gi - r * ncg;
                const int64_t o = (Tl.r0 + r) * g.cols + Tl.c0 + 4 * cg;
                v[k] = *reinterpret_cast<const float4 *>(out + o);
                lb[k] = *reinterpret_cast<const uint32_t *>(root8 + o);
                if constexpr (ABS) pv[k] = *reinterpret_cast<const float4 *>(pcell + o);
            }
        }
    }
    // mu is indexed by the exits' dense numbers; labels name exits only
    uint32_t cm[kRingPerLane];
#pragma unroll
    for (int k = 0; k < kRingPerLane; ++k) {
        const int p = lane + 64 * k;
        cm[k] = p < Tl.P ? cmap[Tl.base + p] : kNone;
    }
    float m[kRingPerLane];
#pragma unroll
    for (int k = 0; k < kRingPerLane; ++k)
        m[k] = cm[k] != kNone ? mu_value(mu[cm[k]]) : 0.0f;
#pragma unroll
    for (int k = 0; k < kRingPerLane; ++k) {
        const int p = lane + 64 * k;
        if (p < Tl.P) mu_l[p] = m[k];
    }
    __syncthreads();
    if (vec) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int gi = lane + 64 * k;
            if (gi < ngr) {
                const int r = (int)(((uint32_t)gi * inv) >> 16), cg = gi - r * ncg;
                const uint32_t l0 = lb[k] & 0xFFu, l1 = (lb[k] >> 8) & 0xFFu;
                const uint32_t l2 = (lb[k] >> 16) & 0xFFu, l3 = lb[k] >> 24;
                float4 x = v[k];
                if constexpr (ABS) {
                    const float4 pk = pv[k];
                    if (l0 < kLabelTerm) x.x += pk.x * mu_l[l0];
                    if (l1 < kLabelTerm) x.y += pk.y * mu_l[l1];
                    if (l2 < kLabelTerm) x.z += pk.z * mu_l[l2];
                    if (l3 < kLabelTerm) x.w += pk.w * mu_l[l3];
                } else {
                    if (l0 < kLabelTerm) x.x += mu_l[l0];
                    if (l1 < kLabelTerm) x.y += mu_l[l1];
                    if (l2 < kLabelTerm) x.z += mu_l[l2];
                    if (l3 < kLabelTerm) x.w += mu_l[l3];
                }
                *reinterpret_cast<float4 *>(out + (Tl.r0 + r) * g.cols + Tl.c0 + 4 * cg) = x;
            }
        }
        return;
    }
    // scalar path: the tile's cells in row-major order, lane + 64 k, 16 per
    // lane at a time with every load issued before use (row = j / w by a
    // scaled reciprocal, exact for j < 4096 and w <= 64)
    const int n = Tl.h * Tl.w;
    const uint32_t invw = ((1u << 20) + (uint32_t)Tl.w - 1u) / (uint32_t)Tl.w;
    for (int j0 = 0; j0 < n; j0 += 64 * 16) {
        int64_t o[16];
        uint32_t l[16];
        float x[16], pc[ABS ? 16 : 1];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int j = j0 + lane + 64 * k;
            l[k] = kLabelTerm;
            o[k] = 0;
            if (j < n) {
                const int r = (int)(((uint64_t)(uint32_t)j * invw) >> 20), c = j - r * Tl.w;
                o[k] = (Tl.r0 + r) * g.cols + Tl.c0 + c;
                l[k] = root8[o[k]];
                x[k] = out[o[k]];
                if constexpr (ABS) pc[k] = pcell[o[k]];
            }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (l[k] < kLabelTerm) out[o[k]] = x[k] + (ABS ? pc[k] * mu_l[l[k]] : mu_l[l[k]]);
    }
}

// ---- kernels: one raster (one wavefront per tile) ------------------------
// Workgroups go to the 8 XCDs in turn (block b to XCD b % 8), and each XCD
// has its own L2.  Block b therefore takes tile (b % 8) * n/8 + b / 8: every
// XCD works through a contiguous eighth of the row-major tile order, so the
// tiles beside and below a tile -- which read the same cache lines of the
// direction raster (row segments, halo cells) -- are served by one L2.
__device__ inline int xcd_tile(int b, int n)
{
    const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + i;
}

template <int PASS, typename T, typename V, typename E>
__global__ void __launch_bounds__(64)
fwd_walk(const uint8_t *__restrict__ dirs, const float *__restrict__ w, Geo g,
         uint16_t *__restrict__ link, T *__restrict__ aloc, uint32_t *__restrict__ indeg,
         uint32_t *__restrict__ cnt, V *__restrict__ acc, E *__restrict__ ext, T *__restrict__ out,
         uint32_t *status, int t0)
{
    // tiles t0 .. t0 + gridDim.x - 1 (a band of tile rows when streaming)
    extern __shared__ __align__(16) uint8_t lds8[];
    fwd_tile<PASS, T, V, E>(dirs, w, g, 0, t0 + xcd_tile(blockIdx.x, gridDim.x), link, aloc, indeg, cnt,
                            acc, ext, out, status, lds8);
}

// Forward passes with absorption (float weights): alpha per cell, and per
// perimeter node its alpha (anode) and an entry's path product (pathp).
template <int PASS>
__global__ void __launch_bounds__(64)
fwd_walk_absorb(const uint8_t *__restrict__ dirs, const float *__restrict__ w,
                const float *__restrict__ alpha, Geo g, uint16_t *__restrict__ link,
                float *__restrict__ aloc, uint32_t *__restrict__ indeg, uint32_t *__restrict__ cnt,
                double *__restrict__ acc, double *__restrict__ ext, float *__restrict__ out,
                uint32_t *status, float *anode, float *pathp)
{
    extern __shared__ __align__(16) uint8_t lds8[];
    fwd_tile<PASS, float, double, double, true>(dirs, w, g, 0, xcd_tile(blockIdx.x, gridDim.x), link,
                                                aloc, indeg, cnt, acc, ext, out, status, lds8, alpha,
                                                anode, pathp);
}

__global__ void __launch_bounds__(64, 3)
adj_walk(const uint8_t *__restrict__ dirs, const float *__restrict__ gin, Geo g,
         uint16_t *__restrict__ link, float *__restrict__ Sg, float *__restrict__ out,
         uint8_t *__restrict__ root8, uint32_t *status)
{
    extern __shared__ __align__(16) uint8_t lds8[];
    adj_tile(dirs, gin, g, 0, xcd_tile(blockIdx.x, gridDim.x), link, Sg, out, root8, status, lds8);
}

// Adjoint over a band of tile rows of a raster streamed from host memory
// (tiles t0 .. t0 + gridDim.x - 1).  Pass 1 writes the perimeter records
// only; pass 2 (mu0 / mu1 given: the jump buffers, jstate[0] naming the
// final one) seeds the exits with mu and writes lambda.
__global__ void __launch_bounds__(64, 3)
adj_walk_band(const uint8_t *__restrict__ dirs, const float *__restrict__ gin, Geo g,
              uint16_t *__restrict__ link, float *__restrict__ Sg, float *__restrict__ out, uint32_t *status,
              const uint32_t *__restrict__ cmap, const unsigned long long *__restrict__ mu0,
              const unsigned long long *__restrict__ mu1, const uint32_t *__restrict__ jstate, int t0)
{
    extern __shared__ __align__(16) uint8_t lds8[];
    const unsigned long long *mu = mu0 ? (jstate[0] == 1 ? mu1 : mu0) : nullptr;
    adj_tile(dirs, gin, g, 0, t0 + xcd_tile(blockIdx.x, gridDim.x), link, Sg, out, nullptr, status, lds8,
             nullptr, nullptr, nullptr, cmap, mu);
}

// Adjoint with absorption: pass 1 also writes P per perimeter node (Pg) and
// per cell (pout); pass 2 reads P and 16-byte exit words.
__global__ void __launch_bounds__(64, 3)
adj_walk_absorb(const uint8_t *__restrict__ dirs, const float *__restrict__ gin,
                const float *__restrict__ alpha, Geo g, uint16_t *__restrict__ link,
                float *__restrict__ Sg, float *__restrict__ Pg, float *__restrict__ out,
                float *__restrict__ pout, uint8_t *__restrict__ root8, uint32_t *status)
{
    extern __shared__ __align__(16) uint8_t lds8[];
    adj_tile<true>(dirs, gin, g, 0, xcd_tile(blockIdx.x, gridDim.x), link, Sg, out, root8, status, lds8,
                   alpha, Pg, pout);
}

__global__ void __launch_bounds__(64)
adj_finish_absorb(Geo g, const uint8_t *__restrict__ root8, const uint32_t *__restrict__ cmap,
                  const uint4 *__restrict__ mu0, const uint4 *__restrict__ mu1,
                  const uint32_t *__restrict__ jstate, const float *__restrict__ pcell,
                  float *__restrict__ out)
{
    __shared__ float mu_l[256];
    const uint4 *mu = jstate[0] == 1 ? mu1 : mu0;
    adj_finish_tile<true>(g, 0, xcd_tile(blockIdx.x, gridDim.x), root8, cmap, mu, out, mu_l, pcell);
}

__global__ void __launch_bounds__(64)
adj_finish(Geo g, const uint8_t *__restrict__ root8, const uint32_t *__restrict__ cmap,
           const unsigned long long *__restrict__ mu0, const unsigned long long *__restrict__ mu1,
           const uint32_t *__restrict__ jstate, float *__restrict__ out)
{
    __shared__ float mu_l[256];
    const unsigned long long *mu = jstate[0] == 1 ? mu1 : mu0;
    adj_finish_tile(g, 0, xcd_tile(blockIdx.x, gridDim.x), root8, cmap, mu, out, mu_l);
}

// ---- kernels: a batch of rasters ----------------------------------------
// One wavefront per tile of a range [t_begin, t_end) of the batch's tile
// list (rasters grouped by tile shape, by decreasing cost within a group,
// tiles row-major); the block-to-tile map is the XCD-aware one above, so
// each XCD works through a contiguous part of the list.  tile_dem[t] is the
// raster of batch tile t.
template <int PASS>
__global__ void __launch_bounds__(64)
fwd_walk_batch(const DemDesc *__restrict__ dems, const uint32_t *__restrict__ tile_dem,
               uint32_t t_begin, uint32_t t_end, uint16_t *__restrict__ link,
               float *__restrict__ aloc, uint32_t *__restrict__ indeg, uint32_t *__restrict__ cnt,
               double *__restrict__ acc, double *__restrict__ ext, uint32_t *status)
{
    extern __shared__ __align__(16) uint8_t lds8[];
    const uint32_t t = t_begin + (uint32_t)xcd_tile(blockIdx.x, gridDim.x);
    if (t >= t_end) return;
    const DemDesc D = dems[tile_dem[t]];
    fwd_tile<PASS, float, double, double>(D.dirs, D.w, D.g, D.node0, (int)(t - D.tile0), link, aloc,
                                          indeg, cnt, acc, ext, D.acc, status, lds8);
}

__global__ void __launch_bounds__(64, 3)
adj_walk_batch(const DemDesc *__restrict__ dems, const uint32_t *__restrict__ tile_dem,
               uint32_t t_begin, uint32_t t_end, uint16_t *__restrict__ link,
               float *__restrict__ Sg, uint32_t *status)
{
    extern __shared__ __align__(16) uint8_t lds8[];
    const uint32_t t = t_begin + (uint32_t)xcd_tile(blockIdx.x, gridDim.x);
    if (t >= t_end) return;
    const DemDesc D = dems[tile_dem[t]];
    adj_tile(D.dirs, D.gacc, D.g, D.node0, (int)(t - D.tile0), link, Sg, D.gw, D.root8, status, lds8);
}

// Batch pass 2: one wavefront per batch tile (an elementwise pass).
__global__ void __launch_bounds__(64)
adj_finish_batch(const DemDesc *__restrict__ dems, const uint32_t *__restrict__ tile_dem,
                 uint32_t ntiles, const uint32_t *__restrict__ cmap,
                 const unsigned long long *__restrict__ mu0,
                 const unsigned long long *__restrict__ mu1, const uint32_t *__restrict__ jstate)
{
    __shared__ float mu_l[256];
    const uint32_t t = (uint32_t)xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const unsigned long long *mu = jstate[0] == 1 ? mu1 : mu0;
    const DemDesc D = dems[tile_dem[t]];
    adj_finish_tile(D.g, D.node0, (int)(t - D.tile0), D.root8, cmap, mu, D.gw, mu_l);
}

__host__ inline size_t walk_lds_bytes(int th, int tw, int kind, int vbytes = 4, bool absorb = false)
{
    return (size_t)walk_layout(th, tw, kind, vbytes, absorb).total;
}


}  // namespace D8_WALK_NS
}  // namespace d8

#undef D8_WALK_KW
#undef D8_WALK_NS
