// walk.h -- one wavefront per tile: flow walkers in LDS.
//
// Tile shape: up to 64 rows x 64 columns.  Lane r owns tile row r during
// setup; its 64 direction codes sit in 16 registers (4 codes per word) and
// the donor counts of all 64 cells are found with byte-parallel compares
// against the rows above and below (fetched from lanes r-1 / r+1).  LDS then
// holds one byte per cell (code | pending donors of a confluence << 4) and
// one 32-bit value per cell (seed, then accumulation), with padded row strides.
//
// Forward walks (Algorithm 1's Kahn order, done by walkers): every source
// (a data cell without in-tile donors) starts a walk downstream.  Entering a
// cell with one donor, the walk simply adds that cell's seed.  Entering a
// confluence, the walk decrements its pending-donor count; only the last
// arriving donor continues, after gathering the donors' totals in fixed
// neighbour order.  All walks of a tile run in one wavefront, so the order of
// LDS operations -- and therefore every float sum -- is fixed by the input.
//
// Link walks (Algorithm 2, FollowPath): from every entry cell (a perimeter
// cell with a donor in another tile) to the end of its in-tile path; the
// adjoint's pass 1 sums g along the way.
#pragma once

#include "d8_common.h"

namespace d8 {
namespace wk {

constexpr int kW = 64;           // max tile width (columns)
constexpr int kH = 64;           // max tile height (rows) = lanes
constexpr int kWords = kW / 4;   // code words per row

struct WTile {
    int ty, tx, h, w, P;
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
    T.r0 = (int64_t)T.ty * g.th;
    T.c0 = (int64_t)T.tx * g.tw;
    T.base = node_base(g, T.ty, T.tx);
    return T;
}

// 0x80 in every zero byte of x, 0 elsewhere (exact, no carries between bytes).
__device__ inline uint32_t zero_bytes(uint32_t x)
{
    return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
}
__device__ inline uint32_t eq_bytes(uint32_t x, uint32_t k) { return zero_bytes(x ^ (k * 0x01010101u)); }
// bytes [4m-1 .. 4m+2] and [4m+1 .. 4m+4] of a row given words m-1, m, m+1
__device__ inline uint32_t left1(uint32_t cur, uint32_t prev) { return __builtin_amdgcn_alignbyte(cur, prev, 3); }
__device__ inline uint32_t right1(uint32_t next, uint32_t cur) { return __builtin_amdgcn_alignbyte(next, cur, 1); }

__device__ inline int lane_id() { return __lane_id(); }

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

// codes of tile row r (lane r), padded with 0xFF outside the tile; codes
// above 9 are reported and replaced by NoData.
__device__ inline void load_row(const uint8_t *__restrict__ dirs, const Geo &g, const WTile &T,
                                uint32_t (&W)[kWords], uint32_t *status)
{
    const int r = lane_id();
#pragma unroll
    for (int m = 0; m < kWords; ++m) W[m] = 0xFFFFFFFFu;
    if (r >= T.h) return;
    const uint8_t *row = dirs + (T.r0 + r) * g.cols + T.c0;
    if ((((uintptr_t)row) & 3) == 0 && (T.w & 3) == 0) {
        const uint32_t *row4 = reinterpret_cast<const uint32_t *>(row);
#pragma unroll
        for (int m = 0; m < kWords; ++m)
            if (4 * m < T.w) W[m] = row4[m];
    } else {
#pragma unroll
        for (int m = 0; m < kWords; ++m) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                int c = 4 * m + b;
                uint32_t k = c < T.w ? row[c] : 0xFFu;
                v |= k << (8 * b);
            }
            W[m] = v;
        }
    }
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

// Donor counts of the 4 cells of word m: each byte += 1 per neighbour whose
// code points at the cell (neighbour in direction j has code 7 - j).
// A/N/B: row above / own / below, words m-1, m, m+1.
__device__ inline uint32_t donor_count_word(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t n0,
                                            uint32_t n1, uint32_t n2, uint32_t b0, uint32_t b1,
                                            uint32_t b2)
{
    uint32_t cnt = 0;
    cnt += eq_bytes(left1(a1, a0), 7) >> 7;   // NW neighbour flows SE
    cnt += eq_bytes(a1, 6) >> 7;              // N flows S
    cnt += eq_bytes(right1(a2, a1), 5) >> 7;  // NE flows SW
    cnt += eq_bytes(left1(n1, n0), 4) >> 7;   // W flows E
    cnt += eq_bytes(right1(n2, n1), 3) >> 7;  // E flows W
    cnt += eq_bytes(left1(b1, b0), 2) >> 7;   // SW flows NE
    cnt += eq_bytes(b1, 1) >> 7;              // S flows N
    cnt += eq_bytes(right1(b2, b1), 0) >> 7;  // SE flows NW
    return cnt;
}

// byte b (0..3) of each 0x80-marker word packed into bit b
__device__ inline uint32_t marker_bits(uint32_t z)
{
    return ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u);
}

// j-th set bit (0-based) of a 64-bit mask
__device__ inline int nth_set_bit(uint64_t s, int j)
{
    int pos = 0;
#pragma unroll
    for (int half = 32; half >= 1; half >>= 1) {
        uint64_t low = s & ((1ull << half) - 1ull);
        int c = __popcll(low);
        if (j >= c) {
            j -= c;
            s >>= half;
            pos += half;
        }
    }
    return pos;
}

__device__ inline uint64_t clear_lowest(uint64_t s, int k)
{
    for (int i = 0; i < k; ++i) s &= s - 1ull;
    return s;
}

// Work dispenser over per-lane bit masks (lane = row, bit = column): hands
// out tasks in row-major order to idle lanes, ranks by lane order.  State is
// wavefront-uniform.
struct Dispenser {
    uint64_t rows_left;  // rows that still have tasks
    int row;             // current row, or -1
    uint64_t pend;       // tasks of the current row not yet handed out

    __device__ void init(uint64_t my_mask)
    {
        rows_left = __ballot(my_mask != 0);
        row = -1;
        pend = 0;
    }
    __device__ bool empty() const { return pend == 0 && rows_left == 0; }
    // Returns true and sets (r, c) for idle lanes that get a task.
    __device__ bool take(bool idle, uint64_t my_mask, int &r, int &c)
    {
        uint64_t free_lanes = __ballot(idle);
        bool got = false;
        while (free_lanes != 0 && !(pend == 0 && rows_left == 0)) {
            if (pend == 0) {
                row = __ffsll((unsigned long long)rows_left) - 1;
                rows_left &= rows_left - 1ull;
                uint32_t lo = __builtin_amdgcn_readlane((uint32_t)my_mask, row);
                uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(my_mask >> 32), row);
                pend = ((uint64_t)hi << 32) | lo;
                continue;
            }
            int nfree = __popcll(free_lanes), ntask = __popcll(pend);
            int k = nfree < ntask ? nfree : ntask;
            if (idle && !got) {
                uint64_t below = free_lanes & ((1ull << lane_id()) - 1ull);
                bool mine = (free_lanes >> lane_id()) & 1ull;
                int rank = __popcll(below);
                if (mine && rank < k) {
                    r = row;
                    c = nth_set_bit(pend, rank);
                    got = true;
                }
            }
            pend = clear_lowest(pend, k);
            free_lanes = clear_lowest(free_lanes, k);
        }
        return got;
    }
};

}  // namespace wk
}  // namespace d8

namespace d8 {
namespace wk {

// Per-tile LDS strides (words), odd so that lanes walking one column hit
// different banks.
struct Layout {
    int cbs, as;  // code-byte row stride, value row stride
    __device__ __host__ static int odd(int x) { return x | 1; }
    __device__ __host__ Layout(int tw) : cbs(odd((tw + 3) / 4 + 1)), as(odd(tw + 1)) {}
    __device__ int cbw(int r, int c) const { return r * cbs + (c >> 2); }
    __device__ int ai(int r, int c) const { return r * as + c; }
};

__device__ inline uint32_t cbyte(const uint32_t *cb, const Layout &L, int r, int c)
{
    return (cb[L.cbw(r, c)] >> (8 * (c & 3))) & 0xFFu;
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
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int c = 4 * m + b;
            uint32_t k = c < T.w ? row[c] : 0xFFu;
            v |= k << (8 * b);
        }
        H[m] = v;
    }
    if (T.c0 > 0) left = row[-1];
    if (T.c0 + T.w < g.cols) right = row[T.w];
}

// Walk state of one lane.
template <typename T>
struct Walker {
    int r = -1, c = -1;  // current cell, r < 0: idle
    uint32_t code = 0;
    T a = (T)0;
};

// One step of a forward walk from (w.r, w.c).  Returns false when the walk ends.
template <typename T>
__device__ inline bool fwd_step(Walker<T> &wk, const WTile &Tl, const Layout &L, uint32_t *cb, T *av,
                                int &visited)
{
    uint32_t k = wk.code;
    if (k >= (uint32_t)kNoFlow) return false;
    int rr = wk.r + dir_dr(k), cc = wk.c + dir_dc(k);
    if (rr < 0 || rr >= Tl.h || cc < 0 || cc >= Tl.w) return false;
    const int wi = L.cbw(rr, cc), sh = 8 * (cc & 3);
    uint32_t b = (cb[wi] >> sh) & 0xFFu;
    uint32_t kn = b & 15u;
    if (kn >= (uint32_t)kNoData) return false;
    const int ai = L.ai(rr, cc);
    if ((b >> 4) != 0u) {
        // confluence: only the last arriving donor continues
        uint32_t old = atomicSub(&cb[wi], 0x10u << sh);
        if (((old >> (sh + 4)) & 15u) != 1u) return false;
        T s = av[ai];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int nr = rr + dir_dr(j), nc = cc + dir_dc(j);
            if (nr < 0 || nr >= Tl.h || nc < 0 || nc >= Tl.w) continue;
            if ((cbyte(cb, L, nr, nc) & 15u) == (uint32_t)(7 - j)) s += av[L.ai(nr, nc)];
        }
        wk.a = s;
    } else {
        wk.a += av[ai];
    }
    av[ai] = wk.a;
    wk.r = rr;
    wk.c = cc;
    wk.code = kn;
    ++visited;
    return true;
}

}  // namespace wk
}  // namespace d8

namespace d8 {
namespace wk {

__device__ inline uint32_t valid_markers(uint32_t x)  // bytes with a data code 0..8
{
    uint32_t ge9 = (((x & 0x7F7F7F7Fu) + 0x77777777u) | x) & 0x80808080u;
    return ~ge9 & 0x80808080u;
}

// Set byte (col - 4m) of word m of a row to `v` when that column falls in the word.
__device__ inline uint32_t put_byte(uint32_t word, int m, int col, uint32_t v)
{
    int b = col - 4 * m;
    if (b < 0 || b > 3) return word;
    return (word & ~(0xFFu << (8 * b))) | (v << (8 * b));
}

// Per-lane setup result.
struct Setup {
    uint64_t src;    // forward: cells without in-tile donors (bit = column)
    uint64_t entry;  // cells with a donor in another tile
    uint64_t root;   // adjoint: cells without an in-tile receiver
    int valid;       // data cells in this row
};

// MODE 0: forward (writes code | confluence count << 4 into cb); MODE 1: adjoint pass 1
// (codes only); MODE 2: adjoint pass 2 (donor masks into cb).  Entries are
// found when WANT_ENTRY, roots when MODE == 2.
template <int MODE, bool WANT_ENTRY>
__device__ inline Setup setup_tile(const uint8_t *__restrict__ dirs, const Geo &g, const WTile &Tl,
                                   const Layout &L, uint32_t *cb, uint32_t *status)
{
    const int r = lane_id();
    uint32_t W[kWords], A[kWords], B[kWords];
    load_row(dirs, g, Tl, W, status);
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        A[m] = from_above(W[m], 0xFFFFFFFFu);
        B[m] = from_below(W[m], 0xFFFFFFFFu);
    }
    Setup S;
    S.src = S.entry = S.root = 0;
    S.valid = 0;
    const uint32_t G = 0xFFFFFFFFu;  // guard word outside the tile
#pragma unroll
    for (int m = 0; m < kWords; ++m) {
        uint32_t a0 = m ? A[m - 1] : G, a2 = m + 1 < kWords ? A[m + 1] : G;
        uint32_t n0 = m ? W[m - 1] : G, n2 = m + 1 < kWords ? W[m + 1] : G;
        uint32_t b0 = m ? B[m - 1] : G, b2 = m + 1 < kWords ? B[m + 1] : G;
        uint32_t vm = valid_markers(W[m]);
        S.valid += __popc(vm);
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
                // only; 0 marks a cell with one donor (or none), so a walk that
                // finds a non-zero nibble knows it entered a confluence
                uint32_t single = (eq_bytes(cnt, 1) >> 7) * 0xFFu;
                if (r < Tl.h && 4 * m < g.tw) cb[r * L.cbs + m] = W[m] | ((cnt & ~single) << 4);
                S.src |= (uint64_t)marker_bits(zero_bytes(cnt) & vm) << (4 * m);
            } else {
                uint32_t mask = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) mask |= (e[j] >> 7) << j;
                if (r < Tl.h && 4 * m < g.tw) cb[r * L.cbs + m] = mask & (vm >> 7) * 0xFFu;
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
                S.root |= (uint64_t)marker_bits(root & vm) << (4 * m);
            }
        } else {
            if (r < Tl.h && 4 * m < g.tw) cb[r * L.cbs + m] = W[m];
        }
    }
    if (WANT_ENTRY) {
        // halo: left / right neighbours of this row, rows above / below the tile
        uint32_t HL = 0xFFu, HR = 0xFFu;
        if (r < Tl.h) {
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
                uint32_t HLb1 = Hl2, HRb1 = Hr2;
                if (HLb1 == 2u) ent |= 1ull;
                if (HRb1 == 0u) ent |= 1ull << (Tl.w - 1);
            }
        }
        // data cells of this row only
        uint64_t vbits = 0;
#pragma unroll
        for (int m = 0; m < kWords; ++m) vbits |= (uint64_t)marker_bits(valid_markers(W[m])) << (4 * m);
        S.entry = (r < Tl.h) ? (ent & vbits) : 0;
    }
    return S;
}

// Algorithm 2's link for a walk from perimeter cell (qr, qc) that ended at
// (er, ec) because its direction leaves the tile (dir_out) or it terminates.
__device__ inline uint16_t link_for(const Geo &g, const WTile &Tl, int qr, int qc, int er, int ec,
                                    uint32_t code_e)
{
    if (code_e >= (uint32_t)kNoFlow) return kLinkTerm;
    int rr = er + dir_dr(code_e), cc = ec + dir_dc(code_e);
    if (rr >= 0 && rr < Tl.h && cc >= 0 && cc < Tl.w) return kLinkTerm;  // into NoData
    int64_t gr = Tl.r0 + rr, gc = Tl.c0 + cc;
    if (gr < 0 || gr >= g.rows || gc < 0 || gc >= g.cols) return kLinkTerm;
    if (er == qr && ec == qc) return kLinkExt;
    return (uint16_t)ring_index(er, ec, Tl.h, Tl.w);
}

// Link walks from every entry cell; SUM: also sum av along the path (the
// adjoint's pass 1).  Results go to ll[p] / sl[p] by ring index.
template <bool SUM>
__device__ inline void link_walks(const Geo &g, const WTile &Tl, const Layout &L, const uint32_t *cb,
                                  const float *av, uint64_t entry, uint16_t *ll, float *sl,
                                  uint32_t *status)
{
    Dispenser ds;
    ds.init(entry);
    int qr = -1, qc = -1, r = -1, c = -1, steps = 0;
    const int max_steps = Tl.h * Tl.w;
    uint32_t code = 0;
    float s = 0.0f;
    for (;;) {
        bool idle = r < 0;
        if (!__any(!idle) && ds.empty()) break;
        int nr, nc;
        if (ds.take(idle, entry, nr, nc)) {
            qr = r = nr;
            qc = c = nc;
            code = cbyte(cb, L, r, c) & 15u;
            s = 0.0f;
            steps = 0;
        }
        if (r < 0) continue;
        if (SUM) s += av[L.ai(r, c)];
        bool end = true;
        if (++steps > max_steps) {
            // longer than the tile has cells: the path runs into a cycle
            set_status(status, kStatusCycle);
            code = kNoFlow;
        }
        if (code < (uint32_t)kNoFlow) {
            int rr = r + dir_dr(code), cc = c + dir_dc(code);
            if (rr >= 0 && rr < Tl.h && cc >= 0 && cc < Tl.w) {
                uint32_t kn = cbyte(cb, L, rr, cc) & 15u;
                if (kn < (uint32_t)kNoData) {
                    r = rr;
                    c = cc;
                    code = kn;
                    end = false;
                }
            }
        }
        if (end) {
            int p = ring_index(qr, qc, Tl.h, Tl.w);
            ll[p] = link_for(g, Tl, qr, qc, r, c, code);
            if (SUM) sl[p] = s;
            r = -1;
        }
    }
}

// Forward walks over all sources; returns the number of cells finished by
// this lane (sources included).
template <typename T>
__device__ inline int forward_walks(const WTile &Tl, const Layout &L, uint32_t *cb, T *av,
                                    uint64_t src)
{
    Dispenser ds;
    ds.init(src);
    Walker<T> wk;
    int visited = 0;
    for (;;) {
        bool idle = wk.r < 0;
        if (!__any(!idle) && ds.empty()) break;
        int nr, nc;
        if (ds.take(idle, src, nr, nc)) {
            wk.r = nr;
            wk.c = nc;
            wk.code = cbyte(cb, L, nr, nc) & 15u;
            wk.a = av[L.ai(nr, nc)];
            ++visited;
        }
        if (wk.r < 0) continue;
        if (!fwd_step(wk, Tl, L, cb, av, visited)) wk.r = -1;
    }
    return visited;
}

__device__ inline int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace wk

// ---------------------------------------------------------------- kernels --
// One wavefront per tile (tiles up to 64 x 64).  Forward:
//   PASS 1: A_loc and links -> one record per perimeter cell, resolve state zeroed
//   PASS 2: seeds w + cross-tile inflow -> A for every cell
template <int PASS, typename T, typename V, typename E>
__global__ void __launch_bounds__(64)
fwd_walk(const uint8_t *__restrict__ dirs, const float *__restrict__ w, Geo g,
         uint16_t *__restrict__ link, T *__restrict__ aloc, uint32_t *__restrict__ indeg,
         V *__restrict__ acc, E *__restrict__ ext, T *__restrict__ out, uint32_t *status)
{
    using namespace wk;
    extern __shared__ uint32_t lds[];
    const WTile Tl = wtile_of(g, blockIdx.x);
    const Layout L(g.tw);
    uint32_t *cb = lds;
    T *av = reinterpret_cast<T *>(lds + g.th * L.cbs);
    uint16_t *ll = reinterpret_cast<uint16_t *>(lds + g.th * (L.cbs + L.as));
    const int r = lane_id();

    Setup S = setup_tile<0, PASS == 1>(dirs, g, Tl, L, cb, status);

    // seeds: own weight (+ resolved inflow on the perimeter in pass 2)
    if (r < Tl.h) {
        const float *wrow = w ? w + (Tl.r0 + r) * g.cols + Tl.c0 : nullptr;
        const bool edge_row = (r == 0 || r == Tl.h - 1);
        for (int c = 0; c < Tl.w; ++c) {
            T s = wrow ? (T)wrow[c] : (T)1;
            if (PASS == 2 && (edge_row || c == 0 || c == Tl.w - 1)) {
                int p = ring_index(r, c, Tl.h, Tl.w);
                s += (T)ext[Tl.base + p];
            }
            av[L.ai(r, c)] = s;
        }
    }
    for (int p = r; p < Tl.P; p += 64) ll[p] = kLinkTerm;
    __syncthreads();

    int visited = forward_walks<T>(Tl, L, cb, av, S.src);
    if (wave_sum(visited) != wave_sum(S.valid) && r == 0) set_status(status, kStatusCycle);

    if (PASS == 2) {
        __syncthreads();
        if (r < Tl.h) {
            T *orow = out + (Tl.r0 + r) * g.cols + Tl.c0;
            for (int c = 0; c < Tl.w; ++c) {
                uint32_t k = cbyte(cb, L, r, c) & 15u;
                orow[c] = k < (uint32_t)kNoData ? av[L.ai(r, c)] : (T)0;
            }
        }
        for (int p = r; p < Tl.P; p += 64) {
            int64_t id = Tl.base + p;
            if (link[id] != kLinkExt) continue;
            bool pending = indeg ? indeg[id] != 0 : (uint32_t)acc[id] != 0;
            if (pending) set_status(status, kStatusCycle);
        }
        return;
    }

    link_walks<false>(g, Tl, L, cb, nullptr, S.entry, ll, nullptr, status);
    __syncthreads();
    for (int p = r; p < Tl.P; p += 64) {
        int qr, qc;
        ring_cell(p, Tl.h, Tl.w, qr, qc);
        uint32_t k = cbyte(cb, L, qr, qc) & 15u;
        uint16_t Lk;
        if (k >= (uint32_t)kNoData) Lk = kLinkNoData;
        else {
            uint16_t out_link = link_for(g, Tl, qr, qc, qr, qc, k);
            Lk = (out_link == kLinkExt) ? kLinkExt : ll[p];
        }
        int64_t id = Tl.base + p;
        link[id] = Lk;
        aloc[id] = k < (uint32_t)kNoData ? av[L.ai(qr, qc)] : (T)0;
        if (indeg) indeg[id] = 0;
        acc[id] = (V)0;
        ext[id] = (E)0;
    }
}

}  // namespace d8

namespace d8 {
namespace wk {

// Upstream walks for the adjoint: lambda(d) = g(d) + lambda(receiver).  A walk
// starts at a root (finished) and moves to one donor at a time; the other
// donors of a branching cell are finished on the spot and queued in a bitmap
// (one 64-bit row mask per tile row plus a summary) for idle lanes.
__device__ inline int upstream_walks(const WTile &Tl, const Layout &L, const uint32_t *cb,
                                     float *av, uint64_t roots, uint32_t *pend, uint32_t *summ)
{
    Dispenser ds;
    ds.init(roots);
    int r = -1, c = -1, visited = 0;
    float a = 0.0f;
    const int lane = lane_id();
    for (;;) {
        bool idle = r < 0;
        uint64_t sm = ((uint64_t)summ[1] << 32) | summ[0];
        if (!__any(!idle) && ds.empty() && sm == 0) break;
        int nr, nc;
        if (ds.take(idle, roots, nr, nc)) {
            r = nr;
            c = nc;
            a = av[L.ai(r, c)];
            ++visited;
            idle = false;
        }
        // queued donors, once the roots are handed out
        if (ds.empty()) {
            uint64_t free_lanes = __ballot(idle);
            bool got = false;
            while (free_lanes != 0 && sm != 0) {
                int R = __ffsll((unsigned long long)sm) - 1;
                uint64_t rb = ((uint64_t)pend[2 * R + 1] << 32) | pend[2 * R];
                int k = __popcll(free_lanes) < __popcll(rb) ? __popcll(free_lanes) : __popcll(rb);
                if (idle && !got) {
                    bool mine = (free_lanes >> lane) & 1ull;
                    int rank = __popcll(free_lanes & ((1ull << lane) - 1ull));
                    if (mine && rank < k) {
                        r = R;
                        c = nth_set_bit(rb, rank);
                        a = av[L.ai(r, c)];
                        got = true;
                    }
                }
                rb = clear_lowest(rb, k);
                free_lanes = clear_lowest(free_lanes, k);
                if (lane == 0) {
                    pend[2 * R] = (uint32_t)rb;
                    pend[2 * R + 1] = (uint32_t)(rb >> 32);
                }
                if (rb == 0) {
                    sm &= ~(1ull << R);
                    if (lane == 0) {
                        summ[0] = (uint32_t)sm;
                        summ[1] = (uint32_t)(sm >> 32);
                    }
                }
            }
        }
        if (r < 0) continue;
        uint32_t mask = cbyte(cb, L, r, c);
        if (mask == 0) {
            r = -1;
            continue;
        }
        int j0 = __ffs(mask) - 1;
        uint32_t rest = mask & (mask - 1u);
        while (rest) {
            int j = __ffs(rest) - 1;
            rest &= rest - 1u;
            // the donor in direction j sits at offset dir(j)
            int dr = r + dir_dr(j), dc = c + dir_dc(j);
            const int ai = L.ai(dr, dc);
            av[ai] += a;
            ++visited;
            atomicOr(&pend[2 * dr + (dc >> 5)], 1u << (dc & 31));
            atomicOr(&summ[dr >> 5], 1u << (dr & 31));
        }
        r += dir_dr(j0);
        c += dir_dc(j0);
        const int ai = L.ai(r, c);
        a += av[ai];
        av[ai] = a;
        ++visited;
    }
    return visited;
}

}  // namespace wk

// Adjoint, one wavefront per tile.
//   PASS 1: per perimeter cell, the link and the sum of g along its in-tile path
//   PASS 2: lambda for every cell, exits seeded with the resolved downstream sum
template <int PASS>
__global__ void __launch_bounds__(64)
adj_walk(const uint8_t *__restrict__ dirs, const float *__restrict__ gin, Geo g,
         uint16_t *__restrict__ link, float *__restrict__ S, const double *__restrict__ mu0,
         const double *__restrict__ mu1, const uint32_t *__restrict__ jstate,
         float *__restrict__ out, uint32_t *status)
{
    using namespace wk;
    extern __shared__ uint32_t lds[];
    const WTile Tl = wtile_of(g, blockIdx.x);
    const Layout L(g.tw);
    uint32_t *cb = lds;
    float *av = reinterpret_cast<float *>(lds + g.th * L.cbs);
    uint32_t *tail = lds + g.th * (L.cbs + L.as);
    const int r = lane_id();

    Setup St = setup_tile<PASS == 1 ? 1 : 2, PASS == 1>(dirs, g, Tl, L, cb, status);
    if (r < Tl.h) {
        const float *grow = gin + (Tl.r0 + r) * g.cols + Tl.c0;
        for (int c = 0; c < Tl.w; ++c) av[L.ai(r, c)] = grow[c];
    }

    if (PASS == 1) {
        uint16_t *ll = reinterpret_cast<uint16_t *>(tail);
        float *sl = reinterpret_cast<float *>(tail + (Tl.P + 1) / 2);
        for (int p = r; p < Tl.P; p += 64) {
            ll[p] = kLinkTerm;
            sl[p] = 0.0f;
        }
        __syncthreads();
        link_walks<true>(g, Tl, L, cb, av, St.entry, ll, sl, status);
        __syncthreads();
        for (int p = r; p < Tl.P; p += 64) {
            int qr, qc;
            ring_cell(p, Tl.h, Tl.w, qr, qc);
            uint32_t k = cbyte(cb, L, qr, qc) & 15u;
            uint16_t Lk;
            if (k >= (uint32_t)kNoData) Lk = kLinkNoData;
            else Lk = (link_for(g, Tl, qr, qc, qr, qc, k) == kLinkExt) ? kLinkExt : ll[p];
            link[Tl.base + p] = Lk;
            S[Tl.base + p] = sl[p];
        }
        return;
    }

    // pass 2: exits get the downstream sum mu of the cell they flow into
    const double *mu = jstate[0] == 1 ? mu1 : mu0;
    uint32_t *pend = tail;       // 2 words per row
    uint32_t *summ = tail + 128;  // 2 words
    for (int i = r; i < 130; i += 64) tail[i] = 0;
    for (int p = r; p < Tl.P; p += 64) {
        int qr, qc;
        ring_cell(p, Tl.h, Tl.w, qr, qc);
        uint32_t k = dirs[(Tl.r0 + qr) * g.cols + Tl.c0 + qc];
        if (k > (uint32_t)kNoData) continue;
        if (link_for(g, Tl, qr, qc, qr, qc, k) == kLinkExt) av[L.ai(qr, qc)] += (float)mu[Tl.base + p];
    }
    __syncthreads();
    int visited = upstream_walks(Tl, L, cb, av, St.root, pend, summ);
    if (wave_sum(visited) != wave_sum(St.valid) && r == 0) set_status(status, kStatusCycle);
    __syncthreads();
    if (r < Tl.h) {
        float *orow = out + (Tl.r0 + r) * g.cols + Tl.c0;
        const uint8_t *drow = dirs + (Tl.r0 + r) * g.cols + Tl.c0;
        for (int c = 0; c < Tl.w; ++c) {
            uint32_t k = drow[c];
            orow[c] = k < (uint32_t)kNoData ? av[L.ai(r, c)] : 0.0f;
        }
    }
}

// LDS bytes per tile for the walker kernels
__host__ inline size_t walk_lds_bytes(int th, int tw)
{
    wk::Layout L(tw);
    size_t base = ((size_t)th * L.cbs + (size_t)th * L.as) * 4;
    size_t tail = (size_t)ring_size(th, tw) * 6 + 8;  // links + sums (pass 1)
    size_t pend = 130 * 4;                              // pending bitmap (adjoint pass 2)
    return base + (tail > pend ? tail : pend) + 16;
}

}  // namespace d8
