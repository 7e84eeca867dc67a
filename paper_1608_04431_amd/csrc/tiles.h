// tiles.h -- per-tile kernels of libd8flow (one workgroup per tile, state in LDS).
//
// Both directions use pointer jumping with gathers only, so float results do
// not depend on thread timing:
//
//   fwd_tile  (Algorithm 1 for one tile): A(x) = seed(x) + sum of A over x's
//             in-tile donors.  Cells with exactly one in-tile donor form
//             chains; pointer jumping UP those chains gives every chain cell
//             its partial sum acc(x) up to the chain's top and the top itself.
//             Tops (cells with zero or several donors) are then finished in
//             dependency rounds, each gathering its donors' acc + A(top), and
//             every chain cell reads A(x) = acc(x) + A(top(x)).
//             Pass 1 also derives Algorithm 2's link of every perimeter cell
//             from the chain/top structure; pass 2 adds the resolved cross-tile
//             inflow to the seed of each receiving perimeter cell (EVICT).
//   adj_tile  lambda(x) = g(x) + lambda(receiver): pointer jumping DOWN the
//             in-tile flow paths; the path end (an exit or an outlet) is seeded
//             with the resolved downstream sum in pass 2.  Pass 1 returns, per
//             perimeter cell, the in-tile path sum and the link.
//
// Each thread keeps kCPT cells' state in registers; the LDS copy is what other
// threads read.  A round is: read phase, barrier, write phase, barrier.
#pragma once

#include "d8_common.h"

namespace d8 {

constexpr int kCPT = 8;                 // cells per thread (blockDim * kCPT >= tile cells)
constexpr uint32_t kPtrMask = 0x3FFFu;  // tile-local cell index (tiles <= 8192 cells)
constexpr uint32_t kTop = 1u << 14;     // forward: a cell without exactly one donor
constexpr uint32_t kDone = 1u << 15;    // jump finished / top value final
constexpr int kEndShift = 16;           // forward tops: (last cell of the chain) + 1

struct Tile {
    int ty, tx, h, w, n, P;
    int64_t r0, c0, base;
};

__device__ inline Tile tile_of(const Geo &g, int t)
{
    Tile T;
    T.ty = t / g.ntx;
    T.tx = t - T.ty * g.ntx;
    T.h = tile_h(g, T.ty);
    T.w = tile_w(g, T.tx);
    T.n = T.h * T.w;
    T.P = ring_size(T.h, T.w);
    T.r0 = (int64_t)T.ty * g.th;
    T.c0 = (int64_t)T.tx * g.tw;
    T.base = node_base(g, T.ty, T.tx);
    return T;
}

__device__ inline int64_t gidx(const Geo &g, const Tile &T, int i)
{
    int r = i / T.w;
    return (T.r0 + r) * g.cols + T.c0 + (i - r * T.w);
}

template <typename T> __device__ inline T from_bits(uint32_t b);
template <> __device__ inline float from_bits<float>(uint32_t b) { return __uint_as_float(b); }
template <> __device__ inline uint32_t from_bits<uint32_t>(uint32_t b) { return b; }
__device__ inline uint32_t to_bits(float v) { return __float_as_uint(v); }
__device__ inline uint32_t to_bits(uint32_t v) { return v; }

// Direction codes of the tile into LDS bytes; codes above 9 are reported and
// then treated as NoData so nothing indexes with them.
__device__ inline void load_codes8(const uint8_t *__restrict__ dirs, const Geo &g, const Tile &T,
                                   uint8_t *code, uint32_t *status)
{
    for (int i = threadIdx.x; i < T.n; i += blockDim.x) {
        uint32_t k = dirs[gidx(g, T, i)];
        if (k > kNoData) {
            set_status(status, kStatusDirCode);
            k = kNoData;
        }
        code[i] = (uint8_t)k;
    }
}

// In-tile receiver of cell i, or -1 (NoFlow / NoData, leaves the tile,
// receiver is NoData).
__device__ inline int rcv8(const uint8_t *code, const Tile &T, int i)
{
    int k = code[i];
    if (k >= kNoFlow) return -1;
    int r0 = i / T.w;
    int r = r0 + dir_dr(k), c = i - r0 * T.w + dir_dc(k);
    if (r < 0 || r >= T.h || c < 0 || c >= T.w) return -1;
    int j = r * T.w + c;
    return code[j] == kNoData ? -1 : j;
}

// Does cell i's direction leave the tile to a cell inside the raster?
__device__ inline bool exits_tile(const Geo &g, const Tile &T, const uint8_t *code, int i)
{
    int k = code[i];
    if (k >= kNoFlow) return false;
    int r0 = i / T.w;
    int r = r0 + dir_dr(k), c = i - r0 * T.w + dir_dc(k);
    if (r >= 0 && r < T.h && c >= 0 && c < T.w) return false;
    int64_t gr = T.r0 + r, gc = T.c0 + c;
    return gr >= 0 && gr < g.rows && gc >= 0 && gc < g.cols;
}

// Bit j set: the in-tile neighbour in direction j flows into cell i (its code
// is 7 - j).
__device__ inline uint32_t donor_mask8(const uint8_t *code, const Tile &T, int i)
{
    int r = i / T.w, c = i - r * T.w;
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        int rr = r + dir_dr(j), cc = c + dir_dc(j);
        if (rr < 0 || rr >= T.h || cc < 0 || cc >= T.w) continue;
        if (code[rr * T.w + cc] == 7 - j) m |= 1u << j;
    }
    return m;
}

__device__ inline int nbr(const Tile &T, int i, int j) { return i + dir_dr(j) * T.w + dir_dc(j); }

// Algorithm 2's link of perimeter cell q whose in-tile path ends at `term`.
__device__ inline uint16_t link_of(const Geo &g, const Tile &T, const uint8_t *code, int q, int term)
{
    if (code[q] == kNoData) return kLinkNoData;
    if (!exits_tile(g, T, code, term)) return kLinkTerm;
    if (term == q) return kLinkExt;
    return (uint16_t)ring_index(term / T.w, term % T.w, T.h, T.w);
}

// ceil(log2(n)) + 2: enough rounds for any acyclic tile; more means a cycle.
__device__ inline int jump_round_limit(int n)
{
    int r = 2;
    while ((1 << (r - 2)) < n) ++r;
    return r;
}

// ------------------------------------------------------------ forward ------
// T: tile arithmetic (uint32_t counts or float); V: resolve state per node
// (packed 64-bit sum:count for counts, double sums with `indeg` for floats);
// E: cross-tile inflow per node (uint32_t or double).
template <int PASS, typename T, typename V, typename E>
__global__ void __launch_bounds__(1024)
fwd_tile(const uint8_t *__restrict__ dirs, const float *__restrict__ w, Geo g,
         uint16_t *__restrict__ link, T *__restrict__ aloc, uint32_t *__restrict__ indeg,
         V *__restrict__ acc, E *__restrict__ ext, T *__restrict__ out, uint32_t *status)
{
    extern __shared__ uint2 lds2[];
    const Tile Tl = tile_of(g, blockIdx.x);
    const int n = Tl.n, B = blockDim.x, tid = threadIdx.x;
    uint2 *st = lds2;
    uint8_t *code = reinterpret_cast<uint8_t *>(lds2 + n);

    load_codes8(dirs, g, Tl, code, status);
    __syncthreads();

    // seeds, donor masks, initial pointers
    T a[kCPT];
    uint32_t y[kCPT];
    uint32_t masks[(kCPT + 3) / 4];
#pragma unroll
    for (int j = 0; j < (kCPT + 3) / 4; ++j) masks[j] = 0;
#pragma unroll
    for (int j = 0; j < kCPT; ++j) {
        int i = tid + j * B;
        a[j] = (T)0;
        y[j] = kTop | kDone;  // inert (outside the tile or NoData)
        if (i < n && code[i] != kNoData) {
            uint32_t m = donor_mask8(code, Tl, i);
            T s = w ? (T)w[gidx(g, Tl, i)] : (T)1;
            if (PASS == 2) {
                int r = i / Tl.w;
                int p = ring_index(r, i - r * Tl.w, Tl.h, Tl.w);
                if (p >= 0) s += (T)ext[Tl.base + p];
            }
            a[j] = s;
            int cnt = __popc(m);
            if (cnt == 1) y[j] = (uint32_t)nbr(Tl, i, __ffs(m) - 1);  // chain cell: points at its donor
            else y[j] = (uint32_t)i | kTop | (cnt == 0 ? kDone : 0u);  // source (final) / confluence
            masks[j >> 2] |= m << (8 * (j & 3));
        }
        if (i < n) st[i] = make_uint2(to_bits(a[j]), y[j]);
    }
    __syncthreads();

    // pointer jumping up the chains: acc(x) = sum of seeds from x up to, not
    // including, ptr(x); finished when ptr(x) is a top
    const int limit = jump_round_limit(n);
    for (int round = 0;; ++round) {
        if (round == limit) {
            if (tid == 0) set_status(status, kStatusCycle);
            break;
        }
        uint2 rd[kCPT];
        bool live = false;
#pragma unroll
        for (int j = 0; j < kCPT; ++j)
            if (!(y[j] & (kTop | kDone))) rd[j] = st[y[j] & kPtrMask];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            if (y[j] & (kTop | kDone)) continue;
            if (rd[j].y & kTop) {
                y[j] |= kDone;  // the pointer already names the top
            } else {
                a[j] += from_bits<T>(rd[j].x);
                y[j] = rd[j].y & (kPtrMask | kDone);
            }
            st[tid + j * B] = make_uint2(to_bits(a[j]), y[j]);
            live |= !(y[j] & kDone);
        }
        if (!__syncthreads_or(live)) break;
    }

    // each chain's last cell: its receiver is a confluence or there is none
#pragma unroll
    for (int j = 0; j < kCPT; ++j) {
        int i = tid + j * B;
        // unfinished chain cells exist only on a cycle (already reported)
        if (i >= n || code[i] == kNoData || (y[j] & (kTop | kDone)) == 0) continue;
        int r = rcv8(code, Tl, i);
        if (r >= 0 && !(st[r].y & kTop)) continue;
        int t = (y[j] & kTop) ? i : (int)(y[j] & kPtrMask);
        atomicOr(&st[t].y, (uint32_t)(i + 1) << kEndShift);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCPT; ++j)
        if ((y[j] & kTop) && tid + j * B < n) y[j] = st[tid + j * B].y;

    // tops in dependency rounds: a confluence finishes once every donor's
    // chain top is final; donors are summed in fixed neighbour order
    for (int round = 0;; ++round) {
        bool live = false, progress = false;
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            if ((y[j] & (kTop | kDone)) != kTop) continue;
            int i = tid + j * B;
            uint32_t m = (masks[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            T sum = a[j];
            bool ready = true;
            for (int k = 0; k < 8 && ready; ++k) {
                if (!(m & (1u << k))) continue;
                uint2 sd = st[nbr(Tl, i, k)];
                if (sd.y & kTop) {
                    if (!(sd.y & kDone)) ready = false;
                    else sum += from_bits<T>(sd.x);
                } else {
                    uint2 stt = st[sd.y & kPtrMask];
                    if ((stt.y & (kTop | kDone)) != (kTop | kDone) || !(sd.y & kDone)) ready = false;
                    else sum += from_bits<T>(sd.x) + from_bits<T>(stt.x);
                }
            }
            if (ready) {
                a[j] = sum;
                y[j] |= kDone;
                st[i] = make_uint2(to_bits(sum), y[j]);
                progress = true;
            } else {
                live = true;
            }
        }
        if (!__syncthreads_or(live)) break;
        if (!__syncthreads_or(progress)) {
            if (tid == 0) set_status(status, kStatusCycle);
            break;
        }
        (void)round;
    }

    // every chain cell: A = acc + A(top); tops already hold A
#pragma unroll
    for (int j = 0; j < kCPT; ++j) {
        int i = tid + j * B;
        if (i >= n || (y[j] & kTop)) continue;
        a[j] += from_bits<T>(st[y[j] & kPtrMask].x);
        if (PASS == 1) st[i].x = to_bits(a[j]);  // others read only tops here
    }

    if (PASS == 2) {
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            int i = tid + j * B;
            if (i < n) out[gidx(g, Tl, i)] = (code[i] == kNoData) ? (T)0 : a[j];
        }
        // an exit cell never reached by the resolve lies on a cycle of tiles
        for (int p = tid; p < Tl.P; p += B) {
            int64_t id = Tl.base + p;
            if (link[id] != kLinkExt) continue;
            bool pending = indeg ? indeg[id] != 0 : (uint32_t)acc[id] != 0;
            if (pending) set_status(status, kStatusCycle);
        }
        return;
    }

    __syncthreads();
    // perimeter records: A_loc and the link, found by following chain ends
    // and confluences down to the end of the in-tile path
    for (int p = tid; p < Tl.P; p += B) {
        int r, c;
        ring_cell(p, Tl.h, Tl.w, r, c);
        int q = r * Tl.w + c;
        int64_t id = Tl.base + p;
        uint16_t L = kLinkNoData;
        T A = (T)0;
        if (code[q] != kNoData) {
            uint2 sq = st[q];
            A = from_bits<T>(sq.x);
            int t = (sq.y & kTop) ? q : (int)(sq.y & kPtrMask);
            int term = q;
            for (int steps = 0; steps <= n; ++steps) {
                int e = (int)(st[t].y >> kEndShift) - 1;
                if (e < 0) break;  // only on a cycle
                int rr = rcv8(code, Tl, e);
                if (rr < 0) {
                    term = e;
                    break;
                }
                t = rr;
            }
            L = link_of(g, Tl, code, q, term);
        }
        link[id] = L;
        aloc[id] = A;
        if (indeg) indeg[id] = 0;
        acc[id] = (V)0;
        ext[id] = (E)0;
    }
}

// ------------------------------------------------------------ adjoint ------
template <int PASS>
__global__ void __launch_bounds__(1024)
adj_tile(const uint8_t *__restrict__ dirs, const float *__restrict__ gin, Geo g,
         uint16_t *__restrict__ link, float *__restrict__ S, const double *__restrict__ mu0,
         const double *__restrict__ mu1, const uint32_t *__restrict__ jstate,
         float *__restrict__ out, uint32_t *status)
{
    extern __shared__ uint2 lds2[];
    const Tile Tl = tile_of(g, blockIdx.x);
    const int n = Tl.n, B = blockDim.x, tid = threadIdx.x;
    uint2 *st = lds2;
    uint8_t *code = reinterpret_cast<uint8_t *>(lds2 + n);
    const double *mu = nullptr;
    if (PASS == 2) mu = jstate[0] == 1 ? mu1 : mu0;

    load_codes8(dirs, g, Tl, code, status);
    __syncthreads();

    // acc(x) = sum of g from x down to, not including, ptr(x); roots (no
    // in-tile receiver) are finished: g plus, for an exit, the downstream sum
    float a[kCPT];
    uint32_t y[kCPT];
#pragma unroll
    for (int j = 0; j < kCPT; ++j) {
        int i = tid + j * B;
        a[j] = 0.0f;
        y[j] = kDone;
        if (i >= n) continue;
        if (code[i] != kNoData) {
            a[j] = gin[gidx(g, Tl, i)];
            int r = rcv8(code, Tl, i);
            if (r >= 0) {
                y[j] = (uint32_t)r;
            } else {
                y[j] = (uint32_t)i | kDone;
                if (PASS == 2 && exits_tile(g, Tl, code, i)) {
                    int rr = i / Tl.w;
                    a[j] += (float)mu[Tl.base + ring_index(rr, i - rr * Tl.w, Tl.h, Tl.w)];
                }
            }
        } else {
            y[j] = (uint32_t)i | kDone;
        }
        st[i] = make_uint2(to_bits(a[j]), y[j]);
    }
    __syncthreads();

    const int limit = jump_round_limit(n);
    for (int round = 0;; ++round) {
        if (round == limit) {
            if (tid == 0) set_status(status, kStatusCycle);
            break;
        }
        uint2 rd[kCPT];
        bool live = false;
#pragma unroll
        for (int j = 0; j < kCPT; ++j)
            if (!(y[j] & kDone)) rd[j] = st[y[j] & kPtrMask];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            if (y[j] & kDone) continue;
            a[j] += __uint_as_float(rd[j].x);
            y[j] = rd[j].y & (kPtrMask | kDone);
            st[tid + j * B] = make_uint2(to_bits(a[j]), y[j]);
            live |= !(y[j] & kDone);
        }
        if (!__syncthreads_or(live)) break;
    }

    if (PASS == 2) {
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            int i = tid + j * B;
            if (i < n) out[gidx(g, Tl, i)] = (code[i] == kNoData) ? 0.0f : a[j];
        }
        return;
    }
    // pass 1: per perimeter cell, its in-tile path sum and link (ptr = path end)
    for (int p = tid; p < Tl.P; p += B) {
        int r, c;
        ring_cell(p, Tl.h, Tl.w, r, c);
        int q = r * Tl.w + c;
        uint2 sq = st[q];
        link[Tl.base + p] = link_of(g, Tl, code, q, (int)(sq.y & kPtrMask));
        S[Tl.base + p] = __uint_as_float(sq.x);
    }
}

}  // namespace d8
