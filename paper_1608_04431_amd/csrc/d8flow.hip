// d8flow.hip -- host side of libd8flow: argument checks, workspace layout,
// launch sequences of the C ABI declared in include/d8flow.h.
#include "d8flow.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"

using namespace d8;

namespace {

constexpr int kDefaultTile = 64;
// Absorption keeps alpha beside the values in LDS, so its tiles default to a
// smaller shape (more tiles resident per CU): 48 x 32, which also takes the
// kernels' narrowest register-row copy.
constexpr int kAbsorbTileRows = 48, kAbsorbTileCols = 32;
inline void absorb_default_tile(int &th, int &tw)
{
    if (th == 0 && tw == 0) {
        th = kAbsorbTileRows;
        tw = kAbsorbTileCols;
    }
}
constexpr int kNodeBlock = 256;

struct Layout {
    size_t status, jstate, link, entry, succ, indeg, val32, acc64, ext64, ptr2, root8, total;
    size_t off, kids, srt, bsum;  // the float forward's children lists, where root8 lies (adjoint only)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Children lists of the float forward's resolve, placed over an area the
// forward does not otherwise use (the adjoint's root labels): offsets,
// children as filled and children in order (a word per node each), and one
// word per 4096 nodes for the scan.  Returns the end of the lists.
size_t csr_place(size_t at, size_t N, size_t &off, size_t &kids, size_t &srt, size_t &bsum)
{
    off = at;
    kids = align256(off + N * sizeof(uint32_t));
    srt = align256(kids + N * sizeof(uint32_t));
    bsum = align256(srt + N * sizeof(uint32_t));
    return align256(bsum + (N / (size_t)kCompactNodes + 2) * sizeof(uint32_t));
}

Layout layout_for(const Geo &g)
{
    size_t N = (size_t)g.nnodes;
    Layout L;
    size_t off = 0;
    L.status = off; off += 256;
    L.jstate = off; off += 256;
    L.link = off;   off = align256(off + N * sizeof(uint16_t));
    L.entry = off;  off = align256(off + N * sizeof(uint32_t));
    L.succ = off;   off = align256(off + N * sizeof(uint32_t));
    L.indeg = off;  off = align256(off + N * sizeof(uint32_t));
    L.ptr2 = off;   off = align256(off + N * sizeof(uint32_t));
    L.val32 = off;  off = align256(off + N * sizeof(uint32_t));
    L.acc64 = off;  off = align256(off + N * sizeof(double));
    L.ext64 = off;  off = align256(off + N * sizeof(double));
    L.root8 = off;  off = align256(off + (size_t)g.rows * (size_t)g.cols);  // adjoint root labels
    L.total = std::max(off, csr_place(L.root8, N, L.off, L.kids, L.srt, L.bsum));
    return L;
}

// Shared argument checks.  Returns D8_OK and fills g (and *empty for a raster
// with no cells), or a negative code.
int check_common(int64_t rows, int64_t cols, int &th, int &tw, Geo &g, bool &empty)
{
    if (rows < 0 || cols < 0 || rows > INT_MAX || cols > INT_MAX) return D8_EINVAL;
    if (th == 0 && tw == 0) th = tw = kDefaultTile;
    if (th < 1 || tw < 1) return D8_EINVAL;
    empty = (rows == 0 || cols == 0);
    if (empty) return D8_OK;
    // a tile larger than the raster is the raster
    if (th > rows) th = (int)rows;
    if (tw > cols) tw = (int)cols;
    if (th > D8_MAX_TILE_SIDE || tw > D8_MAX_TILE_SIDE) return D8_EINVAL;
    g = make_geo(rows, cols, th, tw);
    if (g.nnodes >= (int64_t)kJumpDone || (int64_t)g.nty * g.ntx > INT_MAX) return D8_EINVAL;
    return D8_OK;
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---- optional per-kernel timing: HIP events around each launch, on the
// launch stream, summed per kernel name by d8_timing_report().
struct TimedLaunch {
    const char *name;
    hipEvent_t start, stop;
};
std::mutex g_timing_mu;
int g_timing_on = 0;  // 0 off, 1 every launch, 2 the per-tile passes only
std::vector<TimedLaunch> g_timed;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pooled_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// set while this thread records a graph: no timing events go into it
thread_local bool g_capturing = false;

struct LaunchTimer {
    const char *name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    LaunchTimer(const char *n, hipStream_t s) : name(n), st(s)
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        if (g_timing_on != 0 && !g_capturing && (g_timing_on == 1 || std::strstr(n, "pass") != nullptr)) {
            a = pooled_event();
            (void)hipEventRecord(a, st);
        }
    }
    ~LaunchTimer()
    {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_timing_mu);
        hipEvent_t b = pooled_event();
        (void)hipEventRecord(b, st);
        g_timed.push_back({name, a, b});
    }
};

// The first launch error of a call is kept (kernel name and HIP message) for
// d8_last_error_message().
thread_local std::string g_last_error;
thread_local int g_launch_rc = D8_OK;

#define D8_LAUNCH(name, st, ...)                                                     \
    do {                                                                             \
        LaunchTimer timer_(name, st);                                                \
        __VA_ARGS__;                                                                 \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess && g_launch_rc == D8_OK) {                              \
            g_launch_rc = D8_EHIP;                                                   \
            g_last_error = std::string(name) + ": " + hipGetErrorString(e_);         \
        }                                                                            \
    } while (0)


inline unsigned blocks_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Downstream sums over the exit forest: dense numbering of the exits (count,
// scan, map), initial words, then ceil(log3 N) + 1 pointer-jumping rounds and
// the convergence check.  bsum takes one word per 4096 nodes, cmap one per
// node; the sums end in jw[jstate[0]] at the exits' dense numbers.  Returns
// the number of rounds.
// Dense numbers of the exits among the N perimeter nodes: cmap (node ->
// number), inv (number -> node), *nexit.
void compact_exits(hipStream_t st, int64_t N, const uint16_t *link, uint32_t *bsum, uint32_t *cmap,
                   uint32_t *inv, uint32_t *nexit, bool batch)
{
#define CNAME (batch ? "batch_adj_compact" : "adj_compact")
    const int64_t ncb = (N + kCompactNodes - 1) / kCompactNodes;
    D8_LAUNCH(CNAME, st, (adj_compact_count<<<(unsigned)ncb, kCompactBlock, 0, st>>>(N, link, bsum)));
    D8_LAUNCH(CNAME, st, (adj_compact_scan<<<1, 1024, 0, st>>>(ncb, bsum, nexit)));
    D8_LAUNCH(CNAME, st,
              (adj_compact_map<<<(unsigned)ncb, kCompactBlock, 0, st>>>(N, link, bsum, cmap, inv)));
#undef CNAME
}

int jump_exits(hipStream_t st, int64_t N, const JumpGraph &G, const uint16_t *link, const float *S,
               uint32_t *bsum, uint32_t *cmap, unsigned long long *const jw[2], uint32_t *jstate,
               uint32_t *status, bool batch)
{
    // timing labels are kept by pointer: literals only
#define JNAME(s) (batch ? "batch_" s : s)
    uint32_t *nexit = jstate + 4;
    // inv (dense index -> node) lives in jw[1] until round 0 overwrites it
    uint32_t *inv = reinterpret_cast<uint32_t *>(jw[1]);
    compact_exits(st, N, link, bsum, cmap, inv, nexit, batch);
    const unsigned jb = std::min<unsigned>(blocks_for(N, 2 * kNodeBlock), 4096u);
    D8_LAUNCH(JNAME("adj_jump_init"), st,
              (adj_jump_init<<<jb, kNodeBlock, 0, st>>>(nexit, inv, G, link, S, cmap, jw[0])));
    // each round triples the path a word covers: ceil(log3 N) + 1 rounds
    // leave every chain of an acyclic forest complete
    int rounds = 1;
    for (int64_t span = 1; span <= N; span *= 3) ++rounds;
    for (int r = 0; r < rounds; ++r)
        D8_LAUNCH(JNAME("adj_jump_round"), st,
                  (adj_jump_round<<<jb, kNodeBlock, 0, st>>>(nexit, jw[r & 1], jw[(r + 1) & 1], jstate, r)));
    D8_LAUNCH(JNAME("adj_jump_finish"), st,
              (adj_jump_finish<<<1, 1, 0, st>>>(jstate, rounds, status)));
#undef JNAME
    return rounds;
}

// one wavefront per tile
constexpr int kTileThreads = 64;

__global__ void init_state(uint32_t *status, uint32_t *jstate)
{
    status[0] = kStatusOk;
    jstate[0] = kNone;  // final buffer of the pointer jumping, not yet known
    jstate[1] = 0;      // live flags of rounds r % 3 (round 0 reads slot 2)
    jstate[2] = 0;
    jstate[3] = 1;
}

// Start of a C-ABI call: forget earlier launch errors.
void begin_call()
{
    (void)hipGetLastError();
    g_launch_rc = D8_OK;
    g_last_error.clear();
}

int last_error()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && g_launch_rc == D8_OK) {
        g_launch_rc = D8_EHIP;
        g_last_error = hipGetErrorString(e);
    }
    return g_launch_rc;
}

// The tile kernels compiled for the narrowest register rows that hold the
// tile width (walk.h is compiled for rows of 64, 44 and 32 columns).
inline int row_width(int tw) { return tw <= 32 ? 32 : (tw <= 44 ? 44 : 64); }

template <int PASS, typename T, typename V, typename E>
decltype(&w64::fwd_walk<PASS, T, V, E>) fwd_walk_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::fwd_walk<PASS, T, V, E>;
    case 44: return &w44::fwd_walk<PASS, T, V, E>;
    default: return &w64::fwd_walk<PASS, T, V, E>;
    }
}

template <int PASS>
decltype(&w64::fwd_walk_absorb<PASS>) fwd_walk_absorb_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::fwd_walk_absorb<PASS>;
    case 44: return &w44::fwd_walk_absorb<PASS>;
    default: return &w64::fwd_walk_absorb<PASS>;
    }
}

decltype(&w64::adj_walk_absorb) adj_walk_absorb_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::adj_walk_absorb;
    case 44: return &w44::adj_walk_absorb;
    default: return &w64::adj_walk_absorb;
    }
}

decltype(&w64::adj_walk) adj_walk_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::adj_walk;
    case 44: return &w44::adj_walk;
    default: return &w64::adj_walk;
    }
}

decltype(&w64::adj_walk_band) adj_walk_band_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::adj_walk_band;
    case 44: return &w44::adj_walk_band;
    default: return &w64::adj_walk_band;
    }
}

template <int PASS>
decltype(&w64::fwd_walk_batch<PASS>) fwd_walk_batch_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::fwd_walk_batch<PASS>;
    case 44: return &w44::fwd_walk_batch<PASS>;
    default: return &w64::fwd_walk_batch<PASS>;
    }
}

decltype(&w64::adj_walk_batch) adj_walk_batch_k(int tw)
{
    switch (row_width(tw)) {
    case 32: return &w32::adj_walk_batch;
    case 44: return &w44::adj_walk_batch;
    default: return &w64::adj_walk_batch;
    }
}

// Dynamic LDS above the default 64 KiB must be allowed per kernel.
template <typename K>
int allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return D8_OK;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        g_launch_rc = D8_EHIP;
        g_last_error = std::string("hipFuncSetAttribute(LDS): ") + hipGetErrorString(e);
        (void)hipGetLastError();
        return D8_EHIP;
    }
    return D8_OK;
}

// The float resolve in a fixed order (kernels.h): children lists, walkers
// from the leaves, the cycle check.  V ends in vn (one double per node);
// ext is gathered afterwards by the caller (it needs the rasters' geometry).
// The timing labels are literals: the batch's carry their own.
template <bool ABS>
void resolve_float(hipStream_t st, bool batch, int64_t N, const uint16_t *link, const float *aloc,
                   const uint32_t *succ, const uint32_t *indeg, uint32_t *cnt, char *ws, size_t off_at,
                   size_t kids_at, size_t srt_at, size_t bsum_at, uint32_t *total, double *vn, uint32_t *status,
                   const uint32_t *entry = nullptr, const float *anode = nullptr, const float *pathp = nullptr,
                   double *coef = nullptr)
{
    uint32_t *off = reinterpret_cast<uint32_t *>(ws + off_at);
    uint32_t *kids = reinterpret_cast<uint32_t *>(ws + kids_at);
    uint32_t *srt = reinterpret_cast<uint32_t *>(ws + srt_at);
    uint32_t *bsum = reinterpret_cast<uint32_t *>(ws + bsum_at);
    const unsigned nb = blocks_for(N, kNodeBlock);
    const int64_t ncb = (N + kCompactNodes - 1) / kCompactNodes;
    unsigned long long *vw = reinterpret_cast<unsigned long long *>(vn);
    D8_LAUNCH(batch ? "batch_resolve_lists" : "resolve_lists_count", st,
              (csr_count<<<(unsigned)ncb, kCompactBlock, 0, st>>>(N, indeg, bsum)));
    D8_LAUNCH(batch ? "batch_resolve_lists" : "resolve_lists_scan", st,
              (adj_compact_scan<<<1, 1024, 0, st>>>(ncb, bsum, total)));
    D8_LAUNCH(batch ? "batch_resolve_lists" : "resolve_lists_offsets", st,
              (csr_offsets<<<(unsigned)ncb, kCompactBlock, 0, st>>>(N, indeg, bsum, off, cnt)));
    D8_LAUNCH(batch ? "batch_resolve_lists" : "resolve_lists_fill", st,
              (csr_fill<ABS><<<nb, kNodeBlock, 0, st>>>(N, link, succ, indeg, off, cnt, kids, entry, anode, pathp,
                                                        coef)));
    D8_LAUNCH(batch ? "batch_resolve_lists" : "resolve_lists_rank", st,
              (csr_rank<<<nb, kNodeBlock, 0, st>>>(N, link, succ, indeg, off, kids, srt)));
    D8_LAUNCH(batch ? "batch_resolve_fwd" : "resolve_fwd", st,
              (resolve_fwd_det<float, ABS><<<nb, kNodeBlock, 0, st>>>(N, link, aloc, succ, indeg, off, srt, cnt,
                                                                      vw, coef)));
}

// Unit counts (T = uint32_t): packed 64-bit resolve state, uint32 inflows.
// Float weights (T = float): double resolve sums with separate counts.
template <typename T>
int run_forward(const uint8_t *dirs, const float *w, T *out, const Geo &g, char *ws,
                const Layout &L, hipStream_t st)
{
    constexpr bool kCounts = std::is_same<T, uint32_t>::value;
    using V = typename std::conditional<kCounts, unsigned long long, double>::type;
    using E = typename std::conditional<kCounts, uint32_t, double>::type;
    uint32_t *status = reinterpret_cast<uint32_t *>(ws + L.status);
    uint32_t *jstate = reinterpret_cast<uint32_t *>(ws + L.jstate);
    uint16_t *link = reinterpret_cast<uint16_t *>(ws + L.link);
    uint32_t *entry = reinterpret_cast<uint32_t *>(ws + L.entry);
    uint32_t *succ = reinterpret_cast<uint32_t *>(ws + L.succ);
    uint32_t *indeg = reinterpret_cast<uint32_t *>(ws + L.indeg);
    // float weights: arrival counts; unit counts: donors of each entered node
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + L.ptr2);
    T *aloc = reinterpret_cast<T *>(ws + L.val32);
    V *acc = reinterpret_cast<V *>(ws + L.acc64);
    E *ext = reinterpret_cast<E *>(ws + L.ext64);

    int ntiles = g.nty * g.ntx;
    const int thr = kTileThreads;
    size_t lds1 = walk_lds_bytes(g.th, g.tw, kWalkFwd1, (int)sizeof(FwdLds<1, T>));
    size_t lds2 = walk_lds_bytes(g.th, g.tw, kWalkFwd2, (int)sizeof(FwdLds<2, T>));
    const auto pass1 = fwd_walk_k<1, T, V, E>(g.tw), pass2 = fwd_walk_k<2, T, V, E>(g.tw);
    if (allow_lds(pass1, lds1) || allow_lds(pass2, lds2)) return D8_EHIP;

    init_state<<<1, 1, 0, st>>>(status, jstate);
    unsigned nb = blocks_for(g.nnodes, kNodeBlock);
    D8_LAUNCH("fwd_pass1", st,
              (pass1<<<ntiles, thr, lds1, st>>>(dirs, w, g, link, aloc, indeg, cnt,
                                                               acc, ext, nullptr, status, 0)));
    D8_LAUNCH("graph_build", st,
              (graph_build<<<nb, kNodeBlock, 0, st>>>(dirs, g, link, entry, succ, indeg, 0, g.nnodes)));
    if constexpr (kCounts) {
        D8_LAUNCH("resolve_fwd", st,
                  (resolve_fwd_u32<<<nb, kNodeBlock, 0, st>>>(g.nnodes, link, aloc, entry, succ, indeg, acc,
                                                              ext)));
    } else {
        resolve_float<false>(st, false, g.nnodes, link, aloc, succ, indeg, cnt, ws, L.off, L.kids, L.srt, L.bsum,
                             jstate + 8, acc, status);
        D8_LAUNCH("resolve_ext", st,
                  (resolve_ext<false><<<nb, kNodeBlock, 0, st>>>(dirs, g, link, acc, ext, nullptr, 0, g.nnodes)));
    }
    D8_LAUNCH("fwd_pass2", st,
              (pass2<<<ntiles, thr, lds2, st>>>(dirs, w, g, link, aloc, indeg, cnt,
                                                               acc, ext, out, status, 0)));
    return last_error();
}


// Forward with absorption (float weights): the float path with each cell's
// alpha in the tile passes and per-node coefficients in the resolve.  The
// workspace is the one-raster layout plus anode and pathp (a float per node).
// Absorption's areas after the common layout: per perimeter node its alpha
// (anode, forward) and its path product (pathp: an entry's product in the
// forward pass, every node's P in the adjoint); the adjoint's second buffer
// of 16-byte exit words (the first takes acc64 and ext64, which are
// contiguous and at least 16 bytes per node) and P per cell.
struct AbsorbLayout {
    size_t anode, pathp, jw, pcell, total;
};

AbsorbLayout absorb_layout(const Layout &L, const Geo &g)
{
    const size_t N = (size_t)g.nnodes;
    AbsorbLayout A;
    A.anode = align256(L.total);
    A.pathp = align256(A.anode + N * sizeof(float));
    A.jw = align256(A.pathp + N * sizeof(float));
    A.pcell = align256(A.jw + N * sizeof(uint4));
    A.total = align256(A.pcell + (size_t)g.rows * (size_t)g.cols * sizeof(float));
    return A;
}

int run_forward_absorb(const uint8_t *dirs, const float *w, const float *alpha, float *out, const Geo &g,
                       char *ws, const Layout &L, hipStream_t st)
{
    const AbsorbLayout A = absorb_layout(L, g);
    uint32_t *status = reinterpret_cast<uint32_t *>(ws + L.status);
    uint32_t *jstate = reinterpret_cast<uint32_t *>(ws + L.jstate);
    uint16_t *link = reinterpret_cast<uint16_t *>(ws + L.link);
    uint32_t *entry = reinterpret_cast<uint32_t *>(ws + L.entry);
    uint32_t *succ = reinterpret_cast<uint32_t *>(ws + L.succ);
    uint32_t *indeg = reinterpret_cast<uint32_t *>(ws + L.indeg);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + L.ptr2);
    float *aloc = reinterpret_cast<float *>(ws + L.val32);
    double *acc = reinterpret_cast<double *>(ws + L.acc64);
    double *ext = reinterpret_cast<double *>(ws + L.ext64);
    float *anode = reinterpret_cast<float *>(ws + A.anode);
    float *pathp = reinterpret_cast<float *>(ws + A.pathp);
    const int ntiles = g.nty * g.ntx;
    const size_t lds1 = walk_lds_bytes(g.th, g.tw, kWalkFwd1, 4, true);
    const size_t lds2 = walk_lds_bytes(g.th, g.tw, kWalkFwd2, 4, true);
    const auto pass1 = fwd_walk_absorb_k<1>(g.tw), pass2 = fwd_walk_absorb_k<2>(g.tw);
    if (allow_lds(pass1, lds1) || allow_lds(pass2, lds2)) return D8_EHIP;
    const unsigned nb = blocks_for(g.nnodes, kNodeBlock);
    init_state<<<1, 1, 0, st>>>(status, jstate);
    D8_LAUNCH("absorb_pass1", st,
              (pass1<<<ntiles, kTileThreads, lds1, st>>>(dirs, w, alpha, g, link, aloc, indeg, cnt, acc, ext,
                                                         nullptr, status, anode, pathp)));
    D8_LAUNCH("graph_build", st,
              (graph_build<<<nb, kNodeBlock, 0, st>>>(dirs, g, link, entry, succ, indeg, 0, g.nnodes)));
    // the per-exit coefficients take the adjoint's second word buffer
    resolve_float<true>(st, false, g.nnodes, link, aloc, succ, indeg, cnt, ws, L.off, L.kids, L.srt, L.bsum,
                        jstate + 8, acc, status, entry, anode, pathp,
                        reinterpret_cast<double *>(ws + A.jw));
    D8_LAUNCH("resolve_ext", st,
              (resolve_ext<true><<<nb, kNodeBlock, 0, st>>>(dirs, g, link, acc, ext, anode, 0, g.nnodes)));
    D8_LAUNCH("absorb_pass2", st,
              (pass2<<<ntiles, kTileThreads, lds2, st>>>(dirs, w, alpha, g, link, aloc, indeg, cnt, acc, ext,
                                                         out, status, anode, pathp)));
    return last_error();
}

// ------------------------------------------------------------------ batch --
// A batch plan: rasters with cells, sorted by decreasing cell count (the
// tile work queue hands out the largest rasters' tiles first), their
// descriptors, the raster of every batch tile, and the raster where every
// chunk of 2^kChunkShift nodes starts.
struct BatchLayout {
    size_t status, jstate, desc, tile_dem, chunk_dem;
    size_t link, entry, succ, indeg, cnt, val32, acc64, ext64, root8, total;
    size_t off, kids, srt, bsum;  // the forward's children lists, over the root labels
};

// Rasters of one tile shape: a contiguous range of the batch's tiles, run by
// one launch per stage (a wavefront per tile) with that shape's LDS size.
struct TileGroup {
    int th, tw;
    int64_t t_begin, t_end;
    size_t lds[3];  // fwd pass 1, fwd pass 2, adj pass 1
    int maxw;       // widest tile of the group (selects the kernels' register rows)
};
constexpr int kMaxGroups = 16;  // distinct tile shapes in one batch

struct BatchPlan {
    std::vector<DemDesc> dems;
    std::vector<int64_t> cell0;  // each raster's first cell in the root-label array
    std::vector<uint32_t> tile_dem, chunk_dem;
    std::vector<TileGroup> groups;
    int64_t ntiles = 0, nnodes = 0, ncells = 0;
    BatchLayout L{};
};

int make_plan(const d8_batch_item *items, int n, BatchPlan &P)
{
    if (n < 0 || (n > 0 && !items)) return D8_EINVAL;
    struct Entry { int i; Geo g; };
    std::vector<Entry> order;
    for (int i = 0; i < n; ++i) {
        const d8_batch_item &it = items[i];
        if (it.rows < 0 || it.cols < 0) return D8_EINVAL;
        if (it.rows == 0 || it.cols == 0) continue;
        int th = it.tile_rows, tw = it.tile_cols;
        Geo g;
        bool empty = false;
        int rc = check_common(it.rows, it.cols, th, tw, g, empty);
        if (rc != D8_OK) return rc;
        order.push_back({i, g});
    }
    // group by the requested tile shape (LDS size of a launch), largest
    // rasters first within a group
    std::stable_sort(order.begin(), order.end(), [&](const Entry &a, const Entry &b) {
        const d8_batch_item &x = items[a.i], &y = items[b.i];
        if (x.tile_rows != y.tile_rows) return x.tile_rows > y.tile_rows;
        if (x.tile_cols != y.tile_cols) return x.tile_cols > y.tile_cols;
        return x.rows * x.cols > y.rows * y.cols;
    });
    for (const Entry &e : order) {
        const d8_batch_item &it = items[e.i];
        const Geo &g = e.g;
        DemDesc D;
        D.g = g;
        D.node0 = P.nnodes;
        D.tile0 = P.ntiles;
        D.dirs = it.dirs;
        D.w = it.weights;
        D.acc = it.acc;
        D.gacc = it.grad_acc;
        D.gw = it.grad_weights;
        if (!D.dirs) return D8_EINVAL;
        const int64_t nt = (int64_t)g.nty * g.ntx;
        const int key_th = it.tile_rows, key_tw = it.tile_cols;
        if (P.groups.empty() || P.groups.back().th != key_th || P.groups.back().tw != key_tw) {
            if ((int)P.groups.size() == kMaxGroups) return D8_EINVAL;
            P.groups.push_back({key_th, key_tw, P.ntiles, P.ntiles, {0, 0, 0}, 0});
        }
        TileGroup &G = P.groups.back();
        for (int64_t t = 0; t < nt; ++t) P.tile_dem.push_back((uint32_t)P.dems.size());
        D.root8 = nullptr;  // set when the workspace is known
        P.dems.push_back(D);
        P.cell0.push_back(P.ncells);
        P.ncells += g.rows * g.cols;
        P.ntiles += nt;
        P.nnodes += g.nnodes;
        G.t_end = P.ntiles;
        if (P.nnodes >= (int64_t)kJumpDone || P.ntiles >= (int64_t)INT_MAX) return D8_EINVAL;
        G.maxw = std::max(G.maxw, g.tw);
        G.lds[0] = std::max(G.lds[0], walk_lds_bytes(g.th, g.tw, kWalkFwd1, 4));
        G.lds[1] = std::max(G.lds[1], walk_lds_bytes(g.th, g.tw, kWalkFwd2, 4));
        G.lds[2] = std::max(G.lds[2], walk_lds_bytes(g.th, g.tw, kWalkAdj1, 4));
    }
    const int64_t nchunk = (P.nnodes >> kChunkShift) + 1;
    P.chunk_dem.assign((size_t)nchunk, 0);
    size_t d = 0;
    for (int64_t k = 0; k < nchunk; ++k) {
        const int64_t first = k << kChunkShift;
        while (d + 1 < P.dems.size() && P.dems[d + 1].node0 <= first) ++d;
        P.chunk_dem[(size_t)k] = (uint32_t)d;
    }
    const size_t N = (size_t)P.nnodes;
    BatchLayout &L = P.L;
    size_t off = 0;
    L.status = off; off += 256;
    L.jstate = off; off += 256;
    L.desc = off;      off = align256(off + P.dems.size() * sizeof(DemDesc));
    L.tile_dem = off;  off = align256(off + P.tile_dem.size() * sizeof(uint32_t));
    L.chunk_dem = off; off = align256(off + P.chunk_dem.size() * sizeof(uint32_t));
    L.link = off;  off = align256(off + N * sizeof(uint16_t));
    L.entry = off; off = align256(off + N * sizeof(uint32_t));
    L.succ = off;  off = align256(off + N * sizeof(uint32_t));
    L.indeg = off; off = align256(off + N * sizeof(uint32_t));
    L.cnt = off;   off = align256(off + N * sizeof(uint32_t));
    L.val32 = off; off = align256(off + N * sizeof(float));
    L.acc64 = off; off = align256(off + N * sizeof(double));
    L.ext64 = off; off = align256(off + N * sizeof(double));
    L.root8 = off; off = align256(off + (size_t)P.ncells);
    L.total = std::max(off, csr_place(L.root8, N, L.off, L.kids, L.srt, L.bsum));
    return D8_OK;
}

__global__ void init_batch(uint32_t *status, uint32_t *jstate)
{
    status[0] = kStatusOk;
    jstate[0] = kNone;
    jstate[1] = 0;
    jstate[2] = 0;
    jstate[3] = 1;
}

__global__ void reset_jump(uint32_t *jstate)
{
    jstate[0] = kNone;
    jstate[1] = 0;
    jstate[2] = 0;
    jstate[3] = 1;
}

// Descriptor tables into the workspace without waiting for the stream: the
// tables are packed into a pinned host buffer of the library's own and copied
// from there, stream-ordered before the kernels that read them.  A small ring
// of such buffers is reused; before a buffer is refilled the host waits for
// the event recorded after its last copy (only the copy, which ran at the
// start of that earlier call's work).
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
constexpr int kStagingRing = 4;
std::mutex g_staging_mu;
Staging g_staging[kStagingRing];
int g_staging_next = 0;

int upload_plan(const BatchPlan &P, char *ws, hipStream_t st, bool wait = false)
{
    const BatchLayout &L = P.L;
    if (P.dems.empty()) return D8_OK;
    std::vector<DemDesc> dems = P.dems;
    for (size_t i = 0; i < dems.size(); ++i)
        dems[i].root8 = reinterpret_cast<uint8_t *>(ws + L.root8) + P.cell0[i];
    const size_t b0 = dems.size() * sizeof(DemDesc);
    const size_t b1 = P.tile_dem.size() * sizeof(uint32_t);
    const size_t b2 = P.chunk_dem.size() * sizeof(uint32_t);
    const size_t need = b0 + b1 + b2;
    std::lock_guard<std::mutex> lk(g_staging_mu);
    Staging &S = g_staging[g_staging_next];
    g_staging_next = (g_staging_next + 1) % kStagingRing;
    if (S.done && hipEventSynchronize(S.done) != hipSuccess) return D8_EHIP;
    if (!S.done && hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess) return D8_EHIP;
    if (S.cap < need) {
        if (S.host) (void)hipHostFree(S.host);
        S.host = nullptr;
        S.cap = 0;
        if (hipHostMalloc(&S.host, need, hipHostMallocDefault) != hipSuccess) return D8_EHIP;
        S.cap = need;
    }
    char *h = reinterpret_cast<char *>(S.host);
    std::memcpy(h, dems.data(), b0);
    std::memcpy(h + b0, P.tile_dem.data(), b1);
    std::memcpy(h + b0 + b1, P.chunk_dem.data(), b2);
    if (hipMemcpyAsync(ws + L.desc, h, b0, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(ws + L.tile_dem, h + b0, b1, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(ws + L.chunk_dem, h + b0 + b1, b2, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(S.done, st) != hipSuccess)
        return D8_EHIP;
    if (wait && hipEventSynchronize(S.done) != hipSuccess) return D8_EHIP;
    return D8_OK;
}

int enqueue_batch(const BatchPlan &P, int mode, char *ws, hipStream_t st)
{
    const BatchLayout &L = P.L;
    uint32_t *status = reinterpret_cast<uint32_t *>(ws + L.status);
    uint32_t *jstate = reinterpret_cast<uint32_t *>(ws + L.jstate);
    const DemDesc *dems = reinterpret_cast<const DemDesc *>(ws + L.desc);
    const uint32_t *tile_dem = reinterpret_cast<const uint32_t *>(ws + L.tile_dem);
    const uint32_t *chunk_dem = reinterpret_cast<const uint32_t *>(ws + L.chunk_dem);
    uint16_t *link = reinterpret_cast<uint16_t *>(ws + L.link);
    uint32_t *entry = reinterpret_cast<uint32_t *>(ws + L.entry);
    uint32_t *succ = reinterpret_cast<uint32_t *>(ws + L.succ);
    uint32_t *indeg = reinterpret_cast<uint32_t *>(ws + L.indeg);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
    float *val32 = reinterpret_cast<float *>(ws + L.val32);
    double *acc = reinterpret_cast<double *>(ws + L.acc64);
    double *ext = reinterpret_cast<double *>(ws + L.ext64);
    unsigned long long *jw[2] = {reinterpret_cast<unsigned long long *>(ws + L.acc64),
                                 reinterpret_cast<unsigned long long *>(ws + L.ext64)};
    const int ndem = (int)P.dems.size();
    const int64_t N = P.nnodes;
    const unsigned nb = blocks_for(N, kNodeBlock);

    init_batch<<<1, 1, 0, st>>>(status, jstate);
    if (ndem == 0) return last_error();
    // one launch per tile group and stage, a wavefront per tile of the group
    auto tiles = [&](int stage, auto select, const char *name, auto &&...args) -> int {
        for (size_t k = 0; k < P.groups.size(); ++k) {
            const TileGroup &G = P.groups[k];
            const size_t lds = G.lds[stage];
            const auto kernel = select(G.maxw);
            if (allow_lds(kernel, lds)) return D8_EHIP;
            D8_LAUNCH(name, st,
                      (kernel<<<(unsigned)(G.t_end - G.t_begin), 64, lds, st>>>(
                          dems, tile_dem, (uint32_t)G.t_begin, (uint32_t)G.t_end, args...)));
        }
        return D8_OK;
    };
    if (mode & D8_BATCH_FWD) {
        if (tiles(0, fwd_walk_batch_k<1>, "batch_fwd_pass1", link, val32, indeg, cnt, acc, ext, status))
            return D8_EHIP;
        D8_LAUNCH("batch_graph_build", st,
                  (graph_build_batch<<<nb, kNodeBlock, 0, st>>>(dems, ndem, chunk_dem, N, link, entry,
                                                                succ, indeg)));
        resolve_float<false>(st, true, N, link, val32, succ, indeg, cnt, ws, L.off, L.kids, L.srt, L.bsum,
                             jstate + 8, acc, status);
        D8_LAUNCH("batch_resolve_ext", st,
                  (resolve_ext_batch<<<nb, kNodeBlock, 0, st>>>(dems, ndem, chunk_dem, N, link, acc, ext)));
        if (tiles(1, fwd_walk_batch_k<2>, "batch_fwd_pass2", link, val32, indeg, cnt, acc, ext, status))
            return D8_EHIP;
    }
    if (mode & D8_BATCH_ADJ) {
        reset_jump<<<1, 1, 0, st>>>(jstate);
        if (tiles(2, adj_walk_batch_k, "batch_adj_pass1", link, val32, status)) return D8_EHIP;
        // the exits' edges are found as their jump words are initialised
        const JumpGraph G{nullptr, Geo{}, dems, ndem, chunk_dem};
        jump_exits(st, N, G, link, val32, indeg, cnt, jw, jstate, status, true);
        D8_LAUNCH("batch_adj_pass2", st,
                  (adj_finish_batch<<<(unsigned)P.ntiles, 64, 0, st>>>(dems, tile_dem, (uint32_t)P.ntiles,
                                                                      cnt, jw[0], jw[1], jstate)));
    }
    return last_error();
}

// Checks shared by the batch entry points; fills P.
int batch_prepare(const d8_batch_item *items, int n, int mode, void *ws, size_t ws_bytes, BatchPlan &P)
{
    if (mode <= 0 || (mode & ~(D8_BATCH_FWD | D8_BATCH_ADJ)) != 0) return D8_EINVAL;
    int rc = make_plan(items, n, P);
    if (rc != D8_OK) return rc;
    for (const DemDesc &D : P.dems) {
        if ((mode & D8_BATCH_FWD) && !D.acc) return D8_EINVAL;
        if ((mode & D8_BATCH_ADJ) && (!D.gacc || !D.gw)) return D8_EINVAL;
    }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < P.L.total) return D8_EWORKSPACE;
    return D8_OK;
}

struct GraphHandle {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// --------------------------------------------------------------- streaming --
// A raster in host memory, processed in bands of whole tile rows: pass 1 per
// band (codes of the band plus one halo row above and below), the band's
// graph edges once the next band's links exist, the resolve over the whole
// perimeter graph (which stays in the workspace), then pass 2 per band with
// the counts copied back.  Host-to-device and device-to-host copies run on
// two streams of the library's own (the link is full duplex) and overlap the
// kernels on the caller's stream; events order slot reuse.
struct StreamLayout {
    Layout L;           // perimeter-graph arrays (root8 unused)
    size_t cslot[3];    // codes: (band_rows + 2) x cols bytes each
    size_t oslot[2];    // results: band_rows x cols 4-byte values each
    size_t vslot[2];    // float inputs (weights or cotangents): band_rows x cols each
    size_t total;
    int64_t band_rows;  // a multiple of the tile height
};

int stream_layout(int64_t rows, int64_t cols, int &th, int &tw, int64_t band_rows, Geo &g,
                  bool &empty, StreamLayout &S)
{
    int rc = check_common(rows, cols, th, tw, g, empty);
    if (rc != D8_OK) return rc;
    if (band_rows < 0) return D8_EINVAL;
    if (empty) return D8_OK;
    if (band_rows == 0) band_rows = (int64_t)16 * th;
    if (band_rows % th != 0) return D8_EINVAL;
    if (band_rows > rows) band_rows = ((rows + th - 1) / th) * th;
    S.band_rows = band_rows;
    S.L = layout_for(g);
    size_t off = align256(S.L.root8);
    for (int i = 0; i < 3; ++i) {
        S.cslot[i] = off;
        off = align256(off + (size_t)(band_rows + 2) * (size_t)cols);
    }
    for (int i = 0; i < 2; ++i) {
        S.oslot[i] = off;
        off = align256(off + (size_t)band_rows * (size_t)cols * sizeof(uint32_t));
    }
    for (int i = 0; i < 2; ++i) {
        S.vslot[i] = off;
        off = align256(off + (size_t)band_rows * (size_t)cols * sizeof(float));
    }
    // the float resolve's children lists lie over the slots (they are used
    // between the passes only) and may reach beyond them
    S.total = std::max(off, csr_place(S.L.root8, (size_t)g.nnodes, S.L.off, S.L.kids, S.L.srt, S.L.bsum));
    return D8_OK;
}

// Per device: the copy streams (in, out) and the events of the pipeline.
struct StreamRes {
    hipStream_t cs = nullptr, cs2 = nullptr;
    hipEvent_t ev[20] = {};
};
enum { kEvFree = 0, kEvReady = 3, kEvP1 = 6, kEvCFree = 7, kEvCReady = 9, kEvOFree = 11,
       kEvODone = 13, kEvEnd = 15, kEvVFree = 16, kEvVReady = 18 };

int stream_res(StreamRes *&R)
{
    static std::mutex mu;
    static std::vector<StreamRes> res;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return D8_EHIP;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)res.size() <= dev) res.resize(dev + 1);
    StreamRes &r = res[dev];
    if (!r.cs) {
        if (hipStreamCreateWithFlags(&r.cs, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&r.cs2, hipStreamNonBlocking) != hipSuccess)
            return D8_EHIP;
        for (hipEvent_t &e : r.ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return D8_EHIP;
    }
    R = &r;
    return D8_OK;
}

// What a streamed call computes: unit counts, float weighted sums, or the
// adjoint.  The bands go through the same two-pass pipeline; the float kinds
// also stream one float input per cell (weights or cotangents) in both passes.
enum StreamKind { kStreamU32 = 0, kStreamF32 = 1, kStreamAdj = 2 };

int run_streamed(int kind, const uint8_t *dirs_h, const float *v_h, void *out_h, const Geo &g,
                 const StreamLayout &S, char *ws, hipStream_t st)
{
    StreamRes *R = nullptr;
    if (stream_res(R) != D8_OK) return D8_EHIP;
    hipStream_t cs = R->cs, cs2 = R->cs2;
    hipEvent_t *ev = R->ev;
    const Layout &L = S.L;
    uint32_t *status = reinterpret_cast<uint32_t *>(ws + L.status);
    uint32_t *jstate = reinterpret_cast<uint32_t *>(ws + L.jstate);
    uint16_t *link = reinterpret_cast<uint16_t *>(ws + L.link);
    uint32_t *entry = reinterpret_cast<uint32_t *>(ws + L.entry);
    uint32_t *succ = reinterpret_cast<uint32_t *>(ws + L.succ);
    uint32_t *indeg = reinterpret_cast<uint32_t *>(ws + L.indeg);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + L.ptr2);
    const int64_t cols = g.cols, rows = g.rows;
    const int tb = (int)(S.band_rows / g.th);  // tile rows per band
    const int nband = (g.nty + tb - 1) / tb;
    // float inputs are streamed when given (unit weights need none)
    const bool f32 = kind == kStreamF32, adj = kind == kStreamAdj, vals = v_h != nullptr;
    using VU = unsigned long long;
    const size_t lds1 = adj ? walk_lds_bytes(g.th, g.tw, kWalkAdj1)
                            : walk_lds_bytes(g.th, g.tw, kWalkFwd1, f32 ? 4 : (int)sizeof(FwdLds<1, uint32_t>));
    const size_t lds2 = adj ? lds1 : walk_lds_bytes(g.th, g.tw, kWalkFwd2, 4);
    const auto u1 = fwd_walk_k<1, uint32_t, VU, uint32_t>(g.tw), u2 = fwd_walk_k<2, uint32_t, VU, uint32_t>(g.tw);
    const auto f1 = fwd_walk_k<1, float, double, double>(g.tw), f2 = fwd_walk_k<2, float, double, double>(g.tw);
    const auto ab = adj_walk_band_k(g.tw);
    if (allow_lds(u1, lds1) || allow_lds(u2, lds2) || allow_lds(f1, lds1) || allow_lds(f2, lds2) ||
        allow_lds(ab, lds1))
        return D8_EHIP;
    auto band = [&](int b, int &ty0, int &ty1, int64_t &r0, int64_t &r1) {
        ty0 = b * tb;
        ty1 = std::min(g.nty, ty0 + tb);
        r0 = (int64_t)ty0 * g.th;
        r1 = std::min(rows, (int64_t)ty1 * g.th);
    };
    // a band's codes in slot i: slot row 0 is raster row r0 - 1
    auto codes_ptr = [&](size_t slot, int64_t r0) {
        return reinterpret_cast<const uint8_t *>(ws + slot) - (r0 - 1) * cols;
    };
    // a band's values or results in slot i: slot row 0 is raster row r0
    auto band_ptr = [&](size_t slot, int64_t r0) { return reinterpret_cast<float *>(ws + slot) - r0 * cols; };
    auto nodes_of = [&](int ty0, int ty1, int64_t &n0, int64_t &n1) {
        n0 = (int64_t)ty0 * g.row_nodes;
        n1 = ty1 >= g.nty ? g.nnodes : (int64_t)ty1 * g.row_nodes;
    };
    auto edges = [&](int b) {
        int ty0, ty1;
        int64_t r0, r1, n0, n1;
        band(b, ty0, ty1, r0, r1);
        nodes_of(ty0, ty1, n0, n1);
        D8_LAUNCH("stream_graph_build", st,
                  (graph_build<<<blocks_for(n1 - n0, kNodeBlock), kNodeBlock, 0, st>>>(
                      codes_ptr(S.cslot[b % 3], r0), g, link, entry, succ, adj ? nullptr : indeg, n0, n1)));
        (void)hipEventRecord(ev[kEvFree + b % 3], st);
    };
    // a band's codes (with its halo rows) into code slot `slot` on cs
    auto codes_in = [&](int slot, int64_t r0, int64_t r1) {
        const int64_t h0 = std::max<int64_t>(0, r0 - 1), h1 = std::min(rows, r1 + 1);
        (void)hipMemcpyAsync(ws + S.cslot[slot] + (h0 - (r0 - 1)) * cols, dirs_h + h0 * cols,
                             (size_t)(h1 - h0) * cols, hipMemcpyHostToDevice, cs);
    };
    // a band's float inputs into value slot b & 1 on cs, after the pass that
    // last read the slot (band b - 2 of the same pass)
    auto values_in = [&](int b, int64_t r0, int64_t r1) {
        const int vs = b & 1;
        if (b >= 2) (void)hipStreamWaitEvent(cs, ev[kEvVFree + vs], 0);
        (void)hipMemcpyAsync(ws + S.vslot[vs], v_h + r0 * cols, (size_t)(r1 - r0) * cols * sizeof(float),
                             hipMemcpyHostToDevice, cs);
        (void)hipEventRecord(ev[kEvVReady + vs], cs);
        (void)hipStreamWaitEvent(st, ev[kEvVReady + vs], 0);
    };

    init_state<<<1, 1, 0, st>>>(status, jstate);
    // the copy stream starts after the caller's earlier work on `st`
    (void)hipEventRecord(ev[kEvEnd], st);
    (void)hipStreamWaitEvent(cs, ev[kEvEnd], 0);
    // pass 1 over the bands; band b - 1's edges after band b's links
    for (int b = 0; b < nband; ++b) {
        int ty0, ty1;
        int64_t r0, r1;
        band(b, ty0, ty1, r0, r1);
        const int slot = b % 3;
        if (b >= 3) (void)hipStreamWaitEvent(cs, ev[kEvFree + slot], 0);
        codes_in(slot, r0, r1);
        (void)hipEventRecord(ev[kEvReady + slot], cs);
        (void)hipStreamWaitEvent(st, ev[kEvReady + slot], 0);
        if (vals) values_in(b, r0, r1);
        const int t0 = ty0 * g.ntx, nt = (ty1 - ty0) * g.ntx;
        const uint8_t *dirs = codes_ptr(S.cslot[slot], r0);
        const float *v = vals ? band_ptr(S.vslot[b & 1], r0) : nullptr;
        if (adj)
            D8_LAUNCH("stream_adj_pass1", st,
                      (ab<<<nt, kTileThreads, lds1, st>>>(
                          dirs, v, g, link, reinterpret_cast<float *>(ws + L.val32), nullptr, status, nullptr,
                          nullptr, nullptr, jstate, t0)));
        else if (f32)
            D8_LAUNCH("stream_fwd_pass1", st,
                      (f1<<<nt, kTileThreads, lds1, st>>>(
                          dirs, v, g, link, reinterpret_cast<float *>(ws + L.val32), indeg, cnt,
                          reinterpret_cast<double *>(ws + L.acc64), reinterpret_cast<double *>(ws + L.ext64),
                          nullptr, status, t0)));
        else
            D8_LAUNCH("stream_fwd_pass1", st,
                      (u1<<<nt, kTileThreads, lds1, st>>>(
                          dirs, nullptr, g, link, reinterpret_cast<uint32_t *>(ws + L.val32), indeg, cnt,
                          reinterpret_cast<VU *>(ws + L.acc64), reinterpret_cast<uint32_t *>(ws + L.ext64),
                          nullptr, status, t0)));
        if (vals) (void)hipEventRecord(ev[kEvVFree + (b & 1)], st);
        if (b >= 1) edges(b - 1);
    }
    edges(nband - 1);
    // the resolve over the whole perimeter graph
    unsigned long long *jw[2] = {reinterpret_cast<unsigned long long *>(ws + L.acc64),
                                 reinterpret_cast<unsigned long long *>(ws + L.ext64)};
    const unsigned nbn = blocks_for(g.nnodes, kNodeBlock);
    if (adj) {
        JumpGraph G{nullptr, g, nullptr, 0, nullptr};
        G.entry = entry;
        G.succ = succ;
        jump_exits(st, g.nnodes, G, link, reinterpret_cast<float *>(ws + L.val32), indeg, cnt, jw, jstate, status,
                   false);
    } else if (f32) {
        resolve_float<false>(st, false, g.nnodes, link, reinterpret_cast<float *>(ws + L.val32), succ, indeg, cnt,
                             ws, L.off, L.kids, L.srt, L.bsum, jstate + 8, reinterpret_cast<double *>(ws + L.acc64),
                             status);
    } else {
        VU *acc = reinterpret_cast<VU *>(ws + L.acc64);
        D8_LAUNCH("stream_resolve", st,
                  (resolve_fwd_u32<<<nbn, kNodeBlock, 0, st>>>(g.nnodes, link,
                                                              reinterpret_cast<uint32_t *>(ws + L.val32), entry,
                                                              succ, indeg, acc,
                                                              reinterpret_cast<uint32_t *>(ws + L.ext64))));
    }
    // pass 2 over the bands: code, value and result slots b & 1
    (void)hipEventRecord(ev[kEvP1], st);
    (void)hipStreamWaitEvent(cs, ev[kEvP1], 0);
    for (int b = 0; b < nband; ++b) {
        int ty0, ty1;
        int64_t r0, r1, n0, n1;
        band(b, ty0, ty1, r0, r1);
        nodes_of(ty0, ty1, n0, n1);
        const int cslot = b & 1, oslot = b & 1;
        if (b >= 2) (void)hipStreamWaitEvent(cs, ev[kEvCFree + cslot], 0);
        codes_in(cslot, r0, r1);
        (void)hipEventRecord(ev[kEvCReady + cslot], cs);
        (void)hipStreamWaitEvent(st, ev[kEvCReady + cslot], 0);
        if (vals) values_in(b, r0, r1);
        if (b >= 2) (void)hipStreamWaitEvent(st, ev[kEvOFree + oslot], 0);
        const uint8_t *dirs = codes_ptr(S.cslot[cslot], r0);
        const float *v = vals ? band_ptr(S.vslot[b & 1], r0) : nullptr;
        float *outf = band_ptr(S.oslot[oslot], r0);
        const int t0 = ty0 * g.ntx, nt = (ty1 - ty0) * g.ntx;
        if (adj) {
            D8_LAUNCH("stream_adj_pass2", st,
                      (ab<<<nt, kTileThreads, lds2, st>>>(dirs, v, g, nullptr, nullptr, outf, status, cnt,
                                                                      jw[0], jw[1], jstate, t0)));
        } else if (f32) {
            double *ext = reinterpret_cast<double *>(ws + L.ext64);
            D8_LAUNCH("stream_resolve_ext", st,
                      (resolve_ext<false><<<blocks_for(n1 - n0, kNodeBlock), kNodeBlock, 0, st>>>(
                          dirs, g, link, reinterpret_cast<double *>(ws + L.acc64), ext, nullptr, n0, n1)));
            D8_LAUNCH("stream_fwd_pass2", st,
                      (f2<<<nt, kTileThreads, lds2, st>>>(
                          dirs, v, g, link, reinterpret_cast<float *>(ws + L.val32), indeg, cnt,
                          reinterpret_cast<double *>(ws + L.acc64), ext, outf, status, t0)));
        } else {
            D8_LAUNCH("stream_fwd_pass2", st,
                      (u2<<<nt, kTileThreads, lds2, st>>>(
                          dirs, nullptr, g, link, reinterpret_cast<uint32_t *>(ws + L.val32), indeg, nullptr,
                          reinterpret_cast<VU *>(ws + L.acc64), reinterpret_cast<uint32_t *>(ws + L.ext64),
                          reinterpret_cast<uint32_t *>(outf), status, t0)));
        }
        (void)hipEventRecord(ev[kEvCFree + cslot], st);
        if (vals) (void)hipEventRecord(ev[kEvVFree + (b & 1)], st);
        (void)hipEventRecord(ev[kEvODone + oslot], st);
        (void)hipStreamWaitEvent(cs2, ev[kEvODone + oslot], 0);
        (void)hipMemcpyAsync(reinterpret_cast<char *>(out_h) + r0 * cols * 4, ws + S.oslot[oslot],
                             (size_t)(r1 - r0) * cols * 4, hipMemcpyDeviceToHost, cs2);
        (void)hipEventRecord(ev[kEvOFree + oslot], cs2);
    }
    // the call is complete when `st` is: it waits for the last copy out
    (void)hipEventRecord(ev[kEvEnd], cs2);
    (void)hipStreamWaitEvent(st, ev[kEvEnd], 0);
    return last_error();
}

// D8 (or rho8) over the raster in strips of kD8Rows rows and blocks of
// kD8Cols columns.
template <bool RHO>
int launch_d8(const float *dem, const float *rnd, uint8_t *dirs, int64_t rows, int64_t cols,
              float nodata, hipStream_t st)
{
    if (rows < 0 || cols < 0) return D8_EINVAL;
    if (rows == 0 || cols == 0) return D8_OK;
    if (!dem || !dirs) return D8_EINVAL;
    begin_call();
    const int64_t ncb = (cols + kD8Cols - 1) / kD8Cols, nstrips = (rows + kD8Rows - 1) / kD8Rows;
    const bool vec = cols % 4 == 0 && (reinterpret_cast<uintptr_t>(dem) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(rnd) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(dirs) & 3) == 0;
    const char *name = RHO ? "d8_directions_rho8" : "d8_directions";
    // at most 2^22 blocks per launch (grid size in lanes stays below 2^32)
    const int64_t per = std::max<int64_t>(1, ((int64_t)1 << 22) / ncb);
    for (int64_t s0 = 0; s0 < nstrips; s0 += per) {
        const int64_t ns = nstrips - s0 < per ? nstrips - s0 : per;
        const unsigned nb = (unsigned)(ns * ncb);
        if (vec)
            D8_LAUNCH(name, st,
                      (d8_kernel<true, RHO><<<nb, kD8Threads, 0, st>>>(dem, rnd, dirs, rows, cols, nodata,
                                                                      ncb, s0)));
        else
            D8_LAUNCH(name, st,
                      (d8_kernel<false, RHO><<<nb, kD8Threads, 0, st>>>(dem, rnd, dirs, rows, cols,
                                                                       nodata, ncb, s0)));
    }
    return last_error();
}

// ---- flow_accum without allocation: the workspace is a file-scope device
// array, one copy per GPU.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address comes from hipGetSymbolAddress, once
// per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[D8_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // per device id; null until looked up

int scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return D8_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[(size_t)dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return D8_EHIP;
        }
        g_scratch_ptr[(size_t)dev] = ptr;
    }
    *out = g_scratch_ptr[(size_t)dev];
    return D8_OK;
}

__global__ void copy_status(const uint32_t *status, uint32_t *out) { out[0] = status[0]; }

}  // namespace

extern "C" {

int d8_version(void) { return 100; }

const char *d8_strerror(int code)
{
    switch (code) {
    case D8_OK: return "ok";
    case D8_EINVAL: return "invalid argument";
    case D8_EWORKSPACE: return "workspace missing or too small";
    case D8_EHIP: return "HIP runtime error";
    case D8_EDIRCODE: return "invalid direction code (above 9) in input";
    case D8_ECYCLE: return "flow directions contain a cycle";
    default: return "unknown status code";
    }
}

int d8_directions(const float *dem, uint8_t *dirs, int64_t rows, int64_t cols, float nodata,
                  void *stream)
{
    return launch_d8<false>(dem, nullptr, dirs, rows, cols, nodata, as_stream(stream));
}

int d8_directions_rho8(const float *dem, const float *rnd, uint8_t *dirs, int64_t rows, int64_t cols,
                       float nodata, void *stream)
{
    if (rows > 0 && cols > 0 && !rnd) return D8_EINVAL;
    return launch_d8<true>(dem, rnd, dirs, rows, cols, nodata, as_stream(stream));
}

size_t d8_workspace_bytes(int64_t rows, int64_t cols, int tile_rows, int tile_cols)
{
    Geo g;
    bool empty;
    if (check_common(rows, cols, tile_rows, tile_cols, g, empty) != D8_OK) return 0;
    if (empty) return 512;
    return layout_for(g).total;
}

int flow_accum(const uint8_t *dirs, const float *weights, void *acc, int acc_type, int64_t rows,
               int64_t cols, int tile_rows, int tile_cols, void *ws, size_t ws_bytes, void *stream)
{
    if (acc_type != D8_ACC_U32 && acc_type != D8_ACC_F32) return D8_EINVAL;
    if (acc_type == D8_ACC_U32 && weights) return D8_EINVAL;
    Geo g;
    bool empty;
    int rc = check_common(rows, cols, tile_rows, tile_cols, g, empty);
    if (rc != D8_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return D8_EWORKSPACE;
    if (empty) {
        if (ws_bytes < 512) return D8_EWORKSPACE;
        init_state<<<1, 1, 0, as_stream(stream)>>>(reinterpret_cast<uint32_t *>(ws),
                                                   reinterpret_cast<uint32_t *>((char *)ws + 256));
        return last_error();
    }
    if (!dirs || !acc) return D8_EINVAL;
    Layout L = layout_for(g);
    if (ws_bytes < L.total) return D8_EWORKSPACE;
    char *w8 = reinterpret_cast<char *>(ws);
    begin_call();
    if (acc_type == D8_ACC_U32)
        return run_forward<uint32_t>(dirs, nullptr, reinterpret_cast<uint32_t *>(acc), g, w8, L,
                                     as_stream(stream));
    return run_forward<float>(dirs, weights, reinterpret_cast<float *>(acc), g, w8, L,
                              as_stream(stream));
}

int flow_accum_adjoint(const uint8_t *dirs, const float *grad_acc, float *grad_weights,
                       int64_t rows, int64_t cols, int tile_rows, int tile_cols, void *ws,
                       size_t ws_bytes, void *stream)
{
    Geo g;
    bool empty;
    int rc = check_common(rows, cols, tile_rows, tile_cols, g, empty);
    if (rc != D8_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return D8_EWORKSPACE;
    hipStream_t st = as_stream(stream);
    if (empty) {
        if (ws_bytes < 512) return D8_EWORKSPACE;
        init_state<<<1, 1, 0, st>>>(reinterpret_cast<uint32_t *>(ws),
                                    reinterpret_cast<uint32_t *>((char *)ws + 256));
        return last_error();
    }
    if (!dirs || !grad_acc || !grad_weights) return D8_EINVAL;
    Layout L = layout_for(g);
    if (ws_bytes < L.total) return D8_EWORKSPACE;
    char *w8 = reinterpret_cast<char *>(ws);
    uint32_t *status = reinterpret_cast<uint32_t *>(w8 + L.status);
    uint32_t *jstate = reinterpret_cast<uint32_t *>(w8 + L.jstate);
    uint16_t *link = reinterpret_cast<uint16_t *>(w8 + L.link);
    float *S = reinterpret_cast<float *>(w8 + L.val32);
    unsigned long long *jw[2] = {reinterpret_cast<unsigned long long *>(w8 + L.acc64),
                                 reinterpret_cast<unsigned long long *>(w8 + L.ext64)};

    uint8_t *root8 = reinterpret_cast<uint8_t *>(w8 + L.root8);
    uint32_t *cmap = reinterpret_cast<uint32_t *>(w8 + L.ptr2);
    int ntiles = g.nty * g.ntx;
    const int thr = kTileThreads;
    size_t lds1 = walk_lds_bytes(g.th, g.tw, kWalkAdj1);
    begin_call();
    const auto pass1 = adj_walk_k(g.tw);
    if (allow_lds(pass1, lds1)) return D8_EHIP;
    init_state<<<1, 1, 0, st>>>(status, jstate);
    D8_LAUNCH("adj_pass1", st,
              (pass1<<<ntiles, thr, lds1, st>>>(dirs, grad_acc, g, link, S, grad_weights, root8,
                                                   status)));
    // the exits' edges are found as their jump words are initialised
    const JumpGraph G{dirs, g, nullptr, 0, nullptr};
    const int rounds = jump_exits(st, g.nnodes, G, link, S, reinterpret_cast<uint32_t *>(w8 + L.indeg),
                                  cmap, jw, jstate, status, false);
    D8_LAUNCH("adj_pass2", st,
              (adj_finish<<<ntiles, thr, 0, st>>>(g, root8, cmap, jw[0], jw[1], jstate, grad_weights)));
    (void)rounds;
    return last_error();
}

int flow_accum_noalloc(const uint8_t *dirs, const float *weights, void *acc, int acc_type, int64_t rows,
                       int64_t cols, int tile_rows, int tile_cols, uint32_t *status, void *stream)
{
    const size_t need = d8_workspace_bytes(rows, cols, tile_rows, tile_cols);
    if (need == 0) return D8_EINVAL;
    if (need > (size_t)D8_NOALLOC_SCRATCH_BYTES) return D8_EWORKSPACE;
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc != D8_OK) return rc;
    rc = flow_accum(dirs, weights, acc, acc_type, rows, cols, tile_rows, tile_cols, ws,
                    (size_t)D8_NOALLOC_SCRATCH_BYTES, stream);
    if (rc != D8_OK || !status) return rc;
    hipStream_t st = as_stream(stream);
    copy_status<<<1, 1, 0, st>>>(reinterpret_cast<const uint32_t *>(ws), status);
    return hipGetLastError() == hipSuccess ? D8_OK : D8_EHIP;
}

// ----------------------------------------------------------- absorption --

size_t d8_absorb_workspace_bytes(int64_t rows, int64_t cols, int tile_rows, int tile_cols)
{
    Geo g;
    bool empty;
    absorb_default_tile(tile_rows, tile_cols);
    if (check_common(rows, cols, tile_rows, tile_cols, g, empty) != D8_OK) return 0;
    if (empty) return 512;
    return absorb_layout(layout_for(g), g).total;
}

int flow_accum_absorb(const uint8_t *dirs, const float *weights, const float *alpha, float *acc,
                      int64_t rows, int64_t cols, int tile_rows, int tile_cols, void *ws, size_t ws_bytes,
                      void *stream)
{
    Geo g;
    bool empty;
    absorb_default_tile(tile_rows, tile_cols);
    int rc = check_common(rows, cols, tile_rows, tile_cols, g, empty);
    if (rc != D8_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return D8_EWORKSPACE;
    if (empty) {
        if (ws_bytes < 512) return D8_EWORKSPACE;
        init_state<<<1, 1, 0, as_stream(stream)>>>(reinterpret_cast<uint32_t *>(ws),
                                                   reinterpret_cast<uint32_t *>((char *)ws + 256));
        return last_error();
    }
    if (!dirs || !alpha || !acc) return D8_EINVAL;
    const Layout L = layout_for(g);
    if (ws_bytes < absorb_layout(L, g).total) return D8_EWORKSPACE;
    begin_call();
    return run_forward_absorb(dirs, weights, alpha, acc, g, reinterpret_cast<char *>(ws), L,
                              as_stream(stream));
}

int flow_accum_absorb_adjoint(const uint8_t *dirs, const float *alpha, const float *grad_acc,
                              float *grad_weights, int64_t rows, int64_t cols, int tile_rows, int tile_cols,
                              void *ws, size_t ws_bytes, void *stream)
{
    Geo g;
    bool empty;
    absorb_default_tile(tile_rows, tile_cols);
    int rc = check_common(rows, cols, tile_rows, tile_cols, g, empty);
    if (rc != D8_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return D8_EWORKSPACE;
    hipStream_t st = as_stream(stream);
    if (empty) {
        if (ws_bytes < 512) return D8_EWORKSPACE;
        init_state<<<1, 1, 0, st>>>(reinterpret_cast<uint32_t *>(ws),
                                    reinterpret_cast<uint32_t *>((char *)ws + 256));
        return last_error();
    }
    if (!dirs || !alpha || !grad_acc || !grad_weights) return D8_EINVAL;
    const Layout L = layout_for(g);
    const AbsorbLayout A = absorb_layout(L, g);
    if (ws_bytes < A.total) return D8_EWORKSPACE;
    char *w8 = reinterpret_cast<char *>(ws);
    uint32_t *status = reinterpret_cast<uint32_t *>(w8 + L.status);
    uint32_t *jstate = reinterpret_cast<uint32_t *>(w8 + L.jstate);
    uint16_t *link = reinterpret_cast<uint16_t *>(w8 + L.link);
    float *S = reinterpret_cast<float *>(w8 + L.val32);
    float *P = reinterpret_cast<float *>(w8 + A.pathp);
    float *pcell = reinterpret_cast<float *>(w8 + A.pcell);
    uint8_t *root8 = reinterpret_cast<uint8_t *>(w8 + L.root8);
    uint32_t *cmap = reinterpret_cast<uint32_t *>(w8 + L.ptr2);
    uint32_t *bsum = reinterpret_cast<uint32_t *>(w8 + L.indeg);
    uint4 *jw[2] = {reinterpret_cast<uint4 *>(w8 + L.acc64), reinterpret_cast<uint4 *>(w8 + A.jw)};
    uint32_t *nexit = jstate + 4;
    const int ntiles = g.nty * g.ntx;
    const size_t lds1 = walk_lds_bytes(g.th, g.tw, kWalkAdj1, 4, true);
    begin_call();
    const auto apass1 = adj_walk_absorb_k(g.tw);
    if (allow_lds(apass1, lds1)) return D8_EHIP;
    init_state<<<1, 1, 0, st>>>(status, jstate);
    D8_LAUNCH("absorb_adj_pass1", st,
              (apass1<<<ntiles, kTileThreads, lds1, st>>>(dirs, grad_acc, alpha, g, link, S, P, grad_weights,
                                                          pcell, root8, status)));
    // inv (dense index -> node) lives in jw[1] until round 0 overwrites it
    uint32_t *inv = reinterpret_cast<uint32_t *>(jw[1]);
    compact_exits(st, g.nnodes, link, bsum, cmap, inv, nexit, false);
    const unsigned jb = std::min<unsigned>(blocks_for(g.nnodes, 2 * kNodeBlock), 4096u);
    const JumpGraph G{dirs, g, nullptr, 0, nullptr};
    D8_LAUNCH("absorb_jump_init", st,
              (adj_jump_init_absorb<<<jb, kNodeBlock, 0, st>>>(nexit, inv, G, link, S, P, cmap, jw[0])));
    int rounds = 1;
    for (int64_t span = 1; span <= g.nnodes; span *= 3) ++rounds;
    for (int r = 0; r < rounds; ++r)
        D8_LAUNCH("absorb_jump_round", st,
                  (adj_jump_round_absorb<<<jb, kNodeBlock, 0, st>>>(nexit, jw[r & 1], jw[(r + 1) & 1], jstate,
                                                                    r)));
    D8_LAUNCH("adj_jump_finish", st, (adj_jump_finish<<<1, 1, 0, st>>>(jstate, rounds, status)));
    D8_LAUNCH("absorb_adj_pass2", st,
              (adj_finish_absorb<<<ntiles, kTileThreads, 0, st>>>(g, root8, cmap, jw[0], jw[1], jstate, pcell,
                                                                 grad_weights)));
    return last_error();
}

int flow_accum_absorb_alpha_grad(const uint8_t *dirs, const float *acc, const float *grad_lam,
                                 float *grad_alpha, int64_t rows, int64_t cols, void *stream)
{
    if (rows < 0 || cols < 0 || rows > INT_MAX || cols > INT_MAX) return D8_EINVAL;
    if (rows == 0 || cols == 0) return D8_OK;
    if (!dirs || !acc || !grad_lam || !grad_alpha) return D8_EINVAL;
    begin_call();
    hipStream_t st = as_stream(stream);
    const dim3 grid((unsigned)((cols + kGradBlock - 1) / kGradBlock), (unsigned)std::min<int64_t>(rows, 65535));
    D8_LAUNCH("absorb_alpha_grad", st,
              (absorb_alpha_grad<<<grid, kGradBlock, 0, st>>>(dirs, acc, grad_lam, grad_alpha, rows, cols)));
    return last_error();
}

size_t d8_stream_workspace_bytes(int64_t rows, int64_t cols, int tile_rows, int tile_cols,
                                 int64_t band_rows)
{
    Geo g;
    bool empty;
    StreamLayout S;
    if (stream_layout(rows, cols, tile_rows, tile_cols, band_rows, g, empty, S) != D8_OK) return 0;
    if (empty) return 512;
    return S.total;
}

int flow_accum_streamed(const uint8_t *dirs_host, uint32_t *acc_host, int64_t rows, int64_t cols,
                        int tile_rows, int tile_cols, int64_t band_rows, void *ws, size_t ws_bytes,
                        void *stream)
{
    Geo g;
    bool empty;
    StreamLayout S;
    int rc = stream_layout(rows, cols, tile_rows, tile_cols, band_rows, g, empty, S);
    if (rc != D8_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return D8_EWORKSPACE;
    if (empty) {
        if (ws_bytes < 512) return D8_EWORKSPACE;
        init_state<<<1, 1, 0, as_stream(stream)>>>(reinterpret_cast<uint32_t *>(ws),
                                                   reinterpret_cast<uint32_t *>((char *)ws + 256));
        return last_error();
    }
    if (!dirs_host || !acc_host) return D8_EINVAL;
    if (ws_bytes < S.total) return D8_EWORKSPACE;
    begin_call();
    return run_streamed(kStreamU32, dirs_host, nullptr, acc_host, g, S, reinterpret_cast<char *>(ws),
                        as_stream(stream));
}

// The float kinds: weights (NULL = unit) or cotangents in host memory.
static int streamed_float(int kind, const uint8_t *dirs_host, const float *v_host, float *out_host, int64_t rows,
                   int64_t cols, int tile_rows, int tile_cols, int64_t band_rows, void *ws, size_t ws_bytes,
                   void *stream)
{
    Geo g;
    bool empty;
    StreamLayout S;
    int rc = stream_layout(rows, cols, tile_rows, tile_cols, band_rows, g, empty, S);
    if (rc != D8_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return D8_EWORKSPACE;
    if (empty) {
        if (ws_bytes < 512) return D8_EWORKSPACE;
        init_state<<<1, 1, 0, as_stream(stream)>>>(reinterpret_cast<uint32_t *>(ws),
                                                   reinterpret_cast<uint32_t *>((char *)ws + 256));
        return last_error();
    }
    if (!dirs_host || !out_host || (kind == kStreamAdj && !v_host)) return D8_EINVAL;
    if (ws_bytes < S.total) return D8_EWORKSPACE;
    begin_call();
    return run_streamed(kind, dirs_host, v_host, out_host, g, S, reinterpret_cast<char *>(ws), as_stream(stream));
}

int flow_accum_streamed_f32(const uint8_t *dirs_host, const float *weights_host, float *acc_host, int64_t rows,
                            int64_t cols, int tile_rows, int tile_cols, int64_t band_rows, void *ws,
                            size_t ws_bytes, void *stream)
{
    return streamed_float(kStreamF32, dirs_host, weights_host, acc_host, rows, cols, tile_rows, tile_cols,
                          band_rows, ws, ws_bytes, stream);
}

int flow_accum_adjoint_streamed(const uint8_t *dirs_host, const float *grad_host, float *grad_weights_host,
                                int64_t rows, int64_t cols, int tile_rows, int tile_cols, int64_t band_rows,
                                void *ws, size_t ws_bytes, void *stream)
{
    return streamed_float(kStreamAdj, dirs_host, grad_host, grad_weights_host, rows, cols, tile_rows, tile_cols,
                          band_rows, ws, ws_bytes, stream);
}

size_t d8_batch_workspace_bytes(const d8_batch_item *items, int n)
{
    BatchPlan P;
    if (make_plan(items, n, P) != D8_OK) return 0;
    return P.L.total;
}

int flow_accum_batched(const d8_batch_item *items, int n, int mode, void *ws, size_t ws_bytes,
                       void *stream)
{
    BatchPlan P;
    int rc = batch_prepare(items, n, mode, ws, ws_bytes, P);
    if (rc != D8_OK) return rc;
    begin_call();
    char *w8 = reinterpret_cast<char *>(ws);
    hipStream_t st = as_stream(stream);
    rc = upload_plan(P, w8, st);
    if (rc != D8_OK) return rc;
    return enqueue_batch(P, mode, w8, st);
}

int d8_graph_create(const d8_batch_item *items, int n, int mode, void *ws, size_t ws_bytes,
                    void *stream, void **graph_exec)
{
    if (!graph_exec) return D8_EINVAL;
    *graph_exec = nullptr;
    BatchPlan P;
    int rc = batch_prepare(items, n, mode, ws, ws_bytes, P);
    if (rc != D8_OK) return rc;
    begin_call();
    char *w8 = reinterpret_cast<char *>(ws);
    // a setup call: the tables are in the workspace when it returns, so the
    // graph may be launched on any stream
    rc = upload_plan(P, w8, as_stream(stream), true);
    if (rc != D8_OK) return rc;
    // record on a stream of our own (the caller's may be the legacy default
    // stream, which cannot be captured)
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return D8_EHIP;
    GraphHandle *h = new GraphHandle;
    rc = D8_EHIP;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        g_capturing = true;
        int erc = enqueue_batch(P, mode, w8, cap);
        g_capturing = false;
        hipError_t e = hipStreamEndCapture(cap, &h->graph);
        if (erc == D8_OK && e == hipSuccess &&
            hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) == hipSuccess)
            rc = D8_OK;
        else if (erc != D8_OK)
            rc = erc;
    }
    (void)hipStreamDestroy(cap);
    if (rc != D8_OK) {
        if (h->exec) (void)hipGraphExecDestroy(h->exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        delete h;
        (void)hipGetLastError();
        return rc;
    }
    *graph_exec = h;
    return D8_OK;
}

int d8_graph_launch(void *graph_exec, void *stream)
{
    if (!graph_exec) return D8_EINVAL;
    GraphHandle *h = reinterpret_cast<GraphHandle *>(graph_exec);
    return hipGraphLaunch(h->exec, as_stream(stream)) == hipSuccess ? D8_OK : D8_EHIP;
}

int d8_graph_destroy(void *graph_exec)
{
    if (!graph_exec) return D8_EINVAL;
    GraphHandle *h = reinterpret_cast<GraphHandle *>(graph_exec);
    int rc = D8_OK;
    if (h->exec && hipGraphExecDestroy(h->exec) != hipSuccess) rc = D8_EHIP;
    if (h->graph && hipGraphDestroy(h->graph) != hipSuccess) rc = D8_EHIP;
    delete h;
    return rc;
}

const char *d8_last_error_message(void) { return g_last_error.c_str(); }

int d8_timing_enable(int on)
{
    if (on < 0 || on > 2) return D8_EINVAL;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_on = on;
    return D8_OK;
}

int d8_timing_report(const char **names, double *total_ms, int64_t *launches, int max_entries)
{
    std::vector<TimedLaunch> recs;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        recs.swap(g_timed);
    }
    int n = 0, rc = 0;
    for (const TimedLaunch &t : recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(t.stop) != hipSuccess ||
            hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess)
            rc = D8_EHIP;
        int k = 0;
        while (k < n && std::strcmp(names[k], t.name) != 0) ++k;
        if (k == n) {
            if (n == max_entries) continue;
            names[n] = t.name;
            total_ms[n] = 0.0;
            launches[n] = 0;
            ++n;
        }
        total_ms[k] += ms;
        launches[k] += 1;
    }
    std::lock_guard<std::mutex> lk(g_timing_mu);
    for (const TimedLaunch &t : recs) {
        g_event_pool.push_back(t.start);
        g_event_pool.push_back(t.stop);
    }
    return rc ? rc : n;
}

int d8_check_status(const void *ws, void *stream)
{
    if (!ws) return D8_EINVAL;
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess) return D8_EHIP;
    uint32_t s = 0;
    if (hipMemcpy(&s, ws, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess) return D8_EHIP;
    if (s == kStatusDirCode) return D8_EDIRCODE;
    if (s == kStatusCycle) return D8_ECYCLE;
    return D8_OK;
}

}  // extern "C"
