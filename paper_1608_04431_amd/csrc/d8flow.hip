// d8flow.hip -- host side of libd8flow: argument checks, workspace layout,
// launch sequences of the C ABI declared in include/d8flow.h.
#include "d8flow.h"

#include <hip/hip_runtime.h>

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
constexpr int kNodeBlock = 256;

struct Layout {
    size_t status, jstate, link, entry, succ, indeg, val32, acc64, ext64, ptr2, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

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
    L.total = off;
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
bool g_timing_on = false;
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

struct LaunchTimer {
    const char *name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    LaunchTimer(const char *n, hipStream_t s) : name(n), st(s)
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        if (g_timing_on) {
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
    uint32_t *cnt = kCounts ? nullptr : reinterpret_cast<uint32_t *>(ws + L.ptr2);
    T *aloc = reinterpret_cast<T *>(ws + L.val32);
    V *acc = reinterpret_cast<V *>(ws + L.acc64);
    E *ext = reinterpret_cast<E *>(ws + L.ext64);

    int ntiles = g.nty * g.ntx;
    const int thr = kTileThreads;
    size_t lds1 = walk_lds_bytes(g.th, g.tw, kWalkFwd1, (int)sizeof(FwdLds<1, T>));
    size_t lds2 = walk_lds_bytes(g.th, g.tw, kWalkFwd2, (int)sizeof(FwdLds<2, T>));
    if (allow_lds(fwd_walk<1, T, V, E>, lds1) || allow_lds(fwd_walk<2, T, V, E>, lds2))
        return D8_EHIP;

    init_state<<<1, 1, 0, st>>>(status, jstate);
    unsigned nb = blocks_for(g.nnodes, kNodeBlock);
    D8_LAUNCH("fwd_pass1", st,
              (fwd_walk<1, T, V, E><<<ntiles, thr, lds1, st>>>(dirs, w, g, link, aloc, indeg, cnt,
                                                               acc, ext, nullptr, status)));
    D8_LAUNCH("graph_build", st,
              (graph_build<<<nb, kNodeBlock, 0, st>>>(dirs, g, link, entry, succ, indeg)));
    if constexpr (kCounts) {
        D8_LAUNCH("resolve_fwd", st,
                  (resolve_fwd_u32<<<nb, kNodeBlock, 0, st>>>(g, link, aloc, entry, succ, indeg, acc,
                                                              ext)));
    } else {
        D8_LAUNCH("resolve_fwd", st,
                  (resolve_fwd_f64<T><<<nb, kNodeBlock, 0, st>>>(g, link, aloc, entry, succ, indeg,
                                                                 cnt, acc, ext)));
    }
    D8_LAUNCH("fwd_pass2", st,
              (fwd_walk<2, T, V, E><<<ntiles, thr, lds2, st>>>(dirs, w, g, link, aloc, indeg, cnt,
                                                               acc, ext, out, status)));
    return last_error();
}

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
    if (rows < 0 || cols < 0) return D8_EINVAL;
    if (rows == 0 || cols == 0) return D8_OK;
    if (!dem || !dirs) return D8_EINVAL;
    begin_call();
    dim3 block(64, 4);
    int64_t gx = (cols + 63) / 64, gy = (rows + 3) / 4;
    if (gx > INT_MAX || gy > 65535) {
        // very tall rasters: one launch per band of rows
        for (int64_t r0 = 0; r0 < rows; r0 += 65535 * 4) {
            int64_t nr = rows - r0 < 65535 * 4 ? rows - r0 : 65535 * 4;
            dim3 grid((unsigned)gx, (unsigned)((nr + 3) / 4));
            d8_kernel<<<grid, block, 0, as_stream(stream)>>>(dem + r0 * cols, dirs + r0 * cols, nr,
                                                             cols, nodata);
        }
        return last_error();
    }
    D8_LAUNCH("d8_directions", as_stream(stream),
              (d8_kernel<<<dim3((unsigned)gx, (unsigned)gy), block, 0, as_stream(stream)>>>(
                  dem, dirs, rows, cols, nodata)));
    return last_error();
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
    if (!ws) return D8_EWORKSPACE;
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
    if (!ws) return D8_EWORKSPACE;
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
    uint32_t *entry = reinterpret_cast<uint32_t *>(w8 + L.entry);
    uint32_t *succ = reinterpret_cast<uint32_t *>(w8 + L.succ);
    float *S = reinterpret_cast<float *>(w8 + L.val32);
    unsigned long long *jw[2] = {reinterpret_cast<unsigned long long *>(w8 + L.acc64),
                                 reinterpret_cast<unsigned long long *>(w8 + L.ext64)};

    int ntiles = g.nty * g.ntx;
    const int thr = kTileThreads;
    size_t lds1 = walk_lds_bytes(g.th, g.tw, kWalkAdj1), lds2 = walk_lds_bytes(g.th, g.tw, kWalkAdj2);
    begin_call();
    if (allow_lds(adj_walk<1>, lds1) || allow_lds(adj_walk<2>, lds2)) return D8_EHIP;
    unsigned nb = blocks_for(g.nnodes, kNodeBlock);

    init_state<<<1, 1, 0, st>>>(status, jstate);
    D8_LAUNCH("adj_pass1", st,
              (adj_walk<1><<<ntiles, thr, lds1, st>>>(dirs, grad_acc, g, link, S, nullptr, nullptr,
                                                      jstate, nullptr, status)));
    D8_LAUNCH("graph_build", st,
              (graph_build<<<nb, kNodeBlock, 0, st>>>(dirs, g, link, entry, succ, nullptr)));
    D8_LAUNCH("adj_jump_init", st,
              (adj_jump_init<<<nb, kNodeBlock, 0, st>>>(g, link, entry, succ, S, jw[0], jw[1])));
    int rounds = 1;
    while (((int64_t)1 << (rounds - 1)) <= g.nnodes) ++rounds;
    for (int r = 0; r < rounds; ++r)
        D8_LAUNCH("adj_jump_round", st,
                  (adj_jump_round<<<nb, kNodeBlock, 0, st>>>(g, jw[r & 1], jw[(r + 1) & 1], jstate,
                                                             r)));
    D8_LAUNCH("adj_jump_finish", st, (adj_jump_finish<<<1, 1, 0, st>>>(jstate, rounds, status)));
    D8_LAUNCH("adj_pass2", st,
              (adj_walk<2><<<ntiles, thr, lds2, st>>>(dirs, grad_acc, g, link, nullptr, jw[0],
                                                      jw[1], jstate, grad_weights, status)));
    return last_error();
}

const char *d8_last_error_message(void) { return g_last_error.c_str(); }

int d8_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_on = on != 0;
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
