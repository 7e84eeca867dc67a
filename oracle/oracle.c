/*
 * oracle.c -- plain, serial CPU oracle for D8 flow accumulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library; the two are independent
 * implementations of the same definitions.
 *
 * Everything here is deliberately simple: one thread, no blocking, no fusion,
 * 64-bit integers for unit counts and IEEE double for weighted sums.
 *
 * Direction codes (the paper fixes one byte per cell with ten distinct values,
 * Section "Data Types", but not their encoding; this reading is ours):
 *   0 NW, 1 N, 2 NE, 3 W, 4 E, 5 SW, 6 S, 7 SE  (3x3 scan order without the
 *   centre, so the opposite of k is 7-k), 8 NoFlow, 9 NoData, 10..255 invalid.
 *
 * Return codes: 0 ok, -4 invalid direction code, -5 cycle, -6 overflow,
 * -7 allocation failure, -1 bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_NOFLOW 8
#define OR_NODATA 9
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EDIRCODE (-4)
#define OR_ECYCLE (-5)
#define OR_EOVERFLOW (-6)
#define OR_ENOMEM (-7)

static const int OR_DR[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
static const int OR_DC[8] = {-1, 0, 1, -1, 1, -1, 0, 1};

/* ------------------------------------------------------------------ D8 --- */
/*
 * D8 flow directions (O'Callaghan & Mark 1984, cited by the paper as its
 * non-divergent example in the Introduction; the paper itself treats the
 * direction algorithm as a black box).  Reading used here:
 *   - a cell is NoData if z == nodata or z is NaN (code 9);
 *   - candidates are in-grid, non-NoData neighbours with a strictly positive
 *     float32 drop d = z_c - z_n;
 *   - slope is d / 1 for the four cardinal neighbours and d / sqrt(2) for the
 *     diagonals; comparing squared slopes times two (2 d^2 vs d^2) in double
 *     is exact because a float32 squared fits in a double;
 *   - the largest key wins; equal keys keep the lowest neighbour index;
 *   - no candidate: NoFlow (code 8).
 */
int orc_d8(const float *z, uint8_t *dirs, int64_t rows, int64_t cols, float nodata)
{
    if (rows < 0 || cols < 0) return OR_EINVAL;
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t c = 0; c < cols; ++c) {
            float zc = z[r * cols + c];
            if (zc == nodata || isnan(zc)) { dirs[r * cols + c] = OR_NODATA; continue; }
            int best = OR_NOFLOW;
            double best_key = 0.0;
            for (int k = 0; k < 8; ++k) {
                int64_t rr = r + OR_DR[k], cc = c + OR_DC[k];
                if (rr < 0 || rr >= rows || cc < 0 || cc >= cols) continue;
                float zn = z[rr * cols + cc];
                if (zn == nodata || isnan(zn)) continue;
                volatile float d = zc - zn; /* float32 drop, rounded once */
                if (!(d > 0.0f)) continue;
                double dd = (double)d;
                int cardinal = (OR_DR[k] == 0 || OR_DC[k] == 0);
                double key = cardinal ? 2.0 * dd * dd : dd * dd;
                if (key > best_key) { best_key = key; best = k; }
            }
            dirs[r * cols + c] = (uint8_t)best;
        }
    }
    return OR_OK;
}

/*
 * rho8 directions (Fairfield and Leymarie, 1991), which the paper's
 * Introduction names beside D8 as a non-divergent flow metric: as D8, but the
 * distance to a diagonal neighbour is t = fl32(2 - r) with r in [0, 1) drawn
 * once per cell (given in rnd), instead of sqrt 2 -- so the diagonal factor
 * 1 / t lies in (1/2, 1] with mean ln 2, near 1 / sqrt 2.  The steepest slope
 * d / dist over the strictly lower data neighbours wins, the lowest index on
 * ties; two slopes are compared exactly as d1 * dist2 against d2 * dist1 in
 * double (each product of two floats is exact).
 */
int orc_rho8(const float *z, const float *rnd, uint8_t *dirs, int64_t rows, int64_t cols,
             float nodata)
{
    if (rows < 0 || cols < 0) return OR_EINVAL;
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t c = 0; c < cols; ++c) {
            const int64_t i = r * cols + c;
            float zc = z[i];
            if (zc == nodata || isnan(zc)) { dirs[i] = OR_NODATA; continue; }
            volatile float t = 2.0f - rnd[i];
            int best = OR_NOFLOW;
            double best_d = 0.0, best_dist = 1.0;
            for (int k = 0; k < 8; ++k) {
                int64_t rr = r + OR_DR[k], cc = c + OR_DC[k];
                if (rr < 0 || rr >= rows || cc < 0 || cc >= cols) continue;
                float zn = z[rr * cols + cc];
                if (zn == nodata || isnan(zn)) continue;
                volatile float d = zc - zn;
                if (!(d > 0.0f)) continue;
                double dist = (OR_DR[k] == 0 || OR_DC[k] == 0) ? 1.0 : (double)t;
                if ((double)d * best_dist > best_d * dist) {
                    best = k;
                    best_d = (double)d;
                    best_dist = dist;
                }
            }
            dirs[i] = (uint8_t)best;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------- flow graph --- */
/*
 * The receiver of a cell, from Eq. (1) with alpha in {0,1}: a data cell with
 * code k in 0..7 sends all of its flow to the neighbour in direction k, if that
 * neighbour is inside the raster and is not NoData.  Otherwise (NoFlow, or a
 * direction leaving the raster or entering NoData) the cell is an outlet.
 * Algorithm 1 skips exactly these cases when it counts dependencies.
 * Returns the receiver's index, -1 for none, or -2 for an invalid code.
 */
static int64_t receiver(const uint8_t *dirs, int64_t rows, int64_t cols, int64_t i)
{
    uint8_t k = dirs[i];
    if (k > OR_NODATA) return -2;
    if (k >= OR_NOFLOW) return -1;
    int64_t r = i / cols + OR_DR[k], c = i % cols + OR_DC[k];
    if (r < 0 || r >= rows || c < 0 || c >= cols) return -1;
    int64_t j = r * cols + c;
    if (dirs[j] == OR_NODATA) return -1;
    if (dirs[j] > OR_NODATA) return -2;
    return j;
}

int orc_receivers(const uint8_t *dirs, int64_t rows, int64_t cols, int64_t *recv)
{
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i) {
        if (dirs[i] > OR_NODATA) return OR_EDIRCODE;
        recv[i] = (dirs[i] == OR_NODATA) ? -1 : receiver(dirs, rows, cols, i);
        if (recv[i] == -2) return OR_EDIRCODE;
    }
    return OR_OK;
}

/* ------------------------------------------------------ accumulation --- */
/*
 * Flow accumulation, Eq. (1): A(p) = w(p) + sum over donors n of A(n),
 * computed by the dependency-count (Kahn) order of Algorithm 1 applied to the
 * whole raster as one tile:
 *   1. D(c) = number of data cells whose receiver is c;
 *   2. every data cell with D = 0 is put in a first-in first-out queue, in
 *      row-major order;
 *   3. pop c, add its own weight to A(c); if c has a receiver r, add A(c) to
 *      A(r), decrement D(r) and queue r when D(r) reaches 0.
 * NoData cells hold 0.  If fewer cells are popped than there are data cells
 * the directions contain a cycle (-5).  `order` (optional) receives the pop
 * order, a topological order of the flow forest; *n_order its length.
 *
 * Weights: `w64` (integer, may be NULL for unit weights) for the u64 variant;
 * `w32` (float32) or `wd` (double), both NULL for unit, for the double variant.
 */
static int kahn(const uint8_t *dirs, int64_t rows, int64_t cols, const uint64_t *w64,
                const float *w32, const double *wd, uint64_t *A64, double *Af, int64_t *order,
                int64_t *n_order)
{
    int64_t n = rows * cols;
    if (rows < 0 || cols < 0) return OR_EINVAL;
    uint8_t *D = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *q = order ? order : (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!D || !q) { free(D); if (!order) free(q); return OR_ENOMEM; }
    int64_t n_valid = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (dirs[i] > OR_NODATA) { free(D); if (!order) free(q); return OR_EDIRCODE; }
        if (A64) A64[i] = 0;
        if (Af) Af[i] = 0.0;
        if (dirs[i] == OR_NODATA) continue;
        ++n_valid;
        int64_t r = receiver(dirs, rows, cols, i);
        if (r == -2) { free(D); if (!order) free(q); return OR_EDIRCODE; }
        if (r >= 0) D[r] += 1;
    }
    int64_t head = 0, tail = 0;
    for (int64_t i = 0; i < n; ++i)
        if (dirs[i] != OR_NODATA && D[i] == 0) q[tail++] = i;
    int overflow = 0;
    while (head < tail) {
        int64_t c = q[head++];
        if (A64) {
            uint64_t wc = w64 ? w64[c] : 1u;
            if (A64[c] > UINT64_MAX - wc) overflow = 1;
            A64[c] += wc;
        }
        if (Af) Af[c] += w32 ? (double)w32[c] : (wd ? wd[c] : 1.0);
        int64_t r = receiver(dirs, rows, cols, c);
        if (r < 0) continue;
        if (A64) {
            if (A64[r] > UINT64_MAX - A64[c]) overflow = 1;
            A64[r] += A64[c];
        }
        if (Af) Af[r] += Af[c];
        if (--D[r] == 0) q[tail++] = r;
    }
    if (n_order) *n_order = tail;
    free(D);
    if (!order) free(q);
    if (tail != n_valid) return OR_ECYCLE;
    return overflow ? OR_EOVERFLOW : OR_OK;
}

int orc_accum_u64(const uint8_t *dirs, int64_t rows, int64_t cols, const uint64_t *w,
                  uint64_t *A, int64_t *order, int64_t *n_order)
{
    return kahn(dirs, rows, cols, w, NULL, NULL, A, NULL, order, n_order);
}

int orc_accum_f64(const uint8_t *dirs, int64_t rows, int64_t cols, const float *w, double *A,
                  int64_t *order, int64_t *n_order)
{
    return kahn(dirs, rows, cols, NULL, w, NULL, NULL, A, order, n_order);
}

int orc_accum_f64d(const uint8_t *dirs, int64_t rows, int64_t cols, const double *w, double *A,
                   int64_t *order, int64_t *n_order)
{
    return kahn(dirs, rows, cols, NULL, NULL, w, NULL, A, order, n_order);
}

/*
 * Adjoint (transpose) solve.  Eq. (1) with alpha in {0,1} is linear:
 * A = w + P A, P(p,n) = 1 iff n's receiver is p, so A = (I-P)^-1 w and for a
 * loss L(A) the weight gradient is lambda = (I-P)^-T g with g = dL/dA, i.e.
 * lambda(c) = g(c) + lambda(receiver(c)).  A receiver comes after its donors in
 * a topological (pop) order, so one sweep of that order in reverse computes
 * lambda.  NoData cells hold 0.  `order` must come from orc_accum_*.
 */
int orc_transpose_f64(const uint8_t *dirs, int64_t rows, int64_t cols, const int64_t *order,
                      int64_t n_order, const float *g, double *lam)
{
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i) lam[i] = 0.0;
    for (int64_t t = n_order - 1; t >= 0; --t) {
        int64_t c = order[t];
        int64_t r = receiver(dirs, rows, cols, c);
        if (r == -2) return OR_EDIRCODE;
        lam[c] = (double)g[c] + (r >= 0 ? lam[r] : 0.0);
    }
    return OR_OK;
}

/*
 * Eq. (1) with absorption: alpha(n, p) = alpha(n) in [0, 1] for n's single
 * receiver p (the fraction of n's accumulation that reaches it), so
 * A(p) = w(p) + sum over donors n of alpha(n) A(n).  A cell's accumulation is
 * complete when it is popped in a topological order (from orc_accum_*), so
 * one sweep of that order computes A; its transpose,
 * lambda(c) = g(c) + alpha(c) lambda(receiver(c)), sweeps the order in
 * reverse.  w = NULL means w = 1.  NoData cells hold 0.
 */
int orc_accum_absorb_f64(const uint8_t *dirs, int64_t rows, int64_t cols, const int64_t *order,
                         int64_t n_order, const float *w, const float *alpha, double *A)
{
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i) A[i] = 0.0;
    for (int64_t t = 0; t < n_order; ++t) {
        int64_t c = order[t];
        A[c] += w ? (double)w[c] : 1.0;
    }
    for (int64_t t = 0; t < n_order; ++t) {
        int64_t c = order[t];
        int64_t r = receiver(dirs, rows, cols, c);
        if (r == -2) return OR_EDIRCODE;
        if (r >= 0) A[r] += (double)alpha[c] * A[c];
    }
    return OR_OK;
}

int orc_transpose_absorb_f64(const uint8_t *dirs, int64_t rows, int64_t cols, const int64_t *order,
                             int64_t n_order, const float *g, const float *alpha, double *lam)
{
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i) lam[i] = 0.0;
    for (int64_t t = n_order - 1; t >= 0; --t) {
        int64_t c = order[t];
        int64_t r = receiver(dirs, rows, cols, c);
        if (r == -2) return OR_EDIRCODE;
        lam[c] = (double)g[c] + (r >= 0 ? (double)alpha[c] * lam[r] : 0.0);
    }
    return OR_OK;
}

/*
 * Brute force by path walking (independent of the Kahn order): every data
 * cell y adds w(y) to each cell on its flow path, itself included, so
 * A(x) = sum of w(y) over all y whose path passes x; and lambda(y) is the sum
 * of g over y's path.  O(cells x path length): small rasters only.
 * Returns -5 if a walk exceeds the number of cells (a cycle).
 */
int orc_brute_f64(const uint8_t *dirs, int64_t rows, int64_t cols, const float *w,
                  const float *g, double *A, double *lam)
{
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i) { if (A) A[i] = 0.0; if (lam) lam[i] = 0.0; }
    for (int64_t y = 0; y < n; ++y) {
        if (dirs[y] > OR_NODATA) return OR_EDIRCODE;
        if (dirs[y] == OR_NODATA) continue;
        double wy = w ? (double)w[y] : 1.0, s = 0.0;
        int64_t x = y, steps = 0;
        while (x >= 0) {
            if (++steps > n) return OR_ECYCLE;
            if (A) A[x] += wy;
            if (g) s += (double)g[x];
            x = receiver(dirs, rows, cols, x);
            if (x == -2) return OR_EDIRCODE;
        }
        if (lam) lam[y] = s;
    }
    return OR_OK;
}

int orc_brute_u64(const uint8_t *dirs, int64_t rows, int64_t cols, uint64_t *A)
{
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i) A[i] = 0;
    for (int64_t y = 0; y < n; ++y) {
        if (dirs[y] > OR_NODATA) return OR_EDIRCODE;
        if (dirs[y] == OR_NODATA) continue;
        int64_t x = y, steps = 0;
        while (x >= 0) {
            if (++steps > n) return OR_ECYCLE;
            A[x] += 1;
            x = receiver(dirs, rows, cols, x);
            if (x == -2) return OR_EDIRCODE;
        }
    }
    return OR_OK;
}

/*
 * One value of A, found from its definition alone: breadth-first search over
 * the donors of x (cells whose receiver is x), summing weights.  Cost is the
 * size of x's catchment; used to spot-check rasters too large for a full
 * oracle run.  `w` may be NULL (unit weights).  Returns the sum, or -1 on a
 * cycle / invalid code.
 */
double orc_upstream_sum(const uint8_t *dirs, int64_t rows, int64_t cols, const float *w,
                        int64_t x, int64_t max_cells)
{
    if (dirs[x] >= OR_NODATA) return dirs[x] == OR_NODATA ? 0.0 : -1.0;
    int64_t cap = 1024, head = 0, tail = 0;
    int64_t *q = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    if (!q) return -1.0;
    double s = 0.0;
    q[tail++] = x;
    while (head < tail) {
        int64_t c = q[head++];
        s += w ? (double)w[c] : 1.0;
        if (head > max_cells) { free(q); return -1.0; }
        int64_t r = c / cols, cc = c % cols;
        for (int k = 0; k < 8; ++k) {
            int64_t nr = r + OR_DR[k], nc = cc + OR_DC[k];
            if (nr < 0 || nr >= rows || nc < 0 || nc >= cols) continue;
            int64_t d = nr * cols + nc;
            if (dirs[d] == OR_NODATA) continue;
            if (receiver(dirs, rows, cols, d) != c) continue;
            if (tail == cap) {
                /* reclaim the consumed prefix before growing */
                memmove(q, q + head, (size_t)(tail - head) * sizeof(int64_t));
                tail -= head; head = 0;
                if (tail == cap) {
                    cap *= 2;
                    int64_t *q2 = (int64_t *)realloc(q, (size_t)cap * sizeof(int64_t));
                    if (!q2) { free(q); return -1.0; }
                    q = q2;
                }
            }
            q[tail++] = d;
        }
    }
    free(q);
    return s;
}

/*
 * One value of the adjoint from its definition: lambda(x) = g(x) + lambda of
 * x's receiver, i.e. the sum of g over x's downstream flow path (x, its
 * receiver, that cell's receiver, ... up to a cell without one).  0 for a
 * NoData cell; -1 for an invalid code or a path longer than max_steps (a
 * cycle).
 */
double orc_downstream_sum(const uint8_t *dirs, int64_t rows, int64_t cols, const float *g,
                          int64_t x, int64_t max_steps)
{
    if (dirs[x] >= OR_NODATA) return dirs[x] == OR_NODATA ? 0.0 : -1.0;
    double s = 0.0;
    for (int64_t steps = 0; x >= 0; ++steps) {
        if (steps > max_steps) return -1.0;
        s += (double)g[x];
        x = receiver(dirs, rows, cols, x);
        if (x == -2) return -1.0;
    }
    return s;
}

/*
 * The same two per-cell definitions with absorption (Eq. (1) with alpha per
 * cell): A(x) is the sum over the cells y of x's catchment of w(y) times the
 * product of alpha over y's path up to x (x excluded), so the catchment
 * search carries that product; lambda(x) sums g along x's downstream path,
 * each term scaled by the product of alpha over the cells before it.
 */
double orc_upstream_sum_absorb(const uint8_t *dirs, int64_t rows, int64_t cols, const float *w,
                               const float *alpha, int64_t x, int64_t max_cells)
{
    if (dirs[x] >= OR_NODATA) return dirs[x] == OR_NODATA ? 0.0 : -1.0;
    int64_t cap = 1024, head = 0, tail = 0;
    int64_t *q = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    double *pr = (double *)malloc((size_t)cap * sizeof(double));
    if (!q || !pr) { free(q); free(pr); return -1.0; }
    double s = 0.0;
    q[tail] = x;
    pr[tail++] = 1.0;
    while (head < tail) {
        int64_t c = q[head];
        double p = pr[head++];
        s += p * (w ? (double)w[c] : 1.0);
        if (head > max_cells) { free(q); free(pr); return -1.0; }
        int64_t r = c / cols, cc = c % cols;
        for (int k = 0; k < 8; ++k) {
            int64_t nr = r + OR_DR[k], nc = cc + OR_DC[k];
            if (nr < 0 || nr >= rows || nc < 0 || nc >= cols) continue;
            int64_t d = nr * cols + nc;
            if (dirs[d] == OR_NODATA) continue;
            if (receiver(dirs, rows, cols, d) != c) continue;
            if (tail == cap) {
                memmove(q, q + head, (size_t)(tail - head) * sizeof(int64_t));
                memmove(pr, pr + head, (size_t)(tail - head) * sizeof(double));
                tail -= head; head = 0;
                if (tail == cap) {
                    cap *= 2;
                    int64_t *q2 = (int64_t *)realloc(q, (size_t)cap * sizeof(int64_t));
                    if (!q2) { free(q); free(pr); return -1.0; }
                    q = q2;
                    double *p2 = (double *)realloc(pr, (size_t)cap * sizeof(double));
                    if (!p2) { free(q); free(pr); return -1.0; }
                    pr = p2;
                }
            }
            q[tail] = d;
            pr[tail++] = p * (double)alpha[d];
        }
    }
    free(q);
    free(pr);
    return s;
}

double orc_downstream_sum_absorb(const uint8_t *dirs, int64_t rows, int64_t cols, const float *g,
                                 const float *alpha, int64_t x, int64_t max_steps)
{
    if (dirs[x] >= OR_NODATA) return dirs[x] == OR_NODATA ? 0.0 : -1.0;
    double s = 0.0, p = 1.0;
    for (int64_t steps = 0; x >= 0; ++steps) {
        if (steps > max_steps) return -1.0;
        s += p * (double)g[x];
        p *= (double)alpha[x];
        x = receiver(dirs, rows, cols, x);
        if (x == -2) return -1.0;
    }
    return s;
}

/* --------------------------------------------- tiled scheme, literally --- */
/*
 * The paper's tiled method (Algorithms 1-3), written out literally, for small
 * rasters.  Tiles are th x tw rectangles in row-major tile order; tiles at the
 * right and bottom edges may be smaller (equal tiles are not required, Section
 * "The Algorithm").  Inside a tile, a neighbour outside the tile is treated as
 * NoData (entry conditions of Algorithm 1).
 *
 * Per tile (Algorithm 1): dependencies D counted from in-tile receivers, a
 * queue of D = 0 cells, and the Kahn loop, giving the intermediate A_loc.
 * Per perimeter cell (Algorithm 2, FollowPath): follow the in-tile flow path;
 * reaching a NoData or NoFlow cell gives FlowTerminates; the first step that
 * leaves the tile (to a neighbouring tile or off the raster) gives
 * FlowExternal if it is the cell itself, else the exit cell e.
 *
 * Global solution (Section "Constructing a Global Solution", Algorithm 3): the
 * perimeter cells of all tiles are the nodes of a flow graph.  Edges: q -> L(q)
 * for a perimeter cell linked to an exit cell; e -> receiver(e) for a
 * FlowExternal cell whose receiver (in a neighbouring tile, across an edge or a
 * corner) is a data cell.  Nodes start with A = A_loc for FlowExternal cells
 * and 0 otherwise; Algorithm 1 is run on the graph, passing A + A' downstream
 * and accumulating incoming flow in the offset A'.
 *
 * Finalising (Section "Broadcasting & Finalizing"): the paper adds offsets
 * along each perimeter cell's downstream path.  Reading taken here: what is
 * added along the in-tile path of perimeter cell q is q's own cross-tile
 * inflow ext(q) = sum of (A + A') over q's graph predecessors in OTHER tiles.
 * (A' of an exit cell also holds the inflow of the perimeter cells linked to
 * it, and those cells' paths already pass through the exit, so adding the whole
 * A' along both would count that inflow twice.)  Then
 *     A(x) = A_loc(x) + sum over perimeter q of this tile whose in-tile path
 *            contains x of ext(q).
 *
 * Outputs (all R x C, row-major; unit weights when w is NULL):
 *   A      final accumulation (must equal the untiled Kahn result);
 *   Aloc   the per-tile intermediate of Algorithm 1;
 *   link   for perimeter cells: the exit cell's raster index, or -1
 *          FlowExternal, -2 FlowTerminates; -3 for interior cells;
 *   ext    cross-tile inflow of perimeter cells (0 elsewhere).
 */
#define LINK_EXTERNAL (-1)
#define LINK_TERMINATES (-2)
#define LINK_INTERIOR (-3)

typedef struct { int64_t r0, c0, h, w; } tile_t;

static int in_tile(const tile_t *t, int64_t r, int64_t c)
{
    return r >= t->r0 && r < t->r0 + t->h && c >= t->c0 && c < t->c0 + t->w;
}

static int on_perimeter(const tile_t *t, int64_t r, int64_t c)
{
    return r == t->r0 || c == t->c0 || r == t->r0 + t->h - 1 || c == t->c0 + t->w - 1;
}

/* the in-tile target of cell i's direction, -1 if none (see above) */
static int64_t tile_receiver(const uint8_t *dirs, int64_t rows, int64_t cols, const tile_t *t,
                             int64_t i, int *leaves_tile)
{
    (void)rows;
    uint8_t k = dirs[i];
    *leaves_tile = 0;
    if (k >= OR_NOFLOW) return -1;
    int64_t r = i / cols + OR_DR[k], c = i % cols + OR_DC[k];
    if (!in_tile(t, r, c)) { *leaves_tile = 1; return -1; }
    int64_t j = r * cols + c;
    if (dirs[j] == OR_NODATA) return -1;
    return j;
}

/* Algorithm 1 on one tile with per-cell weights wt (NULL = 1); writes A over the tile */
static int tile_alg1(const uint8_t *dirs, int64_t rows, int64_t cols, const tile_t *t,
                     const double *wt, double *A, uint8_t *D, int64_t *q)
{
    int lv;
    int64_t nvalid = 0;
    for (int64_t r = t->r0; r < t->r0 + t->h; ++r)
        for (int64_t c = t->c0; c < t->c0 + t->w; ++c) { A[r * cols + c] = 0.0; D[r * cols + c] = 0; }
    for (int64_t r = t->r0; r < t->r0 + t->h; ++r)
        for (int64_t c = t->c0; c < t->c0 + t->w; ++c) {
            int64_t i = r * cols + c;
            if (dirs[i] == OR_NODATA) continue;
            ++nvalid;
            int64_t j = tile_receiver(dirs, rows, cols, t, i, &lv);
            if (j >= 0) D[j] += 1;
        }
    int64_t head = 0, tail = 0;
    for (int64_t r = t->r0; r < t->r0 + t->h; ++r)
        for (int64_t c = t->c0; c < t->c0 + t->w; ++c) {
            int64_t i = r * cols + c;
            if (D[i] == 0 && dirs[i] != OR_NODATA) q[tail++] = i;
        }
    while (head < tail) {
        int64_t c = q[head++];
        A[c] += wt ? wt[c] : 1.0;
        int64_t j = tile_receiver(dirs, rows, cols, t, c, &lv);
        if (j < 0) continue;
        A[j] += A[c];
        if (--D[j] == 0) q[tail++] = j;
    }
    return tail == nvalid ? OR_OK : OR_ECYCLE;
}

/* Algorithm 2 (FollowPath) for perimeter cell c0, with a step guard */
static int64_t follow_path(const uint8_t *dirs, int64_t rows, int64_t cols, const tile_t *t,
                           int64_t c0)
{
    (void)rows;
    int64_t c = c0, steps = 0, limit = t->h * t->w + 1;
    for (;;) {
        if (++steps > limit) return -4; /* cycle */
        uint8_t k = dirs[c];
        if (k >= OR_NOFLOW) return LINK_TERMINATES;
        int64_t r = c / cols + OR_DR[k], cc = c % cols + OR_DC[k];
        if (!in_tile(t, r, cc)) {
            /* leaving the tile (possibly off the raster: the global graph then
               has no edge out of this exit) */
            return c == c0 ? LINK_EXTERNAL : c;
        }
        int64_t n = r * cols + cc;
        if (dirs[n] == OR_NODATA) return LINK_TERMINATES;
        c = n;
    }
}

int orc_tiled(const uint8_t *dirs, int64_t rows, int64_t cols, int64_t th, int64_t tw,
              const float *w, double *A, double *Aloc, int64_t *link, double *ext)
{
    if (th <= 0 || tw <= 0 || rows < 0 || cols < 0) return OR_EINVAL;
    int64_t n = rows * cols;
    for (int64_t i = 0; i < n; ++i)
        if (dirs[i] > OR_NODATA) return OR_EDIRCODE;
    int64_t ty = (rows + th - 1) / th, tx = (cols + tw - 1) / tw;
    double *wt = NULL;
    uint8_t *D = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *q = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    double *Ag = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));  /* graph A  */
    double *Ap = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));  /* graph A' */
    int64_t *gq = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    uint8_t *gD = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    tile_t *tiles = (tile_t *)malloc((size_t)(ty * tx > 0 ? ty * tx : 1) * sizeof(tile_t));
    int rc = OR_OK;
    if (w) {
        wt = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        if (wt) for (int64_t i = 0; i < n; ++i) wt[i] = (double)w[i];
    }
    if (!D || !q || !Ag || !Ap || !gq || !gD || !tiles || (w && !wt)) { rc = OR_ENOMEM; goto done; }
    for (int64_t a = 0; a < ty; ++a)
        for (int64_t b = 0; b < tx; ++b) {
            tile_t *t = &tiles[a * tx + b];
            t->r0 = a * th; t->c0 = b * tw;
            t->h = (t->r0 + th <= rows) ? th : rows - t->r0;
            t->w = (t->c0 + tw <= cols) ? tw : cols - t->c0;
        }
    for (int64_t i = 0; i < n; ++i) { link[i] = LINK_INTERIOR; ext[i] = 0.0; }

    /* stage 1: Algorithm 1 + FollowPath per tile */
    for (int64_t ti = 0; ti < ty * tx; ++ti) {
        const tile_t *t = &tiles[ti];
        if ((rc = tile_alg1(dirs, rows, cols, t, wt, Aloc, D, q)) != OR_OK) goto done;
        for (int64_t r = t->r0; r < t->r0 + t->h; ++r)
            for (int64_t c = t->c0; c < t->c0 + t->w; ++c) {
                if (!on_perimeter(t, r, c)) continue;
                int64_t i = r * cols + c;
                if (dirs[i] == OR_NODATA) { link[i] = LINK_TERMINATES; continue; }
                int64_t L = follow_path(dirs, rows, cols, t, i);
                if (L == -4) { rc = OR_ECYCLE; goto done; }
                link[i] = L;
            }
    }

    /* stage 2: the global flow graph over perimeter cells, solved by a
       modified Algorithm 1 (A = A_loc only for FlowExternal, offsets in A') */
    for (int64_t i = 0; i < n; ++i) {
        if (link[i] == LINK_INTERIOR) continue;
        Ag[i] = (link[i] == LINK_EXTERNAL) ? Aloc[i] : 0.0;
        Ap[i] = 0.0;
    }
    /* successor of a node: the exit cell it links to, or across the tile
       boundary for FlowExternal (edge or corner) */
#define GRAPH_SUCC(i, out)                                                         \
    do {                                                                           \
        (out) = -1;                                                                \
        if (link[i] >= 0) (out) = link[i];                                         \
        else if (link[i] == LINK_EXTERNAL) {                                       \
            uint8_t k_ = dirs[i];                                                  \
            int64_t r_ = (i) / cols + OR_DR[k_], c_ = (i) % cols + OR_DC[k_];      \
            if (r_ >= 0 && r_ < rows && c_ >= 0 && c_ < cols &&                    \
                dirs[r_ * cols + c_] != OR_NODATA)                                 \
                (out) = r_ * cols + c_;                                            \
        }                                                                          \
    } while (0)
    int64_t nnodes = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (link[i] == LINK_INTERIOR) continue;
        ++nnodes;
        int64_t s;
        GRAPH_SUCC(i, s);
        if (s >= 0) gD[s] += 1;
    }
    {
        int64_t head = 0, tail = 0;
        for (int64_t i = 0; i < n; ++i)
            if (link[i] != LINK_INTERIOR && gD[i] == 0) gq[tail++] = i;
        while (head < tail) {
            int64_t u = gq[head++];
            int64_t s;
            GRAPH_SUCC(u, s);
            if (s < 0) continue;
            double flow = Ag[u] + Ap[u];
            Ap[s] += flow;
            /* the part of the inflow that crosses a tile boundary */
            if (link[u] == LINK_EXTERNAL) ext[s] += flow;
            if (--gD[s] == 0) gq[tail++] = s;
        }
        if (tail != nnodes) { rc = OR_ECYCLE; goto done; }
    }
#undef GRAPH_SUCC

    /* stage 3: EVICT -- rerun Algorithm 1 per tile, then add each perimeter
       cell's cross-tile inflow along its in-tile downstream path */
    for (int64_t ti = 0; ti < ty * tx; ++ti) {
        const tile_t *t = &tiles[ti];
        if ((rc = tile_alg1(dirs, rows, cols, t, wt, A, D, q)) != OR_OK) goto done;
        for (int64_t r = t->r0; r < t->r0 + t->h; ++r)
            for (int64_t c = t->c0; c < t->c0 + t->w; ++c) {
                int64_t i = r * cols + c;
                if (link[i] == LINK_INTERIOR || ext[i] == 0.0) continue;
                int64_t x = i;
                int lv;
                while (x >= 0) {
                    A[x] += ext[i];
                    x = tile_receiver(dirs, rows, cols, t, x, &lv);
                }
            }
    }
done:
    free(wt); free(D); free(q); free(Ag); free(Ap); free(gq); free(gD); free(tiles);
    return rc;
}

/* ------------------------------------------------------ path statistics --- */
/*
 * Sizes the GPU kernels' critical paths (not a parity check).  With tiles
 * th x tw, for every data cell:
 *   run(c)   = cells on the longest chain of donors ending at c that stays in
 *              c's tile (the dependency depth the in-tile Kahn loop sees);
 *   cross(c) = most tile-boundary crossings on any flow path ending at c.
 * out[0] = max run, out[1] = max cross, out[2] = perimeter cells,
 * out[3] = exit cells (receiver in another tile), out[4] = entry cells (a
 * donor in another tile), out[5] = longest flow path in cells (any tile).
 */
int orc_path_stats(const uint8_t *dirs, int64_t rows, int64_t cols, int64_t th, int64_t tw,
                   int64_t *out)
{
    int64_t n = rows * cols, no = 0;
    int64_t *order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int32_t *run = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *cross = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *len = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    uint8_t *entry = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!order || !run || !cross || !len || !entry) {
        free(order); free(run); free(cross); free(len); free(entry);
        return OR_ENOMEM;
    }
    uint64_t *A = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    int rc = A ? kahn(dirs, rows, cols, NULL, NULL, NULL, A, NULL, order, &no) : OR_ENOMEM;
    free(A);
    for (int k = 0; k < 6; ++k) out[k] = 0;
    if (rc == OR_OK) {
        for (int64_t t = 0; t < no; ++t) {
            int64_t c = order[t];
            run[c] += 1;
            len[c] += 1;
            if (run[c] > out[0]) out[0] = run[c];
            if (cross[c] > out[1]) out[1] = cross[c];
            if (len[c] > out[5]) out[5] = len[c];
            int64_t r = receiver(dirs, rows, cols, c);
            if (r < 0) continue;
            int same = (c / cols / th == r / cols / th) && (c % cols / tw == r % cols / tw);
            if (same) { if (run[c] > run[r]) run[r] = run[c]; }
            else { entry[r] = 1; out[3] += 1; }
            int32_t cr = cross[c] + (same ? 0 : 1);
            if (cr > cross[r]) cross[r] = cr;
            if (len[c] > len[r]) len[r] = len[c];
        }
        for (int64_t i = 0; i < n; ++i) {
            int64_t r = i / cols, c = i % cols;
            int64_t lr = r % th, lc = c % tw;
            int64_t h = (r / th * th + th <= rows) ? th : rows - r / th * th;
            int64_t w = (c / tw * tw + tw <= cols) ? tw : cols - c / tw * tw;
            if (lr == 0 || lc == 0 || lr == h - 1 || lc == w - 1) out[2] += 1;
            out[4] += entry[i];
        }
    }
    free(order); free(run); free(cross); free(len); free(entry);
    return rc;
}
