/*
 * synth.c -- seeded synthetic terrain for the flow-accumulation workloads.
 *
 * This file prepares INPUTS only.  It holds none of the flow-accumulation
 * method: no flow directions, no accumulation.  Both the CPU oracle and the
 * GPU library consume what it writes.
 *
 * What it makes (the paper's own datasets, SRTM / NED / PAMAP, are not
 * available; these rasters stand in for them):
 *   - multi-octave value noise plus a planar tilt (a drainage network with
 *     ridges, valleys and closed depressions);
 *   - optional "ocean" discs of NoData (irregular coastlines);
 *   - a Priority-Flood + epsilon depression fill, so every data cell has a
 *     strictly lower neighbour or is on the border / coast.  The paper
 *     (Introduction) names depression filling by Priority-Flood as the usual
 *     preparation before flow directions are computed; the fill itself is not
 *     part of the accumulation method.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based
 * hash of (seed, octave, lattice row, lattice column).
 *
 * Elevations are quantised to integer millimetres before the fill, so the
 * fill's epsilon is exactly 1 mm and the priority queue is a monotone bucket
 * queue (pops in (elevation, push order) order).  The result is written back
 * as float32 metres.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#define SYN_NODATA (-9999.0f)

/* large arrays are accessed along elevation contours, not rows: back them with
   transparent huge pages where the kernel allows it, to keep TLB misses down */
static void *big_alloc(size_t bytes, int zero)
{
    void *p = NULL;
    size_t align = (size_t)2 << 20;
    size_t sz = (bytes + align - 1) / align * align;
    if (sz == 0) sz = align;
    if (posix_memalign(&p, align, sz) != 0) return NULL;
#ifdef MADV_HUGEPAGE
    madvise(p, sz, MADV_HUGEPAGE);
#endif
    if (zero) memset(p, 0, sz);
    return p;
}

static inline uint64_t sm64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform double in [0,1) from the top 53 bits of a hash */
static inline double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

static inline double lattice(uint64_t seed, int o, int64_t i, int64_t j)
{
    uint64_t h = sm64(sm64(sm64(sm64(seed) ^ (uint64_t)o) ^ (uint64_t)i) ^ (uint64_t)j);
    return 2.0 * u01(h) - 1.0;
}

static inline double fade(double t) { return t * t * (3.0 - 2.0 * t); }

/*
 * z(r,c) = amp * sum_o a_o * n_o(r,c) + tilt * c,
 * a_o = 2^-o / sum_k 2^-k, n_o value noise with lattice spacing lambda0*2^-o.
 * Writes float32 metres.
 */
void syn_value_noise(float *z, int64_t rows, int64_t cols, uint64_t seed, double lambda0,
                     int octaves, double amp, double tilt)
{
    double norm = 0.0;
    for (int k = 0; k < octaves; ++k) norm += ldexp(1.0, -k);
#pragma omp parallel
    {
        /* per-thread scratch: the two lattice rows bracketing the current raster row */
        int64_t maxlat = cols + 3;
        double *row0 = (double *)malloc((size_t)maxlat * sizeof(double));
        double *row1 = (double *)malloc((size_t)maxlat * sizeof(double));
        double *acc = (double *)malloc((size_t)(cols > 0 ? cols : 1) * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            for (int64_t c = 0; c < cols; ++c) acc[c] = 0.0;
            for (int o = 0; o < octaves; ++o) {
                double lam = lambda0 * ldexp(1.0, -o);
                if (lam < 1.0) lam = 1.0;
                double y = (double)r / lam;
                int64_t i0 = (int64_t)floor(y);
                double fy = fade(y - (double)i0), wo = ldexp(1.0, -o) / norm;
                int64_t nlat = (int64_t)floor((double)(cols - 1) / lam) + 2;
                for (int64_t j = 0; j < nlat; ++j) {
                    row0[j] = lattice(seed, o, i0, j);
                    row1[j] = lattice(seed, o, i0 + 1, j);
                }
                for (int64_t c = 0; c < cols; ++c) {
                    double x = (double)c / lam;
                    int64_t j0 = (int64_t)floor(x);
                    double fx = fade(x - (double)j0);
                    double top = row0[j0] + (row0[j0 + 1] - row0[j0]) * fx;
                    double bot = row1[j0] + (row1[j0 + 1] - row1[j0]) * fx;
                    acc[c] += wo * (top + (bot - top) * fy);
                }
            }
            for (int64_t c = 0; c < cols; ++c)
                z[r * cols + c] = (float)(amp * acc[c] + tilt * (double)c);
        }
        free(row0); free(row1); free(acc);
    }
}

/*
 * Ocean discs: draw discs (centre uniform over the raster, radius uniform in
 * [rmin, rmax]) from a counter stream keyed by (seed, "mask") and mark their
 * cells NoData until at least `frac` of the raster is NoData.
 * Returns the number of NoData cells.
 */
int64_t syn_ocean_mask(float *z, int64_t rows, int64_t cols, uint64_t seed, double frac,
                       double rmin, double rmax)
{
    const uint64_t key = sm64(seed ^ 0x6D61736B00000000ULL); /* "mask" */
    int64_t n = rows * cols, masked = 0;
    for (int64_t i = 0; i < n; ++i) masked += (z[i] == SYN_NODATA);
    int64_t target = (int64_t)ceil(frac * (double)n);
    for (uint64_t k = 0; masked < target; ++k) {
        double r0 = floor(u01(sm64(key + 3 * k + 0)) * (double)rows);
        double c0 = floor(u01(sm64(key + 3 * k + 1)) * (double)cols);
        double rad = rmin + (rmax - rmin) * u01(sm64(key + 3 * k + 2));
        int64_t ra = (int64_t)ceil(rad);
        int64_t rlo = (int64_t)r0 - ra, rhi = (int64_t)r0 + ra;
        if (rlo < 0) rlo = 0;
        if (rhi > rows - 1) rhi = rows - 1;
        for (int64_t r = rlo; r <= rhi; ++r) {
            double dr = (double)r - r0;
            for (int64_t c = (int64_t)c0 - ra; c <= (int64_t)c0 + ra; ++c) {
                if (c < 0 || c >= cols) continue;
                double dc = (double)c - c0;
                if (dr * dr + dc * dc <= rad * rad) {
                    float *p = &z[r * cols + c];
                    if (*p != SYN_NODATA) { *p = SYN_NODATA; ++masked; }
                }
            }
        }
    }
    return masked;
}

/* neighbour offsets in the fixed order NW, N, NE, W, E, SW, S, SE */
static const int DR[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
static const int DC[8] = {-1, 0, 1, -1, 1, -1, 0, 1};

/*
 * Priority-Flood + epsilon on integer elevations (eps = 1 unit).
 *   zi:   elevations, modified in place; NODATA_I marks NoData (never touched)
 *   seeds: every data cell on the raster border or with a NoData 8-neighbour,
 *          pushed in row-major order with its own elevation
 *   pop order: increasing elevation, first-in first-out among equals
 *   on pop of c, each in-grid, data, unvisited neighbour n (order NW..SE) is
 *   marked visited; if zi[n] <= zi[c] it is raised to zi[c] + eps; then pushed.
 * Every push lands in a bucket strictly above the one being popped, so a bucket
 * is complete when it is reached and one per-cell link array suffices.
 * Returns 0, or -1 on allocation failure.
 */
#define NODATA_I INT32_MIN
int syn_fill_int(int32_t *zin, int64_t rows, int64_t cols, int32_t eps)
{
    int64_t n = rows * cols;
    if (n == 0) return 0;
    /* Work on a padded copy: a one-cell frame around the raster and a row
       stride that is not a power of two (contours often run down columns, and
       power-of-two strides would map a column walk onto a few cache sets). */
    int64_t ps = cols + 2 + 24;
    int64_t np = (rows + 2) * ps;
    if (np > (int64_t)UINT32_MAX - 1) return -1;
    int32_t zmin = INT32_MAX, zmax = INT32_MIN;
    for (int64_t i = 0; i < n; ++i) {
        if (zin[i] == NODATA_I) continue;
        if (zin[i] < zmin) zmin = zin[i];
        if (zin[i] > zmax) zmax = zin[i];
    }
    if (zmin > zmax) return 0; /* all NoData */
    /* state: 0 = data, not yet reached; 1 = data, reached; 2 = frame or NoData */
    uint8_t *state = (uint8_t *)big_alloc((size_t)np, 0);
    int32_t *zi = (int32_t *)big_alloc((size_t)np * sizeof(int32_t), 0);
    uint32_t *next = (uint32_t *)big_alloc((size_t)np * sizeof(uint32_t), 0);
    int64_t nb = (int64_t)zmax - zmin + 2 + 1024;
    uint32_t *head = (uint32_t *)malloc((size_t)nb * sizeof(uint32_t));
    uint32_t *tail = (uint32_t *)malloc((size_t)nb * sizeof(uint32_t));
    if (!state || !zi || !next || !head || !tail) {
        free(state); free(zi); free(next); free(head); free(tail);
        return -1;
    }
    memset(state, 2, (size_t)np);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c) {
            int64_t p = (r + 1) * ps + (c + 1);
            zi[p] = zin[r * cols + c];
            state[p] = (zi[p] == NODATA_I) ? 2 : 0;
        }
    const int64_t off[8] = {-ps - 1, -ps, -ps + 1, -1, 1, ps - 1, ps, ps + 1};
    const uint32_t NIL = UINT32_MAX;
    for (int64_t b = 0; b < nb; ++b) head[b] = tail[b] = NIL;

#define PUSH(idx, zz)                                                                    \
    do {                                                                                 \
        int64_t b_ = (int64_t)(zz) - zmin;                                               \
        if (b_ >= nb) {                                                                  \
            int64_t nb2 = b_ + 1 + nb / 2;                                               \
            uint32_t *h2 = (uint32_t *)realloc(head, (size_t)nb2 * sizeof(uint32_t));    \
            if (!h2) goto oom;                                                           \
            head = h2;                                                                   \
            uint32_t *t2 = (uint32_t *)realloc(tail, (size_t)nb2 * sizeof(uint32_t));    \
            if (!t2) goto oom;                                                           \
            tail = t2;                                                                   \
            for (int64_t q_ = nb; q_ < nb2; ++q_) head[q_] = tail[q_] = NIL;             \
            nb = nb2;                                                                    \
        }                                                                                \
        next[idx] = NIL;                                                                 \
        if (tail[b_] == NIL) head[b_] = (uint32_t)(idx);                                 \
        else next[tail[b_]] = (uint32_t)(idx);                                           \
        tail[b_] = (uint32_t)(idx);                                                      \
    } while (0)

    /* seeds, row-major: data cells with a frame or NoData neighbour */
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t c = 0; c < cols; ++c) {
            int64_t p = (r + 1) * ps + (c + 1);
            if (state[p] != 0) continue;
            int seed = 0;
            for (int k = 0; k < 8; ++k) seed |= (state[p + off[k]] == 2);
            if (seed) {
                state[p] = 1;
                PUSH(p, zi[p]);
            }
        }
    }
    for (int64_t b = 0; b < nb; ++b) {
        for (uint32_t i = head[b]; i != NIL; i = next[i]) {
            int32_t zc = zi[i];
            for (int k = 0; k < 8; ++k) {
                int64_t j = (int64_t)i + off[k];
                if (state[j] != 0) continue;
                state[j] = 1;
                if (zi[j] <= zc) zi[j] = zc + eps;
                PUSH(j, zi[j]);
            }
        }
    }
#undef PUSH
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c) zin[r * cols + c] = zi[(r + 1) * ps + (c + 1)];
    free(state); free(zi); free(next); free(head); free(tail);
    return 0;
oom:
    free(state); free(zi); free(next); free(head); free(tail);
    return -1;
}

/*
 * Float metres -> integer millimetres -> fill -> float metres.
 * NoData cells (== SYN_NODATA) stay NoData.  `eps_mm` is the fill epsilon in mm.
 * Returns 0 or -1 (allocation failure / range).
 */
int syn_fill_dem(float *z, int64_t rows, int64_t cols, int32_t eps_mm)
{
    int64_t n = rows * cols;
    int32_t *zi = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!zi) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        zi[i] = (z[i] == SYN_NODATA) ? NODATA_I : (int32_t)llround((double)z[i] * 1000.0);
    int rc = syn_fill_int(zi, rows, cols, eps_mm);
    if (rc == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            z[i] = (zi[i] == NODATA_I) ? SYN_NODATA : (float)((double)zi[i] / 1000.0);
    }
    free(zi);
    return rc;
}
