/*
 * mandel.h -- C ABI of libmandel.so, the gfx950 escape-time Mandelbrot library.
 *
 * What is computed (Gamage & Baskaran, "Efficient Generation of Mandelbrot Set
 * using Message Passing Interface", Sec. I, Eq. (1) and Eq. (2)): for every
 * pixel (i, j) of an m x n image, z <- z^2 + c is iterated from z = 0, and the
 * iteration at which |z|^2 first exceeds R^2, or max_iter if that never
 * happens, is stored as a 32-bit count.  The arithmetic is IEEE binary64 with
 * one rounding per operation in this fixed order:
 *     x' = (x*x - y*y) + cx,   y' = 2*(x*y) + cy,   escape iff x'*x' + y'*y' > R*R
 * so that counts are reproducible bit for bit on any conforming machine.
 * Every schedule (Sec. III: naive rows, first-come-first-served, alternating
 * rows; and the tile orders below) yields the same image, because pixels are
 * independent (Sec. II-A, Bernstein's conditions).
 *
 * Conventions for every entry point:
 *   - Pointers named "device" are HIP device pointers on the current device;
 *     "host" pointers are read during the call only.  The library never frees
 *     caller memory.
 *   - stream is a hipStream_t (NULL = the legacy default stream).  Calls
 *     enqueue work and return; results are valid once the stream is
 *     synchronised.  Calls on the same stream run in order; the library keeps
 *     one small workspace (queue head, counters) per (device, stream).
 *   - Return value: MANDEL_OK (0) or a negative code.  On error nothing is
 *     enqueued, and mandel_last_error() returns a description (thread-local).
 *     No C++ exception crosses this interface.
 */
#ifndef MANDEL_H
#define MANDEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MANDEL_OK 0
#define MANDEL_EINVAL (-1) /* bad argument: null pointer, bad size, non-finite value */
#define MANDEL_ENOMEM (-2) /* device or host allocation failed */
#define MANDEL_EHIP (-3)   /* HIP runtime error (launch, copy, graph) */

/*
 * The complex window.  Pixel (i, j) (row i, column j) of an m x n view maps to
 *     cx = cx0 + ((j + 0.5) - n/2) * dx,    cy = cy0 + ((i + 0.5) - m/2) * dy
 * (pixel centres; the bracket is an exact half-integer, then one rounded
 * multiply and one rounded add).  Row i has imaginary part growing with i.
 * Requirements: all four finite, dx > 0, dy > 0, and the corner points finite.
 */
typedef struct mandel_window {
    double cx0, cy0; /* centre of the view */
    double dx, dy;   /* pixel pitch: real part per column, imaginary part per row */
} mandel_window;

/*
 * mandel_render -- the plain entry point: one view, persistent kernel, tiles of
 * 64 x 8 pixels claimed first-come-first-served from a device queue (the
 * device analogue of Sec. III-B).
 *   w        host, the window (see above)
 *   m, n     rows and columns; m == 0 or n == 0 is an empty image (no work,
 *            out may be NULL); negative sizes or m*n >= 2^40 are EINVAL
 *   max_iter iterationMax, 1 <= max_iter <= 2^30
 *   R        escape radius, finite, 0 < R <= 1e150
 *   out      device int32[m*n], row-major, out[i*n + j]; fully overwritten
 * Every count lies in [1, max_iter].
 */
int mandel_render(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter,
                  double R, int32_t *out, void *stream);

/* Work partitions of the kernel family (one kernel template, five sources of work). */
enum mandel_policy {
    /* Sec. III-B, first come first served: a device-wide atomic queue of tiles,
     * claimed `grain` at a time by each wavefront. */
    MANDEL_FCFS_TILES = 0,
    /* Sec. III-A, naive rows: worker r of W (a workgroup) owns rows
     * S_r = floor(m/W)*r .. floor(m/W)*(r+1)-1; the last worker also owns the
     * m mod W leftover rows.  The waves of a worker share its rows. */
    MANDEL_STATIC_ROWS = 1,
    /* Sec. III-C, alternating rows: worker r owns rows r, r+W, r+2W, ...
     * (floor(m/W) of them); worker 0 also owns the leftover rows. */
    MANDEL_ALTERNATING_ROWS = 2,
    /* FCFS over a caller-given permutation of tile ids (e.g. longest
     * predicted first): slot q of the queue renders tile order[q]. */
    MANDEL_ORDERED_TILES = 3,
    /* Non-persistent reference launch: one workgroup per tile, no queue. */
    MANDEL_GRID_TILES = 4
};

/* Per-call schedule; zero-initialised fields take the defaults in brackets. */
typedef struct mandel_sched {
    int32_t policy;          /* enum mandel_policy [FCFS_TILES] */
    int32_t tile_w, tile_h;  /* tile shape in pixels for tile policies [64, 8] */
    int32_t grain;           /* tiles per queue claim [1] */
    int32_t workers;         /* row policies: W workgroups (required >= 1);
                                tile policies: persistent workgroups [fill device] */
    int32_t waves_per_group; /* wavefronts per workgroup, 1..16 [4] */
    int32_t check_every;     /* 1 = test |z|^2 > R^2 after every update only;
                                0 = also allow deferred blocks of tests [0] */
    int32_t block_iters;     /* longest deferred-test block K, 1..1024 [256] */
    int32_t young_iters;     /* pixels younger than this are tested every update [8] */
    int32_t reserved;
    const int32_t *order;    /* device int32[ntiles], ORDERED_TILES only: a permutation */
    int64_t *tile_cost;      /* device int64[ntiles] or NULL: sum of counts per tile
                                (tile policies; cleared by the call) */
    int32_t *claims;         /* device int32[ntiles] or NULL: times each tile was
                                claimed (tile policies; cleared by the call) */
    uint64_t *stats;         /* device uint64[4] or NULL, accumulated (not cleared):
                                [0] wavefront loop iterations, [1] sum of counts,
                                [2] wavefronts that ran, [3] work items taken */
} mandel_sched;

/*
 * mandel_render_sched -- mandel_render with an explicit schedule.  Same
 * arguments and guarantees; the image is identical for every valid schedule.
 * Tiles are numbered row-major over the ceil(m/tile_h) x ceil(n/tile_w) tile
 * grid; edge tiles are clipped to the image.
 */
int mandel_render_sched(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter,
                        double R, int32_t *out, const mandel_sched *s, void *stream);

/* Number of tiles of an m x n view under a tile shape (0 for an empty view). */
int64_t mandel_tile_count(int32_t m, int32_t n, int32_t tile_w, int32_t tile_h);

/* Text of the last error on this thread ("" if none). */
const char *mandel_last_error(void);

/* Library version string. */
const char *mandel_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MANDEL_H */
