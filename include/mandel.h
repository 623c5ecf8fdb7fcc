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
 *     one small workspace (a 256-byte queue head and a 32 KiB order histogram)
 *     per (device, stream) it has seen, until the process ends.  Calls that
 *     overlap in time on different streams never share a workspace.
 *   - Return value: MANDEL_OK (0) or a negative code, and mandel_last_error()
 *     returns a description (thread-local).  An invalid argument (-1) or a
 *     failed allocation (-2) enqueues nothing; a HIP runtime error (-3) in the
 *     middle of a sequence of kernels can leave the kernels before it enqueued.
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
#define MANDEL_EIO (-4)    /* host file could not be written */

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

/* mandel_sched.tile_parts: choose the row parts per tile from the image size */
#define MANDEL_TILE_PARTS_AUTO (-1)

/*
 * mandel_render -- the plain entry point: one view, persistent kernel, tiles of
 * 64 x 8 pixels claimed first-come-first-served from a device queue (the
 * device analogue of Sec. III-B), in row parts chosen as MANDEL_TILE_PARTS_AUTO
 * does.
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

/*
 * Deep zoom: the same escape-time count (Sec. I, Eq. (1)-(2)) evaluated in
 * double-double arithmetic, for pixel pitches below binary64 resolution near c
 * (about 1e-16 |c|), where neighbouring pixels would otherwise share one c.
 * Each value is hi + lo of two binary64 numbers; the operations are Knuth's
 * two-sum, Dekker's fast two-sum and the fma-based exact product, combined into
 * the accurate addition and the products of Hida, Li and Bailey:
 *   add(A, B)  (s, e) = two_sum(A.hi, B.hi); (t, f) = two_sum(A.lo, B.lo);
 *              e = e + t; (s, e) = quick_two_sum(s, e); e = e + f;
 *              (s, e) = quick_two_sum(s, e)
 *   sqr(A)     (p, e) = two_prod(A.hi, A.hi); e = fma(A.hi + A.hi, A.lo, e);
 *              quick_two_sum(p, e)
 *   mul(A, B)  (p, e) = two_prod(A.hi, B.hi); e = fma(A.hi, B.lo, e);
 *              e = fma(A.lo, B.hi, e); quick_two_sum(p, e)
 * update: X' = add(add(sqr(X), -sqr(Y)), Cx),  Y' = add(2 mul(X, Y), Cy);
 * a state escapes when fl(fl(X.hi^2) + fl(Y.hi^2)) > R^2; the count is the
 * first escaping k >= 1, else max_iter.  Pixel centre (j, i):
 *   Cx = add((cx0_hi, cx0_lo), two_prod((j + 0.5) - n/2, dx)), likewise Cy.
 * Every operation is one binary64 rounding in this order, so counts are
 * reproducible bit for bit on any IEEE machine with fma.
 */
typedef struct mandel_window_dd {
    double cx0_hi, cx0_lo;   /* real part of the window centre, hi + lo */
    double cy0_hi, cy0_lo;   /* imaginary part of the window centre, hi + lo */
    double dx, dy;           /* pixel pitch (> 0), binary64 */
} mandel_window_dd;

/*
 * mandel_render_dd -- deep-zoom counts of an m x n view into out (device
 * int32[m*n], row-major, fully overwritten) on `stream`; persistent FCFS tile
 * queue of 64 x 8 tiles.  stats: NULL or device uint64[4] accumulated over
 * calls ([0] wavefront steps, [1] sum of counts, [2] wavefronts, [3] tiles).
 * Same argument limits as mandel_render, and every pixel centre must lie within
 * |re|, |im| <= 1e150.  Returns 0, -1 EINVAL (nothing enqueued) or -3 EHIP.
 */
int mandel_render_dd(const mandel_window_dd *w, int32_t m, int32_t n, int32_t max_iter,
                     double R, int32_t *out, uint64_t *stats, void *stream);

/* ---------------------------------------------------------------------------
 * Output path (Sec. III: one process writes the image file; Sec. I with
 * Eq. (2): each pixel's colour follows from its iteration count).
 * ------------------------------------------------------------------------- */

/*
 * mandel_colour_boolean -- Boolean escape-time colouring on the device: pixel p
 * becomes black (0, 0, 0) when counts[p] >= max_iter (it never escaped) and
 * white (255, 255, 255) otherwise.  counts: device int32[npix]; rgb: device
 * uint8[3 * npix], written as R, G, B per pixel in pixel order (the PPM P6
 * layout).  Enqueued on `stream`.  Returns 0, or -1 EINVAL (npix < 0,
 * max_iter < 1, NULL buffer) / -3 EHIP.
 */
int mandel_colour_boolean(const int32_t *counts, int64_t npix, int32_t max_iter, uint8_t *rgb,
                          void *stream);

/*
 * mandel_write_ppm -- writes a binary PPM (P6, maxval 255) of an m-row,
 * n-column image: the header "P6\n<n> <m>\n255\n", then rgb (host memory,
 * 3 * m * n bytes, row-major) as is.  Synchronous host I/O; the file is
 * replaced.  Returns 0, -1 EINVAL, or -4 EIO.
 */
int mandel_write_ppm(const char *path, const uint8_t *rgb, int32_t m, int32_t n);

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
    int32_t block_iters;     /* longest deferred-test block K, 1..65536 [1024] */
    int32_t young_iters;     /* pixels younger than this are tested every update [4] */
    int32_t refill_lanes;    /* while updates are tested one by one, lanes whose pixel
                                finished are refilled once this many are idle; when a
                                block of untested updates ends, once min(this, 8) are
                                idle (or none is active); 1..64 [16] */
    const int32_t *order;    /* device int32[ntiles], ORDERED_TILES only: a permutation */
    int64_t *tile_cost;      /* device int64[ntiles] or NULL: sum of counts per tile
                                (tile policies; cleared by the call) */
    int32_t *claims;         /* NULL, or a log cleared by the call: tile policies,
                                device int32[ntiles], times a non-empty row part of
                                each tile was claimed (min(tile_parts, rows of the
                                tile) when every tile is rendered once);
                                row policies, device int32[m], the sum of (worker + 1)
                                over the takes of each row (a row taken once by
                                worker r holds r + 1) */
    uint64_t *stats;         /* device uint64[8] or NULL.  [0..3] accumulate over
                                calls (never cleared): [0] wavefront loop iterations,
                                [1] sum of counts, [2] wavefronts that ran, [3] work
                                items taken.  [4..6] are set per call, in wall-clock
                                ticks (hipDeviceAttributeWallClockRate): [4] first
                                queue claim (row policies: first row taken), [5]
                                first claim that found the queue empty (row
                                policies: first worker to run out of rows), [6]
                                last wavefront exit; GRID sets only [6].  [7]
                                accumulates the updates skipped by periodicity
                                detection */
    int32_t tile_parts;      /* FCFS / ORDERED: each tile is queued as this many row
                                parts (rows [p*h/parts, (p+1)*h/parts) of an h-row
                                tile), so one expensive tile can be shared by several
                                wavefronts; 1..64, or MANDEL_TILE_PARTS_AUTO: with r
                                the fewest parts that give at least 24 queue items
                                per resident wavefront, the largest power of two not
                                above r, at most 8, halved while a part would hold
                                fewer than 2^20 pixel-iterations at max_iter (unless
                                the queue holds at most 2 items per wavefront), at
                                most tile_h; 1 when the whole window lies outside
                                1.03 R (every pixel escapes at once) (an image of few
                                tiles is then not left to a few wavefronts, and cheap
                                parts do not queue on the head; first_slot must be 0)
                                [1]; GRID ignores it */
    int32_t periodicity;     /* 1: exact periodicity detection (needs check_every 0):
                                in each deferred block the last 32 states of every
                                lane are compared bit for bit with the block-start
                                state; a lane whose state recurs (and did not escape)
                                is on a cycle of non-escaping states and gets
                                max_iter at once.  Every cycle of period <= 32 is
                                found one block after the orbit reaches it, so
                                short blocks (block_iters 64..256) find cycles
                                sooner: on the 8192 x 8192 view at max_iter 10000
                                they take 5.3 ms instead of 7.4 ms at 1024, and
                                4.2 ms with row stealing.  Zooms centred on the
                                boundary gain little (their orbits rarely settle
                                on a short cycle): there short blocks only add
                                their overhead.  Counts are unchanged; stats[7]
                                adds the updates skipped.  0: off [0] */
    int64_t first_slot;      /* FCFS / ORDERED: the queue starts at this slot (slot
                                q renders row part q mod tile_parts of tile q div
                                tile_parts, through `order` for ORDERED); earlier
                                slots are skipped and their pixels left untouched,
                                so a launch can resume after slot k or cover only
                                part of the queue; >= 0 [0]; must be 0 otherwise */
    uint64_t *tile_time;     /* tile policies: NULL, or device uint64[2 * ntiles] cleared
                                by the call: [2t] the first claim of tile t, [2t + 1]
                                the moment its last pixel finished (wall-clock ticks,
                                as stats[4..6]); for tail analysis -- it adds an
                                atomic per pixel.  Must be NULL for row policies. */
} mandel_sched;

/*
 * mandel_render_sched -- mandel_render with an explicit schedule.  Same
 * arguments and guarantees; the image is identical for every valid schedule.
 * Tiles are numbered row-major over the ceil(m/tile_h) x ceil(n/tile_w) tile
 * grid; edge tiles are clipped to the image.
 */
int mandel_render_sched(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter,
                        double R, int32_t *out, const mandel_sched *s, void *stream);

/*
 * mandel_render_sched_noalloc -- mandel_render_sched for callers that cannot
 * allocate device memory (code under stream or graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, checks, results and
 * error codes; it calls no hipMalloc, hipFree or allocating routine.  Its only
 * scratch is the queue head: one 64-bit counter in a 256-byte file-scope device
 * array that every GPU holds once, from the first call on that GPU until the
 * process ends.  That is the whole of its scratch for any image size, so no size
 * is refused for want of scratch (the image limits are mandel_render_sched's).
 * All calls on one GPU share the array, and each call resets the head before its
 * render: calls that overlap in time on one GPU (different streams without
 * synchronisation between them) race and must not be issued; calls in order on
 * one stream are fine.
 */
int mandel_render_sched_noalloc(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter,
                                double R, int32_t *out, const mandel_sched *s, void *stream);

/* Number of tiles of an m x n view under a tile shape (0 for an empty view). */
int64_t mandel_tile_count(int32_t m, int32_t n, int32_t tile_w, int32_t tile_h);

/* ---------------------------------------------------------------------------
 * Batches: many views of different size, zoom and max_iter rendered by ONE
 * persistent launch over one flat tile space (view k's tiles follow view
 * k-1's, each view row-major over its own tile grid).  The paper renders one
 * image per run (Sec. IV); batching is this library's extension of the same
 * per-pixel definition, so every view's image equals mandel_render's.
 * ------------------------------------------------------------------------- */
typedef struct mandel_view {
    mandel_window w;    /* window of this view */
    int32_t m, n;       /* rows, columns (0 allowed: the view has no tiles) */
    int32_t max_iter;   /* 1 .. 2^30 */
    int32_t reserved;
    double R;           /* escape radius, 0 < R <= 1e150 */
    int64_t out_offset; /* element offset of this view's row-major image in out_base */
} mandel_view;

/* Launch shape of a plan; zero fields take the defaults in brackets. */
typedef struct mandel_tuning {
    int32_t tile_w, tile_h;  /* [64, 8] */
    int32_t grain;           /* tiles per queue claim [1] */
    int32_t waves_per_group; /* [4] */
    int32_t block_iters;     /* [1024] */
    int32_t young_iters;     /* [4] */
    int32_t groups;          /* persistent workgroups [fill the device] */
    int32_t refill_lanes;    /* [16], as in mandel_sched */
    int32_t tile_parts;      /* [1], as in mandel_sched; MANDEL_TILE_PARTS_AUTO is
                                resolved at each launch from its grid, with the
                                smallest max_iter of the views (1 for row stealing and
                                the row partitions; launches must then start at
                                first_slot 0) */
    int32_t collapse_rows;   /* 1: render each distinct row coordinate once.  Where a
                                view's pitch dy lies below the spacing of doubles near
                                its centre, neighbouring rows get the same imaginary part
                                (cy0 + ((i + 0.5) - m/2) dy rounds to equal values) and so
                                the same counts.  2: also merge rows whose imaginary parts
                                differ only in sign (conjugate points have equal counts,
                                bit for bit; a window centred on the real axis renders
                                half its rows).  A view with merged rows is rendered as
                                one row per distinct value, each into the image row where
                                the value first occurs, and every other row is then copied
                                from that row (one more kernel per such view after the
                                render, in the same launch).  At most 2^28 rendered and
                                2^28 copied rows over the collapsed views of a plan.
                                The image is identical; tile ids, tile costs, features,
                                statistics and the row partitions (STATIC_ROWS /
                                ALTERNATING_ROWS) then refer to the rendered rows, and
                                first_slot must be 0.  Views whose rows are all distinct
                                are unchanged.  0: off [0] */
} mandel_tuning;

typedef struct mandel_plan mandel_plan;

/*
 * mandel_plan_create -- validates the views (each as mandel_render would),
 * builds the device view table and allocates the plan's queue head.
 *   views   host array [nviews], copied; 1 <= nviews <= 2^24
 *   tuning  host, or NULL for the defaults (see mandel_plan_autotune)
 *   plan    receives the new plan; owned by the caller, freed by
 *           mandel_plan_destroy.  Synchronous (allocates and copies).
 * Output ranges of different views must not overlap (not checked).
 */
int mandel_plan_create(const mandel_view *views, int32_t nviews, const mandel_tuning *tuning,
                       mandel_plan **plan);

/* Plan geometry: total tiles, total pixels, and the tuning in force (any may be NULL). */
int mandel_plan_info(const mandel_plan *plan, int64_t *ntiles, int64_t *npixels,
                     mandel_tuning *tuning);

/* Launch modes of a plan. */
enum mandel_plan_mode {
    MANDEL_PLAN_FCFS = 0,        /* queue in submission order (the fallback) */
    MANDEL_PLAN_ORDERED = 1,     /* queue over the caller's permutation `order` */
    MANDEL_PLAN_PROBE_LPT = 2,   /* probe features -> key = mean probe cost ->
                                    descending order -> ordered render */
    MANDEL_PLAN_LEARNED_LPT = 3, /* probe features -> cost-model MLP -> descending
                                    order -> ordered render */
    /* The paper's row partitions applied to the whole batch as one image: the rows
     * of all views are concatenated (view 0's rows, then view 1's, ...) and the
     * M rows are split over W = `workers` workgroups as MANDEL_STATIC_ROWS
     * (Sec. III-A) or MANDEL_ALTERNATING_ROWS (Sec. III-C) split one image's rows.
     * No queue, order or cost model; tile_cost must be NULL and first_slot 0.
     * Needs fewer than 2^31 rows in the plan. */
    MANDEL_PLAN_STATIC_ROWS = 4,
    MANDEL_PLAN_ALTERNATING_ROWS = 5
};

typedef struct mandel_launch {
    int32_t mode;            /* enum mandel_plan_mode */
    int32_t use_graph;       /* 1: capture the launch sequence once into a hipGraph
                                (keyed by every field below and out_base; each
                                distinct key keeps its graph until
                                mandel_plan_destroy) and replay it; 0: enqueue the
                                kernels directly */
    const int32_t *order;    /* device int32[ntiles], ORDERED: a permutation of tile ids */
    const float *mlp;        /* device float[MANDEL_MLP_PARAMS], LEARNED_LPT: the cost model */
    int64_t *tile_cost;      /* device int64[ntiles] or NULL: sum of counts per tile */
    uint64_t *stats;         /* device uint64[8] or NULL (as in mandel_sched) */
    int32_t probe_cap;       /* PROBE_LPT / LEARNED_LPT: probe iteration cap of the
                                features, absolute (> 0) or a share of each view's
                                max_iter (< 0; see mandel_plan_features) [128]; a
                                model must be used with the cap it was trained with */
    int32_t workers;         /* STATIC_ROWS / ALTERNATING_ROWS: W workgroups of the
                                plan's waves_per_group wavefronts (required >= 1);
                                must be 0 in the other modes */
    int64_t first_slot;      /* queue modes: the render queue starts at this slot, as
                                in mandel_sched [0] */
    int32_t periodicity;     /* 1: exact periodicity detection, as in mandel_sched [0] */
    int32_t reserved;        /* must be 0 */
    uint64_t *tile_time;     /* device uint64[2 * ntiles] or NULL: per-tile first claim
                                and last finished pixel, as in mandel_sched; queue
                                modes only */
    int32_t steal;           /* queue modes with tile_parts 1: 1 = row stealing.  The
                                rows of a claimed tile are taken one at a time through
                                a per-tile counter, and once the queue is empty a
                                wavefront takes untaken rows of tiles that other
                                wavefronts hold (wavefronts of one SIMD issue unevenly,
                                so a tile claimed early can otherwise finish last).
                                Every row is still rendered once; counts, cost logs and
                                statistics are unchanged.  0: off [0] */
    int32_t reserved2;       /* must be 0 */
} mandel_launch;

/*
 * mandel_plan_launch -- renders every view of the plan into out_base (device
 * int32, each view at its out_offset) on `stream`.  All kernels of a launch
 * go to that stream in order.  A plan has one queue: launches of the same
 * plan must not overlap in time (same stream, or synchronise between them).
 * Different plans share nothing and may run concurrently on different streams.
 * The first launch in PROBE_LPT or LEARNED_LPT mode allocates the plan's order
 * buffers (features, keys, permutation: 280 bytes per tile, and a 32 KiB histogram),
 * and the first launch with steal = 1 its row counters and held-tile table
 * (4 bytes per tile and per wavefront), with hipMalloc (synchronous; -2 ENOMEM
 * on failure); they live until mandel_plan_destroy.  Returns 0, or -1 EINVAL /
 * -2 ENOMEM (nothing enqueued) / -3 EHIP.
 */
int mandel_plan_launch(mandel_plan *plan, int32_t *out_base, const mandel_launch *args,
                       void *stream);

/* Frees the plan, its device buffers and its cached graphs (synchronises the device). */
int mandel_plan_destroy(mandel_plan *plan);

/* ---------------------------------------------------------------------------
 * Learned tile ordering.  The paper balances load by handing out rows on
 * demand (Sec. III-B) or interleaving them (Sec. III-C); here the queue order
 * is chosen so that the most expensive tiles start first (longest-processing-
 * time-first list scheduling), using a small FP32 cost model.  The order never
 * changes a count, only when each tile runs.
 * ------------------------------------------------------------------------- */
#define MANDEL_FEATURES 68   /* per-tile features, see mandel_plan_features */
#define MANDEL_HIDDEN 64     /* width of both hidden layers */
/* Parameter vector of the cost model, FP32, in this order:
 *   mu[68], inv_sd[68]     input standardisation x' = (x - mu) * inv_sd (not trained)
 *   W1[64][68], b1[64]     h1 = relu(W1 x' + b1)
 *   W2[64][64], b2[64]     h2 = relu(W2 h1 + b2)
 *   w3[64], b3[1]          y  = w3 . h2 + b3   (predicted ln of the tile's sum of counts)
 * 136 + 8641 floats; the 8641 after the standardisation are trained. */
#define MANDEL_MLP_NORM 136
#define MANDEL_MLP_PARAMS (136 + 64 * 68 + 64 + 64 * 64 + 64 + 64 + 1)

/*
 * mandel_plan_features -- per-tile features, device float[ntiles][68]:
 *   [0], [1]  real and imaginary part of the tile's centre
 *   [2]       log10 of the tile's width in the complex plane (columns * dx)
 *   [3]       ln(max_iter)
 *   [4 + 8r + k], r, k in 0..7: ln(1 + min(count, cap)) / ln(1 + cap) for the
 *             probe pixel at column x0 + floor((k + 0.5) w / 8) and row
 *             y0 + floor((r + 0.5) h / 8) of the (clipped) w x h tile, where
 *             count is that pixel's escape-time count (same definition and
 *             arithmetic as the render) and cap is the view's probe cap:
 *             min(max_iter, probe_cap) for probe_cap > 0, and
 *             max(1, floor(max_iter / k)) for probe_cap = -k (a share of the
 *             view's own limit, so the probes of deep, high-limit views still
 *             tell late escapes from points that never escape).
 *   probe_cap  -2^20 .. 2^20; 0 means 128.
 */
int mandel_plan_features(mandel_plan *plan, float *feat, int32_t probe_cap, void *stream);

/* Cost-model inference: y[i] = model(x[i]) for i < n; x device float[n][68],
 * y device float[n], params device float[MANDEL_MLP_PARAMS]. */
int mandel_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream);

/* Device floats of scratch that mandel_mlp_train_step needs for a minibatch size. */
int64_t mandel_mlp_work_floats(int32_t batch);

/*
 * mandel_mlp_train_step -- one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected with step number t >= 1) on the mean squared error
 *   L = (1/B) sum_b (model(x[idx[b]]) - target[idx[b]])^2
 * over the minibatch idx (device int32[batch], entries in [0, n)).
 *   params, adam_m, adam_v  device float[MANDEL_MLP_PARAMS] (standardisation
 *                           entries are left unchanged), updated in place
 *   x, target               device float[n][68], float[n]
 *   loss                    device float[1] or NULL: L before the update
 *   work                    device float[mandel_mlp_work_floats(batch)]
 *   1 <= batch <= 4096, lr > 0.
 */
int mandel_mlp_train_step(float *params, float *adam_m, float *adam_v, int32_t t,
                          const float *x, const float *target, const int32_t *idx,
                          int32_t batch, float lr, float *loss, float *work, void *stream);

/*
 * mandel_order_desc -- perm (device int32[n]) becomes a permutation of 0..n-1
 * whose keys (device float[n]) are non-increasing up to the bucket width:
 * numbers are bucketed on a fixed grid of MANDEL_ORDER_BUCKETS - 1 equal
 * buckets over [MANDEL_ORDER_KEY_LO, MANDEL_ORDER_KEY_HI] (keys outside go to
 * the end buckets), NaN keys come after all numbers; the order inside one
 * bucket is unspecified.  0 <= n < 2^31 (n == 0 does nothing).
 */
#define MANDEL_ORDER_BUCKETS 4096
#define MANDEL_ORDER_KEY_LO (-2.0f)
#define MANDEL_ORDER_KEY_HI 50.0f
int mandel_order_desc(const float *keys, int64_t n, int32_t *perm, void *stream);

/* Sets the standardisation entries of params (mu, inv_sd; device) from the
 * column means and standard deviations of feat (device float[n][68], n >= 1):
 * inv_sd = 1 / max(sd, 1e-6).  The trained entries are not touched. */
int mandel_mlp_set_norm(float *params, const float *feat, int64_t n, void *stream);

/* Training targets: target[i] = ln(max(cost[i], 1)) for device int64 cost[n]. */
int mandel_cost_targets(const int64_t *cost, int64_t n, float *target, void *stream);

/*
 * mandel_plan_autotune -- picks the plan tuning (tile shape, claim grain,
 * waves per workgroup, row parts, longest deferred block) for a batch by
 * timing every candidate on a sample of
 * the views (at most max_sample views, spread over the batch's range of
 * pixels x max_iter), and caches the choice per device and batch signature.
 * Synchronous: it allocates a scratch image, renders the sample several
 * times on `stream` and waits.  best receives the chosen tuning; trials
 * (host, may be NULL) receives how many candidate launches were timed.
 */
int mandel_plan_autotune(const mandel_view *views, int32_t nviews, int32_t max_sample,
                         mandel_tuning *best, int32_t *trials, void *stream);

/* Properties of the current device used by the library: compute units and
 * the rate of the wall clock that stamps mandel_sched.stats[4..6] (kHz). */
int mandel_device_info(int32_t *compute_units, int32_t *wall_clock_khz);

/*
 * mandel_fp64_probe -- diagnostic: measures what the FP64 vector units deliver
 * on this device, to put the render kernel's rate next to a measured ceiling.
 *   kind 0: four independent fma chains per lane (peak FMA issue);
 *   kind 1: the escape-time update alone (3 mul, sub, add, fma per iteration, no
 *           test, no scheduling), one pixel per lane;
 *   kind 2: the same update on two pixels per lane.
 *   iters          iterations per lane, 1 .. 2^24 (8 updates or fmas each)
 *   blocks_per_cu  256-thread workgroups per compute unit, 1 .. 8
 *   sink           device double[compute units * blocks_per_cu * 256]: results
 *                  written so the work cannot be optimised away
 *   flops, ms      host: FP64 flops executed (fma = 2; the update counts its 7
 *                  flops) and the kernel time of the second of two launches.
 * Synchronous (waits for the kernel).
 */
int mandel_fp64_probe(int32_t kind, int32_t iters, int32_t blocks_per_cu, double *sink,
                      double *flops, float *ms, void *stream);

/* Text of the last error on this thread ("" if none). */
const char *mandel_last_error(void);

/* Library version string. */
const char *mandel_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MANDEL_H */
