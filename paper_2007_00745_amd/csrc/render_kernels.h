// Shared host/device declarations of the render kernel family.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mandel {

enum : int {
    POLICY_FCFS_TILES = 0,
    POLICY_STATIC_ROWS = 1,
    POLICY_ALTERNATING_ROWS = 2,
    POLICY_ORDERED_TILES = 3,
    POLICY_GRID_TILES = 4,
};

// Bytes of a queue head allocation (one 64-bit counter on its own 256-byte line).
constexpr int HEAD_BYTES = 256;

// One rendered row of a view with collapsed rows: its imaginary part and the element
// offset, in the output buffer, of the image row that receives its counts.
struct RowRef {
    double cy;
    int64_t out;
};

// One view as the kernels see it (96 bytes).
struct ViewDesc {
    double cx0, cy0, dx, dy; // window: centre and pixel pitch
    double R2;               // R*R, rounded once
    double safe2;            // |c|^2 bound below which the deferred test is exact (<0: never)
    int64_t out_off;         // element offset of this view's image in the output buffer
    int64_t tile_off;        // global id of this view's first tile
    int32_t m, n;            // rows, columns
    int32_t max_iter;
    int32_t tiles_x;         // tiles per tile-row
    int32_t tiles_y;
    int32_t rows_off;        // -1: row i has cy = cy0 + ((i + 0.5) - m/2) dy and its
                             // counts go to image row i; >= 0: the view's rows are the
                             // distinct row coordinates of a larger view (collapsed
                             // rows), row i is rows[rows_off + i]
    int64_t row_off;         // batch row policies: index of this view's first row in the
                             // concatenation of all views' rows
};
static_assert(sizeof(ViewDesc) == 96, "ViewDesc layout");

struct RenderArgs {
    ViewDesc v0;                   // the view when there is only one
    const ViewDesc *views;         // batch: device table, ascending tile_off
    int32_t nviews;
    int32_t tile_w, tile_h, grain;
    int64_t ntiles;
    int32_t block_iters;           // K: updates per deferred block
    int32_t young_iters;           // P: pixels younger than P updates are tested every update
    int32_t refill_lanes;          // checked mode refills once this many lanes are idle
    int32_t parts;                 // queue items per tile (row parts), >= 1; 1 for GRID
    int64_t first_slot;            // FCFS / ORDERED: the queue starts at this slot
    int64_t nrows;                 // batch row policies: rows of all views together
    const RowRef *rows;            // rows of views with collapsed rows, or NULL
    int32_t *out;                  // output base
    unsigned long long *head;      // queue head (FCFS / ORDERED)
    const int32_t *order;          // ORDERED: queue slot -> tile id
    int64_t *tile_cost;            // optional: sum of counts per tile
    int32_t *claims;               // optional: claims per tile
    uint64_t *tile_time;           // optional: per tile, first claim and last pixel finished
    int32_t steal;                 // FCFS / ORDERED with parts 1: rows are taken through
                                   // chunk[] and shared out once the queue is dry
    int32_t *chunk;                // steal: next untaken row per tile [ntiles]
    int32_t *active;               // steal: tile held by each wavefront [waves in grid]
    uint64_t *stats;               // optional: uint64[8], see mandel_sched.stats
};

// How the escape test is scheduled: after every update; in deferred blocks (lanes
// inside the safe disk); deferred blocks plus exact periodicity detection.
enum : int {
    TESTS_EVERY_UPDATE = 0,
    TESTS_DEFERRED = 1,
    TESTS_DEFERRED_PERIODIC = 2,
};

hipError_t launch_render(const RenderArgs &a, int policy, bool batch, int tests, dim3 grid,
                         dim3 block, hipStream_t s);
// Clears the queue head and the optional logs; with chunk/active (row stealing) also
// the per-tile row counters [ntiles] and the per-wave held tiles [nwaves].
hipError_t launch_clear(unsigned long long *head, int64_t first_slot, int64_t *tile_cost,
                        int32_t *claims, uint64_t *tile_time, int64_t ntiles, uint64_t *stats,
                        hipStream_t s, int32_t *chunk = nullptr, int32_t *active = nullptr,
                        int64_t nwaves = 0);
int persistent_blocks_per_cu(int policy, bool batch, int tests, int threads);
// Copies whole rows inside one view's image: for each of the npairs pairs (dst, src)
// in pairs[2 * npairs], row dst becomes a copy of row src, n columns per row.  No src
// may be a dst of the same call (the copies run in any order).
hipError_t launch_expand_rows(int32_t *img, int64_t n, const int32_t *pairs, int32_t npairs,
                              hipStream_t s);

} // namespace mandel
