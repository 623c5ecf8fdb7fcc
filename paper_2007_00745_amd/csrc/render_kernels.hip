// Escape-time render kernels for gfx950 (CDNA4, wave64).
//
// The method is the paper's Boolean escape-time generation (Sec. I, Eq. (1)
// and Eq. (2)); its load-imbalance problem (Sec. III: the middle rows cost far
// more than the top and bottom) is handled here inside one GPU:
//
//   * every wavefront is a worker; it pulls work items (tiles or rows) from a
//     source chosen by the policy -- a device-wide atomic queue (the analogue
//     of Sec. III-B), a permuted queue, the contiguous row blocks of Sec. III-A
//     or the alternating rows of Sec. III-C;
//   * lanes whose pixel finished take the next pixels of the wave's current
//     item (ballot + mbcnt compaction), and the wave claims the next item as
//     soon as the current one has no pixels left, so lanes idle only briefly
//     (until a refill round) and in the last items of the whole launch.  A
//     refill round starts once refill_lanes lanes are idle while updates are
//     tested one by one, or min(refill_lanes, 8) when a block of untested
//     updates ends, so refills of finished pixels come in groups;
//   * optionally (a separate instantiation), the rows of tiles other waves
//     hold are shared out once the queue is dry (row stealing);
//   * the |z|^2 > R^2 test may be deferred over blocks of K updates for
//     pixels where an escape provably cannot be undone (R >= 2 and
//     |c| <= (R^2 - R)(1 - 2^-20): after the first escape |z| keeps growing,
//     and inf/NaN never become finite again); a lane found escaped at the end
//     of a block rewinds to its snapshot and replays the block with a test
//     after every update, so the count is exact.
//
// Arithmetic contract (must match the CPU definition bit for bit): IEEE
// binary64, round to nearest even, one rounding per operation, in the order
//     x' = (x*x - y*y) + cx,   y' = 2*(x*y) + cy
// The file is compiled with -ffp-contract=off.  The only fused operation is
// the deliberate fma(2, x*y, cy): multiplying the rounded product by 2 is
// exact, so fma rounds once exactly where 2*(x*y) + cy rounds once.  (It would
// differ only if 2*(x*y) overflowed; before the escape |x|, |y| are bounded by
// about R <= 1e150, so it cannot.)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "render_kernels.h"

#pragma clang fp contract(off)

namespace mandel {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Bit l set iff lane l is active and p holds there (one SGPR pair, no VALU copy).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int32_t bcast_i32(int32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t bcast_i64(int64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Minimum over the 64 lanes (exec must be full): DPP row shifts reduce each
// 16-lane row, two row broadcasts fold the rows, lane 63 holds the result.
#define MANDEL_DPP_MIN(v, ctrl, rmask)                                                        \
    do {                                                                                    \
        const uint32_t o_ = (uint32_t)__builtin_amdgcn_update_dpp((int)(v), (int)(v), ctrl,  \
                                                                  rmask, 0xf, false);       \
        (v) = (v) < o_ ? (v) : o_;                                                          \
    } while (0)

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    MANDEL_DPP_MIN(v, 0x111, 0xf); // row_shr:1
    MANDEL_DPP_MIN(v, 0x112, 0xf); // row_shr:2
    MANDEL_DPP_MIN(v, 0x114, 0xf); // row_shr:4
    MANDEL_DPP_MIN(v, 0x118, 0xf); // row_shr:8
    MANDEL_DPP_MIN(v, 0x142, 0xa); // row_bcast:15 into rows 1 and 3
    MANDEL_DPP_MIN(v, 0x143, 0xc); // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t o = (uint64_t)__shfl_xor((long long)v, off, 64);
        v += o;
    }
    return v;
}

// The view table and the queue order are never written by the render kernel, so they
// are read as constant memory: wave-uniform reads then go through the scalar cache
// into SGPRs instead of 64 per-lane vector loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_const(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// Copy of a descriptor read from constant memory (fields the caller does not use are
// never loaded).
__device__ __forceinline__ ViewDesc load_view(const __attribute__((address_space(4))) ViewDesc *p)
{
    ViewDesc d;
    d.cx0 = p->cx0;
    d.cy0 = p->cy0;
    d.dx = p->dx;
    d.dy = p->dy;
    d.R2 = p->R2;
    d.safe2 = p->safe2;
    d.out_off = p->out_off;
    d.tile_off = p->tile_off;
    d.m = p->m;
    d.n = p->n;
    d.max_iter = p->max_iter;
    d.tiles_x = p->tiles_x;
    d.tiles_y = p->tiles_y;
    d.rows_off = p->rows_off;
    d.row_off = p->row_off;
    return d;
}

// Tile id (or, with ROWS, row index) -> view index in a batch: the last view whose
// first tile (first row) is at or before t.  The offsets ascend; empty views share
// the next view's offset and are never returned for an existing tile or row.
template <bool ROWS = false>
__device__ __forceinline__ int32_t find_view(const ViewDesc *table, int32_t nviews, int64_t t)
{
    const auto *views = as_const(table);
    int32_t lo = 0, hi = nviews - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if ((ROWS ? views[mid].row_off : views[mid].tile_off) <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

} // namespace

// Clears the queue head and the optional per-tile logs before a launch.
__global__ void clear_kernel(unsigned long long *head, int64_t first_slot, int64_t *tile_cost,
                             int32_t *claims, uint64_t *tile_time, int64_t ntiles,
                             uint64_t *stats, int32_t *chunk, int32_t *active, int64_t nwaves)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i == 0 && head)
        *head = (unsigned long long)first_slot;
    if (i == 0 && stats) {
        // per-launch timestamps (wall clock ticks): first claim, queue dry, last exit
        stats[4] = ~0ull;
        stats[5] = ~0ull;
        stats[6] = 0ull;
    }
    for (int64_t t = i; t < ntiles; t += stride) {
        if (tile_cost)
            tile_cost[t] = 0;
        if (claims)
            claims[t] = 0;
        if (tile_time) {
            tile_time[2 * t] = ~0ull; // first claim (atomic min)
            tile_time[2 * t + 1] = 0; // last pixel finished (atomic max)
        }
        if (chunk)
            chunk[t] = 0;
    }
    for (int64_t w = i; active && w < nwaves; w += stride)
        active[w] = -1;
}

// Periodicity detection compares this many of the last states of each deferred block
// with the block-start state, so every cycle of period <= PERIOD_WINDOW is found.
constexpr uint32_t PERIOD_WINDOW = 32;

// Idle lanes that trigger a refill at a round start (capped by refill_lanes).  Swept
// over 1, 2, 4, 8, 16, 32 on the 8192^2 view and the uneven 64-view batch: 8 is 0.5-1 %
// faster on the former and 3 % on the latter than refilling every idle lane at once.
constexpr uint32_t ROUND_REFILL_LANES = 8;

// Longest run of tested updates that a replay or an unsafe lane starts before the mode
// is decided again.  Swept over 16, 64, 256 and 1024 (= K): 64 took a 2048^2
// seahorse-valley view from 2.09 to 1.72 ms and the 8192^2 view 0.5 % faster, with
// the uneven batch unchanged.
constexpr uint32_t CHECKED_RUN = 64;

// Row stealing: a wave stops looking for rows to steal after this many takes that
// found their tile already drained by others.
constexpr int32_t STEAL_MAX_MISSES = 64;

template <int POLICY, bool BATCH, bool DEFER, bool PERIODIC, bool STEAL>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(STEAL ? 7 : 1)))
render_kernel(RenderArgs a)
{
    static_assert(DEFER || !PERIODIC, "periodicity detection runs in the deferred blocks");
    static_assert(!STEAL || POLICY == POLICY_FCFS_TILES || POLICY == POLICY_ORDERED_TILES,
                  "row stealing works on the tile queue");
    __shared__ int32_t lds_next_row;
    if constexpr (POLICY == POLICY_STATIC_ROWS || POLICY == POLICY_ALTERNATING_ROWS) {
        if (threadIdx.x == 0)
            lds_next_row = 0;
        __syncthreads();
    }
    const uint32_t lane = lane_id();

    // ---- wave-uniform state of the current work item ----------------------
    int32_t s_view = 0;          // view of the item
    int32_t s_x0 = 0, s_y0 = 0;  // item origin (column, row)
    int32_t s_w = 1;             // item width in pixels
    int32_t s_next = 0, s_cnt = 0; // next pixel index, pixels in the item
    int32_t s_in = 0, s_jn = 0;  // next pixel as (row, column) within the item (s_w >= 64)
    int64_t s_tile = 0;          // tile id (for the cost log)
    int64_t q_next = 0;          // FCFS: next queue slot of the current claim
    int32_t q_left = 0;          // FCFS: slots left in the current claim
    // STEAL: the tile whose rows this wave takes (-1: none), and the scan position
    // and length over the other waves' tiles once the queue is dry (-1: not yet dry)
    int32_t r_tile = -1;
    int32_t r_scan = -1, r_scanned = 0, r_miss = 0;
    int32_t taken = 0;           // items taken (statistics)
    bool exhausted = false;
    bool grid_done = false;

    // Geometry of tile t: its view and its clipped rectangle.
    auto tile_geometry = [&](int64_t t, int32_t &v, int32_t &x0, int32_t &y0, int32_t &w,
                             int32_t &h) {
        int64_t tile_off;
        int32_t tiles_x, vm, vn;
        v = 0;
        if constexpr (BATCH) {
            v = bcast_i32(find_view(a.views, a.nviews, t));
            const auto *vd = as_const(a.views) + v;
            tile_off = vd->tile_off;
            tiles_x = vd->tiles_x;
            vm = vd->m;
            vn = vd->n;
        } else {
            tile_off = a.v0.tile_off;
            tiles_x = a.v0.tiles_x;
            vm = a.v0.m;
            vn = a.v0.n;
        }
        const int64_t lt = t - tile_off;
        const int32_t ty = (int32_t)(lt / tiles_x);
        const int32_t tx = (int32_t)(lt - (int64_t)ty * tiles_x);
        x0 = tx * a.tile_w;
        y0 = ty * a.tile_h;
        w = vn - x0 < a.tile_w ? vn - x0 : a.tile_w;
        h = vm - y0 < a.tile_h ? vm - y0 : a.tile_h;
    };

    // Row stealing.  A claimed tile's rows are handed out one at a time by its own
    // counter a.chunk[t]; the claiming wave takes them in turn.  Once the queue is
    // dry, a wave looks through the tiles the other waves hold (a.active, one entry
    // per wave) for rows nobody has taken yet and takes them, so the rows of a tile
    // held by a wave that issues slowly are shared out instead of finishing last.
    // Every row is taken exactly once (one atomic increment per take), so counts,
    // cost logs and timestamps are as without stealing.  The held-tile table and the
    // counters are read and written with device-scope atomics: each XCD has its own
    // L2, and a plain load could keep returning a line that another XCD has since
    // changed.  A wave that holds a tile always takes its rows until none is left,
    // so a thief may give up at any time; it gives up after a full pass of the table
    // without a candidate, or after STEAL_MAX_MISSES takes that came too late.
    auto steal_item = [&]() -> bool {
        const int64_t nslots = a.ntiles;
        const int32_t G = (int32_t)(gridDim.x * (blockDim.x >> 6));
        const int32_t gw = (int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
        for (;;) {
            if (r_tile >= 0) {
                int32_t c = 0;
                if (lane == 0)
                    c = atomicAdd(&a.chunk[r_tile], 1);
                c = bcast_i32(c);
                int32_t v, x0, y0, w, h;
                tile_geometry(r_tile, v, x0, y0, w, h);
                if (c < h) {
                    s_view = v;
                    s_x0 = x0;
                    s_y0 = y0 + c;
                    s_w = w;
                    s_next = 0;
                    s_in = 0;
                    s_jn = 0;
                    s_cnt = w;
                    s_tile = r_tile;
                    return true;
                }
                r_tile = -1;
                if (r_scan >= 0)
                    ++r_miss; // a stolen take that found the tile already drained
            }
            if (r_scan < 0) {
                // claim the next tile from the queue
                if (q_left == 0) {
                    unsigned long long q = 0;
                    if (lane == 0)
                        q = atomicAdd(a.head, (unsigned long long)a.grain);
                    const int64_t qb = bcast_i64((int64_t)q);
                    if (a.stats && lane == 0) {
                        if (qb == a.first_slot)
                            atomicMin((unsigned long long *)&a.stats[4],
                                      (unsigned long long)wall_clock64());
                        if (qb >= nslots && qb < nslots + a.grain)
                            atomicMin((unsigned long long *)&a.stats[5],
                                      (unsigned long long)wall_clock64());
                    }
                    if (qb >= nslots) {
                        r_scan = 0; // the queue is dry: steal from now on
                        continue;
                    }
                    q_next = qb;
                    const int64_t left = nslots - qb;
                    q_left = (int32_t)(left < a.grain ? left : a.grain);
                }
                const int64_t slot = q_next++;
                --q_left;
                int64_t t;
                if constexpr (POLICY == POLICY_ORDERED_TILES) {
                    t = (int64_t)as_const(a.order)[slot];
                    if (t < 0 || t >= a.ntiles)
                        continue; // not a tile id: skipped, never dereferenced
                } else {
                    t = slot;
                }
                if (a.claims && lane == 0)
                    atomicAdd(&a.claims[t], 1);
                if (a.tile_time && lane == 0)
                    atomicMin((unsigned long long *)&a.tile_time[2 * t],
                              (unsigned long long)wall_clock64());
                ++taken;
                if (lane == 0)
                    __hip_atomic_store(&a.active[gw], (int32_t)t, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                r_tile = (int32_t)t;
            } else {
                // queue dry: look for a held tile with rows left, 64 entries per step,
                // starting after this wave's own entry; a full pass of the table
                // without a find ends the search
                if (r_scanned >= G || r_miss >= STEAL_MAX_MISSES)
                    return false;
                const int32_t j = (int32_t)(((int64_t)gw + 1 + r_scan + lane) % G);
                const int32_t tj =
                    __hip_atomic_load(&a.active[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bool cand = false;
                if (tj >= 0)
                    cand = __hip_atomic_load(&a.chunk[tj], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < a.tile_h;
                const uint64_t cm = ballot(cand);
                if (cm == 0) {
                    r_scan = (int32_t)(((int64_t)r_scan + 64) % G);
                    r_scanned += 64;
                    continue;
                }
                const int32_t first = (int32_t)__builtin_ctzll(cm);
                r_tile = __builtin_amdgcn_readlane(tj, first);
                r_scan = (int32_t)(((int64_t)r_scan + first + 1) % G);
                r_scanned = 0;
            }
        }
    };

    // Next work item of this wave, or false when the source is empty.
    auto next_item = [&]() -> bool {
        if constexpr (POLICY == POLICY_FCFS_TILES || POLICY == POLICY_ORDERED_TILES ||
                      POLICY == POLICY_GRID_TILES) {
            const int64_t nslots = POLICY == POLICY_GRID_TILES ? a.ntiles : a.ntiles * a.parts;
            for (;;) {
                int64_t t;
                int32_t part = 0;
                if constexpr (POLICY == POLICY_GRID_TILES) {
                    if (grid_done)
                        return false;
                    grid_done = true;
                    t = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
                    if (t >= a.ntiles)
                        return false;
                } else {
                    if constexpr (STEAL)
                        return steal_item();
                    if (q_left == 0) {
                        unsigned long long q = 0;
                        if (lane == 0)
                            q = atomicAdd(a.head, (unsigned long long)a.grain);
                        int64_t qb = bcast_i64((int64_t)q);
                        if (a.stats && lane == 0) {
                            if (qb == a.first_slot)
                                atomicMin((unsigned long long *)&a.stats[4],
                                          (unsigned long long)wall_clock64());
                            if (qb >= nslots && qb < nslots + a.grain)
                                atomicMin((unsigned long long *)&a.stats[5],
                                          (unsigned long long)wall_clock64());
                        }
                        if (qb >= nslots)
                            return false;
                        q_next = qb;
                        int64_t left = nslots - qb;
                        q_left = (int32_t)(left < a.grain ? left : a.grain);
                    }
                    const int64_t slot = q_next++;
                    --q_left;
                    // slot = item * parts + part: the queue hands out row parts of tiles
                    const int64_t item = a.parts == 1 ? slot : slot / a.parts;
                    part = (int32_t)(slot - item * a.parts);
                    if constexpr (POLICY == POLICY_ORDERED_TILES) {
                        t = (int64_t)as_const(a.order)[item];
                        if (t < 0 || t >= a.ntiles)
                            continue; // not a tile id: skipped, never dereferenced
                    } else {
                        t = item;
                    }
                }
                int32_t v = 0;
                int64_t tile_off;
                int32_t tiles_x, vm, vn;
                if constexpr (BATCH) {
                    v = bcast_i32(find_view(a.views, a.nviews, t));
                    const auto *vd = as_const(a.views) + v;
                    tile_off = vd->tile_off;
                    tiles_x = vd->tiles_x;
                    vm = vd->m;
                    vn = vd->n;
                } else {
                    tile_off = a.v0.tile_off;
                    tiles_x = a.v0.tiles_x;
                    vm = a.v0.m;
                    vn = a.v0.n;
                }
                int64_t lt = t - tile_off;
                int32_t ty = (int32_t)(lt / tiles_x);
                int32_t tx = (int32_t)(lt - (int64_t)ty * tiles_x);
                int32_t x0 = tx * a.tile_w, y0 = ty * a.tile_h;
                int32_t w = vn - x0 < a.tile_w ? vn - x0 : a.tile_w;
                int32_t h = vm - y0 < a.tile_h ? vm - y0 : a.tile_h;
                // rows [r0, r1) of the tile form this part
                const int32_t r0 = (int32_t)(((int64_t)part * h) / a.parts);
                const int32_t r1 = (int32_t)(((int64_t)(part + 1) * h) / a.parts);
                if (r1 <= r0)
                    continue; // empty part (a tile with fewer rows than parts)
                if (a.claims && lane == 0)
                    atomicAdd(&a.claims[t], 1);
                if (a.tile_time && lane == 0)
                    atomicMin((unsigned long long *)&a.tile_time[2 * t],
                              (unsigned long long)wall_clock64());
                s_view = v;
                s_x0 = x0;
                s_y0 = y0 + r0;
                s_w = w;
                s_next = 0;
                s_in = 0;
                s_jn = 0;
                s_cnt = w * (r1 - r0);
                s_tile = t;
                ++taken;
                return true;
            }
        } else {
            // Row policies: a workgroup is one worker r of W = gridDim.x.  In a batch the
            // rows of all views form one sequence (view 0's rows, then view 1's, ...)
            // that is partitioned as one image of nrows rows.
            int64_t M;
            if constexpr (BATCH)
                M = a.nrows;
            else
                M = a.v0.m;
            const int64_t W = (int64_t)gridDim.x;
            const int64_t r = (int64_t)blockIdx.x;
            const int64_t q = M / W;
            int32_t k = 0;
            if (lane == 0)
                k = atomicAdd(&lds_next_row, 1);
            k = bcast_i32(k);
            int64_t row, cnt;
            if constexpr (POLICY == POLICY_STATIC_ROWS) {
                // Sec. III-A: S_r = q*r, E_r = q*(r+1) - 1, last worker + (M mod W).
                cnt = q + (r == W - 1 ? M % W : 0);
                row = q * r + k;
            } else {
                // Sec. III-C: rows r + k*W for k < q; worker 0 also does rows q*W .. M-1.
                cnt = q + (r == 0 ? M - q * W : 0);
                row = k < q ? r + (int64_t)k * W : q * W + (k - q);
            }
            if (a.stats && lane == 0) {
                if (k == 0 && cnt > 0)
                    atomicMin((unsigned long long *)&a.stats[4],
                              (unsigned long long)wall_clock64());
                if (k == cnt)
                    atomicMin((unsigned long long *)&a.stats[5],
                              (unsigned long long)wall_clock64());
            }
            if (k >= cnt)
                return false;
            if (a.claims && lane == 0)
                atomicAdd(&a.claims[row], (int32_t)r + 1); // ownership log: worker r + 1 per take
            int32_t v = 0, vrow, vn;
            if constexpr (BATCH) {
                v = bcast_i32(find_view<true>(a.views, a.nviews, row));
                const auto *vd = as_const(a.views) + v;
                vrow = (int32_t)(row - vd->row_off);
                vn = vd->n;
            } else {
                vrow = (int32_t)row;
                vn = a.v0.n;
            }
            s_view = v;
            s_x0 = 0;
            s_y0 = vrow;
            s_w = vn;
            s_next = 0;
            s_in = 0;
            s_jn = 0;
            s_cnt = vn;
            s_tile = row;
            ++taken;
            return true;
        }
    };

    // ---- per-lane state ------------------------------------------------------
    double x = 0.0, y = 0.0, cx = 0.0, cy = 0.0;
    double xs = 0.0, ys = 0.0; // snapshot at the start of a deferred block
    double xm = 0.0, ym = 0.0; // snapshot after the first half of a deferred block
    double R2 = a.v0.R2;
    uint32_t start = 0, deadline = 0; // wave-iteration of z_0 and of z_{max_iter-1}
    int64_t oidx = 0;                 // flat output index
    int64_t ltile = 0;                // tile of the pixel (cost log)
    bool active = false, pending = false, safe = false;
    uint64_t acc = 0;                 // sum of counts finished by this lane
    uint64_t skipped = 0;             // PERIODIC: updates not run thanks to a detected cycle
    uint32_t W = 0;                   // wave iteration counter (uniform)

    auto refill = [&]() {
        for (;;) {
            uint64_t need = ballot(!active);
            if (need == 0 || exhausted)
                break;
            if (s_next >= s_cnt) {
                if (!next_item())
                    exhausted = true;
                continue;
            }
            const int32_t avail = s_cnt - s_next;
            const int32_t k = (int32_t)__popcll(need);
            const int32_t take = k < avail ? k : avail;
            const uint32_t rk = rank_in(need);
            if (!active && (int32_t)rk < take) {
                ViewDesc vv;
                if constexpr (BATCH)
                    vv = load_view(as_const(a.views) + bcast_i32(s_view));
                else
                    vv = a.v0;
                const ViewDesc *vd = &vv;
                // pixel s_next + rk of the item, row-major within it
                int32_t i, j;
                if (s_w >= 64) {
                    // rk < 64 <= s_w: at most one wrap past the item's right edge
                    j = s_jn + (int32_t)rk;
                    i = s_in;
                    if (j >= s_w) {
                        j -= s_w;
                        i += 1;
                    }
                } else {
                    const int32_t p = s_next + (int32_t)rk;
                    i = p / s_w;
                    j = p - i * s_w;
                }
                i += s_y0;
                j += s_x0;
                const double offx = ((double)j + 0.5) - 0.5 * (double)vd->n;
                const double px = offx * vd->dx;
                cx = vd->cx0 + px;
                if (BATCH && vd->rows_off >= 0) {
                    const RowRef rr = a.rows[vd->rows_off + i];
                    cy = rr.cy;
                    oidx = rr.out + j;
                } else {
                    const double offy = ((double)i + 0.5) - 0.5 * (double)vd->m;
                    const double py = offy * vd->dy;
                    cy = vd->cy0 + py;
                    oidx = vd->out_off + (int64_t)i * vd->n + j;
                }
                x = 0.0;
                y = 0.0;
                if constexpr (BATCH)
                    R2 = vd->R2;
                start = W;
                deadline = W + (uint32_t)(vd->max_iter - 1);
                ltile = s_tile;
                if constexpr (DEFER) {
                    const double cc = cx * cx + cy * cy;
                    safe = cc <= vd->safe2;
                }
                pending = false;
                active = true;
            }
            s_next += take;
            if (s_w >= 64) {
                s_jn += take;
                if (s_jn >= s_w) {
                    s_jn -= s_w;
                    s_in += 1;
                }
            }
        }
    };

    auto finalize = [&](bool fin, bool esc) {
        if (fin) {
            const uint32_t cnt = esc ? (W - start) : (deadline - start + 1u);
            a.out[oidx] = (int32_t)cnt;
            if (a.tile_cost)
                atomicAdd((unsigned long long *)&a.tile_cost[ltile], (unsigned long long)cnt);
            if (a.tile_time)
                atomicMax((unsigned long long *)&a.tile_time[2 * ltile + 1],
                          (unsigned long long)wall_clock64());
            acc += cnt;
            active = false;
            pending = false;
        }
    };

    const uint32_t K = (uint32_t)a.block_iters; // longest deferred block
    const uint32_t P = (uint32_t)a.young_iters;
    const uint32_t R = (uint32_t)a.refill_lanes; // idle lanes that trigger a refill round
    // At a round start (a block or a run of tested updates has ended) idle lanes are
    // refilled only once Rs of them are idle, or when no lane is active.  A lane that
    // reached its deadline then waits for a few others, so refills (pixel set-up, young
    // tested updates, budget reduction) come in groups, and lanes refilled together in
    // the set's interior reach their deadlines together again.
    const uint32_t Rs = R < ROUND_REFILL_LANES ? R : ROUND_REFILL_LANES;
    const uint32_t Kmin = K < 8u ? K : 8u;
    uint32_t Kc = K; // current deferred block length (halved after a replay, doubled after a clean block)

    // One update z <- z^2 + c, in the contract's operation order.
    auto update = [&]() {
        const double xx = x * x;
        const double yy = y * y;
        const double t = x * y;
        x = (xx - yy) + cx;
        y = __builtin_fma(2.0, t, cy);
    };
    // One tested update: mask of lanes whose current state has |z|^2 > R^2
    // (tested before the update, so the count of such a lane is its age now).
    auto tested_update = [&]() -> uint64_t {
        const double xx = x * x;
        const double yy = y * y;
        const uint64_t m = ballot(xx + yy > R2);
        const double t = x * y;
        x = (xx - yy) + cx;
        y = __builtin_fma(2.0, t, cy);
        return m;
    };

    // A lower bound of deadline - W over the active lanes, carried from one round to the
    // next: W and the bound advance together, a replay only moves a deadline later and a
    // finished lane leaves the set, so only a refill invalidates it.  While it allows a
    // whole block the exact minimum (a cross-lane reduction) is not needed.
    uint32_t bound = 0;

    // Invariant at the top of each round: every active lane holds the state
    // z_n, n = W - start, not yet tested, and W <= deadline.
    for (;;) {
        const uint64_t idle = ballot(!active);
        if ((uint32_t)__popcll(idle) >= Rs) { // also when no lane is active (Rs <= 8)
            refill();
            bound = 0;
        }
        const uint64_t amask = ballot(active);
        if (amask == 0)
            break;
        // updates until the first lane reaches its last state z_{max_iter-1} (or a lower
        // bound of that, when it still allows a full block: finalisation at a deadline is
        // decided per lane, so a low bound only ends a round early)
        uint32_t budget =
            bound >= Kc ? bound : wave_min_u32(active ? deadline - W : 0xffffffffu);

        if constexpr (DEFER) {
            const bool needc = active && (pending || !safe || (W - start) < P);
            // (budget == 0 means some lane sits at an untested last state: the
            // checked mode below tests it)
            if (ballot(needc) == 0 && budget > 0) {
                // Steady state: blocks of L untested updates.  Every active lane
                // is "safe": once |z|^2 > R^2 its modulus keeps growing (or turns
                // inf/NaN, which never becomes finite again), so one test at the
                // end of a block tells whether the escape happened inside it.
                while (budget > 0) {
                    const uint32_t L = budget < Kc ? budget : Kc;
                    xs = x;
                    ys = y;
                    uint32_t rewind_h = 0; // updates before the checkpoint (0: none)
                    uint64_t pm = 0; // PERIODIC: lanes whose state returned to the block start
                    if constexpr (PERIODIC) {
                        // The last Q states of the block are compared bit for bit with
                        // the block-start state: an orbit that has settled on a cycle of
                        // period p <= Q returns to it at some k in (L - Q, L].
                        const uint32_t Q = L < PERIOD_WINDOW ? L : PERIOD_WINDOW;
                        const uint32_t L0 = L - Q;
                        for (uint32_t u = 0; u < (L0 >> 2); ++u) {
                            update();
                            update();
                            update();
                            update();
                        }
                        for (uint32_t u = 0; u < (L0 & 3u); ++u)
                            update();
                        const uint64_t xb = (uint64_t)__double_as_longlong(xs);
                        const uint64_t yb = (uint64_t)__double_as_longlong(ys);
                        for (uint32_t u = 0; u < Q; ++u) {
                            update();
                            pm |= __builtin_amdgcn_ballot_w64((uint64_t)__double_as_longlong(x) == xb) &
                                  __builtin_amdgcn_ballot_w64((uint64_t)__double_as_longlong(y) == yb);
                        }
                    } else {
                        // A checkpoint after the first Lh updates: a lane found escaped at
                        // the end replays only the half of the block that holds its first
                        // escape.  (Checkpoints after every quarter replayed less but cost
                        // registers and copies: the uneven batch took 314 ms against
                        // 309 ms with one, and the 8192^2 view 1.5 % longer.)
                        const uint32_t Lh = L >> 1;
                        for (uint32_t u = 0; u < (Lh >> 2); ++u) {
                            update();
                            update();
                            update();
                            update();
                        }
                        for (uint32_t u = 0; u < (Lh & 3u); ++u)
                            update();
                        xm = x;
                        ym = y;
                        for (uint32_t u = 0; u < ((L - Lh) >> 2); ++u) {
                            update();
                            update();
                            update();
                            update();
                        }
                        for (uint32_t u = 0; u < ((L - Lh) & 3u); ++u)
                            update();
                        rewind_h = Lh;
                    }
                    W += L;
                    budget -= L;
                    const double sq = x * x + y * y;
                    const uint64_t em = ballot(!(sq <= R2)) & amask;
                    if constexpr (PERIODIC) {
                        // A lane that did not escape in this block and met its block-start
                        // state again is on an exact cycle of non-escaping states (an
                        // escape inside the block would have left |z|^2 > R^2 at its end),
                        // so it never escapes: its count is max_iter.
                        const uint64_t pl = pm & ~em & ballot(active);
                        if (pl != 0) {
                            const bool mine = (pl >> lane) & 1u;
                            if (mine)
                                skipped += deadline - W;
                            finalize(mine, false);
                            if (em == 0 && (uint32_t)__popcll(~ballot(active)) >= Rs)
                                break; // enough idle lanes: refill them
                        }
                    }
                    if (em != 0) {
                        if ((em >> lane) & 1u) {
                            // Rewind and replay with tests.  Escaped states stay escaped
                            // in the safe disk, so the checkpoint state has escaped iff
                            // the first escape lies in the first half: then replay from
                            // the block start, else from the checkpoint (no state before
                            // it escaped).
                            const bool late = rewind_h != 0 && xm * xm + ym * ym <= R2;
                            const uint32_t back = late ? L - rewind_h : L;
                            x = late ? xm : xs;
                            y = late ? ym : ys;
                            start += back;
                            deadline += back;
                            pending = true;
                        }
                        // escapes are near: shorter blocks waste less on replays
                        Kc = Kc >> 1 < Kmin ? Kmin : Kc >> 1;
                        break;
                    }
                    Kc = Kc << 1 > K ? K : Kc << 1;
                }
                // lanes now at z_{max_iter-1} with no escape so far: count = max_iter
                finalize(active && !pending && deadline == W, false);
                bound = budget;
                continue;
            }
        }

        // Checked mode: groups of four tested updates.  A lane's count is the
        // age at its first set mask bit, provided that is not past its deadline.
        // When only young lanes asked for it, P tested updates suffice; replays
        // and unsafe lanes keep it until an event ends it or CHECKED_RUN updates
        // have run (then the mode is decided again, so a wave whose replayed lane
        // has been resolved returns to untested blocks).
        uint32_t climit = K < CHECKED_RUN ? K : CHECKED_RUN;
        if constexpr (DEFER) {
            if (ballot(active && (pending || !safe)) == 0)
                climit = P;
        }
        uint32_t done = 0;
        uint64_t cmask = amask; // lanes still active in this checked run
        for (;;) {
            const uint32_t W0 = W;
            const uint64_t m0 = tested_update();
            const uint64_t m1 = tested_update();
            const uint64_t m2 = tested_update();
            const uint64_t m3 = tested_update();
            W += 4;
            const uint64_t any = (m0 | m1 | m2 | m3) & cmask;
            if (any != 0 || budget < 4) {
                const uint32_t ke = ((m0 >> lane) & 1u) ? 0u
                                  : ((m1 >> lane) & 1u) ? 1u
                                  : ((m2 >> lane) & 1u) ? 2u
                                  : ((m3 >> lane) & 1u) ? 3u : 4u;
                const uint32_t kd = deadline - W0; // steps to the last state
                const bool esc = active && ke < 4u && ke <= kd;
                const bool dl = active && !esc && kd < 4u;
                if (esc || dl) {
                    const uint32_t cnt = esc ? (W0 + ke - start) : (deadline - start + 1u);
                    a.out[oidx] = (int32_t)cnt;
                    if (a.tile_cost)
                        atomicAdd((unsigned long long *)&a.tile_cost[ltile],
                                  (unsigned long long)cnt);
                    if (a.tile_time)
                        atomicMax((unsigned long long *)&a.tile_time[2 * ltile + 1],
                                  (unsigned long long)wall_clock64());
                    acc += cnt;
                    active = false;
                    pending = false;
                }
                // Lazy refill: with budget >= 4 only escapes happened here; while few
                // lanes are idle (or nothing is left to refill from) keep iterating
                // instead of paying for a refill round.  budget - 4 stays a lower
                // bound of every remaining lane's distance to its deadline.
                if (budget >= 4) {
                    cmask = ballot(active);
                    // with deferred tests, only while some lane still needs a test after
                    // every update (a replay, an unsafe or a young lane); otherwise the
                    // round ends and the wave returns to untested blocks
                    if (cmask != 0 && ((uint32_t)__popcll(~cmask) < R || exhausted) &&
                        (!DEFER ||
                         (done + 4 < climit &&
                          ballot(active && (pending || !safe || (W - start) < P)) != 0))) {
                        budget -= 4;
                        done += 4;
                        continue;
                    }
                }
                budget = budget >= 4 ? budget - 4 : 0; // this group's updates
                break;
            }
            budget -= 4;
            done += 4;
            if (DEFER && done >= climit)
                break; // re-evaluate the mode
        }
        bound = budget;
    }

    if (a.stats) {
        const uint64_t tot = wave_sum_u64(acc);
        if (lane == 0) {
            atomicAdd((unsigned long long *)&a.stats[0], (unsigned long long)W);
            atomicAdd((unsigned long long *)&a.stats[1], (unsigned long long)tot);
            atomicAdd((unsigned long long *)&a.stats[2], 1ull);
            atomicAdd((unsigned long long *)&a.stats[3], (unsigned long long)taken);
            atomicMax((unsigned long long *)&a.stats[6], (unsigned long long)wall_clock64());
        }
        if constexpr (PERIODIC) {
            const uint64_t sk = wave_sum_u64(skipped);
            if (lane == 0)
                atomicAdd((unsigned long long *)&a.stats[7], (unsigned long long)sk);
        }
    }
}

// ---- launch helpers (host) ---------------------------------------------------

template <int POLICY, bool BATCH, bool DEFER, bool PERIODIC, bool STEAL = false>
static hipError_t launch_one(const RenderArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    hipLaunchKernelGGL((render_kernel<POLICY, BATCH, DEFER, PERIODIC, STEAL>), grid, block, 0, s,
                       a);
    return hipGetLastError();
}

template <int POLICY, bool BATCH>
static hipError_t launch_mode(const RenderArgs &a, int tests, dim3 grid, dim3 block,
                              hipStream_t s)
{
    if constexpr (BATCH && (POLICY == POLICY_FCFS_TILES || POLICY == POLICY_ORDERED_TILES)) {
        if (a.steal) {
            switch (tests) {
            case TESTS_EVERY_UPDATE:
                return launch_one<POLICY, BATCH, false, false, true>(a, grid, block, s);
            case TESTS_DEFERRED:
                return launch_one<POLICY, BATCH, true, false, true>(a, grid, block, s);
            case TESTS_DEFERRED_PERIODIC:
                return launch_one<POLICY, BATCH, true, true, true>(a, grid, block, s);
            default:
                return hipErrorInvalidValue;
            }
        }
    } else {
        if (a.steal)
            return hipErrorInvalidValue;
    }
    switch (tests) {
    case TESTS_EVERY_UPDATE:
        return launch_one<POLICY, BATCH, false, false>(a, grid, block, s);
    case TESTS_DEFERRED:
        return launch_one<POLICY, BATCH, true, false>(a, grid, block, s);
    case TESTS_DEFERRED_PERIODIC:
        return launch_one<POLICY, BATCH, true, true>(a, grid, block, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_render(const RenderArgs &a, int policy, bool batch, int tests, dim3 grid,
                         dim3 block, hipStream_t s)
{
    if (batch) {
        switch (policy) {
        case POLICY_FCFS_TILES:
            return launch_mode<POLICY_FCFS_TILES, true>(a, tests, grid, block, s);
        case POLICY_ORDERED_TILES:
            return launch_mode<POLICY_ORDERED_TILES, true>(a, tests, grid, block, s);
        case POLICY_GRID_TILES:
            return launch_mode<POLICY_GRID_TILES, true>(a, tests, grid, block, s);
        case POLICY_STATIC_ROWS:
            return launch_mode<POLICY_STATIC_ROWS, true>(a, tests, grid, block, s);
        case POLICY_ALTERNATING_ROWS:
            return launch_mode<POLICY_ALTERNATING_ROWS, true>(a, tests, grid, block, s);
        default:
            return hipErrorInvalidValue;
        }
    }
    switch (policy) {
    case POLICY_FCFS_TILES:
        return launch_mode<POLICY_FCFS_TILES, false>(a, tests, grid, block, s);
    case POLICY_STATIC_ROWS:
        return launch_mode<POLICY_STATIC_ROWS, false>(a, tests, grid, block, s);
    case POLICY_ALTERNATING_ROWS:
        return launch_mode<POLICY_ALTERNATING_ROWS, false>(a, tests, grid, block, s);
    case POLICY_ORDERED_TILES:
        return launch_mode<POLICY_ORDERED_TILES, false>(a, tests, grid, block, s);
    case POLICY_GRID_TILES:
        return launch_mode<POLICY_GRID_TILES, false>(a, tests, grid, block, s);
    default:
        return hipErrorInvalidValue;
    }
}

// Pair p0 + blockIdx.y (dst, src) of an image of n columns: row dst becomes a copy of
// row src, in 16-byte vectors when the rows are 16-byte aligned.
__global__ void expand_rows_kernel(int32_t *img, int64_t n, const int32_t *pairs, int32_t p0,
                                   int32_t npairs)
{
    const int32_t q = p0 + (int32_t)blockIdx.y;
    if (q >= npairs)
        return;
    int32_t *dst = img + (int64_t)pairs[2 * q] * n;
    const int32_t *from = img + (int64_t)pairs[2 * q + 1] * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if ((n & 3) == 0 && (((uintptr_t)img) & 15) == 0) {
        const int64_t n4 = n >> 2;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n4; c += stride)
            ((int4 *)dst)[c] = ((const int4 *)from)[c];
    } else {
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride)
            dst[c] = from[c];
    }
}

hipError_t launch_expand_rows(int32_t *img, int64_t n, const int32_t *pairs, int32_t npairs,
                              hipStream_t s)
{
    if (npairs <= 0 || n <= 0)
        return hipSuccess;
    const int64_t per_row = (n + 4 * 256 - 1) / (4 * 256);
    const unsigned gx = (unsigned)(per_row < 64 ? per_row : 64);
    // grid.y is limited to 65535 rows per launch
    for (int32_t p0 = 0; p0 < npairs; p0 += 65535) {
        const unsigned nr = npairs - p0 < 65535 ? (unsigned)(npairs - p0) : 65535u;
        hipLaunchKernelGGL(expand_rows_kernel, dim3(gx, nr), dim3(256), 0, s, img, n, pairs, p0,
                           npairs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_clear(unsigned long long *head, int64_t first_slot, int64_t *tile_cost,
                        int32_t *claims, uint64_t *tile_time, int64_t ntiles, uint64_t *stats,
                        hipStream_t s, int32_t *chunk, int32_t *active, int64_t nwaves)
{
    int64_t blocks = ((ntiles > nwaves ? ntiles : nwaves) + 255) / 256;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(clear_kernel, dim3((unsigned)blocks), dim3(256), 0, s, head, first_slot,
                       tile_cost, claims, tile_time, ntiles, stats, chunk, active, nwaves);
    return hipGetLastError();
}

int persistent_blocks_per_cu(int policy, bool batch, int tests, int threads)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define MANDEL_OCC(P, B)                                                                       \
    do {                                                                                       \
        if (tests == TESTS_EVERY_UPDATE)                                                       \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                                  \
                &nb, render_kernel<P, B, false, false, false>, threads, 0);                     \
        else if (tests == TESTS_DEFERRED)                                                      \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                                  \
                &nb, render_kernel<P, B, true, false, false>, threads, 0);                      \
        else                                                                                   \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                                  \
                &nb, render_kernel<P, B, true, true, false>, threads, 0);                       \
    } while (0)
    if (batch) {
        if (policy == POLICY_ORDERED_TILES)
            MANDEL_OCC(POLICY_ORDERED_TILES, true);
        else
            MANDEL_OCC(POLICY_FCFS_TILES, true);
    } else {
        if (policy == POLICY_ORDERED_TILES)
            MANDEL_OCC(POLICY_ORDERED_TILES, false);
        else
            MANDEL_OCC(POLICY_FCFS_TILES, false);
    }
#undef MANDEL_OCC
    if (e != hipSuccess || nb < 1)
        return 1;
    return nb;
}

} // namespace mandel
