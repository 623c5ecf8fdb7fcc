// C ABI of libmandel.so: argument checks, workspaces and launches.
// The operation and every argument are specified in include/mandel.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "dd_kernels.h"
#include "mandel.h"
#include "mandel_internal.h"
#include "output.h"
#include "render_kernels.h"

namespace mandel {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(MANDEL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

// ---- per (device, stream) workspace ----------------------------------------
namespace {
struct Workspace {
    unsigned long long *head = nullptr;
    uint32_t *order_hist = nullptr;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
} // namespace

int workspace_head(hipStream_t s, unsigned long long **head)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, s}];
    if (!w.head) {
        e = hipMalloc((void **)&w.head, HEAD_BYTES);
        if (e != hipSuccess) {
            w.head = nullptr;
            return fail(MANDEL_ENOMEM, "hipMalloc(workspace): %s", hipGetErrorString(e));
        }
    }
    *head = w.head;
    return MANDEL_OK;
}

int workspace_order(void *stream, uint32_t **hist)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, (hipStream_t)stream}];
    if (!w.order_hist) {
        e = hipMalloc((void **)&w.order_hist, sizeof(uint32_t) * 2 * MANDEL_ORDER_BUCKETS);
        if (e != hipSuccess) {
            w.order_hist = nullptr;
            return fail(MANDEL_ENOMEM, "hipMalloc(order workspace): %s", hipGetErrorString(e));
        }
    }
    *hist = w.order_hist;
    return MANDEL_OK;
}

// ---- allocation-free variant: the queue head in a file-scope device array ----
// mandel_render_sched_noalloc takes its queue head from `scratch` instead of a
// hipMalloc'd workspace.  Each device holds its own copy of the array, at its own
// address, until the process ends.  In host code the name `scratch` is only a
// host-side stand-in, so host code uses nothing but the device address that
// hipGetSymbolAddress returns, looked up once per device with that device current.
constexpr int NOALLOC_SCRATCH_BYTES = HEAD_BYTES;
static __device__ __align__(256) unsigned long long scratch[NOALLOC_SCRATCH_BYTES / 8];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned long long *> g_scratch; // device -> address of its scratch
} // namespace

int scratch_head(unsigned long long **head)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(MANDEL_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        it = g_scratch.emplace(dev, (unsigned long long *)p).first;
    }
    *head = it->second;
    return MANDEL_OK;
}

int device_cus(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    return MANDEL_OK;
}

// ---- argument checks ----------------------------------------------------------
int64_t tile_count(int32_t m, int32_t n, int32_t tw, int32_t th)
{
    if (m <= 0 || n <= 0 || tw <= 0 || th <= 0)
        return 0;
    // in 64 bits: m + th - 1 overflows int32 for m near 2^31
    return (((int64_t)m + th - 1) / th) * (((int64_t)n + tw - 1) / tw);
}

// Fills d (all but out_off and tile_off) from one view's arguments.
int make_view(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter, double R,
              int32_t tile_w, int32_t tile_h, ViewDesc *d)
{
    if (!w)
        return fail(MANDEL_EINVAL, "window is NULL");
    if (m < 0 || n < 0)
        return fail(MANDEL_EINVAL, "negative size m=%d n=%d", m, n);
    if ((int64_t)m * (int64_t)n >= (int64_t(1) << 40))
        return fail(MANDEL_EINVAL, "image too large: %d x %d", m, n);
    if (max_iter < 1 || max_iter > (1 << 30))
        return fail(MANDEL_EINVAL, "max_iter=%d outside [1, 2^30]", max_iter);
    if (!std::isfinite(R) || !(R > 0.0) || R > 1e150)
        return fail(MANDEL_EINVAL, "escape radius R=%g outside (0, 1e150]", R);
    if (!std::isfinite(w->cx0) || !std::isfinite(w->cy0) || !std::isfinite(w->dx) ||
        !std::isfinite(w->dy))
        return fail(MANDEL_EINVAL, "window has a non-finite value");
    if (!(w->dx > 0.0) || !(w->dy > 0.0))
        return fail(MANDEL_EINVAL, "pixel pitch must be > 0 (dx=%g dy=%g)", w->dx, w->dy);
    // Corner points (extreme offsets); c is monotone in the offset.
    const double ox = 0.5 - 0.5 * (double)n, oy = 0.5 - 0.5 * (double)m;
    const double c0x = w->cx0 + ox * w->dx, c1x = w->cx0 - ox * w->dx;
    const double c0y = w->cy0 + oy * w->dy, c1y = w->cy0 - oy * w->dy;
    if (m > 0 && n > 0 &&
        (!std::isfinite(c0x) || !std::isfinite(c1x) || !std::isfinite(c0y) ||
         !std::isfinite(c1y)))
        return fail(MANDEL_EINVAL, "window corners are not finite");
    std::memset(d, 0, sizeof *d);
    d->cx0 = w->cx0;
    d->cy0 = w->cy0;
    d->dx = w->dx;
    d->dy = w->dy;
    d->R2 = R * R;
    // Deferred tests are exact when R >= 2 and |c| <= (R^2 - R)(1 - 2^-20): after the
    // first |z|^2 > R^2 the modulus then grows at every update, up to overflow to
    // inf/NaN, which stays non-finite.  The bound is taken with a 2^-19 margin so that
    // rounding in the device's |c|^2 cannot cross it.
    if (R >= 2.0) {
        const double b = (R * R - R) * (1.0 - 0x1p-19);
        d->safe2 = b * b;
    } else {
        d->safe2 = -1.0;
    }
    d->m = m;
    d->n = n;
    d->max_iter = max_iter;
    d->tiles_x = (int32_t)(((int64_t)n + tile_w - 1) / tile_w);
    d->tiles_y = (int32_t)(((int64_t)m + tile_h - 1) / tile_h);
    d->rows_off = -1;
    return MANDEL_OK;
}

int check_sched(const mandel_sched *s, mandel_sched *o)
{
    mandel_sched d;
    std::memset(&d, 0, sizeof d);
    if (s)
        d = *s;
    if (d.policy < MANDEL_FCFS_TILES || d.policy > MANDEL_GRID_TILES)
        return fail(MANDEL_EINVAL, "unknown policy %d", d.policy);
    if (d.tile_w == 0)
        d.tile_w = 64;
    if (d.tile_h == 0)
        d.tile_h = 8;
    if (d.tile_w < 1 || d.tile_h < 1 || (int64_t)d.tile_w * d.tile_h > (1 << 20))
        return fail(MANDEL_EINVAL, "bad tile shape %d x %d", d.tile_w, d.tile_h);
    if (d.grain == 0)
        d.grain = 1;
    if (d.grain < 1 || d.grain > (1 << 20))
        return fail(MANDEL_EINVAL, "bad grain %d", d.grain);
    if (d.waves_per_group == 0)
        d.waves_per_group = 4;
    if (d.waves_per_group < 1 || d.waves_per_group > 16)
        return fail(MANDEL_EINVAL, "waves_per_group=%d outside [1, 16]", d.waves_per_group);
    if (d.workers < 0)
        return fail(MANDEL_EINVAL, "negative workers");
    if ((d.policy == MANDEL_STATIC_ROWS || d.policy == MANDEL_ALTERNATING_ROWS) && d.workers < 1)
        return fail(MANDEL_EINVAL, "row policies need workers >= 1");
    if (d.check_every != 0 && d.check_every != 1)
        return fail(MANDEL_EINVAL, "check_every must be 0 or 1");
    if (d.periodicity != 0 && d.periodicity != 1)
        return fail(MANDEL_EINVAL, "periodicity must be 0 or 1");
    if (d.periodicity && d.check_every)
        return fail(MANDEL_EINVAL, "periodicity detection needs deferred tests (check_every 0)");
    if (d.block_iters == 0)
        d.block_iters = 1024;
    if (d.block_iters < 1 || d.block_iters > 65536)
        return fail(MANDEL_EINVAL, "block_iters=%d outside [1, 65536]", d.block_iters);
    if (d.young_iters == 0)
        d.young_iters = 4;
    if (d.young_iters < 0)
        return fail(MANDEL_EINVAL, "negative young_iters");
    if (d.refill_lanes == 0)
        d.refill_lanes = 16;
    if (d.refill_lanes < 1 || d.refill_lanes > 64)
        return fail(MANDEL_EINVAL, "refill_lanes=%d outside [1, 64]", d.refill_lanes);
    if (d.tile_parts == 0)
        d.tile_parts = 1;
    if (d.tile_parts != MANDEL_TILE_PARTS_AUTO && (d.tile_parts < 1 || d.tile_parts > 64))
        return fail(MANDEL_EINVAL, "tile_parts=%d outside [1, 64] and not automatic",
                    d.tile_parts);
    if (d.policy != MANDEL_FCFS_TILES && d.policy != MANDEL_ORDERED_TILES)
        d.tile_parts = 1;
    if (d.tile_parts == MANDEL_TILE_PARTS_AUTO && d.first_slot != 0)
        return fail(MANDEL_EINVAL, "first_slot needs an explicit tile_parts");
    if (d.first_slot < 0)
        return fail(MANDEL_EINVAL, "negative first_slot");
    if (d.first_slot != 0 && d.policy != MANDEL_FCFS_TILES && d.policy != MANDEL_ORDERED_TILES)
        return fail(MANDEL_EINVAL, "first_slot applies to the queue policies only");
    if (d.tile_time && (d.policy == MANDEL_STATIC_ROWS || d.policy == MANDEL_ALTERNATING_ROWS))
        return fail(MANDEL_EINVAL, "tile_time applies to the tile policies only");
    *o = d;
    return MANDEL_OK;
}

// Escape-test schedule of a checked schedule.
int test_mode(const mandel_sched &s)
{
    if (s.check_every)
        return TESTS_EVERY_UPDATE;
    return s.periodicity ? TESTS_DEFERRED_PERIODIC : TESTS_DEFERRED;
}

// Launch geometry for a tile policy: persistent groups or one group per tile.
// MANDEL_TILE_PARTS_AUTO.  Row parts let several wavefronts share one expensive tile, so
// an image of few tiles per wavefront does not end on a few tiles claimed late; but
// every part is a claim on the one queue head, and claims of cheap parts queue there.
// r = the fewest parts that give AUTO_ITEMS_PER_WAVE queue items per resident wavefront;
// the parts are the largest power of two not above r (parts of equal height in a tile of
// 8 rows), at most 8; then halved while a part would hold fewer than AUTO_MIN_PART_WORK
// pixel-iterations at max_iter, unless the whole queue is at most 2 items per
// wavefront; at most the tile's rows.  Measured on single views with 64 x 8 tiles
// (FCFS) over 7168 wavefronts, medians of 7 on several boxes: a 2048^2 full view (8192
// tiles) 4.5-4.7 ms in one part, 2.6 in 4, 2.5 in 8; the 4096^2 one 9.1-9.4 ms in one
// part, 7.5-7.8 in 4, 7.8-8.2 in 8; the 8192^2 one 26.5-27.3 ms in one part, 25.5-26.8
// in 2, 30.3-31.1 in 8 (10^6 claims queue on the head); but at max_iter 200 the 8192^2
// view takes 1.8 ms in one part and 3.3 in 2, and the 8000^2 view at max_iter 2000
// 6.0-6.2 ms in one part and 6.5-6.6 in 2.
constexpr int64_t AUTO_ITEMS_PER_WAVE = 24;
constexpr int64_t AUTO_MIN_PART_WORK = (int64_t)1 << 20;

int32_t auto_tile_parts(int64_t ntiles, int64_t waves, int32_t tile_w, int32_t tile_h,
                        int32_t max_iter)
{
    if (ntiles <= 0)
        return 1;
    const int64_t r = (AUTO_ITEMS_PER_WAVE * waves + ntiles - 1) / ntiles;
    int64_t parts = 1;
    while (parts * 2 <= r && parts < 8)
        parts *= 2;
    const int64_t tile_work = (int64_t)tile_w * tile_h * max_iter;
    while (parts > 1 && ntiles * parts > 2 * waves && tile_work / parts < AUTO_MIN_PART_WORK)
        parts /= 2;
    return (int32_t)(parts < tile_h ? parts : tile_h);
}

int tile_grid(const mandel_sched &s, bool batch, int64_t ntiles, dim3 *grid, dim3 *block)
{
    if (s.policy == MANDEL_GRID_TILES) {
        if (ntiles > (int64_t)1 << 26)
            return fail(MANDEL_EINVAL, "GRID_TILES launch limited to 2^26 tiles");
        unsigned gx = (unsigned)(ntiles < 65535 ? ntiles : 65535);
        unsigned gy = (unsigned)((ntiles + gx - 1) / gx);
        *grid = dim3(gx, gy);
        *block = dim3(64);
        return MANDEL_OK;
    }
    const int threads = 64 * s.waves_per_group;
    int groups = s.workers;
    if (groups == 0) {
        int cus = 0;
        int rc = device_cus(&cus);
        if (rc)
            return rc;
        groups = cus * persistent_blocks_per_cu(s.policy, batch, test_mode(s), threads);
    }
    *grid = dim3((unsigned)groups);
    *block = dim3((unsigned)threads);
    return MANDEL_OK;
}

} // namespace mandel

using namespace mandel;

extern "C" {

const char *mandel_last_error(void) { return g_err.c_str(); }

const char *mandel_version(void) { return "mandel-gfx950 0.1"; }

int mandel_device_info(int32_t *compute_units, int32_t *wall_clock_khz)
{
    clear_error();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    int v = 0;
    if (compute_units) {
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess)
            return hip_fail(e, "hipDeviceGetAttribute");
        *compute_units = v;
    }
    if (wall_clock_khz) {
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess)
            return hip_fail(e, "hipDeviceGetAttribute");
        *wall_clock_khz = v;
    }
    return MANDEL_OK;
}

int64_t mandel_tile_count(int32_t m, int32_t n, int32_t tile_w, int32_t tile_h)
{
    return tile_count(m, n, tile_w, tile_h);
}

static int render_sched(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter, double R,
                        int32_t *out, const mandel_sched *sp, void *stream, bool noalloc)
{
    clear_error();
    mandel_sched s;
    int rc = check_sched(sp, &s);
    if (rc)
        return rc;
    ViewDesc v;
    rc = make_view(w, m, n, max_iter, R, s.tile_w, s.tile_h, &v);
    if (rc)
        return rc;
    if (m == 0 || n == 0)
        return MANDEL_OK; // an empty image: nothing to order either
    if (!out)
        return fail(MANDEL_EINVAL, "out is NULL");
    if (s.policy == MANDEL_ORDERED_TILES && !s.order)
        return fail(MANDEL_EINVAL, "ORDERED_TILES needs an order array");
    hipStream_t st = (hipStream_t)stream;
    const bool rows = s.policy == MANDEL_STATIC_ROWS || s.policy == MANDEL_ALTERNATING_ROWS;
    const int64_t ntiles = rows ? (int64_t)m : tile_count(m, n, s.tile_w, s.tile_h);

    RenderArgs a;
    std::memset(&a, 0, sizeof a);
    a.v0 = v;
    a.v0.out_off = 0;
    a.v0.tile_off = 0;
    a.views = nullptr;
    a.nviews = 1;
    a.tile_w = s.tile_w;
    a.tile_h = s.tile_h;
    a.grain = s.grain;
    a.ntiles = ntiles;
    a.block_iters = s.block_iters;
    a.young_iters = s.young_iters;
    a.refill_lanes = s.refill_lanes;
    a.parts = s.tile_parts;
    a.first_slot = s.first_slot;
    a.out = out;
    a.order = s.order;
    a.tile_cost = rows ? nullptr : s.tile_cost;
    a.claims = s.claims;
    a.tile_time = s.tile_time;
    a.stats = s.stats;

    unsigned long long *head = nullptr;
    rc = noalloc ? scratch_head(&head) : workspace_head(st, &head);
    if (rc)
        return rc;
    a.head = head;

    dim3 grid, block;
    if (rows) {
        grid = dim3((unsigned)s.workers);
        block = dim3((unsigned)(64 * s.waves_per_group));
    } else {
        rc = tile_grid(s, false, ntiles, &grid, &block);
        if (rc)
            return rc;
        if (s.tile_parts == MANDEL_TILE_PARTS_AUTO) {
            // A window whose nearest point to 0 lies well outside the escape radius
            // escapes at the first test everywhere: its tiles are cheap, keep them whole.
            const double hx = 0.5 * (double)n * w->dx, hy = 0.5 * (double)m * w->dy;
            const double nx = std::fmax(0.0, std::fabs(w->cx0) - hx);
            const double ny = std::fmax(0.0, std::fabs(w->cy0) - hy);
            const bool outside = nx * nx + ny * ny > 1.0625 * R * R;
            a.parts = outside ? 1
                              : auto_tile_parts(ntiles,
                                                (int64_t)grid.x * grid.y * (block.x / 64),
                                                s.tile_w, s.tile_h, max_iter);
        }
    }
    hipError_t e = launch_clear(head, s.first_slot, a.tile_cost, a.claims, a.tile_time,
                                a.tile_cost || a.claims || a.tile_time ? ntiles : 0, a.stats,
                                st);
    if (e != hipSuccess)
        return hip_fail(e, "clear launch");
    e = launch_render(a, s.policy, false, test_mode(s), grid, block, st);
    if (e != hipSuccess)
        return hip_fail(e, "render launch");
    return MANDEL_OK;
}

int mandel_render_sched(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter,
                        double R, int32_t *out, const mandel_sched *sp, void *stream)
{
    return render_sched(w, m, n, max_iter, R, out, sp, stream, false);
}

int mandel_render_sched_noalloc(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter,
                                double R, int32_t *out, const mandel_sched *sp, void *stream)
{
    return render_sched(w, m, n, max_iter, R, out, sp, stream, true);
}

int mandel_render(const mandel_window *w, int32_t m, int32_t n, int32_t max_iter, double R,
                  int32_t *out, void *stream)
{
    mandel_sched s;
    std::memset(&s, 0, sizeof s);
    s.policy = MANDEL_FCFS_TILES;
    s.tile_parts = MANDEL_TILE_PARTS_AUTO;
    return mandel_render_sched(w, m, n, max_iter, R, out, &s, stream);
}

int mandel_colour_boolean(const int32_t *counts, int64_t npix, int32_t max_iter, uint8_t *rgb,
                          void *stream)
{
    clear_error();
    if (npix < 0)
        return fail(MANDEL_EINVAL, "negative pixel count");
    if (max_iter < 1)
        return fail(MANDEL_EINVAL, "max_iter=%d < 1", max_iter);
    if (npix == 0)
        return MANDEL_OK;
    if (!counts || !rgb)
        return fail(MANDEL_EINVAL, "counts or rgb is NULL");
    hipError_t e = launch_colour(counts, npix, max_iter, rgb, (hipStream_t)stream);
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "colour launch");
}

int mandel_write_ppm(const char *path, const uint8_t *rgb, int32_t m, int32_t n)
{
    clear_error();
    if (!path)
        return fail(MANDEL_EINVAL, "path is NULL");
    if (m < 0 || n < 0)
        return fail(MANDEL_EINVAL, "negative size m=%d n=%d", m, n);
    if (!rgb && (int64_t)m * n > 0)
        return fail(MANDEL_EINVAL, "rgb is NULL");
    if (write_ppm(path, rgb, m, n) != 0)
        return fail(MANDEL_EIO, "cannot write %s", path);
    return MANDEL_OK;
}

int mandel_render_dd(const mandel_window_dd *w, int32_t m, int32_t n, int32_t max_iter,
                     double R, int32_t *out, uint64_t *stats, void *stream)
{
    clear_error();
    if (!w)
        return fail(MANDEL_EINVAL, "window is NULL");
    if (m < 0 || n < 0)
        return fail(MANDEL_EINVAL, "negative size m=%d n=%d", m, n);
    if ((int64_t)m * (int64_t)n >= (int64_t(1) << 40))
        return fail(MANDEL_EINVAL, "image too large: %d x %d", m, n);
    if (max_iter < 1 || max_iter > (1 << 30))
        return fail(MANDEL_EINVAL, "max_iter=%d outside [1, 2^30]", max_iter);
    if (!std::isfinite(R) || !(R > 0.0) || R > 1e150)
        return fail(MANDEL_EINVAL, "escape radius R=%g outside (0, 1e150]", R);
    const double v[6] = {w->cx0_hi, w->cx0_lo, w->cy0_hi, w->cy0_lo, w->dx, w->dy};
    for (double x : v)
        if (!std::isfinite(x))
            return fail(MANDEL_EINVAL, "window has a non-finite value");
    if (!(w->dx > 0.0) || !(w->dy > 0.0))
        return fail(MANDEL_EINVAL, "pixel pitch must be > 0 (dx=%g dy=%g)", w->dx, w->dy);
    // every pixel centre within |re|, |im| <= 1e150, so no square of a state that
    // has not escaped can overflow
    const double ex = std::fabs(w->cx0_hi) + std::fabs(w->cx0_lo) + 0.5 * (double)n * w->dx;
    const double ey = std::fabs(w->cy0_hi) + std::fabs(w->cy0_lo) + 0.5 * (double)m * w->dy;
    if (!(ex <= 1e150) || !(ey <= 1e150))
        return fail(MANDEL_EINVAL, "window reaches beyond |c| = 1e150");
    if (m == 0 || n == 0)
        return MANDEL_OK;
    if (!out)
        return fail(MANDEL_EINVAL, "out is NULL");
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *head = nullptr;
    int rc = workspace_head(st, &head);
    if (rc)
        return rc;
    int cus = 0;
    rc = device_cus(&cus);
    if (rc)
        return rc;
    DDArgs a;
    std::memset(&a, 0, sizeof a);
    a.cx0h = w->cx0_hi;
    a.cx0l = w->cx0_lo;
    a.cy0h = w->cy0_hi;
    a.cy0l = w->cy0_lo;
    a.dx = w->dx;
    a.dy = w->dy;
    a.R2 = R * R;
    a.m = m;
    a.n = n;
    a.max_iter = max_iter;
    a.tile_w = 64;
    a.tile_h = 8;
    // in 64 bits: n + 63 overflows int32 for n near 2^31 (m = 1 is allowed there)
    a.tiles_x = (int32_t)(((int64_t)n + 63) / 64);
    a.ntiles = tile_count(m, n, 64, 8);
    a.out = out;
    a.head = head;
    a.stats = stats;
    const int threads = 256;
    const dim3 grid((unsigned)(cus * dd_blocks_per_cu(threads))), block(threads);
    hipError_t e = launch_clear(head, 0, nullptr, nullptr, nullptr, 0, nullptr, st);
    if (e != hipSuccess)
        return hip_fail(e, "clear launch");
    e = launch_render_dd(a, grid, block, st);
    if (e != hipSuccess)
        return hip_fail(e, "render launch");
    return MANDEL_OK;
}

} // extern "C"
