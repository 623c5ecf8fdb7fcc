// Batch plans: many views rendered by one persistent launch over one flat tile
// space, optionally through a captured hipGraph, in FCFS, caller-given or
// predicted-longest-first order.  The operations are specified in
// include/mandel.h.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstring>
#include <algorithm>
#include <new>
#include <vector>

#include "costmodel.h"
#include "mandel.h"
#include "mandel_internal.h"
#include "render_kernels.h"
#include "row_collapse.h"

using namespace mandel;

namespace {

struct GraphEntry {
    int32_t *out;
    int32_t mode;
    const int32_t *order;
    const float *mlp;
    int64_t *tile_cost;
    uint64_t *stats;
    int32_t probe_cap;
    int32_t workers;
    int32_t periodicity;
    int64_t first_slot;
    uint64_t *tile_time;
    int32_t steal;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

} // namespace

struct mandel_plan {
    int device = 0;
    std::vector<ViewDesc> views;
    mandel_tuning tune{};
    int64_t ntiles = 0;
    int64_t npixels = 0;
    int64_t nrows = 0;
    int32_t min_max_iter = 1 << 30; // smallest max_iter of the views (automatic row parts)
    ViewDesc *d_views = nullptr;
    unsigned long long *d_head = nullptr;
    // buffers of the ordered modes (allocated on first use)
    float *d_feat = nullptr;
    float *d_keys = nullptr;
    int32_t *d_perm = nullptr;
    uint32_t *d_hist = nullptr;
    // buffers of row stealing (allocated on first use)
    int32_t *d_chunk = nullptr;
    int32_t *d_active = nullptr;
    int64_t active_len = 0;
    // collapsed rows (tuning.collapse_rows): the rendered rows of every collapsed view
    // (imaginary part, destination row) and the row copies that complete its image
    // after the render, as (destination, source) pairs
    RowRef *d_rows = nullptr;
    int32_t *d_pairs = nullptr;
    struct Expand {
        int32_t view;
        int64_t pairs_off; // first pair (pairs are int32[2])
        int32_t npairs;
    };
    std::vector<Expand> expands;
    hipStream_t capture = nullptr;
    std::vector<GraphEntry> graphs;
};


namespace {

// Rendered rows, and copied rows, of the collapsed views of one plan at most (each
// table takes 16 or 8 bytes per row on the host and on the device).
constexpr int64_t MAX_COLLAPSED_ROWS = (int64_t)1 << 28;

int fill_tuning(const mandel_tuning *t, mandel_tuning *o)
{
    mandel_tuning d;
    std::memset(&d, 0, sizeof d);
    if (t)
        d = *t;
    mandel_sched s;
    std::memset(&s, 0, sizeof s);
    s.policy = MANDEL_FCFS_TILES;
    s.tile_w = d.tile_w;
    s.tile_h = d.tile_h;
    s.grain = d.grain;
    s.waves_per_group = d.waves_per_group;
    s.block_iters = d.block_iters;
    s.young_iters = d.young_iters;
    s.refill_lanes = d.refill_lanes;
    s.tile_parts = d.tile_parts;
    s.workers = d.groups;
    mandel_sched c;
    int rc = check_sched(&s, &c);
    if (rc)
        return rc;
    d.tile_w = c.tile_w;
    d.tile_h = c.tile_h;
    d.grain = c.grain;
    d.waves_per_group = c.waves_per_group;
    d.block_iters = c.block_iters;
    d.young_iters = c.young_iters;
    d.refill_lanes = c.refill_lanes;
    d.tile_parts = c.tile_parts;
    d.groups = c.workers;
    if (d.collapse_rows < 0 || d.collapse_rows > 2)
        return fail(MANDEL_EINVAL, "collapse_rows must be 0, 1 or 2");
    *o = d;
    return MANDEL_OK;
}

int ensure_order_buffers(mandel_plan *p, bool need_feat)
{
    hipError_t e;
    if (!p->d_keys) {
        e = hipMalloc((void **)&p->d_keys, sizeof(float) * (size_t)(p->ntiles > 0 ? p->ntiles : 1));
        if (e != hipSuccess)
            return fail(MANDEL_ENOMEM, "hipMalloc(keys): %s", hipGetErrorString(e));
    }
    if (!p->d_perm) {
        e = hipMalloc((void **)&p->d_perm, sizeof(int32_t) * (size_t)(p->ntiles > 0 ? p->ntiles : 1));
        if (e != hipSuccess)
            return fail(MANDEL_ENOMEM, "hipMalloc(perm): %s", hipGetErrorString(e));
    }
    if (!p->d_hist) {
        e = hipMalloc((void **)&p->d_hist, sizeof(uint32_t) * 2 * MANDEL_ORDER_BUCKETS);
        if (e != hipSuccess)
            return fail(MANDEL_ENOMEM, "hipMalloc(order scratch): %s", hipGetErrorString(e));
    }
    if (need_feat && !p->d_feat) {
        e = hipMalloc((void **)&p->d_feat,
                      sizeof(float) * MANDEL_FEATURES * (size_t)(p->ntiles > 0 ? p->ntiles : 1));
        if (e != hipSuccess)
            return fail(MANDEL_ENOMEM, "hipMalloc(features): %s", hipGetErrorString(e));
    }
    return MANDEL_OK;
}

// Render policy of a plan launch mode.
int mode_policy(int32_t mode)
{
    switch (mode) {
    case MANDEL_PLAN_ORDERED:
    case MANDEL_PLAN_PROBE_LPT:
    case MANDEL_PLAN_LEARNED_LPT:
        return POLICY_ORDERED_TILES;
    case MANDEL_PLAN_STATIC_ROWS:
        return POLICY_STATIC_ROWS;
    case MANDEL_PLAN_ALTERNATING_ROWS:
        return POLICY_ALTERNATING_ROWS;
    default:
        return POLICY_FCFS_TILES;
    }
}

// Schedule and launch geometry of the render launch of a plan launch.
int render_grid(mandel_plan *p, const mandel_launch &la, mandel_sched *sc, dim3 *grid,
                dim3 *block)
{
    const int policy = mode_policy(la.mode);
    const bool rows = policy == POLICY_STATIC_ROWS || policy == POLICY_ALTERNATING_ROWS;
    std::memset(sc, 0, sizeof *sc);
    sc->policy = policy;
    sc->waves_per_group = p->tune.waves_per_group;
    sc->workers = rows ? la.workers : p->tune.groups;
    sc->periodicity = la.periodicity;
    return tile_grid(*sc, true, p->ntiles, grid, block);
}

// Row counters (one per tile) and the held-tile table (one entry per wavefront).  The
// table is sized once, at first use, for the largest launch any queue mode of this plan
// can make (FCFS or ordered, with or without periodicity detection: their resident
// group counts differ), so captured graphs, which hold its address and clear length,
// never see it reallocated.
int ensure_steal_buffers(mandel_plan *p)
{
    hipError_t e;
    if (!p->d_chunk) {
        e = hipMalloc((void **)&p->d_chunk, sizeof(int32_t) * (size_t)p->ntiles);
        if (e != hipSuccess)
            return fail(MANDEL_ENOMEM, "hipMalloc(row counters): %s", hipGetErrorString(e));
    }
    if (p->d_active)
        return MANDEL_OK;
    int64_t waves = 0;
    const int32_t modes[2] = {MANDEL_PLAN_FCFS, MANDEL_PLAN_ORDERED};
    for (int32_t mode : modes) {
        for (int32_t per = 0; per <= 1; ++per) {
            mandel_launch la;
            std::memset(&la, 0, sizeof la);
            la.mode = mode;
            la.periodicity = per;
            mandel_sched sc;
            dim3 grid, block;
            int rc = render_grid(p, la, &sc, &grid, &block);
            if (rc)
                return rc;
            const int64_t w = (int64_t)grid.x * (block.x / 64);
            waves = w > waves ? w : waves;
        }
    }
    e = hipMalloc((void **)&p->d_active, sizeof(int32_t) * (size_t)waves);
    if (e != hipSuccess)
        return fail(MANDEL_ENOMEM, "hipMalloc(held tiles): %s", hipGetErrorString(e));
    p->active_len = waves;
    return MANDEL_OK;
}

// Enqueues the whole launch sequence of one plan launch on stream s.
int enqueue(mandel_plan *p, int32_t *out, const mandel_launch &la, hipStream_t s)
{
    hipError_t e;
    const int32_t *order = nullptr;
    const int policy = mode_policy(la.mode);
    if (la.mode == MANDEL_PLAN_ORDERED) {
        order = la.order;
    } else if (la.mode == MANDEL_PLAN_PROBE_LPT || la.mode == MANDEL_PLAN_LEARNED_LPT) {
        e = launch_features(p->d_views, (int32_t)p->views.size(), p->d_rows, p->ntiles,
                            p->tune.tile_w,
                            p->tune.tile_h, la.probe_cap, p->d_feat, s);
        if (e != hipSuccess)
            return hip_fail(e, "features launch");
        if (la.mode == MANDEL_PLAN_PROBE_LPT)
            e = launch_probe_key(p->d_feat, p->ntiles, la.probe_cap, p->d_keys, s);
        else
            e = launch_mlp_forward(la.mlp, p->d_feat, p->ntiles, p->d_keys, s);
        if (e != hipSuccess)
            return hip_fail(e, "key launch");
        e = launch_order_desc(p->d_keys, p->ntiles, p->d_perm, p->d_hist, s);
        if (e != hipSuccess)
            return hip_fail(e, "order launch");
        order = p->d_perm;
    }
    const bool rows = policy == POLICY_STATIC_ROWS || policy == POLICY_ALTERNATING_ROWS;

    RenderArgs a;
    std::memset(&a, 0, sizeof a);
    a.v0 = p->views[0];
    a.views = p->d_views;
    a.nviews = (int32_t)p->views.size();
    a.tile_w = p->tune.tile_w;
    a.tile_h = p->tune.tile_h;
    a.grain = p->tune.grain;
    a.ntiles = p->ntiles;
    a.block_iters = p->tune.block_iters;
    a.young_iters = p->tune.young_iters;
    a.refill_lanes = p->tune.refill_lanes;
    a.first_slot = la.first_slot;
    a.nrows = p->nrows;
    a.rows = p->d_rows;
    a.out = out;
    a.head = rows ? nullptr : p->d_head;
    a.order = order;
    a.tile_cost = la.tile_cost;
    a.claims = nullptr;
    a.tile_time = la.tile_time;
    a.steal = la.steal;
    a.chunk = la.steal ? p->d_chunk : nullptr;
    a.active = la.steal ? p->d_active : nullptr;
    a.stats = la.stats;

    mandel_sched sc;
    dim3 grid, block;
    int rc = render_grid(p, la, &sc, &grid, &block);
    if (rc)
        return rc;
    // automatic row parts (single views: as mandel_render chooses them, but without its
    // test for windows outside the radius; batches with the smallest max_iter of their
    // views); row stealing takes whole tiles
    a.parts = p->tune.tile_parts;
    if (a.parts == MANDEL_TILE_PARTS_AUTO)
        a.parts = la.steal || rows ? 1
                                   : auto_tile_parts(p->ntiles,
                                                     (int64_t)grid.x * grid.y * (block.x / 64),
                                                     p->tune.tile_w, p->tune.tile_h,
                                                     p->min_max_iter);
    if (la.steal && (int64_t)grid.x * (block.x / 64) > p->active_len)
        return fail(MANDEL_EINVAL, "held-tile table smaller than the launch");
    e = launch_clear(rows ? nullptr : p->d_head, la.first_slot, la.tile_cost, nullptr,
                     la.tile_time, la.tile_cost || la.tile_time || la.steal ? p->ntiles : 0,
                     la.stats, s, a.chunk, a.active, la.steal ? p->active_len : 0);
    if (e != hipSuccess)
        return hip_fail(e, "clear launch");
    e = launch_render(a, policy, true, test_mode(sc), grid, block, s);
    if (e != hipSuccess)
        return hip_fail(e, "render launch");
    for (const mandel_plan::Expand &x : p->expands) {
        const ViewDesc &v = p->views[(size_t)x.view];
        e = launch_expand_rows(out + v.out_off, v.n, p->d_pairs + 2 * x.pairs_off, x.npairs, s);
        if (e != hipSuccess)
            return hip_fail(e, "row expansion launch");
    }
    return MANDEL_OK;
}

// Collapsed rows (planned by plan_row_collapse): view k is rendered as its distinct
// rows, each written to the image row where its key first occurs, and the copies of
// the other rows are queued for after the render.
int collapse_rows(mandel_plan *p, int32_t k, bool mirror, std::vector<RowRef> &rows,
                  std::vector<int32_t> &pairs)
{
    ViewDesc &d = p->views[(size_t)k];
    RowCollapse rc;
    plan_row_collapse(d.cy0, d.dy, d.m, mirror, rc);
    const int64_t copies = (int64_t)rc.pairs.size() / 2;
    if (copies == 0)
        return MANDEL_OK; // every row distinct
    if ((int64_t)rows.size() + (int64_t)rc.cy.size() > MAX_COLLAPSED_ROWS ||
        (int64_t)pairs.size() / 2 + copies > MAX_COLLAPSED_ROWS)
        return fail(MANDEL_EINVAL, "view %d: more than 2^28 rendered or copied rows in the "
                    "collapsed views of one plan", k);
    d.rows_off = (int32_t)rows.size();
    for (size_t r = 0; r < rc.cy.size(); ++r)
        rows.push_back({rc.cy[r], d.out_off + (int64_t)rc.first[r] * d.n});
    const int64_t pairs_off = (int64_t)pairs.size() / 2;
    pairs.insert(pairs.end(), rc.pairs.begin(), rc.pairs.end());
    d.m = (int32_t)rc.cy.size();
    d.tiles_y = (int32_t)(((int64_t)d.m + p->tune.tile_h - 1) / p->tune.tile_h);
    p->expands.push_back({k, pairs_off, (int32_t)copies});
    return MANDEL_OK;
}

} // namespace

extern "C" {

int mandel_plan_create(const mandel_view *views, int32_t nviews, const mandel_tuning *tuning,
                       mandel_plan **plan)
{
    clear_error();
    if (!plan)
        return fail(MANDEL_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!views || nviews < 1 || nviews > (1 << 24))
        return fail(MANDEL_EINVAL, "need 1 <= nviews <= 2^24 and a view array");
    mandel_tuning tu;
    int rc = fill_tuning(tuning, &tu);
    if (rc)
        return rc;
    mandel_plan *p = new (std::nothrow) mandel_plan();
    if (!p)
        return fail(MANDEL_ENOMEM, "host allocation failed");
    p->tune = tu;
    int64_t toff = 0, npx = 0;
    std::vector<RowRef> rows;
    std::vector<int32_t> pairs;
    try { // the host tables of a large plan may not fit
        p->views.resize((size_t)nviews);
        for (int32_t k = 0; k < nviews; ++k) {
            const mandel_view &v = views[k];
            rc = make_view(&v.w, v.m, v.n, v.max_iter, v.R, tu.tile_w, tu.tile_h, &p->views[k]);
            if (rc) {
                delete p;
                return fail(rc, "view %d: %s", k, mandel_last_error());
            }
            if (v.out_offset < 0) {
                delete p;
                return fail(MANDEL_EINVAL, "view %d: negative out_offset", k);
            }
            ViewDesc &d = p->views[k];
            d.out_off = v.out_offset;
            if (tu.collapse_rows && v.m > 1 && v.n > 0) {
                rc = collapse_rows(p, k, tu.collapse_rows == 2, rows, pairs);
                if (rc) {
                    delete p;
                    return rc;
                }
            }
            if (d.max_iter < p->min_max_iter)
                p->min_max_iter = d.max_iter;
            d.tile_off = toff;
            d.row_off = p->nrows;
            toff += tile_count(d.m, d.n, tu.tile_w, tu.tile_h);
            p->nrows += d.m;
            npx += (int64_t)v.m * v.n;
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(MANDEL_ENOMEM, "host allocation failed");
    }
    if (toff >= ((int64_t)1 << 31)) {
        delete p;
        return fail(MANDEL_EINVAL, "plan has %lld tiles (limit 2^31 - 1)", (long long)toff);
    }
    p->ntiles = toff;
    p->npixels = npx;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess)
        e = hipMalloc((void **)&p->d_views, sizeof(ViewDesc) * (size_t)nviews);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_views, p->views.data(), sizeof(ViewDesc) * (size_t)nviews,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMalloc((void **)&p->d_head, HEAD_BYTES);
    if (e == hipSuccess && !rows.empty()) {
        e = hipMalloc((void **)&p->d_rows, sizeof(RowRef) * rows.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_rows, rows.data(), sizeof(RowRef) * rows.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMalloc((void **)&p->d_pairs, sizeof(int32_t) * pairs.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_pairs, pairs.data(), sizeof(int32_t) * pairs.size(),
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        mandel_plan_destroy(p);
        return hip_fail(e, "plan allocation");
    }
    *plan = p;
    return MANDEL_OK;
}

int mandel_plan_info(const mandel_plan *p, int64_t *ntiles, int64_t *npixels, mandel_tuning *t)
{
    clear_error();
    if (!p)
        return fail(MANDEL_EINVAL, "plan is NULL");
    if (ntiles)
        *ntiles = p->ntiles;
    if (npixels)
        *npixels = p->npixels;
    if (t)
        *t = p->tune;
    return MANDEL_OK;
}

int mandel_plan_launch(mandel_plan *p, int32_t *out, const mandel_launch *args, void *stream)
{
    clear_error();
    if (!p)
        return fail(MANDEL_EINVAL, "plan is NULL");
    mandel_launch la;
    std::memset(&la, 0, sizeof la);
    if (args)
        la = *args;
    if (la.mode < MANDEL_PLAN_FCFS || la.mode > MANDEL_PLAN_ALTERNATING_ROWS)
        return fail(MANDEL_EINVAL, "unknown plan mode %d", la.mode);
    const bool rows = la.mode == MANDEL_PLAN_STATIC_ROWS || la.mode == MANDEL_PLAN_ALTERNATING_ROWS;
    if (rows) {
        if (la.workers < 1)
            return fail(MANDEL_EINVAL, "row modes need workers >= 1");
        if (la.tile_cost || la.tile_time)
            return fail(MANDEL_EINVAL, "row modes log no per-tile data (tile_cost and tile_time "
                                       "must be NULL)");
        if (la.first_slot != 0)
            return fail(MANDEL_EINVAL, "row modes have no queue (first_slot must be 0)");
        if (p->nrows >= ((int64_t)1 << 31))
            return fail(MANDEL_EINVAL, "row modes need fewer than 2^31 rows (plan has %lld)",
                        (long long)p->nrows);
    } else if (la.workers != 0) {
        return fail(MANDEL_EINVAL, "workers applies to the row modes only");
    }
    if (rows && la.steal)
        return fail(MANDEL_EINVAL, "row stealing applies to the queue modes only");
    if (la.probe_cap == 0)
        la.probe_cap = 128;
    if (la.probe_cap < -(1 << 20) || la.probe_cap > (1 << 20))
        return fail(MANDEL_EINVAL, "probe_cap=%d outside [-2^20, 2^20]", la.probe_cap);
    if (la.first_slot < 0)
        return fail(MANDEL_EINVAL, "negative first_slot");
    if (la.first_slot != 0 && !p->expands.empty())
        return fail(MANDEL_EINVAL, "first_slot must be 0 on a plan with collapsed rows (the "
                                   "row copies after the render would overwrite skipped rows)");
    if (la.periodicity != 0 && la.periodicity != 1)
        return fail(MANDEL_EINVAL, "periodicity must be 0 or 1");
    if (la.reserved != 0)
        return fail(MANDEL_EINVAL, "reserved field must be 0");
    if (la.steal != 0 && la.steal != 1)
        return fail(MANDEL_EINVAL, "steal must be 0 or 1");
    if (la.reserved2 != 0)
        return fail(MANDEL_EINVAL, "reserved2 must be 0");
    if (la.steal && p->tune.tile_parts != 1 && p->tune.tile_parts != MANDEL_TILE_PARTS_AUTO)
        return fail(MANDEL_EINVAL, "row stealing needs tile_parts 1 (or automatic)");
    if (la.first_slot != 0 && p->tune.tile_parts == MANDEL_TILE_PARTS_AUTO)
        return fail(MANDEL_EINVAL, "first_slot needs an explicit tile_parts");
    if (la.steal && p->ntiles > INT32_MAX)
        return fail(MANDEL_EINVAL, "row stealing supports at most 2^31 - 1 tiles");
    if (p->ntiles == 0)
        return MANDEL_OK; // no tiles: nothing to order, no model needed
    if (!out)
        return fail(MANDEL_EINVAL, "out_base is NULL");
    if (la.mode == MANDEL_PLAN_ORDERED && !la.order)
        return fail(MANDEL_EINVAL, "ORDERED needs an order array");
    if (la.mode == MANDEL_PLAN_LEARNED_LPT && !la.mlp)
        return fail(MANDEL_EINVAL, "LEARNED_LPT needs model parameters");
    if (la.mode == MANDEL_PLAN_PROBE_LPT || la.mode == MANDEL_PLAN_LEARNED_LPT) {
        int rc = ensure_order_buffers(p, true);
        if (rc)
            return rc;
    }
    if (la.steal) {
        int rc = ensure_steal_buffers(p);
        if (rc)
            return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!la.use_graph)
        return enqueue(p, out, la, s);

    for (const GraphEntry &g : p->graphs) {
        if (g.out == out && g.mode == la.mode && g.order == la.order && g.mlp == la.mlp &&
            g.tile_cost == la.tile_cost && g.stats == la.stats && g.probe_cap == la.probe_cap &&
            g.workers == la.workers && g.periodicity == la.periodicity &&
            g.first_slot == la.first_slot && g.tile_time == la.tile_time &&
            g.steal == la.steal) {
            hipError_t e = hipGraphLaunch(g.exec, s);
            return e == hipSuccess ? MANDEL_OK : hip_fail(e, "hipGraphLaunch");
        }
    }
    GraphEntry g;
    g.out = out;
    g.mode = la.mode;
    g.order = la.order;
    g.mlp = la.mlp;
    g.tile_cost = la.tile_cost;
    g.stats = la.stats;
    g.probe_cap = la.probe_cap;
    g.workers = la.workers;
    g.periodicity = la.periodicity;
    g.first_slot = la.first_slot;
    g.tile_time = la.tile_time;
    g.steal = la.steal;
    g.graph = nullptr;
    g.exec = nullptr;
    hipError_t e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    int rc = enqueue(p, out, la, p->capture);
    e = hipStreamEndCapture(p->capture, &g.graph);
    if (rc || e != hipSuccess) {
        // nothing ran: drop whatever the capture recorded
        if (e == hipSuccess && g.graph)
            (void)hipGraphDestroy(g.graph);
        return rc ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    p->graphs.push_back(g);
    e = hipGraphLaunch(g.exec, s);
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "hipGraphLaunch");
}

int mandel_plan_features(mandel_plan *p, float *feat, int32_t probe_cap, void *stream)
{
    clear_error();
    if (!p)
        return fail(MANDEL_EINVAL, "plan is NULL");
    if (probe_cap == 0)
        probe_cap = 128;
    if (probe_cap < -(1 << 20) || probe_cap > (1 << 20))
        return fail(MANDEL_EINVAL, "probe_cap=%d outside [-2^20, 2^20]", probe_cap);
    if (p->ntiles == 0)
        return MANDEL_OK;
    if (!feat)
        return fail(MANDEL_EINVAL, "feat is NULL");
    hipError_t e = launch_features(p->d_views, (int32_t)p->views.size(), p->d_rows, p->ntiles,
                                   p->tune.tile_w, p->tune.tile_h, probe_cap, feat,
                                   (hipStream_t)stream);
    return e == hipSuccess ? MANDEL_OK : hip_fail(e, "features launch");
}

int mandel_plan_destroy(mandel_plan *p)
{
    clear_error();
    if (!p)
        return MANDEL_OK;
    (void)hipDeviceSynchronize();
    for (GraphEntry &g : p->graphs) {
        if (g.exec)
            (void)hipGraphExecDestroy(g.exec);
        if (g.graph)
            (void)hipGraphDestroy(g.graph);
    }
    if (p->capture)
        (void)hipStreamDestroy(p->capture);
    (void)hipFree(p->d_views);
    (void)hipFree(p->d_head);
    (void)hipFree(p->d_feat);
    (void)hipFree(p->d_keys);
    (void)hipFree(p->d_perm);
    (void)hipFree(p->d_hist);
    (void)hipFree(p->d_chunk);
    (void)hipFree(p->d_active);
    (void)hipFree(p->d_rows);
    (void)hipFree(p->d_pairs);
    delete p;
    return MANDEL_OK;
}

} // extern "C"
