// Autotuner of batch plans: times candidate launch shapes on a sample of the
// batch and keeps the fastest, cached per device and batch signature.  The
// operation is specified in include/mandel.h (mandel_plan_autotune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "mandel.h"
#include "mandel_internal.h"

using namespace mandel;

namespace {

std::mutex g_tune_mu;
std::map<std::pair<int, uint64_t>, mandel_tuning> g_tune_cache;

uint64_t mix(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

uint64_t bits(double d)
{
    uint64_t u;
    std::memcpy(&u, &d, sizeof u);
    return u;
}

struct Candidate {
    int32_t tw, th, grain, wpg, parts, block;
};

// Tile shape, claim grain, waves per group, row parts, longest deferred block.  Short
// blocks pay where escapes are dense (an escape found at the end of a block replays
// the block with tests): on the uneven boundary-zoom batch 128 took 305 ms against
// 316 ms at 1024, while the 8192^2 full view was alike in FCFS order.
const Candidate kCandidates[] = {
    {64, 8, 1, 4, 1, 1024},  {32, 8, 1, 4, 1, 1024},  {64, 4, 1, 4, 1, 1024},
    {32, 4, 1, 4, 1, 1024},  {128, 4, 1, 4, 1, 1024}, {16, 16, 1, 4, 1, 1024},
    {64, 16, 1, 4, 4, 1024}, {128, 8, 1, 4, 2, 1024}, {64, 8, 4, 4, 1, 1024},
    {64, 8, 1, 4, 4, 1024},  {64, 8, 1, 4, 2, 1024},  {64, 8, 1, 1, 1, 1024},
    {32, 8, 1, 1, 1, 1024},  {64, 4, 1, 1, 1, 1024},  {32, 4, 2, 8, 1, 1024},
    {64, 8, 1, 4, 1, 128},   {64, 8, 1, 4, 4, 128},   {64, 16, 1, 4, 2, 128},
    {128, 16, 1, 4, 4, 128}, {128, 16, 1, 4, 4, 1024},
};

} // namespace

extern "C" int mandel_plan_autotune(const mandel_view *views, int32_t nviews, int32_t max_sample,
                                    mandel_tuning *best, int32_t *trials, void *stream)
{
    clear_error();
    if (!views || nviews < 1 || !best)
        return fail(MANDEL_EINVAL, "need views, nviews >= 1 and best");
    if (trials)
        *trials = 0;
    if (max_sample <= 0)
        max_sample = 8;
    hipStream_t st = (hipStream_t)stream;

    // Validate every view as a plan would, and rank the non-empty ones by a work proxy.
    std::vector<std::pair<double, int32_t>> work;
    for (int32_t k = 0; k < nviews; ++k) {
        ViewDesc d;
        int rc = make_view(&views[k].w, views[k].m, views[k].n, views[k].max_iter, views[k].R, 64,
                           8, &d);
        if (rc)
            return fail(rc, "view %d: %s", k, mandel_last_error());
        const double px = (double)views[k].m * (double)views[k].n;
        if (px > 0)
            work.push_back({px * (double)views[k].max_iter, k});
    }
    std::memset(best, 0, sizeof *best);
    best->tile_w = 64;
    best->tile_h = 8;
    best->grain = 1;
    best->waves_per_group = 4;
    best->block_iters = 1024;
    best->young_iters = 4;
    best->refill_lanes = 16;
    best->tile_parts = 1;
    if (work.empty())
        return MANDEL_OK;
    std::sort(work.begin(), work.end());
    std::vector<int32_t> pick;
    const int32_t ns = std::min<int32_t>(max_sample, (int32_t)work.size());
    for (int32_t q = 0; q < ns; ++q) {
        const size_t r = ns == 1 ? work.size() - 1 : (size_t)q * (work.size() - 1) / (ns - 1);
        if (pick.empty() || pick.back() != work[r].second)
            pick.push_back(work[r].second);
    }

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    uint64_t sig = mix(0, (uint64_t)nviews);
    for (int32_t k : pick) {
        const mandel_view &v = views[k];
        sig = mix(sig, (uint64_t)v.m);
        sig = mix(sig, (uint64_t)v.n);
        sig = mix(sig, (uint64_t)v.max_iter);
        sig = mix(sig, bits(v.R));
        sig = mix(sig, bits(v.w.cx0));
        sig = mix(sig, bits(v.w.cy0));
        sig = mix(sig, bits(v.w.dx));
        sig = mix(sig, bits(v.w.dy));
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find({dev, sig});
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return MANDEL_OK;
        }
    }

    // The sample, packed into one scratch image.
    std::vector<mandel_view> sample;
    int64_t total = 0;
    for (int32_t k : pick) {
        mandel_view v = views[k];
        v.out_offset = total;
        total += (int64_t)v.m * v.n;
        sample.push_back(v);
    }
    int32_t *scratch = nullptr;
    e = hipMalloc((void **)&scratch, sizeof(int32_t) * (size_t)total);
    if (e != hipSuccess)
        return fail(MANDEL_ENOMEM, "hipMalloc(autotune scratch): %s", hipGetErrorString(e));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        (void)hipFree(scratch);
        return hip_fail(e, "hipEventCreate");
    }

    float best_ms = 1e30f;
    int rc = MANDEL_OK;
    int32_t ntrials = 0;
    for (const Candidate &c : kCandidates) {
        mandel_tuning t;
        std::memset(&t, 0, sizeof t);
        t.tile_w = c.tw;
        t.tile_h = c.th;
        t.grain = c.grain;
        t.waves_per_group = c.wpg;
        t.block_iters = c.block;
        t.young_iters = 4;
        t.refill_lanes = 16;
        t.tile_parts = c.parts;
        mandel_plan *p = nullptr;
        rc = mandel_plan_create(sample.data(), (int32_t)sample.size(), &t, &p);
        if (rc)
            break;
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && rc == MANDEL_OK; ++rep) {
            mandel_launch la;
            std::memset(&la, 0, sizeof la);
            (void)hipEventRecord(e0, st);
            rc = mandel_plan_launch(p, scratch, &la, st);
            (void)hipEventRecord(e1, st);
            e = hipEventSynchronize(e1);
            if (rc == MANDEL_OK && e != hipSuccess)
                rc = hip_fail(e, "autotune trial");
            float m = 0.0f;
            if (rc == MANDEL_OK && rep > 0 && hipEventElapsedTime(&m, e0, e1) == hipSuccess)
                ms = std::min(ms, m);
            ++ntrials;
        }
        mandel_plan_destroy(p);
        if (rc)
            break;
        if (ms < best_ms) {
            best_ms = ms;
            *best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (trials)
        *trials = ntrials;
    if (rc)
        return rc;
    clear_error();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[{dev, sig}] = *best;
    return MANDEL_OK;
}
