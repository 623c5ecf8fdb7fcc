// Deep-zoom render in double-double arithmetic for gfx950 (CDNA4, wave64).
//
// The count is the paper's escape-time count (Sec. I, Eq. (1) and Eq. (2));
// only the number format changes.  When the pixel pitch falls below the
// resolution of binary64 near c (about 1e-16 |c|), neighbouring pixels would
// share one c; here every value is an unevaluated sum hi + lo of two binary64
// numbers, built from error-free transformations (Knuth's two-sum, Dekker's
// fast two-sum, and the fma-based exact product), with the accurate addition
// and the products of Hida, Li and Bailey's double-double library:
//   add(A, B)  (s, e) = two_sum(A.hi, B.hi); (t, f) = two_sum(A.lo, B.lo);
//              e += t; (s, e) = quick_two_sum(s, e); e += f; quick_two_sum(s, e)
//   sqr(A)     (p, e) = two_prod(A.hi, A.hi); e = fma(A.hi + A.hi, A.lo, e); ...
//   mul(A, B)  (p, e) = two_prod(A.hi, B.hi); e = fma(A.hi, B.lo, e);
//              e = fma(A.lo, B.hi, e); quick_two_sum(p, e)
// One update is X' = add(add(sqr(X), -sqr(Y)), Cx), Y' = add(2 mul(X, Y), Cy);
// the escape test of a state is fl(fl(X.hi^2) + fl(Y.hi^2)) > R^2 (overflow
// gives inf, which escapes), and X.hi^2 is also the first product of the next
// sqr(X).  Pixel centre: C = add(centre, two_prod((j + 0.5) - n/2, dx)).
// Every operation is one IEEE binary64 rounding (add, mul, fma), evaluated in
// exactly this order, so the counts equal a CPU evaluation bit for bit.
//
// Work distribution: persistent wavefronts claim tiles from a device-wide
// atomic queue (the analogue of the paper's first-come-first-served rows,
// Sec. III-B); lanes whose pixel finished take the next pixels of the tile
// (ballot + mbcnt) once 4 lanes are idle.  Each update is about 80 FP64
// operations, so the test after every update costs little and no deferred
// blocks are used.  The doubling in Y' is folded into the fma's of the add
// (82 FP64 instructions per update instead of 84, the same roundings).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_kernels.h"

#pragma clang fp contract(off)

namespace mandel {

namespace {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b)
{
    const double s = a + b;
    const double v = s - a;
    return {s, (a - (s - v)) + (b - v)};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b)
{
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    double e = s.lo + t.hi;
    s = quick_two_sum(s.hi, e);
    e = s.lo + t.lo;
    return quick_two_sum(s.hi, e);
}

// two_sum(2a, b) and add(2A, B) without forming 2a: 2a is exact, so every
// operation that reads it, fl(2a + t) or fl(t - 2a), is one fma with the factor
// +-2.  Exact when 2a does not overflow; the update applies them to A = mul(X, Y)
// of a state that has not escaped, whose |X|, |Y| <= R <= 1e150.
__device__ __forceinline__ dd two_sum_2a(double a, double b)
{
    const double s = __builtin_fma(2.0, a, b);
    const double v = __builtin_fma(-2.0, a, s);
    return {s, __builtin_fma(2.0, a, -(s - v)) + (b - v)};
}

__device__ __forceinline__ dd dd_add_2a(dd a, dd b)
{
    dd s = two_sum_2a(a.hi, b.hi);
    const dd t = two_sum_2a(a.lo, b.lo);
    double e = s.lo + t.hi;
    s = quick_two_sum(s.hi, e);
    e = s.lo + t.lo;
    return quick_two_sum(s.hi, e);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off >= 1; off >>= 1)
        v += (uint64_t)__shfl_xor((long long)v, off, 64);
    return v;
}

constexpr uint32_t DD_REFILL_LANES = 4; // idle lanes that trigger a refill round (swept: 4, 8, 16)

} // namespace

__global__ void __launch_bounds__(256) render_dd_kernel(DDArgs a)
{
    const uint32_t lane = __lane_id();

    // wave-uniform: current tile and the next pixel within it
    int32_t s_x0 = 0, s_y0 = 0, s_w = 1, s_next = 0, s_cnt = 0;
    int64_t taken = 0;
    bool exhausted = false;

    auto next_tile = [&]() -> bool {
        unsigned long long q = 0;
        if (lane == 0)
            q = atomicAdd(a.head, 1ull);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)q);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(q >> 32));
        const int64_t t = (int64_t)(((uint64_t)hi << 32) | lo);
        if (t >= a.ntiles)
            return false;
        const int32_t ty = (int32_t)(t / a.tiles_x);
        const int32_t tx = (int32_t)(t - (int64_t)ty * a.tiles_x);
        s_x0 = tx * a.tile_w;
        s_y0 = ty * a.tile_h;
        s_w = a.n - s_x0 < a.tile_w ? a.n - s_x0 : a.tile_w;
        const int32_t h = a.m - s_y0 < a.tile_h ? a.m - s_y0 : a.tile_h;
        s_next = 0;
        s_cnt = s_w * h;
        ++taken;
        return true;
    };

    // per lane: state z = (xh + xl) + i (yh + yl), its test products, c, progress
    double xh = 0.0, xl = 0.0, yh = 0.0, yl = 0.0;
    double pxx = 0.0, pyy = 0.0; // fl(xh * xh), fl(yh * yh) of the current state
    double cxh = 0.0, cxl = 0.0, cyh = 0.0, cyl = 0.0;
    int32_t k = 0;               // updates done
    int64_t oidx = 0;
    bool active = false;
    uint64_t acc = 0, steps = 0;

    auto refill = [&]() {
        for (;;) {
            const uint64_t need = ballot(!active);
            if (need == 0 || exhausted)
                break;
            if (s_next >= s_cnt) {
                if (!next_tile())
                    exhausted = true;
                continue;
            }
            const int32_t avail = s_cnt - s_next;
            const int32_t kk = (int32_t)__popcll(need);
            const int32_t take = kk < avail ? kk : avail;
            const uint32_t rk = rank_in(need);
            if (!active && (int32_t)rk < take) {
                const int32_t p = s_next + (int32_t)rk;
                const int32_t i = s_y0 + p / s_w;
                const int32_t j = s_x0 + p % s_w;
                const double offx = ((double)j + 0.5) - 0.5 * (double)a.n;
                const double offy = ((double)i + 0.5) - 0.5 * (double)a.m;
                const dd cx = dd_add({a.cx0h, a.cx0l}, two_prod(offx, a.dx));
                const dd cy = dd_add({a.cy0h, a.cy0l}, two_prod(offy, a.dy));
                cxh = cx.hi;
                cxl = cx.lo;
                cyh = cy.hi;
                cyl = cy.lo;
                xh = xl = yh = yl = 0.0;
                pxx = pyy = 0.0;
                k = 0;
                oidx = (int64_t)i * a.n + j;
                active = true;
            }
            s_next += take;
        }
    };

    // z_k -> z_{k+1}, then the test of z_{k+1}; a lane stops at its count.
    auto step = [&]() {
        if (active) {
            // sqr(X), sqr(Y), mul(X, Y); pxx, pyy are the rounded high products
            double e = __builtin_fma(xh, xh, -pxx);
            e = __builtin_fma(xh + xh, xl, e);
            const dd XX = quick_two_sum(pxx, e);
            e = __builtin_fma(yh, yh, -pyy);
            e = __builtin_fma(yh + yh, yl, e);
            const dd YY = quick_two_sum(pyy, e);
            const double pxy = xh * yh;
            e = __builtin_fma(xh, yh, -pxy);
            e = __builtin_fma(xh, yl, e);
            e = __builtin_fma(xl, yh, e);
            const dd XY = quick_two_sum(pxy, e);
            const dd X = dd_add(dd_add(XX, {-YY.hi, -YY.lo}), {cxh, cxl});
            const dd Y = dd_add_2a(XY, {cyh, cyl}); // add(2 mul(X, Y), Cy)
            xh = X.hi;
            xl = X.lo;
            yh = Y.hi;
            yl = Y.lo;
            pxx = xh * xh;
            pyy = yh * yh;
            ++k;
            const bool esc = pxx + pyy > a.R2;
            if (esc || k == a.max_iter) {
                a.out[oidx] = k;
                acc += (uint64_t)k;
                active = false;
            }
        }
    };

    for (;;) {
        refill();
        if (ballot(active) == 0)
            break;
        for (;;) {
            step();
            step();
            step();
            step();
            steps += 4;
            const uint64_t act = ballot(active);
            if (act == 0 || ((uint32_t)__popcll(~act) >= DD_REFILL_LANES && !exhausted))
                break;
        }
    }

    if (a.stats) {
        const uint64_t tot = wave_sum_u64(acc);
        if (lane == 0) {
            atomicAdd((unsigned long long *)&a.stats[0], (unsigned long long)steps);
            atomicAdd((unsigned long long *)&a.stats[1], (unsigned long long)tot);
            atomicAdd((unsigned long long *)&a.stats[2], 1ull);
            atomicAdd((unsigned long long *)&a.stats[3], (unsigned long long)taken);
        }
    }
}

hipError_t launch_render_dd(const DDArgs &a, dim3 grid, dim3 block, hipStream_t s)
{
    hipLaunchKernelGGL(render_dd_kernel, grid, block, 0, s, a);
    return hipGetLastError();
}

int dd_blocks_per_cu(int threads)
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, render_dd_kernel, threads, 0);
    if (e != hipSuccess || nb < 1)
        return 1;
    return nb;
}

} // namespace mandel
