/*
 * Escape-time Mandelbrot oracle: plain, slow, single-threaded CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the definition that the GPU library
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header or
 * constant with the GPU library, and it must never be called from the product
 * path.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (no -march flag: baseline x86-64 has no FMA, and contraction is off anyway).
 *
 * What is computed (paper, Sec. I, Eq. (1) and Eq. (2)):
 *   each pixel (i, j) of an m x n image I gets a point c of the complex plane;
 *   z <- z^2 + c is applied repeatedly starting from z = 0; the iteration at
 *   which |z|^2 first exceeds the escape radius squared, or iterationMax if
 *   that never happens, is recorded as I[i][j].
 *
 * Readings where the paper is silent:
 *   - the test is |z|^2 > R*R, strict (the paper says the magnitude must
 *     exceed the escape radius);
 *   - count = min(max_iter, first k >= 1 with |z_k|^2 > R^2), so 1 <= count
 *     <= max_iter;
 *   - one IEEE binary64 rounding per written operation, evaluated in this
 *     order, nothing fused:
 *         x' = (x*x - y*y) + cx
 *         y' = 2*(x*y) + cy         (the product x*y is rounded, then doubled)
 *     and the escape test uses s = x'*x' + y'*y';
 *   - pixel centres: the window is given by its centre (cx0, cy0) and pixel
 *     pitch (dx, dy); column j and row i map to
 *         cx = cx0 + ((j + 0.5) - n/2) * dx
 *         cy = cy0 + ((i + 0.5) - m/2) * dy
 *     where the bracketed offset is an exact half-integer, then one multiply
 *     and one add, each rounded.  Output is row-major: out[i*n + j].
 */
#include <stdint.h>
#include <stddef.h>
#include <time.h>

/* Point c of pixel (i, j); window = {cx0, cy0, dx, dy}. */
void oracle_pixel_c(const double win[4], int32_t m, int32_t n,
                    int64_t i, int64_t j, double *cx, double *cy)
{
    double off_x = ((double)j + 0.5) - (double)n / 2.0;
    double off_y = ((double)i + 0.5) - (double)m / 2.0;
    double px = off_x * win[2];
    double py = off_y * win[3];
    *cx = win[0] + px;
    *cy = win[1] + py;
}

/* Eq. (1)-(2) for one point c: the escape-time count. */
int32_t oracle_escape_count(double cx, double cy, int32_t max_iter, double R)
{
    double R2 = R * R;
    double x = 0.0, y = 0.0;
    int32_t k;
    for (k = 1; k <= max_iter; ++k) {
        double xx = x * x;
        double yy = y * y;
        double xy = x * y;
        double diff = xx - yy;
        double twice = 2.0 * xy;
        double xn = diff + cx;
        double yn = twice + cy;
        double sx, sy, s;
        x = xn;
        y = yn;
        sx = x * x;
        sy = y * y;
        s = sx + sy;
        if (s > R2)
            return k;
    }
    return max_iter;
}

/* Whole image, row-major. */
void oracle_render(const double win[4], int32_t m, int32_t n, int32_t max_iter,
                   double R, int32_t *out)
{
    int64_t i, j;
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j) {
            double cx, cy;
            oracle_pixel_c(win, m, n, i, j, &cx, &cy);
            out[i * (int64_t)n + j] = oracle_escape_count(cx, cy, max_iter, R);
        }
}

/*
 * Rows row0, row0 + step, row0 + 2*step, ... (< m) into out, which holds the
 * full m x n image.  Used to split a large image over independent host
 * threads, each of which runs this same single-threaded loop.
 * Returns the seconds spent (CLOCK_MONOTONIC around the loop).
 */
double oracle_render_rows(const double win[4], int32_t m, int32_t n,
                          int32_t max_iter, double R, int64_t row0,
                          int64_t step, int32_t *out)
{
    struct timespec t0, t1;
    int64_t i, j;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (i = row0; i < m; i += step)
        for (j = 0; j < n; ++j) {
            double cx, cy;
            oracle_pixel_c(win, m, n, i, j, &cx, &cy);
            out[i * (int64_t)n + j] = oracle_escape_count(cx, cy, max_iter, R);
        }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}

/* Selected pixels: flat row-major indices idx[0..k) -> out[0..k). */
void oracle_render_pixels(const double win[4], int32_t m, int32_t n,
                          int32_t max_iter, double R, const int64_t *idx,
                          int64_t k, int32_t *out)
{
    int64_t t;
    for (t = 0; t < k; ++t) {
        int64_t i = idx[t] / n, j = idx[t] % n;
        double cx, cy;
        oracle_pixel_c(win, m, n, i, j, &cx, &cy);
        out[t] = oracle_escape_count(cx, cy, max_iter, R);
    }
}

/* Escape counts for an explicit list of points (cx[t], cy[t]). */
void oracle_escape_counts(const double *cx, const double *cy, int64_t k,
                          int32_t max_iter, double R, int32_t *out)
{
    int64_t t;
    for (t = 0; t < k; ++t)
        out[t] = oracle_escape_count(cx[t], cy[t], max_iter, R);
}
