/*
 * Escape-time Mandelbrot in double-double arithmetic: plain, slow,
 * single-threaded CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what the GPU library's
 * double-double render is checked against.  Only the test suite, the smoke
 * check and the CPU baseline leg of the benchmark may load it.  It shares no
 * code, header or constant with the GPU library.
 *
 * Build: gcc -O2 -std=gnu99 -ffp-contract=off -fno-fast-math -fPIC -shared -lm
 * (fma() is the C99 library function: one rounding of a*b + c).
 *
 * What is computed: the escape-time count of the paper (Sec. I, Eq. (1) and
 * Eq. (2)) for pixel spacings below the resolution of binary64, where adjacent
 * pixels would otherwise share one c.  Every quantity is an unevaluated sum
 * hi + lo of two binary64 numbers, and the operations are the classical
 * error-free transformations:
 *   two_sum(a, b)        s = a + b, v = s - a, e = (a - (s - v)) + (b - v)
 *                        (Knuth; s + e == a + b exactly)
 *   quick_two_sum(a, b)  s = a + b, e = b - (s - a)
 *                        (Dekker; exact when |a| >= |b|)
 *   two_prod(a, b)       p = a * b, e = fma(a, b, -p)    (p + e == a * b exactly)
 * built into
 *   add(A, B)  (s, e) = two_sum(A.hi, B.hi); (t, f) = two_sum(A.lo, B.lo);
 *              e = e + t; (s, e) = quick_two_sum(s, e); e = e + f;
 *              (s, e) = quick_two_sum(s, e)
 *   sqr(A)     (p, e) = two_prod(A.hi, A.hi); e = fma(A.hi + A.hi, A.lo, e);
 *              (p, e) = quick_two_sum(p, e)
 *   mul(A, B)  (p, e) = two_prod(A.hi, B.hi); e = fma(A.hi, B.lo, e);
 *              e = fma(A.lo, B.hi, e); (p, e) = quick_two_sum(p, e)
 * (the "accurate" addition and the products of Hida, Li and Bailey's
 * double-double library).  With these, one update is
 *   X' = add(add(sqr(X), -sqr(Y)), Cx),   Y' = add(2 * mul(X, Y), Cy)
 * where negation and doubling act on both parts exactly.  The escape test of a
 * state uses its high parts only, in plain binary64:
 *   escaped  <=>  fl(fl(X.hi * X.hi) + fl(Y.hi * Y.hi)) > R*R
 * (an overflow gives inf, which escapes), and the count is the first k >= 1
 * whose state z_k escapes, else max_iter, as in the binary64 definition.
 * Pixel centres: the window centre is itself double-double, the pitch dx, dy
 * binary64;  Cx = add((cx0_hi, cx0_lo), two_prod(((j + 0.5) - n/2), dx)),
 * likewise Cy with row i, m and dy.  Output is row-major, out[i*n + j].
 */
#include <math.h>
#include <stdint.h>

typedef struct {
    double hi, lo;
} dd;

static dd two_sum(double a, double b)
{
    dd r;
    double s = a + b;
    double v = s - a;
    r.hi = s;
    r.lo = (a - (s - v)) + (b - v);
    return r;
}

static dd quick_two_sum(double a, double b)
{
    dd r;
    double s = a + b;
    r.hi = s;
    r.lo = b - (s - a);
    return r;
}

static dd two_prod(double a, double b)
{
    dd r;
    double p = a * b;
    r.hi = p;
    r.lo = fma(a, b, -p);
    return r;
}

static dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    double e = s.lo + t.hi;
    s = quick_two_sum(s.hi, e);
    e = s.lo + t.lo;
    return quick_two_sum(s.hi, e);
}

static dd dd_sqr(dd a)
{
    dd p = two_prod(a.hi, a.hi);
    double e = fma(a.hi + a.hi, a.lo, p.lo);
    return quick_two_sum(p.hi, e);
}

static dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    double e = fma(a.hi, b.lo, p.lo);
    e = fma(a.lo, b.hi, e);
    return quick_two_sum(p.hi, e);
}

static dd dd_neg(dd a)
{
    dd r;
    r.hi = -a.hi;
    r.lo = -a.lo;
    return r;
}

static dd dd_twice(dd a)
{
    dd r;
    r.hi = 2.0 * a.hi;
    r.lo = 2.0 * a.lo;
    return r;
}

/* Error-free transformations and operations, exported for the pins. */
void oracle_dd_op(int32_t op, double ah, double al, double bh, double bl, double *rh,
                  double *rl)
{
    dd a = {ah, al}, b = {bh, bl}, r = {0.0, 0.0};
    switch (op) {
    case 0: r = two_sum(ah, bh); break;
    case 1: r = quick_two_sum(ah, bh); break;
    case 2: r = two_prod(ah, bh); break;
    case 3: r = dd_add(a, b); break;
    case 4: r = dd_sqr(a); break;
    case 5: r = dd_mul(a, b); break;
    default: break;
    }
    *rh = r.hi;
    *rl = r.lo;
}

/* Pixel centre c of pixel (i, j); window = {cx0_hi, cx0_lo, cy0_hi, cy0_lo, dx, dy};
 * c = {cx_hi, cx_lo, cy_hi, cy_lo}. */
void oracle_dd_pixel_c(const double win[6], int32_t m, int32_t n, int64_t i, int64_t j,
                       double c[4])
{
    dd cx0 = {win[0], win[1]}, cy0 = {win[2], win[3]};
    double off_x = ((double)j + 0.5) - (double)n / 2.0;
    double off_y = ((double)i + 0.5) - (double)m / 2.0;
    dd cx = dd_add(cx0, two_prod(off_x, win[4]));
    dd cy = dd_add(cy0, two_prod(off_y, win[5]));
    c[0] = cx.hi;
    c[1] = cx.lo;
    c[2] = cy.hi;
    c[3] = cy.lo;
}

/* The escape-time count of c = (cx_hi + cx_lo) + i (cy_hi + cy_lo). */
int32_t oracle_dd_escape_count(const double c[4], int32_t max_iter, double R)
{
    const double R2 = R * R;
    dd cx = {c[0], c[1]}, cy = {c[2], c[3]};
    dd x = {0.0, 0.0}, y = {0.0, 0.0};
    int32_t k;
    for (k = 1; k <= max_iter; ++k) {
        dd xx = dd_sqr(x);
        dd yy = dd_sqr(y);
        dd xy = dd_mul(x, y);
        dd xn = dd_add(dd_add(xx, dd_neg(yy)), cx);
        dd yn = dd_add(dd_twice(xy), cy);
        double sx, sy, s;
        x = xn;
        y = yn;
        sx = x.hi * x.hi;
        sy = y.hi * y.hi;
        s = sx + sy;
        if (s > R2)
            return k;
    }
    return max_iter;
}

/* Selected pixels: flat row-major indices idx[0..k) -> out[0..k). */
void oracle_dd_render_pixels(const double win[6], int32_t m, int32_t n, int32_t max_iter,
                             double R, const int64_t *idx, int64_t k, int32_t *out)
{
    int64_t t;
    for (t = 0; t < k; ++t) {
        double c[4];
        oracle_dd_pixel_c(win, m, n, idx[t] / n, idx[t] % n, c);
        out[t] = oracle_dd_escape_count(c, max_iter, R);
    }
}

/* Whole image, row-major. */
void oracle_dd_render(const double win[6], int32_t m, int32_t n, int32_t max_iter, double R,
                      int32_t *out)
{
    int64_t i, j;
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j) {
            double c[4];
            oracle_dd_pixel_c(win, m, n, i, j, c);
            out[i * (int64_t)n + j] = oracle_dd_escape_count(c, max_iter, R);
        }
}
