"""The double-double kernel writes add(2A, B) with the doubling folded into fma's:
every operation that reads 2a is evaluated as fma(+-2, a, t).  That is the same
rounding as fl(+-fl(2a) + t), because 2a is exact unless it overflows.  This test
checks the identity on the CPU (gcc, libm fma, no contraction) for two-sum and
for the accurate double-double addition, on random operands: magnitudes from
subnormal to 1e300, zeros, and near-cancelling pairs."""
import subprocess

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
typedef struct { double hi, lo; } dd;
static dd two_sum(double a, double b) { double s = a + b, v = s - a; dd r = {s, (a - (s - v)) + (b - v)}; return r; }
static dd fast_two_sum(double a, double b) { double s = a + b; dd r = {s, b - (s - a)}; return r; }
static dd add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
    double e = s.lo + t.hi; s = fast_two_sum(s.hi, e); e = s.lo + t.lo; return fast_two_sum(s.hi, e);
}
/* two_sum(2a, b) with 2a never formed */
static dd two_sum_twice(double a, double b) {
    double s = fma(2.0, a, b), v = fma(-2.0, a, s);
    dd r = {s, fma(2.0, a, -(s - v)) + (b - v)}; return r;
}
static dd add_twice(dd a, dd b) {
    dd s = two_sum_twice(a.hi, b.hi), t = two_sum_twice(a.lo, b.lo);
    double e = s.lo + t.hi; s = fast_two_sum(s.hi, e); e = s.lo + t.lo; return fast_two_sum(s.hi, e);
}
static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
static double draw(void) {
    double m = ldexp((double)(next() >> 11), -53) * ((next() & 1) ? -1.0 : 1.0);
    switch (next() % 6) {
    case 0: return ldexp(m, (int)(next() % 100) - 50);
    case 1: return ldexp(m, (int)(next() % 1990) - 1000);
    case 2: return ldexp(m, -1074 + (int)(next() % 60));
    case 3: return ldexp(m, 900 + (int)(next() % 96));
    case 4: return 0.0;
    default: return ldexp(m, (int)(next() % 8) - 4);
    }
}
int main(void) {
    long bad = 0, n = 0;
    for (long i = 0; i < 3000000; i++) {
        dd A = {draw(), 0.0}, B = {draw(), 0.0};
        A.lo = ldexp(draw(), -60) * (A.hi != 0.0 ? fabs(A.hi) : 1e-300);
        B.lo = ldexp(draw(), -60) * (B.hi != 0.0 ? fabs(B.hi) : 1e-300);
        if (i % 3 == 0) B.hi = -2.0 * A.hi * (1.0 + ldexp(draw(), -40));
        if (!(fabs(A.hi) <= 1e300 && fabs(B.hi) <= 1e300 && isfinite(A.lo) && isfinite(B.lo)))
            continue;
        dd A2 = {2.0 * A.hi, 2.0 * A.lo};
        dd p = two_sum(A2.hi, B.hi), q = two_sum_twice(A.hi, B.hi);
        dd r1 = add(A2, B), r2 = add_twice(A, B);
        n++;
        if (memcmp(&p, &q, sizeof p) || memcmp(&r1, &r2, sizeof r1)) bad++;
    }
    printf("%ld %ld\n", n, bad);
    return 0;
}
"""


def test_folded_doubling_is_bit_identical(tmp_path):
    src = tmp_path / "fold.c"
    exe = tmp_path / "fold"
    src.write_text(SRC)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", str(src), "-o", str(exe),
                    "-lm"], check=True)
    n, bad = map(int, subprocess.run([str(exe)], check=True, capture_output=True,
                                     text=True).stdout.split())
    assert n > 2_000_000
    assert bad == 0
