/*
 * Oracle support: the canonical binary64 exponential and natural logarithm
 * used by the oracle's FP32 mode.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.
 *
 * Why it exists.  The FP32 mode must produce per-Gaussian state (scales from
 * exp of log-scales, opacity from the logistic function, the opacity-aware
 * extent k^2 = 2 ln(o / tau) of Eq. 3) whose bits do not depend on which
 * libm evaluated the transcendental.  Each value is therefore computed in
 * binary64 by the fixed sequence of IEEE-754 operations below and rounded once
 * to binary32.  The GPU path carries its own, independently written copy of
 * the same published method; the two share no code.
 *
 * Method (textbook argument reduction, no table):
 *   exp(x): k = floor(x / ln2 + 1/2); r = (x - k*LN2_HI) - k*LN2_LO with ln2
 *           split into a 32-bit head and a tail (Cody & Waite, 1980);
 *           exp(r) by its Taylor series to degree 13 (|r| <= 0.35 so the
 *           truncation error is below 1e-17); result scaled by 2^k through
 *           two exact power-of-two multiplies.
 *   log(x): x = m * 2^e with m in (sqrt(1/2), sqrt(2)]; s = (m-1)/(m+1);
 *           ln m = 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23) (the atanh
 *           series; |s| <= 0.1716 so 11 terms reach 1e-17);
 *           ln x = e*LN2_HI + (ln m + e*LN2_LO).
 * The file is compiled with -ffp-contract=off, so every + - * / above is one
 * correctly rounded binary64 operation in the written order.
 */
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the oracle's parallel loops use (reported with timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of later parallel regions (the benchmark's single-thread baseline). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

#define ORC_LN2_HI 0x1.62e42fee00000p-1
#define ORC_LN2_LO 0x1.a39ef35793c76p-33
#define ORC_INV_LN2 0x1.71547652b82fep+0

static double orc_pow2i(int k) /* exact 2^k for -1022 <= k <= 1023 */
{
    uint64_t bits = (uint64_t)(k + 1023) << 52;
    double d;
    memcpy(&d, &bits, sizeof d);
    return d;
}

static double orc_floor(double x) /* exact floor for |x| < 2^52 */
{
    double t = (double)(int64_t)x;
    return (t > x) ? t - 1.0 : t;
}

double orc_exp_d(double x)
{
    if (x != x) return x;
    if (x > 709.8) return 1.0 / 0.0;
    if (x < -745.2) return 0.0;
    double k = orc_floor(x * ORC_INV_LN2 + 0.5);
    double r = (x - k * ORC_LN2_HI) - k * ORC_LN2_LO;
    /* Taylor coefficients 1/n!, n = 13 .. 2, each the binary64 nearest */
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    int ki = (int)k;
    int k1 = ki / 2;
    int k2 = ki - k1;
    return (p * orc_pow2i(k1)) * orc_pow2i(k2);
}

double orc_log_d(double x)
{
    if (x != x || x < 0.0) return 0.0 / 0.0;
    if (x == 0.0) return -1.0 / 0.0;
    if (x > 1.7976931348623157e308) return x;
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e;
    if ((bits >> 52) == 0) { /* subnormal: scale into the normal range first */
        double y = x * 0x1p64;
        memcpy(&bits, &y, sizeof bits);
        e = (int)((bits >> 52) & 0x7ff) - 1023 - 64;
    } else {
        e = (int)((bits >> 52) & 0x7ff) - 1023;
    }
    bits = (bits & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL;
    double m;
    memcpy(&m, &bits, sizeof m); /* m in [1, 2) */
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    double lnm = (2.0 * s) + (2.0 * s) * (z * p);
    double de = (double)e;
    return de * ORC_LN2_HI + (lnm + de * ORC_LN2_LO);
}
