/*
 * CPU oracle for the Boys functions -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library.  The GPU library never links it, and
 * this file uses no header, table or helper of the GPU library.
 *
 * What it computes: the exact Boys functions
 *
 *     F_k(x) = integral_0^1 t^(2k) exp(-x t^2) dt          (Sec. I, eq. 3)
 *
 * for k = 0..kmax at every argument, in x87 long double (64-bit mantissa),
 * i.e. about three orders of magnitude more accurate than the 5e-14 absolute
 * error the minimax method guarantees.  It is deliberately slow and plain:
 *
 *   x <= SERIES_MAX (30):
 *       F_kmax from the all-positive-terms series used by the paper for its
 *       reference values (Sec. II E, after Shavitt):
 *           F_K(x) = exp(-x)/2 * sum_{l>=0} x^l / prod_{j=0..l} (K + j + 1/2)
 *       then F_{kmax-1}..F_0 by the downward recurrence (Sec. II C)
 *           F_k = (2x F_{k+1} + exp(-x)) / (2k+1),
 *       which does not amplify errors.
 *
 *   x > SERIES_MAX:
 *       F_0 = 1/2 sqrt(pi/x) erf(sqrt(x))  (the k=0 integral in closed form),
 *       then F_1..F_kmax by the upward recurrence (Sec. II C)
 *           F_{k+1} = ((2k+1) F_k - exp(-x)) / (2x).
 *       Upward recurrence multiplies an error in F_k by (k+1/2)/x, and for
 *       x > 30 and k <= ORACLE_KMAX the product of these factors stays below
 *       one (this is the stability criterion of Appendix B, x >= x_0(kmax)).
 *
 * Series truncation.  The appendix states a relative truncation bound for the
 * series, but its last step bounds F_n(x) from above where a lower bound is
 * needed, so it is not a valid bound for small x.  This oracle uses instead
 * the geometric tail bound: the term ratio x/(K+l+1/2) decreases with l, so
 * once it is r < 1 the neglected remainder after term t_L is at most
 * |t_L| r/(1-r).  Summation stops when that is below 2^-72 of the sum.
 *
 * Domain: -1 <= x <= +inf (negative arguments only for finite differences
 * around 0; the series converges for every x).  x < -1 or NaN gives NaN;
 * x = +inf gives 0.  0 <= kmax <= ORACLE_KMAX.
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

#define ORACLE_KMAX 40
#define SERIES_MAX 30.0L

/* F_0..F_kmax at one argument, written to F[0..kmax]. */
static void boys_one(long double x, int kmax, long double *F)
{
    if (isnan(x) || x < -1.0L) {
        for (int k = 0; k <= kmax; ++k) F[k] = NAN;
        return;
    }
    if (isinf(x)) {
        for (int k = 0; k <= kmax; ++k) F[k] = 0.0L;
        return;
    }
    const long double emx = expl(-x);
    if (x <= SERIES_MAX) {
        /* Series for F_K with K = kmax. */
        const long double K = (long double)kmax;
        long double term = 1.0L / (K + 0.5L); /* l = 0 */
        long double sum = term;
        for (int l = 1; l < 100000; ++l) {
            term *= x / (K + (long double)l + 0.5L);
            sum += term;
            long double r = fabsl(x) / (K + (long double)l + 1.5L);
            if (r < 1.0L && fabsl(term) * r / (1.0L - r) <= ldexpl(fabsl(sum), -72))
                break;
        }
        F[kmax] = 0.5L * emx * sum;
        for (int k = kmax - 1; k >= 0; --k)
            F[k] = (2.0L * x * F[k + 1] + emx) / (2.0L * k + 1.0L);
    } else {
        const long double pi = 3.141592653589793238462643383279502884L;
        const long double s = sqrtl(x);
        F[0] = 0.5L * sqrtl(pi / x) * erfl(s);
        for (int k = 0; k < kmax; ++k)
            F[k + 1] = ((2.0L * k + 1.0L) * F[k] - emx) / (2.0L * x);
    }
}

/*
 * out[i*(kmax+1) + k] = F_k(x[i]) for i < n, k <= kmax, in long double.
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 for bad arguments.
 */
int oracle_boys_ld(const long double *x, int64_t n, int kmax, long double *out, int nthreads)
{
    if (n < 0 || kmax < 0 || kmax > ORACLE_KMAX || (n > 0 && (!x || !out)))
        return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i)
        boys_one(x[i], kmax, out + i * (int64_t)(kmax + 1));
    return 0;
}

/* Same as oracle_boys_ld for double arguments, results rounded to double. */
int oracle_boys_f64(const double *x, int64_t n, int kmax, double *out, int nthreads)
{
    if (n < 0 || kmax < 0 || kmax > ORACLE_KMAX || (n > 0 && (!x || !out)))
        return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
        long double F[ORACLE_KMAX + 1];
        boys_one((long double)x[i], kmax, F);
        for (int k = 0; k <= kmax; ++k)
            out[i * (int64_t)(kmax + 1) + k] = (double)F[k];
    }
    return 0;
}

/* Number of threads the OpenMP runtime would use by default. */
int oracle_max_threads(void) { return omp_get_max_threads(); }

int oracle_kmax_limit(void) { return ORACLE_KMAX; }
