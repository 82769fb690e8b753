/*
 * FP64 CPU oracle for the intensity-driven gradient filter.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU library.
 *
 * What it computes (Punzo, van der Hulst & Roerdink, "Finding faint H I
 * structure in and around galaxies: scraping the barrel", Section 3.3,
 * Eqs. 5-7): n explicit Jacobi steps of
 *
 *   I_{i+1}(v) = I_i(v) + tau * sum_a C_a * sum_{s=+-1} w(v, u) * (I_i(u) - I_i(v)),
 *   u = v + s e_a,
 *
 * where the weight w is one of
 *   INTENSITY   (Eq. 6, the paper's filter, Eq. 7):
 *               w = 1 / (1 + I_i(v)^2 / (K rho)^2)       (same for all six edges)
 *   PM_EXP      (Perona-Malik exponential edge-stopping function, per edge):
 *               w = exp(-((I_i(u) - I_i(v)) / (K rho))^2)
 *   PM_RATIONAL (Eq. 5 evaluated per edge with K in rms units):
 *               w = 1 / (1 + ((I_i(u) - I_i(v)) / (K rho))^2)
 *
 * rho is the cube's noise level: the caller's value if > 0, else the root mean
 * square of the input cube over all voxels, computed once before the first
 * step.  A neighbour outside the cube takes the voxel's own value (zero flux
 * through the cube faces).  Every step reads only I_i (two buffers, the
 * result-plus-temporary memory model of Section 5).
 *
 * Optional storage rounding: round_mode 1 (bfloat16), 2 (binary16) or 3
 * (binary32) rounds every voxel to the nearest representable value, ties to
 * even, after each step; the arithmetic of the step itself stays FP64.
 *
 * oracle_error_bound: a first-order running error bound (in the manner of
 * Wilkinson's running error analysis) for any computation of the same steps
 * that works in binary32 and rounds each voxel's new value once per step.
 * If every step adds at voxel v a local error of at most
 *     delta_i(v) = u (|I_{i+1}(v)| + sum_e c_e |T_e(v)|),   u = 2^-24,
 * where T_e is the flux term of edge e (tau C_a w d, or tau S C_a d for the
 * intensity form) and c_e bounds the relative error of computing it, then
 * the accumulated error obeys, to first order,
 *     B_{i+1}(v) = sum_u |dI_{i+1}(v) / dI_i(u)| B_i(u) + delta_i(v),  B_0 = 0,
 * the Jacobian taken at the exact FP64 trajectory.  c_e counts the unit
 * roundoffs one flux term can collect: the difference d (1), the product
 * that forms the term (1), five additions of the terms into the update (5),
 * and for the exponential weight (r = d / (K rho)) an exponential accurate to
 * 2 u whose argument, the base-2 exponent -log2(e) r^2 + log2(tau C) formed
 * from rounded d^2 and 1/(K rho)^2 with one multiply-add, is off by up to
 * u (5.8 r^2 + 4), i.e. a relative error of ln2 times that in the weight:
 * c_e = 12 + 4 r^2; for the rational weight d^2, the multiply-add, the
 * reciprocal (2) and the weight's constant: c_e = 14; for the intensity form
 * the reciprocal 1 / (1 + I^2 / (K rho)^2) and the scaling products: 14.
 * Second-order terms are of the order of B^2 and negligible.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of later parallel loops (n > 0; the calling thread's setting). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of threads the oracle's parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

enum { COND_INTENSITY = 0, COND_PM_EXP = 1, COND_PM_RATIONAL = 2 };
enum { ROUND_NONE = 0, ROUND_BF16 = 1, ROUND_F16 = 2, ROUND_F32 = 3 };

/* Round x to the nearest bfloat16 (8 significant bits), ties to even. */
double oracle_round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                       /* |x| in [2^(e-1), 2^e) */
    double q = ldexp(1.0, e - 1 - 7);   /* spacing of 8-bit significands */
    double qmin = ldexp(1.0, -133);     /* bfloat16 subnormal spacing */
    if (q < qmin) q = qmin;
    double r = nearbyint(x / q) * q;
    if (fabs(r) > 3.3895313892515355e38) r = copysign(INFINITY, x);
    return r;
}

/* Round x to the nearest IEEE binary16 (11 significant bits), ties to even. */
double oracle_round_f16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);
    double q = ldexp(1.0, e - 1 - 10);
    double qmin = ldexp(1.0, -24);      /* binary16 subnormal spacing */
    if (q < qmin) q = qmin;
    double r = nearbyint(x / q) * q;
    if (fabs(r) > 65504.0) r = copysign(INFINITY, x);
    return r;
}

static double round_store(double x, int mode)
{
    if (mode == ROUND_BF16) return oracle_round_bf16(x);
    if (mode == ROUND_F16) return oracle_round_f16(x);
    if (mode == ROUND_F32) return (double)(float)x; /* IEEE conversion: nearest, ties to even */
    return x;
}

/* Storage rounding of n values, and the largest change of that rounding over
 * an interval: y[i] = round(x[i]); if d != NULL, spread[i] = the largest
 * |round(w) - round(x[i])| over |w - x[i]| <= d[i] (rounding is monotone, so
 * it is reached at an end of the interval; zero when no rounding boundary
 * lies within d[i] of x[i]). */
void oracle_round_n(const double* x, const double* d, double* y, double* spread, int64_t n, int mode)
{
    for (int64_t i = 0; i < n; ++i) {
        const double r = round_store(x[i], mode);
        y[i] = r;
        if (d && spread) {
            const double hi = round_store(x[i] + d[i], mode) - r;
            const double lo = r - round_store(x[i] - d[i], mode);
            spread[i] = hi > lo ? hi : lo;
        }
    }
}

/* rms = sqrt(sum I^2 / N) over every voxel; also returns sum I and the number
 * of non-finite voxels (NaN / Inf are skipped in both sums). */
double oracle_rms(const double* in, int64_t n, double* sum_out, int64_t* nonfinite_out)
{
    double s2 = 0.0, s1 = 0.0;
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        double v = in[i];
        if (!isfinite(v)) { ++bad; continue; }
        s1 += v;
        s2 += v * v;
    }
    if (sum_out) *sum_out = s1;
    if (nonfinite_out) *nonfinite_out = bad;
    return n > 0 ? sqrt(s2 / (double)n) : 0.0;
}

static double edge_weight(int cond, double d, double kr)
{
    double r = d / kr;
    if (cond == COND_PM_EXP) return exp(-r * r);
    if (cond == COND_PM_RATIONAL) return 1.0 / (1.0 + r * r);
    return 1.0;
}

/* One Jacobi step src -> dst. */
static void step(const double* src, double* dst, int64_t nx, int64_t ny, int64_t nz,
                 int cond, double K, double rho, double tau, const double C[3], int round_mode)
{
    const double kr = K * rho;
    const int64_t sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t v = x * sx + y * sy + z * sz;
                const double Iv = src[v];
                const int64_t coord[3] = {x, y, z};
                const int64_t extent[3] = {nx, ny, nz};
                const int64_t stride[3] = {sx, sy, sz};
                double acc = 0.0;
                for (int a = 0; a < 3; ++a) {
                    for (int s = -1; s <= 1; s += 2) {
                        const int64_t c = coord[a] + s;
                        const double Iu = (c < 0 || c >= extent[a]) ? Iv : src[v + s * stride[a]];
                        const double d = Iu - Iv;
                        acc += C[a] * edge_weight(cond, d, kr) * d;
                    }
                }
                double out;
                if (cond == COND_INTENSITY)
                    out = Iv + tau * acc / (1.0 + (Iv * Iv) / (kr * kr));
                else
                    out = Iv + tau * acc;
                dst[v] = round_store(out, round_mode);
            }
        }
    }
}

/* dT/dd of one edge's flux term (its derivative in the difference d). */
static double flux_slope(int cond, double d, double kr, double tau_c)
{
    const double r2 = (d / kr) * (d / kr);
    if (cond == COND_PM_EXP) return tau_c * exp(-r2) * (1.0 - 2.0 * r2);
    if (cond == COND_PM_RATIONAL) return tau_c * (1.0 - r2) / ((1.0 + r2) * (1.0 + r2));
    return tau_c;
}

/* One exact step src -> dst together with the bound bsrc -> bdst. */
static void step_bound(const double* src, double* dst, const double* bsrc, double* bdst, int64_t nx, int64_t ny,
                       int64_t nz, int cond, double K, double rho, double tau, const double C[3])
{
    const double kr = K * rho, u = 0x1p-24;
    const int64_t sx = 1, sy = nx, sz = nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t v = x * sx + y * sy + z * sz;
                const double Iv = src[v];
                const int64_t coord[3] = {x, y, z};
                const int64_t extent[3] = {nx, ny, nz};
                const int64_t stride[3] = {sx, sy, sz};
                const double S = cond == COND_INTENSITY ? 1.0 / (1.0 + (Iv * Iv) / (kr * kr)) : 1.0;
                double acc = 0.0, term_err = 0.0, prop = 0.0, self = 1.0, sumcd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    for (int s = -1; s <= 1; s += 2) {
                        const int64_t c = coord[a] + s;
                        if (c < 0 || c >= extent[a]) continue;   /* no edge through a face */
                        const int64_t w = v + s * stride[a];
                        const double d = src[w] - Iv;
                        const double t = C[a] * edge_weight(cond, d, kr) * d;
                        acc += t;
                        sumcd += C[a] * d;
                        const double r2 = (d / kr) * (d / kr);
                        const double ce = cond == COND_PM_EXP ? 12.0 + 4.0 * r2 : 14.0;
                        term_err += ce * fabs(tau * S * t);
                        /* dependence of I_{i+1}(v) on the neighbour through this edge */
                        const double g = cond == COND_INTENSITY ? tau * S * C[a] : flux_slope(cond, d, kr, tau * C[a]);
                        prop += fabs(g) * bsrc[w];
                        self -= g;
                    }
                }
                if (cond == COND_INTENSITY)   /* S depends on I(v) too: dS/dI = -2 I S^2 / (K rho)^2 */
                    self += tau * sumcd * (-2.0 * Iv * S * S / (kr * kr));
                /* the same expression as step(), so `out` is bitwise oracle_run's result */
                const double out = cond == COND_INTENSITY ? Iv + tau * acc / (1.0 + (Iv * Iv) / (kr * kr))
                                                          : Iv + tau * acc;
                dst[v] = out;
                bdst[v] = fabs(self) * bsrc[v] + prop + u * (fabs(out) + term_err);
            }
        }
    }
}

/*
 * The exact FP64 result of n_iter steps (as oracle_run with round_mode 0) in
 * `out`, and in `bound` the first-order bound described at the top of this
 * file on |result of a binary32 computation - exact result|, per voxel.  rms
 * as for oracle_run.  Returns 0, -1 (invalid arguments), -2 (allocation
 * failure) or -3 (non-finite input).
 */
int oracle_error_bound(const double* in, double* out, double* bound, int64_t nx, int64_t ny, int64_t nz, int cond,
                       double K, double tau, int n_iter, double Cx, double Cy, double Cz, double rms,
                       double* rms_used)
{
    if (nx < 1 || ny < 1 || nz < 1 || n_iter < 0 || !(K > 0.0) || !(tau >= 0.0)) return -1;
    if (cond < 0 || cond > 2) return -1;
    const int64_t n = nx * ny * nz;
    double s1;
    int64_t bad;
    double rho_est = oracle_rms(in, n, &s1, &bad);
    if (bad) return -3;
    const double rho = rms > 0.0 ? rms : rho_est;
    if (rms_used) *rms_used = rho;
    const double C[3] = {Cx, Cy, Cz};
    if (!(rho > 0.0)) {
        memmove(out, in, (size_t)n * sizeof(double));
        memset(bound, 0, (size_t)n * sizeof(double));
        return 0;
    }
    double* a = (double*)malloc((size_t)n * sizeof(double));
    double* b = (double*)malloc((size_t)n * sizeof(double));
    double* ba = (double*)calloc((size_t)n, sizeof(double));
    double* bb = (double*)malloc((size_t)n * sizeof(double));
    if (!a || !b || !ba || !bb) { free(a); free(b); free(ba); free(bb); return -2; }
    memcpy(a, in, (size_t)n * sizeof(double));
    for (int i = 0; i < n_iter; ++i) {
        step_bound(a, b, ba, bb, nx, ny, nz, cond, K, rho, tau, C);
        double* t = a; a = b; b = t;
        t = ba; ba = bb; bb = t;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    memcpy(bound, ba, (size_t)n * sizeof(double));
    free(a); free(b); free(ba); free(bb);
    return 0;
}

/*
 * Run n_iter steps on a cube of nx*ny*nz doubles (x fastest).  `in` is not
 * modified; the result goes to `out` (may equal `in`).  rms > 0 is used as
 * the noise level; otherwise it is estimated from `in`.  Returns 0 on
 * success, -1 on invalid arguments, -2 on allocation failure, -3 when the
 * input holds NaN or Inf.
 */
int oracle_run(const double* in, double* out, int64_t nx, int64_t ny, int64_t nz,
               int cond, double K, double tau, int n_iter, double Cx, double Cy, double Cz,
               double rms, int round_mode, double* rms_used)
{
    if (nx < 1 || ny < 1 || nz < 1 || n_iter < 0 || !(K > 0.0) || !(tau >= 0.0)) return -1;
    if (cond < 0 || cond > 2 || round_mode < 0 || round_mode > 3) return -1;
    const int64_t n = nx * ny * nz;
    double s1;
    int64_t bad;
    double rho_est = oracle_rms(in, n, &s1, &bad);
    if (bad) return -3;
    const double rho = rms > 0.0 ? rms : rho_est;
    if (rms_used) *rms_used = rho;
    const double C[3] = {Cx, Cy, Cz};
    if (!(rho > 0.0)) {
        /* An estimated rms of 0 means every voxel is 0: all differences vanish
         * and the cube is a fixed point of the step. */
        memmove(out, in, (size_t)n * sizeof(double));
        return 0;
    }

    double* a = (double*)malloc((size_t)n * sizeof(double));
    double* b = (double*)malloc((size_t)n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, in, (size_t)n * sizeof(double));
    for (int i = 0; i < n_iter; ++i) {
        step(a, b, nx, ny, nz, cond, K, rho, tau, C, round_mode);
        double* t = a; a = b; b = t;
    }
    memcpy(out, a, (size_t)n * sizeof(double));
    free(a);
    free(b);
    return 0;
}
