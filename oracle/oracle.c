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
