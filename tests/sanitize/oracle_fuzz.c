/* Randomised exercise of the FP64 oracle (oracle/oracle.c) on small cubes of
 * every shape class, built with AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_sanitize_cpu.py.  Besides running clean under the sanitizers:
 * results are finite, the per-edge forms conserve the sum, a constant cube is a
 * fixed point, and the error bound's exact part is the plain run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_run(const double* in, double* out, int64_t nx, int64_t ny, int64_t nz, int cond, double K, double tau,
               int n_iter, double Cx, double Cy, double Cz, double rms, int round_mode, double* rms_used);
int oracle_error_bound(const double* in, double* out, double* bound, int64_t nx, int64_t ny, int64_t nz, int cond,
                       double K, double tau, int n_iter, double Cx, double Cy, double Cz, double rms,
                       double* rms_used);
double oracle_rms(const double* in, int64_t n, double* sum_out, int64_t* nonfinite_out);
double oracle_round_bf16(double x);
double oracle_round_f16(double x);

static uint64_t state = 1;
static uint64_t next(void) { /* splitmix64 */
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static double unif(void) { return (double)(next() >> 11) * 0x1p-53; }

int main(int argc, char** argv) {
    state = argc > 1 ? strtoull(argv[1], NULL, 10) : 1;
    const int iters = argc > 2 ? atoi(argv[2]) : 300;
    int failures = 0;
    for (int it = 0; it < iters; ++it) {
        const int64_t nx = 1 + next() % 9, ny = 1 + next() % 9, nz = 1 + next() % 7;
        const int64_t n = nx * ny * nz;
        const int cond = (int)(next() % 3), round_mode = (int)(next() % 4), steps = (int)(next() % 6);
        const double K = 0.5 + 3.0 * unif(), tau = 0.1 * unif();
        const double C[3] = {2.0 * unif(), 2.0 * unif(), 2.0 * unif()};
        double* in = malloc((size_t)n * sizeof(double));
        double* out = malloc((size_t)n * sizeof(double));
        double* ref = malloc((size_t)n * sizeof(double));
        double* bnd = malloc((size_t)n * sizeof(double));
        const int constant = next() % 8 == 0;
        for (int64_t i = 0; i < n; ++i) in[i] = constant ? 1.75 : 4.0 * (unif() - 0.5);
        double used = 0.0, s_in = 0.0;
        int64_t bad = 0;
        oracle_rms(in, n, &s_in, &bad);
        int rc = oracle_run(in, out, nx, ny, nz, cond, K, tau, steps, C[0], C[1], C[2], 0.0, round_mode, &used);
        if (rc != 0) { fprintf(stderr, "run failed %d\n", rc); ++failures; }
        double s_out = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!isfinite(out[i])) { fprintf(stderr, "non-finite output\n"); ++failures; break; }
            s_out += out[i];
            if (constant && out[i] != 1.75) { fprintf(stderr, "constant cube moved\n"); ++failures; break; }
        }
        if (cond != 0 && round_mode == 0 && fabs(s_out - s_in) > 1e-12 * (1.0 + fabs(s_in) + n)) {
            fprintf(stderr, "sum drift %g\n", s_out - s_in);
            ++failures;
        }
        rc = oracle_error_bound(in, ref, bnd, nx, ny, nz, cond, K, tau, steps, C[0], C[1], C[2], 0.0, &used);
        if (rc != 0) { fprintf(stderr, "bound failed %d\n", rc); ++failures; }
        double* plain = malloc((size_t)n * sizeof(double));
        oracle_run(in, plain, nx, ny, nz, cond, K, tau, steps, C[0], C[1], C[2], 0.0, 0, &used);
        if (memcmp(plain, ref, (size_t)n * sizeof(double)) != 0) { fprintf(stderr, "bound's exact part differs\n"); ++failures; }
        for (int64_t i = 0; i < n; ++i)
            if (!(bnd[i] >= 0.0) || !isfinite(bnd[i])) { fprintf(stderr, "bad bound\n"); ++failures; break; }
        /* invalid arguments are refused */
        if (oracle_run(in, out, 0, ny, nz, cond, K, tau, steps, 1, 1, 1, 0.0, 0, &used) != -1) ++failures;
        if (oracle_run(in, out, nx, ny, nz, 7, K, tau, steps, 1, 1, 1, 0.0, 0, &used) != -1) ++failures;
        in[0] = NAN;
        if (oracle_run(in, out, nx, ny, nz, cond, K, tau, steps, 1, 1, 1, 0.0, 0, &used) != -3) ++failures;
        const double x = 1e6 * (unif() - 0.5);
        if (!isfinite(oracle_round_bf16(x)) || !isfinite(oracle_round_f16(x * 1e-3))) ++failures;
        free(in); free(out); free(ref); free(bnd); free(plain);
    }
    printf("oracle_fuzz: %d iterations, %d failures\n", iters, failures);
    return failures ? 1 : 0;
}
