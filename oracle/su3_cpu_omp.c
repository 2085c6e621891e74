/*
 * su3_cpu_omp.c -- multi-core CPU baseline of the SU(3) link multiply.
 *
 * MEASUREMENT INFRASTRUCTURE, not the oracle and not part of the GPU library:
 * only the benchmark's CPU-baseline leg and the tests run it, and it shares
 * no code with either. It times the product
 *
 *     c[s].link[j] = a[s].link[j] * b[j]      (j = 0..3, 3x3 complex, FP64)
 *
 * on every host core, set up the way the paper's best Xeon runs were
 * (arXiv 2103.00571, section Performance on Xeon):
 *
 *  - one OpenMP parallel-for over the sites, with the plain loop nest of
 *    section Background (links j, output entries k and l, dot product over m)
 *    inside it, as in the paper's OpenMP "parallel for" version;
 *  - the arrays are allocated without being touched and then initialised by
 *    a parallel loop with the same static schedule, so every page is first
 *    touched by the thread that later streams it (the paper's fix of empty
 *    constructors plus parallel initialisation);
 *  - the caller binds threads with OMP_PROC_BIND=close and OMP_PLACES=cores.
 *
 * The values are the paper's initialisation (every entry of a is 1+0i, every
 * entry of b is 1/3+0i), so every entry of c is exactly 3 * (1/3) summed in
 * any order = 1+0i in FP64; the program checks that after the timed passes.
 * Arrays are dense, 576 B per site and array (no padded Site struct).
 *
 * usage: su3_cpu_omp SITES WARMUP MIN_PASSES MIN_SECONDS
 * Runs WARMUP untimed passes, then timed passes until at least MIN_PASSES
 * have run and MIN_SECONDS have passed, and prints one JSON line. Exit
 * status 0 on success, 1 on bad arguments or allocation failure, 2 if the
 * result check fails.
 */
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define SITE_DOUBLES 72 /* 4 links x 9 complex x (re, im) */

/* element (k, l) of link j of site s, as a double index (re; im is +1) */
static inline int64_t ix(int64_t s, int j, int k, int l) { return 2 * (((s * 4 + j) * 3 + k) * 3 + l); }

static void product(const double *restrict a, const double *restrict b, double *restrict c, int64_t sites)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < sites; ++s)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double re = 0.0, im = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        const double ar = a[ix(s, j, k, m)], ai = a[ix(s, j, k, m) + 1];
                        const double br = b[2 * ((j * 3 + m) * 3 + l)], bi = b[2 * ((j * 3 + m) * 3 + l) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    c[ix(s, j, k, l)] = re;
                    c[ix(s, j, k, l) + 1] = im;
                }
}

static const char *env_or(const char *name, const char *fallback)
{
    const char *v = getenv(name);
    return v ? v : fallback;
}

int main(int argc, char **argv)
{
    if (argc != 5) {
        fprintf(stderr, "usage: %s SITES WARMUP MIN_PASSES MIN_SECONDS\n", argv[0]);
        return 1;
    }
    const int64_t sites = atoll(argv[1]);
    const int warmup = atoi(argv[2]), min_passes = atoi(argv[3]);
    const double min_seconds = atof(argv[4]);
    if (sites <= 0 || warmup < 0 || min_passes < 1 || min_seconds < 0.0 ||
        sites > INT64_MAX / (SITE_DOUBLES * (int64_t)sizeof(double))) {
        fprintf(stderr, "bad arguments\n");
        return 1;
    }
    const size_t bytes = (size_t)sites * SITE_DOUBLES * sizeof(double);
    /* malloc touches no page of a large block: first touch happens below */
    double *a = malloc(bytes), *c = malloc(bytes);
    double b[SITE_DOUBLES];
    if (!a || !c) {
        fprintf(stderr, "allocation of 2 x %zu bytes failed\n", bytes);
        return 1;
    }
    for (int q = 0; q < SITE_DOUBLES; ++q)
        b[q] = (q % 2 == 0) ? 1.0 / 3.0 : 0.0;

    const double t_init = omp_get_wtime();
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < sites; ++s)
        for (int q = 0; q < SITE_DOUBLES; ++q) {
            a[s * SITE_DOUBLES + q] = (q % 2 == 0) ? 1.0 : 0.0;
            c[s * SITE_DOUBLES + q] = 0.0;
        }
    const double init_seconds = omp_get_wtime() - t_init;

    for (int w = 0; w < warmup; ++w)
        product(a, b, c, sites);
    int passes = 0;
    const double t0 = omp_get_wtime();
    double el = 0.0;
    do {
        product(a, b, c, sites);
        ++passes;
        el = omp_get_wtime() - t0;
    } while (passes < min_passes || el < min_seconds);

    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t s = 0; s < sites; ++s)
        for (int q = 0; q < SITE_DOUBLES; ++q)
            bad += c[s * SITE_DOUBLES + q] != ((q % 2 == 0) ? 1.0 : 0.0);

    const double per_pass = el / passes;
    printf("{\"sites\": %lld, \"threads\": %d, \"passes\": %d, \"seconds\": %.6f, \"seconds_per_pass\": %.9f, "
           "\"sites_per_s\": %.6e, \"gb_s\": %.6e, \"init_seconds\": %.4f, \"omp_proc_bind\": \"%s\", "
           "\"omp_places\": \"%s\", \"check\": \"every c entry == 1+0i\", \"check_ok\": %s}\n",
           (long long)sites, omp_get_max_threads(), passes, el, per_pass, sites / per_pass,
           2.0 * bytes / per_pass / 1e9, init_seconds, env_or("OMP_PROC_BIND", "unset"),
           env_or("OMP_PLACES", "unset"), bad == 0 ? "true" : "false");
    free(a);
    free(c);
    return bad == 0 ? 0 : 2;
}
