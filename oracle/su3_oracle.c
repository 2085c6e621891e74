/*
 * su3_oracle.c -- plain, slow, single-threaded CPU reference for the SU(3)
 * link multiply of SU3_Bench (Tithi, Checconi, Petrini, Doerfler,
 * "Performance Optimization of SU3_Bench on Xeon and Programmable Integrated
 * Unified Memory Architecture", arXiv 2103.00571).
 *
 * TEST INFRASTRUCTURE. This is the oracle the GPU library is checked against.
 * Only the test-suite, the package smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no code, header, helper or constant with the GPU
 * library, and the GPU library never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, no
 * fast-math), so every sum below is evaluated exactly in the order written.
 *
 * Storage conventions (paper, Background / SU3_Bench: an su3_matrix is a 3x3
 * complex matrix; a site holds four links; B is four constant matrices):
 *   - complex numbers are interleaved (re, im);
 *   - a link is row-major 3x3: element (k, l) at complex offset 3k + l;
 *   - a lattice array is site-major: link j of site s at complex offset
 *     (s*4 + j)*9, i.e. shape (sites, 4, 3, 3);
 *   - b is (4, 3, 3): b[j] multiplies link j of every site.
 *
 * Beyond the paper's product the oracle also defines the two other products
 * of the MILC family the benchmark is drawn from (a b^H and a^H b, the
 * adjoint's contractions), the reconstruct-12 product in FP64, and the SU(3)
 * matrix times colour-vector product the paper names as the other building
 * block (section Introduction).
 *
 * Parity status: every function here is pinned by a CPU test against facts
 * fixed by the paper or by the mathematics (identity and signed-permutation
 * products, the paper's constant initialisation, exact rational arithmetic,
 * SU(3) closure, a library matmul, automatic differentiation and central
 * finite differences, bit-level rounding facts). No function is parity
 * unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define LINK_C 9          /* complex entries per link               */
#define SITE_C 36         /* complex entries per site (4 links)     */

/* real-array index of complex element (k, l) of link j of site s */
static inline int64_t ix(int64_t s, int j, int k, int l)
{
    return 2 * ((s * 4 + j) * LINK_C + k * 3 + l);
}

/* real-array index of complex element (m, l) of b[j] */
static inline int bx(int j, int m, int l)
{
    return 2 * (j * LINK_C + m * 3 + l);
}

/* ------------------------------------------------------------------ O1 --
 * Forward product (paper, Background / SU3_Bench, the core kernel): for every
 * site i and link j, C[i].link[j] = A[i].link[j] * B[j], each of the nine
 * outputs the dot product of row k of A[i].link[j] with column l of B[j]
 * (loops i, j, k, l, with the inner m loop the dot product). C is overwritten.
 */
void su3o_mult_nn(const double *a, const double *b, double *c, int64_t sites)
{
    for (int64_t i = 0; i < sites; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double re = 0.0, im = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        const double ar = a[ix(i, j, k, m)];
                        const double ai = a[ix(i, j, k, m) + 1];
                        const double br = b[bx(j, m, l)];
                        const double bi = b[bx(j, m, l) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    c[ix(i, j, k, l)] = re;
                    c[ix(i, j, k, l) + 1] = im;
                }
}

/* Neumaier's improvement of Kahan summation: add x to (sum, comp). */
static inline void neumaier_add(double *sum, double *comp, double x)
{
    const double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/* ------------------------------------------------------------------ O2 --
 * Adjoint of O1 for the real loss Lss = Re sum conj(dC) . C, in the usual
 * complex-gradient convention (dL/dRe z + i dL/dIm z):
 *   dA[s][j](k, m) = sum_l dC[s][j](k, l) * conj(b[j](m, l))      (dC b^H)
 *   dB[j](m, l)    = sum_s sum_k conj(a[s][j](k, m)) * dC[s][j](k, l)
 * The paper has no adjoint; this is the derivative of its product. dB is
 * summed in site order with Neumaier compensation so that it is, in effect,
 * the correctly rounded sum of the rounded terms. db holds 4*9 complex values.
 */
void su3o_mult_nn_bwd(const double *a, const double *b, const double *dc,
                      double *da, double *db, int64_t sites)
{
    double sum[72], comp[72];
    for (int q = 0; q < 72; ++q) { sum[q] = 0.0; comp[q] = 0.0; }

    for (int64_t s = 0; s < sites; ++s)
        for (int j = 0; j < 4; ++j) {
            for (int k = 0; k < 3; ++k)
                for (int m = 0; m < 3; ++m) {
                    double re = 0.0, im = 0.0;
                    for (int l = 0; l < 3; ++l) {
                        const double gr = dc[ix(s, j, k, l)];
                        const double gi = dc[ix(s, j, k, l) + 1];
                        const double br = b[bx(j, m, l)];
                        const double bi = -b[bx(j, m, l) + 1];   /* conj */
                        re += gr * br - gi * bi;
                        im += gr * bi + gi * br;
                    }
                    da[ix(s, j, k, m)] = re;
                    da[ix(s, j, k, m) + 1] = im;
                }
            for (int m = 0; m < 3; ++m)
                for (int l = 0; l < 3; ++l)
                    for (int k = 0; k < 3; ++k) {
                        const double ar = a[ix(s, j, k, m)];
                        const double ai = -a[ix(s, j, k, m) + 1]; /* conj */
                        const double gr = dc[ix(s, j, k, l)];
                        const double gi = dc[ix(s, j, k, l) + 1];
                        const int q = bx(j, m, l);
                        neumaier_add(&sum[q], &comp[q], ar * gr - ai * gi);
                        neumaier_add(&sum[q + 1], &comp[q + 1], ar * gi + ai * gr);
                    }
        }
    for (int q = 0; q < 72; ++q)
        db[q] = sum[q] + comp[q];
}

/* ------------------------------------------------------------------ O3 --
 * Third row of a special unitary 3x3 matrix from its first two rows:
 * r2 = conj(r0 x r1). For U in SU(3), U^-1 = U^H = adj(U), so conj(U(2, l))
 * is the cofactor of element (2, l), which is component l of r0 x r1.
 * r0, r1, r2 each hold three interleaved complex values.
 */
void su3o_recon_row2(const double *r0, const double *r1, double *r2)
{
    for (int l = 0; l < 3; ++l) {
        const int p = (l + 1) % 3, q = (l + 2) % 3;
        /* (r0 x r1)_l = r0_p r1_q - r0_q r1_p */
        const double xr = (r0[2*p] * r1[2*q] - r0[2*p+1] * r1[2*q+1])
                        - (r0[2*q] * r1[2*p] - r0[2*q+1] * r1[2*p+1]);
        const double xi = (r0[2*p] * r1[2*q+1] + r0[2*p+1] * r1[2*q])
                        - (r0[2*q] * r1[2*p+1] + r0[2*q+1] * r1[2*p]);
        r2[2*l] = xr;
        r2[2*l+1] = -xi;
    }
}

/* The same rebuild carried out in single precision (the reconstruct-12
 * form computes in FP32). */
static void recon_row2_f32(const float *r0, const float *r1, float *r2)
{
    for (int l = 0; l < 3; ++l) {
        const int p = (l + 1) % 3, q = (l + 2) % 3;
        const float xr = (r0[2*p] * r1[2*q] - r0[2*p+1] * r1[2*q+1])
                       - (r0[2*q] * r1[2*p] - r0[2*q+1] * r1[2*p+1]);
        const float xi = (r0[2*p] * r1[2*q+1] + r0[2*p+1] * r1[2*q])
                       - (r0[2*q] * r1[2*p+1] + r0[2*q+1] * r1[2*p]);
        r2[2*l] = xr;
        r2[2*l+1] = -xi;
    }
}

/* ------------------------------------------------------------------ O4 --
 * Metrics. Max absolute component error over n reals.
 */
double su3o_max_abs_diff(const double *x, const double *y, int64_t n)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double d = fabs(x[i] - y[i]);
        if (d > m || d != d)
            m = (d != d) ? INFINITY : d;
    }
    return m;
}

/* max over matrices of || M^H M - I ||_F, over `mats` 3x3 complex matrices */
double su3o_unitarity_dev(const double *u, int64_t mats)
{
    double worst = 0.0;
    for (int64_t t = 0; t < mats; ++t) {
        const double *M = u + 18 * t;
        double f = 0.0;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                double re = 0.0, im = 0.0;
                for (int r = 0; r < 3; ++r) {
                    const double xr = M[2*(3*r+p)], xi = -M[2*(3*r+p)+1];
                    const double yr = M[2*(3*r+q)], yi = M[2*(3*r+q)+1];
                    re += xr * yr - xi * yi;
                    im += xr * yi + xi * yr;
                }
                if (p == q) re -= 1.0;
                f += re * re + im * im;
            }
        f = sqrt(f);
        if (f > worst || f != f)
            worst = (f != f) ? INFINITY : f;
    }
    return worst;
}

static void cmul(double ar, double ai, double br, double bi, double *r, double *i)
{
    *r = ar * br - ai * bi;
    *i = ar * bi + ai * br;
}

/* determinant of one 3x3 complex matrix, cofactor expansion along row 0 */
void su3o_det(const double *M, double *re, double *im)
{
    double t1r, t1i, t2r, t2i, mr, mi, sr = 0.0, si = 0.0;
    for (int l = 0; l < 3; ++l) {
        const int p = (l + 1) % 3, q = (l + 2) % 3;
        cmul(M[2*(3+p)], M[2*(3+p)+1], M[2*(6+q)], M[2*(6+q)+1], &t1r, &t1i);
        cmul(M[2*(3+q)], M[2*(3+q)+1], M[2*(6+p)], M[2*(6+p)+1], &t2r, &t2i);
        cmul(M[2*l], M[2*l+1], t1r - t2r, t1i - t2i, &mr, &mi);
        sr += mr;
        si += mi;
    }
    *re = sr;
    *im = si;
}

/* max over matrices of |det M - 1| */
double su3o_det_dev(const double *u, int64_t mats)
{
    double worst = 0.0;
    for (int64_t t = 0; t < mats; ++t) {
        double re, im;
        su3o_det(u + 18 * t, &re, &im);
        const double d = hypot(re - 1.0, im);
        if (d > worst || d != d)
            worst = (d != d) ? INFINITY : d;
    }
    return worst;
}

/* ------------------------------------------------------------------ O5 --
 * Storage forms. Rounding from FP64 is round-to-nearest-even: FP64 -> FP32 by
 * the C conversion (which rounds to nearest even in the default mode); FP32 ->
 * BF16 keeps the upper 16 bits after adding half an ulp with ties to even.
 * BF16 from FP64 goes through FP32.
 */
static uint16_t f32_to_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0)
        return (uint16_t)((u >> 16) | 0x0040u);           /* quiet NaN */
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static float bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
}

void su3o_round_f32(const double *src, float *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = (float)src[i];
}

void su3o_round_bf16(const double *src, uint16_t *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = f32_to_bf16((float)src[i]);
}

void su3o_f32_to_bf16(const float *src, uint16_t *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = f32_to_bf16(src[i]);
}

void su3o_widen_bf16(const uint16_t *src, double *dst, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = (double)bf16_to_f32(src[i]);
}

/* reconstruct-12 storage: rows 0 and 1 of every link, FP32, shape
 * (sites, 4, 2, 3) complex */
void su3o_pack_r12(const double *src, float *dst, int64_t sites)
{
    for (int64_t s = 0; s < sites; ++s)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 3; ++l) {
                    const int64_t o = 2 * (((s * 4 + j) * 2 + k) * 3 + l);
                    dst[o] = (float)src[ix(s, j, k, l)];
                    dst[o + 1] = (float)src[ix(s, j, k, l) + 1];
                }
}

/* widen reconstruct-12 storage to full FP64 links, row 2 rebuilt by O3 in
 * FP64 from the widened rows */
void su3o_unpack_r12(const float *src, double *dst, int64_t sites)
{
    for (int64_t s = 0; s < sites; ++s)
        for (int j = 0; j < 4; ++j) {
            double *L = dst + ix(s, j, 0, 0);
            const float *R = src + 12 * (s * 4 + j);
            for (int q = 0; q < 12; ++q)
                L[q] = (double)R[q];
            su3o_recon_row2(L, L + 6, L + 12);
        }
}

/* Forward product in single precision (the FP32 storage form): the O1 loop
 * with float operands and float accumulators. */
void su3o_mult_nn_f32(const float *a, const float *b, float *c, int64_t sites)
{
    for (int64_t i = 0; i < sites; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    float re = 0.0f, im = 0.0f;
                    for (int m = 0; m < 3; ++m) {
                        const float ar = a[ix(i, j, k, m)];
                        const float ai = a[ix(i, j, k, m) + 1];
                        const float br = b[bx(j, m, l)];
                        const float bi = b[bx(j, m, l) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    c[ix(i, j, k, l)] = re;
                    c[ix(i, j, k, l) + 1] = im;
                }
}

/* BF16 storage form: a and c are BF16, b is FP32, arithmetic is FP32, c is
 * rounded to BF16 with ties to even. Processes one site at a time. */
void su3o_mult_nn_bf16(const uint16_t *a, const float *b, uint16_t *c, int64_t sites)
{
    float aw[72], cw[72];
    for (int64_t s = 0; s < sites; ++s) {
        for (int q = 0; q < 72; ++q)
            aw[q] = bf16_to_f32(a[72 * s + q]);
        su3o_mult_nn_f32(aw, b, cw, 1);
        for (int q = 0; q < 72; ++q)
            c[72 * s + q] = f32_to_bf16(cw[q]);
    }
}

/* Reconstruct-12 form: a holds rows 0-1 in FP32, row 2 is rebuilt in FP32,
 * then the FP32 product; c is full FP32 (sites, 4, 3, 3). */
void su3o_mult_nn_r12(const float *a12, const float *b, float *c, int64_t sites)
{
    float aw[72];
    for (int64_t s = 0; s < sites; ++s) {
        for (int j = 0; j < 4; ++j) {
            const float *R = a12 + 12 * (s * 4 + j);
            float *L = aw + 18 * j;
            for (int q = 0; q < 12; ++q)
                L[q] = R[q];
            recon_row2_f32(L, L + 6, L + 12);
        }
        su3o_mult_nn_f32(aw, b, c + 72 * s, 1);
    }
}

/* ------------------------------------------------------------------ O6 --
 * Structure-of-arrays layout: complex element p = (j*3 + k)*3 + l of site s
 * moves to position p*sites + s (36 planes of `sites` elements). elem_bytes
 * is the size of one complex element (16 for FP64, 8 for FP32).
 */
void su3o_aos_to_soa(const void *src, void *dst, int64_t sites, int elem_bytes)
{
    const char *S = (const char *)src;
    char *D = (char *)dst;
    for (int64_t s = 0; s < sites; ++s)
        for (int p = 0; p < SITE_C; ++p)
            memcpy(D + ((int64_t)p * sites + s) * elem_bytes,
                   S + (s * SITE_C + p) * elem_bytes, (size_t)elem_bytes);
}

void su3o_soa_to_aos(const void *src, void *dst, int64_t sites, int elem_bytes)
{
    const char *S = (const char *)src;
    char *D = (char *)dst;
    for (int64_t s = 0; s < sites; ++s)
        for (int p = 0; p < SITE_C; ++p)
            memcpy(D + (s * SITE_C + p) * elem_bytes,
                   S + ((int64_t)p * sites + s) * elem_bytes, (size_t)elem_bytes);
}

/* ------------------------------------------------------------------ O7 --
 * The other two link products. na: c[s][j] = a[s][j] * b[j]^H, i.e.
 * c(k, l) = sum_m a(k, m) conj(b(l, m)). an: c[s][j] = a[s][j]^H * b[j], i.e.
 * c(k, l) = sum_m conj(a(m, k)) b(m, l). Same loop order as O1.
 */
void su3o_mult_na(const double *a, const double *b, double *c, int64_t sites)
{
    for (int64_t i = 0; i < sites; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double re = 0.0, im = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        const double ar = a[ix(i, j, k, m)];
                        const double ai = a[ix(i, j, k, m) + 1];
                        const double br = b[bx(j, l, m)];
                        const double bi = -b[bx(j, l, m) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    c[ix(i, j, k, l)] = re;
                    c[ix(i, j, k, l) + 1] = im;
                }
}

void su3o_mult_an(const double *a, const double *b, double *c, int64_t sites)
{
    for (int64_t i = 0; i < sites; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double re = 0.0, im = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        const double ar = a[ix(i, j, m, k)];
                        const double ai = -a[ix(i, j, m, k) + 1];
                        const double br = b[bx(j, m, l)];
                        const double bi = b[bx(j, m, l) + 1];
                        re += ar * br - ai * bi;
                        im += ar * bi + ai * br;
                    }
                    c[ix(i, j, k, l)] = re;
                    c[ix(i, j, k, l) + 1] = im;
                }
}

/* ------------------------------------------------------------------ O8 --
 * Reconstruct-12 in FP64: a holds rows 0-1 of every link in FP64, shape
 * (sites, 4, 2, 3) complex; row 2 is rebuilt by O3, then the O1 product.
 */
void su3o_mult_nn_r12_f64(const double *a12, const double *b, double *c, int64_t sites)
{
    double aw[72];
    for (int64_t s = 0; s < sites; ++s) {
        for (int j = 0; j < 4; ++j) {
            const double *R = a12 + 12 * (s * 4 + j);   /* rows 0-1: 6 complex */
            double *L = aw + 18 * j;                     /* full link: 9 complex */
            for (int q = 0; q < 12; ++q)
                L[q] = R[q];
            su3o_recon_row2(L, L + 6, L + 12);
        }
        su3o_mult_nn(aw, b, c + 72 * s, 1);
    }
}

/* ------------------------------------------------------------------ O9 --
 * SU(3) matrix times colour vector over the lattice (the matrix-vector
 * building block; section Introduction): every link of a site applied to the
 * site's own colour vector, w[s][j](k) = sum_m a[s][j](k, m) v[s](m).
 * v is (sites, 3) complex, w is (sites, 4, 3) complex.
 */
void su3o_mat_vec(const double *a, const double *v, double *w, int64_t sites)
{
    for (int64_t i = 0; i < sites; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k) {
                double re = 0.0, im = 0.0;
                for (int m = 0; m < 3; ++m) {
                    const double ar = a[ix(i, j, k, m)];
                    const double ai = a[ix(i, j, k, m) + 1];
                    const double vr = v[2 * (3 * i + m)];
                    const double vi = v[2 * (3 * i + m) + 1];
                    re += ar * vr - ai * vi;
                    im += ar * vi + ai * vr;
                }
                w[2 * ((i * 4 + j) * 3 + k)] = re;
                w[2 * ((i * 4 + j) * 3 + k) + 1] = im;
            }
}
