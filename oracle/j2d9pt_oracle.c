/*
 * j2d9pt_oracle.c -- plain CPU oracle for the j2d9pt (3 x 3 box) iterative
 * stencil.
 *
 * TEST INFRASTRUCTURE ONLY, like j2d5pt_oracle.c: the slow, obviously correct
 * reference the GPU library is checked against; it shares nothing with the
 * HIP library, and only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.
 *
 * What it computes.  The paper presents its method on j2d5pt (Listing 1) as a
 * case study of deep temporal blocking for iterative stencils in general
 * (Title, Section 1); j2d9pt is the next shape in the same framework: every
 * output cell is the weighted sum of the 3 x 3 block of input cells centred on
 * it, read from one buffer and written to another (Jacobi), repeated T times
 * (Section 3.1, Figure 1).  The paper prints no j2d9pt listing; this file
 * fixes the reading used throughout:
 *
 *   coeffs[] holds nine weights in row-major order of the block, rows i-1,
 *   i, i+1 (south to north, the same orientation as j2d5pt: S = row i-1,
 *   N = row i+1), each west to east:
 *     (sw, s, se, w, c, e, nw, n, ne)
 *   and the products are rounded one by one and summed left to right in that
 *   same order.  No multiply-add is fused (-ffp-contract=off).
 *
 *   The one-cell halo ring, corners included (the box reads them), is a fixed
 *   Dirichlet boundary: read, never written.  Storage as for j2d5pt: (rows+2)
 *   lines of `pitch` elements, interior rows 1..rows, columns 1..cols.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE9_OK 0
#define ORACLE9_EINVAL -1
#define ORACLE9_ENOMEM -4

static int threads_or_default(int nthreads)
{
    if (nthreads > 0) return nthreads;
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Advance u by T steps in double precision, in place (see above). */
int oracle_j2d9pt_f64(double* u, int64_t rows, int64_t cols, int64_t pitch,
                      const double* coeffs, int64_t T, int nthreads)
{
    if (!u || !coeffs || rows < 1 || cols < 1 || pitch < cols + 2 || T < 0) return ORACLE9_EINVAL;
    if (T == 0) return ORACLE9_OK;
    double k[9];
    for (int q = 0; q < 9; ++q) k[q] = coeffs[q];
    const size_t n_elem = (size_t)(rows + 2) * (size_t)pitch;
    double* v = (double*)malloc(n_elem * sizeof(double));
    if (!v) return ORACLE9_ENOMEM;
    memcpy(v, u, n_elem * sizeof(double)); /* the second buffer's halo matches */
    double* in = u;
    double* out = v;
    nthreads = threads_or_default(nthreads);
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t i = 1; i <= rows; ++i) {
            const double* s = in + (i - 1) * pitch; /* row i-1 */
            const double* m = in + i * pitch;       /* row i   */
            const double* n = in + (i + 1) * pitch; /* row i+1 */
            double* o = out + i * pitch;
            for (int64_t j = 1; j <= cols; ++j) {
                double acc = k[0] * s[j - 1];
                acc = acc + k[1] * s[j];
                acc = acc + k[2] * s[j + 1];
                acc = acc + k[3] * m[j - 1];
                acc = acc + k[4] * m[j];
                acc = acc + k[5] * m[j + 1];
                acc = acc + k[6] * n[j - 1];
                acc = acc + k[7] * n[j];
                acc = acc + k[8] * n[j + 1];
                o[j] = acc;
            }
        }
        double* tmp = in;
        in = out;
        out = tmp;
    }
    if (in != u) {
        for (int64_t i = 1; i <= rows; ++i)
            memcpy(u + i * pitch + 1, in + i * pitch + 1, (size_t)cols * sizeof(double));
    }
    free(v);
    return ORACLE9_OK;
}

/* The same in single precision: weights rounded to float once, every operation in float, same order. */
int oracle_j2d9pt_f32(float* u, int64_t rows, int64_t cols, int64_t pitch,
                      const double* coeffs, int64_t T, int nthreads)
{
    if (!u || !coeffs || rows < 1 || cols < 1 || pitch < cols + 2 || T < 0) return ORACLE9_EINVAL;
    if (T == 0) return ORACLE9_OK;
    float k[9];
    for (int q = 0; q < 9; ++q) k[q] = (float)coeffs[q];
    const size_t n_elem = (size_t)(rows + 2) * (size_t)pitch;
    float* v = (float*)malloc(n_elem * sizeof(float));
    if (!v) return ORACLE9_ENOMEM;
    memcpy(v, u, n_elem * sizeof(float));
    float* in = u;
    float* out = v;
    nthreads = threads_or_default(nthreads);
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t i = 1; i <= rows; ++i) {
            const float* s = in + (i - 1) * pitch;
            const float* m = in + i * pitch;
            const float* n = in + (i + 1) * pitch;
            float* o = out + i * pitch;
            for (int64_t j = 1; j <= cols; ++j) {
                float acc = k[0] * s[j - 1];
                acc = acc + k[1] * s[j];
                acc = acc + k[2] * s[j + 1];
                acc = acc + k[3] * m[j - 1];
                acc = acc + k[4] * m[j];
                acc = acc + k[5] * m[j + 1];
                acc = acc + k[6] * n[j - 1];
                acc = acc + k[7] * n[j];
                acc = acc + k[8] * n[j + 1];
                o[j] = acc;
            }
        }
        float* tmp = in;
        in = out;
        out = tmp;
    }
    if (in != u) {
        for (int64_t i = 1; i <= rows; ++i)
            memcpy(u + i * pitch + 1, in + i * pitch + 1, (size_t)cols * sizeof(float));
    }
    free(v);
    return ORACLE9_OK;
}
