/*
 * j3d7pt_oracle.c -- plain CPU oracle for the j3d7pt (3-D seven-point)
 * iterative stencil.
 *
 * TEST INFRASTRUCTURE ONLY, like j2d5pt_oracle.c: the slow, obviously correct
 * reference the GPU library is checked against; it shares nothing with the
 * HIP library, and only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.
 *
 * What it computes.  The paper presents its method on j2d5pt (Listing 1) as a
 * case study of deep temporal blocking for iterative stencils in general
 * (Title, Section 1) and names 2.5D/3.5D tiling of 3-D stencils among the
 * related designs (Section 2).  j3d7pt is the 3-D form of Listing 1's update:
 * every interior cell becomes the weighted sum of itself and its six face
 * neighbours, read from one buffer and written to another (Jacobi), repeated T
 * times (Section 3.1, Figure 1).  The paper prints no 3-D listing; this file
 * fixes the reading used throughout:
 *
 *   coeffs[] holds seven weights (c, n, s, e, w, t, b): the five of j2d5pt in
 *   their order, then t for plane z+1 and b for plane z-1.  Orientation as
 *   j2d5pt within a plane (W = column j-1, E = j+1, S = row i-1, N = row
 *   i+1).  The products are rounded one by one and summed left to right in
 *   the order W, E, S, C, N (Listing 1's printed order), then B, T.  No
 *   multiply-add is fused (-ffp-contract=off).
 *
 *   Storage: (depth + 2) planes of `plane_pitch` elements; a plane is
 *   (rows + 2) lines of `pitch` elements; interior planes 1..depth, rows
 *   1..rows, columns 1..cols.  The one-cell halo shell around the interior
 *   (planes 0 and depth+1, and rows / columns 0 and rows+1 / cols+1 of every
 *   plane) is a fixed Dirichlet boundary: read, never written.  Edge and
 *   corner cells of the shell are never read.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE3_OK 0
#define ORACLE3_EINVAL -1
#define ORACLE3_ENOMEM -4

static int threads3(int nthreads)
{
    if (nthreads > 0) return nthreads;
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int bad_shape(int64_t depth, int64_t rows, int64_t cols, int64_t pitch, int64_t plane_pitch, int64_t T)
{
    return depth < 1 || rows < 1 || cols < 1 || pitch < cols + 2 || plane_pitch < (rows + 2) * pitch || T < 0;
}

/* Advance u by T steps in double precision, in place (see above). */
int oracle_j3d7pt_f64(double* u, int64_t depth, int64_t rows, int64_t cols, int64_t pitch, int64_t plane_pitch,
                      const double* coeffs, int64_t T, int nthreads)
{
    if (!u || !coeffs || bad_shape(depth, rows, cols, pitch, plane_pitch, T)) return ORACLE3_EINVAL;
    if (T == 0) return ORACLE3_OK;
    const double wc = coeffs[0], wn = coeffs[1], ws = coeffs[2], we = coeffs[3], ww = coeffs[4];
    const double wt = coeffs[5], wb = coeffs[6];
    const size_t n_elem = (size_t)(depth + 2) * (size_t)plane_pitch;
    double* v = (double*)malloc(n_elem * sizeof(double));
    if (!v) return ORACLE3_ENOMEM;
    memcpy(v, u, n_elem * sizeof(double)); /* the second buffer's halo shell matches */
    double* in = u;
    double* out = v;
    nthreads = threads3(nthreads);
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
        for (int64_t z = 1; z <= depth; ++z) {
            for (int64_t i = 1; i <= rows; ++i) {
                const double* mid = in + z * plane_pitch + i * pitch;    /* plane z, row i */
                const double* up = in + z * plane_pitch + (i - 1) * pitch; /* row i-1: S */
                const double* dn = in + z * plane_pitch + (i + 1) * pitch; /* row i+1: N */
                const double* bel = in + (z - 1) * plane_pitch + i * pitch; /* plane z-1: B */
                const double* abv = in + (z + 1) * plane_pitch + i * pitch; /* plane z+1: T */
                double* o = out + z * plane_pitch + i * pitch;
                for (int64_t j = 1; j <= cols; ++j) {
                    double acc = ww * mid[j - 1];
                    acc = acc + we * mid[j + 1];
                    acc = acc + ws * up[j];
                    acc = acc + wc * mid[j];
                    acc = acc + wn * dn[j];
                    acc = acc + wb * bel[j];
                    acc = acc + wt * abv[j];
                    o[j] = acc;
                }
            }
        }
        double* tmp = in;
        in = out;
        out = tmp;
    }
    if (in != u) {
        for (int64_t z = 1; z <= depth; ++z)
            for (int64_t i = 1; i <= rows; ++i)
                memcpy(u + z * plane_pitch + i * pitch + 1, in + z * plane_pitch + i * pitch + 1,
                       (size_t)cols * sizeof(double));
    }
    free(v);
    return ORACLE3_OK;
}

/* The same in single precision: weights rounded to float once, every operation in float, same order. */
int oracle_j3d7pt_f32(float* u, int64_t depth, int64_t rows, int64_t cols, int64_t pitch, int64_t plane_pitch,
                      const double* coeffs, int64_t T, int nthreads)
{
    if (!u || !coeffs || bad_shape(depth, rows, cols, pitch, plane_pitch, T)) return ORACLE3_EINVAL;
    if (T == 0) return ORACLE3_OK;
    const float wc = (float)coeffs[0], wn = (float)coeffs[1], ws = (float)coeffs[2], we = (float)coeffs[3];
    const float ww = (float)coeffs[4], wt = (float)coeffs[5], wb = (float)coeffs[6];
    const size_t n_elem = (size_t)(depth + 2) * (size_t)plane_pitch;
    float* v = (float*)malloc(n_elem * sizeof(float));
    if (!v) return ORACLE3_ENOMEM;
    memcpy(v, u, n_elem * sizeof(float));
    float* in = u;
    float* out = v;
    nthreads = threads3(nthreads);
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
        for (int64_t z = 1; z <= depth; ++z) {
            for (int64_t i = 1; i <= rows; ++i) {
                const float* mid = in + z * plane_pitch + i * pitch;
                const float* up = in + z * plane_pitch + (i - 1) * pitch;
                const float* dn = in + z * plane_pitch + (i + 1) * pitch;
                const float* bel = in + (z - 1) * plane_pitch + i * pitch;
                const float* abv = in + (z + 1) * plane_pitch + i * pitch;
                float* o = out + z * plane_pitch + i * pitch;
                for (int64_t j = 1; j <= cols; ++j) {
                    float acc = ww * mid[j - 1];
                    acc = acc + we * mid[j + 1];
                    acc = acc + ws * up[j];
                    acc = acc + wc * mid[j];
                    acc = acc + wn * dn[j];
                    acc = acc + wb * bel[j];
                    acc = acc + wt * abv[j];
                    o[j] = acc;
                }
            }
        }
        float* tmp = in;
        in = out;
        out = tmp;
    }
    if (in != u) {
        for (int64_t z = 1; z <= depth; ++z)
            for (int64_t i = 1; i <= rows; ++i)
                memcpy(u + z * plane_pitch + i * pitch + 1, in + z * plane_pitch + i * pitch + 1,
                       (size_t)cols * sizeof(float));
    }
    free(v);
    return ORACLE3_OK;
}
