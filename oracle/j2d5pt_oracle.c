/*
 * j2d5pt_oracle.c -- plain CPU oracle for the j2d5pt iterative stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library, and the
 * library never calls it.
 *
 * What it computes (Zhang et al., "Exploiting Scratchpad Memory for Deep
 * Temporal Blocking", GPGPU '23):
 *
 *   Listing 1 gives the j2d5pt update: every output cell is the weighted sum
 *   of the input cell and its four axis neighbours, read from one buffer and
 *   written to another (Jacobi, not Gauss-Seidel).  Section 3.1 and the
 *   caption of Figure 1 repeat this update for T time steps.
 *
 *   Storage is row-major, (rows + 2) lines of `pitch` elements; the interior
 *   is i = 1..rows, j = 1..cols and the one-cell ring around it is a fixed
 *   Dirichlet halo that is read but never written.
 *
 *   Neighbour names follow Listing 1: x (the thread index, contiguous in
 *   memory) is the column j and y is the row i; W = (i, j-1), E = (i, j+1),
 *   S = (i-1, j), N = (i+1, j), C = (i, j).
 *
 *   Evaluation order: the products are rounded one by one and summed left to
 *   right in the order Listing 1 prints them, W, E, S, C, N.  The file is
 *   compiled with -ffp-contract=off, so no multiply-add is fused.
 *
 *   coeffs[] is passed in the order (c, n, s, e, w).
 *
 * Parallelising the row loop changes no operation order, so the result does
 * not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Return codes. */
#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -4

static int check_args(const void* u, int64_t rows, int64_t cols, int64_t pitch,
                      const double* coeffs, int64_t T)
{
    if (!u || !coeffs) return ORACLE_EINVAL;
    if (rows < 1 || cols < 1 || pitch < cols + 2 || T < 0) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/*
 * Advance u by T steps in double precision, in place.  u holds the (rows+2)
 * x pitch storage described above; on return its interior holds u^T and its
 * halo is untouched.  nthreads <= 0 means the OpenMP default.
 */
int oracle_j2d5pt_f64(double* u, int64_t rows, int64_t cols, int64_t pitch,
                      const double* coeffs, int64_t T, int nthreads)
{
    int rc = check_args(u, rows, cols, pitch, coeffs, T);
    if (rc != ORACLE_OK) return rc;
    if (T == 0) return ORACLE_OK;

    const double wc = coeffs[0], wn = coeffs[1], ws = coeffs[2];
    const double we = coeffs[3], ww = coeffs[4];
    const size_t n_elem = (size_t)(rows + 2) * (size_t)pitch;
    double* v = (double*)malloc(n_elem * sizeof(double));
    if (!v) return ORACLE_ENOMEM;
    /* The second buffer starts as a full copy so that its halo matches. */
    memcpy(v, u, n_elem * sizeof(double));

    double* in = u;
    double* out = v;
    if (nthreads <= 0) {
#ifdef _OPENMP
        nthreads = omp_get_max_threads();
#else
        nthreads = 1;
#endif
    }
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t i = 1; i <= rows; ++i) {
            const double* up = in + (i - 1) * pitch; /* row i-1: S */
            const double* mid = in + i * pitch;      /* row i: W, C, E */
            const double* dn = in + (i + 1) * pitch; /* row i+1: N */
            double* o = out + i * pitch;
            for (int64_t j = 1; j <= cols; ++j) {
                double acc = ww * mid[j - 1];
                acc = acc + we * mid[j + 1];
                acc = acc + ws * up[j];
                acc = acc + wc * mid[j];
                acc = acc + wn * dn[j];
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
    return ORACLE_OK;
}

/*
 * The same definition carried out in single precision: the coefficients are
 * rounded to float once, every product and sum is a float operation in the
 * same order, no fusion.  It is the bit-level reference for the library's
 * FP32 path; the FP64 oracle stays the accuracy reference.
 */
int oracle_j2d5pt_f32(float* u, int64_t rows, int64_t cols, int64_t pitch,
                      const double* coeffs, int64_t T, int nthreads)
{
    int rc = check_args(u, rows, cols, pitch, coeffs, T);
    if (rc != ORACLE_OK) return rc;
    if (T == 0) return ORACLE_OK;

    const float wc = (float)coeffs[0], wn = (float)coeffs[1], ws = (float)coeffs[2];
    const float we = (float)coeffs[3], ww = (float)coeffs[4];
    const size_t n_elem = (size_t)(rows + 2) * (size_t)pitch;
    float* v = (float*)malloc(n_elem * sizeof(float));
    if (!v) return ORACLE_ENOMEM;
    memcpy(v, u, n_elem * sizeof(float));

    float* in = u;
    float* out = v;
    if (nthreads <= 0) {
#ifdef _OPENMP
        nthreads = omp_get_max_threads();
#else
        nthreads = 1;
#endif
    }
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t i = 1; i <= rows; ++i) {
            const float* up = in + (i - 1) * pitch;
            const float* mid = in + i * pitch;
            const float* dn = in + (i + 1) * pitch;
            float* o = out + i * pitch;
            for (int64_t j = 1; j <= cols; ++j) {
                float acc = ww * mid[j - 1];
                acc = acc + we * mid[j + 1];
                acc = acc + ws * up[j];
                acc = acc + wc * mid[j];
                acc = acc + wn * dn[j];
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
    return ORACLE_OK;
}

/* Number of OpenMP threads a call with nthreads <= 0 would use. */
int oracle_default_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
