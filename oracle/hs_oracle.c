/*
 * hs_oracle.c -- FP64 reference for the hyper-systolic matrix product and
 * for the all-pairs n-body interaction (the n^2-problem, at the end).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table
 * or helper with the HIP library.
 *
 * The hyper-systolic method reorders communication but computes exactly the
 * ordinary matrix product (Sec. 3.1, Eq. PRODUCT: c_ij = sum_k a_ik b_kj;
 * Sec. 5.2.3, Thm. GAIN3 -- no extra or fewer multiply-adds).  The oracle is
 * therefore that definition written out: plain triple loops in double
 * precision, contraction index ascending, no blocking, no reordering.
 * OpenMP splits independent output rows only; every output element is one
 * sequential ascending-k sum, so the result does not depend on thread count.
 *
 * All matrices are dense, row-major, with explicit leading dimensions
 * (elements between consecutive rows).  Inputs are the stored values of the
 * caller's matrices promoted to double.
 *
 * Loop order: where the contraction runs over rows of a row-major operand,
 * an output row is accumulated as acc[j] += a_ip * b_pj for p = 0, 1, ...
 * (the p-loop outside the j-loop).  Each acc[j] still receives its terms one
 * at a time in ascending p, so every element is bitwise the same sum as the
 * textbook i-j-p loop; only the memory walk differs.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

/* Threads used by the loops below (n <= 0: the OpenMP default).  Only for
 * timing the oracle; the results do not depend on it. */
void hs_oracle_set_threads(int n)
{
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
}

/* C[m,n] = A[m,k] . B[k,n]  (Eq. PRODUCT, with A n x m and B m x n
 * generalised to rectangular M x Kd times Kd x N). */
void hs_oracle_gemm(int64_t m, int64_t n, int64_t k,
                    const double *A, int64_t lda,
                    const double *B, int64_t ldb,
                    double *C, int64_t ldc)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double a = A[i * lda + p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

/* C[m,n] = A^T . B with A stored as a k x m matrix (the transposed product
 * the paper announces in its abstract and summary): c_ij = sum_p a_pi b_pj. */
void hs_oracle_gemm_tn(int64_t m, int64_t n, int64_t k,
                       const double *A, int64_t lda,
                       const double *B, int64_t ldb,
                       double *C, int64_t ldc)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double a = A[p * lda + i];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

/* y[m] = A[m,n] . x[n]  (the matrix-vector product of the abstract). */
void hs_oracle_gemv(int64_t m, int64_t n,
                    const double *A, int64_t lda,
                    const double *x, double *y)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s += A[i * lda + j] * x[j];
        y[i] = s;
    }
}

/* Gradient of L = sum_ij C_ij G_ij with C = A B (A m x k, B k x n, G m x n):
 *   dL/da_ip = sum_j g_ij b_pj   (dA = G . B^T, m x k)
 *   dL/db_pj = sum_i a_ip g_ij   (dB = A^T . G, k x n)
 * Either output pointer may be NULL to skip it. */
void hs_oracle_backward(int64_t m, int64_t n, int64_t k,
                        const double *A, int64_t lda,
                        const double *B, int64_t ldb,
                        const double *G, int64_t ldg,
                        double *dA, int64_t ldda,
                        double *dB, int64_t lddb)
{
    int64_t i;
    if (dA) {
#pragma omp parallel for schedule(static)
        for (i = 0; i < m; ++i) {
            for (int64_t p = 0; p < k; ++p) {
                double s = 0.0;
                for (int64_t j = 0; j < n; ++j)
                    s += G[i * ldg + j] * B[p * ldb + j];
                dA[i * ldda + p] = s;
            }
        }
    }
    if (dB) {
#pragma omp parallel for schedule(static)
        for (i = 0; i < k; ++i) {
            double *c = dB + i * lddb;
            for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
            for (int64_t q = 0; q < m; ++q) {
                const double a = A[q * lda + i];
                const double *g = G + q * ldg;
                for (int64_t j = 0; j < n; ++j) c[j] += a * g[j];
            }
        }
    }
}

/* Selected rows of C = A . B: out[t, :] = row rows[t] of the product.
 * Used where the full product is too large for the CPU (sampled-row parity). */
void hs_oracle_gemm_rows(int64_t n, int64_t k,
                         const double *A, int64_t lda,
                         const double *B, int64_t ldb,
                         const int64_t *rows, int64_t nrows,
                         double *out, int64_t ldo)
{
    int64_t t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        double *c = out + t * ldo;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double a = A[i * lda + p];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

/* Selected rows of C = A^T . B (A stored k x m). */
void hs_oracle_gemm_tn_rows(int64_t n, int64_t k,
                            const double *A, int64_t lda,
                            const double *B, int64_t ldb,
                            const int64_t *rows, int64_t nrows,
                            double *out, int64_t ldo)
{
    int64_t t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        double *c = out + t * ldo;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double a = A[p * lda + i];
            const double *b = B + p * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

/* Selected rows of dA = G . B^T (row i: sum_j g_ij b_pj). */
void hs_oracle_grad_a_rows(int64_t n, int64_t k,
                           const double *G, int64_t ldg,
                           const double *B, int64_t ldb,
                           const int64_t *rows, int64_t nrows,
                           double *out, int64_t ldo)
{
    int64_t t;
#pragma omp parallel for schedule(static)
    for (t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int64_t p = 0; p < k; ++p) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j)
                s += G[i * ldg + j] * B[p * ldb + j];
            out[t * ldo + p] = s;
        }
    }
}

/*
 * All-pairs gravitational interaction of n bodies: the prototype
 * n^2-problem of Sec. 2.2, which the two-array recipe of Sec. 4.1 computes as
 * F_i = (+)_j f(x_i, z_j) with both data streams x and z equal to the bodies
 * and (+) the sum.  With G = 1 and a softening eps2 >= 0, for body i at r_i:
 *
 *   a_i   =  sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps2)^(3/2)
 *   phi_i = -sum_{j != i} m_j / (|r_j - r_i|^2 + eps2)^(1/2)
 *
 * (acceleration and potential at body i).  The definition written out:
 * plain doubles, j ascending, one sequential sum per output element.
 * bodies: n x 4 doubles (x, y, z, m); out: n x 4 (ax, ay, az, phi).
 * scale (may be NULL): scale[i] = sum_{j != i} m_j |r_j - r_i| / s^(3/2), the
 * sum of the lengths of the terms of a_i (the condition of that sum).
 */
static void nbody_one(int64_t n, const double *bodies, double eps2, int64_t i,
                      double *o, double *scale)
{
    const double xi = bodies[4 * i], yi = bodies[4 * i + 1], zi = bodies[4 * i + 2];
    double ax = 0.0, ay = 0.0, az = 0.0, phi = 0.0, sc = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const double dx = bodies[4 * j] - xi;
        const double dy = bodies[4 * j + 1] - yi;
        const double dz = bodies[4 * j + 2] - zi;
        const double m = bodies[4 * j + 3];
        const double s = dx * dx + dy * dy + dz * dz + eps2;
        const double r = sqrt(s);
        const double w = m / (s * r);
        ax += w * dx;
        ay += w * dy;
        az += w * dz;
        phi -= m / r;
        sc += fabs(w) * sqrt(dx * dx + dy * dy + dz * dz);
    }
    o[0] = ax;
    o[1] = ay;
    o[2] = az;
    o[3] = phi;
    if (scale) *scale = sc;
}

void hs_oracle_nbody(int64_t n, const double *bodies, double eps2, double *out, double *scale)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 64)
    for (i = 0; i < n; ++i)
        nbody_one(n, bodies, eps2, i, out + 4 * i, scale ? scale + i : NULL);
}

/* The same for the bodies rows[0..nrows-1] only (sampled parity at sizes
 * where the full n^2 sum is too slow for the CPU). */
void hs_oracle_nbody_rows(int64_t n, const double *bodies, double eps2,
                          const int64_t *rows, int64_t nrows, double *out, double *scale)
{
    int64_t t;
#pragma omp parallel for schedule(dynamic, 4)
    for (t = 0; t < nrows; ++t)
        nbody_one(n, bodies, eps2, rows[t], out + 4 * t, scale ? scale + t : NULL);
}
