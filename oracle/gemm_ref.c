/*
 * CPU oracle for the batched GEMM  C_b = alpha * op(A_b) * op(B_b) + beta * C0_b.
 *
 * TEST INFRASTRUCTURE ONLY: this file is the checker of the GPU library and
 * is never linked into it.  Only tests/, the smoke entry point and the
 * benchmark's CPU-baseline leg may load it.
 *
 * The operation is the paper's matrix multiply (section 3, "A matrix multiply
 * case study": each output element accumulates the products of one row of the
 * left input and one column of the right input), stated with transposes and
 * alpha/beta.  The oracle is the definition itself: a triple loop in the
 * order (i, j, k) with an FP64 accumulator over the FP32 input values, no
 * blocking and no reordering.  OpenMP splits the (batch, i) loop only.
 *
 * Storage is row-major.  op(A) is M x K: element (i, k) is A[i*lda + k] when
 * transA == 0 and A[k*lda + i] when transA == 1.  op(B) is K x N likewise.
 * Batch item b starts at A + b*strideA (and B + b*strideB, C0 + b*strideC).
 * The result is written dense, out[(b*M + i)*N + j], in FP64.  When beta == 0
 * C0 is not read (it may be NULL and may hold NaN).
 */
#include <stdint.h>
#include <stddef.h>

static inline double a_at(const float* A, int64_t lda, int ta, int64_t i, int64_t k) {
    return ta ? (double)A[k * lda + i] : (double)A[i * lda + k];
}
static inline double b_at(const float* B, int64_t ldb, int tb, int64_t k, int64_t j) {
    return tb ? (double)B[j * ldb + k] : (double)B[k * ldb + j];
}

static double dot_ij(const float* A, int64_t lda, int ta, const float* B, int64_t ldb, int tb,
                     int64_t K, int64_t i, int64_t j) {
    double acc = 0.0;
    for (int64_t k = 0; k < K; ++k) acc += a_at(A, lda, ta, i, k) * b_at(B, ldb, tb, k, j);
    return acc;
}

static double finish(double acc, double alpha, double beta, const float* C0, int64_t ldc,
                     int64_t i, int64_t j) {
    double v = alpha * acc;
    if (beta != 0.0) v += beta * (double)C0[i * ldc + j];
    return v;
}

void kt_oracle_gemm(int64_t M, int64_t N, int64_t K, int64_t batch, int ta, int tb,
                    double alpha, double beta,
                    const float* A, int64_t lda, int64_t strideA,
                    const float* B, int64_t ldb, int64_t strideB,
                    const float* C0, int64_t ldc, int64_t strideC,
                    double* out) {
    int64_t rows = batch * M;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t bi = 0; bi < rows; ++bi) {
        int64_t b = bi / M, i = bi % M;
        const float* Ab = A + b * strideA;
        const float* Bb = B + b * strideB;
        const float* Cb = C0 ? C0 + b * strideC : NULL;
        for (int64_t j = 0; j < N; ++j) {
            double acc = dot_ij(Ab, lda, ta, Bb, ldb, tb, K, i, j);
            out[bi * N + j] = finish(acc, alpha, beta, Cb, ldc, i, j);
        }
    }
}

/*
 * Same definition evaluated only on selected full rows and full columns of
 * every batch item (used where the full product is too large for the CPU):
 * out_rows[(b*nr + r)*N + j] = C_b[rows[r]][j] and
 * out_cols[(b*M + i)*nc + c] = C_b[i][cols[c]].
 */
void kt_oracle_gemm_sampled(int64_t M, int64_t N, int64_t K, int64_t batch, int ta, int tb,
                            double alpha, double beta,
                            const float* A, int64_t lda, int64_t strideA,
                            const float* B, int64_t ldb, int64_t strideB,
                            const float* C0, int64_t ldc, int64_t strideC,
                            const int64_t* rows, int64_t nr, const int64_t* cols, int64_t nc,
                            double* out_rows, double* out_cols) {
    int64_t total = batch * (nr + M);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < total; ++t) {
        int64_t b = t / (nr + M), u = t % (nr + M);
        const float* Ab = A + b * strideA;
        const float* Bb = B + b * strideB;
        const float* Cb = C0 ? C0 + b * strideC : NULL;
        if (u < nr) {
            int64_t i = rows[u];
            for (int64_t j = 0; j < N; ++j)
                out_rows[(b * nr + u) * N + j] =
                    finish(dot_ij(Ab, lda, ta, Bb, ldb, tb, K, i, j), alpha, beta, Cb, ldc, i, j);
        } else {
            int64_t i = u - nr;
            for (int64_t c = 0; c < nc; ++c) {
                int64_t j = cols[c];
                out_cols[(b * M + i) * nc + c] =
                    finish(dot_ij(Ab, lda, ta, Bb, ldb, tb, K, i, j), alpha, beta, Cb, ldc, i, j);
            }
        }
    }
}

int kt_oracle_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of OpenMP threads later calls use (for timing the oracle on one
 * core and on all of them); no effect on the arithmetic. */
void kt_oracle_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
