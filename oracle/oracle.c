/*
 * Oracle for dense C = alpha*A*B + beta*C0.  TEST INFRASTRUCTURE ONLY:
 * nothing on the product path may link, load or call this file.
 *
 * The paper treats classical matrix multiplication C = AB with A m x k and
 * B k x n (section 2.4), and its CDAG fixes the update rule
 *     C(t1,t2,t3) = C(t1,t2,t3-1) + A(t1,t3) * B(t3,t2)
 * i.e. every entry is a sum over the reduction index (section 5.1, the
 * definitions of the MMM CDAG).  The
 * oracle is that definition written out in binary64, with the BLAS scaling
 * convention on top:
 *     C[i][j] = alpha * (sum_{t=0..k-1} A[i][t]*B[t][j]) + beta * C0[i][j]
 *     D[i][j] = |alpha| * sum_t |A[i][t]|*|B[t][j]| + |beta| * |C0[i][j]|
 * D is the denominator of the normalised error metric.
 *
 * Rules that keep the result a plain, checkable function of the inputs:
 *  - t runs in ascending order for every entry; each product is rounded,
 *    then added (built with -ffp-contract=off, no fast-math), so the result
 *    does not depend on vectorisation or on the number of threads.
 *  - k == 0 or alpha == 0: A and B are not read; beta == 0: C0 is not read.
 *  - Rows of C are split over POSIX threads; rows are independent.
 * All matrices are row-major with leading dimensions lda, ldb, ldc.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int64_t m, n, k;
  double alpha;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double beta;
  const double *C0;
  int64_t ldc0;
  double *C;
  int64_t ldc;
  double *D; /* may be NULL */
  int64_t ldd;
  int64_t row_begin, row_end;
  int status;
} oracle_job;

static void *oracle_rows(void *arg) {
  oracle_job *J = (oracle_job *)arg;
  const int64_t n = J->n, k = J->k;
  const int read_ab = (k > 0 && J->alpha != 0.0);
  double *acc = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double *mag = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (!acc || !mag) {
    free(acc);
    free(mag);
    J->status = -1;
    return NULL;
  }
  for (int64_t i = J->row_begin; i < J->row_end; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      acc[j] = 0.0;
      mag[j] = 0.0;
    }
    if (read_ab) {
      for (int64_t t = 0; t < k; ++t) {
        const double a = J->A[i * J->lda + t];
        const double abs_a = fabs(a);
        const double *brow = J->B + t * J->ldb;
        for (int64_t j = 0; j < n; ++j) {
          const double prod = a * brow[j];
          acc[j] = acc[j] + prod;
          const double prod_abs = abs_a * fabs(brow[j]);
          mag[j] = mag[j] + prod_abs;
        }
      }
    }
    for (int64_t j = 0; j < n; ++j) {
      double c = read_ab ? J->alpha * acc[j] : 0.0;
      double d = read_ab ? fabs(J->alpha) * mag[j] : 0.0;
      if (J->beta != 0.0) {
        const double c0 = J->C0[i * J->ldc0 + j];
        c = c + J->beta * c0;
        d = d + fabs(J->beta) * fabs(c0);
      }
      J->C[i * J->ldc + j] = c;
      if (J->D) J->D[i * J->ldd + j] = d;
    }
  }
  free(acc);
  free(mag);
  J->status = 0;
  return NULL;
}

/*
 * Full oracle product.  Returns 0 on success, -1 on invalid arguments or
 * allocation failure.  nthreads <= 0 means one thread.
 */
int oracle_gemm(int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                const double *B, int64_t ldb, double beta, const double *C0, int64_t ldc0,
                double *C, int64_t ldc, double *D, int64_t ldd, int nthreads) {
  if (m < 0 || n < 0 || k < 0) return -1;
  if (m == 0 || n == 0) return 0;
  if (ldc < n || (D && ldd < n)) return -1;
  if (k > 0 && alpha != 0.0 && (!A || !B || lda < k || ldb < n)) return -1;
  if (beta != 0.0 && (!C0 || ldc0 < n)) return -1;
  if (!C) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > m) nthreads = (int)m;
  oracle_job *jobs = (oracle_job *)calloc((size_t)nthreads, sizeof(oracle_job));
  pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !tids) {
    free(jobs);
    free(tids);
    return -1;
  }
  int rc = 0;
  for (int w = 0; w < nthreads; ++w) {
    oracle_job *J = &jobs[w];
    J->m = m; J->n = n; J->k = k;
    J->alpha = alpha; J->A = A; J->lda = lda; J->B = B; J->ldb = ldb;
    J->beta = beta; J->C0 = C0; J->ldc0 = ldc0; J->C = C; J->ldc = ldc; J->D = D; J->ldd = ldd;
    J->row_begin = m * w / nthreads;
    J->row_end = m * (w + 1) / nthreads;
    J->status = -1;
  }
  int started = 0;
  for (int w = 1; w < nthreads; ++w) {
    if (pthread_create(&tids[w], NULL, oracle_rows, &jobs[w]) != 0) break;
    started = w;
  }
  oracle_rows(&jobs[0]);
  for (int w = 1; w <= started; ++w) pthread_join(tids[w], NULL);
  for (int w = started + 1; w < nthreads; ++w) oracle_rows(&jobs[w]); /* threads that failed to start */
  for (int w = 0; w < nthreads; ++w)
    if (jobs[w].status != 0) rc = -1;
  free(jobs);
  free(tids);
  return rc;
}
