/*
 * Plain FP64 CPU oracle for the explicit inverse of a symmetric positive
 * definite matrix.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check
 * and the benchmark's CPU-baseline leg are the only users.  It shares no code
 * with the GPU library and must never be linked into it.
 *
 * What it computes is the plain definition of the method of the paper
 * (Agullo et al., "Towards an Efficient Tile Matrix Inversion of Symmetric
 * Positive Definite Matrices on Multicore Architectures", Section 2,
 * Algorithm 1): the three stages of the tile algorithm collapse, at tile order
 * b = 1, to three unblocked loops.
 *
 *   Stage 1 (Cholesky, Alg. 1 step 1):      A = L L^T, L lower, l_jj > 0
 *   Stage 2 (triangular inverse, step 2):   X = L^{-1}
 *   Stage 3 (product, step 3):              A^{-1} = X^T X
 *
 * Every loop is the textbook definition: no blocking, no reordering of a sum
 * (each sum runs in natural increasing index order), IEEE binary64 with
 * round-to-nearest.  Build with -O2 -ffp-contract=off and never -ffast-math,
 * so that the compiler neither fuses nor reassociates.
 *
 * Storage: every matrix argument is column-major with a leading dimension;
 * only the lower triangle (row >= column) of an input is read.  Internally the
 * stages use private row-major or column-major copies so that every inner
 * sum is a walk over contiguous memory; this changes nothing in the
 * arithmetic.
 *
 * Error behaviour follows LAPACK xPOTRF: the return value is 0 on success,
 * k > 0 when the leading minor of order k is not positive definite (a pivot
 * d <= 0, or NaN), and -1 when memory could not be obtained.
 *
 * Optional OpenMP parallelism runs only over independent outputs (each output
 * element is computed by exactly one thread with the same sequential sum), so
 * the results do not depend on the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CM(a, ld, i, j) ((a)[(size_t)(i) + (size_t)(ld) * (size_t)(j)])

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}

/*
 * Stage 1 -- Cholesky factor (Alg. 1, step 1, at b = 1: SYRK, POTRF, GEMM and
 * TRSM reduce to the scalar left-looking recurrences below).
 *   d      = a_jj - sum_{k<j} l_jk^2          (k increasing)
 *   l_jj   = sqrt(d)                           (INFO = j+1 if d <= 0 or NaN)
 *   l_ij   = (a_ij - sum_{k<j} l_ik l_jk) / l_jj,   i > j
 * Input: lower triangle of A (column-major, lda).  Output: L written to the
 * lower triangle of Lout (column-major, ldl); the strictly upper part of Lout
 * is set to zero.
 */
int oracle_potrf(int n, const double* A, int lda, double* Lout, int ldl) {
  if (n <= 0) return 0;
  /* row-major copy: Lr[i*n + k] = l_ik, so both factors of each sum are rows */
  double* Lr = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  if (!Lr) return -1;
  int info = 0;
  for (int j = 0; j < n && !info; ++j) {
    const double* lj = Lr + (size_t)j * n;
    double d = CM(A, lda, j, j);
    for (int k = 0; k < j; ++k) d -= lj[k] * lj[k];
    if (!(d > 0.0)) { info = j + 1; break; }
    const double ljj = sqrt(d);
    Lr[(size_t)j * n + j] = ljj;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      const double* li = Lr + (size_t)i * n;
      double s = CM(A, lda, i, j);
      for (int k = 0; k < j; ++k) s -= li[k] * lj[k];
      Lr[(size_t)i * n + j] = s / ljj;
    }
  }
  if (!info) {
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        CM(Lout, ldl, i, j) = (i >= j) ? Lr[(size_t)i * n + j] : 0.0;
  }
  free(Lr);
  return info;
}

/*
 * Stage 2 -- inverse of a lower triangular matrix (Alg. 1, step 2, at b = 1).
 * From X L = I, for each column j (taken from the last to the first, since
 * column j uses the columns to its right):
 *   x_jj = 1 / l_jj
 *   x_ij = -( sum_{k=j+1..i} x_ik l_kj ) / l_jj,   i > j   (k increasing)
 * Input: lower triangle of L (column-major, ldl).  Output: X into the lower
 * triangle of Xout (strictly upper part set to zero).  Returns j+1 if a
 * diagonal entry l_jj is zero.
 */
int oracle_trtri(int n, const double* L, int ldl, double* Xout, int ldx) {
  if (n <= 0) return 0;
  for (int j = 0; j < n; ++j)
    if (CM(L, ldl, j, j) == 0.0) return j + 1;
  /* Xr row-major (x_ik contiguous in k), Lc column-major (l_kj contiguous in k) */
  double* Xr = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  double* Lc = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  if (!Xr || !Lc) { free(Xr); free(Lc); return -1; }
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) Lc[(size_t)j * n + i] = CM(L, ldl, i, j);
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = Lc[(size_t)j * n + j];
    Xr[(size_t)j * n + j] = 1.0 / ljj;
    const double* lcol = Lc + (size_t)j * n;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      const double* xi = Xr + (size_t)i * n;
      double s = 0.0;
      for (int k = j + 1; k <= i; ++k) s += xi[k] * lcol[k];
      Xr[(size_t)i * n + j] = -s / ljj;
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      CM(Xout, ldx, i, j) = (i >= j) ? Xr[(size_t)i * n + j] : 0.0;
  free(Xr);
  free(Lc);
  return 0;
}

/*
 * Stage 3 -- product of the transposed inverse factor with itself (Alg. 1,
 * step 3, at b = 1):  y_ij = sum_{k=i..n-1} x_ki x_kj  for i >= j
 * (k increasing), i.e. the lower triangle of X^T X.
 * Input: lower triangle of X (column-major, ldx; strictly upper part ignored).
 * Output: lower triangle of Y (Yout, column-major); the strictly upper part of
 * Yout is left untouched.
 */
void oracle_lauum(int n, const double* X, int ldx, double* Yout, int ldy) {
  if (n <= 0) return;
  /* column-major copy with explicit zeros above the diagonal */
  double* Xc = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  if (!Xc) return;
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) Xc[(size_t)j * n + i] = CM(X, ldx, i, j);
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < n; ++j) {
    const double* xj = Xc + (size_t)j * n;
    for (int i = j; i < n; ++i) {
      const double* xi = Xc + (size_t)i * n;
      double s = 0.0;
      for (int k = i; k < n; ++k) s += xi[k] * xj[k];
      CM(Yout, ldy, i, j) = s;
    }
  }
  free(Xc);
}

/*
 * The whole method: A <- A^{-1} on the lower triangle, in place, as the three
 * stages above.  The strictly upper triangle of A is neither read nor
 * written.  Returns the Cholesky INFO (A is then left unchanged) or 0.
 */
int oracle_spd_inverse(int n, double* A, int lda) {
  if (n <= 0) return 0;
  double* L = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
  double* X = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
  if (!L || !X) { free(L); free(X); return -1; }
  int info = oracle_potrf(n, A, lda, L, n);
  if (!info) info = oracle_trtri(n, L, n, X, n);
  if (!info) oracle_lauum(n, X, n, A, lda);
  free(L);
  free(X);
  return info;
}

/*
 * Gradient of a scalar loss through the inverse: for L(A) with upstream
 * gradient G = dL/d(A^{-1}), the gradient with respect to a symmetric A is
 *   grad = -Y S Y,   S = (G + G^T) / 2,   Y = A^{-1} (full symmetric),
 * the standard differential d(A^{-1}) = -A^{-1} dA A^{-1}.
 * Y is given by its lower triangle (column-major, ldy) and mirrored here.
 * G is a full n x n column-major matrix; grad is written in full.
 * Plain triple loops in natural order: W = Y S, then grad = -(W Y).
 */
int oracle_inverse_grad(int n, const double* Ylow, int ldy, const double* G, int ldg,
                        double* grad, int ldgr) {
  if (n <= 0) return 0;
  const size_t nn = (size_t)n * (size_t)n;
  double* Yr = (double*)malloc(nn * sizeof(double)); /* row-major full Y */
  double* Sc = (double*)malloc(nn * sizeof(double)); /* column-major S   */
  double* Wr = (double*)malloc(nn * sizeof(double)); /* row-major W      */
  double* Yc = (double*)malloc(nn * sizeof(double)); /* column-major Y   */
  if (!Yr || !Sc || !Wr || !Yc) { free(Yr); free(Sc); free(Wr); free(Yc); return -1; }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double y = (i >= j) ? CM(Ylow, ldy, i, j) : CM(Ylow, ldy, j, i);
      Yr[(size_t)i * n + j] = y;
      Yc[(size_t)j * n + i] = y;
    }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      Sc[(size_t)j * n + i] = (CM(G, ldg, i, j) + CM(G, ldg, j, i)) / 2.0;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    const double* yi = Yr + (size_t)i * n;
    for (int j = 0; j < n; ++j) {
      const double* sj = Sc + (size_t)j * n;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += yi[k] * sj[k];
      Wr[(size_t)i * n + j] = s;
    }
  }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    const double* wi = Wr + (size_t)i * n;
    for (int j = 0; j < n; ++j) {
      const double* yj = Yc + (size_t)j * n;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += wi[k] * yj[k];
      CM(grad, ldgr, i, j) = -s;
    }
  }
  free(Yr);
  free(Sc);
  free(Wr);
  free(Yc);
  return 0;
}


/*
 * Solve with the Cholesky factor (the solve that the factor of step 1 of
 * Alg. 1 serves, Section 2): A X = B with A = L L^T, by plain substitutions
 * per right-hand side column, natural order:
 *   forward   y_i = (b_i - sum_{k<i} l_ik y_k) / l_ii,     i = 0..n-1
 *   backward  x_i = (y_i - sum_{k>i} l_ki x_k) / l_ii,     i = n-1..0
 * L: lower triangle (column-major, ldl; the upper part is not read).
 * B: column-major n x nrhs (ldb), overwritten by X.  Returns 0, or i+1 when
 * l_ii = 0.
 */
int oracle_potrs(int n, int nrhs, const double* L, int ldl, double* B, int ldb) {
  for (int i = 0; i < n; ++i)
    if (CM(L, ldl, i, i) == 0.0) return i + 1;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < nrhs; ++c) {
    double* b = B + (size_t)ldb * c;
    for (int i = 0; i < n; ++i) {
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= CM(L, ldl, i, k) * b[k];
      b[i] = s / CM(L, ldl, i, i);
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = b[i];
      for (int k = i + 1; k < n; ++k) s -= CM(L, ldl, k, i) * b[k];
      b[i] = s / CM(L, ldl, i, i);
    }
  }
  return 0;
}
