/* CPU oracle — test infrastructure only.
 *
 * Plain FP64 Cholesky factorisations used by the oracle.  The paper solves
 * the condensed KKT system by P'KP = LDL' with no pivoting (Section 2, LDL^T
 * factorization; Section 3, primal condensed system is SPD so Cholesky
 * needs no pivoting).  For SPD K this is L L' with D folded in; the factor is
 * unique for a given P.
 *
 *   oracle_dense_cholesky   row-major n x n, lower triangle in place
 *   oracle_sparse_cholesky  left-looking column Cholesky on a given column
 *                           structure of L (CSC, diagonal first in each
 *                           column, rows ascending)
 * Both return 0, or j+1 when pivot j is not positive (or not finite).
 *
 *   oracle_sparse_ldlt      the same left-looking loop for P'AP = L D L'
 *                           with unit lower L and a diagonal D of either
 *                           sign (Section 2: an SQD matrix has this
 *                           factorisation for every P, strong factorisability);
 *                           returns j+1 when pivot j is zero or not finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

int oracle_dense_cholesky(int64_t n, double* A) {
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0) || !isfinite(d)) return (int)(j + 1);
    double ljj = sqrt(d);
    A[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / ljj;
    }
  }
  return 0;
}

void oracle_dense_solve(int64_t n, const double* L, double* x) {
  for (int64_t i = 0; i < n; ++i) {
    double s = x[i];
    for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
    x[i] = s / L[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}

int oracle_sparse_cholesky(int64_t n, const int64_t* Lp, const int32_t* Li, double* Lx) {
  double* x = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* link = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int status = 0;
  for (int64_t i = 0; i < n; ++i) head[i] = -1;
  for (int64_t j = 0; j < n && !status; ++j) {
    /* scatter column j of K */
    for (int64_t q = Lp[j]; q < Lp[j + 1]; ++q) x[Li[q]] = Lx[q];
    /* subtract L(j,k) * L(j:n,k) for every earlier column k with L(j,k) != 0 */
    int64_t k = head[j];
    head[j] = -1;
    while (k >= 0) {
      int64_t knext = link[k];
      int64_t p = next[k];
      double ljk = Lx[p];
      for (int64_t q = p; q < Lp[k + 1]; ++q) x[Li[q]] -= Lx[q] * ljk;
      next[k] = p + 1;
      if (p + 1 < Lp[k + 1]) {
        int64_t r = Li[p + 1];
        link[k] = head[r];
        head[r] = k;
      }
      k = knext;
    }
    double d = x[j];
    if (!(d > 0.0) || !isfinite(d)) { status = (int)(j + 1); break; }
    double ljj = sqrt(d);
    Lx[Lp[j]] = ljj;
    x[j] = 0.0;
    for (int64_t q = Lp[j] + 1; q < Lp[j + 1]; ++q) {
      Lx[q] = x[Li[q]] / ljj;
      x[Li[q]] = 0.0;
    }
    next[j] = Lp[j] + 1;
    if (Lp[j] + 1 < Lp[j + 1]) {
      int64_t r = Li[Lp[j] + 1];
      link[j] = head[r];
      head[r] = j;
    }
  }
  free(x); free(head); free(link); free(next);
  return status;
}

void oracle_sparse_solve(int64_t n, const int64_t* Lp, const int32_t* Li, const double* Lx,
                         double* x) {
  for (int64_t j = 0; j < n; ++j) {
    x[j] /= Lx[Lp[j]];
    for (int64_t q = Lp[j] + 1; q < Lp[j + 1]; ++q) x[Li[q]] -= Lx[q] * x[j];
  }
  for (int64_t j = n - 1; j >= 0; --j) {
    double s = x[j];
    for (int64_t q = Lp[j] + 1; q < Lp[j + 1]; ++q) s -= Lx[q] * x[Li[q]];
    x[j] = s / Lx[Lp[j]];
  }
}

int oracle_sparse_ldlt(int64_t n, const int64_t* Lp, const int32_t* Li, double* Lx, double* D) {
  double* x = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* link = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int status = 0;
  for (int64_t i = 0; i < n; ++i) head[i] = -1;
  for (int64_t j = 0; j < n && !status; ++j) {
    /* scatter column j of A */
    for (int64_t q = Lp[j]; q < Lp[j + 1]; ++q) x[Li[q]] = Lx[q];
    /* subtract L(j:n,k) D(k) L(j,k) for every earlier column k with L(j,k) != 0 */
    int64_t k = head[j];
    head[j] = -1;
    while (k >= 0) {
      int64_t knext = link[k];
      int64_t p = next[k];
      double f = Lx[p] * D[k];
      for (int64_t q = p; q < Lp[k + 1]; ++q) x[Li[q]] -= Lx[q] * f;
      next[k] = p + 1;
      if (p + 1 < Lp[k + 1]) {
        int64_t r = Li[p + 1];
        link[k] = head[r];
        head[r] = k;
      }
      k = knext;
    }
    double d = x[j];
    if (d == 0.0 || !isfinite(d)) { status = (int)(j + 1); break; }
    D[j] = d;
    Lx[Lp[j]] = 1.0;
    x[j] = 0.0;
    for (int64_t q = Lp[j] + 1; q < Lp[j + 1]; ++q) {
      Lx[q] = x[Li[q]] / d;
      x[Li[q]] = 0.0;
    }
    next[j] = Lp[j] + 1;
    if (Lp[j] + 1 < Lp[j + 1]) {
      int64_t r = Li[Lp[j] + 1];
      link[j] = head[r];
      head[r] = j;
    }
  }
  free(x); free(head); free(link); free(next);
  return status;
}

void oracle_sparse_ldlt_solve(int64_t n, const int64_t* Lp, const int32_t* Li, const double* Lx,
                              const double* D, double* x) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t q = Lp[j] + 1; q < Lp[j + 1]; ++q) x[Li[q]] -= Lx[q] * x[j];
  for (int64_t j = 0; j < n; ++j) x[j] /= D[j];
  for (int64_t j = n - 1; j >= 0; --j) {
    double s = x[j];
    for (int64_t q = Lp[j] + 1; q < Lp[j + 1]; ++q) s -= Lx[q] * x[Li[q]];
    x[j] = s;
  }
}
