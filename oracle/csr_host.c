/*
 * Host timing variant of the oracle's sparse matrix-vector product and Jacobi-PCG
 * (oracle; test infrastructure only: the CPU baseline of the benchmark and the
 * tests call it, never the GPU library).
 *
 * y = A x on the assembled CSR matrix of "Operator Decomposition" (A = G^t A_E G
 * assembled), one row per iteration of an OpenMP loop over rows.  The PCG is the
 * textbook algorithm of oracle/solvers.py ("Scalable Linear Solvers": CGSolver on
 * the operator; Jacobi preconditioner z = r / diag; stop when the recursive residual
 * ||r_k|| <= tol ||b||, x_0 = 0), its vector updates and dot products also as plain
 * OpenMP loops.  Nothing here is blocked, reordered or tuned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <omp.h>

void csr_spmv(int64_t n, const int64_t* indptr, const int32_t* indices, const double* data,
              const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) s += data[k] * x[indices[k]];
    y[i] = s;
  }
}

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Returns the number of iterations; *rel_res receives ||r_k|| / ||b||. */
int32_t csr_pcg_jacobi(int64_t n, const int64_t* indptr, const int32_t* indices,
                       const double* data, const double* diag, const double* b, double* x,
                       double tol, int32_t maxit, double* rel_res) {
  double* r = malloc(sizeof(double) * n);
  double* z = malloc(sizeof(double) * n);
  double* d = malloc(sizeof(double) * n);
  double* q = malloc(sizeof(double) * n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    x[i] = 0.0;
    r[i] = b[i];
    z[i] = b[i] / diag[i];
    d[i] = z[i];
  }
  const double bnorm = sqrt(dot(n, b, b));
  double rz = dot(n, r, z);
  double rr = dot(n, r, r);
  int32_t k = 0;
  while (k < maxit && sqrt(rr) > tol * bnorm) {
    csr_spmv(n, indptr, indices, data, d, q);
    const double alpha = rz / dot(n, d, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      x[i] += alpha * d[i];
      r[i] -= alpha * q[i];
      z[i] = r[i] / diag[i];
    }
    const double rz_new = dot(n, r, z);
    rr = dot(n, r, r);
    const double beta = rz_new / rz;
    rz = rz_new;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) d[i] = z[i] + beta * d[i];
    ++k;
  }
  *rel_res = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
  free(r);
  free(z);
  free(d);
  free(q);
  return k;
}

int32_t csr_max_threads(void) { return omp_get_max_threads(); }
