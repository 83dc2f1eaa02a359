// Device-resident state of the preconditioned CG solver and its launchers.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace pafem {

// Lives at the start of the solver workspace.  Every scalar of the iteration
// stays on the device; the host only reads `done`/`iter` now and then.
struct CGState {
  double rz;     // r . z of the current residual
  double alpha;  // step length of the current iteration
  double beta;   // direction update factor
  double rr;     // r . r
  double bb;     // b . b
  double tol2;   // rel_tol^2 * b . b
  double res2;   // ||b - A x||^2 computed at exit
  double pad0;
  int32_t iter;  // completed iterations
  int32_t done;  // 0 running, 1 converged, 2 breakdown
  int32_t max_hist;
  int32_t pad1;
  uint32_t ticket[8];  // arrival counters of the last-block reductions
};

constexpr int kCGBlocks = 1024;  // fixed grid of the vector kernels = number of partials
constexpr int kCGThreads = 256;

// zero the state and tickets; hist holds max_hist entries
void launch_cg_reset(CGState* st, int32_t max_hist, hipStream_t s);
// r = b - q (q may be null: r = b); x = 0 if zero_guess; d = z = r / diag;
// rz, rr, bb, tol2, done, hist[0].
void launch_cg_init(CGState* st, double* partials, const double* b, const double* q,
                    const double* diag, double* x, double* r, double* d, int zero_guess,
                    double rel_tol, double* hist, int64_t n, hipStream_t s);
// alpha = rz / (d . q); breakdown if d . q <= 0 or non-finite
void launch_cg_dot(CGState* st, double* partials, const double* d, const double* q, int64_t n,
                   hipStream_t s);
// x += alpha d; r -= alpha q; z = r / diag; rz, rr, beta, iter, hist, convergence
void launch_cg_update(CGState* st, double* partials, double* x, double* r, const double* d,
                      const double* q, const double* diag, double* hist, int64_t n,
                      hipStream_t s);
// d = r / diag + beta d
void launch_cg_direction(CGState* st, const double* r, const double* diag, double* d, int64_t n,
                         hipStream_t s);
// res2 = ||b - q||^2 (always runs, ignores `done`)
void launch_residual_norm(CGState* st, double* partials, const double* b, const double* q,
                          int64_t n, hipStream_t s);

}  // namespace pafem
