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

// The iteration kernels are templated on the vector type TV (double, or float
// for the inner solve of iterative refinement); dot products always accumulate
// in double.
//
// r = b*bscale - q (q may be null); x = 0 if zero_guess; d = z = r / diag;
// rz, rr, bb, tol2, done, hist[0].
template <typename TB, typename TV>
void launch_cg_init(CGState* st, double* partials, const TB* b, double bscale, const TV* q,
                    const TV* diag, TV* x, TV* r, TV* d, int zero_guess, double rel_tol,
                    double* hist, int64_t n, hipStream_t s);
// alpha = rz / (d . q); breakdown if d . q <= 0 or non-finite
template <typename TV>
void launch_cg_dot(CGState* st, double* partials, const TV* d, const TV* q, int64_t n,
                   hipStream_t s);
// x += alpha d; r -= alpha q; z = r / diag; rz, rr, beta, iter, hist, convergence
template <typename TV>
void launch_cg_update(CGState* st, double* partials, TV* x, TV* r, const TV* d, const TV* q,
                      const TV* diag, double* hist, int64_t n, hipStream_t s);
// d = r / diag + beta d
template <typename TV>
void launch_cg_direction(CGState* st, const TV* r, const TV* diag, TV* d, int64_t n,
                         hipStream_t s);
// Flexible CG (done = 3: the preconditioner returned r.z <= 0)
void launch_fcg_init(CGState* st, double* partials, const double* b, const double* q, double* x,
                     double* r, int zero_guess, double rel_tol, double* hist, int64_t n,
                     hipStream_t s);
void launch_fcg_start(CGState* st, double* partials, const double* r, const double* z, double* p,
                      int64_t n, hipStream_t s);
void launch_fcg_update(CGState* st, double* partials, double* x, double* r, const double* p,
                       const double* q, double* hist, int64_t n, hipStream_t s);
void launch_fcg_beta(CGState* st, double* partials, const double* r, const double* z,
                     const double* zold, int64_t n, hipStream_t s);
void launch_fcg_direction(CGState* st, const double* z, double* p, int64_t n, hipStream_t s);
// res2 = ||b - q||^2 and, if r is not null, r = b - q (always runs, ignores `done`)
void launch_residual(CGState* st, double* partials, const double* b, const double* q, double* r,
                     int64_t n, hipStream_t s);
// x += scale * dx (f64 += f32)
void launch_ir_correct(double* x, const float* dx, double scale, int64_t n, hipStream_t s);
// dst = convert(src) to f32 or bf16 (round to nearest even)
void launch_convert(const double* src, void* dst, int dtype, int64_t n, hipStream_t s);

}  // namespace pafem
