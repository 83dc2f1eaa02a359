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
  int32_t done;  // 0 running, 1 converged, 2 breakdown, 3 preconditioner not positive
  int32_t max_hist;
  int32_t pad1;
  uint32_t ticket[8];  // arrival counters of the last-block reductions
};

constexpr int kCGBlocks = 256;  // fixed grid of the vector kernels = number of partials
constexpr int kCGThreads = 1024;

// zero the state and tickets; hist holds max_hist entries
void launch_cg_reset(CGState* st, int32_t max_hist, hipStream_t s);

// The iteration kernels are templated on the vector type TV (double is built);
// dot products always accumulate in double.
//
// r = b*bscale - q (q may be null); x = 0 if zero_guess; d = z = r / diag;
// rz, rr, bb, tol2, done, hist[0].
template <typename TB, typename TV>
void launch_cg_init(CGState* st, double* partials, const TB* b, double bscale, const TV* q,
                    const TV* diag, TV* x, TV* r, TV* d, int zero_guess, double rel_tol,
                    double* hist, int64_t n, hipStream_t s);
// alpha = rz / (d . q) from the apply's element-energy partials (epart, nepart of
// them) plus sum of d_b^2 over the essential dofs (bmask; null for an unconstrained
// operator); breakdown (done = 2) if d . q <= 0 or alpha is not finite
template <typename TV>
void launch_cg_alpha(CGState* st, double* partials, const double* epart, int nepart,
                     const uint8_t* bmask, const TV* d, int64_t n, hipStream_t s);
// x += alpha d; r -= alpha q; z = r / diag; rz, rr, beta, iter, hist, convergence
template <typename TV>
void launch_cg_update(CGState* st, double* partials, TV* x, TV* r, const TV* d, const TV* q,
                      const TV* diag, double* hist, int64_t n, hipStream_t s);
// d = r / diag + beta d
template <typename TV>
void launch_cg_direction(CGState* st, const TV* r, const TV* diag, TV* d, int64_t n,
                         hipStream_t s);
// d = r / diag + beta d (FP64) and q = the apply init of the new d (d on the
// essential dofs given by bmask, 0 elsewhere; bmask null: 0 everywhere)
void launch_cg_direction_init(CGState* st, const double* r, const double* diag, double* d,
                              double* q, const uint8_t* bmask, int64_t n, hipStream_t s);
// Flexible CG (done = 3: the preconditioner returned r.z <= 0)
void launch_fcg_init(CGState* st, double* partials, const double* b, const double* q, double* x,
                     double* r, int zero_guess, double rel_tol, double* hist, int64_t n,
                     hipStream_t s);
void launch_fcg_start(CGState* st, double* partials, const double* r, const double* z, double* p,
                      int64_t n, hipStream_t s);
// x += alpha p; r -= alpha q; zj = r / diag, and zj = r where bmask (may be null) marks
// the essential rows of a constrained operator (unit diagonal there): the Jacobi part
// of the next preconditioned residual
void launch_fcg_update(CGState* st, double* partials, double* x, double* r, const double* p,
                       const double* q, const double* diag, const uint8_t* bmask, double* zj,
                       double* hist, int64_t n, hipStream_t s);
void launch_fcg_beta(CGState* st, double* partials, const double* r, const double* z,
                     const double* zold, int64_t n, hipStream_t s);
void launch_fcg_direction(CGState* st, const double* z, double* p, int64_t n, hipStream_t s);
// res2 = ||b - q||^2 and, if r is not null, r = b - q (always runs, ignores `done`)
void launch_residual(CGState* st, double* partials, const double* b, const double* q, double* r,
                     int64_t n, hipStream_t s);
// Inner PCG of iterative refinement: residual, preconditioned residual, dots and the
// solution x in FP64; direction d and its image q = A_lo d in FP32; dinv = 1/diag in
// FP32 (null: no preconditioner); ess = essential mask of a constrained operator
// (q_b = d_b) or null.  Every kernel that sets the next direction also writes q's
// apply init, so the apply runs without its own init pass.
// r (FP64 residual) *= 1/s; d = z; state restarted with tol2 = tol^2 rr
void launch_ir_start(CGState* st, double* partials, double* r, double s, const float* dinv,
                     float* d, float* q, const uint8_t* ess, double inner_rel_tol, int64_t n,
                     hipStream_t stream);
// x += (s alpha) d; r -= alpha q; rz, rr, beta, iter, convergence
void launch_ir_update(CGState* st, double* partials, double* x, double s, double* r,
                      const float* d, const float* q, const float* dinv, int64_t n,
                      hipStream_t stream);
// d = z + beta d; q = apply init of d
void launch_ir_direction(CGState* st, const double* r, const float* dinv, float* d, float* q,
                         const uint8_t* ess, int64_t n, hipStream_t stream);
// Reliable update after a residual replacement: r (the FP64 residual) *= 1/s_new,
// beta = -(z.q)/(d.q) so that launch_ir_direction continues with a direction
// conjugate to the kept one (done = 2 on breakdown).  partials: 4 * kCGBlocks.
void launch_ir_replace(CGState* st, double* partials, double* r, double s_new, const float* dinv,
                       const float* d, const float* q, double inner_rel_tol, int64_t n,
                       hipStream_t stream);
// dinv = 1/diag rounded to FP32
void launch_ir_dinv(const double* diag, float* dinv, int64_t n, hipStream_t stream);
// dst = convert(src) to f32 or bf16 (round to nearest even)
void launch_convert(const double* src, void* dst, int dtype, int64_t n, hipStream_t s);

}  // namespace pafem
