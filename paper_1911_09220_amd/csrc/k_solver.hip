// Vector kernels of the preconditioned CG solver ("Scalable Linear Solvers":
// CG on the partially assembled operator; the paper notes that Krylov solvers
// run on the device because they are written with Vector operations, "GPU
// Acceleration").
//
// Each kernel is a fixed grid of kCGBlocks x kCGThreads threads (one workgroup per
// compute unit, so the last-block ticket sees few same-address atomics) striding over
// the vectors.  Dot products: wave64 butterfly -> per-wave LDS -> per-block
// partial; the last block to arrive (atomic ticket) sums the partials in index
// order and updates the scalars, so results do not depend on scheduling.
#include <cmath>

#include "device.hpp"
#include "internal.hpp"
#include "solver.hpp"

namespace pafem {

namespace {

__device__ __forceinline__ bool state_done(const CGState* st) {
  return __hip_atomic_load(const_cast<int32_t*>(&st->done), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// grid-stride loop, unrolled so each thread keeps several independent loads in flight
#define GRID_LOOP(i, n)                                                        \
  _Pragma("unroll 4")                                                          \
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < (n);    \
       i += int64_t(gridDim.x) * blockDim.x)

__global__ void cg_reset_kernel(CGState* st, int32_t max_hist) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->rz = st->alpha = st->beta = st->rr = st->bb = st->tol2 = st->res2 = 0.0;
    st->iter = 0;
    st->done = 0;
    st->max_hist = max_hist;
    for (int i = 0; i < 8; ++i) st->ticket[i] = 0u;
  }
}

template <typename TB, typename TV>
__global__ void __launch_bounds__(kCGThreads)
    cg_init_kernel(CGState* st, double* partials, const TB* __restrict__ b, double bscale,
                   const TV* __restrict__ q, const TV* __restrict__ diag, TV* __restrict__ x,
                   TV* __restrict__ r, TV* __restrict__ d, int zero_guess, double rel_tol,
                   double* hist, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double rz = 0.0, rr = 0.0, bb = 0.0;
  GRID_LOOP(i, n) {
    const double bi = double(b[i]) * bscale;
    const TV ri = TV(q ? bi - double(q[i]) : bi);
    if (zero_guess) x[i] = TV(0);
    const TV zi = diag ? ri / diag[i] : ri;
    r[i] = ri;
    d[i] = zi;
    rz += double(ri) * double(zi);
    rr += double(ri) * double(ri);
    bb += bi * bi;
  }
  double* p0 = partials;
  double* p1 = partials + kCGBlocks;
  double* p2 = partials + 2 * kCGBlocks;
  rz = block_sum(rz, scratch);
  rr = block_sum(rr, scratch);
  bb = block_sum(bb, scratch);
  if (threadIdx.x == 0) {
    store_partial(p0, rz);
    store_partial(p1, rr);
    store_partial(p2, bb);
  }
  if (!arrive_last(&st->ticket[0])) return;
  const double trz = sum_partials(p0, scratch);
  const double trr = sum_partials(p1, scratch);
  const double tbb = sum_partials(p2, scratch);
  if (threadIdx.x == 0) {
    st->rz = trz;
    st->rr = trr;
    // reference of the relative stop: ||b||^2, or ||r_0||^2 when b = 0 (the answer is
    // then x = 0 and the iteration reduces the initial residual; both 0: done)
    const double ref = tbb > 0.0 ? tbb : trr;
    st->bb = ref;
    st->tol2 = rel_tol * rel_tol * ref;
    st->iter = 0;
    st->alpha = st->beta = 0.0;
    st->res2 = 0.0;
    const int conv = trr <= st->tol2;
    if (hist && st->max_hist > 0) hist[0] = ref > 0.0 ? sqrt(trr / ref) : 0.0;
    __hip_atomic_store(&st->done, conv ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// alpha = rz / (d . q) with d . q assembled from the apply's per-workgroup element
// energies plus, for a constrained operator, the essential rows (q_b = d_b there):
// d . q = sum(epart) + sum over essential b of d_b^2.  The mask is read eight
// entries at a time; entries at or beyond n are never used.
template <typename TV>
__global__ void __launch_bounds__(kCGThreads)
    cg_alpha_kernel(CGState* st, double* partials, const double* __restrict__ epart,
                    int nepart, const uint8_t* __restrict__ bmask, const TV* __restrict__ d,
                    int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  const int64_t tid = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t nthr = int64_t(gridDim.x) * blockDim.x;
  double s = 0.0;
  for (int64_t i = tid; i < nepart; i += nthr) s += epart[i];
  if (bmask) {
    const int64_t nw = n / 8;
    const uint64_t* mw = reinterpret_cast<const uint64_t*>(bmask);
    for (int64_t w = tid; w < nw; w += nthr) {
      uint64_t m = mw[w];
      while (m) {
        const int b = __builtin_ctzll(m) >> 3;
        const double v = double(d[w * 8 + b]);
        s += v * v;
        m &= ~(uint64_t(0xff) << (8 * b));
      }
    }
    for (int64_t i = nw * 8 + tid; i < n; i += nthr)
      if (bmask[i]) {
        const double v = double(d[i]);
        s += v * v;
      }
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) store_partial(partials, s);
  if (!arrive_last(&st->ticket[1])) return;
  const double pq = sum_partials(partials, scratch);
  if (threadIdx.x == 0) {
    const double alpha = st->rz / pq;
    if (!(pq > 0.0) || !isfinite(alpha))
      __hip_atomic_store(&st->done, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st->alpha = alpha;
    __hip_atomic_store(&st->ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename TV>
__global__ void __launch_bounds__(kCGThreads)
    cg_update_kernel(CGState* st, double* partials, TV* __restrict__ x, TV* __restrict__ r,
                     const TV* __restrict__ d, const TV* __restrict__ q,
                     const TV* __restrict__ diag, double* hist, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  const TV alpha = TV(st->alpha);
  double rz = 0.0, rr = 0.0;
  GRID_LOOP(i, n) {
    const TV di = d[i];
    x[i] += alpha * di;
    const TV ri = r[i] - alpha * q[i];
    r[i] = ri;
    const TV zi = diag ? ri / diag[i] : ri;
    rz += double(ri) * double(zi);
    rr += double(ri) * double(ri);
  }
  double* p0 = partials;
  double* p1 = partials + kCGBlocks;
  rz = block_sum(rz, scratch);
  rr = block_sum(rr, scratch);
  if (threadIdx.x == 0) {
    store_partial(p0, rz);
    store_partial(p1, rr);
  }
  if (!arrive_last(&st->ticket[2])) return;
  const double trz = sum_partials(p0, scratch);
  const double trr = sum_partials(p1, scratch);
  if (threadIdx.x == 0) {
    const double beta = trz / st->rz;
    st->beta = beta;
    st->rz = trz;
    st->rr = trr;
    const int it = st->iter + 1;
    st->iter = it;
    if (hist && it < st->max_hist) hist[it] = sqrt(trr / st->bb);
    int done = 0;
    if (!isfinite(trr) || !isfinite(beta)) done = 2;
    else if (trr <= st->tol2) done = 1;
    if (done) __hip_atomic_store(&st->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename TV>
__global__ void __launch_bounds__(kCGThreads)
    cg_direction_kernel(const CGState* st, const TV* __restrict__ r,
                        const TV* __restrict__ diag, TV* __restrict__ d, int64_t n) {
  if (state_done(st)) return;
  const TV beta = TV(st->beta);
  GRID_LOOP(i, n) {
    const TV zi = diag ? r[i] / diag[i] : r[i];
    d[i] = zi + beta * d[i];
  }
}

// d = r / diag + beta d, and q = the next apply's init: d on essential dofs of a
// constrained operator (bmask non-null), 0 elsewhere
__global__ void __launch_bounds__(kCGThreads)
    cg_direction_init_kernel(const CGState* st, const double* __restrict__ r,
                             const double* __restrict__ diag, double* __restrict__ d,
                             double* __restrict__ q, const uint8_t* __restrict__ bmask,
                             int64_t n) {
  if (state_done(st)) return;
  const double beta = st->beta;
  GRID_LOOP(i, n) {
    const double zi = diag ? r[i] / diag[i] : r[i];
    const double di = zi + beta * d[i];
    d[i] = di;
    q[i] = (bmask && bmask[i]) ? di : 0.0;
  }
}

// ---- flexible CG (variable preconditioner) ----
// r = b - q (q may be null), x = 0 if zero_guess; rr, bb, tol2; iteration count kept
__global__ void __launch_bounds__(kCGThreads)
    fcg_init_kernel(CGState* st, double* partials, const double* __restrict__ b,
                    const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
                    int zero_guess, double rel_tol, double* hist, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double rr = 0.0, bb = 0.0;
  GRID_LOOP(i, n) {
    const double bi = b[i];
    const double ri = q ? bi - q[i] : bi;
    if (zero_guess) x[i] = 0.0;
    r[i] = ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  rr = block_sum(rr, scratch);
  bb = block_sum(bb, scratch);
  if (threadIdx.x == 0) {
    store_partial(partials, rr);
    store_partial(partials + kCGBlocks, bb);
  }
  if (!arrive_last(&st->ticket[0])) return;
  const double trr = sum_partials(partials, scratch);
  const double tbb = sum_partials(partials + kCGBlocks, scratch);
  if (threadIdx.x == 0) {
    st->rr = trr;
    const double ref = tbb > 0.0 ? tbb : trr;  // as in cg_init_kernel
    st->bb = ref;
    st->tol2 = rel_tol * rel_tol * ref;
    const int conv = trr <= st->tol2;
    if (hist && st->max_hist > 0) hist[0] = ref > 0.0 ? sqrt(trr / ref) : 0.0;
    __hip_atomic_store(&st->done, conv ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// rz = r . z (must be > 0: otherwise done = 3, the preconditioner is not positive); p = z
__global__ void __launch_bounds__(kCGThreads)
    fcg_start_kernel(CGState* st, double* partials, const double* __restrict__ r,
                     const double* __restrict__ z, double* __restrict__ p, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  double rz = 0.0;
  GRID_LOOP(i, n) {
    const double zi = z[i];
    p[i] = zi;
    rz += r[i] * zi;
  }
  rz = block_sum(rz, scratch);
  if (threadIdx.x == 0) store_partial(partials, rz);
  if (!arrive_last(&st->ticket[4])) return;
  const double t = sum_partials(partials, scratch);
  if (threadIdx.x == 0) {
    st->rz = t;
    if (!(t > 0.0) || !isfinite(t))
      __hip_atomic_store(&st->done, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[4], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// x += alpha p; r -= alpha q; zj = r / diag (0 on essential dofs: the Jacobi part of
// the next preconditioned residual); rr, iteration count, history, convergence
__global__ void __launch_bounds__(kCGThreads)
    fcg_update_kernel(CGState* st, double* partials, double* __restrict__ x,
                      double* __restrict__ r, const double* __restrict__ p,
                      const double* __restrict__ q, const double* __restrict__ diag,
                      const uint8_t* __restrict__ bmask, double* __restrict__ zj, double* hist,
                      int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  const double alpha = st->alpha;
  double rr = 0.0;
  GRID_LOOP(i, n) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    zj[i] = (bmask && bmask[i]) ? ri : ri / diag[i];
    rr += ri * ri;
  }
  rr = block_sum(rr, scratch);
  if (threadIdx.x == 0) store_partial(partials, rr);
  if (!arrive_last(&st->ticket[2])) return;
  const double t = sum_partials(partials, scratch);
  if (threadIdx.x == 0) {
    st->rr = t;
    const int it = st->iter + 1;
    st->iter = it;
    if (hist && it < st->max_hist) hist[it] = sqrt(t / st->bb);
    int done = 0;
    if (!isfinite(t)) done = 2;
    else if (t <= st->tol2) done = 1;
    if (done) __hip_atomic_store(&st->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// beta = r.(z - z_old) / rz_old (Polak-Ribiere); rz = r.z (> 0 else done = 3)
__global__ void __launch_bounds__(kCGThreads)
    fcg_beta_kernel(CGState* st, double* partials, const double* __restrict__ r,
                    const double* __restrict__ z, const double* __restrict__ zold, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  double rz = 0.0, rzo = 0.0;
  GRID_LOOP(i, n) {
    const double ri = r[i];
    rz += ri * z[i];
    rzo += ri * zold[i];
  }
  rz = block_sum(rz, scratch);
  rzo = block_sum(rzo, scratch);
  if (threadIdx.x == 0) {
    store_partial(partials, rz);
    store_partial(partials + kCGBlocks, rzo);
  }
  if (!arrive_last(&st->ticket[5])) return;
  const double trz = sum_partials(partials, scratch);
  const double trzo = sum_partials(partials + kCGBlocks, scratch);
  if (threadIdx.x == 0) {
    st->beta = (trz - trzo) / st->rz;
    st->rz = trz;
    if (!(trz > 0.0) || !isfinite(st->beta))
      __hip_atomic_store(&st->done, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[5], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// p = z + beta p
__global__ void __launch_bounds__(kCGThreads)
    fcg_direction_kernel(const CGState* st, const double* __restrict__ z, double* __restrict__ p,
                         int64_t n) {
  if (state_done(st)) return;
  const double beta = st->beta;
  GRID_LOOP(i, n) p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kCGThreads)
    residual_kernel(CGState* st, double* partials, const double* __restrict__ b,
                    const double* __restrict__ q, double* __restrict__ r, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double s = 0.0;
  GRID_LOOP(i, n) {
    const double v = b[i] - q[i];
    if (r) r[i] = v;
    s += v * v;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) store_partial(partials, s);
  if (!arrive_last(&st->ticket[3])) return;
  const double t = sum_partials(partials, scratch);
  if (threadIdx.x == 0) {
    st->res2 = t;
    __hip_atomic_store(&st->ticket[3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}


// ---- inner PCG of iterative refinement --------------------------------------
// The inner solve of A_lo d = r / s keeps its residual r, the preconditioned
// residual z, all dot products and the solution x in FP64 (x += s alpha d
// directly, so the FP64 residual b - A x that replaces r carries no rounding of
// an intermediate correction); only what the reduced-precision apply reads and
// writes is FP32: the direction d and its image q = A_lo d.  dinv is the Jacobi
// preconditioner 1/diag rounded to FP32 (a preconditioner, not part of the
// answer); null for none.  Essential rows: q_b = d_b for a constrained operator.

__device__ __forceinline__ double ir_z(const double* r, const float* dinv, int64_t i) {
  return dinv ? r[i] * double(dinv[i]) : r[i];
}

// r *= inv_s (r holds the FP64 residual), d = z, q = apply init of d;
// rz, rr, bb = rr, tol2 = inner_rel_tol^2 rr, iter = 0, done
__global__ void __launch_bounds__(kCGThreads)
    ir_start_kernel(CGState* st, double* partials, double* __restrict__ r, double inv_s,
                    const float* __restrict__ dinv, float* __restrict__ d, float* __restrict__ q,
                    const uint8_t* __restrict__ ess, double inner_rel_tol, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double rz = 0.0, rr = 0.0;
  GRID_LOOP(i, n) {
    const double ri = r[i] * inv_s;
    r[i] = ri;
    const double zi = dinv ? ri * double(dinv[i]) : ri;
    const float di = float(zi);
    d[i] = di;
    q[i] = (ess && ess[i]) ? di : 0.0f;
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = block_sum(rz, scratch);
  rr = block_sum(rr, scratch);
  if (threadIdx.x == 0) {
    store_partial(partials, rz);
    store_partial(partials + kCGBlocks, rr);
  }
  if (!arrive_last(&st->ticket[0])) return;
  const double trz = sum_partials(partials, scratch);
  const double trr = sum_partials(partials + kCGBlocks, scratch);
  if (threadIdx.x == 0) {
    st->rz = trz;
    st->rr = trr;
    st->bb = trr;
    st->tol2 = inner_rel_tol * inner_rel_tol * trr;
    st->iter = 0;
    st->alpha = st->beta = 0.0;
    const int done = trr > 0.0 ? 0 : 1;
    __hip_atomic_store(&st->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// x += (s alpha) d; r -= alpha q (FP64); rz, rr, beta = rz / rz_old, iter, convergence
__global__ void __launch_bounds__(kCGThreads)
    ir_update_kernel(CGState* st, double* partials, double* __restrict__ x, double s,
                     double* __restrict__ r, const float* __restrict__ d,
                     const float* __restrict__ q, const float* __restrict__ dinv, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  const double alpha = st->alpha;
  const double xstep = s * alpha;
  double rz = 0.0, rr = 0.0;
  GRID_LOOP(i, n) {
    x[i] += xstep * double(d[i]);
    const double ri = r[i] - alpha * double(q[i]);
    r[i] = ri;
    const double zi = dinv ? ri * double(dinv[i]) : ri;
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = block_sum(rz, scratch);
  rr = block_sum(rr, scratch);
  if (threadIdx.x == 0) {
    store_partial(partials, rz);
    store_partial(partials + kCGBlocks, rr);
  }
  if (!arrive_last(&st->ticket[2])) return;
  const double trz = sum_partials(partials, scratch);
  const double trr = sum_partials(partials + kCGBlocks, scratch);
  if (threadIdx.x == 0) {
    const double beta = trz / st->rz;
    st->beta = beta;
    st->rz = trz;
    st->rr = trr;
    st->iter = st->iter + 1;
    int done = 0;
    if (!isfinite(trr) || !isfinite(beta)) done = 2;
    else if (trr <= st->tol2) done = 1;
    if (done) __hip_atomic_store(&st->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// d = z + beta d (stored FP32), q = apply init of the new d
__global__ void __launch_bounds__(kCGThreads)
    ir_direction_kernel(const CGState* st, const double* __restrict__ r,
                        const float* __restrict__ dinv, float* __restrict__ d,
                        float* __restrict__ q, const uint8_t* __restrict__ ess, int64_t n) {
  if (state_done(st)) return;
  const double beta = st->beta;
  GRID_LOOP(i, n) {
    const float di = float(ir_z(r, dinv, i) + beta * double(d[i]));
    d[i] = di;
    q[i] = (ess && ess[i]) ? di : 0.0f;
  }
}

// Residual replacement: r holds the FP64 residual b - A_hi x; scale it by 1/s_new
// and continue the recurrence with the kept direction d.  The next
// direction d' = z + beta d is made A_lo-conjugate to d using q = A_lo d of the
// last step: beta = -(z . q) / (d . q).  Without rounding and operator mismatch this
// is the usual beta in the new scaling (times s_old / s_new for the kept direction);
// with a replaced residual it keeps at least the last direction conjugate.
__global__ void __launch_bounds__(kCGThreads)
    ir_replace_kernel(CGState* st, double* partials, double* __restrict__ r, double inv_s_new,
                      const float* __restrict__ dinv, const float* __restrict__ d,
                      const float* __restrict__ q, double inner_rel_tol, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double rz = 0.0, rr = 0.0, zq = 0.0, dq = 0.0;
  GRID_LOOP(i, n) {
    const double ri = r[i] * inv_s_new;
    r[i] = ri;
    const double zi = dinv ? ri * double(dinv[i]) : ri;
    const double qi = double(q[i]);
    rz += ri * zi;
    rr += ri * ri;
    zq += zi * qi;
    dq += double(d[i]) * qi;
  }
  rz = block_sum(rz, scratch);
  rr = block_sum(rr, scratch);
  zq = block_sum(zq, scratch);
  dq = block_sum(dq, scratch);
  if (threadIdx.x == 0) {
    store_partial(partials, rz);
    store_partial(partials + kCGBlocks, rr);
    store_partial(partials + 2 * kCGBlocks, zq);
    store_partial(partials + 3 * kCGBlocks, dq);
  }
  if (!arrive_last(&st->ticket[6])) return;
  const double trz = sum_partials(partials, scratch);
  const double trr = sum_partials(partials + kCGBlocks, scratch);
  const double tzq = sum_partials(partials + 2 * kCGBlocks, scratch);
  const double tdq = sum_partials(partials + 3 * kCGBlocks, scratch);
  if (threadIdx.x == 0) {
    const double beta = -tzq / tdq;
    st->beta = beta;
    st->rz = trz;
    st->rr = trr;
    st->bb = trr;
    st->tol2 = inner_rel_tol * inner_rel_tol * trr;
    const int done = (isfinite(beta) && trz > 0.0 && tdq > 0.0) ? 0 : 2;
    __hip_atomic_store(&st->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[6], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// dinv = 1 / diag rounded to FP32
__global__ void __launch_bounds__(kCGThreads)
    ir_dinv_kernel(const double* __restrict__ diag, float* __restrict__ dinv, int64_t n) {
  GRID_LOOP(i, n) dinv[i] = float(1.0 / diag[i]);
}

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u)  // inf or nan
    return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  const uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);
  return uint16_t((u + rounding) >> 16);
}

__global__ void __launch_bounds__(kCGThreads)
    convert_kernel(const double* __restrict__ src, void* __restrict__ dst, int dtype, int64_t n) {
  GRID_LOOP(i, n) {
    const float f = float(src[i]);
    if (dtype == PAFEM_F32)
      static_cast<float*>(dst)[i] = f;
    else
      static_cast<uint16_t*>(dst)[i] = f32_to_bf16_bits(f);
  }
}

void check_launch(const char* what) {
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

int vec_grid(int64_t n) {
  int64_t g = (n + kCGThreads - 1) / kCGThreads;
  return int(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

void launch_cg_reset(CGState* st, int32_t max_hist, hipStream_t s) {
  hipLaunchKernelGGL(cg_reset_kernel, dim3(1), dim3(64), 0, s, st, max_hist);
  check_launch("cg_reset");
}

template <typename TB, typename TV>
void launch_cg_init(CGState* st, double* partials, const TB* b, double bscale, const TV* q,
                    const TV* diag, TV* x, TV* r, TV* d, int zero_guess, double rel_tol,
                    double* hist, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((cg_init_kernel<TB, TV>), dim3(kCGBlocks), dim3(kCGThreads), 0, s, st,
                     partials, b, bscale, q, diag, x, r, d, zero_guess, rel_tol, hist, n);
  check_launch("cg_init");
}

template <typename TV>
void launch_cg_alpha(CGState* st, double* partials, const double* epart, int nepart,
                     const uint8_t* bmask, const TV* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((cg_alpha_kernel<TV>), dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials,
                     epart, nepart, bmask, d, n);
  check_launch("cg_alpha");
}

template <typename TV>
void launch_cg_update(CGState* st, double* partials, TV* x, TV* r, const TV* d, const TV* q,
                      const TV* diag, double* hist, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((cg_update_kernel<TV>), dim3(kCGBlocks), dim3(kCGThreads), 0, s, st,
                     partials, x, r, d, q, diag, hist, n);
  check_launch("cg_update");
}

template <typename TV>
void launch_cg_direction(CGState* st, const TV* r, const TV* diag, TV* d, int64_t n,
                         hipStream_t s) {
  hipLaunchKernelGGL((cg_direction_kernel<TV>), dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, r,
                     diag, d, n);
  check_launch("cg_direction");
}

template void launch_cg_init<double, double>(CGState*, double*, const double*, double,
                                             const double*, const double*, double*, double*,
                                             double*, int, double, double*, int64_t, hipStream_t);
template void launch_cg_alpha<double>(CGState*, double*, const double*, int, const uint8_t*,
                                      const double*, int64_t, hipStream_t);
template void launch_cg_alpha<float>(CGState*, double*, const double*, int, const uint8_t*,
                                     const float*, int64_t, hipStream_t);
template void launch_cg_update<double>(CGState*, double*, double*, double*, const double*,
                                       const double*, const double*, double*, int64_t,
                                       hipStream_t);
template void launch_cg_direction<double>(CGState*, const double*, const double*, double*,
                                          int64_t, hipStream_t);

void launch_fcg_init(CGState* st, double* partials, const double* b, const double* q, double* x,
                     double* r, int zero_guess, double rel_tol, double* hist, int64_t n,
                     hipStream_t s) {
  hipLaunchKernelGGL(fcg_init_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, b, q,
                     x, r, zero_guess, rel_tol, hist, n);
  check_launch("fcg_init");
}
void launch_fcg_start(CGState* st, double* partials, const double* r, const double* z, double* p,
                      int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fcg_start_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, r, z,
                     p, n);
  check_launch("fcg_start");
}
void launch_fcg_update(CGState* st, double* partials, double* x, double* r, const double* p,
                       const double* q, const double* diag, const uint8_t* bmask, double* zj,
                       double* hist, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fcg_update_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, x,
                     r, p, q, diag, bmask, zj, hist, n);
  check_launch("fcg_update");
}
void launch_fcg_beta(CGState* st, double* partials, const double* r, const double* z,
                     const double* zold, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fcg_beta_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, r, z,
                     zold, n);
  check_launch("fcg_beta");
}
void launch_cg_direction_init(CGState* st, const double* r, const double* diag, double* d,
                              double* q, const uint8_t* bmask, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cg_direction_init_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, r,
                     diag, d, q, bmask, n);
  check_launch("cg_direction_init");
}

void launch_fcg_direction(CGState* st, const double* z, double* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fcg_direction_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, z, p, n);
  check_launch("fcg_direction");
}

void launch_residual(CGState* st, double* partials, const double* b, const double* q, double* r,
                     int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(residual_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, b, q,
                     r, n);
  check_launch("residual");
}


void launch_ir_start(CGState* st, double* partials, double* r, double s, const float* dinv,
                     float* d, float* q, const uint8_t* ess, double inner_rel_tol, int64_t n,
                     hipStream_t stream) {
  hipLaunchKernelGGL(ir_start_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, stream, st, partials,
                     r, 1.0 / s, dinv, d, q, ess, inner_rel_tol, n);
  check_launch("ir_start");
}

void launch_ir_update(CGState* st, double* partials, double* x, double s, double* r,
                      const float* d, const float* q, const float* dinv, int64_t n,
                      hipStream_t stream) {
  hipLaunchKernelGGL(ir_update_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, stream, st,
                     partials, x, s, r, d, q, dinv, n);
  check_launch("ir_update");
}

void launch_ir_direction(CGState* st, const double* r, const float* dinv, float* d, float* q,
                         const uint8_t* ess, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(ir_direction_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, stream, st, r,
                     dinv, d, q, ess, n);
  check_launch("ir_direction");
}

void launch_ir_replace(CGState* st, double* partials, double* r, double s_new, const float* dinv,
                       const float* d, const float* q, double inner_rel_tol, int64_t n,
                       hipStream_t stream) {
  hipLaunchKernelGGL(ir_replace_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, stream, st,
                     partials, r, 1.0 / s_new, dinv, d, q, inner_rel_tol, n);
  check_launch("ir_replace");
}

void launch_ir_dinv(const double* diag, float* dinv, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(ir_dinv_kernel, dim3(vec_grid(n)), dim3(kCGThreads), 0, stream, diag, dinv,
                     n);
  check_launch("ir_dinv");
}

void launch_convert(const double* src, void* dst, int dtype, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(convert_kernel, dim3(vec_grid(n)), dim3(kCGThreads), 0, s, src, dst, dtype,
                     n);
  check_launch("convert");
}

}  // namespace pafem
