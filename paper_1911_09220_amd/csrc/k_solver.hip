// Vector kernels of the preconditioned CG solver ("Scalable Linear Solvers":
// CG on the partially assembled operator; the paper notes that Krylov solvers
// run on the device because they are written with Vector operations, "GPU
// Acceleration").
//
// Each kernel is a fixed grid of kCGBlocks x kCGThreads threads striding over
// the vectors.  Dot products: wave64 butterfly -> per-wave LDS -> per-block
// partial; the last block to arrive (atomic ticket) sums the partials in index
// order and updates the scalars, so results do not depend on scheduling.
#include <cmath>

#include "device.hpp"
#include "internal.hpp"
#include "solver.hpp"

namespace pafem {

namespace {

__device__ __forceinline__ void store_partial(double* partials, double v) {
  __hip_atomic_store(&partials[blockIdx.x], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_partial(const double* partials, int i) {
  return __hip_atomic_load(const_cast<double*>(&partials[i]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes this block's partials (thread 0 already stored them) and returns true in
// every thread of the last block to arrive.
__device__ bool arrive_last(uint32_t* ticket) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

// Sum of partials[0..gridDim.x) in a fixed order, valid in every thread.
__device__ double sum_partials(const double* partials, double* scratch) {
  double v = 0.0;
  for (int i = threadIdx.x; i < int(gridDim.x); i += blockDim.x) v += load_partial(partials, i);
  return block_sum(v, scratch);
}

__device__ __forceinline__ bool state_done(const CGState* st) {
  return __hip_atomic_load(const_cast<int32_t*>(&st->done), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT) != 0;
}

#define GRID_LOOP(i, n)                                                        \
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

__global__ void __launch_bounds__(kCGThreads)
    cg_init_kernel(CGState* st, double* partials, const double* __restrict__ b,
                   const double* __restrict__ q, const double* __restrict__ diag,
                   double* __restrict__ x, double* __restrict__ r, double* __restrict__ d,
                   int zero_guess, double rel_tol, double* hist, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double rz = 0.0, rr = 0.0, bb = 0.0;
  GRID_LOOP(i, n) {
    const double bi = b[i];
    const double ri = q ? bi - q[i] : bi;
    if (zero_guess) x[i] = 0.0;
    const double zi = diag ? ri / diag[i] : ri;
    r[i] = ri;
    d[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
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
    st->bb = tbb;
    st->tol2 = rel_tol * rel_tol * tbb;
    st->iter = 0;
    st->alpha = st->beta = 0.0;
    st->res2 = 0.0;
    const int conv = (trr <= st->tol2) || (tbb == 0.0);
    if (hist && st->max_hist > 0) hist[0] = tbb > 0.0 ? sqrt(trr / tbb) : 0.0;
    __hip_atomic_store(&st->done, conv ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void __launch_bounds__(kCGThreads)
    cg_dot_kernel(CGState* st, double* partials, const double* __restrict__ d,
                  const double* __restrict__ q, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  double s = 0.0;
  GRID_LOOP(i, n) s += d[i] * q[i];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) store_partial(partials, s);
  if (!arrive_last(&st->ticket[1])) return;
  const double pq = sum_partials(partials, scratch);
  if (threadIdx.x == 0) {
    const double alpha = st->rz / pq;
    if (!(pq > 0.0) || !isfinite(alpha)) {
      __hip_atomic_store(&st->done, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    st->alpha = alpha;
    __hip_atomic_store(&st->ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void __launch_bounds__(kCGThreads)
    cg_update_kernel(CGState* st, double* partials, double* __restrict__ x,
                     double* __restrict__ r, const double* __restrict__ d,
                     const double* __restrict__ q, const double* __restrict__ diag,
                     double* hist, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  if (state_done(st)) return;
  const double alpha = st->alpha;
  double rz = 0.0, rr = 0.0;
  GRID_LOOP(i, n) {
    const double di = d[i];
    x[i] += alpha * di;
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    const double zi = diag ? ri / diag[i] : ri;
    rz += ri * zi;
    rr += ri * ri;
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

__global__ void __launch_bounds__(kCGThreads)
    cg_direction_kernel(const CGState* st, const double* __restrict__ r,
                        const double* __restrict__ diag, double* __restrict__ d, int64_t n) {
  if (state_done(st)) return;
  const double beta = st->beta;
  GRID_LOOP(i, n) {
    const double zi = diag ? r[i] / diag[i] : r[i];
    d[i] = zi + beta * d[i];
  }
}

__global__ void __launch_bounds__(kCGThreads)
    residual_norm_kernel(CGState* st, double* partials, const double* __restrict__ b,
                         const double* __restrict__ q, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double s = 0.0;
  GRID_LOOP(i, n) {
    const double v = b[i] - q[i];
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

void check_launch(const char* what) {
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

}  // namespace

void launch_cg_reset(CGState* st, int32_t max_hist, hipStream_t s) {
  hipLaunchKernelGGL(cg_reset_kernel, dim3(1), dim3(64), 0, s, st, max_hist);
  check_launch("cg_reset");
}

void launch_cg_init(CGState* st, double* partials, const double* b, const double* q,
                    const double* diag, double* x, double* r, double* d, int zero_guess,
                    double rel_tol, double* hist, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cg_init_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, b, q,
                     diag, x, r, d, zero_guess, rel_tol, hist, n);
  check_launch("cg_init");
}

void launch_cg_dot(CGState* st, double* partials, const double* d, const double* q, int64_t n,
                   hipStream_t s) {
  hipLaunchKernelGGL(cg_dot_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, d, q,
                     n);
  check_launch("cg_dot");
}

void launch_cg_update(CGState* st, double* partials, double* x, double* r, const double* d,
                      const double* q, const double* diag, double* hist, int64_t n,
                      hipStream_t s) {
  hipLaunchKernelGGL(cg_update_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials, x,
                     r, d, q, diag, hist, n);
  check_launch("cg_update");
}

void launch_cg_direction(CGState* st, const double* r, const double* diag, double* d, int64_t n,
                         hipStream_t s) {
  hipLaunchKernelGGL(cg_direction_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, r, diag, d,
                     n);
  check_launch("cg_direction");
}

void launch_residual_norm(CGState* st, double* partials, const double* b, const double* q,
                          int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(residual_norm_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, s, st, partials,
                     b, q, n);
  check_launch("residual_norm");
}

}  // namespace pafem
