// Kernels of the order (p-) multigrid preconditioner ("Scalable Linear Solvers":
// matrix-free preconditioning of partially assembled operators by multigrid in the
// polynomial order).
//
// * Transfers between two H1 spaces of one mesh: both spaces share the device element
//   order (a Morton order of the mesh's elements), so element k of one is element k of
//   the other.  Prolongation evaluates the coarse function at the fine nodes of each
//   element by three one-axis contractions with the 1D table I[xf][xc] = phi^c_xc at
//   fine node xf; each fine dof is written by one element only, its owner (the first
//   entry of its transposed-map list).  Restriction is the exact transpose: every fine
//   value enters once (through its owner), contracted with I^T, and added into the
//   coarse vector with one atomic per element node.
// * Chebyshev-Jacobi smoothing and power-iteration vector kernels.
#include <cmath>

#include "device.hpp"
#include "internal.hpp"
#include "mg.hpp"
#include "solver.hpp"

namespace pafem {

namespace {

constexpr int kMgThreads = 256;
constexpr int kMgLdsDoubles = 4096;  // 32 KB of LDS per workgroup

#define GRID_LOOP(i, n)                                                     \
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < (n); \
       i += int64_t(gridDim.x) * blockDim.x)

struct TransferArgs {
  const int32_t* gmap_c;  // coarse element->dof map (~g on essential dofs)
  const int32_t* gmap_f;  // fine element->dof map
  const int32_t* toff_f;  // fine transposed-map offsets
  const int32_t* tidx_f;  // fine transposed-map entries (element-vector positions, ascending)
  int64_t ne;
  int dc, df;             // 1D nodes of the coarse / fine order
  int nel;                // elements per workgroup
};

// true if element-vector position `pos` is the first occurrence of dof g
__device__ __forceinline__ bool owns(const TransferArgs& a, int32_t g, int64_t pos) {
  return int64_t(a.tidx_f[a.toff_f[g]]) == pos;
}

__global__ void __launch_bounds__(kMgThreads)
    prolong_kernel(TransferArgs a, Interp1D I, const double* __restrict__ xc,
                   double* __restrict__ out, int add) {
  extern __shared__ double lds[];
  const int dc = a.dc, df = a.df;
  const int dc3 = dc * dc * dc, df3 = df * df * df;
  const int64_t e0 = int64_t(blockIdx.x) * a.nel;
  const int nel = int(min(int64_t(a.nel), a.ne - e0));
  double* u = lds;                          // [nel][dc][dc][dc]
  double* t1 = u + a.nel * dc3;             // [nel][zc][yc][xf]
  double* t2 = t1 + a.nel * dc * dc * df;   // [nel][zc][yf][xf]
  for (int i = threadIdx.x; i < nel * dc3; i += blockDim.x) {
    const int32_t g = a.gmap_c[e0 * dc3 + i];
    u[i] = g >= 0 ? xc[g] : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * dc * dc * df; i += blockDim.x) {
    const int xf = i % df, line = i / df;  // line = (e, zc, yc)
    double s = 0.0;
    for (int k = 0; k < dc; ++k) s += I.v[xf * dc + k] * u[line * dc + k];
    t1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * dc * df * df; i += blockDim.x) {
    const int xf = i % df, yf = (i / df) % df, ez = i / (df * df);  // ez = (e, zc)
    double s = 0.0;
    for (int k = 0; k < dc; ++k) s += I.v[yf * dc + k] * t1[(ez * dc + k) * df + xf];
    t2[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * df3; i += blockDim.x) {
    const int l = i % df3, e = i / df3;
    const int xf = l % df, yf = (l / df) % df, zf = l / (df * df);
    double s = 0.0;
    for (int k = 0; k < dc; ++k) s += I.v[zf * dc + k] * t2[((e * dc + k) * df + yf) * df + xf];
    const int64_t pos = (e0 + e) * df3 + l;
    const int32_t g = a.gmap_f[pos];
    const int32_t gi = g >= 0 ? g : ~g;
    if (!owns(a, gi, pos)) continue;
    const double v = g >= 0 ? s : 0.0;  // free rows only
    if (add)
      out[gi] += v;
    else
      out[gi] = v;
  }
}

__global__ void __launch_bounds__(kMgThreads)
    restrict_kernel(TransferArgs a, Interp1D I, const double* __restrict__ bf,
                    const double* __restrict__ yf, double* __restrict__ rc) {
  extern __shared__ double lds[];
  const int dc = a.dc, df = a.df;
  const int df3 = df * df * df;
  const int64_t e0 = int64_t(blockIdx.x) * a.nel;
  const int nel = int(min(int64_t(a.nel), a.ne - e0));
  double* rf = lds;                          // [nel][zf][yf][xf]
  double* t2 = rf + a.nel * df3;             // [nel][zc][yf][xf]
  double* t1 = t2 + a.nel * dc * df * df;    // [nel][zc][yc][xf]
  for (int i = threadIdx.x; i < nel * df3; i += blockDim.x) {
    const int64_t pos = e0 * df3 + i;
    const int32_t g = a.gmap_f[pos];
    double v = 0.0;
    if (g >= 0 && owns(a, g, pos)) v = yf ? bf[g] - yf[g] : bf[g];
    rf[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * dc * df * df; i += blockDim.x) {
    const int xf = i % df, yfi = (i / df) % df, zc = (i / (df * df)) % dc, e = i / (dc * df * df);
    double s = 0.0;
    for (int k = 0; k < df; ++k) s += I.v[k * dc + zc] * rf[((e * df + k) * df + yfi) * df + xf];
    t2[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * dc * dc * df; i += blockDim.x) {
    const int xf = i % df, yc = (i / df) % dc, ez = i / (df * dc);  // ez = (e, zc)
    double s = 0.0;
    for (int k = 0; k < df; ++k) s += I.v[k * dc + yc] * t2[(ez * df + k) * df + xf];
    t1[i] = s;
  }
  __syncthreads();
  const int dc3 = dc * dc * dc;
  for (int i = threadIdx.x; i < nel * dc3; i += blockDim.x) {
    const int xc = i % dc, line = i / dc;  // line = (e, zc, yc)
    double s = 0.0;
    for (int k = 0; k < df; ++k) s += I.v[k * dc + xc] * t1[line * df + k];
    const int32_t g = a.gmap_c[e0 * dc3 + i];
    if (g >= 0) atomicAdd(&rc[g], s);
  }
}

__global__ void fill_kernel(double* __restrict__ y, double v, int64_t n) {
  GRID_LOOP(i, n) y[i] = v;
}

// r = b - y (y null: r = b); d = c0 r / diag; x = d (zero guess) or x + d
__global__ void cheb_start_kernel(const double* __restrict__ b, const double* __restrict__ y,
                                  const double* __restrict__ diag, double* __restrict__ r,
                                  double* __restrict__ d, double* __restrict__ x, double c0,
                                  int zero_guess, int64_t n) {
  GRID_LOOP(i, n) {
    const double ri = y ? b[i] - y[i] : b[i];
    const double di = c0 * (ri / diag[i]);
    r[i] = ri;
    d[i] = di;
    x[i] = zero_guess ? di : x[i] + di;
  }
}

// r -= y; d = c1 d + c2 r / diag; x += d
__global__ void cheb_step_kernel(const double* __restrict__ y, const double* __restrict__ diag,
                                 double* __restrict__ r, double* __restrict__ d,
                                 double* __restrict__ x, double c1, double c2, int64_t n) {
  GRID_LOOP(i, n) {
    const double ri = r[i] - y[i];
    const double di = c1 * d[i] + c2 * (ri / diag[i]);
    r[i] = ri;
    d[i] = di;
    x[i] += di;
  }
}

// Power iteration.  scal[0]: the last squared D-norm; ticket: last-block counter.
// v_b = 0 on essential dofs (bmask may be null); scal[0] = sum diag v^2
__global__ void __launch_bounds__(kCGThreads)
    power_norm_kernel(double* __restrict__ v, const double* __restrict__ diag,
                      const uint8_t* __restrict__ bmask, double* partials, uint32_t* ticket,
                      double* scal, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double s = 0.0;
  GRID_LOOP(i, n) {
    double vi = v[i];
    if (bmask && bmask[i]) {
      vi = 0.0;
      v[i] = 0.0;
    }
    s += diag[i] * vi * vi;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) store_partial(partials, s);
  if (!arrive_last(ticket)) return;
  const double t = sum_partials(partials, scratch);
  if (threadIdx.x == 0) {
    scal[0] = t;
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// v *= 1 / sqrt(scal[0])
__global__ void power_scale_kernel(double* __restrict__ v, const double* scal, int64_t n) {
  const double f = 1.0 / sqrt(scal[0]);
  GRID_LOOP(i, n) v[i] *= f;
}

// lam = v . w; scal[0] = sum w^2 / diag (the squared D-norm of D^-1 w)
__global__ void __launch_bounds__(kCGThreads)
    power_dots_kernel(const double* __restrict__ v, const double* __restrict__ w,
                      const double* __restrict__ diag, double* partials, uint32_t* ticket,
                      double* scal, double* lam, int64_t n) {
  __shared__ double scratch[kCGThreads / kWave];
  double s1 = 0.0, s3 = 0.0;
  GRID_LOOP(i, n) {
    const double wi = w[i];
    s1 += v[i] * wi;
    s3 += wi * (wi / diag[i]);
  }
  s1 = block_sum(s1, scratch);
  s3 = block_sum(s3, scratch);
  if (threadIdx.x == 0) {
    store_partial(partials, s1);
    store_partial(partials + kCGBlocks, s3);
  }
  if (!arrive_last(ticket)) return;
  const double t1 = sum_partials(partials, scratch);
  const double t3 = sum_partials(partials + kCGBlocks, scratch);
  if (threadIdx.x == 0) {
    *lam = t1;
    scal[0] = t3;
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// v = (w / diag) / sqrt(scal[0])
__global__ void power_update_kernel(double* __restrict__ v, const double* __restrict__ w,
                                    const double* __restrict__ diag, const double* scal,
                                    int64_t n) {
  const double f = 1.0 / sqrt(scal[0]);
  GRID_LOOP(i, n) v[i] = (w[i] / diag[i]) * f;
}

// out[e][*] = mean over the element's points of coeff[e][*] (caller element order)
__global__ void coeff_mean_kernel(const double* __restrict__ coeff, int64_t ne, int nin,
                                  int nout, int kind, double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t e = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) / kWave;
  if (e >= ne) return;
  double s = 0.0;
  for (int q = lane; q < nin; q += kWave) {
    const double c = coeff[e * nin + q];
    s += kind == PAFEM_MEAN_GEOMETRIC ? log(c) : kind == PAFEM_MEAN_HARMONIC ? 1.0 / c : c;
  }
  s = wave_sum(s) / nin;
  const double m = kind == PAFEM_MEAN_GEOMETRIC ? exp(s) : kind == PAFEM_MEAN_HARMONIC ? 1.0 / s : s;
  for (int q = lane; q < nout; q += kWave) out[e * nout + q] = m;
}

int vec_blocks(int64_t n) {
  return int(std::min<int64_t>(kCGBlocks, std::max<int64_t>(1, (n + 255) / 256)));
}

TransferArgs transfer_args(const DevSpace& c, const DevSpace& f, int* lds_bytes, bool prolong) {
  TransferArgs a{};
  a.gmap_c = c.gmap;
  a.gmap_f = f.gmap;
  a.toff_f = f.toff;
  a.tidx_f = f.tidx;
  a.ne = f.ne;
  a.dc = c.p + 1;
  a.df = f.p + 1;
  const int dc = a.dc, df = a.df;
  const int per = prolong ? dc * dc * dc + dc * dc * df + dc * df * df
                          : df * df * df + dc * df * df + dc * dc * df;
  a.nel = std::max(1, std::min(64, kMgLdsDoubles / per));
  *lds_bytes = a.nel * per * int(sizeof(double));
  return a;
}

}  // namespace

void launch_prolongate(const DevSpace& coarse, const DevSpace& fine, const Interp1D& I,
                       const double* xc, double* yf, bool add, hipStream_t st) {
  int lds = 0;
  const TransferArgs a = transfer_args(coarse, fine, &lds, true);
  const int64_t nblk = (a.ne + a.nel - 1) / a.nel;
  if (nblk == 0) return;
  hipLaunchKernelGGL(prolong_kernel, dim3(unsigned(nblk)), dim3(kMgThreads), lds, st, a, I, xc,
                     yf, add ? 1 : 0);
}

void launch_restrict(const DevSpace& fine, const DevSpace& coarse, const Interp1D& I,
                     const double* bf, const double* yf, double* rc, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(coarse.ndofs)), dim3(256), 0, st, rc, 0.0,
                     int64_t(coarse.ndofs));
  int lds = 0;
  const TransferArgs a = transfer_args(coarse, fine, &lds, false);
  const int64_t nblk = (a.ne + a.nel - 1) / a.nel;
  if (nblk == 0) return;
  hipLaunchKernelGGL(restrict_kernel, dim3(unsigned(nblk)), dim3(kMgThreads), lds, st, a, I, bf,
                     yf, rc);
}

void launch_fill(double* y, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, y, v, n);
}

void launch_cheb_start(const double* b, const double* y, const double* diag, double* r,
                       double* d, double* x, double c0, bool zero_guess, int64_t n,
                       hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_start_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, b, y, diag, r, d,
                     x, c0, zero_guess ? 1 : 0, n);
}

void launch_cheb_step(const double* y, const double* diag, double* r, double* d, double* x,
                      double c1, double c2, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_step_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, y, diag, r, d, x,
                     c1, c2, n);
}

void launch_power_norm(double* v, const double* diag, const uint8_t* bmask, double* partials,
                       uint32_t* ticket, double* scal, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(power_norm_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, st, v, diag, bmask,
                     partials, ticket, scal, n);
  hipLaunchKernelGGL(power_scale_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, v,
                     static_cast<const double*>(scal), n);
}

void launch_power_step(double* v, const double* w, const double* diag, double* partials,
                       uint32_t* ticket, double* scal, double* lam, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(power_dots_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, st, v, w, diag,
                     partials, ticket, scal, lam, n);
  hipLaunchKernelGGL(power_update_kernel, dim3(vec_blocks(n)), dim3(256), 0, st, v, w, diag,
                     static_cast<const double*>(scal), n);
}

void launch_coeff_mean(const double* coeff, int64_t ne, int nin, int nout, int kind, double* out,
                       hipStream_t st) {
  if (ne <= 0) return;
  const int64_t threads = ne * kWave;
  const int64_t nblk = (threads + 255) / 256;
  hipLaunchKernelGGL(coeff_mean_kernel, dim3(unsigned(nblk)), dim3(256), 0, st, coeff, ne, nin,
                     nout, kind, out);
}

}  // namespace pafem
