// Kernels of the order (p-) multigrid preconditioner ("Scalable Linear Solvers":
// matrix-free preconditioning of partially assembled operators by multigrid in the
// polynomial order).
//
// * Transfers between two H1 spaces of one mesh: both spaces share the device element
//   order (a Morton order of the mesh's elements), so element k of one is element k of
//   the other.  Across a uniform refinement (h-multigrid) fine element k is child k % 8
//   of coarse element k / 8, and each axis takes the table of its half of the parent's
//   interval.  Prolongation evaluates the coarse function at the fine nodes of each
//   element by three one-axis contractions with the 1D table I[xf][xc] = phi^c_xc at
//   fine node xf (sizes fixed at compile time per pair of orders); each fine dof is
//   written by one element only, its owner (the first entry of its transposed-map list,
//   marked in a per-element bitmask of the space image).  Restriction is the exact transpose: every fine
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

// grid-stride loop, unrolled so each thread keeps several independent loads in flight
#define GRID_LOOP(i, n)                                                     \
  _Pragma("unroll 4")                                                       \
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < (n); \
       i += int64_t(gridDim.x) * blockDim.x)

struct TransferArgs {
  const int32_t* gmap_c;  // coarse element->dof map (~g on essential dofs)
  const int32_t* gmap_f;  // fine element->dof map
  const uint32_t* own_f;  // fine owner bits: node is the first occurrence of its dof
  int64_t ne;             // fine elements
  int h;                  // 1: the fine mesh refines the coarse one
};

// coarse element of fine element e, and the table half of axis `axis`
__device__ __forceinline__ int64_t parent_of(const TransferArgs& a, int64_t e) {
  return a.h ? e >> 3 : e;
}
__device__ __forceinline__ int half_of(const TransferArgs& a, int64_t e, int axis) {
  return a.h ? int((e >> axis) & 1) : 0;
}

template <int DC, int DF>
struct TransferShape {
  static constexpr int DC3 = DC * DC * DC, DF3 = DF * DF * DF;
  static constexpr int W = (DF3 + 31) / 32;  // owner words per element
  // elements per workgroup: as many as fit 32 KB of LDS (at most 64)
  static constexpr int fit(int per) { return (4096 / per) < 1 ? 1 : (4096 / per) > 64 ? 64 : (4096 / per); }
  // a multiple of 8 where 8 or more fit, so that a workgroup holds whole families of
  // children (8 consecutive fine elements) across a refinement
  static constexpr int fit8(int per) { return fit(per) >= 8 ? fit(per) & ~7 : fit(per); }
  static constexpr int NELP = fit(DC3 + DC * DC * DF + DC * DF * DF);  // prolongation
  static constexpr int NELR = fit8(DF3 + DC * DF * DF + DC * DC * DF);  // restriction
};

__device__ __forceinline__ bool owns(const uint32_t* own, int W, int64_t e, int l) {
  return (own[e * W + (l >> 5)] >> (l & 31)) & 1u;
}

static_assert(TransferShape<9, 9>::NELR * (729 * 3) * 8 <= 32768, "transfer LDS");

template <int DC, int DF>
__global__ void __launch_bounds__(kMgThreads)
    prolong_kernel(TransferArgs a, Interp1D I, const double* __restrict__ xc,
                   double* __restrict__ out, int add) {
  using S = TransferShape<DC, DF>;
  constexpr int NEL = S::NELP, DC3 = S::DC3, DF3 = S::DF3;
  __shared__ double u[NEL * DC3];             // [el][zc][yc][xc]
  __shared__ double t1[NEL * DC * DC * DF];   // [el][zc][yc][xf]
  __shared__ double t2[NEL * DC * DF * DF];   // [el][zc][yf][xf]
  const int64_t e0 = int64_t(blockIdx.x) * NEL;
  const int nel = int(min(int64_t(NEL), a.ne - e0));
  for (int i = threadIdx.x; i < nel * DC3; i += kMgThreads) {
    const int el = i / DC3, l = i - el * DC3;
    const int32_t g = a.gmap_c[parent_of(a, e0 + el) * DC3 + l];
    u[i] = g >= 0 ? xc[g] : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * DC * DC * DF; i += kMgThreads) {
    const int xf = i % DF, line = i / DF;  // line = (el, zc, yc)
    const double* T = I.v[half_of(a, e0 + line / (DC * DC), 0)];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DC; ++k) s += T[xf * DC + k] * u[line * DC + k];
    t1[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * DC * DF * DF; i += kMgThreads) {
    const int xf = i % DF, yf = (i / DF) % DF, ez = i / (DF * DF);  // ez = (el, zc)
    const double* T = I.v[half_of(a, e0 + ez / DC, 1)];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DC; ++k) s += T[yf * DC + k] * t1[(ez * DC + k) * DF + xf];
    t2[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * DF3; i += kMgThreads) {
    const int l = i % DF3, el = i / DF3;
    const int xf = l % DF, yf = (l / DF) % DF, zf = l / (DF * DF);
    const int64_t e = e0 + el;
    if (!owns(a.own_f, S::W, e, l)) continue;
    const double* T = I.v[half_of(a, e, 2)];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DC; ++k) s += T[zf * DC + k] * t2[((el * DC + k) * DF + yf) * DF + xf];
    const int32_t g = a.gmap_f[e * DF3 + l];
    const int32_t gi = g >= 0 ? g : ~g;
    const double v = g >= 0 ? s : 0.0;  // free rows only
    if (add)
      out[gi] += v;
    else
      out[gi] = v;
  }
}

template <int DC, int DF>
__global__ void __launch_bounds__(kMgThreads)
    restrict_kernel(TransferArgs a, Interp1D I, const double* __restrict__ bf,
                    const double* __restrict__ yf, double* __restrict__ rc) {
  using S = TransferShape<DC, DF>;
  constexpr int NEL = S::NELR, DC3 = S::DC3, DF3 = S::DF3;
  __shared__ double rf[NEL * DF3];            // [el][zf][yf][xf]
  __shared__ double t2[NEL * DC * DF * DF];   // [el][zc][yf][xf]
  __shared__ double t1[NEL * DC * DC * DF];   // [el][zc][yc][xf]
  const int64_t e0 = int64_t(blockIdx.x) * NEL;
  const int nel = int(min(int64_t(NEL), a.ne - e0));
  for (int i = threadIdx.x; i < nel * DF3; i += kMgThreads) {
    const int el = i / DF3, l = i - el * DF3;
    const int32_t g = a.gmap_f[e0 * DF3 + i];
    double v = 0.0;
    if (g >= 0 && owns(a.own_f, S::W, e0 + el, l)) v = yf ? bf[g] - yf[g] : bf[g];
    rf[i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * DC * DF * DF; i += kMgThreads) {
    const int xf = i % DF, yfi = (i / DF) % DF, zc = (i / (DF * DF)) % DC, el = i / (DC * DF * DF);
    const double* T = I.v[half_of(a, e0 + el, 2)];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DF; ++k) s += T[k * DC + zc] * rf[((el * DF + k) * DF + yfi) * DF + xf];
    t2[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nel * DC * DC * DF; i += kMgThreads) {
    const int xf = i % DF, yc = (i / DF) % DC, ez = i / (DF * DC);  // ez = (el, zc)
    const double* T = I.v[half_of(a, e0 + ez / DC, 1)];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DF; ++k) s += T[k * DC + yc] * t2[(ez * DF + k) * DF + xf];
    t1[i] = s;
  }
  __syncthreads();
  // Across a refinement with whole families in the workgroup, the 8 children of a parent
  // are summed here first (their values go to rf, free since the z stage) and the parent
  // adds once per node: the children's atomics would all hit the same 8 coarse nodes.
  const bool family = NEL % 8 == 0 && a.h;
  for (int i = threadIdx.x; i < nel * DC3; i += kMgThreads) {
    const int xc = i % DC, line = i / DC;  // line = (el, zc, yc)
    const int el = line / (DC * DC);
    const double* T = I.v[half_of(a, e0 + el, 0)];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DF; ++k) s += T[k * DC + xc] * t1[line * DF + k];
    if (family) {
      rf[i] = s;
    } else {
      const int32_t g = a.gmap_c[parent_of(a, e0 + el) * DC3 + (i - el * DC3)];
      if (g >= 0) atomicAdd(&rc[g], s);
    }
  }
  if (family) {
    __syncthreads();
    for (int i = threadIdx.x; i < (nel >> 3) * DC3; i += kMgThreads) {
      const int pp = i / DC3, l = i - pp * DC3;
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) s += rf[(pp * 8 + c) * DC3 + l];
      const int32_t g = a.gmap_c[((e0 >> 3) + pp) * DC3 + l];
      if (g >= 0) atomicAdd(&rc[g], s);
    }
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
  if (zero_guess) {
    GRID_LOOP(i, n) {
      const double ri = b[i];
      const double di = c0 * (ri / diag[i]);
      r[i] = ri;
      d[i] = di;
      x[i] = di;
    }
  } else {
    GRID_LOOP(i, n) {
      const double ri = y ? b[i] - y[i] : b[i];
      const double di = c0 * (ri / diag[i]);
      r[i] = ri;
      d[i] = di;
      x[i] += di;
    }
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

// streaming kernels: the CG grid (one workgroup of kCGThreads per compute unit)
constexpr int kVecThreads = kCGThreads;
int vec_blocks(int64_t n) {
  return int(std::min<int64_t>(kCGBlocks, std::max<int64_t>(1, (n + kVecThreads - 1) / kVecThreads)));
}

template <int DC, int DF>
void prolong_t(const TransferArgs& a, const Interp1D& I, const double* xc, double* yf, bool add,
               hipStream_t st) {
  constexpr int NEL = TransferShape<DC, DF>::NELP;
  const int64_t nblk = (a.ne + NEL - 1) / NEL;
  if (nblk > 0)
    hipLaunchKernelGGL((prolong_kernel<DC, DF>), dim3(unsigned(nblk)), dim3(kMgThreads), 0, st, a,
                       I, xc, yf, add ? 1 : 0);
}

template <int DC, int DF>
void restrict_t(const TransferArgs& a, const Interp1D& I, const double* bf, const double* yf,
                double* rc, hipStream_t st) {
  constexpr int NEL = TransferShape<DC, DF>::NELR;
  const int64_t nblk = (a.ne + NEL - 1) / NEL;
  if (nblk > 0)
    hipLaunchKernelGGL((restrict_kernel<DC, DF>), dim3(unsigned(nblk)), dim3(kMgThreads), 0, st, a,
                       I, bf, yf, rc);
}

TransferArgs transfer_args(const DevSpace& c, const DevSpace& f, const Interp1D& I) {
  TransferArgs a{};
  a.gmap_c = c.gmap;
  a.gmap_f = f.gmap;
  a.own_f = f.owner;
  a.ne = f.ne;
  a.h = I.h ? 1 : 0;
  if (a.h && f.ne != 8 * c.ne) throw Error(PAFEM_EINVAL, "fine mesh is not a refinement of the coarse one");
  if (!a.h && f.ne != c.ne) throw Error(PAFEM_EINVAL, "transfer spaces differ in element count");
  return a;
}

// every (coarse, fine) pair of orders 1 <= pc <= pf <= 8, as 1D node counts
#define PAFEM_TRANSFER_PAIRS(X)                                                              \
  X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(2, 7) X(2, 8) X(2, 9) X(3, 3) X(3, 4) X(3, 5)     \
  X(3, 6) X(3, 7) X(3, 8) X(3, 9) X(4, 4) X(4, 5) X(4, 6) X(4, 7) X(4, 8) X(4, 9) X(5, 5)     \
  X(5, 6) X(5, 7) X(5, 8) X(5, 9) X(6, 6) X(6, 7) X(6, 8) X(6, 9) X(7, 7) X(7, 8) X(7, 9)     \
  X(8, 8) X(8, 9) X(9, 9)

}  // namespace

void launch_prolongate(const DevSpace& coarse, const DevSpace& fine, const Interp1D& I,
                       const double* xc, double* yf, bool add, hipStream_t st) {
  const TransferArgs a = transfer_args(coarse, fine, I);
  const int dc = coarse.p + 1, df = fine.p + 1;
#define PAFEM_PROLONG_CASE(C, F) \
  if (dc == C && df == F) return prolong_t<C, F>(a, I, xc, yf, add, st);
  PAFEM_TRANSFER_PAIRS(PAFEM_PROLONG_CASE)
#undef PAFEM_PROLONG_CASE
  throw Error(PAFEM_EUNSUPPORTED, "transfer between these orders is not built");
}

void launch_restrict(const DevSpace& fine, const DevSpace& coarse, const Interp1D& I,
                     const double* bf, const double* yf, double* rc, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(coarse.ndofs)), dim3(kVecThreads), 0, st, rc, 0.0,
                     int64_t(coarse.ndofs));
  const TransferArgs a = transfer_args(coarse, fine, I);
  const int dc = coarse.p + 1, df = fine.p + 1;
#define PAFEM_RESTRICT_CASE(C, F) \
  if (dc == C && df == F) return restrict_t<C, F>(a, I, bf, yf, rc, st);
  PAFEM_TRANSFER_PAIRS(PAFEM_RESTRICT_CASE)
#undef PAFEM_RESTRICT_CASE
  throw Error(PAFEM_EUNSUPPORTED, "transfer between these orders is not built");
}

void launch_fill(double* y, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, y, v, n);
}

void launch_cheb_start(const double* b, const double* y, const double* diag, double* r,
                       double* d, double* x, double c0, bool zero_guess, int64_t n,
                       hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_start_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, b, y, diag, r, d,
                     x, c0, zero_guess ? 1 : 0, n);
}

void launch_cheb_step(const double* y, const double* diag, double* r, double* d, double* x,
                      double c1, double c2, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_step_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, y, diag, r, d, x,
                     c1, c2, n);
}

void launch_power_norm(double* v, const double* diag, const uint8_t* bmask, double* partials,
                       uint32_t* ticket, double* scal, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(power_norm_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, st, v, diag, bmask,
                     partials, ticket, scal, n);
  hipLaunchKernelGGL(power_scale_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, v,
                     static_cast<const double*>(scal), n);
}

void launch_power_step(double* v, const double* w, const double* diag, double* partials,
                       uint32_t* ticket, double* scal, double* lam, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(power_dots_kernel, dim3(kCGBlocks), dim3(kCGThreads), 0, st, v, w, diag,
                     partials, ticket, scal, lam, n);
  hipLaunchKernelGGL(power_update_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, v, w, diag,
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
