// Element kernels of the learned preconditioner
//     z = r / diag + sum_E R_E^t V diag(c_E / dbar_E) V^t R_E r,   z = 0 on essential dofs,
// with c_E = softplus(N(f_E)) from the element network N (k_mlp.hip) on the 8 octant
// log-ratios f_E of the coefficient, V a learned (p+1)^3 x K basis shared by all
// elements, and dbar_E the mean of diag over the element's non-essential nodes.
// The correction is positive semidefinite for any network and basis, so z(r) is
// an SPD preconditioner; the division by dbar_E makes it invariant to the
// coefficient scale and the element size.
//
// The per-iteration part (lowrank_apply) works on the apply tiles: the tile's
// unique dofs are gathered once into LDS, each element contracts with V^t and V
// in FP32, the outputs are summed per unique dof in LDS and added with one atomic
// per unique dof.  The network runs once per operator (lowrank_coeffs).
#include <math.h>

#include <algorithm>

#include "device.hpp"
#include "mlp.hpp"

namespace pafem {

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int kFeat = 9;  // kbar + 8 octant log-ratios

__global__ void patch_features_kernel(const int32_t* __restrict__ orig, const double* __restrict__ kappa,
                                      int Q, float* __restrict__ feats, int64_t ne) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < ne;
       e += int64_t(gridDim.x) * blockDim.x) {
    float* f = feats + e * kFeat;
    if (!kappa) {
      f[0] = 1.f;
      for (int o = 0; o < 8; ++o) f[1 + o] = 0.f;
      continue;
    }
    const double* k = kappa + size_t(orig[e]) * Q * Q * Q;
    double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0}, tot = 0.0;
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int half = Q / 2;
    for (int qz = 0; qz < Q; ++qz)
      for (int qy = 0; qy < Q; ++qy)
        for (int qx = 0; qx < Q; ++qx) {
          const double v = k[(qz * Q + qy) * Q + qx];
          const int o = (qx >= half) | ((qy >= half) << 1) | ((qz >= half) << 2);
          sum[o] += v;
          cnt[o]++;
          tot += v;
        }
    const double kbar = tot / double(Q * Q * Q);
    f[0] = float(kbar);
    for (int o = 0; o < 8; ++o) f[1 + o] = float(log((sum[o] / cnt[o]) / kbar));
  }
}

// X[e] = bf16([f_E (8 log-ratios), 0 ...]), in_pad columns
__global__ void net_inputs_kernel(const float* __restrict__ feats, int in_pad,
                                  uint16_t* __restrict__ X, int64_t ne) {
  const int64_t n = ne * in_pad;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = i / in_pad;
    const int j = int(i - e * in_pad);
    X[i] = f2bf(j < 8 ? feats[e * kFeat + 1 + j] : 0.f);
  }
}

// One wave per element: c[e][k] = softplus(a[e][k]) and idb[e] = 1 / dbar_E.
__global__ void lowrank_coeffs_kernel(const int32_t* __restrict__ gmap, const double* __restrict__ diag,
                                      int dpe, const float* __restrict__ a, int K,
                                      float* __restrict__ c, float* __restrict__ idb, int64_t ne) {
  const int lane = threadIdx.x % kWave;
  const int64_t e = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) / kWave;
  if (e >= ne) return;
  const int32_t* g = gmap + e * dpe;
  double sum = 0.0, cnt = 0.0;
  for (int i = lane; i < dpe; i += kWave) {
    const int d = g[i];
    if (d >= 0) {
      sum += diag[d];
      cnt += 1.0;
    }
  }
  sum = wave_sum(sum);
  cnt = wave_sum(cnt);
  if (lane == 0) idb[e] = cnt > 0.0 ? float(cnt / sum) : 1.f;
  for (int k = lane; k < K; k += kWave) {
    const float x = a[e * K + k];
    c[e * K + k] = x > 20.f ? x : log1pf(expf(x));
  }
}

template <int P, int K>
struct LowRankShape {
  static constexpr int D = P + 1, DDD = D * D * D;
  static constexpr int NE = qdata_tile(P + 2);  // elements per apply tile
  static constexpr int VK = DDD * K;
};

// z += sum_E R_E^t V diag(c_E idb_E) V^t R_E r over the non-essential dofs (z holds
// the Jacobi part on entry).  Persistent: each workgroup loads V into LDS once and
// walks one contiguous range of apply tiles (ranges of the workgroups of one XCD
// are adjacent, so tiles that share dofs share an L2).  Per tile every global load
// (unique dofs, r, slot map, coefficients) is issued before the first barrier, and
// each thread keeps the unique dofs it gathered for its scatter, so a tile waits on
// one round of memory latency.
template <int P, int K>
__global__ void __launch_bounds__(256)
    lowrank_apply_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                         const uint16_t* __restrict__ tile_slot, const float* __restrict__ V,
                         const float* __restrict__ c, const float* __restrict__ idb,
                         const double* __restrict__ r, double* __restrict__ z, int ne, int ntiles) {
  using S = LowRankShape<P, K>;
  constexpr int DDD = S::DDD, NE = S::NE;
  constexpr int MU = (NE * DDD + 255) / 256;  // unique dofs per thread (at most)
  __shared__ float sV[DDD * K];    // [i][k]
  __shared__ float sVt[K * DDD];   // [k][i]
  __shared__ float sU[NE * DDD];   // the tile's unique dofs: r, later the summed outputs
  __shared__ float sRE[NE * DDD];  // element node values
  __shared__ float sT[NE * K];
  __shared__ float sC[NE * K];     // c_E idb_E per element and column
  __shared__ uint16_t sSlot[NE * DDD];
  const int tid = threadIdx.x;
  for (int j = tid; j < DDD * K; j += 256) {
    const float v = V[j];
    sV[j] = v;
    sVt[(j % K) * DDD + j / K] = v;
  }
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int t0 = b * per, t1 = min(ntiles, t0 + per);
  for (int tile = t0; tile < t1; ++tile) {
    const int e0 = tile * NE;
    const int nel = min(NE, ne - e0);
    const int u0 = tile_off[tile];
    const int nu = tile_off[tile + 1] - u0;
    int gk[MU];
#pragma unroll
    for (int m = 0; m < MU; ++m) {
      const int s = tid + 256 * m;
      gk[m] = s < nu ? tile_dofs[u0 + s] : -1;
    }
    float rv[MU];
#pragma unroll
    for (int m = 0; m < MU; ++m) rv[m] = gk[m] < 0 ? 0.f : float(r[gk[m]]);
    uint16_t sl[MU];  // slot map entries j = tid + 256 m < nel * DDD
#pragma unroll
    for (int m = 0; m < MU; ++m) {
      const int j = tid + 256 * m;
      sl[m] = j < nel * DDD ? tile_slot[size_t(e0) * DDD + j] : uint16_t(0);
    }
    constexpr int MC = (NE * K + 255) / 256;
    float cv[MC];
#pragma unroll
    for (int m = 0; m < MC; ++m) {
      const int j = tid + 256 * m;
      cv[m] = j < nel * K ? c[size_t(e0) * K + j] * idb[e0 + j / K] : 0.f;
    }
    __syncthreads();  // V is in place; the previous tile's outputs are out
#pragma unroll
    for (int m = 0; m < MU; ++m) {
      const int j = tid + 256 * m;
      if (j < nu) sU[j] = rv[m];
      if (j < nel * DDD) sSlot[j] = sl[m];
    }
#pragma unroll
    for (int m = 0; m < MC; ++m)
      if (tid + 256 * m < nel * K) sC[tid + 256 * m] = cv[m];
    __syncthreads();
    for (int j = tid; j < nel * DDD; j += 256) sRE[j] = sU[sSlot[j]];
    __syncthreads();
    for (int s = tid; s < nu; s += 256) sU[s] = 0.f;
    // t = V^t r_E, scaled by c_E / dbar_E
    for (int j = tid; j < nel * K; j += 256) {
      const int el = j / K, k = j - el * K;
      const float* re = sRE + el * DDD;
      float acc = 0.f;
#pragma unroll 8
      for (int i = 0; i < DDD; ++i) acc += sV[i * K + k] * re[i];
      sT[j] = acc * sC[j];
    }
    __syncthreads();
    // y_E = V t, summed per unique dof
    for (int j = tid; j < nel * DDD; j += 256) {
      const int el = j / DDD, i = j - el * DDD;
      const float* t = sT + el * K;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) acc += sVt[k * DDD + i] * t[k];
      atomicAdd(&sU[sSlot[j]], acc);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MU; ++m)
      if (gk[m] >= 0) unsafeAtomicAdd(&z[gk[m]], double(sU[tid + 256 * m]));
  }
}

// Backward of the low-rank term for dL/dz = gscale * g (essential entries are read
// as 0):
//   s_E = V^t R_E g,  t_E = V^t R_E r,
//   dout[e][k] = s_k t_k idb_E sigmoid(a_k)   (bf16, the network's output gradient;
//                                              sigmoid(a) = 1 - exp(-softplus(a)))
//   dV = sum_E R_E g (c idb t)^t + R_E r (c idb s)^t,
// the sum over elements taken in a fixed order: each workgroup walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ... and each thread owns fixed entries of
// dV; part[blockIdx.x] receives the workgroup's partial sum.
template <int P, int K>
__global__ void __launch_bounds__(256)
    lowrank_grad_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                        const uint16_t* __restrict__ tile_slot, const float* __restrict__ V,
                        const float* __restrict__ c, const float* __restrict__ idb,
                        const double* __restrict__ r, const double* __restrict__ g,
                        const double* __restrict__ gscale, uint16_t* __restrict__ dout,
                        float* __restrict__ part, int ne, int ntiles) {
  using S = LowRankShape<P, K>;
  constexpr int DDD = S::DDD, NE = S::NE, VK = S::VK;
  constexpr int OWN = (VK + 255) / 256;
  __shared__ float sV[DDD * K];
  __shared__ float sUr[NE * DDD];
  __shared__ float sUg[NE * DDD];
  __shared__ float sRE[NE * DDD];
  __shared__ float sGE[NE * DDD];
  __shared__ float sA[NE * K];
  __shared__ float sB[NE * K];
  const int tid = threadIdx.x;
  const float gs = float(*gscale);
  for (int j = tid; j < VK; j += 256) sV[j] = V[j];
  float acc[OWN];
#pragma unroll
  for (int m = 0; m < OWN; ++m) acc[m] = 0.f;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int e0 = tile * NE;
    const int nel = min(NE, ne - e0);
    const int u0 = tile_off[tile];
    const int nu = tile_off[tile + 1] - u0;
    __syncthreads();  // the previous tile's readers are done
    for (int s = tid; s < nu; s += 256) {
      const int d = tile_dofs[u0 + s];
      sUr[s] = d < 0 ? 0.f : float(r[d]);
      sUg[s] = d < 0 ? 0.f : float(g[d]) * gs;
    }
    __syncthreads();
    for (int j = tid; j < nel * DDD; j += 256) {
      const int sl = tile_slot[size_t(e0) * DDD + j];
      sRE[j] = sUr[sl];
      sGE[j] = sUg[sl];
    }
    __syncthreads();
    for (int j = tid; j < nel * K; j += 256) {
      const int el = j / K, k = j - el * K;
      const float* re = sRE + el * DDD;
      const float* ge = sGE + el * DDD;
      float t = 0.f, s = 0.f;
#pragma unroll 8
      for (int i = 0; i < DDD; ++i) {
        const float v = sV[i * K + k];
        t += v * re[i];
        s += v * ge[i];
      }
      const size_t ek = size_t(e0 + el) * K + k;
      const float ce = c[ek], ib = idb[e0 + el];
      dout[ek] = f2bf(s * t * ib * (-expm1f(-ce)));
      sA[j] = ce * ib * t;
      sB[j] = ce * ib * s;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < OWN; ++m) {
      const int j = tid + 256 * m;
      if (j < VK) {
        const int i = j / K, k = j - i * K;
        float a = acc[m];
        for (int el = 0; el < nel; ++el)
          a += sGE[el * DDD + i] * sA[el * K + k] + sRE[el * DDD + i] * sB[el * K + k];
        acc[m] = a;
      }
    }
  }
#pragma unroll
  for (int m = 0; m < OWN; ++m) {
    const int j = tid + 256 * m;
    if (j < VK) part[size_t(blockIdx.x) * VK + j] = acc[m];
  }
}

__global__ void diff_kernel(const double* __restrict__ a, const double* __restrict__ b,
                            double* __restrict__ t, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    t[i] = a[i] - b[i];
}

// v = u / diag (0 on essential dofs); scal[0] = loss = (u.D^-1 u) / (r.D^-1 r),
// scal[1] = -2 / (r.D^-1 r) (the factor of dL/dz = scal[1] * A v)
__global__ void __launch_bounds__(256)
    loss_kernel(const double* __restrict__ u, const double* __restrict__ r,
                const double* __restrict__ diag, const uint8_t* __restrict__ bmask,
                double* __restrict__ v, double* partials, uint32_t* ticket, double* scal,
                int64_t n) {
  __shared__ double scratch[256 / kWave];
  double num = 0.0, den = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double vi = bmask[i] ? 0.0 : u[i] / diag[i];
    v[i] = vi;
    num += u[i] * vi;
    den += r[i] * r[i] / diag[i];
  }
  num = block_sum(num, scratch);
  den = block_sum(den, scratch);
  double* p0 = partials;
  double* p1 = partials + gridDim.x;
  if (threadIdx.x == 0) {
    store_partial(p0, num);
    store_partial(p1, den);
  }
  if (!arrive_last(ticket)) return;
  const double tn = sum_partials(p0, scratch);
  const double td = sum_partials(p1, scratch);
  if (threadIdx.x == 0) {
    scal[0] = tn / td;
    scal[1] = -2.0 / td;
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// z = r / diag off the essential dofs; on them per ess_mode (kJacobiEss*)
__global__ void jacobi_kernel(const double* __restrict__ r, const double* __restrict__ diag,
                              const uint8_t* __restrict__ bmask, int ess_mode,
                              double* __restrict__ z, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const bool b = bmask[i] && ess_mode != kJacobiEssDiag;
    z[i] = b ? (ess_mode == kJacobiEssKeep ? r[i] : 0.0) : r[i] / diag[i];
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return int(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

void check(const char* what) {
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

int ntiles_of(const DevSpace& sp) { return int((sp.ne + sp.tile_ne - 1) / sp.tile_ne); }

template <int P>
void lowrank_apply_p(const DevSpace& sp, const float* V, const float* c, const float* idb,
                     const double* r, double* z, hipStream_t st) {
  if (sp.tile_ne != LowRankShape<P, kLowRank>::NE)
    throw Error(PAFEM_EINVAL, "low-rank apply: tile size differs from the apply tiles");
  const int nt = ntiles_of(sp);
  // persistent grid: at most as many workgroups as are resident at once on this device
  // (a second, partial wave of workgroups would double the time of its tiles)
  static int resident[64] = {0};
  auto ok = [](hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  int dev = 0;
  ok(hipGetDevice(&dev), "device");
  if (dev < 0 || dev >= 64) dev = 0;
  if (resident[dev] == 0) {
    int per_cu = 0, cus = 0;
    ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lowrank_apply_kernel<P, kLowRank>,
                                                    256, 0),
       "occupancy");
    ok(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CUs");
    resident[dev] = std::max(1, std::min(kLowRankApplyBlocks, per_cu * cus));
  }
  hipLaunchKernelGGL((lowrank_apply_kernel<P, kLowRank>), dim3(std::min(nt, resident[dev])),
                     dim3(256), 0, st, sp.tile_off, sp.tile_dofs, sp.tile_slot, V, c, idb, r, z,
                     int(sp.ne), nt);
}

template <int P>
void lowrank_grad_p(const DevSpace& sp, const float* V, const float* c, const float* idb,
                    const double* r, const double* g, const double* gscale, uint16_t* dout,
                    float* part, hipStream_t st) {
  if (sp.tile_ne != LowRankShape<P, kLowRank>::NE)
    throw Error(PAFEM_EINVAL, "low-rank gradient: tile size differs from the apply tiles");
  const int nt = ntiles_of(sp);
  hipLaunchKernelGGL((lowrank_grad_kernel<P, kLowRank>), dim3(std::min(nt, kLowRankGradBlocks)),
                     dim3(256), 0, st, sp.tile_off, sp.tile_dofs, sp.tile_slot, V, c, idb, r, g,
                     gscale, dout, part, int(sp.ne), nt);
}

}  // namespace

constexpr int kLossBlocks = 512;

void launch_diff(const double* a, const double* b, double* t, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(diff_kernel, dim3(grid_for(n)), dim3(256), 0, st, a, b, t, n);
  check("diff");
}

void launch_loss(const DevSpace& sp, const double* u, const double* r, const double* diag,
                 double* v, double* partials, uint32_t* ticket, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(loss_kernel, dim3(kLossBlocks), dim3(256), 0, st, u, r, diag, sp.bmask, v,
                     partials, ticket, scal, sp.ndofs);
  check("loss");
}

void launch_jacobi(const DevSpace& sp, const double* r, const double* diag, double* z,
                   hipStream_t st, int ess_mode) {
  hipLaunchKernelGGL(jacobi_kernel, dim3(grid_for(sp.ndofs)), dim3(256), 0, st, r, diag, sp.bmask,
                     ess_mode, z, sp.ndofs);
  check("jacobi");
}

void launch_patch_features(const DevSpace& sp, const double* kappa, int q1d, float* feats,
                           hipStream_t st) {
  hipLaunchKernelGGL(patch_features_kernel, dim3(grid_for(sp.ne)), dim3(256), 0, st, sp.elem_orig,
                     kappa, q1d, feats, sp.ne);
  check("patch_features");
}

void launch_net_inputs(const DevSpace& sp, const float* feats, int in_pad, uint16_t* X,
                       hipStream_t st) {
  hipLaunchKernelGGL(net_inputs_kernel, dim3(grid_for(sp.ne * in_pad)), dim3(256), 0, st, feats,
                     in_pad, X, sp.ne);
  check("net_inputs");
}

void launch_lowrank_coeffs(const DevSpace& sp, const double* diag, const float* a, float* c,
                           float* idb, hipStream_t st) {
  const int dpe = (sp.p + 1) * (sp.p + 1) * (sp.p + 1);
  const int64_t threads = sp.ne * kWave;
  hipLaunchKernelGGL(lowrank_coeffs_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0,
                     st, sp.gmap, diag, dpe, a, kLowRank, c, idb, sp.ne);
  check("lowrank_coeffs");
}

void launch_lowrank_apply(const DevSpace& sp, const float* V, const float* c, const float* idb,
                          const double* r, double* z, hipStream_t st) {
  switch (sp.p) {
    case 1: lowrank_apply_p<1>(sp, V, c, idb, r, z, st); break;
    case 2: lowrank_apply_p<2>(sp, V, c, idb, r, z, st); break;
    case 3: lowrank_apply_p<3>(sp, V, c, idb, r, z, st); break;
    case 4: lowrank_apply_p<4>(sp, V, c, idb, r, z, st); break;
    default: throw Error(PAFEM_EUNSUPPORTED, "learned preconditioner: orders 1..4");
  }
  check("lowrank_apply");
}

void launch_lowrank_grad(const DevSpace& sp, const float* V, const float* c, const float* idb,
                         const double* r, const double* g, const double* gscale, uint16_t* dout,
                         float* part, float* gV, hipStream_t st) {
  switch (sp.p) {
    case 1: lowrank_grad_p<1>(sp, V, c, idb, r, g, gscale, dout, part, st); break;
    case 2: lowrank_grad_p<2>(sp, V, c, idb, r, g, gscale, dout, part, st); break;
    case 3: lowrank_grad_p<3>(sp, V, c, idb, r, g, gscale, dout, part, st); break;
    case 4: lowrank_grad_p<4>(sp, V, c, idb, r, g, gscale, dout, part, st); break;
    default: throw Error(PAFEM_EUNSUPPORTED, "learned preconditioner: orders 1..4");
  }
  check("lowrank_grad");
  const int dpe = (sp.p + 1) * (sp.p + 1) * (sp.p + 1);
  launch_reduce_parts(part, gV, std::min(ntiles_of(sp), kLowRankGradBlocks), dpe * kLowRank, st);
}

}  // namespace pafem
