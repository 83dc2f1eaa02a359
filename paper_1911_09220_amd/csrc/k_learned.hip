// Element-patch kernels of the learned preconditioner
//     z = r / diag + G^t( w * (s_E / kbar_E) * N([r_E / s_E, f_E]) ),
// with s_E = ||r_E||, kbar_E the element mean of the coefficient, f_E the 8
// octant log-ratios of the coefficient, w = 1 / (number of element nodes that
// share the dof).  The network N runs on matrix cores (k_mlp.hip).
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

// one wave per element: lane i < D^3 owns node i
__global__ void patch_inputs_kernel(const int32_t* __restrict__ gmap, const double* __restrict__ r,
                                    const float* __restrict__ feats, int dpe, int in_pad,
                                    uint16_t* __restrict__ X, float* __restrict__ s, int64_t ne) {
  const int lane = threadIdx.x % kWave;
  const int64_t e = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) / kWave;
  if (e >= ne) return;
  const int32_t* g = gmap + e * dpe;
  double ss = 0.0;
  for (int i = lane; i < dpe; i += kWave) {
    const int d = g[i];
    const double v = r[d < 0 ? ~d : d];
    ss += v * v;
  }
  ss = wave_sum(ss);
  const double sc = sqrt(ss) + 1e-300;
  if (lane == 0) s[e] = float(sc);
  uint16_t* x = X + e * in_pad;
  for (int i = lane; i < in_pad; i += kWave) {
    float v = 0.f;
    if (i < dpe) {
      const int d = g[i];
      v = float(r[d < 0 ? ~d : d] / sc);
    } else if (i < dpe + 8) {
      v = feats[e * kFeat + 1 + (i - dpe)];
    }
    x[i] = f2bf(v);
  }
}

__global__ void patch_outputs_kernel(const float* __restrict__ out, int out_pad, int dpe,
                                     const float* __restrict__ s, const float* __restrict__ feats,
                                     double* __restrict__ ye, int64_t ne) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < ne * dpe;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = i / dpe;
    const int k = int(i - e * dpe);
    ye[i] = double(s[e]) / double(feats[e * kFeat]) * double(out[e * out_pad + k]);
  }
}

__global__ void precond_gather_kernel(const int32_t* __restrict__ toff,
                                      const int32_t* __restrict__ tidx,
                                      const uint8_t* __restrict__ bmask,
                                      const double* __restrict__ ye, const double* __restrict__ r,
                                      const double* __restrict__ diag, double* __restrict__ z,
                                      int64_t n) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n;
       g += int64_t(gridDim.x) * blockDim.x) {
    if (bmask[g]) {
      z[g] = 0.0;
      continue;
    }
    const int32_t k0 = toff[g], k1 = toff[g + 1];
    double acc = 0.0;
    for (int32_t k = k0; k < k1; ++k) acc += ye[tidx[k]];
    z[g] = r[g] / diag[g] + acc / double(k1 - k0);
  }
}

__global__ void patch_output_grad_kernel(const int32_t* __restrict__ gmap,
                                         const int32_t* __restrict__ toff,
                                         const double* __restrict__ gz,
                                         const double* __restrict__ gscale,
                                         const float* __restrict__ s,
                                         const float* __restrict__ feats, int dpe, int out_pad,
                                         uint16_t* __restrict__ dout, int64_t ne) {
  const double c = gscale ? gscale[0] : 1.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < ne * out_pad;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = i / out_pad;
    const int k = int(i - e * out_pad);
    float v = 0.f;
    if (k < dpe) {
      const int d = gmap[e * dpe + k];
      if (d >= 0) {  // essential dofs carry no correction
        const double m = double(toff[d + 1] - toff[d]);
        v = float(c * double(s[e]) / double(feats[e * kFeat]) * gz[d] / m);
      }
    }
    dout[i] = f2bf(v);
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

__global__ void jacobi_kernel(const double* __restrict__ r, const double* __restrict__ diag,
                              const uint8_t* __restrict__ bmask, double* __restrict__ z, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    z[i] = bmask[i] ? 0.0 : r[i] / diag[i];
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return int(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

void check(const char* what) {
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
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
                   hipStream_t st) {
  hipLaunchKernelGGL(jacobi_kernel, dim3(grid_for(sp.ndofs)), dim3(256), 0, st, r, diag, sp.bmask,
                     z, sp.ndofs);
  check("jacobi");
}

void launch_patch_features(const DevSpace& sp, const double* kappa, int q1d, float* feats,
                           hipStream_t st) {
  hipLaunchKernelGGL(patch_features_kernel, dim3(grid_for(sp.ne)), dim3(256), 0, st, sp.elem_orig,
                     kappa, q1d, feats, sp.ne);
  check("patch_features");
}

void launch_patch_inputs(const DevSpace& sp, const double* r, const float* feats, int in_pad,
                         uint16_t* X, float* s, hipStream_t st) {
  const int dpe = (sp.p + 1) * (sp.p + 1) * (sp.p + 1);
  const int64_t threads = sp.ne * kWave;
  hipLaunchKernelGGL(patch_inputs_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, st,
                     sp.gmap, r, feats, dpe, in_pad, X, s, sp.ne);
  check("patch_inputs");
}

void launch_patch_outputs(const DevSpace& sp, const float* out, int out_pad, const float* s,
                          const float* feats, double* ye, hipStream_t st) {
  const int dpe = (sp.p + 1) * (sp.p + 1) * (sp.p + 1);
  hipLaunchKernelGGL(patch_outputs_kernel, dim3(grid_for(sp.ne * dpe)), dim3(256), 0, st, out,
                     out_pad, dpe, s, feats, ye, sp.ne);
  check("patch_outputs");
}

void launch_precond_gather(const DevSpace& sp, const double* ye, const double* r,
                           const double* diag, double* z, hipStream_t st) {
  hipLaunchKernelGGL(precond_gather_kernel, dim3(grid_for(sp.ndofs)), dim3(256), 0, st, sp.toff,
                     sp.tidx, sp.bmask, ye, r, diag, z, sp.ndofs);
  check("precond_gather");
}

void launch_patch_output_grad(const DevSpace& sp, const double* g, const double* gscale,
                              const float* s, const float* feats, int out_pad, uint16_t* dout,
                              hipStream_t st) {
  const int dpe = (sp.p + 1) * (sp.p + 1) * (sp.p + 1);
  hipLaunchKernelGGL(patch_output_grad_kernel, dim3(grid_for(sp.ne * out_pad)), dim3(256), 0, st,
                     sp.gmap, sp.toff, g, gscale, s, feats, dpe, out_pad, dout, sp.ne);
  check("patch_output_grad");
}

}  // namespace pafem
