// Setup kernels: geometric factors + quadrature data (PA setup), the linear
// form, the operator diagonal, and the transposed element restriction G^t.
//
// These run once per solve, so they are written for clarity with runtime sizes
// (one workgroup per element, dynamic LDS).  All arithmetic is FP64.
#include <climits>

#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

#define HIP_LAUNCH_CHECK()                                                        \
  do {                                                                            \
    hipError_t err_ = hipGetLastError();                                          \
    if (err_ != hipSuccess)                                                       \
      throw Error(PAFEM_EHIP, std::string("kernel launch: ") + hipGetErrorString(err_)); \
  } while (0)

struct TabView {
  const double *pts, *wts, *B, *G, *Bg, *Gg;
};

TabView tab_view(const DevSpace& sp, int Q) {
  const int D = sp.p + 1, NG = sp.ng;
  const double* t = sp.tables + table_offset_doubles(Q, D, NG);
  TabView v;
  v.pts = t;
  v.wts = t + Q;
  v.B = t + 2 * Q;
  v.G = v.B + Q * D;
  v.Bg = v.G + Q * D;
  v.Gg = v.Bg + Q * NG;
  return v;
}

// Jacobian J_ab = d x_a / d xhat_b of the element map at quadrature point q, from
// the element's geometry nodes X[k][3] and the 1D geometry tables Bg, Gg [Q][NG].
__device__ void element_jacobian(int q, int Q, int NG, const double* X, const double* Bg,
                                 const double* Gg, double J[3][3], double x[3]) {
  const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
  for (int a = 0; a < 3; ++a) {
    x[a] = 0.0;
    for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
  }
  for (int k3 = 0; k3 < NG; ++k3)
    for (int k2 = 0; k2 < NG; ++k2)
      for (int k1 = 0; k1 < NG; ++k1) {
        const double b1 = Bg[q1 * NG + k1], g1 = Gg[q1 * NG + k1];
        const double b2 = Bg[q2 * NG + k2], g2 = Gg[q2 * NG + k2];
        const double b3 = Bg[q3 * NG + k3], g3 = Gg[q3 * NG + k3];
        const double w = b1 * b2 * b3;
        const double d0 = g1 * b2 * b3, d1 = b1 * g2 * b3, d2 = b1 * b2 * g3;
        const double* Xk = X + 3 * (k1 + NG * (k2 + NG * k3));
        for (int a = 0; a < 3; ++a) {
          x[a] += w * Xk[a];
          J[a][0] += Xk[a] * d0;
          J[a][1] += Xk[a] * d1;
          J[a][2] += Xk[a] * d2;
        }
      }
}

__global__ void qdata_kernel(const double* __restrict__ gnodes, const int32_t* __restrict__ orig,
                             int NG, TabView tv, int Q, int kind,
                             const double* __restrict__ coeff, double scale,
                             double* __restrict__ qd, int32_t* status) {
  extern __shared__ double smem[];
  const int e = blockIdx.x;
  const int NN = NG * NG * NG, QQQ = Q * Q * Q;
  double* sX = smem;
  double* sBg = sX + 3 * NN;
  double* sGg = sBg + Q * NG;
  for (int i = threadIdx.x; i < 3 * NN; i += blockDim.x) sX[i] = gnodes[size_t(e) * 3 * NN + i];
  for (int i = threadIdx.x; i < Q * NG; i += blockDim.x) {
    sBg[i] = tv.Bg[i];
    sGg[i] = tv.Gg[i];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < QQQ; q += blockDim.x) {
    double J[3][3], x[3];
    element_jacobian(q, Q, NG, sX, sBg, sGg, J, x);
    // adjugate A = det(J) J^{-1}
    const double A00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double A01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    const double A02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const double A10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double A11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    const double A12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const double A20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double A21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    const double A22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * A00 + J[0][1] * A10 + J[0][2] * A20;
    if (!(det > 0.0)) atomicMin(&status[0], orig[e]);
    const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
    const double w = tv.wts[q1] * tv.wts[q2] * tv.wts[q3];
    // scalar coefficient per point (convection, elasticity and the definite Maxwell
    // form read theirs below)
    const double c = (kind == PAFEM_CONVECTION || kind == PAFEM_ELASTICITY ||
                      kind == PAFEM_HCURL_MAXWELL || kind == PAFEM_DG_CONVECTION)
                         ? 0.0
                         : scale * (coeff ? coeff[size_t(orig[e]) * QQQ + q] : 1.0);
    if (kind == PAFEM_HCURL_CURLCURL || kind == PAFEM_HCURL_MAXWELL) {
      // curl-curl: w alpha J^T J / det J (the reference curl maps with J / det J);
      // Maxwell: that with alpha, then the mass part w beta A A^T / det J with beta,
      // (alpha, beta) the point's coefficient pair
      const int nc = kind == PAFEM_HCURL_MAXWELL ? 12 : 6;
      double ca = c, cb = 0.0;
      if (kind == PAFEM_HCURL_MAXWELL) {
        const double* ab = coeff + (size_t(orig[e]) * QQQ + q) * 2;
        ca = scale * ab[0];
        cb = scale * ab[1];
      }
      const double f = w * ca / det;
      double T[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) T[a][b] = J[0][a] * J[0][b] + J[1][a] * J[1][b] + J[2][a] * J[2][b];
      qd[qdata_index(e, 0, q, Q, nc)] = f * T[0][0];
      qd[qdata_index(e, 1, q, Q, nc)] = f * T[0][1];
      qd[qdata_index(e, 2, q, Q, nc)] = f * T[0][2];
      qd[qdata_index(e, 3, q, Q, nc)] = f * T[1][1];
      qd[qdata_index(e, 4, q, Q, nc)] = f * T[1][2];
      qd[qdata_index(e, 5, q, Q, nc)] = f * T[2][2];
      if (kind == PAFEM_HCURL_MAXWELL) {
        const double g = w * cb / det;
        qd[qdata_index(e, 6, q, Q, 12)] = g * (A00 * A00 + A01 * A01 + A02 * A02);
        qd[qdata_index(e, 7, q, Q, 12)] = g * (A00 * A10 + A01 * A11 + A02 * A12);
        qd[qdata_index(e, 8, q, Q, 12)] = g * (A00 * A20 + A01 * A21 + A02 * A22);
        qd[qdata_index(e, 9, q, Q, 12)] = g * (A10 * A10 + A11 * A11 + A12 * A12);
        qd[qdata_index(e, 10, q, Q, 12)] = g * (A10 * A20 + A11 * A21 + A12 * A22);
        qd[qdata_index(e, 11, q, Q, 12)] = g * (A20 * A20 + A21 * A21 + A22 * A22);
      }
    } else if (kind == PAFEM_MASS) {
      qd[qdata_index(e, 0, q, Q, 1)] = w * c * det;
    } else if (kind == PAFEM_GRADIENT || kind == PAFEM_DIVERGENCE) {
      // w kappa det J J^{-T} as D[c][b] = w kappa adj(J)[b][c]: physical derivative c
      // (the gradient's output component, the divergence's input component),
      // reference derivative b
      const double f = w * c;
      qd[qdata_index(e, 0, q, Q, 9)] = f * A00;
      qd[qdata_index(e, 1, q, Q, 9)] = f * A10;
      qd[qdata_index(e, 2, q, Q, 9)] = f * A20;
      qd[qdata_index(e, 3, q, Q, 9)] = f * A01;
      qd[qdata_index(e, 4, q, Q, 9)] = f * A11;
      qd[qdata_index(e, 5, q, Q, 9)] = f * A21;
      qd[qdata_index(e, 6, q, Q, 9)] = f * A02;
      qd[qdata_index(e, 7, q, Q, 9)] = f * A12;
      qd[qdata_index(e, 8, q, Q, 9)] = f * A22;
    } else if (kind == PAFEM_ELASTICITY) {
      // J^{-1} = A / det J as [b][d] = d xhat_b / d x_d, then w det J lambda and
      // w det J mu, lambda and mu from the point's coefficient pair
      const double* lm = coeff + (size_t(orig[e]) * QQQ + q) * 2;
      const double id = 1.0 / det, wd = scale * w * det;
      const double Kinv[9] = {A00, A01, A02, A10, A11, A12, A20, A21, A22};
      for (int k = 0; k < 9; ++k) qd[qdata_index(e, k, q, Q, 11)] = Kinv[k] * id;
      qd[qdata_index(e, 9, q, Q, 11)] = wd * lm[0];
      qd[qdata_index(e, 10, q, Q, 11)] = wd * lm[1];
    } else if (kind == PAFEM_CONVECTION || kind == PAFEM_DG_CONVECTION) {
      // alpha det J J^{-1} beta = alpha adj(J) beta, beta = scale * velocity at the point
      // (the DG convection: one constant velocity)
      const double* v =
          kind == PAFEM_DG_CONVECTION ? coeff : coeff + (size_t(orig[e]) * QQQ + q) * 3;
      const double b0 = scale * v[0], b1 = scale * v[1], b2 = scale * v[2];
      qd[qdata_index(e, 0, q, Q, 3)] = w * (A00 * b0 + A01 * b1 + A02 * b2);
      qd[qdata_index(e, 1, q, Q, 3)] = w * (A10 * b0 + A11 * b1 + A12 * b2);
      qd[qdata_index(e, 2, q, Q, 3)] = w * (A20 * b0 + A21 * b1 + A22 * b2);
    } else if (kind == PAFEM_DIFFUSION_GEOM) {
      qd[qdata_index(e, 0, q, Q, 1)] = w * c;  // the apply recomputes the geometric part
    } else {
      // diffusion and the H(curl) mass: alpha kappa det J J^{-1} J^{-T} = alpha kappa
      // A A^T / det J
      const double f = w * c / det;
      qd[qdata_index(e, 0, q, Q, 6)] = f * (A00 * A00 + A01 * A01 + A02 * A02);
      qd[qdata_index(e, 1, q, Q, 6)] = f * (A00 * A10 + A01 * A11 + A02 * A12);
      qd[qdata_index(e, 2, q, Q, 6)] = f * (A00 * A20 + A01 * A21 + A02 * A22);
      qd[qdata_index(e, 3, q, Q, 6)] = f * (A10 * A10 + A11 * A11 + A12 * A12);
      qd[qdata_index(e, 4, q, Q, 6)] = f * (A10 * A20 + A11 * A21 + A12 * A22);
      qd[qdata_index(e, 5, q, Q, 6)] = f * (A20 * A20 + A21 * A21 + A22 * A22);
    }
  }
}

// out[i1,i2,i3] (+)= factor * sum_q T1[q1,i1] T2[q2,i2] T3[q3,i3] in[q1,q2,q3] by three
// one-axis contractions through LDS (sum factorization of B^t).
__device__ void contract_to_dofs(int Q, int D, const double* in, double* t1, double* t2,
                                 double* out, const double* T1, const double* T2,
                                 const double* T3, double factor, bool accumulate) {
  const int nt = blockDim.x, tid = threadIdx.x;
  for (int idx = tid; idx < Q * Q * D; idx += nt) {
    const int i1 = idx % D, q23 = idx / D;
    double s = 0.0;
    for (int q1 = 0; q1 < Q; ++q1) s += T1[q1 * D + i1] * in[q23 * Q + q1];
    t1[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < Q * D * D; idx += nt) {
    const int i1 = idx % D, i2 = (idx / D) % D, q3 = idx / (D * D);
    double s = 0.0;
    for (int q2 = 0; q2 < Q; ++q2) s += T2[q2 * D + i2] * t1[(q3 * Q + q2) * D + i1];
    t2[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < D * D * D; idx += nt) {
    const int i1 = idx % D, i2 = (idx / D) % D, i3 = idx / (D * D);
    double s = 0.0;
    for (int q3 = 0; q3 < Q; ++q3) s += T3[q3 * D + i3] * t2[(q3 * D + i2) * D + i1];
    out[idx] = (accumulate ? out[idx] : 0.0) + factor * s;
  }
  __syncthreads();
}

__global__ void linear_form_kernel(const double* __restrict__ gnodes,
                                   const int32_t* __restrict__ orig, int NG, TabView tv, int Q,
                                   int D, int source, const double* __restrict__ fqp,
                                   double scale, double* __restrict__ ye) {
  extern __shared__ double smem[];
  const int e = blockIdx.x;
  const int NN = NG * NG * NG, QQQ = Q * Q * Q, DDD = D * D * D;
  double* sX = smem;
  double* sBg = sX + 3 * NN;
  double* sGg = sBg + Q * NG;
  double* sB = sGg + Q * NG;
  double* sF = sB + Q * D;
  double* t1 = sF + QQQ;
  double* t2 = t1 + Q * Q * D;
  double* out = t2 + Q * D * D;
  for (int i = threadIdx.x; i < 3 * NN; i += blockDim.x) sX[i] = gnodes[size_t(e) * 3 * NN + i];
  for (int i = threadIdx.x; i < Q * NG; i += blockDim.x) {
    sBg[i] = tv.Bg[i];
    sGg[i] = tv.Gg[i];
  }
  for (int i = threadIdx.x; i < Q * D; i += blockDim.x) sB[i] = tv.B[i];
  __syncthreads();
  const double pi = 3.14159265358979323846;
  for (int q = threadIdx.x; q < QQQ; q += blockDim.x) {
    double J[3][3], x[3];
    element_jacobian(q, Q, NG, sX, sBg, sGg, J, x);
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
    const double w = tv.wts[q1] * tv.wts[q2] * tv.wts[q3];
    double f;
    if (source == PAFEM_SOURCE_ARRAY)
      f = scale * fqp[size_t(orig[e]) * QQQ + q];
    else if (source == PAFEM_SOURCE_CONST)
      f = scale;
    else
      f = scale * 3.0 * pi * pi * sin(pi * x[0]) * sin(pi * x[1]) * sin(pi * x[2]);
    sF[q] = w * det * f;
  }
  __syncthreads();
  contract_to_dofs(Q, D, sF, t1, t2, out, sB, sB, sB, 1.0, false);
  for (int i = threadIdx.x; i < DDD; i += blockDim.x) ye[size_t(e) * DDD + i] = out[i];
}

__global__ void diagonal_kernel(TabView tv, int Q, int D, int kind,
                                const double* __restrict__ qd, double* __restrict__ ye) {
  extern __shared__ double smem[];
  const int e = blockIdx.x;
  const int QQQ = Q * Q * Q, DDD = D * D * D, QD = Q * D;
  double* sBB = smem;      // B o B
  double* sGG = sBB + QD;  // G o G
  double* sBG = sGG + QD;  // B o G
  double* sF = sBG + QD;
  double* t1 = sF + QQQ;
  double* t2 = t1 + Q * Q * D;
  double* out = t2 + Q * D * D;
  for (int i = threadIdx.x; i < QD; i += blockDim.x) {
    const double b = tv.B[i], g = tv.G[i];
    sBB[i] = b * b;
    sGG[i] = g * g;
    sBG[i] = b * g;
  }
  __syncthreads();
  if (kind == PAFEM_MASS) {
    for (int q = threadIdx.x; q < QQQ; q += blockDim.x) sF[q] = qd[qdata_index(e, 0, q, Q, 1)];
    __syncthreads();
    contract_to_dofs(Q, D, sF, t1, t2, out, sBB, sBB, sBB, 1.0, false);
  } else {
    // diag_i = sum_q sum_ab D_ab(q) d_a phi_i(q) d_b phi_i(q); d_a phi_i is a product of
    // G in direction a and B in the others, so each (a,b) term is a tensor
    // contraction with elementwise products of the 1D tables.
    int comp = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b, ++comp) {
        for (int q = threadIdx.x; q < QQQ; q += blockDim.x)
          sF[q] = qd[qdata_index(e, comp, q, Q, 6)];
        __syncthreads();
        const double* T[3];
        for (int d = 0; d < 3; ++d) {
          const int hits = (d == a) + (d == b);
          T[d] = hits == 2 ? sGG : (hits == 1 ? sBG : sBB);
        }
        contract_to_dofs(Q, D, sF, t1, t2, out, T[0], T[1], T[2], a == b ? 1.0 : 2.0, comp > 0);
      }
  }
  for (int i = threadIdx.x; i < DDD; i += blockDim.x) ye[size_t(e) * DDD + i] = out[i];
}

template <typename T>
__global__ void evec_gather_kernel(const int32_t* __restrict__ toff,
                                   const int32_t* __restrict__ tidx,
                                   const uint8_t* __restrict__ bmask, const T* __restrict__ ye,
                                   const T* __restrict__ x, int bc_mode, T bc_value,
                                   T* __restrict__ y, int64_t n) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n;
       g += int64_t(gridDim.x) * blockDim.x) {
    if (bc_mode != 0 && bmask[g]) {
      y[g] = (bc_mode == 1) ? x[g] : bc_value;
      continue;
    }
    T s = T(0);
    const int32_t k1 = toff[g + 1];
    for (int32_t k = toff[g]; k < k1; ++k) s += ye[tidx[k]];
    y[g] = s;
  }
}

template <typename T>
__global__ void scatter_init_kernel(const uint8_t* __restrict__ bmask, const T* __restrict__ x,
                                    int constrained, T* __restrict__ y, int64_t begin, int64_t n) {
#pragma unroll 4
  for (int64_t g = begin + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < n;
       g += int64_t(gridDim.x) * blockDim.x)
    y[g] = (constrained && bmask[g]) ? x[g] : T(0);
}

// Four dofs per thread: one 4-byte mask load and 16-byte stores (vectors aligned to
// 16 bytes, mask to 4).  Covers [0, 4 * n4).
__global__ void scatter_init_f64x4_kernel(const uint32_t* __restrict__ mask4,
                                          const double2* __restrict__ x2, int constrained,
                                          double2* __restrict__ y2, int64_t n4) {
  for (int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; w < n4;
       w += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t m = constrained ? mask4[w] : 0u;
    double2 lo = {0.0, 0.0}, hi = {0.0, 0.0};
    if (m) {
      const double2 xl = x2[2 * w], xh = x2[2 * w + 1];
      lo.x = (m & 0xffu) ? xl.x : 0.0;
      lo.y = (m & 0xff00u) ? xl.y : 0.0;
      hi.x = (m & 0xff0000u) ? xh.x : 0.0;
      hi.y = (m & 0xff000000u) ? xh.y : 0.0;
    }
    y2[2 * w] = lo;
    y2[2 * w + 1] = hi;
  }
}

__global__ void scatter_init_f32x4_kernel(const uint32_t* __restrict__ mask4,
                                          const float4* __restrict__ x4, int constrained,
                                          float4* __restrict__ y4, int64_t n4) {
  for (int64_t w = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; w < n4;
       w += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t m = constrained ? mask4[w] : 0u;
    float4 v = {0.f, 0.f, 0.f, 0.f};
    if (m) {
      const float4 xv = x4[w];
      v.x = (m & 0xffu) ? xv.x : 0.f;
      v.y = (m & 0xff00u) ? xv.y : 0.f;
      v.z = (m & 0xff0000u) ? xv.z : 0.f;
      v.w = (m & 0xff000000u) ? xv.w : 0.f;
    }
    y4[w] = v;
  }
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > (1 << 20)) g = 1 << 20;
  return int(g < 1 ? 1 : g);
}

}  // namespace

void launch_qdata(const DevSpace& sp, int kind, int q1d, const double* coeff, double scale,
                  double* qd, hipStream_t st) {
  if (sp.dim == 2) {
    launch_qdata_2d(sp, kind, q1d, coeff, scale, qd, st);
    HIP_LAUNCH_CHECK();
    return;
  }
  const TabView tv = tab_view(sp, q1d);
  const int NN = sp.ng * sp.ng * sp.ng;
  const size_t lds = sizeof(double) * (3 * NN + 2 * q1d * sp.ng);
  hipLaunchKernelGGL(qdata_kernel, dim3(unsigned(sp.ne)), dim3(256), lds, st, sp.gnodes,
                     sp.elem_orig, sp.ng, tv, q1d, kind, coeff, scale, qd, sp.status);
  HIP_LAUNCH_CHECK();
}

void launch_linear_form_evec(const DevSpace& sp, int q1d, int source, const double* fqp,
                             double scale, double* ye, hipStream_t st) {
  if (sp.dim == 2) {
    launch_linear_form_evec_2d(sp, q1d, source, fqp, scale, ye, st);
    HIP_LAUNCH_CHECK();
    return;
  }
  const TabView tv = tab_view(sp, q1d);
  const int NN = sp.ng * sp.ng * sp.ng, Q = q1d, D = sp.p + 1;
  const size_t lds = sizeof(double) * (3 * NN + 2 * Q * sp.ng + Q * D + Q * Q * Q + Q * Q * D +
                                       Q * D * D + D * D * D);
  hipLaunchKernelGGL(linear_form_kernel, dim3(unsigned(sp.ne)), dim3(256), lds, st, sp.gnodes,
                     sp.elem_orig, sp.ng, tv, Q, D, source, fqp, scale, ye);
  HIP_LAUNCH_CHECK();
}

void launch_diagonal_evec(const DevSpace& sp, int kind, int q1d, const double* qd, double* ye,
                          hipStream_t st) {
  if (sp.dim == 2) {
    launch_diagonal_evec_2d(sp, kind, q1d, qd, ye, st);
    HIP_LAUNCH_CHECK();
    return;
  }
  const TabView tv = tab_view(sp, q1d);
  const int Q = q1d, D = sp.p + 1;
  const size_t lds =
      sizeof(double) * (3 * Q * D + Q * Q * Q + Q * Q * D + Q * D * D + D * D * D);
  hipLaunchKernelGGL(diagonal_kernel, dim3(unsigned(sp.ne)), dim3(256), lds, st, tv, Q, D, kind,
                     qd, ye);
  HIP_LAUNCH_CHECK();
}

void launch_evec_gather(const DevSpace& sp, const double* ye, const double* x, int bc_mode,
                        double bc_value, double* y, hipStream_t st) {
  hipLaunchKernelGGL(evec_gather_kernel<double>, dim3(grid_for(sp.ndofs, 256)), dim3(256), 0, st,
                     sp.toff, sp.tidx, sp.bmask, ye, x, bc_mode, bc_value, y, sp.ndofs);
  HIP_LAUNCH_CHECK();
}

void launch_evec_gather_f32(const DevSpace& sp, const float* ye, const float* x, int bc_mode,
                            float* y, hipStream_t st) {
  hipLaunchKernelGGL(evec_gather_kernel<float>, dim3(grid_for(sp.ndofs, 256)), dim3(256), 0, st,
                     sp.toff, sp.tidx, sp.bmask, ye, x, bc_mode, 0.0f, y, sp.ndofs);
  HIP_LAUNCH_CHECK();
}

void launch_scatter_init(const DevSpace& sp, const double* x, bool constrained, double* y,
                         hipStream_t st) {
  const int64_t n = sp.ndofs;
  int64_t done = 0;
  if (aligned(x, 16) && aligned(y, 16) && aligned(sp.bmask, 4)) {
    const int64_t n4 = n / 4;
    if (n4 > 0)
      hipLaunchKernelGGL(scatter_init_f64x4_kernel, dim3(grid_for(n4, 256)), dim3(256), 0, st,
                         reinterpret_cast<const uint32_t*>(sp.bmask),
                         reinterpret_cast<const double2*>(x), int(constrained),
                         reinterpret_cast<double2*>(y), n4);
    done = 4 * n4;
  }
  if (done < n)
    hipLaunchKernelGGL(scatter_init_kernel<double>, dim3(grid_for(n - done, 256)), dim3(256), 0,
                       st, sp.bmask, x, int(constrained), y, done, n);
  HIP_LAUNCH_CHECK();
}

void launch_scatter_init_f32(const DevSpace& sp, const float* x, bool constrained, float* y,
                             hipStream_t st) {
  const int64_t n = sp.ndofs;
  int64_t done = 0;
  if (aligned(x, 16) && aligned(y, 16) && aligned(sp.bmask, 4)) {
    const int64_t n4 = n / 4;
    if (n4 > 0)
      hipLaunchKernelGGL(scatter_init_f32x4_kernel, dim3(grid_for(n4, 256)), dim3(256), 0, st,
                         reinterpret_cast<const uint32_t*>(sp.bmask),
                         reinterpret_cast<const float4*>(x), int(constrained),
                         reinterpret_cast<float4*>(y), n4);
    done = 4 * n4;
  }
  if (done < n)
    hipLaunchKernelGGL(scatter_init_kernel<float>, dim3(grid_for(n - done, 256)), dim3(256), 0,
                       st, sp.bmask, x, int(constrained), y, done, n);
  HIP_LAUNCH_CHECK();
}

}  // namespace pafem
