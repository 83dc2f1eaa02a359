// Partial assembly on quadrilaterals ("High-Order Partial Assembly" in 2D, the
// setting of the paper's GPU experiment): quadrature data, load vector, diagonal
// and the fused apply y = G^t B^t D B G x for H1 mass and diffusion.
//
// Apply: one workgroup of 256 threads holds one tile of NE = floor(256/Q) elements
// (the tile of the tile-interleaved quadrature data, [c][qy][element][qx]); each
// element gets Q threads.  As in 3D every contraction is one 1D line per thread with
// wave-uniform table entries:
//   G    gather the tile's unique dofs once into LDS (essential dofs read as 0 when
//        constrained)
//   B    x-lines: thread dy (< D) contracts its row of D values into Q values along x
//        (B and G tables), written to LDS
//   D    y-lines: thread qx reads its column of D values per array, contracts along y
//        to the two derivatives at its Q points, applies the symmetric 2x2 D (loaded
//        with non-temporal loads before the gather) and contracts back along y in
//        registers, writing in place the entries it read
//   B^t  x-lines again: thread dy produces its D outputs
//   G^t  summed per unique dof of the tile in LDS, then one FP64 atomic per unique dof
//        into y (pre-set by the init kernel: x on essential dofs when constrained)
// With DOT each workgroup writes the sum of its elements' energies (B G u) . D (B G u)
// for the CG step length.
#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

constexpr int k2dThreads = 256;

struct Tab2 {
  const double *wts, *B, *G, *Bg, *Gg;
};

Tab2 tab2(const DevSpace& sp, int Q) {
  const int D = sp.p + 1;
  const double* t = sp.tables + table_offset_doubles(Q, D, sp.ng);
  Tab2 v;
  v.wts = t + Q;
  v.B = t + 2 * Q;
  v.G = v.B + Q * D;
  v.Bg = v.G + Q * D;
  v.Gg = v.Bg + Q * sp.ng;
  return v;
}

// J at (qx, qy) from the 4 lexicographic corners X[c][a] of a bilinear element
__device__ __forceinline__ void jacobian2d(const double* X, const double* Bg, const double* Gg,
                                           int qx, int qy, double J[2][2], double x[2]) {
  for (int a = 0; a < 2; ++a) {
    double j0 = 0.0, j1 = 0.0, v = 0.0;
    for (int k2 = 0; k2 < 2; ++k2)
      for (int k1 = 0; k1 < 2; ++k1) {
        const double xa = X[(k1 + 2 * k2) * 2 + a];
        j0 += xa * Gg[qx * 2 + k1] * Bg[qy * 2 + k2];
        j1 += xa * Bg[qx * 2 + k1] * Gg[qy * 2 + k2];
        v += xa * Bg[qx * 2 + k1] * Bg[qy * 2 + k2];
      }
    J[a][0] = j0;
    J[a][1] = j1;
    x[a] = v;
  }
}

// one thread per (device element, point)
__global__ void qdata2d_kernel(const double* __restrict__ gnodes, const int32_t* __restrict__ orig,
                               Tab2 tv, int Q, int kind, const double* __restrict__ coeff,
                               double scale, double* __restrict__ qd, int32_t* status, int64_t ne) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= ne * Q * Q) return;
  const int64_t e = i / (Q * Q);
  const int q = int(i - e * Q * Q), qx = q % Q, qy = q / Q;
  double J[2][2], x[2];
  jacobian2d(gnodes + e * 8, tv.Bg, tv.Gg, qx, qy, J, x);
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  if (!(det > 0.0)) atomicMin(&status[0], orig[e]);
  const double w = tv.wts[qx] * tv.wts[qy];
  const double c = scale * (coeff ? coeff[size_t(orig[e]) * Q * Q + q] : 1.0);
  if (kind == PAFEM_MASS) {
    qd[qdata_index_2d(e, 0, q, Q, 1)] = w * c * det;
  } else {
    // alpha kappa det J J^-1 J^-T = alpha kappa adj(J) adj(J)^T / det J,
    // adj(J) = [[J11, -J01], [-J10, J00]]
    const double f = w * c / det;
    qd[qdata_index_2d(e, 0, q, Q, 3)] = f * (J[1][1] * J[1][1] + J[0][1] * J[0][1]);
    qd[qdata_index_2d(e, 1, q, Q, 3)] = -f * (J[1][1] * J[1][0] + J[0][1] * J[0][0]);
    qd[qdata_index_2d(e, 2, q, Q, 3)] = f * (J[1][0] * J[1][0] + J[0][0] * J[0][0]);
  }
}

// element load vectors ye [device element][D^2]; one wave per element
__global__ void linear_form2d_kernel(const double* __restrict__ gnodes,
                                     const int32_t* __restrict__ orig, Tab2 tv, int Q, int D,
                                     int source, const double* __restrict__ fqp, double scale,
                                     double* __restrict__ ye) {
  extern __shared__ double smem[];
  const int64_t e = blockIdx.x;
  double* F = smem;          // [qy][qx]
  double* T = F + Q * Q;     // [qy][i1]
  const double pi = 3.14159265358979323846;
  for (int q = threadIdx.x; q < Q * Q; q += blockDim.x) {
    const int qx = q % Q, qy = q / Q;
    double J[2][2], x[2];
    jacobian2d(gnodes + e * 8, tv.Bg, tv.Gg, qx, qy, J, x);
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double f;
    if (source == PAFEM_SOURCE_ARRAY)
      f = scale * fqp[size_t(orig[e]) * Q * Q + q];
    else if (source == PAFEM_SOURCE_CONST)
      f = scale;
    else
      f = scale * 2.0 * pi * pi * sin(pi * x[0]) * sin(pi * x[1]);
    F[q] = tv.wts[qx] * tv.wts[qy] * det * f;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < Q * D; k += blockDim.x) {
    const int i1 = k % D, qy = k / D;
    double s = 0.0;
    for (int qx = 0; qx < Q; ++qx) s += tv.B[qx * D + i1] * F[qy * Q + qx];
    T[k] = s;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < D * D; k += blockDim.x) {
    const int i1 = k % D, i2 = k / D;
    double s = 0.0;
    for (int qy = 0; qy < Q; ++qy) s += tv.B[qy * D + i2] * T[qy * D + i1];
    ye[e * D * D + k] = s;
  }
}

// element diagonals ye [device element][D^2]: sum_q grad phi_i . D grad phi_i (or
// D phi_i^2 for mass), one thread per (element, dof)
__global__ void diagonal2d_kernel(Tab2 tv, int Q, int D, int kind, const double* __restrict__ qd,
                                  double* __restrict__ ye, int64_t ne) {
  const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (k >= ne * D * D) return;
  const int64_t e = k / (D * D);
  const int i = int(k - e * D * D), i1 = i % D, i2 = i / D;
  double s = 0.0;
  for (int qy = 0; qy < Q; ++qy)
    for (int qx = 0; qx < Q; ++qx) {
      const int q = qx + Q * qy;
      const double bx = tv.B[qx * D + i1], by = tv.B[qy * D + i2];
      if (kind == PAFEM_MASS) {
        s += qd[qdata_index_2d(e, 0, q, Q, 1)] * (bx * by) * (bx * by);
      } else {
        const double gx = tv.G[qx * D + i1] * by, gy = bx * tv.G[qy * D + i2];
        s += qd[qdata_index_2d(e, 0, q, Q, 3)] * gx * gx +
             2.0 * qd[qdata_index_2d(e, 1, q, Q, 3)] * gx * gy +
             qd[qdata_index_2d(e, 2, q, Q, 3)] * gy * gy;
      }
    }
  ye[k] = s;
}

template <int Q>
constexpr int elems2d() {
  return qdata_tile_2d(Q);
}

template <int P, int Q, int KIND, bool DOT>
__global__ void __launch_bounds__(k2dThreads)
    pa_apply2d_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                      const uint16_t* __restrict__ tile_slot, const double* __restrict__ tabB,
                      const double* __restrict__ tabG, const double* __restrict__ qd,
                      const double* __restrict__ x, double* __restrict__ y,
                      double* __restrict__ dotp, int ne, int constrained) {
  constexpr int D = P + 1, DD = D * D;
  constexpr int NE = elems2d<Q>();
  static_assert(NE * Q <= k2dThreads, "tile does not fit the workgroup");
  constexpr bool DIFF = (KIND == PAFEM_DIFFUSION);
  constexpr int NC = DIFF ? 3 : 1;  // stored values per point
  constexpr int NA = DIFF ? 2 : 1;  // arrays between the stages
  // row stride: odd (no bank conflicts between rows) while the tile fits 3 workgroups per CU
  constexpr int LQ = (Q | 1) * NA * D * NE * 8 + NE * DD * 8 <= 52 * 1024 ? (Q | 1) : Q;
  constexpr int ELEM = NA * D * LQ;

  __shared__ double sW[NE * ELEM];
  __shared__ double sX[NE * DD];

  const int tid = threadIdx.x;
  const int el = tid / Q;
  const int r = tid - el * Q;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int e = tile * NE + el;
  const bool act = tid < NE * Q && e < ne;
  const int u0 = tile_off[tile];
  const int nu = tile_off[tile + 1] - u0;
  double* const W = sW + (act ? el : 0) * ELEM;
  auto at = [&](int a, int dy, int qx) -> double& { return W[(a * D + dy) * LQ + qx]; };
  // Row q (forward stages) or column d (back stage) of a 1D table.  At p = 8 loaded per
  // loop iteration (opaque_ptr): up front, the compiler spilled the 180 entries through
  // VGPR lanes (1248 lane reads per wave against 750 FMAs).
  constexpr bool OPQ = P >= 8;
  auto tab = [&](const double* t) {
    if constexpr (OPQ)
      return opaque_ptr(t);
    else
      return t;
  };
  auto rowB = [&](int q) { return tab(tabB + q * D); };
  auto rowG = [&](int q) { return tab(tabG + q * D); };
  auto colB = [&](int d) { return tab(tabB + d); };
  auto colG = [&](int d) { return tab(tabG + d); };

  // D of this thread's column qx = r
  double dq[Q][NC];
  if (act) {
    const double* qe = qd + size_t(tile) * NC * Q * NE * Q + tid;
#pragma unroll
    for (int qy = 0; qy < Q; ++qy)
#pragma unroll
      for (int c = 0; c < NC; ++c) dq[qy][c] = __builtin_nontemporal_load(qe + (c * Q + qy) * (NE * Q));
  }

  // G: the tile's unique dofs
  for (int s0 = tid; s0 < nu; s0 += 4 * k2dThreads) {
    int gg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * k2dThreads;
      gg[k] = s < nu ? tile_dofs[u0 + s] : 0;
    }
    double xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = gg[k];
      xv[k] = (s0 + k * k2dThreads < nu && !(constrained && g < 0)) ? x[g < 0 ? ~g : g] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s0 + k * k2dThreads < nu) sX[s0 + k * k2dThreads] = xv[k];
  }
  const bool xline = act && r < D;
  int slot[D];
  if (xline) {
    const uint16_t* sl = tile_slot + size_t(e) * DD + r * D;
#pragma unroll
    for (int dx = 0; dx < D; ++dx) slot[dx] = sl[dx];
  }
  __syncthreads();

  // B (and G) along x: thread dy = r
  if (xline) {
    double u[D];
#pragma unroll
    for (int dx = 0; dx < D; ++dx) u[dx] = sX[slot[dx]];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      const auto rb = rowB(qx);
      const auto rg = rowG(qx);
      double b = 0.0, g = 0.0;
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        b += rb[dx] * u[dx];
        if (DIFF) g += rg[dx] * u[dx];
      }
      at(0, r, qx) = b;
      if (DIFF) at(1, r, qx) = g;
    }
  }
  __syncthreads();
  for (int s = tid; s < nu; s += k2dThreads) sX[s] = 0.0;

  // along y, D, back along y: thread qx = r
  double energy = 0.0;
  if (act) {
    double a0[D], a1[D], t0[D], t1[D];
#pragma unroll
    for (int dy = 0; dy < D; ++dy) {
      a0[dy] = at(0, dy, r);
      if (DIFF) a1[dy] = at(1, dy, r);
      t0[dy] = t1[dy] = 0.0;
    }
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      const auto rb = rowB(qy);
      const auto rg = rowG(qy);
      if constexpr (DIFF) {
        double ux = 0.0, uy = 0.0;
#pragma unroll
        for (int dy = 0; dy < D; ++dy) {
          ux += rb[dy] * a1[dy];  // G along x, B along y
          uy += rg[dy] * a0[dy];  // B along x, G along y
        }
        const double vx = dq[qy][0] * ux + dq[qy][1] * uy;
        const double vy = dq[qy][1] * ux + dq[qy][2] * uy;
        if (DOT) energy += ux * vx + uy * vy;
#pragma unroll
        for (int dy = 0; dy < D; ++dy) {
          t1[dy] += rb[dy] * vx;
          t0[dy] += rg[dy] * vy;
        }
      } else {
        double u = 0.0;
#pragma unroll
        for (int dy = 0; dy < D; ++dy) u += rb[dy] * a0[dy];
        const double v = dq[qy][0] * u;
        if (DOT) energy += u * v;
#pragma unroll
        for (int dy = 0; dy < D; ++dy) t0[dy] += rb[dy] * v;
      }
    }
#pragma unroll
    for (int dy = 0; dy < D; ++dy) {
      at(0, dy, r) = t0[dy];
      if (DIFF) at(1, dy, r) = t1[dy];
    }
  }
  __syncthreads();

  // back along x and G^t into the tile's unique dofs: thread dy = r
  if (xline) {
    double w0[Q], w1[Q];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      w0[qx] = at(0, r, qx);
      if (DIFF) w1[qx] = at(1, r, qx);
    }
#pragma unroll
    for (int dx = 0; dx < D; ++dx) {
      const auto cb = colB(dx);
      const auto cg = colG(dx);
      double acc = 0.0;
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        acc += cb[qx * D] * w0[qx];
        if (DIFF) acc += cg[qx * D] * w1[qx];
      }
      atomicAdd(&sX[slot[dx]], acc);
    }
  }
  if (DOT) {
    __shared__ double sDot[k2dThreads / kWave];
    energy = block_sum(energy, sDot);
    if (tid == 0) dotp[blockIdx.x] = energy;
  }
  __syncthreads();
#pragma unroll 4
  for (int s = tid; s < nu; s += k2dThreads) {
    const int g = tile_dofs[u0 + s];
    if (!(constrained && g < 0)) unsafeAtomicAdd(&y[g < 0 ? ~g : g], sX[s]);
  }
}

template <int P, int KIND, bool DOT>
void launch2d(const DevSpace& sp, bool constrained, const double* qd, const double* x, double* y,
              double* dotp, hipStream_t st) {
  constexpr int Q = P + 2;
  constexpr int NE = elems2d<Q>();
  const int nblk = int((sp.ne + NE - 1) / NE);
  const Tab2 tv = tab2(sp, Q);
  hipLaunchKernelGGL((pa_apply2d_kernel<P, Q, KIND, DOT>), dim3(nblk), dim3(k2dThreads), 0, st,
                     sp.tile_off, sp.tile_dofs, sp.tile_slot, tv.B, tv.G, qd, x, y, dotp,
                     int(sp.ne), int(constrained));
}

template <int P>
void launch2d_order(const DevSpace& sp, int kind, bool constrained, const double* qd,
                    const double* x, double* y, double* dotp, hipStream_t st) {
  if (kind == PAFEM_DIFFUSION) {
    if (dotp)
      launch2d<P, PAFEM_DIFFUSION, true>(sp, constrained, qd, x, y, dotp, st);
    else
      launch2d<P, PAFEM_DIFFUSION, false>(sp, constrained, qd, x, y, dotp, st);
  } else {
    if (dotp)
      launch2d<P, PAFEM_MASS, true>(sp, constrained, qd, x, y, dotp, st);
    else
      launch2d<P, PAFEM_MASS, false>(sp, constrained, qd, x, y, dotp, st);
  }
}

}  // namespace

void launch_qdata_2d(const DevSpace& sp, int kind, int q1d, const double* coeff, double scale,
                     double* qd, hipStream_t st) {
  const int64_t n = sp.ne * q1d * q1d;
  hipLaunchKernelGGL(qdata2d_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, sp.gnodes,
                     sp.elem_orig, tab2(sp, q1d), q1d, kind, coeff, scale, qd, sp.status, sp.ne);
}

void launch_linear_form_evec_2d(const DevSpace& sp, int q1d, int source, const double* fqp,
                                double scale, double* ye, hipStream_t st) {
  const int D = sp.p + 1;
  const size_t lds = sizeof(double) * (q1d * q1d + q1d * D);
  hipLaunchKernelGGL(linear_form2d_kernel, dim3(unsigned(sp.ne)), dim3(64), lds, st, sp.gnodes,
                     sp.elem_orig, tab2(sp, q1d), q1d, D, source, fqp, scale, ye);
}

void launch_diagonal_evec_2d(const DevSpace& sp, int kind, int q1d, const double* qd, double* ye,
                             hipStream_t st) {
  const int D = sp.p + 1;
  const int64_t n = sp.ne * D * D;
  hipLaunchKernelGGL(diagonal2d_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
                     tab2(sp, q1d), q1d, D, kind, qd, ye, sp.ne);
}

int pa_apply2d_blocks(const DevSpace& sp) {
  const int NE = qdata_tile_2d(sp.p + 2);
  return int((sp.ne + NE - 1) / NE);
}

bool launch_pa_apply_2d(const DevSpace& sp, int kind, bool constrained, const double* qd,
                        const double* x, double* y, hipStream_t st, double* dotp) {
  switch (sp.p) {
    case 1: launch2d_order<1>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 2: launch2d_order<2>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 3: launch2d_order<3>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 4: launch2d_order<4>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 5: launch2d_order<5>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 6: launch2d_order<6>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 7: launch2d_order<7>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 8: launch2d_order<8>(sp, kind, constrained, qd, x, y, dotp, st); break;
    default: return false;
  }
  return true;
}

}  // namespace pafem
