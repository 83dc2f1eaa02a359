// Partially assembled isotropic linear elasticity on the vector H1 space (the
// vector-valued integrators among the paper's GPU kernels, "GPU Acceleration"):
//
//   a(u, v) = int lambda (div u)(div v) + 2 mu eps(u) : eps(v),  eps(u) = (grad u + grad u^T)/2
//
// u and v have three components in the scalar H1 space, stored component-major
// (x[c * ndofs + i]).  Quadrature data per point (11 values): K = J^{-1} (K[b][d] =
// d xhat_b / d x_d, 9 values), w det J lambda and w det J mu.
//
// Same tiles and line-per-thread contractions as the scalar fused apply, but the
// point operation needs the gradients of all three components at once:
//   forward, per input component c: gather, x-lines, y-lines, z-lines; the z-line
//     thread keeps the reference gradient of u_c at its Q points in registers
//   point stage: F = ghat K (physical gradient), sigma = w det J (lambda tr F I +
//     mu (F + F^T)), output coefficients o = sigma K^T per point, in registers
//   backward, per output component c: z-lines (B, B, G), y-lines, x-lines of the
//     diffusion back contractions, summed per unique dof of the tile in LDS, one FP64
//     atomic per unique dof into y + c * ndofs (y pre-set by the init kernel: x on
//     essential dofs when constrained, 0 elsewhere)
#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

constexpr int kElasticValues = 11;

template <int P, int Q>
__global__ void __launch_bounds__(qdata_tile(Q) * Q * Q, P == 7 ? 2 : 1)
    elasticity_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                      const uint16_t* __restrict__ tile_slot, const double* __restrict__ tabB,
                      const double* __restrict__ tabG, const double* __restrict__ qd,
                      const double* __restrict__ x, double* __restrict__ y, int ne,
                      int constrained, int64_t nd) {
  constexpr int D = P + 1, DD = D * D, QQ = Q * Q, QQQ = QQ * Q, DDD = DD * D;
  constexpr int NE = qdata_tile(Q);
  constexpr int LC = D | 1;  // odd line stride
  constexpr int ELEM = 3 * QQ * LC;
  static_assert(2 * D <= 3 * Q, "x-line outputs must fit the element region");
  __shared__ double sW[NE * ELEM];
  __shared__ double sX[NE * DDD];

  const int tid = threadIdx.x;
  const int el = tid / QQ;
  const int r = tid - el * QQ;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int e = tile * NE + el;
  const bool act = e < ne;
  const int u0 = tile_off[tile];
  const int nu = tile_off[tile + 1] - u0;
  double* const W = sW + el * ELEM;
  // entry (c, qy, qx, dz) of the element region; x-line outputs (a, dz, dy, qx) at
  // c*Q + qy = a*D + dy
  auto at = [&](int c, int qy, int qx, int dz) -> double& {
    return W[((c * Q + qy) * Q + qx) * LC + dz];
  };
  // Row q (forward stages) or column d (back stages) of a 1D table.  At p = 7, 8 loaded
  // per loop iteration (opaque_ptr): loading every entry of the unrolled stages up front
  // overflowed the scalar registers (312 and 1784 spilled through VGPR lanes; p = 8 2.98 ->
  // 1.42 ms at 1e7 dofs; at p = 7 it also frees the registers for the two-wave launch
  // bound, 1.99 -> 1.23 ms).  At p = 5, 6, where 56-148 spill, the per-iteration loads
  // were 1-6% slower.
  constexpr bool OPQ = P >= 7;
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

  const bool xline = act && r < DD;  // x-line (dz, dy)
  const int xz = r / D, xy = r - (r / D) * D;
  const bool yline = act && r < D * Q;  // y-line (dz, qx)
  const int yz = r / Q, yx = r - (r / Q) * Q;
  const int zy = r / Q, zx = r - (r / Q) * Q;  // z-line (qy, qx)
  int slot[D];
  if (xline) {
    const uint16_t* sl = tile_slot + size_t(e) * DDD + r * D;
#pragma unroll
    for (int dx = 0; dx < D; ++dx) slot[dx] = sl[dx];
  }

  // g[c][qz][b]: reference derivative b of component c at the point (zx, zy, qz);
  // after the point stage, the coefficient of reference derivative b in output c
  double g[3][Q][3];

#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    const double* const xc = x + comp * nd;
    for (int s = tid; s < nu; s += NE * QQ) {
      const int gd = tile_dofs[u0 + s];
      sX[s] = (constrained && gd < 0) ? 0.0 : xc[gd < 0 ? ~gd : gd];
    }
    __syncthreads();
    if (xline) {
      double u[D];
#pragma unroll
      for (int dx = 0; dx < D; ++dx) u[dx] = sX[slot[dx]];
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        const auto rb = rowB(qx);
        const auto rg = rowG(qx);
        double b = 0.0, gg = 0.0;
#pragma unroll
        for (int dx = 0; dx < D; ++dx) {
          b += rb[dx] * u[dx];
          gg += rg[dx] * u[dx];
        }
        at(xy / Q, xy % Q, qx, xz) = b;
        at((D + xy) / Q, (D + xy) % Q, qx, xz) = gg;
      }
    }
    __syncthreads();
    if (yline) {
      double aB[D], aG[D];
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        aB[dy] = at(dy / Q, dy % Q, yx, yz);
        aG[dy] = at((D + dy) / Q, (D + dy) % Q, yx, yz);
      }
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        const auto rb = rowB(qy);
        const auto rg = rowG(qy);
        double gb = 0.0, bgv = 0.0, bb = 0.0;
#pragma unroll
        for (int dy = 0; dy < D; ++dy) {
          gb += rb[dy] * aG[dy];
          bgv += rg[dy] * aB[dy];
          bb += rb[dy] * aB[dy];
        }
        at(0, qy, yx, yz) = gb;
        at(1, qy, yx, yz) = bgv;
        at(2, qy, yx, yz) = bb;
      }
    }
    __syncthreads();
    if (act) {
      double c0[D], c1[D], c2[D];
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        c0[dz] = at(0, zy, zx, dz);
        c1[dz] = at(1, zy, zx, dz);
        c2[dz] = at(2, zy, zx, dz);
      }
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        const auto rb = rowB(qz);
        const auto rg = rowG(qz);
        double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          ux += rb[dz] * c0[dz];
          uy += rb[dz] * c1[dz];
          uz += rg[dz] * c2[dz];
        }
        g[comp][qz][0] = ux;
        g[comp][qz][1] = uy;
        g[comp][qz][2] = uz;
      }
    }
    // no barrier here: the next gather writes only sX, which nothing reads after the
    // x-lines, and the next x-lines write the element regions only after the barrier
    // that follows the gather, which every thread reaches after its z-line
  }

  // point stage
  if (act) {
    const double* qe = qd + size_t(tile) * kElasticValues * QQQ * NE + tid;
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      double K[3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          K[b][d] = __builtin_nontemporal_load(qe + ((3 * b + d) * Q + qz) * (NE * QQ));
      const double lw = __builtin_nontemporal_load(qe + (9 * Q + qz) * (NE * QQ));
      const double mw = __builtin_nontemporal_load(qe + (10 * Q + qz) * (NE * QQ));
      double F[3][3];  // F[c][d] = d u_c / d x_d
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          F[c][d] = g[c][qz][0] * K[0][d] + g[c][qz][1] * K[1][d] + g[c][qz][2] * K[2][d];
      const double ld = lw * (F[0][0] + F[1][1] + F[2][2]);
      double S[3][3];  // w det J sigma, symmetric
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) S[c][d] = mw * (F[c][d] + F[d][c]) + (c == d ? ld : 0.0);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          g[c][qz][b] = S[c][0] * K[b][0] + S[c][1] * K[b][1] + S[c][2] * K[b][2];
    }
  }

#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    // the previous component's scatter is done with sX and its x-lines with the regions
    __syncthreads();
    for (int s = tid; s < nu; s += NE * QQ) sX[s] = 0.0;
    if (act) {
      double t0[D], t1[D], t2[D];
#pragma unroll
      for (int dz = 0; dz < D; ++dz) t0[dz] = t1[dz] = t2[dz] = 0.0;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        const auto rb = rowB(qz);
        const auto rg = rowG(qz);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          t0[dz] += rb[dz] * g[comp][qz][0];
          t1[dz] += rb[dz] * g[comp][qz][1];
          t2[dz] += rg[dz] * g[comp][qz][2];
        }
      }
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        at(0, zy, zx, dz) = t0[dz];
        at(1, zy, zx, dz) = t1[dz];
        at(2, zy, zx, dz) = t2[dz];
      }
    }
    __syncthreads();
    if (yline) {
      double v0[Q], v1[Q], v2[Q];
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        v0[qy] = at(0, qy, yx, yz);
        v1[qy] = at(1, qy, yx, yz);
        v2[qy] = at(2, qy, yx, yz);
      }
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        const auto cb = colB(dy);
        const auto cg = colG(dy);
        double b = 0.0, gg = 0.0;
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          gg += cb[qy * D] * v0[qy];
          b += cg[qy * D] * v1[qy] + cb[qy * D] * v2[qy];
        }
        at(dy / Q, dy % Q, yx, yz) = b;
        at((D + dy) / Q, (D + dy) % Q, yx, yz) = gg;
      }
    }
    __syncthreads();
    if (xline) {
      double wB[Q], wG[Q];
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        wB[qx] = at(xy / Q, xy % Q, qx, xz);
        wG[qx] = at((D + xy) / Q, (D + xy) % Q, qx, xz);
      }
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        const auto cb = colB(dx);
        const auto cg = colG(dx);
        double acc = 0.0;
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) acc += cb[qx * D] * wB[qx] + cg[qx * D] * wG[qx];
        atomicAdd(&sX[slot[dx]], acc);
      }
    }
    __syncthreads();
    double* const yc = y + comp * nd;
    for (int s = tid; s < nu; s += NE * QQ) {
      const int gd = tile_dofs[u0 + s];
      if (!(constrained && gd < 0)) unsafeAtomicAdd(&yc[gd < 0 ? ~gd : gd], sX[s]);
    }
  }
}

template <int P>
void launch_elastic_order(const DevSpace& sp, bool constrained, const double* qd,
                          const double* x, double* y, hipStream_t st) {
  constexpr int Q = P + 2;
  constexpr int NE = qdata_tile(Q);
  const int nblk = int((sp.ne + NE - 1) / NE);
  const double* tabB = sp.tables + table_offset_doubles(Q, P + 1, sp.ng) + 2 * Q;
  const double* tabG = tabB + Q * (P + 1);
  hipLaunchKernelGGL((elasticity_kernel<P, Q>), dim3(nblk), dim3(NE * Q * Q), 0, st,
                     sp.tile_off, sp.tile_dofs, sp.tile_slot, tabB, tabG, qd, x, y, int(sp.ne),
                     int(constrained), int64_t(sp.ndofs));
}

}  // namespace

bool launch_elasticity(const DevSpace& sp, bool constrained, const double* qd, const double* x,
                       double* y, hipStream_t st) {
  switch (sp.p) {
    case 1: launch_elastic_order<1>(sp, constrained, qd, x, y, st); return true;
    case 2: launch_elastic_order<2>(sp, constrained, qd, x, y, st); return true;
    case 3: launch_elastic_order<3>(sp, constrained, qd, x, y, st); return true;
    case 4: launch_elastic_order<4>(sp, constrained, qd, x, y, st); return true;
    case 5: launch_elastic_order<5>(sp, constrained, qd, x, y, st); return true;
    case 6: launch_elastic_order<6>(sp, constrained, qd, x, y, st); return true;
    case 7: launch_elastic_order<7>(sp, constrained, qd, x, y, st); return true;
    case 8: launch_elastic_order<8>(sp, constrained, qd, x, y, st); return true;
    default: return false;
  }
}

}  // namespace pafem
