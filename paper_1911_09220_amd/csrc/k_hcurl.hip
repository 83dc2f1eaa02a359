// Partial-assembly action of the H(curl) mass and curl-curl forms on a Nedelec
// space of hexahedra ("Discrete de Rham Complex"; the H(curl) integrators among the
// partially assembled kernels of "GPU Acceleration"), y = G^t B^t D B G x with
//   B    per component a: the open 1D basis along axis a, the closed one along the
//        other two (value), and for the curl the closed basis' derivative along one
//        of the other two axes;
//   D    at each point the symmetric 3x3 w beta det J J^{-1} J^{-T} acting on the
//        reference field (mass) and w alpha J^T J / det J acting on the reference
//        curl (curl-curl), so that v_ref = D_m u_ref, w_ref = D_c curl_ref;
//   G    the tile's unique dofs with each element's orientation signs.
// Same tiles, quadrature-data layout and scatter as the H1 apply: one workgroup holds
// NE elements of one quadrature-data tile, Q*Q threads each; the tile's unique dofs
// are gathered once into LDS, element outputs are summed per unique dof in LDS and
// added with one FP64 atomic each.  Per component, the forward contractions run
// x -> y -> z one 1D line per thread; the z-line thread keeps the point values of all
// three components (field and curl) in registers, applies D there and starts the
// transposed contractions z -> y -> x.  Array bookkeeping: component a carries its
// value and, with the curl, one derivative array per axis b != a, created by the
// forward stage along b and merged back into the value by the transposed stage
// along b (the derivative arrays are kept in increasing axis order, so the one a
// stage creates or merges is always the last).
#include <type_traits>

#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

// Levi-Civita symbol for distinct indices (c, b, a)
__host__ __device__ constexpr int eps3(int c, int b, int a) {
  return ((b - c + 3) % 3 == 1) ? 1 : -1;
}
// the k-th axis (k = 0, 1) other than a
__host__ __device__ constexpr int other_axis(int a, int k) { return k < a ? k : k + 1; }

template <int P, int KIND, bool DOT>
__global__ void __launch_bounds__(qdata_tile(P + 2) * (P + 2) * (P + 2), P >= 5 ? 2 : 1)
    nd_apply_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                    const uint16_t* __restrict__ tile_slot, const int8_t* __restrict__ esign,
                    const double* __restrict__ tabB, const double* __restrict__ tabG,
                    const double* __restrict__ tabO, const double* __restrict__ qd,
                    const double* __restrict__ x, double* __restrict__ y,
                    double* __restrict__ dotp, int ne, int constrained) {
  constexpr int Q = P + 2, QQ = Q * Q, QQQ = Q * Q * Q;
  constexpr int DC = P + 1, DO = P;  // closed and open 1D sizes
  constexpr int NE = qdata_tile(Q);
  constexpr int NDE = 3 * DO * DC * DC;  // dofs per element
  constexpr int CB = DO * DC * DC;       // dofs per component block
  constexpr bool MASS = KIND != PAFEM_HCURL_CURLCURL;
  constexpr bool CURL = KIND != PAFEM_HCURL_MASS;
  constexpr int NCT = KIND == PAFEM_HCURL_MAXWELL ? 12 : 6;
  constexpr int CP0 = 0;                 // first pair of the curl D
  constexpr int MP0 = KIND == PAFEM_HCURL_MAXWELL ? 3 : 0;  // first pair of the mass D
  // One LDS region per element holds every intermediate of a component's contractions:
  // Q x DC columns (q, i2), each of RS rows.  The x contraction of line (i1, i2) writes
  // row k*n1 + i1 of columns (q, i2); the y contraction of line (q0, i2) reads those rows
  // of its own column and writes rows k*Q + q of the same column; the z contraction of
  // line (q0, q1) reads (and on the way back writes) row k*Q + q1 of the columns (q0, i2).
  // Every y-line thread reads all its inputs before writing, so the stages work in place
  // (LDS per element 3Q^2 DC instead of 2Q DC^2 + 3Q^2 DC: twice the workgroups per CU
  // at p >= 6).  RS is odd, so that y-line threads walking their columns hit distinct banks.
  constexpr int RS = (3 * Q) | 1;
  constexpr int REG = Q * DC * RS;
  static_assert(2 * DC <= RS && 3 * Q <= RS, "rows of a column");

  __shared__ double sR[NE * REG];
  __shared__ double sX[NE * NDE];

  const int tid = threadIdx.x;
  const int el = tid / QQ;
  const int r = tid - el * QQ;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int e = tile * NE + el;
  const bool act = e < ne;
  const int u0 = tile_off[tile];
  const int nu = tile_off[tile + 1] - u0;
  double* const R = sR + el * REG;
  auto at = [&](int col_q, int col_i2, int row) -> double& { return R[(col_i2 * Q + col_q) * RS + row]; };
  const uint16_t* const slots = tile_slot + size_t(e) * NDE;
  const int8_t* const signs = esign + size_t(e) * NDE;
  // Row q (forward stages, transposed z) or column d (transposed y and x) of a 1D
  // table.  At p = 8 loaded per loop iteration (opaque_ptr): loading every entry of the
  // unrolled stages up front overflows the scalar registers (spilled through VGPR lanes;
  // 0.797 -> 0.614 ms at 1e7 dofs).  At p = 3..7 the spills are smaller and the
  // per-iteration loads were 1-12% slower.
  constexpr int OPQ_MIN = 8;
  auto tab = [&](const double* t) {
    if constexpr (P >= OPQ_MIN)
      return opaque_ptr(t);
    else
      return t;
  };
  auto rowB = [&](int q) { return tab(tabB + q * DC); };
  auto rowG = [&](int q) { return tab(tabG + q * DC); };
  auto rowO = [&](int q) { return tab(tabO + q * DO); };
  auto colB = [&](int d) { return tab(tabB + d); };  // entry q at [q * DC]
  auto colG = [&](int d) { return tab(tabG + d); };
  auto colO = [&](int d) { return tab(tabO + d); };  // entry q at [q * DO]

  // G: the tile's unique dofs, essential ones read as 0 when constrained
  for (int s0 = tid; s0 < nu; s0 += 4 * NE * QQ) {
    int gg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * NE * QQ;
      gg[k] = s < nu ? tile_dofs[u0 + s] : 0;
    }
    double xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = gg[k];
      xv[k] = (s0 + k * NE * QQ < nu && !(constrained && g < 0)) ? x[g < 0 ? ~g : g] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s0 + k * NE * QQ < nu) sX[s0 + k * NE * QQ] = xv[k];
  }
  __syncthreads();

  // point values of this thread's z-line (qx, qy) = r: field (MASS) and curl (CURL)
  double uq[3][Q], cq[3][Q];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int q = 0; q < Q; ++q) uq[c][q] = cq[c][q] = 0.0;

  // ---------------- forward: one component at a time ----------------------------
  auto forward = [&](auto Atag) {
    constexpr int A = decltype(Atag)::value;
    constexpr int n0 = A == 0 ? DO : DC, n1 = A == 1 ? DO : DC, n2 = A == 2 ? DO : DC;
    constexpr int NX = 1 + ((CURL && A != 0) ? 1 : 0);  // arrays after the x contraction
    constexpr int NY = NX + ((CURL && A != 1) ? 1 : 0);  // after the y contraction
    // the previous component's z contraction has read the region
    if constexpr (A > 0) __syncthreads();
    // x contraction: line (i1, i2)
    if (act && r < n1 * n2) {
      const int i1 = r % n1, i2 = r / n1;
      double in[n0];
#pragma unroll
      for (int i0 = 0; i0 < n0; ++i0) {
        const int j = A * CB + i0 + n0 * (i1 + n1 * i2);
        in[i0] = double(signs[j]) * sX[slots[j]];
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const auto ro = rowO(q);
        const auto rb = rowB(q);
        const auto rg = rowG(q);
        double v = 0.0, d = 0.0;
#pragma unroll
        for (int i0 = 0; i0 < n0; ++i0) {
          if constexpr (A == 0) {
            v += ro[i0] * in[i0];
          } else {
            v += rb[i0] * in[i0];
            if constexpr (CURL) d += rg[i0] * in[i0];
          }
        }
        at(q, i2, i1) = v;
        if constexpr (NX == 2) at(q, i2, n1 + i1) = d;
      }
    }
    __syncthreads();
    // y contraction: line (q0, i2)
    if (act && r < Q * n2) {
      const int q0 = r % Q, i2 = r / Q;
      double in[NX][n1];
#pragma unroll
      for (int k = 0; k < NX; ++k)
#pragma unroll
        for (int i1 = 0; i1 < n1; ++i1) in[k][i1] = at(q0, i2, k * n1 + i1);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const auto ro = rowO(q);
        const auto rb = rowB(q);
        const auto rg = rowG(q);
        double out[NY];
#pragma unroll
        for (int k = 0; k < NY; ++k) out[k] = 0.0;
#pragma unroll
        for (int i1 = 0; i1 < n1; ++i1) {
          if constexpr (A == 1) {
#pragma unroll
            for (int k = 0; k < NX; ++k) out[k] += ro[i1] * in[k][i1];
          } else {
#pragma unroll
            for (int k = 0; k < NX; ++k) out[k] += rb[i1] * in[k][i1];
            if constexpr (CURL) out[NY - 1] += rg[i1] * in[0][i1];
          }
        }
#pragma unroll
        for (int k = 0; k < NY; ++k) at(q0, i2, k * Q + q) = out[k];
      }
    }
    __syncthreads();
    // z contraction: line (q0, q1) = r, into the point registers
    if (act) {
      const int q0 = r % Q, q1 = r / Q;
      double in[NY][n2];
#pragma unroll
      for (int k = 0; k < NY; ++k)
#pragma unroll
        for (int i2 = 0; i2 < n2; ++i2) in[k][i2] = at(q0, i2, k * Q + q1);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const auto ro = rowO(q);
        const auto rb = rowB(q);
        const auto rg = rowG(q);
        double out[NY + 1];
#pragma unroll
        for (int k = 0; k <= NY; ++k) out[k] = 0.0;
#pragma unroll
        for (int i2 = 0; i2 < n2; ++i2) {
          if constexpr (A == 2) {
#pragma unroll
            for (int k = 0; k < NY; ++k) out[k] += ro[i2] * in[k][i2];
          } else {
#pragma unroll
            for (int k = 0; k < NY; ++k) out[k] += rb[i2] * in[k][i2];
            if constexpr (CURL) out[NY] += rg[i2] * in[0][i2];
          }
        }
        if (MASS) uq[A][q] = out[0];
        if constexpr (CURL) {
          // derivative arrays along the two other axes, in increasing order
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int b = other_axis(A, k);
            const int c = 3 - A - b;
            cq[c][q] += double(eps3(c, b, A)) * out[1 + k];
          }
        }
      }
    }
  };
  forward(std::integral_constant<int, 0>{});
  forward(std::integral_constant<int, 1>{});
  forward(std::integral_constant<int, 2>{});

  // sX was last read by the x contraction of component 2, before the barrier that
  // precedes its y contraction: clear it for the per-unique-dof sums
  for (int s = tid; s < nu; s += NE * QQ) sX[s] = 0.0;

  // ---------------- D at the points ---------------------------------------------
  double energy = 0.0;
  if (act) {
    const double* const qe0 = qd + size_t(tile) * NCT * QQQ * NE + 2 * tid;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if constexpr (MASS) {
        double d[6];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          load_pair<double, double>(qe0 + 2 * (((MP0 + k) * Q + q) * (NE * QQ)), d[2 * k],
                                    d[2 * k + 1]);
        const double a0 = uq[0][q], a1 = uq[1][q], a2 = uq[2][q];
        const double v0 = d[0] * a0 + d[1] * a1 + d[2] * a2;
        const double v1 = d[1] * a0 + d[3] * a1 + d[4] * a2;
        const double v2 = d[2] * a0 + d[4] * a1 + d[5] * a2;
        if (DOT) energy += a0 * v0 + a1 * v1 + a2 * v2;
        uq[0][q] = v0;
        uq[1][q] = v1;
        uq[2][q] = v2;
      }
      if constexpr (CURL) {
        double d[6];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          load_pair<double, double>(qe0 + 2 * (((CP0 + k) * Q + q) * (NE * QQ)), d[2 * k],
                                    d[2 * k + 1]);
        const double a0 = cq[0][q], a1 = cq[1][q], a2 = cq[2][q];
        const double v0 = d[0] * a0 + d[1] * a1 + d[2] * a2;
        const double v1 = d[1] * a0 + d[3] * a1 + d[4] * a2;
        const double v2 = d[2] * a0 + d[4] * a1 + d[5] * a2;
        if (DOT) energy += a0 * v0 + a1 * v1 + a2 * v2;
        cq[0][q] = v0;
        cq[1][q] = v1;
        cq[2][q] = v2;
      }
    }
  }

  // ---------------- transposed contractions, one component at a time -------------
  auto back = [&](auto Atag) {
    constexpr int A = decltype(Atag)::value;
    constexpr int n0 = A == 0 ? DO : DC, n1 = A == 1 ? DO : DC, n2 = A == 2 ? DO : DC;
    // arrays after the transposed z contraction: the value and the derivatives along
    // the axes below 2 other than A; after the y one: those below 1
    constexpr int NZ = 1 + (CURL ? ((A == 2) ? 2 : 1) : 0);
    constexpr int NYB = 1 + (CURL ? ((A == 0) ? 0 : 1) : 0);
    // the previous component's transposed x contraction has read the region
    if constexpr (A > 0) __syncthreads();
    // z: thread (q0, q1); coefficients of the value and of d/d(axis b) at the points
    if (act) {
      const int q0 = r % Q, q1 = r / Q;
      double out[NZ][n2];
#pragma unroll
      for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int i2 = 0; i2 < n2; ++i2) out[k][i2] = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const auto ro = rowO(q);
        const auto rb = rowB(q);
        const auto rg = rowG(q);
        const double V = MASS ? uq[A][q] : 0.0;
        double Wd[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int b = other_axis(A, k);
          const int c = 3 - A - b;
          Wd[k] = CURL ? double(eps3(c, b, A)) * cq[c][q] : 0.0;
        }
#pragma unroll
        for (int i2 = 0; i2 < n2; ++i2) {
          if constexpr (A == 2) {
            out[0][i2] += ro[i2] * V;
            if constexpr (CURL) {
              out[1][i2] += ro[i2] * Wd[0];
              out[2][i2] += ro[i2] * Wd[1];
            }
          } else {
            // the derivative along z (the last of the two) merges into the value
            out[0][i2] += rb[i2] * V;
            if constexpr (CURL) {
              out[0][i2] += rg[i2] * Wd[1];
              out[1][i2] += rb[i2] * Wd[0];
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int i2 = 0; i2 < n2; ++i2) at(q0, i2, k * Q + q1) = out[k][i2];
    }
    __syncthreads();
    // y: line (q0, i2)
    if (act && r < Q * n2) {
      const int q0 = r % Q, i2 = r / Q;
      double in[NZ][Q];
#pragma unroll
      for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q) in[k][q] = at(q0, i2, k * Q + q);
#pragma unroll
      for (int i1 = 0; i1 < n1; ++i1) {
        const auto co = colO(i1);
        const auto cb = colB(i1);
        const auto cg = colG(i1);
        double out[NYB];
#pragma unroll
        for (int k = 0; k < NYB; ++k) out[k] = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if constexpr (A == 1) {
#pragma unroll
            for (int k = 0; k < NYB; ++k) out[k] += co[q * DO] * in[k][q];
          } else {
            // the derivative along y (the last array) merges into the value
            out[0] += cb[q * DC] * in[0][q];
            if constexpr (CURL) out[0] += cg[q * DC] * in[NZ - 1][q];
#pragma unroll
            for (int k = 1; k < NYB; ++k) out[k] += cb[q * DC] * in[k][q];
          }
        }
#pragma unroll
        for (int k = 0; k < NYB; ++k) at(q0, i2, k * n1 + i1) = out[k];
      }
    }
    __syncthreads();
    // x: line (i1, i2), then the signed sums per unique dof
    if (act && r < n1 * n2) {
      const int i1 = r % n1, i2 = r / n1;
      double in[NYB][Q];
#pragma unroll
      for (int k = 0; k < NYB; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q) in[k][q] = at(q, i2, k * n1 + i1);
#pragma unroll
      for (int i0 = 0; i0 < n0; ++i0) {
        const auto co = colO(i0);
        const auto cb = colB(i0);
        const auto cg = colG(i0);
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if constexpr (A == 0) {
            acc += co[q * DO] * in[0][q];
          } else {
            acc += cb[q * DC] * in[0][q];
            if constexpr (CURL) acc += cg[q * DC] * in[NYB - 1][q];
          }
        }
        const int j = A * CB + i0 + n0 * (i1 + n1 * i2);
        atomicAdd(&sX[slots[j]], double(signs[j]) * acc);
      }
    }
  };
  back(std::integral_constant<int, 0>{});
  back(std::integral_constant<int, 1>{});
  back(std::integral_constant<int, 2>{});

  if (DOT) {
    __shared__ double sDot[(qdata_tile(P + 2) * (P + 2) * (P + 2) + kWave - 1) / kWave];
    energy = block_sum(energy, sDot);
    if (tid == 0) dotp[blockIdx.x] = energy;
  }
  __syncthreads();
  // G^t: one global atomic per unique dof of the tile
  for (int s = tid; s < nu; s += NE * QQ) {
    const int g = tile_dofs[u0 + s];
    if (!(constrained && g < 0)) unsafeAtomicAdd(&y[g < 0 ? ~g : g], sX[s]);
  }
}

template <int P, int KIND, bool DOT>
void launch_nd_one(const DevSpace& sp, bool constrained, const double* qd, const double* x,
                   double* y, double* dotp, hipStream_t st) {
  constexpr int Q = P + 2;
  constexpr int NE = qdata_tile(Q);
  const int nblk = int((sp.ne + NE - 1) / NE);
  const double* tb = sp.tables + table_offset_doubles(Q, P + 1, sp.ng) + 2 * Q;
  const double* tg = tb + Q * (P + 1);
  const double* to = sp.tables_open + nd_open_offset(Q, P);
  hipLaunchKernelGGL((nd_apply_kernel<P, KIND, DOT>), dim3(nblk), dim3(NE * Q * Q), 0, st,
                     sp.tile_off, sp.tile_dofs, sp.tile_slot, sp.sign, tb, tg, to, qd, x, y, dotp,
                     int(sp.ne), int(constrained));
}

template <int P>
bool launch_nd_order(const DevSpace& sp, int kind, bool constrained, const double* qd,
                     const double* x, double* y, double* dotp, hipStream_t st) {
  switch (kind) {
    case PAFEM_HCURL_MASS:
      if (dotp) launch_nd_one<P, PAFEM_HCURL_MASS, true>(sp, constrained, qd, x, y, dotp, st);
      else launch_nd_one<P, PAFEM_HCURL_MASS, false>(sp, constrained, qd, x, y, dotp, st);
      return true;
    case PAFEM_HCURL_CURLCURL:
      if (dotp) launch_nd_one<P, PAFEM_HCURL_CURLCURL, true>(sp, constrained, qd, x, y, dotp, st);
      else launch_nd_one<P, PAFEM_HCURL_CURLCURL, false>(sp, constrained, qd, x, y, dotp, st);
      return true;
    case PAFEM_HCURL_MAXWELL:
      if (dotp) launch_nd_one<P, PAFEM_HCURL_MAXWELL, true>(sp, constrained, qd, x, y, dotp, st);
      else launch_nd_one<P, PAFEM_HCURL_MAXWELL, false>(sp, constrained, qd, x, y, dotp, st);
      return true;
    default:
      return false;
  }
}

}  // namespace

bool launch_nd_apply(const DevSpace& sp, int kind, int q1d, bool constrained, const double* qd,
                     const double* x, double* y, hipStream_t st, double* dotp) {
  if (sp.family != kFamilyND || q1d != sp.p + 2 || sp.sign == nullptr) return false;
  bool ok = false;
  switch (sp.p) {
    case 1: ok = launch_nd_order<1>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 2: ok = launch_nd_order<2>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 3: ok = launch_nd_order<3>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 4: ok = launch_nd_order<4>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 5: ok = launch_nd_order<5>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 6: ok = launch_nd_order<6>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 7: ok = launch_nd_order<7>(sp, kind, constrained, qd, x, y, dotp, st); break;
    case 8: ok = launch_nd_order<8>(sp, kind, constrained, qd, x, y, dotp, st); break;
    default: return false;
  }
  if (ok) {
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
      throw Error(PAFEM_EHIP, std::string("H(curl) apply launch: ") + hipGetErrorString(err));
  }
  return ok;
}

}  // namespace pafem
