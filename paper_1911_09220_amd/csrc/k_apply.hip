// Fused partial-assembly operator action y = G^t B^t D B G x for H1 mass and
// diffusion on hexahedra ("Operator Decomposition", "High-Order Partial
// Assembly").
//
// One workgroup holds NE elements; each element gets a Q x Q plane of threads
// (qx, qy) that walks the third direction in registers.  Per element:
//   G    gather x_E = x[gmap] into LDS (essential dofs read as 0 when constrained)
//   B    three one-axis contractions with the 1D tables (sum factorization):
//        x-axis through LDS, y-axis through LDS into registers, z-axis in registers
//   D    pointwise: 1 value (mass) or a symmetric 3x3 (diffusion) per point,
//        streamed from HBM once with non-temporal loads, issued before the gather
//   B^t  the transposed contractions in reverse order (z in registers, y and x
//        through LDS)
//   G^t  either hardware FP atomics into y (y pre-set by a init kernel) or a
//        plain store of the element vector for the deterministic transposed gather.
// Blocks are remapped so each XCD processes one contiguous range of elements.
#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

template <int Q>
constexpr int elems_per_block() {
  return (256 / (Q * Q)) > 0 ? (256 / (Q * Q)) : 1;
}

template <int P, int Q, int KIND, bool EVEC, typename TV, typename TD, typename TC>
__global__ void __launch_bounds__(elems_per_block<Q>() * Q * Q)
    pa_apply_kernel(const int32_t* __restrict__ gmap, const double* __restrict__ tabB,
                    const double* __restrict__ tabG, const TD* __restrict__ qd,
                    const TV* __restrict__ x, TV* __restrict__ y, int ne, int constrained) {
  constexpr int D = P + 1, QQ = Q * Q, QQQ = Q * Q * Q, DDD = D * D * D;
  constexpr int NE = elems_per_block<Q>();
  constexpr bool DIFF = (KIND == PAFEM_DIFFUSION);
  constexpr int NC = DIFF ? 6 : 1;   // stored values per quadrature point
  constexpr int NA = DIFF ? 2 : 1;   // x-contraction outputs (B, G)
  constexpr int NCC = DIFF ? 3 : 1;  // z^t-contraction outputs

  __shared__ TC sB[Q][D];
  __shared__ TC sG[Q][D];
  __shared__ TC sU[NE][D][D][D];
  __shared__ TC sA[NE][NA][D][D][Q];
  __shared__ TC sC[NE][NCC][D][Q][Q];

  const int tid = threadIdx.x;
  const int el = tid / QQ;
  const int r = tid - el * QQ;
  const int qx = r % Q, qy = r / Q;
  const int e = xcd_remap(blockIdx.x, gridDim.x) * NE + el;
  const bool act = e < ne;

  for (int i = tid; i < Q * D; i += NE * QQ) {
    (&sB[0][0])[i] = TC(tabB[i]);
    if (DIFF) (&sG[0][0])[i] = TC(tabG[i]);
  }

  // D for this thread's (qx, qy) column: issued first so the HBM stream overlaps
  // the gather and the forward contractions
  TC dq[Q][NC];
  if (act) {
    const TD* qe = qd + size_t(e) * NC * QQQ + r;
#pragma unroll
    for (int qz = 0; qz < Q; ++qz)
#pragma unroll
      for (int c = 0; c < NC; ++c) dq[qz][c] = load_value<TC, TD>(qe + c * QQQ + qz * QQ);
  }

  // G: gather
  int gidx[D];
  const bool dof_thread = act && qx < D && qy < D;
  if (dof_thread) {
    const int32_t* ge = gmap + size_t(e) * DDD + qy * D + qx;
#pragma unroll
    for (int dz = 0; dz < D; ++dz) {
      const int g = ge[dz * D * D];
      gidx[dz] = g;
      TC v = TC(0);
      if (!(constrained && g < 0)) v = TC(x[g < 0 ? ~g : g]);
      sU[el][dz][qy][qx] = v;
    }
  }
  __syncthreads();

  // B, x-axis: thread (qx, dy = qy)
  if (qy < D) {
#pragma unroll
    for (int dz = 0; dz < D; ++dz) {
      TC b = TC(0), g = TC(0);
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        const TC u = sU[el][dz][qy][dx];
        b += sB[qx][dx] * u;
        if (DIFF) g += sG[qx][dx] * u;
      }
      sA[el][0][dz][qy][qx] = b;
      if (DIFF) sA[el][NA - 1][dz][qy][qx] = g;
    }
  }
  __syncthreads();

  // B, y-axis into registers: thread (qx, qy)
  TC BB[D], GB[D], BG[D];
#pragma unroll
  for (int dz = 0; dz < D; ++dz) {
    TC bb = TC(0), gb = TC(0), bg = TC(0);
#pragma unroll
    for (int dy = 0; dy < D; ++dy) {
      const TC a0 = sA[el][0][dz][dy][qx];
      const TC by = sB[qy][dy];
      bb += by * a0;
      if (DIFF) {
        const TC a1 = sA[el][NA - 1][dz][dy][qx];
        gb += by * a1;
        bg += sG[qy][dy] * a0;
      }
    }
    BB[dz] = bb;
    GB[dz] = gb;
    BG[dz] = bg;
  }

  // B z-axis, D, B^t z-axis: all in registers
  TC tBB[D], tGB[D], tBG[D];
#pragma unroll
  for (int dz = 0; dz < D; ++dz) tBB[dz] = tGB[dz] = tBG[dz] = TC(0);
#pragma unroll
  for (int qz = 0; qz < Q; ++qz) {
    if (DIFF) {
      TC ux = TC(0), uy = TC(0), uz = TC(0);
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        const TC bz = sB[qz][dz], gz = sG[qz][dz];
        ux += bz * GB[dz];
        uy += bz * BG[dz];
        uz += gz * BB[dz];
      }
      const TC vx = dq[qz][0] * ux + dq[qz][1] * uy + dq[qz][2] * uz;
      const TC vy = dq[qz][1] * ux + dq[qz][3] * uy + dq[qz][4] * uz;
      const TC vz = dq[qz][2] * ux + dq[qz][4] * uy + dq[qz][5] * uz;
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        const TC bz = sB[qz][dz], gz = sG[qz][dz];
        tGB[dz] += bz * vx;
        tBG[dz] += bz * vy;
        tBB[dz] += gz * vz;
      }
    } else {
      TC u = TC(0);
#pragma unroll
      for (int dz = 0; dz < D; ++dz) u += sB[qz][dz] * BB[dz];
      const TC v = dq[qz][0] * u;
#pragma unroll
      for (int dz = 0; dz < D; ++dz) tBB[dz] += sB[qz][dz] * v;
    }
  }
#pragma unroll
  for (int dz = 0; dz < D; ++dz) {
    if (DIFF) {
      sC[el][0][dz][qy][qx] = tGB[dz];
      sC[el][1][dz][qy][qx] = tBG[dz];
      sC[el][2][dz][qy][qx] = tBB[dz];
    } else {
      sC[el][0][dz][qy][qx] = tBB[dz];
    }
  }
  __syncthreads();

  // B^t, y-axis: thread (qx, dy = qy)
  if (qy < D) {
#pragma unroll
    for (int dz = 0; dz < D; ++dz) {
      TC bx = TC(0), gx = TC(0);
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const TC by = sB[q2][qy];
        if (DIFF) {
          gx += by * sC[el][0][dz][q2][qx];
          bx += sG[q2][qy] * sC[el][1][dz][q2][qx] + by * sC[el][2][dz][q2][qx];
        } else {
          bx += by * sC[el][0][dz][q2][qx];
        }
      }
      sA[el][0][dz][qy][qx] = bx;
      if (DIFF) sA[el][NA - 1][dz][qy][qx] = gx;
    }
  }
  __syncthreads();

  // B^t, x-axis and G^t: thread (dx = qx, dy = qy)
  if (dof_thread) {
#pragma unroll
    for (int dz = 0; dz < D; ++dz) {
      TC acc = TC(0);
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        acc += sB[q1][qx] * sA[el][0][dz][qy][q1];
        if (DIFF) acc += sG[q1][qx] * sA[el][NA - 1][dz][qy][q1];
      }
      if (EVEC) {
        y[size_t(e) * DDD + dz * D * D + qy * D + qx] = TV(acc);
      } else {
        const int g = gidx[dz];
        if (!(constrained && g < 0)) unsafeAtomicAdd(&y[g < 0 ? ~g : g], TV(acc));
      }
    }
  }
}

template <int P, int KIND, bool EVEC, typename TV, typename TD, typename TC>
void launch_one(const DevSpace& sp, const double* tab, bool constrained, const void* qd,
                const void* x, void* out, hipStream_t st) {
  constexpr int Q = P + 2;
  constexpr int NE = elems_per_block<Q>();
  const int nblk = int((sp.ne + NE - 1) / NE);
  const double* tabB = tab + 2 * Q;
  const double* tabG = tabB + Q * (P + 1);
  hipLaunchKernelGGL((pa_apply_kernel<P, Q, KIND, EVEC, TV, TD, TC>), dim3(nblk),
                     dim3(NE * Q * Q), 0, st, sp.gmap, tabB, tabG,
                     static_cast<const TD*>(qd), static_cast<const TV*>(x),
                     static_cast<TV*>(out), int(sp.ne), int(constrained));
}

template <int P, int KIND, typename TV, typename TD, typename TC>
void launch_mode(const DevSpace& sp, const double* tab, bool constrained, bool evec,
                 const void* qd, const void* x, void* out, hipStream_t st) {
  if (evec)
    launch_one<P, KIND, true, TV, TD, TC>(sp, tab, constrained, qd, x, out, st);
  else
    launch_one<P, KIND, false, TV, TD, TC>(sp, tab, constrained, qd, x, out, st);
}

template <int P>
bool launch_order(const DevSpace& sp, int kind, int qdtype, int vdtype, const double* tab,
                  bool constrained, bool evec, const void* qd, const void* x, void* out,
                  hipStream_t st) {
  if (vdtype == PAFEM_F64 && qdtype == PAFEM_F64) {
    if (kind == PAFEM_DIFFUSION)
      launch_mode<P, PAFEM_DIFFUSION, double, double, double>(sp, tab, constrained, evec, qd, x,
                                                              out, st);
    else
      launch_mode<P, PAFEM_MASS, double, double, double>(sp, tab, constrained, evec, qd, x, out,
                                                         st);
    return true;
  }
  if (vdtype == PAFEM_F32 && qdtype == PAFEM_F32) {
    if (kind == PAFEM_DIFFUSION)
      launch_mode<P, PAFEM_DIFFUSION, float, float, float>(sp, tab, constrained, evec, qd, x, out,
                                                           st);
    else
      launch_mode<P, PAFEM_MASS, float, float, float>(sp, tab, constrained, evec, qd, x, out, st);
    return true;
  }
  if (vdtype == PAFEM_F32 && qdtype == PAFEM_BF16) {
    if (kind == PAFEM_DIFFUSION)
      launch_mode<P, PAFEM_DIFFUSION, float, bf16, float>(sp, tab, constrained, evec, qd, x, out,
                                                          st);
    else
      launch_mode<P, PAFEM_MASS, float, bf16, float>(sp, tab, constrained, evec, qd, x, out, st);
    return true;
  }
  return false;
}

}  // namespace

bool launch_pa_apply(const DevSpace& sp, int kind, int q1d, int qdtype, bool constrained,
                     bool evec, const void* qd, const void* x, void* out, int vdtype,
                     hipStream_t st) {
  if (q1d != sp.p + 2) return false;
  const double* tab = sp.tables + table_offset_doubles(q1d, sp.p + 1, sp.ng);
  bool ok = false;
  switch (sp.p) {
    case 1: ok = launch_order<1>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 2: ok = launch_order<2>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 3: ok = launch_order<3>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 4: ok = launch_order<4>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 5: ok = launch_order<5>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 6: ok = launch_order<6>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 7: ok = launch_order<7>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    case 8: ok = launch_order<8>(sp, kind, qdtype, vdtype, tab, constrained, evec, qd, x, out, st); break;
    default: ok = false;
  }
  if (ok) {
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
      throw Error(PAFEM_EHIP, std::string("apply launch: ") + hipGetErrorString(err));
  }
  return ok;
}

}  // namespace pafem
