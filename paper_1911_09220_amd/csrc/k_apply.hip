// Fused partial-assembly operator action y = G^t B^t D B G x for H1 mass and
// diffusion on hexahedra ("Operator Decomposition", "High-Order Partial
// Assembly").
//
// One workgroup holds NE elements; each element gets a Q x Q plane of threads
// (qx, qy) that walks the third direction in registers.  Per element:
//   G    gather the tile's unique dofs once into LDS (essential dofs read as 0 when
//        constrained) and expand them to the element nodes through a slot map
//   B    three one-axis contractions with the 1D tables (sum factorization):
//        x-axis through LDS, y-axis through LDS into registers, z-axis in registers
//   D    pointwise: 1 value (mass) or a symmetric 3x3 (diffusion) per point,
//        streamed from HBM once with non-temporal loads, issued before the gather
//   B^t  the transposed contractions in reverse order (z in registers, y and x
//        through LDS)
//   G^t  either: sum the element outputs per unique dof of the tile in LDS, then one
//        hardware FP atomic per unique dof into y (y pre-set by an init kernel); or
//        a plain store of the element vector for the deterministic transposed gather.
// Blocks are remapped so each XCD processes one contiguous range of elements.
#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

// one workgroup = one tile of the tile-interleaved quadrature data
template <int Q>
constexpr int elems_per_block() {
  return qdata_tile(Q);
}

template <int P, int Q, int KIND, bool EVEC, typename TV, typename TD, typename TC>
__global__ void __launch_bounds__(elems_per_block<Q>() * Q * Q)
    pa_apply_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                    const uint16_t* __restrict__ tile_slot, const double* __restrict__ tabB,
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

  // The tile's unique dofs: x is gathered once per unique dof into sX, and the
  // element outputs are summed per unique dof in sY before one global atomic
  // per unique dof.  sX aliases sC (not live before the z-loop ends), sY aliases
  // sU (not live after the x-contraction).
  TC* const sX = &sC[0][0][0][0][0];
  TC* const sY = &sU[0][0][0][0];

  const int tid = threadIdx.x;
  const int el = tid / QQ;
  const int r = tid - el * QQ;
  const int qx = r % Q, qy = r / Q;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int e = tile * NE + el;
  const bool act = e < ne;
  const int u0 = tile_off[tile];
  const int nu = tile_off[tile + 1] - u0;

  for (int i = tid; i < Q * D; i += NE * QQ) {
    (&sB[0][0])[i] = TC(tabB[i]);
    if (DIFF) (&sG[0][0])[i] = TC(tabG[i]);
  }

  // D for this thread's (qx, qy) column: issued first so the HBM stream overlaps
  // the gather and the forward contractions
  // (tile-interleaved: for each (c, qz) the workgroup reads one contiguous run)
  TC dq[Q][NC];
  if (act) {
    const TD* qe = qd + size_t(e / NE) * NC * QQQ * NE + tid;
#pragma unroll
    for (int qz = 0; qz < Q; ++qz)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        dq[qz][c] = load_value<TC, TD>(qe + (c * Q + qz) * (NE * QQ));
  }

  // G: gather the tile's unique dofs, then expand to the element nodes
  // four unique dofs per thread per step keep several gathers in flight
  for (int s0 = tid; s0 < nu; s0 += 4 * NE * QQ) {
    int gg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * NE * QQ;
      gg[k] = s < nu ? tile_dofs[u0 + s] : 0;
    }
    TC xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = gg[k];
      xv[k] = (s0 + k * NE * QQ < nu && !(constrained && g < 0)) ? TC(x[g < 0 ? ~g : g]) : TC(0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s0 + k * NE * QQ < nu) sX[s0 + k * NE * QQ] = xv[k];
  }
  int slot[D];
  const bool dof_thread = act && qx < D && qy < D;
  if (dof_thread) {
    const uint16_t* sl = tile_slot + size_t(e) * DDD + qy * D + qx;
#pragma unroll
    for (int dz = 0; dz < D; ++dz) slot[dz] = sl[dz * D * D];
  }
  __syncthreads();
  if (dof_thread) {
#pragma unroll
    for (int dz = 0; dz < D; ++dz) sU[el][dz][qy][qx] = sX[slot[dz]];
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

  // sU is dead from here on: clear the per-unique-dof accumulators it now holds
  if (!EVEC)
    for (int s = tid; s < nu; s += NE * QQ) sY[s] = TC(0);

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
      if (EVEC)
        y[size_t(e) * DDD + dz * D * D + qy * D + qx] = TV(acc);
      else
        atomicAdd(&sY[slot[dz]], acc);
    }
  }
  if (EVEC) return;
  __syncthreads();
  // G^t: one global atomic per unique dof of the tile
#pragma unroll 4
  for (int s = tid; s < nu; s += NE * QQ) {
    const int g = tile_dofs[u0 + s];
    if (!(constrained && g < 0)) unsafeAtomicAdd(&y[g < 0 ? ~g : g], TV(sY[s]));
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
                     dim3(NE * Q * Q), 0, st, sp.tile_off, sp.tile_dofs, sp.tile_slot, tabB, tabG,
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
