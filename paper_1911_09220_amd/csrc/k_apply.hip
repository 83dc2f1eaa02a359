// Fused partial-assembly operator action y = G^t B^t D B G x for H1 mass and
// diffusion on hexahedra ("Operator Decomposition", "High-Order Partial
// Assembly"), and on the same skeleton the other integrators of "GPU Acceleration":
// diffusion with recomputed geometry, convection, gradient (vector output; from
// p = 5 one pass per component), divergence (vector input) and the three-component
// vector forms of mass and diffusion (elasticity has its own kernel, k_elastic.hip).
//
// One workgroup holds NE elements (one tile of the tile-interleaved quadrature
// data); each element gets Q*Q threads.  Every contraction is done one 1D line per
// thread: a thread loads the D (or Q) inputs of its line into registers and
// produces all Q (or D) outputs of that line, so the 1D table entries it multiplies
// by are the same for every thread of the wave and are read as scalars, and each
// intermediate value passes through LDS once.  Per element:
//   G    gather the tile's unique dofs once into LDS (essential dofs read as 0 when
//        constrained); a thread owning the x-line (dz, dy) picks its D values
//        through the tile slot map.  The index lists are read once per apply and
//        loaded non-temporally; at p <= 4 every thread keeps the dof ids it gathered
//        for the scatter instead of reading the list again
//   B    x-lines (dz, dy) -> y-lines (dz, qx) -> z-lines (qy, qx)
//   D    pointwise on the z-line: 1 value (mass) or a symmetric 3x3 (diffusion) per
//        point, streamed from HBM with non-temporal loads issued before the gather
//        (at some orders only the first planes, the rest one z-iteration ahead)
//   B^t  z-lines (in registers) -> y-lines -> x-lines
//   G^t  either: sum the element outputs per unique dof of the tile in LDS, then one
//        hardware FP atomic per unique dof into y (y pre-set by an init kernel); or
//        a plain store of the element vector for the deterministic transposed gather.
// With DOT, each workgroup also writes the sum of its elements' energies
// u_E . (A_E u_E) (u_E the gathered input, essential entries 0 when constrained) to
// dotp[blockIdx.x], taken at the quadrature points as the sum of (B G u) . D (B G u):
// the x.Ax of the CG step without another pass over x and y.
// All intermediate arrays of an element share one LDS region: every stage writes
// only entries that the same thread has just read, so a region of 3*Q*Q lines of
// D values (1*Q*Q for mass) holds them all.
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

template <int P, int Q, int KIND, bool EVEC, bool DOT, typename TV, typename TD, typename TC>
__global__ void __launch_bounds__(elems_per_block<Q>() * Q * Q, KIND != PAFEM_DIFFUSION ? 1 : sizeof(TC) == 4 ? (P == 6 ? 5 : 1) : (P == 4 || P == 5) ? 4 : P == 2 ? 5 : P >= 6 ? 3 : 1)
    pa_apply_kernel(const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_dofs,
                    const uint16_t* __restrict__ tile_slot, const TC* __restrict__ tabB,
                    const TC* __restrict__ tabG, const TD* __restrict__ qd,
                    const TV* __restrict__ x, TV* __restrict__ y, double* __restrict__ dotp,
                    const double* __restrict__ gnodes, const TC* __restrict__ tabBg,
                    const TC* __restrict__ tabGg, int ne, int constrained, int64_t ystride) {
  constexpr int D = P + 1, DD = D * D, QQ = Q * Q, QQQ = Q * Q * Q, DDD = D * D * D;
  constexpr int NE = elems_per_block<Q>();
  // GEOM: diffusion storing alpha kappa per point; J recomputed from the 8 corners
  // kinds from kVectorKind on: the same operator on each of 3 components (x and y hold
  // 3 vectors at stride ystride), D read once and kept in registers for all three
  // GRADC: output component GC of the gradient operator alone: the convection
  // contractions with that component's row of the gradient's D (9 values stored per point)
  constexpr bool GRADC = KIND >= kGradCompKind;
  constexpr int GC = GRADC ? KIND - kGradCompKind : 0;
  constexpr bool VEC3 = KIND >= kVectorKind && !GRADC;
  constexpr int K0 = GRADC ? PAFEM_CONVECTION : VEC3 ? KIND - kVectorKind : KIND;
  // DIVV: divergence of a vector-valued input into a scalar output: the three input
  // components pass the forward contractions one after the other, their point values
  // summed in registers, then one back contraction of values
  constexpr bool DIVV = (K0 == PAFEM_DIVERGENCE);
  constexpr int NV = (VEC3 || DIVV) ? 3 : 1;
  constexpr bool GEOM = (K0 == PAFEM_DIFFUSION_GEOM);
  constexpr bool DIFF = (K0 == PAFEM_DIFFUSION) || GEOM;  // gradient in, gradient out
  // CONV: convection, gradient in, value out (the back contractions are the mass ones)
  constexpr bool CONV = (K0 == PAFEM_CONVECTION);
  // DGV: volume term of the DG convection, -(u, beta . grad v): value in, gradient out
  // (the forward contractions are the mass ones, the back ones the diffusion ones)
  constexpr bool DGV = (K0 == PAFEM_DG_CONVECTION);
  // GRADV: gradient into a vector-valued output, gradient in, 3 values out (each
  // contracted back with B only), output component c at y + c * ystride
  constexpr bool GRADV = (K0 == PAFEM_GRADIENT);
  constexpr bool GRAD = DIFF || CONV || GRADV || DIVV;  // the forward contractions produce the gradient
  constexpr bool BACK3 = DIFF || GRADV || DGV;  // three arrays in the back contractions
  constexpr bool BACKD = DIFF || DGV;           // gradient back contractions
  // values per point in registers; DIVV stores 9 and reads those of one input component
  constexpr int NC = GEOM ? 1 : DIFF ? 6 : (CONV || DIVV || DGV) ? 3 : GRADV ? 9 : 1;
  constexpr int NCT = (DIVV || GRADC) ? 9 : NC;  // stored values per point
  constexpr int NA = GRAD ? 2 : 1;   // arrays after the x-lines (B and G along x)
  constexpr int NCC = (GRAD || DGV) ? 3 : 1;  // arrays after the y-lines (one per derivative)
  constexpr int NOUT = GRADV ? 3 : 1;  // output components
  static_assert(!((CONV || GRADV || DIVV || DGV) && DOT), "the convection, gradient and divergence operators have no energy");
  static_assert(!(DGV && EVEC), "the DG volume term stores through the tile lists");
  static_assert(!((GRADV || DIVV) && EVEC), "the gradient and divergence operators use the atomic scatter");
  static_assert(NOUT * D <= NCC * Q, "back x-line arrays must fit the element region");
  static_assert(NV == 1 || DIVV || (!DOT && !EVEC && (K0 == PAFEM_MASS || K0 == PAFEM_DIFFUSION)),
                "vector operators: stored-D mass or diffusion, atomic scatter, no energy");
  // Line stride: odd, so that threads walking consecutive lines hit distinct banks.
  // Stored-D scalar FP64 diffusion at p = 5 keeps the even stride D instead: the 1029 ->
  // 882 values per element region are what lets four tiles share a CU (four waves per
  // SIMD, with the unique dofs in the region tails below), which outweighs the conflicts
  // (0.401 -> 0.386 ms at 1e7 dofs).
  constexpr int LC =
      (P == 5 && KIND == PAFEM_DIFFUSION && sizeof(TC) == 8) ? D : (D | 1);
  constexpr int ELEM = NCC * QQ * LC;
  static_assert(NA * D <= NCC * Q, "x-line outputs must fit the element region");
  // XTAIL (scalar FP64 diffusion, p >= 5): the rows (c*Q + qy) of the element region
  // from NA*D on are dead from the back y-lines until the forward y-lines, while the
  // tile's unique-dof array is live exactly then (gather to forward x-lines, back
  // x-lines to the scatter).  Those rows of all elements of the tile are one
  // contiguous block after the leading rows, and the unique-dof array lives in it:
  // 11-12 KB less LDS per tile, three tiles per CU instead of two (one more barrier,
  // to clear the accumulators once the back y-lines have read the rows).
  constexpr bool XTAIL = DIFF && NV == 1 && P >= 5 && sizeof(TC) == 8;
  constexpr int HR = XTAIL ? NA * D : NCC * Q;  // leading rows of an element
  constexpr int HEAD = HR * Q * LC, TAIL = ELEM - HEAD;
  static_assert(!XTAIL || NE * TAIL >= NE * DDD, "the unique dofs must fit the region tails");

  __shared__ TC sW[NE * ELEM];
  // The tile's unique dofs: x gathered once per unique dof, later the element
  // outputs summed per unique dof before one global atomic each.
  __shared__ TC sXa[XTAIL ? 1 : NOUT * NE * DDD];
  TC* const sX = XTAIL ? sW + NE * HEAD : sXa;

  const int tid = threadIdx.x;
  const int el = tid / QQ;
  const int r = tid - el * QQ;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int e = tile * NE + el;
  const bool act = e < ne;
  const int u0 = tile_off[tile];
  const int nu = tile_off[tile + 1] - u0;
  TC* const W = sW + el * HEAD;
  TC* const WT = sW + NE * HEAD + el * TAIL;
  // entry (c, qy, qx, dz) of the element region; the x-line outputs (a, dz, dy, qx)
  // live at c*Q + qy = a*D + dy
  auto at = [&](int c, int qy, int qx, int dz) -> TC& {
    const int row = c * Q + qy;
    if constexpr (XTAIL)
      return row < HR ? W[(row * Q + qx) * LC + dz] : WT[((row - HR) * Q + qx) * LC + dz];
    else
      return W[(row * Q + qx) * LC + dz];
  };
  // Row q (forward stages) or column d (back stages) of a 1D table.  At p = 8 loaded per
  // loop iteration (opaque_ptr): the 180 FP64 table entries outgrow the scalar registers
  // and the compiler, loading them all up front, spilled them through VGPR lanes (1674
  // lane reads per wave; 0.483 -> 0.363 ms at 1e7 dofs with the changes below).  At
  // p = 6, 7 its up-front loads spill far less and are 2-4% faster than the per-iteration
  // ones, except in the FP64 variant with the fused energy (the CG apply), where they
  // spilled 374 / 804 / 1464 lane reads at p = 5 / 6 / 7 (CG iteration at p = 7 0.594 ->
  // 0.542 ms with the per-iteration loads).
  constexpr bool OPQ = P >= 8 || (DOT && !EVEC && P >= 5 && sizeof(TC) == 8);
  auto tab = [&](const TC* t) {
    if constexpr (OPQ)
      return opaque_ptr(t);
    else
      return t;
  };
  auto rowB = [&](int q) { return tab(tabB + q * D); };
  auto rowG = [&](int q) { return tab(tabG + q * D); };
  auto colB = [&](int d) { return tab(tabB + d); };
  auto colG = [&](int d) { return tab(tabG + d); };

  // D for this thread's z-line (qx, qy) = r: issued first so the HBM stream
  // overlaps the gather and the forward contractions (tile-interleaved: for each
  // (c, qz) the workgroup reads one contiguous run)
  // Stored-D scalar diffusion at p = 2 and p >= 4 in FP64 and at p = 6 in FP32 (the
  // refinement's inner operator): only the first PD planes are loaded here and each later
  // plane PD z-iterations ahead of its use.  The registers of the other planes lift the
  // occupancy, with the launch bound's request where needed: FP64 p = 4 from 3 to 4 waves
  // per SIMD (0.431 -> 0.419 ms at 1e7 dofs), p = 5 from 2 to 3 (0.434 -> 0.383 ms), FP32
  // p = 6 from 4 to 5 (0.462 -> 0.445 ms at 2e7 dofs), FP64 p = 6..8 from 2 to 3 together
  // with the smaller LDS footprint of XTAIL (p = 6 0.382 -> 0.326 ms, p = 7 0.377 -> 0.342
  // ms; p = 8 one plane ahead, fewer spills), p = 5 from 3 to 4 with XTAIL, the even line
  // stride and one plane ahead, and p = 2 from 4 to 5 (0.777 -> 0.770 ms, its CG iteration
  // 0.988 -> 0.968 ms).  Measured and not kept: p = 2 at 6 waves (spills, 12% slower), p = 3
  // at 5 waves (spills, 4% slower), FP64 p = 6..8 streamed at 2 waves (1-2% slower), FP32
  // p = 6 at 6 waves with XTAIL (spills; the refinement 8% slower).
  constexpr bool STREAM_D =
      K0 == PAFEM_DIFFUSION && NV == 1 && (sizeof(TC) == 8 ? (P == 2 || P >= 4) : P == 6);
  constexpr int PD = STREAM_D ? ((P == 5 || P == 8) ? 1 : 2) : Q;
  TC dq[Q][NC];
  // stored diffusion D: components in pairs per point, one load per pair
  constexpr bool PAIRS = (NCT == 6);
  const TD* const qe0 = qd + size_t(tile) * NCT * QQQ * NE + (PAIRS ? 2 * tid : tid);
  auto load_plane = [&](int qz, int cbase) {
    if constexpr (PAIRS) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        load_pair<TC, TD>(qe0 + 2 * ((k * Q + qz) * (NE * QQ)), dq[qz][2 * k], dq[qz][2 * k + 1]);
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        dq[qz][c] = load_value<TC, TD>(qe0 + ((cbase + c) * Q + qz) * (NE * QQ));
    }
  };
  auto load_dq = [&](int cbase) {
    if (act) {
#pragma unroll
      for (int qz = 0; qz < PD; ++qz) load_plane(qz, cbase);
    }
  };
  if (!DIVV) load_dq(GRADC ? 3 * GC : 0);
  TC sdiv[DIVV ? Q : 1];  // DIVV: the divergence at this thread's points, summed over components
#pragma unroll
  for (int qz = 0; qz < (DIVV ? Q : 1); ++qz) sdiv[qz] = TC(0);

  for (int comp = 0; comp < NV; ++comp) {
  const TV* const xv_in = x + comp * ystride;
  if (DIVV) load_dq(3 * comp);  // w kappa adj(J)[b][comp], b = 0..2
  // G: gather the tile's unique dofs; four per thread per step keep several
  // gathers in flight
  // at p <= 4 a tile's unique dofs fit one pass of four per thread: the dof ids stay
  // in registers for the scatter
  constexpr bool ONEPASS = DDD <= 4 * QQ;
  int gkeep[4] = {0, 0, 0, 0};
  for (int s0 = tid; s0 < nu; s0 += 4 * NE * QQ) {
    int gg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = s0 + k * NE * QQ;
      gg[k] = s < nu ? __builtin_nontemporal_load(tile_dofs + u0 + s) : 0;
      gkeep[k] = gg[k];
    }
    TC xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int g = gg[k];
      xv[k] = (s0 + k * NE * QQ < nu && !(constrained && g < 0)) ? TC(xv_in[g < 0 ? ~g : g]) : TC(0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s0 + k * NE * QQ < nu) sX[s0 + k * NE * QQ] = xv[k];
  }
  // x-line (dz, dy) = r < D*D: its D slots in the tile's unique dofs
  const bool xline = act && r < DD;
  const int xz = r / D, xy = r - (r / D) * D;
  int slot[D];
  if (xline) {
    const uint16_t* sl = tile_slot + size_t(e) * DDD + r * D;
#pragma unroll
    for (int dx = 0; dx < D; ++dx) slot[dx] = __builtin_nontemporal_load(sl + dx);
  }
  __syncthreads();

  // B along x: thread (dz, dy)
  if (xline) {
    TC u[D];
#pragma unroll
    for (int dx = 0; dx < D; ++dx) u[dx] = sX[slot[dx]];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      const auto rb = rowB(qx);
      const auto rg = rowG(qx);
      TC b = TC(0), g = TC(0);
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        b += rb[dx] * u[dx];
        if (GRAD) g += rg[dx] * u[dx];
      }
      at(xy / Q, xy % Q, qx, xz) = b;
      if (GRAD) at((D + xy) / Q, (D + xy) % Q, qx, xz) = g;
    }
  }
  __syncthreads();

  // sX is dead from here on: clear the per-unique-dof accumulators it now holds
  if (!EVEC && !XTAIL)
    for (int s = tid; s < nu; s += NE * QQ)
#pragma unroll
      for (int oc = 0; oc < NOUT; ++oc) sX[oc * NE * DDD + s] = TC(0);

  // B along y: thread (dz, qx) = r < D*Q
  const bool yline = act && r < D * Q;
  const int yz = r / Q, yx = r - (r / Q) * Q;
  if (yline) {
    TC aB[D], aG[D];
#pragma unroll
    for (int dy = 0; dy < D; ++dy) {
      aB[dy] = at(dy / Q, dy % Q, yx, yz);
      if (GRAD) aG[dy] = at((D + dy) / Q, (D + dy) % Q, yx, yz);
    }
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      const auto rb = rowB(qy);
      const auto rg = rowG(qy);
      TC gb = TC(0), bg = TC(0), bb = TC(0);
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        bb += rb[dy] * aB[dy];
        if (GRAD) {
          gb += rb[dy] * aG[dy];
          bg += rg[dy] * aB[dy];
        }
      }
      if (GRAD) {
        at(0, qy, yx, yz) = gb;
        at(1, qy, yx, yz) = bg;
        at(2, qy, yx, yz) = bb;
      } else {
        at(0, qy, yx, yz) = bb;
      }
    }
  }
  __syncthreads();

  // B along z, D, B^t along z: thread (qy, qx) = r, in registers, written back in place
  double energy = 0.0;  // sum of u . D u over this thread's points (DOT)
  if (act) {
    const int zy = r / Q, zx = r - (r / Q) * Q;
    // GEOM: the corners contracted over this thread's (qx, qy), per z-corner k and
    // coordinate a: value, x-derivative and y-derivative parts of J
    TC gv[3][2], gx[3][2], gy[3][2];
    if constexpr (GEOM) {
      const double* X = gnodes + size_t(e) * 24;  // [k3][k2][k1][a], k1 fastest
      const TC b1[2] = {tabBg[zx * 2], tabBg[zx * 2 + 1]}, g1[2] = {tabGg[zx * 2], tabGg[zx * 2 + 1]};
      const TC b2[2] = {tabBg[zy * 2], tabBg[zy * 2 + 1]}, g2[2] = {tabGg[zy * 2], tabGg[zy * 2 + 1]};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k3 = 0; k3 < 2; ++k3) {
          TC v = TC(0), dx = TC(0), dy = TC(0);
#pragma unroll
          for (int k2 = 0; k2 < 2; ++k2)
#pragma unroll
            for (int k1 = 0; k1 < 2; ++k1) {
              const TC xa = X[3 * (k1 + 2 * (k2 + 2 * k3)) + a];
              v += xa * (b1[k1] * b2[k2]);
              dx += xa * (g1[k1] * b2[k2]);
              dy += xa * (b1[k1] * g2[k2]);
            }
          gv[a][k3] = v;
          gx[a][k3] = dx;
          gy[a][k3] = dy;
        }
    }
    TC c0[D], c1[D], c2[D];
#pragma unroll
    for (int dz = 0; dz < D; ++dz) {
      c0[dz] = at(0, zy, zx, dz);
      if (GRAD) {
        c1[dz] = at(1, zy, zx, dz);
        c2[dz] = at(2, zy, zx, dz);
      }
    }
    TC t0[D], t1[D], t2[D];
#pragma unroll
    for (int dz = 0; dz < D; ++dz) t0[dz] = t1[dz] = t2[dz] = TC(0);
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      const auto rb = rowB(qz);
      const auto rg = rowG(qz);
      if constexpr (PD < Q) {
        if (qz + PD < Q) load_plane(qz + PD, 0);
        __asm__ volatile("" ::: "memory");  // keep the next plane's loads in this iteration
      }
      if constexpr (DIFF) {
        TC ux = TC(0), uy = TC(0), uz = TC(0);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          ux += rb[dz] * c0[dz];
          uy += rb[dz] * c1[dz];
          uz += rg[dz] * c2[dz];
        }
        TC vx, vy, vz;
        if constexpr (GEOM) {
          // J[a][b] = dx_a / dxi_b at (qx, qy, qz); D = w kappa adj(J) adj(J)^t / det J
          TC J[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            J[a][0] = gx[a][0] * tabBg[qz * 2] + gx[a][1] * tabBg[qz * 2 + 1];
            J[a][1] = gy[a][0] * tabBg[qz * 2] + gy[a][1] * tabBg[qz * 2 + 1];
            J[a][2] = gv[a][0] * tabGg[qz * 2] + gv[a][1] * tabGg[qz * 2 + 1];
          }
          const TC A00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
          const TC A01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
          const TC A02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
          const TC A10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
          const TC A11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
          const TC A12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
          const TC A20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
          const TC A21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
          const TC A22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          const TC det = J[0][0] * A00 + J[0][1] * A10 + J[0][2] * A20;
          const TC f = dq[qz][0] / det;
          // D u = f A (A^t u) without forming D (21 instead of 33 operations per point)
          const TC w0 = f * (A00 * ux + A10 * uy + A20 * uz);
          const TC w1 = f * (A01 * ux + A11 * uy + A21 * uz);
          const TC w2 = f * (A02 * ux + A12 * uy + A22 * uz);
          vx = A00 * w0 + A01 * w1 + A02 * w2;
          vy = A10 * w0 + A11 * w1 + A12 * w2;
          vz = A20 * w0 + A21 * w1 + A22 * w2;
        } else {
          vx = dq[qz][0] * ux + dq[qz][1] * uy + dq[qz][2] * uz;
          vy = dq[qz][1] * ux + dq[qz][3] * uy + dq[qz][4] * uz;
          vz = dq[qz][2] * ux + dq[qz][4] * uy + dq[qz][5] * uz;
        }
        if (DOT) energy += double(ux) * double(vx) + double(uy) * double(vy) + double(uz) * double(vz);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          t0[dz] += rb[dz] * vx;
          t1[dz] += rb[dz] * vy;
          t2[dz] += rg[dz] * vz;
        }
      } else if constexpr (GRADV) {
        // w kappa adj(J)^t (reference gradient): the physical gradient times w det J
        TC ux = TC(0), uy = TC(0), uz = TC(0);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          ux += rb[dz] * c0[dz];
          uy += rb[dz] * c1[dz];
          uz += rg[dz] * c2[dz];
        }
        const TC v0 = dq[qz][0] * ux + dq[qz][1] * uy + dq[qz][2] * uz;
        const TC v1 = dq[qz][3] * ux + dq[qz][4] * uy + dq[qz][5] * uz;
        const TC v2 = dq[qz][6] * ux + dq[qz][7] * uy + dq[qz][8] * uz;
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          t0[dz] += rb[dz] * v0;
          t1[dz] += rb[dz] * v1;
          t2[dz] += rb[dz] * v2;
        }
      } else if constexpr (DIVV) {
        // d u_comp / d x_comp times w kappa det J: sum_b w kappa adj(J)[b][comp] d_b u_comp
        TC ux = TC(0), uy = TC(0), uz = TC(0);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          ux += rb[dz] * c0[dz];
          uy += rb[dz] * c1[dz];
          uz += rg[dz] * c2[dz];
        }
        sdiv[qz] += dq[qz][0] * ux + dq[qz][1] * uy + dq[qz][2] * uz;
        if (comp == NV - 1) {
#pragma unroll
          for (int dz = 0; dz < D; ++dz) t0[dz] += rb[dz] * sdiv[qz];
        }
      } else if constexpr (DGV) {
        // -u (w adj(J) beta) . grad_ref v: the value at the point times minus the stored
        // vector, contracted back against the reference gradient
        TC u = TC(0);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) u += rb[dz] * c0[dz];
        const TC vx = -dq[qz][0] * u, vy = -dq[qz][1] * u, vz = -dq[qz][2] * u;
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          t0[dz] += rb[dz] * vx;
          t1[dz] += rb[dz] * vy;
          t2[dz] += rg[dz] * vz;
        }
      } else if constexpr (CONV) {
        // (beta . grad u) at the point: w adj(J) beta . (reference gradient)
        TC ux = TC(0), uy = TC(0), uz = TC(0);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) {
          ux += rb[dz] * c0[dz];
          uy += rb[dz] * c1[dz];
          uz += rg[dz] * c2[dz];
        }
        const TC v = dq[qz][0] * ux + dq[qz][1] * uy + dq[qz][2] * uz;
#pragma unroll
        for (int dz = 0; dz < D; ++dz) t0[dz] += rb[dz] * v;
      } else {
        TC u = TC(0);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) u += rb[dz] * c0[dz];
        const TC v = dq[qz][0] * u;
        if (DOT) energy += double(u) * double(v);
#pragma unroll
        for (int dz = 0; dz < D; ++dz) t0[dz] += rb[dz] * v;
      }
    }
    if (!DIVV || comp == NV - 1) {
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        at(0, zy, zx, dz) = t0[dz];
        if (BACK3) {
          at(1, zy, zx, dz) = t1[dz];
          at(2, zy, zx, dz) = t2[dz];
        }
      }
    }
  }
  // DIVV: the next component's gather writes only sX, which no thread reads after the
  // x-lines, and its x-lines write the element regions only after the barrier that
  // follows the gather, which every thread reaches after its z-line
  if (DIVV && comp < NV - 1) continue;
  __syncthreads();

  // B^t along y: thread (dz, qx)
  if (yline) {
    TC v0[Q], v1[Q], v2[Q];
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      v0[qy] = at(0, qy, yx, yz);
      if (BACK3) {
        v1[qy] = at(1, qy, yx, yz);
        v2[qy] = at(2, qy, yx, yz);
      }
    }
    if constexpr (GRADV) {
      // three value contractions: component c of the output to x-line array c
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        const auto cb = colB(dy);
        TC o0 = TC(0), o1 = TC(0), o2 = TC(0);
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          o0 += cb[qy * D] * v0[qy];
          o1 += cb[qy * D] * v1[qy];
          o2 += cb[qy * D] * v2[qy];
        }
        at(dy / Q, dy % Q, yx, yz) = o0;
        at((D + dy) / Q, (D + dy) % Q, yx, yz) = o1;
        at((2 * D + dy) / Q, (2 * D + dy) % Q, yx, yz) = o2;
      }
    } else {
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        const auto cb = colB(dy);
        const auto cg = colG(dy);
        TC b = TC(0), g = TC(0);
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          if (BACKD) {
            g += cb[qy * D] * v0[qy];
            b += cg[qy * D] * v1[qy] + cb[qy * D] * v2[qy];
          } else {
            b += cb[qy * D] * v0[qy];
          }
        }
        at(dy / Q, dy % Q, yx, yz) = b;
        if (BACKD) at((D + dy) / Q, (D + dy) % Q, yx, yz) = g;
      }
    }
  }
  __syncthreads();
  if constexpr (XTAIL && !EVEC) {
    // the region tails are dead now: clear the per-unique-dof accumulators there
    for (int s = tid; s < nu; s += NE * QQ) sX[s] = TC(0);
    __syncthreads();
  }

  // B^t along x and G^t: thread (dz, dy)
  if constexpr (GRADV) {
   if (xline) {
    TC w0[Q], w1[Q], w2[Q];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      w0[qx] = at(xy / Q, xy % Q, qx, xz);
      w1[qx] = at((D + xy) / Q, (D + xy) % Q, qx, xz);
      w2[qx] = at((2 * D + xy) / Q, (2 * D + xy) % Q, qx, xz);
    }
#pragma unroll
    for (int dx = 0; dx < D; ++dx) {
      const auto cb = colB(dx);
      TC a0 = TC(0), a1 = TC(0), a2 = TC(0);
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        a0 += cb[qx * D] * w0[qx];
        a1 += cb[qx * D] * w1[qx];
        a2 += cb[qx * D] * w2[qx];
      }
      atomicAdd(&sX[slot[dx]], a0);
      atomicAdd(&sX[NE * DDD + slot[dx]], a1);
      atomicAdd(&sX[2 * NE * DDD + slot[dx]], a2);
    }
   }
  } else if (xline) {
    TC wB[Q], wG[Q];
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      wB[qx] = at(xy / Q, xy % Q, qx, xz);
      if (BACKD) wG[qx] = at((D + xy) / Q, (D + xy) % Q, qx, xz);
    }
#pragma unroll
    for (int dx = 0; dx < D; ++dx) {
      const auto cb = colB(dx);
      const auto cg = colG(dx);
      TC acc = TC(0);
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        acc += cb[qx * D] * wB[qx];
        if (BACKD) acc += cg[qx * D] * wG[qx];
      }
      if (EVEC)
        y[size_t(e) * DDD + r * D + dx] = TV(acc);
      else
        atomicAdd(&sX[slot[dx]], acc);
    }
  }
  if (DOT) {
    __shared__ double sDot[(elems_per_block<Q>() * Q * Q + kWave - 1) / kWave];
    energy = block_sum(energy, sDot);
    if (tid == 0) dotp[blockIdx.x] = energy;
  }
  if (EVEC) return;
  __syncthreads();
  // G^t: one global atomic per unique dof of the tile.  The DG volume term's dofs belong
  // to one element each (no dof is shared between tiles), so it stores instead, and the
  // call needs no y-init (the face kernel adds its atomics afterwards).
  auto put = [&](TV* dst, TV v) {
    if constexpr (DGV)
      *dst = v;
    else
      unsafeAtomicAdd(dst, v);
  };
  if constexpr (ONEPASS && NV == 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = tid + k * NE * QQ;
      const int g = gkeep[k];
      if (s < nu && !(constrained && g < 0))
#pragma unroll
        for (int oc = 0; oc < NOUT; ++oc)
          put(&y[(DIVV ? 0 : GRADC ? GC : comp + oc) * ystride + (g < 0 ? ~g : g)],
              TV(sX[oc * NE * DDD + s]));
    }
  } else {
#pragma unroll 4
    for (int s = tid; s < nu; s += NE * QQ) {
      const int g = tile_dofs[u0 + s];
      if (!(constrained && g < 0))
#pragma unroll
        for (int oc = 0; oc < NOUT; ++oc)
          put(&y[(DIVV ? 0 : GRADC ? GC : comp + oc) * ystride + (g < 0 ? ~g : g)],
              TV(sX[oc * NE * DDD + s]));
    }
  }
  if (NV > 1) __syncthreads();  // sX is gathered again for the next component
  }
}

// the 1D tables in the compute precision
template <typename TC>
const TC* table_block(const DevSpace& sp, int q1d);
template <>
const double* table_block<double>(const DevSpace& sp, int q1d) {
  return sp.tables + table_offset_doubles(q1d, sp.p + 1, sp.ng);
}
template <>
const float* table_block<float>(const DevSpace& sp, int q1d) {
  return sp.tables32 + table_offset_doubles(q1d, sp.p + 1, sp.ng);
}

template <int P, int KIND, bool EVEC, bool DOT, typename TV, typename TD, typename TC>
void launch_one(const DevSpace& sp, bool constrained, const void* qd, const void* x, void* out,
                double* dotp, hipStream_t st) {
  constexpr int Q = P + 2;
  constexpr int NE = elems_per_block<Q>();
  const int nblk = int((sp.ne + NE - 1) / NE);
  const TC* tabB = table_block<TC>(sp, Q) + 2 * Q;
  const TC* tabG = tabB + Q * (P + 1);
  // geometry tables (Bg, Gg of the ng-node geometry basis) follow B and G
  const TC* tabBg = tabG + Q * (P + 1);
  const TC* tabGg = tabBg + Q * sp.ng;
  hipLaunchKernelGGL((pa_apply_kernel<P, Q, KIND, EVEC, DOT, TV, TD, TC>), dim3(nblk),
                     dim3(NE * Q * Q), 0, st, sp.tile_off, sp.tile_dofs, sp.tile_slot, tabB, tabG,
                     static_cast<const TD*>(qd), static_cast<const TV*>(x),
                     static_cast<TV*>(out), dotp, sp.gnodes, tabBg, tabGg, int(sp.ne),
                     int(constrained), int64_t(sp.ndofs));
}

template <int P, int KIND, typename TV, typename TD, typename TC>
void launch_mode(const DevSpace& sp, bool constrained, bool evec, const void* qd, const void* x,
                 void* out, double* dotp, hipStream_t st) {
  if (evec) {
    if (dotp)
      launch_one<P, KIND, true, true, TV, TD, TC>(sp, constrained, qd, x, out, dotp, st);
    else
      launch_one<P, KIND, true, false, TV, TD, TC>(sp, constrained, qd, x, out, dotp, st);
  } else {
    if (dotp)
      launch_one<P, KIND, false, true, TV, TD, TC>(sp, constrained, qd, x, out, dotp, st);
    else
      launch_one<P, KIND, false, false, TV, TD, TC>(sp, constrained, qd, x, out, dotp, st);
  }
}

template <int P>
bool launch_order(const DevSpace& sp, int kind, int qdtype, int vdtype, bool constrained,
                  bool evec, const void* qd, const void* x, void* out, double* dotp,
                  hipStream_t st) {
  const bool diff = kind == PAFEM_DIFFUSION;
  if (kind == kVectorKind + PAFEM_DIFFUSION || kind == kVectorKind + PAFEM_MASS) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || dotp || evec) return false;
    if constexpr (P >= 7) {
      // the three-component kernel runs out of registers at p >= 7: one scalar apply per
      // component (measured faster there)
      for (int c = 0; c < 3; ++c) {
        const double* xc = static_cast<const double*>(x) + c * sp.ndofs;
        double* yc = static_cast<double*>(out) + c * sp.ndofs;
        if (kind == kVectorKind + PAFEM_DIFFUSION)
          launch_one<P, PAFEM_DIFFUSION, false, false, double, double, double>(sp, constrained, qd,
                                                                                xc, yc, nullptr, st);
        else
          launch_one<P, PAFEM_MASS, false, false, double, double, double>(sp, constrained, qd, xc,
                                                                           yc, nullptr, st);
      }
      return true;
    }
    if (kind == kVectorKind + PAFEM_DIFFUSION)
      launch_one<P, kVectorKind + PAFEM_DIFFUSION, false, false, double, double, double>(
          sp, constrained, qd, x, out, nullptr, st);
    else
      launch_one<P, kVectorKind + PAFEM_MASS, false, false, double, double, double>(
          sp, constrained, qd, x, out, nullptr, st);
    return true;
  }
  if (kind == PAFEM_GRADIENT) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || dotp || evec) return false;
    if constexpr (P <= 4) {
      // all three output components at once: three accumulators in LDS (51 KB at p = 4)
      launch_one<P, PAFEM_GRADIENT, false, false, double, double, double>(sp, constrained, qd, x,
                                                                           out, nullptr, st);
    } else {
      // three accumulators no longer fit a workgroup's LDS: one pass per component
      launch_one<P, kGradCompKind + 0, false, false, double, double, double>(sp, constrained, qd,
                                                                             x, out, nullptr, st);
      launch_one<P, kGradCompKind + 1, false, false, double, double, double>(sp, constrained, qd,
                                                                             x, out, nullptr, st);
      launch_one<P, kGradCompKind + 2, false, false, double, double, double>(sp, constrained, qd,
                                                                             x, out, nullptr, st);
    }
    return true;
  }
  if (kind == PAFEM_DIVERGENCE) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || dotp || evec) return false;
    launch_one<P, PAFEM_DIVERGENCE, false, false, double, double, double>(sp, constrained, qd, x,
                                                                           out, nullptr, st);
    return true;
  }
  if (kind == PAFEM_DG_CONVECTION) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || dotp || evec) return false;
    launch_one<P, PAFEM_DG_CONVECTION, false, false, double, double, double>(sp, false, qd, x,
                                                                              out, nullptr, st);
    return true;
  }
  if (kind == PAFEM_CONVECTION) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || dotp) return false;
    if (evec)
      launch_one<P, PAFEM_CONVECTION, true, false, double, double, double>(sp, constrained, qd, x,
                                                                            out, nullptr, st);
    else
      launch_one<P, PAFEM_CONVECTION, false, false, double, double, double>(sp, constrained, qd, x,
                                                                             out, nullptr, st);
    return true;
  }
  if (kind == PAFEM_DIFFUSION_GEOM) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || sp.ng != 2) return false;
    launch_mode<P, PAFEM_DIFFUSION_GEOM, double, double, double>(sp, constrained, evec, qd, x, out,
                                                                 dotp, st);
    return true;
  }
  if (vdtype == PAFEM_F64 && qdtype == PAFEM_F64) {
    if (diff)
      launch_mode<P, PAFEM_DIFFUSION, double, double, double>(sp, constrained, evec, qd, x, out, dotp, st);
    else
      launch_mode<P, PAFEM_MASS, double, double, double>(sp, constrained, evec, qd, x, out, dotp, st);
    return true;
  }
  if (vdtype == PAFEM_F32 && qdtype == PAFEM_F32) {
    if (diff)
      launch_mode<P, PAFEM_DIFFUSION, float, float, float>(sp, constrained, evec, qd, x, out, dotp, st);
    else
      launch_mode<P, PAFEM_MASS, float, float, float>(sp, constrained, evec, qd, x, out, dotp, st);
    return true;
  }
  if (vdtype == PAFEM_F32 && qdtype == PAFEM_BF16) {
    if (diff)
      launch_mode<P, PAFEM_DIFFUSION, float, bf16, float>(sp, constrained, evec, qd, x, out, dotp, st);
    else
      launch_mode<P, PAFEM_MASS, float, bf16, float>(sp, constrained, evec, qd, x, out, dotp, st);
    return true;
  }
  return false;
}

}  // namespace

int pa_apply_blocks(const DevSpace& sp) {
  if (sp.dim == 2) return pa_apply2d_blocks(sp);
  return int((sp.ne + qdata_tile(sp.p + 2) - 1) / qdata_tile(sp.p + 2));
}

bool launch_pa_apply(const DevSpace& sp, int kind, int q1d, int qdtype, bool constrained,
                     bool evec, const void* qd, const void* x, void* out, int vdtype,
                     hipStream_t st, double* dotp) {
  if (q1d != sp.p + 2) return false;
  bool ok = false;
  if (sp.dim == 2) {
    if (evec || qdtype != PAFEM_F64 || vdtype != PAFEM_F64 ||
        (kind != PAFEM_DIFFUSION && kind != PAFEM_MASS))
      return false;
    ok = launch_pa_apply_2d(sp, kind, constrained, static_cast<const double*>(qd),
                            static_cast<const double*>(x), static_cast<double*>(out), st, dotp);
    if (ok) {
      hipError_t err = hipGetLastError();
      if (err != hipSuccess)
        throw Error(PAFEM_EHIP, std::string("apply launch: ") + hipGetErrorString(err));
    }
    return ok;
  }
  if (kind == PAFEM_ELASTICITY) {
    if (evec || dotp || qdtype != PAFEM_F64 || vdtype != PAFEM_F64) return false;
    ok = launch_elasticity(sp, constrained, static_cast<const double*>(qd),
                           static_cast<const double*>(x), static_cast<double*>(out), st);
  } else {
#define PAFEM_ORDER_CASE(P_)                                                                   \
  case P_:                                                                                     \
    ok = launch_order<P_>(sp, kind, qdtype, vdtype, constrained, evec, qd, x, out, dotp, st); \
    break;
  switch (sp.p) {
    PAFEM_ORDER_CASE(1)
    PAFEM_ORDER_CASE(2)
    PAFEM_ORDER_CASE(3)
    PAFEM_ORDER_CASE(4)
    PAFEM_ORDER_CASE(5)
    PAFEM_ORDER_CASE(6)
    PAFEM_ORDER_CASE(7)
    PAFEM_ORDER_CASE(8)
    default: ok = false;
  }
#undef PAFEM_ORDER_CASE
  }
  if (ok) {
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
      throw Error(PAFEM_EHIP, std::string("apply launch: ") + hipGetErrorString(err));
  }
  return ok;
}

}  // namespace pafem
