// Batched operator action: many right-hand sides over many meshes.
//
// Each mesh m holds nrhs vectors stored right-hand-side fastest, X_m[dof][rhs],
// so the gather of one dof reads one contiguous run of nrhs values.  The
// partial-assembly stages are those of the single-vector kernel (G, B, D, B^t,
// G^t; "Operator Decomposition"), one 1D line per thread, applied to NRB
// right-hand sides at once: the tile of a workgroup is NE elements x Q*Q lines x
// NRB right-hand sides with the rhs index fastest (coalesced X loads and Y
// atomics, broadcast D loads, conflict-free LDS).  Table entries are the same for
// every lane and come from scalar loads; the quadrature data D of a z-line is
// loaded once into registers and reused for every right-hand side.  The
// workgroup loops over the nrhs/NRB chunks.  All meshes of one order share one
// grouped launch: a workgroup finds its mesh from a prefix table of tile counts.
#include "batch.hpp"
#include "device.hpp"

namespace pafem {

namespace {

template <int P, int Q, int NE, int NRB, int KIND, typename TV, typename TD, typename TC>
__global__ void __launch_bounds__(NE * Q * Q * NRB)
    pa_apply_mrhs_kernel(const BatchMesh* __restrict__ meshes, int nmesh,
                         const TC* __restrict__ tabB, const TC* __restrict__ tabG, int nrhs) {
  constexpr int D = P + 1, DD = D * D, QQ = Q * Q;
  constexpr bool DIFF = (KIND == PAFEM_DIFFUSION);
  constexpr int NC = DIFF ? 6 : 1;
  constexpr int NCC = DIFF ? 3 : 1;
  constexpr int ELEM = NCC * QQ * D;  // entries of one element region (per rhs)
  static_assert((DIFF ? 2 : 1) * D <= NCC * Q, "x-line outputs must fit the element region");

  __shared__ TC sW[NE * ELEM * NRB];

  // which mesh and which tile of it
  int m = 0;
  const int blk = blockIdx.x;
  while (m + 1 < nmesh && meshes[m + 1].block_begin <= blk) ++m;
  const BatchMesh& M = meshes[m];
  const int tile = blk - M.block_begin;

  const int tid = threadIdx.x;
  const int rb = tid % NRB;
  const int pl = tid / NRB;  // line thread: (el, r)
  const int el = pl / QQ;
  const int r = pl - el * QQ;
  const int e = tile * NE + el;
  const bool act = e < M.ne;
  const int constrained = M.constrained;
  TC* const W = sW + el * ELEM * NRB + rb;
  // entry (c, qy, qx, dz) of this element and rhs; the x-line outputs (a, dz, dy, qx)
  // live at c*Q + qy = a*D + dy
  auto at = [&](int c, int qy, int qx, int dz) -> TC& {
    return W[(((c * Q + qy) * Q + qx) * D + dz) * NRB];
  };
  auto bB = [&](int q, int d) -> TC { return tabB[q * D + d]; };
  auto bG = [&](int q, int d) -> TC { return tabG[q * D + d]; };

  // D of this thread's z-line (qy, qx) = r, reused for every chunk of right-hand sides
  TC dq[Q][NC];
  if (act) {
    const TD* qd = static_cast<const TD*>(M.qdata);
#pragma unroll
    for (int qz = 0; qz < Q; ++qz)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        dq[qz][c] = load_value<TC, TD>(qd + qdata_index(e, c, qz * QQ + r, Q, NC));
  }
  // x-line (dz, dy) = r < D*D: the dofs of its D nodes (re-read where used: cached)
  const bool xline = act && r < DD;
  const int xz = r / D, xy = r - (r / D) * D;
  const int32_t* __restrict__ gline = M.gmap + size_t(e) * (DD * D) + r * D;
  const bool yline = act && r < D * Q;
  const int yz = r / Q, yx = r - (r / Q) * Q;
  const int zy = r / Q, zx = r - (r / Q) * Q;
  const TV* __restrict__ X = static_cast<const TV*>(M.x);
  TV* __restrict__ Y = static_cast<TV*>(M.y);

  for (int r0 = 0; r0 < nrhs; r0 += NRB) {
    const int rr = r0 + rb;
    // G and B along x: thread (dz, dy)
    if (xline) {
      TC u[D];
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        const int g = gline[dx];
        u[dx] = (constrained && g < 0) ? TC(0) : TC(X[size_t(g < 0 ? ~g : g) * nrhs + rr]);
      }
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        TC b = TC(0), g = TC(0);
#pragma unroll
        for (int dx = 0; dx < D; ++dx) {
          b += bB(qx, dx) * u[dx];
          if (DIFF) g += bG(qx, dx) * u[dx];
        }
        at(xy / Q, xy % Q, qx, xz) = b;
        if (DIFF) at((D + xy) / Q, (D + xy) % Q, qx, xz) = g;
      }
    }
    __syncthreads();
    // B along y: thread (dz, qx)
    if (yline) {
      TC aB[D], aG[D];
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        aB[dy] = at(dy / Q, dy % Q, yx, yz);
        if (DIFF) aG[dy] = at((D + dy) / Q, (D + dy) % Q, yx, yz);
      }
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        TC gb = TC(0), bg = TC(0), bb = TC(0);
#pragma unroll
        for (int dy = 0; dy < D; ++dy) {
          bb += bB(qy, dy) * aB[dy];
          if (DIFF) {
            gb += bB(qy, dy) * aG[dy];
            bg += bG(qy, dy) * aB[dy];
          }
        }
        if (DIFF) {
          at(0, qy, yx, yz) = gb;
          at(1, qy, yx, yz) = bg;
          at(2, qy, yx, yz) = bb;
        } else {
          at(0, qy, yx, yz) = bb;
        }
      }
    }
    __syncthreads();
    // B along z, D, B^t along z: thread (qy, qx), in place
    if (act) {
      TC c0[D], c1[D], c2[D];
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        c0[dz] = at(0, zy, zx, dz);
        if (DIFF) {
          c1[dz] = at(1, zy, zx, dz);
          c2[dz] = at(2, zy, zx, dz);
        }
      }
      TC t0[D], t1[D], t2[D];
#pragma unroll
      for (int dz = 0; dz < D; ++dz) t0[dz] = t1[dz] = t2[dz] = TC(0);
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        if (DIFF) {
          TC ux = TC(0), uy = TC(0), uz = TC(0);
#pragma unroll
          for (int dz = 0; dz < D; ++dz) {
            ux += bB(qz, dz) * c0[dz];
            uy += bB(qz, dz) * c1[dz];
            uz += bG(qz, dz) * c2[dz];
          }
          const TC vx = dq[qz][0] * ux + dq[qz][1] * uy + dq[qz][2] * uz;
          const TC vy = dq[qz][1] * ux + dq[qz][3] * uy + dq[qz][4] * uz;
          const TC vz = dq[qz][2] * ux + dq[qz][4] * uy + dq[qz][5] * uz;
#pragma unroll
          for (int dz = 0; dz < D; ++dz) {
            t0[dz] += bB(qz, dz) * vx;
            t1[dz] += bB(qz, dz) * vy;
            t2[dz] += bG(qz, dz) * vz;
          }
        } else {
          TC u = TC(0);
#pragma unroll
          for (int dz = 0; dz < D; ++dz) u += bB(qz, dz) * c0[dz];
          const TC v = dq[qz][0] * u;
#pragma unroll
          for (int dz = 0; dz < D; ++dz) t0[dz] += bB(qz, dz) * v;
        }
      }
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        at(0, zy, zx, dz) = t0[dz];
        if (DIFF) {
          at(1, zy, zx, dz) = t1[dz];
          at(2, zy, zx, dz) = t2[dz];
        }
      }
    }
    __syncthreads();
    // B^t along y: thread (dz, qx)
    if (yline) {
      TC v0[Q], v1[Q], v2[Q];
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        v0[qy] = at(0, qy, yx, yz);
        if (DIFF) {
          v1[qy] = at(1, qy, yx, yz);
          v2[qy] = at(2, qy, yx, yz);
        }
      }
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        TC b = TC(0), g = TC(0);
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          if (DIFF) {
            g += bB(qy, dy) * v0[qy];
            b += bG(qy, dy) * v1[qy] + bB(qy, dy) * v2[qy];
          } else {
            b += bB(qy, dy) * v0[qy];
          }
        }
        at(dy / Q, dy % Q, yx, yz) = b;
        if (DIFF) at((D + dy) / Q, (D + dy) % Q, yx, yz) = g;
      }
    }
    __syncthreads();
    // B^t along x and G^t: thread (dz, dy)
    if (xline) {
      TC wB[Q], wG[Q];
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        wB[qx] = at(xy / Q, xy % Q, qx, xz);
        if (DIFF) wG[qx] = at((D + xy) / Q, (D + xy) % Q, qx, xz);
      }
#pragma unroll
      for (int dx = 0; dx < D; ++dx) {
        TC acc = TC(0);
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) {
          acc += bB(qx, dx) * wB[qx];
          if (DIFF) acc += bG(qx, dx) * wG[qx];
        }
        const int g = gline[dx];
        if (!(constrained && g < 0))
          unsafeAtomicAdd(&Y[size_t(g < 0 ? ~g : g) * nrhs + rr], TV(acc));
      }
    }
    // the next chunk overwrites the element regions only after every thread is done
    __syncthreads();
  }
}

// Y = X on essential dofs (constrained) and 0 elsewhere, for every mesh of the
// batch; blockIdx.y selects the mesh.
template <typename TV>
__global__ void batch_init_kernel(const BatchMesh* __restrict__ meshes, int nrhs) {
  const BatchMesh& M = meshes[blockIdx.y];
  const int64_t total = int64_t(M.ndofs) * nrhs;
  const TV* __restrict__ X = static_cast<const TV*>(M.x);
  TV* __restrict__ Y = static_cast<TV*>(M.y);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += int64_t(gridDim.x) * blockDim.x)
    Y[k] = (M.constrained && M.bmask[k / nrhs]) ? X[k] : TV(0);
}

template <int P, int NE, int NRB, typename TV, typename TD, typename TC>
void launch_cfg(const BatchMesh* meshes, int nmesh, int nblocks, int kind, const void* tab,
                int nrhs, hipStream_t st) {
  constexpr int Q = P + 2;
  const TC* tabB = static_cast<const TC*>(tab);
  const TC* tabG = tabB + Q * (P + 1);
  if (kind == PAFEM_DIFFUSION)
    hipLaunchKernelGGL((pa_apply_mrhs_kernel<P, Q, NE, NRB, PAFEM_DIFFUSION, TV, TD, TC>),
                       dim3(nblocks), dim3(NE * Q * Q * NRB), 0, st, meshes, nmesh, tabB, tabG,
                       nrhs);
  else
    hipLaunchKernelGGL((pa_apply_mrhs_kernel<P, Q, NE, NRB, PAFEM_MASS, TV, TD, TC>),
                       dim3(nblocks), dim3(NE * Q * Q * NRB), 0, st, meshes, nmesh, tabB, tabG,
                       nrhs);
}

// Candidate tiles per order (elements x right-hand sides per workgroup), limited
// by 1024 threads per workgroup and the LDS of the FP64 diffusion variant.
template <int P, typename TV, typename TD, typename TC>
bool launch_tile(int cand, const BatchMesh* meshes, int nmesh, int nblocks, int kind,
                 const void* tab, int nrhs, hipStream_t st) {
  if (cand == 0) {
    launch_cfg<P, 1, 4, TV, TD, TC>(meshes, nmesh, nblocks, kind, tab, nrhs, st);
    return true;
  }
  if (cand == 4) {
    launch_cfg<P, 1, 2, TV, TD, TC>(meshes, nmesh, nblocks, kind, tab, nrhs, st);
    return true;
  }
  if constexpr (P <= 5) {
    if (cand == 1) {
      launch_cfg<P, 1, 8, TV, TD, TC>(meshes, nmesh, nblocks, kind, tab, nrhs, st);
      return true;
    }
  }
  if constexpr (P <= 3) {
    if (cand == 2) {
      launch_cfg<P, 1, 16, TV, TD, TC>(meshes, nmesh, nblocks, kind, tab, nrhs, st);
      return true;
    }
  }
  if constexpr (P <= 3) {
    if (cand == 3) {
      launch_cfg<P, 2, 8, TV, TD, TC>(meshes, nmesh, nblocks, kind, tab, nrhs, st);
      return true;
    }
  }
  return false;
}

}  // namespace

int batch_tile_elems(int cand) {
  switch (cand) {
    case 3: return 2;
    default: return 1;
  }
}
int batch_tile_rhs(int cand) {
  switch (cand) {
    case 0: return 4;
    case 1: return 8;
    case 2: return 16;
    case 3: return 8;
    case 4: return 2;
    case kBatchMfmaCandidate: return 16;
    default: return 0;
  }
}

bool launch_batch_apply(int p, int cand, int vdtype, int qdtype, int kind,
                        const BatchMesh* meshes, int nmesh, int nblocks, const void* tab,
                        int nrhs, hipStream_t st) {
  if (cand == kBatchMfmaCandidate) {
    if (vdtype != PAFEM_F64 || qdtype != PAFEM_F64 || nrhs % 16) return false;
    return launch_batch_apply_mfma(p, kind, meshes, nmesh, nblocks,
                                   static_cast<const double*>(tab), nrhs, st);
  }
  bool ok = false;
#define PAFEM_BATCH_ORDER(PP)                                                                   \
  case PP:                                                                                      \
    if (vdtype == PAFEM_F64 && qdtype == PAFEM_F64)                                             \
      ok = launch_tile<PP, double, double, double>(cand, meshes, nmesh, nblocks, kind, tab,     \
                                                   nrhs, st);                                   \
    else if (vdtype == PAFEM_F32 && qdtype == PAFEM_F32)                                        \
      ok = launch_tile<PP, float, float, float>(cand, meshes, nmesh, nblocks, kind, tab, nrhs,  \
                                                st);                                            \
    break;
  switch (p) {
    PAFEM_BATCH_ORDER(1)
    PAFEM_BATCH_ORDER(2)
    PAFEM_BATCH_ORDER(3)
    PAFEM_BATCH_ORDER(4)
    PAFEM_BATCH_ORDER(5)
    PAFEM_BATCH_ORDER(6)
    default: ok = false;
  }
#undef PAFEM_BATCH_ORDER
  if (ok) {
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
      throw Error(PAFEM_EHIP, std::string("batch apply launch: ") + hipGetErrorString(err));
  }
  return ok;
}

void launch_batch_init(int vdtype, const BatchMesh* meshes, int nmesh, int nrhs,
                       hipStream_t st) {
  const dim3 grid(512, unsigned(nmesh));
  if (vdtype == PAFEM_F64)
    hipLaunchKernelGGL(batch_init_kernel<double>, grid, dim3(256), 0, st, meshes, nrhs);
  else
    hipLaunchKernelGGL(batch_init_kernel<float>, grid, dim3(256), 0, st, meshes, nrhs);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    throw Error(PAFEM_EHIP, std::string("batch init launch: ") + hipGetErrorString(err));
}

}  // namespace pafem
