// Batched operator action: many right-hand sides over many meshes.
//
// Each mesh m holds nrhs vectors stored right-hand-side fastest, X_m[dof][rhs],
// so the gather of one dof reads one contiguous run of nrhs values.  The
// partial-assembly stages are those of the single-vector kernel (G, B, D, B^t,
// G^t; "Operator Decomposition"), applied to NRB right-hand sides at once: the
// tile of a workgroup is NE elements x NRB right-hand sides, the rhs index is
// the fastest thread index (coalesced X loads, broadcast D loads, conflict-free
// LDS), and the quadrature data D of an element is loaded once into registers
// and reused for every right-hand side.  The workgroup loops over the nrhs/NRB
// chunks.  All meshes of one order share one grouped launch: a workgroup finds
// its mesh from a prefix table of tile counts.
#include "batch.hpp"
#include "device.hpp"

namespace pafem {

namespace {

template <int P, int Q, int NE, int NRB, int KIND, typename TV, typename TD, typename TC>
__global__ void __launch_bounds__(NE * Q * Q * NRB)
    pa_apply_mrhs_kernel(const BatchMesh* __restrict__ meshes, int nmesh,
                         const double* __restrict__ tabB, const double* __restrict__ tabG,
                         int nrhs) {
  constexpr int D = P + 1, QQ = Q * Q, DDD = D * D * D;
  constexpr bool DIFF = (KIND == PAFEM_DIFFUSION);
  constexpr int NC = DIFF ? 6 : 1;
  constexpr int NA = DIFF ? 2 : 1;
  constexpr int NCC = DIFF ? 3 : 1;

  __shared__ TC sB[Q][D];
  __shared__ TC sG[Q][D];
  __shared__ TC sU[NE][D][D][D][NRB];
  __shared__ TC sA[NE][NA][D][D][Q][NRB];
  __shared__ TC sC[NE][NCC][D][Q][Q][NRB];

  // which mesh and which tile of it
  int m = 0;
  const int blk = blockIdx.x;
  while (m + 1 < nmesh && meshes[m + 1].block_begin <= blk) ++m;
  const BatchMesh& M = meshes[m];
  const int tile = blk - M.block_begin;

  const int tid = threadIdx.x;
  const int rb = tid % NRB;
  const int pl = tid / NRB;  // plane thread: (el, qy, qx)
  const int el = pl / QQ;
  const int r = pl - el * QQ;
  const int qx = r % Q, qy = r / Q;
  const int e = tile * NE + el;
  const bool act = e < M.ne;
  const int constrained = M.constrained;

  for (int i = tid; i < Q * D; i += NE * QQ * NRB) {
    (&sB[0][0])[i] = TC(tabB[i]);
    if (DIFF) (&sG[0][0])[i] = TC(tabG[i]);
  }
  TC dq[Q][NC];
  if (act) {
    const TD* qd = static_cast<const TD*>(M.qdata);
#pragma unroll
    for (int qz = 0; qz < Q; ++qz)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        dq[qz][c] = load_value<TC, TD>(qd + qdata_index(e, c, qz * QQ + r, Q, NC));
  }
  int gidx[D];
  const bool dof_thread = act && qx < D && qy < D;
  if (dof_thread) {
    const int32_t* ge = M.gmap + size_t(e) * DDD + qy * D + qx;
#pragma unroll
    for (int dz = 0; dz < D; ++dz) gidx[dz] = ge[dz * D * D];
  }
  const TV* __restrict__ X = static_cast<const TV*>(M.x);
  TV* __restrict__ Y = static_cast<TV*>(M.y);

  for (int r0 = 0; r0 < nrhs; r0 += NRB) {
    const int rr = r0 + rb;
    // G: gather NRB right-hand sides of every element node
    if (dof_thread) {
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        const int g = gidx[dz];
        TC v = TC(0);
        if (!(constrained && g < 0)) v = TC(X[size_t(g < 0 ? ~g : g) * nrhs + rr]);
        sU[el][dz][qy][qx][rb] = v;
      }
    }
    __syncthreads();
    if (qy < D) {
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        TC b = TC(0), g = TC(0);
#pragma unroll
        for (int dx = 0; dx < D; ++dx) {
          const TC u = sU[el][dz][qy][dx][rb];
          b += sB[qx][dx] * u;
          if (DIFF) g += sG[qx][dx] * u;
        }
        sA[el][0][dz][qy][qx][rb] = b;
        if (DIFF) sA[el][NA - 1][dz][qy][qx][rb] = g;
      }
    }
    __syncthreads();
    TC BB[D], GB[D], BG[D];
#pragma unroll
    for (int dz = 0; dz < D; ++dz) {
      TC bb = TC(0), gb = TC(0), bg = TC(0);
#pragma unroll
      for (int dy = 0; dy < D; ++dy) {
        const TC a0 = sA[el][0][dz][dy][qx][rb];
        const TC by = sB[qy][dy];
        bb += by * a0;
        if (DIFF) {
          gb += by * sA[el][NA - 1][dz][dy][qx][rb];
          bg += sG[qy][dy] * a0;
        }
      }
      BB[dz] = bb;
      GB[dz] = gb;
      BG[dz] = bg;
    }
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
        sC[el][0][dz][qy][qx][rb] = tGB[dz];
        sC[el][1][dz][qy][qx][rb] = tBG[dz];
        sC[el][2][dz][qy][qx][rb] = tBB[dz];
      } else {
        sC[el][0][dz][qy][qx][rb] = tBB[dz];
      }
    }
    __syncthreads();
    if (qy < D) {
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        TC bx = TC(0), gx = TC(0);
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const TC by = sB[q2][qy];
          if (DIFF) {
            gx += by * sC[el][0][dz][q2][qx][rb];
            bx += sG[q2][qy] * sC[el][1][dz][q2][qx][rb] + by * sC[el][2][dz][q2][qx][rb];
          } else {
            bx += by * sC[el][0][dz][q2][qx][rb];
          }
        }
        sA[el][0][dz][qy][qx][rb] = bx;
        if (DIFF) sA[el][NA - 1][dz][qy][qx][rb] = gx;
      }
    }
    __syncthreads();
    if (dof_thread) {
#pragma unroll
      for (int dz = 0; dz < D; ++dz) {
        TC acc = TC(0);
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          acc += sB[q1][qx] * sA[el][0][dz][qy][q1][rb];
          if (DIFF) acc += sG[q1][qx] * sA[el][NA - 1][dz][qy][q1][rb];
        }
        const int g = gidx[dz];
        if (!(constrained && g < 0))
          unsafeAtomicAdd(&Y[size_t(g < 0 ? ~g : g) * nrhs + rr], TV(acc));
      }
    }
    // the next chunk overwrites sU only after every thread finished this one
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
void launch_cfg(const BatchMesh* meshes, int nmesh, int nblocks, int kind, const double* tabB,
                const double* tabG, int nrhs, hipStream_t st) {
  constexpr int Q = P + 2;
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
                 const double* tabB, const double* tabG, int nrhs, hipStream_t st) {
  if (cand == 0) {
    launch_cfg<P, 1, 4, TV, TD, TC>(meshes, nmesh, nblocks, kind, tabB, tabG, nrhs, st);
    return true;
  }
  if (cand == 4) {
    launch_cfg<P, 1, 2, TV, TD, TC>(meshes, nmesh, nblocks, kind, tabB, tabG, nrhs, st);
    return true;
  }
  if constexpr (P <= 5) {
    if (cand == 1) {
      launch_cfg<P, 1, 8, TV, TD, TC>(meshes, nmesh, nblocks, kind, tabB, tabG, nrhs, st);
      return true;
    }
  }
  if constexpr (P <= 4) {
    if (cand == 2) {
      launch_cfg<P, 1, 16, TV, TD, TC>(meshes, nmesh, nblocks, kind, tabB, tabG, nrhs, st);
      return true;
    }
  }
  if constexpr (P <= 3) {
    if (cand == 3) {
      launch_cfg<P, 2, 8, TV, TD, TC>(meshes, nmesh, nblocks, kind, tabB, tabG, nrhs, st);
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
    default: return 0;
  }
}

bool launch_batch_apply(int p, int cand, int vdtype, int qdtype, int kind,
                        const BatchMesh* meshes, int nmesh, int nblocks, const double* tabB,
                        const double* tabG, int nrhs, hipStream_t st) {
  bool ok = false;
#define PAFEM_BATCH_ORDER(PP)                                                                   \
  case PP:                                                                                      \
    if (vdtype == PAFEM_F64 && qdtype == PAFEM_F64)                                             \
      ok = launch_tile<PP, double, double, double>(cand, meshes, nmesh, nblocks, kind, tabB,    \
                                                   tabG, nrhs, st);                             \
    else if (vdtype == PAFEM_F32 && qdtype == PAFEM_F32)                                        \
      ok = launch_tile<PP, float, float, float>(cand, meshes, nmesh, nblocks, kind, tabB, tabG, \
                                                nrhs, st);                                      \
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
