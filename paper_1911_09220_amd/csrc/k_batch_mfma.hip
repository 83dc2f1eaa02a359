// Batched operator action on the matrix cores (FP64 MFMA), for the many-right-hand-side
// form: with 16 right-hand sides the one-axis contractions of sum factorization
// ("High-Order Partial Assembly") are dense products
//     out[(m) ; (line, rhs)] = T[m ; k] . in[k ; (line, rhs)],
// the 1D table T as the 16 x 4 A operand (its rows padded to 16, k to a multiple of 4)
// and, for each line of the element, the k x 16 slice of the data (k along the axis,
// the right-hand sides across) as the B operand of v_mfma_f64_16x16x4f64.  The tables
// sit in registers for the whole kernel; data pass through LDS between stages (each
// stage's output rows are the next stage's k).  One workgroup = one element x 16
// right-hand sides, 4 waves sharing each stage's lines:
//   x:  [B;G] (2Q rows) on each (dz, dy) line          -> W1[arr][dz][qx][dy][rhs]
//   y:  [B;G] on the B array, B on the G array          -> W2[c][qx][qy][dz][rhs]
//   z:  B, B, G on the three arrays of each (qx, qy) line, D at the points (FP64, the
//       quadrature data of the single apply), then B^t, B^t, G^t back along z, in place
//   y^t, x^t: the transposed tables; the x^t output (rows dx, columns rhs) goes to Y
//       with FP64 atomics, 16 consecutive right-hand sides of a dof per row.
// Operand layout of v_mfma_f64_16x16x4f64 (checked on the device): lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and, in its result register i, D[l / 16 + 4 i][l % 16].
#include "batch.hpp"
#include "device.hpp"

namespace pafem {

namespace {

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mfma_d4 mfma16(double a, double b, mfma_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int P, int KIND>
__global__ void __launch_bounds__(256)
    pa_apply_mrhs_mfma_kernel(const BatchMesh* __restrict__ meshes, int nmesh,
                              const double* __restrict__ tabB, const double* __restrict__ tabG,
                              int nrhs) {
  constexpr int D = P + 1, Q = P + 2, QQ = Q * Q, R = 16;
  constexpr bool DIFF = (KIND == PAFEM_DIFFUSION);
  constexpr int KD = (D + 3) / 4, KQ = (Q + 3) / 4;  // k-steps over D and over Q
  constexpr int NA = DIFF ? 2 : 1;                   // arrays after x (and before x^t)
  constexpr int NC = DIFF ? 3 : 1;                   // arrays after y (and before y^t)
  constexpr int W1N = NA * D * Q * D * R;
  constexpr int W2N = NC * Q * Q * D * R;
  constexpr int INN = D * D * D * R;
  static_assert(2 * Q <= 16, "table rows must fit one 16-row operand");
  static_assert(INN <= W2N, "the gathered element must fit the y-stage region");
  __shared__ double sW1[W1N];
  __shared__ double sW2[W2N];   // also holds the gathered input before the y stage
  __shared__ double sT[4][16 * R];  // per-wave transposes of point values
  double* const sIn = sW2;

  int m = 0;
  const int blk = blockIdx.x;
  while (m + 1 < nmesh && meshes[m + 1].block_begin <= blk) ++m;
  const BatchMesh& M = meshes[m];
  const int e = blk - M.block_begin;  // one element per workgroup
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int lr = lane % 16, lg = lane / 16;  // operand column (rhs) / row group
  const int32_t* __restrict__ gmap = M.gmap + size_t(e) * D * D * D;
  const double* __restrict__ X = static_cast<const double*>(M.x);
  double* __restrict__ Y = static_cast<double*>(M.y);
  const double* __restrict__ qd = static_cast<const double*>(M.qdata);

  // A operands: forward tables (rows = outputs, k = inputs) and transposed ones
  auto tB = [&](int q, int d) { return (q < Q && d < D) ? tabB[q * D + d] : 0.0; };
  auto tG = [&](int q, int d) { return (q < Q && d < D) ? tabG[q * D + d] : 0.0; };
  double aBG[KD], aB[KD], aG[KD], aBt[KQ], aGt[KQ];
#pragma unroll
  for (int s = 0; s < KD; ++s) {
    const int k = 4 * s + lg, row = lr;
    aB[s] = tB(row, k);
    aG[s] = tG(row, k);
    aBG[s] = row < Q ? tB(row, k) : tG(row - Q, k);
  }
#pragma unroll
  for (int s = 0; s < KQ; ++s) {
    const int k = 4 * s + lg, row = lr;  // row: output dof index, k: point index
    aBt[s] = tB(k, row);
    aGt[s] = tG(k, row);
  }

  for (int r0 = 0; r0 < nrhs; r0 += R) {
    // gather: node n = dx + D (dy + D dz), rhs r -> sIn[n * R + r]
    for (int i = tid; i < INN; i += 256) {
      const int n = i / R, r = i % R;
      const int g = gmap[n];
      sIn[i] = (M.constrained && g < 0) ? 0.0 : X[size_t(g < 0 ? ~g : g) * nrhs + r0 + r];
    }
    __syncthreads();

    // x: line (dz, dy), k = dx
    for (int b = wave; b < D * D; b += 4) {
      const int dz = b / D, dy = b % D;
      mfma_d4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KD; ++s) {
        const int k = 4 * s + lg;
        const double bv = k < D ? sIn[((dz * D + dy) * D + k) * R + lr] : 0.0;
        c = mfma16(DIFF ? aBG[s] : aB[s], bv, c);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = lg + 4 * i;
        if (row < NA * Q) {
          const int arr = row / Q, qx = row - arr * Q;
          sW1[(((arr * D + dz) * Q + qx) * D + dy) * R + lr] = c[i];
        }
      }
    }
    __syncthreads();

    // y: line (arr, dz, qx), k = dy; arr 0 (B along x) -> bb (c = 2) and bg (c = 1),
    // arr 1 (G along x) -> gb (c = 0); mass: one array, c = 0
    for (int b = wave; b < NA * D * Q; b += 4) {
      const int arr = b / (D * Q), dz = (b / Q) % D, qx = b % Q;
      mfma_d4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KD; ++s) {
        const int k = 4 * s + lg;
        const double bv = k < D ? sW1[(((arr * D + dz) * Q + qx) * D + k) * R + lr] : 0.0;
        c = mfma16((DIFF && arr == 0) ? aBG[s] : aB[s], bv, c);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = lg + 4 * i;
        int cc = -1, qy = 0;
        if (!DIFF) {
          if (row < Q) cc = 0, qy = row;
        } else if (arr == 0) {
          if (row < Q) cc = 2, qy = row;
          else if (row < 2 * Q) cc = 1, qy = row - Q;
        } else if (row < Q) {
          cc = 0, qy = row;
        }
        if (cc >= 0) sW2[(((cc * Q + qx) * Q + qy) * D + dz) * R + lr] = c[i];
      }
    }
    __syncthreads();

    // z, D, z^t: line (qx, qy), k = dz forward, k = qz back; in place in sW2
    double* const tw = sT[wave];
    for (int b = wave; b < QQ; b += 4) {
      const int qx = b % Q, qy = b / Q;
      mfma_d4 u[NC];
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        u[cc] = mfma_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KD; ++s) {
          const int k = 4 * s + lg;
          const double bv = k < D ? sW2[(((cc * Q + qx) * Q + qy) * D + k) * R + lr] : 0.0;
          // gb -> d/dx (B along z), bg -> d/dy (B), bb -> d/dz (G); mass: B
          u[cc] = mfma16((DIFF && cc == 2) ? aG[s] : aB[s], bv, u[cc]);
        }
      }
      // point operator at rows qz = lg + 4 i (all right-hand sides share D)
      mfma_d4 v[NC];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int qz = lg + 4 * i;
        if (qz < Q) {
          const int q = qz * QQ + qy * Q + qx;
          if constexpr (DIFF) {
            double d[6];
#pragma unroll
            for (int k = 0; k < 3; ++k)
              load_pair<double, double>(qd + qdata_index(e, 2 * k, q, Q, 6), d[2 * k],
                                        d[2 * k + 1]);
            const double ux = u[0][i], uy = u[1][i], uz = u[2][i];
            v[0][i] = d[0] * ux + d[1] * uy + d[2] * uz;
            v[1][i] = d[1] * ux + d[3] * uy + d[4] * uz;
            v[2][i] = d[2] * ux + d[4] * uy + d[5] * uz;
          } else {
            v[0][i] = __builtin_nontemporal_load(qd + qdata_index(e, 0, q, Q, 1)) * u[0][i];
          }
        } else {
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) v[cc][i] = 0.0;
        }
      }
      // back along z: rows (dz) from k = qz; v goes through the wave's LDS scratch to
      // become a B operand (rows qz across the lane groups)
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
#pragma unroll
        for (int i = 0; i < 4; ++i) tw[(lg + 4 * i) * R + lr] = v[cc][i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        mfma_d4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KQ; ++s) {
          const int k = 4 * s + lg;
          const double bv = k < 16 ? tw[k * R + lr] : 0.0;
          t = mfma16((DIFF && cc == 2) ? aGt[s] : aBt[s], bv, t);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int dz = lg + 4 * i;
          if (dz < D) sW2[(((cc * Q + qx) * Q + qy) * D + dz) * R + lr] = t[i];
        }
      }
    }
    __syncthreads();

    // y^t: line (dz, qx), k = qy; diffusion: g = B^t t0 -> arr 1, b = G^t t1 + B^t t2
    // -> arr 0; mass: B^t t0 -> arr 0.  Output rows dy, layout W1[arr][dz][dy][qx][rhs]
    for (int b = wave; b < D * Q; b += 4) {
      const int dz = b / Q, qx = b % Q;
      mfma_d4 g = {0.0, 0.0, 0.0, 0.0}, bb = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KQ; ++s) {
        const int k = 4 * s + lg;
        auto at = [&](int cc) {
          return k < Q ? sW2[(((cc * Q + qx) * Q + k) * D + dz) * R + lr] : 0.0;
        };
        if constexpr (DIFF) {
          g = mfma16(aBt[s], at(0), g);
          bb = mfma16(aGt[s], at(1), bb);
          bb = mfma16(aBt[s], at(2), bb);
        } else {
          bb = mfma16(aBt[s], at(0), bb);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int dy = lg + 4 * i;
        if (dy < D) {
          sW1[(((0 * D + dz) * D + dy) * Q + qx) * R + lr] = bb[i];
          if (DIFF) sW1[(((1 * D + dz) * D + dy) * Q + qx) * R + lr] = g[i];
        }
      }
    }
    __syncthreads();

    // x^t: line (dz, dy), k = qx: B^t on arr 0 plus G^t on arr 1; rows dx -> Y
    for (int b = wave; b < D * D; b += 4) {
      const int dz = b / D, dy = b % D;
      mfma_d4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KQ; ++s) {
        const int k = 4 * s + lg;
        const double b0 = k < Q ? sW1[(((0 * D + dz) * D + dy) * Q + k) * R + lr] : 0.0;
        c = mfma16(aBt[s], b0, c);
        if constexpr (DIFF) {
          const double b1 = k < Q ? sW1[(((1 * D + dz) * D + dy) * Q + k) * R + lr] : 0.0;
          c = mfma16(aGt[s], b1, c);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int dx = lg + 4 * i;
        if (dx < D) {
          const int g = gmap[dx + D * (dy + D * dz)];
          if (!(M.constrained && g < 0))
            unsafeAtomicAdd(&Y[size_t(g < 0 ? ~g : g) * nrhs + r0 + lr], c[i]);
        }
      }
    }
    // the next chunk's gather overwrites sW2 only after every wave is done here
    __syncthreads();
  }
}

}  // namespace

bool launch_batch_apply_mfma(int p, int kind, const BatchMesh* meshes, int nmesh, int nblocks,
                             const double* tabB, int nrhs, hipStream_t st) {
  const double* tabG = tabB + (p + 2) * (p + 1);
#define PAFEM_MFMA_ORDER(PP)                                                                  \
  case PP:                                                                                    \
    if (kind == PAFEM_DIFFUSION)                                                              \
      hipLaunchKernelGGL((pa_apply_mrhs_mfma_kernel<PP, PAFEM_DIFFUSION>), dim3(nblocks),     \
                         dim3(256), 0, st, meshes, nmesh, tabB, tabG, nrhs);                  \
    else                                                                                      \
      hipLaunchKernelGGL((pa_apply_mrhs_mfma_kernel<PP, PAFEM_MASS>), dim3(nblocks),          \
                         dim3(256), 0, st, meshes, nmesh, tabB, tabG, nrhs);                  \
    return true;
  switch (p) {
    PAFEM_MFMA_ORDER(1)
    PAFEM_MFMA_ORDER(2)
    PAFEM_MFMA_ORDER(3)
    PAFEM_MFMA_ORDER(4)
    default:
      return false;
  }
#undef PAFEM_MFMA_ORDER
}

}  // namespace pafem
