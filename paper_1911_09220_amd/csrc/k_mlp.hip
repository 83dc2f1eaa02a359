// BF16 matrix-core (MFMA) kernels of the element-patch network: forward layers,
// backward layers, weight gradients and Adam.  Inputs and weights are bfloat16,
// accumulation is FP32 (v_mfma_f32_16x16x16_bf16), master weights FP32.
//
// Operand layout of the 16x16x16 bf16 MFMA on a 64-lane wave (lane l, j = 0..3):
//   A[i][k]: lane l holds A[l % 16][4 * (l / 16) + j]
//   B[k][n]: lane l holds B[4 * (l / 16) + j][l % 16]
//   C[i][n]: lane l holds C[4 * (l / 16) + j][l % 16]
#include "device.hpp"
#include "mlp.hpp"

namespace pafem {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

constexpr int kRowsPerBlock = 64;  // 4 waves x 16 rows
constexpr int kPad = 8;            // LDS row padding (bf16 elements)

// C[M][N] = epilogue(A[M][K] . B[N][K]^T), K and N multiples of 16, N <= 128, K <= 256.
//   EPI_RELU_BF16: out bf16 = relu(acc + bias)
//   EPI_BIAS_F32:  out f32  = acc + bias
//   EPI_MASK_BF16: out bf16 = acc * (mask > 0)   (mask: bf16 [M][N], the forward activation)
template <int EPI>
__global__ void __launch_bounds__(256)
    gemm_rows_kernel(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                     const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                     void* __restrict__ out, int M, int N, int K) {
  extern __shared__ uint16_t lds[];
  const int ldk = K + kPad;
  uint16_t* sA = lds;
  uint16_t* sB = lds + kRowsPerBlock * ldk;
  const int row0 = blockIdx.x * kRowsPerBlock;
  for (int i = threadIdx.x; i < kRowsPerBlock * K; i += blockDim.x) {
    const int r = i / K, k = i - r * K;
    sA[r * ldk + k] = (row0 + r < M) ? A[size_t(row0 + r) * K + k] : uint16_t(0);
  }
  for (int i = threadIdx.x; i < N * K; i += blockDim.x) {
    const int n = i / K, k = i - n * K;
    sB[n * ldk + k] = B[i];
  }
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int li = lane % 16, lk = 4 * (lane / 16);
  v4f acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  const int ntiles = N / 16;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const uint16_t* pa = sA + (wave * 16 + li) * ldk + k0 + lk;
    const v4s a = {short(pa[0]), short(pa[1]), short(pa[2]), short(pa[3])};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t < ntiles) {
        const uint16_t* pb = sB + (t * 16 + li) * ldk + k0 + lk;
        const v4s b = {short(pb[0]), short(pb[1]), short(pb[2]), short(pb[3])};
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (t >= ntiles) continue;
    const int n = t * 16 + li;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row0 + wave * 16 + lk + j;
      if (row >= M) continue;
      float v = acc[t][j];
      if (EPI == kEpiReluBf16) {
        v = fmaxf(v + bias[n], 0.f);
        static_cast<uint16_t*>(out)[size_t(row) * N + n] = f2bf(v);
      } else if (EPI == kEpiBiasF32) {
        static_cast<float*>(out)[size_t(row) * N + n] = v + bias[n];
      } else {
        const float mk = bf2f(mask[size_t(row) * N + n]);
        static_cast<uint16_t*>(out)[size_t(row) * N + n] = f2bf(mk > 0.f ? v : 0.f);
      }
    }
  }
}

constexpr int kWgradRows = 128;  // rows reduced per workgroup

// Partial weight gradient of one row chunk: P[blk][N][K] = sum_m Z[m][n] X[m][k] and
// Pb[blk][n] = sum_m Z[m][n], rows m of the chunk.  Z: bf16 [M][N], X: bf16 [M][K].
__global__ void __launch_bounds__(256)
    gemm_wgrad_kernel(const uint16_t* __restrict__ Z, const uint16_t* __restrict__ X,
                      float* __restrict__ part, float* __restrict__ partb, int M, int N, int K) {
  extern __shared__ uint16_t lds[];
  uint16_t* sZ = lds;                        // [kWgradRows][N]
  uint16_t* sX = lds + kWgradRows * N;       // [kWgradRows][K]
  const int m0 = blockIdx.x * kWgradRows;
  for (int i = threadIdx.x; i < kWgradRows * N; i += blockDim.x) {
    const int r = i / N;
    sZ[i] = (m0 + r < M) ? Z[size_t(m0) * N + i] : uint16_t(0);
  }
  for (int i = threadIdx.x; i < kWgradRows * K; i += blockDim.x) {
    const int r = i / K;
    sX[i] = (m0 + r < M) ? X[size_t(m0) * K + i] : uint16_t(0);
  }
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int li = lane % 16, lk = 4 * (lane / 16);
  const int tn = N / 16, tk = K / 16, ntile = tn * tk;
  float* P = part + size_t(blockIdx.x) * N * K;
  // each wave takes every 4th output tile
  for (int t0 = wave; t0 < ntile; t0 += 4 * 4) {
    v4f acc[4];
    int tiles[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
      tiles[u] = t0 + 4 * u;
    }
    for (int mm = 0; mm < kWgradRows; mm += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = tiles[u];
        if (t >= ntile) continue;
        const int nt = t / tk, kt = t - nt * tk;
        // A'[n][m] = Z[m][n]; B'[m][k] = X[m][k]
        const int n = nt * 16 + li, k = kt * 16 + li;
        const v4s a = {short(sZ[(mm + lk + 0) * N + n]), short(sZ[(mm + lk + 1) * N + n]),
                       short(sZ[(mm + lk + 2) * N + n]), short(sZ[(mm + lk + 3) * N + n])};
        const v4s b = {short(sX[(mm + lk + 0) * K + k]), short(sX[(mm + lk + 1) * K + k]),
                       short(sX[(mm + lk + 2) * K + k]), short(sX[(mm + lk + 3) * K + k])};
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[u], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = tiles[u];
      if (t >= ntile) continue;
      const int nt = t / tk, kt = t - nt * tk;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        P[size_t(nt * 16 + lk + j) * K + kt * 16 + li] = acc[u][j];
    }
  }
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    float s = 0.f;
    for (int r = 0; r < kWgradRows; ++r) s += bf2f(sZ[r * N + n]);
    partb[size_t(blockIdx.x) * N + n] = s;
  }
}

// grad[i] = sum over blocks of part[blk][i], in a fixed order: a workgroup takes
// kRedEntries consecutive entries; lane group j (kRedLanes of them) sums the blocks
// b = j, j + kRedLanes, ... and the groups' sums are added in index order.
constexpr int kRedEntries = 32, kRedLanes = 8;  // kRedEntries * kRedLanes = 256 threads
__global__ void __launch_bounds__(256)
    reduce_parts_kernel(const float* __restrict__ part, float* __restrict__ grad, int nblk,
                        int n) {
  __shared__ float sp[kRedLanes][kRedEntries];
  const int e = threadIdx.x % kRedEntries, j = threadIdx.x / kRedEntries;
  const int i = blockIdx.x * kRedEntries + e;
  float s = 0.f;
  if (i < n)
    for (int b = j; b < nblk; b += kRedLanes) s += part[size_t(b) * n + i];
  sp[j][e] = s;
  __syncthreads();
  if (j == 0 && i < n) {
    float t = sp[0][e];
    for (int k = 1; k < kRedLanes; ++k) t += sp[k][e];
    grad[i] = t;
  }
}

int reduce_grid(int n) { return (n + kRedEntries - 1) / kRedEntries; }

// Adam on the FP32 master parameters, then refresh the bf16 copies (weights and
// the transposed weights used by the input-gradient GEMMs).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int n, float lr,
                            float beta1, float beta2, float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void cast_weights_kernel(const float* __restrict__ W, uint16_t* __restrict__ Wb,
                                    uint16_t* __restrict__ Wtb, int rows, int cols) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows * cols;
       i += gridDim.x * blockDim.x) {
    const int r = i / cols, c = i - r * cols;
    const uint16_t b = f2bf(W[i]);
    Wb[i] = b;
    if (Wtb) Wtb[size_t(c) * rows + r] = b;
  }
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                   int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = f2bf(src[i]);
}

void check(const char* what) {
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

int grid1d(int64_t n) {
  int64_t g = (n + 255) / 256;
  return int(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

void launch_gemm_rows(int epi, const uint16_t* A, const uint16_t* B, const float* bias,
                      const uint16_t* mask, void* out, int M, int N, int K, hipStream_t st) {
  if (N % 16 || K % 16 || N > 128 || K > 256 || N <= 0 || K <= 0)
    throw Error(PAFEM_EINVAL, "gemm_rows: N, K multiples of 16, N <= 128, K <= 256");
  if (M <= 0) return;
  const dim3 grid((M + kRowsPerBlock - 1) / kRowsPerBlock);
  const size_t lds = sizeof(uint16_t) * size_t(kRowsPerBlock + N) * (K + kPad);
  if (epi == kEpiReluBf16)
    hipLaunchKernelGGL(gemm_rows_kernel<kEpiReluBf16>, grid, dim3(256), lds, st, A, B, bias, mask,
                       out, M, N, K);
  else if (epi == kEpiBiasF32)
    hipLaunchKernelGGL(gemm_rows_kernel<kEpiBiasF32>, grid, dim3(256), lds, st, A, B, bias, mask,
                       out, M, N, K);
  else
    hipLaunchKernelGGL(gemm_rows_kernel<kEpiMaskBf16>, grid, dim3(256), lds, st, A, B, bias, mask,
                       out, M, N, K);
  check("gemm_rows");
}

int wgrad_blocks(int M) { return (M + kWgradRows - 1) / kWgradRows; }

void launch_gemm_wgrad(const uint16_t* Z, const uint16_t* X, float* part, float* partb,
                       float* gW, float* gb, int M, int N, int K, hipStream_t st) {
  if (N % 16 || K % 16 || N > 128 || K > 256 || N <= 0 || K <= 0)
    throw Error(PAFEM_EINVAL, "gemm_wgrad: N, K multiples of 16, N <= 128, K <= 256");
  const int nblk = wgrad_blocks(M);
  const size_t lds = sizeof(uint16_t) * size_t(kWgradRows) * (N + K);
  hipLaunchKernelGGL(gemm_wgrad_kernel, dim3(nblk), dim3(256), lds, st, Z, X, part, partb, M, N, K);
  check("gemm_wgrad");
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(reduce_grid(N * K)), dim3(256), 0, st, part, gW,
                     nblk, N * K);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(reduce_grid(N)), dim3(256), 0, st, partb, gb, nblk,
                     N);
  check("reduce_parts");
}

void launch_reduce_parts(const float* part, float* out, int nblk, int n, hipStream_t st) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(reduce_grid(n)), dim3(256), 0, st, part, out, nblk,
                     n);
  check("reduce_parts");
}

void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float beta1,
                 float beta2, float eps, int step, hipStream_t st) {
  const float c1 = 1.f - powf(beta1, float(step)), c2 = 1.f - powf(beta2, float(step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid1d(n)), dim3(256), 0, st, p, g, m, v, n, lr, beta1,
                     beta2, eps, c1, c2);
  check("adam");
}

void launch_cast_weights(const float* W, uint16_t* Wb, uint16_t* Wtb, int rows, int cols,
                         hipStream_t st) {
  hipLaunchKernelGGL(cast_weights_kernel, dim3(grid1d(int64_t(rows) * cols)), dim3(256), 0, st, W,
                     Wb, Wtb, rows, cols);
  check("cast_weights");
}

void launch_f32_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(grid1d(n)), dim3(256), 0, st, src, dst, n);
  check("f32_to_bf16");
}

}  // namespace pafem
