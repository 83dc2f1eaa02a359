// Element-patch network kernels (k_mlp.hip) and learned-preconditioner
// kernels (k_learned.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "internal.hpp"

namespace pafem {

constexpr int kEpiReluBf16 = 0;  // out bf16 = relu(acc + bias)
constexpr int kEpiBiasF32 = 1;   // out f32 = acc + bias
constexpr int kEpiMaskBf16 = 2;  // out bf16 = acc * (mask > 0)

// C[M][N] = epilogue(A[M][K] . B[N][K]^T): bf16 operands, FP32 MFMA accumulation.
void launch_gemm_rows(int epi, const uint16_t* A, const uint16_t* B, const float* bias,
                      const uint16_t* mask, void* out, int M, int N, int K, hipStream_t st);
// gW[N][K] = sum_m Z[m][n] X[m][k], gb[n] = sum_m Z[m][n] (two deterministic passes
// through part [wgrad_blocks(M)][N][K] and partb [wgrad_blocks(M)][N]).
int wgrad_blocks(int M);
void launch_gemm_wgrad(const uint16_t* Z, const uint16_t* X, float* part, float* partb,
                       float* gW, float* gb, int M, int N, int K, hipStream_t st);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float beta1,
                 float beta2, float eps, int step, hipStream_t st);
void launch_cast_weights(const float* W, uint16_t* Wb, uint16_t* Wtb, int rows, int cols,
                         hipStream_t st);
void launch_f32_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t st);

// part [nblk][n] -> out[n], summed over blocks in index order
void launch_reduce_parts(const float* part, float* out, int nblk, int n, hipStream_t st);

// ---- learned preconditioner (k_learned.hip) ----
constexpr int kLowRank = 16;            // columns of the learned element basis V
constexpr int kLowRankGradBlocks = 256;  // workgroups of the basis-gradient reduction
constexpr int kLowRankApplyBlocks = 2048;  // persistent workgroups of the per-iteration apply

// feats[e] = {kbar_e, 8 octant log-ratios} per device element, from kappa [E][Q^3]
// in caller element order (NULL: kbar = 1, ratios 0).
void launch_patch_features(const DevSpace& sp, const double* kappa, int q1d, float* feats,
                           hipStream_t st);
// X[e] = bf16([8 log-ratios, 0...]), in_pad columns
void launch_net_inputs(const DevSpace& sp, const float* feats, int in_pad, uint16_t* X,
                       hipStream_t st);
// c[e][k] = softplus(a[e][k]) (a: network output [E][kLowRank]); idb[e] = 1 / dbar_E
void launch_lowrank_coeffs(const DevSpace& sp, const double* diag, const float* a, float* c,
                           float* idb, hipStream_t st);
// z += sum_E R_E^t V diag(c_E idb_E) V^t R_E r on non-essential dofs; V [(p+1)^3][kLowRank]
void launch_lowrank_apply(const DevSpace& sp, const float* V, const float* c, const float* idb,
                          const double* r, double* z, hipStream_t st);
// For dL/dz = gscale[0] * g: network output gradient dout (bf16 [E][kLowRank]) and the
// basis gradient gV [(p+1)^3][kLowRank]; part holds kLowRankGradBlocks * (p+1)^3 * kLowRank floats
void launch_lowrank_grad(const DevSpace& sp, const float* V, const float* c, const float* idb,
                         const double* r, const double* g, const double* gscale, uint16_t* dout,
                         float* part, float* gV, hipStream_t st);

// t = a - b
void launch_diff(const double* a, const double* b, double* t, int64_t n, hipStream_t st);
// training loss: v = u / diag, scal = {loss, -2 / (r.D^-1 r)}; partials >= 2*512 doubles
void launch_loss(const DevSpace& sp, const double* u, const double* r, const double* diag,
                 double* v, double* partials, uint32_t* ticket, double* scal, hipStream_t st);
// z = r / diag, and on the essential dofs: 0 (kJacobiEssZero, the learned
// preconditioner's own definition), r (kJacobiEssKeep: a constrained operator is the
// identity there) or r / diag as elsewhere (kJacobiEssDiag: an unconstrained operator)
constexpr int kJacobiEssZero = 0, kJacobiEssKeep = 1, kJacobiEssDiag = 2;
void launch_jacobi(const DevSpace& sp, const double* r, const double* diag, double* z,
                   hipStream_t st, int ess_mode = kJacobiEssZero);

}  // namespace pafem
