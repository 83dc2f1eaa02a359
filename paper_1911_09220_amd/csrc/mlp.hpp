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

// ---- learned preconditioner (k_learned.hip) ----
// feats[e] = {kbar_e, 8 octant log-ratios} per device element, from kappa [E][Q^3]
// in caller element order (NULL: kbar = 1, ratios 0).
void launch_patch_features(const DevSpace& sp, const double* kappa, int q1d, float* feats,
                           hipStream_t st);
// X[e] = bf16([r_E / s_e, ratios, 0...]) and s[e] = ||r_E||
void launch_patch_inputs(const DevSpace& sp, const double* r, const float* feats, int in_pad,
                         uint16_t* X, float* s, hipStream_t st);
// ye[e][i] = (s_e / kbar_e) out[e][i]
void launch_patch_outputs(const DevSpace& sp, const float* out, int out_pad, const float* s,
                          const float* feats, double* ye, hipStream_t st);
// z = r / diag + (sum of ye over the dof's element nodes) / multiplicity; 0 on essential dofs
void launch_precond_gather(const DevSpace& sp, const double* ye, const double* r,
                           const double* diag, double* z, hipStream_t st);
// dout[e][i] = (s_e / kbar_e) * g[dof] / multiplicity(dof) * gscale[0], as bf16 [E][out_pad]
void launch_patch_output_grad(const DevSpace& sp, const double* g, const double* gscale,
                              const float* s, const float* feats, int out_pad, uint16_t* dout,
                              hipStream_t st);

// t = a - b
void launch_diff(const double* a, const double* b, double* t, int64_t n, hipStream_t st);
// training loss: v = u / diag, scal = {loss, -2 / (r.D^-1 r)}; partials >= 2*512 doubles
void launch_loss(const DevSpace& sp, const double* u, const double* r, const double* diag,
                 double* v, double* partials, uint32_t* ticket, double* scal, hipStream_t st);
// z = r / diag, 0 on essential dofs
void launch_jacobi(const DevSpace& sp, const double* r, const double* diag, double* z,
                   hipStream_t st);

}  // namespace pafem
