// Host-callable kernel launchers (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime_api.h>

#include "internal.hpp"

namespace pafem {

// ---- setup (k_setup.hip) ----
// status[0] must hold INT32_MAX on entry; receives the smallest element with det J <= 0.
void launch_qdata(const DevSpace& sp, int kind, int q1d, const double* coeff, double scale,
                  double* qd, hipStream_t st);
// element vectors of the linear form into ye [ne][D^3]
void launch_linear_form_evec(const DevSpace& sp, int q1d, int source, const double* fqp,
                             double scale, double* ye, hipStream_t st);
// element diagonals into ye [ne][D^3]
void launch_diagonal_evec(const DevSpace& sp, int kind, int q1d, const double* qd,
                          double* ye, hipStream_t st);
// y[g] = sum of element-vector entries of dof g; essential dofs per bc_mode:
// 0 plain sum, 1 y = x (x required), 2 y = bc_value
void launch_evec_gather(const DevSpace& sp, const double* ye, const double* x, int bc_mode,
                        double bc_value, double* y, hipStream_t st);
void launch_evec_gather_f32(const DevSpace& sp, const float* ye, const float* x, int bc_mode,
                            float* y, hipStream_t st);
// y = x on essential dofs (constrained) and 0 elsewhere: start of an atomic scatter
void launch_scatter_init(const DevSpace& sp, const double* x, bool constrained, double* y,
                         hipStream_t st);
void launch_scatter_init_f32(const DevSpace& sp, const float* x, bool constrained, float* y,
                             hipStream_t st);

// ---- apply (k_apply.hip) ----
// Fused G -> B -> D -> B^t -> G^t.  evec: write element vectors to `out`
// [ne][D^3] instead of atomically adding into the dof vector `out`.  dotp (may be
// null): receives pa_apply_blocks(sp) partial sums of the element energies
// u_E . A_E u_E (essential inputs 0 when constrained), one per workgroup.
// Returns false if (p, q1d, dtype) is not instantiated.
// isotropic linear elasticity on the vector space (k_elastic.hip); false when the order
// is not built
bool launch_elasticity(const DevSpace& sp, bool constrained, const double* qd, const double* x,
                       double* y, hipStream_t st);
bool launch_pa_apply(const DevSpace& sp, int kind, int q1d, int qdtype, bool constrained,
                     bool evec, const void* qd, const void* x, void* out, int vdtype,
                     hipStream_t st, double* dotp = nullptr);
int pa_apply_blocks(const DevSpace& sp);
// DG convection (k_dg.hip): the face values w (beta . N) of every interior face, then of
// every boundary face, Q^2 per face (beta = scale * beta3[0..2], device)
void launch_dg_face_qdata(const DevSpace& sp, int q1d, const double* beta3, double scale,
                          double* fq, hipStream_t st);
// adds the upwind face terms of the DG convection to y
void launch_dg_faces(const DevSpace& sp, int q1d, const double* fq, const double* x, double* y,
                     hipStream_t st);
// H(curl) mass / curl-curl / definite Maxwell apply on a Nedelec space (k_hcurl.hip);
// false when the order, q1d or kind is not built
bool launch_nd_apply(const DevSpace& sp, int kind, int q1d, bool constrained, const double* qd,
                     const double* x, double* y, hipStream_t st, double* dotp = nullptr);

// ---- quadrilaterals (k_2d.hip); the launchers above dispatch to these when sp.dim == 2 ----
void launch_qdata_2d(const DevSpace& sp, int kind, int q1d, const double* coeff, double scale,
                     double* qd, hipStream_t st);
void launch_linear_form_evec_2d(const DevSpace& sp, int q1d, int source, const double* fqp,
                                double scale, double* ye, hipStream_t st);
void launch_diagonal_evec_2d(const DevSpace& sp, int kind, int q1d, const double* qd, double* ye,
                             hipStream_t st);
int pa_apply2d_blocks(const DevSpace& sp);
// FP64, atomic scatter only
bool launch_pa_apply_2d(const DevSpace& sp, int kind, bool constrained, const double* qd,
                        const double* x, double* y, hipStream_t st, double* dotp);

}  // namespace pafem
