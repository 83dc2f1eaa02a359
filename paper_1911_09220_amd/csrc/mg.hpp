// Order-multigrid kernels (k_mg.hip) and the host side of the preconditioner (mg.cpp).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "internal.hpp"

namespace pafem {

// 1D interpolation tables passed by value: v[half][xf * dc + xc] = coarse Lagrange basis
// function xc (Gauss-Lobatto nodes of the coarse order) at fine Gauss-Lobatto node xf.
// Within one mesh (h == 0) only half 0 is used, at the fine node itself.  Across a
// uniform refinement (h == 1) the fine node is mapped into the lower (half 0) or upper
// (half 1) half of the parent's interval, (half + xf) / 2; fine device element k then
// lies in coarse device element k / 8, octant k % 8 (bit a: upper half along axis a).
constexpr int kMaxInterpNodes = 9;  // orders up to 8
struct Interp1D {
  double v[2][kMaxInterpNodes * kMaxInterpNodes];
  int32_t h;
};

// yf = P xc on free fine dofs (0 on essential ones), or yf += P xc when `add`;
// coarse essential values are read as 0.  Both spaces on one mesh (I.h == 0), or the
// fine one on a uniform refinement of the coarse one's mesh (I.h == 1).
void launch_prolongate(const DevSpace& coarse, const DevSpace& fine, const Interp1D& I,
                       const double* xc, double* yf, bool add, hipStream_t st);
// rc = P^T (bf - yf) (yf may be null), 0 on essential coarse dofs
void launch_restrict(const DevSpace& fine, const DevSpace& coarse, const Interp1D& I,
                     const double* bf, const double* yf, double* rc, hipStream_t st);
void launch_fill(double* y, double v, int64_t n, hipStream_t st);
// Chebyshev-Jacobi: r = b - y (y null: b); d = c0 r/diag; x = d or x + d
void launch_cheb_start(const double* b, const double* y, const double* diag, double* r,
                       double* d, double* x, double c0, bool zero_guess, int64_t n,
                       hipStream_t st);
// r -= y; d = c1 d + c2 r/diag; x += d
void launch_cheb_step(const double* y, const double* diag, double* r, double* d, double* x,
                      double c1, double c2, int64_t n, hipStream_t st);
// Power iteration on D^-1 A.  partials: 2 * kCGBlocks doubles; scal: 1 double.
// v: zero on essential dofs (bmask, may be null), then v /= ||v||_D
void launch_power_norm(double* v, const double* diag, const uint8_t* bmask, double* partials,
                       uint32_t* ticket, double* scal, int64_t n, hipStream_t st);
// w = A v given: *lam = v . w; v = D^-1 w / ||D^-1 w||_D
void launch_power_step(double* v, const double* w, const double* diag, double* partials,
                       uint32_t* ticket, double* scal, double* lam, int64_t n, hipStream_t st);
// out[e][0..nout) = mean of coeff[e][0..nin) (arithmetic, geometric or harmonic)
void launch_coeff_mean(const double* coeff, int64_t ne, int nin, int nout, int kind, double* out,
                       hipStream_t st);

}  // namespace pafem
