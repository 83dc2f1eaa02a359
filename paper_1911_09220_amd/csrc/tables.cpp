// 1D quadrature rules and basis tables on [0,1] (host).
//
// The basis B and its derivative G are the 1D factors B^{1d}_{kj} = phi_j(x_k)
// of the tensor-product basis evaluator ("High-Order Partial Assembly",
// eq. (paB)); quadrature points and weights are the {xhat_k, alpha_k} of the
// mass-matrix equations of the same section.  The H1 basis is nodal at
// Gauss-Lobatto points ("Finite Elements").
//
// Gauss points come from Newton's method on the three-term Legendre
// recurrence; Lobatto points from Newton's method on P_p' using the Legendre
// differential equation for P_p''.  Basis values use barycentric weights and
// derivatives use the nodal differentiation matrix.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace pafem {

namespace {

// Legendre P_n(x) and P_n'(x) on [-1,1].
void legendre(int n, double x, double* pn, double* dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *pn = 1.0;
    *dpn = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *pn = p1;
  // derivative from (1-x^2) P_n' = n (P_{n-1} - x P_n), valid away from +-1
  *dpn = n * (p0 - x * p1) / (1.0 - x * x);
}

}  // namespace

void gauss_legendre_01(int q, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double t = std::cos(pi * (i + 0.75) / (q + 0.5));
    double pn = 0, dpn = 0;
    for (int it = 0; it < 100; ++it) {
      legendre(q, t, &pn, &dpn);
      double dt = pn / dpn;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre(q, t, &pn, &dpn);
    x[i] = 0.5 * (1.0 - t);  // ascending order on [0,1]
    w[i] = 1.0 / ((1.0 - t * t) * dpn * dpn);  // = (2 / ((1-t^2) P'^2)) / 2
  }
}

void gauss_lobatto_01(int n, double* x) {
  const int p = n - 1;
  const double pi = 3.14159265358979323846;
  x[0] = 0.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, dpn;
      legendre(p, t, &pn, &dpn);
      // Legendre ODE: (1-t^2) P'' = 2 t P' - p(p+1) P
      double d2 = (2.0 * t * dpn - p * (p + 1.0) * pn) / (1.0 - t * t);
      double dt = dpn / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = 0.5 * (t + 1.0);
  }
  std::sort(x, x + n);
}

void lagrange_tables(int n, const double* nodes, int npts, const double* pts, double* B,
                     double* G) {
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m)
      if (m != j) lam[j] /= (nodes[j] - nodes[m]);
  // nodal differentiation matrix Dn[k][j] = phi_j'(node_k)
  std::vector<double> Dn(size_t(n) * n, 0.0);
  for (int k = 0; k < n; ++k) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == k) continue;
      double v = (lam[j] / lam[k]) / (nodes[k] - nodes[j]);
      Dn[k * n + j] = v;
      diag -= v;
    }
    Dn[k * n + k] = diag;
  }
  for (int k = 0; k < npts; ++k) {
    const double t = pts[k];
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (t == nodes[j]) hit = j;
    double* b = B + size_t(k) * n;
    if (hit >= 0) {
      for (int j = 0; j < n; ++j) b[j] = (j == hit) ? 1.0 : 0.0;
    } else {
      double s = 0.0;
      for (int j = 0; j < n; ++j) {
        b[j] = lam[j] / (t - nodes[j]);
        s += b[j];
      }
      for (int j = 0; j < n; ++j) b[j] /= s;
    }
    // phi_j' is a polynomial of degree n-2 < n, so it is interpolated exactly
    // by the nodal basis: phi_j'(t) = sum_m phi_m(t) phi_j'(node_m)
    double* g = G + size_t(k) * n;
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int m = 0; m < n; ++m) acc += b[m] * Dn[m * n + j];
      g[j] = acc;
    }
  }
}

std::vector<double> build_tables(int p, int ng) {
  const int D = p + 1;
  std::vector<double> nodes(D), gnodes(ng);
  gauss_lobatto_01(D, nodes.data());
  for (int i = 0; i < ng; ++i) gnodes[i] = double(i) / double(ng - 1);
  std::vector<double> out(table_offset_doubles(kMaxQ1d + 1, D, ng), 0.0);
  for (int Q = 1; Q <= kMaxQ1d; ++Q) {
    double* t = out.data() + table_offset_doubles(Q, D, ng);
    double* pts = t;
    double* wts = t + Q;
    double* B = wts + Q;
    double* G = B + Q * D;
    double* Bg = G + Q * D;
    double* Gg = Bg + Q * ng;
    gauss_legendre_01(Q, pts, wts);
    lagrange_tables(D, nodes.data(), Q, pts, B, G);
    lagrange_tables(ng, gnodes.data(), Q, pts, Bg, Gg);
  }
  return out;
}

// Value tables of the open basis of a Nedelec space (Lagrange polynomials on the p
// Gauss-Legendre points) at the Gauss-Legendre quadrature points, for every q1d.
std::vector<double> build_open_tables(int p) {
  std::vector<double> nodes(p), wdummy(p);
  gauss_legendre_01(p, nodes.data(), wdummy.data());
  std::vector<double> out(nd_open_offset(kMaxQ1d + 1, p), 0.0);
  for (int Q = 1; Q <= kMaxQ1d; ++Q) {
    std::vector<double> pts(Q), wts(Q), G(size_t(Q) * p);
    gauss_legendre_01(Q, pts.data(), wts.data());
    lagrange_tables(p, nodes.data(), Q, pts.data(), out.data() + nd_open_offset(Q, p), G.data());
  }
  return out;
}

}  // namespace pafem
