// Face terms of the upwind DG convection on a discontinuous nodal space of hexahedra
// (convection "including DG" among the partially assembled integrators of "GPU
// Acceleration"); the volume term runs in the fused apply (k_apply.hip).
//
// With the Gauss-Lobatto nodes the trace of an element function on one of its faces
// depends only on the (p+1)^2 dofs of that face, so a face needs no more than its two
// sides' face dofs: each side's trace is evaluated at the Q x Q Gauss points of the
// face by two one-axis contractions, the upwind value times the stored w (beta . N)
// is formed at each point (the "+" side's points reached through the face's
// orientation), and the flux is contracted back onto both sides' face dofs (with
// opposite signs) and added to y with FP64 atomics.  Boundary faces keep the outflow
// part only (zero inflow data).  One workgroup holds several faces, Q*Q threads each.
#include "device.hpp"
#include "launch.hpp"

namespace pafem {

namespace {

#define HIP_LAUNCH_CHECK_DG()                                                     \
  do {                                                                            \
    hipError_t err_ = hipGetLastError();                                          \
    if (err_ != hipSuccess)                                                       \
      throw Error(PAFEM_EHIP, std::string("kernel launch: ") + hipGetErrorString(err_)); \
  } while (0)

// tangential axes of face f = 2 a + side, in increasing order
__host__ __device__ inline void face_axes(int f, int& a, int& b, int& c) {
  a = f / 2;
  b = (a == 0) ? 1 : 0;
  c = (a == 2) ? 1 : 2;
}

// index of the "+" side's point / node for the "-" side's (is, it) on an n x n grid
__device__ inline int face_perm(int orient, int is, int it, int n) {
  int u, v;
  if (orient & 1) {
    u = it;
    v = is;
  } else {
    u = is;
    v = it;
  }
  if (orient & 2) u = n - 1 - u;
  if (orient & 4) v = n - 1 - v;
  return u + n * v;
}

// 1D Lagrange basis on NG equispaced nodes of [0, 1]: value and derivative of node j at x
__device__ inline void geom_basis(int NG, int j, double x, double& val, double& der) {
  const double xj = double(j) / (NG - 1);
  val = 1.0;
  der = 0.0;
  for (int m = 0; m < NG; ++m) {
    if (m == j) continue;
    const double xm = double(m) / (NG - 1);
    double prod = 1.0 / (xj - xm);
    for (int l = 0; l < NG; ++l)
      if (l != j && l != m) prod *= (x - double(l) / (NG - 1)) / (xj - double(l) / (NG - 1));
    der += prod;
    val *= (x - xm) / (xj - xm);
  }
}

// w_s w_t scale (beta . N) at the Q x Q Gauss points of every face, N = T_b x T_c
// oriented outward from the face's first element (the interior face's "-" side); after
// them, one 8-byte slot per face with its two elements' caller indices (the dof blocks
// the face kernel reads and writes), so the apply needs no lookup through elem_orig
__global__ void dg_face_qdata_kernel(const int32_t* __restrict__ faces,
                                     const int32_t* __restrict__ bfaces, int64_t nf, int64_t nb,
                                     const int32_t* __restrict__ orig,
                                     const double* __restrict__ gnodes, int NG,
                                     const double* __restrict__ pts,
                                     const double* __restrict__ wts, int Q,
                                     const double* __restrict__ beta3, double scale,
                                     double* __restrict__ fq) {
  const int64_t g = blockIdx.x;
  if (g >= nf + nb) return;
  int e, f;
  if (g < nf) {
    e = faces[g * kFaceInts + 0];
    f = faces[g * kFaceInts + 2] & 7;
  } else {
    e = bfaces[(g - nf) * 2 + 0];
    f = bfaces[(g - nf) * 2 + 1];
  }
  if (threadIdx.x == 0) {
    int2 o;
    o.x = orig[e];
    o.y = g < nf ? orig[faces[g * kFaceInts + 1]] : 0;
    reinterpret_cast<int2*>(fq + (nf + nb) * Q * Q)[g] = o;
  }
  int a, b, c;
  face_axes(f, a, b, c);
  const int side = f & 1;
  const double* X = gnodes + size_t(e) * NG * NG * NG * 3;
  const double be0 = scale * beta3[0], be1 = scale * beta3[1], be2 = scale * beta3[2];
  // (a, b, c) cyclic: T_b x T_c points along +e_a for the reference cube
  const double sgn = ((a == 1) ? -1.0 : 1.0) * (side ? 1.0 : -1.0);
  for (int q = threadIdx.x; q < Q * Q; q += blockDim.x) {
    const int qs = q % Q, qt = q / Q;
    double xi[3];
    xi[a] = side;
    xi[b] = pts[qs];
    xi[c] = pts[qt];
    double Tb[3] = {0, 0, 0}, Tc[3] = {0, 0, 0};
    for (int k3 = 0; k3 < NG; ++k3)
      for (int k2 = 0; k2 < NG; ++k2)
        for (int k1 = 0; k1 < NG; ++k1) {
          const int kk[3] = {k1, k2, k3};
          double v[3], d[3];
          for (int t = 0; t < 3; ++t) geom_basis(NG, kk[t], xi[t], v[t], d[t]);
          double wb = d[b], wc = d[c];
          for (int t = 0; t < 3; ++t) {
            if (t != b) wb *= v[t];
            if (t != c) wc *= v[t];
          }
          const double* Xk = X + 3 * (k1 + NG * (k2 + NG * k3));
          for (int t = 0; t < 3; ++t) {
            Tb[t] += wb * Xk[t];
            Tc[t] += wc * Xk[t];
          }
        }
    const double N0 = Tb[1] * Tc[2] - Tb[2] * Tc[1];
    const double N1 = Tb[2] * Tc[0] - Tb[0] * Tc[2];
    const double N2 = Tb[0] * Tc[1] - Tb[1] * Tc[0];
    fq[size_t(g) * Q * Q + q] = wts[qs] * wts[qt] * sgn * (be0 * N0 + be1 * N1 + be2 * N2);
  }
}

template <int P>
constexpr int faces_per_block() {
  return (256 / ((P + 2) * (P + 2))) > 0 ? (256 / ((P + 2) * (P + 2))) : 1;
}

template <int P>
__global__ void __launch_bounds__(faces_per_block<P>() * (P + 2) * (P + 2))
    dg_face_kernel(const int32_t* __restrict__ faces, const int32_t* __restrict__ bfaces,
                   int64_t nf, int64_t nb, const double* __restrict__ tabB,
                   const double* __restrict__ fq,
                   const double* __restrict__ x, double* __restrict__ y) {
  constexpr int Q = P + 2, D = P + 1, QQ = Q * Q, DD = D * D, DDD = D * D * D;
  constexpr int FPB = faces_per_block<P>();
  constexpr int PER = 2 * DD + 4 * Q * D + 4 * QQ;  // LDS values per face
  __shared__ double sm[FPB * PER];
  const int lf = threadIdx.x / QQ, r = threadIdx.x - lf * QQ;
  const int64_t g = int64_t(blockIdx.x) * FPB + lf;
  const bool act = g < nf + nb;
  const bool inner = g < nf;
  double* uM = sm + lf * PER;
  double* uP = uM + DD;
  double* tM = uP + DD;
  double* tP = tM + Q * D;
  double* vM = tP + Q * D;
  double* vP = vM + QQ;
  double* FM = vP + QQ;
  double* FP = FM + QQ;
  double* sM = FP + QQ;
  double* sP = sM + Q * D;
  auto bB = [&](int q, int d) { return tabB[q * D + d]; };

  int fm = 0, fp = 0, orient = 0;
  int2 eo = {0, 0};  // the two sides' caller element indices
  if (act) {
    eo = reinterpret_cast<const int2*>(fq + (nf + nb) * QQ)[g];
    if (inner) {
      const int code = faces[g * kFaceInts + 2];
      fm = code & 7;
      fp = (code >> 3) & 7;
      orient = code >> 6;
    } else {
      fm = bfaces[(g - nf) * 2 + 1];
    }
  }
  // face node (i, j) of face f of an element -> lexicographic element dof
  auto face_dof = [&](int f, int i, int j) {
    int a, b, c;
    face_axes(f, a, b, c);
    int idx[3];
    idx[a] = (f & 1) ? P : 0;
    idx[b] = i;
    idx[c] = j;
    return idx[0] + D * (idx[1] + D * idx[2]);
  };
  const int64_t baseM = int64_t(eo.x) * DDD;
  const int64_t baseP = inner ? int64_t(eo.y) * DDD : 0;

  if (act && r < DD) {
    const int i = r % D, j = r / D;
    uM[r] = x[baseM + face_dof(fm, i, j)];
    uP[r] = inner ? x[baseP + face_dof(fp, i, j)] : 0.0;
  }
  __syncthreads();
  if (act && r < Q * D) {
    const int q = r % Q, j = r / Q;
    double am = 0.0, ap = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      am += bB(q, i) * uM[i + D * j];
      ap += bB(q, i) * uP[i + D * j];
    }
    tM[r] = am;
    tP[r] = ap;
  }
  __syncthreads();
  if (act) {
    const int qs = r % Q, qt = r / Q;
    double am = 0.0, ap = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      am += bB(qt, j) * tM[qs + Q * j];
      ap += bB(qt, j) * tP[qs + Q * j];
    }
    vM[r] = am;
    vP[r] = ap;
  }
  __syncthreads();
  if (act) {
    // upwind flux at the "-" side's point r; the "+" side's value at its own index
    const int qs = r % Q, qt = r / Q;
    const double w = fq[size_t(g) * QQ + r];
    if (inner) {
      const int rp = face_perm(orient, qs, qt, Q);
      const double F = w > 0.0 ? w * vM[r] : w * vP[rp];
      FM[r] = F;
      FP[rp] = -F;
    } else {
      FM[r] = w > 0.0 ? w * vM[r] : 0.0;
      FP[r] = 0.0;
    }
  }
  __syncthreads();
  if (act && r < Q * D) {
    const int q = r % Q, j = r / Q;
    double am = 0.0, ap = 0.0;
#pragma unroll
    for (int qt = 0; qt < Q; ++qt) {
      am += bB(qt, j) * FM[q + Q * qt];
      ap += bB(qt, j) * FP[q + Q * qt];
    }
    sM[r] = am;
    sP[r] = ap;
  }
  __syncthreads();
  if (act && r < DD) {
    const int i = r % D, j = r / D;
    double am = 0.0, ap = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      am += bB(q, i) * sM[q + Q * j];
      ap += bB(q, i) * sP[q + Q * j];
    }
    unsafeAtomicAdd(&y[baseM + face_dof(fm, i, j)], am);
    if (inner) unsafeAtomicAdd(&y[baseP + face_dof(fp, i, j)], ap);
  }
}

template <int P>
void launch_faces_p(const DevSpace& sp, const double* tabB, const double* fq, const double* x,
                    double* y, hipStream_t st) {
  constexpr int Q = P + 2, FPB = faces_per_block<P>();
  const int64_t total = sp.nfaces + sp.nbfaces;
  if (total == 0) return;
  const unsigned nblk = unsigned((total + FPB - 1) / FPB);
  hipLaunchKernelGGL((dg_face_kernel<P>), dim3(nblk), dim3(FPB * Q * Q), 0, st, sp.faces,
                     sp.bfaces, sp.nfaces, sp.nbfaces, tabB, fq, x, y);
}

}  // namespace

void launch_dg_face_qdata(const DevSpace& sp, int q1d, const double* beta3, double scale,
                          double* fq, hipStream_t st) {
  const int64_t total = sp.nfaces + sp.nbfaces;
  if (total == 0) return;
  const double* t = sp.tables + table_offset_doubles(q1d, sp.p + 1, sp.ng);
  hipLaunchKernelGGL(dg_face_qdata_kernel, dim3(unsigned(total)), dim3(128), 0, st, sp.faces,
                     sp.bfaces, sp.nfaces, sp.nbfaces, sp.elem_orig, sp.gnodes, sp.ng, t, t + q1d,
                     q1d, beta3, scale, fq);
  HIP_LAUNCH_CHECK_DG();
}

void launch_dg_faces(const DevSpace& sp, int q1d, const double* fq, const double* x, double* y,
                     hipStream_t st) {
  if (q1d != sp.p + 2) throw Error(PAFEM_EUNSUPPORTED, "DG faces are built for q1d = p + 2");
  const double* tabB = sp.tables + table_offset_doubles(q1d, sp.p + 1, sp.ng) + 2 * q1d;
  switch (sp.p) {
    case 1: launch_faces_p<1>(sp, tabB, fq, x, y, st); break;
    case 2: launch_faces_p<2>(sp, tabB, fq, x, y, st); break;
    case 3: launch_faces_p<3>(sp, tabB, fq, x, y, st); break;
    case 4: launch_faces_p<4>(sp, tabB, fq, x, y, st); break;
    case 5: launch_faces_p<5>(sp, tabB, fq, x, y, st); break;
    case 6: launch_faces_p<6>(sp, tabB, fq, x, y, st); break;
    case 7: launch_faces_p<7>(sp, tabB, fq, x, y, st); break;
    case 8: launch_faces_p<8>(sp, tabB, fq, x, y, st); break;
    default: throw Error(PAFEM_EUNSUPPORTED, "DG faces: order not built");
  }
  HIP_LAUNCH_CHECK_DG();
}

}  // namespace pafem
