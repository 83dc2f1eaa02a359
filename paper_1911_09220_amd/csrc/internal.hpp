// Internal declarations shared by the host code and the kernel launchers of
// the partial-assembly library.  Not part of the public C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "pafem.h"

namespace pafem {

constexpr int kMaxOrder = 8;
// kernel-internal operator kinds: kVectorKind + kind applies `kind` to each of three
// components (PAFEM_OP_VECTOR3)
constexpr int kVectorKind = 16;
// kernel-internal: kGradCompKind + c is output component c of PAFEM_GRADIENT alone
// (its one-accumulator form, used from p = 5 on)
constexpr int kGradCompKind = 32;
constexpr int kMaxQ1d = 12;  // 1D tables are built for every q1d in [1, kMaxQ1d]

inline bool known_kind(int kind) {
  return kind == PAFEM_MASS || kind == PAFEM_DIFFUSION || kind == PAFEM_DIFFUSION_GEOM ||
         kind == PAFEM_CONVECTION || kind == PAFEM_GRADIENT || kind == PAFEM_DIVERGENCE ||
         kind == PAFEM_ELASTICITY || kind == PAFEM_HCURL_MASS || kind == PAFEM_HCURL_CURLCURL ||
         kind == PAFEM_HCURL_MAXWELL || kind == PAFEM_DG_CONVECTION;
}
// operators on L2 spaces
inline bool l2_kind(int kind) { return kind == PAFEM_DG_CONVECTION; }

// operators on Nedelec spaces
inline bool nd_kind(int kind) {
  return kind == PAFEM_HCURL_MASS || kind == PAFEM_HCURL_CURLCURL || kind == PAFEM_HCURL_MAXWELL;
}
// stored values per quadrature point of each operator kind (hexahedra)
inline int qdata_components(int kind) {
  switch (kind) {
    case PAFEM_DIFFUSION: case PAFEM_HCURL_MASS: case PAFEM_HCURL_CURLCURL: return 6;
    case PAFEM_HCURL_MAXWELL: return 12;
    case PAFEM_DG_CONVECTION: return 3;
    case PAFEM_CONVECTION: return 3;
    case PAFEM_GRADIENT: case PAFEM_DIVERGENCE: return 9;
    case PAFEM_ELASTICITY: return 11;
    default: return 1;
  }
}
// operators that are not symmetric positive definite on one scalar space (mixed,
// non-symmetric or vector-valued): no diagonal, no CG
inline bool mixed_or_nonsymmetric(int kind) {
  return kind == PAFEM_CONVECTION || kind == PAFEM_GRADIENT || kind == PAFEM_DIVERGENCE ||
         kind == PAFEM_ELASTICITY;
}

// Thrown inside the library and turned into a status at the C boundary.
struct Error : std::runtime_error {
  pafem_status code;
  Error(pafem_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Quadrature data is stored tile-interleaved: elements are grouped in tiles of
// qdata_tile(Q) consecutive elements, and within a tile the values are ordered
// [component][qz][element in tile][qy][qx] (the diffusion D in component pairs, below).  One load instruction of the fused
// apply (all threads of a tile reading component c at plane qz) is then one
// contiguous run.  The last tile is padded.
constexpr int qdata_tile(int Q) { return (256 / (Q * Q)) > 0 ? (256 / (Q * Q)) : 1; }
// Offset of value (e, component c, point q = qz*Q*Q + r) with nc components.
// The six values of the diffusion D (and the twelve of the definite Maxwell form)
// are stored in pairs: components 2k and 2k+1 of a point are adjacent ([pair][qz][element in tile][qy][qx][2]), so the apply reads a
// pair with one 16-byte load per thread (FP64) and a workgroup's pair plane is still
// one contiguous run.
constexpr size_t qdata_index(int64_t e, int c, int q, int Q, int nc) {
  const int nt = qdata_tile(Q), qq = Q * Q;
  const int64_t tile = e / nt;
  const int el = int(e - tile * nt);
  const int qz = q / qq, r = q - qz * qq;
  if (nc == 6 || nc == 12)
    return ((size_t(tile) * (nc / 2) + c / 2) * Q + qz) * size_t(nt * qq) * 2 +
           (size_t(el) * qq + r) * 2 + (c & 1);
  return ((size_t(tile) * nc + c) * Q + qz) * size_t(nt * qq) + size_t(el) * qq + r;
}
// Quadrilaterals: tiles of qdata_tile_2d(Q) elements (Q threads per element in the
// apply), within a tile [component][qy][element in tile][qx].
constexpr int qdata_tile_2d(int Q) { return (256 / Q) > 0 ? (256 / Q) : 1; }
constexpr size_t qdata_index_2d(int64_t e, int c, int q, int Q, int nc) {
  const int nt = qdata_tile_2d(Q);
  const int64_t tile = e / nt;
  const int el = int(e - tile * nt);
  const int qy = q / Q, qx = q - qy * Q;
  return ((size_t(tile) * nc + c) * Q + qy) * size_t(nt * Q) + size_t(el) * Q + qx;
}
inline int64_t qdata_values_2d(int64_t ne, int Q, int nc) {
  const int nt = qdata_tile_2d(Q);
  return ((ne + nt - 1) / nt) * nt * int64_t(nc) * Q * Q;
}
inline int64_t qdata_values(int64_t ne, int Q, int nc) {
  const int nt = qdata_tile(Q);
  return ((ne + nt - 1) / nt) * nt * int64_t(nc) * Q * Q * Q;
}

// ---- 1D tables (tables.cpp) -------------------------------------------------
// Gauss-Legendre rule on [0,1]: points and weights, ascending.
void gauss_legendre_01(int q, double* x, double* w);
// Gauss-Lobatto points on [0,1], ascending, n >= 2.
void gauss_lobatto_01(int n, double* x);
// Lagrange basis on `nodes` (n of them): B[k*n+j] = phi_j(pts[k]),
// G[k*n+j] = phi_j'(pts[k]).
void lagrange_tables(int n, const double* nodes, int npts, const double* pts, double* B,
                     double* G);

// Per-q1d table block, in doubles: pts[Q] wts[Q] B[Q*D] G[Q*D] Bg[Q*NG] Gg[Q*NG]
// (D = basis dofs per direction, NG = geometry nodes per direction).
inline size_t table_block_doubles(int Q, int D, int NG) {
  return size_t(2 * Q + 2 * Q * D + 2 * Q * NG);
}
inline size_t table_offset_doubles(int Q, int D, int NG) {
  size_t off = 0;
  for (int q = 1; q < Q; ++q) off += table_block_doubles(q, D, NG);
  return off;
}
std::vector<double> build_tables(int p, int ng);

// ---- device image of a space -------------------------------------------------
// Device image.  Element arrays are in the device element order (a Morton order
// of element centroids, so consecutive elements -- and each apply tile -- are
// spatially compact); elem_orig maps back to the caller's element numbering.
struct DevSpace {
  const int32_t* gmap = nullptr;       // [ne][dpe], essential dofs stored as ~g
  const double* gnodes = nullptr;      // [ne][NG^3][3]
  const uint8_t* bmask = nullptr;      // [ndofs] 1 on essential dofs
  const int32_t* toff = nullptr;       // [ndofs+1] transposed map offsets
  const int32_t* tidx = nullptr;       // [ne*D^3] element-vector entries per dof (ascending)
  const double* tables = nullptr;      // 1D tables for q1d = 1..kMaxQ1d
  const float* tables32 = nullptr;     // the same tables rounded to FP32 (FP32 kernels)
  int32_t* status = nullptr;           // [64] small device status words
  const int32_t* elem_orig = nullptr;  // [ne] caller element id of each device element
  const int32_t* tile_off = nullptr;   // [ntiles+1] offsets into tile_dofs
  const int32_t* tile_dofs = nullptr;  // unique dofs of each apply tile (~g if essential)
  const uint16_t* tile_slot = nullptr; // [ntiles*tile_ne*D^3] node -> index in its tile's list
  const uint32_t* owner = nullptr;     // [ne][owner_words(D^dim)] first-occurrence bits
  const int8_t* sign = nullptr;        // Nedelec: [ne][dpe] orientation sign of each local dof
  const double* tables_open = nullptr; // Nedelec: open-basis tables for q1d = 1..kMaxQ1d
  const int32_t* faces = nullptr;      // L2: interior faces [nfaces][kFaceInts]
  const int32_t* bfaces = nullptr;     // L2: boundary faces [nbfaces][2]
  int64_t nfaces = 0, nbfaces = 0;
  int64_t ne = 0, ndofs = 0;
  int p = 0, ng = 0, tile_ne = 0;
  int dim = 3;                         // 3: hexahedra, 2: quadrilaterals
  int family = 0;                      // kFamilyH1 or kFamilyND
};

struct Mesh {
  int dim = 3;                 // 3: hexahedra, 2: quadrilaterals
  int64_t nv = 0, ne = 0;
  std::vector<double> xyz;     // [nv][dim]
  std::vector<int64_t> hex;    // [ne][8] (dim 3)
  std::vector<int64_t> quad;   // [ne][4] counter-clockwise (dim 2)
  int geom_order = 1;
  std::vector<double> gnodes;  // [ne][27][3] for geom_order 2
  uint64_t id = 0;             // unique per mesh object (next_mesh_id)
  uint64_t parent_id = 0;      // id of the mesh this one refines uniformly (0: none)
  std::vector<int32_t> elem_order;  // device element order of a refined mesh (else Morton)
};

uint64_t next_mesh_id();
// Device element order of the mesh: Morton order of the element centroids, or for a
// refined mesh the children 8 e + 0..7 of each parent e in the parent's device order,
// so that device element k of the refined mesh lies in device element k / 8 of its
// parent, octant k % 8.
std::vector<int32_t> mesh_element_order(const Mesh& m);
// Uniform refinement of a hexahedral mesh: child 8 e + o (o = ox + 2 oy + 4 oz) of
// element e covers the octant [o/2, (o+1)/2] of its reference cube, axes kept; new
// vertices at the edge midpoints, face and cell centres of the parent's map (coarse
// vertices keep their ids, then one vertex per edge, face and element); a quadratic
// geometry gives each child the parent's map at its 27 nodes.
void refine_mesh(const Mesh& c, Mesh& f);

// space families: nodal H1 (Gauss-Lobatto nodes) and Nedelec H(curl)
constexpr int kFamilyH1 = 0;
constexpr int kFamilyND = 1;
constexpr int kFamilyL2 = 2;
// interior face of an L2 space: device elements of its two sides and
// code = f_minus | f_plus << 3 | orientation << 6 (f = 2 * axis + side; orientation:
// bit 0 swap, bit 1 reverse u, bit 2 reverse v, mapping the "-" side's face indices
// (s, t) to the "+" side's (u, v); s, u along the lower tangential axis)
constexpr int kFaceInts = 3;
// the family an operator kind needs
inline int kind_family(int kind) {
  return nd_kind(kind) ? kFamilyND : l2_kind(kind) ? kFamilyL2 : kFamilyH1;
}

// Open-basis (Gauss-Legendre nodes, p of them) value table B_o[q][k] for each q1d,
// stored one block after another: block Q starts at nd_open_offset(Q, p) doubles.
inline size_t nd_open_offset(int Q, int p) { return size_t(p) * size_t(Q - 1) * size_t(Q) / 2; }
std::vector<double> build_open_tables(int p);

struct Space {
  const Mesh* mesh = nullptr;
  int family = kFamilyH1;
  int dim = 3;
  int p = 0, D1 = 0, dpe = 0, ng = 0;
  int64_t ne = 0, ndofs = 0;
  std::vector<int32_t> gmap;      // [ne][dpe] dof ids, caller element order
  std::vector<int32_t> dev_order; // device element position -> caller element id
  int tile_ne = 0;                // elements per apply tile (qdata_tile(p + 2), 2D: qdata_tile_2d)
  std::vector<int32_t> tile_off, tile_dofs;
  std::vector<uint16_t> tile_slot;
  std::vector<uint8_t> bmask;     // [ndofs]
  std::vector<int32_t> bdr;       // essential dofs ascending
  std::vector<double> ref_nodes;  // Gauss-Lobatto nodes [D1]
  std::vector<double> tables;     // build_tables(p, ng)
  std::vector<int8_t> gsign;      // Nedelec: [ne][dpe] dof signs, caller element order
  std::vector<int32_t> faces;     // L2: [nfaces][kFaceInts] interior faces (device elements)
  std::vector<int32_t> bfaces;    // L2: [nbfaces][2] boundary faces (device element, face)
  std::vector<double> tables_open;  // Nedelec: build_open_tables(p)
  // device image (caller-owned buffer)
  void* dev_buf = nullptr;
  size_t dev_bytes = 0;
  DevSpace dev;
  bool uploaded = false;
};

// space.cpp
Space* build_space(const Mesh* mesh, int order, int flags);
// Nedelec space of order p on hexahedra: local dof (a, i0, i1, i2) component-major,
// lexicographic (first index fastest), open index along a, closed along the others
Space* build_nd_space(const Mesh* mesh, int order, int flags);
inline int nd_dofs_per_elem(int p) { return 3 * p * (p + 1) * (p + 1); }
// Discontinuous nodal space of order p on hexahedra: element e (caller order) owns dofs
// e * (p+1)^3 + i, i lexicographic on the Gauss-Lobatto nodes; interior and boundary
// face lists for the face terms
Space* build_l2_space(const Mesh* mesh, int order, int flags);
void space_dof_coords(const Space& s, double* xyz);
constexpr int kSpaceSegments = 17;
// words of the per-element owner bitmask (bit i of element k: node i is the first
// occurrence of its dof in device element order)
inline int owner_words(int dpe) { return (dpe + 31) / 32; }
void space_device_layout(const Space& s, size_t* offsets /*[kSpaceSegments+1]*/, size_t* total);
// host copies of every device array, in upload order
void space_pack(const Space& s, std::vector<int32_t>& gmap_enc, std::vector<double>& gnodes,
                std::vector<int32_t>& toff, std::vector<int32_t>& tidx,
                std::vector<uint32_t>& owner);

struct Op {
  const Space* space = nullptr;
  int kind = PAFEM_DIFFUSION;
  int q1d = 0;
  const void* qdata = nullptr;
  int qdtype = PAFEM_F64;
  int flags = 0;
};

}  // namespace pafem
