/*
 * pafem.h -- C ABI of the MI355X partial-assembly finite element library.
 *
 * The library computes the matrix-free ("partially assembled") action of H1
 * diffusion and mass operators on unstructured hexahedral meshes,
 *      y = G^t B^t D B G x,
 * where G is the element restriction (global dofs -> element dofs), B the
 * basis evaluation at quadrature points (applied by sum factorization with 1D
 * tables), and D the stored quadrature-point operator.  Notation and the
 * factorization follow the MFEM paper (arXiv:1911.09220), sections
 * "Operator Decomposition" and "High-Order Partial Assembly"; the problem is
 * the weak form of "Finite Element Abstractions": find u_h in V_h with
 * a(u_h, v_h) = l(v_h) for all v_h, a(u,v) = int kappa grad u . grad v,
 * l(v) = int f v, with essential (Dirichlet) boundary conditions imposed as
 * in FormLinearSystem ("Finite Element Linear Systems").
 *
 * Conventions (every call):
 *  - Return value: PAFEM_OK (0) or a negative status; a message describing the
 *    last error of the calling thread is available from pafem_last_error().
 *    No C++ exception crosses this boundary.
 *  - Handles (mesh, space, op) are host objects owned by the library; release
 *    them with the matching *_destroy call.  Destroying a space or mesh that an
 *    op still references is undefined.
 *  - "device" pointers are HIP device memory owned by the caller (typically
 *    torch tensors); the library never frees caller memory and never
 *    allocates device memory itself.  Scratch memory comes from caller
 *    workspaces whose size is queried first (pafem_op_apply_noalloc instead
 *    uses one fixed device array of the library, loaded with its code).
 *  - stream is a hipStream_t (NULL = default stream).  Calls are asynchronous
 *    on that stream unless marked SYNCHRONOUS.  An asynchronous HIP failure is
 *    reported as PAFEM_EHIP by a later synchronous call.
 *  - Reference element [0,1]^3.  Element dofs are lexicographic
 *    i = i1 + D1*(i2 + D1*i3), D1 = p+1, nodes at Gauss-Lobatto points.
 *    Quadrature points are tensor Gauss-Legendre points, lexicographic
 *    q = q1 + Q*(q2 + Q*q3), Q = q1d.
 *  - Hex connectivity: 8 vertex indices per element in the usual order, bottom
 *    face (0,0,0) (1,0,0) (1,1,0) (0,1,0), then the top face in the same order.
 */
#ifndef PAFEM_H
#define PAFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pafem_status;

#define PAFEM_OK 0
#define PAFEM_EINVAL (-1)       /* invalid argument: null pointer, bad index, bad mesh, det J <= 0 */
#define PAFEM_ESHAPE (-2)       /* buffer or workspace too small, size mismatch */
#define PAFEM_EUNSUPPORTED (-3) /* order / q1d / dtype / kind combination not built */
#define PAFEM_EHIP (-4)         /* HIP runtime error (launch, copy, asynchronous fault) */
#define PAFEM_ENOTCONV (-5)     /* solver stopped at max_iter before reaching the tolerance */
#define PAFEM_EBREAKDOWN (-6)   /* CG breakdown: p.Ap <= 0 or a non-finite scalar */

/* Operator kinds ("High-Order Partial Assembly": mass; "Finite Element
 * Abstractions": diffusion). */
#define PAFEM_MASS 0
#define PAFEM_DIFFUSION 1
/* The diffusion operator storing only a portion of D ("High-Order Partial
 * Assembly" lets PA store portions of D and recompute the rest): qdata holds
 * alpha_q kappa_q per point, and the apply recomputes J, det J and J^{-1} J^{-T}
 * from the element's trilinear geometry nodes.  Same operator as
 * PAFEM_DIFFUSION up to rounding; FP64, trilinear meshes only; the diagonal is
 * taken from a PAFEM_DIFFUSION operator of the same space and coefficient. */
#define PAFEM_DIFFUSION_GEOM 2
/* Convection a(u, v) = int (beta . grad u) v, one of the integrators the paper
 * lists among its partially assembled kernels ("GPU Acceleration"): D_q =
 * alpha_q det J_q J_q^{-1} beta_q (3 values per point), applied as
 * B^t (D . (B G u)).  Not symmetric: no diagonal, no CG.  FP64, hexahedra. */
#define PAFEM_CONVECTION 3
/* Gradient, the mixed form (grad u, v) with v vector-valued in the same H1
 * space (the gradient integrator of "GPU Acceleration"): D_q = alpha_q kappa_q
 * det J_q J_q^{-T} (9 values per point), applied as three value contractions
 * B^t (D (B G u))_c.  The output has 3 * ndofs values, component-major
 * (y[c * ndofs + i]).  Unconstrained (flags 0), atomic scatter, FP64,
 * hexahedra, orders 1..8 (from p = 5 on, one pass per output component). */
#define PAFEM_GRADIENT 4
/* Divergence, the mixed form (div u, q) with u vector-valued in the same H1
 * space as the scalar test function q (the divergence integrator of "GPU
 * Acceleration"): the same D_q as PAFEM_GRADIENT (the qdata of either kind
 * serves both), applied as B^t (sum_c (D (B G u_c))_c).  The input has
 * 3 * ndofs values, component-major (x[c * ndofs + i]), the output ndofs.
 * Unconstrained (flags 0), atomic scatter, FP64, hexahedra. */
#define PAFEM_DIVERGENCE 5
/* Isotropic linear elasticity on the vector H1 space, a(u, v) = int lambda
 * (div u)(div v) + 2 mu eps(u) : eps(v) with eps(u) = (grad u + grad u^T)/2 (the
 * vector-valued integrators of "GPU Acceleration"): qdata per point J^{-1} (9
 * values), alpha det J lambda and alpha det J mu, from a coefficient array of
 * (lambda, mu) pairs per point, [E][Q^3][2].  x and y have 3 * ndofs values,
 * component-major; PAFEM_OP_CONSTRAINED eliminates the essential dofs of every
 * component (y_c = x_c there).  Atomic scatter, FP64, hexahedra, orders 1..8; no
 * diagonal or CG on it. */
#define PAFEM_ELASTICITY 6

/* Nedelec (H(curl)) operators, on a space from pafem_space_create_nd: the forms of
 * the definite Maxwell problem of the paper's Example 3 ("Discrete de Rham
 * Complex"; the H(curl) integrators of "GPU Acceleration").  With the covariant
 * map u = J^{-T} uhat and curl u = J curlhat uhat / det J:
 *   PAFEM_HCURL_MASS      (beta u, v):           D_q = w beta det J J^{-1} J^{-T}
 *                          (the same 6 values per point as PAFEM_DIFFUSION)
 *   PAFEM_HCURL_CURLCURL  (alpha curl u, curl v): D_q = w alpha J^T J / det J (6 values)
 *   PAFEM_HCURL_MAXWELL   the sum of both, coefficients as (alpha, beta) pairs per
 *                          point [E][Q^3][2] (12 values per point)
 * Constrained (tangential essential dofs eliminated) or not; atomic scatter; FP64. */
#define PAFEM_HCURL_MASS 7
#define PAFEM_HCURL_CURLCURL 8
#define PAFEM_HCURL_MAXWELL 9

/* Upwind DG convection on a space from pafem_space_create_l2 (convection "including
 * DG" among the partially assembled integrators of "GPU Acceleration"): the steady
 * transport term div(beta u) with a constant velocity beta, zero inflow data,
 *   a(u, v) = -sum_K int_K u beta . grad v + sum_F int_F (beta . n) u_up (v^- - v^+)
 *             + int_{outflow} (beta . n) u v,
 * n from the face's "-" element to its "+" element, u_up the trace on the side the
 * flow leaves.  qdata: per volume point w adj(J) beta (3 values, the layout of
 * PAFEM_CONVECTION), then per interior face and per boundary face the Q^2 values
 * w (beta . N) at the face's Gauss points (N the area-weighted normal, outward from
 * the face's "-" element), then per face one 8-byte slot holding its "-" and "+"
 * elements' indices (caller order, int32 each; 0 for the "+" side of a boundary face);
 * coeff of pafem_qdata_assemble: device beta[3].
 * Unconstrained, atomic scatter, FP64, not symmetric (no diagonal or CG). */
#define PAFEM_DG_CONVECTION 10

/* Space families (pafem_space_family). */
#define PAFEM_SPACE_H1 0
#define PAFEM_SPACE_ND 1
#define PAFEM_SPACE_L2 2

/* Storage types. */
#define PAFEM_F64 0
#define PAFEM_F32 1
#define PAFEM_BF16 2

/* Space creation flags. */
#define PAFEM_SPACE_RENUMBER 1 /* number dofs by first touch in element order (locality);
                                  default is vertices, edges, faces, interiors */

/* Operator flags. */
#define PAFEM_OP_CONSTRAINED 1  /* eliminate essential dofs: y_b = x_b on boundary dofs and
                                   boundary columns dropped (symmetric elimination) */
#define PAFEM_OP_SCATTER_EVEC 2 /* G^t by writing element vectors and gathering them per dof
                                   through the transposed element->dof map: deterministic,
                                   needs a workspace.  Default: hardware FP atomics. */
#define PAFEM_OP_VECTOR3 4      /* the operator on each component of a vector-valued H1
                                   function (vector mass / vector diffusion): x and y hold
                                   3 * ndofs values, component-major; D is read once for the
                                   three components.  Mass or diffusion, FP64, hexahedra,
                                   atomic scatter; no diagonal or solvers (use the scalar
                                   operator per component). */

/* Built-in sources for pafem_linear_form. */
#define PAFEM_SOURCE_ARRAY 0 /* f given at quadrature points, device [E][Q^3] f64 */
#define PAFEM_SOURCE_CONST 1 /* f = scale */
#define PAFEM_SOURCE_SINE 2  /* f = scale * 3 pi^2 sin(pi x) sin(pi y) sin(pi z) */

/* Preconditioners for pafem_pcg_solve. */
#define PAFEM_PRECOND_NONE 0
#define PAFEM_PRECOND_JACOBI 1

typedef struct pafem_mesh_s* pafem_mesh;
typedef struct pafem_space_s* pafem_space;
typedef struct pafem_op_s* pafem_op;

/* Message of the last failed call on this thread ("" if none). */
const char* pafem_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int32_t pafem_version(void);

/* ---------------------------------------------------------------- mesh --- */

/* Conforming hexahedral mesh ("Meshes / Conforming Meshes").  Host call.
 *  nv, xyz:        vertex count and coordinates, host [nv][3] f64 (copied).
 *  ne, hex8:       element count and connectivity, host [ne][8] int64 (copied).
 *  geom_order:     1 = trilinear map from the vertices; 2 = quadratic map from
 *                  27 nodes per element (the nodal mesh description).
 *  geom_nodes:     NULL for geom_order 1; host [ne][27][3] f64 lexicographic
 *                  nodes at reference positions {0,1/2,1}^3 for geom_order 2.
 * Errors: EINVAL on null pointers, nv/ne <= 0, an index outside [0,nv), or an
 * element repeating a vertex. */
pafem_status pafem_mesh_create_hex(int64_t nv, const double* xyz, int64_t ne,
                                   const int64_t* hex8, int32_t geom_order,
                                   const double* geom_nodes, pafem_mesh* out);

/* A conforming quadrilateral mesh ("Meshes", 2D): nv vertices xy[nv][2], ne
 * elements quad4[ne][4] listing each element's vertices counter-clockwise from
 * its reference origin ((0,0), (1,0), (1,1), (0,1)); bilinear geometry.  Spaces
 * on it are 2D: (p+1)^2 dofs per element, Q^2 quadrature points per element,
 * diffusion qdata holds the symmetric 2x2 operator (3 values per point).  2D
 * operators are FP64 with the atomic scatter; the mixed-precision, batched,
 * learned and multigrid entry points return EUNSUPPORTED for them.
 * Errors: EINVAL (index out of range, repeated vertex). */
pafem_status pafem_mesh_create_quad(int64_t nv, const double* xy, int64_t ne, const int64_t* quad4,
                                    pafem_mesh* out);
/* Uniform refinement of a hexahedral mesh ("Meshes"; the nested mesh hierarchy of
 * multigrid in the mesh size, "Scalable Linear Solvers").  Child 8 e + o
 * (o = ox + 2 oy + 4 oz) of element e covers the octant [o/2, (o+1)/2]^3 of e's
 * reference cube with its axes along e's, so its map is e's map on the octant and the
 * coarse mesh's spaces lie in the refined mesh's.  Vertices: the coarse ones keep
 * their ids, then one per edge midpoint, face centre and element centre (placed by
 * the parent's map); a quadratic geometry gives each child the parent's map at its 27
 * nodes.  The refined mesh records its parent, for transfers between spaces of the
 * two (pafem_prolongate); it does not reference the coarse object, which may be
 * destroyed first.  Host call.  Errors: EUNSUPPORTED (quadrilateral mesh), ESHAPE
 * (more than 2^27 coarse elements). */
pafem_status pafem_mesh_refine(pafem_mesh coarse, pafem_mesh* fine);
/* Vertex and element counts of a mesh ("Meshes"), e.g. of a refined one.  Either
 * pointer may be NULL.  Host call.  Errors: EINVAL (null mesh). */
pafem_status pafem_mesh_info(pafem_mesh mesh, int64_t* nv, int64_t* ne);
/* Copies of the vertex coordinates (host [nv][dim] f64) and the connectivity (host
 * [ne][8] in the usual hexahedron vertex order, or [ne][4] counter-clockwise for
 * quadrilaterals, int64) of a mesh ("Meshes"), sized by pafem_mesh_info; either
 * pointer may be NULL.  Caller-owned host memory.  Host call.  Errors: EINVAL (null
 * mesh). */
pafem_status pafem_mesh_vertices(pafem_mesh mesh, double* xyz, int64_t* elems);
void pafem_mesh_destroy(pafem_mesh mesh);

/* --------------------------------------------------------------- space --- */

/* Order-p H1 space with nodal Lagrange basis at Gauss-Lobatto points
 * ("Finite Element Discretization"): builds the element->dof map G with
 * orientation-consistent edge and face dofs, the essential (boundary) dof
 * set -- every dof on a face that belongs to one element only -- and the
 * transposed map used by the deterministic scatter.  Host call.
 *  order: 1..8.  flags: PAFEM_SPACE_RENUMBER or 0.
 * Errors: EUNSUPPORTED for order outside 1..8; EINVAL on a non-conforming mesh
 * (a face shared by more than two elements). */
pafem_status pafem_space_create_h1(pafem_mesh mesh, int32_t order, int32_t flags,
                                   pafem_space* out);
void pafem_space_destroy(pafem_space space);

/* Nedelec (H(curl)-conforming) space of order 1..8 on a hexahedral mesh
 * ("Discrete de Rham Complex"; vector dofs as in "Finite Elements": the dof of a
 * basis function is its dot product with a fixed vector at its node).  Local dof
 * (a, i0, i1, i2), component-major, first index fastest: component a is the
 * product of the open basis (Lagrange on the p Gauss-Legendre points) along axis
 * a and the closed basis (Lagrange on the p+1 Gauss-Lobatto points) along the
 * other two; 3 p (p+1)^2 dofs per element.  Global numbering: edge dofs (p per
 * edge, from its smaller to its larger vertex id), face dofs (2 p (p-1) per face),
 * interiors.  Orientation: the global basis function along local axis a is the
 * local one when the smallest vertex id among the dof entity's corners with c_a = 1
 * exceeds the smallest among those with c_a = 0, else its negative (interior dofs
 * are never negated); pafem_space_elem_signs returns these signs.  Essential dofs:
 * every dof on a boundary face (the tangential trace).  The other pafem_space_*
 * calls work as for H1 spaces (dof coordinates are the dof nodes).  Host call.
 * Errors: EINVAL (bad mesh), EUNSUPPORTED (order, quadrilateral mesh). */
pafem_status pafem_space_create_nd(pafem_mesh mesh, int32_t order, int32_t flags,
                                   pafem_space* out);
/* Discontinuous (L2) space of order 1..8 on a hexahedral mesh ("Discrete de Rham
 * Complex"; nodal Lagrange basis on the (p+1)^3 Gauss-Lobatto points of every
 * element, no continuity): element e of the caller's numbering owns dofs
 * e * (p+1)^3 + i, i lexicographic; no essential dofs.  The space also records its
 * interior faces (with the orientation between the two sides) and boundary faces
 * for the face terms of PAFEM_DG_CONVECTION.  Host call.  Errors as
 * pafem_space_create_h1. */
pafem_status pafem_space_create_l2(pafem_mesh mesh, int32_t order, int32_t flags,
                                   pafem_space* out);
/* PAFEM_SPACE_H1, PAFEM_SPACE_ND or PAFEM_SPACE_L2. */
pafem_status pafem_space_family(pafem_space space, int32_t* family);
/* signs[ne * dofs_per_elem] (+1 / -1) of each element's local dofs in the global
 * basis, caller element order; all +1 for an H1 space.  Host call. */
pafem_status pafem_space_elem_signs(pafem_space space, int8_t* signs);

/* Sizes: global dofs, elements, dofs per element ((p+1)^3), essential dofs. */
pafem_status pafem_space_info(pafem_space space, int64_t* ndofs, int64_t* nelem,
                              int32_t* dofs_per_elem, int64_t* nbdr);

/* Spatial dimension of the space's mesh (3 hexahedra, 2 quadrilaterals). */
pafem_status pafem_space_dim(pafem_space space, int32_t* dim);
/* Host copies: dof node coordinates [ndofs][dim] f64; essential dof indices
 * [nbdr] int32 ascending; element->dof map [nelem][(p+1)^dim] int32. */
pafem_status pafem_space_dof_coords(pafem_space space, double* xyz);
pafem_status pafem_space_boundary_dofs(pafem_space space, int32_t* idx);
pafem_status pafem_space_elem_dofs(pafem_space space, int32_t* gmap);

/* Device image of the space (element->dof map, geometry nodes, transposed map,
 * boundary mask, 1D tables).  Query the size, allocate a device buffer of at
 * least that many bytes (256-byte aligned), then upload.  The buffer must stay
 * alive and unmodified while the space is used.  pafem_space_upload is
 * SYNCHRONOUS.  Errors: ESHAPE if nbytes is too small. */
pafem_status pafem_space_device_bytes(pafem_space space, size_t* nbytes);
pafem_status pafem_space_upload(pafem_space space, void* device_buf, size_t nbytes,
                                void* stream);

/* ------------------------------------------------------ quadrature data --- */

/* Number of stored values of the quadrature-point operator D
 * ("High-Order Partial Assembly": storing only D):
 *   mass:      E * Q^3       D_q = alpha_q det J_q rho_q
 *   diffusion: E * 6 * Q^3   D_q = alpha_q kappa_q det J_q J_q^{-1} J_q^{-T},
 *                            symmetric, components (00,01,02,11,12,22),
 *                            layout [E][6][Q^3].
 *   diffusion with recomputed geometry (PAFEM_DIFFUSION_GEOM): E * Q^3 values
 *                            alpha_q kappa_q.
 *   convection: E * 3 * Q^3  D_q = alpha_q det J_q J_q^{-1} beta_q.
 *   gradient:   E * 9 * Q^3  D_q = alpha_q kappa_q det J_q J_q^{-T}, [c][b] with c the
 *                            output component and b the reference derivative.
 *   divergence: the gradient's layout and values (c the input component).
 *   elasticity: E * 11 * Q^3  J^{-1} as [b][d] (9), alpha det J lambda, alpha det J mu.
 * Quadrilateral spaces: Q^2 points per element, diffusion 3 components
 * (00, 01, 11), mass 1.  All layouts are padded to whole apply tiles.
 * Errors: EUNSUPPORTED if q1d is not one of the built rules (q1d = p+2). */
pafem_status pafem_qdata_size(pafem_space space, int32_t kind, int32_t q1d, int64_t* nvalues);

/* PA setup: geometric factors (Jacobian of the element map at every
 * quadrature point) and D, written as f64 to device `qdata`.
 *  coeff: device [E][Q^3] f64 coefficient (kappa or rho) or NULL for 1; for
 *         PAFEM_CONVECTION the velocity [E][Q^3][3] (required).
 *  coeff_scale: multiplies the coefficient.
 * SYNCHRONOUS: returns EINVAL naming the first element with det J <= 0. */
pafem_status pafem_qdata_assemble(pafem_space space, int32_t kind, int32_t q1d,
                                  const double* coeff, double coeff_scale,
                                  double* qdata, void* stream);

/* ------------------------------------------------------------ operator --- */

/* Operator y = G^t B^t D B G x on the space, reading `qdata` (device, layout
 * of pafem_qdata_size, f64).  flags: PAFEM_OP_* bits.  Host call; the op
 * keeps the qdata pointer. */
pafem_status pafem_op_create(pafem_space space, int32_t kind, int32_t q1d,
                             const void* qdata, int32_t qdata_dtype, int32_t flags,
                             pafem_op* out);
void pafem_op_destroy(pafem_op op);

/* Workspace bytes needed by pafem_op_apply / pafem_op_diagonal (0 if none). */
pafem_status pafem_op_workspace_bytes(pafem_op op, size_t* nbytes);

/* y = A x on device vectors (f64; f32 for an operator on f32 or bf16 qdata).
 * Lengths: ndofs, except 3 * ndofs (component-major) for y of PAFEM_GRADIENT,
 * x of PAFEM_DIVERGENCE, and x and y of PAFEM_ELASTICITY and of operators
 * created with PAFEM_OP_VECTOR3; the library cannot check lengths.  x and y
 * must not alias.  With PAFEM_OP_CONSTRAINED, y_b = x_b on essential dofs and
 * the essential columns are dropped (per component for vector operators).
 * Asynchronous.  Errors: EINVAL (null or aliased pointers), ESHAPE (workspace
 * too small for the deterministic scatter), EUNSUPPORTED (no kernel built for
 * the order, q1d or dtype). */
pafem_status pafem_op_apply(pafem_op op, const double* x, double* y, void* work,
                            size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid hipMalloc): pafem_op_apply without a
 * workspace.  The element vectors of the deterministic scatter
 * (PAFEM_OP_SCATTER_EVEC) go to a library-held device buffer of
 * PAFEM_NOALLOC_SCRATCH_BYTES on each GPU, set up on the first call on that GPU
 * and held until the process ends; operators with the atomic scatter need none.
 * Same vectors, semantics and results as pafem_op_apply (bitwise, for the
 * deterministic scatter).  Calls whose executions overlap on one GPU share that
 * GPU's buffer and race: serialize them (one stream, or events).  Allocates
 * nothing.  Asynchronous.  Errors: as pafem_op_apply, and ESHAPE when the element
 * vectors (8 bytes per element dof: ne * (p+1)^dim * 8) exceed the buffer. */
#define PAFEM_NOALLOC_SCRATCH_BYTES (64u << 20)
pafem_status pafem_op_apply_noalloc(pafem_op op, const double* x, double* y, void* stream);

/* diag[ndofs] = diagonal of the operator (1 on essential dofs if constrained),
 * by sum factorization with products of the 1D tables.  Asynchronous.
 * EUNSUPPORTED for PAFEM_DIFFUSION_GEOM (use the PAFEM_DIFFUSION operator). */
pafem_status pafem_op_diagonal(pafem_op op, double* diag, void* work, size_t work_bytes,
                               void* stream);

/* b[ndofs] = int f phi_i ("Finite Element Abstractions", l(v)), zero on
 * essential dofs.  f per `source` (PAFEM_SOURCE_*), f_qp used only for
 * PAFEM_SOURCE_ARRAY.  work >= E*(p+1)^3*8 bytes.  Asynchronous. */
pafem_status pafem_linear_form(pafem_space space, int32_t q1d, int32_t source,
                               const double* f_qp, double scale, double* b, void* work,
                               size_t work_bytes, void* stream);

/* -------------------------------------------------------------- solver --- */

typedef struct {
  double rel_tol;       /* stop when ||r_k||_2 <= rel_tol * ||b||_2 (recursive residual); for b = 0, relative to ||r_0||_2 */
  int32_t max_iter;     /* iteration cap (the paper's ex1p uses 2000) */
  int32_t precond;      /* PAFEM_PRECOND_* */
  int32_t check_every;  /* host reads the convergence flag every this many iterations */
  int32_t zero_guess;   /* 1: start from x = 0 (x is overwritten); 0: start from x */
  double* res_hist;     /* optional host array of ||r_k||/||b||, k = 0..iters */
  int32_t res_hist_cap; /* its capacity */
} pafem_solve_opts;

typedef struct {
  int32_t iters;        /* CG iterations performed */
  int32_t converged;    /* 1 if the tolerance was met */
  double rel_res;       /* final recursive ||r||/||b|| */
  double true_rel_res;  /* ||b - A x|| / ||b|| recomputed at exit */
  double seconds;       /* wall time of the call */
} pafem_solve_result;

/* Workspace bytes for pafem_pcg_solve on this op with at most max_iter
 * iterations (three dof vectors, reduction partials, the residual history and
 * the operator's own workspace). */
pafem_status pafem_pcg_workspace_bytes(pafem_op op, int32_t max_iter, size_t* nbytes);

/* Preconditioned CG ("Scalable Linear Solvers", CGSolver on the PA operator;
 * Jacobi preconditioner z = r / diag).  Vectors are device f64 [ndofs]; diag
 * may be NULL for PAFEM_PRECOND_NONE.  All vector work and the dot products
 * run on the device; the host reads a convergence flag every check_every
 * iterations.  SYNCHRONOUS.  Returns ENOTCONV at max_iter, EBREAKDOWN on
 * p.Ap <= 0 or a non-finite scalar (result filled in either case). */
pafem_status pafem_pcg_solve(pafem_op op, const double* diag, const double* b, double* x,
                             void* work, size_t work_bytes, const pafem_solve_opts* opts,
                             pafem_solve_result* result, void* stream);


/* ------------------------------------------- mixed precision refinement --- */

/* dst[i] = src[i] rounded to PAFEM_F32 or PAFEM_BF16 (round to nearest even),
 * device arrays of n values.  Makes the reduced-precision copies of quadrature
 * data for an inner operator (pafem_op_create with that qdata_dtype).
 * Asynchronous.  Errors: EINVAL for another dtype. */
pafem_status pafem_convert(int64_t n, const double* src, void* dst, int32_t dtype, void* stream);

typedef struct {
  double rel_tol;       /* outer stop: ||b - A_hi x||_2 <= rel_tol ||b||_2, FP64 residual */
  double inner_rel_tol; /* inner stop: reduction of the reduced-precision PCG residual */
  int32_t max_outer;    /* refinement steps */
  int32_t max_inner;    /* inner PCG iterations per step */
  int32_t check_every;  /* host reads the inner convergence flag every this many iterations */
  int32_t precond;      /* PAFEM_PRECOND_NONE or PAFEM_PRECOND_JACOBI (diag rounded to f32) */
  int32_t keep_direction; /* 1: the inner PCG keeps its search direction across steps
                             (residual replacement); 0: it restarts from d = 0 each step */
  double* res_hist;     /* optional host array: outer ||r_k||/||b||, k = 0..outer */
  int32_t res_hist_cap;
} pafem_ir_opts;

typedef struct {
  int32_t outer;        /* refinement steps taken */
  int32_t inner_total;  /* inner PCG iterations summed over the steps */
  int32_t converged;    /* 1 if rel_tol was met */
  double rel_res;       /* final ||b - A_hi x|| / ||b|| (FP64) */
  double seconds;       /* wall time of the call */
} pafem_ir_result;

/* Workspace bytes of pafem_ir_solve for this pair of operators. */
pafem_status pafem_ir_workspace_bytes(pafem_op a_hi, pafem_op a_lo, size_t* nbytes);

/* Iterative refinement: x = 0; repeat r = b - A_hi x (FP64 apply, FP64 residual
 * and norms), solve A_lo d = r/||r|| approximately with Jacobi-PCG, x += ||r|| d
 * (FP64).  The inner PCG keeps its residual, preconditioned residual and dot
 * products in FP64; only the reduced-precision apply's input (the search
 * direction) and output, and the correction d, are FP32 (the Jacobi scaling is
 * 1/diag rounded to FP32).  With keep_direction the inner PCG is one continuing
 * iteration whose residual is replaced by the FP64 residual at every step (a
 * reliable update: the recurrence and its search direction survive, so the inner
 * iteration count stays close to that of FP64 PCG); a step that ends on max_inner
 * instead of inner_rel_tol restarts the inner PCG.  One step = one FP64 residual =
 * one `outer`.
 * a_hi: an FP64 operator; a_lo: the same operator (same space, kind and flags)
 * built on F32 or BF16 quadrature data.  diag: FP64 diagonal of a_hi (NULL for
 * PAFEM_PRECOND_NONE).  b, x: device f64 [ndofs].  SYNCHRONOUS.  Returns
 * ENOTCONV if max_outer steps do not reach rel_tol (result filled in). */
pafem_status pafem_ir_solve(pafem_op a_hi, pafem_op a_lo, const double* diag, const double* b,
                            double* x, void* work, size_t work_bytes, const pafem_ir_opts* opts,
                            pafem_ir_result* result, void* stream);


/* ------------------------------------------------------------- batched --- */

/* Many right-hand sides over many meshes in one graph launch.  Each operator
 * (one per mesh; same kind; all F64 or all F32 quadrature data; orders 1..6,
 * q1d = p+2) applies to nrhs vectors stored right-hand-side fastest:
 * x_m[dof][rhs], y_m[dof][rhs] (device, f64 for F64 operators, f32 for F32).
 * The batch groups the meshes by order (one grouped launch per order), and
 * captures the whole batch into a HIP graph that replays on the caller's stream.
 * The tile shape of each order (elements x right-hand sides per workgroup) is
 * chosen by pafem_batch_autotune, or set by hand. */
typedef struct pafem_batch_s* pafem_batch;

/* Device workspace for the mesh descriptors of a batch of nops operators. */
pafem_status pafem_batch_workspace_bytes(int32_t nops, size_t* nbytes);

/* nrhs: even and >= 2.  work: device workspace (kept by the batch). */
pafem_status pafem_batch_create(int32_t nops, const pafem_op* ops, int32_t nrhs, void* work,
                                size_t work_bytes, pafem_batch* out);
void pafem_batch_destroy(pafem_batch batch);

/* y_m = A_m x_m for every mesh m (x, y: host arrays of nops device pointers).
 * Constrained operators return y_b = x_b on essential dofs.  Asynchronous; the
 * graph is (re)captured when the pointers or tiles change. */
pafem_status pafem_batch_apply(pafem_batch batch, const void* const* x, void* const* y,
                               void* stream);

/* Time every tile candidate of every order `reps` times on these vectors (their
 * y contents are overwritten) and keep the fastest; results are read from and
 * written to the text cache `cache_path` (NULL: no cache), keyed by GPU
 * architecture, kind, dtype, nrhs and order.  SYNCHRONOUS. */
pafem_status pafem_batch_autotune(pafem_batch batch, const void* const* x, void* const* y,
                                  const char* cache_path, int32_t reps, void* stream);

/* Force the tile candidate (-1 = default) for the meshes of one order.  0..4: vector-unit
 * tiles of 4, 8, 16, 2x8 (two elements) and 2 right-hand sides; 5: FP64 matrix cores
 * (v_mfma_f64_16x16x4f64, the sum-factorization contractions as dense products over 16
 * right-hand sides; one element per workgroup), FP64 batches of orders 1..4 with nrhs a
 * multiple of 16 ("High-Order Partial Assembly").  EINVAL for a candidate the order,
 * dtype or nrhs does not allow. */
pafem_status pafem_batch_set_tile(pafem_batch batch, int32_t order, int32_t candidate);

/* JSON description of the groups, chosen tiles and tuning timings into buf. */
pafem_status pafem_batch_describe(pafem_batch batch, char* buf, size_t len);


/* ------------------------------------------- learned element preconditioner --- */

/* A small network N on element patches (BF16 weights and activations, FP32
 * accumulation on matrix cores, FP32 master weights and Adam) defines the
 * preconditioner
 *     z = r / diag + G^t( w * (s_E / kbar_E) * N([r_E / s_E, f_E]) ),
 * s_E = ||r_E||, kbar_E the element mean of the coefficient, f_E the 8 octant
 * log-ratios of the coefficient, w = 1 / (element nodes sharing the dof), z = 0
 * on essential dofs.  N: in -> hidden (relu) -> hidden (relu) -> out with
 * in = roundup16((p+1)^3 + 8), out = roundup16((p+1)^3).  Parameters (FP32):
 * W1 [hidden][in], b1, W2 [hidden][hidden], b2, W3 [out][hidden], b3.
 * Not in the paper: an addition to CG on partially assembled operators.  Built
 * for orders 1..4. */
typedef struct pafem_net_s* pafem_net;

/* Device storage of a network that runs on up to max_rows element patches and
 * trains on up to max_train_rows. */
pafem_status pafem_net_storage_bytes(int32_t order, int32_t hidden, int64_t max_rows,
                                     int64_t max_train_rows, size_t* nbytes);
pafem_status pafem_net_create(int32_t order, int32_t hidden, int64_t max_rows,
                              int64_t max_train_rows, void* storage, size_t nbytes,
                              pafem_net* out);
void pafem_net_destroy(pafem_net net);
pafem_status pafem_net_dims(pafem_net net, int32_t* in_dim, int32_t* hidden, int32_t* out_dim,
                            int64_t* nparams);
/* Host FP32 parameters in, or out; set also clears the Adam state.  SYNCHRONOUS. */
pafem_status pafem_net_set_params(pafem_net net, const float* host_params, void* stream);
pafem_status pafem_net_get_params(pafem_net net, float* host_params, void* stream);
/* Gradients of the last backward pass (host FP32).  SYNCHRONOUS. */
pafem_status pafem_net_get_grads(pafem_net net, float* host_grads, void* stream);
/* Training state for checkpoint and resume.  host_state [3][nparams] f32: the
 * parameters (same order as pafem_net_set_params), then Adam's first and second
 * moment estimates; *step / step: the number of Adam steps taken, which sets the
 * bias correction of the next one.  set_state clears the kept gradients; the
 * next pafem_net_adam_step then continues as if training had not stopped.
 * Host memory is the caller's.  EINVAL on a null pointer or a negative step.
 * SYNCHRONOUS.  (Checkpoints of the state are an addition to the paper's
 * data-collection output.) */
pafem_status pafem_net_get_state(pafem_net net, float* host_state, int32_t* step, void* stream);
pafem_status pafem_net_set_state(pafem_net net, const float* host_state, int32_t step,
                                 void* stream);
/* out [rows][out] f32 = N(x), x device bf16 [rows][in]. */
pafem_status pafem_net_forward(pafem_net net, const uint16_t* x, float* out, int64_t rows,
                               void* stream);
/* Gradients of sum(dout * N(x)) w.r.t. the parameters, kept in the network;
 * dout device bf16 [rows][out]. */
pafem_status pafem_net_backward(pafem_net net, const uint16_t* x, const uint16_t* dout,
                                int64_t rows, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the kept gradients. */
pafem_status pafem_net_adam_step(pafem_net net, float lr, void* stream);

/* feats [E][9] f32 per element (kbar, 8 octant log-ratios) from the coefficient
 * kappa [E][q1d^3] f64 (device; NULL: constant 1). */
pafem_status pafem_learned_features(pafem_space space, const double* kappa, int32_t q1d,
                                    float* feats, void* stream);
/* Workspace of pafem_learned_precond / pafem_learned_loss_grad on this op. */
pafem_status pafem_learned_workspace_bytes(pafem_op op, size_t* nbytes);
/* z = M(r) as above (device f64 vectors). */
pafem_status pafem_learned_precond(pafem_net net, pafem_op op, const float* feats,
                                   const double* diag, const double* r, double* z, void* work,
                                   size_t work_bytes, void* stream);
/* Training loss on a pair (r, e) with A e = r:
 *     L = ||A (e - M(r))||^2_{D^-1} / ||r||^2_{D^-1},
 * written to the device scalar *loss (may be NULL); its parameter gradients are
 * kept in the network for pafem_net_adam_step. */
pafem_status pafem_learned_loss_grad(pafem_net net, pafem_op op, const float* feats,
                                     const double* diag, const double* r, const double* e,
                                     double* loss, void* work, size_t work_bytes, void* stream);

typedef struct {
  int32_t iters;          /* iterations (across a fallback restart) */
  int32_t converged;
  int32_t fell_back;      /* 1 if the learned preconditioner was abandoned for Jacobi */
  int32_t fallback_iter;  /* iteration at which it was abandoned (-1: never) */
  double rel_res;
  double true_rel_res;
  double seconds;
} pafem_fcg_result;

pafem_status pafem_fcg_workspace_bytes(pafem_op op, int32_t max_iter, size_t* nbytes);
/* Flexible CG (Polak-Ribiere beta) with the learned preconditioner (net != NULL)
 * or Jacobi (net == NULL).  If r.z <= 0, a non-finite scalar or a residual
 * growth by 1e6 appears with the network, it restarts from the current iterate
 * with Jacobi (result->fell_back).  opts->precond is ignored.  On the essential
 * dofs the preconditioner returns r when the operator is constrained (its rows
 * there are the identity, so b and x may hold any values on them) and r / diag
 * otherwise; the learned correction acts on the other dofs only.  SYNCHRONOUS. */
pafem_status pafem_fcg_solve(pafem_op op, pafem_net net, const float* feats, const double* diag,
                             const double* b, double* x, void* work, size_t work_bytes,
                             const pafem_solve_opts* opts, pafem_fcg_result* result,
                             void* stream);

/* Solver iterations (pafem_pcg_solve batches, pafem_pmg_fcg_solve pairs of
 * iterations) are captured once per solve into a HIP graph (kernels only) and
 * replayed on the caller's stream.  mode 0 launches every kernel directly
 * instead; process-wide, returns the previous mode.  Results are the same up to
 * the order of atomic sums. */
int32_t pafem_set_graph_mode(int32_t mode);

/* ---------------------------------------------------- order multigrid --- */
/* Matrix-free preconditioning of PA operators by multigrid in the polynomial
 * order ("Scalable Linear Solvers" names it without fixing an algorithm; the
 * definitions below are this library's).  Levels are H1 spaces of orders
 * p_0 >= p_1 >= ... on ONE mesh object (the spaces share the device element
 * order), each with its constrained diffusion operator and diagonal. */

#define PAFEM_MEAN_ARITHMETIC 0
#define PAFEM_MEAN_GEOMETRIC 1
#define PAFEM_MEAN_HARMONIC 2

/* out[e][q'] = mean over q of coeff[e][q], for every q' < q1d_out^3: the
 * per-element mean (PAFEM_MEAN_*) of a coefficient given per quadrature point
 * (q1d_in^3 values per element, caller element order) spread over the points
 * of another rule; the coarse-level coefficient of the multigrid.  Device f64
 * arrays.  Asynchronous.  Errors: EINVAL (kind, sizes). */
pafem_status pafem_coeff_element_mean(pafem_space space, int32_t kind, const double* coeff,
                                      int32_t q1d_in, int32_t q1d_out, double* out,
                                      void* stream);

/* Prolongation from the order-pc space `coarse` to the order-pf space `fine`
 * (pc <= pf; both on one mesh, or `fine` on pafem_mesh_refine of `coarse`'s mesh):
 * yf[i] = sum_j phi^c_j(x_i) xc[j] over free coarse dofs j, for free fine dofs i
 * (the coarse function evaluated at the fine node; across a refinement, the parent's
 * basis at the child's nodes mapped into the parent's octant); essential fine
 * entries are set to 0, or left unchanged when add != 0, in which case the result
 * is added to yf.  Device f64 vectors.  Asynchronous.  Deterministic (each fine dof
 * is written by one element).
 * Errors: EINVAL (unrelated meshes, pc > pf, order above 8). */
pafem_status pafem_prolongate(pafem_space coarse, pafem_space fine, const double* xc, double* yf,
                              int32_t add, void* stream);

/* coeff_parent_mean: out [Ec][q1d_out^3] f64 = the mean (kind as above) of the
 * coefficient coeff [Ef][q1d_in^3] given on `fine` (a space on pafem_mesh_refine
 * of `coarse`'s mesh) over the points of each coarse element's 8 children, at every
 * point of the coarse element; caller element order (children 8 e .. 8 e + 7).  The
 * coefficient of a multigrid level one refinement coarser.  Device arrays.
 * Asynchronous.  Errors: EINVAL (kind, sizes, unrelated meshes). */
pafem_status pafem_coeff_parent_mean(pafem_space fine, pafem_space coarse, int32_t kind,
                                     const double* coeff, int32_t q1d_in, int32_t q1d_out,
                                     double* out, void* stream);

/* Restriction, the transpose of the prolongation on free dofs:
 * rc = P^T (bf - yf) (yf may be NULL), 0 on essential coarse dofs.  Sums with
 * device atomics (order not fixed).  Asynchronous. */
pafem_status pafem_restrict(pafem_space fine, pafem_space coarse, const double* bf,
                            const double* yf, double* rc, void* stream);

/* Workspace of pafem_op_lambda_max and pafem_chebyshev_smooth on op. */
pafem_status pafem_smoother_workspace_bytes(pafem_op op, size_t* nbytes);

/* Power iteration for the largest eigenvalue of D^-1 A (D = diag(diag)):
 * v (device f64 [ndofs], the start vector, overwritten) is zeroed on essential
 * dofs and normalised in the D-norm; then `iters` times w = A v,
 * lambda = v . w, v = D^-1 w / ||D^-1 w||_D.  *lambda (host) is the last
 * estimate, a lower bound of the largest eigenvalue.  SYNCHRONOUS. */
pafem_status pafem_op_lambda_max(pafem_op op, const double* diag, double* v, int32_t iters,
                                 void* work, size_t work_bytes, double* lambda, void* stream);

/* `degree` steps of Chebyshev iteration with the Jacobi preconditioner on
 * A x = b (Saad, Iterative Methods for Sparse Linear Systems, Chebyshev
 * acceleration): eigenvalue interval [lo*lmax, hi*lmax] of D^-1 A, centre
 * theta, half width delta, sigma = theta/delta; r = b - A x, rho = 1/sigma,
 * d = D^-1 r / theta; repeat: x += d, and before each further step
 * r -= A d, rho' = 1/(2 sigma - rho), d = rho' rho d + (2 rho'/delta) D^-1 r.
 * zero_guess: x_0 = 0 (saves one apply).  Asynchronous. */
pafem_status pafem_chebyshev_smooth(pafem_op op, const double* diag, double lmax, double lo,
                                    double hi, int32_t degree, const double* b, double* x,
                                    int32_t zero_guess, void* work, size_t work_bytes,
                                    void* stream);

typedef struct pafem_pmg_s* pafem_pmg;

typedef struct {
  int32_t degree;        /* Chebyshev steps before and after the coarse correction */
  double lo, hi;         /* Chebyshev interval [lo*lmax, hi*lmax] */
  int32_t coarse_iters;  /* Jacobi-PCG iterations on the coarsest level (from zero) */
} pafem_pmg_opts;

/* A V-cycle hierarchy over nlevels >= 1 levels, finest first: ops[l] an f64
 * constrained diffusion operator (PAFEM_DIFFUSION or PAFEM_DIFFUSION_GEOM) of
 * order p_l (non-increasing); each level's space is on the previous level's mesh
 * (a step in the order) or on the mesh that one was refined from
 * (pafem_mesh_refine: a step in the mesh size, h-multigrid); diags[l] its diagonal
 * (device f64, caller-owned, kept by pointer); lmax[l] the largest-eigenvalue
 * estimate of diags[l]^-1 ops[l] (pafem_op_lambda_max).  The operators and
 * diagonals must outlive the hierarchy.  Orders up to 8. */
pafem_status pafem_pmg_create(int32_t nlevels, const pafem_op* ops, const double* const* diags,
                              const double* lmax, const pafem_pmg_opts* opts, pafem_pmg* out);
void pafem_pmg_destroy(pafem_pmg pmg);
/* Workspace bytes of pafem_pmg_vcycle (max_iter < 0) or of pafem_pmg_fcg_solve
 * with at most max_iter iterations. */
pafem_status pafem_pmg_workspace_bytes(pafem_pmg pmg, int32_t max_iter, size_t* nbytes);
/* z = V(r), one V-cycle from a zero guess: pre-smoothing, residual,
 * restriction, recursion (coarsest: opts.coarse_iters Jacobi-PCG iterations),
 * prolongation added, post-smoothing.  Device f64 [ndofs of level 0].
 * Asynchronous. */
pafem_status pafem_pmg_vcycle(pafem_pmg pmg, const double* r, double* z, void* work,
                              size_t work_bytes, void* stream);
/* Flexible CG on ops[0] preconditioned by one V-cycle per iteration (the
 * coarse PCG makes the cycle a nonlinear map).  opts->precond is ignored.
 * SYNCHRONOUS.  Returns ENOTCONV / EBREAKDOWN with the result filled in. */
pafem_status pafem_pmg_fcg_solve(pafem_pmg pmg, const double* b, double* x, void* work,
                                 size_t work_bytes, const pafem_solve_opts* opts,
                                 pafem_solve_result* result, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PAFEM_H */
