// C ABI of the library: argument checking, host orchestration, launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "internal.hpp"
#include "batch_host.hpp"
#include "capi.hpp"
#include "graph.hpp"
#include "launch.hpp"
#include "mg.hpp"
#include "solver.hpp"

using namespace pafem;

struct pafem_batch_s {
  Batch* b;
};


namespace {
const Space& uploaded_space(pafem_space sp) {
  require(sp != nullptr && sp->s != nullptr, PAFEM_EINVAL, "null space");
  require(sp->s->uploaded, PAFEM_EINVAL, "space has no device image: call pafem_space_upload");
  return *sp->s;
}

size_t dtype_size(int dt) {
  switch (dt) {
    case PAFEM_F64: return 8;
    case PAFEM_F32: return 4;
    case PAFEM_BF16: return 2;
    default: return 0;
  }
}

// vector type used by an operator with the given qdata type
int vector_dtype(int qdtype) { return qdtype == PAFEM_F64 ? PAFEM_F64 : PAFEM_F32; }

}  // namespace

size_t pafem::op_work_bytes(const Op& op) {
  const Space& s = *op.space;
  const size_t evec = size_t(s.ne) * s.dpe;
  // diagonal needs an f64 element vector; the deterministic scatter an element
  // vector of the operator's vector type
  size_t need = evec * sizeof(double);
  return align256(need);
}

namespace {

}  // namespace

namespace pafem {
// One application of the operator; `work` must hold op_work_bytes(op).  dotp (may be
// null): pa_apply_blocks partial element energies for launch_cg_alpha.
void apply_op(const Op& op, const void* x, void* y, void* work, hipStream_t st, double* dotp,
              bool y_ready) {
  const Space& s = *op.space;
  const bool constrained = op.flags & PAFEM_OP_CONSTRAINED;
  const bool evec = op.flags & PAFEM_OP_SCATTER_EVEC;
  const int vdt = vector_dtype(op.qdtype);
  if (op.kind == PAFEM_DG_CONVECTION) {
    const double* qd = static_cast<const double*>(op.qdata);
    // the volume kernel stores every dof (each belongs to one element); the faces add
    require(launch_pa_apply(s.dev, op.kind, op.q1d, PAFEM_F64, false, false, qd, x, y,
                            PAFEM_F64, st, nullptr),
            PAFEM_EUNSUPPORTED, "DG volume kernel not built for this order/q1d");
    launch_dg_faces(s.dev, op.q1d, qd + qdata_values(s.ne, op.q1d, 3),
                    static_cast<const double*>(x), static_cast<double*>(y), st);
    return;
  }
  if (nd_kind(op.kind)) {
    if (!y_ready)
      launch_scatter_init(s.dev, static_cast<const double*>(x), constrained,
                          static_cast<double*>(y), st);
    require(launch_nd_apply(s.dev, op.kind, op.q1d, constrained,
                            static_cast<const double*>(op.qdata), static_cast<const double*>(x),
                            static_cast<double*>(y), st, dotp),
            PAFEM_EUNSUPPORTED, "H(curl) apply not built for this order/q1d");
    return;
  }
  if (evec) {
    require(launch_pa_apply(s.dev, op.kind, op.q1d, op.qdtype, constrained, true, op.qdata, x,
                            work, vdt, st, dotp),
            PAFEM_EUNSUPPORTED, "apply kernel not built for this order/q1d/dtype");
    if (vdt == PAFEM_F64)
      launch_evec_gather(s.dev, static_cast<const double*>(work), static_cast<const double*>(x),
                         constrained ? 1 : 0, 0.0, static_cast<double*>(y), st);
    else
      launch_evec_gather_f32(s.dev, static_cast<const float*>(work), static_cast<const float*>(x),
                             constrained ? 1 : 0, static_cast<float*>(y), st);
  } else {
    if (y_ready) {
      // the caller already set y = x on essential dofs (constrained) and 0 elsewhere
    } else if (op.kind == PAFEM_GRADIENT) {
      launch_fill(static_cast<double*>(y), 0.0, 3 * s.ndofs, st);  // three output components
    } else if (op.kind == PAFEM_DIVERGENCE) {
      launch_fill(static_cast<double*>(y), 0.0, s.ndofs, st);
    } else if ((op.flags & PAFEM_OP_VECTOR3) || op.kind == PAFEM_ELASTICITY) {
      for (int c = 0; c < 3; ++c)
        launch_scatter_init(s.dev, static_cast<const double*>(x) + c * s.ndofs, constrained,
                            static_cast<double*>(y) + c * s.ndofs, st);
    } else if (vdt == PAFEM_F64) {
      launch_scatter_init(s.dev, static_cast<const double*>(x), constrained,
                          static_cast<double*>(y), st);
    } else {
      launch_scatter_init_f32(s.dev, static_cast<const float*>(x), constrained,
                              static_cast<float*>(y), st);
    }
    const int kkind = (op.flags & PAFEM_OP_VECTOR3) ? kVectorKind + op.kind : op.kind;
    require(launch_pa_apply(s.dev, kkind, op.q1d, op.qdtype, constrained, false, op.qdata, x,
                            y, vdt, st, dotp),
            PAFEM_EUNSUPPORTED, "apply kernel not built for this order/q1d/dtype");
  }
}
}  // namespace pafem

namespace pafem {
thread_local std::string g_last_error;
std::atomic<int>& graph_mode_flag() {
  static std::atomic<int> flag{1};
  return flag;
}
}

extern "C" {

const char* pafem_last_error(void) { return g_last_error.c_str(); }

int32_t pafem_version(void) { return 274; }

int32_t pafem_set_graph_mode(int32_t mode) {
  return graph_mode_flag().exchange(mode != 0 ? 1 : 0);
}

pafem_status pafem_mesh_create_hex(int64_t nv, const double* xyz, int64_t ne, const int64_t* hex8,
                                   int32_t geom_order, const double* geom_nodes,
                                   pafem_mesh* out) {
  return guarded([&] {
    require(out && xyz && hex8, PAFEM_EINVAL, "null pointer argument");
    require(nv > 0 && ne > 0, PAFEM_EINVAL, "mesh needs vertices and elements");
    require(geom_order == 1 || geom_order == 2, PAFEM_EINVAL, "geom_order must be 1 or 2");
    require(geom_order == 1 || geom_nodes, PAFEM_EINVAL, "geom_order 2 needs geom_nodes");
    for (int64_t e = 0; e < ne; ++e) {
      const int64_t* h = hex8 + e * 8;
      for (int k = 0; k < 8; ++k) {
        if (h[k] < 0 || h[k] >= nv)
          throw Error(PAFEM_EINVAL,
                      "element " + std::to_string(e) + " has a vertex index out of range");
        for (int j = 0; j < k; ++j)
          if (h[j] == h[k])
            throw Error(PAFEM_EINVAL, "element " + std::to_string(e) + " repeats a vertex");
      }
    }
    auto* m = new pafem_mesh_s();
    m->m.nv = nv;
    m->m.ne = ne;
    m->m.xyz.assign(xyz, xyz + nv * 3);
    m->m.hex.assign(hex8, hex8 + ne * 8);
    m->m.geom_order = geom_order;
    if (geom_order == 2) m->m.gnodes.assign(geom_nodes, geom_nodes + ne * 27 * 3);
    m->m.id = next_mesh_id();
    *out = m;
  });
}

pafem_status pafem_mesh_create_quad(int64_t nv, const double* xy, int64_t ne, const int64_t* quad4,
                                    pafem_mesh* out) {
  return guarded([&] {
    require(out && xy && quad4, PAFEM_EINVAL, "null pointer argument");
    require(nv > 0 && ne > 0, PAFEM_EINVAL, "mesh needs vertices and elements");
    for (int64_t e = 0; e < ne; ++e) {
      const int64_t* q = quad4 + e * 4;
      for (int k = 0; k < 4; ++k) {
        if (q[k] < 0 || q[k] >= nv)
          throw Error(PAFEM_EINVAL,
                      "element " + std::to_string(e) + " has a vertex index out of range");
        for (int j = 0; j < k; ++j)
          if (q[j] == q[k])
            throw Error(PAFEM_EINVAL, "element " + std::to_string(e) + " repeats a vertex");
      }
    }
    auto* m = new pafem_mesh_s();
    m->m.dim = 2;
    m->m.nv = nv;
    m->m.ne = ne;
    m->m.xyz.assign(xy, xy + nv * 2);
    m->m.quad.assign(quad4, quad4 + ne * 4);
    m->m.geom_order = 1;
    m->m.id = next_mesh_id();
    *out = m;
  });
}

pafem_status pafem_mesh_refine(pafem_mesh coarse, pafem_mesh* fine) {
  return guarded([&] {
    require(coarse && fine, PAFEM_EINVAL, "null pointer argument");
    auto m = std::make_unique<pafem_mesh_s>();
    refine_mesh(coarse->m, m->m);
    *fine = m.release();
  });
}

pafem_status pafem_mesh_info(pafem_mesh mesh, int64_t* nv, int64_t* ne) {
  return guarded([&] {
    require(mesh, PAFEM_EINVAL, "null mesh");
    if (nv) *nv = mesh->m.nv;
    if (ne) *ne = mesh->m.ne;
  });
}

pafem_status pafem_mesh_vertices(pafem_mesh mesh, double* xyz, int64_t* elems) {
  return guarded([&] {
    require(mesh, PAFEM_EINVAL, "null mesh");
    const Mesh& m = mesh->m;
    if (xyz) std::copy(m.xyz.begin(), m.xyz.end(), xyz);
    if (elems) {
      const std::vector<int64_t>& conn = m.dim == 2 ? m.quad : m.hex;
      std::copy(conn.begin(), conn.end(), elems);
    }
  });
}

void pafem_mesh_destroy(pafem_mesh mesh) { delete mesh; }

pafem_status pafem_space_create_h1(pafem_mesh mesh, int32_t order, int32_t flags,
                                   pafem_space* out) {
  return guarded([&] {
    require(mesh && out, PAFEM_EINVAL, "null pointer argument");
    auto* s = new pafem_space_s();
    try {
      s->s = build_space(&mesh->m, order, flags);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

pafem_status pafem_space_create_nd(pafem_mesh mesh, int32_t order, int32_t flags,
                                   pafem_space* out) {
  return guarded([&] {
    require(mesh && out, PAFEM_EINVAL, "null pointer argument");
    auto* s = new pafem_space_s();
    try {
      s->s = build_nd_space(&mesh->m, order, flags);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

pafem_status pafem_space_create_l2(pafem_mesh mesh, int32_t order, int32_t flags,
                                   pafem_space* out) {
  return guarded([&] {
    require(mesh && out, PAFEM_EINVAL, "null pointer argument");
    auto* s = new pafem_space_s();
    try {
      s->s = build_l2_space(&mesh->m, order, flags);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

pafem_status pafem_space_family(pafem_space space, int32_t* family) {
  return guarded([&] {
    require(space && space->s && family, PAFEM_EINVAL, "null pointer argument");
    const int f = space->s->family;
    *family = f == kFamilyND ? PAFEM_SPACE_ND : f == kFamilyL2 ? PAFEM_SPACE_L2 : PAFEM_SPACE_H1;
  });
}

pafem_status pafem_space_elem_signs(pafem_space space, int8_t* signs) {
  return guarded([&] {
    require(space && space->s && signs, PAFEM_EINVAL, "null pointer argument");
    const Space& s = *space->s;
    if (s.family == kFamilyND)
      std::copy(s.gsign.begin(), s.gsign.end(), signs);
    else
      std::fill(signs, signs + size_t(s.ne) * s.dpe, int8_t(1));
  });
}

void pafem_space_destroy(pafem_space space) {
  if (!space) return;
  delete space->s;
  delete space;
}

pafem_status pafem_space_info(pafem_space space, int64_t* ndofs, int64_t* nelem,
                              int32_t* dofs_per_elem, int64_t* nbdr) {
  return guarded([&] {
    require(space && space->s, PAFEM_EINVAL, "null space");
    const Space& s = *space->s;
    if (ndofs) *ndofs = s.ndofs;
    if (nelem) *nelem = s.ne;
    if (dofs_per_elem) *dofs_per_elem = s.dpe;
    if (nbdr) *nbdr = int64_t(s.bdr.size());
  });
}

pafem_status pafem_space_dim(pafem_space space, int32_t* dim) {
  return guarded([&] {
    require(space && space->s && dim, PAFEM_EINVAL, "null pointer argument");
    *dim = space->s->dim;
  });
}

pafem_status pafem_space_dof_coords(pafem_space space, double* xyz) {
  return guarded([&] {
    require(space && space->s && xyz, PAFEM_EINVAL, "null pointer argument");
    space_dof_coords(*space->s, xyz);
  });
}

pafem_status pafem_space_boundary_dofs(pafem_space space, int32_t* idx) {
  return guarded([&] {
    require(space && space->s, PAFEM_EINVAL, "null pointer argument");
    require(idx || space->s->bdr.empty(), PAFEM_EINVAL, "null pointer argument");
    std::copy(space->s->bdr.begin(), space->s->bdr.end(), idx);
  });
}

pafem_status pafem_space_elem_dofs(pafem_space space, int32_t* gmap) {
  return guarded([&] {
    require(space && space->s && gmap, PAFEM_EINVAL, "null pointer argument");
    std::copy(space->s->gmap.begin(), space->s->gmap.end(), gmap);
  });
}

pafem_status pafem_space_device_bytes(pafem_space space, size_t* nbytes) {
  return guarded([&] {
    require(space && space->s && nbytes, PAFEM_EINVAL, "null pointer argument");
    size_t off[kSpaceSegments + 1];
    space_device_layout(*space->s, off, nbytes);
  });
}

pafem_status pafem_space_upload(pafem_space space, void* device_buf, size_t nbytes,
                                void* stream) {
  return guarded([&] {
    require(space && space->s && device_buf, PAFEM_EINVAL, "null pointer argument");
    require((reinterpret_cast<uintptr_t>(device_buf) & 255) == 0, PAFEM_EINVAL,
            "device buffer must be 256-byte aligned");
    Space& s = *space->s;
    size_t off[kSpaceSegments + 1], total = 0;
    space_device_layout(s, off, &total);
    require(nbytes >= total, PAFEM_ESHAPE,
            "device buffer too small: need " + std::to_string(total) + " bytes");
    std::vector<int32_t> gmap_enc, toff, tidx;
    std::vector<double> gnodes;
    std::vector<uint32_t> owner;
    space_pack(s, gmap_enc, gnodes, toff, tidx, owner);
    auto st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(device_buf);
    auto up = [&](int seg, const void* src, size_t bytes, const char* what) {
      if (bytes) hip_check(hipMemcpyAsync(base + off[seg], src, bytes, hipMemcpyHostToDevice, st), what);
    };
    up(0, gmap_enc.data(), gmap_enc.size() * 4, "upload gmap");
    up(1, gnodes.data(), gnodes.size() * 8, "upload geometry");
    up(2, s.bmask.data(), s.bmask.size(), "upload boundary mask");
    up(3, toff.data(), toff.size() * 4, "upload transposed offsets");
    up(4, tidx.data(), tidx.size() * 4, "upload transposed map");
    up(5, s.tables.data(), s.tables.size() * 8, "upload tables");
    hip_check(hipMemsetAsync(base + off[6], 0, 64 * 4, st), "clear status");
    up(7, s.dev_order.data(), s.dev_order.size() * 4, "upload element order");
    up(8, s.tile_off.data(), s.tile_off.size() * 4, "upload tile offsets");
    up(9, s.tile_dofs.data(), s.tile_dofs.size() * 4, "upload tile dofs");
    up(10, s.tile_slot.data(), s.tile_slot.size() * 2, "upload tile slots");
    const std::vector<float> tables32(s.tables.begin(), s.tables.end());
    up(11, tables32.data(), tables32.size() * 4, "upload FP32 tables");
    up(12, owner.data(), owner.size() * 4, "upload owner bits");
    std::vector<int8_t> sign_dev(s.gsign.size());
    for (int64_t k = 0; k < s.ne && !s.gsign.empty(); ++k)
      std::copy_n(s.gsign.data() + size_t(s.dev_order[size_t(k)]) * s.dpe, s.dpe,
                  sign_dev.data() + size_t(k) * s.dpe);
    up(13, sign_dev.data(), sign_dev.size(), "upload dof signs");
    up(14, s.tables_open.data(), s.tables_open.size() * 8, "upload open-basis tables");
    up(15, s.faces.data(), s.faces.size() * 4, "upload faces");
    up(16, s.bfaces.data(), s.bfaces.size() * 4, "upload boundary faces");
    hip_check(hipStreamSynchronize(st), "upload sync");
    s.dev_buf = device_buf;
    s.dev_bytes = nbytes;
    s.dev.gmap = reinterpret_cast<const int32_t*>(base + off[0]);
    s.dev.gnodes = reinterpret_cast<const double*>(base + off[1]);
    s.dev.bmask = reinterpret_cast<const uint8_t*>(base + off[2]);
    s.dev.toff = reinterpret_cast<const int32_t*>(base + off[3]);
    s.dev.tidx = reinterpret_cast<const int32_t*>(base + off[4]);
    s.dev.tables = reinterpret_cast<const double*>(base + off[5]);
    s.dev.status = reinterpret_cast<int32_t*>(base + off[6]);
    s.dev.elem_orig = reinterpret_cast<const int32_t*>(base + off[7]);
    s.dev.tile_off = reinterpret_cast<const int32_t*>(base + off[8]);
    s.dev.tile_dofs = reinterpret_cast<const int32_t*>(base + off[9]);
    s.dev.tile_slot = reinterpret_cast<const uint16_t*>(base + off[10]);
    s.dev.tables32 = reinterpret_cast<const float*>(base + off[11]);
    s.dev.owner = reinterpret_cast<const uint32_t*>(base + off[12]);
    s.dev.sign = s.gsign.empty() ? nullptr : reinterpret_cast<const int8_t*>(base + off[13]);
    s.dev.tables_open =
        s.tables_open.empty() ? nullptr : reinterpret_cast<const double*>(base + off[14]);
    s.dev.family = s.family;
    s.dev.faces = s.faces.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + off[15]);
    s.dev.bfaces = s.bfaces.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + off[16]);
    s.dev.nfaces = int64_t(s.faces.size() / kFaceInts);
    s.dev.nbfaces = int64_t(s.bfaces.size() / 2);
    s.dev.ne = s.ne;
    s.dev.ndofs = s.ndofs;
    s.dev.p = s.p;
    s.dev.ng = s.ng;
    s.dev.tile_ne = s.tile_ne;
    s.dev.dim = s.dim;
    s.uploaded = true;
  });
}

pafem_status pafem_qdata_size(pafem_space space, int32_t kind, int32_t q1d, int64_t* nvalues) {
  return guarded([&] {
    require(space && space->s && nvalues, PAFEM_EINVAL, "null pointer argument");
    require(known_kind(kind), PAFEM_EINVAL, "unknown operator kind");
    require(q1d >= 1 && q1d <= kMaxQ1d, PAFEM_EUNSUPPORTED, "q1d out of range");
    if (space->s->dim == 2) {
      require(kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, PAFEM_EUNSUPPORTED,
              "quadrilaterals support the mass and diffusion operators");
      *nvalues = qdata_values_2d(space->s->ne, q1d, kind == PAFEM_DIFFUSION ? 3 : 1);
    } else {
      require(kind_family(kind) == space->s->family, PAFEM_EUNSUPPORTED,
              "operator kind and space family do not match (H1, Nedelec or L2)");
      *nvalues = qdata_values(space->s->ne, q1d, qdata_components(kind));
      if (kind == PAFEM_DG_CONVECTION)
        // per face the Q^2 weights and one slot with its two elements' caller indices
        *nvalues += int64_t(space->s->faces.size() / kFaceInts + space->s->bfaces.size() / 2) *
                    (q1d * q1d + 1);
    }
  });
}

pafem_status pafem_qdata_assemble(pafem_space space, int32_t kind, int32_t q1d,
                                  const double* coeff, double coeff_scale, double* qdata,
                                  void* stream) {
  return guarded([&] {
    const Space& s = uploaded_space(space);
    require(qdata != nullptr, PAFEM_EINVAL, "null qdata");
    require(known_kind(kind), PAFEM_EINVAL, "unknown operator kind");
    require(q1d >= 1 && q1d <= kMaxQ1d, PAFEM_EUNSUPPORTED, "q1d out of range");
    require(s.dim == 3 || kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, PAFEM_EUNSUPPORTED,
            "quadrilaterals support the mass and diffusion operators");
    require(kind != PAFEM_CONVECTION || coeff, PAFEM_EINVAL,
            "the convection operator needs the velocity field");
    require(kind != PAFEM_ELASTICITY || coeff, PAFEM_EINVAL,
            "the elasticity operator needs the (lambda, mu) pairs");
    require(kind != PAFEM_HCURL_MAXWELL || coeff, PAFEM_EINVAL,
            "the definite Maxwell operator needs the (alpha, beta) pairs");
    require(kind_family(kind) == s.family, PAFEM_EUNSUPPORTED,
            "operator kind and space family do not match (H1, Nedelec or L2)");
    require(kind != PAFEM_DG_CONVECTION || coeff, PAFEM_EINVAL,
            "the DG convection operator needs the velocity (3 values)");
    auto st = static_cast<hipStream_t>(stream);
    hip_check(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(s.dev.status), INT_MAX, 1, st),
              "status init");
    launch_qdata(s.dev, kind, q1d, coeff, coeff_scale, qdata, st);
    if (kind == PAFEM_DG_CONVECTION)
      launch_dg_face_qdata(s.dev, q1d, coeff, coeff_scale,
                           qdata + qdata_values(s.ne, q1d, qdata_components(kind)), st);
    int32_t bad = INT_MAX;
    hip_check(hipMemcpyAsync(&bad, s.dev.status, 4, hipMemcpyDeviceToHost, st), "status read");
    hip_check(hipStreamSynchronize(st), "qdata sync");
    require(bad == INT_MAX, PAFEM_EINVAL,
            "non-positive Jacobian determinant in element " + std::to_string(bad));
  });
}

pafem_status pafem_op_create(pafem_space space, int32_t kind, int32_t q1d, const void* qdata,
                             int32_t qdata_dtype, int32_t flags, pafem_op* out) {
  return guarded([&] {
    const Space& s = uploaded_space(space);
    require(out && qdata, PAFEM_EINVAL, "null pointer argument");
    require(known_kind(kind), PAFEM_EINVAL, "unknown operator kind");
    require(kind_family(kind) == s.family, PAFEM_EUNSUPPORTED,
            "operator kind and space family do not match (H1, Nedelec or L2)");
    if (kind == PAFEM_DG_CONVECTION) {
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "the DG convection operator is FP64");
      require(flags == 0, PAFEM_EUNSUPPORTED,
              "the DG convection operator is unconstrained with the atomic scatter");
    }
    if (nd_kind(kind)) {
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "the H(curl) operators are FP64");
      require((flags & ~PAFEM_OP_CONSTRAINED) == 0, PAFEM_EUNSUPPORTED,
              "the H(curl) operators use the atomic scatter");
    }
    if (kind == PAFEM_GRADIENT) {
      require(s.dim == 3, PAFEM_EUNSUPPORTED, "the gradient operator is built for hexahedra");
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "the gradient operator is FP64");
      require(flags == 0, PAFEM_EUNSUPPORTED,
              "the gradient operator is unconstrained with the atomic scatter");
    }
    if (kind == PAFEM_ELASTICITY) {
      require(s.dim == 3, PAFEM_EUNSUPPORTED, "the elasticity operator is built for hexahedra");
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "the elasticity operator is FP64");
      require((flags & ~PAFEM_OP_CONSTRAINED) == 0, PAFEM_EUNSUPPORTED,
              "the elasticity operator is vector-valued by itself, with the atomic scatter");
    }
    if (kind == PAFEM_DIVERGENCE) {
      require(s.dim == 3, PAFEM_EUNSUPPORTED, "the divergence operator is built for hexahedra");
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "the divergence operator is FP64");
      require(flags == 0, PAFEM_EUNSUPPORTED,
              "the divergence operator is unconstrained with the atomic scatter");
    }
    if (kind == PAFEM_CONVECTION) {
      require(s.dim == 3, PAFEM_EUNSUPPORTED, "the convection operator is built for hexahedra");
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "the convection operator is FP64");
    }
    if (s.dim == 2) {
      require(kind != PAFEM_DIFFUSION_GEOM, PAFEM_EUNSUPPORTED,
              "recomputed geometry is built for hexahedra only");
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "quadrilateral operators are FP64");
      require(!(flags & PAFEM_OP_SCATTER_EVEC), PAFEM_EUNSUPPORTED,
              "quadrilateral operators use the atomic scatter");
    }
    if (kind == PAFEM_DIFFUSION_GEOM) {
      require(s.ng == 2, PAFEM_EUNSUPPORTED, "recomputed geometry needs trilinear elements");
      require(qdata_dtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "recomputed geometry is FP64");
    }
    require(dtype_size(qdata_dtype) != 0, PAFEM_EINVAL, "unknown qdata dtype");
    require(q1d == s.p + 2, PAFEM_EUNSUPPORTED,
            "the fused apply is built for q1d = p + 2 only");
    require((flags & ~(PAFEM_OP_CONSTRAINED | PAFEM_OP_SCATTER_EVEC | PAFEM_OP_VECTOR3)) == 0,
            PAFEM_EINVAL, "unknown operator flags");
    if (flags & PAFEM_OP_VECTOR3) {
      require(kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, PAFEM_EUNSUPPORTED,
              "vector operators: mass or diffusion");
      require(s.dim == 3 && qdata_dtype == PAFEM_F64 && !(flags & PAFEM_OP_SCATTER_EVEC),
              PAFEM_EUNSUPPORTED, "vector operators are FP64, hexahedra, atomic scatter");
    }
    auto* o = new pafem_op_s();
    o->op.space = &s;
    o->op.kind = kind;
    o->op.q1d = q1d;
    o->op.qdata = qdata;
    o->op.qdtype = qdata_dtype;
    o->op.flags = flags;
    *out = o;
  });
}

void pafem_op_destroy(pafem_op op) { delete op; }

pafem_status pafem_op_workspace_bytes(pafem_op op, size_t* nbytes) {
  return guarded([&] {
    require(op && nbytes, PAFEM_EINVAL, "null pointer argument");
    *nbytes = op_work_bytes(op->op);
  });
}

pafem_status pafem_op_apply(pafem_op op, const double* x, double* y, void* work,
                            size_t work_bytes, void* stream) {
  return guarded([&] {
    require(op && x && y, PAFEM_EINVAL, "null pointer argument");
    require(x != y, PAFEM_EINVAL, "x and y must not alias");
    if (op->op.flags & PAFEM_OP_SCATTER_EVEC)
      require(work && work_bytes >= op_work_bytes(op->op), PAFEM_ESHAPE, "workspace too small");
    apply_op(op->op, x, y, work, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_op_diagonal(pafem_op op, double* diag, void* work, size_t work_bytes,
                               void* stream) {
  return guarded([&] {
    require(op && diag, PAFEM_EINVAL, "null pointer argument");
    require(op->op.qdtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "diagonal needs f64 qdata");
    require(op->op.kind != PAFEM_DIFFUSION_GEOM, PAFEM_EUNSUPPORTED,
            "diagonal: use the PAFEM_DIFFUSION operator of the same space and coefficient");
    require(!mixed_or_nonsymmetric(op->op.kind), PAFEM_EUNSUPPORTED,
            "diagonal of the convection, gradient, divergence and elasticity operators is not built");
    require(!(op->op.flags & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED,
            "vector operator: every component has the scalar operator's diagonal");
    require(work && work_bytes >= op_work_bytes(op->op), PAFEM_ESHAPE, "workspace too small");
    const Op& o = op->op;
    const Space& s = *o.space;
    auto st = static_cast<hipStream_t>(stream);
    double* ye = static_cast<double*>(work);
    launch_diagonal_evec(s.dev, o.kind, o.q1d, static_cast<const double*>(o.qdata), ye, st);
    const bool constrained = o.flags & PAFEM_OP_CONSTRAINED;
    launch_evec_gather(s.dev, ye, nullptr, constrained ? 2 : 0, 1.0, diag, st);
  });
}

pafem_status pafem_linear_form(pafem_space space, int32_t q1d, int32_t source,
                               const double* f_qp, double scale, double* b, void* work,
                               size_t work_bytes, void* stream) {
  return guarded([&] {
    const Space& s = uploaded_space(space);
    require(b != nullptr, PAFEM_EINVAL, "null output");
    require(q1d >= 1 && q1d <= kMaxQ1d, PAFEM_EUNSUPPORTED, "q1d out of range");
    require(source >= PAFEM_SOURCE_ARRAY && source <= PAFEM_SOURCE_SINE, PAFEM_EINVAL,
            "unknown source");
    require(source != PAFEM_SOURCE_ARRAY || f_qp, PAFEM_EINVAL, "source array missing");
    const size_t need = size_t(s.ne) * s.dpe * sizeof(double);
    require(work && work_bytes >= need, PAFEM_ESHAPE, "workspace too small");
    auto st = static_cast<hipStream_t>(stream);
    double* ye = static_cast<double*>(work);
    launch_linear_form_evec(s.dev, q1d, source, f_qp, scale, ye, st);
    launch_evec_gather(s.dev, ye, nullptr, 2, 0.0, b, st);
  });
}

pafem_status pafem_pcg_workspace_bytes(pafem_op op, int32_t max_iter, size_t* nbytes) {
  return guarded([&] {
    require(op && nbytes, PAFEM_EINVAL, "null pointer argument");
    require(op->op.qdtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "PCG needs an f64 operator");
    require(max_iter >= 0, PAFEM_EINVAL, "negative max_iter");
    const size_t n = size_t(op->op.space->ndofs);
    *nbytes = align256(sizeof(CGState)) + align256(3 * kCGBlocks * sizeof(double)) +
              align256((size_t(max_iter) + 1) * sizeof(double)) + 3 * align256(n * 8) +
              align256(size_t(pa_apply_blocks(op->op.space->dev)) * sizeof(double)) +
              op_work_bytes(op->op);
  });
}

pafem_status pafem_pcg_solve(pafem_op op, const double* diag, const double* b, double* x,
                             void* work, size_t work_bytes, const pafem_solve_opts* opts,
                             pafem_solve_result* result, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  pafem_status status = PAFEM_OK;
  pafem_status rc = guarded([&] {
    require(op && b && x && work && opts && result, PAFEM_EINVAL, "null pointer argument");
    const Op& o = op->op;
    require(o.qdtype == PAFEM_F64, PAFEM_EUNSUPPORTED, "PCG needs an f64 operator");
    require(!mixed_or_nonsymmetric(o.kind), PAFEM_EINVAL,
            "CG needs a symmetric operator on a scalar space");
    require(!(o.flags & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED,
            "CG on vector operators: solve each component with the scalar operator");
    require(opts->precond == PAFEM_PRECOND_NONE || opts->precond == PAFEM_PRECOND_JACOBI,
            PAFEM_EINVAL, "unknown preconditioner");
    require(opts->precond == PAFEM_PRECOND_NONE || diag, PAFEM_EINVAL,
            "Jacobi preconditioner needs diag");
    require(opts->max_iter >= 0 && opts->rel_tol >= 0.0, PAFEM_EINVAL, "bad solver options");
    size_t need = 0;
    require(pafem_pcg_workspace_bytes(op, opts->max_iter, &need) == PAFEM_OK, PAFEM_EINVAL,
            g_last_error);
    require(work_bytes >= need, PAFEM_ESHAPE, "workspace too small: need " + std::to_string(need));
    const Space& s = *o.space;
    const int64_t n = s.ndofs;
    const double* dg = opts->precond == PAFEM_PRECOND_JACOBI ? diag : nullptr;
    char* w = static_cast<char*>(work);
    auto* state = reinterpret_cast<CGState*>(w);
    w += align256(sizeof(CGState));
    auto* partials = reinterpret_cast<double*>(w);
    w += align256(3 * kCGBlocks * sizeof(double));
    auto* hist = reinterpret_cast<double*>(w);
    w += align256((size_t(opts->max_iter) + 1) * sizeof(double));
    auto* r = reinterpret_cast<double*>(w);
    w += align256(n * 8);
    auto* d = reinterpret_cast<double*>(w);
    w += align256(n * 8);
    auto* q = reinterpret_cast<double*>(w);
    w += align256(n * 8);
    const int nap = pa_apply_blocks(s.dev);
    auto* dotp = reinterpret_cast<double*>(w);
    w += align256(size_t(nap) * sizeof(double));
    void* opwork = w;
    auto st = static_cast<hipStream_t>(stream);
    const int check = std::max(1, opts->check_every);
    const uint8_t* ess = (o.flags & PAFEM_OP_CONSTRAINED) ? s.dev.bmask : nullptr;

    launch_cg_reset(state, opts->max_iter + 1, st);
    if (!opts->zero_guess) apply_op(o, x, q, opwork, st);
    launch_cg_init<double, double>(state, partials, b, 1.0, opts->zero_guess ? nullptr : q, dg,
                                   x, r, d, opts->zero_guess, opts->rel_tol, hist, n, st);
    // the atomic scatter's y-init of each apply is written by the preceding kernel
    const bool evec = o.flags & PAFEM_OP_SCATTER_EVEC;
    if (!evec) launch_scatter_init(s.dev, d, ess != nullptr, q, st);
    auto iterations = [&](hipStream_t s2, int count) {
      for (int k = 0; k < count; ++k) {
        apply_op(o, d, q, opwork, s2, dotp, !evec);
        launch_cg_alpha(state, partials, dotp, nap, ess, d, n, s2);
        launch_cg_update(state, partials, x, r, d, q, dg, hist, n, s2);
        if (evec)
          launch_cg_direction(state, r, dg, d, n, s2);
        else
          launch_cg_direction_init(state, r, dg, d, q, ess, n, s2);
      }
    };
    CapturedGraph graph;
    CGState host{};
    int launched = 0;
    while (true) {
      hip_check(hipMemcpyAsync(&host, state, sizeof(CGState), hipMemcpyDeviceToHost, st),
                "state read");
      hip_check(hipStreamSynchronize(st), "solver sync");
      if (host.done || launched >= opts->max_iter) break;
      const int batch = std::min(check, opts->max_iter - launched);
      if (graphs_enabled() && batch == check && check >= 2) {
        if (!graph.ready()) graph.capture([&](hipStream_t cs) { iterations(cs, check); });
        graph.launch(st);
      } else {
        iterations(st, batch);
      }
      launched += batch;
    }
    // true residual ||b - A x||
    apply_op(o, x, q, opwork, st);
    launch_residual(state, partials, b, q, nullptr, n, st);
    hip_check(hipMemcpyAsync(&host, state, sizeof(CGState), hipMemcpyDeviceToHost, st),
              "state read");
    hip_check(hipStreamSynchronize(st), "solver sync");
    result->iters = host.iter;
    result->converged = host.done == 1;
    result->rel_res = host.bb > 0 ? std::sqrt(host.rr / host.bb) : 0.0;
    result->true_rel_res = host.bb > 0 ? std::sqrt(host.res2 / host.bb) : 0.0;
    if (opts->res_hist && opts->res_hist_cap > 0) {
      const int nh = std::min(opts->res_hist_cap, host.iter + 1);
      hip_check(hipMemcpy(opts->res_hist, hist, size_t(nh) * sizeof(double),
                          hipMemcpyDeviceToHost), "history read");
    }
    if (host.done == 2)
      status = fail(PAFEM_EBREAKDOWN, "CG breakdown at iteration " + std::to_string(host.iter));
    else if (host.done != 1)
      status = fail(PAFEM_ENOTCONV, "CG did not converge in " + std::to_string(host.iter) +
                                        " iterations");
  });
  if (result)
    result->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc != PAFEM_OK ? rc : status;
}


pafem_status pafem_convert(int64_t n, const double* src, void* dst, int32_t dtype, void* stream) {
  return guarded([&] {
    require(n >= 0, PAFEM_EINVAL, "negative length");
    require(dtype == PAFEM_F32 || dtype == PAFEM_BF16, PAFEM_EINVAL, "dtype must be F32 or BF16");
    if (n == 0) return;
    require(src && dst, PAFEM_EINVAL, "null pointer argument");
    launch_convert(src, dst, dtype, n, static_cast<hipStream_t>(stream));
  });
}

namespace {

struct IRLayout {
  size_t state_hi, state_lo, partials, r64, q64, d32, q32, dinv32, dotp, opwork, total;
};

IRLayout ir_layout(const Op& hi, const Op& lo) {
  const size_t n = size_t(hi.space->ndofs);
  IRLayout L{};
  size_t o = 0;
  L.state_hi = o; o += align256(sizeof(CGState));
  L.state_lo = o; o += align256(sizeof(CGState));
  L.partials = o; o += align256(4 * kCGBlocks * sizeof(double));
  L.r64 = o; o += align256(n * 8);
  L.q64 = o; o += align256(n * 8);
  L.d32 = o; o += align256(n * 4);
  L.q32 = o; o += align256(n * 4);
  L.dinv32 = o; o += align256(n * 4);
  L.dotp = o; o += align256(size_t(pa_apply_blocks(hi.space->dev)) * sizeof(double));
  L.opwork = o; o += std::max(op_work_bytes(hi), op_work_bytes(lo));
  L.total = o;
  return L;
}

void check_ir_pair(const Op& hi, const Op& lo) {
  require(hi.qdtype == PAFEM_F64, PAFEM_EINVAL, "a_hi must be an FP64 operator");
  require(lo.qdtype == PAFEM_F32 || lo.qdtype == PAFEM_BF16, PAFEM_EINVAL,
          "a_lo must use F32 or BF16 quadrature data");
  require(hi.space == lo.space && hi.kind == lo.kind && hi.q1d == lo.q1d &&
              hi.flags == lo.flags,
          PAFEM_EINVAL, "a_hi and a_lo must be the same operator on the same space");
}

}  // namespace

pafem_status pafem_ir_workspace_bytes(pafem_op a_hi, pafem_op a_lo, size_t* nbytes) {
  return guarded([&] {
    require(a_hi && a_lo && nbytes, PAFEM_EINVAL, "null pointer argument");
    check_ir_pair(a_hi->op, a_lo->op);
    *nbytes = ir_layout(a_hi->op, a_lo->op).total;
  });
}

pafem_status pafem_ir_solve(pafem_op a_hi, pafem_op a_lo, const double* diag, const double* b,
                            double* x, void* work, size_t work_bytes, const pafem_ir_opts* opts,
                            pafem_ir_result* result, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  pafem_status status = PAFEM_OK;
  pafem_status rc = guarded([&] {
    require(a_hi && a_lo && b && x && work && opts && result, PAFEM_EINVAL,
            "null pointer argument");
    require(!((a_hi->op.flags | a_lo->op.flags) & PAFEM_OP_VECTOR3), PAFEM_EUNSUPPORTED,
            "refinement needs scalar operators");
    const Op& hi = a_hi->op;
    const Op& lo = a_lo->op;
    check_ir_pair(hi, lo);
    require(opts->precond == PAFEM_PRECOND_NONE || (opts->precond == PAFEM_PRECOND_JACOBI && diag),
            PAFEM_EINVAL, "Jacobi preconditioner needs diag");
    require(opts->max_outer >= 0 && opts->max_inner >= 1 && opts->rel_tol >= 0.0 &&
                opts->inner_rel_tol > 0.0,
            PAFEM_EINVAL, "bad solver options");
    const IRLayout L = ir_layout(hi, lo);
    require(work_bytes >= L.total, PAFEM_ESHAPE,
            "workspace too small: need " + std::to_string(L.total));
    const int64_t n = hi.space->ndofs;
    char* w = static_cast<char*>(work);
    auto* st_hi = reinterpret_cast<CGState*>(w + L.state_hi);
    auto* st_lo = reinterpret_cast<CGState*>(w + L.state_lo);
    auto* partials = reinterpret_cast<double*>(w + L.partials);
    auto* r64 = reinterpret_cast<double*>(w + L.r64);
    auto* q64 = reinterpret_cast<double*>(w + L.q64);
    auto* d32 = reinterpret_cast<float*>(w + L.d32);
    auto* q32 = reinterpret_cast<float*>(w + L.q32);
    auto* dinv = opts->precond == PAFEM_PRECOND_JACOBI ? reinterpret_cast<float*>(w + L.dinv32)
                                                       : nullptr;
    void* opwork = w + L.opwork;
    auto* dotp = reinterpret_cast<double*>(w + L.dotp);
    const int nap = pa_apply_blocks(hi.space->dev);
    const uint8_t* ess = (lo.flags & PAFEM_OP_CONSTRAINED) ? hi.space->dev.bmask : nullptr;
    auto st = static_cast<hipStream_t>(stream);
    const int check = std::max(1, opts->check_every);
    if (dinv) launch_ir_dinv(diag, dinv, n, st);
    hip_check(hipMemsetAsync(x, 0, size_t(n) * 8, st), "zero x");
    launch_cg_reset(st_hi, 0, st);
    launch_cg_reset(st_lo, 0, st);
    // r = b, ||b||
    hip_check(hipMemsetAsync(q64, 0, size_t(n) * 8, st), "zero q");
    launch_residual(st_hi, partials, b, q64, r64, n, st);
    CGState h{};
    hip_check(hipMemcpyAsync(&h, st_hi, sizeof(CGState), hipMemcpyDeviceToHost, st), "state read");
    hip_check(hipStreamSynchronize(st), "ir sync");
    const double bb = h.res2;
    double rr = bb;
    int outer = 0, inner_total = 0, inner_seen = 0;
    bool converged = bb == 0.0;
    if (opts->res_hist && opts->res_hist_cap > 0) opts->res_hist[0] = bb > 0 ? 1.0 : 0.0;
    double s = std::sqrt(rr);
    bool restart = true;  // the inner PCG (re)starts from d = z on r / s
    while (!converged && outer < opts->max_outer) {
      if (restart)
        launch_ir_start(st_lo, partials, r64, s, dinv, d32, q32, ess, opts->inner_rel_tol, n, st);
      // inner: Jacobi-PCG on A_lo d = r / ||r|| with the reduced-precision apply, x += ||r|| d
      int launched = 0;
      CGState hl{};
      while (true) {
        hip_check(hipMemcpyAsync(&hl, st_lo, sizeof(CGState), hipMemcpyDeviceToHost, st),
                  "state read");
        hip_check(hipStreamSynchronize(st), "ir sync");
        if (hl.done || launched >= opts->max_inner) break;
        const int batch = std::min(check, opts->max_inner - launched);
        for (int k = 0; k < batch; ++k) {
          apply_op(lo, d32, q32, opwork, st, dotp, /*y_ready=*/true);
          launch_cg_alpha<float>(st_lo, partials, dotp, nap, ess, d32, n, st);
          launch_ir_update(st_lo, partials, x, s, r64, d32, q32, dinv, n, st);
          launch_ir_direction(st_lo, r64, dinv, d32, q32, ess, n, st);
        }
        launched += batch;
      }
      // the inner iteration counter restarts with the inner PCG and continues otherwise
      inner_total += hl.iter - (restart ? 0 : inner_seen);
      inner_seen = hl.iter;
      ++outer;
      // FP64 residual of the refined iterate, into the inner residual's buffer
      apply_op(hi, x, q64, opwork, st);
      launch_residual(st_hi, partials, b, q64, r64, n, st);
      hip_check(hipMemcpyAsync(&h, st_hi, sizeof(CGState), hipMemcpyDeviceToHost, st),
                "state read");
      hip_check(hipStreamSynchronize(st), "ir sync");
      rr = h.res2;
      if (opts->res_hist && outer < opts->res_hist_cap) opts->res_hist[outer] = std::sqrt(rr / bb);
      converged = rr <= opts->rel_tol * opts->rel_tol * bb;
      if (!std::isfinite(rr)) break;
      if (converged) break;
      const double s_new = std::sqrt(rr);
      restart = !(opts->keep_direction && hl.done == 1);
      if (!restart) {
        launch_ir_replace(st_lo, partials, r64, s_new, dinv, d32, q32, opts->inner_rel_tol, n, st);
        launch_ir_direction(st_lo, r64, dinv, d32, q32, ess, n, st);
      }
      s = s_new;
    }
    result->outer = outer;
    result->inner_total = inner_total;
    result->converged = converged;
    result->rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (!converged)
      status = fail(PAFEM_ENOTCONV, "iterative refinement did not reach the tolerance in " +
                                        std::to_string(outer) + " steps");
  });
  if (result)
    result->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc != PAFEM_OK ? rc : status;
}


pafem_status pafem_batch_workspace_bytes(int32_t nops, size_t* nbytes) {
  return guarded([&] {
    require(nops > 0 && nbytes, PAFEM_EINVAL, "bad arguments");
    *nbytes = Batch::workspace_bytes(nops);
  });
}

pafem_status pafem_batch_create(int32_t nops, const pafem_op* ops, int32_t nrhs, void* work,
                                size_t work_bytes, pafem_batch* out) {
  return guarded([&] {
    require(nops > 0 && ops && out, PAFEM_EINVAL, "bad arguments");
    std::vector<const Op*> v;
    for (int i = 0; i < nops; ++i) {
      require(ops[i] != nullptr, PAFEM_EINVAL, "null operator in batch");
      v.push_back(&ops[i]->op);
    }
    auto* b = new pafem_batch_s();
    try {
      b->b = new Batch(v, nrhs, work, work_bytes);
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
  });
}

void pafem_batch_destroy(pafem_batch batch) {
  if (!batch) return;
  delete batch->b;
  delete batch;
}

pafem_status pafem_batch_apply(pafem_batch batch, const void* const* x, void* const* y,
                               void* stream) {
  return guarded([&] {
    require(batch && x && y, PAFEM_EINVAL, "null pointer argument");
    batch->b->apply(x, y, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_batch_autotune(pafem_batch batch, const void* const* x, void* const* y,
                                  const char* cache_path, int32_t reps, void* stream) {
  return guarded([&] {
    require(batch && x && y, PAFEM_EINVAL, "null pointer argument");
    batch->b->autotune(x, y, cache_path, reps, static_cast<hipStream_t>(stream));
  });
}

pafem_status pafem_batch_set_tile(pafem_batch batch, int32_t order, int32_t candidate) {
  return guarded([&] {
    require(batch != nullptr, PAFEM_EINVAL, "null batch");
    batch->b->set_candidate(order, candidate);
  });
}

pafem_status pafem_batch_describe(pafem_batch batch, char* buf, size_t len) {
  return guarded([&] {
    require(batch && buf && len > 0, PAFEM_EINVAL, "bad arguments");
    const std::string d = batch->b->describe();
    require(d.size() < len, PAFEM_ESHAPE, "buffer too small: need " + std::to_string(d.size() + 1));
    std::memcpy(buf, d.c_str(), d.size() + 1);
  });
}

}  // extern "C"
