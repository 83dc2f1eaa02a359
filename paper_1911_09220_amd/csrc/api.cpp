// C ABI of the library: argument checking, host orchestration, launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"
#include "launch.hpp"
#include "solver.hpp"

using namespace pafem;

struct pafem_mesh_s {
  Mesh m;
};
struct pafem_space_s {
  Space* s;
};
struct pafem_op_s {
  Op op;
};

namespace {

thread_local std::string g_last_error;

pafem_status fail(pafem_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

void hip_check(hipError_t err, const char* what) {
  if (err != hipSuccess) throw Error(PAFEM_EHIP, std::string(what) + ": " + hipGetErrorString(err));
}

void require(bool cond, pafem_status code, const std::string& msg) {
  if (!cond) throw Error(code, msg);
}

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

size_t op_work_bytes(const Op& op) {
  const Space& s = *op.space;
  const size_t evec = size_t(s.ne) * s.dpe;
  // diagonal needs an f64 element vector; the deterministic scatter an element
  // vector of the operator's vector type
  size_t need = evec * sizeof(double);
  return align256(need);
}

template <typename F>
pafem_status guarded(F&& f) {
  try {
    f();
    return PAFEM_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "out of host memory";
    return PAFEM_EINVAL;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PAFEM_EINVAL;
  }
}

// One application of the operator; `work` must hold op_work_bytes(op).
void apply_op(const Op& op, const void* x, void* y, void* work, hipStream_t st) {
  const Space& s = *op.space;
  const bool constrained = op.flags & PAFEM_OP_CONSTRAINED;
  const bool evec = op.flags & PAFEM_OP_SCATTER_EVEC;
  const int vdt = vector_dtype(op.qdtype);
  if (evec) {
    require(launch_pa_apply(s.dev, op.kind, op.q1d, op.qdtype, constrained, true, op.qdata, x,
                            work, vdt, st),
            PAFEM_EUNSUPPORTED, "apply kernel not built for this order/q1d/dtype");
    if (vdt == PAFEM_F64)
      launch_evec_gather(s.dev, static_cast<const double*>(work), static_cast<const double*>(x),
                         constrained ? 1 : 0, 0.0, static_cast<double*>(y), st);
    else
      launch_evec_gather_f32(s.dev, static_cast<const float*>(work), static_cast<const float*>(x),
                             constrained ? 1 : 0, static_cast<float*>(y), st);
  } else {
    if (vdt == PAFEM_F64)
      launch_scatter_init(s.dev, static_cast<const double*>(x), constrained,
                          static_cast<double*>(y), st);
    else
      launch_scatter_init_f32(s.dev, static_cast<const float*>(x), constrained,
                              static_cast<float*>(y), st);
    require(launch_pa_apply(s.dev, op.kind, op.q1d, op.qdtype, constrained, false, op.qdata, x,
                            y, vdt, st),
            PAFEM_EUNSUPPORTED, "apply kernel not built for this order/q1d/dtype");
  }
}

}  // namespace

extern "C" {

const char* pafem_last_error(void) { return g_last_error.c_str(); }

int32_t pafem_version(void) { return 100; }

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
    *out = m;
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

pafem_status pafem_space_dof_coords(pafem_space space, double* xyz) {
  return guarded([&] {
    require(space && space->s && xyz, PAFEM_EINVAL, "null pointer argument");
    space_dof_coords(*space->s, xyz);
  });
}

pafem_status pafem_space_boundary_dofs(pafem_space space, int32_t* idx) {
  return guarded([&] {
    require(space && space->s && idx, PAFEM_EINVAL, "null pointer argument");
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
    size_t off[8];
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
    size_t off[8], total = 0;
    space_device_layout(s, off, &total);
    require(nbytes >= total, PAFEM_ESHAPE,
            "device buffer too small: need " + std::to_string(total) + " bytes");
    std::vector<int32_t> gmap_enc, toff, tidx;
    std::vector<double> gnodes;
    space_pack(s, gmap_enc, gnodes, toff, tidx);
    auto st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(device_buf);
    hip_check(hipMemcpyAsync(base + off[0], gmap_enc.data(), gmap_enc.size() * 4,
                             hipMemcpyHostToDevice, st), "upload gmap");
    hip_check(hipMemcpyAsync(base + off[1], gnodes.data(), gnodes.size() * 8,
                             hipMemcpyHostToDevice, st), "upload geometry");
    hip_check(hipMemcpyAsync(base + off[2], s.bmask.data(), s.bmask.size(),
                             hipMemcpyHostToDevice, st), "upload boundary mask");
    hip_check(hipMemcpyAsync(base + off[3], toff.data(), toff.size() * 4,
                             hipMemcpyHostToDevice, st), "upload transposed offsets");
    hip_check(hipMemcpyAsync(base + off[4], tidx.data(), tidx.size() * 4,
                             hipMemcpyHostToDevice, st), "upload transposed map");
    hip_check(hipMemcpyAsync(base + off[5], s.tables.data(), s.tables.size() * 8,
                             hipMemcpyHostToDevice, st), "upload tables");
    hip_check(hipMemsetAsync(base + off[6], 0, 64 * 4, st), "clear status");
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
    s.dev.ne = s.ne;
    s.dev.ndofs = s.ndofs;
    s.dev.p = s.p;
    s.dev.ng = s.ng;
    s.uploaded = true;
  });
}

pafem_status pafem_qdata_size(pafem_space space, int32_t kind, int32_t q1d, int64_t* nvalues) {
  return guarded([&] {
    require(space && space->s && nvalues, PAFEM_EINVAL, "null pointer argument");
    require(kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, PAFEM_EINVAL, "unknown operator kind");
    require(q1d >= 1 && q1d <= kMaxQ1d, PAFEM_EUNSUPPORTED, "q1d out of range");
    const int64_t qqq = int64_t(q1d) * q1d * q1d;
    *nvalues = space->s->ne * qqq * (kind == PAFEM_DIFFUSION ? 6 : 1);
  });
}

pafem_status pafem_qdata_assemble(pafem_space space, int32_t kind, int32_t q1d,
                                  const double* coeff, double coeff_scale, double* qdata,
                                  void* stream) {
  return guarded([&] {
    const Space& s = uploaded_space(space);
    require(qdata != nullptr, PAFEM_EINVAL, "null qdata");
    require(kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, PAFEM_EINVAL, "unknown operator kind");
    require(q1d >= 1 && q1d <= kMaxQ1d, PAFEM_EUNSUPPORTED, "q1d out of range");
    auto st = static_cast<hipStream_t>(stream);
    hip_check(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(s.dev.status), INT_MAX, 1, st),
              "status init");
    launch_qdata(s.dev, kind, q1d, coeff, coeff_scale, qdata, st);
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
    require(kind == PAFEM_MASS || kind == PAFEM_DIFFUSION, PAFEM_EINVAL, "unknown operator kind");
    require(dtype_size(qdata_dtype) != 0, PAFEM_EINVAL, "unknown qdata dtype");
    require(q1d == s.p + 2, PAFEM_EUNSUPPORTED,
            "the fused apply is built for q1d = p + 2 only");
    require((flags & ~(PAFEM_OP_CONSTRAINED | PAFEM_OP_SCATTER_EVEC)) == 0, PAFEM_EINVAL,
            "unknown operator flags");
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
    void* opwork = w;
    auto st = static_cast<hipStream_t>(stream);
    const int check = std::max(1, opts->check_every);

    launch_cg_reset(state, opts->max_iter + 1, st);
    if (!opts->zero_guess) apply_op(o, x, q, opwork, st);
    launch_cg_init(state, partials, b, opts->zero_guess ? nullptr : q, dg, x, r, d,
                   opts->zero_guess, opts->rel_tol, hist, n, st);
    CGState host{};
    int launched = 0;
    while (true) {
      hip_check(hipMemcpyAsync(&host, state, sizeof(CGState), hipMemcpyDeviceToHost, st),
                "state read");
      hip_check(hipStreamSynchronize(st), "solver sync");
      if (host.done || launched >= opts->max_iter) break;
      const int batch = std::min(check, opts->max_iter - launched);
      for (int k = 0; k < batch; ++k) {
        apply_op(o, d, q, opwork, st);
        launch_cg_dot(state, partials, d, q, n, st);
        launch_cg_update(state, partials, x, r, d, q, dg, hist, n, st);
        launch_cg_direction(state, r, dg, d, n, st);
      }
      launched += batch;
    }
    // true residual ||b - A x||
    apply_op(o, x, q, opwork, st);
    launch_residual_norm(state, partials, b, q, n, st);
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

}  // extern "C"
