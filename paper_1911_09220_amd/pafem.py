"""Thin ctypes binding of libpafem.so (argument marshalling only).

Every function named ``pafem_*`` here calls the C entry point of the same name
declared in ``include/pafem.h``; device buffers are torch tensors on the GPU
and the stream is torch's current stream.  The classes below only hold handles
and the caller-owned device buffers the C calls need.  No computation happens in
Python: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpafem.so")

MASS, DIFFUSION, DIFFUSION_GEOM, CONVECTION, GRADIENT, DIVERGENCE, ELASTICITY = 0, 1, 2, 3, 4, 5, 6
HCURL_MASS, HCURL_CURLCURL, HCURL_MAXWELL = 7, 8, 9
DG_CONVECTION = 10
SPACE_H1, SPACE_ND, SPACE_L2 = 0, 1, 2
F64, F32, BF16 = 0, 1, 2
SPACE_RENUMBER = 1
OP_CONSTRAINED, OP_SCATTER_EVEC, OP_VECTOR3 = 1, 2, 4
SOURCE_ARRAY, SOURCE_CONST, SOURCE_SINE = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI = 0, 1
MEAN_ARITHMETIC, MEAN_GEOMETRIC, MEAN_HARMONIC = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "EUNSUPPORTED", -4: "EHIP",
          -5: "ENOTCONV", -6: "EBREAKDOWN"}


class PafemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_iter", C.c_int32), ("precond", C.c_int32),
                ("check_every", C.c_int32), ("zero_guess", C.c_int32),
                ("res_hist", C.POINTER(C.c_double)), ("res_hist_cap", C.c_int32)]


class SolveResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("seconds", C.c_double)]


class IROpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("inner_rel_tol", C.c_double), ("max_outer", C.c_int32),
                ("max_inner", C.c_int32), ("check_every", C.c_int32), ("precond", C.c_int32),
                ("keep_direction", C.c_int32), ("res_hist", C.POINTER(C.c_double)),
                ("res_hist_cap", C.c_int32)]


class IRResult(C.Structure):
    _fields_ = [("outer", C.c_int32), ("inner_total", C.c_int32), ("converged", C.c_int32),
                ("rel_res", C.c_double), ("seconds", C.c_double)]


class PMGOpts(C.Structure):
    _fields_ = [("degree", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("coarse_iters", C.c_int32)]


class FCGResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("fell_back", C.c_int32),
                ("fallback_iter", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("seconds", C.c_double)]


ABI_VERSION = 274  # pafem_version() of the library whose structs are declared above


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch first: the library then binds to the HIP runtime torch already loaded, so
    # both share one runtime (two runtimes in one process do not see the same device)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "pafem_last_error": (C.c_char_p, []),
        "pafem_version": (I32, []),
        "pafem_set_graph_mode": (I32, [I32]),
        "pafem_mesh_create_hex": (I32, [I64, P, I64, P, I32, P, C.POINTER(P)]),
        "pafem_mesh_create_quad": (I32, [I64, P, I64, P, C.POINTER(P)]),
        "pafem_mesh_destroy": (None, [P]),
        "pafem_mesh_refine": (I32, [P, C.POINTER(P)]),
        "pafem_mesh_info": (I32, [P, C.POINTER(I64), C.POINTER(I64)]),
        "pafem_mesh_vertices": (I32, [P, P, P]),
        "pafem_space_dim": (I32, [P, C.POINTER(I32)]),
        "pafem_space_create_h1": (I32, [P, I32, I32, C.POINTER(P)]),
        "pafem_space_destroy": (None, [P]),
        "pafem_space_info": (I32, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32),
                                   C.POINTER(I64)]),
        "pafem_space_dof_coords": (I32, [P, P]),
        "pafem_space_boundary_dofs": (I32, [P, P]),
        "pafem_space_elem_dofs": (I32, [P, P]),
        "pafem_space_create_nd": (I32, [P, I32, I32, C.POINTER(P)]),
        "pafem_space_create_l2": (I32, [P, I32, I32, C.POINTER(P)]),
        "pafem_space_family": (I32, [P, C.POINTER(I32)]),
        "pafem_space_elem_signs": (I32, [P, P]),
        "pafem_space_device_bytes": (I32, [P, C.POINTER(SZ)]),
        "pafem_space_upload": (I32, [P, P, SZ, P]),
        "pafem_qdata_size": (I32, [P, I32, I32, C.POINTER(I64)]),
        "pafem_qdata_assemble": (I32, [P, I32, I32, P, D, P, P]),
        "pafem_op_create": (I32, [P, I32, I32, P, I32, I32, C.POINTER(P)]),
        "pafem_op_destroy": (None, [P]),
        "pafem_op_workspace_bytes": (I32, [P, C.POINTER(SZ)]),
        "pafem_op_apply": (I32, [P, P, P, P, SZ, P]),
        "pafem_op_apply_noalloc": (I32, [P, P, P, P]),
        "pafem_op_diagonal": (I32, [P, P, P, SZ, P]),
        "pafem_linear_form": (I32, [P, I32, I32, P, D, P, P, SZ, P]),
        "pafem_pcg_workspace_bytes": (I32, [P, I32, C.POINTER(SZ)]),
        "pafem_pcg_solve": (I32, [P, P, P, P, P, SZ, C.POINTER(SolveOpts),
                                  C.POINTER(SolveResult), P]),
        "pafem_convert": (I32, [I64, P, P, I32, P]),
        "pafem_batch_workspace_bytes": (I32, [I32, C.POINTER(SZ)]),
        "pafem_batch_create": (I32, [I32, P, I32, P, SZ, C.POINTER(P)]),
        "pafem_batch_destroy": (None, [P]),
        "pafem_batch_apply": (I32, [P, P, P, P]),
        "pafem_batch_autotune": (I32, [P, P, P, C.c_char_p, I32, P]),
        "pafem_batch_set_tile": (I32, [P, I32, I32]),
        "pafem_batch_describe": (I32, [P, C.c_char_p, SZ]),
        "pafem_net_storage_bytes": (I32, [I32, I32, I64, I64, C.POINTER(SZ)]),
        "pafem_net_create": (I32, [I32, I32, I64, I64, P, SZ, C.POINTER(P)]),
        "pafem_net_destroy": (None, [P]),
        "pafem_net_dims": (I32, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                 C.POINTER(I64)]),
        "pafem_net_set_params": (I32, [P, P, P]),
        "pafem_net_get_params": (I32, [P, P, P]),
        "pafem_net_get_grads": (I32, [P, P, P]),
        "pafem_net_forward": (I32, [P, P, P, I64, P]),
        "pafem_net_backward": (I32, [P, P, P, I64, P]),
        "pafem_net_adam_step": (I32, [P, C.c_float, P]),
        "pafem_net_get_state": (I32, [P, P, P, P]),
        "pafem_net_set_state": (I32, [P, P, I32, P]),
        "pafem_learned_features": (I32, [P, P, I32, P, P]),
        "pafem_learned_workspace_bytes": (I32, [P, C.POINTER(SZ)]),
        "pafem_learned_precond": (I32, [P, P, P, P, P, P, P, SZ, P]),
        "pafem_learned_loss_grad": (I32, [P, P, P, P, P, P, P, P, SZ, P]),
        "pafem_fcg_workspace_bytes": (I32, [P, I32, C.POINTER(SZ)]),
        "pafem_fcg_solve": (I32, [P, P, P, P, P, P, P, SZ, C.POINTER(SolveOpts),
                                  C.POINTER(FCGResult), P]),
        "pafem_coeff_element_mean": (I32, [P, I32, P, I32, I32, P, P]),
        "pafem_coeff_parent_mean": (I32, [P, P, I32, P, I32, I32, P, P]),
        "pafem_prolongate": (I32, [P, P, P, P, I32, P]),
        "pafem_restrict": (I32, [P, P, P, P, P, P]),
        "pafem_smoother_workspace_bytes": (I32, [P, C.POINTER(SZ)]),
        "pafem_op_lambda_max": (I32, [P, P, P, I32, P, SZ, C.POINTER(D), P]),
        "pafem_chebyshev_smooth": (I32, [P, P, D, D, D, I32, P, P, I32, P, SZ, P]),
        "pafem_pmg_create": (I32, [I32, P, P, P, C.POINTER(PMGOpts), C.POINTER(P)]),
        "pafem_pmg_destroy": (None, [P]),
        "pafem_pmg_workspace_bytes": (I32, [P, I32, C.POINTER(SZ)]),
        "pafem_pmg_vcycle": (I32, [P, P, P, P, SZ, P]),
        "pafem_pmg_fcg_solve": (I32, [P, P, P, P, SZ, C.POINTER(SolveOpts),
                                      C.POINTER(SolveResult), P]),
        "pafem_ir_workspace_bytes": (I32, [P, P, C.POINTER(SZ)]),
        "pafem_ir_solve": (I32, [P, P, P, P, P, P, SZ, C.POINTER(IROpts), C.POINTER(IRResult), P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.pafem_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {lib.pafem_version()}, this binding "
                          f"expects {ABI_VERSION}; rebuild with __graft_entry__.build()")
    return lib


lib = _load()


def _check(rc):
    if rc != 0:
        raise PafemError(rc, lib.pafem_last_error().decode())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _device_bytes(nbytes, device="cuda"):
    import torch
    # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---- thin wrappers with the C names -------------------------------------------------

def pafem_version():
    return lib.pafem_version()


def pafem_set_graph_mode(mode):
    """1: replay solver iterations from HIP graphs (default); 0: direct launches.
    Returns the previous mode."""
    return lib.pafem_set_graph_mode(int(mode))


def pafem_mesh_create_hex(vertices, hexes, geom_order=1, geom_nodes=None):
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    h = np.ascontiguousarray(hexes, dtype=np.int64)
    g = None if geom_nodes is None else np.ascontiguousarray(geom_nodes, dtype=np.float64)
    out = C.c_void_p()
    _check(lib.pafem_mesh_create_hex(v.shape[0], _np_ptr(v), h.shape[0], _np_ptr(h),
                                     int(geom_order), None if g is None else _np_ptr(g),
                                     C.byref(out)))
    return out


def pafem_mesh_create_quad(vertices, quads):
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    q = np.ascontiguousarray(quads, dtype=np.int64)
    out = C.c_void_p()
    _check(lib.pafem_mesh_create_quad(v.shape[0], _np_ptr(v), q.shape[0], _np_ptr(q), C.byref(out)))
    return out


def pafem_space_dim(space):
    d = C.c_int32()
    _check(lib.pafem_space_dim(space, C.byref(d)))
    return d.value


def pafem_space_create_h1(mesh, order, flags=0):
    out = C.c_void_p()
    _check(lib.pafem_space_create_h1(mesh, int(order), int(flags), C.byref(out)))
    return out


def pafem_space_create_nd(mesh, order, flags=0):
    out = C.c_void_p()
    _check(lib.pafem_space_create_nd(mesh, int(order), int(flags), C.byref(out)))
    return out


def pafem_space_create_l2(mesh, order, flags=0):
    out = C.c_void_p()
    _check(lib.pafem_space_create_l2(mesh, int(order), int(flags), C.byref(out)))
    return out


def pafem_space_info(space):
    nd, ne, nb = C.c_int64(), C.c_int64(), C.c_int64()
    dpe = C.c_int32()
    _check(lib.pafem_space_info(space, C.byref(nd), C.byref(ne), C.byref(dpe), C.byref(nb)))
    return nd.value, ne.value, dpe.value, nb.value


def pafem_space_device_bytes(space):
    n = C.c_size_t()
    _check(lib.pafem_space_device_bytes(space, C.byref(n)))
    return n.value


def pafem_space_upload(space, buf):
    _check(lib.pafem_space_upload(space, _ptr(buf), buf.numel() * buf.element_size(), _stream()))


def pafem_qdata_size(space, kind, q1d):
    n = C.c_int64()
    _check(lib.pafem_qdata_size(space, int(kind), int(q1d), C.byref(n)))
    return n.value


def pafem_qdata_assemble(space, kind, q1d, coeff, scale, qdata):
    _check(lib.pafem_qdata_assemble(space, int(kind), int(q1d), _ptr(coeff), float(scale),
                                    _ptr(qdata), _stream()))


def pafem_op_create(space, kind, q1d, qdata, qdata_dtype, flags):
    out = C.c_void_p()
    _check(lib.pafem_op_create(space, int(kind), int(q1d), _ptr(qdata), int(qdata_dtype),
                               int(flags), C.byref(out)))
    return out


def pafem_op_workspace_bytes(op):
    n = C.c_size_t()
    _check(lib.pafem_op_workspace_bytes(op, C.byref(n)))
    return n.value


def pafem_op_apply(op, x, y, work):
    _check(lib.pafem_op_apply(op, _ptr(x), _ptr(y), _ptr(work),
                              0 if work is None else work.numel(), _stream()))


def pafem_op_apply_noalloc(op, x, y):
    _check(lib.pafem_op_apply_noalloc(op, _ptr(x), _ptr(y), _stream()))


def pafem_op_diagonal(op, diag, work):
    _check(lib.pafem_op_diagonal(op, _ptr(diag), _ptr(work), work.numel(), _stream()))


def pafem_linear_form(space, q1d, source, f_qp, scale, b, work):
    _check(lib.pafem_linear_form(space, int(q1d), int(source), _ptr(f_qp), float(scale),
                                 _ptr(b), _ptr(work), work.numel(), _stream()))


def pafem_pcg_workspace_bytes(op, max_iter):
    n = C.c_size_t()
    _check(lib.pafem_pcg_workspace_bytes(op, int(max_iter), C.byref(n)))
    return n.value


def pafem_pcg_solve(op, diag, b, x, work, opts: SolveOpts):
    res = SolveResult()
    rc = lib.pafem_pcg_solve(op, _ptr(diag), _ptr(b), _ptr(x), _ptr(work), work.numel(),
                             C.byref(opts), C.byref(res), _stream())
    return rc, res


def pafem_convert(src, dst, dtype):
    _check(lib.pafem_convert(src.numel(), _ptr(src), _ptr(dst), int(dtype), _stream()))


def pafem_ir_workspace_bytes(a_hi, a_lo):
    n = C.c_size_t()
    _check(lib.pafem_ir_workspace_bytes(a_hi, a_lo, C.byref(n)))
    return n.value


def pafem_ir_solve(a_hi, a_lo, diag, b, x, work, opts: IROpts):
    res = IRResult()
    rc = lib.pafem_ir_solve(a_hi, a_lo, _ptr(diag), _ptr(b), _ptr(x), _ptr(work), work.numel(),
                            C.byref(opts), C.byref(res), _stream())
    return rc, res


def _ptr_array(tensors):
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


def pafem_batch_workspace_bytes(nops):
    n = C.c_size_t()
    _check(lib.pafem_batch_workspace_bytes(int(nops), C.byref(n)))
    return n.value


def pafem_batch_create(ops, nrhs, work):
    handles = (C.c_void_p * len(ops))(*[o.value for o in ops])
    out = C.c_void_p()
    _check(lib.pafem_batch_create(len(ops), handles, int(nrhs), _ptr(work), work.numel(),
                                  C.byref(out)))
    return out


def pafem_batch_apply(batch, xs, ys):
    _check(lib.pafem_batch_apply(batch, _ptr_array(xs), _ptr_array(ys), _stream()))


def pafem_batch_autotune(batch, xs, ys, cache_path=None, reps=5):
    _check(lib.pafem_batch_autotune(batch, _ptr_array(xs), _ptr_array(ys),
                                    None if cache_path is None else cache_path.encode(),
                                    int(reps), _stream()))


def pafem_batch_set_tile(batch, order, candidate):
    _check(lib.pafem_batch_set_tile(batch, int(order), int(candidate)))


def pafem_batch_describe(batch):
    buf = C.create_string_buffer(1 << 16)
    _check(lib.pafem_batch_describe(batch, buf, len(buf)))
    return buf.value.decode()


def pafem_coeff_parent_mean(fine, coarse, kind, coeff, q1d_in, q1d_out, out):
    _check(lib.pafem_coeff_parent_mean(fine, coarse, int(kind), _ptr(coeff), int(q1d_in),
                                       int(q1d_out), _ptr(out), _stream()))


def pafem_coeff_element_mean(space, kind, coeff, q1d_in, q1d_out, out):
    _check(lib.pafem_coeff_element_mean(space, int(kind), _ptr(coeff), int(q1d_in), int(q1d_out),
                                        _ptr(out), _stream()))


def pafem_prolongate(coarse, fine, xc, yf, add=False):
    _check(lib.pafem_prolongate(coarse, fine, _ptr(xc), _ptr(yf), int(bool(add)), _stream()))


def pafem_restrict(fine, coarse, bf, yf, rc):
    _check(lib.pafem_restrict(fine, coarse, _ptr(bf), _ptr(yf), _ptr(rc), _stream()))


def pafem_smoother_workspace_bytes(op):
    n = C.c_size_t()
    _check(lib.pafem_smoother_workspace_bytes(op, C.byref(n)))
    return n.value


def pafem_op_lambda_max(op, diag, v, iters, work):
    lam = C.c_double()
    _check(lib.pafem_op_lambda_max(op, _ptr(diag), _ptr(v), int(iters), _ptr(work), work.numel(),
                                   C.byref(lam), _stream()))
    return lam.value


def pafem_chebyshev_smooth(op, diag, lmax, lo, hi, degree, b, x, zero_guess, work):
    _check(lib.pafem_chebyshev_smooth(op, _ptr(diag), float(lmax), float(lo), float(hi),
                                      int(degree), _ptr(b), _ptr(x), int(bool(zero_guess)),
                                      _ptr(work), work.numel(), _stream()))


def pafem_pmg_create(ops, diags, lmax, opts: PMGOpts):
    n = len(ops)
    oh = (C.c_void_p * n)(*[o.value for o in ops])
    dh = _ptr_array(diags)
    lm = (C.c_double * n)(*[float(v) for v in lmax])
    out = C.c_void_p()
    _check(lib.pafem_pmg_create(n, oh, dh, lm, C.byref(opts), C.byref(out)))
    return out


def pafem_pmg_workspace_bytes(pmg, max_iter):
    n = C.c_size_t()
    _check(lib.pafem_pmg_workspace_bytes(pmg, int(max_iter), C.byref(n)))
    return n.value


def pafem_pmg_vcycle(pmg, r, z, work):
    _check(lib.pafem_pmg_vcycle(pmg, _ptr(r), _ptr(z), _ptr(work), work.numel(), _stream()))


def pafem_pmg_fcg_solve(pmg, b, x, work, opts: SolveOpts):
    res = SolveResult()
    rc = lib.pafem_pmg_fcg_solve(pmg, _ptr(b), _ptr(x), _ptr(work), work.numel(), C.byref(opts),
                                 C.byref(res), _stream())
    return rc, res


def lowered_qdata(qdata, dtype):
    """Reduced-precision copy (F32 or BF16 bits) of f64 quadrature data, on the device."""
    import torch
    out = torch.empty(qdata.numel(), dtype=torch.float32 if dtype == F32 else torch.int16,
                      device=qdata.device)
    pafem_convert(qdata, out, dtype)
    return out


# ---- handle-owning conveniences -----------------------------------------------------

class Mesh:
    """Hexahedral mesh, or quadrilateral with ``quads`` (2D vertices) instead of hexes."""

    def __init__(self, vertices, hexes=None, geom_order=1, geom_nodes=None, quads=None):
        if quads is not None:
            self.dim = 2
            self.handle = pafem_mesh_create_quad(vertices, quads)
        else:
            self.dim = 3
            self.handle = pafem_mesh_create_hex(vertices, hexes, geom_order, geom_nodes)

    @classmethod
    def from_dict(cls, m):
        if "quad" in m:
            return cls(m["vertices"], quads=m["quad"])
        return cls(m["vertices"], m["hex"], m.get("geom_order", 1), m.get("geom_nodes"))

    def refine(self):
        """Uniform refinement (pafem_mesh_refine): child 8 e + o covers octant o of
        element e's reference cube; spaces on the result take transfers from spaces on
        this mesh."""
        out = C.c_void_p()
        _check(lib.pafem_mesh_refine(self.handle, C.byref(out)))
        m = Mesh.__new__(Mesh)
        m.dim, m.handle = self.dim, out
        return m

    def counts(self):
        nv, ne = C.c_int64(), C.c_int64()
        _check(lib.pafem_mesh_info(self.handle, C.byref(nv), C.byref(ne)))
        return nv.value, ne.value

    def arrays(self):
        """(vertices [nv, dim], elements [ne, 8 or 4]) host copies."""
        nv, ne = self.counts()
        v = np.empty((nv, self.dim), dtype=np.float64)
        e = np.empty((ne, 8 if self.dim == 3 else 4), dtype=np.int64)
        _check(lib.pafem_mesh_vertices(self.handle, _np_ptr(v), _np_ptr(e)))
        return v, e

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "handle", None) and lib is not None:
            lib.pafem_mesh_destroy(self.handle)
            self.handle = None


class Space:
    """H1 space of order p; uploads its device image on construction."""

    def __init__(self, mesh: Mesh, order: int, renumber: bool = False, device="cuda",
                 family="h1"):
        """family "h1" (nodal Gauss-Lobatto), "nd" (Nedelec, H(curl)) or "l2"
        (discontinuous nodal Gauss-Lobatto)."""
        self.mesh = mesh  # keeps the mesh alive
        self.p = int(order)
        creators = {"h1": pafem_space_create_h1, "nd": pafem_space_create_nd,
                    "l2": pafem_space_create_l2}
        if family not in creators:
            raise ValueError("family must be 'h1', 'nd' or 'l2'")
        self.family = family
        create = creators[family]
        self.handle = create(mesh.handle, order, SPACE_RENUMBER if renumber else 0)
        self.ndofs, self.nelem, self.dofs_per_elem, self.nbdr = pafem_space_info(self.handle)
        self.dim = pafem_space_dim(self.handle)
        self.device = device
        self.buf = None
        if device is not None:
            self.buf = _device_bytes(pafem_space_device_bytes(self.handle), device)
            pafem_space_upload(self.handle, self.buf)

    def dof_coords(self):
        out = np.empty((self.ndofs, self.dim))
        _check(lib.pafem_space_dof_coords(self.handle, _np_ptr(out)))
        return out

    def boundary_dofs(self):
        out = np.empty(self.nbdr, dtype=np.int32)
        _check(lib.pafem_space_boundary_dofs(self.handle, _np_ptr(out)))
        return out

    def elem_dofs(self):
        out = np.empty((self.nelem, self.dofs_per_elem), dtype=np.int32)
        _check(lib.pafem_space_elem_dofs(self.handle, _np_ptr(out)))
        return out

    def elem_signs(self):
        """Orientation sign (+1 / -1) of every element's local dofs in the global basis."""
        out = np.empty((self.nelem, self.dofs_per_elem), dtype=np.int8)
        _check(lib.pafem_space_elem_signs(self.handle, _np_ptr(out)))
        return out

    def _check_qp_array(self, a, q1d, name):
        if a is None:
            return
        need = self.nelem * q1d ** self.dim
        if a.numel() != need or a.dtype != __import__("torch").float64 or not a.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 array of {need} values")

    def qdata(self, kind, q1d=None, coeff=None, scale=1.0):
        """Quadrature data of an operator kind; coeff per point [E*Q^dim] (for
        CONVECTION the velocity, [E*Q^3*3]; for ELASTICITY (lambda, mu) pairs, [E*Q^3*2])."""
        import torch
        q1d = self.p + 2 if q1d is None else q1d
        if kind == CONVECTION:
            if coeff is None or coeff.numel() != self.nelem * q1d ** 3 * 3 or not coeff.is_contiguous():
                raise ValueError("convection needs a contiguous velocity [E][Q^3][3]")
        elif kind == DG_CONVECTION:
            if coeff is None or coeff.numel() != 3 or coeff.dtype != torch.float64 or not coeff.is_cuda:
                raise ValueError("DG convection needs the constant velocity as a float64 device "
                                 "tensor of 3 values")
        elif kind in (ELASTICITY, HCURL_MAXWELL):
            if (coeff is None or coeff.numel() != self.nelem * q1d ** 3 * 2 or not coeff.is_contiguous()
                    or coeff.dtype != torch.float64):
                raise ValueError("this operator needs contiguous float64 coefficient pairs "
                                 "[E][Q^3][2]")
        else:
            self._check_qp_array(coeff, q1d, "coeff")
        qd = torch.empty(pafem_qdata_size(self.handle, kind, q1d), dtype=torch.float64,
                         device=self.device)
        pafem_qdata_assemble(self.handle, kind, q1d, coeff, scale, qd)
        return qd

    def coeff_mean(self, coeff, q1d_in=None, q1d_out=None, kind=MEAN_ARITHMETIC):
        """Per-element mean of a per-point coefficient, spread over another rule."""
        import torch
        q1d_in = self.p + 2 if q1d_in is None else q1d_in
        q1d_out = self.p + 2 if q1d_out is None else q1d_out
        self._check_qp_array(coeff, q1d_in, "coeff")
        out = torch.empty(self.nelem * q1d_out ** 3, dtype=torch.float64, device=self.device)
        pafem_coeff_element_mean(self.handle, kind, coeff, q1d_in, q1d_out, out)
        return out

    def coeff_parent_mean(self, coarse, coeff, q1d_in=None, q1d_out=None, kind=MEAN_ARITHMETIC):
        """Mean of a per-point coefficient on this space's (refined) mesh over the 8
        children of each element of ``coarse``'s mesh, spread over ``coarse``'s rule."""
        import torch
        q1d_in = self.p + 2 if q1d_in is None else q1d_in
        q1d_out = coarse.p + 2 if q1d_out is None else q1d_out
        self._check_qp_array(coeff, q1d_in, "coeff")
        out = torch.empty(coarse.nelem * q1d_out ** 3, dtype=torch.float64, device=self.device)
        pafem_coeff_parent_mean(self.handle, coarse.handle, kind, coeff, q1d_in, q1d_out, out)
        return out

    def linear_form(self, source=SOURCE_SINE, q1d=None, f_qp=None, scale=1.0):
        import torch
        q1d = self.p + 2 if q1d is None else q1d
        self._check_qp_array(f_qp, q1d, "f_qp")
        b = torch.empty(self.ndofs, dtype=torch.float64, device=self.device)
        work = _device_bytes(self.nelem * self.dofs_per_elem * 8, self.device)
        pafem_linear_form(self.handle, q1d, source, f_qp, scale, b, work)
        return b

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "handle", None) and lib is not None:
            lib.pafem_space_destroy(self.handle)
            self.handle = None


class Operator:
    """y = A x for the PA mass or diffusion operator on a Space."""

    def __init__(self, space: Space, kind, qdata, q1d=None, constrained=True,
                 scatter="atomic", qdata_dtype=F64, vector=False):
        """vector=True: the operator on each of 3 components (vectors of 3 * ndofs)."""
        self.space, self.kind, self.qdata = space, kind, qdata
        self.q1d = space.p + 2 if q1d is None else q1d
        self.vector = bool(vector)
        flags = ((OP_CONSTRAINED if constrained else 0) | (OP_SCATTER_EVEC if scatter == "evec" else 0)
                 | (OP_VECTOR3 if vector else 0))
        self.handle = pafem_op_create(space.handle, kind, self.q1d, qdata, qdata_dtype, flags)
        self.work = _device_bytes(pafem_op_workspace_bytes(self.handle), space.device)
        self.vec_dtype = "float64" if qdata_dtype == F64 else "float32"

    def _check_vec(self, v, name, dtype=None):
        want = self.vec_dtype if dtype is None else dtype
        if (v.numel() != self.space.ndofs or not v.is_contiguous() or not v.is_cuda
                or str(v.dtype) != "torch." + want):
            raise ValueError(f"{name} must be a contiguous {want} device vector of "
                             f"{self.space.ndofs}")

    def apply(self, x, y=None):
        """y = A x; GRADIENT writes, DIVERGENCE reads, ELASTICITY and vector operators
        read and write 3 * ndofs values (component-major)."""
        import torch
        nout = 3 if self.kind == GRADIENT else 1
        if self.kind == DIVERGENCE:
            n3 = 3 * self.space.ndofs
            if x.numel() != n3 or not x.is_contiguous() or not x.is_cuda or x.dtype != torch.float64:
                raise ValueError(f"x must be a contiguous float64 device vector of {n3}")
            if y is None:
                y = torch.empty(self.space.ndofs, dtype=x.dtype, device=x.device)
            self._check_vec(y, "y")
            pafem_op_apply(self.handle, x, y, self.work)
            return y
        if y is None:
            y = torch.empty(nout * x.numel(), dtype=x.dtype, device=x.device)
        if self.vector or self.kind == ELASTICITY:
            for v, nm in ((x, "x"), (y, "y")):
                if (v.numel() != 3 * self.space.ndofs or not v.is_contiguous() or not v.is_cuda
                        or v.dtype != torch.float64):
                    raise ValueError(f"{nm} must be a contiguous float64 device vector of "
                                     f"{3 * self.space.ndofs}")
            pafem_op_apply(self.handle, x, y, self.work)
            return y
        self._check_vec(x, "x")
        if nout == 1:
            self._check_vec(y, "y")
        elif (y.numel() != 3 * self.space.ndofs or not y.is_contiguous() or not y.is_cuda
              or y.dtype != x.dtype):
            raise ValueError(f"y must be a contiguous device vector of {3 * self.space.ndofs}")
        pafem_op_apply(self.handle, x, y, self.work)
        return y

    def apply_noalloc(self, x, y):
        """y = A x through pafem_op_apply_noalloc: no workspace and no allocation (the
        caller passes y).  Scalar operators only."""
        if self.vector or self.kind in (GRADIENT, DIVERGENCE, ELASTICITY):
            raise ValueError("apply_noalloc: scalar operators only")
        self._check_vec(x, "x")
        self._check_vec(y, "y")
        pafem_op_apply_noalloc(self.handle, x, y)
        return y

    def diagonal(self):
        import torch
        d = torch.empty(self.space.ndofs, dtype=torch.float64, device=self.space.device)
        pafem_op_diagonal(self.handle, d, self.work)
        return d

    def pcg(self, b, x=None, diag=None, rel_tol=1e-10, max_iter=2000, precond=PRECOND_JACOBI,
            check_every=8, history=True):
        import torch
        if precond == PRECOND_JACOBI and diag is None:
            diag = self.diagonal()
        zero = x is None
        if x is None:
            x = torch.zeros_like(b)
        for v, nm in ((b, "b"), (x, "x")) + (((diag, "diag"),) if diag is not None else ()):
            self._check_vec(v, nm)
        work = _device_bytes(pafem_pcg_workspace_bytes(self.handle, max_iter), self.space.device)
        hist = np.zeros(max_iter + 1) if history else None
        opts = SolveOpts(float(rel_tol), int(max_iter), int(precond), int(check_every), int(zero),
                         None if hist is None else hist.ctypes.data_as(C.POINTER(C.c_double)),
                         0 if hist is None else hist.size)
        rc, res = pafem_pcg_solve(self.handle, diag if precond == PRECOND_JACOBI else None,
                                  b, x, work, opts)
        if rc not in (0, -5, -6):
            _check(rc)
        info = {"status": STATUS.get(rc, rc), "iters": res.iters, "converged": bool(res.converged),
                "rel_res": res.rel_res, "true_rel_res": res.true_rel_res, "seconds": res.seconds}
        if hist is not None:
            info["history"] = hist[: res.iters + 1].copy()
        return x, info

    def lambda_max(self, diag, v, iters=20):
        """Power-iteration estimate of the largest eigenvalue of diag^-1 A (v: start
        vector, overwritten)."""
        self._check_vec(v, "v")
        self._check_vec(diag, "diag")
        work = _device_bytes(pafem_smoother_workspace_bytes(self.handle), self.space.device)
        return pafem_op_lambda_max(self.handle, diag, v, iters, work)

    def chebyshev(self, diag, lmax, b, x=None, degree=2, lo=0.3, hi=1.1):
        """degree Chebyshev-Jacobi steps on A x = b (x None: from zero)."""
        import torch
        zero = x is None
        if zero:
            x = torch.empty_like(b)
        for v, nm in ((b, "b"), (x, "x"), (diag, "diag")):
            self._check_vec(v, nm)
        work = _device_bytes(pafem_smoother_workspace_bytes(self.handle), self.space.device)
        pafem_chebyshev_smooth(self.handle, diag, lmax, lo, hi, degree, b, x, zero, work)
        return x

    def ir_solve(self, lo, b, diag=None, rel_tol=1e-10, inner_rel_tol=1e-2, max_outer=50,
                 max_inner=5000, check_every=8, precond=PRECOND_JACOBI, keep_direction=True):
        """Iterative refinement with `lo` (same operator on F32/BF16 qdata) as inner solver.

        keep_direction: the inner PCG continues across steps with its residual replaced
        by the FP64 one (reliable update); False restarts it at every step."""
        import torch
        if precond == PRECOND_JACOBI and diag is None:
            diag = self.diagonal()
        self._check_vec(b, "b")
        x = torch.empty_like(b)
        work = _device_bytes(pafem_ir_workspace_bytes(self.handle, lo.handle), self.space.device)
        hist = np.zeros(max_outer + 1)
        opts = IROpts(float(rel_tol), float(inner_rel_tol), int(max_outer), int(max_inner),
                      int(check_every), int(precond), int(bool(keep_direction)),
                      hist.ctypes.data_as(C.POINTER(C.c_double)), hist.size)
        rc, res = pafem_ir_solve(self.handle, lo.handle,
                                 diag if precond == PRECOND_JACOBI else None, b, x, work, opts)
        if rc not in (0, -5):
            _check(rc)
        return x, {"status": STATUS.get(rc, rc), "outer": res.outer, "inner_total": res.inner_total,
                   "converged": bool(res.converged), "rel_res": res.rel_res,
                   "seconds": res.seconds, "history": hist[: res.outer + 1].copy()}

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "handle", None) and lib is not None:
            lib.pafem_op_destroy(self.handle)
            self.handle = None


def prolongate(coarse: Space, fine: Space, xc, yf=None, add=False):
    """yf (+)= P xc: the coarse function at the fine nodes (free dofs)."""
    import torch
    if yf is None:
        yf = torch.empty(fine.ndofs, dtype=torch.float64, device=fine.device)
    for v, S, nm in ((xc, coarse, "xc"), (yf, fine, "yf")):
        if v.numel() != S.ndofs or v.dtype != torch.float64 or not v.is_contiguous() or not v.is_cuda:
            raise ValueError(f"{nm} must be a contiguous float64 device vector of {S.ndofs}")
    pafem_prolongate(coarse.handle, fine.handle, xc, yf, add)
    return yf


def restrict(fine: Space, coarse: Space, bf, yf=None, rc=None):
    """rc = P^T (bf - yf) on free dofs."""
    import torch
    if rc is None:
        rc = torch.empty(coarse.ndofs, dtype=torch.float64, device=coarse.device)
    for v, S, nm in ((bf, fine, "bf"), (yf, fine, "yf"), (rc, coarse, "rc")):
        if v is None:
            continue
        if v.numel() != S.ndofs or v.dtype != torch.float64 or not v.is_contiguous() or not v.is_cuda:
            raise ValueError(f"{nm} must be a contiguous float64 device vector of {S.ndofs}")
    pafem_restrict(fine.handle, coarse.handle, bf, yf, rc)
    return rc


class PMG:
    """Multigrid V-cycle over constrained diffusion operators (finest first): each
    level on the previous level's Mesh (lower order) or on the Mesh it was refined from
    (Mesh.refine; h-multigrid); diagonals and largest-eigenvalue estimates per level."""

    def __init__(self, ops, diags, lmax, degree=2, lo=0.3, hi=1.1, coarse_iters=20):
        self.ops, self.diags = list(ops), list(diags)  # kept alive: the library holds pointers
        for o, d in zip(self.ops, self.diags):
            o._check_vec(d, "diag")
        self.lmax = [float(v) for v in lmax]
        self.opts = PMGOpts(int(degree), float(lo), float(hi), int(coarse_iters))
        self.handle = pafem_pmg_create([o.handle for o in self.ops], self.diags, self.lmax,
                                       self.opts)
        self.device = self.ops[0].space.device
        self._vwork = None

    def vcycle(self, r, z=None):
        import torch
        if z is None:
            z = torch.empty_like(r)
        self.ops[0]._check_vec(r, "r")
        self.ops[0]._check_vec(z, "z")
        if self._vwork is None:
            self._vwork = _device_bytes(pafem_pmg_workspace_bytes(self.handle, -1), self.device)
        pafem_pmg_vcycle(self.handle, r, z, self._vwork)
        return z

    def fcg(self, b, x=None, rel_tol=1e-8, max_iter=500, check_every=4, history=True):
        import torch
        zero = x is None
        if x is None:
            x = torch.zeros_like(b)
        self.ops[0]._check_vec(b, "b")
        self.ops[0]._check_vec(x, "x")
        work = _device_bytes(pafem_pmg_workspace_bytes(self.handle, max_iter), self.device)
        hist = np.zeros(max_iter + 1) if history else None
        opts = SolveOpts(float(rel_tol), int(max_iter), PRECOND_NONE, int(check_every), int(zero),
                         None if hist is None else hist.ctypes.data_as(C.POINTER(C.c_double)),
                         0 if hist is None else hist.size)
        rc, res = pafem_pmg_fcg_solve(self.handle, b, x, work, opts)
        if rc not in (0, -5, -6):
            _check(rc)
        info = {"status": STATUS.get(rc, rc), "iters": res.iters, "converged": bool(res.converged),
                "rel_res": res.rel_res, "true_rel_res": res.true_rel_res, "seconds": res.seconds}
        if hist is not None:
            info["history"] = hist[: res.iters + 1].copy()
        return x, info

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "handle", None) and lib is not None:
            lib.pafem_pmg_destroy(self.handle)
            self.handle = None


class Batch:
    """Many meshes x nrhs right-hand sides in one graph launch (vectors [ndofs, nrhs])."""

    def __init__(self, ops, nrhs=16):
        self.ops = list(ops)  # keep operators (and their spaces) alive
        self.nrhs = int(nrhs)
        dev = self.ops[0].space.device
        self.work = _device_bytes(pafem_batch_workspace_bytes(len(self.ops)), dev)
        self.handle = pafem_batch_create([o.handle for o in self.ops], self.nrhs, self.work)

    def _check(self, xs, ys):
        if len(xs) != len(self.ops) or len(ys) != len(self.ops):
            raise ValueError("one x and one y per operator")
        for o, x, y in zip(self.ops, xs, ys):
            for v in (x, y):
                if v.numel() != o.space.ndofs * self.nrhs or not v.is_contiguous() or not v.is_cuda:
                    raise ValueError("batch vectors must be contiguous [ndofs, nrhs] device arrays")

    def apply(self, xs, ys):
        self._check(xs, ys)
        pafem_batch_apply(self.handle, xs, ys)
        return ys

    def autotune(self, xs, ys, cache_path=None, reps=5):
        self._check(xs, ys)
        pafem_batch_autotune(self.handle, xs, ys, cache_path, reps)

    def set_tile(self, order, candidate):
        pafem_batch_set_tile(self.handle, order, candidate)

    def describe(self):
        import json
        return json.loads(pafem_batch_describe(self.handle))

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "handle", None) and lib is not None:
            lib.pafem_batch_destroy(self.handle)
            self.handle = None


class Net:
    """Learned element preconditioner parameters: the element network (BF16 MFMA
    kernels, FP32 master weights) and the element basis V [(p+1)^3, out_dim]; Adam."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "V")

    def __init__(self, order, hidden=128, max_rows=1, max_train_rows=0, device="cuda"):
        n = C.c_size_t()
        _check(lib.pafem_net_storage_bytes(int(order), int(hidden), int(max_rows),
                                           int(max_train_rows), C.byref(n)))
        self.storage = _device_bytes(n.value, device)
        self.handle = C.c_void_p()
        _check(lib.pafem_net_create(int(order), int(hidden), int(max_rows), int(max_train_rows),
                                    _ptr(self.storage), self.storage.numel(),
                                    C.byref(self.handle)))
        i, h, o, npar = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib.pafem_net_dims(self.handle, C.byref(i), C.byref(h), C.byref(o), C.byref(npar)))
        self.in_dim, self.hidden, self.out_dim, self.nparams = i.value, h.value, o.value, npar.value
        self.order = int(order)
        self.shapes = {"W1": (self.hidden, self.in_dim), "b1": (self.hidden,),
                       "W2": (self.hidden, self.hidden), "b2": (self.hidden,),
                       "W3": (self.out_dim, self.hidden), "b3": (self.out_dim,),
                       "V": ((self.order + 1) ** 3, self.out_dim)}

    def flatten(self, params):
        return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1)
                               for k in self.NAMES]).astype(np.float32)

    def unflatten(self, flat):
        out, o = {}, 0
        for k in self.NAMES:
            n = int(np.prod(self.shapes[k]))
            out[k] = flat[o:o + n].reshape(self.shapes[k]).astype(np.float64)
            o += n
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(params if isinstance(params, np.ndarray) else self.flatten(params),
                                    dtype=np.float32)
        assert flat.size == self.nparams
        _check(lib.pafem_net_set_params(self.handle, _np_ptr(flat), _stream()))

    def get_params(self):
        flat = np.empty(self.nparams, dtype=np.float32)
        _check(lib.pafem_net_get_params(self.handle, _np_ptr(flat), _stream()))
        return self.unflatten(flat)

    def get_grads(self):
        flat = np.empty(self.nparams, dtype=np.float32)
        _check(lib.pafem_net_get_grads(self.handle, _np_ptr(flat), _stream()))
        return self.unflatten(flat)

    def get_state(self):
        """Training state: {"params", "adam_m", "adam_v"} (flat FP32) and "adam_step"."""
        flat = np.empty(3 * self.nparams, dtype=np.float32)
        step = C.c_int32()
        _check(lib.pafem_net_get_state(self.handle, _np_ptr(flat), C.byref(step), _stream()))
        n = self.nparams
        return {"params": flat[:n], "adam_m": flat[n:2 * n], "adam_v": flat[2 * n:],
                "adam_step": int(step.value)}

    def set_state(self, state):
        flat = np.ascontiguousarray(np.concatenate([np.asarray(state[k], dtype=np.float32).ravel()
                                                    for k in ("params", "adam_m", "adam_v")]))
        if flat.size != 3 * self.nparams:
            raise ValueError(f"state holds {flat.size // 3} parameters, the network "
                             f"{self.nparams}")
        _check(lib.pafem_net_set_state(self.handle, _np_ptr(flat), int(state["adam_step"]),
                                       _stream()))

    def forward(self, x_bf16, rows):
        import torch
        out = torch.empty(rows, self.out_dim, dtype=torch.float32, device=x_bf16.device)
        _check(lib.pafem_net_forward(self.handle, _ptr(x_bf16), _ptr(out), int(rows), _stream()))
        return out

    def backward(self, x_bf16, dout_bf16, rows):
        _check(lib.pafem_net_backward(self.handle, _ptr(x_bf16), _ptr(dout_bf16), int(rows),
                                      _stream()))

    def adam_step(self, lr):
        _check(lib.pafem_net_adam_step(self.handle, float(lr), _stream()))

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared
        if getattr(self, "handle", None) and lib is not None:
            lib.pafem_net_destroy(self.handle)
            self.handle = None


def learned_features(space, kappa=None, q1d=None):
    import torch
    q1d = space.p + 2 if q1d is None else q1d
    space._check_qp_array(kappa, q1d, "kappa")
    feats = torch.empty(space.nelem, 9, dtype=torch.float32, device=space.device)
    _check(lib.pafem_learned_features(space.handle, _ptr(kappa), int(q1d), _ptr(feats), _stream()))
    return feats


def _learned_work(op):
    n = C.c_size_t()
    _check(lib.pafem_learned_workspace_bytes(op.handle, C.byref(n)))
    return _device_bytes(n.value, op.space.device)


def learned_precond(net, op, feats, diag, r, work=None):
    import torch
    z = torch.empty_like(r)
    work = _learned_work(op) if work is None else work
    _check(lib.pafem_learned_precond(net.handle, op.handle, _ptr(feats), _ptr(diag), _ptr(r),
                                     _ptr(z), _ptr(work), work.numel(), _stream()))
    return z


def learned_loss_grad(net, op, feats, diag, r, e, loss=None, work=None):
    import torch
    loss = torch.zeros(1, dtype=torch.float64, device=r.device) if loss is None else loss
    work = _learned_work(op) if work is None else work
    _check(lib.pafem_learned_loss_grad(net.handle, op.handle, _ptr(feats), _ptr(diag), _ptr(r),
                                       _ptr(e), _ptr(loss), _ptr(work), work.numel(), _stream()))
    return loss


def fcg_solve(op, b, diag, net=None, feats=None, rel_tol=1e-8, max_iter=2000, check_every=8,
              history=True, x=None):
    """Flexible CG; x: starting guess, overwritten with the solution (None: from zero)."""
    import torch
    zero = x is None
    if zero:
        x = torch.zeros_like(b)
    op._check_vec(x, "x")
    n = C.c_size_t()
    _check(lib.pafem_fcg_workspace_bytes(op.handle, int(max_iter), C.byref(n)))
    work = _device_bytes(n.value, op.space.device)
    hist = np.zeros(max_iter + 1) if history else None
    opts = SolveOpts(float(rel_tol), int(max_iter), 0, int(check_every), int(zero),
                     None if hist is None else hist.ctypes.data_as(C.POINTER(C.c_double)),
                     0 if hist is None else hist.size)
    res = FCGResult()
    rc = lib.pafem_fcg_solve(op.handle, None if net is None else net.handle, _ptr(feats),
                             _ptr(diag), _ptr(b), _ptr(x), _ptr(work), work.numel(),
                             C.byref(opts), C.byref(res), _stream())
    if rc not in (0, -5, -6):
        _check(rc)
    info = {"status": STATUS.get(rc, rc), "iters": res.iters, "converged": bool(res.converged),
            "fell_back": bool(res.fell_back), "fallback_iter": res.fallback_iter,
            "rel_res": res.rel_res, "true_rel_res": res.true_rel_res, "seconds": res.seconds}
    if hist is not None:
        info["history"] = hist[: res.iters + 1].copy()
    return x, info
