"""ctypes binding of oracle/csr_host.c, the host timing variant of the oracle's CSR
matrix-vector product and Jacobi-PCG (oracle; test infrastructure only).

Built by ``build_library()`` (gcc -O2 -fopenmp), which __graft_entry__.build() calls;
the tests pin it against scipy's product and the oracle's Python PCG.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csr_host.c")
LIB = os.path.join(HERE, "libcsr_host.so")


def build_library():
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"],
                   check=True, capture_output=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built; run __graft_entry__.build()")
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.csr_spmv.argtypes = [C.c_int64, P, P, P, P, P]
        lib.csr_spmv.restype = None
        lib.csr_pcg_jacobi.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_double, C.c_int32,
                                       C.POINTER(C.c_double)]
        lib.csr_pcg_jacobi.restype = C.c_int32
        lib.csr_max_threads.restype = C.c_int32
        _lib = lib
    return _lib


def _csr_arrays(A):
    A = A.tocsr()
    return (np.ascontiguousarray(A.indptr, dtype=np.int64),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class HostCSR:
    """A CSR matrix prepared once for repeated host products and solves."""

    def __init__(self, A):
        self.n = A.shape[0]
        self.indptr, self.indices, self.data = _csr_arrays(A)

    def matvec(self, x, y=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n) if y is None else y
        _load().csr_spmv(self.n, _p(self.indptr), _p(self.indices), _p(self.data), _p(x), _p(y))
        return y

    def pcg_jacobi(self, b, diag, tol=1e-8, maxit=20000):
        b = np.ascontiguousarray(b, dtype=np.float64)
        diag = np.ascontiguousarray(diag, dtype=np.float64)
        x = np.empty(self.n)
        rel = C.c_double()
        its = _load().csr_pcg_jacobi(self.n, _p(self.indptr), _p(self.indices), _p(self.data),
                                     _p(diag), _p(b), _p(x), tol, maxit, C.byref(rel))
        return x, int(its), float(rel.value)


def threads():
    return int(_load().csr_max_threads())
