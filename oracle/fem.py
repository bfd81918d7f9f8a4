"""ctypes front end of the oracle's C element loops (test infrastructure only).

Sec. II, eq. (1)-(2): P1 semi-discretisation M dx/dt + K(x)x = b; Sec. III:
K(x)x is formed element by element without assembling K(x).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import scipy.sparse as sp

from . import build as _build

EPS0 = 8.8541878128e-12  # vacuum permittivity, F/m (CODATA 2018)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64 = C.c_int64
        L.orc_element_matrix.argtypes = [P, P, P]
        L.orc_element_matrix.restype = C.c_int
        L.orc_first_flat_tet.argtypes = [P, i64, P]
        L.orc_first_flat_tet.restype = i64
        L.orc_assemble.argtypes = [i64, P, i64, P, P, i64, P, P, P]
        L.orc_assemble.restype = i64
        L.orc_apply_K.argtypes = [i64, P, i64, P, P, P, P, P, P, P, P, P, P]
        L.orc_apply_K.restype = C.c_int
        L.orc_element_kappa.argtypes = [P, i64, P, P, P, P, P, P, P, P]
        L.orc_element_kappa.restype = C.c_int
        L.orc_p2_element_matrix.argtypes = [P, P, P]
        L.orc_p2_element_matrix.restype = C.c_int
        L.orc_p2_assemble.argtypes = [i64, P, i64, P, P, i64, P, P, P]
        L.orc_p2_assemble.restype = i64
        L.orc_p2_apply_K.argtypes = [i64, P, i64, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_p2_apply_K.restype = C.c_int
        L.orc_csr_matvec.argtypes = [i64, P, P, P, P, P]
        L.orc_csr_matvec.restype = None
        L.orc_pcg_sgs.argtypes = [i64, P, P, P, P, P, C.c_double, C.c_int32, P, P]
        L.orc_pcg_sgs.restype = C.c_int
        L.orc_pcg_jacobi.argtypes = [i64, P, P, P, P, P, C.c_double, C.c_int32, C.c_int32, P, P]
        L.orc_pcg_jacobi.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def element_matrix(p):
    """Unit-coefficient P1 element matrix A_e (4x4) and volume of the tet p (4x3)."""
    p = _f64(p).reshape(4, 3)
    A = np.zeros(16)
    vol = np.zeros(1)
    if lib().orc_element_matrix(_p(p), _p(A), _p(vol)) != 0:
        raise ValueError("flat tetrahedron")
    return A.reshape(4, 4), float(vol[0])


def element_matrix_p2(p):
    """Unit-coefficient second-order (10-node) element matrix and volume of the
    tet with vertices p (4x3); nodes: vertices, then edge midpoints."""
    p = _f64(p).reshape(4, 3)
    A = np.zeros(100)
    vol = np.zeros(1)
    if lib().orc_p2_element_matrix(_p(p), _p(A), _p(vol)) != 0:
        raise ValueError("flat tetrahedron")
    return A.reshape(10, 10), float(vol[0])


def first_flat_tet(xyz, tets) -> int:
    xyz, tets = _f64(xyz), _i32(np.asarray(tets)[:, :4])
    return int(lib().orc_first_flat_tet(_p(xyz), tets.shape[0], _p(tets)))


def is_p2(tets) -> bool:
    """10-node (second-order) tets, else 4-node."""
    return np.asarray(tets).shape[1] == 10


def assemble(xyz, tets, w_tet) -> sp.csr_matrix:
    """Full nodal matrix sum_e w_e A_e (all nodes, sorted CSR); 4- or 10-node tets."""
    if is_p2(tets):
        return assemble_p2_points(xyz, tets, np.repeat(_f64(w_tet), 4))
    xyz, tets, w = _f64(xyz), _i32(tets), _f64(w_tet)
    n = xyz.shape[0]
    L = lib()
    nnz = L.orc_assemble(n, _p(xyz), tets.shape[0], _p(tets), _p(w), 0, None, None, None)
    if nnz < 0:
        raise ValueError("assembly failed (%d)" % nnz)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float64)
    got = L.orc_assemble(n, _p(xyz), tets.shape[0], _p(tets), _p(w), nnz, _p(rowptr), _p(col), _p(val))
    if got != nnz:
        raise ValueError("assembly failed (%d)" % got)
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


def assemble_p2_points(xyz, tets, w_q) -> sp.csr_matrix:
    """sum_e sum_q w_q (|T_e|/4) grad N_i . grad N_j over 10-node tets, with a
    weight per element and quadrature point (w_q: n_tets x 4)."""
    xyz, tets, w = _f64(xyz), _i32(tets), _f64(w_q).reshape(-1)
    n = xyz.shape[0]
    L = lib()
    nnz = L.orc_p2_assemble(n, _p(xyz), tets.shape[0], _p(tets), _p(w), 0, None, None, None)
    if nnz < 0:
        raise ValueError("assembly failed (%d)" % nnz)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float64)
    got = L.orc_p2_assemble(n, _p(xyz), tets.shape[0], _p(tets), _p(w), nnz, _p(rowptr), _p(col), _p(val))
    if got != nnz:
        raise ValueError("assembly failed (%d)" % got)
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


def _mat_arrays(case):
    return (
        _f64(case.eps_r),
        _f64(case.kappa0),
        _f64(case.e_s),
        _f64(case.alpha),
        _i32(case.nonlinear),
    )


def apply_K(case, x, with_rate: bool = False):
    """y = K(x)x over all nodes (element loop). Optionally max_e sigma_e/eps_e
    (10-node tets: over the quadrature points)."""
    xyz, tets, tm = _f64(case.xyz), _i32(case.tets), _i32(case.tet_mat)
    eps, k0, es, al, nl = _mat_arrays(case)
    x = _f64(x)
    y = np.zeros_like(x)
    rate = np.zeros(1)
    if is_p2(tets):
        rc = lib().orc_p2_apply_K(xyz.shape[0], _p(xyz), tets.shape[0], _p(tets), _p(tm), _p(eps), _p(k0), _p(es),
                                  _p(al), _p(nl), _p(x), _p(y), None, _p(rate) if with_rate else None)
        if rc != 0:
            raise ValueError("flat tetrahedron")
        return (y, float(rate[0])) if with_rate else y
    rc = lib().orc_apply_K(
        xyz.shape[0], _p(xyz), tets.shape[0], _p(tets), _p(tm), _p(eps), _p(k0), _p(es), _p(al), _p(nl),
        _p(x), _p(y), _p(rate) if with_rate else None,
    )
    if rc != 0:
        raise ValueError("flat tetrahedron")
    return (y, float(rate[0])) if with_rate else y


def element_kappa(case, x):
    """Per-element conductivity kappa_e(|E_e(x)|) (10-node tets: n_tets x 4,
    one per quadrature point)."""
    xyz, tets, tm = _f64(case.xyz), _i32(case.tets), _i32(case.tet_mat)
    _, k0, es, al, nl = _mat_arrays(case)
    x = _f64(x)
    if is_p2(tets):
        eps = _f64(case.eps_r)
        kq = np.zeros(tets.shape[0] * 4)
        if lib().orc_p2_apply_K(xyz.shape[0], _p(xyz), tets.shape[0], _p(tets), _p(tm), _p(eps), _p(k0), _p(es),
                                _p(al), _p(nl), _p(x), None, _p(kq), None):
            raise ValueError("flat tetrahedron")
        return kq.reshape(-1, 4)
    out = np.zeros(tets.shape[0])
    if lib().orc_element_kappa(_p(xyz), tets.shape[0], _p(tets), _p(tm), _p(k0), _p(es), _p(al), _p(nl), _p(x), _p(out)):
        raise ValueError("flat tetrahedron")
    return out


def assemble_M(case) -> sp.csr_matrix:
    """Permittivity matrix M = sum_e eps0 eps_r,e A_e over all nodes (eq. (2))."""
    return assemble(case.xyz, case.tets, EPS0 * np.asarray(case.eps_r)[case.tet_mat])


def assemble_K_frozen(case, x) -> sp.csr_matrix:
    """Frozen conductivity matrix K(x) = sum_e kappa_e(x) A_e (for checks only;
    10-node tets: kappa at each quadrature point)."""
    if is_p2(case.tets):
        return assemble_p2_points(case.xyz, case.tets, element_kappa(case, x))
    return assemble(case.xyz, case.tets, element_kappa(case, x))


def csr_matvec(A: sp.csr_matrix, x):
    A = A.tocsr()
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = _i32(A.indices)
    val = _f64(A.data)
    x = _f64(x)
    y = np.zeros(A.shape[0])
    lib().orc_csr_matvec(A.shape[0], _p(rowptr), _p(col), _p(val), _p(x), _p(y))
    return y


class PcgResult:
    def __init__(self, x, iters, relres, status):
        self.x, self.iters, self.relres, self.status = x, iters, relres, status


def pcg_sgs(A: sp.csr_matrix, rhs, x0=None, rtol=1e-13, maxit=100000) -> PcgResult:
    """SGS-preconditioned CG to a true relative residual rtol."""
    A = A.tocsr()
    n = A.shape[0]
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = _i32(A.indices)
    val = _f64(A.data)
    rhs = _f64(rhs)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    it = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1)
    st = lib().orc_pcg_sgs(n, _p(rowptr), _p(col), _p(val), _p(rhs), _p(x), rtol, maxit, _p(it), _p(rr))
    return PcgResult(x, int(it[0]), float(rr[0]), int(st))


def default_threads() -> int:
    """Threads for the Jacobi-PCG reference solver: OMP_NUM_THREADS if set,
    else the CPUs this process may run on."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    if v.isdigit() and int(v) > 0:
        return int(v)
    return max(1, len(os.sched_getaffinity(0)))


def pcg_jacobi(A: sp.csr_matrix, rhs, x0=None, rtol=1e-13, maxit=1000000, threads=None) -> PcgResult:
    """Jacobi-preconditioned CG to a true relative residual rtol (same CG loop
    as pcg_sgs; row loops on ``threads`` OpenMP threads)."""
    A = A.tocsr()
    n = A.shape[0]
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = _i32(A.indices)
    val = _f64(A.data)
    rhs = _f64(rhs)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    it = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1)
    nt = default_threads() if threads is None else int(threads)
    st = lib().orc_pcg_jacobi(n, _p(rowptr), _p(col), _p(val), _p(rhs), _p(x), rtol, maxit, nt, _p(it), _p(rr))
    return PcgResult(x, int(it[0]), float(rr[0]), int(st))
