"""CPU oracle for the P1 system (rho*K + M) u = f of eq. (5) -- TEST INFRASTRUCTURE.

This package is the plain, slow, double-precision reference against which the
GPU library is checked.  Only the test suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does, and it imports nothing from the product package.  Its only shared
dependency with the GPU side is ``ocp_inputs`` (seeded meshes and target
descriptors, no method arithmetic).

Contents
  * ``oracle.c``  (this package's C part, built with gcc + OpenMP):
    element matrices and load by the 4-point rule, row-by-row assembly of
    A = rho*K + M and f on the interior vertices (Section 2, system (linsys)),
    sampled rows, CSR SpMV and Jacobi-PCG from x0 = 0.
  * ``dense.py``: numpy element-by-element dense assembly and a Cholesky solve
    for tiny meshes.
  * ``norms.py``: L2 / H1 errors against the closed-form solutions of
    Section 4.1 and its sine-mode superpositions.
  * ``amg.py``: the smoothed-aggregation hierarchy written out from its
    definitions (aggregation, tentative and smoothed prolongators, Galerkin
    coarse operators) for the parity checks of the GPU setup.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Target(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_modes", C.c_int),
                ("k", C.POINTER(C.c_int32)), ("amp", C.POINTER(C.c_double)),
                ("offset", C.c_double), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("nodal", C.POINTER(C.c_double))]


class _System(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double)), ("valK", C.POINTER(C.c_double)),
                ("valM", C.POINTER(C.c_double)), ("f", C.POINTER(C.c_double)),
                ("dof_of_vertex", C.POINTER(C.c_int32)),
                ("vertex_of_dof", C.POINTER(C.c_int32))]


_lib_handle = None


def lib():
    global _lib_handle
    if _lib_handle is None:
        build(force=False)
        L = C.CDLL(_SO)
        dp, ip, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.orc_assemble.argtypes = [C.c_int64, dp, C.c_int64, ip, C.POINTER(C.c_uint8),
                                   C.c_double, C.POINTER(_Target), C.c_int, C.POINTER(_System)]
        L.orc_assemble.restype = C.c_int
        L.orc_free.argtypes = [C.POINTER(_System)]
        L.orc_sample_rows.argtypes = [C.c_int64, dp, C.c_int64, ip, C.POINTER(C.c_uint8),
                                      C.c_double, C.POINTER(_Target), C.c_int64, ip, C.c_int,
                                      ip, dp, ip, dp]
        L.orc_sample_rows.restype = C.c_int
        L.orc_spmv.argtypes = [C.c_int64, i64p, ip, dp, dp, dp]
        L.orc_pcg.argtypes = [C.c_int64, i64p, ip, dp, dp, dp, C.c_double, C.c_int, dp]
        L.orc_pcg.restype = C.c_int
        L.orc_element.argtypes = [dp, ip, C.POINTER(_Target), dp, dp, dp, dp]
        L.orc_element.restype = C.c_int
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        _lib_handle = L
    return _lib_handle


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _target_struct(target, keep):
    t = _Target()
    kind = target.kind
    if kind == "sine":
        k = np.ascontiguousarray(target.k, dtype=np.int32)
        amp = np.ascontiguousarray(target.amp, dtype=np.float64)
        keep += [k, amp]
        t.kind = 0
        t.n_modes = int(k.shape[0])
        t.k = _ptr(k, C.c_int32)
        t.amp = _ptr(amp, C.c_double)
        t.offset = float(target.offset)
    elif kind == "box":
        t.kind = 1
        for d in range(3):
            t.lo[d] = float(target.lo[d])
            t.hi[d] = float(target.hi[d])
    elif kind == "nodal":
        v = np.ascontiguousarray(target.values, dtype=np.float64)
        keep.append(v)
        t.kind = 2
        t.nodal = _ptr(v, C.c_double)
    else:
        raise ValueError(kind)
    return t


@dataclass
class System:
    """Assembled interior system: CSR (sorted columns), load, dof maps."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    f: np.ndarray
    dof_of_vertex: np.ndarray
    vertex_of_dof: np.ndarray
    valK: Optional[np.ndarray] = None
    valM: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def csr(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def assemble(mesh, rho: float, target, keep_km: bool = False) -> System:
    """A = rho*K + M and f = (int ubar phi_i) on the interior vertices."""
    L = lib()
    keep = []
    t = _target_struct(target, keep)
    xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
    tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
    mask = np.ascontiguousarray(mesh.dirichlet, dtype=np.uint8)
    s = _System()
    rc = L.orc_assemble(xyz.shape[0], _ptr(xyz, C.c_double), tets.shape[0],
                        _ptr(tets, C.c_int32), _ptr(mask, C.c_uint8), float(rho),
                        C.byref(t), int(keep_km), C.byref(s))
    if rc != 0:
        raise RuntimeError(f"oracle assembly failed ({rc})")
    n, nnz = int(s.n), int(s.nnz)
    nv = xyz.shape[0]

    def arr(p, cnt, dt):
        if cnt == 0:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(p, shape=(cnt,)).astype(dt, copy=True)

    out = System(n=n, row_ptr=arr(s.row_ptr, n + 1, np.int64), col=arr(s.col, nnz, np.int32),
                 val=arr(s.val, nnz, np.float64), f=arr(s.f, n, np.float64),
                 dof_of_vertex=arr(s.dof_of_vertex, nv, np.int32),
                 vertex_of_dof=arr(s.vertex_of_dof, n, np.int32),
                 valK=arr(s.valK, nnz, np.float64) if keep_km else None,
                 valM=arr(s.valM, nnz, np.float64) if keep_km else None)
    L.orc_free(C.byref(s))
    return out


def sample_rows(mesh, rho: float, target, vertices, cap: int = 64):
    """Rows of A and entries of f for the given interior vertex ids.

    Returns (cols [ns, cap] int32 dof ids, vals [ns, cap], counts [ns], f [ns]).
    """
    L = lib()
    keep = []
    t = _target_struct(target, keep)
    xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
    tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
    mask = np.ascontiguousarray(mesh.dirichlet, dtype=np.uint8)
    rows = np.ascontiguousarray(vertices, dtype=np.int32)
    ns = rows.size
    cols = np.full((ns, cap), -1, dtype=np.int32)
    vals = np.zeros((ns, cap), dtype=np.float64)
    cnt = np.zeros(ns, dtype=np.int32)
    f = np.zeros(ns, dtype=np.float64)
    rc = L.orc_sample_rows(xyz.shape[0], _ptr(xyz, C.c_double), tets.shape[0],
                           _ptr(tets, C.c_int32), _ptr(mask, C.c_uint8), float(rho),
                           C.byref(t), ns, _ptr(rows, C.c_int32), cap,
                           _ptr(cols, C.c_int32), _ptr(vals, C.c_double),
                           _ptr(cnt, C.c_int32), _ptr(f, C.c_double))
    if rc != 0:
        raise RuntimeError(f"oracle row sampling failed ({rc})")
    return cols, vals, cnt, f


def spmv(sys: System, x: np.ndarray) -> np.ndarray:
    L = lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(sys.n, dtype=np.float64)
    L.orc_spmv(sys.n, _ptr(sys.row_ptr, C.c_int64), _ptr(sys.col, C.c_int32),
               _ptr(sys.val, C.c_double), _ptr(x, C.c_double), _ptr(y, C.c_double))
    return y


def pcg(sys: System, f: Optional[np.ndarray] = None, rtol: float = 1e-14, maxit: int = 100000):
    """Jacobi-PCG from x0 = 0; returns (x, iterations, relative residual)."""
    L = lib()
    f = sys.f if f is None else np.ascontiguousarray(f, dtype=np.float64)
    x = np.zeros(sys.n, dtype=np.float64)
    rr = C.c_double(0.0)
    it = L.orc_pcg(sys.n, _ptr(sys.row_ptr, C.c_int64), _ptr(sys.col, C.c_int32),
                   _ptr(sys.val, C.c_double), _ptr(f, C.c_double), _ptr(x, C.c_double),
                   float(rtol), int(maxit), C.byref(rr))
    return x, int(it), float(rr.value)


def element(pts: np.ndarray, target):
    """(Ke, Me, fe, vol) of one tetrahedron with vertices pts[4,3]."""
    L = lib()
    keep = []
    t = _target_struct(target, keep)
    xyz = np.ascontiguousarray(pts, dtype=np.float64).reshape(4, 3)
    tv = np.arange(4, dtype=np.int32)
    Ke = np.zeros(16)
    Me = np.zeros(16)
    fe = np.zeros(4)
    vol = C.c_double(0.0)
    rc = L.orc_element(_ptr(xyz, C.c_double), _ptr(tv, C.c_int32), C.byref(t),
                       _ptr(Ke, C.c_double), _ptr(Me, C.c_double), _ptr(fe, C.c_double),
                       C.byref(vol))
    if rc != 0:
        raise RuntimeError("degenerate element")
    return Ke.reshape(4, 4), Me.reshape(4, 4), fe, float(vol.value)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


def solve(mesh, rho: float, target, rtol: float = 1e-14, maxit: int = 100000):
    """Discrete solution u = A^{-1} f on the interior, plus the system."""
    sys = assemble(mesh, rho, target)
    x, it, rr = pcg(sys, rtol=rtol, maxit=maxit)
    return x, sys, it, rr


def to_vertices(sys: System, u_interior: np.ndarray, n_vertices: int) -> np.ndarray:
    """Scatter interior coefficients to all vertices (0 on Gamma)."""
    out = np.zeros(n_vertices, dtype=np.float64)
    out[sys.vertex_of_dof] = u_interior
    return out
