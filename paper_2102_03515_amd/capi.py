"""ctypes binding of libocpamg.so -- argument marshalling only.

Every computation runs in the HIP library; this module converts torch tensors
and target descriptors to the C structures of ``include/ocpamg.h`` and back.
PyTorch supplies device memory (through the library's allocator callbacks)
and the stream.  There is no CPU fallback: if the library is missing, every
call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libocpamg.so")

OK, MAXIT = 0, 1
ERR_INVALID_ARG, ERR_BAD_MESH, ERR_OOM, ERR_BREAKDOWN, ERR_HIP, ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6
KEEP_KM = 1
NO_LOAD = 2
PREC_FP64, PREC_MIXED = 0, 1
SMOOTH_L1JACOBI, SMOOTH_CHEBYSHEV = 0, 1
AMG_AGGREGATION, AMG_REDBLACK = 0, 1
STOP_L2, STOP_PRECOND = 0, 1
FLEXIBLE = 2
TARGET_SINE, TARGET_BOX, TARGET_NODAL = 0, 1, 2


class OcpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ocpamg error {code}: {msg}")
        self.code = code


# --------------------------------------------------------------- structures
class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_tets", C.c_int32), ("xyz", C.c_void_p),
                ("tets", C.c_void_p), ("dirichlet", C.c_void_p)]


class _Target(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_modes", C.c_int32), ("k", C.POINTER(C.c_int32)),
                ("amp", C.POINTER(C.c_double)), ("offset", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("nodal", C.c_void_p)]


class _SystemView(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_dofs", C.c_int32), ("nnz", C.c_int64),
                ("rho", C.c_double), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("f", C.c_void_p), ("dof_of_vertex", C.c_void_p),
                ("vertex_of_dof", C.c_void_p), ("sell_coded", C.c_int32), ("sell_entries", C.c_int64)]


class _AmgParams(C.Structure):
    _fields_ = [("precision", C.c_int32), ("smoother", C.c_int32), ("degree", C.c_int32),
                ("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("theta", C.c_double),
                ("omega", C.c_double), ("cheb_ratio", C.c_double), ("method", C.c_int32)]


class _LevelView(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level", C.c_int32), ("n", C.c_int32),
                ("n_coarse", C.c_int32), ("nnz_A", C.c_int64), ("nnz_P", C.c_int64),
                ("A_row_ptr", C.c_void_p), ("A_col", C.c_void_p), ("A_val", C.c_void_p),
                ("P_row_ptr", C.c_void_p), ("P_col", C.c_void_p), ("P_val", C.c_void_p),
                ("R_row_ptr", C.c_void_p), ("R_col", C.c_void_p), ("R_val", C.c_void_p),
                ("agg", C.c_void_p), ("dense_inv", C.c_void_p), ("lambda_max", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("rel_res_l2", C.c_double),
                ("rel_res_precond", C.c_double), ("true_rel_res", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

# every exported entry point and its ctypes signature
_SIGS = {
    "ocp_version": (C.c_char_p, []),
    "ocp_ctx_create": (C.c_int, [C.c_void_p, ALLOC_FN, FREE_FN, C.c_void_p, C.POINTER(C.c_void_p)]),
    "ocp_ctx_destroy": (None, [C.c_void_p]),
    "ocp_last_error": (C.c_char_p, [C.c_void_p]),
    "fe_assemble": (C.c_int, [C.c_void_p, C.POINTER(_Mesh), C.c_double, C.POINTER(_Target), C.c_int32,
                              C.POINTER(C.c_void_p)]),
    "ocp_system_destroy": (None, [C.c_void_p]),
    "fe_set_rho": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double]),
    "fe_derive": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_void_p)]),
    "fe_load": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(_Target), C.c_void_p]),
    "fe_load_multi": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(_Target), C.c_void_p]),
    "ocp_system_get_view": (C.c_int, [C.c_void_p, C.POINTER(_SystemView)]),
    "ocp_spmv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "amg_default_params": (None, [C.POINTER(_AmgParams)]),
    "amg_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(_AmgParams), C.POINTER(C.c_void_p)]),
    "ocp_hierarchy_destroy": (None, [C.c_void_p]),
    "ocp_hierarchy_get_level": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(_LevelView)]),
    "amg_vcycle": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pcg_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                            C.c_int32, C.c_int32, C.POINTER(SolveInfo)]),
    "pcg_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_int32, C.c_int32, C.POINTER(SolveInfo)]),
    "pcg_solve_multi": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_double, C.c_int32, C.c_int32, C.POINTER(SolveInfo)]),
    "pcg_solve_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_double, C.c_int32, C.c_int32,
                                  C.POINTER(SolveInfo)]),
    "pcg_begin": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                            C.POINTER(C.c_void_p)]),
    "pcg_advance": (C.c_int, [C.c_void_p, C.c_int32]),
    "pcg_poll": (C.c_int, [C.c_void_p, C.POINTER(SolveInfo)]),
    "pcg_end": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SolveInfo)]),
    "fe_recover": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(_Target), C.c_void_p, C.c_void_p, C.c_void_p]),
    "fe_error_norms": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(_Target), C.c_void_p,
                                 C.POINTER(C.c_double)]),
    "fe_error_indicator": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(_Target), C.c_void_p, C.c_void_p]),
    "ocp_refiner_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "ocp_refiner_destroy": (None, [C.c_void_p]),
    "ocp_refiner_refine": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_int32)]),
    "ocp_refiner_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ocp_refiner_get": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ocp_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "ocp_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
}

(KERNEL_CG_SPMV, KERNEL_VC_PRE0, KERNEL_VC_POST0, KERNEL_VC_RESTRICT0, KERNEL_VC_PROLONG0, KERNEL_VC_PRE0_B,
 KERNEL_VC_POST0_A, KERNEL_BLK_SPMM) = range(8)

_lib = None


def lib():
    """Load libocpamg.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


# ---------------------------------------------------------------- helpers
def _torch():
    import torch
    return torch


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _torch()  # the HIP runtime is loaded with torch
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipDeviceSynchronize.restype = C.c_int
    return _hip


_DT = {"i4": ("int32", 4), "f8": ("float64", 8), "f4": ("float32", 4), "u1": ("uint8", 1)}


def device_view(ptr: int, shape, dtype: str):
    """A torch tensor holding a copy of library-owned device memory."""
    torch = _torch()
    shape = (int(shape),) if np.isscalar(shape) else tuple(int(s) for s in shape)
    name, size = _DT[dtype]
    out = torch.zeros(shape, dtype=getattr(torch, name), device="cuda")
    nbytes = int(np.prod(shape)) * size
    if ptr and nbytes:
        hip = _hip_runtime()
        if hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("hipDeviceSynchronize failed")
        rc = hip.hipMemcpy(C.c_void_p(out.data_ptr()), C.c_void_p(int(ptr)), nbytes, 4)  # hipMemcpyDefault
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


# ---------------------------------------------------------------- context
class Context:
    """Library context bound to a torch stream and torch's caching allocator."""

    def __init__(self, stream=None, torch_allocator: bool = True, on_alloc=None):
        """on_alloc: optional callable(nbytes) run on every device allocation
        the library requests through this context (tests count them)."""
        torch = _torch()
        L = lib()
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        sp = int(self.stream.cuda_stream)
        if torch_allocator:
            dev, st = self.device, self.stream

            def _alloc(nbytes, user):
                if on_alloc is not None:
                    on_alloc(int(nbytes))
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
                except Exception:
                    return None

            def _free(ptr, user):
                try:
                    torch.cuda.caching_allocator_delete(int(ptr))
                except Exception:
                    pass

            self._alloc = ALLOC_FN(_alloc)
            self._free = FREE_FN(_free)
        else:
            self._alloc = ALLOC_FN()
            self._free = FREE_FN()
        h = C.c_void_p()
        rc = L.ocp_ctx_create(C.c_void_p(sp), self._alloc, self._free, None, C.byref(h))
        if rc != OK:
            raise OcpError(rc, "context creation failed")
        self.handle = h

    def last_error(self) -> str:
        return lib().ocp_last_error(self.handle).decode()

    def check(self, rc: int, ok=(OK,)):
        if rc not in ok:
            raise OcpError(rc, self.last_error())
        return rc

    def profile(self, on: bool = True):
        self.check(lib().ocp_profile_enable(self.handle, int(bool(on))))

    def kernel_timing(self, kernel: int):
        """(launches, total milliseconds) of a profiled kernel."""
        n = C.c_int64()
        ms = C.c_double()
        self.check(lib().ocp_profile_read(self.handle, int(kernel), C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().ocp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------- mesh
@dataclass
class DeviceMesh:
    xyz: object        # torch float64 [nv,3] on the GPU
    tets: object       # torch int32 [nt,4]
    dirichlet: object  # torch uint8 [nv]

    @property
    def n_vertices(self):
        return int(self.xyz.shape[0])

    @property
    def n_tets(self):
        return int(self.tets.shape[0])

    def struct(self) -> _Mesh:
        return _Mesh(self.n_vertices, self.n_tets, _ptr(self.xyz), _ptr(self.tets), _ptr(self.dirichlet))


def upload_mesh(mesh) -> DeviceMesh:
    """Copy an ``ocp_inputs.Mesh`` to the GPU."""
    torch = _torch()
    return DeviceMesh(xyz=torch.from_numpy(np.ascontiguousarray(mesh.xyz)).cuda(),
                      tets=torch.from_numpy(np.ascontiguousarray(mesh.tets, dtype=np.int32)).cuda(),
                      dirichlet=torch.from_numpy(np.ascontiguousarray(mesh.dirichlet, dtype=np.uint8)).cuda())


def target_struct(target, keep: list) -> _Target:
    t = _Target()
    if target.kind == "sine":
        k = np.ascontiguousarray(target.k, dtype=np.int32)
        a = np.ascontiguousarray(target.amp, dtype=np.float64)
        keep += [k, a]
        t.kind = TARGET_SINE
        t.n_modes = int(k.shape[0])
        t.k = k.ctypes.data_as(C.POINTER(C.c_int32))
        t.amp = a.ctypes.data_as(C.POINTER(C.c_double))
        t.offset = float(target.offset)
    elif target.kind == "box":
        t.kind = TARGET_BOX
        for d in range(3):
            t.lo[d] = float(target.lo[d])
            t.hi[d] = float(target.hi[d])
    elif target.kind == "nodal":
        torch = _torch()
        v = target.values
        if not (hasattr(v, "is_cuda") and v.is_cuda):
            v = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
        keep.append(v)
        t.kind = TARGET_NODAL
        t.nodal = _ptr(v)
    else:
        raise ValueError(f"unknown target kind {target.kind!r}")
    return t


# ----------------------------------------------------------------- system
class System:
    def __init__(self, ctx: Context, handle, mesh: DeviceMesh):
        self.ctx = ctx
        self.handle = handle
        self.mesh = mesh   # keeps the device mesh alive (the system borrows it; fe_load reads it)

    def view(self) -> _SystemView:
        v = _SystemView()
        self.ctx.check(lib().ocp_system_get_view(self.handle, C.byref(v)))
        return v

    @property
    def n(self) -> int:
        return int(self.view().n_dofs)

    @property
    def nnz(self) -> int:
        return int(self.view().nnz)

    @property
    def sell_coded(self) -> bool:
        """True when the solve-phase sliced-ELL matrix reads 4-bit column codes."""
        return bool(self.view().sell_coded)

    @property
    def sell_entries(self) -> int:
        """Stored entries of the solve-phase sliced-ELL matrix (slices padded)."""
        return int(self.view().sell_entries)

    def csr(self):
        """(row_ptr, col, val) as torch tensors viewing the library's arrays."""
        v = self.view()
        return (device_view(v.row_ptr, (v.n_dofs + 1,), "i4"), device_view(v.col, (v.nnz,), "i4"),
                device_view(v.val, (v.nnz,), "f8"))

    def f(self):
        v = self.view()
        return device_view(v.f, (v.n_dofs,), "f8")

    def dof_of_vertex(self):
        v = self.view()
        return device_view(v.dof_of_vertex, (v.n_vertices,), "i4")

    def vertex_of_dof(self):
        v = self.view()
        return device_view(v.vertex_of_dof, (v.n_dofs,), "i4")

    def spmv(self, x, y=None):
        torch = _torch()
        if y is None:
            y = torch.empty_like(x)
        self.ctx.check(lib().ocp_spmv(self.ctx.handle, self.handle, _ptr(x), _ptr(y)))
        return y

    def set_rho(self, rho: float):
        self.ctx.check(lib().fe_set_rho(self.ctx.handle, self.handle, float(rho)))

    def load(self, target, out=None, ctx: Optional["Context"] = None):
        """Load vector of a target; runs on `ctx` (default: the creating
        context)."""
        torch = _torch()
        ctx = ctx or self.ctx
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        keep = []
        t = target_struct(target, keep)
        ctx.check(lib().fe_load(ctx.handle, self.handle, C.byref(t), _ptr(out)))
        return out

    def load_multi(self, targets, out=None, ctx: Optional["Context"] = None):
        """Load vectors of several targets as one row-major block [n][k];
        runs on `ctx` (default: the creating context)."""
        torch = _torch()
        ctx = ctx or self.ctx
        k = len(targets)
        if out is None:
            out = torch.empty((self.n, k), dtype=torch.float64, device="cuda")
        keep = []
        arr = (_Target * k)(*[target_struct(t, keep) for t in targets])
        ctx.check(lib().fe_load_multi(ctx.handle, self.handle, k, arr, _ptr(out)))
        return out

    def recover(self, target, u, ctx: Optional["Context"] = None):
        """(p, z) on all vertices: adjoint -rho u and control (ubar - u)/rho
        from the state u (device [n_vertices])."""
        torch = _torch()
        ctx = ctx or self.ctx
        nv = self.view().n_vertices
        p = torch.empty(nv, dtype=torch.float64, device="cuda")
        z = torch.empty(nv, dtype=torch.float64, device="cuda")
        keep = []
        t = target_struct(target, keep)
        ctx.check(lib().fe_recover(ctx.handle, self.handle, C.byref(t), _ptr(u), _ptr(p), _ptr(z)))
        return p, z

    def error_indicator(self, target, u, ctx: Optional["Context"] = None):
        """Squared residual error indicator per tetrahedron (torch, device)."""
        torch = _torch()
        ctx = ctx or self.ctx
        nt = self.mesh.n_tets
        eta2 = torch.empty(nt, dtype=torch.float64, device="cuda")
        keep = []
        t = target_struct(target, keep)
        ctx.check(lib().fe_error_indicator(ctx.handle, self.handle, C.byref(t), _ptr(u), _ptr(eta2)))
        return eta2

    def error_norms(self, target, u, ctx: Optional["Context"] = None):
        """(||u_rho - u||_L2, ||grad(u_rho - u)||_L2, ||ubar - u||_L2); the
        first two are NaN for targets without a closed-form solution."""
        ctx = ctx or self.ctx
        keep = []
        t = target_struct(target, keep)
        out = (C.c_double * 3)()
        ctx.check(lib().fe_error_norms(ctx.handle, self.handle, C.byref(t), _ptr(u), out))
        return float(out[0]), float(out[1]), float(out[2])

    def close(self):
        if getattr(self, "handle", None):
            lib().ocp_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Refiner:
    """Host mesh under bisection refinement (ocp_refiner_*)."""

    def __init__(self, xyz, tets):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        h = C.c_void_p()
        rc = lib().ocp_refiner_create(xyz.ctypes.data, int(xyz.shape[0]), tets.ctypes.data, int(tets.shape[0]),
                                      C.byref(h))
        if rc != OK:
            raise OcpError(rc, "refiner creation failed")
        self.handle = h

    def refine(self, eta2, theta: float = 0.5) -> int:
        """Doerfler-mark by the squared indicators (host, one per tetrahedron)
        and bisect; returns the number marked."""
        e = np.ascontiguousarray(eta2, dtype=np.float64)
        m = C.c_int32()
        rc = lib().ocp_refiner_refine(self.handle, e.ctypes.data, float(theta), C.byref(m))
        if rc != OK:
            raise OcpError(rc, "refinement failed")
        return int(m.value)

    def get(self):
        """(xyz [nv,3], tets [nt,4], dirichlet [nv]) of the current mesh."""
        nv, nt = C.c_int32(), C.c_int32()
        rc = lib().ocp_refiner_sizes(self.handle, C.byref(nv), C.byref(nt))
        if rc != OK:
            raise OcpError(rc, "refiner sizes")
        xyz = np.empty((nv.value, 3), dtype=np.float64)
        tets = np.empty((nt.value, 4), dtype=np.int32)
        d = np.empty(nv.value, dtype=np.uint8)
        rc = lib().ocp_refiner_get(self.handle, xyz.ctypes.data, tets.ctypes.data, d.ctypes.data)
        if rc != OK:
            raise OcpError(rc, "refiner get")
        return xyz, tets, d

    def close(self):
        if getattr(self, "handle", None):
            lib().ocp_refiner_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fe_assemble(ctx: Context, mesh: DeviceMesh, rho: float, target, flags: int = 0) -> System:
    """A = rho K + M and f on the mesh; with NO_LOAD in flags, A only (f zero,
    target may be None)."""
    keep = []
    t = C.byref(target_struct(target, keep)) if target is not None else None
    m = mesh.struct()
    h = C.c_void_p()
    ctx.check(lib().fe_assemble(ctx.handle, C.byref(m), float(rho), t, int(flags), C.byref(h)))
    return System(ctx, h, mesh)


def fe_derive(ctx: Context, base: System, rho: float) -> System:
    """System with A = rho*K + M from base's stored K and M (base assembled
    with KEEP_KM); pattern, maps and f are copied."""
    h = C.c_void_p()
    ctx.check(lib().fe_derive(ctx.handle, base.handle, float(rho), C.byref(h)))
    return System(ctx, h, base.mesh)


# -------------------------------------------------------------- hierarchy
def default_params() -> _AmgParams:
    p = _AmgParams()
    lib().amg_default_params(C.byref(p))
    return p


class Hierarchy:
    def __init__(self, ctx: Context, handle, system: System, params: _AmgParams):
        self.ctx = ctx
        self.handle = handle
        self.system = system
        self.params = params

    def level(self, l: int) -> _LevelView:
        v = _LevelView()
        self.ctx.check(lib().ocp_hierarchy_get_level(self.handle, int(l), C.byref(v)))
        return v

    @property
    def n_levels(self) -> int:
        return int(self.level(0).n_levels)

    def level_arrays(self, l: int) -> dict:
        v = self.level(l)
        out = {"n": v.n, "nc": v.n_coarse, "lambda_max": v.lambda_max,
               "A": (device_view(v.A_row_ptr, (v.n + 1,), "i4"), device_view(v.A_col, (v.nnz_A,), "i4"),
                     device_view(v.A_val, (v.nnz_A,), "f8"))}
        if v.P_row_ptr:
            out["P"] = (device_view(v.P_row_ptr, (v.n + 1,), "i4"), device_view(v.P_col, (v.nnz_P,), "i4"),
                        device_view(v.P_val, (v.nnz_P,), "f8"))
            out["R"] = (device_view(v.R_row_ptr, (v.n_coarse + 1,), "i4"), device_view(v.R_col, (v.nnz_P,), "i4"),
                        device_view(v.R_val, (v.nnz_P,), "f8"))
            out["agg"] = device_view(v.agg, (v.n,), "i4")
        if v.dense_inv:
            out["dense_inv"] = device_view(v.dense_inv, (v.n, v.n), "f8")
        return out

    def vcycle(self, r, z=None):
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        self.ctx.check(lib().amg_vcycle(self.ctx.handle, self.handle, _ptr(r), _ptr(z)))
        return z

    def close(self):
        if getattr(self, "handle", None):
            lib().ocp_hierarchy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amg_setup(ctx: Context, system: System, precision: int = PREC_FP64, **kw) -> Hierarchy:
    p = default_params()
    p.precision = int(precision)
    for k, v in kw.items():
        setattr(p, k, v)
    h = C.c_void_p()
    ctx.check(lib().amg_setup(ctx.handle, system.handle, C.byref(p), C.byref(h)))
    return Hierarchy(ctx, h, system, p)


# ------------------------------------------------------------------ solve
def pcg_solve(ctx: Context, system: System, hierarchy: Optional[Hierarchy] = None, f=None, u=None,
              rtol: float = 1e-8, maxit: int = 500, stop: int = STOP_L2, raise_on_maxit: bool = False,
              flexible: bool = False):
    """Returns (u on all vertices, SolveInfo, status).  flexible: the
    Polak-Ribiere beta (for an FP32 V-cycle)."""
    torch = _torch()
    nv = system.view().n_vertices
    if u is None:
        u = torch.empty(nv, dtype=torch.float64, device="cuda")
    info = SolveInfo()
    flags = int(stop) | (FLEXIBLE if flexible else 0)
    rc = lib().pcg_solve(ctx.handle, system.handle, hierarchy.handle if hierarchy is not None else None,
                         _ptr(f), _ptr(u), float(rtol), int(maxit), flags, C.byref(info))
    ok = (OK,) if raise_on_maxit else (OK, MAXIT)
    ctx.check(rc, ok=ok)
    return u, info, rc


def pcg_solve_noalloc(ctx: Context, system: System, hierarchy: Optional[Hierarchy] = None, f=None, u=None,
                      rtol: float = 1e-8, maxit: int = 500, stop: int = STOP_L2, flexible: bool = False):
    """pcg_solve with its work memory carved from the library's fixed scratch
    region (no device allocation in the call).  u must be given (or is
    allocated here, before the call).  Returns (u, SolveInfo, status)."""
    torch = _torch()
    nv = system.view().n_vertices
    if u is None:
        u = torch.empty(nv, dtype=torch.float64, device="cuda")
    info = SolveInfo()
    flags = int(stop) | (FLEXIBLE if flexible else 0)
    rc = lib().pcg_solve_noalloc(ctx.handle, system.handle, hierarchy.handle if hierarchy is not None else None,
                                 _ptr(f), _ptr(u), float(rtol), int(maxit), flags, C.byref(info))
    ctx.check(rc, ok=(OK, MAXIT))
    return u, info, rc


def pcg_solve_multi(ctx: Context, system: System, hierarchy: Optional[Hierarchy], F, k: Optional[int] = None,
                    U=None, rtol: float = 1e-8, maxit: int = 500, stop: int = STOP_L2, tile: int = 0):
    """Block PCG over the k columns of F (device [n][k] row-major, or None for
    k copies of the system's f).  tile forces the column-panel width of the
    block kernels (8/16/32/64; 0 = chosen by timing).  Returns
    (U [n_vertices][k], [SolveInfo]*k, status)."""
    torch = _torch()
    if F is not None:
        if F.dim() != 2 or not F.is_contiguous() or F.dtype != torch.float64:
            raise ValueError("F must be a contiguous float64 [n][k] tensor")
        k = F.shape[1]
    if k is None:
        raise ValueError("k is needed when F is None")
    nv = system.view().n_vertices
    if U is None:
        U = torch.empty((nv, k), dtype=torch.float64, device="cuda")
    infos = (SolveInfo * k)()
    rc = lib().pcg_solve_multi(ctx.handle, system.handle, hierarchy.handle if hierarchy is not None else None,
                               int(k), _ptr(F), _ptr(U), float(rtol), int(maxit), int(stop) | (int(tile) << 8),
                               infos)
    ctx.check(rc, ok=(OK, MAXIT))
    return U, list(infos), rc


class SolveHandle:
    """A PCG solve driven in steps (pcg_begin / advance / poll / end)."""

    def __init__(self, ctx: Context, handle, system: System, u):
        self.ctx, self.handle, self.system, self.u = ctx, handle, system, u

    def advance(self, iters: int):
        self.ctx.check(lib().pcg_advance(self.handle, int(iters)))

    def poll(self):
        """(state, SolveInfo): 0 stopped, 1 ready for more iterations, 2 the
        last advance is still running."""
        info = SolveInfo()
        rc = lib().pcg_poll(self.handle, C.byref(info))
        if rc < 0:
            self.ctx.check(rc)
        return rc, info

    def end(self):
        info = SolveInfo()
        rc = lib().pcg_end(self.handle, _ptr(self.u), C.byref(info))
        self.handle = None
        self.ctx.check(rc, ok=(OK, MAXIT))
        return self.u, info, rc


def pcg_begin(ctx: Context, system: System, hierarchy: Optional[Hierarchy] = None, f=None, u=None,
              rtol: float = 1e-8, maxit: int = 500, stop: int = STOP_L2) -> SolveHandle:
    torch = _torch()
    if u is None:
        u = torch.empty(system.view().n_vertices, dtype=torch.float64, device="cuda")
    h = C.c_void_p()
    ctx.check(lib().pcg_begin(ctx.handle, system.handle, hierarchy.handle if hierarchy is not None else None,
                              _ptr(f), float(rtol), int(maxit), int(stop), C.byref(h)))
    return SolveHandle(ctx, h, system, u)


BATCH_GRAPH = 1 << 16


def pcg_solve_batch(ctx: Context, systems, hierarchies=None, fs=None, us=None, rtol: float = 1e-8,
                    maxit: int = 500, stop: int = STOP_L2, graph: bool = False):
    """Many independent solves packed together: small ones in one persistent
    launch (one workgroup per solve), the others (or all, with graph=True)
    in one graph launch per iteration.  Returns ([u_i], [SolveInfo_i],
    worst status)."""
    torch = _torch()
    m = len(systems)
    if us is None:
        us = [torch.empty(s.view().n_vertices, dtype=torch.float64, device="cuda") for s in systems]
    arr = lambda xs: (C.c_void_p * m)(*[None if x is None else C.c_void_p(x) for x in xs])
    sys_a = arr([s.handle.value for s in systems])
    h_a = arr([None if h is None else h.handle.value for h in hierarchies]) if hierarchies is not None else None
    f_a = arr([_ptr(f) for f in fs]) if fs is not None else None
    u_a = arr([_ptr(u) for u in us])
    infos = (SolveInfo * m)()
    flags = int(stop) | (BATCH_GRAPH if graph else 0)
    rc = lib().pcg_solve_batch(ctx.handle, m, sys_a, h_a, f_a, u_a, float(rtol), int(maxit), flags, infos)
    ctx.check(rc, ok=(OK, MAXIT))
    return us, list(infos), rc
