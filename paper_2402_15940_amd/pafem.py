"""Thin ctypes binding of libpafem.so (the C ABI in include/pafem.h).

Argument marshalling only: every step of the operator, diagonal, right-hand
side and solve runs in the library's HIP kernels.  Device vectors are torch
tensors on the GPU (contiguous, float64 or float32); their data pointers and
torch's current HIP stream are handed to the library.  If the library is not
built the first call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAFEM_LIB selects another build of the library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PAFEM_LIB") or os.path.join(_HERE, "libpafem.so")

MASS = 0
DIFFUSION = 1
FP64 = 1
FP32 = 2
BF16 = 4
SCATTER_ATOMIC = 0
SCATTER_DETERMINISTIC = 1
INDEX_LATTICE = 0
INDEX_MAP = 1
APPLY_CONSTRAINED = 1
APPLY_ACCUMULATE = 2
SOLVE_PLAIN_FP64 = 0
SOLVE_IR_FP32 = 1
SOLVE_IR_BF16 = 2
SOLVE_MIXED_FP32 = 3
SOLVE_MIXED_BF16 = 4
LAUNCH_KERNELS = 0
ASSEMBLY_PARTIAL = 0
ASSEMBLY_MATRIX_FREE = 1
LAUNCH_GRAPH = 1
LAUNCH_PERSISTENT = 2

_ERRORS = {0: "OK", -1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "HIP", -4: "NOT_CONVERGED",
           -5: "UNSUPPORTED", -6: "NO_DEVICE"}


class PafemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pafem error {_ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = _ERRORS.get(code, str(code))


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("rtol", C.c_double), ("inner_rtol", C.c_double),
                ("maxit", C.c_int), ("max_outer", C.c_int), ("check_every", C.c_int),
                ("launch", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer_iterations", C.c_int), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("seconds", C.c_double),
                ("fp64_inner_solves", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("p", C.c_int),
                ("verts_host", C.c_void_p), ("coef_kind", C.c_int), ("coef_value", C.c_double),
                ("mode", C.c_int), ("rtol", C.c_double), ("inner_rtol", C.c_double),
                ("maxit", C.c_int), ("max_outer", C.c_int)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("error", C.c_int), ("ndofs", C.c_int64),
                ("footprint_bytes", C.c_int64), ("iterations", C.c_int),
                ("outer_iterations", C.c_int), ("rel_res", C.c_double),
                ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("rounds", C.c_int64), ("peak_bytes", C.c_int64), ("max_active", C.c_int),
                ("dof_iterations", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MgOpts(C.Structure):
    _fields_ = [("cheb_degree", C.c_int), ("cheb_lower", C.c_double), ("lmax_safety", C.c_double),
                ("power_iters", C.c_int), ("coarse_iters", C.c_int)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
COEF_CONST, COEF_SINX = 0, 1

_P = C.c_void_p
_I = C.c_int
_I64 = C.c_int64
_D = C.c_double
_PP = C.POINTER(C.c_void_p)

# name: (restype, argtypes)
_SIGNATURES = {
    "pafem_last_error": (C.c_char_p, []),
    "pafem_version": (_I, []),
    "pafem_ctx_create": (_I, [_I, _PP]),
    "pafem_ctx_destroy": (_I, [_P]),
    "pafem_mesh_create_structured": (_I, [_P, _I, _I, _I, _P, _PP]),
    "pafem_mesh_destroy": (_I, [_P]),
    "pafem_space_create": (_I, [_P, _I, _PP]),
    "pafem_space_destroy": (_I, [_P]),
    "pafem_space_ndofs": (_I64, [_P]),
    "pafem_space_nelems": (_I64, [_P]),
    "pafem_space_num_ess": (_I64, [_P]),
    "pafem_space_get_restriction": (_I, [_P, _P]),
    "pafem_space_get_restriction_transpose": (_I, [_P, _P, _P]),
    "pafem_space_get_ess_dofs": (_I, [_P, _P]),
    "pafem_basis_tables": (_I, [_I, _I, _P, _P, _P, _P, _P]),
    "pafem_op_create": (_I, [_P, _I, _I, _PP]),
    "pafem_op_destroy": (_I, [_P]),
    "pafem_op_q1d": (_I, [_P]),
    "pafem_op_qpoint_coords": (_I, [_P, _P, _P]),
    "pafem_op_set_coefficient_const": (_I, [_P, _D]),
    "pafem_op_set_coefficient_qpts": (_I, [_P, _P, _P]),
    "pafem_op_set_coefficient_sinx": (_I, [_P, _D]),
    "pafem_op_assemble": (_I, [_P, _I, _P]),
    "pafem_op_qdata_bytes": (_I64, [_P, _I]),
    "pafem_op_footprint_bytes": (_I64, [_P, _I]),
    "pafem_op_get_qdata": (_I, [_P, _I, _P, _P]),
    "pafem_op_set_scatter_mode": (_I, [_P, _I]),
    "pafem_op_set_assembly_level": (_I, [_P, _I]),
    "pafem_op_set_restriction_mode": (_I, [_P, _I]),
    "pafem_op_apply": (_I, [_P, _I, _P, _P, _I, _P]),
    "pafem_op_apply_evector": (_I, [_P, _I, _P, _P, _I, _P]),
    "pafem_op_apply_noalloc": (_I, [_P, _I, _P, _P, _I, _P]),
    "pafem_op_diagonal": (_I, [_P, _P, _I, _P]),
    "pafem_rhs_assemble": (_I, [_P, _P, _P, _P]),
    "pafem_solve_cg": (_I, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveStats), _P]),
    "pafem_dot": (_I, [_P, _I64, _P, _P, _P, _P]),
    "pafem_mg_default_opts": (None, [C.POINTER(MgOpts)]),
    "pafem_mg_create": (_I, [_P, C.POINTER(MgOpts), _PP]),
    "pafem_mg_destroy": (_I, [_P]),
    "pafem_mg_num_levels": (_I, [_P]),
    "pafem_mg_level_info": (_I, [_P, _I, C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_double)]),
    "pafem_mg_set_lmax": (_I, [_P, _I, _D]),
    "pafem_mg_prolong": (_I, [_P, _I, _P, _P, _P]),
    "pafem_mg_restrict": (_I, [_P, _I, _P, _P, _P]),
    "pafem_mg_smooth": (_I, [_P, _I, _P, _P, _P]),
    "pafem_mg_vcycle": (_I, [_P, _P, _P, _P]),
    "pafem_mg_solve": (_I, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveStats), _P]),
    "pafem_request_footprint": (_I64, [C.POINTER(Request)]),
    "pafem_server_create": (_I, [_P, _I64, _I, _I, _PP]),
    "pafem_server_submit": (_I, [_P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "pafem_server_poll": (_I, [_P, C.c_uint64, C.POINTER(Result)]),
    "pafem_server_get_solution": (_I, [_P, C.c_uint64, _P, _I64]),
    "pafem_server_drain": (_I, [_P]),
    "pafem_server_stats": (_I, [_P, C.POINTER(ServerStats)]),
    "pafem_server_destroy": (_I, [_P]),
}

_lib = None


def lib() -> C.CDLL:
    """Load libpafem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2402_15940_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(rc: int):
    if rc != 0:
        msg = lib().pafem_last_error().decode(errors="replace")
        raise PafemError(rc, msg)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous GPU tensor, with dtype/length checks."""
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data)


def version() -> int:
    return lib().pafem_version()


def basis_tables(p: int, q: int) -> dict:
    """GLL nodes, GL points/weights and B/G tables from the library (host)."""
    out = {"nodes": np.empty(p + 1), "points": np.empty(q), "weights": np.empty(q),
           "B": np.empty((q, p + 1)), "G": np.empty((q, p + 1))}
    _check(lib().pafem_basis_tables(p, q, *[_np_ptr(out[k]) for k in
                                            ("nodes", "points", "weights", "B", "G")]))
    return out


class Context:
    """Binding of a pafem context: device >= 0 for a GPU, -1 for host-only queries."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().pafem_ctx_create(device, C.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def dot(self, x, y, stream=None):
        import torch
        n = x.numel()
        out = torch.empty(1, dtype=torch.float64, device=x.device)
        _check(lib().pafem_dot(self._h, n, _dptr(x, torch.float64, None, "x"),
                               _dptr(y, torch.float64, n, "y"), _dptr(out), _stream(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().pafem_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """Structured nx*ny*nz hexahedral mesh from a [(nx+1)(ny+1)(nz+1), 3] vertex array."""

    def __init__(self, ctx: Context, nx: int, ny: int, nz: int, verts: np.ndarray):
        v = np.ascontiguousarray(verts, dtype=np.float64)
        if v.shape != ((nx + 1) * (ny + 1) * (nz + 1), 3):
            raise ValueError(f"verts must have shape {((nx + 1) * (ny + 1) * (nz + 1), 3)}")
        h = C.c_void_p()
        _check(lib().pafem_mesh_create_structured(ctx.handle, nx, ny, nz, _np_ptr(v), C.byref(h)))
        self._h = h
        self.ctx = ctx
        self.shape = (nx, ny, nz)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().pafem_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Space:
    """Order-p H1 space on a mesh; exposes the integer maps."""

    def __init__(self, mesh: Mesh, p: int):
        h = C.c_void_p()
        _check(lib().pafem_space_create(mesh.handle, p, C.byref(h)))
        self._h = h
        self.mesh = mesh
        self.p = p

    @property
    def handle(self):
        return self._h

    @property
    def ndofs(self) -> int:
        return lib().pafem_space_ndofs(self._h)

    @property
    def nelems(self) -> int:
        return lib().pafem_space_nelems(self._h)

    @property
    def num_ess(self) -> int:
        return lib().pafem_space_num_ess(self._h)

    def restriction(self) -> np.ndarray:
        E = np.empty((self.nelems, (self.p + 1) ** 3), dtype=np.int32)
        _check(lib().pafem_space_get_restriction(self._h, _np_ptr(E)))
        return E

    def restriction_transpose(self):
        off = np.empty(self.ndofs + 1, dtype=np.int32)
        idx = np.empty(self.nelems * (self.p + 1) ** 3, dtype=np.int32)
        _check(lib().pafem_space_get_restriction_transpose(self._h, _np_ptr(off), _np_ptr(idx)))
        return off, idx

    def ess_dofs(self) -> np.ndarray:
        out = np.empty(self.num_ess, dtype=np.int32)
        _check(lib().pafem_space_get_ess_dofs(self._h, _np_ptr(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().pafem_space_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """Partially assembled MASS or DIFFUSION operator (see include/pafem.h)."""

    def __init__(self, space: Space, kind: int = DIFFUSION, q1d: int = 0):
        h = C.c_void_p()
        _check(lib().pafem_op_create(space.handle, kind, q1d, C.byref(h)))
        self._h = h
        self.space = space
        self.kind = kind
        self.q = lib().pafem_op_q1d(h)

    @property
    def handle(self):
        return self._h

    @property
    def ncomp(self) -> int:
        return 6 if self.kind == DIFFUSION else 1

    def _torch(self):
        import torch
        return torch

    def qpoint_coords(self, stream=None):
        torch = self._torch()
        n = self.space.nelems * 3 * self.q ** 3
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().pafem_op_qpoint_coords(self._h, _dptr(out), _stream(stream)))
        return out.view(self.space.nelems, 3, self.q ** 3)

    def set_coefficient_const(self, c: float):
        _check(lib().pafem_op_set_coefficient_const(self._h, float(c)))

    def set_coefficient_qpts(self, k, stream=None):
        torch = self._torch()
        n = self.space.nelems * self.q ** 3
        _check(lib().pafem_op_set_coefficient_qpts(self._h, _dptr(k, torch.float64, n, "k"),
                                                   _stream(stream)))

    def set_coefficient_sinx(self, amp: float = 0.5):
        _check(lib().pafem_op_set_coefficient_sinx(self._h, float(amp)))

    def assemble(self, prec_mask: int = FP64, stream=None):
        _check(lib().pafem_op_assemble(self._h, prec_mask, _stream(stream)))

    def footprint_bytes(self, prec_mask: int = FP64) -> int:
        return lib().pafem_op_footprint_bytes(self._h, prec_mask)

    def qdata_bytes(self, prec_mask: int = FP64) -> int:
        return lib().pafem_op_qdata_bytes(self._h, prec_mask)

    def qdata(self, prec: int = FP64, stream=None):
        """Stored quadrature data [ne, C, q^3]; the bfloat16 copy comes back as int16 bits."""
        torch = self._torch()
        dt = {FP64: torch.float64, FP32: torch.float32, BF16: torch.int16}[prec]
        out = torch.empty(self.space.nelems * self.ncomp * self.q ** 3, dtype=dt, device="cuda")
        _check(lib().pafem_op_get_qdata(self._h, prec, _dptr(out), _stream(stream)))
        return out.view(self.space.nelems, self.ncomp, self.q ** 3)

    def set_assembly_level(self, level: int):
        _check(lib().pafem_op_set_assembly_level(self._h, level))

    def set_scatter_mode(self, mode: int):
        _check(lib().pafem_op_set_scatter_mode(self._h, mode))

    def set_restriction_mode(self, mode: int):
        _check(lib().pafem_op_set_restriction_mode(self._h, mode))

    def apply(self, x, y=None, constrained: bool = False, accumulate: bool = False,
              bf16: bool = False, stream=None):
        """y = A x; float vectors use the FP32 quadrature data, or the bfloat16 copy."""
        torch = self._torch()
        prec = FP64 if x.dtype == torch.float64 else (BF16 if bf16 else FP32)
        n = self.space.ndofs
        if y is None:
            if accumulate:
                raise ValueError("accumulate needs y")
            y = torch.empty_like(x)
        flags = (APPLY_CONSTRAINED if constrained else 0) | (APPLY_ACCUMULATE if accumulate else 0)
        _check(lib().pafem_op_apply(self._h, prec, _dptr(x, x.dtype, n, "x"),
                                    _dptr(y, x.dtype, n, "y"), flags, _stream(stream)))
        return y

    def apply_noalloc(self, x, y, constrained: bool = False, accumulate: bool = False,
                      bf16: bool = False, stream=None):
        """y = A x through the allocation-free entry point (y must be given)."""
        torch = self._torch()
        prec = FP64 if x.dtype == torch.float64 else (BF16 if bf16 else FP32)
        n = self.space.ndofs
        flags = (APPLY_CONSTRAINED if constrained else 0) | (APPLY_ACCUMULATE if accumulate else 0)
        _check(lib().pafem_op_apply_noalloc(self._h, prec, _dptr(x, x.dtype, n, "x"),
                                            _dptr(y, x.dtype, n, "y"), flags, _stream(stream)))
        return y

    def apply_evector(self, x, yE=None, constrained: bool = False, bf16: bool = False,
                      stream=None):
        """Element results before assembly, shape [nelems, (p+1)^3]."""
        torch = self._torch()
        prec = FP64 if x.dtype == torch.float64 else (BF16 if bf16 else FP32)
        m = self.space.nelems * (self.space.p + 1) ** 3
        if yE is None:
            yE = torch.empty(m, dtype=x.dtype, device=x.device)
        _check(lib().pafem_op_apply_evector(self._h, prec, _dptr(x, x.dtype, self.space.ndofs, "x"),
                                            _dptr(yE, x.dtype, m, "yE"),
                                            APPLY_CONSTRAINED if constrained else 0,
                                            _stream(stream)))
        return yE.view(self.space.nelems, (self.space.p + 1) ** 3)

    def diagonal(self, constrained: bool = False, out=None, stream=None):
        torch = self._torch()
        n = self.space.ndofs
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().pafem_op_diagonal(self._h, _dptr(out, torch.float64, n, "d"),
                                       int(constrained), _stream(stream)))
        return out

    def rhs(self, f_q=None, out=None, stream=None):
        torch = self._torch()
        n = self.space.ndofs
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device="cuda")
        fp = C.c_void_p(0) if f_q is None else _dptr(
            f_q, torch.float64, self.space.nelems * self.q ** 3, "f_q")
        _check(lib().pafem_rhs_assemble(self._h, fp, _dptr(out, torch.float64, n, "b"),
                                        _stream(stream)))
        return out

    def solve(self, b, x=None, mode: int = SOLVE_PLAIN_FP64, rtol: float = 1e-10,
              inner_rtol: float = 1e-4, maxit: int = 10000, max_outer: int = 50,
              check_every: int = 1, stream=None, raise_on_nonconvergence: bool = True,
              launch: int = LAUNCH_KERNELS):
        torch = self._torch()
        n = self.space.ndofs
        if x is None:
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
        o = SolveOpts(mode, rtol, inner_rtol, maxit, max_outer, check_every, launch)
        st = SolveStats()
        rc = lib().pafem_solve_cg(self._h, _dptr(b, torch.float64, n, "b"),
                                  _dptr(x, torch.float64, n, "x"), C.byref(o), C.byref(st),
                                  _stream(stream))
        if rc != 0 and not (rc == -4 and not raise_on_nonconvergence):
            _check(rc)
        return x, st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().pafem_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f64():
    import torch
    return torch.float64


class Multigrid:
    """p-multigrid hierarchy (orders p, p/2, ..., 1) of an FP64-assembled operator."""

    def __init__(self, op: "Operator", cheb_degree=None, cheb_lower=None, lmax_safety=None,
                 power_iters=None, coarse_iters=None):
        o = MgOpts()
        lib().pafem_mg_default_opts(C.byref(o))
        for k, v in (("cheb_degree", cheb_degree), ("cheb_lower", cheb_lower),
                     ("lmax_safety", lmax_safety), ("power_iters", power_iters),
                     ("coarse_iters", coarse_iters)):
            if v is not None:
                setattr(o, k, v)
        self.op = op
        self.opts = o
        h = C.c_void_p()
        _check(lib().pafem_mg_create(op.handle, C.byref(o), C.byref(h)))
        self._h = h

    @property
    def num_levels(self) -> int:
        return lib().pafem_mg_num_levels(self._h)

    def level_info(self, level: int) -> dict:
        p, n, lm = C.c_int(), C.c_int64(), C.c_double()
        _check(lib().pafem_mg_level_info(self._h, level, C.byref(p), C.byref(n), C.byref(lm)))
        return {"p": p.value, "ndofs": n.value, "lmax": lm.value}

    def set_lmax(self, level: int, lmax: float):
        _check(lib().pafem_mg_set_lmax(self._h, level, float(lmax)))

    def _vec(self, level):
        import torch
        return torch.empty(self.level_info(level)["ndofs"], dtype=torch.float64, device="cuda")

    def prolong(self, level: int, uc, out=None, stream=None):
        nf, nc = self.level_info(level)["ndofs"], self.level_info(level + 1)["ndofs"]
        uf = self._vec(level) if out is None else out
        _check(lib().pafem_mg_prolong(self._h, level, _dptr(uc, _f64(), nc, "uc"),
                                      _dptr(uf, _f64(), nf, "uf"), _stream(stream)))
        return uf

    def restrict(self, level: int, rf, out=None, stream=None):
        nf, nc = self.level_info(level)["ndofs"], self.level_info(level + 1)["ndofs"]
        rc = self._vec(level + 1) if out is None else out
        _check(lib().pafem_mg_restrict(self._h, level, _dptr(rf, _f64(), nf, "rf"),
                                       _dptr(rc, _f64(), nc, "rc"), _stream(stream)))
        return rc

    def smooth(self, level: int, b, out=None, stream=None):
        n = self.level_info(level)["ndofs"]
        x = self._vec(level) if out is None else out
        _check(lib().pafem_mg_smooth(self._h, level, _dptr(b, _f64(), n, "b"), _dptr(x, _f64(), n, "x"),
                                     _stream(stream)))
        return x

    def vcycle(self, r, out=None, stream=None):
        n = self.level_info(0)["ndofs"]
        z = self._vec(0) if out is None else out
        _check(lib().pafem_mg_vcycle(self._h, _dptr(r, _f64(), n, "r"), _dptr(z, _f64(), n, "z"),
                                     _stream(stream)))
        return z

    def solve(self, b, x=None, rtol: float = 1e-10, maxit: int = 1000, stream=None):
        """Flexible CG with one V-cycle per iteration; returns (x, stats dict)."""
        import torch
        n = self.level_info(0)["ndofs"]
        if x is None:
            x = torch.zeros_like(b)
        o = SolveOpts(SOLVE_PLAIN_FP64, rtol, 0.0, maxit, 0, 1)
        st = SolveStats()
        rc = lib().pafem_mg_solve(self._h, _dptr(b, _f64(), n, "b"), _dptr(x, _f64(), n, "x"),
                                  C.byref(o), C.byref(st), _stream(stream))
        if rc not in (0, -4):
            _check(rc)
        d = st.as_dict()
        d["converged"] = rc == 0
        return x, d

    def close(self):
        if getattr(self, "_h", None):
            lib().pafem_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_request(nx, ny, nz, p, verts, coef_kind=COEF_CONST, coef_value=1.0,
                 mode=SOLVE_IR_FP32, rtol=1e-10, inner_rtol=1e-4, maxit=20000, max_outer=30):
    """Request structure plus the vertex array it points to (keep both alive)."""
    v = np.ascontiguousarray(verts, dtype=np.float64)
    if v.shape != ((nx + 1) * (ny + 1) * (nz + 1), 3):
        raise ValueError("verts has the wrong shape")
    req = Request(nx, ny, nz, p, v.ctypes.data, coef_kind, coef_value, mode, rtol, inner_rtol,
                  maxit, max_outer)
    return req, v


def request_footprint(nx, ny, nz, p, mode=SOLVE_IR_FP32) -> int:
    dummy = np.zeros(((nx + 1) * (ny + 1) * (nz + 1), 3))
    req, _ = make_request(nx, ny, nz, p, dummy, mode=mode)
    return lib().pafem_request_footprint(C.byref(req))


class Server:
    """Continuous-batching Poisson solve server on one GPU (see include/pafem.h)."""

    def __init__(self, ctx: Context, budget_bytes: int, max_slots: int = 16,
                 iters_per_round: int = 10):
        h = C.c_void_p()
        _check(lib().pafem_server_create(ctx.handle, int(budget_bytes), max_slots,
                                         iters_per_round, C.byref(h)))
        self._h = h
        self.ctx = ctx

    def submit(self, nx, ny, nz, p, verts, **kw) -> int:
        req, v = make_request(nx, ny, nz, p, verts, **kw)
        t = C.c_uint64()
        _check(lib().pafem_server_submit(self._h, C.byref(req), C.byref(t)))
        return t.value

    def poll(self, ticket: int) -> dict:
        r = Result()
        _check(lib().pafem_server_poll(self._h, ticket, C.byref(r)))
        return r.as_dict()

    def solution(self, ticket: int) -> np.ndarray:
        n = self.poll(ticket)["ndofs"]
        x = np.empty(n)
        _check(lib().pafem_server_get_solution(self._h, ticket, _np_ptr(x), n))
        return x

    def drain(self):
        _check(lib().pafem_server_drain(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().pafem_server_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().pafem_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
