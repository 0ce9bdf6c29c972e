"""ctypes binding of libhhg.so.  Argument marshalling only: every numerical step runs in the
HIP library; PyTorch supplies device memory and the stream.

The raw C entry points are exposed under their C names (``hhg_setup``, ``hhg_fmg_solve``, ...);
:class:`HHG` wraps one context with tensors.  Importing fails loudly when the library has not
been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhhg.so")

HHG_OK, HHG_EINVAL, HHG_EMESH, HHG_ENOMEM, HHG_EHIP, HHG_ENOTCONV, HHG_ESTATE = 0, -1, -2, -3, -4, -5, -6
HHG_KAPPA_MACRO, HHG_KAPPA_P1 = 0, 1
HHG_GS_REDBLACK, HHG_GS_MULTICOLOR, HHG_JACOBI = 0, 1, 2
HHG_FP64, HHG_FP32_REFINED = 0, 1
HHG_OP_STIFFNESS, HHG_OP_MASS = 0, 1
HHG_NORM_L2, HHG_NORM_ENERGY, HHG_NORM_LUMPED = 0, 1, 2
HHG_LOCAL_L1, HHG_LOCAL_UNSCALED, HHG_LOCAL_SCALED = 0, 1, 2
_NORMS = {"l2": HHG_NORM_L2, "energy": HHG_NORM_ENERGY, "lumped": HHG_NORM_LUMPED}
_LOCALS = {"l1": HHG_LOCAL_L1, "unscaled": HHG_LOCAL_UNSCALED, "scaled": HHG_LOCAL_SCALED}
HHG_FLAG_NO_FUSED = 1
HHG_FLAG_NO_LANE_IFACE = 2
HHG_FLAG_NO_GRAPH = 4
HHG_FLAG_NO_PRELOAD = 8
HHG_FLAG_ROWS3D = 16
HHG_FLAG_STREAM3D = 32
HHG_FLAG_GENERIC_EST = 64
HHG_FLAG_CLASSWISE_IFACE = 128
HHG_FLAG_NO_PLANES3D = 256
HHG_FLAG_PLANES3D = 512
HHG_FLAG_TWO_LAUNCH_IFACE = 1024
HHG_FLAG_NO_DENSE_COARSE = 2048
HHG_FLAG_DENSE_COARSE = 4096
HHG_FLAG_NO_FUSED_PROLONG = 8192

SMOOTHERS = {"redblack": HHG_GS_REDBLACK, "multicolour": HHG_GS_MULTICOLOR, "jacobi": HHG_JACOBI}
PRECISIONS = {"fp64": HHG_FP64, "fp32_refined": HHG_FP32_REFINED}


class hhg_mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_vertices", C.c_int64), ("coords", C.POINTER(C.c_double)),
                ("n_cells", C.c_int64), ("cells", C.POINTER(C.c_int32)),
                ("dirichlet", C.POINTER(C.c_uint8)), ("kappa_cell", C.POINTER(C.c_double))]


class hhg_options(C.Structure):
    _fields_ = [("coefficient", C.c_int), ("smoother", C.c_int), ("jacobi_omega", C.c_double), ("flags", C.c_int)]


class hhg_solve_params(C.Structure):
    _fields_ = [("nu", C.c_int), ("pre", C.c_int), ("post", C.c_int), ("precision", C.c_int),
                ("rtol", C.c_double), ("max_iter", C.c_int)]


class hhg_solve_stats(C.Structure):
    _fields_ = [("vcycles", C.c_int), ("ir_steps", C.c_int), ("final_rel_residual", C.c_double),
                ("ms_total", C.c_double), ("dense_level", C.c_int)]


_ctx = C.c_void_p
_dp = C.c_void_p   # device pointers travel as integers
_SIGS = {
    "hhg_setup": (C.c_int, [C.POINTER(hhg_mesh), C.c_int, C.POINTER(hhg_options), C.POINTER(_ctx)]),
    "hhg_workspace_bytes": (C.c_int, [_ctx, C.POINTER(C.c_size_t)]),
    "hhg_bind_workspace": (C.c_int, [_ctx, _dp, C.c_size_t, C.c_void_p]),
    "hhg_bind_static_workspace": (C.c_int, [_ctx, C.c_void_p]),
    "hhg_num_dofs": (C.c_int, [_ctx, C.c_int, C.POINTER(C.c_int64)]),
    "hhg_dof_coords": (C.c_int, [_ctx, C.c_int, _dp]),
    "hhg_set_kappa_cell": (C.c_int, [_ctx, C.POINTER(C.c_double)]),
    "hhg_set_kappa_nodal": (C.c_int, [_ctx, _dp]),
    "hhg_fmg_solve": (C.c_int, [_ctx, _dp, _dp, _dp, C.POINTER(hhg_solve_params), C.POINTER(hhg_solve_stats)]),
    "hhg_estimate": (C.c_int, [_ctx, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "hhg_estimate_ex": (C.c_int, [_ctx, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "hhg_macro_norms": (C.c_int, [_ctx, _dp, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "hhg_cycle_solve": (C.c_int, [_ctx, _dp, _dp, _dp, C.POINTER(hhg_solve_params), C.POINTER(hhg_solve_stats)]),
    "hhg_transfer": (C.c_int, [_ctx, _ctx, _dp, _dp]),
    "hhg_apply": (C.c_int, [_ctx, C.c_int, C.c_int, _dp, _dp]),
    "hhg_mass_apply": (C.c_int, [_ctx, _dp, _dp]),
    "hhg_smooth": (C.c_int, [_ctx, C.c_int, _dp, _dp, C.c_int]),
    "hhg_restrict": (C.c_int, [_ctx, C.c_int, _dp, _dp]),
    "hhg_prolongate": (C.c_int, [_ctx, C.c_int, _dp, _dp]),
    "hhg_adjoint": (C.c_int, [_ctx, _dp, _dp, _dp, _dp, C.POINTER(C.c_double), C.POINTER(hhg_solve_params)]),
    "hhg_bench_smoother": (C.c_int, [_ctx, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "hhg_residual_history": (C.c_int, [_ctx, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int)]),
    "hhg_status_string": (C.c_char_p, [C.c_int]),
    "hhg_last_error": (C.c_char_p, [_ctx]),
    "hhg_destroy": (None, [_ctx]),
}

_lib = None


def load() -> C.CDLL:
    """Load libhhg.so from the package directory (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_06049_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list[str]:
    return sorted(_SIGS)


class HHGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status: int, ctx=None):
    if status != HHG_OK:
        lib = load()
        msg = lib.hhg_last_error(ctx).decode()
        raise HHGError(status, msg or lib.hhg_status_string(status).decode())


def _dptr(t, n: int | None = None) -> int:
    """Device address of a contiguous float64 CUDA tensor; with n, its length must be n (the
    C entry points take raw pointers and cannot check sizes themselves)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("device tensor expected")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("contiguous float64 tensor expected")
    if n is not None and t.numel() != n:
        raise ValueError(f"vector of length {n} expected, got {t.numel()}")
    return t.data_ptr()


def _dbl(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class SolveStats:
    vcycles: int
    ir_steps: int
    final_rel_residual: float
    ms_total: float
    dense_level: int = -1


def setup_host(coords, cells, L: int, smoother: str = "redblack", coefficient: str = "macro",
               kappa_cell=None, dirichlet=None, omega: float = 0.0, flags: int = 0):
    """Call hhg_setup (host only).  Returns (ctx handle, keep-alive arrays)."""
    lib = load()
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    m = hhg_mesh()
    m.dim = coords.shape[1]
    m.n_vertices = coords.shape[0]
    m.coords = _dbl(coords)
    m.n_cells = cells.shape[0]
    m.cells = cells.ctypes.data_as(C.POINTER(C.c_int32))
    keep = [coords, cells]
    if dirichlet is not None:
        d = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        keep.append(d)
        m.dirichlet = d.ctypes.data_as(C.POINTER(C.c_uint8))
    if kappa_cell is not None:
        k = np.ascontiguousarray(kappa_cell, dtype=np.float64)
        keep.append(k)
        m.kappa_cell = _dbl(k)
    o = hhg_options()
    o.coefficient = HHG_KAPPA_P1 if coefficient == "p1" else HHG_KAPPA_MACRO
    o.smoother = SMOOTHERS[smoother]
    o.jacobi_omega = omega
    o.flags = flags
    ctx = _ctx()
    _check(lib.hhg_setup(C.byref(m), L, C.byref(o), C.byref(ctx)), None)
    return ctx, keep


class HHG:
    """One HHG context bound to a torch-allocated workspace on a CUDA (HIP) device."""

    def __init__(self, coords, cells, L: int, smoother: str = "redblack", coefficient: str = "macro",
                 kappa_cell=None, dirichlet=None, omega: float = 0.0, device="cuda:0", flags: int = 0,
                 workspace: str = "torch"):
        """workspace: "torch" (device memory allocated here by torch, hhg_bind_workspace) or
        "static" (the library's static workspace, hhg_bind_static_workspace: no allocation)."""
        import torch
        self.lib = load()
        self.dim = int(np.asarray(coords).shape[1])
        self.n_cells = int(np.asarray(cells).shape[0])
        self.L = L
        self.coefficient = coefficient
        self.ctx, _ = setup_host(coords, cells, L, smoother, coefficient, kappa_cell, dirichlet, omega, flags)
        nb = C.c_size_t()
        _check(self.lib.hhg_workspace_bytes(self.ctx, C.byref(nb)), self.ctx)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        if workspace == "static":
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(self.lib.hhg_bind_static_workspace(self.ctx, C.c_void_p(self.stream.cuda_stream)), self.ctx)
        elif workspace == "torch":
            self.workspace = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            _check(self.lib.hhg_bind_workspace(self.ctx, aligned, int(nb.value), C.c_void_p(self.stream.cuda_stream)),
                   self.ctx)
        else:
            raise ValueError(f"workspace must be 'torch' or 'static', not {workspace!r}")
        self.workspace_bytes = int(nb.value)

    # --- basics -----------------------------------------------------------------------------
    def num_dofs(self, level: int | None = None) -> int:
        n = C.c_int64()
        _check(self.lib.hhg_num_dofs(self.ctx, self.L if level is None else level, C.byref(n)), self.ctx)
        return int(n.value)

    def _nd(self, level: int | None = None) -> int:
        lvl = self.L if level is None else level
        if not 0 <= lvl <= self.L:
            raise HHGError(HHG_EINVAL, f"level {lvl} outside 0..{self.L}")
        if not hasattr(self, "_ndofs"):
            self._ndofs = [self.num_dofs(l) for l in range(self.L + 1)]
        return self._ndofs[lvl]

    def dof_coords(self, level: int | None = None):
        import torch
        lvl = self.L if level is None else level
        out = torch.empty((self.num_dofs(lvl), self.dim), dtype=torch.float64, device=self.device)
        _check(self.lib.hhg_dof_coords(self.ctx, lvl, _dptr(out)), self.ctx)
        return out

    def set_kappa_cell(self, kappa):
        k = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64))
        _check(self.lib.hhg_set_kappa_cell(self.ctx, _dbl(k)), self.ctx)

    def set_kappa_nodal(self, kappa):
        _check(self.lib.hhg_set_kappa_nodal(self.ctx, _dptr(kappa, self._nd())), self.ctx)

    @staticmethod
    def params(nu=1, pre=2, post=2, precision="fp64", rtol=0.0, max_iter=0) -> hhg_solve_params:
        p = hhg_solve_params()
        p.nu, p.pre, p.post = nu, pre, post
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        p.rtol, p.max_iter = rtol, max_iter
        return p

    def fmg_solve(self, f, g, u_out=None, **kw):
        import torch
        p = self.params(**kw)
        u = torch.empty_like(f) if u_out is None else u_out
        st = hhg_solve_stats()
        n = self._nd()
        _check(self.lib.hhg_fmg_solve(self.ctx, _dptr(f, n), _dptr(g, n), _dptr(u, n), C.byref(p), C.byref(st)),
               self.ctx)
        return u, SolveStats(st.vcycles, st.ir_steps, st.final_rel_residual, st.ms_total, st.dense_level)

    def cycle_solve(self, f, g, u0, **kw):
        """hhg_cycle_solve: V-cycles from the iterate u0 (copied); returns (u, stats)."""
        p = self.params(**kw)
        u = u0.clone()
        st = hhg_solve_stats()
        n = self._nd()
        _check(self.lib.hhg_cycle_solve(self.ctx, _dptr(f, n), _dptr(g, n), _dptr(u, n), C.byref(p), C.byref(st)),
               self.ctx)
        return u, SolveStats(st.vcycles, st.ir_steps, st.final_rel_residual, st.ms_total, st.dense_level)

    def transfer_from(self, old: "HHG", u_old):
        """hhg_transfer: u_old on old's level L evaluated at this context's level-L DoFs."""
        import torch
        out = torch.empty(self._nd(), dtype=torch.float64, device=self.device)
        _check(self.lib.hhg_transfer(self.ctx, old.ctx, _dptr(u_old, old._nd()), _dptr(out)), self.ctx)
        return out

    def residual_history(self) -> np.ndarray:
        n = C.c_int()
        _check(self.lib.hhg_residual_history(self.ctx, None, 0, C.byref(n)), self.ctx)
        out = np.zeros(max(n.value, 1))
        _check(self.lib.hhg_residual_history(self.ctx, _dbl(out), n.value, C.byref(n)), self.ctx)
        return out[:n.value]

    def estimate(self, j: int = 1, norm: str | None = None, local: str | None = None) -> dict:
        """hhg_estimate; with ``norm`` ("l2", "energy", "lumped") or ``local`` ("l1",
        "unscaled", "scaled") given, hhg_estimate_ex."""
        eta = np.zeros(self.n_cells)
        ej, th, ne = C.c_double(), C.c_double(), C.c_double()
        if norm is None and local is None:
            st = self.lib.hhg_estimate(self.ctx, j, _dbl(eta), C.byref(ej), C.byref(th), C.byref(ne))
        else:
            st = self.lib.hhg_estimate_ex(self.ctx, j, _NORMS[norm or "l2"], _LOCALS[local or "l1"], _dbl(eta),
                                          C.byref(ej), C.byref(th), C.byref(ne))
        _check(st, self.ctx)
        return dict(eta_T=eta, eta_j=ej.value, theta=th.value, norm_e=ne.value)

    def macro_norms(self, x=None, level: int = -1, norm: str = "l2") -> np.ndarray:
        """hhg_macro_norms: per-macro squared norms of x (level -1), x - u_L (level L) or
        x - I w_level (0 <= level < L); x None means u_L of the last solve."""
        out = np.zeros(self.n_cells)
        _check(self.lib.hhg_macro_norms(self.ctx, None if x is None else _dptr(x, self._nd()), level, _NORMS[norm], _dbl(out)),
               self.ctx)
        return out

    def apply(self, level: int, op: str, x):
        import torch
        y = torch.empty_like(x)
        _check(self.lib.hhg_apply(self.ctx, level, HHG_OP_MASS if op == "mass" else HHG_OP_STIFFNESS,
                                  _dptr(x, self._nd(level)), _dptr(y)), self.ctx)
        return y

    def mass_apply(self, x):
        import torch
        y = torch.empty_like(x)
        _check(self.lib.hhg_mass_apply(self.ctx, _dptr(x, self._nd()), _dptr(y)), self.ctx)
        return y

    def smooth(self, level: int, u, b, sweeps: int = 1):
        _check(self.lib.hhg_smooth(self.ctx, level, _dptr(u, self._nd(level)), _dptr(b, self._nd(level)), sweeps),
               self.ctx)
        return u

    def restrict(self, level: int, r_fine):
        import torch
        out = torch.empty(self.num_dofs(level - 1), dtype=torch.float64, device=self.device)
        _check(self.lib.hhg_restrict(self.ctx, level, _dptr(r_fine, self._nd(level)), _dptr(out)), self.ctx)
        return out

    def prolongate(self, level: int, e_coarse):
        import torch
        out = torch.empty(self.num_dofs(level), dtype=torch.float64, device=self.device)
        _check(self.lib.hhg_prolongate(self.ctx, level, _dptr(e_coarse, self._nd(level - 1)), _dptr(out)), self.ctx)
        return out

    def adjoint(self, f, g, dJdu, **kw):
        import torch
        p = self.params(**kw)
        dJdf = torch.empty_like(f)
        dJdk = np.zeros(self.n_cells)
        n = self._nd()
        _check(self.lib.hhg_adjoint(self.ctx, _dptr(f, n), _dptr(g, n), _dptr(dJdu, n), _dptr(dJdf, n), _dbl(dJdk),
                                    C.byref(p)),
               self.ctx)
        return dJdf, dJdk

    def bench_smoother(self, precision="fp64", sweeps: int = 10, per_launch: bool = True) -> dict:
        ms, nbytes, lms, lbytes = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        _check(self.lib.hhg_bench_smoother(self.ctx, PRECISIONS[precision], sweeps, C.byref(ms), C.byref(nbytes),
                                           C.byref(lms) if per_launch else None,
                                           C.byref(lbytes) if per_launch else None), self.ctx)
        return dict(ms=ms.value, bytes=nbytes.value, launch_ms=lms.value, launch_bytes=lbytes.value)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hhg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
