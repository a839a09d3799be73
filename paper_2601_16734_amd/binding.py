"""Thin ctypes binding of libseemps_hip.so (include/seemps_hip.h).

Argument marshalling only: every step of apply/compress, scalar product and
norm runs in the library's HIP kernels.  PyTorch is used, when present, only
to obtain the current HIP stream (and device buffers for *_create_device).
Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int, c_size_t, c_ulonglong, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libseemps_hip.so")

OK, EINVAL, ENOMEM, EHIP, ENUMERIC, EUNSUPPORTED, ENODEV = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16x3": PREC_BF16X3, "bf16": PREC_BF16}
TRUNC_REL_NORM2, TRUNC_REL_SV = 0, 1
FACT_SVD, FACT_RSVD_MLP, FACT_RSVD_PREV, FACT_RSVD_FIXED = 0, 1, 2, 3
MLP_PARAMS = 64 * 32 + 64 + 64 * 64 + 64 + 64 + 1

# every symbol the header declares, in declaration order
EXPORTS = [
    "smps_ctx_create", "smps_ctx_create_planning", "smps_ctx_destroy", "smps_last_error",
    "smps_ctx_workspace_bytes", "smps_ctx_set_workspace_limit", "smps_ctx_set_split",
    "smps_ctx_set_profiling",
    "smps_ctx_kernel_time",
    "smps_mps_create", "smps_mps_create_device", "smps_mps_destroy", "smps_mps_shape", "smps_mps_read",
    "smps_mps_device_ptr", "smps_mpo_create", "smps_mpo_destroy", "smps_mpo_apply", "smps_simplify",
    "smps_last_info", "smps_last_log", "smps_last_factor_log", "smps_combine", "smps_mpo_transpose",
    "smps_mpo_apply_right", "smps_mpo_list_apply", "smps_mpo_simplify", "smps_mpo_shape", "smps_mpo_read",
    "smps_mpo_apply_batched", "smps_mpo_apply_batched_caps", "smps_plan_apply", "smps_plan_apply_batched",
    "smps_scprod", "smps_norm",
    "smps_scprod_noalloc",
    "smps_rank_mlp_init", "smps_rank_mlp_train", "smps_rank_mlp_predict", "smps_rank_mlp_get",
    "smps_rank_mlp_set", "smps_rank_mlp_grad", "smps_rank_training_pairs",
    "smps_autotune_apply", "smps_autotune_gemm", "smps_autotune_save", "smps_autotune_load", "smps_autotune_clear",
    "smps_autotune_entries", "smps_dmrg", "smps_last_jacobi_log",
    "smps_zmps_create", "smps_zmps_destroy", "smps_zmps_shape", "smps_zmps_read", "smps_zmpo_create",
    "smps_zmpo_destroy", "smps_zmpo_apply", "smps_zscprod",
]


class Strategy(ctypes.Structure):
    _fields_ = [("max_bond", c_int), ("tol", c_double), ("trunc_mode", c_int), ("max_sweeps", c_int),
                ("sweep_tol", c_double), ("precision", c_int), ("factorization", c_int)]


class ApplyInfo(ctypes.Structure):
    _fields_ = [("error_bound", c_double), ("discarded", c_double), ("norm", c_double), ("sweeps_done", c_int),
                ("steps", c_int), ("rsvd_accepted", c_int), ("rsvd_fallbacks", c_int), ("jacobi_sweeps", c_int),
                ("reserved", c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("workspace_bytes", c_size_t), ("steps", ctypes.c_longlong), ("operations", ctypes.c_longlong),
                ("launches", ctypes.c_longlong), ("graph_kernels", ctypes.c_longlong),
                ("descriptor_bytes", c_size_t)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class SmpsError(RuntimeError):
    def __init__(self, code: int, msg: str, info: dict | None = None):
        super().__init__(f"[{code}] {msg}")
        self.code = code
        self.info = info


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the library (once).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} (run __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    vp, ip, dp = c_void_p, POINTER(c_int), POINTER(c_double)
    sig = {
        "smps_ctx_create": (c_int, [c_int, vp, POINTER(vp)]),
        "smps_ctx_create_planning": (c_int, [POINTER(vp)]),
        "smps_ctx_set_workspace_limit": (c_int, [vp, c_size_t]),
        "smps_plan_apply": (c_int, [vp, vp, vp, POINTER(Strategy), POINTER(PlanInfo)]),
        "smps_plan_apply_batched": (c_int, [vp, c_int, POINTER(vp), POINTER(vp), ip, POINTER(Strategy),
                                            POINTER(PlanInfo)]),
        "smps_mpo_apply_batched_caps": (c_int, [vp, c_int, POINTER(vp), POINTER(vp), ip, POINTER(Strategy),
                                                POINTER(vp), dp]),
        "smps_ctx_destroy": (c_int, [vp]),
        "smps_last_error": (ctypes.c_char_p, [vp]),
        "smps_ctx_workspace_bytes": (c_int, [vp, POINTER(c_size_t)]),
        "smps_ctx_set_split": (c_int, [vp, c_int]),
        "smps_ctx_set_profiling": (c_int, [vp, c_int]),
        "smps_ctx_kernel_time": (c_int, [vp, c_int, POINTER(c_double), POINTER(ctypes.c_longlong)]),
        "smps_mps_create": (c_int, [vp, c_int, ip, ip, c_int, POINTER(vp), POINTER(vp)]),
        "smps_mps_create_device": (c_int, [vp, c_int, ip, ip, c_int, POINTER(vp), POINTER(vp)]),
        "smps_mps_destroy": (c_int, [vp]),
        "smps_mps_shape": (c_int, [vp, ip, ip, ip, ip]),
        "smps_mps_read": (c_int, [vp, vp, c_int, dp, c_size_t]),
        "smps_mps_device_ptr": (c_int, [vp, c_int, POINTER(vp)]),
        "smps_mpo_create": (c_int, [vp, c_int, ip, ip, ip, c_int, POINTER(vp), POINTER(vp)]),
        "smps_mpo_destroy": (c_int, [vp]),
        "smps_mpo_apply": (c_int, [vp, vp, vp, POINTER(Strategy), POINTER(vp), dp]),
        "smps_simplify": (c_int, [vp, vp, POINTER(Strategy), POINTER(vp), dp]),
        "smps_last_info": (c_int, [vp, POINTER(ApplyInfo)]),
        "smps_last_log": (c_int, [vp, c_int, dp, ip, dp, ip]),
        "smps_last_factor_log": (c_int, [vp, c_int, ip, ip]),
        "smps_combine": (c_int, [vp, c_int, dp, POINTER(vp), POINTER(vp), POINTER(Strategy), POINTER(vp), dp]),
        "smps_mpo_transpose": (c_int, [vp, vp, POINTER(vp)]),
        "smps_mpo_shape": (c_int, [vp, ip, ip, ip, ip]),
        "smps_mpo_read": (c_int, [vp, vp, c_int, dp, c_size_t]),
        "smps_mpo_apply_right": (c_int, [vp, vp, vp, POINTER(Strategy), POINTER(vp), dp]),
        "smps_mpo_list_apply": (c_int, [vp, c_int, POINTER(vp), vp, POINTER(Strategy), POINTER(vp), dp]),
        "smps_mpo_simplify": (c_int, [vp, vp, POINTER(Strategy), POINTER(vp), dp]),
        "smps_mpo_apply_batched": (c_int, [vp, c_int, POINTER(vp), POINTER(vp), POINTER(Strategy), POINTER(vp), dp]),
        "smps_scprod": (c_int, [vp, vp, vp, dp]),
        "smps_norm": (c_int, [vp, vp, dp]),
        "smps_scprod_noalloc": (c_int, [vp, vp, vp, vp]),
        "smps_rank_mlp_init": (c_int, [vp, c_ulonglong]),
        "smps_rank_mlp_train": (c_int, [vp, c_int, POINTER(c_float), POINTER(c_float), c_int, c_int, c_float,
                                        POINTER(c_float)]),
        "smps_rank_mlp_predict": (c_int, [vp, c_int, POINTER(c_float), POINTER(c_float)]),
        "smps_rank_mlp_get": (c_int, [vp, POINTER(c_float), c_int]),
        "smps_rank_mlp_set": (c_int, [vp, POINTER(c_float), c_int]),
        "smps_rank_training_pairs": (c_int, [vp, c_int, POINTER(c_float), POINTER(c_float), ip]),
        "smps_autotune_apply": (c_int, [vp, vp, vp, POINTER(Strategy), c_int, ip]),
        "smps_autotune_gemm": (c_int, [vp, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                                       c_int, ip]),
        "smps_autotune_save": (c_int, [vp, ctypes.c_char_p]),
        "smps_autotune_load": (c_int, [vp, ctypes.c_char_p]),
        "smps_autotune_clear": (c_int, [vp]),
        "smps_autotune_entries": (c_int, [vp, ip]),
        "smps_last_jacobi_log": (c_int, [vp, c_int, ip, ip]),
        "smps_zmps_create": (c_int, [vp, c_int, ip, ip, POINTER(dp), POINTER(vp)]),
        "smps_zmps_destroy": (c_int, [vp]),
        "smps_zmps_shape": (c_int, [vp, ip, ip, ip]),
        "smps_zmps_read": (c_int, [vp, vp, c_int, dp, ctypes.c_size_t]),
        "smps_zmpo_create": (c_int, [vp, c_int, ip, ip, ip, POINTER(dp), POINTER(vp)]),
        "smps_zmpo_destroy": (c_int, [vp]),
        "smps_zmpo_apply": (c_int, [vp, vp, vp, POINTER(Strategy), POINTER(vp), dp]),
        "smps_zscprod": (c_int, [vp, vp, vp, dp, dp]),
        "smps_dmrg": (c_int, [vp, vp, vp, POINTER(Strategy), c_int, POINTER(vp), dp]),
        "smps_rank_mlp_grad": (c_int, [vp, c_int, POINTER(c_float), POINTER(c_float), POINTER(c_float),
                                       POINTER(c_float), c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def strategy(max_bond: int, tol: float, *, sweeps: int = 4, precision="fp64", trunc_mode: int = TRUNC_REL_NORM2,
             sweep_tol: float = 0.0, factorization: int = FACT_SVD) -> Strategy:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return Strategy(int(max_bond), float(tol), int(trunc_mode), int(sweeps), float(sweep_tol), prec, int(factorization))


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_float))


class MPS:
    """Handle of a device MPS (owned; freed on destroy / garbage collection)."""

    def __init__(self, ctx: "Context", handle: c_void_p):
        self.ctx = ctx
        self.h = handle

    def shape(self):
        if not self.h:
            raise SmpsError(EINVAL, "MPS handle was destroyed")
        L = c_int()
        self.ctx._check(self.ctx.lib.smps_mps_shape(self.h, byref(L), None, None, None))
        phys = (c_int * L.value)()
        bonds = (c_int * (L.value + 1))()
        center = c_int()
        self.ctx._check(self.ctx.lib.smps_mps_shape(self.h, None, phys, bonds, byref(center)))
        return list(phys), list(bonds), center.value

    def read(self) -> list[np.ndarray]:
        phys, bonds, _ = self.shape()
        out = []
        for k in range(len(phys)):
            a = np.empty((bonds[k], phys[k], bonds[k + 1]), dtype=np.float64)
            self.ctx._check(self.ctx.lib.smps_mps_read(self.ctx.h, self.h, k, a.ctypes.data_as(POINTER(c_double)),
                                                      a.size))
            out.append(a)
        return out

    def device_ptr(self, site: int) -> int:
        p = c_void_p()
        self.ctx._check(self.ctx.lib.smps_mps_device_ptr(self.h, site, byref(p)))
        return p.value

    def destroy(self):
        if self.h:
            self.ctx.lib.smps_mps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                self.destroy()
        except Exception:
            pass


class MPO:
    """Handle of a device MPO (owned; freed on destroy / garbage collection)."""

    def __init__(self, ctx: "Context", handle: c_void_p, L: int):
        self.ctx = ctx
        self.h = handle
        self.L = L

    def shape(self):
        if not self.h:
            raise SmpsError(EINVAL, "MPO handle was destroyed")
        pout = (c_int * self.L)()
        pin = (c_int * self.L)()
        bonds = (c_int * (self.L + 1))()
        self.ctx._check(self.ctx.lib.smps_mpo_shape(self.h, None, pout, pin, bonds))
        return list(pout), list(pin), list(bonds)

    def read(self) -> list[np.ndarray]:
        pout, pin, bonds = self.shape()
        out = []
        for k in range(self.L):
            a = np.empty((bonds[k], pout[k], pin[k], bonds[k + 1]), dtype=np.float64)
            self.ctx._check(self.ctx.lib.smps_mpo_read(self.ctx.h, self.h, k, a.ctypes.data_as(POINTER(c_double)),
                                                      a.size))
            out.append(a)
        return out

    def destroy(self):
        if self.h:
            self.ctx.lib.smps_mpo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                self.destroy()
        except Exception:
            pass


class ZMPS:
    """Handle of a device complex MPS (owned; freed on destroy / garbage collection)."""

    def __init__(self, ctx: "Context", handle: c_void_p):
        self.ctx = ctx
        self.h = handle

    def shape(self):
        L = c_int()
        self.ctx._check(self.ctx.lib.smps_zmps_shape(self.h, byref(L), None, None))
        phys = (c_int * L.value)()
        bonds = (c_int * (L.value + 1))()
        self.ctx._check(self.ctx.lib.smps_zmps_shape(self.h, None, phys, bonds))
        return list(phys), list(bonds)

    def read(self) -> list[np.ndarray]:
        phys, bonds = self.shape()
        out = []
        for k in range(len(phys)):
            a = np.empty((bonds[k], phys[k], bonds[k + 1]), dtype=np.complex128)
            self.ctx._check(self.ctx.lib.smps_zmps_read(self.ctx.h, self.h, k, a.ctypes.data_as(POINTER(c_double)),
                                                        a.size))
            out.append(a)
        return out

    def destroy(self):
        if self.h:
            self.ctx.lib.smps_zmps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.ctx.h:
                self.destroy()
        except Exception:
            pass


class ZMPO:
    """Handle of a device complex MPO."""

    def __init__(self, ctx: "Context", handle: c_void_p):
        self.ctx = ctx
        self.h = handle

    def destroy(self):
        if self.h:
            self.ctx.lib.smps_zmpo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.ctx.h:
                self.destroy()
        except Exception:
            pass


class Context:
    """A library context bound to one device and one HIP stream (torch's
    current stream by default), or a planning context (Context.planning())
    with no device."""

    def __init__(self, device: int = 0, stream: int | None = None, *, _planning: bool = False):
        self.lib = load()
        if _planning:
            h = c_void_p()
            rc = self.lib.smps_ctx_create_planning(byref(h))
            if rc != OK:
                raise SmpsError(rc, "smps_ctx_create_planning failed")
            self.h = h
            self.device = -1
            return
        if stream is None:
            import torch
            torch.cuda.set_device(device)
            stream = torch.cuda.current_stream(device).cuda_stream
        h = c_void_p()
        rc = self.lib.smps_ctx_create(int(device), c_void_p(stream), byref(h))
        if rc != OK:
            raise SmpsError(rc, f"smps_ctx_create(device={device}) failed")
        self.h = h
        self.device = device

    @classmethod
    def planning(cls) -> "Context":
        """Context with no device: shapes, validation and planning only."""
        return cls(_planning=True)

    def _check(self, rc: int):
        if rc != OK:
            raise SmpsError(rc, self.lib.smps_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.lib.smps_ctx_destroy(self.h)
            self.h = None

    # ---- handles
    def mps_create(self, tensors, dtype=np.float64) -> MPS:
        arrs = [np.ascontiguousarray(t, dtype=dtype) for t in tensors]
        L = len(arrs)
        phys = (c_int * L)(*[a.shape[1] for a in arrs])
        bonds = (c_int * (L + 1))(*([a.shape[0] for a in arrs] + [arrs[-1].shape[2]]))
        ptrs = (c_void_p * L)(*[a.ctypes.data for a in arrs])
        h = c_void_p()
        self._check(self.lib.smps_mps_create(self.h, L, phys, bonds, F64 if dtype == np.float64 else F32, ptrs,
                                             byref(h)))
        return MPS(self, h)

    def mps_zeros(self, phys, bonds) -> MPS:
        """MPS of the given shape with zero tensors (no host data passed); in a
        planning context a shape-only handle."""
        L = len(phys)
        h = c_void_p()
        self._check(self.lib.smps_mps_create(self.h, L, (c_int * L)(*phys), (c_int * (L + 1))(*bonds), F64, None,
                                             byref(h)))
        return MPS(self, h)

    def mpo_zeros(self, pout, pin, bonds) -> MPO:
        """MPO of the given shape with zero tensors; shape-only in a planning context."""
        L = len(pout)
        h = c_void_p()
        self._check(self.lib.smps_mpo_create(self.h, L, (c_int * L)(*pout), (c_int * L)(*pin),
                                             (c_int * (L + 1))(*bonds), F64, None, byref(h)))
        return MPO(self, h, L)

    def mps_create_device(self, tensors) -> MPS:
        """From torch device tensors (float64 or float32), copied on the stream."""
        import torch
        L = len(tensors)
        dt = F64 if tensors[0].dtype == torch.float64 else F32
        ts = [t.contiguous() for t in tensors]
        phys = (c_int * L)(*[t.shape[1] for t in ts])
        bonds = (c_int * (L + 1))(*([t.shape[0] for t in ts] + [ts[-1].shape[2]]))
        ptrs = (c_void_p * L)(*[t.data_ptr() for t in ts])
        h = c_void_p()
        self._check(self.lib.smps_mps_create_device(self.h, L, phys, bonds, dt, ptrs, byref(h)))
        return MPS(self, h)

    def mpo_create(self, tensors, dtype=np.float64) -> MPO:
        arrs = [np.ascontiguousarray(t, dtype=dtype) for t in tensors]
        L = len(arrs)
        pout = (c_int * L)(*[a.shape[1] for a in arrs])
        pin = (c_int * L)(*[a.shape[2] for a in arrs])
        bonds = (c_int * (L + 1))(*([a.shape[0] for a in arrs] + [arrs[-1].shape[3]]))
        ptrs = (c_void_p * L)(*[a.ctypes.data for a in arrs])
        h = c_void_p()
        self._check(self.lib.smps_mpo_create(self.h, L, pout, pin, bonds, F64 if dtype == np.float64 else F32, ptrs,
                                             byref(h)))
        return MPO(self, h, L)

    # ---- the hot path
    def mpo_apply(self, U: MPO, v: MPS, st: Strategy):
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_mpo_apply(self.h, U.h, v.h, byref(st), byref(out), byref(err)))
        return MPS(self, out), err.value

    def simplify(self, v: MPS, st: Strategy):
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_simplify(self.h, v.h, byref(st), byref(out), byref(err)))
        return MPS(self, out), err.value

    def combine(self, terms, st: Strategy):
        """Compress sum_l w_l U_l v_l; terms = [(w, MPO or None, MPS)]."""
        n = len(terms)
        w = (c_double * n)(*[float(t[0]) for t in terms])
        U = (c_void_p * n)(*[t[1].h if t[1] is not None else None for t in terms])
        v = (c_void_p * n)(*[t[2].h for t in terms])
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_combine(self.h, n, w, U, v, byref(st), byref(out), byref(err)))
        return MPS(self, out), err.value

    def mpo_transpose(self, U: "MPO") -> "MPO":
        out = c_void_p()
        self._check(self.lib.smps_mpo_transpose(self.h, U.h, byref(out)))
        return MPO(self, out, U.L)

    def mpo_apply_right(self, v: "MPS", U: "MPO", st: Strategy):
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_mpo_apply_right(self.h, v.h, U.h, byref(st), byref(out), byref(err)))
        return MPS(self, out), err.value

    def mpo_list_apply(self, Us, v: "MPS", st: Strategy):
        n = len(Us)
        uh = (c_void_p * n)(*[u.h for u in Us])
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_mpo_list_apply(self.h, n, uh, v.h, byref(st), byref(out), byref(err)))
        return MPS(self, out), err.value

    def mpo_simplify(self, U: "MPO", st: Strategy):
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_mpo_simplify(self.h, U.h, byref(st), byref(out), byref(err)))
        return MPO(self, out, U.L), err.value

    def dmrg(self, H: "MPO", guess: MPS, st: Strategy, krylov_dim: int = 24):
        """Two-site DMRG ground-state search (Sec. 3.1.1); returns (state, energy)."""
        out = c_void_p()
        e = c_double()
        self._check(self.lib.smps_dmrg(self.h, H.h, guess.h, byref(st), int(krylov_dim), byref(out), byref(e)))
        return MPS(self, out), e.value

    # ---- complex states and operators (interleaved complex128 on the host side)
    def zmps_create(self, tensors) -> "ZMPS":
        arrs = [np.ascontiguousarray(t, dtype=np.complex128) for t in tensors]
        L = len(arrs)
        phys = (c_int * L)(*[a.shape[1] for a in arrs])
        bonds = (c_int * (L + 1))(*([arrs[0].shape[0]] + [a.shape[2] for a in arrs]))
        dpt = POINTER(c_double)
        ptrs = (dpt * L)(*[a.ctypes.data_as(dpt) for a in arrs])
        out = c_void_p()
        self._check(self.lib.smps_zmps_create(self.h, L, phys, bonds, ptrs, byref(out)))
        return ZMPS(self, out)

    def zmpo_create(self, tensors) -> "ZMPO":
        arrs = [np.ascontiguousarray(t, dtype=np.complex128) for t in tensors]
        L = len(arrs)
        pout = (c_int * L)(*[a.shape[1] for a in arrs])
        pin = (c_int * L)(*[a.shape[2] for a in arrs])
        bonds = (c_int * (L + 1))(*([arrs[0].shape[0]] + [a.shape[3] for a in arrs]))
        dpt = POINTER(c_double)
        ptrs = (dpt * L)(*[a.ctypes.data_as(dpt) for a in arrs])
        out = c_void_p()
        self._check(self.lib.smps_zmpo_create(self.h, L, pout, pin, bonds, ptrs, byref(out)))
        return ZMPO(self, out)

    def zmpo_apply(self, U: "ZMPO", v: "ZMPS", st: Strategy):
        out = c_void_p()
        err = c_double()
        self._check(self.lib.smps_zmpo_apply(self.h, U.h, v.h, byref(st), byref(out), byref(err)))
        return ZMPS(self, out), err.value

    def zscprod(self, a: "ZMPS", b: "ZMPS") -> complex:
        re, im = c_double(), c_double()
        self._check(self.lib.smps_zscprod(self.h, a.h, b.h, byref(re), byref(im)))
        return complex(re.value, im.value)

    def mpo_apply_batched(self, Us, vs, st: Strategy, max_bonds=None):
        """Batched apply; max_bonds (one cap per problem) replaces st.max_bond."""
        n = len(vs)
        uh = (c_void_p * n)(*[u.h for u in Us])
        vh = (c_void_p * n)(*[v.h for v in vs])
        outs = (c_void_p * n)()
        errs = (c_double * n)()
        if max_bonds is None:
            rc = self.lib.smps_mpo_apply_batched(self.h, n, uh, vh, byref(st), outs, errs)
        else:
            caps = (c_int * n)(*[int(x) for x in max_bonds])
            rc = self.lib.smps_mpo_apply_batched_caps(self.h, n, uh, vh, caps, byref(st), outs, errs)
        self._check(rc)
        return [MPS(self, c_void_p(outs[i])) for i in range(n)], list(errs)

    def scprod(self, a: MPS, b: MPS) -> float:
        r = c_double()
        self._check(self.lib.smps_scprod(self.h, a.h, b.h, byref(r)))
        return r.value

    def scprod_noalloc(self, a: MPS, b: MPS, out_dev_ptr: int) -> None:
        """<a|b> into the device double at out_dev_ptr (stream-ordered, no sync)."""
        self._check(self.lib.smps_scprod_noalloc(self.h, a.h, b.h, c_void_p(out_dev_ptr)))

    def norm(self, a: MPS) -> float:
        r = c_double()
        self._check(self.lib.smps_norm(self.h, a.h, byref(r)))
        return r.value

    def last_info(self) -> dict:
        info = ApplyInfo()
        self._check(self.lib.smps_last_info(self.h, byref(info)))
        return {f: getattr(info, f) for f, _ in ApplyInfo._fields_}

    def last_log(self):
        n = c_int()
        self._check(self.lib.smps_last_log(self.h, 0, None, None, None, byref(n)))
        m = n.value
        deltas = np.zeros(m)
        ranks = np.zeros(m, dtype=np.int32)
        spec = np.zeros((m, 32))
        self._check(self.lib.smps_last_log(self.h, m, deltas.ctypes.data_as(POINTER(c_double)),
                                           ranks.ctypes.data_as(POINTER(c_int)),
                                           spec.ctypes.data_as(POINTER(c_double)), byref(n)))
        return deltas, ranks, spec

    def last_jacobi_log(self) -> list:
        """Rotating Jacobi sweeps of each step's exact factorization in the last apply."""
        n = c_int()
        self._check(self.lib.smps_last_jacobi_log(self.h, 0, None, byref(n)))
        out = (c_int * max(1, n.value))()
        self._check(self.lib.smps_last_jacobi_log(self.h, n.value, out, byref(n)))
        return list(out)[:n.value]

    def last_factor_log(self) -> np.ndarray:
        n = c_int()
        self._check(self.lib.smps_last_factor_log(self.h, 0, None, byref(n)))
        kinds = np.zeros(n.value, dtype=np.int32)
        self._check(self.lib.smps_last_factor_log(self.h, n.value, kinds.ctypes.data_as(POINTER(c_int)), byref(n)))
        return kinds

    def set_profiling(self, on: bool):
        self._check(self.lib.smps_ctx_set_profiling(self.h, 1 if on else 0))

    def kernel_time(self, category: int = 0):
        """(total milliseconds, launches) of timed launches of a category since
        profiling was enabled: 0 factorizations, 1 contractions, 2 bulk splits,
        3 X tensors, 4 theta products, 5 environment updates, 6 other launches."""
        ms = c_double()
        n = ctypes.c_longlong()
        self._check(self.lib.smps_ctx_kernel_time(self.h, int(category), byref(ms), byref(n)))
        return ms.value, n.value

    def set_split(self, method: str) -> None:
        """'auto' (the library's choice), 'jacobi' or 'gram' (Gram / tridiagonal split for short vectors)."""
        self._check(self.lib.smps_ctx_set_split(self.h, {"auto": 0, "jacobi": 1, "gram": 2}[method]))

    def set_workspace_limit(self, nbytes: int) -> None:
        """Upper bound on the workspace arena (0: none); larger calls fail with ENOMEM."""
        self._check(self.lib.smps_ctx_set_workspace_limit(self.h, int(nbytes)))

    def plan_apply(self, U: MPO, v: MPS, st: Strategy) -> dict:
        """What mpo_apply would allocate and enqueue (host only).  On a refusal
        the SmpsError carries the filled sizes in .info."""
        info = PlanInfo()
        rc = self.lib.smps_plan_apply(self.h, U.h, v.h, byref(st), byref(info))
        if rc != OK:
            raise SmpsError(rc, self.lib.smps_last_error(self.h).decode(), info.as_dict())
        return info.as_dict()

    def plan_apply_batched(self, Us, vs, st: Strategy, max_bonds=None) -> dict:
        n = len(vs)
        uh = (c_void_p * n)(*[u.h for u in Us])
        vh = (c_void_p * n)(*[v.h for v in vs])
        caps = None if max_bonds is None else (c_int * n)(*[int(x) for x in max_bonds])
        info = PlanInfo()
        rc = self.lib.smps_plan_apply_batched(self.h, n, uh, vh, caps, byref(st), byref(info))
        if rc != OK:
            raise SmpsError(rc, self.lib.smps_last_error(self.h).decode(), info.as_dict())
        return info.as_dict()

    def workspace_bytes(self) -> int:
        b = c_size_t()
        self._check(self.lib.smps_ctx_workspace_bytes(self.h, byref(b)))
        return b.value

    # ---- rank predictor
    def rank_mlp_init(self, seed: int = 0):
        self._check(self.lib.smps_rank_mlp_init(self.h, c_ulonglong(seed)))

    def rank_mlp_train(self, feats, labels, epochs: int, batch: int, lr: float) -> float:
        f = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        loss = c_float()
        self._check(self.lib.smps_rank_mlp_train(self.h, len(y), _fptr(f), _fptr(y), int(epochs), int(batch),
                                                 float(lr), byref(loss)))
        return loss.value

    def rank_mlp_predict(self, feats) -> np.ndarray:
        f = np.ascontiguousarray(feats, dtype=np.float32)
        out = np.zeros(f.shape[0], dtype=np.float32)
        self._check(self.lib.smps_rank_mlp_predict(self.h, f.shape[0], _fptr(f), _fptr(out)))
        return out

    def rank_mlp_get(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(self.lib.smps_rank_mlp_get(self.h, _fptr(p), MLP_PARAMS))
        return p

    def rank_mlp_set(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.smps_rank_mlp_set(self.h, _fptr(p), p.size))

    # ---- GEMM tile autotuner
    def autotune_apply(self, U: "MPO", v: "MPS", st: Strategy, reps: int = 5) -> int:
        n = c_int()
        self._check(self.lib.smps_autotune_apply(self.h, U.h, v.h, byref(st), int(reps), byref(n)))
        return n.value

    def autotune_gemm(self, precision, M, N, K, ta=0, tb=0, tc=0, a_type=0, b_type=0, c_type=0, reps=5) -> int:
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        best = c_int()
        self._check(self.lib.smps_autotune_gemm(self.h, prec, M, N, K, ta, tb, tc, a_type, b_type, c_type, reps,
                                                byref(best)))
        return best.value

    def autotune_save(self, path: str):
        self._check(self.lib.smps_autotune_save(self.h, str(path).encode()))

    def autotune_load(self, path: str):
        self._check(self.lib.smps_autotune_load(self.h, str(path).encode()))

    def autotune_clear(self):
        self._check(self.lib.smps_autotune_clear(self.h))

    def autotune_entries(self) -> int:
        n = c_int()
        self._check(self.lib.smps_autotune_entries(self.h, byref(n)))
        return n.value

    def rank_training_pairs(self):
        n = c_int()
        self._check(self.lib.smps_rank_training_pairs(self.h, 0, None, None, byref(n)))
        f = np.zeros((n.value, 32), dtype=np.float32)
        y = np.zeros(n.value, dtype=np.float32)
        self._check(self.lib.smps_rank_training_pairs(self.h, n.value, _fptr(f), _fptr(y), byref(n)))
        return f, y

    def rank_mlp_grad(self, feats, labels):
        f = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(labels, dtype=np.float32)
        loss = c_float()
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._check(self.lib.smps_rank_mlp_grad(self.h, len(y), _fptr(f), _fptr(y), byref(loss), _fptr(g), g.size))
        return loss.value, g


# names of the boundary, as module-level calls on a context
def mps_create(ctx: Context, tensors, dtype=np.float64) -> MPS:
    return ctx.mps_create(tensors, dtype)


def mpo_create(ctx: Context, tensors, dtype=np.float64) -> MPO:
    return ctx.mpo_create(tensors, dtype)


def mpo_apply(ctx: Context, U: MPO, v: MPS, st: Strategy):
    return ctx.mpo_apply(U, v, st)


def simplify(ctx: Context, v: MPS, st: Strategy):
    return ctx.simplify(v, st)


def scprod(ctx: Context, a: MPS, b: MPS) -> float:
    return ctx.scprod(a, b)


def norm(ctx: Context, a: MPS) -> float:
    return ctx.norm(a)
