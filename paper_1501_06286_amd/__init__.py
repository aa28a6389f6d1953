"""Fast QMC matrix products on AMD MI355X (gfx950).

X = Y A for QMC point matrices Y (rank-1 lattice rules with prime N, and
polynomial lattice rules over GF(2) with N = 2^m), computed through the
circulant factorisation of Dick, Kuo, Le Gia and Schwab (Section 2.1,
eq. (ZPa); Remark 1) without forming Y.

This module is argument marshalling only: every step runs in the HIP library
``libqmcfast.so`` built from ``csrc/`` (see ``build.py``).  PyTorch provides
device memory and streams.  There is no CPU fallback: if the library is
missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqmcfast.so")

RULE_LATTICE = 0
RULE_POLY_GF2 = 1
PHI_IDENTITY = 0
PHI_CENTERED = 1
PHI_INVNORM = 2
PHI_TENT = 3
F32 = 0
F64 = 1

EXPORTED = [
    "qmc_plan_create", "qmc_plan_destroy", "qmc_plan_info", "qmc_plan_tables",
    "qmc_workspace_size", "qmc_matmul", "qmc_matmul_epilogue", "qmc_matmul_adjoint",
    "qmc_explicit_points",
    "qmc_dense_matmul", "qmc_batched_workspace_size", "qmc_matmul_batched", "qmc_strerror",
    "qmc_profile_enable", "qmc_profile_collect", "qmc_profile_slot_name",
    "qmc_plan_set_tuning", "qmc_plan_get_tuning", "qmc_plan_set_row_order",
    "qmc_batch_create", "qmc_batch_set_chunk", "qmc_batch_set_epilogue",
    "qmc_batch_workspace_size", "qmc_batch_run",
    "qmc_batch_destroy",
    "qmc_korobov_create", "qmc_korobov_destroy", "qmc_korobov_info", "qmc_korobov_set_chunk",
    "qmc_korobov_workspace_size", "qmc_korobov_plan", "qmc_korobov_matmul",
    "qmc_korobov_matmul_epilogue", "qmc_korobov_matmul_adjoint", "qmc_matmul_noalloc",
]
PROF_SLOTS = 10
BATCH_CHUNK_DEFAULT = 256 << 20  # QMC_BATCH_CHUNK_DEFAULT
ROWS_CONVENTIONAL, ROWS_GROUP = 0, 1


class QMCError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {lib().qmc_strerror(code).decode()} (code {code})")
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("chunk_pairs", ctypes.c_int64), ("streams", ctypes.c_int), ("nt_store", ctypes.c_int),
                ("front", ctypes.c_int), ("outer_q", ctypes.c_int), ("nt_inter", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("s", ctypes.c_int64), ("L", ctypes.c_int64),
                ("M", ctypes.c_int64), ("M1", ctypes.c_int64), ("M2", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("beta", ctypes.c_uint64),
                ("rule", ctypes.c_int), ("phi_kind", ctypes.c_int), ("dtype", ctypes.c_int),
                ("embedded", ctypes.c_int), ("phi0", ctypes.c_double), ("P2", ctypes.c_int),
                ("Q2", ctypes.c_int), ("blocks", ctypes.c_int64), ("direct_rows", ctypes.c_int64)]


class KorobovInfo(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("s", ctypes.c_int64), ("N", ctypes.c_int64),
                ("L", ctypes.c_int64), ("M", ctypes.c_int64), ("M1", ctypes.c_int64),
                ("M2", ctypes.c_int64), ("blocks", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("beta", ctypes.c_uint64), ("phi_kind", ctypes.c_int), ("dtype", ctypes.c_int),
                ("chunk_blocks", ctypes.c_int64)]


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libqmcfast.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_1501_06286_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i64, u64, vp, ip = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        sz = ctypes.c_size_t
        L.qmc_plan_create.argtypes = [ctypes.POINTER(vp), ip, i64, i64, ctypes.POINTER(u64), u64,
                                      ip, i64, i64, ip, vp]
        L.qmc_plan_destroy.argtypes = [vp]
        L.qmc_plan_destroy.restype = None
        L.qmc_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        pi32 = ctypes.POINTER(ctypes.c_int32)
        L.qmc_plan_tables.argtypes = [vp, pi32, pi32, pi32, ctypes.POINTER(ctypes.c_double)]
        L.qmc_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
        L.qmc_matmul.argtypes = [vp, vp, i64, i64, vp, i64, vp, sz, vp]
        L.qmc_matmul_adjoint.argtypes = [vp, vp, i64, i64, vp, i64, vp, sz, vp]
        L.qmc_matmul_noalloc.argtypes = [vp, vp, i64, i64, vp, i64, vp]
        L.qmc_matmul_epilogue.argtypes = [vp, vp, i64, i64, vp, i64, ip, vp, vp, vp, sz, vp]
        L.qmc_explicit_points.argtypes = [vp, vp, i64, vp]
        L.qmc_dense_matmul.argtypes = [vp, vp, i64, vp, i64, i64, vp, i64, vp]
        L.qmc_batched_workspace_size.argtypes = [ip, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                                 ctypes.POINTER(sz)]
        L.qmc_matmul_batched.argtypes = [ip, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(i64), ctypes.POINTER(vp), vp, sz, vp]
        L.qmc_strerror.argtypes = [ip]
        L.qmc_strerror.restype = ctypes.c_char_p
        L.qmc_batch_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), vp]
        L.qmc_batch_set_chunk.argtypes = [vp, i64, ip, vp]
        L.qmc_batch_set_epilogue.argtypes = [vp, ip, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.qmc_batch_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
        L.qmc_batch_run.argtypes = [vp, vp, sz, vp]
        L.qmc_batch_destroy.argtypes = [vp]
        L.qmc_batch_destroy.restype = None
        L.qmc_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.qmc_plan_set_row_order.argtypes = [vp, ip]
        L.qmc_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.qmc_profile_enable.argtypes = [vp, ip]
        L.qmc_profile_collect.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.qmc_profile_slot_name.argtypes = [ip]
        L.qmc_profile_slot_name.restype = ctypes.c_char_p
        L.qmc_korobov_create.argtypes = [ctypes.POINTER(vp), i64, i64, ip, i64, i64, ip, vp]
        L.qmc_korobov_destroy.argtypes = [vp]
        L.qmc_korobov_destroy.restype = None
        L.qmc_korobov_info.argtypes = [vp, ctypes.POINTER(KorobovInfo)]
        L.qmc_korobov_set_chunk.argtypes = [vp, i64]
        L.qmc_korobov_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
        L.qmc_korobov_plan.argtypes = [vp]
        L.qmc_korobov_plan.restype = vp
        L.qmc_korobov_matmul.argtypes = [vp, vp, i64, i64, vp, i64, vp, sz, vp]
        L.qmc_korobov_matmul_epilogue.argtypes = [vp, vp, i64, i64, vp, i64, ip, vp, vp, vp, sz,
                                                  vp]
        L.qmc_korobov_matmul_adjoint.argtypes = [vp, vp, i64, i64, vp, i64, vp, sz, vp]
        for name in EXPORTED:
            if name not in ("qmc_plan_destroy", "qmc_strerror", "qmc_profile_slot_name",
                            "qmc_batch_destroy", "qmc_korobov_destroy", "qmc_korobov_plan"):
                getattr(L, name).restype = ip
        _LIB = L
    return _LIB


def _check(code: int, where: str) -> None:
    if code != 0:
        raise QMCError(code, where)


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> Optional[int]:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(dtype) -> int:
    torch = _torch()
    if dtype in ("f32", "float32", torch.float32, F32):
        return F32
    if dtype in ("f64", "float64", torch.float64, F64):
        return F64
    raise ValueError(f"unsupported dtype {dtype}")


class Plan:
    """Everything that depends only on the point set (Section 2.1): primitive
    element, exponents l_j, phi table, generator spectrum, schedules."""

    def __init__(self, rule: int, N: int, gen, phi: int = PHI_IDENTITY,
                 shift: Tuple[int, int] = (0, 1), dtype="f32", modulus: int = 0,
                 stream=None):
        gen = np.ascontiguousarray(np.asarray(gen, dtype=np.uint64))
        self.rule, self.N, self.s = int(rule), int(N), int(gen.shape[0])
        self.phi, self.shift, self.modulus = int(phi), (int(shift[0]), int(shift[1])), int(modulus)
        self.dtype_code = _dtype_code(dtype)
        torch = _torch()
        self.torch_dtype = torch.float32 if self.dtype_code == F32 else torch.float64
        handle = ctypes.c_void_p()
        code = lib().qmc_plan_create(
            ctypes.byref(handle), self.rule, self.N, self.s,
            gen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), self.modulus, self.phi,
            self.shift[0], self.shift[1], self.dtype_code, _stream_handle(stream))
        _check(code, "qmc_plan_create")
        self._h = handle
        self._owned = True
        self._ws = None

    @classmethod
    def from_instance(cls, inst, dtype=None, stream=None) -> "Plan":
        return cls(inst.rule, inst.N, inst.gen, inst.phi, inst.shift,
                   dtype or inst.dtype, inst.modulus, stream)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            if getattr(self, "_owned", True):
                lib().qmc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().qmc_plan_info(self.handle, ctypes.byref(inf)), "qmc_plan_info")
        return {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    def tables(self):
        """(pow, log, ell, phi) copied to host numpy arrays (bit-exact tables)."""
        inf = self.info()
        L, N, s = inf["L"], inf["N"], inf["s"]
        pw = np.empty(L, dtype=np.int32)
        lg = np.empty(N, dtype=np.int32)
        el = np.empty(s, dtype=np.int32)
        ph = np.empty(N, dtype=np.float64)
        p32 = ctypes.POINTER(ctypes.c_int32)
        _check(lib().qmc_plan_tables(self.handle, pw.ctypes.data_as(p32), lg.ctypes.data_as(p32),
                                     el.ctypes.data_as(p32),
                                     ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "qmc_plan_tables")
        return pw, lg, el, ph

    def set_tuning(self, chunk_pairs: int = 0, streams: int = 1, nt_store: int = 0,
                   front: int = 0, outer_q: int = 0, nt_inter: int = 0) -> None:
        """Launch tuning (see autotune.py); changes the workspace size."""
        tu = Tuning(int(chunk_pairs), int(streams), int(nt_store), int(front), int(outer_q),
                    int(nt_inter))
        _check(lib().qmc_plan_set_tuning(self.handle, ctypes.byref(tu)), "qmc_plan_set_tuning")

    def set_row_order(self, order: int) -> None:
        """ROWS_CONVENTIONAL (row n = point n) or ROWS_GROUP (row 1 + e = the
        point of beta^e) for X and, in the adjoint, G."""
        _check(lib().qmc_plan_set_row_order(self.handle, int(order)), "qmc_plan_set_row_order")

    def get_tuning(self) -> dict:
        tu = Tuning()
        _check(lib().qmc_plan_get_tuning(self.handle, ctypes.byref(tu)), "qmc_plan_get_tuning")
        return {"chunk_pairs": tu.chunk_pairs, "streams": tu.streams, "nt_store": tu.nt_store,
                "front": tu.front, "outer_q": tu.outer_q, "nt_inter": tu.nt_inter}

    def profile(self, on: bool = True) -> None:
        """Bracket every kernel launch of this plan with HIP events."""
        _check(lib().qmc_profile_enable(self.handle, 1 if on else 0), "qmc_profile_enable")

    def profile_collect(self) -> dict:
        """{kernel: (total_ms, launches)} since the last collect (waits for the events)."""
        ms = (ctypes.c_double * PROF_SLOTS)()
        n = (ctypes.c_int64 * PROF_SLOTS)()
        _check(lib().qmc_profile_collect(self.handle, ms, n), "qmc_profile_collect")
        out = {}
        for k in range(PROF_SLOTS):
            if n[k]:
                out[lib().qmc_profile_slot_name(k).decode()] = (float(ms[k]), int(n[k]))
        return out

    def workspace_bytes(self, t: int) -> int:
        n = ctypes.c_size_t()
        _check(lib().qmc_workspace_size(self.handle, int(t), ctypes.byref(n)), "qmc_workspace_size")
        return int(n.value)

    def workspace(self, t: int, device=None):
        """A cached device workspace large enough for t columns."""
        torch = _torch()
        need = self.workspace_bytes(t)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device or "cuda")
        return self._ws


def _check_tensor(x, plan: Plan, rows: int, name: str):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != plan.torch_dtype:
        raise TypeError(f"{name} has dtype {x.dtype}, plan computes in {plan.torch_dtype}")
    if x.dim() != 2 or x.shape[0] != rows or x.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major {rows} x t matrix (unit column stride)")


EPILOGUES = {None: 0, "none": 0, "affine": 1, "exp": 2}


def _vec_ptr(v, plan: Plan, t: int, name: str):
    if v is None:
        return None
    torch = _torch()
    if not isinstance(v, torch.Tensor) or not v.is_cuda or v.dtype != plan.torch_dtype:
        raise TypeError(f"{name} must be a CUDA tensor of the plan dtype")
    if v.dim() != 1 or v.shape[0] != t or v.stride(0) != 1:
        raise ValueError(f"{name} must be a contiguous vector of t = {t} entries")
    return ctypes.c_void_p(v.data_ptr())


def matmul(plan: Plan, A, out=None, workspace=None, stream=None, epilogue=None, bias=None,
           scale=None):
    """X = Y A (N x t) on the GPU.  epilogue "affine": X = scale * (bias + Y A),
    "exp": X = scale * exp(bias + Y A), per column (Sections 3.2, 3.3)."""
    torch = _torch()
    _check_tensor(A, plan, plan.s, "A")
    t = A.shape[1]
    X = torch.empty((plan.N, t), dtype=A.dtype, device=A.device) if out is None else out
    _check_tensor(X, plan, plan.N, "out")
    ws = plan.workspace(t, A.device) if workspace is None else workspace
    kind = EPILOGUES[epilogue]
    if kind == 0 and bias is None and scale is None:
        _check(lib().qmc_matmul(plan.handle, ctypes.c_void_p(A.data_ptr()), t, A.stride(0),
                                ctypes.c_void_p(X.data_ptr()), X.stride(0),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                _stream_handle(stream)), "qmc_matmul")
        return X
    _check(lib().qmc_matmul_epilogue(plan.handle, ctypes.c_void_p(A.data_ptr()), t, A.stride(0),
                                     ctypes.c_void_p(X.data_ptr()), X.stride(0), kind,
                                     _vec_ptr(bias, plan, t, "bias"),
                                     _vec_ptr(scale, plan, t, "scale"),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                     _stream_handle(stream)), "qmc_matmul_epilogue")
    return X


def matmul_noalloc(plan: Plan, A, out, stream=None):
    """X = Y A into the preallocated `out` through qmc_matmul_noalloc: the
    library's static device scratch serves as workspace, nothing is allocated
    (same result as matmul)."""
    _check_tensor(A, plan, plan.s, "A")
    _check_tensor(out, plan, plan.N, "out")
    t = A.shape[1]
    if out.shape[1] != t:
        raise ValueError(f"out has {out.shape[1]} columns, A has {t}")
    _check(lib().qmc_matmul_noalloc(plan.handle, ctypes.c_void_p(A.data_ptr()), t, A.stride(0),
                                    ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                    _stream_handle(stream)), "qmc_matmul_noalloc")
    return out


def matmul_adjoint(plan: Plan, G, out=None, workspace=None, stream=None):
    """dA = Y^T G (s x t) on the GPU."""
    torch = _torch()
    _check_tensor(G, plan, plan.N, "G")
    t = G.shape[1]
    dA = torch.empty((plan.s, t), dtype=G.dtype, device=G.device) if out is None else out
    _check_tensor(dA, plan, plan.s, "out")
    ws = plan.workspace(t, G.device) if workspace is None else workspace
    _check(lib().qmc_matmul_adjoint(plan.handle, ctypes.c_void_p(G.data_ptr()), t, G.stride(0),
                                    ctypes.c_void_p(dA.data_ptr()), dA.stride(0),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                    _stream_handle(stream)), "qmc_matmul_adjoint")
    return dA


def explicit_points(plan: Plan, out=None, stream=None):
    """The N x s point matrix Y itself (conventional order), built on the GPU."""
    torch = _torch()
    Y = torch.empty((plan.N, plan.s), dtype=plan.torch_dtype, device="cuda") if out is None else out
    _check(lib().qmc_explicit_points(plan.handle, ctypes.c_void_p(Y.data_ptr()), Y.stride(0),
                                     _stream_handle(stream)), "qmc_explicit_points")
    return Y


def dense_matmul(plan: Plan, Y, A, out=None, stream=None):
    """The standard approach: X = Y A with an explicit Y, on the MFMA cores."""
    torch = _torch()
    _check_tensor(Y, plan, plan.N, "Y")
    _check_tensor(A, plan, plan.s, "A")
    t = A.shape[1]
    X = torch.empty((plan.N, t), dtype=A.dtype, device=A.device) if out is None else out
    _check(lib().qmc_dense_matmul(plan.handle, ctypes.c_void_p(Y.data_ptr()), Y.stride(0),
                                  ctypes.c_void_p(A.data_ptr()), t, A.stride(0),
                                  ctypes.c_void_p(X.data_ptr()), X.stride(0),
                                  _stream_handle(stream)), "qmc_dense_matmul")
    return X


def batched_workspace_bytes(plans: Sequence[Plan], ts: Sequence[int]) -> int:
    n = len(plans)
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    tt = (ctypes.c_int64 * n)(*[int(t) for t in ts])
    out = ctypes.c_size_t()
    _check(lib().qmc_batched_workspace_size(n, hs, tt, ctypes.byref(out)),
           "qmc_batched_workspace_size")
    return int(out.value)


def matmul_batched(plans: Sequence[Plan], As: Sequence, outs: Optional[Sequence] = None,
                   workspace=None, stream=None) -> List:
    """X_i = Y_i A_i for many plans in one call (dense row-major A_i, X_i)."""
    torch = _torch()
    n = len(plans)
    Xs = []
    for i, (p, A) in enumerate(zip(plans, As)):
        _check_tensor(A, p, p.s, f"A[{i}]")
        if A.stride(0) != A.shape[1]:
            raise ValueError("batched inputs must be dense row-major")
        X = torch.empty((p.N, A.shape[1]), dtype=A.dtype, device=A.device) if outs is None else outs[i]
        Xs.append(X)
    ts = [A.shape[1] for A in As]
    need = batched_workspace_bytes(plans, ts)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda") if workspace is None else workspace
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    ap = (ctypes.c_void_p * n)(*[A.data_ptr() for A in As])
    xp = (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])
    tt = (ctypes.c_int64 * n)(*ts)
    _check(lib().qmc_matmul_batched(n, hs, ap, tt, xp, ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel(), _stream_handle(stream)), "qmc_matmul_batched")
    return Xs


class Batch:
    """Many products X_i = Y_i A_i bound once; run() is, per run of products
    sized to the Infinity Cache, one persistent launch of each pass over the
    run (per transform size and radix where the kernels differ) and can be
    captured in a graph (torch.cuda.graph) and replayed.  The plans and
    tensors must stay alive."""

    def __init__(self, plans: Sequence[Plan], As: Sequence, Xs: Optional[Sequence] = None,
                 stream=None, chunk_bytes: Optional[int] = None):
        torch = _torch()
        self.plans = list(plans)
        self.As = list(As)
        if Xs is None:
            Xs = [torch.empty((p.N, A.shape[1]), dtype=A.dtype, device=A.device)
                  for p, A in zip(self.plans, self.As)]
        self.Xs = list(Xs)
        n = len(self.plans)
        for i, (p, A, X) in enumerate(zip(self.plans, self.As, self.Xs)):
            _check_tensor(A, p, p.s, f"A[{i}]")
            _check_tensor(X, p, p.N, f"X[{i}]")
            if X.shape[1] != A.shape[1]:
                raise ValueError(f"X[{i}] and A[{i}] column counts differ")
        hs = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        tt = (ctypes.c_int64 * n)(*[A.shape[1] for A in self.As])
        ap = (ctypes.c_void_p * n)(*[A.data_ptr() for A in self.As])
        la = (ctypes.c_int64 * n)(*[A.stride(0) for A in self.As])
        xp = (ctypes.c_void_p * n)(*[X.data_ptr() for X in self.Xs])
        lx = (ctypes.c_int64 * n)(*[X.stride(0) for X in self.Xs])
        h = ctypes.c_void_p()
        _check(lib().qmc_batch_create(ctypes.byref(h), n, hs, tt, ap, la, xp, lx,
                                      _stream_handle(stream)), "qmc_batch_create")
        self._h = h
        self._stream = stream
        if chunk_bytes is not None:
            self.set_chunk(chunk_bytes)
        else:
            self._alloc_workspace()

    def _alloc_workspace(self) -> None:
        torch = _torch()
        nb = ctypes.c_size_t()
        _check(lib().qmc_batch_workspace_size(self._h, ctypes.byref(nb)),
               "qmc_batch_workspace_size")
        self.workspace = torch.empty(max(1, nb.value), dtype=torch.uint8, device="cuda")

    def set_chunk(self, chunk_bytes: int, nt_inter: int = 0) -> None:
        """Runs of products whose intermediates take at most chunk_bytes
        together (0: one run per layout group), with cached (1), streaming (2)
        or automatic (0) stores of the intermediates; reallocates the
        workspace."""
        _check(lib().qmc_batch_set_chunk(self._h, int(chunk_bytes), int(nt_inter),
                                         _stream_handle(self._stream)), "qmc_batch_set_chunk")
        self._alloc_workspace()

    def set_epilogue(self, epilogue, biases=None, scales=None) -> None:
        """One epilogue kind ("affine", "exp" or None) for every product, with
        per-product bias and scale vectors (device tensors of t_i values, or
        None); the vectors must stay alive while the batch is run."""
        kind = EPILOGUES[epilogue]
        n = len(self.plans)

        def ptrs(vs, what):
            if vs is None:
                return None
            out = []
            for i, (v, p, A) in enumerate(zip(vs, self.plans, self.As)):
                out.append(None if v is None else _vec_ptr(v, p, A.shape[1], f"{what}[{i}]").value)
            return (ctypes.c_void_p * n)(*out)

        self._epi = (biases, scales)  # keep the vectors referenced
        _check(lib().qmc_batch_set_epilogue(self._h, kind, ptrs(biases, "bias"),
                                            ptrs(scales, "scale"), _stream_handle(self._stream)),
               "qmc_batch_set_epilogue")

    def run(self, stream=None) -> List:
        _check(lib().qmc_batch_run(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                   self.workspace.numel(), _stream_handle(stream)), "qmc_batch_run")
        return self.Xs

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().qmc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class KorobovUnion:
    """The union of all Korobov lattice point sets with a prime K (Section 2.2):
    N = (K-1)^2 points x_{b,n} = ({n b^j / K + Delta})_{j < s}, b, n = 1..K-1,
    row (b-1)(K-1) + (n-1).  The K-1 blocks share one generator spectrum."""

    def __init__(self, K: int, s: int, phi: int = PHI_INVNORM,
                 shift: Tuple[int, int] = (0, 1), dtype="f32", stream=None):
        self.K, self.s = int(K), int(s)
        self.N = (self.K - 1) ** 2
        self.phi, self.shift = int(phi), (int(shift[0]), int(shift[1]))
        self.dtype_code = _dtype_code(dtype)
        torch = _torch()
        self.torch_dtype = torch.float32 if self.dtype_code == F32 else torch.float64
        h = ctypes.c_void_p()
        _check(lib().qmc_korobov_create(ctypes.byref(h), self.K, self.s, self.phi, self.shift[0],
                                        self.shift[1], self.dtype_code, _stream_handle(stream)),
               "qmc_korobov_create")
        self._h = h
        self._ws = None
        # the shared lattice plan of K points (owned by the union)
        base = Plan.__new__(Plan)
        base.rule, base.N, base.s = RULE_LATTICE, self.K, self.s
        base.phi, base.shift, base.modulus = self.phi, self.shift, 0
        base.dtype_code, base.torch_dtype = self.dtype_code, self.torch_dtype
        base._h = ctypes.c_void_p(lib().qmc_korobov_plan(h))
        base._owned = False
        base._ws = None
        self.plan = base

    @classmethod
    def from_instance(cls, inst, dtype=None, stream=None) -> "KorobovUnion":
        return cls(inst.modulus, inst.s, inst.phi, inst.shift, dtype or inst.dtype, stream)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("union plan destroyed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            self.plan._h = None
            lib().qmc_korobov_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = KorobovInfo()
        _check(lib().qmc_korobov_info(self.handle, ctypes.byref(inf)), "qmc_korobov_info")
        return {k: getattr(inf, k) for k, _ in KorobovInfo._fields_}

    def set_chunk(self, blocks: int) -> None:
        """Blocks per run of the passes (0: all); changes the workspace size."""
        _check(lib().qmc_korobov_set_chunk(self.handle, int(blocks)), "qmc_korobov_set_chunk")

    def workspace_bytes(self, t: int) -> int:
        n = ctypes.c_size_t()
        _check(lib().qmc_korobov_workspace_size(self.handle, int(t), ctypes.byref(n)),
               "qmc_korobov_workspace_size")
        return int(n.value)

    def workspace(self, t: int, device=None):
        torch = _torch()
        need = self.workspace_bytes(t)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device or "cuda")
        return self._ws


def korobov_matmul(U: KorobovUnion, A, out=None, workspace=None, stream=None, epilogue=None,
                   bias=None, scale=None):
    """X = Y A for the union of Korobov lattice point sets ((K-1)^2 x t), with
    the optional per-column epilogue of ``matmul``."""
    torch = _torch()
    _check_tensor(A, U, U.s, "A")
    t = A.shape[1]
    X = torch.empty((U.N, t), dtype=A.dtype, device=A.device) if out is None else out
    _check_tensor(X, U, U.N, "out")
    ws = U.workspace(t, A.device) if workspace is None else workspace
    kind = EPILOGUES[epilogue]
    _check(lib().qmc_korobov_matmul_epilogue(
        U.handle, ctypes.c_void_p(A.data_ptr()), t, A.stride(0), ctypes.c_void_p(X.data_ptr()),
        X.stride(0), kind, _vec_ptr(bias, U, t, "bias"), _vec_ptr(scale, U, t, "scale"),
        ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), _stream_handle(stream)),
        "qmc_korobov_matmul_epilogue")
    return X


def korobov_matmul_adjoint(U: KorobovUnion, G, out=None, workspace=None, stream=None):
    """dA = Y^T G for the union of Korobov lattice point sets (s x t)."""
    torch = _torch()
    _check_tensor(G, U, U.N, "G")
    t = G.shape[1]
    dA = torch.empty((U.s, t), dtype=G.dtype, device=G.device) if out is None else out
    _check_tensor(dA, U, U.s, "out")
    ws = U.workspace(t, G.device) if workspace is None else workspace
    _check(lib().qmc_korobov_matmul_adjoint(
        U.handle, ctypes.c_void_p(G.data_ptr()), t, G.stride(0), ctypes.c_void_p(dA.data_ptr()),
        dA.stride(0), ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
        _stream_handle(stream)), "qmc_korobov_matmul_adjoint")
    return dA


def _autograd():
    torch = _torch()

    class QMCMatmul(torch.autograd.Function):
        """X = Y A with dA = Y^T dX in backward (no gradient for the point set)."""

        @staticmethod
        def forward(ctx, A, plan):
            ctx.plan = plan
            return matmul(plan, A.contiguous())

        @staticmethod
        def backward(ctx, gX):
            return matmul_adjoint(ctx.plan, gX.contiguous()), None

    class KorobovMatmul(torch.autograd.Function):
        """The union's X = Y A with dA = Y^T dX in backward."""

        @staticmethod
        def forward(ctx, A, U):
            ctx.U = U
            return korobov_matmul(U, A.contiguous())

        @staticmethod
        def backward(ctx, gX):
            return korobov_matmul_adjoint(ctx.U, gX.contiguous()), None

    return QMCMatmul, KorobovMatmul


_QMC_FN = None


def qmc_matmul(A, plan: Plan):
    """Differentiable X = Y A (torch.autograd)."""
    global _QMC_FN
    if _QMC_FN is None:
        _QMC_FN = _autograd()
    return _QMC_FN[0].apply(A, plan)


def korobov_qmc_matmul(A, U: KorobovUnion):
    """Differentiable X = Y A for the union of Korobov lattice point sets."""
    global _QMC_FN
    if _QMC_FN is None:
        _QMC_FN = _autograd()
    return _QMC_FN[1].apply(A, U)
