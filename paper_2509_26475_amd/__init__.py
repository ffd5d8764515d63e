"""phicomb: linear combinations of phi-function actions on MI355X (gfx950).

Thin Python binding of ``libphicomb.so`` (C ABI in ``include/phicomb.h``).
Functions named ``phicomb_*`` mirror the C entry points one to one
(argument marshalling only: every step of the method runs in the HIP
library).  PyTorch provides device memory and the current HIP stream.

The method is the block truncated-Taylor scaling-and-recovering algorithm
of Al-Mohy, "Computing Linear Combinations of phi-Function Actions for
Exponential Integrators" (arXiv 2509.26475): Algorithm 1 chooses the shift
and scaling, Algorithm 3 evaluates w_i = sum_j beta_ij phi_j(t_i A) v_j.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphicomb.so")

OK, PENDING = 0, 1
EINVAL, ENOMEM, EADMIT, ENOCONV, EOVERFLOW, EDEVICE = -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
MAX_P, MAX_R, MAX_M = 7, 4, 100


class PhicombError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = _lib().phicomb_strerror(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{where}: status {status} ({msg})")


class ParamsT(C.Structure):
    _fields_ = [("shift", C.c_double), ("s0", C.c_double), ("zstar", C.c_double),
                ("fstar", C.c_double), ("s", C.c_double), ("tol", C.c_double),
                ("m", C.c_int32), ("r_acc", C.c_int32), ("n_feval", C.c_int32),
                ("status", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class StatsT(C.Structure):
    _fields_ = [("s_int", C.c_int32), ("terms_S", C.c_int32), ("terms_rec", C.c_int32),
                ("max_terms_step", C.c_int32), ("status", C.c_int32),
                ("fp32_terms", C.c_int32), ("bytes_alg", C.c_double), ("ms", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ExprkStatsT(C.Structure):
    _fields_ = [("steps", C.c_int32), ("calls", C.c_int32), ("max_s_int", C.c_int32),
                ("status", C.c_int32), ("terms", C.c_int64), ("fp32_terms", C.c_int64),
                ("ms", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchItemT(C.Structure):
    _fields_ = [("op", C.c_void_p), ("prm", C.POINTER(ParamsT)), ("p", C.c_int32),
                ("r", C.c_int32), ("t", C.c_void_p), ("beta", C.c_void_p), ("V", C.c_void_p),
                ("W", C.c_void_p), ("tol", C.c_double)]


_LIB = None


def _lib():
    """Load the HIP library; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2509_26475_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
        sig = {
            "phicomb_op_create_csr": ([I64, P, P, P, P], I32),
            "phicomb_op_create_stencil": ([I32, P, P, D, P], I32),
            "phicomb_op_create_dense": ([I64, P, P], I32),
            "phicomb_op_create_lowrank": ([I64, I32, P, P, P], I32),
            "phicomb_op_destroy": ([P], I32),
            "phicomb_op_n": ([P], I64),
            "phicomb_params": ([P, D, I32, P, C.c_uint64, P, P], I32),
            "phicomb_solve": ([P, P, I32, I32, P, P, P, D, I32, P, P, P], I32),
            "phicomb_solve_static": ([P, P, I32, I32, P, P, P, D, I32, P, P, P], I32),
            "phicomb_submit": ([P, P, I32, I32, P, P, P, D, I32, P, P], I32),
            "phicomb_poll": ([P, P], I32),
            "phicomb_serve_config": ([I64, I32], I32),
            "phicomb_request_bytes": ([I64, I32, I32, I32], I64),
            "phicomb_strerror": ([I32], C.c_char_p),
            "phicomb_batch_create": ([I32, P, I32, P], I32),
            "phicomb_batch_run": ([P, P, P], I32),
            "phicomb_batch_info": ([P, P, P, P], I32),
            "phicomb_batch_destroy": ([P], I32),
            "phicomb_batch_model": ([P, P, P], I32),
            "phicomb_batch_fit": ([P, P, P, P], I32),
            "phicomb_batch_times": ([P, P, P], I32),
            "phicomb_exprk4s6": ([P, P, P, D, I32, D, I32, P, P, P], I32),
            "phicomb_solve_series": ([P, I32, I32, P, P, P, D, P, P, P], I32),
            "phicomb_op_apply": ([P, P, I32, D, P, P, P], I32),
            "phicomb_zop_create_csr": ([I64, P, P, P, P], I32),
            "phicomb_zop_create_dense": ([I64, P, P], I32),
            "phicomb_zop_destroy": ([P], I32),
            "phicomb_zparams": ([P, D, I32, P, C.c_uint64, P, P], I32),
            "phicomb_zsolve": ([P, P, P, I32, I32, P, P, P, D, P, P, P], I32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = lib
    return _LIB


def _check(st: int, where: str):
    if st != OK:
        raise PhicombError(st, where)


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("phicomb needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- C entry points
def phicomb_op_create_csr(n: int, rowptr, col, val) -> C.c_void_p:
    _require_gpu()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    h = C.c_void_p()
    _check(_lib().phicomb_op_create_csr(n, _np_ptr(rp), _np_ptr(ci), _np_ptr(va), C.byref(h)),
           "phicomb_op_create_csr")
    return h


def phicomb_op_create_stencil(dim: int, grid: Sequence[int], coef: Sequence[float],
                              superdiag: float = 0.0) -> C.c_void_p:
    _require_gpu()
    g = np.ascontiguousarray(list(grid) + [1] * (3 - len(grid)), dtype=np.int32)
    c = np.ascontiguousarray(coef, dtype=np.float64)
    h = C.c_void_p()
    _check(_lib().phicomb_op_create_stencil(dim, _np_ptr(g), _np_ptr(c), float(superdiag),
                                            C.byref(h)), "phicomb_op_create_stencil")
    return h


def phicomb_op_create_dense(n: int, A) -> C.c_void_p:
    _require_gpu()
    a = np.ascontiguousarray(A, dtype=np.float64)
    h = C.c_void_p()
    _check(_lib().phicomb_op_create_dense(n, _np_ptr(a), C.byref(h)), "phicomb_op_create_dense")
    return h


def phicomb_op_create_lowrank(n: int, U, W) -> C.c_void_p:
    """A = U W^T applied matrix-free; U, W host arrays n x rank (rank <= 16)."""
    _require_gpu()
    u = np.ascontiguousarray(U, dtype=np.float64)
    w = np.ascontiguousarray(W, dtype=np.float64)
    if u.ndim != 2 or u.shape != w.shape or u.shape[0] != n:
        raise ValueError("U and W must both be n x rank")
    h = C.c_void_p()
    _check(_lib().phicomb_op_create_lowrank(n, u.shape[1], _np_ptr(u), _np_ptr(w), C.byref(h)),
           "phicomb_op_create_lowrank")
    return h


def phicomb_op_destroy(h) -> None:
    _check(_lib().phicomb_op_destroy(h), "phicomb_op_destroy")


def phicomb_params(h, tol: float, m: int = 61, v: Optional[np.ndarray] = None, seed: int = 1,
                   stream=None) -> ParamsT:
    out = ParamsT()
    va = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    st = _lib().phicomb_params(h, float(tol), int(m), _np_ptr(va) if va is not None else None,
                               int(seed), _stream_ptr(stream), C.byref(out))
    _check(st, "phicomb_params")
    return out


def phicomb_solve(h, prm: ParamsT, p: int, r: int, t, beta, V, tol: float, precision: int,
                  W, stream=None) -> StatsT:
    """V: torch float64 cuda tensor [n][p+1]; W: torch float64 cuda tensor [n][r]."""
    ta = np.ascontiguousarray(t, dtype=np.float64)
    ba = np.ascontiguousarray(beta, dtype=np.float64)
    _check_device_tensor(V, (None, p + 1), "V")
    _check_device_tensor(W, (None, r), "W")
    stats = StatsT()
    st = _lib().phicomb_solve(h, C.byref(prm), int(p), int(r), _np_ptr(ta), _np_ptr(ba),
                              C.c_void_p(V.data_ptr()), float(tol), int(precision),
                              C.c_void_p(W.data_ptr()), _stream_ptr(stream), C.byref(stats))
    _check(st, "phicomb_solve")
    return stats


def phicomb_solve_static(h, prm: ParamsT, p: int, r: int, t, beta, V, tol: float,
                         precision: int, W, stream=None) -> StatsT:
    """phicomb_solve with the work blocks in the library's static device
    array (no allocation in the call); same arguments."""
    ta = np.ascontiguousarray(t, dtype=np.float64)
    ba = np.ascontiguousarray(beta, dtype=np.float64)
    _check_device_tensor(V, (None, p + 1), "V")
    _check_device_tensor(W, (None, r), "W")
    stats = StatsT()
    st = _lib().phicomb_solve_static(h, C.byref(prm), int(p), int(r), _np_ptr(ta), _np_ptr(ba),
                                     C.c_void_p(V.data_ptr()), float(tol), int(precision),
                                     C.c_void_p(W.data_ptr()), _stream_ptr(stream),
                                     C.byref(stats))
    _check(st, "phicomb_solve_static")
    return stats


STATIC_BYTES = 64 << 20   # PHICOMB_STATIC_BYTES


def phicomb_op_apply(h, X, shift: float, Y, stream=None, timed: bool = False) -> float:
    """Y = (A - shift I) X; X, Y: torch float64 cuda tensors [ncols][n]
    (column-major blocks).  Returns the device time in ms when timed."""
    import torch
    for name, x in (("X", X), ("Y", Y)):
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64 \
                or not x.is_contiguous() or x.dim() != 2:
            raise TypeError(f"{name} must be a contiguous float64 cuda tensor [ncols][n]")
    if X.shape != Y.shape:
        raise ValueError("X and Y must have the same shape")
    ms = C.c_double(0.0)
    st = _lib().phicomb_op_apply(h, C.c_void_p(X.data_ptr()), int(X.shape[0]), float(shift),
                                 C.c_void_p(Y.data_ptr()), _stream_ptr(stream),
                                 C.byref(ms) if timed else None)
    _check(st, "phicomb_op_apply")
    return ms.value


def phicomb_solve_series(h, p: int, r: int, t, beta, V, tol: float, W, stream=None) -> StatsT:
    """The Proposition's single block series (no shift, no scaling)."""
    ta = np.ascontiguousarray(t, dtype=np.float64)
    ba = np.ascontiguousarray(beta, dtype=np.float64)
    _check_device_tensor(V, (None, p + 1), "V")
    _check_device_tensor(W, (None, r), "W")
    stats = StatsT()
    st = _lib().phicomb_solve_series(h, int(p), int(r), _np_ptr(ta), _np_ptr(ba),
                                     C.c_void_p(V.data_ptr()), float(tol),
                                     C.c_void_p(W.data_ptr()), _stream_ptr(stream),
                                     C.byref(stats))
    _check(st, "phicomb_solve_series")
    return stats


def phicomb_exprk4s6(h, prm: ParamsT, g, step: float, nsteps: int, tol: float, precision: int,
                     u, stream=None) -> ExprkStatsT:
    """expRK4s6 for u' = A u + g(u), g(u) = g[0] + g[1] u + g[2] u^2 + g[3] u^3;
    u: torch float64 cuda tensor [n] (or [n][1]), advanced in place."""
    ga = np.ascontiguousarray(g, dtype=np.float64)
    if ga.shape != (4,):
        raise ValueError("g must hold 4 cubic coefficients")
    uu = u.view(-1, 1) if u.dim() == 1 else u
    _check_device_tensor(uu, (None, 1), "u")
    stats = ExprkStatsT()
    st = _lib().phicomb_exprk4s6(h, C.byref(prm), _np_ptr(ga), float(step), int(nsteps),
                                 float(tol), int(precision), C.c_void_p(u.data_ptr()),
                                 _stream_ptr(stream), C.byref(stats))
    _check(st, "phicomb_exprk4s6")
    return stats


def phicomb_submit(h, prm: ParamsT, p: int, r: int, t, beta, V, tol: float, precision: int,
                   W) -> C.c_void_p:
    ta = np.ascontiguousarray(t, dtype=np.float64)
    ba = np.ascontiguousarray(beta, dtype=np.float64)
    _check_device_tensor(V, (None, p + 1), "V")
    _check_device_tensor(W, (None, r), "W")
    req = C.c_void_p()
    st = _lib().phicomb_submit(h, C.byref(prm), int(p), int(r), _np_ptr(ta), _np_ptr(ba),
                               C.c_void_p(V.data_ptr()), float(tol), int(precision),
                               C.c_void_p(W.data_ptr()), C.byref(req))
    _check(st, "phicomb_submit")
    return req


def phicomb_poll(req) -> tuple:
    """Returns (status, StatsT).  status PENDING leaves the ticket valid."""
    stats = StatsT()
    st = _lib().phicomb_poll(req, C.byref(stats))
    return st, stats


def phicomb_serve_config(budget_bytes: int, slots: int) -> None:
    _check(_lib().phicomb_serve_config(int(budget_bytes), int(slots)), "phicomb_serve_config")


def phicomb_request_bytes(n: int, p: int, r: int, precision: int = FP64) -> int:
    return int(_lib().phicomb_request_bytes(n, p, r, precision))


def phicomb_strerror(status: int) -> str:
    return _lib().phicomb_strerror(status).decode()


def phicomb_batch_create(items, precision: int = FP64):
    """items: sequence of (op_handle, ParamsT, p, r, t, beta, V, W, tol) with V, W
    float64 CUDA tensors ([n][p+1], [n][r]).  Returns the plan handle."""
    keep = []
    arr = (BatchItemT * len(items))()
    for k, (h, prm, p, r, t, beta, V, W, tol) in enumerate(items):
        ta = np.ascontiguousarray(t, dtype=np.float64)
        ba = np.ascontiguousarray(beta, dtype=np.float64)
        _check_device_tensor(V, (None, p + 1), "V")
        _check_device_tensor(W, (None, r), "W")
        keep += [ta, ba, prm]
        arr[k].op = h.value if isinstance(h, C.c_void_p) else h
        arr[k].prm = C.pointer(prm)
        arr[k].p, arr[k].r = int(p), int(r)
        arr[k].t, arr[k].beta = ta.ctypes.data, ba.ctypes.data
        arr[k].V, arr[k].W = V.data_ptr(), W.data_ptr()
        arr[k].tol = float(tol)
    out = C.c_void_p()
    _check(_lib().phicomb_batch_create(len(items), arr, int(precision), C.byref(out)),
           "phicomb_batch_create")
    return out


def phicomb_batch_run(b, count: int, stream=None):
    """Runs the plan; returns (status, [StatsT] * count)."""
    stats = (StatsT * count)()
    st = _lib().phicomb_batch_run(b, _stream_ptr(stream), stats)
    return st, list(stats)


def phicomb_batch_model(b, new=None) -> list:
    """The plan's cost-model constants (5 doubles); with new, replace them
    (the schedule is rebuilt) and return the new ones."""
    out = (C.c_double * 5)()
    if new is not None:
        arr = (C.c_double * 5)(*[float(x) for x in new])
        _check(_lib().phicomb_batch_model(b, None, arr), "phicomb_batch_model")
    _check(_lib().phicomb_batch_model(b, out, None), "phicomb_batch_model")
    return list(out)


def phicomb_batch_fit(b) -> dict:
    """Last run: measured launch ms and the model's prediction before and
    after its refit."""
    m, p0, p1 = C.c_double(), C.c_double(), C.c_double()
    _check(_lib().phicomb_batch_fit(b, C.byref(m), C.byref(p0), C.byref(p1)),
           "phicomb_batch_fit")
    return {"measured_ms": m.value, "predicted_ms_before": p0.value,
            "predicted_ms_after": p1.value}


def phicomb_batch_times(b, count: int):
    """Per instance of the last run: (microseconds, workgroups of its group)."""
    us = (C.c_double * count)()
    gs = (C.c_int * count)()
    _check(_lib().phicomb_batch_times(b, us, gs), "phicomb_batch_times")
    return list(us), list(gs)


def phicomb_batch_info(b) -> dict:
    g, w, ms = C.c_int(), C.c_int(), C.c_double()
    _check(_lib().phicomb_batch_info(b, C.byref(g), C.byref(w), C.byref(ms)),
           "phicomb_batch_info")
    return {"groups": g.value, "workgroups": w.value, "predicted_ms": ms.value}


def phicomb_batch_destroy(b) -> None:
    _check(_lib().phicomb_batch_destroy(b), "phicomb_batch_destroy")


def _check_device_tensor(x, shape, name):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 torch tensor on the GPU")
    if not x.is_contiguous() or x.dim() != 2 or (shape[1] is not None and x.shape[1] != shape[1]):
        raise ValueError(f"{name} must be contiguous [n][{shape[1]}], got {tuple(x.shape)}")


# ---------------------------------------------------------------- complex data
def phicomb_zop_create_csr(n: int, rowptr, col, val):
    """Complex CSR operator; val complex [nnz] (host)."""
    _require_gpu()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.complex128)
    h = C.c_void_p()
    _check(_lib().phicomb_zop_create_csr(int(n), _np_ptr(rp), _np_ptr(ci), _np_ptr(va),
                                         C.byref(h)), "phicomb_zop_create_csr")
    return h


def phicomb_zop_create_dense(A):
    """Complex dense operator from a complex [n][n] array (host)."""
    _require_gpu()
    a = np.ascontiguousarray(A, dtype=np.complex128)
    h = C.c_void_p()
    _check(_lib().phicomb_zop_create_dense(int(a.shape[0]), _np_ptr(a), C.byref(h)),
           "phicomb_zop_create_dense")
    return h


def phicomb_zop_destroy(h) -> None:
    _check(_lib().phicomb_zop_destroy(h), "phicomb_zop_destroy")


def phicomb_zparams(h, tol: float, m: int = 61, v: Optional[np.ndarray] = None, seed: int = 1,
                    stream=None) -> ParamsT:
    out = ParamsT()
    va = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    st = _lib().phicomb_zparams(h, float(tol), int(m), _np_ptr(va) if va is not None else None,
                                int(seed), _stream_ptr(stream), C.byref(out))
    _check(st, "phicomb_zparams")
    return out


def phicomb_zsolve(h, prm: ParamsT, p: int, r: int, t, beta, V, tol: float, W, shift=None,
                   stream=None) -> StatsT:
    """V: torch complex128 cuda tensor [n][p+1]; W: torch complex128 [n][r];
    t [r] and beta [r][p+1] complex (host); shift complex or None (prm.shift)."""
    import torch
    ta = np.ascontiguousarray(t, dtype=np.complex128)
    ba = np.ascontiguousarray(beta, dtype=np.complex128)
    for x, name, c in ((V, "V", p + 1), (W, "W", r)):
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.complex128:
            raise TypeError(f"{name} must be a complex128 torch tensor on the GPU")
        if not x.is_contiguous() or x.dim() != 2 or x.shape[1] != c:
            raise ValueError(f"{name} must be contiguous [n][{c}], got {tuple(x.shape)}")
    xa = None if shift is None else np.array([complex(shift)], dtype=np.complex128)
    stats = StatsT()
    st = _lib().phicomb_zsolve(h, C.byref(prm), _np_ptr(xa) if xa is not None else None,
                               int(p), int(r), _np_ptr(ta), _np_ptr(ba),
                               C.c_void_p(V.data_ptr()), float(tol), C.c_void_p(W.data_ptr()),
                               _stream_ptr(stream), C.byref(stats))
    _check(st, "phicomb_zsolve")
    return stats


# ---------------------------------------------------------------- conveniences
class Operator:
    """Resident operator handle built from a workloads description
    (Stencil, CSR, Dense or LowRank)."""

    def __init__(self, desc):
        kind = desc.kind
        if kind == "stencil":
            self.h = phicomb_op_create_stencil(desc.dim, desc.grid, desc.coef, desc.superdiag)
        elif kind == "dense":
            self.h = phicomb_op_create_dense(desc.n, desc.A)
        elif kind == "lowrank":
            self.h = phicomb_op_create_lowrank(desc.n, desc.U, desc.W)
        else:
            rp, ci, va = desc.csr()
            self.h = phicomb_op_create_csr(len(rp) - 1, rp, ci, va)
        self.n = int(_lib().phicomb_op_n(self.h))
        self.kind = kind

    def close(self):
        if self.h:
            phicomb_op_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, tol: float, m: int = 61, v=None, seed: int = 1) -> ParamsT:
        return phicomb_params(self.h, tol, m, v, seed)

    def solve(self, prm: ParamsT, t, beta, V, tol: float, precision: int = FP64, W=None):
        torch = _require_gpu()
        beta = np.atleast_2d(np.asarray(beta, dtype=np.float64))
        r, P1 = beta.shape
        if W is None:
            W = torch.empty((self.n, r), dtype=torch.float64, device=V.device)
        stats = phicomb_solve(self.h, prm, P1 - 1, r, t, beta, V, tol, precision, W)
        return W, stats


def params_from_dict(d: dict) -> ParamsT:
    """Pin parameters computed elsewhere (e.g. by a reference)."""
    p = ParamsT()
    for f, _ in ParamsT._fields_:
        if f in d:
            setattr(p, f, d[f])
    p.status = OK
    return p
