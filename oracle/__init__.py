"""CPU oracle for the phi-combination method -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded IEEE-double C (``phicomb_oracle.c``) following
Algorithms 1-3 of Al-Mohy, "Computing Linear Combinations of phi-Function
Actions for Exponential Integrators" (arXiv 2509.26475), step by step.
Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the HIP library never does, and
neither includes, links or calls the other.  Two published routines that
both sides must compute exactly (the correctly rounded binomial coefficient
and Brent's localmin) are written separately on each side and pinned here
on their own.

Blocks cross this wrapper row-major ([n][p+1] for V, [n][r] for W) to match
the library's layout; the C code works column-major internally, so the
wrapper transposes (a layout change only).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phicomb_oracle.c")
_ZSRC = os.path.join(_HERE, "phicomb_oracle_complex.c")   # Algorithms 1 and 3 over C
_LIB = os.path.join(_HERE, "libphicomb_oracle.so")
_lib = None

BRENT_REL = 1.4901161193847656e-08   # sqrt(2^-52)
BRENT_ABS = 1e-6                     # absolute tolerance in z = -xi/s0
BRENT_MAXIT = 100
KCAP = 150                           # Taylor-term cap per loop (sigma = k! < 2^1024)

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -4: "ENOCONV", -5: "EOVERFLOW"}


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status} ({STATUS.get(status, '?')})")
        self.status = status


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, _ZSRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Op(C.Structure):
    _fields_ = [("n", C.c_int64), ("kind", C.c_int32), ("rank", C.c_int32),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("dense", C.c_void_p), ("lr_u", C.c_void_p), ("lr_w", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("shift", C.c_double), ("s0", C.c_double), ("zstar", C.c_double),
                ("fstar", C.c_double), ("s", C.c_double), ("m", C.c_int32),
                ("r_acc", C.c_int32), ("n_feval", C.c_int32), ("status", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("s_int", C.c_int32), ("terms_S", C.c_int32), ("terms_rec", C.c_int32),
                ("max_terms_step", C.c_int32), ("status", C.c_int32), ("pad", C.c_int32)]


_FUN = C.CFUNCTYPE(C.c_double, C.c_double, C.c_void_p)


def _configure(lib):
    P = C.c_void_p
    lib.orc_params.argtypes = [P, C.c_double, C.c_int, P, C.c_double, C.c_double,
                               C.c_int, P, P, P]
    lib.orc_params.restype = C.c_int
    lib.orc_solve.argtypes = [P, C.c_int, C.c_int, P, P, P, C.c_int, P, C.c_double,
                              C.c_double, C.c_double, C.c_int, P, P]
    lib.orc_solve.restype = C.c_int
    lib.orc_solve_single.argtypes = [P, C.c_int, C.c_double, C.c_double, P, C.c_double,
                                     C.c_double, C.c_double, C.c_int, P, P]
    lib.orc_solve_single.restype = C.c_int
    lib.orc_brent_min.argtypes = [_FUN, P, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_int, P, P]
    lib.orc_brent_min.restype = C.c_double
    lib.orc_apply.argtypes = [P, P, P]
    lib.orc_apply.restype = None
    lib.orc_binom.argtypes = [C.c_int, C.c_int]
    lib.orc_binom.restype = C.c_double
    if hasattr(lib, "orz_solve"):   # builds of the real source alone lack them
        lib.orz_params.argtypes = [P, C.c_double, C.c_int, P, C.c_double, C.c_double,
                                   C.c_int, P]
        lib.orz_params.restype = C.c_int
        lib.orz_solve.argtypes = [P, C.c_int, C.c_int, P, P, P, C.c_int, P, C.c_double, P,
                                  C.c_double, C.c_int, P, P]
        lib.orz_solve.restype = C.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _configure(C.CDLL(_LIB))
    return _lib


class using_library:
    """Context manager: route every call through another build of the
    oracle source (the mutation tests compile planted-mistake copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _configure(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Operator:
    """Keeps the arrays alive and exposes the C descriptor."""

    def __init__(self, op):
        kind = getattr(op, "kind", None)
        self.keep = []
        s = _Op()
        if kind == "dense":
            A = np.ascontiguousarray(op.A, dtype=np.float64)
            self.keep.append(A)
            s.n, s.kind, s.dense = A.shape[0], 1, A.ctypes.data
        elif kind == "lowrank":
            U = np.ascontiguousarray(op.U, dtype=np.float64)
            W = np.ascontiguousarray(op.W, dtype=np.float64)
            if U.shape != W.shape or U.shape[1] > 16:
                raise ValueError("low-rank operator: U and W must be n x r, r <= 16")
            self.keep += [U, W]
            s.n, s.kind, s.rank = U.shape[0], 2, U.shape[1]
            s.lr_u, s.lr_w = U.ctypes.data, W.ctypes.data
        else:
            rp, ci, va = op.csr()
            rp = np.ascontiguousarray(rp, dtype=np.int32)
            ci = np.ascontiguousarray(ci, dtype=np.int32)
            va = np.ascontiguousarray(va, dtype=np.float64)
            self.keep += [rp, ci, va]
            s.n, s.kind = rp.shape[0] - 1, 0
            s.rowptr, s.col, s.val = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
        self.s = s
        self.n = int(s.n)

    @property
    def ref(self):
        return C.byref(self.s)


def _as_op(op):
    return op if isinstance(op, Operator) else Operator(op)


def apply(op, x: np.ndarray) -> np.ndarray:
    o = _as_op(op)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    _load().orc_apply(o.ref, _ptr(x), _ptr(y))
    return y


def binom(m: int, k: int) -> float:
    return float(_load().orc_binom(m, k))


def params(op, tol: float, v: np.ndarray, m: int = 61, brent_rel: float = BRENT_REL,
           brent_abs: float = BRENT_ABS, brent_maxit: int = BRENT_MAXIT,
           want_basis: bool = False) -> dict:
    """Algorithm 1.  Returns a dict with shift, s0, zstar, fstar, s, m,
    r_acc, n_feval, L (log-norms of the accepted powers) and optionally
    the normalised basis [m+1][n]."""
    o = _as_op(op)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = _Params()
    L = np.zeros(m + 1)
    basis = np.zeros((m + 1, o.n)) if want_basis else None
    st = _load().orc_params(o.ref, tol, m, _ptr(v), brent_rel, brent_abs, brent_maxit,
                            C.byref(out), _ptr(L), _ptr(basis) if want_basis else None)
    if st != 0:
        raise OracleError(st)
    res = {f: getattr(out, f) for f, _ in _Params._fields_}
    res["L"] = L
    res["tol"] = tol
    if want_basis:
        res["basis"] = basis
    return res


def solve(op, p: int, r: int, t, beta, V: np.ndarray, tol: float, shift: float, s: float,
          form: str = "beta", alpha=None, kcap: int = KCAP):
    """Algorithm 3.  V: [n][p+1] row-major.  Returns (W [n][r], stats)."""
    o = _as_op(op)
    n = o.n
    t = np.ascontiguousarray(t, dtype=np.float64)
    Vc = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)   # column-major
    assert Vc.shape == (p + 1, n)
    beta_a = np.ascontiguousarray(beta, dtype=np.float64) if beta is not None else None
    alpha_a = np.ascontiguousarray(alpha, dtype=np.float64) if alpha is not None else None
    Wc = np.zeros((r, n))
    stt = _Stats()
    st = _load().orc_solve(o.ref, p, r, _ptr(t), _ptr(beta_a) if beta_a is not None else None,
                           _ptr(alpha_a) if alpha_a is not None else None,
                           0 if form == "beta" else 1, _ptr(Vc), tol, shift, s, kcap,
                           _ptr(Wc), C.byref(stt))
    if st != 0:
        raise OracleError(st)
    stats = {f: getattr(stt, f) for f, _ in _Stats._fields_ if f != "pad"}
    return np.ascontiguousarray(Wc.T), stats


def solve_single(op, p: int, t: float, alpha: float, V: np.ndarray, tol: float,
                 shift: float, s: float, kcap: int = KCAP):
    """Algorithm 2.  Returns (w [n], stats)."""
    o = _as_op(op)
    Vc = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)
    w = np.zeros(o.n)
    stt = _Stats()
    st = _load().orc_solve_single(o.ref, p, float(t), float(alpha), _ptr(Vc), tol, shift, s,
                                  kcap, _ptr(w), C.byref(stt))
    if st != 0:
        raise OracleError(st)
    return w, {f: getattr(stt, f) for f, _ in _Stats._fields_ if f != "pad"}


def brent_min(f, a: float, b: float, rel: float = BRENT_REL, abs_tol: float = BRENT_ABS,
              maxit: int = BRENT_MAXIT):
    cb = _FUN(lambda x, ctx: float(f(x)))
    fmin = C.c_double()
    nfev = C.c_int()
    x = _load().orc_brent_min(cb, None, a, b, rel, abs_tol, maxit, C.byref(fmin), C.byref(nfev))
    return x, fmin.value, nfev.value


def full(problem, m: int = 61, form: str = "beta", kcap: int = KCAP, prm: Optional[dict] = None):
    """Algorithm 1 then Algorithm 3 on a workloads.Problem."""
    o = Operator(problem.op)
    if prm is None:
        prm = params(o, problem.tol, problem.v, m=m)
    W, st = solve(o, problem.p, problem.r, problem.t, problem.beta, problem.V, problem.tol,
                  prm["shift"], prm["s"], form=form, alpha=problem.alpha, kcap=kcap)
    return W, st, prm


# ------------------------------------------------------------ expRK4s6
# Nodes of the fourth-order six-stage exponential Runge-Kutta scheme
# (Sec. 1, eq. (expRK4s6)).
EXPRK_C = {2: 0.5, 3: 0.5, 4: 1.0 / 3.0, 5: 5.0 / 6.0, 6: 1.0 / 3.0}


def _cubic(gc, u):
    """Pointwise reaction g(u) = gc[0] + gc[1] u + gc[2] u^2 + gc[3] u^3."""
    return gc[0] + u * (gc[1] + u * (gc[2] + u * gc[3]))


def exprk4s6(op, gc, u0: np.ndarray, h: float, nsteps: int, tol: float, shift: float,
             s: float):
    """u' = A u + g(u) over nsteps steps of size h with the scheme of Sec. 1,
    eq. (expRK4s6), every phi-combination evaluated by Algorithm 3 with the
    parameters (shift, s) of Algorithm 1 reused for all calls.  The stages
    that the scheme allows to be computed together are one block call each
    (Sec. 5, fourth experiment): U2; {U3, U4}; {U5, U6}; u_{n+1}.  Every
    call has v_0 = 0 and v_1 = h f(u_n).  Returns (u, per-call stats)."""
    o = _as_op(op)
    c = EXPRK_C
    u = np.array(u0, dtype=np.float64)
    calls = []

    def call(t, beta, cols):
        V = np.stack([np.zeros_like(u)] + cols, axis=1)
        W, st = solve(o, V.shape[1] - 1, len(t), np.asarray(t), np.asarray(beta), V, tol,
                      shift, s)
        calls.append(st)
        return W

    for _ in range(nsteps):
        gu = _cubic(gc, u)
        f = apply(o, u) + gu
        hf = h * f
        # U2 = u + phi_1(c2 h A) c2 h f
        W = call([c[2] * h], [[0.0, c[2]]], [hf])
        D2 = _cubic(gc, u + W[:, 0]) - gu
        # U_k = u + phi_1(c_k h A) c_k h f + phi_2(c_k h A) (c_k^2/c2) h D2, k = 3, 4
        W = call([c[3] * h, c[4] * h],
                 [[0.0, c[k], c[k] ** 2 / c[2]] for k in (3, 4)], [hf, h * D2])
        D3 = _cubic(gc, u + W[:, 0]) - gu
        D4 = _cubic(gc, u + W[:, 1]) - gu
        # U_j, j = 5, 6: phi_2 weight c_j^2/(c3-c4), phi_3 weight 2 c_j^3/(c3-c4)
        q2 = h * (-(c[4] / c[3]) * D3 + (c[3] / c[4]) * D4)
        q3 = h * (D3 / c[3] - D4 / c[4])
        W = call([c[5] * h, c[6] * h],
                 [[0.0, c[j], c[j] ** 2 / (c[3] - c[4]), 2.0 * c[j] ** 3 / (c[3] - c[4])]
                  for j in (5, 6)], [hf, q2, q3])
        D5 = _cubic(gc, u + W[:, 0]) - gu
        D6 = _cubic(gc, u + W[:, 1]) - gu
        # u_{n+1}: phi_2 weight 1/(c5-c6), phi_3 weight 2/(c5-c6)
        q2 = h * (-(c[6] / c[5]) * D5 + (c[5] / c[6]) * D6)
        q3 = h * (D5 / c[5] - D6 / c[6])
        W = call([h], [[0.0, 1.0, 1.0 / (c[5] - c[6]), 2.0 / (c[5] - c[6])]], [hf, q2, q3])
        u = u + W[:, 0]
    return u, calls


# ------------------------------------------------ the Proposition's series
def series_block(op, p: int, r: int, t, beta, V: np.ndarray, tol: float, kcap: int = KCAP):
    """The single series of the Proposition in Sec. 4 with g_i = phi_i:
    G = sum_j A^j V D_j Gamma T^j, D_j = diag(1/(i+j)!, i = 0..p), with the
    Vandermonde Gamma replaced by a general weight table (Gamma[i, k] =
    beta[k, i]; the proof is unchanged).  Column k of G is
    w_k = sum_i beta[k, i] phi_i(t_k A) v_i.  No shift and no scaling: terms
    are added until two consecutive ones are below tol times the block norm
    (the stopping rule (stopTm) of Algorithm 3, block infinity norm).
    Returns (W [n][r], stats)."""
    o = _as_op(op)
    t = np.asarray(t, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64).reshape(r, p + 1)
    X = np.array(V, dtype=np.float64)            # A^j V, column i = A^j v_i
    tj = np.ones(r)                              # t_k^j
    fact = np.array([float(math.factorial(i)) for i in range(p + 1)])   # (i+j)!

    def term():
        # column k: sum_i beta[k, i] t_k^j / (i+j)! A^j v_i
        return X @ (beta / fact[None, :]).T * tj[None, :]

    G = term()
    c1, c2 = math.inf, np.abs(G).sum(axis=1).max()
    j = 0
    while c1 + c2 > tol * np.abs(G).sum(axis=1).max():
        if j + 1 >= kcap:
            raise OracleError(-4)
        j += 1
        X = np.stack([apply(o, X[:, i]) for i in range(p + 1)], axis=1)
        tj = tj * t
        fact = fact * (np.arange(p + 1) + j)
        T = term()
        G = G + T
        c1, c2 = c2, np.abs(T).sum(axis=1).max()
    return G, {"terms": j + 1}


# ----------------------------------------------------------- complex data
class _ZOp(C.Structure):
    _fields_ = [("n", C.c_int64), ("kind", C.c_int32), ("pad", C.c_int32),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("dense", C.c_void_p)]


class ZOperator:
    """A complex operator for the complex oracle: a dense n x n array, or CSR
    (rowptr, col, val) with complex values.  Keeps the arrays alive."""

    def __init__(self, dense=None, csr=None):
        s = _ZOp()
        self.keep = []
        if dense is not None:
            A = np.ascontiguousarray(dense, dtype=np.complex128)
            self.keep.append(A)
            s.n, s.kind, s.dense = A.shape[0], 1, A.ctypes.data
        else:
            rp, ci, va = csr
            rp = np.ascontiguousarray(rp, dtype=np.int32)
            ci = np.ascontiguousarray(ci, dtype=np.int32)
            va = np.ascontiguousarray(va, dtype=np.complex128)
            self.keep += [rp, ci, va]
            s.n, s.kind = rp.shape[0] - 1, 0
            s.rowptr, s.col, s.val = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
        self.s = s
        self.n = int(s.n)

    @property
    def ref(self):
        return C.byref(self.s)


def zparams(op: ZOperator, tol: float, v: np.ndarray, m: int = 61,
            brent_rel: float = BRENT_REL, brent_abs: float = BRENT_ABS,
            brent_maxit: int = BRENT_MAXIT) -> dict:
    """Algorithm 1 for a complex operator from a real start vector v; the
    shift is searched on the real line as in the listing (real xi*)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = _Params()
    st = _load().orz_params(op.ref, tol, m, _ptr(v), brent_rel, brent_abs, brent_maxit,
                            C.byref(out))
    if st != 0:
        raise OracleError(st)
    res = {f: getattr(out, f) for f, _ in _Params._fields_}
    res["tol"] = tol
    return res


def zsolve(op: ZOperator, p: int, r: int, t, beta, V: np.ndarray, tol: float, shift,
           s: float, form: str = "beta", alpha=None, kcap: int = KCAP):
    """Algorithm 3 over C.  t [r], beta [r][p+1] (form "beta") or alpha [r]
    (form "alpha"), V [n][p+1], shift complex.  Returns (W [n][r], stats)."""
    n = op.n
    t = np.ascontiguousarray(t, dtype=np.complex128)
    Vc = np.ascontiguousarray(np.asarray(V, dtype=np.complex128).T)
    assert Vc.shape == (p + 1, n)
    b = np.ascontiguousarray(beta, dtype=np.complex128) if beta is not None else None
    a = np.ascontiguousarray(alpha, dtype=np.complex128) if alpha is not None else None
    xi = np.array([complex(shift)], dtype=np.complex128)
    Wc = np.zeros((r, n), dtype=np.complex128)
    stt = _Stats()
    st = _load().orz_solve(op.ref, p, r, _ptr(t), _ptr(b) if b is not None else None,
                           _ptr(a) if a is not None else None, 0 if form == "beta" else 1,
                           _ptr(Vc), tol, _ptr(xi), s, kcap, _ptr(Wc), C.byref(stt))
    if st != 0:
        raise OracleError(st)
    stats = {f: getattr(stt, f) for f, _ in _Stats._fields_ if f != "pad"}
    return np.ascontiguousarray(Wc.T), stats
