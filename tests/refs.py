"""Exact references used to pin the oracle (test helpers; no oracle code).

Each helper computes w_i = sum_j beta_ij phi_j(t_i A) v_j (paper, Sec. 1,
(phi.comb)) by a route that is independent of the method:

* ``phi_mp`` / ``phi_ld``: the scalar phi-functions from their definition
  (Sec. 1, (def.phik)): series sum_k z^k/(k+j)! near 0, otherwise
  phi_0 = e^z and phi_{j+1}(z) = (phi_j(z) - 1/j!)/z.
* ``augmented_mp``: the exact augmented-matrix form used by the paper for
  its reference solutions (Sec. 5, first experiment; Theorem 1's proof):
  w = [I 0] exp([[tA, [w_p .. w_1]], [0, J_p(0)]]) [w_0; e_p] with
  w_j = beta_j v_j, evaluated by mpmath at high precision.
* ``dst_laplacian``: the textbook eigen-decomposition of a Dirichlet
  Laplacian stencil (orthonormal DST-I), scalar phi at every eigenvalue.
* ``expm_multiply_aug`` / ``expm_multiply_dense_aug``: scipy's
  expm_multiply on the augmented matrix (Al-Mohy & Higham 2011, the paper's
  [alhi11]).
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def phi_mp(j: int, z, dps: int = 50):
    """phi_j(z) at ``dps`` digits (definition (def.phik))."""
    with mpmath.workdps(dps):
        z = mpmath.mpf(z) if not isinstance(z, mpmath.mpc) else z
        if abs(z) < 2:
            acc = mpmath.mpf(0)
            term = mpmath.mpf(1) / mpmath.factorial(j)
            k = 0
            while True:
                acc += term
                k += 1
                term = term * z / (k + j)
                if abs(term) < mpmath.mpf(10) ** (-dps - 5) * (abs(acc) + 1):
                    break
            return acc
        s = mpmath.exp(z)
        for k in range(j):
            s -= z ** k / mpmath.factorial(k)
        return s / z ** j


def phi_ld(j: int, z: np.ndarray) -> np.ndarray:
    """Vectorised phi_j in extended (80-bit) precision, returned as float64.
    Series for |z| < 8, recurrence from e^z otherwise (stable there since
    every step divides by |z| > j)."""
    z = np.asarray(z, dtype=np.longdouble)
    out = np.empty(z.shape, dtype=np.longdouble)
    small = np.abs(z) < 8
    if small.any():
        zs = z[small]
        acc = np.zeros_like(zs)
        term = np.full_like(zs, 1) / np.longdouble(math.factorial(j))
        for k in range(1, 90):
            acc += term
            term = term * zs / (k + j)
        out[small] = acc
    big = ~small
    if big.any():
        zb = z[big]
        ph = np.exp(zb)
        fact = np.longdouble(1)
        for k in range(j):
            ph = (ph - 1 / fact) / zb
            fact *= (k + 1)
        out[big] = ph
    return out.astype(np.float64)


def augmented_mp(A: np.ndarray, t_i: float, beta_i: np.ndarray, V: np.ndarray,
                 dps: int = 40) -> np.ndarray:
    """Exact w_i from the augmented exponential (V: [n][p+1])."""
    n, P1 = V.shape
    p = P1 - 1
    with mpmath.workdps(dps):
        M = mpmath.zeros(n + p, n + p)
        for a in range(n):
            for b in range(n):
                M[a, b] = mpmath.mpf(t_i) * mpmath.mpf(A[a, b])
        # columns n..n+p-1 of the (1,2) block: [w_p, w_{p-1}, ..., w_1]
        for c in range(p):
            j = p - c
            for a in range(n):
                M[a, n + c] = mpmath.mpf(beta_i[j]) * mpmath.mpf(V[a, j])
        for c in range(p - 1):
            M[n + c, n + c + 1] = 1
        E = mpmath.expm(M)
        rhs = mpmath.zeros(n + p, 1)
        for a in range(n):
            rhs[a] = mpmath.mpf(beta_i[0]) * mpmath.mpf(V[a, 0])
        if p > 0:
            rhs[n + p - 1] = 1
        w = E * rhs
        return np.array([float(w[a]) for a in range(n)])


def augmented_mp_c(A: np.ndarray, t_i: complex, beta_i: np.ndarray, V: np.ndarray,
                   dps: int = 40) -> np.ndarray:
    """Exact w_i over C from the augmented exponential (Theorem 1):
    w_i = [I 0] exp([[t_i A, W_i], [0, J_p(0)]]) [beta_i0 v_0; e_p], with
    W_i = [beta_ip v_p, ..., beta_i1 v_1]; complex A, t_i, beta_i, V."""
    n, P1 = V.shape
    p = P1 - 1
    mc = lambda z: mpmath.mpc(complex(z).real, complex(z).imag)
    with mpmath.workdps(dps):
        M = mpmath.zeros(n + p, n + p)
        for a in range(n):
            for b in range(n):
                M[a, b] = mc(t_i) * mc(A[a, b])
        for c in range(p):
            j = p - c
            for a in range(n):
                M[a, n + c] = mc(beta_i[j]) * mc(V[a, j])
        for c in range(p - 1):
            M[n + c, n + c + 1] = 1
        E = mpmath.expm(M)
        rhs = mpmath.zeros(n + p, 1)
        for a in range(n):
            rhs[a] = mc(beta_i[0]) * mc(V[a, 0])
        if p > 0:
            rhs[n + p - 1] = 1
        w = E * rhs
        return np.array([complex(w[a]) for a in range(n)])


def exact_dense_mp_c(A, t, beta, V, dps=40):
    return np.stack([augmented_mp_c(A, t[i], beta[i], V, dps) for i in range(len(t))], axis=1)


def exact_dense_mp(A, t, beta, V, dps=40):
    return np.stack([augmented_mp(A, t[i], beta[i], V, dps) for i in range(len(t))], axis=1)


def _lap_eigs_1d(m: int, c_off: float) -> np.ndarray:
    k = np.arange(1, m + 1)
    return c_off * (2.0 * np.cos(k * np.pi / (m + 1)) - 2.0)


def dst_laplacian(stencil, t, beta, V) -> np.ndarray:
    """Exact W for a symmetric constant-coefficient Dirichlet Laplacian
    stencil (centre = -sum of the off-diagonal coefficients, equal +/- pair
    in every direction, no superdiagonal perturbation)."""
    nx, ny, nz = stencil.grid
    c = np.asarray(stencil.coef)
    assert stencil.superdiag == 0.0
    assert c[1] == c[2] and c[3] == c[4] and c[5] == c[6]
    assert abs(c[0] + 2 * (c[1] + c[3] + c[5])) <= 1e-12 * abs(c[0])
    shape = (nz, ny, nx)
    lam = (_lap_eigs_1d(nz, c[5])[:, None, None] + _lap_eigs_1d(ny, c[3])[None, :, None]
           + _lap_eigs_1d(nx, c[1])[None, None, :])
    axes = (0, 1, 2) if nz > 1 else (1, 2)
    P1 = V.shape[1]
    coeffs = [scipy.fft.dstn(V[:, j].reshape(shape), type=1, norm="ortho", axes=axes)
              for j in range(P1)]
    W = np.empty((V.shape[0], len(t)))
    for i, ti in enumerate(t):
        acc = np.zeros(shape)
        for j in range(P1):
            acc += beta[i][j] * phi_ld(j, ti * lam) * coeffs[j]
        W[:, i] = scipy.fft.idstn(acc, type=1, norm="ortho", axes=axes).ravel()
    return W


def expm_multiply_aug(csr, t, beta, V) -> np.ndarray:
    """Exact-to-~1e-14 W via scipy expm_multiply on the augmented sparse
    matrix, one abscissa at a time.  csr = (rowptr, col, val)."""
    rp, ci, va = csr
    n = len(rp) - 1
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    P1 = V.shape[1]
    p = P1 - 1
    W = np.empty((n, len(t)))
    for i, ti in enumerate(t):
        blocks_top = [ti * A]
        if p > 0:
            Wb = np.stack([beta[i][p - c] * V[:, p - c] for c in range(p)], axis=1)
            blocks_top.append(sp.csr_matrix(Wb))
            Jp = sp.diags([np.ones(p - 1)], [1], shape=(p, p)) if p > 1 else sp.csr_matrix((1, 1))
            M = sp.bmat([blocks_top, [None, Jp]], format="csr")
        else:
            M = (ti * A).tocsr()
        rhs = np.zeros(n + p)
        rhs[:n] = beta[i][0] * V[:, 0]
        if p > 0:
            rhs[n + p - 1] = 1.0
        W[:, i] = spla.expm_multiply(M, rhs)[:n]
    return W


def expm_multiply_dense_aug(A, t, beta, V) -> np.ndarray:
    """W for a dense operator via scipy expm_multiply on the dense augmented
    matrix of Theorem 1 (same construction as expm_multiply_aug)."""
    rp = np.arange(0, A.size + 1, A.shape[1], dtype=np.int64)
    ci = np.tile(np.arange(A.shape[1]), A.shape[0])
    return expm_multiply_aug((rp, ci, np.ascontiguousarray(A).ravel()), t, beta, V)


_EXACT_Q = None


def _exact_q_lib():
    """Build (once, with gcc) and load the quadruple-precision augmented
    exponential of exact_q.c."""
    global _EXACT_Q
    if _EXACT_Q is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        out_dir = os.path.join(here, "_build")
        os.makedirs(out_dir, exist_ok=True)
        lib = os.path.join(out_dir, "libexact_q.so")
        src = os.path.join(here, "exact_q.c")
        if os.environ.get("PHICOMB_EXACT_Q_LIB"):   # a sanitized build (test_sanitizers)
            lib = os.environ["PHICOMB_EXACT_Q_LIB"]
        elif not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            subprocess.run(["gcc", "-O2", "-shared", "-fPIC", src, "-o", lib + ".tmp",
                            "-lquadmath"], check=True)
            os.replace(lib + ".tmp", lib)
        L = ctypes.CDLL(lib)
        P = ctypes.c_void_p
        L.aug_expm_q.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_double, P, P, P]
        L.aug_expm_q.restype = ctypes.c_int
        _EXACT_Q = L
    return _EXACT_Q


def exact_dense_q(A, t, beta, V) -> np.ndarray:
    """W[:, i] = sum_j beta_ij phi_j(t_i A) v_j from the augmented exponential
    in __float128 (Taylor, scaling and squaring); dense A only."""
    L = _exact_q_lib()
    A = np.ascontiguousarray(A, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, P1 = V.shape
    W = np.empty((n, len(t)))
    for i, ti in enumerate(t):
        b = np.ascontiguousarray(beta[i], dtype=np.float64)
        w = np.empty(n)
        rc = L.aug_expm_q(n, P1 - 1, A.ctypes.data, float(ti), b.ctypes.data, V.ctypes.data,
                          w.ctypes.data)
        assert rc == 0
        W[:, i] = w
    return W


def phi_matrix_mp(k: int, X: np.ndarray, dps: int = 60):
    """phi_k(X) for a small square X: the (1, k+1) block of the exponential of
    the block matrix with X in the corner and identities on the block
    superdiagonal (the standard augmented form), at dps digits."""
    r = X.shape[0]
    N = r * (k + 1)
    with mpmath.workdps(dps):
        B = mpmath.zeros(N, N)
        for a in range(r):
            for b in range(r):
                B[a, b] = mpmath.mpf(X[a, b])
        for blk in range(k):
            for a in range(r):
                B[blk * r + a, (blk + 1) * r + a] = 1
        E = mpmath.expm(B)
        return [[E[a, k * r + b] for b in range(r)] for a in range(r)]


def lowrank_exact(op, t: float, beta_i, V, dps: int = 60) -> np.ndarray:
    """w = sum_j beta_j phi_j(tA) v_j for A = U W^T in closed form (Sec. 5,
    third experiment): sum_j beta_j v_j / j! + U (t sum_j beta_j phi_{j+1}(tM)
    (W^T v_j)); the small phi_{j+1}(tM) at dps digits."""
    U, W, M = op.U, op.W, op.M
    P1 = V.shape[1]
    r = M.shape[0]
    with mpmath.workdps(dps):
        acc = [mpmath.mpf(0)] * r
        for j in range(P1):
            phi = phi_matrix_mp(j + 1, np.asarray(M) * t, dps)
            wv = W.T @ V[:, j]          # r inner products in double (inputs are double)
            for a in range(r):
                s = mpmath.mpf(0)
                for b in range(r):
                    s += phi[a][b] * mpmath.mpf(wv[b])
                acc[a] += mpmath.mpf(beta_i[j]) * mpmath.mpf(t) * s
        coef = np.array([float(x) for x in acc])
    w = U @ coef
    for j in range(P1):
        w = w + beta_i[j] * V[:, j] / math.factorial(j)
    return w


def rel1_cols(a, b) -> np.ndarray:
    """Relative 1-norm error per column (the error measure of Table 1)."""
    a = np.asarray(a).reshape(b.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return np.abs(a - b).sum(axis=0) / np.abs(b).sum(axis=0)


def rel2(a, b) -> float:
    """Relative 2-norm error ||a-b||/||b|| (Frobenius over all columns)."""
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def rel2_cols(a, b) -> np.ndarray:
    a = np.asarray(a).reshape(b.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def ode_reference(op, gc, u0, t_end: float, rtol: float = 1e-12):
    """u(t_end) of u' = A u + g(u) (g the cubic with coefficients gc) by
    scipy's explicit Runge-Kutta DOP853 at rtol = atol (the paper's fourth
    experiment uses a stiff solver at 1e-12 for its reference)."""
    from scipy.integrate import solve_ivp
    import scipy.sparse as sp
    rp, ci, va = op.csr()
    A = sp.csr_matrix((va, ci, rp), shape=(op.n, op.n))

    def rhs(_t, u):
        return A @ u + (gc[0] + u * (gc[1] + u * (gc[2] + u * gc[3])))

    sol = solve_ivp(rhs, (0.0, t_end), np.asarray(u0, dtype=np.float64), method="DOP853",
                    rtol=rtol, atol=rtol, t_eval=[t_end])
    assert sol.success, sol.message
    return sol.y[:, -1]
