"""Seeded synthetic workloads for the phi-combination method.

This module only *builds inputs*: operators (as stencil descriptions, CSR
arrays or dense matrices), the vectors v_0..v_p, abscissae t_i, weight
tables, tolerances and the unit-vector seed for the parameter search.
It contains none of the method's arithmetic, and it is the only code that
the CPU oracle and the HIP library both consume.

Problem statement being fed: w_i = sum_j beta_ij phi_j(t_i A) v_j,
i = 1..r (paper, Sec. 1, eq. (phi.comb)); the paper's case is
beta_ij = alpha_i^j.

Layouts handed out:
  * V: float64 [n][p+1], row-major, natural order j = 0..p.
  * beta: float64 [r][p+1], row-major.
  * CSR: int32 rowptr[n+1], int32 col[nnz] (ascending within a row),
    float64 val[nnz].
  * dense: float64 [n][n], row-major.
  * stencil: 7 coefficients (centre, -x, +x, -y, +y, -z, +z) plus an
    optional constant added on the matrix superdiagonal (i, i+1) for every
    i < n-1 (a non-normal perturbation; at the end of a grid line it is a
    new "wrap" entry).  Grid index i = x + nx*(y + ny*z), x fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Stencil", "Dense", "Problem", "stencil_to_csr", "laplacian_2d",
    "laplacian_3d", "convdiff_2d_upwind", "dense_upper_nonnormal",
    "config1", "config2", "config3", "config4", "config5_stream",
    "small_problem", "params_vector", "LowRank", "dct2_basis", "lowrank_cores",
    "lowrank_operator", "exp3_problem", "EXP3_SHAPES", "ADR", "adr_operator",
    "adr_initial", "adr_reaction", "adr_steps",
]


# --------------------------------------------------------------------------
# operators
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Stencil:
    """Constant-coefficient 5-point (dim=2) or 7-point (dim=3) stencil."""
    dim: int
    grid: tuple          # (nx, ny, nz); nz == 1 for dim == 2
    coef: np.ndarray     # float64[7]: centre, -x, +x, -y, +y, -z, +z
    superdiag: float = 0.0
    kind: str = "stencil"

    @property
    def n(self) -> int:
        nx, ny, nz = self.grid
        return nx * ny * nz

    def csr(self):
        return stencil_to_csr(self)

    def dense(self) -> np.ndarray:
        rp, ci, va = self.csr()
        n = self.n
        A = np.zeros((n, n))
        rows = np.repeat(np.arange(n), np.diff(rp))
        A[rows, ci] = va
        return A


@dataclasses.dataclass
class Dense:
    A: np.ndarray        # float64 [n][n] row-major
    kind: str = "dense"

    @property
    def n(self) -> int:
        return self.A.shape[0]

    def csr(self):
        n = self.n
        rp = (np.arange(n + 1, dtype=np.int64) * n).astype(np.int32)
        ci = np.tile(np.arange(n, dtype=np.int32), n)
        return rp, ci, np.ascontiguousarray(self.A, dtype=np.float64).ravel()

    def dense(self) -> np.ndarray:
        return self.A


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    kind: str = "csr"

    def csr(self):
        return self.rowptr, self.col, self.val

    def dense(self) -> np.ndarray:
        A = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        A[rows, self.col] = self.val
        return A


def stencil_to_csr(st: Stencil):
    """Expand a stencil description to CSR (ascending columns per row)."""
    nx, ny, nz = st.grid
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    c = np.asarray(st.coef, dtype=np.float64)
    slots = []  # (offset, valid mask, value array) in ascending column order
    if st.dim == 3:
        slots.append((-nx * ny, z > 0, np.full(n, c[5])))
    slots.append((-nx, y > 0, np.full(n, c[3])))
    slots.append((-1, x > 0, np.full(n, c[1])))
    slots.append((0, np.ones(n, bool), np.full(n, c[0])))
    xp_valid = x < nx - 1
    sd_valid = (idx < n - 1) & (st.superdiag != 0.0)
    xp_val = np.where(xp_valid, c[2], 0.0) + np.where(sd_valid, st.superdiag, 0.0)
    slots.append((1, xp_valid | sd_valid, xp_val))
    slots.append((nx, y < ny - 1, np.full(n, c[4])))
    if st.dim == 3:
        slots.append((nx * ny, z < nz - 1, np.full(n, c[6])))
    valid = np.stack([s[1] for s in slots], axis=1)
    cols = np.stack([idx + s[0] for s in slots], axis=1)
    vals = np.stack([s[2] for s in slots], axis=1)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[valid].astype(np.int32)
    val = vals[valid].astype(np.float64)
    return rowptr.astype(np.int32), col, val


def laplacian_2d(nx: int, ny: Optional[int] = None, kappa: float = 1.0) -> Stencil:
    """kappa * 5-point Dirichlet Laplacian on an nx*ny interior grid of the
    unit square, mesh width h = 1/(nx+1) (and 1/(ny+1) in y)."""
    ny = nx if ny is None else ny
    hx2 = (nx + 1.0) ** 2
    hy2 = (ny + 1.0) ** 2
    coef = np.array([-2 * kappa * (hx2 + hy2), kappa * hx2, kappa * hx2,
                     kappa * hy2, kappa * hy2, 0.0, 0.0])
    return Stencil(2, (nx, ny, 1), coef)


def laplacian_3d(nside: int, kappa: float = 1.0, superdiag: float = 0.0) -> Stencil:
    """kappa * 7-point Dirichlet Laplacian on an nside^3 interior grid,
    h = 1/(nside+1); optional constant on the matrix superdiagonal."""
    h2 = (nside + 1.0) ** 2
    coef = np.array([-6 * kappa * h2] + [kappa * h2] * 6)
    return Stencil(3, (nside, nside, nside), coef, float(superdiag))


def convdiff_2d_upwind(nside: int, diff: float = 1.0, vel=(50.0, 50.0)) -> Stencil:
    """u_t = diff*Lap(u) - b.grad(u) on the unit square, Dirichlet, nside^2
    interior points, h = 1/(nside+1), first-order upwind (backward
    differences for b > 0)."""
    h = 1.0 / (nside + 1.0)
    d = diff / h ** 2
    bx, by = vel
    coef = np.array([-4 * d - (bx + by) / h,
                     d + bx / h, d,      # -x (upwind side), +x
                     d + by / h, d,      # -y (upwind side), +y
                     0.0, 0.0])
    return Stencil(2, (nside, nside, 1), coef)


def dense_upper_nonnormal(n: int, rng: np.random.Generator, diag_max: float = 50.0) -> Dense:
    """Upper-triangular dense A: strictly-upper entries N(0,1), diagonal
    -U(0, diag_max)."""
    A = np.triu(rng.standard_normal((n, n)), 1)
    A[np.arange(n), np.arange(n)] = -rng.uniform(0.0, diag_max, n)
    return Dense(np.ascontiguousarray(A))


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    name: str
    op: object            # Stencil | Dense | CSR
    p: int
    r: int
    t: np.ndarray         # float64[r]
    beta: np.ndarray      # float64[r][p+1]
    V: np.ndarray         # float64[n][p+1] row-major
    tol: float
    v: np.ndarray         # float64[n]: start vector of the parameter search
    alpha: Optional[np.ndarray] = None   # float64[r] when beta_ij = alpha_i^j

    @property
    def n(self) -> int:
        return self.op.n


def vandermonde(alpha: Sequence[float], p: int) -> np.ndarray:
    a = np.asarray(alpha, dtype=np.float64)
    return np.ascontiguousarray(a[:, None] ** np.arange(p + 1)[None, :])


def params_vector(n: int, seed: int = 1) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


def _V_normal(n, p, seed, normalise=False):
    V = np.random.default_rng(seed).standard_normal((p + 1, n))
    if normalise:
        V /= np.linalg.norm(V, axis=1, keepdims=True)
    return np.ascontiguousarray(V.T)


def _V_uniform(n, p, seed):
    V = np.random.default_rng(seed).uniform(-1.0, 1.0, (p + 1, n))
    return np.ascontiguousarray(V.T)


def config1() -> Problem:
    """2-D Laplacian, 20x20 interior (n=400), p=3, r=1, t=1e-3, alpha=1,
    tol=2^-53, V ~ N(0,1) from seed 0."""
    op = laplacian_2d(20)
    p, r = 3, 1
    alpha = np.ones(r)
    return Problem("cfg1_lap2d_20", op, p, r, np.array([1e-3]),
                   vandermonde(alpha, p), _V_normal(op.n, p, 0),
                   2.0 ** -53, params_vector(op.n, 1), alpha)


def config2(nside: int = 512, as_csr: bool = True) -> Problem:
    """2-D upwind convection-diffusion 512^2 (n=262144), velocity (50,50),
    p=3, r=3, t_i = c_i*1e-4 with c = (1/2, 1/3, 1), beta_ij = c_i^j,
    v_j ~ N(0,1) normalised, tol=1e-12."""
    st = convdiff_2d_upwind(nside)
    op = st
    if as_csr:
        rp, ci, va = st.csr()
        op = CSR(st.n, rp, ci, va)
    p, r = 3, 3
    c = np.array([0.5, 1.0 / 3.0, 1.0])
    return Problem(f"cfg2_convdiff2d_{nside}", op, p, r, c * 1e-4,
                   vandermonde(c, p), _V_normal(st.n, p, 0, normalise=True),
                   1e-12, params_vector(st.n, 1), c)


def config3(nside: int = 128, nonnormal: bool = False, tol: float = 1e-12) -> Problem:
    """3-D Laplacian 128^3 (n=2097152), optional +100 on the matrix
    superdiagonal, p=2, r=2, t = (0.5, 1)*1e-3, alpha_i = t_i/1e-3,
    v_j ~ U(-1,1)."""
    op = laplacian_3d(nside, superdiag=100.0 if nonnormal else 0.0)
    p, r = 2, 2
    c = np.array([0.5, 1.0])
    return Problem(f"cfg3_lap3d_{nside}{'_nn' if nonnormal else ''}", op, p, r,
                   c * 1e-3, vandermonde(c, p), _V_uniform(op.n, p, 0), tol,
                   params_vector(op.n, 1), c)


def chebyshev_laplacian(N: int = 100, L: float = 2.0) -> Dense:
    """Second-derivative operator on [0, L] with homogeneous Dirichlet
    conditions by Chebyshev spectral collocation (Sec. 5, second experiment).

    Built from the entrywise definition of the first-derivative collocation
    matrix on the Chebyshev extreme points xi_k = cos(k pi / N), k = 0..N, of
    [-1, 1] (Trefethen, Spectral Methods in MATLAB, ch. 6): for k != l,
        D[k, l] = (w_k / w_l) (-1)^(k+l) / (xi_k - xi_l),
    with w_0 = w_N = 2 and w_k = 1 otherwise; each diagonal entry is minus
    the sum of the other entries of its row (D annihilates constants).  The
    affine map x = (xi + 1) L / 2 scales d/dx = (2/L) d/dxi, so the second
    derivative is (2/L)^2 D^2; the Dirichlet conditions remove the two
    boundary rows and columns.  A is (N-1) x (N-1), dense, non-normal, with
    eigenvalues on the negative real axis."""
    xi = [math.cos(k * math.pi / N) for k in range(N + 1)]
    w = [2.0 if k in (0, N) else 1.0 for k in range(N + 1)]
    D = np.zeros((N + 1, N + 1))
    for k in range(N + 1):
        off = 0.0
        for l in range(N + 1):
            if l == k:
                continue
            sign = -1.0 if (k + l) % 2 else 1.0
            D[k, l] = (w[k] / w[l]) * sign / (xi[k] - xi[l])
            off += D[k, l]
        D[k, k] = -off
    A = (2.0 / L) ** 2 * (D @ D)
    return Dense(np.ascontiguousarray(A[1:N, 1:N]))


def exp2_problems(seed: int = 0, N: int = 100) -> List[Problem]:
    """Second experiment of Sec. 5: the collocation Laplacian above (N = 100,
    L = 2, n = 99), p = 6, one solve per t_i = 10^(i-5), i = 1..5 (Table 1
    reports each t on its own), weights t_i^j (alpha = t_i), the same
    v_j ~ N(0,1) for every t, tol = 2^-53."""
    op = chebyshev_laplacian(N)
    p = 6
    V = _V_normal(op.n, p, seed)
    out = []
    for i in range(1, 6):
        t = np.array([10.0 ** (i - 5)])
        out.append(Problem(f"exp2_cheb_lap_99_t1e{i - 5}", op, p, 1, t, vandermonde(t, p), V,
                           2.0 ** -53, params_vector(op.n, 1), t))
    return out


@dataclasses.dataclass
class LowRank:
    """Matrix-free A = U W^T (third experiment of Sec. 5): U, W are n x r."""
    U: np.ndarray
    W: np.ndarray
    M: np.ndarray        # the r x r core, W = U M^T
    kind: str = "lowrank"

    @property
    def n(self) -> int:
        return self.U.shape[0]


def dct2_basis(n: int, r: int) -> np.ndarray:
    """First r columns of the orthonormal DCT-II matrix:
    U_ik = sqrt(2/n) a_k cos(pi (i + 1/2) k / n), a_0 = 1/sqrt(2), a_k = 1."""
    i = np.arange(n)[:, None] + 0.5
    k = np.arange(r)[None, :]
    a = np.where(k == 0, 1.0 / math.sqrt(2.0), 1.0)
    return np.ascontiguousarray(math.sqrt(2.0 / n) * a * np.cos(np.pi * i * k / n))


def lowrank_cores() -> dict:
    """The three cores of the third experiment (Sec. 5): M1 skew-symmetric
    (normal A, eigenvalues +-10i), M2 upper triangular with a 1e5 coupling
    (non-normal), M3 Moler's 3 x 3 core (eigenvalues about -63.4, -6.2,
    -0.11, departure from normality ~2.8e10)."""
    a, b, c, d, e = 2e10, 4e8 / 6.0, 200.0 / 3.0, 3.0, 1e-8
    return {
        "M1": np.array([[0.0, 10.0], [-10.0, 0.0]]),
        "M2": np.array([[-1.0, 1e5], [0.0, -10.0]]),
        "M3": np.array([[0.0, e, 0.0], [-(a + b), -d, a], [c, 0.0, -c]]),
    }


def lowrank_operator(core: np.ndarray, n: int) -> LowRank:
    U = dct2_basis(n, core.shape[0])
    return LowRank(U, np.ascontiguousarray(U @ core.T), np.asarray(core, dtype=np.float64))


# sizes and p of the three cores in the paper (n, p)
EXP3_SHAPES = {"M1": (200000, 3), "M2": (400000, 4), "M3": (500000, 2)}


def exp3_problem(core_name: str, t: float, n: Optional[int] = None, seed: int = 0) -> Problem:
    """One solve of the third experiment: A = U W^T with the named core, the
    paper's n and p (or a given n), alpha = 1 (beta_j = 1), V ~ N(0,1),
    tol = 2^-53, a single abscissa t."""
    n0, p = EXP3_SHAPES[core_name]
    n = n0 if n is None else n
    op = lowrank_operator(lowrank_cores()[core_name], n)
    ta = np.array([float(t)])
    return Problem(f"exp3_{core_name}_n{n}_t{t:g}", op, p, 1, ta, np.ones((1, p + 1)),
                   _V_normal(n, p, seed), 2.0 ** -53, params_vector(n, 1), np.ones(1))


# Fourth experiment of Sec. 5: 2-D advection-diffusion-reaction
#   u_t = eps Lap u - alpha (u_x + u_y) + gamma u (u - 1/2)(1 - u)  on [0,1]^2,
# homogeneous Neumann on x = 0 and y = 0, homogeneous Dirichlet on x = 1 and
# y = 1, u(0) = 256 x^2 y^2 (1-x)^2 (1-y)^2, t in [0, 1/2].
ADR = {"eps": 1e-3, "alpha": -0.5, "gamma": 1000.0, "t_end": 0.5, "N": 100}


def adr_operator(N: int = 100, eps: float = 1e-3, alpha: float = -0.5) -> CSR:
    """Second-order finite differences of eps Lap - alpha (d/dx + d/dy) on the
    N x N unknowns x_i = i/N, i = 0..N-1 (x = 1 is the Dirichlet boundary and
    carries no unknown), the same in y, grid index i + N j.  The Neumann
    condition at x = 0 (y = 0) is imposed with the mirrored ghost value
    u_{-1} = u_1: the diffusion row becomes (2 u_1 - 2 u_0)/h^2 and the
    central advection difference vanishes there."""
    h = 1.0 / N
    d2 = eps / h ** 2
    d1 = -alpha / (2.0 * h)        # coefficient of (u_{i+1} - u_{i-1})
    rows, cols, vals = [], [], []
    for j in range(N):
        for i in range(N):
            k = i + N * j
            ent = {k: -4.0 * d2}
            for (ii, jj, axis) in ((i, j, 0), (j, i, 1)):
                step = 1 if axis == 0 else N
                if ii == 0:              # mirrored ghost: u_{-1} = u_1
                    ent[k + step] = ent.get(k + step, 0.0) + 2.0 * d2
                else:
                    ent[k - step] = ent.get(k - step, 0.0) + d2 - d1
                    if ii < N - 1:
                        ent[k + step] = ent.get(k + step, 0.0) + d2 + d1
            for c in sorted(ent):
                rows.append(k)
                cols.append(c)
                vals.append(ent[c])
    rows = np.asarray(rows)
    rp = np.zeros(N * N + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return CSR(N * N, rp, np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float64))


def adr_initial(N: int = 100) -> np.ndarray:
    x = np.arange(N) / N
    X, Y = np.meshgrid(x, x, indexing="xy")      # X varies along the fast index
    return np.ascontiguousarray((256.0 * X ** 2 * Y ** 2 * (1 - X) ** 2 * (1 - Y) ** 2).ravel())


def adr_reaction(gamma: float = 1000.0) -> np.ndarray:
    """g(u) = gamma u (u - 1/2)(1 - u) as cubic coefficients c0 + c1 u + c2 u^2 + c3 u^3."""
    return np.array([0.0, -0.5 * gamma, 1.5 * gamma, -gamma])


def adr_steps(i: int) -> tuple:
    """Step size h_i = 2^-8 (t_end - t0)/(i + 1), i = 1..7, and the number
    of steps that reach t_end."""
    nsteps = 256 * (i + 1)
    return ADR["t_end"] / nsteps, nsteps


def config4(count: int = 256, seed: int = 0, side_range=(32, 256)) -> List[Problem]:
    """Batched uneven instances: 2-D kappa*Laplacians, side ~ U{32..256},
    kappa ~ logU[1e-2, 1e2], p ~ U{1,2,3}, r ~ U{1,2,3},
    t_i ~ logU[1e-5, 1e-2], beta = 1, v_j ~ N(0,1), tol = 1e-8."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        kappa = float(10.0 ** rng.uniform(-2, 2))
        p = int(rng.integers(1, 4))
        r = int(rng.integers(1, 4))
        t = 10.0 ** rng.uniform(-5, -2, r)
        op = laplacian_2d(side, kappa=kappa)
        V = np.ascontiguousarray(rng.standard_normal((p + 1, op.n)).T)
        out.append(Problem(f"cfg4_{k}", op, p, r, t, np.ones((r, p + 1)), V,
                           1e-8, params_vector(op.n, 1), np.ones(r)))
    return out


def config5_stream(duration_s: float = 60.0, rate: float = 200.0, seed: int = 0,
                   n_stencil_ops: int = 64, n_dense_ops: int = 32,
                   n_range=(4096, 1 << 20), dense_sizes=(256, 512, 1024, 2048)):
    """Served stream: Poisson arrivals; 70% stencil requests (2-D/3-D,
    n ~ logU[4096, 2^20]) and 30% dense non-normal requests.  Operators
    come from a resident pool; each request draws p ~ U{1..4},
    r ~ U{1..3}, tol in {1e-6, 1e-10}, alpha = 1,
    t_i = (i/r) * gamma / ||A||_inf with gamma ~ logU[0.1, 100].

    Returns (ops, requests) where requests are dicts with keys
    arrival, op_index, p, r, t, tol, seed (V is drawn from the seed)."""
    rng = np.random.default_rng(seed)
    ops = []
    for k in range(n_stencil_ops):
        dim = 2 if k % 2 == 0 else 3
        n_target = 10.0 ** rng.uniform(math.log10(n_range[0]), math.log10(n_range[1]))
        side = max(4, int(round(n_target ** (1.0 / dim))))
        ops.append(laplacian_2d(side) if dim == 2 else laplacian_3d(side))
    for k in range(n_dense_ops):
        ops.append(dense_upper_nonnormal(int(dense_sizes[k % len(dense_sizes)]), rng))
    t_now = 0.0
    reqs = []
    while True:
        t_now += rng.exponential(1.0 / rate)
        if t_now >= duration_s:
            break
        if rng.uniform() < 0.7:
            oi = int(rng.integers(0, n_stencil_ops))
        else:
            oi = n_stencil_ops + int(rng.integers(0, n_dense_ops))
        p = int(rng.integers(1, 5))
        r = int(rng.integers(1, 4))
        gamma = 10.0 ** rng.uniform(-1, 2)
        tol = 1e-6 if rng.uniform() < 0.5 else 1e-10
        reqs.append(dict(arrival=t_now, op_index=oi, p=p, r=r, gamma=gamma,
                         tol=tol, seed=int(rng.integers(0, 2 ** 31))))
    return ops, reqs


def inf_norm_bound(op) -> float:
    """max_i sum_j |a_ij| of an operator description (problem setup only)."""
    if op.kind == "dense":
        return float(np.abs(op.A).sum(axis=1).max())
    rp, ci, va = op.csr()
    rows = np.repeat(np.arange(op.n), np.diff(rp))
    return float(np.bincount(rows, weights=np.abs(va), minlength=op.n).max())


def stream_request_inputs(op, req):
    """Materialise t, beta and V of one served request."""
    rng = np.random.default_rng(req["seed"])
    r, p = req["r"], req["p"]
    t = (np.arange(1, r + 1) / r) * req["gamma"] / inf_norm_bound(op)
    V = np.ascontiguousarray(rng.standard_normal((p + 1, op.n)).T)
    return t, np.ones((r, p + 1)), V


def small_problem(n: int, p: int, r: int, seed: int = 0, kind: str = "dense",
                  spread: float = 10.0, vandermonde_weights: bool = False,
                  t_scale: float = 1.0) -> Problem:
    """Tiny random non-normal test problem (for exact-reference checks)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * (spread / math.sqrt(n))
    A -= np.diag(rng.uniform(0, spread, n))
    op = Dense(np.ascontiguousarray(A))
    t = t_scale * rng.uniform(0.2, 1.0, r) * np.where(rng.uniform(size=r) < 0.2, -1, 1)
    if vandermonde_weights:
        alpha = rng.uniform(0.3, 1.5, r)
        beta = vandermonde(alpha, p)
    else:
        alpha = None
        beta = rng.uniform(-1.5, 1.5, (r, p + 1))
    V = np.ascontiguousarray(rng.standard_normal((n, p + 1)))
    return Problem(f"small_{kind}_{n}_{p}_{r}_{seed}", op, p, r, t, beta, V,
                   2.0 ** -53, params_vector(n, seed + 1), alpha)
