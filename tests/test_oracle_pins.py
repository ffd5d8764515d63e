"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check compares the oracle with something computed another way:
closed forms of the phi-functions (Sec. 1, (def.phik)), the exact
augmented-matrix exponential (Theorem 1 and the reference solutions of
Sec. 5), eigen-decompositions of Laplacians, scipy's expm_multiply, or
invariants the method must satisfy (independence of the shift and the
scaling, Corollary of Theorem 1, Algorithm 3 with r = 1 = Algorithm 2).
"""
import math

import numpy as np
import pytest

import refs
import workloads as wl


def _diag_op(lams):
    n = len(lams)
    return wl.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                  np.asarray(lams, dtype=np.float64))


# ---------------------------------------------------------------- Alg 1 parts
def test_binomials_are_correctly_rounded(orc):
    for m in (5, 61, 100):
        for k in range(m + 1):
            assert orc.binom(m, k) == float(math.comb(m, k))


@pytest.mark.parametrize("f,a,b,xmin", [
    (lambda x: (x - 0.3) ** 2 + 1.0, -10.0, 10.0, 0.3),
    (lambda x: abs(x - 1.7) + 2.0, -5.0, 9.0, 1.7),
    (lambda x: math.cos(x), 2.0, 5.0, math.pi),
    (lambda x: (x + 400.0) ** 4, -512.0, 512.0, -400.0),
    (lambda x: x, -3.0, 4.0, -3.0),                    # minimum at the end point
])
def test_brent_finds_known_minima(orc, f, a, b, xmin):
    x, fx, nfev = orc.brent_min(f, a, b, abs_tol=1e-7)
    tol = 3 * (1.5e-8 * abs(xmin) + 1e-7) + 1e-6
    if abs(xmin - a) < 1e-12 or abs(xmin - b) < 1e-12:
        tol = 1e-5
    assert abs(x - xmin) <= max(tol, 2e-3 if "abs" in str(f) else tol), (x, xmin)
    assert nfev <= 101


def test_power_basis_guard_and_s0_for_scaled_identity(orc):
    """A = c I with log c = 20: L_k = 20 k, the guard of Algorithm 1 accepts
    k while 20k + log(k+1)/2 + max_j log binom(61,j) <= 0.8 log(realmax):
    k <= 26; s0 is exactly c; the objective |c - xi|/c is minimised at xi = c."""
    c = math.exp(20.0)
    n = 7
    op = _diag_op([c] * n)
    v = np.random.default_rng(3).standard_normal(n)
    prm = orc.params(op, 2.0 ** -53, v)
    lmax = max(math.lgamma(62) - math.lgamma(j + 1) - math.lgamma(62 - j) for j in range(62))
    gmax = 0.8 * math.log(np.finfo(float).max)
    k_expected = max(k for k in range(1, 62) if 20.0 * k + 0.5 * math.log(k + 1) + lmax <= gmax)
    assert k_expected == 26
    assert prm["r_acc"] == k_expected
    np.testing.assert_allclose(prm["L"][1:k_expected + 1], 20.0 * np.arange(1, k_expected + 1),
                               rtol=1e-14)
    assert abs(prm["s0"] / c - 1) < 1e-13
    # With m = 61 the objective sum_k binom(m,k) z^(m-k) V_k = (1+z)^m v is
    # evaluated with cancellation of size (1+|z|)^m, so the computed f has a
    # floor near eps^(1/m)(1+|z|) and its minimiser sits where
    # 1+z = eps^(1/m)(1-z), i.e. z ~ -0.29, not at z = -1 (xi = c).
    assert 0.15 < prm["shift"] / c < 0.45
    assert 0.6 < prm["fstar"] < 0.8
    # A low degree has a negligible floor: the minimiser is xi = c.
    prm4 = orc.params(op, 2.0 ** -53, v, m=4)
    assert abs(prm4["s0"] / c - 1) < 1e-13
    assert abs(prm4["shift"] / c - 1) < 1e-3
    assert prm4["fstar"] < 1e-3


def test_power_basis_log_norms_match_direct_powers(orc):
    rng = np.random.default_rng(5)
    n = 12
    A = rng.standard_normal((n, n)) * 3 - 4 * np.eye(n)
    v = rng.standard_normal(n)
    prm = orc.params(wl.Dense(A), 1e-10, v)
    x = v / np.linalg.norm(v)
    for k in range(1, prm["r_acc"] + 1):
        x = A @ x
        assert abs(prm["L"][k] - math.log(np.linalg.norm(x))) < 1e-12 * max(1.0, k)


def test_params_objective_is_minimised_over_the_bracket(orc):
    """f(xi*) is no larger than f at the interval centre xi = 0, which for a
    diagonal operator is ||A^m v||^(1/m)/s0 (direct evaluation)."""
    lam = -np.linspace(1.0, 300.0, 40)
    op = _diag_op(lam)
    v = np.random.default_rng(0).standard_normal(40)
    prm = orc.params(op, 1e-8, v)
    u = v / np.linalg.norm(v)
    f0 = math.exp((math.log(np.linalg.norm(np.abs(lam) ** 61 * u)) / 61)) / prm["s0"]
    assert prm["fstar"] <= f0 * (1 + 1e-12)
    # the shift lies inside the spectral interval and s obeys s0 f*/theta
    assert -300 <= prm["shift"] <= -1
    theta = math.exp((math.log(1e-8) + math.lgamma(62)) / 61)
    assert abs(prm["s"] - prm["s0"] * prm["fstar"] / theta) <= 1e-12 * prm["s"]


@pytest.mark.parametrize("m", [4, 6, 8])
def test_params_two_point_spectrum(orc, m):
    """Spectrum {-c, 0} with equal weights on a unit v: every power has the
    growth ratio c, so s0 = c; the objective is
    f(z)^(2m) = ((z-1)^(2m) + z^(2m))/2, minimised at z = 1/2, so
    xi* = -c/2 and f* = 1/2 (low m: negligible rounding floor)."""
    c = 300.0
    op = _diag_op([-c] * 4 + [0.0] * 4)
    prm = orc.params(op, 1e-10, np.ones(8), m=m)
    assert abs(prm["s0"] / c - 1) < 1e-13
    assert abs(prm["shift"] / (-0.5 * c) - 1) < 1e-4
    assert abs(prm["fstar"] / 0.5 - 1) < 1e-6


def test_params_short_basis_fallback(orc):
    """m = 2 accepts only two powers: s0 = exp(L_2/2) (the reading for a
    basis too short for the mean of the last ratios); here L_2 = log(c^2/sqrt 2)."""
    c = 300.0
    prm = orc.params(_diag_op([-c] * 4 + [0.0] * 4), 1e-10, np.ones(8), m=2)
    assert prm["r_acc"] == 2
    assert abs(prm["s0"] / (c * 2.0 ** -0.25) - 1) < 1e-13


def test_params_zero_operator(orc):
    op = _diag_op(np.zeros(5))
    prm = orc.params(op, 1e-10, np.ones(5))
    assert prm["r_acc"] == 0 and prm["shift"] == 0.0 and prm["s"] == 1.0


def test_params_overflow_guard(orc):
    op = _diag_op(np.full(4, math.exp(600.0)))
    with pytest.raises(orc.OracleError) as e:
        orc.params(op, 1e-10, np.ones(4))
    assert e.value.status == -5


# ------------------------------------------------------------ scalar closed forms
@pytest.mark.parametrize("z", [-60.0, -3.0, -0.25, 0.7, 2.5])
def test_phi1_closed_form(orc, z):
    """1x1 A = [z]: w = phi_1(z) = (e^z - 1)/z."""
    op = _diag_op([z])
    V = np.array([[0.0, 1.0]])
    beta = np.array([[1.0, 1.0]])
    prm = orc.params(op, 2.0 ** -53, np.ones(1))
    for xi, s in [(prm["shift"], prm["s"]), (0.0, max(abs(z), 1.0)), (0.5 * z, 2 * abs(z) + 1)]:
        W, _ = orc.solve(op, 1, 1, [1.0], beta, V, 2.0 ** -53, xi, s)
        exact = math.expm1(z) / z
        assert abs(W[0, 0] - exact) <= 2e-14 * abs(exact), (xi, s, W[0, 0], exact)


@pytest.mark.parametrize("z", [-40.0, -2.0, -0.3, 1.2])
def test_phi_recurrence_and_closed_forms(orc, z):
    """phi_j(z) = z phi_{j+1}(z) + 1/j!, phi_2(z) = (e^z - 1 - z)/z^2."""
    op = _diag_op([z])
    p = 4
    V = np.ones((1, p + 1))
    prm = orc.params(op, 2.0 ** -53, np.ones(1))
    vals = []
    for j in range(p + 1):
        beta = np.zeros((1, p + 1))
        beta[0, j] = 1.0
        W, _ = orc.solve(op, p, 1, [1.0], beta, V, 2.0 ** -53, prm["shift"], prm["s"])
        vals.append(W[0, 0])
    for j in range(p):
        lhs, rhs = vals[j], z * vals[j + 1] + 1.0 / math.factorial(j)
        assert abs(lhs - rhs) <= 2e-14 * max(abs(lhs), 1.0)
    # phi_0 = e^z is only accurate relative to the whole tracked block (the
    # stopping test uses the block infinity norm), so tiny e^z is checked
    # with an absolute floor; every other phi_j relative to itself.
    for j in range(p + 1):
        ex = float(refs.phi_mp(j, z))
        assert abs(vals[j] - ex) <= 2e-14 * abs(ex) + (1e-20 if j == 0 else 0.0), (j, vals[j], ex)


# ------------------------------------------------------------- whole method
def test_diagonal_operator_elementwise(orc):
    rng = np.random.default_rng(11)
    n, p, r = 30, 4, 3
    lam = np.concatenate([-np.geomspace(0.01, 250.0, n - 3), [0.0, 0.8, 3.0]])
    op = _diag_op(lam)
    t = np.array([0.4, -0.15, 1.3])
    beta = rng.uniform(-1.5, 1.5, (r, p + 1))
    V = rng.standard_normal((n, p + 1))
    prm = orc.params(op, 2.0 ** -53, rng.standard_normal(n))
    exact = np.zeros((n, r))
    for i in range(r):
        for k in range(n):
            exact[k, i] = sum(beta[i, j] * float(refs.phi_mp(j, t[i] * lam[k])) * V[k, j]
                              for j in range(p + 1))
    for xi, s in [(prm["shift"], prm["s"]), (-100.0, prm["s"] * 1.3), (0.0, prm["s"] * 2.0)]:
        W, st = orc.solve(op, p, r, t, beta, V, 2.0 ** -53, xi, s)
        assert st["s_int"] >= 2
        assert refs.rel2(W, exact) <= 2e-14, (xi, s, refs.rel2(W, exact))


def test_scaled_identity_whole_method(orc):
    c, n, p, r = -37.0, 9, 3, 2
    rng = np.random.default_rng(2)
    op = _diag_op([c] * n)
    t = np.array([0.3, 1.0])
    beta = wl.vandermonde([0.5, 2.0], p)
    V = rng.standard_normal((n, p + 1))
    W, st, prm = orc.full(wl.Problem("cI", op, p, r, t, beta, V, 2.0 ** -53, np.ones(n),
                                     np.array([0.5, 2.0])))
    phis = [[float(refs.phi_mp(j, ti * c)) for j in range(p + 1)] for ti in t]
    exact = np.stack([V @ (beta[i] * np.array(phis[i])) for i in range(r)], axis=1)
    assert refs.rel2(W, exact) <= 1e-14
    # with the exact shift xi = c the shifted operator vanishes and every
    # Taylor loop stops after its first term
    W2, st2 = orc.solve(op, p, r, t, beta, V, 2.0 ** -53, c, 40.0)
    assert st2["s_int"] == 40 and st2["terms_rec"] <= 2 * 39
    assert refs.rel2(W2, exact) <= 1e-14


@pytest.mark.parametrize("n,p,r,seed,ts", [
    (6, 3, 2, 0, 1.0), (8, 0, 1, 1, 5.0), (7, 5, 3, 2, 20.0), (5, 2, 3, 3, 3.0),
    (9, 1, 1, 4, 12.0), (4, 6, 2, 5, 6.0),
])
def test_small_dense_against_augmented_exponential(orc, n, p, r, seed, ts):
    """Exact w_i = [I 0] exp([[t_i A, W], [0, J_p(0)]]) [beta_i0 v_0; e_p]."""
    pr = wl.small_problem(n, p, r, seed, t_scale=ts, spread=4.0,
                          vandermonde_weights=(seed % 2 == 0))
    exact = refs.exact_dense_mp(pr.op.A, pr.t, pr.beta, pr.V, dps=34)
    W, st, prm = orc.full(pr)
    assert refs.rel2_cols(W, exact).max() <= 1e-12, refs.rel2_cols(W, exact)
    if pr.alpha is not None:
        Wa, st_a = orc.solve(pr.op, p, r, pr.t, None, pr.V, pr.tol, prm["shift"], prm["s"],
                             form="alpha", alpha=pr.alpha)
        assert refs.rel2_cols(Wa, exact).max() <= 1e-12


def test_corollary_alpha_form_equals_prescaled_form(orc):
    pr = wl.small_problem(10, 4, 3, 6, t_scale=15.0, spread=5.0, vandermonde_weights=True)
    prm = orc.params(pr.op, pr.tol, pr.v)
    Wb, sb = orc.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    Wa, sa = orc.solve(pr.op, pr.p, pr.r, pr.t, None, pr.V, pr.tol, prm["shift"], prm["s"],
                       form="alpha", alpha=pr.alpha)
    assert sb["s_int"] >= 3
    assert refs.rel2_cols(Wa, Wb).max() <= 1e-13


@pytest.mark.parametrize("p", [0, 1, 3, 5])
def test_block_with_r1_reduces_to_algorithm2(orc, p):
    pr = wl.small_problem(12, p, 1, 7 + p, t_scale=30.0, spread=6.0, vandermonde_weights=True)
    prm = orc.params(pr.op, pr.tol, pr.v)
    a = float(pr.alpha[0])
    t = float(pr.t[0])
    Wb, sb = orc.solve(pr.op, p, 1, [t], None, pr.V, pr.tol, prm["shift"], prm["s"],
                       form="alpha", alpha=[a])
    ws, ss = orc.solve_single(pr.op, p, t, a, pr.V, pr.tol, prm["shift"], prm["s"])
    assert sb["s_int"] == ss["s_int"] >= 2
    assert refs.rel2(Wb[:, 0], ws) <= 5e-14
    assert abs(sb["terms_S"] - ss["terms_S"]) <= 1
    assert abs(sb["terms_rec"] - ss["terms_rec"]) <= sb["s_int"]


def test_result_is_independent_of_shift_and_scaling(orc):
    pr = wl.config2(nside=24)
    prm = orc.params(pr.op, pr.tol, pr.v)
    t = pr.t * 100.0
    base, st0 = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    assert st0["s_int"] >= 3
    # variants that keep ||t(A - xi I)/s|| no larger than the chosen pair:
    # xi moved towards the spectral centre, or s enlarged
    for dxi, fs in [(-0.1, 1.0), (0.1, 1.5), (-0.15, 1.3), (0.0, 2.0)]:
        W, _ = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol,
                         prm["shift"] + dxi * prm["s0"], prm["s"] * fs)
        assert refs.rel2_cols(W, base).max() <= 1e-11


def test_config1_against_dst(orc):
    pr = wl.config1()
    W, st, prm = orc.full(pr)
    exact = refs.dst_laplacian(pr.op, pr.t, pr.beta, pr.V)
    assert refs.rel2(W, exact) <= 5e-15


@pytest.mark.parametrize("t_mult", [1.0, 60.0])
def test_config1_operator_recovery_steps_against_dst(orc, t_mult):
    pr = wl.config1()
    t = pr.t * t_mult
    prm = orc.params(pr.op, pr.tol, pr.v)
    W, st = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    exact = refs.dst_laplacian(pr.op, t, pr.beta, pr.V)
    assert refs.rel2(W, exact) <= 2e-14
    if t_mult > 1:
        assert st["s_int"] >= 5


@pytest.mark.parametrize("nside,t_mult", [(48, 1.0), (48, 25.0)])
def test_config2_operator_against_expm_multiply(orc, nside, t_mult):
    pr = wl.config2(nside=nside)
    t = pr.t * t_mult
    prm = orc.params(pr.op, pr.tol, pr.v)
    W, st = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    exact = refs.expm_multiply_aug(pr.op.csr(), t, pr.beta, pr.V)
    assert refs.rel2_cols(W, exact).max() <= 2e-13


@pytest.mark.parametrize("nonnormal", [False, True])
def test_config3_operator_reduced(orc, nonnormal):
    pr = wl.config3(nside=20, nonnormal=nonnormal, tol=1e-12)
    t = pr.t * 30.0
    prm = orc.params(pr.op, pr.tol, pr.v)
    W, st = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    assert st["s_int"] >= 3
    if nonnormal:
        exact = refs.expm_multiply_aug(pr.op.csr(), t, pr.beta, pr.V)
    else:
        exact = refs.dst_laplacian(pr.op, t, pr.beta, pr.V)
    assert refs.rel2_cols(W, exact).max() <= 1e-12


@pytest.mark.slow
def test_config2_full_size_against_expm_multiply(orc):
    pr = wl.config2()
    W, st, prm = orc.full(pr)
    exact = refs.expm_multiply_aug(pr.op.csr(), pr.t, pr.beta, pr.V)
    assert st["s_int"] >= 5
    assert refs.rel2_cols(W, exact).max() <= 1e-13


# --------------------------------------------------------------- edge cases
def test_p0_returns_exponential_action(orc):
    pr = wl.config2(nside=20)
    V = pr.V[:, :1]
    t = pr.t * 30
    prm = orc.params(pr.op, pr.tol, pr.v)
    W, st = orc.solve(pr.op, 0, 3, t, np.ones((3, 1)), V, pr.tol, prm["shift"], prm["s"])
    exact = refs.expm_multiply_aug(pr.op.csr(), t, np.ones((3, 1)), V)
    assert refs.rel2_cols(W, exact).max() <= 1e-12


def test_t_zero_gives_weighted_sum(orc):
    rng = np.random.default_rng(1)
    pr = wl.config2(nside=16)
    beta = rng.uniform(-1, 1, (2, 4))
    t = np.array([0.0, 0.0])
    prm = orc.params(pr.op, pr.tol, pr.v)
    W, st = orc.solve(pr.op, 3, 2, t, beta, pr.V, pr.tol, prm["shift"], prm["s"])
    fact = np.array([1.0 / math.factorial(j) for j in range(4)])
    exact = pr.V @ (beta * fact).T
    assert st["s_int"] == 1
    assert refs.rel2(W, exact) <= 1e-15


def test_zero_operator(orc):
    n, p = 6, 2
    op = _diag_op(np.zeros(n))
    V = np.random.default_rng(4).standard_normal((n, p + 1))
    W, st, prm = orc.full(wl.Problem("zero", op, p, 1, np.array([0.7]), np.ones((1, p + 1)), V,
                                     1e-12, np.ones(n), np.ones(1)))
    exact = V @ np.array([1.0, 1.0, 0.5])
    assert refs.rel2(W[:, 0], exact) <= 1e-15


def test_v0_zero(orc):
    pr = wl.small_problem(7, 3, 2, 9, t_scale=4.0, spread=4.0)
    pr.V[:, 0] = 0.0
    exact = refs.exact_dense_mp(pr.op.A, pr.t, pr.beta, pr.V, dps=34)
    W, st, prm = orc.full(pr)
    assert refs.rel2_cols(W, exact).max() <= 1e-12


def test_invalid_inputs_and_term_cap(orc):
    pr = wl.config2(nside=16)
    with pytest.raises(orc.OracleError) as e:
        orc.solve(pr.op, 3, 3, [np.nan, 1e-4, 1e-4], pr.beta, pr.V, 1e-12, 0.0, 1e5)
    assert e.value.status == -1
    with pytest.raises(orc.OracleError) as e:
        orc.solve(pr.op, 3, 3, pr.t, pr.beta, pr.V, 1e-12, 0.0, 1e5, kcap=3)
    assert e.value.status == -4
    with pytest.raises(orc.OracleError) as e:
        orc.solve(pr.op, 3, 3, [1e300, 1, 1], pr.beta, pr.V, 1e-12, 0.0, 1e5)
    assert e.value.status == -1


def test_cost_grows_linearly_with_scaling_count(orc):
    """Total Taylor terms are essentially proportional to ceil(|t| s)."""
    pr = wl.config1()
    prm = orc.params(pr.op, pr.tol, pr.v)
    per_step = []
    for mult in (20.0, 40.0, 80.0):
        _, st = orc.solve(pr.op, pr.p, pr.r, pr.t * mult, pr.beta, pr.V, pr.tol,
                          prm["shift"], prm["s"])
        per_step.append(st["terms_rec"] / (st["s_int"] - 1))
    assert max(per_step) / min(per_step) < 1.15


# ------------------------------------------- second experiment (Sec. 5, Table 1)
def test_exact_q_reference_against_multiprecision():
    """The quadruple-precision augmented exponential used below agrees with
    the 30-digit mpmath one on a small non-normal case."""
    pr = wl.small_problem(7, 3, 2, seed=4, t_scale=3.0)
    Wq = refs.exact_dense_q(pr.op.A, pr.t, pr.beta, pr.V)
    Wm = refs.exact_dense_mp(pr.op.A, pr.t, pr.beta, pr.V, dps=30)
    assert refs.rel2(Wq, Wm) < 1e-15


def test_chebyshev_laplacian_structure():
    """Collocation matrix of the second experiment: 99 x 99, non-normal,
    eigenvalues on the negative real axis, smallest in modulus close to the
    continuous Dirichlet eigenvalue -(pi/L)^2."""
    A = wl.chebyshev_laplacian(100, 2.0).A
    assert A.shape == (99, 99)
    ev = np.linalg.eigvals(A)
    assert np.abs(ev.imag).max() < 1e-6 * np.abs(ev.real).max()
    assert ev.real.max() < 0
    assert abs(ev.real.max() + (math.pi / 2.0) ** 2) < 1e-9
    assert np.linalg.norm(A @ A.T - A.T @ A) > 1e-3 * np.linalg.norm(A) ** 2


@pytest.mark.parametrize("L", [2.0, 3.0])
def test_chebyshev_laplacian_differentiates_polynomials_exactly(L):
    """Collocation is exact on polynomials of degree <= N: for
    u = x (L - x) x^k (zero at both ends, degree k + 2 <= N) the matrix maps
    the interior values of u to those of u'' up to rounding (the
    differentiation matrices amplify it by about N^4 u)."""
    N = 100
    A = wl.chebyshev_laplacian(N, L).A
    x = (np.cos(np.arange(1, N) * math.pi / N) + 1.0) * L / 2.0
    for k in (0, 1, 5, 30, 98):
        u = x * (L - x) * x ** k
        # u = L x^(k+1) - x^(k+2)
        upp = L * (k + 1) * k * x ** max(k - 1, 0) - (k + 2) * (k + 1) * x ** k
        assert np.abs(A @ u - upp).max() <= 1e-9 * np.abs(upp).max(), k


def test_second_experiment_within_table1_envelope(orc):
    """The oracle (Algorithm 1 + Algorithm 3 at tol 2^-53, one solve per t)
    reaches the accuracy the paper reports for its implementation in Table 1
    (relative 1-norm error against an exact reference), within a factor 10,
    for t = 1e-4 .. 1e-1 (t = 1 needs ~2.4e5 scaling steps)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_phimv.json")))
    for pr, env in zip(wl.exp2_problems()[:4], g["rel_err_1norm"][:4]):
        Wq = refs.exact_dense_q(pr.op.A, pr.t, pr.beta, pr.V)
        Wo, st, prm = orc.full(pr)
        err = refs.rel1_cols(Wo, Wq)[0]
        assert err <= 10 * env, (pr.name, err, env)


# ------------------------------------------------ third experiment (low rank)
def test_dct2_basis_is_orthonormal_and_cores_have_stated_spectra():
    """U has orthonormal columns (so A^j = U M^(j-1) W^T), M3 has the
    eigenvalues -63.4, -6.2, -0.11 quoted with it, M1 is skew-symmetric."""
    U = wl.dct2_basis(1000, 4)
    assert np.abs(U.T @ U - np.eye(4)).max() < 1e-13
    cores = wl.lowrank_cores()
    ev = np.sort(np.linalg.eigvals(cores["M3"]).real)
    assert np.allclose(ev, [-63.4, -6.2, -0.11], rtol=2e-2, atol=5e-3), ev
    assert np.array_equal(cores["M1"], -cores["M1"].T)
    op = wl.lowrank_operator(cores["M2"], 500)
    A = op.U @ op.W.T
    assert np.abs(A @ A - op.U @ cores["M2"] @ op.W.T).max() < 1e-8 * np.abs(A).max() ** 2


def test_lowrank_operator_application(orc):
    """The oracle's matrix-free product x -> U (W^T x) equals the assembled
    n x n matrix times x."""
    op = wl.lowrank_operator(wl.lowrank_cores()["M3"], 300)
    x = np.random.default_rng(5).standard_normal(300)
    y = orc.apply(op, x)
    ref = (op.U @ op.W.T) @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(op.U @ op.W.T).max() * np.abs(x).sum()


@pytest.mark.parametrize("core,t", [("M1", 1.0), ("M2", 0.1), ("M3", 1e-5)])
def test_lowrank_closed_form_against_augmented_exponential(core, t):
    """The closed form used as the reference for the third experiment (Sec. 5,
    separating the j = 0 term and using A^j = U M^(j-1) W^T) agrees with the
    quadruple-precision augmented exponential of the assembled matrix at
    n = 40; this pins the reference, not the oracle."""
    pr = wl.exp3_problem(core, t, n=40, seed=3)
    A = pr.op.U @ pr.op.W.T
    Wq = refs.exact_dense_q(A, pr.t, pr.beta, pr.V)
    ref = refs.lowrank_exact(pr.op, t, pr.beta[0], pr.V)
    # assembling A = U W^T in double perturbs it by ~u |U||W^T|; the non-normal
    # cores amplify that (M2 couples with 1e5; for M3 a random elementwise
    # relative perturbation of A by u moves the exact result by up to 1.7e-8)
    scale = {"M1": 1e-13, "M2": 1e-12, "M3": 5e-8}[core]
    assert refs.rel1_cols(ref[:, None], Wq)[0] < scale


def _exp3_env():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tables2to4_phimv.json")))


@pytest.mark.parametrize("core", ["M1", "M2", "M3"])
def test_third_experiment_within_tables2to4_envelope(orc, core):
    """The oracle (Algorithm 1 + Algorithm 3, alpha = 1, tol 2^-53) on the
    low-rank operator at the paper's p and a reduced n = 4000 is as accurate
    as the paper's implementation in Tables 2-4 (within a factor 10, floor
    100 u) for every abscissa of the tables (s_int up to 73 here; M3 needs
    s_int = 1, 5 and 45 at t = 0.1, 1 and 10)."""
    env = _exp3_env()[core]
    u = 2.0 ** -53
    for t, e in zip(env["t"], env["rel_err_1norm"]):
        pr = wl.exp3_problem(core, t, n=4000, seed=0)
        ref = refs.lowrank_exact(pr.op, t, pr.beta[0], pr.V)
        Wo, st, prm = orc.full(pr)
        err = refs.rel1_cols(Wo, ref[:, None])[0]
        bar = max(10 * e, 100 * u)
        assert err <= bar, (core, t, st["s_int"], err, e)


def test_lowrank_inner_products_are_compensated(orc):
    """The oracle's W^T x (the only n-term sums of a low-rank product) is the
    exact inner product rounded once: ones summed while +2^60 sits in the
    accumulator (cancelled later by -2^60) are lost by a plain row-order sum
    but counted exactly here, and random data of widely spread magnitudes
    agrees with the exact rational sum rounded once."""
    from fractions import Fraction
    n = 4001
    U = np.zeros((n, 1))
    U[0, 0] = 1.0
    W = np.ones((n, 1))
    x = np.ones(n)
    x[0] = 2.0 ** 60
    x[2000] = -(2.0 ** 60)
    op = wl.LowRank(U, W, np.ones((1, 1)))
    y = orc.apply(op, x)
    assert y[0] == float(n - 2), y[0]
    acc = 0.0
    for v in x:
        acc += v
    assert acc != float(n - 2)   # the plain sum fails here
    rng = np.random.default_rng(3)
    W = rng.standard_normal((n, 1))
    x = rng.standard_normal(n) * 10.0 ** rng.uniform(-8, 8, n)
    op = wl.LowRank(U, np.ascontiguousarray(W), np.ones((1, 1)))
    exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(W[:, 0], x))
    assert orc.apply(op, x)[0] == float(exact)


# ------------------------------------------- fourth experiment (expRK4s6, ADR)
def test_adr_operator_second_order():
    """The ADR operator of the fourth experiment applied to the grid values of
    u = cos(pi x/2) cos(pi y/2) (zero slope at x = 0 and y = 0, zero at x = 1
    and y = 1) approaches eps Lap u - alpha (u_x + u_y) at second order."""
    eps, alpha = 1e-3, -0.5
    errs = []
    for N in (20, 40, 80):
        x = np.arange(N) / N
        X, Y = np.meshgrid(x, x, indexing="xy")
        cx, cy = np.cos(np.pi * X / 2), np.cos(np.pi * Y / 2)
        sx, sy = np.sin(np.pi * X / 2), np.sin(np.pi * Y / 2)
        u = (cx * cy).ravel()
        Lu = (eps * (-(np.pi ** 2) / 2) * cx * cy
              - alpha * (-(np.pi / 2) * sx * cy - (np.pi / 2) * cx * sy)).ravel()
        op = wl.adr_operator(N, eps, alpha)
        errs.append(np.abs(op.dense() @ u - Lu).max())
    assert 3.2 < errs[0] / errs[1] < 4.8 and 3.2 < errs[1] / errs[2] < 4.8, errs


def test_exprk4s6_fourth_order(orc):
    """expRK4s6 (Sec. 1, eq. (expRK4s6)) on the ADR problem at N = 10 with a
    milder reaction (gamma = 20) to t = 1/2 converges at order four against a
    1e-12 Runge-Kutta reference: halving h divides the error by about 16.  A
    wrong stage weight or node drops the order."""
    N, T = 10, 0.5
    op = wl.adr_operator(N)
    gc = wl.adr_reaction(20.0)
    u0 = wl.adr_initial(N)
    ref = refs.ode_reference(op, gc, u0, T)
    o = orc.Operator(op)
    prm = orc.params(o, 1e-14, wl.params_vector(op.n))
    errs = []
    for ns in (16, 32, 64):
        u, calls = orc.exprk4s6(o, gc, u0, T / ns, ns, 1e-14, prm["shift"], prm["s"])
        assert len(calls) == 4 * ns
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20, errs


def test_exprk4s6_linear_problem_is_exponential(orc):
    """With g = 0 every stage and the update are exact phi-combinations, so the
    scheme returns e^(T A) u0 up to the solver tolerance."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import expm_multiply
    N, T, ns = 10, 0.5, 8
    op = wl.adr_operator(N)
    u0 = wl.adr_initial(N)
    o = orc.Operator(op)
    prm = orc.params(o, 1e-14, wl.params_vector(op.n))
    u, _ = orc.exprk4s6(o, np.zeros(4), u0, T / ns, ns, 1e-14, prm["shift"], prm["s"])
    rp, ci, va = op.csr()
    ref = expm_multiply(T * sp.csr_matrix((va, ci, rp), shape=(op.n, op.n)), u0)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------ the Proposition's block series
@pytest.mark.parametrize("seed,ts", [(4, 0.5), (5, 0.3), (6, 0.2)])
def test_series_block_against_augmented_exponential(orc, seed, ts):
    """The single series of the Proposition (Sec. 4) with g_i = phi_i against
    the exact augmented exponential (Theorem 1) on small non-normal matrices
    with |t| ||A||_inf up to about 18 (at 24 the unscaled series already
    loses a digit to cancellation: 1.2e-13)."""
    pr = wl.small_problem(7, 3, 3, seed=seed, t_scale=ts)
    W, st = orc.series_block(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, 2.0 ** -53)
    Wq = refs.exact_dense_q(pr.op.A, pr.t, pr.beta, pr.V)
    assert refs.rel2(W, Wq) < 1e-14


def test_series_block_single_phi_for_many_abscissae(orc):
    """The Remark after the Proposition: with every v_i zero except v_k the
    columns are phi_k(t_i A) v_k; on a diagonal operator these are scalar
    phi_k values (50-digit mpmath)."""
    lams = np.array([-3.0, -1.0, -0.25, 0.0, 0.5, 1.5])
    op = _diag_op(lams)
    k, p = 2, 3
    t = np.array([0.1, 0.4, 0.7, 1.0])
    V = np.zeros((len(lams), p + 1))
    V[:, k] = np.arange(1.0, len(lams) + 1)
    beta = np.ones((len(t), p + 1))
    W, _ = orc.series_block(op, p, len(t), t, beta, V, 2.0 ** -53)
    for c, tc in enumerate(t):
        ref = np.array([float(refs.phi_mp(k, tc * lam)) for lam in lams]) * V[:, k]
        assert np.abs(W[:, c] - ref).max() <= 2e-16 * np.abs(ref).max() * 4


def test_series_block_agrees_with_algorithm3(orc):
    """Two different evaluations of the same combinations: the unscaled,
    unshifted series and Algorithm 3 with Algorithm 1's parameters."""
    pr = wl.config1()
    t = pr.t * np.array([1.0])
    prm = orc.params(pr.op, pr.tol, pr.v)
    W3, _ = orc.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    Ws, st = orc.series_block(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol)
    assert refs.rel2(Ws, W3) < 1e-14
