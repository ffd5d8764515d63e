"""Pins of the complex oracle (Algorithms 1 and 3 over C; Sec. 1 poses the
problem for complex A, V, t and weights, Algorithm 3 takes a complex shift).

Each check compares it with something computed another way: the scalar
closed form of phi_j at 50 digits on a complex diagonal operator, the
exact augmented exponential (Theorem 1) in complex mpmath on small
non-normal matrices, the real oracle on real data, and the invariance of
the result under a change of shift.
"""
import numpy as np
import pytest

import refs

TOL = 2.0 ** -53


def _rng_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _diag_zop(orc, lams):
    n = len(lams)
    return orc.ZOperator(csr=(np.arange(n + 1), np.arange(n), np.asarray(lams, np.complex128)))


def _closed_form_diag(lams, t, beta, V):
    """w_i[k] = sum_j beta_ij phi_j(t_i lambda_k) V[k, j] at 50 digits."""
    n, P1 = V.shape
    W = np.zeros((n, len(t)), dtype=np.complex128)
    for i, ti in enumerate(t):
        for k in range(n):
            z = complex(ti) * complex(lams[k])
            import mpmath
            acc = mpmath.mpc(0)
            with mpmath.workdps(50):
                for j in range(P1):
                    acc += (mpmath.mpc(beta[i][j].real, beta[i][j].imag)
                            * refs.phi_mp(j, mpmath.mpc(z.real, z.imag), 50)
                            * mpmath.mpc(V[k, j].real, V[k, j].imag))
            W[k, i] = complex(acc)
    return W


@pytest.mark.parametrize("seed,tscale", [(0, 1.0), (1, 10.0), (2, 40.0)])
def test_complex_diagonal_closed_form(orc, seed, tscale):
    """Complex spectrum (rotating and decaying modes), complex t, a complex
    weight table and complex V, with Algorithm 1's (real) shift and with a
    complex shift: the scalar closed form of every component."""
    rng = np.random.default_rng(seed)
    n, p, r = 12, 3, 3
    lams = -rng.uniform(0.0, 4.0, n) + 1j * rng.uniform(-6.0, 6.0, n)
    t = tscale * (rng.uniform(0.2, 1.0, r) * np.exp(1j * rng.uniform(-0.4, 0.4, r)))
    beta = _rng_c(rng, r, p + 1)
    V = _rng_c(rng, n, p + 1)
    op = _diag_zop(orc, lams)
    prm = orc.zparams(op, TOL, rng.standard_normal(n))
    exact = _closed_form_diag(lams, t, beta, V)
    W, st = orc.zsolve(op, p, r, t, beta, V, TOL, prm["shift"], prm["s"])
    assert st["s_int"] >= 1
    assert refs.rel2_cols(W, exact).max() <= 1e-13, refs.rel2_cols(W, exact)
    W2, st2 = orc.zsolve(op, p, r, t, beta, V, TOL, prm["shift"] - 1.5 + 2.0j, prm["s"])
    assert refs.rel2_cols(W2, exact).max() <= 1e-13, refs.rel2_cols(W2, exact)


@pytest.mark.parametrize("n,p,r,seed,ts", [(6, 3, 2, 0, 1.0), (7, 5, 3, 1, 8.0),
                                           (5, 0, 1, 2, 3.0), (8, 2, 2, 3, 15.0)])
def test_complex_dense_against_augmented_exponential(orc, n, p, r, seed, ts):
    """Small non-normal complex A: Algorithm 1 and 3 end to end against the
    exact augmented exponential in complex mpmath, in the beta-prescaled form
    and (alpha_i^j weights) the literal alpha-form."""
    rng = np.random.default_rng(seed)
    A = _rng_c(rng, n, n) * (3.0 / np.sqrt(n)) - np.diag(rng.uniform(0.0, 3.0, n))
    t = ts * rng.uniform(0.3, 1.0, r) * np.exp(1j * rng.uniform(-1.0, 1.0, r))
    alpha = rng.uniform(0.5, 1.5, r) * np.exp(1j * rng.uniform(-3.0, 3.0, r))
    beta = np.array([[a ** j for j in range(p + 1)] for a in alpha])
    V = _rng_c(rng, n, p + 1)
    op = orc.ZOperator(dense=A)
    prm = orc.zparams(op, TOL, rng.standard_normal(n))
    exact = refs.exact_dense_mp_c(A, t, beta, V, dps=34)
    Wb, sb = orc.zsolve(op, p, r, t, beta, V, TOL, prm["shift"], prm["s"])
    assert refs.rel2_cols(Wb, exact).max() <= 1e-12, refs.rel2_cols(Wb, exact)
    Wa, sa = orc.zsolve(op, p, r, t, None, V, TOL, prm["shift"], prm["s"], form="alpha",
                        alpha=alpha)
    assert refs.rel2_cols(Wa, exact).max() <= 1e-12, refs.rel2_cols(Wa, exact)
    assert sa["s_int"] == sb["s_int"]


def test_complex_path_on_real_data_equals_real_oracle(orc):
    """Zero imaginary parts: the complex algorithms do the real ones' arithmetic
    (multiplications by exact zeros), so parameters, term counts and results
    agree with the real oracle."""
    import workloads as wl
    pr = wl.small_problem(10, 4, 3, 7, t_scale=12.0, spread=5.0)
    prm = orc.params(pr.op, pr.tol, pr.v)
    zop = orc.ZOperator(dense=pr.op.A.astype(np.complex128))
    zprm = orc.zparams(zop, pr.tol, pr.v)
    assert zprm["r_acc"] == prm["r_acc"]
    assert abs(zprm["s0"] / prm["s0"] - 1) <= 1e-15
    assert abs(zprm["s"] / prm["s"] - 1) <= 1e-13
    W, st = orc.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    Wz, stz = orc.zsolve(zop, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    assert (stz["s_int"], stz["terms_S"], stz["terms_rec"]) == \
        (st["s_int"], st["terms_S"], st["terms_rec"])
    assert np.abs(Wz.imag).max() == 0.0
    assert refs.rel2_cols(Wz.real, W).max() <= 1e-15


def test_complex_csr_equals_dense(orc):
    rng = np.random.default_rng(5)
    n, p, r = 9, 2, 2
    A = _rng_c(rng, n, n) * (rng.uniform(size=(n, n)) < 0.4) - 2.0 * np.eye(n)
    rp = np.zeros(n + 1, np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols += list(nz)
        vals += list(A[i, nz])
        rp[i + 1] = len(cols)
    dop = orc.ZOperator(dense=A)
    cop = orc.ZOperator(csr=(rp, np.array(cols), np.array(vals)))
    t = np.array([0.7 + 0.2j, -0.4j])
    beta = _rng_c(rng, r, p + 1)
    V = _rng_c(rng, n, p + 1)
    prm = orc.zparams(dop, TOL, np.ones(n))
    Wd, _ = orc.zsolve(dop, p, r, t, beta, V, TOL, prm["shift"], prm["s"])
    Wc, _ = orc.zsolve(cop, p, r, t, beta, V, TOL, prm["shift"], prm["s"])
    assert refs.rel2_cols(Wc, Wd).max() <= 1e-15


def test_complex_params_conjugate_pair_and_scalar(orc):
    """Algorithm 1 over C.  A = c I with complex c: every growth ratio is |c|,
    so s0 = |c|.  A conjugate pair a +- ib from a real start vector at low
    degree: f(xi)^m = ||((A - xi I)/s0)^m v|| is symmetric about xi = a and
    smallest there, so Brent's real search returns xi* = a."""
    n = 6
    c = -2.0 + 3.0j
    prm = orc.zparams(_diag_zop(orc, [c] * n), TOL, np.arange(1.0, n + 1))
    assert abs(prm["s0"] / abs(c) - 1) <= 1e-14
    a, b = -3.0, 5.0
    prm2 = orc.zparams(_diag_zop(orc, [a + 1j * b, a - 1j * b]), TOL, np.array([1.0, 1.0]), m=4)
    assert abs(prm2["shift"] - a) <= 1e-5 * prm2["s0"]


def test_complex_purely_imaginary_data(orc):
    """Purely imaginary V: by linearity W(iV) = i W(V), and every product by i
    is exact, so the complex path on iV reproduces i times the real oracle
    bit for bit, with the same term counts (the block norms must use moduli:
    the real parts are all zero).  Purely imaginary t (a Schroedinger-type
    step e^{i tau A}) against the scalar closed form, with the number of
    scaling steps ceil(s max|t_i|) of the moduli."""
    import workloads as wl
    pr = wl.small_problem(9, 3, 2, 4, t_scale=6.0, spread=4.0)
    prm = orc.params(pr.op, pr.tol, pr.v)
    W, st = orc.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    zop = orc.ZOperator(dense=pr.op.A.astype(np.complex128))
    Wz, stz = orc.zsolve(zop, pr.p, pr.r, pr.t, pr.beta, 1j * pr.V, pr.tol, prm["shift"],
                         prm["s"])
    assert (stz["terms_S"], stz["terms_rec"]) == (st["terms_S"], st["terms_rec"])
    assert np.array_equal(Wz, 1j * W)
    rng = np.random.default_rng(8)
    n, p, r = 10, 2, 2
    lams = rng.uniform(-5.0, 5.0, n) - 0.1
    t = 1j * np.array([3.0, -7.0])
    beta = _rng_c(rng, r, p + 1)
    V = _rng_c(rng, n, p + 1)
    op = _diag_zop(orc, lams)
    zprm = orc.zparams(op, TOL, rng.standard_normal(n))
    Wt, stt = orc.zsolve(op, p, r, t, beta, V, TOL, zprm["shift"], zprm["s"])
    assert stt["s_int"] == max(1, int(np.ceil(zprm["s"] * 7.0)))
    exact = _closed_form_diag(lams, t, beta, V)
    # |t lambda| up to 35 on the imaginary axis: the solution oscillates and
    # the scaling steps add their rounding (measured 3.6e-13)
    assert refs.rel2_cols(Wt, exact).max() <= 1e-12
