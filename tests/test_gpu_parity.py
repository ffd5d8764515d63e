"""GPU (HIP, through the C ABI) versus the CPU oracle, element by element.

Tolerance on the FP64 path: relative 2-norm 1e-12 per column with the
parameters pinned to the oracle's.  With independently computed
parameters both sides are approximations of the exact result within their
own truncation error, so they are compared with a bound derived from tol
and checked against an exact reference where one exists.
"""
import math

import numpy as np
import pytest

import oracle
import refs
import workloads as wl
from gpu_util import gpu_solve, load_golden, sampled_err, say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


def _pinned(problem, t=None, beta=None, V=None, p=None, r=None):
    prm = oracle.params(problem.op, problem.tol, problem.v)
    t = problem.t if t is None else t
    beta = problem.beta if beta is None else beta
    V = problem.V if V is None else V
    p = problem.p if p is None else p
    r = problem.r if r is None else r
    Wo, so = oracle.solve(problem.op, p, r, t, beta, V, problem.tol, prm["shift"], prm["s"])
    return prm, Wo, so


def _compare(problem, **kw):
    say(f"[gpu] {problem.name} n={problem.n} {kw.get('label', '')}")
    prm, Wo, so = _pinned(problem, kw.get("t"), kw.get("beta"), kw.get("V"))
    Wg, sg, _ = gpu_solve(problem, prm=prm, t=kw.get("t"), beta=kw.get("beta"), V=kw.get("V"))
    err = refs.rel2_cols(Wg, Wo)
    say(f"      s_int={so['s_int']} terms S {so['terms_S']}/{sg['terms_S']} "
        f"rec {so['terms_rec']}/{sg['terms_rec']} err={err.max():.2e}")
    assert sg["s_int"] == so["s_int"]
    assert abs(sg["terms_S"] - so["terms_S"]) <= 1
    assert abs(sg["terms_rec"] - so["terms_rec"]) <= max(1, so["s_int"] // 4)
    assert err.max() <= TOL_FP64, err
    return Wg, Wo, sg, so


# --------------------------------------------------------------- configs
def test_config1_pinned():
    _compare(wl.config1())


def test_config1_end_to_end():
    pr = wl.config1()
    say("[gpu] cfg1 end-to-end")
    Wg, sg, prm = gpu_solve(pr)
    po = oracle.params(pr.op, pr.tol, pr.v)
    Wo, so = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, po["shift"], po["s"])
    exact = refs.dst_laplacian(pr.op, pr.t, pr.beta, pr.V)
    assert prm.r_acc == po["r_acc"]
    assert abs(prm.s0 / po["s0"] - 1) < 1e-12
    assert abs(prm.s / po["s"] - 1) < 0.1
    assert refs.rel2(Wg, exact) <= 1e-14
    assert refs.rel2(Wg, Wo) <= TOL_FP64


@pytest.mark.parametrize("nside", [16, 48, 100])
@pytest.mark.parametrize("kind", ["csr", "stencil"])
@pytest.mark.parametrize("t_mult", [1.0, 40.0])
def test_config2_operator_reduced(nside, kind, t_mult):
    pr = wl.config2(nside=nside, as_csr=(kind == "csr"))
    _compare(pr, t=pr.t * t_mult, label=f"{kind} t*{t_mult}")


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_config2_full_size_pinned(kind):
    pr = wl.config2(as_csr=(kind == "csr"))
    Wg, Wo, sg, so = _compare(pr, label=kind)
    assert so["s_int"] >= 5


def test_config2_full_size_end_to_end():
    pr = wl.config2()
    say("[gpu] cfg2 end-to-end params")
    op = pc.Operator(pr.op)
    prm = op.params(pr.tol, v=pr.v)
    po = oracle.params(pr.op, pr.tol, pr.v)
    say(f"      gpu s={prm.s:.6g} xi={prm.shift:.6g} nf={prm.n_feval}; "
        f"oracle s={po['s']:.6g} xi={po['shift']:.6g} nf={po['n_feval']}")
    assert prm.r_acc == po["r_acc"]
    assert abs(prm.s0 / po["s0"] - 1) < 1e-10
    assert abs(prm.s / po["s"] - 1) < 0.1
    Wg, sg, _ = gpu_solve(pr, prm=prm, op=op)
    Wo, so = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, po["shift"], po["s"])
    err = refs.rel2_cols(Wg, Wo)
    say(f"      err vs oracle (own params) {err.max():.2e}")
    assert err.max() <= 100 * pr.tol
    op.close()


@pytest.mark.parametrize("nonnormal", [False, True])
def test_config3_operator_reduced_pinned(nonnormal):
    pr = wl.config3(nside=24, nonnormal=nonnormal, tol=1e-12)
    _compare(pr, t=pr.t * 20, label="3d")


@pytest.mark.parametrize("tol", [1e-12, 1e-6])
def test_config3_full_size_against_dst(tol):
    pr = wl.config3(tol=tol)
    say(f"[gpu] cfg3 full n={pr.n} tol={tol}")
    Wg, sg, prm = gpu_solve(pr)
    exact = refs.dst_laplacian(pr.op, pr.t, pr.beta, pr.V)
    err = refs.rel2_cols(Wg, exact)
    say(f"      s_int={sg['s_int']} terms {sg['terms_S']}/{sg['terms_rec']} err={err.max():.2e}")
    assert err.max() <= max(10 * tol, 1e-12)


@pytest.mark.parametrize("tol", [1e-6, 1e-12])
def test_config3_nonnormal_full_size_sampled(tol):
    pr = wl.config3(nonnormal=True, tol=tol)
    g = load_golden(tol)
    say(f"[gpu] {pr.name} full n={pr.n} tol={tol:g} (sampled oracle rows)")
    Wg, sg, _ = gpu_solve(pr, prm=g["params"])
    err = sampled_err(Wg, g)
    so = g["stats"]
    say(f"      s_int={sg['s_int']} terms S {so['terms_S']}/{sg['terms_S']} "
        f"rec {so['terms_rec']}/{sg['terms_rec']} sampled err {np.array2string(err, precision=2)}")
    assert sg["s_int"] == so["s_int"]
    assert abs(sg["terms_S"] - so["terms_S"]) <= 1
    assert abs(sg["terms_rec"] - so["terms_rec"]) <= max(1, so["s_int"] // 4)
    assert err.max() <= TOL_FP64
    # the column norms of the full result agree as well
    cn = np.linalg.norm(Wg, axis=0)
    assert np.allclose(cn, g["col_norm2"], rtol=TOL_FP64, atol=0)


def test_large_nonsymmetric_stencil_row_pairs_pinned():
    """Past 2^20 rows the partial sums E live in memory and stencil products
    run by row pairs (x-neighbours across lanes).  A non-symmetric 3-D stencil
    (every neighbour weight different, plus a superdiagonal) on a 104^3 grid
    (n = 1 124 864: 256 workgroups of 4394 rows, pairs straddling waves and
    a ragged last workgroup), p = 1, r = 2, against the oracle with pinned
    parameters at the FP64 parity bar."""
    rng = np.random.default_rng(31)
    h2 = 105.0 ** 2
    coef = np.array([-6.0, 1.3, 0.7, 1.1, 0.9, 1.2, 0.8]) * h2
    st = wl.Stencil(3, (104, 104, 104), coef, 0.03 * h2)
    V = np.ascontiguousarray(rng.standard_normal((st.n, 2)))
    pr = wl.Problem("stencil3d_104_nonsym", st, 1, 2, np.array([2e-4, 5e-4]),
                    rng.uniform(-1, 1, (2, 2)), V, 1e-12, wl.params_vector(st.n))
    _compare(pr, label="E in memory, row pairs")


# --------------------------------------------------------------- edge cases
def test_p0_exponential_only():
    pr = wl.config2(nside=40)
    prm = oracle.params(pr.op, pr.tol, pr.v)
    V = np.ascontiguousarray(pr.V[:, :1])
    beta = np.ones((3, 1))
    t = pr.t * 30
    Wo, so = oracle.solve(pr.op, 0, 3, t, beta, V, pr.tol, prm["shift"], prm["s"])
    Wg, sg, _ = gpu_solve(pr, prm=prm, t=t, beta=beta, V=V)
    assert refs.rel2_cols(Wg, Wo).max() <= TOL_FP64


@pytest.mark.parametrize("p,r", [(1, 1), (2, 4), (5, 2), (7, 1), (7, 4)])
def test_p_r_range_general_weights(p, r):
    rng = np.random.default_rng(p * 10 + r)
    st = wl.convdiff_2d_upwind(37)      # ragged: n = 1369
    rp, ci, va = st.csr()
    op = wl.CSR(st.n, rp, ci, va)
    V = np.ascontiguousarray(rng.standard_normal((st.n, p + 1)))
    beta = rng.uniform(-1, 1, (r, p + 1))
    t = rng.uniform(-1, 1, r) * 2e-3
    pr = wl.Problem(f"pr_{p}_{r}", op, p, r, t, beta, V, 1e-12, wl.params_vector(st.n))
    _compare(pr, label=f"p={p} r={r}")


def test_v0_zero_and_t_zero():
    pr = wl.config2(nside=30)
    V = pr.V.copy()
    V[:, 0] = 0.0
    _compare(pr, V=V, t=pr.t * 10, label="v0=0")
    _compare(pr, t=np.array([0.0, 1e-4, 0.0]), label="t has zeros")


def test_tiny_sizes():
    for n in (1, 2, 5):
        st = wl.laplacian_2d(n, 1)
        # a random start vector: a constant one can be an eigenvector here,
        # which hides the rest of the spectrum from Algorithm 1
        pr = wl.Problem(f"tiny{n}", st, 2, 2, np.array([0.3, 1.0]), np.ones((2, 3)),
                        np.random.default_rng(n).standard_normal((n, 3)), 1e-12,
                        wl.params_vector(n, 7))
        _compare(pr, label="tiny")


def test_small_dense_nonnormal():
    pr = wl.small_problem(24, 3, 3, 5, t_scale=5.0, spread=6.0)
    _compare(pr, label="dense")


# Dense operators of at most 112 rows run on one workgroup with A and the
# term blocks in LDS when they fit (p = 7, r = 4 at n = 112 does not and takes
# the global-memory kernel, as do n = 113 and 128 on one workgroup); ragged
# 16-row tiles at n = 1, 17, 63, 99 and 112; past 128 rows one 16-row tile a
# workgroup, the last one ragged (n = 129: a single row; n = 257).
@pytest.mark.parametrize("n,p,r", [(1, 2, 1), (17, 1, 2), (63, 6, 1), (99, 6, 1), (99, 3, 4),
                                   (112, 4, 3), (112, 7, 4), (113, 2, 2), (128, 6, 1),
                                   (129, 2, 1), (257, 3, 2)])
def test_dense_lds_sizes(n, p, r):
    pr = wl.small_problem(n, p, r, 11 + n, t_scale=3.0, spread=8.0)
    _compare(pr, label="dense")


def test_deterministic_reruns():
    pr = wl.config2(nside=64)
    op = pc.Operator(pr.op)
    p1 = op.params(pr.tol, v=pr.v)
    p2 = op.params(pr.tol, v=pr.v)
    assert p1.s == p2.s and p1.shift == p2.shift
    W1, _, _ = gpu_solve(pr, prm=p1, op=op)
    W2, _, _ = gpu_solve(pr, prm=p1, op=op)
    assert np.array_equal(W1, W2)
    op.close()


# --------------------------------------------------------------- error paths
def test_overflow_guard_and_invalid_inputs():
    n = 8
    op = pc.Operator(wl.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                            np.full(n, math.exp(600.0))))
    with pytest.raises(pc.PhicombError) as e:
        op.params(1e-10, v=np.ones(n))
    assert e.value.status == pc.EOVERFLOW
    op.close()
    pr = wl.config2(nside=16)
    op = pc.Operator(pr.op)
    prm = op.params(pr.tol, v=pr.v)
    import torch
    V = torch.from_numpy(pr.V).cuda()
    with pytest.raises(pc.PhicombError) as e:
        op.solve(prm, [np.nan, 1e-4, 1e-4], pr.beta, V, pr.tol)
    assert e.value.status == pc.EINVAL
    with pytest.raises(pc.PhicombError) as e:
        op.solve(prm, [1e300, 1e-4, 1e-4], pr.beta, V, pr.tol)
    assert e.value.status == pc.EINVAL
    with pytest.raises(pc.PhicombError) as e:
        op.solve(prm, pr.t, pr.beta, V, -1.0)
    assert e.value.status == pc.EINVAL
    # a non-finite entry of V is found in the device's first pass over V
    Vbad = V.clone()
    Vbad[100, 2] = float("nan")
    with pytest.raises(pc.PhicombError) as e:
        op.solve(prm, pr.t, pr.beta, Vbad, pr.tol)
    assert e.value.status == pc.EINVAL
    Vbad[100, 2] = float("inf")
    with pytest.raises(pc.PhicombError) as e:
        op.solve(prm, pr.t, pr.beta, Vbad, pr.tol)
    assert e.value.status == pc.EINVAL
    # the operator still solves normally afterwards
    W, st = op.solve(prm, pr.t, pr.beta, V, pr.tol)
    assert st.status == pc.OK
    op.close()


# ------------------------------------------- second experiment (Sec. 5, Table 1)
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_second_experiment_chebyshev(k):
    """Dense, highly non-normal collocation Laplacian (n = 99), p = 6, one
    solve per t = 1e-4 .. 1e-1 at tol 2^-53.  Parity with the oracle at the
    oracle's parameters and at the GPU's own parameters; end to end
    (parameters from the GPU) within 10x the paper's Table 1 error against
    an exact reference, or within 10x the error the oracle itself reaches
    with the same parameters where that is larger (xi* and s are set by a
    rounding-limited objective and the error of this non-normal matrix moves
    with them)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_phimv.json")))
    pr, env = wl.exp2_problems()[k], g["rel_err_1norm"][k]
    say(f"[gpu] {pr.name}")
    Wq = refs.exact_dense_q(pr.op.A, pr.t, pr.beta, pr.V)
    Wg, sg, prm = gpu_solve(pr)
    e_end = refs.rel1_cols(Wg, Wq)[0]
    po = oracle.params(pr.op, pr.tol, pr.v)
    Wo, so = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, po["shift"], po["s"])
    Wp, sp_, _ = gpu_solve(pr, prm=po)
    e_par = refs.rel2_cols(Wp, Wo)[0]
    # the oracle at the GPU's own parameters
    Wog, sog = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, prm.shift, prm.s)
    e_par_g = refs.rel2_cols(Wg, Wog)[0]
    # where the method's own rounding error exceeds 1e-12 (tens of
    # thousands of scaling steps on a non-normal matrix; Table 1 reports
    # 1.2e-12 at t = 0.1), two correct FP64 evaluations differ by up to
    # that error: the bar is the oracle's own error against the exact one
    e_orc = refs.rel2_cols(Wo, Wq)[0]
    e_orc1 = refs.rel1_cols(Wo, Wq)[0]
    e_orc1_g = refs.rel1_cols(Wog, Wq)[0]
    say(f"      params gpu: shift {prm.shift:.6e} s {prm.s:.6e} n_feval {prm.n_feval} "
        f"s_int {sg['s_int']}; oracle: shift {po['shift']:.6e} s {po['s']:.6e} "
        f"n_feval {po['n_feval']} s_int {so['s_int']}")
    say(f"      end-to-end rel1 err {e_end:.2e} (Table 1: {env:.1e}); oracle at its own "
        f"parameters {e_orc1:.2e}, at the GPU's {e_orc1_g:.2e}; pinned vs oracle "
        f"{e_par:.2e} / {e_par_g:.2e} (oracle vs exact {e_orc:.2e})")
    assert e_end <= 10 * max(env, e_orc1_g)
    assert sp_["s_int"] == so["s_int"]
    assert sog["s_int"] == sg["s_int"]
    assert e_par <= max(TOL_FP64, e_orc)
    assert e_par_g <= max(TOL_FP64, refs.rel2_cols(Wog, Wq)[0])


def test_second_experiment_chebyshev_t1():
    """Table 1's t = 1 row (2.6e5 scaling steps, 1.2e7 Taylor terms on one
    workgroup with A in registers, about 25 s): end to end within 10x the
    paper's 1.5e-10 against the exact reference.  The oracle is not run here
    (its single-threaded C needs minutes for this many terms)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_phimv.json")))
    pr, env = wl.exp2_problems()[4], g["rel_err_1norm"][4]
    say(f"[gpu] {pr.name}")
    Wq = refs.exact_dense_q(pr.op.A, pr.t, pr.beta, pr.V)
    Wg, sg, prm = gpu_solve(pr)
    e_end = refs.rel1_cols(Wg, Wq)[0]
    say(f"      s_int {sg['s_int']} terms {sg['terms_S']} + {sg['terms_rec']}: "
        f"end-to-end rel1 err {e_end:.2e} (Table 1: {env:.1e})")
    assert sg["status"] == pc.OK
    assert e_end <= 10 * env
