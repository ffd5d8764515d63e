"""Mixed-precision solve (FP64 head, FP32 tail of every Taylor loop) on the
GPU versus the FP64 CPU oracle.

Bar: relative 2-norm per column within 10 * tol of the FP64 oracle with the
parameters (shift, s) pinned to the oracle's, and within 10 * tol (plus the
FP64 path's own 1e-12) of the exact DST result on the 3-D Laplacian.  The
error of every result is printed.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import refs
import workloads as wl
from gpu_util import gpu_solve, load_golden, sampled_err, say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu


def _mixed_vs_oracle(pr, t=None, label=""):
    t = pr.t if t is None else t
    say(f"[gpu-mixed] {pr.name} n={pr.n} tol={pr.tol:g} {label}")
    prm = oracle.params(pr.op, pr.tol, pr.v)
    Wo, so = oracle.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    Wg, sg, _ = gpu_solve(pr, prm=prm, t=t, precision=pc.MIXED)
    err = refs.rel2_cols(Wg, Wo)
    nterms = sg["terms_S"] + sg["terms_rec"]
    say(f"      s_int={sg['s_int']} terms {sg['terms_S']}+{sg['terms_rec']} "
        f"fp32 {sg['fp32_terms']}/{nterms}  err per column {np.array2string(err, precision=2)}")
    assert sg["s_int"] == so["s_int"]
    assert err.max() <= 10 * pr.tol, err
    return sg, err


@pytest.mark.parametrize("tol", [1e-6, 1e-9, 1e-12])
@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_config2_reduced_mixed(tol, kind):
    pr = dataclasses.replace(wl.config2(nside=96, as_csr=(kind == "csr")), tol=tol)
    sg, _ = _mixed_vs_oracle(pr, t=pr.t * 20, label=kind)
    if tol >= 1e-9:
        assert sg["fp32_terms"] > 0


@pytest.mark.parametrize("nonnormal", [False, True])
def test_config3_reduced_mixed(nonnormal):
    pr = wl.config3(nside=24, nonnormal=nonnormal, tol=1e-6)
    sg, _ = _mixed_vs_oracle(pr, t=pr.t * 20, label="3d")
    assert sg["fp32_terms"] > 0


@pytest.mark.parametrize("p,r", [(0, 1), (2, 4), (7, 2)])
def test_p_r_range_mixed(p, r):
    rng = np.random.default_rng(100 + p * 10 + r)
    st = wl.convdiff_2d_upwind(37)      # ragged: n = 1369
    V = np.ascontiguousarray(rng.standard_normal((st.n, p + 1)))
    beta = rng.uniform(-1, 1, (r, p + 1))
    t = rng.uniform(-1, 1, r) * 2e-3
    pr = wl.Problem(f"mix_{p}_{r}", st, p, r, t, beta, V, 1e-7, wl.params_vector(st.n))
    _mixed_vs_oracle(pr, label=f"p={p} r={r}")


def test_config2_full_size_mixed():
    pr = dataclasses.replace(wl.config2(), tol=1e-6)
    sg, _ = _mixed_vs_oracle(pr, label="csr full")
    assert sg["fp32_terms"] > 0


@pytest.mark.parametrize("tol", [1e-6, 1e-12])
def test_config3_full_size_mixed_vs_dst(tol):
    pr = wl.config3(tol=tol)
    say(f"[gpu-mixed] {pr.name} full n={pr.n} tol={tol:g}")
    Wm, sm, prm = gpu_solve(pr, precision=pc.MIXED)
    nterms = sm["terms_S"] + sm["terms_rec"]
    exact = refs.dst_laplacian(pr.op, pr.t, pr.beta, pr.V)
    em = refs.rel2_cols(Wm, exact)
    say(f"      s_int={sm['s_int']} terms {sm['terms_S']}+{sm['terms_rec']} "
        f"fp32 {sm['fp32_terms']}/{nterms} vs exact {np.array2string(em, precision=2)}")
    assert em.max() <= 10 * tol + 1e-12
    if tol >= 1e-6:
        assert sm["fp32_terms"] > 0


@pytest.mark.parametrize("tol", [1e-6, 1e-12])
def test_config3_nonnormal_full_size_mixed_sampled(tol):
    pr = wl.config3(nonnormal=True, tol=tol)
    g = load_golden(tol)
    say(f"[gpu-mixed] {pr.name} full n={pr.n} tol={tol:g} (sampled oracle rows)")
    Wm, sm, _ = gpu_solve(pr, prm=g["params"], precision=pc.MIXED)
    err = sampled_err(Wm, g)
    nterms = sm["terms_S"] + sm["terms_rec"]
    say(f"      s_int={sm['s_int']} terms {sm['terms_S']}+{sm['terms_rec']} "
        f"fp32 {sm['fp32_terms']}/{nterms} sampled err {np.array2string(err, precision=2)}")
    assert sm["s_int"] == g["stats"]["s_int"]
    assert err.max() <= 10 * tol
    if tol >= 1e-6:
        assert sm["fp32_terms"] > 0


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_series_only_mixed_tail(kind):
    """With s_int = 1 every term is in the S-series: its FP32 tail (the same
    head/tail rule as the recovery steps) is used and the result stays within
    10 tol of the FP64 oracle."""
    pr = dataclasses.replace(wl.config2(nside=96, as_csr=(kind == "csr")), tol=1e-6)
    sg, _ = _mixed_vs_oracle(pr, label=f"{kind} s_int=1")
    assert sg["s_int"] == 1
    assert sg["fp32_terms"] > 0
