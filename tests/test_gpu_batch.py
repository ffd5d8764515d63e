"""Batched solves (phicomb_batch_*): many instances of uneven size in one
persistent launch, replayed from a captured HIP graph.

Every instance is compared with the FP64 oracle (parameters pinned to the
oracle's) at the parity bar of a single solve: 1e-12 relative 2-norm per
column for FP64, 10 tol for mixed precision.  Graph replays are checked one
by one, with the program's own eager work between them.
"""
import numpy as np
import pytest

import oracle
import refs
import workloads as wl
from gpu_util import say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


def _instances(count, seed, tol, kind="stencil"):
    """2-D kappa-Laplacians of ragged sizes, p in 1..3, r in 1..3, t spread so
    that s_int runs from 1 to a few dozen."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        side = int(rng.integers(9, 80))
        kappa = float(10.0 ** rng.uniform(-1, 1))
        st = wl.laplacian_2d(side, kappa=kappa)
        op = st
        if kind == "csr":
            rp, ci, va = st.csr()
            op = wl.CSR(st.n, rp, ci, va)
        p = int(rng.integers(1, 4))
        r = int(rng.integers(1, 4))
        t = 10.0 ** rng.uniform(-5, -2.5, r) / kappa
        beta = rng.uniform(-1, 1, (r, p + 1))
        V = np.ascontiguousarray(rng.standard_normal((st.n, p + 1)))
        out.append(wl.Problem(f"b{k}", op, p, r, t, beta, V, tol, wl.params_vector(st.n)))
    return out


def _plan(probs, precision):
    import torch
    ops = [pc.Operator(pr.op) for pr in probs]
    po = [oracle.params(pr.op, pr.tol, pr.v) for pr in probs]
    prms = [pc.params_from_dict(d) for d in po]
    Vd = [torch.from_numpy(pr.V).cuda() for pr in probs]
    Wd = [torch.full((pr.n, pr.r), np.nan, dtype=torch.float64, device="cuda") for pr in probs]
    items = [(ops[k].h, prms[k], pr.p, pr.r, pr.t, pr.beta, Vd[k], Wd[k], pr.tol)
             for k, pr in enumerate(probs)]
    torch.cuda.synchronize()
    b = pc.phicomb_batch_create(items, precision)
    return b, ops, po, Vd, Wd


def _check_against_oracle(probs, po, Wd, stats, bar):
    worst = 0.0
    for k, pr in enumerate(probs):
        Wo, so = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol,
                              po[k]["shift"], po[k]["s"])
        err = refs.rel2_cols(Wd[k].cpu().numpy(), Wo).max()
        worst = max(worst, err)
        st = stats[k]
        assert st.status == pc.OK
        assert st.s_int == so["s_int"], (k, st.s_int, so["s_int"])
        assert err <= bar, (k, pr.n, pr.p, pr.r, err)
    return worst


@pytest.mark.parametrize("kind", ["stencil", "csr"])
def test_batch_fp64_matches_oracle(kind):
    import torch
    probs = _instances(24, 5 if kind == "stencil" else 6, 1e-10, kind)
    b, ops, po, Vd, Wd = _plan(probs, pc.FP64)
    info = pc.phicomb_batch_info(b)
    st, stats = pc.phicomb_batch_run(b, len(probs))
    torch.cuda.synchronize()
    assert st == pc.OK, pc.phicomb_strerror(st)
    say(f"[gpu-batch] {kind}: {len(probs)} instances, n {min(p.n for p in probs)}.."
        f"{max(p.n for p in probs)}, s_int up to {max(s.s_int for s in stats)}; "
        f"{info['groups']} groups / {info['workgroups']} workgroups, "
        f"{stats[0].ms:.2f} ms (model {info['predicted_ms']:.2f} ms)")
    worst = _check_against_oracle(probs, po, Wd, stats, TOL_FP64)
    say(f"      worst error vs oracle {worst:.2e}")
    pc.phicomb_batch_destroy(b)
    for o in ops:
        o.close()


def test_batch_mixed_matches_oracle():
    import torch
    probs = _instances(16, 7, 1e-6)
    b, ops, po, Vd, Wd = _plan(probs, pc.MIXED)
    st, stats = pc.phicomb_batch_run(b, len(probs))
    torch.cuda.synchronize()
    assert st == pc.OK
    worst = _check_against_oracle(probs, po, Wd, stats, 10 * 1e-6)
    n32 = sum(s.fp32_terms for s in stats)
    say(f"[gpu-batch] mixed: worst error vs oracle {worst:.2e}, fp32 terms {n32}")
    pc.phicomb_batch_destroy(b)
    for o in ops:
        o.close()


def test_batch_graph_replays():
    """Replays of the captured launch, with eager work in between: each run is
    bitwise equal to the first, and new V contents give the new results."""
    import torch
    probs = _instances(10, 11, 1e-10)
    b, ops, po, Vd, Wd = _plan(probs, pc.FP64)
    st, stats = pc.phicomb_batch_run(b, len(probs))
    torch.cuda.synchronize()
    assert st == pc.OK
    first = [w.cpu().numpy().copy() for w in Wd]
    for rep in range(3):
        # eager work between replays: clear W and run an unrelated solve
        for w in Wd:
            w.zero_()
        other = wl.config2(nside=20)
        h = pc.Operator(other.op)
        h.solve(h.params(other.tol, v=other.v), other.t, other.beta,
                torch.from_numpy(other.V).cuda(), other.tol)
        torch.cuda.synchronize()
        h.close()
        st, stats = pc.phicomb_batch_run(b, len(probs))
        torch.cuda.synchronize()
        assert st == pc.OK
        for k, w in enumerate(Wd):
            assert np.array_equal(w.cpu().numpy(), first[k]), (rep, k)
    # new inputs through the same pointers
    rng = np.random.default_rng(99)
    for k, pr in enumerate(probs):
        pr.V[:] = rng.standard_normal(pr.V.shape)
        Vd[k].copy_(torch.from_numpy(pr.V))
    torch.cuda.synchronize()
    st, stats = pc.phicomb_batch_run(b, len(probs))
    torch.cuda.synchronize()
    assert st == pc.OK
    _check_against_oracle(probs, po, Wd, stats, TOL_FP64)
    pc.phicomb_batch_destroy(b)
    for o in ops:
        o.close()


def test_batch_rejects_mixed_kinds():
    import torch
    a = _instances(1, 1, 1e-8, "stencil")[0]
    c = _instances(1, 2, 1e-8, "csr")[0]
    ops = [pc.Operator(a.op), pc.Operator(c.op)]
    prms = [pc.params_from_dict(oracle.params(pr.op, pr.tol, pr.v)) for pr in (a, c)]
    items = []
    for k, pr in enumerate((a, c)):
        items.append((ops[k].h, prms[k], pr.p, pr.r, pr.t, pr.beta,
                      torch.from_numpy(pr.V).cuda(),
                      torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda"), pr.tol))
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_batch_create(items, pc.FP64)
    assert e.value.status == pc.EINVAL
    for o in ops:
        o.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config4_full_batch_against_closed_form(precision):
    """The whole benchmark batch (256 kappa-Laplacians, side U{32..256},
    kappa logU[1e-2, 1e2], p, r U{1,2,3}, t logU[1e-5, 1e-2], tol 1e-8,
    s_int up to ~16 000), one launch with the GPU's own parameters: every
    instance against the DST-I eigen-decomposition closed form, within
    max(10 tol, 1e-12) relative 2-norm per column in FP64 and 10 tol in
    mixed precision."""
    import torch
    prec = pc.FP64 if precision == "fp64" else pc.MIXED
    probs = wl.config4()
    ops = [pc.Operator(pr.op) for pr in probs]
    prms = [o.params(pr.tol, v=pr.v) for o, pr in zip(ops, probs)]
    Vd = [torch.from_numpy(pr.V).cuda() for pr in probs]
    Wd = [torch.full((pr.n, pr.r), np.nan, dtype=torch.float64, device="cuda") for pr in probs]
    items = [(ops[k].h, prms[k], pr.p, pr.r, pr.t, pr.beta, Vd[k], Wd[k], pr.tol)
             for k, pr in enumerate(probs)]
    torch.cuda.synchronize()
    b = pc.phicomb_batch_create(items, prec)
    say(f"[gpu-batch] config 4, {precision}: {len(probs)} instances, one launch")
    st, stats = pc.phicomb_batch_run(b, len(probs))
    torch.cuda.synchronize()
    assert st == pc.OK, pc.phicomb_strerror(st)
    bar = 10 * probs[0].tol if prec == pc.MIXED else max(10 * probs[0].tol, 1e-12)
    worst, wk = 0.0, -1
    for k, pr in enumerate(probs):
        assert stats[k].status == pc.OK, k
        ref = refs.dst_laplacian(pr.op, pr.t, pr.beta, pr.V)
        err = refs.rel2_cols(Wd[k].cpu().numpy(), ref).max()
        if err > worst:
            worst, wk = err, k
        assert err <= bar, (k, pr.n, pr.p, pr.r, stats[k].s_int, err)
    say(f"      {stats[0].ms:.0f} ms, s_int up to {max(s.s_int for s in stats)}, "
        f"fp32 terms {sum(s.fp32_terms for s in stats)}; worst error vs closed form "
        f"{worst:.2e} (instance {wk}, n={probs[wk].n})")
    pc.phicomb_batch_destroy(b)
    for o in ops:
        o.close()
