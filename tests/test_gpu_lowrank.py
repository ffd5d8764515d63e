"""Low-rank operators A = U W^T (Sec. 5, third experiment) on the HIP path,
through the C ABI, against the CPU oracle and the closed form of the
low-rank linear combination.

Both sides form the n-term inner products W^T x compensated (exact products
and sums carried as double-double pairs, rounded once), so the order in
which they are summed no longer matters.  Parity with the parameters pinned
to the oracle's: relative 2-norm 1e-12 per column, or, where the method's
own rounding is larger (the strongly non-normal M3 core amplifies the
rounding of the row products and Taylor sums), ten times the oracle's own
relative error against the closed form; the GPU result must then also be
that close to the closed form itself.  End to end (the GPU's own
parameters), at the paper's n and p, for every row of Tables 2-4: within
the paper's accuracy (factor 10, floor 100 u).
"""
import json
import os

import numpy as np
import pytest

import oracle
import refs
import workloads as wl
from gpu_util import gpu_solve, say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12
U53 = 2.0 ** -53
# phimv column of Tables 2-4 (relative 1-norm errors), stored with its citation
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "tables2to4_phimv.json")) as _f:
    _G = json.load(_f)
TABLE = {c: dict(zip([float(t) for t in _G[c]["t"]], _G[c]["rel_err_1norm"]))
         for c in ("M1", "M2", "M3")}
ROWS = [(c, t) for c in ("M1", "M2", "M3") for t in TABLE[c]]
# rows whose oracle solve at the paper's n takes more than a few seconds on
# one core (s_int from 5 to 73): pinned parity runs at n = 20 000 for them
LONG = {("M1", 50.0), ("M1", 100.0), ("M2", 50.0), ("M2", 100.0),
        ("M3", 1.0), ("M3", 10.0)}


def _exact(pr):
    return np.stack([refs.lowrank_exact(pr.op, float(pr.t[i]), pr.beta[i], pr.V)
                     for i in range(pr.r)], axis=1)


def _pinned(pr, label=""):
    say(f"[gpu] lowrank {pr.name} n={pr.n} p={pr.p} r={pr.r} {label}")
    prm = oracle.params(pr.op, pr.tol, pr.v)
    Wo, so = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol, prm["shift"], prm["s"])
    Wg, sg, _ = gpu_solve(pr, prm=prm)
    ex = _exact(pr)
    e_orc = refs.rel2_cols(Wo, ex).max()
    e_gpu = refs.rel2_cols(Wg, ex).max()
    err = refs.rel2_cols(Wg, Wo).max()
    bar = max(TOL_FP64, 10 * e_orc)
    say(f"      s_int={so['s_int']} terms S {so['terms_S']}/{sg['terms_S']} "
        f"rec {so['terms_rec']}/{sg['terms_rec']} gpu-oracle {err:.2e} "
        f"oracle-exact {e_orc:.2e} gpu-exact {e_gpu:.2e}")
    assert sg["status"] == pc.OK
    assert sg["s_int"] == so["s_int"]
    assert abs(sg["terms_S"] - so["terms_S"]) <= 1
    assert abs(sg["terms_rec"] - so["terms_rec"]) <= max(1, so["s_int"] // 4)
    assert err <= bar, (err, bar)
    assert e_gpu <= bar, (e_gpu, bar)
    return Wg, Wo, ex


@pytest.mark.parametrize("core", ["M1", "M2", "M3"])
def test_lowrank_params_match_oracle(core):
    pr = wl.exp3_problem(core, 1.0, n=4000)
    say(f"[gpu] lowrank params {core}")
    op = pc.Operator(pr.op)
    pg = op.params(pr.tol, v=pr.v)
    op.close()
    po = oracle.params(pr.op, pr.tol, pr.v)
    say(f"      r_acc {pg.r_acc}/{po['r_acc']} s0 {pg.s0:.6e}/{po['s0']:.6e} s {pg.s:.4e}/{po['s']:.4e}")
    assert pg.status == pc.OK
    assert pg.r_acc == po["r_acc"]
    # the power norms go through n-term sums W^T x summed in different
    # orders; the Moler core M3 (departure from normality ~2.8e10) amplifies
    # that rounding difference in its powers (observed 6e-8)
    assert abs(pg.s0 / po["s0"] - 1) < (1e-6 if core == "M3" else 1e-11)
    # s = s0 f(xi*) / (tol m!)^(1/m) with f limited by rounding near its
    # minimum (a floor of about eps^(1/m) (1 + |z|)); on the non-normal M2
    # core the two minimisers land on that floor 12 % apart
    assert abs(pg.s / po["s"] - 1) < 0.2


@pytest.mark.parametrize("core,t,n", [
    ("M1", 1.0, 37),          # one workgroup
    ("M1", 1.0, 4000),
    ("M1", 10.0, 4000),       # recovery steps
    ("M2", 0.1, 4000),
    ("M2", 10.0, 4000),
    ("M3", 1e-5, 4000),
    ("M3", 1e-3, 4000),
    ("M1", 10.0, 100003),     # many workgroups, ragged last one
    ("M1", 50.0, 20000),
    ("M1", 100.0, 20000),
    ("M2", 50.0, 20000),
    ("M2", 100.0, 20000),
    ("M3", 0.1, 20000),
    ("M3", 1.0, 20000),
    ("M3", 10.0, 20000),
])
def test_lowrank_pinned(core, t, n):
    _pinned(wl.exp3_problem(core, t, n=n, seed=1), f"t={t}")


def test_lowrank_block_of_abscissae_general_weights():
    """r = 3 abscissae and a general weight table on the M2 core."""
    base = wl.exp3_problem("M2", 1.0, n=50001, seed=2)
    rng = np.random.default_rng(7)
    p, r = 2, 3
    pr = wl.Problem("exp3_M2_block", base.op, p, r, np.array([0.25, 0.5, 1.0]),
                    rng.uniform(-1, 1, (r, p + 1)), np.ascontiguousarray(base.V[:, :p + 1]),
                    2.0 ** -53, base.v)
    _pinned(pr, "r=3")


def test_lowrank_p0_is_exponential_action():
    base = wl.exp3_problem("M1", 10.0, n=20000, seed=3)
    pr = wl.Problem("exp3_M1_p0", base.op, 0, 1, base.t, np.ones((1, 1)),
                    np.ascontiguousarray(base.V[:, :1]), 2.0 ** -53, base.v)
    _pinned(pr, "p=0")


@pytest.mark.parametrize("core,t", ROWS)
def test_lowrank_paper_sizes(core, t):
    """Every row of Tables 2-4 at the paper's n and p: the end-to-end result
    (GPU parameters) against the closed form within 10x the paper's error;
    pinned parity with the oracle over every entry where the oracle finishes
    in seconds at that size (the other rows: at n = 20 000 above, and the
    GPU with the oracle's parameters against the closed form here)."""
    pr = wl.exp3_problem(core, t, seed=0)
    ex = _exact(pr)
    bar = max(10 * TABLE[core][t], 100 * U53)
    if (core, t) in LONG:
        say(f"[gpu] lowrank {pr.name} n={pr.n} p={pr.p} (paper size, oracle parameters)")
        prm = oracle.params(pr.op, pr.tol, pr.v)
        Wg, sg, _ = gpu_solve(pr, prm=prm)
        e_pin = refs.rel1_cols(Wg, ex)[0]
        say(f"      s_int={sg['s_int']} rel1 err {e_pin:.2e}")
        assert sg["status"] == pc.OK
        assert e_pin <= bar, (e_pin, bar)
    else:
        _pinned(pr, f"t={t} (paper size)")
    Wg2, sg2, prm = gpu_solve(pr)
    err = refs.rel1_cols(Wg2, ex)[0]
    say(f"      end to end: s_int={sg2['s_int']} rel1 err {err:.2e} (paper {TABLE[core][t]:.2e})")
    assert sg2["status"] == pc.OK
    assert err <= bar, (err, bar)


def test_lowrank_mixed_precision_within_tol():
    """FP32 recovery-term tails on the low-rank operator: within 10 tol of
    the FP64 result (tol = 1e-8)."""
    pr = wl.exp3_problem("M1", 10.0, seed=4)
    pr.tol = 1e-8
    prm = oracle.params(pr.op, pr.tol, pr.v)
    W64, s64, _ = gpu_solve(pr, prm=prm)
    W32, s32, _ = gpu_solve(pr, prm=prm, precision=pc.MIXED)
    err = refs.rel2_cols(W32, W64).max()
    say(f"[gpu] lowrank mixed: fp32 terms {s32['fp32_terms']} err {err:.2e}")
    assert s32["status"] == pc.OK
    assert err <= 10 * pr.tol


def test_lowrank_rejects_bad_shapes():
    import torch
    n = 64
    U = np.ones((n, 17))
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_op_create_lowrank(n, U, U)
    assert e.value.status == pc.EINVAL
    bad = np.ones((n, 2))
    bad[3, 1] = np.nan
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_op_create_lowrank(n, bad, bad)
    assert e.value.status == pc.EINVAL
    # rank 16 with p = 7, r = 4 exchanges 16 * 36 > 256 entries per term
    core = np.diag(-np.arange(1.0, 17.0))
    op = wl.lowrank_operator(core, 200)
    h = pc.Operator(op)
    prm = h.params(1e-8)
    V = torch.from_numpy(np.random.default_rng(0).standard_normal((200, 8))).cuda()
    with pytest.raises(pc.PhicombError) as e:
        h.solve(prm, np.full(4, 0.1), np.ones((4, 8)), V, 1e-8)
    assert e.value.status == pc.EINVAL
    # the batched launch takes no low-rank operator
    W = torch.empty((200, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_batch_create([(h.h, prm, 1, 1, np.array([0.1]), np.ones((1, 2)),
                                  V[:, :2].contiguous(), W, 1e-8)], pc.FP64)
    assert e.value.status == pc.EINVAL
    h.close()


def test_lowrank_maximum_rank():
    """rank 16 (the largest accepted) with r = 2 abscissae: 96 entries of W^T X
    per exchange; a diagonal core with eigenvalues -1 .. -16."""
    core = np.diag(-np.arange(1.0, 17.0))
    op = wl.lowrank_operator(core, 5000)
    rng = np.random.default_rng(9)
    p, r = 1, 2
    pr = wl.Problem("lowrank_rank16", op, p, r, np.array([0.3, 1.0]),
                    rng.uniform(-1, 1, (r, p + 1)),
                    np.ascontiguousarray(rng.standard_normal((op.n, p + 1))), 2.0 ** -53,
                    wl.params_vector(op.n))
    _pinned(pr, "rank 16")


def test_lowrank_served_matches_blocking_solve():
    """Low-rank requests through phicomb_submit / phicomb_poll (the worker's
    workspace includes the W^T X exchange area) give the blocking solve's
    result bit for bit; three cores in flight together."""
    import time
    import torch
    pc.phicomb_serve_config(0, 4)
    probs = [wl.exp3_problem(c, t, n=30000, seed=5) for c, t in
             (("M1", 10.0), ("M2", 1.0), ("M3", 1e-3))]
    ops = [pc.Operator(pr.op) for pr in probs]
    prms = [pc.params_from_dict(oracle.params(pr.op, pr.tol, pr.v)) for pr in probs]
    Vd = [torch.from_numpy(pr.V).cuda() for pr in probs]
    Wb = [torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda") for pr in probs]
    Ws = [torch.full((pr.n, pr.r), np.nan, dtype=torch.float64, device="cuda") for pr in probs]
    for k, pr in enumerate(probs):
        pc.phicomb_solve(ops[k].h, prms[k], pr.p, pr.r, pr.t, pr.beta, Vd[k], pr.tol, pc.FP64,
                         Wb[k])
    torch.cuda.synchronize()
    tickets = [pc.phicomb_submit(ops[k].h, prms[k], pr.p, pr.r, pr.t, pr.beta, Vd[k], pr.tol,
                                 pc.FP64, Ws[k]) for k, pr in enumerate(probs)]
    done = [None] * len(tickets)
    t_end = time.perf_counter() + 60.0
    while any(d is None for d in done):
        assert time.perf_counter() < t_end, "served requests did not complete"
        for i, tk in enumerate(tickets):
            if done[i] is None:
                st, _ = pc.phicomb_poll(tk)
                if st != pc.PENDING:
                    done[i] = st
        time.sleep(0.0005)
    torch.cuda.synchronize()
    say(f"[gpu] lowrank served: statuses {done}")
    assert all(d == pc.OK for d in done)
    for k in range(len(probs)):
        assert torch.equal(Ws[k], Wb[k]), k
    for o in ops:
        o.close()
