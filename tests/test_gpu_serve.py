"""Serving (phicomb_submit / phicomb_poll): continuous batching of requests
on several resident operators.

Checks, for a mix of operators and shapes:
  * every served result matches the FP64 oracle (parameters pinned) within
    the parity bar, and the same request solved alone with phicomb_solve;
  * admission by footprint: with a budget that holds one request at a time
    everything still completes, in order; a request larger than the budget
    is refused with EADMIT;
  * poll reports PENDING before completion and frees the ticket after.
"""
import time

import numpy as np
import pytest

import oracle
import refs
import workloads as wl
from gpu_util import say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


def _mix_problems():
    """Requests over four resident operators of different kinds and sizes
    (2-D CSR, 2-D stencil, 3-D stencil, small dense), uneven p and r."""
    rng = np.random.default_rng(7)
    ops = [wl.config2(nside=64).op,                     # CSR, n = 4096
           wl.convdiff_2d_upwind(80),                    # stencil, n = 6400
           wl.laplacian_3d(20, superdiag=100.0),         # 3-D stencil, n = 8000
           wl.small_problem(300, 1, 1, seed=3, spread=20.0).op]   # dense, n = 300
    reqs = []
    for k in range(12):
        oi = k % len(ops)
        op = ops[oi]
        p = int(rng.integers(1, 5))
        r = int(rng.integers(1, 4))
        t = rng.uniform(0.2, 1.0, r) * (2e-4 if oi < 3 else 0.3)
        beta = rng.uniform(-1, 1, (r, p + 1))
        V = np.ascontiguousarray(rng.standard_normal((op.n, p + 1)))
        reqs.append((oi, wl.Problem(f"req{k}", op, p, r, t, beta, V, 1e-10,
                                    wl.params_vector(op.n))))
    return ops, reqs


def _serve(handles, prms, reqs, Vd, Wd, precision=pc.FP64, timeout=60.0):
    tickets = []
    t_sub = []
    for (oi, pr), V, W in zip(reqs, Vd, Wd):
        tickets.append(pc.phicomb_submit(handles[oi].h, prms[oi], pr.p, pr.r, pr.t, pr.beta,
                                         V, pr.tol, precision, W))
        t_sub.append(time.perf_counter())
    done = [None] * len(tickets)
    lat = [0.0] * len(tickets)
    t_end = time.perf_counter() + timeout
    saw_pending = False
    while any(d is None for d in done):
        assert time.perf_counter() < t_end, "served requests did not complete"
        for i, tk in enumerate(tickets):
            if done[i] is None:
                st, stats = pc.phicomb_poll(tk)
                if st == pc.PENDING:
                    saw_pending = True
                    continue
                done[i] = (st, stats.as_dict())
                lat[i] = time.perf_counter() - t_sub[i]
        time.sleep(0.0005)
    return done, lat, saw_pending


def test_served_mix_matches_alone_and_oracle():
    import torch
    ops, reqs = _mix_problems()
    handles = [pc.Operator(o) for o in ops]
    prms_o = [oracle.params(o, 1e-10, wl.params_vector(o.n)) for o in ops]
    prms = [pc.params_from_dict(d) for d in prms_o]
    Vd = [torch.from_numpy(pr.V).cuda() for _, pr in reqs]
    alone = []
    for (oi, pr), V in zip(reqs, Vd):
        W, st = handles[oi].solve(prms[oi], pr.t, pr.beta, V, pr.tol)
        alone.append(W.cpu().numpy())
    pc.phicomb_serve_config(0, 4)
    Wd = [torch.full((pr.n, pr.r), np.nan, dtype=torch.float64, device="cuda")
          for _, pr in reqs]
    torch.cuda.synchronize()
    done, lat, _ = _serve(handles, prms, reqs, Vd, Wd)
    say(f"[gpu-serve] {len(reqs)} requests, latency ms p50 "
        f"{1e3 * np.median(lat):.2f} max {1e3 * max(lat):.2f}")
    n_bitexact = 0
    for i, ((oi, pr), W) in enumerate(zip(reqs, Wd)):
        st, stats = done[i]
        assert st == pc.OK, pc.phicomb_strerror(st)
        Wm = W.cpu().numpy()
        po = prms_o[oi]
        Wo, so = oracle.solve(pr.op, pr.p, pr.r, pr.t, pr.beta, pr.V, pr.tol,
                              po["shift"], po["s"])
        e_or = refs.rel2_cols(Wm, Wo).max()
        e_al = refs.rel2_cols(Wm, alone[i]).max()
        n_bitexact += int(np.array_equal(Wm, alone[i]))
        say(f"      req{i} op{oi} n={pr.n} p={pr.p} r={pr.r} s_int={stats['s_int']} "
            f"vs oracle {e_or:.2e} vs alone {e_al:.2e}")
        assert stats["s_int"] == so["s_int"]
        assert e_or <= TOL_FP64
        assert e_al <= TOL_FP64
    say(f"      bit-identical to the alone result: {n_bitexact}/{len(reqs)}")
    for h in handles:
        h.close()


def test_served_admission_by_footprint():
    import torch
    pr = wl.config2(nside=48)
    h = pc.Operator(pr.op)
    prm = pc.params_from_dict(oracle.params(pr.op, pr.tol, pr.v))
    po = oracle.params(pr.op, pr.tol, pr.v)
    Wo, _ = oracle.solve(pr.op, pr.p, pr.r, pr.t * 10, pr.beta, pr.V, pr.tol,
                         po["shift"], po["s"])
    one = pc.phicomb_request_bytes(pr.n, pr.p, pr.r, pc.FP64)
    assert one > 0
    # a budget for exactly one request: the others wait for memory
    pc.phicomb_serve_config(one, 4)
    V = torch.from_numpy(pr.V).cuda()
    reqs = [(0, wl.Problem(f"adm{k}", pr.op, pr.p, pr.r, pr.t * 10, pr.beta, pr.V, pr.tol,
                           pr.v)) for k in range(5)]
    Wd = [torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda") for _ in reqs]
    torch.cuda.synchronize()
    done, lat, saw_pending = _serve([h], [prm], reqs, [V] * len(reqs), Wd)
    say(f"[gpu-serve] budget for one request: latencies ms "
        f"{[round(1e3 * x, 2) for x in lat]}")
    assert saw_pending
    for (st, _), W in zip(done, Wd):
        assert st == pc.OK
        assert refs.rel2_cols(W.cpu().numpy(), Wo).max() <= TOL_FP64
    # a request that can never fit
    pc.phicomb_serve_config(one - 1, 0)
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_submit(h.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, pc.FP64, Wd[0])
    assert e.value.status == pc.EADMIT
    pc.phicomb_serve_config(1 << 34, 0)
    h.close()


def test_served_mixed_precision():
    import torch
    pr = wl.config3(nside=24, nonnormal=True, tol=1e-6)
    h = pc.Operator(pr.op)
    po = oracle.params(pr.op, pr.tol, pr.v)
    prm = pc.params_from_dict(po)
    t = pr.t * 20
    Wo, _ = oracle.solve(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, po["shift"], po["s"])
    V = torch.from_numpy(pr.V).cuda()
    reqs = [(0, wl.Problem(f"mx{k}", pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol, pr.v))
            for k in range(6)]
    Wd = [torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda") for _ in reqs]
    pc.phicomb_serve_config(0, 4)
    torch.cuda.synchronize()
    done, _, _ = _serve([h], [prm], reqs, [V] * len(reqs), Wd, precision=pc.MIXED)
    for (st, stats), W in zip(done, Wd):
        assert st == pc.OK
        err = refs.rel2_cols(W.cpu().numpy(), Wo).max()
        assert err <= 10 * pr.tol, err
        assert stats["fp32_terms"] > 0
    h.close()
