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


def test_served_stream_sample_at_config5_sizes():
    """Five seconds of the served stream (Poisson arrivals at 200/s over the
    resident pool of 64 stencils with n up to 2^20 and 32 dense non-normal
    operators with n in 256..2048; p, r, tol and precision per request as in
    the benchmark), submitted at their arrival times; a seeded 2 % sample is
    checked: stencil requests against the DST-I closed form within
    max(10 tol, 1e-12), dense requests against the oracle run with the same
    (GPU) parameters at the parity bar (1e-12 FP64)."""
    import torch
    ops, reqs = wl.config5_stream(duration_s=5.0)
    handles = [pc.Operator(o) for o in ops]
    prms = {}
    for i, h in enumerate(handles):
        for tol in (1e-6, 1e-10):
            prms[(i, tol)] = h.params(tol, v=wl.params_vector(ops[i].n))
    pc.phicomb_serve_config(0, 8)
    pick = np.random.default_rng(2024).uniform(size=len(reqs)) < 0.02
    say(f"[gpu] served stream: {len(reqs)} requests over 5 s, {int(pick.sum())} sampled")
    pending, sampled = [], []
    t0 = time.perf_counter()
    i = 0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        assert now < 120.0, "served stream did not drain"
        while i < len(reqs) and reqs[i]["arrival"] <= now:
            q = reqs[i]
            op = ops[q["op_index"]]
            t, beta, V = wl.stream_request_inputs(op, q)
            prec = pc.MIXED if (q["tol"] == 1e-6 and op.kind != "dense") else pc.FP64
            Vd = torch.from_numpy(V).cuda()
            Wd = torch.empty((op.n, q["r"]), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            tk = pc.phicomb_submit(handles[q["op_index"]].h, prms[(q["op_index"], q["tol"])],
                                   q["p"], q["r"], t, beta, Vd, q["tol"], prec, Wd)
            pending.append((tk, i, Vd, Wd, t, beta, V, prec))
            i += 1
        still = []
        for item in pending:
            st, _ = pc.phicomb_poll(item[0])
            if st == pc.PENDING:
                still.append(item)
                continue
            assert st == pc.OK, pc.phicomb_strerror(st)
            if pick[item[1]]:
                sampled.append((item[1], item[5], item[4], item[6], item[3].cpu().numpy(),
                                item[7]))
        pending = still
        time.sleep(0.0003)
    worst = {}
    for k, beta, t, V, W, prec in sampled:
        q = reqs[k]
        op = ops[q["op_index"]]
        if op.kind == "stencil":
            ref = refs.dst_laplacian(op, t, beta, V)
            bar = max(10 * q["tol"], 1e-12)
        else:
            pg = prms[(q["op_index"], q["tol"])]
            ref, _ = oracle.solve(op, q["p"], q["r"], t, beta, V, q["tol"], pg.shift, pg.s)
            bar = TOL_FP64 if prec == pc.FP64 else 10 * q["tol"]
        err = refs.rel2_cols(W, ref).max()
        key = f"{op.kind} n={op.n} tol={q['tol']:g}"
        worst[key] = max(worst.get(key, 0.0), err)
        assert err <= bar, (k, key, q["p"], q["r"], err, bar)
    for key in sorted(worst):
        say(f"      {key}: {worst[key]:.2e}")
    assert any(ops[reqs[k]["op_index"]].kind == "dense" for k, *_ in sampled)
    assert max(ops[reqs[k]["op_index"]].n for k, *_ in sampled) > 100000
    for h in handles:
        h.close()
