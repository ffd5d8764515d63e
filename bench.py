#!/usr/bin/env python3
"""Throughput of the phi-combination hot path on one MI355X.

One step = one pass of the whole path over one synthetic problem:
parameter selection (Algorithm 1: power basis, objective, Brent) followed
by the block solve (Algorithm 3) for r abscissae, with the operator and
the vectors already resident in HBM.

Workload (default): 3-D Dirichlet Laplacian, 7-point stencil on a 128^3
grid (n = 2^21, h = 1/129), p = 2, r = 2, t_i = c_i * 1e-3 with
c = (1/2, 1), beta_ij = c_i^j, v_j ~ U(-1, 1), tol = 1e-12, FP64: the
largest single-GPU configuration, whose working set (about 350 MB) exceeds
the 256 MB Infinity Cache.  --workload selects the others (the 512^2
convection-diffusion operator is cache resident: its bandwidth is
effective, not HBM).

Prints one JSON line.  ``roofline`` describes the solve kernel (the
dominant kernel): algorithmic bytes per launch / its average duration
measured with HIP events on the launch stream; ``traffic`` is the HBM
traffic per launch from the committed rocprofv3 counter summary when it was
taken on the current kernel source.  ``cpu_baseline`` times the CPU oracle
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "phi-comb solves/s + block-SpMM HBM GB/s at tol; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("internal.h", "solve_body.h", "solve.hip"):
        with open(os.path.join(ROOT, "paper_2509_26475_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only
    if they were taken on the current kernel source."""
    path = os.path.join(PROFILE_DIR, "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(f"{kernel}|{workload}")
        if not e or e.get("source_hash") != kernel_source_hash():
            return None
        return float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(problem, gpu_stats: dict, extras: bool = True) -> dict:
    """The oracle (single-threaded C) on a bounded sample of the headline
    step: Algorithm 1 in full, and Algorithm 3 with the same operator,
    vectors, weights and parameters at t/8 (s_int about 1/8 of the full
    solve), scaled to the full solve by its column-terms (Taylor terms times
    block width, S-series and recovery, from the GPU's statistics)."""
    import oracle
    pr = problem
    t0 = time.perf_counter()
    prm = oracle.params(pr.op, pr.tol, pr.v)
    t_par = time.perf_counter() - t0
    t1 = time.perf_counter()
    _, st = oracle.solve(pr.op, pr.p, pr.r, pr.t / 8.0, pr.beta, pr.V, pr.tol, prm["shift"],
                         prm["s"])
    t_smp = time.perf_counter() - t1
    cS, cR = (pr.p + 1) * pr.r, 2 * pr.r
    col_smp = (st["terms_S"] - 1) * cS + st["terms_rec"] * cR
    col_full = (gpu_stats["terms_S"] - 1) * cS + gpu_stats["terms_rec"] * cR
    t_solve = t_smp * col_full / max(1, col_smp)
    out = {"value": 1.0 / (t_par + t_solve), "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": (f"Algorithm 1 in full ({t_par:.1f} s) and Algorithm 3 at t/8 "
                      f"(s_int {st['s_int']}, {st['terms_S']}+{st['terms_rec']} terms, "
                      f"{t_smp:.1f} s) scaled by column-terms to the full solve "
                      f"({gpu_stats['terms_S']}+{gpu_stats['terms_rec']} terms: {t_solve:.1f} s); "
                      "single-threaded C"),
           "cpu_model": _cpu_model(), "host_cores": len(os.sched_getaffinity(0))}
    if extras:
        out["others"] = cpu_baseline_others(oracle)
    return out


def cpu_baseline_others(oracle) -> dict:
    """The oracle (single thread) on bounded samples of the other measured
    workloads, in the units of their bench sections."""
    import workloads as wl
    res = {}
    # third experiment: one (core, t), parameters + solve
    pr = wl.exp3_problem("M2", 10.0, seed=0)
    t0 = time.perf_counter()
    oracle.full(pr)
    res["exp3_M2_t10_total_ms"] = 1e3 * (time.perf_counter() - t0)
    # fourth experiment: the first 64 steps at h_1 (the integration has 512)
    op = wl.adr_operator(wl.ADR["N"])
    gc = wl.adr_reaction(wl.ADR["gamma"])
    u0 = wl.adr_initial(wl.ADR["N"])
    po = oracle.params(op, 1e-7, wl.params_vector(op.n))
    h, _ = wl.adr_steps(1)
    t0 = time.perf_counter()
    oracle.exprk4s6(op, gc, u0, h, 64, 1e-7, po["shift"], po["s"])
    res["exp4_h1_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / 64
    # single block series: convection-diffusion 512^2 at |t| ||A|| = 1
    pr = wl.config2()
    t = pr.t / pr.t.max() * (1.0 / _norm_inf(pr.op))
    t0 = time.perf_counter()
    oracle.series_block(pr.op, pr.p, pr.r, t, pr.beta, pr.V, pr.tol)
    res["series_tnorm1_ms"] = 1e3 * (time.perf_counter() - t0)
    return res


def _norm_inf(op) -> float:
    """max_i sum_j |a_ij| of an operator description (interior stencil row)."""
    if op.kind == "stencil":
        k = 5 if op.dim == 2 else 7
        return float(abs(op.coef[:k]).sum() + abs(op.superdiag))
    import numpy as np
    if op.kind == "csr":
        rp, _, va = op.csr()
        return float(np.add.reduceat(np.abs(va), rp[:-1].astype(np.int64)).max())
    return float(np.abs(op.A).sum(axis=1).max())


def bench_mixed(pc, wl, torch, reps: int) -> list:
    """Solves/s of FP64 and mixed precision on the 128^3 Laplacian and its
    nonnormal variant at tol 1e-6 (parameters computed once per operator)."""
    out = []
    for nonnormal in (False, True):
        pr = wl.config3(nonnormal=nonnormal, tol=1e-6)
        op = pc.Operator(pr.op)
        prm = pc.phicomb_params(op.h, pr.tol, 61, None, 1)
        V = torch.from_numpy(pr.V).cuda()
        W = torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda")
        row = {"workload": pr.name + "_p2_r2_tol1e-6"}
        for name, prec in (("fp64", pc.FP64), ("mixed", pc.MIXED)):
            pc.phicomb_solve(op.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, prec, W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = [pc.phicomb_solve(op.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, prec, W)
                   for _ in range(reps)]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            st = sts[-1]
            row[name + "_solves_per_s"] = 1.0 / dt
            row[name + "_kernel_ms"] = st.ms
            # algorithmic bytes over the kernel time, against the HBM peak
            row[name + "_achieved_GBps"] = st.bytes_alg / (st.ms * 1e-3) / 1e9
            row[name + "_hbm_frac"] = row[name + "_achieved_GBps"] / HBM_PEAK_GBS
            if prec == pc.MIXED:
                row["fp32_term_fraction"] = st.fp32_terms / max(1, st.terms_S + st.terms_rec)
        row["mixed_over_fp64"] = row["mixed_solves_per_s"] / row["fp64_solves_per_s"]
        out.append(row)
        op.close()
    return out


def bench_batched(pc, wl, torch, reps: int) -> dict:
    """256 kappa-Laplacians of uneven size (side U{32..256}, kappa
    logU[1e-2, 1e2], p, r U{1,2,3}, t logU[1e-5, 1e-2], tol 1e-8) in one
    persistent launch (graph replay), FP32 bulk (mixed) and FP64."""
    probs = wl.config4()
    ops = [pc.Operator(pr.op) for pr in probs]
    prms = [pc.phicomb_params(o.h, pr.tol, 61, None, 1) for o, pr in zip(ops, probs)]
    Vd = [torch.from_numpy(pr.V).cuda() for pr in probs]
    Wd = [torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda") for pr in probs]
    items = [(ops[k].h, prms[k], pr.p, pr.r, pr.t, pr.beta, Vd[k], Wd[k], pr.tol)
             for k, pr in enumerate(probs)]
    torch.cuda.synchronize()
    out = {"workload": "256 kappa-Laplacians 2-D, side U{32..256}, p,r U{1,2,3}, tol 1e-8",
           "instances": len(probs)}
    for name, prec in (("mixed", pc.MIXED), ("fp64", pc.FP64)):
        print(f"[bench] batched {name}: plan", file=sys.stderr, flush=True)
        b = pc.phicomb_batch_create(items, prec)
        info = pc.phicomb_batch_info(b)
        st, stats = pc.phicomb_batch_run(b, len(probs))      # first run captures the graph
        print(f"[bench] batched {name}: first run {stats[0].ms:.0f} ms", file=sys.stderr,
              flush=True)
        if st != pc.OK:
            raise RuntimeError(f"batch failed: {pc.phicomb_strerror(st)}")
        ms = []
        for _ in range(reps):
            st, stats = pc.phicomb_batch_run(b, len(probs))
            ms.append(stats[0].ms)
        pc.phicomb_batch_destroy(b)
        best = min(ms)
        out[name] = {"solves_per_s": len(probs) / (best * 1e-3), "launch_ms": best,
                     "predicted_ms": info["predicted_ms"], "groups": info["groups"],
                     "workgroups": info["workgroups"],
                     "max_s_int": max(s.s_int for s in stats),
                     "fp32_terms": sum(s.fp32_terms for s in stats),
                     "terms": sum(s.terms_S + s.terms_rec for s in stats)}
    for o in ops:
        o.close()
    return out


def bench_exp2(pc, wl, torch) -> dict:
    """Second experiment of the paper (collocation Laplacian, n = 99, dense,
    p = 6, tol 2^-53), one solve per t = 1e-4 .. 1 (Table 1's rows) with
    parameters from the GPU; accuracy against an exact reference is checked
    by the tests for t <= 0.1 (t = 1 takes 2.6e5 scaling steps)."""
    out = {"workload": "chebyshev collocation Laplacian N=100 L=2 (n=99), p=6, tol 2^-53",
           "t": [], "solve_ms": [], "s_int": []}
    for pr in wl.exp2_problems():
        op = pc.Operator(pr.op)
        prm = pc.phicomb_params(op.h, pr.tol, 61, pr.v, 1)
        V = torch.from_numpy(pr.V).cuda()
        W = torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = pc.phicomb_solve(op.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, pc.FP64, W)
        torch.cuda.synchronize()
        print(f"[bench] second experiment t={pr.t[0]:g}: {st.ms:.0f} ms", file=sys.stderr,
              flush=True)
        out["t"].append(float(pr.t[0]))
        out["solve_ms"].append(1e3 * (time.perf_counter() - t0))
        out["s_int"].append(st.s_int)
        op.close()
    return out


def bench_exp3(pc, wl, torch) -> dict:
    """Third experiment of the paper (A = U W^T, DCT-II basis, cores M1-M3 at
    the paper's n and p, alpha = 1, tol 2^-53): parameters (Algorithm 1) and
    solve (Algorithm 3) per (core, t) on the GPU, timed end to end like the
    paper's Tables 2-4; accuracy against the closed form is checked by the
    tests."""
    cases = [("M1", 0.1), ("M1", 1.0), ("M1", 10.0), ("M1", 50.0), ("M1", 100.0),
             ("M2", 0.1), ("M2", 1.0), ("M2", 10.0), ("M2", 50.0), ("M2", 100.0),
             ("M3", 1e-5), ("M3", 1e-3), ("M3", 0.1), ("M3", 1.0), ("M3", 10.0)]
    out = {"workload": "low-rank A = U W^T (DCT-II U, W = U M^T); M1 n=2e5 p=3, "
                       "M2 n=4e5 p=4, M3 n=5e5 p=2; alpha=1, tol 2^-53",
           "core": [], "t": [], "params_ms": [], "solve_ms": [], "total_ms": [], "s_int": []}
    ops = {}
    for core, t in cases:
        pr = wl.exp3_problem(core, t, seed=0)
        if core not in ops:
            ops[core] = pc.Operator(pr.op)
        op = ops[core]
        V = torch.from_numpy(pr.V).cuda()
        W = torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prm = pc.phicomb_params(op.h, pr.tol, 61, pr.v, 1)
        t1 = time.perf_counter()
        st = pc.phicomb_solve(op.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, pc.FP64, W)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        print(f"[bench] third experiment {core} t={t:g}: s_int={st.s_int} "
              f"{1e3 * (t2 - t0):.1f} ms", file=sys.stderr, flush=True)
        out["core"].append(core)
        out["t"].append(t)
        out["params_ms"].append(1e3 * (t1 - t0))
        out["solve_ms"].append(1e3 * (t2 - t1))
        out["total_ms"].append(1e3 * (t2 - t0))
        out["s_int"].append(st.s_int)
    for op in ops.values():
        op.close()
    return out


def bench_exp4(pc, wl, torch) -> dict:
    """Fourth experiment of the paper: expRK4s6 on the 2-D ADR problem (N = 100,
    n = 10^4) to t = 1/2 with h_i = 2^-8 (1/2)/(i + 1), i = 1..7, tol 1e-7;
    device time of each whole integration (4 block calls per step) and its
    relative max-norm error against a 1e-12 Runge-Kutta reference."""
    import numpy as np
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    import refs
    op = wl.adr_operator(wl.ADR["N"])
    gc = wl.adr_reaction(wl.ADR["gamma"])
    u0 = wl.adr_initial(wl.ADR["N"])
    ref = refs.ode_reference(op, gc, u0, wl.ADR["t_end"])
    H = pc.Operator(op)
    prm = pc.phicomb_params(H.h, 1e-7, 61, None, 1)
    out = {"workload": "ADR 2-D, N=100 (n=1e4), eps=1e-3, alpha=-1/2, gamma=1000, t in [0, 1/2], "
                       "expRK4s6, tol 1e-7",
           "h": [], "steps": [], "ms": [], "rel_err_inf": [], "calls": []}
    for i in range(1, 8):
        h, ns = wl.adr_steps(i)
        u = torch.from_numpy(u0.copy()).cuda()
        torch.cuda.synchronize()
        st = pc.phicomb_exprk4s6(H.h, prm, gc, h, ns, 1e-7, pc.FP64, u)
        torch.cuda.synchronize()
        err = float(np.abs(u.cpu().numpy() - ref).max() / np.abs(ref).max())
        print(f"[bench] fourth experiment h_{i}: {ns} steps {st.ms:.0f} ms err {err:.2e}",
              file=sys.stderr, flush=True)
        out["h"].append(h)
        out["steps"].append(ns)
        out["ms"].append(st.ms)
        out["rel_err_inf"].append(err)
        out["calls"].append(st.calls)
    H.close()
    return out


def bench_series(pc, wl, torch) -> dict:
    """The Proposition's single block series against Algorithm 3 on the
    convection-diffusion operator (512^2, CSR, p = 3, r = 3, tol 1e-12) at
    steps scaled so that |t| ||A||_inf is about 0.1, 1 and 10; both timed on
    the device (kernel events), Algorithm 1 excluded."""
    import numpy as np
    pr = wl.config2()
    op = pc.Operator(pr.op)
    prm = pc.phicomb_params(op.h, pr.tol, 61, pr.v, 1)
    nrm = _norm_inf(pr.op)
    V = torch.from_numpy(pr.V).cuda()
    W1 = torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda")
    W2 = torch.empty_like(W1)
    out = {"workload": "convdiff 512^2 CSR, p=3, r=3, tol 1e-12", "t_norm": [],
           "series_ms": [], "series_terms": [], "alg3_ms": [], "alg3_s_int": [],
           "rel_diff": []}
    for target in (0.1, 1.0, 10.0):
        t = pr.t / pr.t.max() * (target / nrm)
        best_s, best_a = None, None
        for _ in range(3):
            s1 = pc.phicomb_solve_series(op.h, pr.p, pr.r, t, pr.beta, V, pr.tol, W1)
            s2 = pc.phicomb_solve(op.h, prm, pr.p, pr.r, t, pr.beta, V, pr.tol, pc.FP64, W2)
            best_s = s1 if best_s is None or s1.ms < best_s.ms else best_s
            best_a = s2 if best_a is None or s2.ms < best_a.ms else best_a
        torch.cuda.synchronize()
        diff = float((torch.linalg.norm(W1 - W2, dim=0) / torch.linalg.norm(W2, dim=0)).max())
        print(f"[bench] series |t|A|| = {target:g}: {best_s.ms:.3f} ms ({best_s.terms_S} terms)"
              f" vs Algorithm 3 {best_a.ms:.3f} ms", file=sys.stderr, flush=True)
        out["t_norm"].append(target)
        out["series_ms"].append(best_s.ms)
        out["series_terms"].append(best_s.terms_S)
        out["alg3_ms"].append(best_a.ms)
        out["alg3_s_int"].append(best_a.s_int)
        out["rel_diff"].append(diff)
    op.close()
    return out


def bench_complex(pc, wl, torch) -> dict:
    """Complex data (Sec. 1): A = (1 + 0.5i) L + diag(pot), L the 2-D 5-point
    Laplacian on a 512 x 512 grid (CSR, n = 2^18), pot complex N(0, 50^2),
    p = 2, r = 2, complex t, complex weights and V, tol 1e-12: Algorithm 1
    on the real representation, Algorithm 3 in the complex kernel."""
    import numpy as np
    import scipy.sparse as sp
    m = 512
    n = m * m
    rng = np.random.default_rng(7)
    h2 = (m + 1.0) ** 2
    T = sp.diags([np.full(m - 1, h2), np.full(m, -2.0 * h2), np.full(m - 1, h2)], [-1, 0, 1])
    L = sp.kron(sp.identity(m), T) + sp.kron(T, sp.identity(m))
    pot = 50.0 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    A = ((1.0 + 0.5j) * L + sp.diags(pot)).tocsr()
    A.sort_indices()
    p, r, tol = 2, 2, 1e-12
    t = 2e-4 * np.array([1.0, 0.5]) * np.exp(0.3j)
    beta = rng.standard_normal((r, p + 1)) + 1j * rng.standard_normal((r, p + 1))
    V = torch.from_numpy(rng.standard_normal((n, p + 1)) + 1j * rng.standard_normal((n, p + 1))).cuda()
    W = torch.empty((n, r), dtype=torch.complex128, device="cuda")
    h = pc.phicomb_zop_create_csr(n, A.indptr, A.indices, A.data)
    try:
        t0 = time.perf_counter()
        prm = pc.phicomb_zparams(h, tol, 61, None, 1)
        torch.cuda.synchronize()
        t_par = time.perf_counter() - t0
        st = None
        for _ in range(2):
            st = pc.phicomb_zsolve(h, prm, p, r, t, beta, V, tol, W)
        terms = st.terms_S + st.terms_rec
        return {"workload": "complex (1+0.5i) 2-D Laplacian 512^2 + complex potential, CSR, "
                            "p=2, r=2, complex t, tol 1e-12",
                "params_ms": 1e3 * t_par, "solve_kernel_ms": st.ms, "s_int": st.s_int,
                "terms_S": st.terms_S, "terms_rec": st.terms_rec,
                "us_per_term": 1e3 * st.ms / max(1, terms)}
    finally:
        pc.phicomb_zop_destroy(h)


def bench_spmm(pc, wl, torch) -> dict:
    """The block product Y = (A - xi I) X alone on the 128^3 Laplacian
    (n = 2^21) as a 7-point stencil and as CSR, c = 4, 6, 12 columns:
    algorithmic bytes (X read and Y written once, 16 n c, plus the CSR arrays
    12 nnz + 4 (n + 1)) over the device time per launch: 20 launches back to
    back on torch's current stream between two events (so the host's launch
    gaps are hidden), best of 3 such runs."""
    pr = wl.config3()
    st = pr.op
    rp, ci, va = st.csr()
    out = {"workload": "128^3 Laplacian, n=2^21, Y = (A - xi I) X", "rows": []}
    for kind, desc in (("stencil", st), ("csr", wl.CSR(st.n, rp, ci, va))):
        op = pc.Operator(desc)
        opb = 0.0 if kind == "stencil" else 12.0 * len(va) + 4.0 * (st.n + 1)
        for c in (4, 6, 12):
            X = torch.randn((c, st.n), dtype=torch.float64, device="cuda")
            Y = torch.empty_like(X)
            pc.phicomb_op_apply(op.h, X, 0.5, Y)
            best = None
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(20):
                    pc.phicomb_op_apply(op.h, X, 0.5, Y)
                e1.record()
                e1.synchronize()
                ms = e0.elapsed_time(e1) / 20
                best = ms if best is None else min(best, ms)
            gbs = (16.0 * st.n * c + opb) / (best * 1e-3) / 1e9
            print(f"[bench] block product {kind} c={c}: {best * 1e3:.1f} us {gbs:.0f} GB/s",
                  file=sys.stderr, flush=True)
            out["rows"].append({"kind": kind, "cols": c, "us": best * 1e3, "GBps": gbs,
                                "hbm_frac": gbs / HBM_PEAK_GBS})
        op.close()
    return out


def _served_reference(job):
    """Exact result of one sampled served request (run in a worker process):
    stencils (Dirichlet Laplacians) by the DST-I eigen-decomposition closed
    form, dense operators by scipy's expm_multiply (Al-Mohy & Higham 2011)
    on the augmented matrix of Theorem 1, one abscissa at a time."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import refs
    op, t, beta, V, W = job
    if op.kind == "stencil":
        ref = refs.dst_laplacian(op, t, beta, V)
    else:
        ref = refs.expm_multiply_dense_aug(op.A, t, beta, V)
    return float(refs.rel2_cols(W, ref).max())


def bench_served(pc, wl, torch, duration: float, rate: float, slots: int,
                 sample_frac: float = 0.02, capacity_window: float = 10.0) -> dict:
    """Poisson request stream over a resident operator pool (70 % 2-D/3-D
    stencils n ~ logU[4096, 2^20], 30 % dense nonnormal n in 256..2048),
    p ~ U{1..4}, r ~ U{1..3}, tol 1e-6 (mixed; dense FP64) or 1e-10 (FP64).
    Latency = completion seen by polling - scheduled arrival.  A seeded
    sample of the requests (sample_frac) is checked against exact
    references after the stream.  Capacity: the requests of the stream's
    first capacity_window seconds submitted at once, completions per second."""
    import numpy as np
    ops, reqs = wl.config5_stream(duration_s=duration, rate=rate)
    handles = [pc.Operator(o) for o in ops]
    norms = [_norm_inf(o) for o in ops]
    prms = {}
    for i, h in enumerate(handles):
        for tol in (1e-6, 1e-10):
            prms[(i, tol)] = pc.phicomb_params(h.h, tol, 61, None, 1)
    pc.phicomb_serve_config(0, slots)
    gen = torch.Generator(device="cuda")
    pick = np.random.default_rng(20250).uniform(size=len(reqs)) < sample_frac

    def make(q):
        op = ops[q["op_index"]]
        p, r = q["p"], q["r"]
        t = (np.arange(1, r + 1) / r) * q["gamma"] / norms[q["op_index"]]
        gen.manual_seed(q["seed"])
        V = torch.randn((op.n, p + 1), generator=gen, dtype=torch.float64, device="cuda")
        W = torch.empty((op.n, r), dtype=torch.float64, device="cuda")
        prec = pc.MIXED if (q["tol"] == 1e-6 and op.kind != "dense") else pc.FP64
        return op, t, V, W, prec

    def submit(q, t, V, W, prec):
        return pc.phicomb_submit(handles[q["op_index"]].h, prms[(q["op_index"], q["tol"])],
                                 q["p"], q["r"], t, np.ones((q["r"], q["p"] + 1)), V, q["tol"],
                                 prec, W)

    lat, pending, kernel_ms, sampled = [], [], [], []
    i, n_done = 0, 0
    t0 = time.perf_counter()
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i]["arrival"] <= now:
            q = reqs[i]
            op, t, V, W, prec = make(q)
            torch.cuda.current_stream().synchronize()
            tk = submit(q, t, V, W, prec)
            pending.append((tk, q["arrival"], V, W, i, t))
            i += 1
        still = []
        for tk, arr, V, W, k, t in pending:
            st, stats = pc.phicomb_poll(tk)
            if st == pc.PENDING:
                still.append((tk, arr, V, W, k, t))
                continue
            if st != pc.OK:
                raise RuntimeError(f"served request failed: {pc.phicomb_strerror(st)}")
            lat.append(time.perf_counter() - t0 - arr)
            kernel_ms.append(stats.ms)
            n_done += 1
            if pick[k]:
                sampled.append((k, t, V.cpu().numpy(), W.cpu().numpy()))
        pending = still
        if pending or i < len(reqs):
            time.sleep(0.0002)
    wall = time.perf_counter() - t0
    print(f"[bench] served stream: {n_done} requests in {wall:.1f} s", file=sys.stderr,
          flush=True)

    # capacity: the first capacity_window seconds of the stream, all at once
    first = [q for q in reqs if q["arrival"] < capacity_window]
    inflight = [make(q) for q in first]
    torch.cuda.synchronize()
    tc = time.perf_counter()
    tks = [submit(q, t, V, W, prec) for q, (op, t, V, W, prec) in zip(first, inflight)]
    left = list(tks)
    while left:
        nxt = []
        for tk in left:
            st, _ = pc.phicomb_poll(tk)
            if st == pc.PENDING:
                nxt.append(tk)
            elif st != pc.OK:
                raise RuntimeError(f"capacity request failed: {pc.phicomb_strerror(st)}")
        left = nxt
        if left:
            time.sleep(0.0002)
    cap_wall = time.perf_counter() - tc
    del inflight
    for h in handles:
        h.close()

    # the seeded sample against exact references, in worker processes
    from concurrent.futures import ProcessPoolExecutor
    jobs = []
    for k, t, V, W in sampled:
        q = reqs[k]
        jobs.append((ops[q["op_index"]], t, np.ones((q["r"], q["p"] + 1)), V, W))
    tv = time.perf_counter()
    with ProcessPoolExecutor(max_workers=8) as ex:
        errs = list(ex.map(_served_reference, jobs))
    worst = {"stencil_tol1e-6": 0.0, "stencil_tol1e-10": 0.0, "dense_tol1e-6": 0.0,
             "dense_tol1e-10": 0.0}
    bad = 0
    for (k, _, _, _), e in zip(sampled, errs):
        q = reqs[k]
        key = f"{ops[q['op_index']].kind}_tol{q['tol']:.0e}".replace("e-0", "e-")
        worst[key] = max(worst[key], e)
        bad += int(e > max(10.0 * q["tol"], 1e-12))
    print(f"[bench] served sample of {len(jobs)} checked in {time.perf_counter() - tv:.1f} s",
          file=sys.stderr, flush=True)
    lat_ms = 1e3 * np.asarray(lat)
    return {"workload": f"poisson {rate:g}/s x {duration:g} s, 64 stencil + 32 dense ops",
            "requests": n_done, "slots": slots, "p50_ms": float(np.percentile(lat_ms, 50)),
            "p99_ms": float(np.percentile(lat_ms, 99)), "mean_ms": float(lat_ms.mean()),
            "offered_req_per_s": len(reqs) / duration,
            "completed_req_per_s": n_done / wall,
            "capacity_req_per_s": len(first) / cap_wall,
            "capacity_requests": len(first),
            "mean_kernel_ms": float(np.mean(kernel_ms)),
            "verified": {"sample": len(jobs), "fraction": sample_frac,
                         "over_bar": bad, "bar": "max(10 tol, 1e-12) relative 2-norm per column",
                         "worst_rel_err": worst}}


def dense_workload(wl):
    """Dense non-normal operator of the served stream at its largest size:
    upper triangular n = 2048, strictly upper N(0,1), diagonal -U(0, 50);
    p = 3, r = 3, t_i = (i/3) * 10 / ||A||_inf, beta = 1, V ~ N(0,1),
    tol 1e-10 (FP64)."""
    import numpy as np
    rng = np.random.default_rng(5)
    op = wl.dense_upper_nonnormal(2048, rng)
    t = (np.arange(1, 4) / 3.0) * 10.0 / _norm_inf(op)
    V = np.ascontiguousarray(rng.standard_normal((4, op.n)).T)
    return wl.Problem("dense_upper_2048", op, 3, 3, t, np.ones((3, 4)), V, 1e-10,
                      wl.params_vector(op.n, 1))


WORKLOADS = {
    # name: (description, builder)
    "lap3d128": ("7-point Dirichlet Laplacian 128^3 (stencil), FP64",
                 lambda wl: wl.config3(tol=1e-12)),
    "lap3d128-nonnormal": ("7-point Laplacian 128^3 + 100 on the superdiagonal (stencil), FP64",
                           lambda wl: wl.config3(nonnormal=True, tol=1e-12)),
    "convdiff512-csr": ("csr 5-point upwind convection-diffusion 512x512 (cache resident)",
                        lambda wl: wl.config2(as_csr=True)),
    "convdiff512-stencil": ("stencil 5-point upwind convection-diffusion 512x512 "
                            "(cache resident)", lambda wl: wl.config2(as_csr=False)),
    "dense2048": ("dense upper-triangular non-normal 2048x2048 (MFMA)", None),
}


def _workload_name(key: str, pr) -> str:
    tol = f"tol{pr.tol:.0e}".replace("e-0", "e-")
    return {"lap3d128": f"lap3d_128_stencil_p2_r2_{tol}",
            "lap3d128-nonnormal": f"lap3d_128_nonnormal_stencil_p2_r2_{tol}",
            "convdiff512-csr": f"convdiff2d_512_csr_p3_r3_{tol}",
            "convdiff512-stencil": f"convdiff2d_512_stencil_p3_r3_{tol}",
            "dense2048": f"dense_upper_nonnormal_2048_p3_r3_{tol}"}[key]


def timed_steps(pc, torch, pr, steps: int, warmup: int):
    """Warm-up, then `steps` timed steps (Algorithm 1 + Algorithm 3) bracketed
    by device synchronisations; returns (seconds, per-step stats, params
    seconds, last parameters)."""
    op = pc.Operator(pr.op)
    V = torch.from_numpy(pr.V).cuda()
    W = torch.empty((pr.n, pr.r), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        prm = pc.phicomb_params(op.h, pr.tol, 61, None, 1)
        pc.phicomb_solve(op.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, pc.FP64, W)
    torch.cuda.synchronize()
    stats, t_par = [], 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        prm = pc.phicomb_params(op.h, pr.tol, 61, None, 1)
        b = time.perf_counter()
        st = pc.phicomb_solve(op.h, prm, pr.p, pr.r, pr.t, pr.beta, V, pr.tol, pc.FP64, W)
        t_par += b - a
        stats.append(st.as_dict())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    op.close()
    return dt, stats, t_par, prm


def bench_convdiff_effective(pc, wl, torch) -> dict:
    """The 512^2 convection-diffusion operator (CSR and stencil, p = 3, r = 3,
    tol 1e-12): its ~50 MB working set stays in the 256 MB Infinity Cache, so
    the bandwidth here is effective (algorithmic bytes / kernel time), not
    HBM bandwidth."""
    import numpy as np
    out = {"note": "cache-resident working set: effective bandwidth, not HBM"}
    for key in ("convdiff512-csr", "convdiff512-stencil"):
        pr = WORKLOADS[key][1](wl)
        dt, stats, t_par, _ = timed_steps(pc, torch, pr, 10, 2)
        ms = float(np.mean([s["ms"] for s in stats]))
        byt = float(np.mean([s["bytes_alg"] for s in stats]))
        out[key] = {"workload": _workload_name(key, pr), "steps_per_s": 10 / dt,
                    "solve_kernel_ms": ms, "effective_GBps": byt / (ms * 1e-3) / 1e9,
                    "s_int": stats[-1]["s_int"], "terms_S": stats[-1]["terms_S"],
                    "terms_rec": stats[-1]["terms_rec"]}
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="lap3d128",
                    help="headline workload (default: the 128^3 Laplacian at tol 1e-12)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra sections (mixed precision, batched, experiments, "
                         "block product, served stream)")
    ap.add_argument("--extras", default=None,
                    help="comma-separated subset of the extra sections to run (mixed_tol1e-6, "
                         "convdiff512, batched, exp2, exp3, exp4, series, spmm, complex, served); "
                         "default all")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU layout is described in the design notes, not built)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2509_26475_amd as pc
    import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    desc, builder = WORKLOADS[args.workload]
    pr = dense_workload(wl) if builder is None else builder(wl)
    t_start = time.perf_counter()
    dt, stats, t_par, prm = timed_steps(pc, torch, pr, args.steps, args.warmup)
    value = args.steps / dt
    ms_kernel = float(np.mean([s["ms"] for s in stats]))
    bytes_launch = float(np.mean([s["bytes_alg"] for s in stats]))
    achieved = bytes_launch / (ms_kernel * 1e-3) / 1e9
    kind = pr.op.kind
    kernel_name = f"solve_kernel<{kind},r={pr.r}>"
    workload = _workload_name(args.workload, pr)
    traffic = measured_traffic(kernel_name, workload)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": pr.n, "p": pr.p, "r": pr.r, "operator": desc,
                   "tol": pr.tol, "step": "Algorithm 1 + Algorithm 3"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": kernel_name,
                     "bytes_per_launch": bytes_launch, "ms_per_launch": ms_kernel,
                     "traffic_GBps": (None if traffic is None
                                      else traffic / (ms_kernel * 1e-3) / 1e9)},
        "solve_only_per_s": 1e3 / ms_kernel,
        "params_ms": 1e3 * t_par / args.steps,
        "s_int": stats[-1]["s_int"], "terms_S": stats[-1]["terms_S"],
        "terms_rec": stats[-1]["terms_rec"],
        "shift": prm.shift, "s": prm.s,
    }

    def progress(what, t0):
        print(f"[bench] {what} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)

    progress("headline workload", t_start)
    sections = [
        ("mixed_tol1e-6", "mixed precision", lambda: bench_mixed(pc, wl, torch, reps=5)),
        ("convdiff512", "convection-diffusion 512^2 (effective)",
         lambda: bench_convdiff_effective(pc, wl, torch)),
        ("batched", "batched", lambda: bench_batched(pc, wl, torch, reps=1)),
        ("exp2", "second experiment", lambda: bench_exp2(pc, wl, torch)),
        ("exp3", "third experiment", lambda: bench_exp3(pc, wl, torch)),
        ("exp4", "fourth experiment", lambda: bench_exp4(pc, wl, torch)),
        ("series", "single block series", lambda: bench_series(pc, wl, torch)),
        ("spmm", "block product", lambda: bench_spmm(pc, wl, torch)),
        ("complex", "complex data", lambda: bench_complex(pc, wl, torch)),
    ]
    if args.serve_seconds > 0:
        sections.append(("served", "served stream",
                         lambda: bench_served(pc, wl, torch, args.serve_seconds,
                                              args.serve_rate, args.serve_slots)))
    wanted = None if args.extras is None else set(args.extras.split(","))
    if not args.no_extras:
        for key, what, fn in sections:
            if wanted is not None and key not in wanted:
                continue
            t1 = time.perf_counter()
            line[key] = fn()
            progress(what, t1)
    if not args.no_cpu:
        t1 = time.perf_counter()
        line["cpu_baseline"] = cpu_baseline(pr, stats[-1], extras=not args.no_extras)
        progress("cpu baseline", t1)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
