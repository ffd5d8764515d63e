"""expRK4s6 time stepping on the GPU (Sec. 1, eq. (expRK4s6); Sec. 5, fourth
experiment: 2-D advection-diffusion-reaction, N = 100, n = 10^4, tol 1e-7)
through the C ABI, against the oracle's integrator and a 1e-12 Runge-Kutta
reference of the same semi-discrete system.

Parity: with the oracle's Algorithm 1 parameters both sides make the same
block calls with the same stopping decisions, so after 16 steps the states
agree to 1e-10 (relative, max norm); 64 calls of a 1e-12-parity solve plus
the pointwise stage arithmetic.  End to end: at the paper's largest step the
error against the reference is the scheme's own (the oracle's, within 5 %),
and the smallest step is at least 100 times more accurate (order four
predicts 256).
"""
import numpy as np
import pytest

import oracle
import refs
import workloads as wl
from gpu_util import say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu

N = 100
TOL = 1e-7


def _setup():
    op = wl.adr_operator(N)
    return op, wl.adr_reaction(), wl.adr_initial(N)


def _run_gpu(op_h, prm, gc, u0, h, ns, precision=pc.FP64):
    import torch
    u = torch.from_numpy(u0.copy()).cuda()
    st = pc.phicomb_exprk4s6(op_h.h, prm, gc, h, ns, TOL, precision, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st.as_dict()


def test_exprk4s6_matches_oracle_pinned():
    op, gc, u0 = _setup()
    h, _ = wl.adr_steps(1)
    po = oracle.params(op, TOL, wl.params_vector(op.n))
    say(f"[gpu] expRK4s6 ADR N={N} 16 steps h={h:.3e} pinned")
    uo, calls = oracle.exprk4s6(op, gc, u0, h, 16, TOL, po["shift"], po["s"])
    H = pc.Operator(op)
    ug, st = _run_gpu(H, pc.params_from_dict(po), gc, u0, h, 16)
    H.close()
    err = np.abs(ug - uo).max() / np.abs(uo).max()
    terms_o = sum(c["terms_S"] + c["terms_rec"] for c in calls)
    say(f"      calls {st['calls']} terms {st['terms']}/{terms_o} err {err:.2e}")
    assert st["status"] == pc.OK and st["steps"] == 16 and st["calls"] == 64
    assert abs(st["terms"] - terms_o) <= 4
    assert err <= 1e-10, err


def test_exprk4s6_end_to_end_accuracy():
    op, gc, u0 = _setup()
    ref = refs.ode_reference(op, gc, u0, wl.ADR["t_end"])
    H = pc.Operator(op)
    prm = H.params(TOL, v=wl.params_vector(op.n))
    errs = {}
    for i in (1, 7):
        h, ns = wl.adr_steps(i)
        ug, st = _run_gpu(H, prm, gc, u0, h, ns)
        errs[i] = np.abs(ug - ref).max() / np.abs(ref).max()
        say(f"[gpu] expRK4s6 ADR h_{i}={h:.3e} steps {ns}: rel err {errs[i]:.3e}, "
            f"{st['ms']:.0f} ms, max s_int {st['max_s_int']}")
        assert st["status"] == pc.OK and st["steps"] == ns
    H.close()
    h, ns = wl.adr_steps(1)
    po = oracle.params(op, TOL, wl.params_vector(op.n))
    uo, _ = oracle.exprk4s6(op, gc, u0, h, ns, TOL, po["shift"], po["s"])
    e_orc = np.abs(uo - ref).max() / np.abs(ref).max()
    say(f"      oracle h_1: rel err {e_orc:.3e}")
    assert abs(errs[1] / e_orc - 1) < 0.05
    assert errs[7] * 100 <= errs[1]


def test_exprk4s6_mixed_precision():
    """The mixed-precision path through the integrator.  At these steps every
    call has s_int = 1 (no recovery steps), so no term runs in FP32 and the
    result must equal the FP64 one to 10 tol (in practice exactly)."""
    op, gc, u0 = _setup()
    h, _ = wl.adr_steps(1)
    H = pc.Operator(op)
    prm = H.params(TOL, v=wl.params_vector(op.n))
    u64, _ = _run_gpu(H, prm, gc, u0, h, 32)
    u32, st = _run_gpu(H, prm, gc, u0, h, 32, pc.MIXED)
    H.close()
    err = np.abs(u32 - u64).max() / np.abs(u64).max()
    say(f"[gpu] expRK4s6 mixed: fp32 terms {st['fp32_terms']} err {err:.2e}")
    assert err <= 10 * TOL


def test_exprk4s6_rejects_bad_arguments():
    import torch
    op, gc, u0 = _setup()
    H = pc.Operator(op)
    prm = H.params(TOL)
    u = torch.from_numpy(u0.copy()).cuda()
    for args in ((0.0, 4), (-1e-3, 4), (1e-3, -1)):
        with pytest.raises(pc.PhicombError) as e:
            pc.phicomb_exprk4s6(H.h, prm, gc, args[0], args[1], TOL, pc.FP64, u)
        assert e.value.status == pc.EINVAL
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_exprk4s6(H.h, prm, [0.0, np.nan, 0.0, 0.0], 1e-3, 1, TOL, pc.FP64, u)
    assert e.value.status == pc.EINVAL
    H.close()
    lr = pc.Operator(wl.lowrank_operator(wl.lowrank_cores()["M1"], N * N))
    prm = lr.params(TOL)
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_exprk4s6(lr.h, prm, gc, 1e-3, 1, TOL, pc.FP64, u)
    assert e.value.status == pc.EINVAL
    lr.close()


@pytest.mark.parametrize("kind", ["stencil", "dense", "dense2048"])
def test_exprk4s6_other_operator_kinds(kind):
    """The right-hand side through the stencil row product (a 2-D Laplacian
    stencil) and through a dense operator's CSR form, against the oracle's
    integrator with pinned parameters.  The n = 2048 dense operator (the
    served stream's largest, upper triangular non-normal) needs more solve
    workgroups (one per 32 rows) than its row count alone asks for."""
    steps = 20
    if kind == "stencil":
        op = wl.laplacian_2d(40, kappa=1e-3)
        u0 = wl.adr_initial(40)
    elif kind == "dense":
        rng = np.random.default_rng(5)
        A = rng.standard_normal((300, 300)) * 0.2 - np.diag(rng.uniform(0, 30, 300))
        op = wl.Dense(np.ascontiguousarray(A))
        u0 = rng.uniform(0, 1, 300)
    else:
        rng = np.random.default_rng(6)
        op = wl.dense_upper_nonnormal(2048, rng)
        u0 = rng.uniform(0, 1, 2048)
        steps = 3
    gc = wl.adr_reaction(50.0)
    h = 1e-3
    po = oracle.params(op, TOL, wl.params_vector(op.n))
    say(f"[gpu] expRK4s6 {kind} n={op.n} {steps} steps pinned")
    uo, calls = oracle.exprk4s6(op, gc, u0, h, steps, TOL, po["shift"], po["s"])
    H = pc.Operator(op)
    ug, st = _run_gpu(H, pc.params_from_dict(po), gc, u0, h, steps)
    H.close()
    err = np.abs(ug - uo).max() / np.abs(uo).max()
    say(f"      err {err:.2e} terms {st['terms']}")
    assert st["status"] == pc.OK and st["calls"] == 4 * steps
    assert err <= 1e-10, err


def test_exprk4s6_failing_call_leaves_last_completed_step():
    """A tolerance no Taylor sum can meet makes the first call of the first
    step stop with ENOCONV: with a unit step the scaled steps have norm
    about 17 (the parameters are chosen for tol 1e-7), whose Taylor terms
    are still ~1e-77 of the sum at the 150-term cap, far above 1e-300 (a
    small step's terms would underflow to zero first and end the loop).
    The status comes back and u keeps its initial value (every step's
    update is skipped once a call has failed)."""
    import torch
    op, gc, u0 = _setup()
    h, _ = wl.adr_steps(1)
    H = pc.Operator(op)
    prm = H.params(TOL, v=wl.params_vector(op.n))
    u = torch.from_numpy(u0.copy()).cuda()
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_exprk4s6(H.h, prm, gc, 1.0, 3, 1e-300, pc.FP64, u)
    torch.cuda.synchronize()
    assert e.value.status == pc.ENOCONV
    assert np.array_equal(u.cpu().numpy(), u0)
    # and the operator still integrates normally afterwards
    ug, st = _run_gpu(H, prm, gc, u0, h, 4)
    assert st["status"] == pc.OK and st["steps"] == 4
    H.close()
