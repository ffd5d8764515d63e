"""Helpers for the GPU tests: run the HIP path through the C ABI."""
import sys

import numpy as np

import paper_2509_26475_amd as pc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_solve(problem, prm=None, precision=pc.FP64, op=None, t=None, beta=None, V=None,
              tol=None):
    import torch
    own = op is None
    if own:
        op = pc.Operator(problem.op)
    t = problem.t if t is None else t
    beta = problem.beta if beta is None else beta
    V = problem.V if V is None else V
    tol = problem.tol if tol is None else tol
    if prm is None:
        prm = op.params(tol, v=problem.v)
    elif isinstance(prm, dict):
        prm = pc.params_from_dict(prm)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    W, st = op.solve(prm, t, beta, Vd, tol, precision)
    torch.cuda.synchronize()
    out = W.cpu().numpy()
    if own:
        op.close()
    return out, st.as_dict(), prm
