"""Helpers for the GPU tests: run the HIP path through the C ABI."""
import json
import os
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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(tol: float) -> dict:
    """Sampled rows of the oracle's result on the full-size nonnormal 3-D
    Laplacian, written by golden/make_lap3d_nonnormal.py."""
    with open(os.path.join(GOLDEN, f"lap3d_128_nonnormal_tol{tol:.0e}.json")) as f:
        return json.load(f)


def sampled_err(W, g: dict) -> np.ndarray:
    """Per-column relative 2-norm error over the sampled rows (difference
    and reference restricted to the same rows)."""
    rows = np.asarray(g["rows"])
    ref = np.asarray(g["W"])
    return np.linalg.norm(W[rows] - ref, axis=0) / np.linalg.norm(ref, axis=0)
