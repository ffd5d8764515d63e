"""The block product Y = (A - shift I) X on the GPU through the C ABI
against the oracle's operator product, column by column (relative max-norm
1e-14 of the row-sum scale: the two sum each row in their own order, the
GPU with fused multiply-adds)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import say

import paper_2509_26475_amd as pc

pytestmark = pytest.mark.gpu


def _check(desc, ncols, shift, seed=0):
    import torch
    n = desc.n
    X = np.random.default_rng(seed).standard_normal((ncols, n))
    op = pc.Operator(desc)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full_like(Xd, np.nan)
    pc.phicomb_op_apply(op.h, Xd, shift, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    op.close()
    o = oracle.Operator(desc)
    err = 0.0
    for c in range(ncols):
        ref = oracle.apply(o, X[c]) - shift * X[c]
        scale = np.abs(ref).max() + abs(shift) * np.abs(X[c]).max() + 1e-300
        err = max(err, np.abs(Y[c] - ref).max() / scale)
    say(f"[gpu] apply {getattr(desc, 'kind', '?')} n={n} ncols={ncols}: err {err:.2e}")
    assert err <= 1e-14, err


@pytest.mark.parametrize("ncols", [1, 3, 4, 6, 7, 12, 16, 64])
def test_apply_stencil_and_csr(ncols):
    st = wl.laplacian_3d(24, superdiag=100.0)
    _check(st, ncols, 0.5)
    rp, ci, va = st.csr()
    _check(wl.CSR(st.n, rp, ci, va), ncols, -3.0)


def test_apply_dense_and_ragged():
    pr = wl.small_problem(300, 1, 1, seed=2)
    _check(pr.op, 5, 1.25)
    _check(wl.convdiff_2d_upwind(37), 6, 0.0)      # n = 1369: ragged last workgroup


def test_apply_full_size_stencil():
    _check(wl.laplacian_3d(128), 6, 0.0)


def test_apply_rejects_low_rank_and_bad_shapes():
    import torch
    lr = pc.Operator(wl.lowrank_operator(wl.lowrank_cores()["M1"], 64))
    X = torch.zeros((2, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_op_apply(lr.h, X, 0.0, torch.zeros_like(X))
    assert e.value.status == pc.EINVAL
    lr.close()
    op = pc.Operator(wl.laplacian_2d(8))
    X = torch.zeros((65, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PhicombError) as e:
        pc.phicomb_op_apply(op.h, X, 0.0, torch.zeros_like(X))
    assert e.value.status == pc.EINVAL
    op.close()


@pytest.mark.parametrize("grid,dim,sd", [
    ((2, 3, 5), 3, 0.0),       # two-point grid lines: every pair is a whole line
    ((6, 5, 4), 3, 100.0),     # superdiagonal across grid-line ends
    ((30, 17, 1), 2, 0.0),     # 255 pairs: a partial last wave
    ((64, 64, 1), 2, -7.0),
    ((130, 3, 2), 3, 1.0),     # a grid line longer than a wave of pairs
])
@pytest.mark.parametrize("ncols", [1, 5, 13, 16])
def test_apply_stencil_row_pairs(grid, dim, sd, ncols):
    """Stencils with an even grid line take the row-pair kernel (x-neighbours
    across lanes, first and last lane of a wave loading their own); random
    non-symmetric coefficients so that every neighbour's weight is seen."""
    rng = np.random.default_rng(sum(grid) + ncols)
    coef = rng.uniform(-2, 2, 7)
    if dim == 2:
        coef[5:] = 0.0
    st = wl.Stencil(dim, grid, coef, sd)
    _check(st, ncols, 0.75, seed=ncols)
