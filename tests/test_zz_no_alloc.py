"""The application entry point that allocates nothing (marker: gpu).

fl_apply_fractional_noalloc keeps its intermediates in a fixed device array
of the library: called through the C ABI, its result matches
fl_apply_fractional's on the same inputs (the same kernels; at these sizes
the same split of V^T G, so bit for bit), on two calls in a row, the second
smaller, and sizes beyond the array are refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1911_11906_amd import inputs

pytestmark = pytest.mark.gpu
P = ctypes.c_void_p


def note(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_11906_amd.api import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def noalloc(op, F, al, paired, U):
    from paper_1911_11906_amd import _lib
    from paper_1911_11906_amd.api import _ld, _ptr
    f = _lib.load().fl_apply_fractional_noalloc
    al = np.ascontiguousarray(al, dtype=np.float64)
    op.ctx._sync_stream()
    return f(op.ptr, F.shape[1], _ptr(F), _ld(F), al.size, al.ctypes.data_as(P), int(paired), _ptr(U), _ld(U))


def test_noalloc_matches_allocating_entry_point(ctx):
    from paper_1911_11906_amd.api import Operator, colmajor, empty_colmajor
    mesh = inputs.q1_rectangle(40, 40)
    op = Operator.assemble(ctx, mesh)
    op.eigensolve("fp64")
    n = op.n
    for call, (nf, na, paired) in enumerate(((48, 3, False), (16, 2, False), (8, 8, True))):
        note("noalloc call", call, nf, na, paired)
        F = colmajor(inputs.polynomial_forcings(mesh, nf, tag=90 + call), ctx.device)
        al = inputs.alphas_uniform(na, tag=90 + call)
        ncol = nf if paired else nf * na
        U = empty_colmajor(n, ncol, ctx.device)
        U.fill_(np.nan)
        assert noalloc(op, F, al, paired, U) == 0
        Ue = op.apply(F, al, paired=paired)
        torch.cuda.synchronize()
        assert torch.equal(U, Ue)
    # a second, smaller operator on the same device
    small = inputs.q1_rectangle(12, 9)
    op2 = Operator.assemble(ctx, small)
    op2.eigensolve("fp64")
    F = colmajor(inputs.polynomial_forcings(small, 5, tag=95), ctx.device)
    al = np.array([0.0, 0.7, 2.0])
    U = empty_colmajor(op2.n, 15, ctx.device)
    assert noalloc(op2, F, al, False, U) == 0
    Ue = op2.apply(F, al)
    torch.cuda.synchronize()
    assert torch.equal(U, Ue)
    op.close()
    op2.close()


def test_noalloc_refuses_oversize_and_bad_arguments(ctx):
    from paper_1911_11906_amd import _lib
    from paper_1911_11906_amd.api import Operator, colmajor, empty_colmajor
    mesh = inputs.q1_rectangle(40, 40)
    op = Operator.assemble(ctx, mesh)
    op.eigensolve("fp64")
    n = op.n
    # (2 nf + na) n doubles must fit in 64 MiB: nf = 2700 at n = 1600 does not
    nf = 2700
    F = colmajor(np.ones((n, nf)), ctx.device)
    U = empty_colmajor(n, nf, ctx.device)
    assert noalloc(op, F, [1.0], False, U) == _lib.FL_EINVAL
    assert "limit" in _lib.load().fl_last_error(ctx.ptr).decode()
    assert noalloc(op, F[:, :4], [2.5], False, U) == _lib.FL_EINVAL
    fresh = Operator.assemble(ctx, mesh)
    assert noalloc(fresh, F[:, :4], [1.0], False, U) == _lib.FL_ESTATE
    op.close()
    fresh.close()
