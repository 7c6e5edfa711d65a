"""Eigenvalue counting on the GPU by Sylvester's law of inertia (Section
"Eigenvalue counting"; marker: gpu).  The counts are integers and must equal
exactly: the index of the shift in the exact discrete Q1 spectrum (closed
form), the oracle's banded LDL^T counts, and, at full size on the P1 polygon
mesh (n = 16384), the positions of the shifts in the stored oracle
reference spectrum.  Shifts sit midway between consecutive eigenvalues that
are at least 1e-6 apart (relative), below the spectrum and above it."""
import glob
import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle.closed_form import Q1Rectangle
from paper_1911_11906_amd import inputs

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1911_11906_amd.api import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def midpoint_shifts(th, count, seed):
    rng = np.random.default_rng(seed)
    ks = [k for k in rng.permutation(th.size - 1) if th[k + 1] - th[k] > 1e-6 * th[k + 1]][:count]
    sig = np.array([0.5 * (th[k] + th[k + 1]) for k in ks] + [0.5 * th[0], 2.0 * th[-1]])
    want = np.array([k + 1 for k in ks] + [0, th.size])
    return sig, want


@pytest.mark.parametrize("mx,my,ly", [(24, 24, 1.0), (37, 11, 0.4)])
def test_counts_match_closed_form_q1(ctx, oracle_mod, mx, my, ly):
    note("inertia q1", mx, my)
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.q1_rectangle(mx, my, ly=ly)
    op = Operator.assemble(ctx, mesh)
    th = Q1Rectangle(mx, my, 1.0, ly).eigenvalues()
    sig, want = midpoint_shifts(th, 40, mx)
    cnt, bw = op.inertia(sig)
    assert bw <= mx + 1
    assert np.array_equal(cnt, want)
    K, M = oracle_mod.assemble(mesh)
    for s, c in zip(sig[:6], cnt[:6]):
        assert oracle_mod.inertia_count_banded(K, M, s) == c
    op.close()


@pytest.mark.parametrize("which", ["p1", "lshape"])
def test_counts_match_oracle_reordered(ctx, oracle_mod, which):
    """Unstructured numbering (reverse Cuthill-McKee chosen on the device
    side) and an L-shaped domain: counts = oracle's LAPACK-spectrum index and
    the oracle's banded counts."""
    note("inertia", which)
    import scipy.linalg as sl
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.p1_polygon_with_holes(1500, seed=12) if which == "p1" else inputs.q1_lshape(17)
    op = Operator.assemble(ctx, mesh)
    K, M = oracle_mod.assemble(mesh)
    th = sl.eigh(K, M, eigvals_only=True)
    sig, want = midpoint_shifts(th, 48, 5)
    cnt, bw = op.inertia(sig)
    assert np.array_equal(cnt, want)
    for s, c in zip(sig[:5], cnt[:5]):
        assert oracle_mod.inertia_count_banded(K, M, s) == c
    op.close()


def test_counts_at_full_size_p1(ctx):
    note("inertia c3 n=16384")
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.p1_polygon_with_holes(16384)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"c3_{mesh.sha256()[:16]}.npz")
    th = np.load(path, allow_pickle=False)["theta"]
    op = Operator.assemble(ctx, mesh)
    sig, want = midpoint_shifts(th, 126, 16384)
    cnt, bw = op.inertia(sig)
    note(f"c3 bandwidth {bw}")
    assert np.array_equal(cnt, want)
    op.close()


def test_inertia_rejects_dense_pencils_and_bad_shifts(ctx):
    from paper_1911_11906_amd.api import FraclapError, Operator
    rng = np.random.default_rng(0)
    X = rng.standard_normal((600, 600))
    op = Operator.from_dense(ctx, X @ X.T + 600 * np.eye(600), np.eye(600))
    with pytest.raises(FraclapError, match="bandwidth"):
        op.inertia([1.0])
    mesh = inputs.q1_rectangle(8, 8)
    op2 = Operator.assemble(ctx, mesh)
    with pytest.raises(FraclapError, match="FL_EINVAL"):
        op2.inertia([np.inf])
    op.close()
    op2.close()
