"""GPU parity of the building blocks against the CPU oracle (marker: gpu).

Tolerances follow from FP64 rounding: a length-k dot product errs by at most
~k eps |a||b|; factorisations by ~n eps kappa.  Every test prints its case
before touching the device.
"""
import numpy as np
import pytest

from paper_1911_11906_amd import inputs

pytestmark = pytest.mark.gpu


def note(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1911_11906_amd.api import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def to_np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (300, 257, 129), (128, 128, 16), (513, 70, 1000),
                                   (530, 64, 301), (700, 64, 600), (1100, 37, 3000)])
def test_dgemm_matches_numpy(ctx, ta, tb, m, n, k):
    note("dgemm", ta, tb, m, n, k)
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((n, k) if tb else (k, n))
    C0 = rng.standard_normal((m, n))
    from paper_1911_11906_amd.api import colmajor
    C = colmajor(C0)
    ctx.dgemm(A, B, C, ta=bool(ta), tb=bool(tb), alpha=-0.5, beta=2.0)
    ref = -0.5 * (A.T if ta else A) @ (B.T if tb else B) + 2.0 * C0
    bound = 4 * k * np.finfo(float).eps * (np.abs(A).max() * np.abs(B).max() * k + np.abs(C0).max())
    assert np.abs(to_np(C) - ref).max() <= bound


@pytest.mark.parametrize("which", ["q1", "p1"])
def test_assembly_matches_oracle(ctx, oracle_mod, which):
    note("assemble", which)
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.q1_rectangle(13, 9, lx=1.3, ly=0.7) if which == "q1" else inputs.p1_polygon_with_holes(500, seed=4)
    op = Operator.assemble(ctx, mesh)
    K, M = op.matrices()
    Ko, Mo = oracle_mod.assemble(mesh)
    assert op.n == mesh.n_dof
    assert np.abs(to_np(K) - Ko).max() <= 1e-13 * np.abs(Ko).max()
    assert np.abs(to_np(M) - Mo).max() <= 1e-13 * np.abs(Mo).max()
    assert np.array_equal(op.dof_of_node, mesh.dof_of_node())


def test_assembly_is_bitwise_reproducible(ctx):
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.p1_polygon_with_holes(800, seed=8)
    K1, M1 = Operator.assemble(ctx, mesh).matrices()
    K2, M2 = Operator.assemble(ctx, mesh).matrices()
    assert np.array_equal(to_np(K1), to_np(K2)) and np.array_equal(to_np(M1), to_np(M2))


@pytest.mark.parametrize("n", [1, 100, 128, 300, 576])
def test_potrf_matches_oracle(ctx, oracle_mod, n):
    note("potrf", n)
    if n == 576:
        _, M = oracle_mod.assemble(inputs.q1_rectangle(24, 24))
    else:
        rng = np.random.default_rng(n)
        X = rng.standard_normal((n, n))
        M = X @ X.T + n * np.eye(n)
    L = to_np(ctx.dpotrf(M))
    Lo = oracle_mod.cholesky(M)
    assert np.abs(L - np.tril(Lo)).max() <= 1e-13 * np.abs(Lo).max()


def test_potrf_reports_pivot(ctx):
    from paper_1911_11906_amd._lib import FraclapError
    A = np.eye(200)
    A[150, 150] = -1.0
    with pytest.raises(FraclapError, match="pivot 151"):
        ctx.dpotrf(A)


@pytest.mark.parametrize("mesh_name", ["q1_24", "p1_300"])
def test_sygst_matches_oracle(ctx, oracle_mod, mesh_name):
    note("sygst", mesh_name)
    mesh = inputs.q1_rectangle(24, 24) if mesh_name == "q1_24" else inputs.p1_polygon_with_holes(300, seed=1)
    K, M = oracle_mod.assemble(mesh)
    Lo = oracle_mod.cholesky(M)
    Co = oracle_mod.standard_form(Lo, K)
    L = ctx.dpotrf(M)
    C = to_np(ctx.dsygst(L, K))
    assert np.abs(C - Co).max() <= 1e-12 * np.abs(Co).max()
    assert np.array_equal(C, C.T)


@pytest.fixture(scope="module")
def c1_oracle(oracle_mod):
    mesh = inputs.q1_rectangle(24, 24)
    K, M = oracle_mod.assemble(mesh)
    th, V = oracle_mod.eigensolve(K, M)
    return mesh, K, M, th, V


def test_apply_with_oracle_basis(ctx, oracle_mod, c1_oracle):
    note("apply c1 with oracle basis")
    from paper_1911_11906_amd.api import Operator
    mesh, K, M, th, V = c1_oracle
    op = Operator.assemble(ctx, mesh)
    op.set_eigenpairs(th, V)
    F = np.concatenate([inputs.sine_mode(mesh), inputs.polynomial_forcings(mesh, 4, tag=1)], axis=1)
    al = np.array([0.0, 0.5, 1.0, 1.5, 2.0])
    U = to_np(op.apply(F, al))
    Uo = oracle_mod.apply_fractional(th, V, M, F, al)
    assert U.shape == Uo.shape
    assert np.abs(U - Uo).max() <= 1e-12 * np.abs(Uo).max()
    # alpha = 0 reproduces f; eigenfunction forcing gives theta_11^(-alpha/2) f
    assert np.abs(U[:, 0] - F[:, 0]).max() < 1e-12
    th11 = th[0]
    for i, a in enumerate(al):
        assert np.abs(U[:, i * 5] - th11 ** (-a / 2) * F[:, 0]).max() < 5e-13
    Up = to_np(op.apply(F, al, paired=True))
    for b in range(5):
        assert np.abs(Up[:, b] - Uo[:, b + 5 * b]).max() <= 1e-12 * np.abs(Uo).max()


def test_grad_with_oracle_basis(ctx, oracle_mod, c1_oracle):
    note("grad c1 with oracle basis")
    from paper_1911_11906_amd.api import Operator
    mesh, K, M, th, V = c1_oracle
    op = Operator.assemble(ctx, mesh)
    op.set_eigenpairs(th, V)
    F = inputs.polynomial_forcings(mesh, 6, tag=11)
    al = inputs.alphas_uniform(6, tag=11)
    GU = np.random.default_rng(2).standard_normal(F.shape)
    GF, ga = op.grad(F, al, GU)
    GFo, gao = oracle_mod.grad_apply(th, V, M, F, al, GU)
    assert np.abs(to_np(GF) - GFo).max() <= 1e-12 * np.abs(GFo).max()
    assert np.abs(ga.numpy() - gao).max() <= 1e-11 * np.abs(gao).max()


def test_error_paths(ctx, c1_oracle):
    from paper_1911_11906_amd.api import Operator
    from paper_1911_11906_amd._lib import FraclapError, FL_ESTATE, FL_EINVAL
    mesh = c1_oracle[0]
    op = Operator.assemble(ctx, mesh)
    F = inputs.sine_mode(mesh)
    with pytest.raises(FraclapError) as e:
        op.apply(F, [1.0])
    assert e.value.status == FL_ESTATE
    op.set_eigenpairs(c1_oracle[3], c1_oracle[4])
    with pytest.raises(FraclapError) as e:
        op.apply(F, [2.5])
    assert e.value.status == FL_EINVAL
    bad = inputs.q1_rectangle(4, 4)
    bad.conn = bad.conn[:, ::-1].copy()  # clockwise
    with pytest.raises(FraclapError) as e:
        Operator.assemble(ctx, bad)
    assert e.value.status == FL_EINVAL


def test_apply_uniform_tile_path(ctx, oracle_mod, c1_oracle):
    """nf a multiple of 128: every GEMM tile shares one alpha (the weight is
    applied once per k-row); same answer as the oracle."""
    note("apply nf=256 uniform-tile path")
    from paper_1911_11906_amd.api import Operator
    mesh, K, M, th, V = c1_oracle
    op = Operator.assemble(ctx, mesh)
    op.set_eigenpairs(th, V)
    F = inputs.polynomial_forcings(mesh, 256, tag=31)
    al = np.array([0.0, 0.8, 2.0])
    U = to_np(op.apply(F, al))
    Uo = oracle_mod.apply_fractional(th, V, M, F, al)
    assert np.abs(U - Uo).max() <= 1e-12 * np.abs(Uo).max()
    assert np.abs(U[:, :256] - F).max() <= 2e-12 * np.abs(F).max()


@pytest.mark.parametrize("nf,na", [(256, 4), (100, 10)])
def test_apply_grouped_tile_grid(ctx, oracle_mod, c1_oracle, nf, na):
    """Tile grids of 5 x 8 (n = 576 rows, 1024 or 1000 columns): the tile
    count is a multiple of 8, so the XCD-aware order splits it into eighths,
    and the band of 8 row tiles is cut to 5.  Both the uniform-alpha tiles
    (nf = 256) and the per-column weights (nf = 100) match the oracle."""
    note(f"apply grouped tile grid nf={nf} na={na}")
    from paper_1911_11906_amd.api import Operator
    mesh, K, M, th, V = c1_oracle
    op = Operator.assemble(ctx, mesh)
    op.set_eigenpairs(th, V)
    F = inputs.polynomial_forcings(mesh, nf, tag=41)
    al = np.linspace(0.0, 2.0, na)
    U = to_np(op.apply(F, al))
    Uo = oracle_mod.apply_fractional(th, V, M, F, al)
    assert U.shape == Uo.shape == (576, nf * na)
    assert np.abs(U - Uo).max() <= 1e-12 * np.abs(Uo).max()
    assert np.abs(U[:, :nf] - F).max() <= 2e-12 * np.abs(F).max()
