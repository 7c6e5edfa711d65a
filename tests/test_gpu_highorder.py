"""Tensor-product elements of order p = 2..8 on the GPU (the order sweep of
Section "Accuracy"; marker: gpu).

* Assembly of every order against the oracle's (2-D Gauss quadrature of the
  products of the basis functions, written independently).
* The order sweep of the accuracy experiment: on 2 x 2 elements of order
  p = 2..8, the GPU eigensolve and the solutions v for the eigenfunction
  forcing of equations poisson_f / poisson_u at the paper's 11 orders agree
  with the oracle (Jacobi), and their error against the continuum solution
  falls by orders of magnitude with p (below 1e-9 at p = 8).
* A larger mesh (16 x 16 elements of order 4, n = 3969) in both precisions
  against the oracle's library-eigensolver step: every eigenvalue to
  1e-12, solutions to 1e-10.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

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


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_assembly_matches_oracle(ctx, oracle_mod, p):
    note("assemble order", p)
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.qp_rectangle(3, 2, p, lx=1.2, ly=0.7)
    op = Operator.assemble(ctx, mesh)
    K, M = op.matrices()
    Ko, Mo = oracle_mod.assemble(mesh)
    assert op.n == mesh.n_dof
    assert np.abs(K.cpu().numpy() - Ko).max() <= 1e-12 * np.abs(Ko).max()
    assert np.abs(M.cpu().numpy() - Mo).max() <= 1e-13 * np.abs(Mo).max()
    op.close()


def test_order_sweep_of_the_accuracy_experiment(ctx, oracle_mod):
    from paper_1911_11906_amd.api import Operator
    al = inputs.paper_alpha_sweep()
    errs = []
    for p in range(2, 9):
        note("order sweep p", p)
        mesh = inputs.qp_rectangle(2, 2, p)
        op = Operator.assemble(ctx, mesh)
        op.eigensolve("fp64")
        th, _ = op.eigenpairs(want_vectors=False)
        K, M = oracle_mod.assemble(mesh)
        tho, Vo = oracle_mod.eigensolve(K, M)
        assert np.max(np.abs(th.cpu().numpy() - tho) / tho) <= 1e-12
        f = inputs.sine_mode(mesh)
        U = op.apply(f, al).cpu().numpy()
        Uo = oracle_mod.apply_fractional(tho, Vo, M, f, al)
        assert np.abs(U - Uo).max() <= 1e-10 * np.abs(Uo).max()
        exact = np.stack([(2 * np.pi ** 2) ** (-a / 2) * f[:, 0] for a in al], 1)
        errs.append(np.abs(U - exact).max() / np.abs(exact).max())
        op.close()
    note("order sweep errors", ["%.2e" % e for e in errs])
    assert all(errs[i + 1] < 0.2 * errs[i] for i in range(len(errs) - 1))
    assert errs[-1] < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_order4_mesh_against_library_step(ctx, oracle_mod, prec):
    note("order 4, 16 x 16 elements", prec)
    from oracle import certify
    from paper_1911_11906_amd.api import Operator
    mesh = inputs.qp_rectangle(16, 16, 4)
    op = Operator.assemble(ctx, mesh)
    op.eigensolve(prec)
    th, V = op.eigenpairs()
    K, M = oracle_mod.assemble(mesh)
    thl, Vl = certify.eigensolve_lapack(K, M)
    rq = certify.rayleigh_quotients(sp.csr_matrix(K), sp.csr_matrix(M), Vl)
    order = np.argsort(rq)
    rq, Vl = rq[order], Vl[:, order]
    err = np.max(np.abs(th.cpu().numpy() - rq) / rq)
    Vg = V.cpu().numpy()
    orth = np.abs(Vg.T @ M @ Vg - np.eye(op.n)).max()
    F = inputs.polynomial_forcings(mesh, 6, tag=41)
    al = inputs.alphas_uniform(4, tag=41)
    U = op.apply(F, al).cpu().numpy()
    Uo = oracle_mod.apply_fractional(rq, Vl, M, F, al)
    D = U - Uo
    uerr = np.sqrt(np.einsum("ij,ij->j", D, M @ D) / np.einsum("ij,ij->j", Uo, M @ Uo)).max()
    note(f"order 4 {prec}: eig err {err:.2e}, orth {orth:.2e}, solution err {uerr:.2e}")
    assert err <= 1e-12 and orth <= 1e-11 and uerr <= 1e-10
    op.close()


def test_order_p_element_validation(ctx):
    from paper_1911_11906_amd.api import FraclapError, Operator
    mesh = inputs.qp_rectangle(2, 2, 3)
    bad = inputs.Mesh(mesh.elem, mesh.xy.copy(), mesh.conn[:, ::-1].copy(), mesh.dirichlet)
    with pytest.raises(FraclapError, match="tensor lattice"):
        Operator.assemble(ctx, bad)
    wrong = inputs.Mesh(10, mesh.xy, mesh.conn[:, :10].copy(), mesh.dirichlet)
    with pytest.raises(FraclapError, match="elem must be"):
        Operator.assemble(ctx, wrong)
