"""Pins of the oracle's tensor-product elements of order p = 2..8 (the order
sweep of Section "Accuracy"; CPU only).

* One-dimensional check: the order-2 element matrices on an interval are
  the textbook quadratic-element matrices (1/(3h)) [[7,-8,1],[-8,16,-8],
  [1,-8,7]] and (h/30) [[4,2,-1],[2,16,2],[-1,2,4]]; in 2-D the order-2
  element is their tensor product.
* Partition of unity: the full mass matrix sums to the area and the
  Neumann stiffness annihilates constants, for every order.
* Conforming Galerkin eigenvalues lie above the continuum ones
  pi^2 (j^2 + l^2) (min-max), and the error of the lowest one falls
  exponentially with the order.
* The eigenfunction forcing of equations poisson_f / poisson_u: the error of
  v against the continuum solution falls by orders of magnitude from p = 2
  to p = 8 on a 2 x 2 element mesh.
"""
import numpy as np
import pytest

from paper_1911_11906_amd import inputs


def test_gll_points():
    for p in range(2, 9):
        g = inputs.gll_points(p)
        assert g.size == p + 1 and g[0] == -1 and g[-1] == 1 and np.all(np.diff(g) > 0)
        assert np.allclose(g, -g[::-1], atol=1e-15)
    assert np.allclose(inputs.gll_points(2), [-1, 0, 1])
    assert np.allclose(inputs.gll_points(3), [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1])


def test_order2_element_is_textbook_tensor_product(oracle_mod):
    hx, hy = 0.5, 0.25
    m = inputs.qp_rectangle(1, 1, 2, lx=hx, ly=hy)
    _, _, Kf, Mf = oracle_mod.assemble(m, full=True)
    k = lambda h: np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * h)
    mm = lambda h: np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) * h / 30
    Ke = np.kron(mm(hy), k(hx)) + np.kron(k(hy), mm(hx))   # local index a + 3 b, a along x
    Me = np.kron(mm(hy), mm(hx))
    assert np.abs(Kf - Ke).max() < 1e-13 * np.abs(Ke).max()
    assert np.abs(Mf - Me).max() < 1e-14 * np.abs(Me).max()


@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_partition_of_unity(oracle_mod, p):
    m = inputs.qp_rectangle(2, 3, p, lx=1.3, ly=0.7)
    _, _, Kf, Mf = oracle_mod.assemble(m, full=True)
    assert Mf.sum() == pytest.approx(1.3 * 0.7, rel=1e-13)
    assert np.abs(Kf.sum(axis=1)).max() < 1e-11 * np.abs(Kf).max()
    assert np.abs(Kf - Kf.T).max() < 1e-12 * np.abs(Kf).max()


def test_spectra_bound_the_continuum_and_converge(oracle_mod):
    import scipy.linalg as sl
    lam = np.sort([np.pi ** 2 * (a * a + b * b) for a in range(1, 60) for b in range(1, 60)])
    errs = []
    for p in range(2, 9):
        m = inputs.qp_rectangle(2, 2, p)
        K, M = oracle_mod.assemble(m)
        th = sl.eigh(K, M, eigvals_only=True)
        assert np.all(th >= lam[:th.size] * (1 - 1e-12))
        errs.append(th[0] / (2 * np.pi ** 2) - 1)
    errs = np.array(errs)
    assert np.all(np.diff(np.log10(errs[:5])) < -0.9)   # at least a factor ~8 per order up to p = 6
    assert errs[-1] < 1e-11


def test_eigenfunction_forcing_converges_with_order(oracle_mod):
    al = 1.0
    err = []
    for p in (2, 4, 6, 8):
        m = inputs.qp_rectangle(2, 2, p)
        K, M = oracle_mod.assemble(m)
        th, V = oracle_mod.eigensolve(K, M)
        f = inputs.sine_mode(m)
        u = oracle_mod.apply_fractional(th, V, M, f, [al])[:, 0]
        exact = (2 * np.pi ** 2) ** (-al / 2) * f[:, 0]
        err.append(np.abs(u - exact).max() / np.abs(exact).max())
    assert err[0] > 1e2 * err[1] > 1e4 * err[2] or err[2] < 1e-9
    assert err[-1] < 1e-9
