"""Pins of the oracle's certificate and library-eigensolver steps (CPU).

* Weinstein's residual bound and the Kato-Temple refinement must contain the
  exact discrete eigenvalues of bilinear elements on a rectangle (closed
  form), for exact and for deliberately perturbed eigenvectors, and must be
  small for accurate ones (accuracy certificate of the eigenpairs; equation
  discrete_laplace, orthonormality of Section "Post-processing").
* The library eigensolver step gives the same eigenvalues and the same
  solutions v = sum theta^(-alpha/2) <f, phi> phi (Section "Method") as the
  cyclic-Jacobi oracle on a P1 polygon mesh.
* The stored reference of the n = 16384 P1 workload belongs to the mesh the
  generator produces, and its eigenvalues are certified far below the
  1e-12 target.
"""
import glob
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import certify
from oracle.closed_form import Q1Rectangle
from paper_1911_11906_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
# rounding of a Rayleigh quotient evaluated in FP64 (and of the closed form):
# a few tens of units in the last place, outside what the bounds cover
ROUND = 64 * np.finfo(float).eps


@pytest.fixture(scope="module")
def rect(oracle_mod):
    # aspect ratio 0.618: no two closed-form eigenvalues coincide
    mx, my, ly = 14, 9, 0.6180339887
    m = inputs.q1_rectangle(mx, my, ly=ly)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    exact = Q1Rectangle(mx, my, 1.0, ly).eigenvalues()
    return sp.csr_matrix(K), sp.csr_matrix(M), th, V, exact


def test_weinstein_contains_exact_and_is_tight(rect):
    Ks, Ms, th, V, exact = rect
    rq = certify.rayleigh_quotients(Ks, Ms, V)
    eta = certify.weinstein_bounds(Ks, Ms, rq, V)
    err = np.abs(rq - exact)
    assert np.all(err <= eta + ROUND * exact)
    assert np.max(eta / rq) < 1e-12
    kt = certify.kato_temple_bounds(rq, eta)
    assert np.all(np.isfinite(kt)) and np.all(kt <= eta)
    assert np.all(err <= kt + ROUND * exact)


def test_bounds_hold_for_perturbed_vectors(rect):
    Ks, Ms, th, V, exact = rect
    rng = np.random.default_rng(5)
    X = V + 1e-5 * rng.standard_normal(V.shape) * np.abs(V).max()
    rq = certify.rayleigh_quotients(Ks, Ms, X)
    order = np.argsort(rq)
    rq, X = rq[order], X[:, order]
    eta = certify.weinstein_bounds(Ks, Ms, rq, X)
    err = np.abs(rq - exact)
    assert np.all(err <= eta + ROUND * exact)
    # the radius is first order in the perturbation, not vacuous
    assert np.max(eta / rq) < 1e-2
    kt = certify.kato_temple_bounds(rq, eta)
    assert np.all(err <= kt * (1 + 1e-9) + ROUND * exact)


def test_weinstein_radius_of_shifted_values(rect):
    """For an exact eigenvector v and a wrong value t, K v - t M v =
    (lambda - t) M v, whose M^-1 norm over ||v||_M is exactly |lambda - t|: the
    radius equals the error.  The same residual measured in the M norm (a
    plausible slip) is far smaller and would not contain the eigenvalue."""
    Ks, Ms, th, V, exact = rect
    t = exact * (1 + 1e-7)
    eta = certify.weinstein_bounds(Ks, Ms, t, V)
    err = np.abs(t - exact)
    assert np.all(eta >= err * (1 - 1e-6)) and np.all(eta <= err * (1 + 1e-6))
    R = Ks @ V - (Ms @ V) * t[None, :]
    rM = np.sqrt(np.einsum("ij,ij->j", R, Ms @ R) / np.einsum("ij,ij->j", V, Ms @ V))
    assert np.all(rM < 0.5 * err)


def test_lapack_step_matches_jacobi_on_p1(oracle_mod):
    m = inputs.p1_polygon_with_holes(900, seed=11)
    K, M = oracle_mod.assemble(m)
    th_j, V_j = oracle_mod.eigensolve(K, M)
    th_l, V_l = certify.eigensolve_lapack(K, M)
    Ks, Ms = sp.csr_matrix(K), sp.csr_matrix(M)
    rq_j = certify.rayleigh_quotients(Ks, Ms, V_j)
    rq_l = certify.rayleigh_quotients(Ks, Ms, V_l)
    assert np.max(np.abs(np.sort(rq_l) - np.sort(rq_j)) / np.sort(rq_j)) < 1e-12
    assert np.abs(V_l.T @ M @ V_l - np.eye(m.n_dof)).max() < 1e-12
    F = inputs.polynomial_forcings(m, 3, tag=17)
    al = np.array([0.37, 1.0, 1.81])
    Uj = oracle_mod.apply_fractional(rq_j, V_j, M, F, al)
    Ul = oracle_mod.apply_fractional(rq_l, V_l, M, F, al)
    D = Ul - Uj
    rel = np.sqrt(np.einsum("ij,ij->j", D, M @ D) / np.einsum("ij,ij->j", Uj, M @ Uj))
    assert rel.max() < 1e-12


def test_c3_reference_file_is_certified(oracle_mod):
    paths = glob.glob(os.path.join(HERE, "golden", "c3_*.npz"))
    assert len(paths) == 1
    d = np.load(paths[0], allow_pickle=False)
    mesh = inputs.p1_polygon_with_holes(16384)
    assert str(d["sha256"]) == mesh.sha256()
    assert os.path.basename(paths[0]) == f"c3_{mesh.sha256()[:16]}.npz"
    th, eta = d["theta"], d["eta"]
    assert th.size == mesh.n_dof == 16384 and np.all(np.diff(th) > 0)
    kt = certify.kato_temple_bounds(th, eta)
    assert np.max(kt / th) < 1e-14
    for s, c in zip(d["shifts"], d["counts"]):
        assert c == np.searchsorted(th, s)
    assert np.array_equal(d["alpha"], inputs.alphas_uniform(3, tag=3))
    assert d["U"].shape == (16384, 4 * 3) and np.all(np.isfinite(d["U"]))
