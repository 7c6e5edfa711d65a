"""Eigenpairs of the pencil at sizes where cyclic Jacobi is out of reach, and
residual certificates for any computed eigenpairs.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by the tests and by
the committed script that writes the stored P1 reference under
``tests/golden/``; never by the product package, and no code is shared with it.

* ``eigensolve_lapack``: all pairs K phi = theta M phi with phi^T M phi = I
  (equation discrete_laplace; M-orthonormality from Section "Post-processing")
  by a library generalized symmetric eigensolver (LAPACK's divide-and-conquer
  driver through scipy) used as a single step.  At n = 16384 the plain Jacobi
  of ``fl_oracle.c`` would stream both n x n arrays once per rotation step,
  ~10 sweeps x 16383 steps x 8 GB, which is days on a host; the library
  routine is the same definition reached by another published algorithm.
* ``rayleigh_quotients``: theta_k = v_k^T K v_k / v_k^T M v_k with the sparse
  K and M.  For an approximate eigenvector its error is second order in the
  vector's error, so it is a more accurate eigenvalue than the solver's own
  value, whose error is normwise (eps * ||M^-1 K||).
* ``weinstein_bounds``: for any vector v and number t there is an eigenvalue
  of the pencil within ||K v - t M v||_{M^-1} / ||v||_M of t (Weinstein's
  residual bound, written for the pencil through the M-inner product; see
  Parlett, The Symmetric Eigenvalue Problem).  This certifies each computed
  eigenvalue independently of how the vector was obtained (the accuracy
  certificate of the eigenpairs).
"""
from __future__ import annotations

import numpy as np


def eigensolve_lapack(K: np.ndarray, M: np.ndarray):
    """theta ascending and V (n x n) with V^T M V = I, by scipy/LAPACK
    (``driver="gvd"``)."""
    import scipy.linalg as sl
    theta, V = sl.eigh(K, M, driver="gvd", check_finite=True)
    return theta, np.asfortranarray(V)


def _csr(A):
    import scipy.sparse as sp
    return A if sp.issparse(A) else sp.csr_matrix(A)


def rayleigh_quotients(K, M, V: np.ndarray, block: int = 1024) -> np.ndarray:
    """theta_k = v_k^T K v_k / v_k^T M v_k for every column of V (K, M dense or
    sparse; the products are taken with the sparse matrices)."""
    Ks, Ms = _csr(K), _csr(M)
    n, m = V.shape
    out = np.empty(m)
    for c0 in range(0, m, block):
        X = np.asarray(V[:, c0:c0 + block])
        out[c0:c0 + X.shape[1]] = np.einsum("ij,ij->j", X, Ks @ X) / np.einsum("ij,ij->j", X, Ms @ X)
    return out


def weinstein_bounds(K, M, theta: np.ndarray, V: np.ndarray, block: int = 1024) -> np.ndarray:
    """eta_k = ||K v_k - theta_k M v_k||_{M^-1} / ||v_k||_M for every column:
    some eigenvalue of (K, M) lies in [theta_k - eta_k, theta_k + eta_k].
    The M^-1 norm uses a sparse LU factorisation of M (a library step)."""
    import scipy.sparse.linalg as spl
    Ks, Ms = _csr(K), _csr(M)
    lu = spl.splu(Ms.tocsc())
    n, m = V.shape
    out = np.empty(m)
    for c0 in range(0, m, block):
        X = np.asarray(V[:, c0:c0 + block])
        t = theta[c0:c0 + X.shape[1]]
        MX = Ms @ X
        R = Ks @ X - MX * t[None, :]
        Z = lu.solve(np.asfortranarray(R))
        rn = np.sqrt(np.maximum(np.einsum("ij,ij->j", R, Z), 0.0))
        vn = np.sqrt(np.einsum("ij,ij->j", X, MX))
        out[c0:c0 + X.shape[1]] = rn / vn
    return out


def kato_temple_bounds(theta: np.ndarray, eta: np.ndarray) -> np.ndarray:
    """Bounds on |theta_k - lambda_k| for Rayleigh quotients theta (ascending)
    with Weinstein radii eta; where the conditions below do not hold, the
    Weinstein radius eta_k itself.

    When the n intervals [theta_k - eta_k, theta_k + eta_k] are pairwise
    disjoint, each holds at least one of the n eigenvalues (Weinstein), hence
    exactly one, in order.  Then (a, b) = (theta_{k-1} + eta_{k-1},
    theta_{k+1} - eta_{k+1}) holds only lambda_k, and the Kato-Temple
    inequality gives theta_k - eta_k^2 / (b - theta_k) <= lambda_k <=
    theta_k + eta_k^2 / (theta_k - a).  At the ends of the spectrum one side
    needs no bound: every Rayleigh quotient lies in [lambda_1, lambda_n]."""
    theta = np.asarray(theta, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    n = theta.size
    if n == 0:
        return eta.copy()
    lo, hi = theta - eta, theta + eta
    if n > 1 and not np.all(hi[:-1] < lo[1:]):
        return eta.copy()
    a = np.r_[-np.inf, hi[:-1]]
    b = np.r_[lo[1:], np.inf]
    with np.errstate(divide="ignore"):
        up = np.where(np.isfinite(a), eta ** 2 / (theta - a), 0.0)
        dn = np.where(np.isfinite(b), eta ** 2 / (b - theta), 0.0)
    return np.minimum(np.maximum(up, dn), eta)
