"""CPU oracle for the fractional Poisson eigen-expansion path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.  It shares
no code with the GPU library.

``liboracle.so`` (plain C, OpenMP, FP64; source ``fl_oracle.c``) does the
finite-element assembly, the Cholesky / standard-form / cyclic-Jacobi
eigensolve, the spectral application and its adjoint.  ``closed_form`` holds
the exact discrete spectrum of bilinear elements on rectangles.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "fl_oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile fl_oracle.c with gcc (-O2 -fopenmp); returns the .so path."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.or_assemble.argtypes = [ctypes.c_int, i64, P, i64, P, P, i64, P, P, P, P]
        L.or_assemble.restype = ctypes.c_int
        L.or_cholesky.argtypes = [i64, P]
        L.or_cholesky.restype = ctypes.c_int
        L.or_standard_form.argtypes = [i64, P, P, P]
        L.or_solve_lt.argtypes = [i64, P, i64, P]
        L.or_jacobi.argtypes = [i64, P, P, ctypes.c_int]
        L.or_jacobi.restype = ctypes.c_int
        L.or_eigensolve.argtypes = [i64, P, P, P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.or_eigensolve.restype = ctypes.c_int
        L.or_apply.argtypes = [i64, P, P, P, i64, P, i64, P, P]
        L.or_grad.argtypes = [i64, P, P, P, i64, P, P, P, P, P]
        L.or_apply_diffusion.argtypes = [i64, P, P, P, i64, P, i64, P, P, P, P]
        L.or_grad_diffusion.argtypes = [i64, P, P, P, i64, P, P, P, P, P, P, P, P, P]
        L.or_inertia_negative.argtypes = [i64, P]
        L.or_inertia_negative.restype = i64
        L.or_inertia_negative_band.argtypes = [i64, i64, P]
        L.or_inertia_negative_band.restype = i64
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().or_num_threads())


def assemble(mesh, full: bool = False):
    """Dense K, M over interior DOFs (Fortran order).  With ``full`` also the
    un-eliminated matrices over all nodes."""
    xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
    conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
    dof = np.ascontiguousarray(mesh.dof_of_node(), dtype=np.int64)
    n = mesh.n_dof
    K = np.zeros((n, n), order="F")
    M = np.zeros((n, n), order="F")
    Kf = Mf = None
    if full:
        Kf = np.zeros((mesh.n_nodes, mesh.n_nodes), order="F")
        Mf = np.zeros((mesh.n_nodes, mesh.n_nodes), order="F")
    rc = lib().or_assemble(mesh.elem, mesh.n_nodes, _p(xy), mesh.n_elem, _p(conn), _p(dof), n,
                           _p(K), _p(M), _p(Kf) if full else None, _p(Mf) if full else None)
    if rc:
        raise ValueError(f"degenerate element {-rc - 1}")
    return (K, M, Kf, Mf) if full else (K, M)


def cholesky(M: np.ndarray) -> np.ndarray:
    L = np.array(M, order="F", dtype=np.float64, copy=True)
    rc = lib().or_cholesky(L.shape[0], _p(L))
    if rc:
        raise np.linalg.LinAlgError(f"matrix not positive definite at pivot {rc}")
    return L


def standard_form(L: np.ndarray, K: np.ndarray) -> np.ndarray:
    n = L.shape[0]
    C = np.zeros((n, n), order="F")
    lib().or_standard_form(n, _p(np.asfortranarray(L)), _p(np.asfortranarray(K)), _p(C))
    return C


def jacobi(C: np.ndarray, max_sweeps: int = 40):
    """Returns (diag, Q, sweeps) with C = Q diag Q^T (unsorted)."""
    A = np.array(C, order="F", dtype=np.float64, copy=True)
    Q = np.zeros_like(A, order="F")
    sw = lib().or_jacobi(A.shape[0], _p(A), _p(Q), max_sweeps)
    return np.diag(A).copy(), Q, sw


def eigensolve(K: np.ndarray, M: np.ndarray, max_sweeps: int = 40):
    """All generalized eigenpairs: theta ascending, V M-orthonormal."""
    K = np.asfortranarray(K, dtype=np.float64)
    M = np.asfortranarray(M, dtype=np.float64)
    n = K.shape[0]
    theta = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sw = ctypes.c_int(0)
    rc = lib().or_eigensolve(n, _p(K), _p(M), _p(theta), _p(V), max_sweeps, ctypes.byref(sw))
    if rc > 0:
        raise np.linalg.LinAlgError(f"M not positive definite at pivot {rc}")
    if rc < 0:
        raise RuntimeError("Jacobi did not converge")
    return theta, V


def apply_fractional(theta, V, M, F, alpha):
    """U[:, j + i*nf] = v(alpha_i, f_j)."""
    F = np.asfortranarray(np.atleast_2d(F.T).T, dtype=np.float64)
    n, nf = F.shape
    alpha = np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64)
    U = np.zeros((n, nf * alpha.size), order="F")
    lib().or_apply(n, _p(np.ascontiguousarray(theta, dtype=np.float64)), _p(np.asfortranarray(V)),
                   _p(np.asfortranarray(M)), nf, _p(F), alpha.size, _p(alpha), _p(U))
    return U


def grad_apply(theta, V, M, F, alpha, GU):
    """Adjoint of the paired map (f_b, alpha_b) -> u_b: returns (GF, galpha)."""
    F = np.asfortranarray(F, dtype=np.float64)
    GU = np.asfortranarray(GU, dtype=np.float64)
    n, nb = F.shape
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    GF = np.zeros((n, nb), order="F")
    ga = np.zeros(nb)
    lib().or_grad(n, _p(np.ascontiguousarray(theta, dtype=np.float64)), _p(np.asfortranarray(V)),
                  _p(np.asfortranarray(M)), nb, _p(F), _p(alpha), _p(GU), _p(GF), _p(ga))
    return GF, ga


def apply_diffusion(theta, V, M, U0, alpha, t, mu):
    """U[:, j + i*nf] = u(t_i; alpha_i, mu_i, u0_j) of the fractional
    diffusion equation (alpha, t, mu: one value each per i)."""
    U0 = np.asfortranarray(np.atleast_2d(U0.T).T, dtype=np.float64)
    n, nf = U0.shape
    alpha = np.ascontiguousarray(np.atleast_1d(alpha), dtype=np.float64)
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), alpha.shape))
    mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), alpha.shape))
    U = np.zeros((n, nf * alpha.size), order="F")
    lib().or_apply_diffusion(n, _p(np.ascontiguousarray(theta, dtype=np.float64)), _p(np.asfortranarray(V)),
                             _p(np.asfortranarray(M)), nf, _p(U0), alpha.size, _p(alpha), _p(t), _p(mu), _p(U))
    return U


def grad_diffusion(theta, V, M, U0, alpha, t, mu, GU):
    """Adjoint of the paired diffusion map: returns (GU0, galpha, gt, gmu)."""
    U0 = np.asfortranarray(U0, dtype=np.float64)
    GU = np.asfortranarray(GU, dtype=np.float64)
    n, nb = U0.shape
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), alpha.shape))
    mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), alpha.shape))
    GU0 = np.zeros((n, nb), order="F")
    ga, gt, gm = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    lib().or_grad_diffusion(n, _p(np.ascontiguousarray(theta, dtype=np.float64)), _p(np.asfortranarray(V)),
                            _p(np.asfortranarray(M)), nb, _p(U0), _p(alpha), _p(t), _p(mu), _p(GU), _p(GU0),
                            _p(ga), _p(gt), _p(gm))
    return GU0, ga, gt, gm


def inertia_count(K, M, sigma: float) -> int:
    """# of eigenvalues of K - theta M below sigma (negative LDL^T pivots)."""
    A = np.array(K - sigma * M, order="F", dtype=np.float64, copy=True)
    r = lib().or_inertia_negative(A.shape[0], _p(A))
    if r < 0:
        raise ZeroDivisionError("zero pivot")
    return int(r)


def inertia_count_banded(K, M, sigma: float) -> int:
    """# of eigenvalues of K - theta M below sigma, for sparse K and M of any
    size: reverse Cuthill-McKee ordering (a congruence, so the inertia is
    unchanged), then the banded LDL^T count."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    A = sp.csr_matrix(K - sigma * M)
    perm = reverse_cuthill_mckee(A, symmetric_mode=True)
    A = A[perm][:, perm].tocoo()
    n = A.shape[0]
    low = A.row >= A.col
    r, c, v = A.row[low], A.col[low], A.data[low]
    bw = int((r - c).max()) if r.size else 0
    AB = np.zeros((n, bw + 1), dtype=np.float64)   # row c holds column c of the band
    AB[c, r - c] = v
    AB = np.ascontiguousarray(AB)
    res = lib().or_inertia_negative_band(n, bw, _p(AB))
    if res < 0:
        raise ZeroDivisionError("zero pivot")
    return int(res)
