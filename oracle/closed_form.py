"""Exact discrete spectrum of bilinear (Q1) elements on a rectangle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With an mx x my interior grid of spacing hx, hy and homogeneous Dirichlet
data, K = Kx (x) My + Mx (x) Ky and M = Mx (x) My, where the 1-D factors are
Kh = (1/h) tridiag(-1, 2, -1) and Mh = (h/6) tridiag(1, 4, 1).  Both are
diagonalised by the sine vectors s_j(i) = sin(i phi_j), phi_j = j pi/(m+1):
  Kh s_j = (4/h) sin^2(phi_j/2) s_j,   Mh s_j = (h/3)(2 + cos phi_j) s_j,
so the pencil (K, M) has eigenvalues theta_jk = t^x_j + t^y_k with
  t_j = (12/h^2) sin^2(phi_j/2) / (2 + cos phi_j)
and eigenvectors s^x_j (x) s^y_k whose squared M-norm is
  mu^x_j mu^y_k (mx+1)(my+1)/4,  mu_j = (h/3)(2 + cos phi_j).
This is the discrete counterpart of the Fourier-mode solutions of the paper
(Section "Method", generalized Fourier series on squares; Section
"Accuracy").  DOFs are numbered with x fastest.
"""
from __future__ import annotations

import numpy as np


def _one_d(m: int, h: float):
    j = np.arange(1, m + 1)
    phi = j * np.pi / (m + 1)
    t = (12.0 / h ** 2) * np.sin(phi / 2) ** 2 / (2.0 + np.cos(phi))
    mu = (h / 3.0) * (2.0 + np.cos(phi))
    S = np.sin(np.outer(np.arange(1, m + 1), phi))     # S[i, j] = sin(i phi_j)
    return t, mu, S


class Q1Rectangle:
    def __init__(self, mx: int, my: int, lx: float = 1.0, ly: float = 1.0):
        self.mx, self.my = mx, my
        self.hx, self.hy = lx / (mx + 1), ly / (my + 1)
        self.tx, self.mux, self.Sx = _one_d(mx, self.hx)
        self.ty, self.muy, self.Sy = _one_d(my, self.hy)
        # M-normalised 1-D factors: columns s_j / sqrt(mu_j (m+1)/2)
        self.Nx = self.Sx / np.sqrt(self.mux * (mx + 1) / 2.0)
        self.Ny = self.Sy / np.sqrt(self.muy * (my + 1) / 2.0)

    @property
    def n(self) -> int:
        return self.mx * self.my

    def eigenvalues(self) -> np.ndarray:
        """All n eigenvalues, ascending."""
        return np.sort(np.add.outer(self.ty, self.tx).ravel())

    def theta_grid(self) -> np.ndarray:
        """theta[k, j] for x-mode j and y-mode k (row-major, x fastest)."""
        return np.add.outer(self.ty, self.tx)

    def eigenvector(self, jx: int, ky: int) -> np.ndarray:
        """M-normalised eigenvector for modes (jx, ky), 1-based."""
        return np.kron(self.Ny[:, ky - 1], self.Nx[:, jx - 1])

    def apply(self, F: np.ndarray, alpha) -> np.ndarray:
        """u = sum_k theta_k^(-alpha/2) (phi_k^T M f) phi_k for every column of F
        and every alpha: returns n x (nf * na), column j + i*nf.

        Uses the separable transform: phi^T M f = (Nx (x) Ny)^T (Mx (x) My) f and
        (Mx N)_j = mu_j N_j, so coefficients are mu-weighted sine transforms."""
        F = np.atleast_2d(np.asarray(F, dtype=np.float64).T).T
        n, nf = F.shape
        alphas = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
        mx, my = self.mx, self.my
        G = F.T.reshape(nf, my, mx)                       # [f, y, x]
        # c[f, ky, jx] = sum_{y,x} (muy_k Ny[y,k]) (mux_j Nx[x,j]) G[f,y,x]
        Ax = self.Nx * self.mux[None, :]
        Ay = self.Ny * self.muy[None, :]
        C = np.einsum("yk,fyx,xj->fkj", Ay, G, Ax, optimize=True)
        th = self.theta_grid()
        out = np.empty((n, nf * alphas.size))
        for i, a in enumerate(alphas):
            W = np.exp(-0.5 * a * np.log(th)) if a != 0.0 else np.ones_like(th)
            U = np.einsum("yk,fkj,xj->fyx", self.Ny, C * W[None], self.Nx, optimize=True)
            out[:, i * nf:(i + 1) * nf] = U.reshape(nf, n).T
        return out
