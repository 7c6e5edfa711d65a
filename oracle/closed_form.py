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

    def _coeffs(self, F: np.ndarray) -> np.ndarray:
        """c[f, ky, jx] = phi_(jx,ky)^T M f for every column f of F (mu-weighted
        separable sine transform: (Mx N)_j = mu_j N_j)."""
        nf = F.shape[1]
        G = F.T.reshape(nf, self.my, self.mx)                # [f, y, x]
        Ax = self.Nx * self.mux[None, :]
        Ay = self.Ny * self.muy[None, :]
        return np.einsum("yk,fyx,xj->fkj", Ay, G, Ax, optimize=True)

    def _proj(self, G: np.ndarray) -> np.ndarray:
        """p[f, ky, jx] = phi_(jx,ky)^T g (no mass matrix) for columns g of G."""
        nf = G.shape[1]
        return np.einsum("yk,fyx,xj->fkj", self.Ny, G.T.reshape(nf, self.my, self.mx), self.Nx, optimize=True)

    def _synth(self, C: np.ndarray, mass: bool = False) -> np.ndarray:
        """sum_k C[f, k] phi_k (times M when mass) as an n x nf array."""
        Nx = self.Nx * self.mux[None, :] if mass else self.Nx
        Ny = self.Ny * self.muy[None, :] if mass else self.Ny
        U = np.einsum("yk,fkj,xj->fyx", Ny, C, Nx, optimize=True)
        return U.reshape(C.shape[0], self.n).T

    def weights(self, alpha: float, mu_t=None) -> np.ndarray:
        """W[k, j]: theta^(-alpha/2) (Poisson) or, given mu_t = mu t,
        exp(-mu t theta^(alpha/2)) (diffusion, equation diffusion_solution)."""
        th = self.theta_grid()
        if mu_t is None:
            return np.exp(-0.5 * alpha * np.log(th)) if alpha != 0.0 else np.ones_like(th)
        return np.exp(-mu_t * np.exp(0.5 * alpha * np.log(th)))

    def apply(self, F: np.ndarray, alpha, mu_t=None) -> np.ndarray:
        """u = sum_k w_k (phi_k^T M f) phi_k for every column of F and every
        alpha (w = theta^(-alpha/2), or exp(-mu_t theta^(alpha/2)) with mu_t
        given, one per alpha): returns n x (nf * na), column j + i*nf.

        Uses the separable transform: phi^T M f = (Nx (x) Ny)^T (Mx (x) My) f and
        (Mx N)_j = mu_j N_j, so coefficients are mu-weighted sine transforms."""
        F = np.atleast_2d(np.asarray(F, dtype=np.float64).T).T
        n, nf = F.shape
        alphas = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
        mts = None if mu_t is None else np.broadcast_to(np.asarray(mu_t, dtype=np.float64), alphas.shape)
        C = self._coeffs(F)
        out = np.empty((n, nf * alphas.size))
        for i, a in enumerate(alphas):
            W = self.weights(a, None if mts is None else mts[i])
            out[:, i * nf:(i + 1) * nf] = self._synth(C * W[None])
        return out

    def grad(self, F: np.ndarray, alpha, GU: np.ndarray, mu_t=None):
        """Adjoint of the paired map u_b = sum_k w_kb (phi_k^T M f_b) phi_k:
        given GU = dL/dU (n x nb) returns (GF, galpha, gs) with GF = M V (w o p),
        p = V^T GU, galpha_b = sum_k p c dw/dalpha, gs_b = sum_k p c dw/d(mu t)
        (gs is None for the Poisson weights)."""
        F = np.asarray(F, dtype=np.float64)
        GU = np.asarray(GU, dtype=np.float64)
        alphas = np.asarray(alpha, dtype=np.float64)
        nb = F.shape[1]
        C = self._coeffs(F)
        P = self._proj(GU)
        lt = np.log(self.theta_grid())
        W = np.empty_like(C)
        ga = np.empty(nb)
        gs = None if mu_t is None else np.empty(nb)
        mts = None if mu_t is None else np.broadcast_to(np.asarray(mu_t, dtype=np.float64), alphas.shape)
        for b in range(nb):
            w = self.weights(alphas[b], None if mts is None else mts[b])
            W[b] = w
            q = P[b] * C[b] * w
            if mts is None:
                ga[b] = np.sum(q * (-0.5 * lt))
            else:
                e = np.exp(0.5 * alphas[b] * lt)
                ga[b] = np.sum(q * (-0.5 * mts[b] * e * lt))
                gs[b] = np.sum(q * (-e))
        GF = self._synth(W * P, mass=True)
        return GF, ga, gs
