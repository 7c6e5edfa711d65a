"""Planted mistakes in the oracle (CPU only): each mutant of fl_oracle.c
(a dropped term, a wrong sign, index or weight, a transposed operand) is
compiled into a scratch library and must fail at least one pin that does
not depend on the oracle's own code.  The unmutated source passes all."""
import contextlib
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from oracle.closed_form import Q1Rectangle
from paper_1911_11906_amd import inputs

SRC = os.path.join(os.path.dirname(oracle.__file__), "fl_oracle.c")

MUTANTS = {
    "q1_mass_index": ("Me[i * 4 + j] += det * N[i] * N[j];", "Me[i * 4 + j] += det * N[i] * N[i];"),
    "q1_stiff_drop_y": ("(dNx[i] * dNx[j] + dNy[i] * dNy[j])", "(dNx[i] * dNx[j])"),
    "p1_stiff_transposed": ("area * (gx[i] * gx[j] + gy[i] * gy[j])", "area * (gx[i] * gy[j] + gy[i] * gx[j])"),
    "p1_mass_weight": ("m += (area / 3.0) * mid[q][i] * mid[q][j];", "m += (area / 2.0) * mid[q][i] * mid[q][j];"),
    "chol_index": ("s -= A[IDX(i, k, n)] * A[IDX(j, k, n)];", "s -= A[IDX(i, k, n)] * A[IDX(k, j, n)];"),
    "stdform_transposed_L": ("for (int64_t k = 0; k < i; ++k) s -= L[IDX(i, k, n)] * w[k];",
                             "for (int64_t k = 0; k < i; ++k) s -= L[IDX(k, i, n)] * w[k];"),
    "backsub_index": ("for (int64_t k = i + 1; k < n; ++k) s -= L[IDX(k, i, n)] * x[k];",
                      "for (int64_t k = i + 1; k < n; ++k) s -= L[IDX(i, k, n)] * x[k];"),
    "jacobi_tan_sign": ("double t = (tau >= 0.0 ? 1.0 : -1.0)", "double t = (tau >= 0.0 ? -1.0 : 1.0)"),
    "jacobi_row_sign": ("xp[r2] = s2 * a1 + c2 * a2;", "xp[r2] = s2 * a1 - c2 * a2;"),
    "apply_half_dropped": ("double w = pow(theta[k], -0.5 * alpha[i]);", "double w = pow(theta[k], -alpha[i]);"),
    "apply_mass_dropped": ("for (int64_t c = 0; c < n; ++c) s += M[IDX(r, c, n)] * F[IDX(c, j, n)];",
                           "for (int64_t c = 0; c < n; ++c) s += (r == c) * F[IDX(c, j, n)];"),
    "grad_log_weight": ("ga += sp * sc * w * (-0.5 * log(theta[k]));", "ga += sp * sc * w * (-log(theta[k]));"),
    "grad_mass_dropped": ("for (int64_t q = 0; q < n; ++q) s += M[IDX(r, q, n)] * y[q];",
                          "for (int64_t q = 0; q < n; ++q) s += (r == q) * y[q];"),
    "diffusion_half_dropped": ("double w = exp(-mu[i] * pow(theta[k], 0.5 * alpha[i]) * t[i]);",
                               "double w = exp(-mu[i] * pow(theta[k], alpha[i]) * t[i]);"),
    "diffusion_sign": ("double w = exp(-mu[b] * e * t[b]);", "double w = exp(mu[b] * e * t[b]);"),
    "diffusion_grad_t_weight": ("g_t += q * (-mu[b] * e);", "g_t += q * (-t[b] * e);"),
    "diffusion_grad_alpha_half": ("ga += q * (-mu[b] * t[b] * e * 0.5 * log(theta[k]));",
                                  "ga += q * (-mu[b] * t[b] * e * log(theta[k]));"),
    "diffusion_grad_mass_dropped": ("for (int64_t q = 0; q < n; ++q) s += M[IDX(r, q, n)] * gy[q];",
                                    "for (int64_t q = 0; q < n; ++q) s += (r == q) * gy[q];"),
    "band_ldl_index": ("-= l * AB[(size_t)(r - j) + (size_t)j * ld];", "-= l * AB[(size_t)(c - j) + (size_t)j * ld];"),
}


@contextlib.contextmanager
def swapped_lib(so_path):
    saved = oracle._lib
    oracle._lib = None
    real_so = oracle._SO
    oracle._SO = so_path
    real_build = oracle.build
    oracle.build = lambda force=False: so_path
    try:
        yield
    finally:
        oracle._lib = saved
        oracle._SO = real_so
        oracle.build = real_build


def failing_pins():
    """Run small versions of the independent pins; return the names that fail."""
    bad = []

    def check(name, cond):
        if not cond:
            bad.append(name)

    with np.errstate(all="ignore"):
        try:
            m = inputs.q1_rectangle(7, 7)
            K, M = oracle.assemble(m)
            h = 1 / 8
            i = 24
            check("q1_stencil_K", abs(K[i, i] - 8 / 3) < 1e-13 and abs(K[i, i + 8] + 1 / 3) < 1e-13)
            check("q1_stencil_M", abs(M[i, i] * 36 / h ** 2 - 16) < 1e-10 and abs(M[i, i + 1] * 36 / h ** 2 - 4) < 1e-10)
            mp = inputs.p1_right_triangles(6)
            Kp, Mp = oracle.assemble(mp)
            j = 14
            check("p1_five_point", abs(Kp[j, j] - 4) < 1e-13 and abs(Kp[j, j + 7]) < 1e-13)
            check("p1_mass", abs(Mp[j, j] - (1 / 7) ** 2 / 2) < 1e-14)
            q = inputs.q1_rectangle(8, 6, lx=1.0, ly=0.8)
            Kq, Mq = oracle.assemble(q)
            th, V = oracle.eigensolve(Kq, Mq)
            ref = Q1Rectangle(8, 6, 1.0, 0.8).eigenvalues()
            check("q1_spectrum", np.all(np.isfinite(th)) and np.max(np.abs(th - ref) / ref) < 1e-12)
            check("m_orthonormal", np.abs(V.T @ Mq @ V - np.eye(48)).max() < 1e-12)
            pp = inputs.p1_polygon_with_holes(120, seed=2)
            Kr, Mr = oracle.assemble(pp)
            thr, _ = oracle.eigensolve(Kr, Mr)
            w = sl.eigh(Kr, Mr, eigvals_only=True)
            check("p1_vs_lapack", np.max(np.abs(thr - w) / w) < 1e-11)
            f = inputs.sine_mode(q, lx=1.0, ly=0.8)
            cf = Q1Rectangle(8, 6, 1.0, 0.8)
            th11 = cf.tx[0] + cf.ty[0]
            u = oracle.apply_fractional(th, V, Mq, f, [1.0])
            check("eigenfunction_forcing", np.abs(u[:, 0] - th11 ** -0.5 * f[:, 0]).max() < 1e-12)
            F = inputs.polynomial_forcings(q, 2, tag=3)
            U2 = oracle.apply_fractional(th, V, Mq, F, [2.0])
            check("alpha2_laplacian", np.abs(Kq @ U2 - Mq @ F).max() < 1e-11 * np.abs(Mq @ F).max())
            al = np.array([0.4, 1.1])
            Uo = oracle.apply_fractional(th, V, Mq, F, [0.9])

            def loss(Fx, ax):
                tot = 0.0
                for b in range(2):
                    r = oracle.apply_fractional(th, V, Mq, Fx[:, b], [ax[b]])[:, 0] - Uo[:, b]
                    tot += r @ Mq @ r
                return tot
            U = np.stack([oracle.apply_fractional(th, V, Mq, F[:, b], [al[b]])[:, 0] for b in range(2)], 1)
            GF, ga = oracle.grad_apply(th, V, Mq, F, al, 2 * Mq @ (U - Uo))
            hh = 1e-5
            fd = (loss(F, al + [hh, 0]) - loss(F, al - [hh, 0])) / (2 * hh)
            check("grad_alpha_fd", abs(ga[0] - fd) < 1e-6 * max(1.0, abs(fd)))
            D = np.random.default_rng(0).standard_normal(F.shape)
            fd = (loss(F + hh * D, al) - loss(F - hh * D, al)) / (2 * hh)
            check("grad_f_fd", abs(np.sum(GF * D) - fd) < 1e-6 * max(1.0, abs(fd)))
            # fractional diffusion: the (1,1) mode decays by exp(-mu theta_11^(alpha/2) t)
            ud = oracle.apply_diffusion(th, V, Mq, f, [1.3], [0.4], [1.0])
            check("diffusion_eigenfunction",
                  np.abs(ud[:, 0] - np.exp(-th11 ** 0.65 * 0.4) * f[:, 0]).max() < 1e-12)
            # alpha = 2: M du/dt = -mu K u (central difference in t)
            tt, mu_, hd = 0.01, 0.7, 1e-5
            up = oracle.apply_diffusion(th, V, Mq, F[:, :1], [2.0], [tt + hd], [mu_])[:, 0]
            um = oracle.apply_diffusion(th, V, Mq, F[:, :1], [2.0], [tt - hd], [mu_])[:, 0]
            u0 = oracle.apply_diffusion(th, V, Mq, F[:, :1], [2.0], [tt], [mu_])[:, 0]
            lhs = Mq @ (up - um) / (2 * hd)
            check("diffusion_alpha2_ode", np.abs(lhs + mu_ * Kq @ u0).max() < 1e-5 * np.abs(lhs).max())
            ad, td, md = np.array([0.6, 1.5]), np.array([0.3, 0.05]), np.array([1.0, 2.0])
            Uod = oracle.apply_diffusion(th, V, Mq, F, [0.9], [0.2], [1.0])

            def dloss(ax, tx, mx):
                tot = 0.0
                for b in range(2):
                    r = oracle.apply_diffusion(th, V, Mq, F[:, b], [ax[b]], [tx[b]], [mx[b]])[:, 0] - Uod[:, b]
                    tot += r @ Mq @ r
                return tot
            Ud = np.stack([oracle.apply_diffusion(th, V, Mq, F[:, b], [ad[b]], [td[b]], [md[b]])[:, 0]
                           for b in range(2)], 1)
            _, gad, gtd, gmd = oracle.grad_diffusion(th, V, Mq, F, ad, td, md, 2 * Mq @ (Ud - Uod))
            e0 = np.array([hh, 0.0])
            fa = (dloss(ad + e0, td, md) - dloss(ad - e0, td, md)) / (2 * hh)
            ft = (dloss(ad, td + e0, md) - dloss(ad, td - e0, md)) / (2 * hh)
            fm = (dloss(ad, td, md + e0) - dloss(ad, td, md - e0)) / (2 * hh)
            check("diffusion_grad_fd", abs(gad[0] - fa) < 1e-6 * max(1.0, abs(fa)) and
                  abs(gtd[0] - ft) < 1e-6 * max(1.0, abs(ft)) and abs(gmd[0] - fm) < 1e-6 * max(1.0, abs(fm)))
            GU0 = oracle.grad_diffusion(th, V, Mq, F, ad, td, md, 2 * Mq @ (Ud - Uod))[0]
            Dd = np.random.default_rng(1).standard_normal(F.shape)

            def floss(Fx):
                tot = 0.0
                for b in range(2):
                    r = oracle.apply_diffusion(th, V, Mq, Fx[:, b], [ad[b]], [td[b]], [md[b]])[:, 0] - Uod[:, b]
                    tot += r @ Mq @ r
                return tot
            fd = (floss(F + hh * Dd) - floss(F - hh * Dd)) / (2 * hh)
            check("diffusion_grad_u0_fd", abs(np.sum(GU0 * Dd) - fd) < 1e-6 * max(1.0, abs(fd)))
            # Sylvester counts of the banded LDL^T against LAPACK
            ok = True
            for k in (5, 40, 90):
                sig = 0.5 * (w[k] + w[k + 1])
                ok = ok and oracle.inertia_count_banded(Kr, Mr, sig) == k + 1
            check("band_inertia", ok)
        except Exception as e:  # a mutant may also break the pipeline outright
            bad.append(f"raised:{type(e).__name__}")
    return bad


def test_unmutated_oracle_passes_all_pins():
    oracle.build()
    assert failing_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", so,
                           str(mutated), "-lm"])
    with swapped_lib(so):
        bad = failing_pins()
    assert bad, f"mutant {name} passed every pin"
