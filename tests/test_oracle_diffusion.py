"""Pins of the oracle's fractional diffusion solution and of the closed-form
adjoints (CPU only).

Fractional diffusion (Section "Method", equations model_diffusion and
diffusion_solution): u(t) = sum_k exp(-mu theta_k^(alpha/2) t) <u0, phi_k>
phi_k.  The exact solution of Section "Accuracy" (equations diffusion_ics and
diffusion_sols: u0 = sin(pi x) sin(pi y), with the factor 1 instead of 2
since the map is linear) at t = 0.4, mu = 1 for the paper's 11 orders; the
t = 0 and mu = 0 limits; the semigroup property in t; the alpha = 2 case,
which solves the heat equation M du/dt = -mu K u; and the closed form on
rectangles.  The closed-form adjoints (Poisson and diffusion) are pinned
against the oracle's adjoints and central finite differences.
"""
import numpy as np
import pytest

from oracle.closed_form import Q1Rectangle
from paper_1911_11906_amd import inputs


@pytest.fixture(scope="module")
def basis(oracle_mod):
    m = inputs.q1_rectangle(24, 24)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    return m, K, M, th, V


def test_eigenfunction_initial_condition(basis, oracle_mod):
    """u0 = the (1,1) discrete mode decays as exp(-mu theta_11^(alpha/2) t);
    against the continuum exp(-mu (2 pi^2)^(alpha/2) t) sin sin the gap is
    exactly the change of that exponent."""
    m, K, M, th, V = basis
    u0 = inputs.sine_mode(m)
    cf = Q1Rectangle(24, 24)
    th11 = cf.tx[0] + cf.ty[0]
    al = inputs.paper_alpha_sweep()
    t, mu = 0.4, 1.0
    U = oracle_mod.apply_diffusion(th, V, M, u0, al, t, mu)
    for i, a in enumerate(al):
        disc = np.exp(-mu * th11 ** (a / 2) * t)
        cont = np.exp(-mu * (2 * np.pi ** 2) ** (a / 2) * t)
        assert np.abs(U[:, i] - disc * u0[:, 0]).max() < 5e-13
        gap = np.abs(U[:, i] - cont * u0[:, 0]).max()
        assert gap == pytest.approx(abs(disc - cont) * np.abs(u0).max(), rel=1e-6, abs=5e-13)


def test_limits_and_semigroup(basis, oracle_mod):
    m, K, M, th, V = basis
    F = inputs.polynomial_forcings(m, 3, tag=21)
    U = oracle_mod.apply_diffusion(th, V, M, F, [1.2], [0.0], [1.0])
    assert np.abs(U - F).max() < 1e-12 * np.abs(F).max()
    U = oracle_mod.apply_diffusion(th, V, M, F, [0.7], [0.3], [0.0])
    assert np.abs(U - F).max() < 1e-12 * np.abs(F).max()
    a, mu = 1.4, 0.8
    U1 = oracle_mod.apply_diffusion(th, V, M, F, [a], [0.01], [mu])
    U12 = oracle_mod.apply_diffusion(th, V, M, U1, [a], [0.02], [mu])
    U3 = oracle_mod.apply_diffusion(th, V, M, F, [a], [0.03], [mu])
    assert np.abs(U12 - U3).max() < 1e-12 * np.abs(U3).max()
    # mu and t enter only through their product
    Ua = oracle_mod.apply_diffusion(th, V, M, F, [a], [0.02], [1.5])
    Ub = oracle_mod.apply_diffusion(th, V, M, F, [a], [0.03], [1.0])
    assert np.abs(Ua - Ub).max() < 1e-12 * np.abs(Ub).max()


def test_alpha2_is_the_heat_equation(basis, oracle_mod):
    m, K, M, th, V = basis
    F = inputs.polynomial_forcings(m, 2, tag=22)
    t, mu, h = 0.002, 1.3, 1e-6
    up = oracle_mod.apply_diffusion(th, V, M, F, [2.0], [t + h], [mu])
    um = oracle_mod.apply_diffusion(th, V, M, F, [2.0], [t - h], [mu])
    u = oracle_mod.apply_diffusion(th, V, M, F, [2.0], [t], [mu])
    lhs = M @ (up - um) / (2 * h)
    assert np.abs(lhs + mu * K @ u).max() < 1e-6 * np.abs(lhs).max()


@pytest.mark.parametrize("mx,my,ly", [(24, 24, 1.0), (13, 9, 0.7)])
def test_closed_form_diffusion_matches_oracle(oracle_mod, mx, my, ly):
    m = inputs.q1_rectangle(mx, my, ly=ly)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    cf = Q1Rectangle(mx, my, 1.0, ly)
    F = inputs.polynomial_forcings(m, 4, tag=23)
    al, t, mu = np.array([0.0, 0.5, 1.3, 2.0]), np.array([0.4, 0.1, 0.02, 0.003]), np.array([1.0, 2.0, 0.5, 1.0])
    Uo = oracle_mod.apply_diffusion(th, V, M, F, al, t, mu)
    Uc = cf.apply(F, al, mu_t=mu * t)
    assert np.abs(Uo - Uc).max() < 1e-12 * np.abs(Uo).max()


def test_closed_form_adjoints_match_oracle(oracle_mod):
    mx, my, ly = 13, 9, 0.7
    m = inputs.q1_rectangle(mx, my, ly=ly)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    cf = Q1Rectangle(mx, my, 1.0, ly)
    F = inputs.polynomial_forcings(m, 4, tag=24)
    GU = np.random.default_rng(4).standard_normal(F.shape)
    al = np.array([0.2, 0.9, 1.5, 2.0])
    GF, ga, gs = cf.grad(F, al, GU)
    GFo, gao = oracle_mod.grad_apply(th, V, M, F, al, GU)
    assert gs is None
    assert np.abs(GF - GFo).max() < 1e-12 * np.abs(GFo).max()
    assert np.abs(ga - gao).max() < 1e-12 * np.abs(gao).max()
    t, mu = np.array([0.4, 0.1, 0.02, 0.003]), np.array([1.0, 2.0, 0.5, 1.0])
    GFd, gad, gsd = cf.grad(F, al, GU, mu_t=mu * t)
    GU0o, gado, gto, gmo = oracle_mod.grad_diffusion(th, V, M, F, al, t, mu, GU)
    assert np.abs(GFd - GU0o).max() < 1e-12 * np.abs(GU0o).max()
    assert np.abs(gad - gado).max() < 1e-11 * np.abs(gado).max()
    assert np.abs(mu * gsd - gto).max() < 1e-11 * np.abs(gto).max()
    assert np.abs(t * gsd - gmo).max() < 1e-11 * np.abs(gmo).max()


def test_closed_form_gradient_finite_differences():
    """The closed-form adjoint of the L2 misfit against central differences
    of the closed-form forward map (Poisson and diffusion weights)."""
    mx, my = 11, 8
    m = inputs.q1_rectangle(mx, my)
    cf = Q1Rectangle(mx, my)
    F = inputs.polynomial_forcings(m, 3, tag=25)
    al = np.array([0.3, 1.0, 1.7])
    mt = np.array([0.02, 0.1, 0.05])
    # mass matrix applied through the transform: M x = sum_k (phi_k^T M x) M phi_k
    for mu_t in (None, mt):
        obs = np.stack([cf.apply(F[:, b], [1.1], None if mu_t is None else [0.07])[:, 0] for b in range(3)], 1)

        def fwd(Fx, ax, sx):
            return np.stack([cf.apply(Fx[:, b], [ax[b]], None if sx is None else [sx[b]])[:, 0]
                             for b in range(3)], 1)

        def loss(Fx, ax, sx):
            R = fwd(Fx, ax, sx) - obs
            MR = cf._synth(cf._coeffs(R), mass=True)   # M R via M = M V V^T M
            return float(np.sum(R * MR))
        U = fwd(F, al, mu_t)
        R = U - obs
        GU = 2 * cf._synth(cf._coeffs(R), mass=True)
        GF, ga, gs = cf.grad(F, al, GU, mu_t=mu_t)
        h = 1e-6
        for b in range(3):
            e = np.zeros(3)
            e[b] = h
            fd = (loss(F, al + e, mu_t) - loss(F, al - e, mu_t)) / (2 * h)
            assert ga[b] == pytest.approx(fd, rel=1e-6, abs=1e-12)
            if mu_t is not None:
                fd = (loss(F, al, mu_t + e) - loss(F, al, mu_t - e)) / (2 * h)
                assert gs[b] == pytest.approx(fd, rel=1e-6, abs=1e-12)
        D = np.random.default_rng(9).standard_normal(F.shape)
        fd = (loss(F + h * D, al, mu_t) - loss(F - h * D, al, mu_t)) / (2 * h)
        assert float(np.sum(GF * D)) == pytest.approx(fd, rel=1e-6)
