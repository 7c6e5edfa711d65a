"""Pins of the CPU oracle against facts fixed by the mathematics and the
paper, independent of the oracle's own code (CPU only).

Each test names the passage it follows:
  * stencils / mass sums: Galerkin definition of K and M (Section "Method",
    equation discrete_laplace and the definition of K_ij and M_ij);
  * spectra: the generalized Fourier series on squares (Section "Method") in
    its exact discrete form (bilinear elements), and library LAPACK for P1;
  * inertia counts: Sylvester's law (Section "Eigenvalue counting");
  * apply: the expansion v = sum theta^(-alpha/2) <f,phi> phi (Section
    "Method"), the eigenfunction forcing of Section "Accuracy", and the
    alpha = 0 / alpha = 2 limits stated with the title figure.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1911_11906_amd import inputs
from oracle.closed_form import Q1Rectangle


# ----------------------------------------------------------------- assembly
def test_q1_stencil_values(oracle_mod):
    """Interior rows of Q1 on a uniform grid: K = {8/3 centre, -1/3 at all 8
    neighbours}, M = h^2/36 {16 centre, 4 edge, 1 corner neighbours}."""
    m = inputs.q1_rectangle(7, 7)
    K, M = oracle_mod.assemble(m)
    h = 1.0 / 8
    i = 3 * 7 + 3  # node (3,3): all neighbours interior
    row_k = K[:, i].reshape(7, 7)
    row_m = M[:, i].reshape(7, 7) * 36 / h ** 2
    expect_k = np.zeros((7, 7)); expect_m = np.zeros((7, 7))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            expect_k[3 + dy, 3 + dx] = 8 / 3 if (dx, dy) == (0, 0) else -1 / 3
            expect_m[3 + dy, 3 + dx] = {0: 16, 1: 4, 2: 1}[abs(dx) + abs(dy)]
    assert np.allclose(row_k, expect_k, atol=1e-14, rtol=0)
    assert np.allclose(row_m, expect_m, atol=1e-12, rtol=0)


def test_q1_rectangle_stencil_anisotropic(oracle_mod):
    """Q1 on hx != hy: K centre = 4/3 (hy/hx + hx/hy) (tensor product of the 1-D
    factors (1/h)[2,-1] and (h/6)[4,1])."""
    m = inputs.q1_rectangle(5, 3, lx=1.0, ly=2.0)
    K, M = oracle_mod.assemble(m)
    hx, hy = 1.0 / 6, 2.0 / 4
    i = 1 * 5 + 2
    assert K[i, i] == pytest.approx((2 / hx) * (4 * hy / 6) + (4 * hx / 6) * (2 / hy), rel=1e-14)
    assert K[i, i + 1] == pytest.approx((-1 / hx) * (4 * hy / 6) + (hx / 6) * (2 / hy), rel=1e-13)
    assert M[i, i] == pytest.approx((4 * hx / 6) * (4 * hy / 6), rel=1e-14)


def test_p1_structured_is_five_point(oracle_mod):
    """P1 on the right-triangle mesh: K is the 5-point Laplacian (4, -1)."""
    m = inputs.p1_right_triangles(6)
    K, M = oracle_mod.assemble(m)
    i = 2 * 6 + 2
    row = K[:, i].reshape(6, 6)
    expect = np.zeros((6, 6))
    expect[2, 2] = 4
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        expect[2 + dy, 2 + dx] = -1
    assert np.allclose(row, expect, atol=1e-14)
    h = 1 / 7
    # consistent mass: diagonal = 6 triangles * 2*area/12 = h^2/2; edge neighbours h^2/12
    assert M[i, i] == pytest.approx(h * h / 2, rel=1e-14)
    assert M[i, i + 1] == pytest.approx(h * h / 12, rel=1e-14)


@pytest.mark.parametrize("which", ["q1", "lshape", "p1poly"])
def test_full_mass_integrates_area_and_neumann_kernel(oracle_mod, which):
    """sum_ij M_ij = |Omega| (integral of 1 = sum of basis functions), and the
    un-eliminated K annihilates constants (row sums 0)."""
    if which == "q1":
        m = inputs.q1_rectangle(6, 4, lx=1.5, ly=0.7)
        area = 1.5 * 0.7
    elif which == "lshape":
        m = inputs.q1_lshape(3)
        area = 0.75
    else:
        m = inputs.p1_polygon_with_holes(300, seed=11)
        p = m.xy[m.conn]
        area = 0.5 * np.sum((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                            - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    K, M, Kf, Mf = oracle_mod.assemble(m, full=True)
    assert Mf.sum() == pytest.approx(area, rel=1e-13)
    assert np.abs(Kf.sum(axis=1)).max() < 1e-12 * np.abs(Kf).max()
    assert np.allclose(K, K.T, atol=0) and np.allclose(M, M.T, atol=0)


def test_p1_delaunay_offdiagonal_nonpositive(oracle_mod):
    """Delaunay triangulations give K_ij <= 0 off the diagonal (sum of
    cotangents of opposite angles is >= 0)."""
    m = inputs.p1_polygon_with_holes(400, seed=5)
    K, _ = oracle_mod.assemble(m)
    off = K - np.diag(np.diag(K))
    assert off.max() < 1e-10


# -------------------------------------------------------------- eigensolve
@pytest.mark.parametrize("mx,my,lx,ly", [(12, 12, 1.0, 1.0), (10, 7, 1.0, 0.6), (24, 24, 1.0, 1.0)])
def test_q1_spectrum_matches_closed_form(oracle_mod, mx, my, lx, ly):
    m = inputs.q1_rectangle(mx, my, lx=lx, ly=ly)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    ref = Q1Rectangle(mx, my, lx, ly).eigenvalues()
    assert np.max(np.abs(th - ref) / ref) < 2e-13 * max(1.0, mx * my / 144)
    assert np.abs(V.T @ M @ V - np.eye(m.n_dof)).max() < 1e-12
    R = K @ V - (M @ V) * th[None, :]
    assert np.abs(R).max() < 1e-11 * th.max()


def test_p1_spectrum_vs_lapack_and_trace(oracle_mod):
    m = inputs.p1_polygon_with_holes(350, seed=7)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    w = sl.eigh(K, M, eigvals_only=True)
    assert np.max(np.abs(th - w) / w) < 1e-11
    assert np.sum(th) == pytest.approx(np.trace(np.linalg.solve(M, K)), rel=1e-12)
    assert np.abs(V.T @ M @ V - np.eye(m.n_dof)).max() < 1e-12


def test_p1_minmax_upper_bounds(oracle_mod):
    """Conforming Galerkin eigenvalues bound the continuum ones from above:
    theta_k >= lambda_k = pi^2 (j^2 + l^2) (sorted) on the unit square."""
    m = inputs.p1_right_triangles(12)
    K, M = oracle_mod.assemble(m)
    th, _ = oracle_mod.eigensolve(K, M)
    lam = np.sort([np.pi ** 2 * (a * a + b * b) for a in range(1, 40) for b in range(1, 40)])[: th.size]
    assert np.all(th >= lam * (1 - 1e-12))
    assert th[0] == pytest.approx(2 * np.pi ** 2, rel=0.1)


def test_inertia_counts_index_completeness(oracle_mod):
    """Sylvester: #negative pivots of LDL^T(K - sigma M) = #theta < sigma."""
    m = inputs.p1_polygon_with_holes(200, seed=9)
    K, M = oracle_mod.assemble(m)
    th, _ = oracle_mod.eigensolve(K, M)
    rng = np.random.default_rng(0)
    for k in sorted(rng.choice(th.size - 1, 8, replace=False)):
        if th[k + 1] - th[k] < 1e-8 * th[k]:
            continue
        sigma = 0.5 * (th[k] + th[k + 1])
        assert oracle_mod.inertia_count(K, M, sigma) == k + 1


@pytest.mark.parametrize("which", ["p1", "lshape"])
def test_banded_inertia_matches_dense_and_lapack(oracle_mod, which):
    """The banded count (reverse Cuthill-McKee, banded LDL^T) equals the dense
    count and the number of LAPACK eigenvalues below sigma."""
    import scipy.linalg
    m = inputs.p1_polygon_with_holes(260, seed=5) if which == "p1" else inputs.q1_lshape(7)
    K, M = oracle_mod.assemble(m)
    w = scipy.linalg.eigh(K, M, eigvals_only=True)
    rng = np.random.default_rng(1)
    for k in sorted(rng.choice(w.size - 1, 6, replace=False)):
        if w[k + 1] - w[k] < 1e-8 * w[k + 1]:
            continue
        sigma = 0.5 * (w[k] + w[k + 1])
        nb = oracle_mod.inertia_count_banded(K, M, sigma)
        assert nb == oracle_mod.inertia_count(K, M, sigma) == k + 1
    assert oracle_mod.inertia_count_banded(K, M, 0.5 * w[0]) == 0
    assert oracle_mod.inertia_count_banded(K, M, 2.0 * w[-1]) == w.size


def test_jacobi_on_a_textbook_matrix(oracle_mod):
    """Tridiagonal (2,-1) of size m has eigenvalues 2 - 2 cos(j pi/(m+1))."""
    mm = 31
    A = 2 * np.eye(mm) - np.eye(mm, k=1) - np.eye(mm, k=-1)
    d, Q, sw = oracle_mod.jacobi(A)
    ref = 2 - 2 * np.cos(np.arange(1, mm + 1) * np.pi / (mm + 1))
    assert np.allclose(np.sort(d), ref, atol=1e-13, rtol=0)
    assert np.abs(Q @ np.diag(d) @ Q.T - A).max() < 1e-13
    assert 0 < sw < 20


# -------------------------------------------------------------------- apply
@pytest.fixture(scope="module")
def c1_basis(oracle_mod):
    m = inputs.q1_rectangle(24, 24)
    K, M = oracle_mod.assemble(m)
    th, V = oracle_mod.eigensolve(K, M)
    return m, K, M, th, V


def test_eigenfunction_forcing(c1_basis, oracle_mod):
    """f = sin(pi x) sin(pi y) sampled at the nodes is exactly the (1,1)
    discrete mode, so u = theta_11^(-alpha/2) f; against the continuum
    (2 pi^2)^(-alpha/2) sin sin the gap is the discretisation error
    1 - (theta_11/(2 pi^2))^(-alpha/2)."""
    m, K, M, th, V = c1_basis
    f = inputs.sine_mode(m)
    cf = Q1Rectangle(24, 24)
    th11 = cf.tx[0] + cf.ty[0]
    alphas = inputs.paper_alpha_sweep()
    U = oracle_mod.apply_fractional(th, V, M, f, alphas)
    for i, a in enumerate(alphas):
        u = U[:, i]
        assert np.abs(u - th11 ** (-a / 2) * f[:, 0]).max() < 5e-13
        cont = (2 * np.pi ** 2) ** (-a / 2) * f[:, 0]
        gap = abs(1 - (th11 / (2 * np.pi ** 2)) ** (-a / 2))
        err = np.abs(u - cont).max() / np.abs(cont).max()
        assert err == pytest.approx(gap, rel=1e-6, abs=1e-12)
        assert err <= (a / 2) * 1.4e-3 + 1e-12


def test_alpha_limits_semigroup_linearity(c1_basis, oracle_mod):
    m, K, M, th, V = c1_basis
    F = inputs.polynomial_forcings(m, 3, tag=1)
    U0 = oracle_mod.apply_fractional(th, V, M, F, [0.0])
    assert np.abs(U0 - F).max() < 2e-12 * np.abs(F).max()          # alpha = 0: g = f
    U2 = oracle_mod.apply_fractional(th, V, M, F, [2.0])
    assert np.abs(K @ U2 - M @ F).max() < 1e-11 * np.abs(M @ F).max()  # alpha = 2: K u = M f
    a, b = 0.7, 0.9
    Uab = oracle_mod.apply_fractional(th, V, M, F, [a + b])
    Ub = oracle_mod.apply_fractional(th, V, M, F, [b])
    Uab2 = oracle_mod.apply_fractional(th, V, M, Ub, [a])
    assert np.abs(Uab - Uab2).max() < 1e-12 * np.abs(Uab).max()
    G = oracle_mod.apply_fractional(th, V, M, F @ np.array([[2.0], [-1.0], [0.5]]), [1.3])
    Gs = oracle_mod.apply_fractional(th, V, M, F, [1.3]) @ np.array([[2.0], [-1.0], [0.5]])
    assert np.abs(G - Gs).max() < 1e-12 * np.abs(G).max()


def test_closed_form_apply_matches_oracle(c1_basis, oracle_mod):
    m, K, M, th, V = c1_basis
    F = inputs.polynomial_forcings(m, 4, tag=7)
    al = np.array([0.0, 0.5, 1.25, 2.0])
    U = oracle_mod.apply_fractional(th, V, M, F, al)
    Uc = Q1Rectangle(24, 24).apply(F, al)
    assert np.abs(U - Uc).max() < 1e-11 * np.abs(U).max()
    cf = Q1Rectangle(24, 24)
    for jx, ky in ((1, 1), (3, 2), (24, 24)):
        v = cf.eigenvector(jx, ky)
        t = cf.tx[jx - 1] + cf.ty[ky - 1]
        assert np.abs(K @ v - t * (M @ v)).max() < 1e-11 * t
        assert v @ M @ v == pytest.approx(1.0, rel=1e-13)


# ----------------------------------------------------------------- gradient
def test_gradient_finite_differences(c1_basis, oracle_mod):
    """L = (u - u_obs)^T M (u - u_obs): dL/du = 2 M (u - u_obs); the adjoint
    gives dL/df and dL/dalpha; check by central differences."""
    m, K, M, th, V = c1_basis
    F = inputs.polynomial_forcings(m, 2, tag=9)
    al = np.array([0.6, 1.4])
    al_obs = np.array([1.0, 0.3])
    Uobs = np.stack([oracle_mod.apply_fractional(th, V, M, F[:, b], [al_obs[b]])[:, 0] for b in range(2)], 1)

    def loss(Fx, ax):
        tot = 0.0
        for b in range(2):
            u = oracle_mod.apply_fractional(th, V, M, Fx[:, b], [ax[b]])[:, 0]
            r = u - Uobs[:, b]
            tot += r @ M @ r
        return tot

    U = np.stack([oracle_mod.apply_fractional(th, V, M, F[:, b], [al[b]])[:, 0] for b in range(2)], 1)
    GU = 2 * M @ (U - Uobs)
    GF, ga = oracle_mod.grad_apply(th, V, M, F, al, GU)
    h = 1e-5
    for b in range(2):
        e = np.zeros(2); e[b] = h
        fd = (loss(F, al + e) - loss(F, al - e)) / (2 * h)
        assert ga[b] == pytest.approx(fd, rel=1e-7)
    D = np.random.default_rng(1).standard_normal(F.shape)
    fd = (loss(F + h * D, al) - loss(F - h * D, al)) / (2 * h)
    assert np.sum(GF * D) == pytest.approx(fd, rel=1e-7)


def test_gradient_eigenfunction_closed_form(c1_basis, oracle_mod):
    """For f the (1,1) mode, du/dalpha = -1/2 ln(theta_11) u, so with
    L = g^T u the alpha-gradient is -1/2 ln(theta_11) g^T u."""
    m, K, M, th, V = c1_basis
    f = inputs.sine_mode(m)
    cf = Q1Rectangle(24, 24)
    th11 = cf.tx[0] + cf.ty[0]
    g = np.random.default_rng(3).standard_normal((m.n_dof, 1))
    a = np.array([0.8])
    u = oracle_mod.apply_fractional(th, V, M, f, a)
    _, ga = oracle_mod.grad_apply(th, V, M, f, a, g)
    assert ga[0] == pytest.approx(-0.5 * np.log(th11) * float(g[:, 0] @ u[:, 0]), rel=1e-11)
