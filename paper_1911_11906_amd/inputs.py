"""Seeded synthetic inputs: meshes, forcings and fractional orders.

This module holds no arithmetic of the method (no element integrals, no
eigen-solve, no spectral weights).  It only produces the discretised domain
(node coordinates, element connectivity, Dirichlet flags) and the values fed
to the solver (forcing samples at the nodes, fractional orders), so that the
GPU path and the CPU oracle can be driven by identical data.

Workloads follow the paper's accuracy setup (unit square, homogeneous
Dirichlet data, Fourier-mode forcing; Section "Accuracy") and stand-ins for
its complex-geometry meshes (Section "Test Meshes"), which are not available:
a seeded star polygon with two circular holes triangulated by Delaunay.

Every random draw comes from ``numpy.random.default_rng(SeedSequence([1911,
11906, tag]))`` so that a (workload, seed) pair fixes the data bit for bit.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

Q1 = 4  # bilinear quadrilateral: 4 nodes per element, counter-clockwise
P1 = 3  # linear triangle: 3 nodes per element, counter-clockwise


def rng_for(tag: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([1911, 11906, int(tag), *map(int, extra)]))


@dataclass
class Mesh:
    elem: int                 # nodes per element: P1 (3), Q1 (4) or (p+1)^2 for order p
    xy: np.ndarray            # (n_nodes, 2) float64
    conn: np.ndarray          # (n_elem, elem) int32, CCW
    dirichlet: np.ndarray     # (n_nodes,) uint8, 1 = boundary node (eliminated)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_dof(self) -> int:
        return int(self.n_nodes - int(self.dirichlet.sum()))

    def dof_of_node(self) -> np.ndarray:
        """Interior nodes numbered in node order; -1 for Dirichlet nodes."""
        d = np.full(self.n_nodes, -1, dtype=np.int64)
        inner = np.nonzero(self.dirichlet == 0)[0]
        d[inner] = np.arange(inner.size, dtype=np.int64)
        return d

    def interior_xy(self) -> np.ndarray:
        return self.xy[self.dirichlet == 0]

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.xy, self.conn, self.dirichlet):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def q1_rectangle(mx: int, my: int, x0: float = 0.0, y0: float = 0.0,
                 lx: float = 1.0, ly: float = 1.0) -> Mesh:
    """Uniform Q1 grid with mx x my interior nodes on [x0,x0+lx]x[y0,y0+ly].

    Nodes are numbered lexicographically with x fastest; interior DOFs follow
    the same order.  Elements are counter-clockwise.
    """
    nx, ny = mx + 2, my + 2
    xs = x0 + lx * np.arange(nx) / (mx + 1)
    ys = y0 + ly * np.arange(ny) / (my + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    n00 = (j * nx + i).ravel()
    conn = np.stack([n00, n00 + 1, n00 + 1 + nx, n00 + nx], axis=1).astype(np.int32)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    bnd = ((ii == 0) | (ii == nx - 1) | (jj == 0) | (jj == ny - 1)).ravel()
    return Mesh(Q1, xy, conn, bnd.astype(np.uint8), name=f"q1_rect_{mx}x{my}",
                meta={"mx": mx, "my": my, "lx": lx, "ly": ly})


def gll_points(p: int) -> np.ndarray:
    """The p + 1 Gauss-Lobatto-Legendre points on [-1, 1] (the endpoints and
    the roots of P_p'), ascending: the node positions of an order-p element
    along each direction."""
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def qp_rectangle(ex: int, ey: int, p: int, lx: float = 1.0, ly: float = 1.0) -> Mesh:
    """ex x ey elements of order p (2 <= p <= 8) on [0,lx]x[0,ly]: each element
    carries the (p+1) x (p+1) tensor lattice of Gauss-Lobatto-Legendre points
    mapped to it, numbered lexicographically (a + (p+1) b, a along x);
    elements share their edge nodes.  Global nodes: the (ex p + 1) x (ey p + 1)
    lattice, x fastest; the boundary lattice nodes are Dirichlet."""
    if not 2 <= p <= 8:
        raise ValueError("order must be in [2, 8]")
    g = 0.5 * (gll_points(p) + 1.0)                     # on [0, 1]
    xs = np.concatenate([(i + g[:-1]) * lx / ex for i in range(ex)] + [[lx]])
    ys = np.concatenate([(j + g[:-1]) * ly / ey for j in range(ey)] + [[ly]])
    nx, ny = xs.size, ys.size
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    a = np.arange(p + 1)
    loc = (a[None, :] + nx * a[:, None]).ravel()          # local (a, b) -> offset, a fastest
    conn = np.array([loc + (i * p) + nx * (j * p) for j in range(ey) for i in range(ex)], dtype=np.int32)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    bnd = ((ii == 0) | (ii == nx - 1) | (jj == 0) | (jj == ny - 1)).ravel()
    return Mesh((p + 1) ** 2, xy, conn, bnd.astype(np.uint8), name=f"q{p}_rect_{ex}x{ey}",
                meta={"ex": ex, "ey": ey, "p": p, "lx": lx, "ly": ly})


def q1_lshape(m: int) -> Mesh:
    """L-shaped Q1 mesh: the unit square grid with (2m+1)^2 interior nodes of
    spacing 1/(2m+2), minus the upper-right quadrant.  Boundary nodes of the
    L (including the re-entrant edges) are Dirichlet."""
    full = 2 * m + 3                      # nodes per side of the enclosing square grid
    h = 1.0 / (full - 1)
    keep_node = np.zeros((full, full), dtype=bool)
    half = (full - 1) // 2
    for j in range(full):
        for i in range(full):
            keep_node[j, i] = not (i > half and j > half)
    idx = -np.ones((full, full), dtype=np.int64)
    idx[keep_node] = np.arange(int(keep_node.sum()))
    jj, ii = np.nonzero(keep_node)
    xy = np.stack([ii * h, jj * h], axis=1).astype(np.float64)
    conn = []
    for j in range(full - 1):
        for i in range(full - 1):
            if i >= half and j >= half:
                continue
            conn.append([idx[j, i], idx[j, i + 1], idx[j + 1, i + 1], idx[j + 1, i]])
    conn = np.asarray(conn, dtype=np.int32)
    # boundary: a node is Dirichlet if it lies on the outer square boundary or
    # on the re-entrant edges x=0.5 (y>=0.5) / y=0.5 (x>=0.5)
    bnd = np.zeros(xy.shape[0], dtype=np.uint8)
    for k, (i, j) in enumerate(zip(ii, jj)):
        on_outer = i == 0 or j == 0 or i == full - 1 or j == full - 1
        on_inner = (i == half and j >= half) or (j == half and i >= half)
        bnd[k] = 1 if (on_outer or on_inner) else 0
    return Mesh(Q1, xy, conn, bnd, name=f"q1_lshape_{m}", meta={"m": m})


def p1_right_triangles(m: int) -> Mesh:
    """Structured P1 mesh of the unit square: each grid cell cut along the
    diagonal from its lower-left to upper-right corner (m x m interior nodes)."""
    q = q1_rectangle(m, m)
    tri = []
    for a, b, c, d in q.conn:
        tri.append([a, b, c])
        tri.append([a, c, d])
    return Mesh(P1, q.xy, np.asarray(tri, dtype=np.int32), q.dirichlet,
                name=f"p1_square_{m}x{m}", meta={"m": m})


def _point_in_polygon(px, py, poly):
    """Even-odd rule, vectorised over points."""
    inside = np.zeros(px.shape, dtype=bool)
    n = len(poly)
    for k in range(n):
        x1, y1 = poly[k]
        x2, y2 = poly[(k + 1) % n]
        cond = (y1 > py) != (y2 > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = x1 + (py - y1) * (x2 - x1) / (y2 - y1)
        inside ^= cond & (px < xint)
    return inside


def _dist_to_polygon(px, py, poly):
    d = np.full(px.shape, np.inf)
    n = len(poly)
    for k in range(n):
        x1, y1 = poly[k]
        x2, y2 = poly[(k + 1) % n]
        ex, ey = x2 - x1, y2 - y1
        t = np.clip(((px - x1) * ex + (py - y1) * ey) / (ex * ex + ey * ey), 0.0, 1.0)
        d = np.minimum(d, np.hypot(px - (x1 + t * ex), py - (y1 + t * ey)))
    return d


def p1_polygon_with_holes(n_target: int = 16384, seed: int = 3) -> Mesh:
    """Seeded star-shaped 12-gon with two circular holes, P1 Delaunay mesh of a
    jittered grid, trimmed to exactly ``n_target`` interior nodes.

    Stand-in for the paper's complex 2-D geometry (its site mesh is not
    available).  Recipe: 12 vertices at sorted U(0,2pi) angles with radius
    0.5(0.7+0.3U) about (0.5,0.5); two holes of radius U(0.06,0.10) placed by
    rejection; interior points on a grid of spacing h jittered by U(+-h/4),
    kept at least h/2 from every boundary; boundary points every ~h; h chosen
    by bisection so that at least n_target interior points exist, the surplus
    removed by a seeded draw; Delaunay triangles whose centroid lies outside
    the domain are dropped.
    """
    from scipy.spatial import Delaunay

    rng = rng_for(3, seed)
    ang = np.sort(rng.uniform(0, 2 * np.pi, 12))
    rad = 0.5 * (0.7 + 0.3 * rng.uniform(size=12))
    poly = np.stack([0.5 + rad * np.cos(ang), 0.5 + rad * np.sin(ang)], axis=1)
    holes = []
    tries = 0
    while len(holes) < 2:
        tries += 1
        if tries > 100000:
            raise RuntimeError("hole placement failed")
        r = rng.uniform(0.06, 0.10)
        c = rng.uniform(0.1, 0.9, size=2)
        if not _point_in_polygon(np.array([c[0]]), np.array([c[1]]), poly)[0]:
            continue
        if _dist_to_polygon(np.array([c[0]]), np.array([c[1]]), poly)[0] < r + 0.04:
            continue
        if any(np.hypot(*(c - hc)) < r + hr + 0.04 for hc, hr in holes):
            continue
        holes.append((c, r))

    def interior_points(h, jitter_rng):
        g = np.arange(0.0, 1.0 + h, h)
        X, Y = np.meshgrid(g, g, indexing="xy")
        px = X.ravel() + jitter_rng.uniform(-h / 4, h / 4, X.size)
        py = Y.ravel() + jitter_rng.uniform(-h / 4, h / 4, Y.size)
        ok = _point_in_polygon(px, py, poly) & (_dist_to_polygon(px, py, poly) >= h / 2)
        for hc, hr in holes:
            ok &= np.hypot(px - hc[0], py - hc[1]) >= hr + h / 2
        return px[ok], py[ok]

    lo, hi = 1e-4, 0.05
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        px, _py = interior_points(mid, rng_for(3, seed, 1))
        if px.size >= n_target:
            lo = mid
        else:
            hi = mid
    h = lo
    px, py = interior_points(h, rng_for(3, seed, 1))
    assert px.size >= n_target
    keep = np.sort(rng_for(3, seed, 2).choice(px.size, n_target, replace=False))
    px, py = px[keep], py[keep]

    bx, by = [], []
    for k in range(len(poly)):
        x1, y1 = poly[k]
        x2, y2 = poly[(k + 1) % len(poly)]
        m = max(1, int(np.ceil(np.hypot(x2 - x1, y2 - y1) / h)))
        t = np.arange(m) / m
        bx.append(x1 + t * (x2 - x1))
        by.append(y1 + t * (y2 - y1))
    for hc, hr in holes:
        m = max(8, int(np.ceil(2 * np.pi * hr / h)))
        t = 2 * np.pi * np.arange(m) / m
        bx.append(hc[0] + hr * np.cos(t))
        by.append(hc[1] + hr * np.sin(t))
    bx, by = np.concatenate(bx), np.concatenate(by)

    xy = np.concatenate([np.stack([px, py], 1), np.stack([bx, by], 1)]).astype(np.float64)
    dirichlet = np.concatenate([np.zeros(px.size, np.uint8), np.ones(bx.size, np.uint8)])
    tri = Delaunay(xy).simplices.astype(np.int64)
    cen = xy[tri].mean(axis=1)
    ok = _point_in_polygon(cen[:, 0], cen[:, 1], poly)
    for hc, hr in holes:
        ok &= np.hypot(cen[:, 0] - hc[0], cen[:, 1] - hc[1]) >= hr
    tri = tri[ok]
    # orient counter-clockwise
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    flip = cross < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    # drop degenerate slivers (zero area)
    tri = tri[np.abs(cross) > 1e-14]
    used = np.zeros(xy.shape[0], bool)
    used[tri.ravel()] = True
    if not used[: px.size].all():
        raise RuntimeError("interior node not covered by any triangle")
    return Mesh(P1, xy, tri.astype(np.int32), dirichlet, name=f"p1_polyholes_{n_target}",
                meta={"h": h, "poly": poly.tolist(),
                      "holes": [(hc.tolist(), hr) for hc, hr in holes]})


def sine_mode(mesh: Mesh, kx: int = 1, ky: int = 1, lx: float = 1.0, ly: float = 1.0) -> np.ndarray:
    """Forcing sin(kx pi x/lx) sin(ky pi y/ly) sampled at the interior nodes (n, 1)."""
    p = mesh.interior_xy()
    return (np.sin(kx * np.pi * p[:, 0] / lx) * np.sin(ky * np.pi * p[:, 1] / ly))[:, None].copy()


def polynomial_forcings(mesh: Mesh, count: int, tag: int, degree: int = 3) -> np.ndarray:
    """``count`` random bivariate polynomials sum_{a+b<=degree} c_ab x^a y^b,
    c_ab ~ N(0,1), sampled at the interior nodes: column-major (n, count)."""
    rng = rng_for(tag, 100)
    p = mesh.interior_xy()
    terms = [(a, b) for a in range(degree + 1) for b in range(degree + 1 - a)]
    coef = rng.standard_normal((count, len(terms)))
    basis = np.stack([p[:, 0] ** a * p[:, 1] ** b for a, b in terms], axis=1)
    return np.asfortranarray(basis @ coef.T)


def alphas_uniform(count: int, tag: int, lo: float = 0.0, hi: float = 2.0) -> np.ndarray:
    return rng_for(tag, 200).uniform(lo, hi, count)


def paper_alpha_sweep() -> np.ndarray:
    """Eleven equally spaced fractional orders on [0,2] (the accuracy sweep)."""
    return np.linspace(0.0, 2.0, 11)


def _lshape_ndof(m: int) -> int:
    """Interior nodes of q1_lshape(m): the (2m+1)^2 interior grid minus the
    (m+1)^2 nodes of the removed quadrant (its re-entrant edges included)."""
    return (2 * m + 1) ** 2 - (m + 1) ** 2


def batched_problem_meshes(count: int = 256, tag: int = 4, nmin: int = 64, nmax: int = 1024):
    """Rectangles (aspect U(0.5,2)) and L-shapes with interior size near
    n_target ~ U{nmin..nmax}."""
    rng = rng_for(tag, 300)
    out = []
    for _ in range(count):
        nt = int(rng.integers(nmin, nmax + 1))
        if rng.uniform() < 0.5:
            aspect = rng.uniform(0.5, 2.0)
            mx = max(2, int(round(np.sqrt(nt * aspect))))
            my = max(2, int(round(nt / mx)))
            while mx * my > nmax:          # keep n inside [nmin, nmax]
                if mx >= my:
                    mx -= 1
                else:
                    my -= 1
            while mx * my < nmin:
                if mx <= my:
                    mx += 1
                else:
                    my += 1
            out.append(q1_rectangle(mx, my, lx=1.0, ly=float(my + 1) / float(mx + 1)))
        else:
            best = None
            for m in range(1, 40):
                nn = _lshape_ndof(m)
                if nn < nmin or nn > nmax:
                    continue
                if best is None or abs(nn - nt) < abs(best[1] - nt):
                    best = (m, nn)
            out.append(q1_lshape(best[0]))
    return out


def workload(name: str):
    """Named workloads (see the design doc for the recipe of each)."""
    if name == "c1":
        m = q1_rectangle(24, 24)
        return {"mesh": m, "F": sine_mode(m), "alpha": np.array([0.5, 1.0, 1.5])}
    if name == "c2":
        m = q1_rectangle(96, 96)
        return {"mesh": m, "F": polynomial_forcings(m, 64, tag=2), "alpha": alphas_uniform(16, tag=2)}
    if name == "c3":
        m = p1_polygon_with_holes(16384)
        return {"mesh": m}
    if name == "c4_apply":
        m = q1_rectangle(128, 128)
        return {"mesh": m, "F": polynomial_forcings(m, 1024, tag=4), "alpha": alphas_uniform(32, tag=4)}
    if name == "c5":
        m = q1_rectangle(181, 181)
        rng = rng_for(5, 400)
        return {"mesh": m, "F": polynomial_forcings(m, 128, tag=5),
                "alpha": rng.uniform(0, 2, 128), "alpha_obs": rng_for(5, 401).uniform(0, 2, 128)}
    raise KeyError(name)
