"""Seeded synthetic inputs: meshes, targets and densities.

This module holds no part of the evaluator's arithmetic (no quadrature, no
kernel, no basis): it only produces the inputs that the library and the test
oracle both consume.  All randomness uses ``numpy.random.default_rng(seed)``.

Every mesh it returns has counter-clockwise triangles, so the vertex order
(A, B, C) it stores is the order in which the reference nodes are mapped:
node xi = (xi1, xi2) of triangle (A, B, C) sits at A + xi1 (B-A) + xi2 (C-A).

Workloads (sizes are those the benchmark and the tests use):
  * unit square [0,1]^2, n x n cells, "/" split (quadrature mesh) and "\\"
    split (staggered target mesh);
  * star r(theta) = 1 + 0.3 cos(5 theta): equispaced boundary points plus a
    jittered hexagonal lattice inside, Delaunay-triangulated; a staggered
    copy with the lattice shifted by (h/2, h sqrt(3)/6) and the boundary by
    half a step;
  * polygonal disk (unit-density check);
  * graded L-shape [-1,1]^2 minus [0,1]^2 with h ~ r^0.5 toward the corner.
"""

import math

import numpy as np
from scipy.spatial import Delaunay, cKDTree


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def _ccw(vert, tri):
    tri = np.asarray(tri, dtype=np.int32).copy()
    a, b, c = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    flip = det < 0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def node_positions(vert, tri, ref_nodes):
    """Physical positions [T, n, 2] of reference nodes in every triangle
    (triangles must be counter-clockwise)."""
    vert = np.asarray(vert, dtype=np.float64)
    tri = np.asarray(tri)
    a, b, c = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    if np.any(det <= 0):
        raise ValueError("node_positions expects counter-clockwise triangles")
    X = np.asarray(ref_nodes, dtype=np.float64)
    return (a[:, None, :] + X[None, :, :1] * (b - a)[:, None, :]
            + X[None, :, 1:2] * (c - a)[:, None, :])


def sample_density(fn, vert, tri, ref_nodes):
    """F[t, i] = f(node i of triangle t); fn maps ([n], [n]) -> [n] or
    [n, R].  Returns [T, n_p] or [T, n_p, R]."""
    pos = node_positions(vert, tri, ref_nodes)
    T, n = pos.shape[:2]
    val = np.asarray(fn(pos[..., 0].ravel(), pos[..., 1].ravel()), dtype=np.float64)
    return val.reshape((T, n) + val.shape[1:])


# ----------------------------------------------------------------------------
# unit square
# ----------------------------------------------------------------------------

def unit_square(n=8, split="/"):
    """[0,1]^2 in n x n cells, each cut in two along "/" or "\\"."""
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    vert = np.stack([X.ravel(), Y.ravel()], axis=1)
    idx = lambda i, j: i * (n + 1) + j  # noqa: E731
    tri = []
    for i in range(n):
        for j in range(n):
            v00, v10, v01, v11 = idx(i, j), idx(i + 1, j), idx(i, j + 1), idx(i + 1, j + 1)
            if split == "/":
                tri += [(v00, v10, v11), (v00, v11, v01)]
            else:
                tri += [(v00, v10, v01), (v10, v11, v01)]
    return vert, _ccw(vert, np.array(tri))


def gaussian_bump(x, y):
    """exp(-((x-0.5)^2 + (y-0.5)^2) / 0.05): the unit-square density."""
    return np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / 0.05)


# ----------------------------------------------------------------------------
# star-shaped and disk domains
# ----------------------------------------------------------------------------

def star_radius(theta):
    return 1.0 + 0.3 * np.cos(5.0 * theta)


STAR_AREA = math.pi * (1.0 + 0.3 ** 2 / 2.0)


def _radial_polygon_mesh(radius_fn, area, n_tri, n_boundary, seed, staggered=False):
    """Mesh of the polygon through n_boundary points equispaced in theta on
    r(theta), star-shaped about the origin.  Interior: jittered hexagonal
    lattice (jitter U[-h/4, h/4]^2), points closer than h/2 to the boundary
    dropped; Delaunay; triangles whose centroid lies outside removed."""
    rng = np.random.default_rng(seed)
    dth = 2.0 * math.pi / n_boundary
    th = np.arange(n_boundary) * dth + (0.5 * dth if staggered else 0.0)
    rb = radius_fn(th)
    bnd = np.stack([rb * np.cos(th), rb * np.sin(th)], axis=1)
    tree = cKDTree(bnd)
    rmax = float(np.max(rb))

    def inside(pts):
        ang = np.mod(np.arctan2(pts[:, 1], pts[:, 0]) - th[0], 2.0 * math.pi)
        k = np.minimum((ang / dth).astype(np.int64), n_boundary - 1)
        p0 = bnd[k]
        p1 = bnd[(k + 1) % n_boundary]
        cr = (p1[:, 0] - p0[:, 0]) * (pts[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (pts[:, 0] - p0[:, 0])
        return cr > 0.0

    n_int_goal = max(1, (n_tri - n_boundary + 2) // 2)
    h = math.sqrt(2.0 * area / (math.sqrt(3.0) * n_int_goal))
    for _ in range(4):
        ny = int(math.ceil(2 * rmax / (h * math.sqrt(3) / 2))) + 2
        nx = int(math.ceil(2 * rmax / h)) + 2
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        px = -rmax - h + ii * h + (jj % 2) * (h / 2)
        py = -rmax - h + jj * (h * math.sqrt(3) / 2)
        if staggered:
            px = px + h / 2
            py = py + h * math.sqrt(3) / 6
        lat = np.stack([px.ravel(), py.ravel()], axis=1)
        lat = lat + rng.uniform(-0.25 * h, 0.25 * h, size=lat.shape)
        keep = inside(lat)
        lat = lat[keep]
        dist, _ = tree.query(lat)
        lat = lat[dist > 0.5 * h]
        pts = np.concatenate([bnd, lat])
        dl = Delaunay(pts)
        tri = dl.simplices
        cen = pts[tri].mean(axis=1)
        tri = tri[inside(cen)]
        if abs(len(tri) - n_tri) <= 0.02 * n_tri:
            break
        h *= math.sqrt(len(tri) / n_tri)
    return pts, _ccw(pts, tri)


def star_mesh(n_tri=20000, n_boundary=2000, seed=20, staggered=False):
    """Star r(theta) = 1 + 0.3 cos(5 theta), about n_tri triangles."""
    return _radial_polygon_mesh(star_radius, STAR_AREA, n_tri, n_boundary, seed, staggered)


def disk_mesh(n_tri=500, n_boundary=60, seed=1, radius=1.0):
    """Polygonal disk of the given radius (vertices on the circle)."""
    return _radial_polygon_mesh(lambda t: np.full_like(t, radius), math.pi * radius ** 2,
                                n_tri, n_boundary, seed)


def polar_curved_sides(vert, tri, radius_fn, n_boundary, staggered=False, deg=16):
    """Curved sides for a mesh of ``_radial_polygon_mesh``: every triangle
    edge joining consecutive boundary points k, k+1 becomes the arc of
    r(theta) between them, given as deg+1 points at the Chebyshev-Lobatto
    parameters u_i = (1 - cos(pi i / deg)) / 2 of theta between the two
    vertices (end points copied from ``vert``).  Returns (curved_tri,
    curved_side, curved_pts [n, deg+1, 2]); side e is the edge from local
    vertex e to local vertex e+1."""
    vert = np.asarray(vert, dtype=np.float64)
    tri = np.asarray(tri)
    dth = 2.0 * math.pi / n_boundary
    off = 0.5 * dth if staggered else 0.0
    u = 0.5 * (1.0 - np.cos(np.pi * np.arange(deg + 1) / deg))
    ct, cs, cp = [], [], []
    for t in range(len(tri)):
        sides = []
        for e in range(3):
            a, b = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            if a < n_boundary and b < n_boundary and (b - a) % n_boundary in (1, n_boundary - 1):
                sides.append((e, a, b))
        if len(sides) > 1:
            raise ValueError("a triangle with two boundary edges cannot take one curved side")
        for e, a, b in sides:
            step = dth if (b - a) % n_boundary == 1 else -dth
            th = a * dth + off + u * step
            r = radius_fn(th)
            pts = np.stack([r * np.cos(th), r * np.sin(th)], 1)
            pts[0], pts[-1] = vert[a], vert[b]
            ct.append(t)
            cs.append(e)
            cp.append(pts)
    return np.array(ct, dtype=np.int32), np.array(cs, dtype=np.int32), np.array(cp)


def curved_disk(n_tri=500, n_boundary=60, seed=1, radius=1.0, deg=16):
    """The disk mesh with its boundary edges replaced by circular arcs:
    (vert, tri, curved_tri, curved_side, curved_pts)."""
    v, t = disk_mesh(n_tri=n_tri, n_boundary=n_boundary, seed=seed, radius=radius)
    return (v, t) + polar_curved_sides(v, t, lambda th: np.full_like(th, radius), n_boundary, deg=deg)


def curved_star(n_tri=20000, n_boundary=2000, seed=20, staggered=False, deg=12):
    """The star mesh with its boundary edges on r = 1 + 0.3 cos(5 theta)."""
    v, t = star_mesh(n_tri=n_tri, n_boundary=n_boundary, seed=seed, staggered=staggered)
    return (v, t) + polar_curved_sides(v, t, star_radius, n_boundary, staggered=staggered, deg=deg)


def polygon_area(vert, tri):
    a, b, c = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    return 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1])
                        - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])).sum()


def gaussian_sum(seed, vert, tri, n_terms=10, width=(0.05, 0.3)):
    """f(x) = sum_i a_i exp(-|x - c_i|^2 / s_i), a ~ U[-1,1], s ~ U[width],
    centres uniform over the mesh (a triangle picked by area, then a
    uniform point in it).  Returns the callable f(x, y)."""
    rng = np.random.default_rng(seed)
    vert = np.asarray(vert)
    a, b, c = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    ar = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    k = rng.choice(len(tri), size=n_terms, p=ar / ar.sum())
    r1, r2 = rng.uniform(size=n_terms), rng.uniform(size=n_terms)
    s1 = np.sqrt(r1)
    cen = (1 - s1)[:, None] * a[k] + (s1 * (1 - r2))[:, None] * b[k] + (s1 * r2)[:, None] * c[k]
    amp = rng.uniform(-1.0, 1.0, size=n_terms)
    wid = rng.uniform(width[0], width[1], size=n_terms)

    def f(x, y):
        x = np.asarray(x)[..., None]
        y = np.asarray(y)[..., None]
        return (amp * np.exp(-((x - cen[:, 0]) ** 2 + (y - cen[:, 1]) ** 2) / wid)).sum(axis=-1)

    return f


# ----------------------------------------------------------------------------
# graded L-shape
# ----------------------------------------------------------------------------

def l_shape_graded(n_tri=250000, seed=50, staggered=False, grade=0.5):
    """[-1,1]^2 minus [0,1]^2 with local size h ~ r^grade toward the
    re-entrant corner (grade = 0.5).  Points: a jittered hexagonal lattice in
    a reference plane xi, mapped by x = xi |xi|^(1/grade - 1), which spreads
    uniform spacing into h ~ |x|^grade (radial and tangential stretches
    differ by the factor 1/grade, so triangles stay within aspect ~2);
    boundary points spaced by the same local size; Delaunay; triangles with
    centroid in the removed quadrant dropped.  The staggered copy shifts the
    lattice by (h/2, h sqrt(3)/6) and the boundary by half a step."""
    rng = np.random.default_rng(seed)
    alpha = 1.0 / grade - 1.0

    def fwd(xi):
        rr = np.hypot(xi[:, 0], xi[:, 1])
        return xi * (rr ** alpha)[:, None]

    def inside(pts):
        return ((np.abs(pts[:, 0]) < 1) & (np.abs(pts[:, 1]) < 1) & ~((pts[:, 0] > 0) & (pts[:, 1] > 0)))

    corners = np.array([[0.0, 0.0], [0.0, 1.0], [-1.0, 1.0], [-1.0, -1.0], [1.0, -1.0], [1.0, 0.0]])
    rmax = math.sqrt(2.0) ** (1.0 / (1.0 + alpha))
    h = math.sqrt(2.0 * 1.6 / (math.sqrt(3.0) * n_tri / 2.0))
    for _ in range(5):
        ny = int(math.ceil(2 * rmax / (h * math.sqrt(3) / 2))) + 2
        nx = int(math.ceil(2 * rmax / h)) + 2
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        px = -rmax - h + ii * h + (jj % 2) * (h / 2)
        py = -rmax - h + jj * (h * math.sqrt(3) / 2)
        if staggered:
            px = px + h / 2
            py = py + h * math.sqrt(3) / 6
        xi = np.stack([px.ravel(), py.ravel()], axis=1)
        xi = xi + rng.uniform(-0.15 * h, 0.15 * h, size=xi.shape)
        pts = fwd(xi)
        rxi = np.hypot(xi[:, 0], xi[:, 1])
        hloc = h * (1.0 + alpha) * np.maximum(rxi, h) ** alpha  # local size in x
        keep = inside(pts)
        pts, hloc = pts[keep], hloc[keep]
        # distance to the boundary polyline
        dmin = np.full(len(pts), np.inf)
        for k in range(len(corners)):
            p0, p1 = corners[k], corners[(k + 1) % len(corners)]
            d = p1 - p0
            t = np.clip(((pts - p0) @ d) / (d @ d), 0.0, 1.0)
            dmin = np.minimum(dmin, np.hypot(*(pts - (p0 + t[:, None] * d)).T))
        pts = pts[dmin > 0.5 * hloc]
        # boundary points spaced by the local size
        bpts = []
        for k in range(len(corners)):
            p0, p1 = corners[k], corners[(k + 1) % len(corners)]
            L = float(np.hypot(*(p1 - p0)))
            bpts.append(p0)  # corners always belong to the boundary
            rloc = math.hypot(p0[0], p0[1]) ** (1.0 / (1.0 + alpha))
            s = h * (1.0 + alpha) * max(rloc, h) ** alpha * (0.5 if staggered else 1.0)
            while s < L:
                pt = p0 + (p1 - p0) * (s / L)
                rloc = math.hypot(pt[0], pt[1]) ** (1.0 / (1.0 + alpha))
                step = h * (1.0 + alpha) * max(rloc, h) ** alpha
                if L - s > 0.5 * step:
                    bpts.append(pt)
                s += step
        allp = np.concatenate([np.array(bpts), pts])
        dl = Delaunay(allp)
        tri = dl.simplices
        cen = allp[tri].mean(axis=1)
        tri = tri[inside(cen)]
        if abs(len(tri) - n_tri) <= 0.02 * n_tri:
            break
        h *= math.sqrt(len(tri) / n_tri)
    return allp, _ccw(allp, tri)


def l_shape_density(seed):
    """r^(2/3) sin(2 theta'/3) exp(-r^2) + a seeded Gaussian sum, with
    theta' in [0, 3 pi/2] measured from the positive y axis counter-clockwise
    around the domain."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-1, 1, size=(10, 2))
    cen[(cen[:, 0] > 0) & (cen[:, 1] > 0)] *= -1
    amp = rng.uniform(-1, 1, size=10)
    wid = rng.uniform(0.05, 0.3, size=10)

    def f(x, y):
        x = np.asarray(x)
        y = np.asarray(y)
        r = np.hypot(x, y)
        th = np.mod(np.arctan2(y, x) - math.pi / 2, 2 * math.pi)
        sing = r ** (2.0 / 3.0) * np.sin(2.0 * th / 3.0) * np.exp(-r * r)
        g = (amp * np.exp(-((x[..., None] - cen[:, 0]) ** 2 + (y[..., None] - cen[:, 1]) ** 2) / wid)).sum(-1)
        return sing + g

    return f
