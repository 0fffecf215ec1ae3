"""Pins for the oracle evaluator against closed forms, brute force and
invariances.  Each check targets a part of the oracle where a plausible
mistake (a dropped term, a wrong sign, a wrong index or panel) would show."""

import math

import numpy as np
import pytest

import pins
from oracle import potential, rules
from paper_2205_04401_amd import workloads as W

SQRT2 = math.sqrt(2.0)

TRIANGLES = {
    "regular": np.array([[0.0, 0.0], [1.0, 0.0], [0.3, 0.8]]),
    "small": np.array([[0.2, 0.1], [0.23, 0.1], [0.21, 0.125]]),
    "stretched": np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 0.12]]),
    "clockwise": np.array([[0.0, 0.0], [0.3, 0.8], [1.0, 0.0]]),
}


def one_triangle(name, p=3, q=8, eps=1e-13):
    v = TRIANGLES[name]
    return potential.Oracle(v, np.array([[0, 1, 2]]), p, q, eps), v


def sample_points(v, rng, n):
    """Targets inside, on edges, at vertices and just outside."""
    A, B, C = v
    pts = [A, B, C, (A + B) / 2, (B + C) / 2, 0.3 * A + 0.7 * C]
    bc = rng.dirichlet([1, 1, 1], size=n)
    pts += list(bc @ v)
    cen = v.mean(0)
    size = max(np.hypot(*(B - A)), np.hypot(*(C - B)), np.hypot(*(A - C)))
    for d in (1e-9, 1e-5, 1e-2, 0.1, 0.4):
        for e0, e1 in ((A, B), (B, C), (C, A)):
            m = 0.37 * e0 + 0.63 * e1
            out = m + (m - cen) / np.hypot(*(m - cen)) * d * size
            pts.append(out)
    pts.append(A + (A - cen) * 0.05)
    return [np.asarray(p_, float) for p_ in pts]


# -- P2: A_0 against the closed-form integral of log over a triangle --------

@pytest.mark.parametrize("name", list(TRIANGLES))
def test_A0_matches_closed_form(name):
    o, v = one_triangle(name)
    rng = np.random.default_rng(3)
    for x in sample_points(v, rng, 6):
        exact = pins.triangle_log_integral(*v, x)
        cls = o.classify_target(x)
        kind = cls[0][1] if cls else 2
        if kind == 0:
            got = o.self_A(0, x)[0] / SQRT2
        elif kind == 1:
            got = o.near_A(0, x)[0] / SQRT2
        else:
            got = o.far_B(0, x)[0] / SQRT2
        # eps is an absolute tolerance per interaction (Sec. 4.1, eq.
        # precise_far); a near pair sums many sub-triangles, each within eps,
        # and a stretched triangle's ellipse union is slightly too small
        # (Sec. 4.1, the stretched-triangle caveat): allow 4 eps.
        assert abs(got - exact) <= 4 * o.eps, (name, x, kind)


# -- P6: all A_k against mpmath brute force ---------------------------------

@pytest.mark.parametrize("case", ["inside", "edge", "vertex", "near", "near_close", "near_far"])
def test_Ak_brute_force(case):
    p = 3
    o, v = one_triangle("regular", p=p)
    A, B, C = v
    nrm = np.array([C[1] - B[1], B[0] - C[0]])
    nrm /= np.hypot(*nrm)
    nrm *= -np.sign(np.dot(nrm, v.mean(0) - B))
    x = {"inside": np.array([0.41, 0.27]), "edge": (A + B) * 0.5 + np.array([0.07, 0.0]),
         "vertex": C.copy(), "near": np.array([0.5, -0.06]),
         "near_close": 0.6 * B + 0.4 * C + 1e-3 * nrm,
         "near_far": 0.6 * B + 0.4 * C + 0.3 * nrm}[case]
    cls = o.classify_target(x)
    kind = cls[0][1]
    assert kind == (0 if case in ("inside", "edge", "vertex") else 1)
    got = o.self_A(0, x) if kind == 0 else o.near_A(0, x)
    e1, e2, D = B - A, C - A, o.D[0]

    def g(y0, y1):
        d0, d1 = y0 - A[0], y1 - A[1]
        xi1 = (d0 * e2[1] - d1 * e2[0]) / D
        xi2 = (e1[0] * d1 - e1[1] * d0) / D
        return rules.koornwinder(p, xi1, xi2)

    ref = pins.brute_triangle_integral(A, B, C, x, g, inside=(kind == 0))
    assert np.abs(got - ref).max() < 4 * o.eps, (case, got, ref)


# -- P3: end-to-end, unit density, polygon closed form ----------------------

def c1_problem(p=4, q=8, eps=1e-13):
    vq, tq = W.unit_square(8, "/")
    vt, tt = W.unit_square(8, "\\")
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    return vq, tq, tg, nodes


def test_unit_square_unit_density_matches_polygon_closed_form():
    vq, tq, tg, nodes = c1_problem()
    rng = np.random.default_rng(5)
    sel = rng.choice(len(tg), 240, replace=False)
    F = np.ones((len(tq), rules.n_basis(4)))
    o = potential.Oracle(vq, tq, 4, 8, 1e-13)
    u = o.evaluate(F, tg[sel])
    ex = np.array([pins.mesh_unit_potential(vq, tq, x) for x in tg[sel]])
    assert np.abs(u - ex).max() <= 1e-12 * np.abs(ex).max()


def test_far_only_differs_and_corrections_matter():
    """The far rule alone is visibly wrong near the mesh; the corrections fix
    it (guards against a correction that is silently zero)."""
    vq, tq, tg, nodes = c1_problem()
    F = np.ones((len(tq), rules.n_basis(4)))
    o = potential.Oracle(vq, tq, 4, 8, 1e-13)
    x = tg[:40]
    u_far = o.evaluate(F, x, far_only=True)
    ex = np.array([pins.mesh_unit_potential(vq, tq, t) for t in x])
    assert np.abs(u_far - ex).max() > 1e-6


# -- P4: disk closed form ----------------------------------------------------

def test_naive_ball_model_converges_to_the_exact_integral():
    """The naive near field (a ball of kappa times the centroid radius, the
    paper's comparison setting) reaches the exact integral only as kappa
    grows, and at far more sub-triangles than the Bernstein ellipses need
    for a smaller error (Sec. 4.1, Remark rem:near_zero)."""
    vq, tq = W.unit_square(4, "/")
    rng = np.random.default_rng(5)
    tg = rng.uniform(-0.2, 1.2, (40, 2))
    exact = np.array([pins.mesh_unit_potential(vq, tq, x) for x in tg])
    F = np.ones((len(tq), rules.n_basis(1)))
    errs, subs = [], []
    for kappa in (1.0, 2.0, 3.0, 5.0):
        o = potential.Oracle(vq, tq, 1, 4, 1e-12, near_model="ball", ball_factor=kappa)
        errs.append(np.abs(o.evaluate(F, tg) - exact).max() / np.abs(exact).max())
        subs.append(o.stats["near_subtriangles"])
    assert all(b < 0.2 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[0] > 1e-7 and errs[-1] < 1e-10
    o = potential.Oracle(vq, tq, 1, 4, 1e-12)
    e_ell = np.abs(o.evaluate(F, tg) - exact).max() / np.abs(exact).max()
    assert e_ell < 1e-12 and e_ell < errs[-1]
    assert o.stats["near_subtriangles"] < subs[-1] / 4


def test_disk_unit_density_polygon_exact_and_circle_converges():
    R = 1.0
    rng = np.random.default_rng(2)
    radii = np.array([0.0, 0.3, 0.77, 1.6, 3.0])
    ang = rng.uniform(0, 2 * math.pi, size=len(radii))
    tgt = np.stack([radii * np.cos(ang), radii * np.sin(ang)], 1)
    errs_circle = []
    for nb, nt in ((24, 120), (48, 480)):
        v, t = W.disk_mesh(n_tri=nt, n_boundary=nb, seed=1, radius=R)
        o = potential.Oracle(v, t, 2, 6, 1e-13)
        u = o.evaluate(np.ones((len(t), 6)), tgt)
        poly = np.array([pins.mesh_unit_potential(v, t, x) for x in tgt])
        assert np.abs(u - poly).max() < 1e-12
        circ = np.array([pins.disk_potential(R, x) for x in tgt])
        errs_circle.append(np.abs(u - circ).max())
    rate = math.log(errs_circle[0] / errs_circle[1]) / math.log(2.0)
    assert 1.7 < rate < 2.3, errs_circle


def test_disk_golden_values_from_paper():
    """The paper's unit-disk check (Sec. 5.1.1): u = (|x|^2 - 1)/4 inside.
    The fixture holds values of that formula; the closed form used by the
    other pins must reproduce them, and the oracle on a fine polygonal disk
    must approach them within the inscribed polygon's area deficit."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "unit_disk_potential.txt")
    rows = np.loadtxt(path, comments="#")
    for r, u in rows:
        assert abs(pins.disk_potential(1.0, (r, 0.0)) - u) < 1e-15
    v, t = W.disk_mesh(n_tri=480, n_boundary=48, seed=1)
    o = potential.Oracle(v, t, 2, 6, 1e-13)
    pts = np.stack([rows[:, 0], np.zeros(len(rows))], 1)
    got = o.evaluate(np.ones((len(t), 6)), pts)
    deficit = math.pi - W.polygon_area(v, t)
    assert np.abs(got - rows[:, 1]).max() < 2.0 * deficit


# -- P5: far-field asymptote -------------------------------------------------

def test_far_field_asymptote():
    vq, tq, tg, nodes = c1_problem(p=4)
    f = W.gaussian_bump
    F = W.sample_density(f, vq, tq, nodes)
    o = potential.Oracle(vq, tq, 4, 8, 1e-13)
    c = o.coefficients(F)
    mass = float(np.sum(o.D * c[:, 0]) / SQRT2)
    # first moment of the interpolant, with the far rule (exact: degree p+1)
    pos, charge = o.far_sources(c)
    dip = (pos * charge).sum(0)
    for R in (1e2, 1e3, 1e5):
        x = np.array([R * 0.6, R * 0.8])
        u = o.evaluate(F, x[None, :])[0]
        pred = (mass * math.log(R) - np.dot(x, dip) / R ** 2) / (2 * math.pi)
        assert abs(u - pred) < 5.0 / R ** 2 + 1e-13 * abs(pred), R


# -- P7: invariances ---------------------------------------------------------

def small_star():
    v, t = W.star_mesh(n_tri=300, n_boundary=40, seed=7)
    vt, tt = W.star_mesh(n_tri=300, n_boundary=40, seed=8, staggered=True)
    return v, t, vt, tt


def test_translation_rotation_invariance_and_linearity():
    v, t, vt, tt = small_star()
    p, q = 3, 6
    nodes = rules.interp_nodes(p)
    rng = np.random.default_rng(0)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)[rng.choice(len(tt) * 10, 60, replace=False)]
    f1 = W.gaussian_sum(1, v, t)
    f2 = W.gaussian_sum(2, v, t)
    F = np.stack([W.sample_density(f1, v, t, nodes), W.sample_density(f2, v, t, nodes)], -1)
    o = potential.Oracle(v, t, p, q, 1e-12)
    u = o.evaluate(F, tg)
    # translation
    sh = np.array([1e3, -1e3])
    u_t = potential.Oracle(v + sh, t, p, q, 1e-12).evaluate(F, tg + sh)
    assert np.abs(u_t - u).max() <= 1e-9 * np.abs(u).max()
    # rotation
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    u_r = potential.Oracle(v @ Rm.T, t, p, q, 1e-12).evaluate(F, tg @ Rm.T)
    assert np.abs(u_r - u).max() <= 1e-11 * np.abs(u).max()
    # linearity and column independence
    u1 = o.evaluate(F[..., 0], tg)
    u2 = o.evaluate(2.0 * F[..., 1] - F[..., 0], tg)
    assert np.abs(u1 - u[:, 0]).max() <= 1e-14 * np.abs(u).max()
    assert np.abs(u2 - (2 * u[:, 1] - u[:, 0])).max() <= 1e-13 * np.abs(u).max()


def test_scaling_law():
    """u_lambda(lambda x) = lambda^2 [u(x) + (M / 2pi) log lambda]."""
    v, t, vt, tt = small_star()
    p, q = 2, 6
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)[::23]
    F = W.sample_density(W.gaussian_sum(3, v, t), v, t, nodes)
    o = potential.Oracle(v, t, p, q, 1e-13)
    u = o.evaluate(F, tg)
    mass = float(np.sum(o.D * o.coefficients(F)[:, 0]) / SQRT2)
    lam = 3.0
    u_l = potential.Oracle(lam * v, t, p, q, 1e-13).evaluate(F, lam * tg)
    pred = lam ** 2 * (u + mass * math.log(lam) / (2 * math.pi))
    assert np.abs(u_l - pred).max() <= 1e-11 * np.abs(pred).max()


# -- P8: polynomial reproduction end to end ---------------------------------

@pytest.mark.slow
def test_polynomial_density_end_to_end_brute_force():
    """For f in P_p the interpolant is f itself; u then equals the exact
    potential of f, computed here by brute force triangle by triangle."""
    vert = np.array([[0.0, 0.0], [1.0, 0.1], [0.2, 0.9], [1.1, 1.0]])
    tri = np.array([[0, 1, 2], [1, 3, 2]])
    p = 2
    nodes = rules.interp_nodes(p)

    def f(x, y):
        return 1.0 + x - 0.5 * y + 0.7 * x * y - y * y

    F = W.sample_density(f, vert, tri, nodes)
    o = potential.Oracle(vert, tri, p, 6, 1e-14)
    targets = np.array([[0.4, 0.3], [0.6, 0.55], [1.2, 0.2], [0.5, -0.02], [-0.3, 0.5], [3.0, 2.0]])
    u = o.evaluate(F, targets)
    for i, x in enumerate(targets):
        ref = 0.0
        for tr in tri:
            A, B, C = vert[tr]
            lam = np.linalg.solve(np.array([[B[0] - A[0], C[0] - A[0]], [B[1] - A[1], C[1] - A[1]]]), x - A)
            inside = lam.min() >= 0 and lam.sum() <= 1
            ref += pins.brute_triangle_integral(A, B, C, x, f, inside)
        assert abs(u[i] - ref / (2 * math.pi)) < 1e-13, (x, u[i], ref / (2 * math.pi))


# -- P9: containment of the far field ---------------------------------------

@pytest.mark.parametrize("q,eps", [(4, 1e-10), (8, 1e-13), (8, 1e-10), (12, 1e-13)])
def test_far_pairs_meet_tolerance(q, eps):
    """Every target the classification calls far gets the far rule's value of
    int log within 2 eps (unit density; exact value by the closed form)."""
    v = TRIANGLES["regular"] * 0.1
    o = potential.Oracle(v, np.array([[0, 1, 2]]), 2, q, eps)
    rng = np.random.default_rng(q)
    worst = 0.0
    g = np.linspace(-0.12, 0.22, 69)
    for x0 in g:
        for y0 in g:
            x = np.array([x0, y0]) + rng.uniform(-1e-3, 1e-3, 2)
            if o.classify_target(x):
                continue
            err = abs(o.far_B(0, x)[0] / SQRT2 - pins.triangle_log_integral(*v, x))
            worst = max(worst, err)
    assert worst <= 2.0 * eps, worst


def test_near_field_shrinks_with_order():
    """Sec. 4.2: the ellipse-union near field shrinks as the far order grows."""
    v = TRIANGLES["regular"]
    g = np.linspace(-1.0, 2.0, 61)
    counts = []
    for q in (4, 8, 12, 16, 20):
        o = potential.Oracle(v, np.array([[0, 1, 2]]), 2, q, 1e-12)
        counts.append(sum(1 for a in g for b in g if any(k == 1 for _, k in o.classify_target(np.array([a, b])))))
    assert all(counts[i] > counts[i + 1] for i in range(len(counts) - 1)), counts


# -- P10: self machinery converged -----------------------------------------

def test_self_rows_converged_in_panel_order():
    v = TRIANGLES["stretched"]
    base = potential.Oracle(v, np.array([[0, 1, 2]]), 4, 8, 1e-13)
    fine = potential.Oracle(v, np.array([[0, 1, 2]]), 4, 8, 1e-13, n_l=30)
    for x in (np.array([0.5, 0.05]), np.array([0.5, 1e-7]), np.array([0.99, 0.002]), v[2]):
        a, b = base.self_A(0, x), fine.self_A(0, x)
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max(), x


# -- planted mistakes: each must break at least one pin ----------------------

def test_planted_mistakes_are_caught(monkeypatch):
    v = TRIANGLES["regular"]
    x_in = np.array([0.41, 0.27])
    x_near = np.array([0.5, -0.05])
    exact_in = pins.triangle_log_integral(*v, x_in)
    exact_near = pins.triangle_log_integral(*v, x_near)

    def a0(o, x, kind):
        return (o.self_A(0, x) if kind == 0 else o.near_A(0, x))[0] / SQRT2

    o, _ = one_triangle("regular")
    assert abs(a0(o, x_in, 0) - exact_in) < 1e-14
    assert abs(a0(o, x_near, 1) - exact_near) < 1e-14
    # 1) dropped log r0 term of the radial rule
    o1, _ = one_triangle("regular")
    o1.rad_alpha = o1.rad_alpha * 0.0
    assert abs(a0(o1, x_in, 0) - exact_in) > 1e-6
    # 2) the last dyadic panel (the one next to the foot point) dropped
    orig = potential.Oracle.dyadic_panels
    o2, _ = one_triangle("regular")
    monkeypatch.setattr(potential.Oracle, "dyadic_panels",
                        lambda self, s, L, d: orig(self, s, L, d)[:-1] or orig(self, s, L, d))
    assert abs(a0(o2, x_in, 0) - exact_in) > 1e-6
    monkeypatch.setattr(potential.Oracle, "dyadic_panels", orig)
    # 3) near rule never subdivides (ellipse test ignored)
    o3, _ = one_triangle("regular")
    monkeypatch.setattr(o3, "in_ellipses", lambda *a, **k: False)
    assert abs(a0(o3, x_near, 1) - exact_near) > 1e-9
    # 4) area scaling of w forgotten (rho from the reference weight alone):
    #    on a large triangle the ellipses become too small and far pairs
    #    miss the tolerance
    big = v * 6.0
    o4 = potential.Oracle(big, np.array([[0, 1, 2]]), 2, 8, 1e-13)
    o4.far_what = o4.far_what / o4.D[0]
    worst = 0.0
    for a in np.linspace(-10.0, 16.0, 40):
        for b in np.linspace(-10.0, 14.0, 37):
            x = np.array([a, b])
            if o4.classify_target(x):
                continue
            worst = max(worst, abs(o4.far_B(0, x)[0] / SQRT2 - pins.triangle_log_integral(*big, x)))
    assert worst > 2 * o4.eps


# ---------------------------------------------------------------------------
# curved boundary elements (Sec. 3.1, eq. blend)
# ---------------------------------------------------------------------------

def _disk_targets(seed=2):
    rng = np.random.default_rng(seed)
    r = np.concatenate([rng.uniform(0, 0.99, 6), [1.0, 1.0], rng.uniform(1.01, 3, 4), [0.995, 1.005]])
    a = rng.uniform(0, 2 * math.pi, len(r))
    return r, np.stack([r * np.cos(a), r * np.sin(a)], 1)


def test_curved_disk_area_and_unit_density_closed_form():
    """Boundary triangles with circular sides: the far rule integrates the
    disk's area, and unit density reproduces u = r^2/4 - 1/4 inside,
    (1/2) log r outside (the disk closed form, R = 1) to rounding, at
    targets inside, outside and on the circle."""
    from oracle import curved
    v, t, ct, cs, cp = W.curved_disk(n_tri=200, n_boundary=30, seed=1, deg=16)
    o = curved.CurvedOracle(v, t, ct, cs, cp, 1, 8, 1e-12)
    F = np.ones((len(t), rules.n_basis(1)))
    _, charge = o.far_sources(o.coefficients(F))
    assert abs(charge.sum() - math.pi) < 1e-14
    r, tg = _disk_targets()
    exact = np.where(r <= 1, r ** 2 / 4 - 0.25, 0.5 * np.log(r))
    u = o.evaluate(F, tg)
    assert np.abs(u - exact).max() < 1e-12 * np.abs(exact).max()


def test_curved_disk_r2_density_converges_to_closed_form():
    """f = r^2 on the curved disk: u = r^4/16 - 1/16 inside, (1/4) log r
    outside.  f composed with the blending map is not a polynomial, so the
    error is the interpolant's, falling with p."""
    from oracle import curved
    v, t, ct, cs, cp = W.curved_disk(n_tri=200, n_boundary=30, seed=1, deg=16)
    r, tg = _disk_targets(3)
    exact = np.where(r <= 1, r ** 4 / 16 - 1 / 16, 0.25 * np.log(r))
    errs = []
    for p in (4, 6, 8):
        o = curved.CurvedOracle(v, t, ct, cs, cp, p, 8, 1e-13)
        Y = o.node_positions(rules.interp_nodes(p))
        u = o.evaluate(Y[:, :, 0] ** 2 + Y[:, :, 1] ** 2, tg)
        errs.append(np.abs(u - exact).max() / np.abs(exact).max())
    assert errs[0] < 1e-8 and errs[1] < 1e-12 and errs[2] < 1e-13 and errs[2] < errs[0] / 1e4, errs


def test_curved_map_inverse_round_trip_and_straight_limit():
    """Newton inversion undoes the blending map; with every 'curved' side
    placed on its chord the curved oracle equals the straight one."""
    from oracle import curved
    v, t, ct, cs, cp = W.curved_disk(n_tri=120, n_boundary=24, seed=4, deg=10)
    o = curved.CurvedOracle(v, t, ct, cs, cp, 3, 6, 1e-12)
    rng = np.random.default_rng(9)
    X = rng.dirichlet([1, 1, 1], 20)[:, 1:]
    for tc in list(o.curves)[:5]:
        Y = o.blend(tc, X)[0]
        Z = np.array([o.inverse(tc, y) for y in Y])
        assert np.abs(Z - X).max() < 1e-13
    # straight limit: points on the chords
    u01 = curved.lobatto_params(cp.shape[1] - 1)
    flat = np.array([[v[t[k, e]] + s * (v[t[k, (e + 1) % 3]] - v[t[k, e]]) for s in u01] for k, e in zip(ct, cs)])
    of = curved.CurvedOracle(v, t, ct, cs, flat, 3, 6, 1e-12)
    os_ = potential.Oracle(v, t, 3, 6, 1e-12)
    # a global cubic, reproduced exactly by both interpolants (each samples
    # it at its own node positions: a curved triangle orders its vertices
    # from its curved side)
    X = rules.interp_nodes(3)

    def f(Y):
        x, y = Y[..., 0], Y[..., 1]
        return 1.0 + x + 2.0 * y * y - x * y + x ** 3

    Ys = os_.A[:, None, :] + X[None, :, :1] * (os_.B - os_.A)[:, None, :] + X[None, :, 1:2] * (os_.C - os_.A)[:, None, :]
    _, tg = _disk_targets(5)
    ref = os_.evaluate(f(Ys), tg)
    assert np.abs(of.evaluate(f(of.node_positions(X)), tg) - ref).max() < 1e-12 * np.abs(ref).max()



# ---------------------------------------------------------------------------
# interpolation of the potential over a mesh element (Sec. 3.5)
# ---------------------------------------------------------------------------

def test_interpolation_reproduces_polynomials_and_marks_outside_points():
    """A global cubic given at the p = 3 nodes of every triangle is
    reproduced exactly anywhere in the mesh; points outside give NaN."""
    from oracle import interp
    v, t = W.disk_mesh(n_tri=120, n_boundary=24, seed=4)
    o = potential.Oracle(v, t, 3, 4, 1e-10)
    X = rules.interp_nodes(3)
    Y = o.A[:, None, :] + X[None, :, :1] * (o.B - o.A)[:, None, :] + X[None, :, 1:2] * (o.C - o.A)[:, None, :]

    def g(x, y):
        return 1.0 - 2.0 * x + x * y + 3.0 * y ** 3 - x * x * y

    rng = np.random.default_rng(8)
    r, a = np.sqrt(rng.uniform(0, 0.9, 30)), rng.uniform(0, 2 * math.pi, 30)
    pts = np.stack([r * np.cos(a), r * np.sin(a)], 1)
    u = interp.interpolate(o, 3, g(Y[..., 0], Y[..., 1]), pts)
    assert np.abs(u - g(pts[:, 0], pts[:, 1])).max() < 1e-13
    assert np.all(np.isnan(interp.interpolate(o, 3, g(Y[..., 0], Y[..., 1]), [[2.0, 0.0], [0.0, -1.5]])))


def test_interpolation_boundary_trace_on_curved_sides():
    """Remark rem:bndry_interp: the point gamma(u) of a curved side lies at
    reference point (1 - u, 0) of its triangle (the side runs from B at
    u = 0 to A at u = 1); point location by Newton's method finds it there,
    and a polynomial in reference coordinates is reproduced."""
    from oracle import curved, interp
    from numpy.polynomial import chebyshev as cheb
    v, t, ct, cs, cp = W.curved_disk(n_tri=120, n_boundary=24, seed=4, deg=12)
    o = curved.CurvedOracle(v, t, ct, cs, cp, 4, 6, 1e-10)
    X = rules.interp_nodes(4)
    g = lambda a, b: 0.5 + a - 2.0 * b + a * b * b + a ** 4  # noqa: E731
    un = np.broadcast_to(g(X[:, 0], X[:, 1])[None, :], (len(t), len(X)))
    rng = np.random.default_rng(13)
    worst_ref = worst_val = 0.0
    for tc in list(o.curves)[:8]:
        cx, cy = o.curves[tc][0], o.curves[tc][1]
        for uu in rng.uniform(0.05, 0.95, 3):
            x = np.array([cheb.chebval(2 * uu - 1, cx), cheb.chebval(2 * uu - 1, cy)])
            tt, z = interp.locate(o, x)
            assert tt == tc
            worst_ref = max(worst_ref, abs(z[0] - (1 - uu)) + abs(z[1]))
            worst_val = max(worst_val, abs(interp.evaluate(4, un, tt, z) - g(1 - uu, 0.0)))
    assert worst_ref < 1e-12 and worst_val < 1e-11
