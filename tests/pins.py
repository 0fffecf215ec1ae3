"""Independent references that pin the oracle (closed forms and brute force).

None of this uses the oracle's rules or machinery:
  * ``triangle_log_integral``: int_Delta log|x - y| dA_y in closed form.  From
    Laplacian[r^2 (log r - 1) / 4] = log r and the divergence theorem, the
    integral is sum over edges of h_e (2 I_e - l_e) / 4 with h_e the signed
    distance from x to the edge line (outward normal), l_e the edge length and
    I_e = int_e log|x - y| ds = [t log(h^2 + t^2)/2 - t + h atan(t/h)] over
    the edge's coordinate t along it, measured from the foot of x.
  * ``disk_potential``: Newtonian potential of unit density on a disk of
    radius R, (1/2pi) int log|x-y| dA = r^2/4 + (R^2/2) log R - R^2/4 inside
    and (R^2/2) log r outside.
  * ``brute_triangle_integral``: int_Delta log|x - y| g(y) dA by composite
    Gauss-Legendre quadrature in Duffy coordinates about the target (or its
    nearest point on the triangle), with panels graded geometrically toward
    the (near-)singularity.
"""

import math

import numpy as np


def triangle_log_integral(A, B, C, x):
    P = [np.asarray(A, float), np.asarray(B, float), np.asarray(C, float)]
    x = np.asarray(x, float)
    # orient counter-clockwise
    det = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0])
    if det < 0:
        P[1], P[2] = P[2], P[1]
    total = 0.0
    for i in range(3):
        p0, p1 = P[i], P[(i + 1) % 3]
        L = math.hypot(*(p1 - p0))
        t = (p1 - p0) / L
        n = np.array([t[1], -t[0]])
        h = float(np.dot(p0 - x, n))
        t1, t2 = float(np.dot(p0 - x, t)), float(np.dot(p1 - x, t))

        def F(s):
            if h == 0.0:
                return 0.0 if s == 0.0 else s * math.log(abs(s)) - s
            return 0.5 * s * math.log(h * h + s * s) - s + h * math.atan(s / h)

        total += h * (2.0 * (F(t2) - F(t1)) - L) / 4.0
    return total


def mesh_unit_potential(vert, tri, x):
    """(1/2pi) sum over triangles of the closed form: exact potential of unit
    density on the polygonal mesh at x."""
    return sum(triangle_log_integral(vert[a], vert[b], vert[c], x) for a, b, c in tri) / (2 * math.pi)


def disk_potential(R, x):
    r = math.hypot(x[0], x[1])
    if r <= R:
        return r * r / 4.0 + 0.5 * R * R * math.log(R) - R * R / 4.0
    return 0.5 * R * R * math.log(r)


def _graded_panels(center, n_levels=56):
    """Panels of [0, 1] shrinking geometrically (ratio 2) toward center."""
    edges = {0.0, 1.0, center}
    for side_len, sgn in ((center, -1.0), (1.0 - center, 1.0)):
        for k in range(1, n_levels):
            w = side_len * 0.5 ** k
            if w < 1e-17:
                break
            edges.add(center + sgn * w)
    e = np.array(sorted(edges))
    return e[:-1], e[1:]


def _gl_panels(lo, hi, n):
    x, w = np.polynomial.legendre.leggauss(n)
    mid, half = (lo + hi) / 2, (hi - lo) / 2
    return (mid[:, None] + half[:, None] * x[None, :]).ravel(), (half[:, None] * w[None, :]).ravel()


def _duffy_piece(x, c, P, Q, g, n):
    """int over triangle (c, P, Q) of log|y - x| g(y) dA with
    y = c + s (P - c) + s t (Q - P), dA = s |det(P - c, Q - P)| ds dt.
    s-panels graded toward 0 (the target, or its foot point, sits at s = 0);
    t-panels graded toward the foot of c on PQ."""
    jac = abs((P[0] - c[0]) * (Q[1] - P[1]) - (P[1] - c[1]) * (Q[0] - P[0]))
    if jac == 0.0:
        return 0.0
    qp = Q - P
    tstar = min(max(-np.dot(P - c, qp) / np.dot(qp, qp), 0.0), 1.0)
    s, ws = _gl_panels(*_graded_panels(0.0), n)
    t, wt = _gl_panels(*_graded_panels(tstar, 30), n)
    S, Tt = np.meshgrid(s, t, indexing="ij")
    Wt = np.outer(ws, wt)
    y0 = c[0] + S * (P[0] - c[0]) + S * Tt * qp[0]
    y1 = c[1] + S * (P[1] - c[1]) + S * Tt * qp[1]
    r2 = (y0 - x[0]) ** 2 + (y1 - x[1]) ** 2
    with np.errstate(divide="ignore"):
        lg = np.where(r2 > 0, 0.5 * np.log(np.where(r2 > 0, r2, 1.0)), 0.0)
    gv = np.asarray(g(y0.ravel(), y1.ravel()))
    gv = gv.reshape(y0.shape + gv.shape[1:])
    wl = (Wt * S * jac * lg).reshape(y0.shape + (1,) * (gv.ndim - 2))
    return np.sum(wl * gv, axis=(0, 1))


def _closest_point(A, B, C, x):
    best, bd = None, np.inf
    for P, Q in ((A, B), (B, C), (C, A)):
        d = Q - P
        t = min(max(np.dot(x - P, d) / np.dot(d, d), 0.0), 1.0)
        y = P + t * d
        dist = np.hypot(*(x - y))
        if dist < bd:
            best, bd = y, dist
    return best


def brute_triangle_integral(A, B, C, x, g, inside, n=20):
    """int_Delta log|x - y| g(y) dA by composite Gauss-Legendre in Duffy
    coordinates about a centre c: c = x when x is in the closed triangle,
    else the point of the triangle nearest x.  The triangle is split at c;
    every piece has c as a vertex, where the (near-)singularity sits, and
    the panels are graded toward it.  g(y0, y1) must be vectorised; it may
    return [n] (scalar integrand) or [n, m] (m integrands at once)."""
    A, B, C, x = (np.asarray(z, float) for z in (A, B, C, x))
    c = x if inside else _closest_point(A, B, C, x)
    area = 0.5 * abs((B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]))
    total = 0.0
    for P, Q in ((A, B), (B, C), (C, A)):
        sub = 0.5 * abs((P[0] - c[0]) * (Q[1] - c[1]) - (P[1] - c[1]) * (Q[0] - c[0]))
        if sub <= 1e-15 * area:
            continue
        total += _duffy_piece(x, c, P, Q, g, n)
    return total
