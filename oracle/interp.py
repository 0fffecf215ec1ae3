"""Interpolation of the potential over a mesh element (Sec. 3.5) for the
oracle (TEST INFRASTRUCTURE ONLY).

Given u at the order-p interpolation nodes of every triangle of a mesh, u at
a point x is sum_k c_k K_k(rho^{-1}(x)) with c = V^{-1} u of the triangle
containing x: point location by testing every triangle (the lowest index
whose closure contains x, barycentric tolerance 1e-13; Newton's method on a
curved triangle), then the interpolation matrix and the Koornwinder basis.
"""

import numpy as np

from . import rules
from .potential import to_reference

TAU = 1e-13


def locate(o, x):
    """(triangle, rho^{-1}(x)) for the mesh of oracle o (an Oracle or a
    CurvedOracle); (-1, (0, 0)) if no triangle contains x."""
    x = np.asarray(x, dtype=np.float64)
    e1 = o.B - o.A
    e2 = o.C - o.A
    d = x[None, :] - o.A
    z1 = (d[:, 0] * e2[:, 1] - d[:, 1] * e2[:, 0]) / o.D
    z2 = (e1[:, 0] * d[:, 1] - e1[:, 1] * d[:, 0]) / o.D
    inside = np.minimum(np.minimum(1.0 - z1 - z2, z1), z2) >= -TAU
    curves = getattr(o, "curves", {})
    for t in curves:
        inside[t] = False
    best, ref = -1, np.zeros(2)
    hits = np.nonzero(inside)[0]
    if len(hits):
        best = int(hits[0])
        ref = np.array([z1[best], z2[best]])
    for t in sorted(curves):
        if best >= 0 and t > best:
            break
        if not o.in_box(t, x):
            continue
        z = o.inverse(t, x)
        if np.all(np.isfinite(z)) and min(1.0 - z[0] - z[1], z[0], z[1]) >= -TAU:
            best, ref = t, z
            break
    return best, ref


def evaluate(p, u_nodes, t, ref):
    """sum_k c_k K_k(ref), c = V^{-1} u_nodes[t] (u_nodes [T, n_p] or
    [T, n_p, R])."""
    u = np.asarray(u_nodes, dtype=np.float64)
    c = rules.vandermonde_inverse(p) @ u[t]
    K = rules.koornwinder(p, np.array([ref[0]]), np.array([ref[1]]))[0]
    return K @ c


def interpolate(o, p, u_nodes, points):
    """u at every point [n] (or [n, R]); NaN outside the mesh."""
    out = []
    for x in np.asarray(points, dtype=np.float64).reshape(-1, 2):
        t, z = locate(o, x)
        if t < 0:
            u = np.asarray(u_nodes)
            out.append(np.full(u.shape[2:] if u.ndim == 3 else (), np.nan))
        else:
            out.append(evaluate(p, u_nodes, t, z))
    return np.array(out)
