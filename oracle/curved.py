"""Curved boundary elements for the oracle (TEST INFRASTRUCTURE ONLY).

A triangle may have one curved side (Sec. 3.1, eq. blend).  Input format,
shared with the library: curved triangle t, its curved side e (the edge
from its local vertex e to local vertex e+1 mod 3, in the order given) and
d+1 points of the side at the Chebyshev-Lobatto parameters
u_i = (1 - cos(pi i / d)) / 2 (u_0 = 0 at local vertex e, u_d = 1 at local
vertex e+1).  gamma(u) is the polynomial through those points.

With B = gamma(0), A = gamma(1) and C the opposite vertex (swapped, with the
curve reversed, if (A, B, C) would be clockwise), the blending map of eq.
blend with the parameter u = 1 - xi in place of the arc length reads

    rho(xi, eta) = A + xi (B - A) + eta (C - A) + ((u - eta) / u) beta(u),
    beta(u) = gamma(u) - (B + u (A - B))      (the side's offset from its chord)

which is affine when the side is straight.  Every step of the method then
runs in the reference simplex (Thm. smooth_int_jac):

  * far rule: nodes rho(xi_j), weights w_j |J(xi_j)|;
  * classification: self if rho^{-1}(x) (Newton) lies in the closed simplex
    up to tau; otherwise near if x is inside the chord triangle or inside
    the chord triangle's three ellipses (the paper's advice to treat the
    curved side as straight), with the weight scale |J| taken as the largest
    |J| at the far nodes;
  * near pairs: the subdivision of Sec. 3.3 in the reference simplex, each
    sub-triangle's vertices mapped by rho for the ellipse test (same |J|
    scale times its reference area) and its near-rule nodes mapped with
    weights w |J|;
  * self pairs (reading: the paper integrates along the true curve in
    physical space; here the same radius-arc-length construction runs in
    the reference simplex about rho^{-1}(x), where
    log|rho(y) - x| = log r + log(|rho(y) - x| / r) splits into the radial
    rule's log part and a smooth remainder), with a radial rule of
    ``radial_curved`` points per part.
"""

import math

import numpy as np
from numpy.polynomial import chebyshev as cheb

from . import rules
from .potential import Oracle, to_reference


def lobatto_params(d):
    """Chebyshev-Lobatto parameters on [0, 1], increasing."""
    return 0.5 * (1.0 - np.cos(np.pi * np.arange(d + 1) / d))


class CurvedOracle(Oracle):
    """Oracle for a mesh with curved boundary triangles.

    curved_tri [n], curved_side [n] (0, 1, 2), curved_pts [n, d+1, 2] as in
    the module docstring; radial_curved = points per part of the radial
    rule on curved self pieces.  Other arguments as ``Oracle``."""

    def __init__(self, vert, tri, curved_tri, curved_side, curved_pts, p, q, eps, radial_curved=12, **kw):
        super().__init__(vert, tri, p, q, eps, **kw)
        vert = np.asarray(vert, dtype=np.float64)
        tri = np.asarray(tri, dtype=np.int64)
        curved_pts = np.asarray(curved_pts, dtype=np.float64)
        d = curved_pts.shape[1] - 1
        s_nodes = 2.0 * lobatto_params(d) - 1.0
        self.curves = {}
        for t, e, P in zip(np.asarray(curved_tri), np.asarray(curved_side), curved_pts):
            t, e = int(t), int(e)
            B, A, C = (vert[tri[t, (e + k) % 3]] for k in range(3))
            P = P.copy()
            if (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]) < 0:
                A, B = B, A
                P = P[::-1]
            self.A[t], self.B[t], self.C[t] = A, B, C
            self.D[t] = (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0])
            cx = cheb.chebfit(s_nodes, P[:, 0], d)
            cy = cheb.chebfit(s_nodes, P[:, 1], d)
            self.curves[t] = (cx, cy, cheb.chebder(cx), cheb.chebder(cy))
        self.rad_c_r, self.rad_c_alpha, self.rad_c_beta = rules.radial_rule(2 * int(radial_curved) - 3)
        self.Deff = self.D.copy()
        self.box = {}
        for t in self.curves:
            self.Deff[t] = self.blend(t, self.far_X)[1].max()
            # box of the element: its vertices and 65 points of its curved side, padded
            u = np.linspace(0.0, 1.0, 65)
            cx, cy = self.curves[t][0], self.curves[t][1]
            pts = np.concatenate([np.stack([cheb.chebval(2 * u - 1, cx), cheb.chebval(2 * u - 1, cy)], 1),
                                  self.C[t][None, :]])
            lo, hi = pts.min(0), pts.max(0)
            pad = 0.05 * (hi - lo).max()
            self.box[t] = (lo - pad, hi + pad)

    # -- the blending map (eq. blend) -----------------------------------------
    def blend_full(self, t, X):
        """rho(X) [n,2] and its partial derivatives d/dxi, d/deta [n,2] for
        reference points X [n,2] with xi < 1."""
        A, B, C = self.A[t], self.B[t], self.C[t]
        cx, cy, dcx, dcy = self.curves[t]
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        xi, eta = X[:, 0], X[:, 1]
        u = 1.0 - xi
        s = 2.0 * u - 1.0
        g = np.stack([cheb.chebval(s, cx), cheb.chebval(s, cy)], 1)
        dg = 2.0 * np.stack([cheb.chebval(s, dcx), cheb.chebval(s, dcy)], 1)
        beta = g - (B[None, :] + u[:, None] * (A - B)[None, :])
        dbeta = dg - (A - B)[None, :]
        f = ((u - eta) / u)[:, None]
        Y = A[None, :] + xi[:, None] * (B - A)[None, :] + eta[:, None] * (C - A)[None, :] + f * beta
        d_eta = (C - A)[None, :] - beta / u[:, None]
        d_xi = (B - A)[None, :] - (eta / (u * u))[:, None] * beta - (1.0 - eta / u)[:, None] * dbeta
        return Y, d_xi, d_eta

    def blend(self, t, X):
        """rho(X) and |J(X)| = det[d rho/d xi, d rho/d eta]."""
        Y, dx, de = self.blend_full(t, X)
        return Y, dx[:, 0] * de[:, 1] - dx[:, 1] * de[:, 0]

    def vertices(self, t, X):
        """Images of reference vertices X [n,2]; the point xi = 1 (vertex B,
        where u = 0) maps to B."""
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        Y = np.empty_like(X)
        at_b = X[:, 0] >= 1.0
        if np.any(~at_b):
            Y[~at_b] = self.blend(t, X[~at_b])[0]
        Y[at_b] = self.B[t]
        return Y

    def inverse(self, t, x, iters=60):
        """rho^{-1}(x) by Newton's method from the chord's affine inverse
        (Sec. 3.1, point location for curved elements); NaNs if it does not
        converge (x far from the element)."""
        x = np.asarray(x, dtype=np.float64)
        z = to_reference(self.A[t], self.B[t], self.C[t], self.D[t], x[None, :])[0].copy()
        with np.errstate(all="ignore"):
            for _ in range(iters):
                z[0] = min(z[0], 1.0 - 1e-12)
                Y, dx, de = self.blend_full(t, z[None, :])
                r = Y[0] - x
                J = dx[0, 0] * de[0, 1] - dx[0, 1] * de[0, 0]
                dz = np.array([(de[0, 1] * r[0] - de[0, 0] * r[1]) / J, (dx[0, 0] * r[1] - dx[0, 1] * r[0]) / J])
                z = z - dz
                if not np.all(np.isfinite(z)):
                    return np.full(2, np.nan)
                if abs(dz[0]) + abs(dz[1]) < 1e-16:
                    return z
        return z if abs(dz[0]) + abs(dz[1]) < 1e-12 else np.full(2, np.nan)

    def in_box(self, t, x):
        lo, hi = self.box[t]
        return bool(np.all(x >= lo) and np.all(x <= hi))

    def node_positions(self, X):
        """Physical positions [T, n, 2] of reference points X in every
        triangle (curved triangles through the blending map)."""
        X = np.asarray(X, dtype=np.float64)
        out = (self.A[:, None, :] + X[None, :, :1] * (self.B - self.A)[:, None, :]
               + X[None, :, 1:2] * (self.C - self.A)[:, None, :])
        for t in self.curves:
            out[t] = self.blend(t, X)[0]
        return out

    # -- far rule (Sec. 3.2 with Thm. smooth_int_jac) -------------------------
    def far_sources(self, c):
        pos, charge = super().far_sources(c)
        nf = self.far_X.shape[0]
        c = np.asarray(c, dtype=np.float64)
        if c.ndim == 2:
            c = c[:, :, None]
        for t in self.curves:
            Y, J = self.blend(t, self.far_X)
            pos[t * nf:(t + 1) * nf] = Y
            fh = self.far_K @ c[t]
            charge[t * nf:(t + 1) * nf] = fh * (self.far_W * J)[:, None]
        return pos, charge

    def far_B(self, t_idx, x):
        if t_idx not in self.curves:
            return super().far_B(t_idx, x)
        Y, J = self.blend(t_idx, self.far_X)
        r2 = (x[0] - Y[:, 0]) ** 2 + (x[1] - Y[:, 1]) ** 2
        keep = r2 > 0.0
        lg = np.zeros_like(r2)
        lg[keep] = 0.5 * np.log(r2[keep])
        return (self.far_W * J * lg) @ self.far_K

    # -- classification ------------------------------------------------------
    def classify_target(self, x):
        x = np.asarray(x, dtype=np.float64)
        base = dict(super().classify_target(x))
        N = 2 * self.q - 1
        for t in self.curves:
            base.pop(t, None)
            z = self.inverse(t, x) if self.in_box(t, x) else np.full(2, np.nan)
            if min(1.0 - z[0] - z[1], z[0], z[1]) >= -self.tau:
                base[t] = 0
                continue
            lam = self.barycentric(t, x)
            P3 = (self.A[t], self.B[t], self.C[t])
            near = lam.min() >= -self.tau
            if not near and self.near_model == "ball":
                near = self.in_ball(x, P3)
            elif not near:
                near = self.in_ellipses(x, P3, self.Deff[t], self.far_what, N)
            if near:
                base[t] = 1
        return sorted(base.items())

    # -- near pairs (Sec. 3.3 in the reference simplex) -----------------------
    def near_A(self, t_idx, x, eps=None):
        if t_idx not in self.curves:
            return super().near_A(t_idx, x, eps)
        x = np.asarray(x, dtype=np.float64)
        Nn = 2 * self.q_near - 1
        leaves = []
        stack = [(np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0]), 0)]
        while stack:
            a, b, c, depth = stack.pop()
            ref_area2 = abs((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
            P3 = self.vertices(t_idx, np.stack([a, b, c]))
            if self.near_model == "ball":
                split = self.in_ball(x, P3)
            else:
                split = self.in_ellipses(x, P3, ref_area2 * self.Deff[t_idx], self.near_what, Nn)
            if depth < self.depth_cap and split:
                mab, mbc, mca = (a + b) / 2, (b + c) / 2, (c + a) / 2
                stack.extend([(a, mab, mca, depth + 1), (mab, b, mbc, depth + 1),
                              (mca, mbc, c, depth + 1), (mbc, mca, mab, depth + 1)])
                continue
            if depth >= self.depth_cap:
                self.n_subdiv_cap_hits += 1
            leaves.append((a, b, c, ref_area2))
        self.stats["near_subtriangles"] += len(leaves)
        Xn, Wn = self.near_X, self.near_W
        xi = np.concatenate([a[None, :] + Xn[:, :1] * (b - a)[None, :] + Xn[:, 1:2] * (c - a)[None, :]
                             for a, b, c, _ in leaves])
        w = np.concatenate([Wn * ra for _, _, _, ra in leaves])
        Y, J = self.blend(t_idx, xi)
        lg = 0.5 * np.log((x[0] - Y[:, 0]) ** 2 + (x[1] - Y[:, 1]) ** 2)
        K = rules.koornwinder(self.p, xi[:, 0], xi[:, 1])
        return (w * J * lg) @ K

    # -- self pairs (reference-simplex radius-arc-length coordinates) ---------
    def self_A(self, t_idx, v):
        if t_idx not in self.curves:
            return super().self_A(t_idx, v)
        x = np.asarray(v, dtype=np.float64)
        z = self.inverse(t_idx, x)
        Pr = (np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0]))
        ys, ws, als, rs = [], [], [], []
        for P, Q in ((Pr[0], Pr[1]), (Pr[1], Pr[2]), (Pr[2], Pr[0])):
            area_sub = 0.5 * abs((P[0] - z[0]) * (Q[1] - z[1]) - (P[1] - z[1]) * (Q[0] - z[0]))
            if area_sub <= self.tau * 0.5:
                continue
            L = math.hypot(Q[0] - P[0], Q[1] - P[1])
            e = (Q - P) / L
            h = abs((P[0] - z[0]) * (Q[1] - P[1]) - (P[1] - z[1]) * (Q[0] - P[0])) / L
            s_t = min(max((z[0] - P[0]) * e[0] + (z[1] - P[1]) * e[1], 0.0), L)
            foot = P + s_t * e
            d = math.hypot(z[0] - foot[0], z[1] - foot[1])
            panels = self.dyadic_panels(s_t, L, d)
            self.stats["self_panels"] += len(panels)
            for s0, s1 in panels:
                s = s0 + (s1 - s0) * self.gl_s
                wsv = (s1 - s0) * self.gl_w
                g = P[None, :] + s[:, None] * e[None, :]
                y = z[None, None, :] + self.rad_c_r[None, :, None] * (g[:, None, :] - z[None, None, :])
                ys.append(y.reshape(-1, 2))
                ws.append((h * wsv[:, None] * np.ones_like(self.rad_c_r)[None, :]).reshape(-1))
                als.append(np.broadcast_to(np.arange(len(self.rad_c_r))[None, :], (len(s), len(self.rad_c_r)))
                           .reshape(-1))
                rs.append(np.broadcast_to(self.rad_c_r[None, :], (len(s), len(self.rad_c_r))).reshape(-1))
        if not ys:
            return np.zeros(self.n_p)
        Yr = np.concatenate(ys)
        w = np.concatenate(ws)
        idx = np.concatenate(als)
        r = np.concatenate(rs)
        Y, J = self.blend(t_idx, Yr)
        alpha, beta = self.rad_c_alpha[idx], self.rad_c_beta[idx]
        # log|rho(y) - x| = log r + smooth: the radial rule's log-weight
        # nodes (beta) take the log r part, its Gauss-Legendre nodes (alpha)
        # the smooth remainder log(|rho(y) - x| / r)
        rem = np.zeros_like(r)
        on = alpha != 0.0
        rem[on] = 0.5 * np.log((Y[on, 0] - x[0]) ** 2 + (Y[on, 1] - x[1]) ** 2) - np.log(r[on])
        coef = w * (alpha * rem + beta) * J
        K = rules.koornwinder(self.p, Yr[:, 0], Yr[:, 1])
        return coef @ K
