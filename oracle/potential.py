"""The oracle evaluator (TEST INFRASTRUCTURE ONLY; see package doc).

Computes, for targets x_t and a density given by its values at the
interpolation nodes of every triangle,

    u(x_t) = (1/2pi) sum_Delta int_Delta log|x_t - y| f_h(y) dA_y

where f_h is the per-triangle degree-p interpolant of the density (Sec. 3.5
map applied to the density), with the method of the paper:

  * far field: every far-rule node of every triangle is a point charge
    (Sec. 3.6, first step), summed directly over all targets;
  * classification of each (target, triangle) pair into self / near / far
    (Def. of far/near field in Sec. 3.2; near field = union of three
    Bernstein ellipses, Sec. 4.1, eqs. rho0 and threeE);
  * subtract-and-add (Sec. 3.6): for each self or near pair, remove the far
    rule's contribution B and add the accurate integral A, where A comes from
    adaptive subdivision for near pairs (Sec. 3.3, eq. sum_near, with the
    Sec. 4.1 ellipse test deciding every split) and from radius-arc-length
    coordinates with dyadic arc-length panels for self pairs (Sec. 3.4, eq.
    volpot_self_single).

All arithmetic is float64 (sums over many terms accumulate in extended
precision).  Readings of points the paper leaves open are stated where they
are used.
"""

import math

import numpy as np

from . import rules

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# Geometry (Sec. 3.1: the affine map of a triangle)
# ----------------------------------------------------------------------------

def orient(vert, tri):
    """Return (A, B, C, D) for every triangle with counter-clockwise vertex
    order.  D = det[B-A, C-A] = |J| = 2 area.  A triangle stored clockwise has
    its local vertices 1 and 2 swapped (reading: this fixes which vertex the
    collapsed rules collapse onto, vertex B)."""
    vert = np.asarray(vert, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64).copy()
    A, B, C = vert[tri[:, 0]], vert[tri[:, 1]], vert[tri[:, 2]]
    D = (B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (B[:, 1] - A[:, 1]) * (C[:, 0] - A[:, 0])
    flip = D < 0
    B2 = np.where(flip[:, None], C, B)
    C2 = np.where(flip[:, None], B, C)
    return A, B2, C2, np.abs(D)


def to_physical(A, B, C, X):
    """rho(xi) = A + xi_1 (B - A) + xi_2 (C - A) for reference points X [n,2]
    and one triangle (A, B, C as length-2 arrays)."""
    return A[None, :] + X[:, :1] * (B - A)[None, :] + X[:, 1:2] * (C - A)[None, :]


def to_reference(A, B, C, D, Y):
    """Inverse affine map for one triangle: reference coordinates of Y [n,2]."""
    e1, e2 = B - A, C - A
    d = Y - A[None, :]
    xi1 = (d[:, 0] * e2[1] - d[:, 1] * e2[0]) / D
    xi2 = (e1[0] * d[:, 1] - e1[1] * d[:, 0]) / D
    return np.stack([xi1, xi2], axis=1)


# ----------------------------------------------------------------------------
# The evaluator
# ----------------------------------------------------------------------------

class Oracle:
    """Plain evaluator for one (mesh, p, q, eps) problem.

    Parameters mirror the paper's notation: p = interpolation order of the
    density, q = points per direction of the far rule (exact through total
    degree N = 2q - 1), eps = tolerance of the far/near rules, c_n = the
    constant C_N of eq. rho0 (reading: 1 for the collapsed Gauss rules, whose
    C_N the paper does not tabulate), q_near = points per direction of the
    rule used on sub-triangles (N_n = 2 q_near - 1), n_l = Gauss-Legendre
    points per arc-length panel, tau = barycentric tolerance of the self test.
    near_model = "ellipse" (the union of Bernstein ellipses, Sec. 4.1) or
    "ball" (the naive near field the paper compares against, the opening of Sec. 4 and
    the superscript-0 setting of Table near_corr): a target is near a
    triangle, and a sub-triangle is split, when the target lies within
    ball_factor times R of the centroid c, R = the largest vertex distance
    from c (reading: the paper tunes the ball's size, not its shape).
    """

    def __init__(self, vert, tri, p, q, eps, c_n=1.0, q_near=7, n_l=16, tau=1e-13,
                 depth_cap=50, dyadic_cap=60, near_model="ellipse", ball_factor=2.0):
        if near_model not in ("ellipse", "ball"):
            raise ValueError("near_model must be 'ellipse' or 'ball'")
        self.near_model, self.ball_factor = near_model, float(ball_factor)
        self.p, self.q, self.eps, self.c_n = int(p), int(q), float(eps), float(c_n)
        self.q_near, self.n_l, self.tau = int(q_near), int(n_l), float(tau)
        self.depth_cap, self.dyadic_cap = int(depth_cap), int(dyadic_cap)
        self.A, self.B, self.C, self.D = orient(vert, tri)
        self.T = self.A.shape[0]
        self.n_p = rules.n_basis(self.p)
        # reference data
        self.Vinv = rules.vandermonde_inverse(self.p)
        self.far_X, self.far_W = rules.collapsed_gauss(self.q)
        self.far_K = rules.koornwinder(self.p, self.far_X[:, 0], self.far_X[:, 1])
        self.far_what = rules.edge_weights(self.q)
        self.near_X, self.near_W = rules.collapsed_gauss(self.q_near)
        self.near_what = rules.edge_weights(self.q_near)
        self.gl_s, self.gl_w = rules.gauss_legendre01(self.n_l)
        self.rad_r, self.rad_alpha, self.rad_beta = rules.radial_rule(self.p)
        self.n_subdiv_cap_hits = 0
        self.stats = {"near_subtriangles": 0, "self_panels": 0}

    # -- step 3: values -> Koornwinder coefficients (Sec. 2.2, Sec. 3.5) -----
    def coefficients(self, F):
        """F: [T, n_p] or [T, n_p, R] values at the interpolation nodes.
        Returns c with the same shape: c(Delta) = V^{-1} F(Delta)."""
        F = np.asarray(F, dtype=np.float64)
        squeeze = F.ndim == 2
        if squeeze:
            F = F[:, :, None]
        c = np.einsum("ki,tir->tkr", self.Vinv, F)
        return c[:, :, 0] if squeeze else c

    # -- step 4: far sum over all far-rule nodes (Sec. 3.2 rule, Sec. 3.6) ----
    def far_sources(self, c):
        """Node positions [T*q^2, 2] and charges [T*q^2, R]:
        charge_j = w_j |J| f_h(y_j) (the 1/2pi is applied at the end)."""
        c = np.asarray(c, dtype=np.float64)
        if c.ndim == 2:
            c = c[:, :, None]
        nf = self.far_X.shape[0]
        pos = (self.A[:, None, :] + self.far_X[None, :, :1] * (self.B - self.A)[:, None, :]
               + self.far_X[None, :, 1:2] * (self.C - self.A)[:, None, :])
        fh = np.einsum("jk,tkr->tjr", self.far_K, c)
        charge = fh * (self.far_W[None, :, None] * self.D[:, None, None])
        return pos.reshape(self.T * nf, 2), charge.reshape(self.T * nf, -1)

    @staticmethod
    def far_sum(pos, charge, targets):
        """sum_j charge_j log|x_t - y_j| for every target; a pair at distance
        exactly 0 contributes 0 (reading: the paper is silent; the same skip
        is applied to the subtracted far-rule part, so it cancels).
        Accumulated in extended precision."""
        targets = np.asarray(targets, dtype=np.float64)
        out = np.empty((targets.shape[0], charge.shape[1]))
        qx = charge.astype(np.longdouble)
        chunk = max(1, int(2_000_000 // max(1, pos.shape[0])))
        for s in range(0, targets.shape[0], chunk):
            tx = targets[s:s + chunk]
            dx = tx[:, None, 0] - pos[None, :, 0]
            dy = tx[:, None, 1] - pos[None, :, 1]
            r2 = dx * dx + dy * dy
            with np.errstate(divide="ignore"):
                lg = np.where(r2 > 0.0, 0.5 * np.log(np.where(r2 > 0.0, r2, 1.0)), 0.0)
            out[s:s + chunk] = (lg.astype(np.longdouble) @ qx).astype(np.float64)
        return out

    # -- step 5: classification (Def. far/near field; Sec. 4.1) ---------------
    def ellipse_params(self, P, Q, area2, what, order):
        """rho and focal-sum threshold of one edge's Bernstein ellipse.

        rho = (w / (eps C_N))^(1/N) with w = w-hat * |J| (eq. rho0 and the
        area scaling that follows Table CN_values); the ellipse is the image
        of E_rho under the map of [-1, 1] onto the edge PQ, i.e. the points
        whose distances to P and Q sum to less than |PQ| (rho + 1/rho) / 2.
        Returns (rho, threshold)."""
        rho = (what * area2 / (self.eps * self.c_n)) ** (1.0 / order)
        ell = math.hypot(Q[0] - P[0], Q[1] - P[1])
        return rho, 0.5 * ell * (rho + 1.0 / rho)

    def in_ellipses(self, x, P3, area2, what, order):
        """True if x lies inside one of the three edge ellipses (eq. threeE)
        of the triangle with vertices P3[0..2] (edges 01, 12, 20)."""
        for e in range(3):
            P, Q = P3[e], P3[(e + 1) % 3]
            rho, thr = self.ellipse_params(P, Q, area2, what[e], order)
            if rho <= 1.0:
                continue
            fs = math.hypot(x[0] - P[0], x[1] - P[1]) + math.hypot(x[0] - Q[0], x[1] - Q[1])
            if fs < thr:
                return True
        return False

    def in_ball(self, x, P3):
        """True if x lies within ball_factor R of the centroid c of the
        triangle P3[0..2], R = max_i |P3[i] - c| (the naive near field).
        Distances as sqrt(dx^2 + dy^2), so that a decision is the same in
        any IEEE evaluation of this formula."""
        cx = (P3[0][0] + P3[1][0] + P3[2][0]) / 3.0
        cy = (P3[0][1] + P3[1][1] + P3[2][1]) / 3.0

        def dist(ax, ay):
            dx, dy = ax - cx, ay - cy
            return math.sqrt(dx * dx + dy * dy)

        R = max(dist(P3[i][0], P3[i][1]) for i in range(3))
        return dist(x[0], x[1]) < self.ball_factor * R

    def barycentric(self, t_idx, x):
        """Barycentric coordinates (lambda_A, lambda_B, lambda_C) of x with
        respect to triangle t_idx."""
        A, B, C, D = self.A[t_idx], self.B[t_idx], self.C[t_idx], self.D[t_idx]
        xi = to_reference(A, B, C, D, np.asarray(x, dtype=np.float64)[None, :])[0]
        return np.array([1.0 - xi[0] - xi[1], xi[0], xi[1]])

    def classify_target(self, x):
        """List of (triangle, kind) for one target, kind 0 = self, 1 = near,
        triangles ascending.  Self: x in the closure of the triangle, up to a
        barycentric tolerance tau (a target on a shared edge or vertex is self
        for every triangle containing it).  Near: not self and inside the
        ellipse union of the far rule (N = 2q - 1), or, for the ball model,
        inside the naive ball (``in_ball``).  Everything else is far.
        The tests are those of ``barycentric`` and ``in_ellipses``, written
        over all triangles at once."""
        x = np.asarray(x, dtype=np.float64)
        e1 = self.B - self.A
        e2 = self.C - self.A
        d = x[None, :] - self.A
        xi1 = (d[:, 0] * e2[:, 1] - d[:, 1] * e2[:, 0]) / self.D
        xi2 = (e1[:, 0] * d[:, 1] - e1[:, 1] * d[:, 0]) / self.D
        lam_min = np.minimum(np.minimum(1.0 - xi1 - xi2, xi1), xi2)
        is_self = lam_min >= -self.tau
        N = 2 * self.q - 1
        is_near = np.zeros(self.T, dtype=bool)
        if self.near_model == "ball":
            c = (self.A + self.B + self.C) / 3.0

            def dist(P):
                d = P - c
                return np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1])

            R = np.maximum(np.maximum(dist(self.A), dist(self.B)), dist(self.C))
            is_near = dist(np.broadcast_to(x, c.shape)) < self.ball_factor * R
        else:
            for e, (P, Q) in enumerate(((self.A, self.B), (self.B, self.C), (self.C, self.A))):
                rho = (self.far_what[e] * self.D / (self.eps * self.c_n)) ** (1.0 / N)
                ell = np.hypot(Q[:, 0] - P[:, 0], Q[:, 1] - P[:, 1])
                thr = 0.5 * ell * (rho + 1.0 / rho)
                fs = np.hypot(x[0] - P[:, 0], x[1] - P[:, 1]) + np.hypot(x[0] - Q[:, 0], x[1] - Q[:, 1])
                is_near |= (rho > 1.0) & (fs < thr)
        is_near &= ~is_self
        out = [(int(t), 0 if is_self[t] else 1) for t in np.nonzero(is_self | is_near)[0]]
        return out

    # -- step 6a: far rule's own contribution B (subtract half, Sec. 3.6) -----
    def far_B(self, t_idx, x):
        """B_k = sum_j w_j |J| log|x - y_j| K_k(xi_j) over the far nodes of
        one triangle; r = 0 terms skipped."""
        A, B, C, D = self.A[t_idx], self.B[t_idx], self.C[t_idx], self.D[t_idx]
        Y = to_physical(A, B, C, self.far_X)
        r2 = (x[0] - Y[:, 0]) ** 2 + (x[1] - Y[:, 1]) ** 2
        with np.errstate(divide="ignore"):
            lg = np.where(r2 > 0.0, 0.5 * np.log(np.where(r2 > 0.0, r2, 1.0)), 0.0)
        return (self.far_W * D * lg) @ self.far_K

    # -- step 6b: near pair, adaptive subdivision (Sec. 3.3, Sec. 4.1) --------
    def near_A(self, t_idx, x, eps=None):
        """A_k = int_Delta log|x - y| K_k(rho^{-1} y) dA for x outside Delta.

        Start from the reference simplex; a sub-triangle tau (reference
        vertices a, b, c) is integrated with the near rule (mapped by
        xi' -> a + xi'_1 (b - a) + xi'_2 (c - a)) once x lies outside the
        three ellipses of its physical image for the near rule, with weights
        scaled by its own |J| (Sec. 4.1: subdivision decided by the same
        analysis).  Otherwise it splits into four by edge midpoints (reading:
        the paper's figure of the subdivision is not available):
            (a, m_ab, m_ca), (m_ab, b, m_bc), (m_ca, m_bc, c), (m_bc, m_ca, m_ab)
        which keeps every child's orientation.  Depth capped at depth_cap
        (a capped leaf is integrated anyway and counted)."""
        saved = self.eps
        if eps is not None:
            self.eps = float(eps)
        try:
            A, B, C, D = self.A[t_idx], self.B[t_idx], self.C[t_idx], self.D[t_idx]
            Nn = 2 * self.q_near - 1
            leaves = []
            stack = [(np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0]), 0)]
            while stack:
                a, b, c, depth = stack.pop()
                ref_area2 = abs((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
                area2 = ref_area2 * D
                P3 = to_physical(A, B, C, np.stack([a, b, c]))
                if self.near_model == "ball":
                    split = self.in_ball(x, P3)
                else:
                    split = self.in_ellipses(x, P3, area2, self.near_what, Nn)
                if depth < self.depth_cap and split:
                    mab, mbc, mca = (a + b) / 2, (b + c) / 2, (c + a) / 2
                    stack.extend([(a, mab, mca, depth + 1), (mab, b, mbc, depth + 1),
                                  (mca, mbc, c, depth + 1), (mbc, mca, mab, depth + 1)])
                    continue
                if depth >= self.depth_cap:
                    self.n_subdiv_cap_hits += 1
                leaves.append((a, b, c, ref_area2))
            self.stats["near_subtriangles"] += len(leaves)
            # integrate all leaves with the near rule
            Xn, Wn = self.near_X, self.near_W
            xis, wts = [], []
            for a, b, c, ref_area2 in leaves:
                xis.append(a[None, :] + Xn[:, :1] * (b - a)[None, :] + Xn[:, 1:2] * (c - a)[None, :])
                wts.append(Wn * ref_area2 * D)
            xi = np.concatenate(xis)
            w = np.concatenate(wts)
            Y = to_physical(A, B, C, xi)
            lg = 0.5 * np.log((x[0] - Y[:, 0]) ** 2 + (x[1] - Y[:, 1]) ** 2)
            K = rules.koornwinder(self.p, xi[:, 0], xi[:, 1])
            return (w * lg) @ K
        finally:
            self.eps = saved

    # -- step 6c: self pair, radius-arc-length coordinates (Sec. 3.4) ---------
    def dyadic_panels(self, s_tilde, length, d):
        """Arc-length panels on [0, length] toward s_tilde (Sec. 3.4, steps
        1-3).  On [0, s~]: [(1 - 2^-(i-1)) s~, (1 - 2^-i) s~] for i = 1..N and
        [(1 - 2^-N) s~, s~], N = min{N >= 0 : 2^-N s~ < d}; mirrored on
        [s~, L] with M.  An empty side gives no panels."""
        panels = []
        if s_tilde > 0.0:
            n = 0
            while not (s_tilde * 0.5 ** n < d) and n < self.dyadic_cap:
                n += 1
            for i in range(1, n + 1):
                panels.append(((1.0 - 0.5 ** (i - 1)) * s_tilde, (1.0 - 0.5 ** i) * s_tilde))
            panels.append(((1.0 - 0.5 ** n) * s_tilde, s_tilde))
        rest = length - s_tilde
        if rest > 0.0:
            m = 0
            while not (rest * 0.5 ** m < d) and m < self.dyadic_cap:
                m += 1
            for i in range(1, m + 1):
                panels.append((length - (1.0 - 0.5 ** i) * rest, length - (1.0 - 0.5 ** (i - 1)) * rest))
            panels.append((s_tilde, length - (1.0 - 0.5 ** m) * rest))
        return panels

    def self_A(self, t_idx, v):
        """A_k = int_Delta log|v - y| K_k(rho^{-1} y) dA for v in the closure
        of Delta.  Delta splits at v into (v, A, B), (v, B, C), (v, C, A); a
        piece with area <= tau * area(Delta) is skipped (v on that edge).  On
        a piece with opposite side PQ (length L, unit-speed gamma(s) =
        P + s (Q-P)/L), eq. volpot_self_single reads
            int_0^L int_0^1 log(r0(s) r) f(v + r (gamma(s) - v)) r dr h ds
        where r0(s) = |gamma(s) - v| and h = |(gamma - v) x gamma'| is the
        distance from v to the line PQ (constant on a straight side).  The
        s-integral uses n_l-point Gauss-Legendre on the dyadic panels, the
        r-integral the radial rule (exact for the degree-p interpolant)."""
        A, B, C, D = self.A[t_idx], self.B[t_idx], self.C[t_idx], self.D[t_idx]
        v = np.asarray(v, dtype=np.float64)
        area = 0.5 * D
        ys, ws = [], []
        for P, Q in ((A, B), (B, C), (C, A)):
            area_sub = 0.5 * abs((P[0] - v[0]) * (Q[1] - v[1]) - (P[1] - v[1]) * (Q[0] - v[0]))
            if area_sub <= self.tau * area:
                continue
            L = math.hypot(Q[0] - P[0], Q[1] - P[1])
            e = (Q - P) / L
            h = abs((P[0] - v[0]) * (Q[1] - P[1]) - (P[1] - v[1]) * (Q[0] - P[0])) / L
            s_t = min(max((v[0] - P[0]) * e[0] + (v[1] - P[1]) * e[1], 0.0), L)
            foot = P + s_t * e
            d = math.hypot(v[0] - foot[0], v[1] - foot[1])
            panels = self.dyadic_panels(s_t, L, d)
            self.stats["self_panels"] += len(panels)
            for s0, s1 in panels:
                s = s0 + (s1 - s0) * self.gl_s
                wsv = (s1 - s0) * self.gl_w
                g = P[None, :] + s[:, None] * e[None, :]
                r0 = np.hypot(g[:, 0] - v[0], g[:, 1] - v[1])
                # all (s, r) combinations
                y = v[None, None, :] + self.rad_r[None, :, None] * (g[:, None, :] - v[None, None, :])
                coef = (h * wsv[:, None]) * (self.rad_alpha[None, :] * np.log(r0)[:, None]
                                             + self.rad_beta[None, :])
                ys.append(y.reshape(-1, 2))
                ws.append(coef.reshape(-1))
        if not ys:
            return np.zeros(self.n_p)
        Y = np.concatenate(ys)
        w = np.concatenate(ws)
        xi = to_reference(A, B, C, D, Y)
        K = rules.koornwinder(self.p, xi[:, 0], xi[:, 1])
        return w @ K

    # -- rows and the end-to-end result --------------------------------------
    def row(self, t_idx, x, kind):
        """Correction row (A_k - B_k) / 2pi for one (target, triangle) pair."""
        x = np.asarray(x, dtype=np.float64)
        Ak = self.self_A(t_idx, x) if kind == 0 else self.near_A(t_idx, x)
        return (Ak - self.far_B(t_idx, x)) / TWO_PI

    def evaluate(self, F, targets, far_only=False, return_parts=False):
        """u at every target [n_tgt, R] (or [n_tgt] for a single density).

        u = far sum / 2pi + sum over self and near pairs of row . c(Delta)."""
        F = np.asarray(F, dtype=np.float64)
        single = F.ndim == 2
        c = self.coefficients(F)
        if single:
            c = c[:, :, None]
        targets = np.asarray(targets, dtype=np.float64).reshape(-1, 2)
        pos, charge = self.far_sources(c)
        u_far = self.far_sum(pos, charge, targets) / TWO_PI
        corr = np.zeros_like(u_far)
        pairs = []
        if not far_only:
            for i, x in enumerate(targets):
                for t_idx, kind in self.classify_target(x):
                    r = self.row(t_idx, x, kind)
                    corr[i] += r @ c[t_idx]
                    pairs.append((i, t_idx, kind))
        u = u_far + corr
        if single:
            u, u_far, corr = u[:, 0], u_far[:, 0], corr[:, 0]
        if return_parts:
            return u, u_far, corr, pairs
        return u
