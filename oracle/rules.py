"""Reference data for the oracle (TEST INFRASTRUCTURE ONLY; see package doc).

Everything here lives on the standard simplex
    T = {(x, y): 0 <= x <= 1, 0 <= y <= 1 - x}
with vertex order A=(0,0), B=(1,0), C=(0,1).  Each routine is written from
the definition the paper gives; library primitives (SciPy's Gauss-Jacobi and
Gauss-Legendre nodes, mpmath's symmetric eigensolver, LAPACK's LU inverse)
serve as steps.
"""

import functools

import mpmath
import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import eval_jacobi, eval_legendre, roots_jacobi, roots_legendre


def n_basis(p):
    """dim P_p = (p+1)(p+2)/2 (Sec. 2.1)."""
    return (p + 1) * (p + 2) // 2


def koornwinder(p, x, y):
    """Orthonormal Koornwinder basis of P_p on T, Sec. 2.1.

    K_mn(x,y) = c_mn (1-x)^m P^{(2m+1,0)}_{n-m}(2x-1) P_m(2y/(1-x) - 1), m <= n,
    with c_mn = sqrt(2 (2m+1) (n+1)) so that the integral of K_mn^2 over T is 1.
    Column k = n(n+1)/2 + m.  Returns an array of shape (len(x), n_basis(p)).

    The factor (1-x)^m P_m(2y/(1-x)-1) is a polynomial of degree m; at the
    collapsed vertex B (x = 1, hence y = 0) its value is 1 for m = 0 and 0
    otherwise, which is the limit used there.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    t = 1.0 - x
    safe_t = np.where(t != 0.0, t, 1.0)
    s = np.where(t != 0.0, 2.0 * y / safe_t - 1.0, 0.0)
    out = np.empty((x.size, n_basis(p)))
    for n in range(p + 1):
        for m in range(n + 1):
            c = np.sqrt(2.0 * (2 * m + 1) * (n + 1))
            leg = np.where(t != 0.0, t ** m * eval_legendre(m, s), 1.0 if m == 0 else 0.0)
            out[:, n * (n + 1) // 2 + m] = c * eval_jacobi(n - m, 2 * m + 1, 0, 2.0 * x - 1.0) * leg
    return out


@functools.lru_cache(maxsize=None)
def gauss_legendre01(n):
    """n-point Gauss-Legendre rule on [0, 1] (nodes ascending, weights sum 1)."""
    x, w = roots_legendre(n)
    return (x + 1.0) / 2.0, w / 2.0


@functools.lru_cache(maxsize=None)
def collapsed_gauss(q):
    """q x q collapsed Gauss rule on T (far and near rules, Sec. 3.2).

    The integral over T equals the integral over the unit square of
    g(u, (1-u) v) (1-u) du dv.  u-nodes: Gauss-Jacobi with weight (1-u) on
    [0, 1] (alpha = 1, beta = 0 on [-1, 1], weights / 4); v-nodes:
    Gauss-Legendre on [0, 1].  Node (u_a, (1-u_a) v_b) has weight
    wu_a * wv_b; node index = a*q + b.  The map collapses the edge u = 1 onto
    vertex B.  Exact for total degree <= 2q - 1.
    """
    u, wu = roots_jacobi(q, 1.0, 0.0)
    u = (u + 1.0) / 2.0
    wu = wu / 4.0
    v, wv = gauss_legendre01(q)
    X = np.empty((q * q, 2))
    W = np.empty(q * q)
    for a in range(q):
        for b in range(q):
            X[a * q + b] = (u[a], (1.0 - u[a]) * v[b])
            W[a * q + b] = wu[a] * wv[b]
    return X, W


def edge_distances(X):
    """Distances of reference points to the three edges of T: AB (y=0),
    BC (x+y=1) and CA (x=0), in that order (columns)."""
    return np.stack([X[:, 1], (1.0 - X[:, 0] - X[:, 1]) / np.sqrt(2.0), X[:, 0]], axis=1)


@functools.lru_cache(maxsize=None)
def edge_weights(q):
    """Per-edge weight w-hat_i of the q x q collapsed rule (Sec. 4.1, eq. rho0).

    The paper takes the largest quadrature weight among the nodes closest to
    an edge.  Reading used here: for each edge of T, the largest weight among
    the q nodes nearest that edge.  Returns an array of 3 (edges AB, BC, CA).
    """
    X, W = collapsed_gauss(q)
    d = edge_distances(X)
    out = np.empty(3)
    for e in range(3):
        nearest = np.argsort(d[:, e], kind="stable")[:q]
        out[e] = W[nearest].max()
    return out


@functools.lru_cache(maxsize=None)
def log_gauss01(n):
    """n-point Gauss rule for the weight -log(r) on [0, 1].

    Built at 80 digits with mpmath from the exact moments
    int_0^1 -log(r) r^k dr = 1/(k+1)^2: Chebyshev's algorithm gives the
    three-term recurrence, the eigen-decomposition of its Jacobi matrix the
    nodes and weights (Golub-Welsch).  Returns (nodes, weights) as float64.
    """
    with mpmath.workdps(80):
        mom = [mpmath.mpf(1) / (k + 1) ** 2 for k in range(2 * n)]
        # Chebyshev algorithm (ordinary moments -> recurrence coefficients).
        alpha = [mpmath.mpf(0)] * n
        beta = [mpmath.mpf(0)] * n
        sig_prev = [mpmath.mpf(0)] * (2 * n)
        sig = list(mom)
        alpha[0] = mom[1] / mom[0]
        beta[0] = mom[0]
        for k in range(1, n):
            sig_new = [mpmath.mpf(0)] * (2 * n)
            for l in range(k, 2 * n - k):
                sig_new[l] = sig[l + 1] - alpha[k - 1] * sig[l] - beta[k - 1] * sig_prev[l]
            alpha[k] = sig_new[k + 1] / sig_new[k] - sig[k] / sig[k - 1]
            beta[k] = sig_new[k] / sig[k - 1]
            sig_prev, sig = sig, sig_new
        J = mpmath.zeros(n, n)
        for k in range(n):
            J[k, k] = alpha[k]
            if k + 1 < n:
                J[k, k + 1] = J[k + 1, k] = mpmath.sqrt(beta[k + 1])
        evals, evecs = mpmath.eigsy(J)
        nodes = np.array([float(evals[i]) for i in range(n)])
        weights = np.array([float(mom[0] * evecs[0, i] ** 2) for i in range(n)])
    order = np.argsort(nodes)
    return nodes[order], weights[order]


def radial_half(p):
    """Points per half of the radial rule: exact for r * phi(r) with phi of
    degree <= p needs 2n - 1 >= p + 1; at least 4 (8 points in total, the
    paper's GGQ length)."""
    return max(4, (p + 3) // 2)


@functools.lru_cache(maxsize=None)
def radial_rule(p):
    """Radial rule for the self-interaction inner integral (Sec. 3.4).

    For phi of degree <= p the inner integral
        int_0^1 r log(r0 r) phi(r) dr = log(r0) int_0^1 r phi(r) dr
                                         + int_0^1 r log(r) phi(r) dr
    is integrated exactly: the first part by Gauss-Legendre, the second by
    the Gauss rule for weight -log(r).  Node j contributes
    (alpha_j log r0 + beta_j) phi(r_j).  Returns (r, alpha, beta).
    """
    n = radial_half(p)
    rg, wg = gauss_legendre01(n)
    rl, wl = log_gauss01(n)
    r = np.concatenate([rg, rl])
    alpha = np.concatenate([wg * rg, np.zeros(n)])
    beta = np.concatenate([np.zeros(n), -wl * rl])
    return r, alpha, beta


@functools.lru_cache(maxsize=None)
def gauss_lobatto_legendre01(M):
    """M+1 Gauss-Lobatto-Legendre points on [0, 1]: the end points and the
    roots of P_M'."""
    c = np.zeros(M + 1)
    c[-1] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(c)).real)
    return np.concatenate([[0.0], (inner + 1.0) / 2.0, [1.0]])


@functools.lru_cache(maxsize=None)
def interp_nodes(p):
    """Interpolation nodes on T for degree p (stand-in for the
    Vioreanu-Rokhlin nodes of Sec. 2.2, whose tables are not printed).

    Blyth-Pozrikidis construction from the Gauss-Lobatto-Legendre points
    v_0..v_M of order M = p + 3: for i + j + k = M with i, j, k >= 1,
        x = (1 + 2 v_i - v_j - v_k) / 3,   y = (1 + 2 v_j - v_i - v_k) / 3.
    This gives exactly (p+1)(p+2)/2 interior nodes.  Order: i ascending,
    then j ascending.
    """
    M = p + 3
    v = gauss_lobatto_legendre01(M)
    pts = []
    for i in range(1, M):
        for j in range(1, M - i):
            k = M - i - j
            pts.append(((1 + 2 * v[i] - v[j] - v[k]) / 3.0, (1 + 2 * v[j] - v[i] - v[k]) / 3.0))
    return np.array(pts)


@functools.lru_cache(maxsize=None)
def vandermonde_inverse(p):
    """Interpolation matrix V^{-1} of Sec. 2.2: V[i, k] = K_k(node_i);
    V^{-1} maps values at the nodes to Koornwinder coefficients.  LU with
    partial pivoting (LAPACK) inverts it."""
    X = interp_nodes(p)
    V = koornwinder(p, X[:, 0], X[:, 1])
    return np.linalg.inv(V)
