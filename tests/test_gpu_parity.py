"""GPU parity: the HIP library (through its C ABI) against the oracle.

Bars (FP64 path): far sum alone <= 1e-13 relative L-infinity, end to end
<= 1e-11 relative L-infinity (max_t |u_gpu - u_oracle| / max_t |u_oracle|
per right-hand side), pair lists equal except pairs whose classification
margin is within 1e-12 of the decision boundary (both sides then sit within
rounding of an ellipse or an edge, where either answer meets eps).
"""

import math
import sys

import numpy as np
import pytest

from oracle import potential, rules
from paper_2205_04401_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_FAR = 1e-13
REL_E2E = 1e-11
BAND = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vp_ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2205_04401_amd import vp
    ctx = vp.Context(0)
    yield ctx


def rel_linf(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return float((np.abs(a - b).max(0) / np.abs(b).max(0)).max())


def oracle_pairs_rows(o, targets):
    pairs, rows = [], {}
    for i, x in enumerate(targets):
        for t, k in o.classify_target(x):
            pairs.append((i, t, k))
            rows[(i, t)] = o.row(t, x, k)
    return pairs, rows


def margin(o, x, t, kind_gpu):
    """Relative distance of (x, t) from the boundary of the test that decides
    its class: self test (barycentric vs -tau) and each ellipse."""
    lam = o.barycentric(t, x)
    m = [abs(lam.min() + o.tau)]
    N = 2 * o.q - 1
    P3 = (o.A[t], o.B[t], o.C[t])
    if getattr(o, "curves", None) and t in o.curves:
        z = o.inverse(t, x)
        if np.all(np.isfinite(z)):
            m.append(abs(min(1.0 - z[0] - z[1], z[0], z[1]) + o.tau))
        for e in range(3):
            P, Q = P3[e], P3[(e + 1) % 3]
            rho, thr = o.ellipse_params(P, Q, o.Deff[t], o.far_what[e], N)
            if rho > 1:
                m.append(abs(math.hypot(*(x - P)) + math.hypot(*(x - Q)) - thr) / thr)
        return min(m)
    if o.near_model == "ball":
        c = (P3[0] + P3[1] + P3[2]) / 3.0
        r = o.ball_factor * max(math.hypot(*(v - c)) for v in P3)
        return min(m + [abs(math.hypot(*(x - c)) - r) / r])
    for e in range(3):
        P, Q = P3[e], P3[(e + 1) % 3]
        rho, thr = o.ellipse_params(P, Q, o.D[t], o.far_what[e], N)
        if rho > 1:
            fs = math.hypot(*(x - P)) + math.hypot(*(x - Q))
            m.append(abs(fs - thr) / thr)
    return min(m)


def compare_pairs(plan, o, targets, sample=None, pairs=None):
    """Pair lists of the plan (or `pairs`, its copy from plan.pairs()) vs the
    oracle's classification.  Returns the number of band flips; fails on any
    other difference."""
    rp, tri, kind = plan.pairs() if pairs is None else pairs
    idx = range(len(targets)) if sample is None else sample
    flips = 0
    for i in idx:
        x = targets[i]
        g = {(int(t), int(k)) for t, k in zip(tri[rp[i]:rp[i + 1]], kind[rp[i]:rp[i + 1]])}
        r = set(o.classify_target(x))
        assert list(tri[rp[i]:rp[i + 1]]) == sorted(tri[rp[i]:rp[i + 1]]), "triangles not ascending"
        for t, k in g ^ r:
            assert margin(o, x, t, k) < BAND, (i, t, k, margin(o, x, t, k))
            flips += 1
    return flips


def special_targets(vq, tq, seed, n_vert=8, n_edge=8, n_sliver=4):
    """Targets where the near-field decisions are hardest: interior mesh
    vertices (self pairs with every triangle around them), points on shared
    edges (self pairs with both sides), and, on the n_sliver triangles of
    largest aspect ratio (longest edge squared over area), the centroid, a
    point just inside each edge's midpoint and a point just outside."""
    rng = np.random.default_rng(seed)
    tq = np.asarray(tq)
    e = np.sort(np.concatenate([tq[:, [0, 1]], tq[:, [1, 2]], tq[:, [2, 0]]]), axis=1)
    edges, count = np.unique(e, axis=0, return_counts=True)
    shared = edges[count == 2]
    interior = np.unique(shared.ravel())
    on_boundary = np.unique(edges[count == 1].ravel())
    interior = np.setdiff1d(interior, on_boundary)
    pts = [vq[rng.choice(interior, n_vert, replace=False)]]
    pick = shared[rng.choice(len(shared), n_edge, replace=False)]
    s_ = rng.uniform(0.1, 0.9, n_edge)[:, None]
    pts.append(vq[pick[:, 0]] + s_ * (vq[pick[:, 1]] - vq[pick[:, 0]]))
    a, b, c = vq[tq[:, 0]], vq[tq[:, 1]], vq[tq[:, 2]]
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    longest = np.maximum.reduce([np.sum((b - a) ** 2, 1), np.sum((c - b) ** 2, 1), np.sum((a - c) ** 2, 1)])
    for t in np.argsort(longest / area)[-n_sliver:]:
        P = vq[tq[t]]
        cen = P.mean(0)
        pts.append(cen[None])
        for k in range(3):
            mid = 0.5 * (P[k] + P[(k + 1) % 3])
            pts.append(np.stack([mid + 1e-3 * (cen - mid), mid - 1e-3 * (cen - mid)]))
    return np.concatenate(pts)


def sample_with_special(tg, vq, tq, n_random, seed, extra=()):
    """Targets with special ones appended (a ragged tail), and the sorted
    indices of n_random seeded targets plus every appended one."""
    sp = [special_targets(vq, tq, seed)] + [np.asarray(x, dtype=np.float64).reshape(-1, 2) for x in extra]
    sp = np.concatenate(sp)
    rng = np.random.default_rng(seed)
    sample = np.concatenate([rng.choice(len(tg), n_random, replace=False), len(tg) + np.arange(len(sp))])
    return np.ascontiguousarray(np.concatenate([tg, sp])), np.sort(sample)


def compare_rows(plan, o, tg, sample, rp, tri, kind, area, tol):
    """Every row of the sampled targets (copied pair range by pair range)
    against the oracle's row, relative to the triangle's area; pairs whose
    class differs (a decision on its boundary, checked by compare_pairs)
    are skipped.  Returns (worst, rows compared per kind)."""
    worst, seen = 0.0, {0: 0, 1: 0}
    for i in sample:
        ref = {t: (k, o.row(t, tg[i], k)) for t, k in o.classify_target(tg[i])}
        rows = plan.rows_range(rp[i], rp[i + 1] - rp[i])
        for j, p_ in enumerate(range(rp[i], rp[i + 1])):
            t = int(tri[p_])
            if t not in ref or ref[t][0] != int(kind[p_]):
                continue
            seen[ref[t][0]] += 1
            worst = max(worst, np.abs(rows[j] - ref[t][1]).max() / area[t])
    assert worst <= tol, worst
    return worst, seen


def tri_area(vq, tq):
    e1, e2 = vq[tq[:, 1]] - vq[tq[:, 0]], vq[tq[:, 2]] - vq[tq[:, 0]]
    return 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])


# ---------------------------------------------------------------------------
# unit square, p = 4, q = 8, eps = 1e-13 (1920 targets, 128 triangles)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1(vp_ctx):
    p, q, eps = 4, 8, 1e-13
    vq, tq = W.unit_square(8, "/")
    vt, tt = W.unit_square(8, "\\")
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_bump, vq, tq, nodes)
    say("c1: oracle")
    o = potential.Oracle(vq, tq, p, q, eps)
    pairs, rows = oracle_pairs_rows(o, tg)
    c = o.coefficients(F)
    pos, charge = o.far_sources(c)
    u_far = o.far_sum(pos, charge, tg)[:, 0] / (2 * math.pi)
    corr = np.zeros(len(tg))
    for i, t, k in pairs:
        corr[i] += rows[(i, t)] @ c[t]
    say("c1: plan")
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    return dict(o=o, tg=tg, F=F, pairs=pairs, rows=rows, u_far=u_far, u=u_far + corr, c=c, pos=pos,
                charge=charge, plan=plan, mesh=mesh, vq=vq, tq=tq)


def test_c1_coefficients_and_charges(c1):
    coef, charge = c1["plan"].coefficients(c1["F"])
    assert np.abs(coef[:, :, 0] - c1["c"]).max() <= 1e-13 * np.abs(c1["c"]).max()
    ref = c1["charge"][:, 0] / (4 * math.pi)
    assert np.abs(charge[:, 0] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(c1["plan"].sources() - c1["pos"]).max() < 1e-15


def test_c1_pair_lists(c1):
    flips = compare_pairs(c1["plan"], c1["o"], c1["tg"])
    info = c1["plan"].info()
    assert info["near_subtri"] >= info["n_pairs"] - info["n_self"]
    say("c1 pairs", info["n_pairs"], "oracle", len(c1["pairs"]), "band flips", flips)
    assert abs(info["n_pairs"] - len(c1["pairs"])) <= flips
    assert info["n_self"] == sum(1 for _, _, k in c1["pairs"] if k == 0)


def test_c1_rows(c1):
    rp, tri, kind = c1["plan"].pairs()
    rows = c1["plan"].rows()
    scale = max(np.abs(r).max() for r in c1["rows"].values())
    worst = 0.0
    for i in range(len(c1["tg"])):
        for p_ in range(rp[i], rp[i + 1]):
            key = (i, int(tri[p_]))
            if key in c1["rows"]:
                worst = max(worst, np.abs(rows[p_] - c1["rows"][key]).max())
    say("c1 rows worst abs diff", worst, "scale", scale)
    assert worst <= 1e-12 * scale


def test_c1_far_only(c1):
    u = c1["plan"].execute(c1["F"], far_only=True)
    err = rel_linf(u, c1["u_far"])
    say("c1 far-only rel", err)
    assert err <= REL_FAR


def test_c1_end_to_end(c1):
    u = c1["plan"].execute(c1["F"])
    err = rel_linf(u, c1["u"])
    say("c1 end-to-end rel", err)
    assert err <= REL_E2E


@pytest.mark.parametrize("p", list(range(1, 11)))
def test_every_order_small_square(vp_ctx, p):
    """Orders 1 to 10, every instantiation of the per-order kernels (basis,
    coefficients, correction rows and their wavefront reduction, apply) on a
    3 x 3 unit square with the staggered targets: the potential at up to 64
    seeded targets against the oracle, and the two far-sum precisions."""
    q, eps = 8, 1e-12
    vq, tq = W.unit_square(3, "/")
    vt, tt = W.unit_square(3, "\\")
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_bump, vq, tq, nodes)
    sample = np.sort(np.random.default_rng(100 + p).choice(len(tg), min(64, len(tg)), replace=False))
    say(f"order {p}: {len(tg)} targets, {len(sample)} sampled")
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    u = plan.execute(F)
    u_mixed = plan.execute(F, mixed=True)
    plan.close()
    mesh.close()
    ref = potential.Oracle(vq, tq, p, q, eps).evaluate(F, tg[sample])
    err = rel_linf(u[sample], ref)
    say(f"order {p}: rel {err:.2e}")
    assert err <= REL_E2E
    assert rel_linf(u_mixed[sample], ref) <= 1e-6


REL_MIXED = 1e-6


def test_c1_mixed_precision(c1):
    """Mixed path (FP32 far sum, FP64 rows) against the FP64 oracle."""
    u = c1["plan"].execute(c1["F"], mixed=True)
    err = rel_linf(u, c1["u"])
    say("c1 mixed rel", err)
    assert err <= REL_MIXED
    u_far = c1["plan"].execute(c1["F"], mixed=True, far_only=True)
    assert rel_linf(u_far, c1["u_far"]) <= REL_MIXED


def test_c1_multi_rhs_and_device_pointers(c1):
    import torch
    F3 = np.stack([c1["F"], 2.0 * c1["F"] - 1.0, np.sin(c1["F"])], -1)
    u3 = c1["plan"].execute(F3)
    for r in range(3):
        ur = c1["plan"].execute(np.ascontiguousarray(F3[:, :, r]))
        assert np.abs(u3[:, r] - ur).max() <= 1e-15 * np.abs(ur).max()
    Fd = torch.from_numpy(F3).cuda()
    ud = c1["plan"].execute(Fd).cpu().numpy()
    assert np.array_equal(ud, u3)


def c1_oracle_u(c1, F):
    """Oracle potential of the C1 targets for density F, reusing the pairs
    and rows the fixture computed."""
    o = c1["o"]
    c = o.coefficients(F)
    pos, charge = o.far_sources(c)
    u = o.far_sum(pos, charge, c1["tg"])[:, 0] / (2 * math.pi)
    for i, t, k in c1["pairs"]:
        u[i] += c1["rows"][(i, t)] @ c[t]
    return u


def test_c1_many_rhs_matrix_core_blocks(c1):
    """87 right-hand sides: the far sum runs blocks of 64 and 16 on the
    matrix cores (FP64 MFMA, and FP32 MFMA in mixed precision) and the last
    seven on the vector ALUs (4 + 2 + 1).  Every column matches its
    single-RHS evaluation; three columns, one from each kind of block, also
    match the oracle."""
    rng = np.random.default_rng(87)
    base, R = c1["F"], 87
    coef = rng.uniform(-1.0, 1.0, (R, 3))
    FR = np.ascontiguousarray(np.stack(
        [coef[r, 0] * base + coef[r, 1] + coef[r, 2] * np.sin(3.0 * base + r) for r in range(R)], -1))
    plan = c1["plan"]
    u64 = plan.execute(FR)
    umx = plan.execute(FR, mixed=True)
    e64 = emx = 0.0
    for r in range(R):
        ur = plan.execute(np.ascontiguousarray(FR[:, :, r]))
        e64 = max(e64, rel_linf(u64[:, r], ur))
        emx = max(emx, rel_linf(umx[:, r], ur))
    eo = max(rel_linf(u64[:, r], c1_oracle_u(c1, np.ascontiguousarray(FR[:, :, r]))) for r in (5, 70, 86))
    say("c1 87 RHS: fp64 vs single", e64, "mixed vs fp64 single", emx, "fp64 vs oracle", eo)
    assert e64 <= REL_FAR and emx <= 1e-6 and eo <= REL_E2E


def test_graph_replays_equal_eager(c1, vp_ctx):
    """A captured evaluation (HIP graph), FP64 and mixed, replayed several
    times with other eager work and output clears in between: every replay
    equals vp_execute's result bit for bit, also after new density values
    are written into the same buffer."""
    import time
    import torch
    from paper_2205_04401_amd import vp
    plan = c1["plan"]
    F3 = np.ascontiguousarray(np.stack([c1["F"], 2.0 * c1["F"] - 1.0, np.sin(c1["F"])], -1))
    Fd = torch.from_numpy(F3).cuda()
    Ud = torch.empty((len(c1["tg"]), 3), dtype=torch.float64, device="cuda")
    for mixed in (False, True):
        g = vp.Graph(plan, Fd, Ud, mixed=mixed)
        ref = plan.execute(Fd, mixed=mixed).cpu().numpy()
        for k in range(4):
            plan.execute(Fd * (k + 2.0), mixed=not mixed)
            Ud.zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(Ud.cpu().numpy(), ref), (mixed, k)
        Fd.mul_(-0.5)
        ref2 = plan.execute(Fd, mixed=mixed).cpu().numpy()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Ud.cpu().numpy(), ref2)
        Fd.mul_(-2.0)
        if not mixed:
            n = 200
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n):
                plan.execute(Fd, out=Ud, asynchronous=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(n):
                g.launch()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            say("c1 evaluation latency: eager", (t1 - t0) / n * 1e6, "us, graph", (t2 - t1) / n * 1e6, "us")
        g.close()


def test_c1_every_far_shape_and_autotune(c1, vp_ctx):
    """Every launch shape of the far sum (wide / narrow blocks, 1, 2 or 4
    matrix-core tiles, 1 to the most source chunks) gives the oracle's
    potential for one density and the default shape's for 17 (16 on the
    matrix cores + 1 on the vector ALUs), FP64 and mixed; the tuner returns
    one of its candidates with a positive time, and out-of-range shapes are
    refused."""
    from paper_2205_04401_amd import vp
    plan = vp_ctx.plan(c1["mesh"], 4, 8, 1e-13, c1["tg"])
    most = max(1, (plan.info()["n_src"] + 255) // 256 * 256 // 64)
    F1 = c1["F"]
    F17 = np.ascontiguousarray(np.stack([(1.0 + 0.1 * r) * F1 - 0.01 * r for r in range(17)], -1))
    ref17 = {m: plan.execute(F17, mixed=m) for m in (False, True)}
    worst = {}
    for mixed in (False, True):
        tol = REL_MIXED if mixed else REL_E2E
        for shape in ("wide", "narrow1", "narrow2"):
            for split in (1, 8, 40, most):
                plan.set_far_config(shape, 4, split, n_rhs=1, mixed=mixed)
                assert plan.far_config(1, mixed) == dict(shape=vp.FAR_SHAPES[shape], mfma_tiles=4, n_split=split)
                e = rel_linf(plan.execute(F1, mixed=mixed), c1["u"])
                worst[(mixed, 1)] = max(worst.get((mixed, 1), 0.0), e)
                assert e <= tol, (mixed, shape, split, e)
            for tiles in (1, 2, 4):
                for split in (8, most):
                    plan.set_far_config(shape, tiles, split, n_rhs=17, mixed=mixed)
                    u = plan.execute(F17, mixed=mixed)
                    e = max(rel_linf(u[:, r], ref17[mixed][:, r]) for r in range(17))
                    worst[(mixed, 17)] = max(worst.get((mixed, 17), 0.0), e)
                    assert e <= (2e-6 if mixed else REL_FAR), (mixed, shape, tiles, split, e)
    say("c1 far shapes: worst rel", worst)
    for mixed in (False, True):
        for R in (1, 17):
            cfg, ms = plan.autotune(n_rhs=R, mixed=mixed, reps=2)
            say("c1 autotune R", R, "mixed", mixed, cfg, f"{ms * 1e3:.1f} us")
            assert ms > 0 and plan.far_config(R, mixed) == cfg and 1 <= cfg["n_split"] <= most
    assert rel_linf(plan.execute(F1), c1["u"]) <= REL_E2E
    for bad in (dict(shape=3, mfma_tiles=4, n_split=8), dict(shape=0, mfma_tiles=3, n_split=8),
                dict(shape=0, mfma_tiles=4, n_split=0), dict(shape=0, mfma_tiles=4, n_split=most + 1)):
        with pytest.raises(vp.VPError):
            plan.set_far_config(bad["shape"], bad["mfma_tiles"], bad["n_split"])
    plan.close()


def test_matrix_core_corrections_shuffled_ragged_targets(vp_ctx):
    """The correction apply on the matrix cores (blocks of 16+ densities,
    16-target clusters) on a 1000-triangle star whose 14 790 staggered
    targets are shuffled (clusters of unrelated targets: long, mostly empty
    union lists) plus 7 more targets (a ragged last cluster).  33 densities
    (32 on the matrix cores, 1 on the vector ALUs) match each density's own
    one-RHS evaluation, far-only included; the shuffled plan gives the
    unshuffled plan's potential, and the oracle's at sampled targets."""
    p, q, eps = 4, 6, 1e-12
    vq, tq = W.star_mesh(n_tri=1000, n_boundary=200, seed=61)
    vt, tt = W.star_mesh(n_tri=1000, n_boundary=200, seed=62, staggered=True)
    nodes = rules.interp_nodes(p)
    tg0 = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    rng = np.random.default_rng(33)
    perm = rng.permutation(len(tg0))
    tg = np.concatenate([tg0[perm], rng.uniform(-1.0, 1.0, (7, 2))])
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    # the clusters are built by the first evaluation of 16 or more densities
    assert plan.info()["cluster_entries"] == 0
    R = 33
    F1 = W.sample_density(W.gaussian_sum(64, vq, tq), vq, tq, nodes)
    FR = np.ascontiguousarray(np.stack([(1.0 + 0.2 * r) * F1 + np.cos(r + F1) for r in range(R)], -1))
    for far_only in (False, True):
        uR = plan.execute(FR, far_only=far_only)
        info = plan.info()
        say("shuffled star:", len(tg), "targets,", info["n_pairs"], "pairs,", info["cluster_entries"],
            "cluster entries, row fill", info["n_pairs"] / (16 * info["cluster_entries"]))
        assert info["cluster_entries"] > 0 and len(tg) >= 512 * 16
        worst = 0.0
        for r in (0, 7, 15, 16, 31, 32):
            u1 = plan.execute(np.ascontiguousarray(FR[:, :, r]), far_only=far_only)
            worst = max(worst, rel_linf(uR[:, r], u1))
        say("33 RHS, far_only", far_only, "worst rel vs one-RHS", worst)
        assert worst <= REL_FAR
    plan0 = vp_ctx.plan(mesh, p, q, eps, tg0)
    u0 = plan0.execute(FR)
    uR = plan.execute(FR)
    assert rel_linf(uR[: len(perm)], u0[perm]) <= REL_FAR
    sample = np.sort(rng.choice(len(tg), 12, replace=False))
    ref = potential.Oracle(vq, tq, p, q, eps).evaluate(FR[:, :, 20], tg[sample])
    e = rel_linf(uR[sample, 20], ref)
    say("shuffled star sampled rel vs oracle", e)
    assert e <= REL_E2E
    plan0.close()
    plan.close()
    mesh.close()


def test_c1_deterministic(c1, vp_ctx):
    plan2 = vp_ctx.plan(c1["mesh"], 4, 8, 1e-13, c1["tg"])
    a, b = c1["plan"].pairs(), plan2.pairs()
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert np.array_equal(c1["plan"].rows(), plan2.rows())
    assert np.array_equal(c1["plan"].execute(c1["F"]), plan2.execute(c1["F"]))
    plan2.close()


# ---------------------------------------------------------------------------
# independent closed forms and edge cases
# ---------------------------------------------------------------------------

def test_disk_unit_density_polygon_closed_form(vp_ctx):
    import pins
    v, t = W.disk_mesh(n_tri=496, n_boundary=60, seed=1)
    rng = np.random.default_rng(2)
    r = rng.uniform(0, 3, 400)
    a = rng.uniform(0, 2 * math.pi, 400)
    tg = np.stack([r * np.cos(a), r * np.sin(a)], 1)
    mesh = vp_ctx.mesh(v, t)
    plan = vp_ctx.plan(mesh, 2, 8, 1e-13, tg)
    u = plan.execute(np.ones((len(t), 6)))
    ex = np.array([pins.mesh_unit_potential(v, t, x) for x in tg])
    err = rel_linf(u, ex)
    say("disk rel vs polygon closed form", err)
    assert err <= REL_E2E
    plan.close()
    mesh.close()


def test_targets_on_vertices_edges_far_and_ragged(vp_ctx):
    """Targets exactly on vertices and edges (several self pairs), outside
    every near field (no pair), and a count that is not a multiple of any
    block size."""
    p, q = 3, 6
    vq, tq = W.unit_square(4, "/")
    rng = np.random.default_rng(11)
    tg = np.concatenate([vq, (vq[tq[:, 0]] + vq[tq[:, 1]]) / 2, rng.uniform(-0.2, 1.2, (251, 2)),
                         np.array([[5.0, 5.0], [-40.0, 3.0]])])
    nodes = rules.interp_nodes(p)
    F = W.sample_density(lambda x, y: np.cos(3 * x) * y + 0.5, vq, tq, nodes)
    o = potential.Oracle(vq, tq, p, q, 1e-12)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, 1e-12, tg)
    compare_pairs(plan, o, tg)
    rp, _, _ = plan.pairs()
    assert rp[-2] == rp[-3] and rp[-1] == rp[-2]  # far-away targets: no pairs
    u = plan.execute(F)
    ref = o.evaluate(F, tg)
    err = rel_linf(u, ref)
    say("edge-case targets rel", err)
    assert err <= REL_E2E
    plan.close()
    mesh.close()


def test_targets_on_far_nodes(vp_ctx):
    """Targets exactly at far quadrature nodes: the library gives such a pair
    the same finite kernel value in the far sum and in the subtracted rule,
    which cancel; the oracle skips the pair in both.  The potentials agree
    (FP64 and mixed)."""
    p, q = 3, 5
    vq, tq = W.unit_square(3, "/")
    nodes = rules.interp_nodes(p)
    F = W.sample_density(lambda x, y: 1.0 + x * y, vq, tq, nodes)
    mesh = vp_ctx.mesh(vq, tq)
    probe = vp_ctx.plan(mesh, p, q, 1e-12, np.zeros((1, 2)))
    src = probe.sources()
    probe.close()
    tg = np.concatenate([src[::7], np.array([[0.31, 0.52]])])
    plan = vp_ctx.plan(mesh, p, q, 1e-12, tg)
    ref = potential.Oracle(vq, tq, p, q, 1e-12).evaluate(F, tg)
    e64 = rel_linf(plan.execute(F), ref)
    emx = rel_linf(plan.execute(F, mixed=True), ref)
    say("targets on far nodes: rel", e64, "mixed", emx)
    assert e64 <= REL_E2E and emx <= 1e-6
    plan.close()
    mesh.close()


def test_naive_ball_near_model_matches_oracle(vp_ctx):
    """The naive ball near field (ablation model): pair sets, every row and
    u equal the oracle's running the same model (kappa = 2)."""
    p, q, eps, kappa = 3, 4, 1e-12, 2.0
    vq, tq = W.unit_square(4, "/")
    vt, tt = W.unit_square(4, "\\")
    nodes = rules.interp_nodes(p)
    rng = np.random.default_rng(17)
    tg = np.concatenate([W.node_positions(vt, tt, nodes).reshape(-1, 2), rng.uniform(-0.3, 1.3, (40, 2))])
    F = W.sample_density(W.gaussian_bump, vq, tq, nodes)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg, near_model="ball", ball_factor=kappa)
    o = potential.Oracle(vq, tq, p, q, eps, near_model="ball", ball_factor=kappa)
    flips = compare_pairs(plan, o, tg)
    rp, tri, kind = plan.pairs()
    rows = plan.rows()
    worst = scale = 0.0
    for i in range(0, len(tg), 3):
        for j in range(rp[i], rp[i + 1]):
            ref = o.row(int(tri[j]), tg[i], int(kind[j]))
            worst = max(worst, np.abs(rows[j] - ref).max())
            scale = max(scale, np.abs(ref).max())
    e = rel_linf(plan.execute(F), o.evaluate(F, tg))
    say("ball model: flips", flips, "worst row abs", worst, "scale", scale, "u rel", e, plan.info()["near_subtri"])
    assert flips == 0 and worst <= 1e-12 * scale and e <= REL_E2E
    plan.close()
    mesh.close()


def test_ablation_driver_small_star(vp_ctx):
    """The ablation driver on a small star: its eps = 1e-15 reference agrees
    with the oracle, every setting stays within its tolerance, and the
    ellipse near field integrates fewer near sub-triangles than the ball
    tuned to the same error (on so small a mesh the ball may need fewer
    corrections; the counts are reported)."""
    from paper_2205_04401_amd import ablation
    res = ablation.run(vp_ctx, eps_list=(1e-10,), q=6, n_tri=600, n_sample=6, seed=60)
    prob = res["problem"]
    o = potential.Oracle(prob["vq"], prob["tq"], prob["p"], 6, 1e-15)
    x = prob["stag"][res["sample_stag"][:3]]
    ref = ablation.reference(vp_ctx, vp_ctx.mesh(prob["vq"], prob["tq"]), prob, 6, x)
    e_ref = rel_linf(ref, o.evaluate(prob["F"], x))
    r = res["rows"][0]
    say("ablation small:", ablation.table(res), "reference vs oracle", e_ref)
    assert e_ref <= REL_E2E
    assert r["star"]["E_abs"] < 1e-8 and r["plus"]["E_abs"] < 1e-8 and r["zero"]["E_abs"] <= 2 * r["star"]["E_abs"]
    assert r["star"]["s_n"] < r["zero"]["s_n"]


# ---------------------------------------------------------------------------
# curved boundary triangles (Sec. 3.1, eq. blend)
# ---------------------------------------------------------------------------

def _disk_targets(seed):
    rng = np.random.default_rng(seed)
    r = np.concatenate([rng.uniform(0, 0.99, 24), [1.0, 1.0, 1.0], rng.uniform(1.01, 3, 12), [0.995, 1.005]])
    a = rng.uniform(0, 2 * math.pi, len(r))
    return r, np.stack([r * np.cos(a), r * np.sin(a)], 1)


@pytest.fixture(scope="module")
def cdisk(vp_ctx):
    from oracle import curved
    v, t, ct, cs, cp = W.curved_disk(n_tri=200, n_boundary=30, seed=1, deg=16)
    mesh = vp_ctx.mesh(v, t, curved=(ct, cs, cp))
    return dict(v=v, t=t, curved=(ct, cs, cp), mesh=mesh, make=lambda p, q, eps: curved.CurvedOracle(
        v, t, ct, cs, cp, p, q, eps))


def test_curved_disk_map_points_and_unit_density_closed_form(vp_ctx, cdisk):
    """Mapped interpolation nodes equal the oracle's; unit density on the
    disk with circular boundary sides gives u = r^2/4 - 1/4 inside and
    (1/2) log r outside (the disk closed form) to within 1e-11, in FP64, at
    targets inside, outside and on the circle; mixed within 1e-6."""
    o = cdisk["make"](1, 8, 1e-13)
    X = rules.interp_nodes(4)
    dmap = np.abs(cdisk["mesh"].map_points(X) - o.node_positions(X)).max()
    r, tg = _disk_targets(11)
    plan = vp_ctx.plan(cdisk["mesh"], 1, 8, 1e-13, tg)
    F = np.ones((len(cdisk["t"]), 3))
    exact = np.where(r <= 1, r ** 2 / 4 - 0.25, 0.5 * np.log(r))
    e64 = np.abs(plan.execute(F) - exact).max() / np.abs(exact).max()
    emx = np.abs(plan.execute(F, mixed=True) - exact).max() / np.abs(exact).max()
    say("curved disk: map diff", dmap, "unit density vs closed form", e64, "mixed", emx)
    assert dmap < 1e-14 and e64 <= 1e-11 and emx <= 1e-6
    plan.close()


def test_curved_disk_pairs_rows_and_r2_density(vp_ctx, cdisk):
    """f = r^2 (p = 6): pair sets and rows match the oracle's (self pairs on
    curved triangles by Newton point location, near pairs on curved
    triangles, straight ones), u matches the oracle and the closed form
    r^4/16 - 1/16 inside, (1/4) log r outside."""
    p, q, eps = 6, 8, 1e-13
    o = cdisk["make"](p, q, eps)
    r, tg = _disk_targets(12)
    plan = vp_ctx.plan(cdisk["mesh"], p, q, eps, tg)
    flips = compare_pairs(plan, o, tg)
    rp, tri, kind = plan.pairs()
    rows = plan.rows()
    worst = scale = 0.0
    n_curved_pairs = 0
    for i in range(len(tg)):
        for j in range(rp[i], rp[i + 1]):
            if int(tri[j]) not in o.curves and i % 4:
                continue
            n_curved_pairs += int(tri[j]) in o.curves
            ref = o.row(int(tri[j]), tg[i], int(kind[j]))
            worst = max(worst, np.abs(rows[j] - ref).max())
            scale = max(scale, np.abs(ref).max())
    Y = o.node_positions(rules.interp_nodes(p))
    F = Y[:, :, 0] ** 2 + Y[:, :, 1] ** 2
    u = plan.execute(F)
    e_orc = rel_linf(u, o.evaluate(F, tg))
    exact = np.where(r <= 1, r ** 4 / 16 - 1 / 16, 0.25 * np.log(r))
    e_cf = np.abs(u - exact).max() / np.abs(exact).max()
    say("curved disk r^2: flips", flips, "pairs on curved triangles", n_curved_pairs, "rows worst", worst, "scale",
        scale, "vs oracle", e_orc, "vs closed form", e_cf)
    assert n_curved_pairs > 10 and worst <= 1e-12 * scale and e_orc <= REL_E2E and e_cf <= 1e-11
    plan.close()


def test_curved_star_sampled(vp_ctx):
    """The star with its boundary sides on r = 1 + 0.3 cos(5 theta) (2000
    triangles, p = 4, q = 6): sampled targets, incl. points on and next to
    the curved boundary, match the oracle."""
    from oracle import curved
    v, t, ct, cs, cp = W.curved_star(n_tri=2000, n_boundary=300, seed=70, deg=12)
    o = curved.CurvedOracle(v, t, ct, cs, cp, 4, 6, 1e-12)
    mesh = vp_ctx.mesh(v, t, curved=(ct, cs, cp))
    rng = np.random.default_rng(71)
    th = rng.uniform(0, 2 * math.pi, 8)
    onb = np.stack([W.star_radius(th) * np.cos(th), W.star_radius(th) * np.sin(th)], 1)
    tg = np.concatenate([rng.uniform(-1.2, 1.2, (10, 2)), onb, onb * 1.001, onb * 0.999])
    Y = o.node_positions(rules.interp_nodes(4))
    f = W.gaussian_sum(72, v, t)
    F = f(Y[:, :, 0], Y[:, :, 1])
    plan = vp_ctx.plan(mesh, 4, 6, 1e-12, tg)
    flips = compare_pairs(plan, o, tg)
    e = rel_linf(plan.execute(F), o.evaluate(F, tg))
    say("curved star: flips", flips, "rel vs oracle", e, "curved sides", len(ct))
    assert e <= REL_E2E
    plan.close()
    mesh.close()


# ---------------------------------------------------------------------------
# the potential anywhere: interpolation over a mesh element (Sec. 3.5)
# ---------------------------------------------------------------------------

def test_interp_locate_and_eval_match_oracle(vp_ctx):
    """Point location (straight and curved triangles, points on the curved
    boundary, outside points) and evaluation match the oracle's."""
    from numpy.polynomial import chebyshev as cheb
    from oracle import curved, interp
    v, t, ct, cs, cp = W.curved_star(n_tri=2000, n_boundary=300, seed=74, deg=12)
    o = curved.CurvedOracle(v, t, ct, cs, cp, 4, 6, 1e-10)
    mesh = vp_ctx.mesh(v, t, curved=(ct, cs, cp))
    it = vp_ctx.interp(mesh, 4)
    rng = np.random.default_rng(75)
    th = rng.uniform(0, 2 * math.pi, 40)
    rad = W.star_radius(th) * rng.uniform(0.0, 1.0, 40)
    pts = [np.stack([rad * np.cos(th), rad * np.sin(th)], 1)]
    for tc in list(o.curves)[:10]:  # points of curved sides
        uu = rng.uniform(0.05, 0.95)
        pts.append(np.array([[cheb.chebval(2 * uu - 1, o.curves[tc][0]), cheb.chebval(2 * uu - 1, o.curves[tc][1])]]))
    pts.append(np.array([[2.0, 2.0], [-1.4, 0.0]]))
    pts = np.concatenate(pts)
    tri, ref = it.locate(pts)
    n_same = worst_ref = 0
    for i, x in enumerate(pts):
        to, zo = interp.locate(o, x)
        assert (tri[i] < 0) == (to < 0), (i, tri[i], to)
        if to >= 0 and tri[i] == to:
            n_same += 1
            worst_ref = max(worst_ref, np.abs(ref[i] - zo).max())
    Y = o.node_positions(rules.interp_nodes(4))
    un = W.gaussian_sum(76, v, t)(Y[:, :, 0], Y[:, :, 1])
    u = it.eval(un, tri, ref)
    ref_u = np.array([interp.evaluate(4, un, tri[i], ref[i]) if tri[i] >= 0 else np.nan for i in range(len(pts))])
    inside = tri >= 0
    e = np.abs(u[inside] - ref_u[inside]).max() / np.abs(ref_u[inside]).max()
    say("interp: located", inside.sum(), "same triangle as the oracle", n_same, "ref diff", worst_ref, "eval rel", e)
    assert n_same >= inside.sum() - 2 and worst_ref < 1e-12 and e < 1e-13 and np.all(np.isnan(u[~inside]))
    it.close()
    mesh.close()


def test_potential_anywhere_on_a_curved_disk(vp_ctx):
    """Unit density on the curved disk: the potential computed at the p = 6
    nodes of a second, curved target mesh of the disk, then interpolated to
    arbitrary points and to points of the boundary (Sec. 3.5), matches the
    disk closed form to the interpolation error."""
    vq, tq, cq, sq, pq = W.curved_disk(n_tri=200, n_boundary=30, seed=1, deg=16)
    vt, tt, ctt, stt, ptt = W.curved_disk(n_tri=160, n_boundary=26, seed=5, deg=16)
    src = vp_ctx.mesh(vq, tq, curved=(cq, sq, pq))
    tgt = vp_ctx.mesh(vt, tt, curved=(ctt, stt, ptt))
    p = 6
    nodes = tgt.map_points(rules.interp_nodes(p)).reshape(-1, 2)
    plan = vp_ctx.plan(src, 1, 8, 1e-13, nodes)
    u_nodes = plan.execute(np.ones((len(tq), 3))).reshape(len(tt), -1)
    it = vp_ctx.interp(tgt, p)
    rng = np.random.default_rng(77)
    r = np.concatenate([np.sqrt(rng.uniform(0, 0.98, 30)), np.ones(10)])
    a = rng.uniform(0, 2 * math.pi, len(r))
    pts = np.stack([r * np.cos(a), r * np.sin(a)], 1)
    tri, ref = it.locate(pts)
    u = it.eval(u_nodes, tri, ref)
    exact = r ** 2 / 4 - 0.25
    e = np.abs(u - exact).max() / np.abs(exact).max()
    say("potential anywhere: located", (tri >= 0).sum(), "of", len(pts), "rel vs closed form", e)
    assert np.all(tri >= 0) and e < 1e-9
    it.close()
    plan.close()
    tgt.close()
    src.close()


def test_empty_target_set_and_single_triangle(vp_ctx):
    v = np.array([[0.0, 0.0], [1.0, 0.2], [0.1, 0.9]])
    t = np.array([[0, 2, 1]], dtype=np.int32)  # clockwise: the library swaps B and C
    mesh = vp_ctx.mesh(v, t)
    plan = vp_ctx.plan(mesh, 2, 5, 1e-12, np.zeros((0, 2)))
    assert plan.execute(np.ones((1, 6))).shape == (0,)
    plan.close()
    tg = np.array([[0.3, 0.3], [0.0, 0.0], [1.5, 1.5], [0.55, 0.1]])
    plan = vp_ctx.plan(mesh, 2, 5, 1e-12, tg)
    o = potential.Oracle(v, t, 2, 5, 1e-12)
    F = np.arange(6.0)[None, :] * 0.1 + 1.0
    assert rel_linf(plan.execute(F), o.evaluate(F, tg)) <= REL_E2E
    plan.close()
    mesh.close()


def test_sliver_triangles_depth_first_subdivision(vp_ctx):
    """Near pairs of triangles with aspect ratio ~1e3 need more sub-triangles
    per level than the breadth-first buffers hold; the kernel then walks the
    subdivision depth-first.  Results must still match the oracle."""
    vert = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 1e-3], [0.5, -8e-4], [1.2, 0.3], [-0.1, 0.25]])
    tri = np.array([[0, 1, 2], [0, 3, 1], [1, 4, 2], [0, 2, 5]], dtype=np.int32)
    p, q = 3, 6
    tg = np.array([[0.3, 2e-3], [0.7, -1.5e-3], [0.5, 0.01], [0.45, 4e-4], [0.2, -3e-4], [0.9, 0.05]])
    nodes = rules.interp_nodes(p)
    F = W.sample_density(lambda x, y: np.cos(2 * x) + y * y, vert, tri, nodes)
    mesh = vp_ctx.mesh(vert, tri)
    plan = vp_ctx.plan(mesh, p, q, 1e-12, tg)
    info = plan.info()
    say("sliver plan", {k: info[k] for k in ("n_pairs", "near_subtri", "depth_first_pairs", "capped_leaves")})
    assert info["depth_first_pairs"] > 0
    o = potential.Oracle(vert, tri, p, q, 1e-12)
    compare_pairs(plan, o, tg)
    err = rel_linf(plan.execute(F), o.evaluate(F, tg))
    say("sliver rel", err)
    assert err <= REL_E2E
    plan.close()
    mesh.close()


def test_error_paths(vp_ctx):
    from paper_2205_04401_amd import vp
    vq, tq = W.unit_square(2, "/")
    mesh = vp_ctx.mesh(vq, tq)
    tg = np.array([[0.5, 0.5]])
    for kw in (dict(p=0, q=8, eps=1e-12), dict(p=11, q=8, eps=1e-12), dict(p=2, q=1, eps=1e-12),
               dict(p=2, q=33, eps=1e-12), dict(p=2, q=8, eps=0.0), dict(p=2, q=8, eps=-1.0)):
        with pytest.raises(vp.VPError) as e:
            vp_ctx.plan(mesh, kw["p"], kw["q"], kw["eps"], tg)
        assert e.value.status == vp.VP_EINVAL
    with pytest.raises(vp.VPError) as e:
        vp_ctx.plan(mesh, 2, 8, 1e-12, np.array([[np.nan, 0.0]]))
    assert e.value.status == vp.VP_EINVAL
    bad = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 2.0]])
    with pytest.raises(vp.VPError) as e:
        vp_ctx.mesh(bad, np.array([[0, 1, 2]]))
    assert e.value.status == vp.VP_EINVAL
    with pytest.raises(vp.VPError) as e:
        vp_ctx.mesh(vq, np.array([[0, 1, 99]]))
    assert e.value.status == vp.VP_EINVAL
    plan = vp_ctx.plan(mesh, 2, 8, 1e-12, tg)
    with pytest.raises(vp.VPError) as e:
        mesh.close()
    assert e.value.status == vp.VP_EBUSY
    with pytest.raises(vp.VPError) as e:  # n_rhs = 0
        vp._check(vp.load().vp_execute(plan.h, 0, None, None, vp.VP_FP64, 0))
    assert e.value.status == vp.VP_EINVAL
    with pytest.raises(vp.VPError) as e:  # unknown precision
        vp._check(vp.load().vp_execute(plan.h, 1, vp._ptr(np.ones((len(tq), 6))), vp._ptr(np.zeros(1)), 7, 0))
    assert e.value.status == vp.VP_EINVAL
    plan.close()
    mesh.close()
    small = vp.Context(0, hbm_budget_bytes=4096)
    m2 = small.mesh(vq, tq)
    with pytest.raises(vp.VPError) as e:
        small.plan(m2, 6, 16, 1e-13, np.random.default_rng(0).uniform(0, 1, (500, 2)))
    assert e.value.status == vp.VP_ENOMEM
    m2.close()
    small.close()


# ---------------------------------------------------------------------------
# full-size star (the benchmark's workload): sampled targets vs the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q", [6, 8])
def test_star_mixed_loose_eps_plan(vp_ctx, q):
    """A mixed-precision plan with eps = 1e-8 (smaller near field) still meets
    1e-6 against the FP64, eps = 1e-13 oracle (q = 8: the configuration of
    the bench's C2 mixed sweep)."""
    p = 6
    vq, tq = W.star_mesh(n_tri=20000, seed=20)
    vt, tt = W.star_mesh(n_tri=20000, seed=21, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_sum(22, vq, tq), vq, tq, nodes)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, 1e-8, tg)
    u = plan.execute(F, mixed=True)
    rng = np.random.default_rng(99 + q)
    sample = np.sort(rng.choice(len(tg), 16, replace=False))
    ref = potential.Oracle(vq, tq, p, q, 1e-13).evaluate(F, tg[sample])
    err = np.abs(u[sample] - ref).max() / np.abs(ref).max()
    say("star mixed eps=1e-8 plan: pairs/target", plan.info()["n_pairs"] / len(tg), "rel", err)
    assert err <= REL_MIXED
    plan.close()
    mesh.close()

@pytest.mark.parametrize("q", [8, 4])
def test_star_full_size_sampled(vp_ctx, q):
    """The 20k-triangle star with its 559k staggered targets plus special
    ones (vertices, shared edges, slivers): pair lists, every row, the far
    sum and the potential at 64 seeded and all special targets."""
    p, eps = 6, 1e-13
    vq, tq = W.star_mesh(n_tri=20000, seed=20)
    vt, tt = W.star_mesh(n_tri=20000, seed=21, staggered=True)
    nodes = rules.interp_nodes(p)
    tg, sample = sample_with_special(W.node_positions(vt, tt, nodes).reshape(-1, 2), vq, tq, 64, 123 + q)
    F = W.sample_density(W.gaussian_sum(22, vq, tq), vq, tq, nodes)
    say("star: plan", len(tq), "triangles", len(tg), "targets,", len(sample), "sampled")
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    u = plan.execute(F)
    u_far = plan.execute(F, far_only=True)
    info = plan.info()
    say("star plan", {k: info[k] for k in ("n_pairs", "n_self", "near_subtri", "self_panels", "ms_classify",
                                          "ms_rows", "capped_leaves")})
    # every near pair integrates at least one leaf, every self pair one panel
    assert info["near_subtri"] >= info["n_pairs"] - info["n_self"]
    assert info["self_panels"] >= info["n_self"]
    o = potential.Oracle(vq, tq, p, q, eps)
    rp, tri, kind = plan.pairs()
    flips = compare_pairs(plan, o, tg, sample, (rp, tri, kind))
    worst, seen = compare_rows(plan, o, tg, sample, rp, tri, kind, tri_area(vq, tq), 10 * eps)
    ref_u, ref_far, _, _ = o.evaluate(F, tg[sample], return_parts=True)
    e_far = np.abs(u_far[sample] - ref_far).max() / np.abs(ref_far).max()
    e_all = np.abs(u[sample] - ref_u).max() / np.abs(ref_u).max()
    u_mix = plan.execute(F, mixed=True)
    e_mix = np.abs(u_mix[sample] - ref_u).max() / np.abs(ref_u).max()
    say("star sampled: band flips", flips, "rows compared", seen, "worst / area", worst, "rel far", e_far,
        "end-to-end", e_all, "mixed", e_mix)
    assert seen[0] > 0 and seen[1] > 0
    assert e_far <= REL_FAR
    assert e_all <= REL_E2E
    assert e_mix <= REL_MIXED
    plan.close()
    mesh.close()


def test_rows_near_and_self_launched_apart(vp_ctx):
    """At q = 16 on a star a quarter or more of the pairs are self pairs, so
    near and self rows come from two separate launches: each row equals the
    oracle's, and the end-to-end result meets the bar."""
    p, q, eps = 6, 16, 1e-13
    vq, tq = W.star_mesh(n_tri=1500, n_boundary=250, seed=60)  # a third of the pairs are self pairs
    vt, tt = W.star_mesh(n_tri=1500, n_boundary=250, seed=61, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_sum(62, vq, tq), vq, tq, nodes)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    info = plan.info()
    say("split rows: pairs", info["n_pairs"], "self", info["n_self"])
    assert 4 * info["n_self"] >= info["n_pairs"] > info["n_self"] > 0
    rp, tri, kind = plan.pairs()
    rows = plan.rows()
    o = potential.Oracle(vq, tq, p, q, eps)
    rng = np.random.default_rng(63)
    sample = np.sort(rng.choice(len(tg), 40, replace=False))
    # a row is a near integral minus its far-rule sum, both of the size of the
    # triangle's area times a logarithm: the bar is 10 eps times the area
    e1, e2 = vq[tq[:, 1]] - vq[tq[:, 0]], vq[tq[:, 2]] - vq[tq[:, 0]]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    worst, n_self, n_near = 0.0, 0, 0
    for i in sample:
        ref = {t: (k, o.row(t, tg[i], k)) for t, k in o.classify_target(tg[i])}
        for p_ in range(rp[i], rp[i + 1]):
            t = int(tri[p_])
            if t not in ref or ref[t][0] != int(kind[p_]):
                continue  # a pair on a decision boundary (checked by the pair-list tests)
            n_self += ref[t][0] == 0
            n_near += ref[t][0] == 1
            worst = max(worst, np.abs(rows[p_] - ref[t][1]).max() / area[t])
    u = plan.execute(F)
    ref_u = o.evaluate(F, tg[sample])
    e_all = np.abs(u[sample] - ref_u).max() / np.abs(ref_u).max()
    say("split rows: compared", n_self, "self and", n_near, "near rows, worst difference / area", worst,
        "end-to-end", e_all)
    assert n_self > 0 and n_near > 0
    assert worst <= 10 * eps
    assert e_all <= REL_E2E
    plan.close()
    mesh.close()


def near_depth_class(o, t, x):
    """Depth class of a near pair in the oracle's subdivision: 0 if the
    triangle itself is a leaf, 1 if it splits once into four leaves, else 2."""
    A, B, C, D = o.A[t], o.B[t], o.C[t], o.D[t]
    Nn = 2 * o.q_near - 1
    stack = [(np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0]), 0)]
    deepest = 0
    while stack:
        a, b, c, d = stack.pop()
        ra = abs((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]))
        P3 = potential.to_physical(A, B, C, np.stack([a, b, c]))
        if o.in_ellipses(x, P3, ra * D, o.near_what, Nn):
            m_ab, m_bc, m_ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            stack += [(a, m_ab, m_ca, d + 1), (m_ab, b, m_bc, d + 1), (m_ca, m_bc, c, d + 1), (m_bc, m_ca, m_ab, d + 1)]
        else:
            deepest = max(deepest, d)
    return min(deepest, 2)


@pytest.mark.parametrize("p", [4, 6])
def test_rows_of_every_depth_class(vp_ctx, p):
    """Near pairs whose subdivision stops at the triangle (class 0) or after
    one split (class 1) take the matrix-core row path, deeper near pairs and
    self pairs the per-pair path: on a graded L-shape at q = 4, where all
    four kinds are common, every sampled row of each kind equals the
    oracle's, and the end-to-end result meets the bar."""
    q, eps = 4, 1e-13
    vq, tq = W.l_shape_graded(n_tri=3000, seed=70)
    vt, tt = W.l_shape_graded(n_tri=3000, seed=71, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.l_shape_density(72), vq, tq, nodes)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    info = plan.info()
    rp, tri, kind = plan.pairs()
    rows = plan.rows()
    o = potential.Oracle(vq, tq, p, q, eps)
    rng = np.random.default_rng(73)
    sample = np.sort(np.concatenate([rng.choice(len(tg), 40, replace=False),
                                     np.argsort(np.hypot(tg[:, 0], tg[:, 1]))[:4]]))
    e1, e2 = vq[tq[:, 1]] - vq[tq[:, 0]], vq[tq[:, 2]] - vq[tq[:, 0]]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    worst = {0: 0.0, 1: 0.0, 2: 0.0, "self": 0.0}
    seen = {0: 0, 1: 0, 2: 0, "self": 0}
    for i in sample:
        ref = {t: (k, o.row(t, tg[i], k)) for t, k in o.classify_target(tg[i])}
        for p_ in range(rp[i], rp[i + 1]):
            t = int(tri[p_])
            if t not in ref or ref[t][0] != int(kind[p_]):
                continue  # a pair on a decision boundary (checked by the pair-list tests)
            cls = "self" if ref[t][0] == 0 else near_depth_class(o, t, tg[i])
            seen[cls] += 1
            worst[cls] = max(worst[cls], np.abs(rows[p_] - ref[t][1]).max() / area[t])
    u = plan.execute(F)
    ref_u = o.evaluate(F, tg[sample])
    e_all = np.abs(u[sample] - ref_u).max() / np.abs(ref_u).max()
    say("depth classes: pairs", info["n_pairs"], "compared", seen, "worst difference / area", worst,
        "end-to-end", e_all)
    assert all(v > 0 for v in seen.values()), seen
    assert max(worst.values()) <= 10 * eps
    assert e_all <= REL_E2E
    plan.close()
    mesh.close()


# ---------------------------------------------------------------------------
# serving: each result is the same alone and in the mix
# ---------------------------------------------------------------------------

def test_serving_results_equal_alone_and_in_mix(vp_ctx):
    import torch
    rng = np.random.default_rng(5)
    plans, inputs = [], []
    for k, (T, p) in enumerate(((600, 3), (1500, 4))):
        vq, tq = W.star_mesh(n_tri=T, n_boundary=120, seed=300 + k)
        vt, tt = W.star_mesh(n_tri=T, n_boundary=120, seed=310 + k, staggered=True)
        nodes = rules.interp_nodes(p)
        tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
        mesh = vp_ctx.mesh(vq, tq)
        plans.append((mesh, vp_ctx.plan(mesh, p, 6, 1e-12, tg), vq, tq, nodes))
    server = vp_ctx.server(n_slots=3, max_batch_rhs=24)
    inputs = []
    for i in range(40):
        k = int(rng.integers(2))
        mesh, plan, vq, tq, nodes = plans[k]
        R = int(rng.integers(1, 9))
        F = np.stack([W.sample_density(W.gaussian_sum(700 + 13 * i + r, vq, tq), vq, tq, nodes)
                      for r in range(R)], -1)
        mixed = bool(i % 3 == 0)
        Fd = torch.from_numpy(F).cuda()
        out = torch.full((plan.n_tgt, R), np.nan, dtype=torch.float64, device="cuda")
        inputs.append((k, F, mixed, out, Fd))
    torch.cuda.synchronize()
    # all requests arrive while the first batches run: later ones are packed
    reqs = [(k, F, mixed, out, server.submit(plans[k][1], Fd, out, mixed=mixed))
            for k, F, mixed, out, Fd in inputs]
    for _, _, _, _, t in reqs:
        server.wait(t)
    st = server.stats()
    say("serving stats", st)
    assert st["requests_done"] == 40 and st["batches"] < 40  # some requests were packed together
    # FP64: the same up to summation order.  Mixed: a request packed with
    # others into 16+ columns has its far sum on the FP32 matrix cores
    # instead of the FP32 vector ALUs, a different FP32 rounding; both are
    # within the mixed tolerance of the FP64 result, so they agree to twice it.
    worst = {False: 0.0, True: 0.0}
    for k, F, mixed, out, _ in reqs:
        alone = plans[k][1].execute(F, mixed=mixed)
        got = out.cpu().numpy()
        worst[mixed] = max(worst[mixed], rel_linf(got, alone))
        if mixed:  # and within the mixed tolerance of the FP64 evaluation
            assert rel_linf(got, plans[k][1].execute(F)) <= REL_MIXED
    say("serving: worst rel difference alone vs in the mix (fp64, mixed)", worst[False], worst[True])
    assert worst[False] <= 1e-14 and worst[True] <= 2 * REL_MIXED
    server.close()
    for mesh, plan, *_ in plans:
        plan.close()
        mesh.close()


def test_serving_poisson_run_reports_latency(vp_ctx):
    from paper_2205_04401_amd import serving
    for res in serving.run(vp_ctx, n_requests=40, tri_range=(500, 2000), n_meshes=2, budget_gb=4.0):
        say("serving run", res)
        assert res["p50_ms"] > 0 and res["p99_ms"] >= res["p50_ms"] and res["evals_per_s"] > 0
        assert res["rejected"] == 0
        assert res["in_use_bytes_at_end"] + res["cached_bytes_at_end"] <= res["hbm_budget_bytes"]


# ---------------------------------------------------------------------------
# graded L-shape (about 250k triangles, p = 4, the 16-node far rule, 3.7M
# targets) and the batched star (100k triangles, 64 densities)
# ---------------------------------------------------------------------------

def test_graded_l_shape_full_size_sampled(vp_ctx):
    """The graded L-shape at full size (250k triangles, 3.75M targets) plus
    special targets: interior vertices, shared edges, slivers, the
    re-entrant corner itself, points approaching it inside the domain and
    along its two boundary edges, and one in the removed quadrant.  Pair
    lists and every row of the 64 seeded, 8 nearest-corner and special
    targets against the oracle, then the potential (FP64 and mixed)."""
    p, q, eps = 4, 4, 1e-13
    vq, tq = W.l_shape_graded(n_tri=250000, seed=50)
    vt, tt = W.l_shape_graded(n_tri=250000, seed=51, staggered=True)
    nodes = rules.interp_nodes(p)
    tg0 = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    d = np.array([1e-8, 1e-5, 1e-3])[:, None]
    corner = np.concatenate([[[0.0, 0.0]], d * [-1.0, -1.0], d * [-1.0, 1.0], d * [1.0, -1.0],
                             d * [0.0, 1.0], d * [1.0, 0.0], [[1e-3, 1e-3]]])
    near_corner = tg0[np.argsort(np.hypot(tg0[:, 0], tg0[:, 1]))[:8]]
    tg, sample = sample_with_special(tg0, vq, tq, 64, 55, extra=(corner, near_corner))
    F = W.sample_density(W.l_shape_density(52), vq, tq, nodes)
    say("L-shape:", len(tq), "triangles", len(tg), "targets,", len(sample), "sampled")
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    info = plan.info()
    say("L-shape plan", {k: info[k] for k in ("n_pairs", "n_self", "tab_pairs", "near_subtri", "ms_classify",
                                              "ms_rows", "capped_leaves", "bytes_resident")})
    assert info["near_subtri"] >= info["n_pairs"] - info["n_self"]
    u = plan.execute(F)
    u_mix = plan.execute(F, mixed=True)
    o = potential.Oracle(vq, tq, p, q, eps)
    rp, tri, kind = plan.pairs()
    flips = compare_pairs(plan, o, tg, sample, (rp, tri, kind))
    worst, seen = compare_rows(plan, o, tg, sample, rp, tri, kind, tri_area(vq, tq), 10 * eps)
    ref = o.evaluate(F, tg[sample])
    e = np.abs(u[sample] - ref).max() / np.abs(ref).max()
    e_mix = np.abs(u_mix[sample] - ref).max() / np.abs(ref).max()
    say("L-shape sampled: band flips", flips, "rows compared", seen, "worst / area", worst, "rel", e,
        "mixed", e_mix)
    assert seen[0] > 0 and seen[1] > 0
    assert e <= REL_E2E and e_mix <= REL_MIXED
    plan.close()
    mesh.close()


@pytest.mark.parametrize("q,n_sample", [(8, 64), (12, 16)])
def test_batched_star_100k_64_densities(vp_ctx, q, n_sample):
    import torch
    p, eps, R = 6, 1e-13, 64
    vq, tq = W.star_mesh(n_tri=100000, n_boundary=2000, seed=30)
    vt, tt = W.star_mesh(n_tri=100000, n_boundary=2000, seed=31, staggered=True)
    nodes = rules.interp_nodes(p)
    tg_all = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    rng = np.random.default_rng(33)
    tg = tg_all[np.sort(rng.choice(len(tg_all), 2048, replace=False))]  # seeded target subset
    F = np.stack([W.sample_density(W.gaussian_sum(1000 + r, vq, tq), vq, tq, nodes) for r in range(R)], -1)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg)
    Fd = torch.from_numpy(F).cuda()
    u = plan.execute(Fd).cpu().numpy()
    u_mix = plan.execute(Fd, mixed=True).cpu().numpy()
    # every column equals its own single-density evaluation (batch invariance)
    for r in (0, 17, 63):
        assert rel_linf(u[:, r], plan.execute(np.ascontiguousarray(F[:, :, r]))) <= 1e-14
    # oracle on n_sample targets (the first, the last and seeded ones) and 8
    # columns (the oracle's extended-precision far sum over the 6.4M / 14.4M
    # sources takes about a second per target)
    cols = [0, 9, 17, 31, 40, 52, 58, 63]
    rest = np.random.default_rng(34 + q).choice(np.arange(1, len(tg) - 1), n_sample - 2, replace=False)
    sample = np.sort(np.concatenate([[0, len(tg) - 1], rest]))
    ref = potential.Oracle(vq, tq, p, q, eps).evaluate(np.ascontiguousarray(F[:, :, cols]), tg[sample])
    e = rel_linf(u[sample][:, cols], ref)
    e_mix = rel_linf(u_mix[sample][:, cols], ref)
    say(f"batched star q={q}: rel {e}, mixed {e_mix}")
    assert e <= REL_E2E and e_mix <= REL_MIXED
    plan.close()
    mesh.close()
