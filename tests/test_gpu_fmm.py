"""GPU parity of the FMM far sum (plan option fmm_terms > 0) against the
oracle's direct sum and the library's own direct-sum path.

The FMM approximates the direct sum of the far-rule point charges with an
error bound of 1.2 (sum |Q|) 0.547^p (p expansion terms); at the p used here
that is far below the FP64 bars of the direct path, which the FMM must meet
as well: far sum alone <= 1e-13 and end to end <= 1e-11 relative L-infinity
against the oracle.
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
REL_MIXED = 1e-6
P_FMM = 48


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_linf(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return float((np.abs(a - b).max(0) / np.abs(b).max(0)).max())


@pytest.fixture(scope="module")
def vp_ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2205_04401_amd import vp
    yield vp.Context(0)


@pytest.fixture(scope="module")
def square(vp_ctx):
    """Unit square 8x8 cells, p = 4, q = 8, eps = 1e-13, 1920 staggered
    targets: oracle far sum and potential, and an FMM plan (3 levels)."""
    p, q, eps = 4, 8, 1e-13
    vq, tq = W.unit_square(8, "/")
    vt, tt = W.unit_square(8, "\\")
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_bump, vq, tq, nodes)
    o = potential.Oracle(vq, tq, p, q, eps)
    u, u_far, _, _ = o.evaluate(F, tg, return_parts=True)
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, eps, tg, fmm_terms=P_FMM, fmm_leaf=64)
    return dict(vq=vq, tq=tq, tg=tg, F=F, o=o, u=u, u_far=u_far, mesh=mesh, plan=plan, p=p, q=q, eps=eps)


def test_fmm_square_far_sum_and_potential(square):
    plan = square["plan"]
    info = plan.info()
    say("fmm square: terms", info["fmm_terms"], "levels", info["fmm_levels"], "far_split", info["far_split"])
    assert info["fmm_terms"] == P_FMM and info["fmm_levels"] >= 2 and info["far_split"] == 1
    e_far = rel_linf(plan.execute(square["F"], far_only=True), square["u_far"])
    e_all = rel_linf(plan.execute(square["F"]), square["u"])
    e_mix = rel_linf(plan.execute(square["F"], mixed=True), square["u"])
    say("fmm square rel far", e_far, "end-to-end", e_all, "mixed", e_mix)
    assert e_far <= REL_FAR and e_all <= REL_E2E and e_mix <= REL_MIXED


def test_fmm_square_many_rhs_graph_and_determinism(square, vp_ctx):
    """17 densities (16 with matrix-core corrections + 1) match their
    one-density evaluations; a captured graph replays the eager result bit
    for bit; two evaluations agree bit for bit."""
    import torch
    from paper_2205_04401_amd import vp
    plan = square["plan"]
    F = square["F"]
    FR = np.ascontiguousarray(np.stack([(1.0 + 0.1 * r) * F - 0.02 * r for r in range(17)], -1))
    uR = plan.execute(FR)
    worst = max(rel_linf(uR[:, r], plan.execute(np.ascontiguousarray(FR[:, :, r]))) for r in (0, 9, 16))
    say("fmm 17 RHS worst rel vs one-RHS", worst)
    assert worst <= 1e-14
    assert np.array_equal(plan.execute(F), plan.execute(F))
    Fd = torch.from_numpy(FR[:, :, :3].copy()).cuda()
    Ud = torch.empty((len(square["tg"]), 3), dtype=torch.float64, device="cuda")
    ref = plan.execute(Fd).cpu().numpy()
    g = vp.Graph(plan, Fd, Ud)
    for k in range(3):
        Ud.zero_()
        plan.execute(Fd * 2.0)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Ud.cpu().numpy(), ref), k
    g.close()


def test_fmm_targets_on_sources_and_outside(square, vp_ctx):
    """Targets on far-rule nodes (a source at distance 0: the near-field sum
    of the FMM uses the direct sum's kernel, so the correction rows cancel
    it), on vertices, and outside the mesh (boxes of the grid that hold no
    sources)."""
    plan0 = square["plan"]
    src = plan0.sources()
    rng = np.random.default_rng(7)
    tg = np.concatenate([src[rng.choice(len(src), 40, replace=False)], square["vq"][:10],
                         rng.uniform(-2.0, 3.0, (30, 2))])
    plan = vp_ctx.plan(square["mesh"], square["p"], square["q"], square["eps"], tg, fmm_terms=P_FMM)
    direct = vp_ctx.plan(square["mesh"], square["p"], square["q"], square["eps"], tg)
    u = plan.execute(square["F"])
    ud = direct.execute(square["F"])
    ref = square["o"].evaluate(square["F"], tg)
    say("fmm on-source targets: rel vs direct", rel_linf(u, ud), "vs oracle", rel_linf(u, ref))
    assert rel_linf(u, ud) <= REL_FAR and rel_linf(u, ref) <= REL_E2E
    plan.close()
    direct.close()


@pytest.mark.parametrize("terms, leaf", [(56, 128), (40, 32)])
def test_fmm_star_matches_direct_sum(vp_ctx, terms, leaf):
    """A 3000-triangle star (p = 6, q = 6, 83 048 targets, 107 568 sources):
    the FMM far sum equals the direct far sum to <= 1e-13 (and to the
    oracle's at sampled targets), at two tree depths and expansion lengths."""
    p, q, eps = 6, 6, 1e-13
    vq, tq = W.star_mesh(n_tri=3000, n_boundary=300, seed=41)
    vt, tt = W.star_mesh(n_tri=3000, n_boundary=300, seed=141, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_sum(42, vq, tq), vq, tq, nodes)
    mesh = vp_ctx.mesh(vq, tq)
    fmm = vp_ctx.plan(mesh, p, q, eps, tg, fmm_terms=terms, fmm_leaf=leaf)
    direct = vp_ctx.plan(mesh, p, q, eps, tg)
    info = fmm.info()
    uf = fmm.execute(F, far_only=True)
    ud = direct.execute(F, far_only=True)
    e = rel_linf(uf, ud)
    say("fmm star terms", terms, "leaf", leaf, "levels", info["fmm_levels"], "rel vs direct far", e)
    assert e <= REL_FAR
    rng = np.random.default_rng(terms)
    sample = np.sort(rng.choice(len(tg), 8, replace=False))
    ref_u, ref_far, _, _ = potential.Oracle(vq, tq, p, q, eps).evaluate(F, tg[sample], return_parts=True)
    assert rel_linf(uf[sample], ref_far) <= REL_FAR
    assert rel_linf(fmm.execute(F)[sample], ref_u) <= REL_E2E
    fmm.close()
    direct.close()
    mesh.close()


def test_fmm_star_blocks_of_16_densities(vp_ctx):
    """81 densities on a 3000-triangle star: a pass of 64 and a pass of 16
    on the matrix cores (P2M, M2L, L2P and the near-field sum as products
    with the densities as columns) and one density alone; every column's far
    sum equals the direct far sum to <= 1e-13, and the potentials equal the
    one-density FMM evaluations."""
    p, q, eps = 6, 6, 1e-13
    vq, tq = W.star_mesh(n_tri=3000, n_boundary=300, seed=43)
    vt, tt = W.star_mesh(n_tri=3000, n_boundary=300, seed=143, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    R = 81
    base = [W.sample_density(W.gaussian_sum(500 + r, vq, tq), vq, tq, nodes) for r in range(9)]
    FR = np.ascontiguousarray(np.stack([(1.0 + 0.05 * r) * base[r % 9] - 0.3 * base[(r // 9) % 9] for r in range(R)],
                                       -1))
    mesh = vp_ctx.mesh(vq, tq)
    fmm = vp_ctx.plan(mesh, p, q, eps, tg, fmm_terms=40, fmm_leaf=64)
    direct = vp_ctx.plan(mesh, p, q, eps, tg)
    uf = fmm.execute(FR, far_only=True)
    ud = direct.execute(FR, far_only=True)
    e = rel_linf(uf, ud)
    u = fmm.execute(FR)
    e1 = max(rel_linf(u[:, r], fmm.execute(np.ascontiguousarray(FR[:, :, r]))) for r in (0, 37, 63, 64, 79, 80))
    say("fmm star 81 densities: far rel vs direct", e, "potential rel vs one-density FMM", e1)
    assert e <= REL_FAR and e1 <= REL_FAR
    fmm.close()
    direct.close()
    mesh.close()


@pytest.mark.parametrize("R", [7, 23])
def test_fmm_partial_blocks_of_densities(vp_ctx, R):
    """A number of densities that does not fill the blocks of 16: the rest
    (7 of 7, 7 of 23) runs as one block padded with zero columns in the FMM
    passes and in the matrix-core correction apply (84k targets, 5250
    clusters of 16); every column equals its one-density evaluation and the
    direct far sum, and sampled targets the oracle."""
    p, q, eps = 6, 6, 1e-13
    vq, tq = W.star_mesh(n_tri=3000, n_boundary=300, seed=44)
    vt, tt = W.star_mesh(n_tri=3000, n_boundary=300, seed=144, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    base = [W.sample_density(W.gaussian_sum(600 + r, vq, tq), vq, tq, nodes) for r in range(5)]
    FR = np.ascontiguousarray(np.stack([(1.0 + 0.1 * r) * base[r % 5] - 0.2 * base[(r // 5) % 5] for r in range(R)],
                                       -1))
    mesh = vp_ctx.mesh(vq, tq)
    fmm = vp_ctx.plan(mesh, p, q, eps, tg, fmm_terms=40, fmm_leaf=64)
    direct = vp_ctx.plan(mesh, p, q, eps, tg)
    uf = fmm.execute(FR, far_only=True)
    ud = direct.execute(FR, far_only=True)
    e = rel_linf(uf, ud)
    u = fmm.execute(FR)
    assert fmm.info()["cluster_entries"] > 0
    cols = sorted({0, R // 2, R - 2, R - 1})
    e1 = max(rel_linf(u[:, r], fmm.execute(np.ascontiguousarray(FR[:, :, r]))) for r in cols)
    ud_all = direct.execute(FR)
    e2 = rel_linf(u, ud_all)
    sample = np.sort(np.random.default_rng(45 + R).choice(len(tg), 6, replace=False))
    o = potential.Oracle(vq, tq, p, q, eps)
    e3 = max(rel_linf(u[sample, r], o.evaluate(np.ascontiguousarray(FR[:, :, r]), tg[sample])) for r in (0, R - 1))
    say(f"fmm star {R} densities: far rel vs direct", e, "vs one-density", e1, "vs direct path", e2, "vs oracle", e3)
    assert e <= REL_FAR and e1 <= REL_FAR and e2 <= REL_FAR and e3 <= REL_E2E
    fmm.close()
    direct.close()
    mesh.close()


@pytest.mark.parametrize("terms", [16, 32])
def test_fmm_mixed_precision_blocks(vp_ctx, terms):
    """Mixed precision on an FMM plan (the leaf passes of blocks of
    densities on the FP32 matrix cores, a plan at eps = 1e-8, 16 or 32
    expansion terms): 23 densities (a block of 16 and a padded block of 7)
    within 1e-6 of the FP64 eps = 1e-13 oracle at sampled targets."""
    p, q = 6, 6
    vq, tq = W.star_mesh(n_tri=3000, n_boundary=300, seed=46)
    vt, tt = W.star_mesh(n_tri=3000, n_boundary=300, seed=146, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    R = 23
    base = [W.sample_density(W.gaussian_sum(700 + r, vq, tq), vq, tq, nodes) for r in range(5)]
    FR = np.ascontiguousarray(np.stack([(1.0 + 0.1 * r) * base[r % 5] - 0.2 * base[(r // 5) % 5] for r in range(R)],
                                       -1))
    mesh = vp_ctx.mesh(vq, tq)
    plan = vp_ctx.plan(mesh, p, q, 1e-8, tg, fmm_terms=terms, fmm_leaf=64)
    u = plan.execute(FR, mixed=True)
    sample = np.sort(np.random.default_rng(47).choice(len(tg), 8, replace=False))
    o = potential.Oracle(vq, tq, p, q, 1e-13)
    e = max(rel_linf(u[sample, r], o.evaluate(np.ascontiguousarray(FR[:, :, r]), tg[sample])) for r in (0, 9, 16, 22))
    say(f"fmm mixed, {terms} terms, {R} densities: rel vs FP64 oracle", e)
    assert e <= REL_MIXED
    plan.close()
    mesh.close()


def test_fmm_star_100k_all_targets_64_densities(vp_ctx):
    """The batched configuration at full size: the 100k-triangle star, all
    2.8M staggered targets, 64 densities, q = 8, far sum by the FMM (32
    terms, leaves of 64) in passes of 16 densities; FP64 and mixed (a plan
    at eps = 1e-8 with 16 terms, FP32 leaf passes).  16 sampled targets
    (first, last, 14 seeded) x 8 columns against the oracle, and two columns
    against their one-density evaluation."""
    import torch
    p, q, eps, R = 6, 8, 1e-13, 64
    vq, tq = W.star_mesh(n_tri=100000, n_boundary=2000, seed=30)
    vt, tt = W.star_mesh(n_tri=100000, n_boundary=2000, seed=31, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = np.ascontiguousarray(np.stack([W.sample_density(W.gaussian_sum(1000 + r, vq, tq), vq, tq, nodes)
                                       for r in range(R)], -1))
    say("star 100k:", len(tq), "triangles", len(tg), "targets", R, "densities")
    mesh = vp_ctx.mesh(vq, tq)
    Fd = torch.from_numpy(F).cuda()
    cols = [0, 9, 17, 31, 40, 52, 58, 63]
    rest = np.random.default_rng(36).choice(np.arange(1, len(tg) - 1), 14, replace=False)
    sample = np.sort(np.concatenate([[0, len(tg) - 1], rest]))
    sample_d = torch.from_numpy(sample).cuda()
    got = {}
    for mixed, eps_plan, terms in ((False, eps, 32), (True, 1e-8, 16)):
        plan = vp_ctx.plan(mesh, p, q, eps_plan, tg, fmm_terms=terms, fmm_leaf=64)
        u = plan.execute(Fd, mixed=mixed)
        got[mixed] = u[sample_d].cpu().numpy()
        if not mixed:
            for r in (5, 63):
                one = plan.execute(Fd[:, :, r:r + 1].contiguous())
                assert rel_linf(got[mixed][:, r], one[sample_d].cpu().numpy()) <= REL_FAR
        say("plan", "mixed" if mixed else "fp64", {k: plan.info()[k] for k in ("n_pairs", "n_src", "ms_rows")})
        del u
        plan.close()
    ref = potential.Oracle(vq, tq, p, q, eps).evaluate(np.ascontiguousarray(F[:, :, cols]), tg[sample])
    e = rel_linf(got[False][:, cols], ref)
    e_mix = rel_linf(got[True][:, cols], ref)
    say("star 100k, 64 densities, FMM: rel vs oracle", e, "mixed", e_mix)
    assert e <= REL_E2E and e_mix <= REL_MIXED
    mesh.close()


def test_fmm_curved_disk_closed_form(vp_ctx):
    """Unit density on a disk with circular boundary sides (curved
    triangles, blending map), far sum by the FMM: u = r^2/4 - 1/4 inside and
    (1/2) log r outside, to within 1e-11, at targets inside, on and outside
    the circle."""
    v, t, ct, cs, cp = W.curved_disk(n_tri=200, n_boundary=30, seed=1, deg=16)
    mesh = vp_ctx.mesh(v, t, curved=(ct, cs, cp))
    rng = np.random.default_rng(11)
    r = np.concatenate([rng.uniform(0, 0.99, 24), [1.0, 1.0, 1.0], rng.uniform(1.01, 3, 12), [0.995, 1.005]])
    a = rng.uniform(0, 2 * math.pi, len(r))
    tg = np.stack([r * np.cos(a), r * np.sin(a)], 1)
    plan = vp_ctx.plan(mesh, 1, 8, 1e-13, tg, fmm_terms=40, fmm_leaf=16)
    exact = np.where(r <= 1, r ** 2 / 4 - 0.25, 0.5 * np.log(r))
    e = np.abs(plan.execute(np.ones((len(t), 3))) - exact).max() / np.abs(exact).max()
    say("fmm curved disk: levels", plan.info()["fmm_levels"], "unit density vs closed form", e)
    assert e <= 1e-11
    plan.close()
    mesh.close()


def test_fmm_serving_alone_and_in_mix(vp_ctx):
    """Requests of 1-8 densities on FMM plans through the continuous-batching
    server: packed batches of 16+ columns run the matrix-core passes, a lone
    request the one-density passes; every result agrees with the request's
    own evaluation to 1e-13."""
    import torch
    rng = np.random.default_rng(9)
    plans = []
    for k, (T, p) in enumerate(((600, 3), (1500, 4))):
        vq, tq = W.star_mesh(n_tri=T, n_boundary=120, seed=320 + k)
        vt, tt = W.star_mesh(n_tri=T, n_boundary=120, seed=330 + k, staggered=True)
        nodes = rules.interp_nodes(p)
        tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
        mesh = vp_ctx.mesh(vq, tq)
        plans.append((mesh, vp_ctx.plan(mesh, p, 6, 1e-12, tg, fmm_terms=40, fmm_leaf=32), vq, tq, nodes))
    server = vp_ctx.server(n_slots=3, max_batch_rhs=32)
    reqs = []
    for i in range(30):
        k = int(rng.integers(2))
        mesh, plan, vq, tq, nodes = plans[k]
        R = int(rng.integers(1, 9))
        F = np.stack([W.sample_density(W.gaussian_sum(900 + 7 * i + r, vq, tq), vq, tq, nodes) for r in range(R)], -1)
        out = torch.full((plan.n_tgt, R), np.nan, dtype=torch.float64, device="cuda")
        reqs.append((k, F, out, torch.from_numpy(F).cuda()))
    torch.cuda.synchronize()
    tickets = [server.submit(plans[k][1], Fd, out) for k, F, out, Fd in reqs]
    for t in tickets:
        server.wait(t)
    st = server.stats()
    worst = max(rel_linf(out.cpu().numpy(), plans[k][1].execute(F)) for k, F, out, _ in reqs)
    say("fmm serving:", st, "worst rel alone vs in the mix", worst)
    assert st["requests_done"] == 30 and st["batches"] < 30 and worst <= 1e-13
    server.close()
    for mesh, plan, *_ in plans:
        plan.close()
        mesh.close()


def test_fmm_option_errors(square, vp_ctx):
    from paper_2205_04401_amd import vp
    for terms, leaf in ((5, 128), (64, 128), (40, 4), (40, 5000)):
        with pytest.raises(vp.VPError):
            vp_ctx.plan(square["mesh"], 4, 8, 1e-13, square["tg"][:10], fmm_terms=terms, fmm_leaf=leaf)
    plan = square["plan"]
    with pytest.raises(vp.VPError):
        plan.set_far_config("wide", 4, 8)  # an FMM plan has one partial sum per target
    plan.set_far_config("wide", 4, 1)
    cfg, ms = plan.autotune(n_rhs=1, reps=2)  # nothing to choose: times the one shape
    assert cfg["n_split"] == 1 and ms > 0
