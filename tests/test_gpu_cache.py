"""The context's cache of device blocks: plans built from blocks that earlier
plans used (and left full of their own data) give the same potentials as
plans built on fresh allocations, and the oracle's at sampled targets; the
cache empties on trim and stays inside an HBM budget."""

import sys

import numpy as np
import pytest

from oracle import potential, rules
from paper_2205_04401_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_E2E = 1e-11


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case(p, n_tri, seed):
    vq, tq = W.star_mesh(n_tri=n_tri, seed=seed)
    vt, tt = W.star_mesh(n_tri=n_tri, seed=seed + 1, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_sum(seed + 2, vq, tq), vq, tq, nodes)
    return vq, tq, tg, F


def run(ctx, vq, tq, tg, F, p, q, eps):
    mesh = ctx.mesh(vq, tq)
    plan = ctx.plan(mesh, p, q, eps, tg)
    u = plan.execute(F)
    held = plan.info()["bytes_resident"]
    plan.close()
    mesh.close()
    return u, held


def check_oracle(vq, tq, tg, F, p, q, eps, u, seed):
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(len(tg), 8, replace=False))
    ref = potential.Oracle(vq, tq, p, q, eps).evaluate(F, tg[sample])
    return float(np.abs(u[sample] - ref).max() / np.abs(ref).max())


def test_plans_on_cached_blocks():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2205_04401_amd import vp
    ctx = vp.Context(0)
    try:
        a = case(4, 1500, 40)
        b = case(6, 1200, 50)
        say("cache: plan A on fresh blocks")
        u_a, held_a = run(ctx, *a, 4, 8, 1e-12)
        cached = ctx.cached_bytes()
        say("cache: held", held_a, "cached after close", cached)
        assert cached >= held_a > 0
        # B reuses A's blocks where sizes allow (then holding A's data)
        say("cache: plan B on A's blocks")
        u_b, _ = run(ctx, *b, 6, 8, 1e-12)
        err_b = check_oracle(*b, 6, 8, 1e-12, u_b, 1)
        say("cache: B vs oracle", err_b)
        assert err_b <= REL_E2E
        # A again, now on blocks that held A's and B's data
        say("cache: plan A again")
        u_a2, _ = run(ctx, *a, 4, 8, 1e-12)
        rel = float(np.abs(u_a2 - u_a).max() / np.abs(u_a).max())
        err_a = check_oracle(*a, 4, 8, 1e-12, u_a2, 2)
        say("cache: A repeat vs first", rel, "vs oracle", err_a)
        assert rel <= 1e-15 and err_a <= REL_E2E
        ctx.trim()
        assert ctx.cached_bytes() == 0
        # after the trim every block is fresh again
        u_a3, _ = run(ctx, *a, 4, 8, 1e-12)
        assert float(np.abs(u_a3 - u_a).max() / np.abs(u_a).max()) <= 1e-15
    finally:
        ctx.close()


def test_cache_within_budget():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2205_04401_amd import vp
    a = case(4, 1500, 40)
    probe = vp.Context(0)
    try:
        _, held = run(probe, *a, 4, 8, 1e-12)
    finally:
        probe.close()
    # room for the mesh, one plan and its workspace, not for a second plan
    budget = int(1.6 * held) + (8 << 20)
    ctx = vp.Context(0, hbm_budget_bytes=budget)

    def within():
        in_use, cached = ctx.memory()
        say("cache budget", budget, "in use", in_use, "cached", cached)
        assert in_use + cached <= budget
        return in_use, cached

    try:
        vq, tq, tg, F = a
        mesh = ctx.mesh(vq, tq)
        plan = ctx.plan(mesh, 4, 8, 1e-12, tg)
        in_use, _ = within()
        # every block the plan holds is counted (rounded sizes included)
        assert in_use >= plan.info()["bytes_resident"]
        u1 = plan.execute(F)  # the workspace joins the plan
        in_use2, _ = within()
        assert in_use2 >= plan.info()["bytes_resident"] > 0
        plan.close()
        within()
        # a second plan on the cached blocks, then one more than the budget
        # holds next to it: refused, everything still within the budget
        plan = ctx.plan(mesh, 4, 8, 1e-12, tg)
        u2 = plan.execute(F)
        within()
        with pytest.raises(vp.VPError) as ei:
            ctx.plan(mesh, 4, 8, 1e-12, tg)
        assert ei.value.status == vp.VP_ENOMEM
        within()
        assert float(np.abs(u2 - u1).max() / np.abs(u1).max()) <= 1e-15
        plan.close()
        mesh.close()
        in_use, cached = within()
        assert in_use == 0
        ctx.trim()
        assert ctx.memory() == (0, 0)
    finally:
        ctx.close()
