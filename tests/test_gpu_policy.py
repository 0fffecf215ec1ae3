"""The far-order policy (vp_choose_q) on a 3000-triangle star through the C
ABI: every order in the range is measured, the returned order has the least
plan + n_solves x evaluation time of the reported ones, a plan serving many
evaluations takes an order no higher than a plan used once (with the direct
far sum the evaluation grows with q^2 while the plan shrinks with the near
field), and a plan at the chosen order meets the end-to-end bar against the
oracle."""

import math

import numpy as np
import pytest

from oracle import potential, rules
from paper_2205_04401_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_choose_q_direct_and_fmm():
    import torch
    assert torch.cuda.is_available()
    from paper_2205_04401_amd import vp
    p, eps = 6, 1e-13
    vq, tq = W.star_mesh(n_tri=3000, n_boundary=300, seed=80)
    vt, tt = W.star_mesh(n_tri=3000, n_boundary=300, seed=81, staggered=True)
    nodes = rules.interp_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    ctx = vp.Context(0)
    mesh = ctx.mesh(vq, tq)
    chosen = {}
    for label, opts, n_solves in (("direct, 1", {}, 1.0), ("direct, 1000", {}, 1000.0),
                                  ("fmm, 1", {"fmm_terms": 32, "fmm_leaf": 64}, 1.0)):
        q, times = ctx.choose_q(mesh, p, eps, tg, q_min=4, q_max=10, n_solves=n_solves, **opts)
        say(label, "->", q, {k: (round(a, 2), round(b, 3)) for k, (a, b) in times.items()})
        assert sorted(times) == list(range(4, 11))
        assert all(math.isfinite(a) and a > 0 and math.isfinite(b) and b > 0 for a, b in times.values())
        cost = {k: a + n_solves * b for k, (a, b) in times.items()}
        assert cost[q] == min(cost.values())
        chosen[label] = (q, times)
    assert chosen["direct, 1000"][0] <= chosen["direct, 1"][0]
    # the evaluation time of the direct sum grows with the order
    t = chosen["direct, 1"][1]
    assert t[10][1] > t[4][1]
    # a plan at the order chosen for one evaluation meets the bar
    q = chosen["direct, 1"][0]
    F = W.sample_density(W.gaussian_sum(82, vq, tq), vq, tq, nodes)
    plan = ctx.plan(mesh, p, q, eps, tg)
    u = plan.execute(F)
    sample = np.sort(np.random.default_rng(83).choice(len(tg), 12, replace=False))
    ref = potential.Oracle(vq, tq, p, q, eps).evaluate(F, tg[sample])
    err = float(np.abs(u[sample] - ref).max() / np.abs(ref).max())
    say("plan at q =", q, "rel vs oracle", err)
    assert err <= 1e-11
    with pytest.raises(vp.VPError) as ei:
        ctx.choose_q(mesh, p, eps, tg, q_min=9, q_max=4)
    assert ei.value.status == vp.VP_EINVAL
    plan.close()
    mesh.close()
    ctx.close()
