"""Serving under an HBM budget, through the C ABI: with a budget that holds
the plans and about one slot's workspace, batches wait for running ones to
retire (the server counts the waits), every request still completes, and
each served result matches the oracle at sampled targets and the same
evaluation made alone."""

import numpy as np
import pytest

from oracle import potential, rules
from paper_2205_04401_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_E2E = 1e-11


def say(*a):
    print(*a, flush=True)


def meshes():
    out = []
    for k, (n_tri, p) in enumerate(((900, 4), (1300, 6))):
        vq, tq = W.star_mesh(n_tri=n_tri, n_boundary=200, seed=90 + k)
        vt, tt = W.star_mesh(n_tri=n_tri, n_boundary=200, seed=95 + k, staggered=True)
        nodes = rules.interp_nodes(p)
        tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
        out.append(dict(vq=vq, tq=tq, tg=tg, p=p, nodes=nodes))
    return out


def densities(m, R, seed):
    return np.ascontiguousarray(np.stack(
        [W.sample_density(W.gaussian_sum(seed + r, m["vq"], m["tq"]), m["vq"], m["tq"], m["nodes"])
         for r in range(R)], -1))


def build(ctx, ms, q=6, eps=1e-12):
    for m in ms:
        m["mesh"] = ctx.mesh(m["vq"], m["tq"])
        m["plan"] = ctx.plan(m["mesh"], m["p"], q, eps, m["tg"])


def close(ms):
    for m in ms:
        m["plan"].close()
        m["mesh"].close()


def test_serving_waits_for_budget_and_matches_oracle():
    import torch
    from paper_2205_04401_amd import vp
    assert torch.cuda.is_available()
    ms = meshes()
    width = 8
    rng = np.random.default_rng(91)
    reqs = []
    for i in range(12):
        k = int(rng.integers(len(ms)))
        R = int(rng.integers(2, width + 1))
        reqs.append(dict(k=k, R=R, F=densities(ms[k], R, 1000 + 37 * i)))
    # probe (no budget): memory of the plans, then of one slot's workspace at
    # full width; each request's evaluation alone
    probe = vp.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    build(probe, ms)
    base, _ = probe.memory()
    srv = probe.server(n_slots=1, max_batch_rhs=width)
    slot = 0
    for m in ms:  # the slot grows to the larger plan's workspace
        F = torch.from_numpy(densities(m, width, 300)).cuda()
        out = torch.empty((m["plan"].n_tgt, width), dtype=torch.float64, device="cuda")
        srv.wait(srv.submit(m["plan"], F, out))
        slot = max(slot, probe.memory()[0] - base)
    srv.close()
    for r in reqs:
        r["alone"] = ms[r["k"]]["plan"].execute(r["F"])
    close(ms)
    probe.close()
    budget = base + int(1.4 * slot)
    say("plans", base, "bytes; one slot at width", width, ":", slot, "bytes; budget", budget)

    ctx = vp.Context(0, stream=torch.cuda.current_stream().cuda_stream, hbm_budget_bytes=budget)
    build(ctx, ms)
    srv = ctx.server(n_slots=3, max_batch_rhs=width)
    # the server keeps its context alive
    with pytest.raises(vp.VPError) as ei:
        vp._check(vp.load().vp_ctx_destroy(ctx.h))
    assert ei.value.status == vp.VP_EBUSY
    for r in reqs:
        r["F_d"] = torch.from_numpy(r["F"]).cuda()
        r["out"] = torch.full((ms[r["k"]]["plan"].n_tgt, r["R"]), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    tickets = [srv.submit(ms[r["k"]]["plan"], r["F_d"], r["out"]) for r in reqs]
    in_use, cached = ctx.memory()
    assert in_use + cached <= budget
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    in_use, cached = ctx.memory()
    say("served", st, "in use", in_use, "cached", cached)
    assert st["requests_done"] == len(reqs) and st["rejected"] == 0
    assert st["budget_waits"] > 0, "the budget never made a batch wait"
    assert in_use + cached <= budget
    worst_alone, worst_oracle = 0.0, 0.0
    oracles = [potential.Oracle(m["vq"], m["tq"], m["p"], 6, 1e-12) for m in ms]
    for i, r in enumerate(reqs):
        m = ms[r["k"]]
        u = r["out"].cpu().numpy()
        alone = r["alone"]
        worst_alone = max(worst_alone, float(np.abs(u - alone).max() / np.abs(alone).max()))
        sample = np.sort(np.random.default_rng(500 + i).choice(len(m["tg"]), 4, replace=False))
        col = i % r["R"]
        ref = oracles[r["k"]].evaluate(np.ascontiguousarray(r["F"][:, :, col]), m["tg"][sample])
        worst_oracle = max(worst_oracle, float(np.abs(u[sample, col] - ref).max() / np.abs(ref).max()))
    say("served vs alone", worst_alone, "vs oracle", worst_oracle)
    assert worst_alone <= 1e-13 and worst_oracle <= REL_E2E
    srv.close()
    close(ms)
    ctx.close()
