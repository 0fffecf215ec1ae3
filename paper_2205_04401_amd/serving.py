"""Request-serving workload: Poisson arrivals over resident meshes.

Seeded star meshes of log-uniform sizes stay resident on the device with
their plans (near lists, FP64 correction rows, the far sum's FMM tree);
requests of 1-32 right-hand sides arrive as a Poisson process and go
through the library's continuous-batching server (vp_server_*) under a
stated HBM budget.  Reports p50/p99 latency (arrival to observed
completion) beside throughput in potential evaluations per second (targets
x right-hand sides).

Each request's densities are a seeded combination of eight Gaussian-sum
densities of its mesh, formed on the device when the request arrives (input
generation: the densities of a request on a 200k-triangle mesh are ~1 GB,
a thousand of them do not fit anywhere at once).  Only argument
marshalling, input generation and clocks live here; all evaluation work
runs in libvp.
"""

import math
import time

import numpy as np

from . import vp
from . import workloads as W

N_BASIS = 8  # Gaussian-sum densities per mesh that requests combine


def build_meshes(ctx, n_meshes=8, tri_range=(1000, 200000), seed=40, device="cuda:0"):
    """Meshes (log-uniform triangle counts), their staggered target nodes for
    p = 4 and 6, and density bases on the device."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1]), n_meshes))).astype(int)
    meshes = []
    for k, T in enumerate(sizes):
        nb = int(min(2000, max(200, math.sqrt(T) * 4.5)))
        vq, tq = W.star_mesh(n_tri=int(T), n_boundary=nb, seed=seed + 1 + k)
        vt, tt = W.star_mesh(n_tri=int(T), n_boundary=nb, seed=seed + 101 + k, staggered=True)
        entry = dict(vq=vq, tq=tq, mesh=ctx.mesh(vq, tq), plans={}, basis={}, tg={})
        for p in (4, 6):
            nodes = vp.ref_nodes(p)
            entry["tg"][p] = torch.from_numpy(W.node_positions(vt, tt, nodes).reshape(-1, 2)).to(device)
            cols = [W.sample_density(W.gaussian_sum(seed + 1000 * k + 10 * p + b, vq, tq), vq, tq, nodes)
                    .reshape(-1) for b in range(N_BASIS)]
            entry["basis"][p] = torch.from_numpy(np.ascontiguousarray(np.stack(cols, -1))).to(device)
        meshes.append(entry)
    return meshes, [int(s) for s in sizes]


def build_plans(ctx, meshes, q, eps, fmm_terms):
    for m in meshes:
        for p in (4, 6):
            opts = {"fmm_terms": fmm_terms, "fmm_leaf": 64} if fmm_terms else {}
            m["plans"][p] = ctx.plan(m["mesh"], p, q, eps, m["tg"][p], **opts)


def close_plans(meshes):
    for m in meshes:
        for p in list(m["plans"]):
            m["plans"].pop(p).close()


def requests(meshes, n_requests=1000, max_rhs=32, seed=49):
    """The request list: mesh, order p (4 or 6), R ~ U{1..max_rhs}, and the
    seed of its combination of the mesh's basis densities."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_requests):
        k = int(rng.integers(len(meshes)))
        p = int(rng.choice([4, 6]))
        R = int(rng.integers(1, max_rhs + 1))
        n_tgt = meshes[k]["tg"][p].shape[0]
        reqs.append(dict(mesh=k, p=p, R=R, seed=10_000 + i, evals=n_tgt * R))
    return reqs


def request_inputs(wl, r, device="cuda:0"):
    """The request's densities [n_tri, n_p, R] (a seeded combination of the
    mesh's basis densities) and an output buffer, on the device."""
    import torch
    m = wl["meshes"][r["mesh"]]
    plan = m["plans"][r["p"]]
    g = torch.Generator(device="cpu").manual_seed(r["seed"])
    coef = torch.randn((N_BASIS, r["R"]), generator=g, dtype=torch.float64).to(device)
    F = (m["basis"][r["p"]] @ coef).reshape(plan.n_tri, plan.n_p, r["R"]).contiguous()
    out = torch.empty((plan.n_tgt, r["R"]), dtype=torch.float64, device=device)
    return F, out


def drive(server, wl, mixed, arrivals=None, max_outstanding=24):
    """Submit every request (at its arrival time, or as soon as fewer than
    max_outstanding are in flight when arrivals is None) and poll until all
    are done.  Returns (latencies s, total s, evals/s)."""
    import torch
    n = len(wl["reqs"])
    done_at = np.zeros(n)
    start_at = np.zeros(n)
    outstanding = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while i < n or outstanding:
        now = time.perf_counter() - t0
        while i < n and (arrivals[i] <= now if arrivals is not None else len(outstanding) < max_outstanding):
            r = wl["reqs"][i]
            F, out = request_inputs(wl, r)
            plan = wl["meshes"][r["mesh"]]["plans"][r["p"]]
            start_at[i] = arrivals[i] if arrivals is not None else time.perf_counter() - t0
            outstanding[server.submit(plan, F, out, mixed=mixed)] = (i, F, out)
            i += 1
            now = time.perf_counter() - t0
        for t in list(outstanding):
            if server.poll(t):
                j = outstanding.pop(t)[0]
                done_at[j] = time.perf_counter() - t0
        if outstanding and (i >= n or arrivals is None or arrivals[i] > time.perf_counter() - t0):
            time.sleep(2e-4)
        elif not outstanding and i < n and arrivals is not None:
            time.sleep(max(0.0, min(1e-3, arrivals[i] - (time.perf_counter() - t0))))
    total = time.perf_counter() - t0
    return done_at - start_at, total, sum(r["evals"] for r in wl["reqs"]) / total


def run(ctx, n_requests=1000, modes=("fp64", "mixed"), n_slots=4, max_batch_rhs=32, load=0.8, budget_gb=128.0,
        q=8, n_meshes=8, tri_range=(1000, 200000), seed=40):
    """For each mode, on the same meshes and request list: plans, saturated
    throughput (requests kept in flight), then a Poisson run at `load` times
    the saturated request rate.  Modes: "fp64" (plans at eps = 1e-13, FMM
    with 32 terms, FP64 evaluation) and "mixed" (plans at eps = 1e-8, FMM
    with 16 terms, VP_MIXED evaluation: the FMM's leaf passes on the FP32
    matrix cores).  The run makes its own context with the HBM budget on
    ctx's device.  Returns one dict of metrics per mode."""
    import torch
    budget = int(budget_gb * (1 << 30))
    sctx = vp.Context(ctx.device, stream=torch.cuda.current_stream().cuda_stream, hbm_budget_bytes=budget)
    t0 = time.perf_counter()
    meshes, sizes = build_meshes(sctx, n_meshes=n_meshes, tri_range=tri_range, seed=seed)
    t_meshes = time.perf_counter() - t0
    reqs = requests(meshes, n_requests=n_requests)
    out = []
    for mode in modes:
        mixed = mode == "mixed"
        eps, terms = (1e-8, 16) if mixed else (1e-13, 32)
        t0 = time.perf_counter()
        build_plans(sctx, meshes, q, eps, terms)
        t_plans = time.perf_counter() - t0
        wl = dict(meshes=meshes, reqs=reqs)
        server = sctx.server(n_slots=n_slots, max_batch_rhs=max_batch_rhs)
        drive(server, dict(meshes=meshes, reqs=reqs[:64]), mixed)  # workspaces, code objects, FMM tables
        _, dt_sat, evals_sat = drive(server, wl, mixed)
        rate = load * len(reqs) / dt_sat
        arrivals = np.cumsum(np.random.default_rng(49).exponential(1.0 / rate, len(reqs)))
        lat, total, evals = drive(server, wl, mixed, arrivals=arrivals)
        st = server.stats()
        in_use, cached = sctx.memory()
        server.close()
        resident = sum(m["plans"][p].info()["bytes_resident"] for m in meshes for p in (4, 6))
        close_plans(meshes)
        out.append({
            "precision": mode, "far": "fmm", "fmm_terms": terms, "plan_eps": eps, "q": q,
            "requests": len(reqs), "mesh_triangles": sizes, "rhs_per_request": "U{1..32}",
            "setup_s": {"meshes": t_meshes, "plans": t_plans}, "plans_resident_bytes": resident,
            "hbm_budget_bytes": budget, "in_use_bytes_at_end": in_use, "cached_bytes_at_end": cached,
            "saturated_evals_per_s": evals_sat, "arrival_rate_per_s": rate, "evals_per_s": evals,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "batches": st["batches"], "columns": st["columns"], "budget_waits": st["budget_waits"],
            "rejected": st["rejected"], "slots": n_slots, "max_batch_rhs": max_batch_rhs,
        })
    for m in meshes:
        m["mesh"].close()
    sctx.close()
    return out
