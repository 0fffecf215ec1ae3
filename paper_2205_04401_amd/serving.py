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


def build_workload(ctx, n_meshes=8, tri_range=(1000, 200000), q=8, eps=1e-13, seed=40, n_requests=1000,
                   max_rhs=32, device="cuda:0", fmm_terms=32):
    """Meshes (log-uniform triangle counts; p = 4 or 6 per request), their
    plans, density bases on the device, and the request list (mesh, p, R,
    combination seed).  Returns a dict."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1]), n_meshes))).astype(int)
    meshes = []
    for k, T in enumerate(sizes):
        nb = int(min(2000, max(200, math.sqrt(T) * 4.5)))
        vq, tq = W.star_mesh(n_tri=int(T), n_boundary=nb, seed=seed + 1 + k)
        vt, tt = W.star_mesh(n_tri=int(T), n_boundary=nb, seed=seed + 101 + k, staggered=True)
        mesh = ctx.mesh(vq, tq)
        entry = dict(vq=vq, tq=tq, mesh=mesh, plans={}, basis={}, tg={})
        for p in (4, 6):
            nodes = vp.ref_nodes(p)
            tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
            cols = [W.sample_density(W.gaussian_sum(seed + 1000 * k + 10 * p + b, vq, tq), vq, tq, nodes)
                    .reshape(-1) for b in range(N_BASIS)]
            entry["basis"][p] = torch.from_numpy(np.ascontiguousarray(np.stack(cols, -1))).to(device)
            entry["tg"][p] = tg
            opts = {"fmm_terms": fmm_terms, "fmm_leaf": 64} if fmm_terms else {}
            entry["plans"][p] = ctx.plan(mesh, p, q, eps, torch.from_numpy(tg).to(device), **opts)
        meshes.append(entry)
    reqs = []
    for i in range(n_requests):
        k = int(rng.integers(n_meshes))
        p = int(rng.choice([4, 6]))
        R = int(rng.integers(1, max_rhs + 1))
        plan = meshes[k]["plans"][p]
        reqs.append(dict(mesh=k, p=p, R=R, seed=10_000 + i, evals=plan.n_tgt * R))
    return dict(meshes=meshes, reqs=reqs, sizes=[int(s) for s in sizes], q=q, eps=eps)


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


def drive(server, wl, mixed, arrivals=None, max_outstanding=48):
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


def run(ctx, n_requests=1000, mixed=False, eps=None, n_slots=4, max_batch_rhs=64, load=0.8, budget_gb=200.0,
        **kw):
    """Saturated throughput (requests kept in flight), then a Poisson run at
    `load` times the saturated request rate.  Returns a dict of metrics.
    The context passed in is only used for its device; the run makes its own
    context with the HBM budget."""
    import torch
    eps = eps if eps is not None else (1e-8 if mixed else 1e-13)
    budget = int(budget_gb * (1 << 30))
    sctx = vp.Context(ctx.device, stream=torch.cuda.current_stream().cuda_stream, hbm_budget_bytes=budget)
    t_build = time.perf_counter()
    wl = build_workload(sctx, n_requests=n_requests, eps=eps, **kw)
    t_build = time.perf_counter() - t_build
    server = sctx.server(n_slots=n_slots, max_batch_rhs=max_batch_rhs)
    warm = dict(wl, reqs=wl["reqs"][:64])
    drive(server, warm, mixed)  # workspaces, code objects, FMM tables of 16+ densities
    _, dt_sat, evals_sat = drive(server, wl, mixed)
    rate = load * len(wl["reqs"]) / dt_sat
    arrivals = np.cumsum(np.random.default_rng(49).exponential(1.0 / rate, len(wl["reqs"])))
    lat, total, evals = drive(server, wl, mixed, arrivals=arrivals)
    st = server.stats()
    in_use, cached = sctx.memory()
    server.close()
    resident = sum(m["plans"][p].info()["bytes_resident"] for m in wl["meshes"] for p in (4, 6))
    for m in wl["meshes"]:
        for p in (4, 6):
            m["plans"][p].close()
        m["mesh"].close()
    sctx.close()
    return {
        "precision": "mixed" if mixed else "fp64",
        "far": "fmm" if kw.get("fmm_terms", 32) else "direct",
        "plan_eps": eps,
        "q": wl["q"],
        "requests": len(wl["reqs"]),
        "mesh_triangles": wl["sizes"],
        "rhs_per_request": "U{1..32}",
        "setup_s": t_build,
        "plans_resident_bytes": resident,
        "hbm_budget_bytes": budget,
        "in_use_bytes_at_end": in_use,
        "cached_bytes_at_end": cached,
        "saturated_evals_per_s": evals_sat,
        "arrival_rate_per_s": rate,
        "evals_per_s": evals,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "batches": st["batches"],
        "columns": st["columns"],
        "budget_waits": st["budget_waits"],
        "rejected": st["rejected"],
        "slots": n_slots,
        "max_batch_rhs": max_batch_rhs,
    }
