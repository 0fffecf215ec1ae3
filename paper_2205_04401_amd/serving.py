"""Request-serving workload: Poisson arrivals over several resident meshes.

Several seeded star meshes of different sizes stay resident on the device
with their plans (near lists and FP64 correction rows); requests of 1-32
right-hand sides arrive as a Poisson process and go through the library's
continuous-batching server (vp_server_*).  Reports p50/p99 latency (arrival
to observed completion) beside throughput in potential evaluations per
second (targets x right-hand sides).

Only argument marshalling and clocks live here; all evaluation work runs in
libvp.
"""

import math
import time

import numpy as np

from . import vp
from . import workloads as W


def build_workload(ctx, n_meshes=4, tri_range=(1000, 8000), q=6, eps=1e-13, seed=40, n_requests=300,
                   max_rhs=32, device="cuda:0", fmm_terms=0):
    """Meshes (log-uniform triangle counts), plans (p = 4 or 6 per mesh) and
    a request list (mesh, R, density tensor).  Returns a dict."""
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1]), n_meshes))).astype(int)
    orders = rng.choice([4, 6], size=n_meshes)
    meshes = []
    for k, (T, p) in enumerate(zip(sizes, orders)):
        vq, tq = W.star_mesh(n_tri=int(T), n_boundary=max(200, int(T) // 10), seed=seed + 1 + k)
        vt, tt = W.star_mesh(n_tri=int(T), n_boundary=max(200, int(T) // 10), seed=seed + 101 + k, staggered=True)
        nodes = vp.ref_nodes(int(p))
        tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
        mesh = ctx.mesh(vq, tq)
        plan = ctx.plan(mesh, int(p), q, eps, tg, **({"fmm_terms": fmm_terms, "fmm_leaf": 64} if fmm_terms else {}))
        meshes.append(dict(vq=vq, tq=tq, tg=tg, p=int(p), nodes=nodes, mesh=mesh, plan=plan))
    reqs = []
    for i in range(n_requests):
        k = int(rng.integers(n_meshes))
        R = int(rng.integers(1, max_rhs + 1))
        m = meshes[k]
        cols = [W.sample_density(W.gaussian_sum(1000 + 97 * i + r, m["vq"], m["tq"]), m["vq"], m["tq"], m["nodes"])
                for r in range(R)]
        F = torch.from_numpy(np.ascontiguousarray(np.stack(cols, -1))).to(device)
        out = torch.empty((m["plan"].n_tgt, R), dtype=torch.float64, device=device)
        reqs.append(dict(mesh=k, R=R, F=F, out=out, evals=m["plan"].n_tgt * R))
    return dict(meshes=meshes, reqs=reqs)


def saturated(server, wl, mixed):
    """All requests submitted at once; returns (seconds, evals/s)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [server.submit(wl["meshes"][r["mesh"]]["plan"], r["F"], r["out"], mixed=mixed) for r in wl["reqs"]]
    for t in tickets:
        server.wait(t)
    dt = time.perf_counter() - t0
    return dt, sum(r["evals"] for r in wl["reqs"]) / dt


def poisson_run(server, wl, mixed, rate, seed=49):
    """Requests arrive at the given mean rate (per second); returns
    per-request latencies (s) and the achieved evals/s."""
    import torch
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, len(wl["reqs"]))
    arrivals = np.cumsum(gaps)
    done_at = np.zeros(len(wl["reqs"]))
    outstanding = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while i < len(wl["reqs"]) or outstanding:
        now = time.perf_counter() - t0
        while i < len(wl["reqs"]) and arrivals[i] <= now:
            r = wl["reqs"][i]
            outstanding[server.submit(wl["meshes"][r["mesh"]]["plan"], r["F"], r["out"], mixed=mixed)] = i
            i += 1
        for t in list(outstanding):
            if server.poll(t):
                done_at[outstanding.pop(t)] = time.perf_counter() - t0
        if not outstanding and i < len(wl["reqs"]):
            time.sleep(max(0.0, min(1e-3, arrivals[i] - (time.perf_counter() - t0))))
    total = time.perf_counter() - t0
    return done_at - arrivals, sum(r["evals"] for r in wl["reqs"]) / total


def run(ctx, n_requests=300, mixed=False, eps=None, n_slots=4, max_batch_rhs=32, load=0.8, **kw):
    """Saturated throughput, then a Poisson run at `load` times the saturated
    request rate.  Returns a dict of metrics."""
    eps = eps if eps is not None else (1e-8 if mixed else 1e-13)
    wl = build_workload(ctx, n_requests=n_requests, eps=eps, **kw)
    server = ctx.server(n_slots=n_slots, max_batch_rhs=max_batch_rhs)
    saturated(server, wl, mixed)  # warm-up (workspaces, code objects)
    dt_sat, evals_sat = saturated(server, wl, mixed)
    rate = load * len(wl["reqs"]) / dt_sat
    lat, evals = poisson_run(server, wl, mixed, rate)
    st = server.stats()
    server.close()
    for m in wl["meshes"]:
        m["plan"].close()
        m["mesh"].close()
    return {
        "precision": "mixed" if mixed else "fp64",
        "far": "fmm" if kw.get("fmm_terms") else "direct",
        "plan_eps": eps,
        "requests": len(wl["reqs"]),
        "meshes": [int(m["plan"].n_tri) for m in wl["meshes"]],
        "orders_p": [m["p"] for m in wl["meshes"]],
        "saturated_evals_per_s": evals_sat,
        "arrival_rate_per_s": rate,
        "evals_per_s": evals,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "batches": st["batches"],
        "columns": st["columns"],
        "slots": n_slots,
        "max_batch_rhs": max_batch_rhs,
    }
