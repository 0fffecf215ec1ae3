"""Benchmark: potential evaluations per second on one MI355X.

Headline workload: the graded L-shaped domain [-1,1]^2 minus [0,1]^2
(249 721 triangles, mesh size h ~ r^0.5 toward the re-entrant corner), its
staggered target mesh's 3 749 550 order-4 nodes as targets, p = 4, a 4 x 4
collapsed Gauss far rule (3 995 536 far sources), eps = 1e-13, one density,
FP64.  One step is one pass of the whole hot path: plan creation (far
sources, near-field pair lists from the Bernstein-ellipse test, FP64
correction rows) followed by one evaluation (coefficients and far charges,
the far-field sum, the correction apply).  The headline's far sum is the
plan option that sums the far rule's point charges by the fast multipole
method (the paper's own coupling of Sec. 3.6); the tiled direct sum of the
same step is timed beside it.  Mesh, targets and density are resident in
device memory before the timed region; the output stays on the device.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line (the contract) after progress lines.  Beside the
headline it carries: the same step with the direct far sum and in mixed
precision, the error of each against the oracle at sampled targets, the
far-order sweep on the star (Sec. 4.2) and on the 100k-triangle star with
64 densities, the batched and small-case sections, the serving run, and the
oracle's own rate on the host's cores.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "potential evals/s at rel err 1e-11 (FP64) vs 1e-6 (mixed); p50/p99 solve latency"
# MI355X published peaks
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
FLOPS_PER_PAIR = 8  # 2 sub, 1 mul, 1 FMA (r^2), 1 FMA (accumulate), log counted as 1
# vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64
# instruction occupies a 16-lane SIMD for 4 cycles)
PEAK_VALU_LANE_INSTS = 256 * 4 * 16 * 2.4e9
FMM = {"fmm_terms": 32, "fmm_leaf": 64}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# workloads (seeded, synthetic; the generators hold none of the method)
# ---------------------------------------------------------------------------

def l_shape(p=4):
    from paper_2205_04401_amd import workloads as W
    from paper_2205_04401_amd import vp
    vq, tq = W.l_shape_graded(n_tri=250000, seed=50)
    vt, tt = W.l_shape_graded(n_tri=250000, seed=51, staggered=True)
    tg = W.node_positions(vt, tt, vp.ref_nodes(p)).reshape(-1, 2)
    F = W.sample_density(W.l_shape_density(52), vq, tq, vp.ref_nodes(p))
    return vq, tq, tg, F


def star(n_tri, seeds=(20, 21, 22), p=6):
    from paper_2205_04401_amd import workloads as W
    from paper_2205_04401_amd import vp
    vq, tq = W.star_mesh(n_tri=n_tri, n_boundary=2000, seed=seeds[0])
    vt, tt = W.star_mesh(n_tri=n_tri, n_boundary=2000, seed=seeds[1], staggered=True)
    nodes = vp.ref_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = W.sample_density(W.gaussian_sum(seeds[2], vq, tq), vq, tq, nodes)
    return vq, tq, tg, F


# ---------------------------------------------------------------------------
# the oracle on the host's cores (worker processes started before any GPU
# call; they import no GPU code)
# ---------------------------------------------------------------------------

def _oracle_chunk(args):
    """Oracle u at a chunk of targets; returns (u, seconds)."""
    vq, tq, p, q, eps, F, targets = args
    from oracle import potential
    t0 = time.perf_counter()
    u = potential.Oracle(vq, tq, p, q, eps).evaluate(F, targets)
    return u, time.perf_counter() - t0


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def start_pool(n):
    import multiprocessing as mp
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    return mp.get_context("spawn").Pool(n)


def oracle_at(pool, n_workers, vq, tq, p, q, eps, F, targets):
    """The oracle at `targets`, split over the pool; (u, wall seconds)."""
    chunks = np.array_split(np.arange(len(targets)), n_workers)
    t0 = time.perf_counter()
    res = pool.map(_oracle_chunk, [(vq, tq, p, q, eps, F, targets[c]) for c in chunks if len(c)])
    wall = time.perf_counter() - t0
    return np.concatenate([r[0] for r in res]), wall


def rel_err(u, ref):
    return float(np.abs(u - ref).max() / np.abs(ref).max())


# ---------------------------------------------------------------------------
# rooflines
# ---------------------------------------------------------------------------

# Algorithmic FP64 flops of one node evaluation in the correction rows:
# geometry and weight 10, the log counted as 1, 2 per basis function to
# accumulate, and the basis values: up to order 6 the product basis of the
# row kernels (4 for the collapsed coordinates, 2 per step of the Legendre
# recurrence in 2x-1 and 3 per step of the one in the collapsed direction,
# p - 1 steps each, and p + 1 products with the weight), above it 3 per
# basis function for the Koornwinder recurrences (k_rows); with the
# Koornwinder values from a table (k_rows_tab) only the 2 of the
# contraction, on the matrix cores.
def rows_flops_per_node(n_p, p):
    basis = 4 + 5 * (p - 1) + (p + 1) if p <= 6 else 3 * n_p
    return 11 + 2 * n_p + basis


def tab_flops_per_node(n_p):
    return 11 + 2 * n_p


def stage_rooflines(info, tm, steps, q_near=7, n_l=16):
    """Every stage of a step against the resource that bounds it (per launch:
    work over the stage's average device time)."""
    n_p, n_tgt, n_pairs, T = info["n_p"], info["n_tgt"], info["n_pairs"], info["n_tri"]
    n_f, nn = info["n_f"], q_near * q_near
    # radial nodes per ray of a straight self piece (the folded radial rule)
    # other than its apex, which is the target on every ray: evaluated once
    # per pair
    n_r = info["p"]
    n_self, tab_pairs, tab_leaves = info["n_self"], info["tab_pairs"], info["tab_leaves"]
    out = {}

    def alu(name, stage, nodes, fpn, kernel):
        # nodes are one step's; a stage of several launches per step (the
        # table path runs one per pair of depth classes) is taken as a whole
        ms, n = tm.get(stage, (0.0, 0))
        if not n:
            return
        sec = ms / 1e3 / steps
        ach = nodes * fpn / sec / 1e12
        out[name] = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_FP64_VECTOR_TFLOPS, "node_evaluations": nodes, "flops_per_node": fpn,
                     "ms_per_step": sec * 1e3, "launches_per_step": n / steps, "kernel": kernel}
        if n == steps:
            out[name]["avg_launch_ms"] = sec * 1e3

    near_deep = n_pairs - n_self - tab_pairs
    p = info["p"]
    alu("rows_tab", "rows_tab", tab_pairs * n_f + tab_leaves * nn, tab_flops_per_node(n_p), f"k_rows_tab<{p}, *>")
    alu("rows_near", "rows_near", (info["near_subtri"] - tab_leaves) * nn + near_deep * n_f,
        rows_flops_per_node(n_p, p), f"k_rows_deep<{p}>")
    alu("rows_self", "rows_self", info["self_panels"] * n_l * n_r + n_self * (n_f + 1), rows_flops_per_node(n_p, p),
        f"k_rows<{p}, false, 2>")
    if "rows_tab" not in out and "rows_near" not in out:
        nodes = info["near_subtri"] * nn + info["self_panels"] * n_l * n_r + n_pairs * n_f + n_self
        alu("rows", "rows", nodes, rows_flops_per_node(n_p, p), f"k_rows<{p}>")
    # near lists: targets read in the count and fill passes, CSR and pairs written
    ms, n = tm.get("classify", (0.0, 0))
    if n:
        nbytes = 2 * 16 * n_tgt + 8 * (n_tgt + 1) + 9 * n_pairs
        sec = ms / 1e3 / n
        out["near_lists"] = {"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": nbytes / sec / 1e9 / PEAK_HBM_GBS, "bytes": nbytes, "avg_ms": sec * 1e3}
    # correction apply + partial-sum join: far partials, rows, row pointers,
    # pair triangles, coefficients, output
    ms, n = tm.get("finish", (0.0, 0))
    if n:
        nbytes = 8 * (info["far_split"] * n_tgt + n_pairs * n_p + (n_tgt + 1) + T * n_p + n_tgt) + 4 * n_pairs
        sec = ms / 1e3 / n
        out["correction_apply"] = {"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": PEAK_HBM_GBS,
                                   "unit": "GB/s", "frac": nbytes / sec / 1e9 / PEAK_HBM_GBS,
                                   "bytes_per_launch": nbytes, "avg_launch_ms": sec * 1e3,
                                   "kernel": f"k_finish<{p}> / k_finish_flat<{p}, 16>"}
    return out


def far_roofline(n_src, n_tgt, far_ms, launches, kernel, peak):
    sec = far_ms / 1e3 / max(launches, 1)
    pairs = n_src * n_tgt
    ach = FLOPS_PER_PAIR * pairs / sec / 1e12
    return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
            "flops_per_pair": FLOPS_PER_PAIR, "pairs_per_launch": pairs, "avg_launch_ms": sec * 1e3,
            "pairs_per_s": pairs / sec, "kernel": kernel}


def counter_summary(name):
    """Fields of a committed counter summary under profiles/ (rocprofv3 --pmc
    runs), or {} when absent."""
    path = os.path.join(ROOT, "profiles", name)
    fields = {}
    if os.path.exists(path):
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    return fields


def source_digest(parts):
    """First 16 hex digits of the SHA-256 of the named source regions:
    [(file under csrc, first marker, last marker)]: each region runs from the
    first marker to the end of the function that follows the last."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2205_04401_amd", "csrc")
    text = ""
    for fname, a, b in parts:
        src = open(os.path.join(csrc, fname)).read()
        i = src.index(a)
        j = src.index("\n}\n", src.index(b, i)) + 3
        text += src[i:j]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


LOG_DIGEST_PART = ("vp_internal.h", "constexpr double kR2Bias", "void vp_log_wide_parts(")
FAR64_DIGEST_PARTS = [("vp_exec.hip", "template <int S, int RB>\nstruct FarShape {", "void k_far("), LOG_DIGEST_PART]
FAR32_DIGEST_PARTS = [("vp_exec.hip", "template <int RB, int TPT>\n__global__ __launch_bounds__(kBlock) void k_far32(",
                       "void k_far32("), LOG_DIGEST_PART]
# the row kernels and the pair classification that decides which of them takes a pair
ROWS_DIGEST_PARTS = [("vp_rows.hip", "__device__ __forceinline__ int dyadic_count", "hipError_t rows_by_class(")]


def traffic_from(summary, digest, kernel_key):
    f = counter_summary(summary)
    if f.get("kernel_source_sha256_16") != digest:
        return None
    v = f.get(f"{kernel_key}_traffic_bytes_per_step")
    return float(v) if v else None


# ---------------------------------------------------------------------------
# sections
# ---------------------------------------------------------------------------

def timed_steps(ctx, step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    marks = []
    for _ in range(steps):
        info = step()
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    gaps = np.diff(np.concatenate([[t0], marks])) * 1e3
    say(f"  {steps} steps: host return times per step (ms) min {gaps.min():.1f} median {np.median(gaps):.1f} "
        f"max {gaps.max():.1f}")
    tm = ctx.timings()
    ctx.profile(False)
    return dt, info, tm


def sweep_star(ctx, qs, steps=1):
    """Far order q on the star (Sec. 4.2 trade-off): per q the plan + one
    evaluation with the direct far sum and with the FMM far sum."""
    import torch
    p, eps = 6, 1e-13
    vq, tq, tg, F = star(20000)
    mesh = ctx.mesh(vq, tq)
    tg_d = torch.from_numpy(tg).cuda()
    F_d = torch.from_numpy(F).cuda()
    out = torch.empty((len(tg), 1), dtype=torch.float64, device="cuda")
    lines = []
    for q in qs:
        for far, opts in (("direct", {}), ("fmm", FMM)):
            def step():
                plan = ctx.plan(mesh, p, q, eps, tg_d, **opts)
                plan.execute(F_d, out=out)
                info = plan.info()
                plan.close()
                return info
            dt, info, tm = timed_steps(ctx, step, steps, 1)
            line = {"q": q, "far": far, "ms_per_step": dt * 1e3, "evals_per_s": len(tg) / dt,
                    "far_ms": tm["far"][0] / steps, "classify_ms": tm["classify"][0] / steps,
                    "rows_ms": tm["rows"][0] / steps, "finish_ms": tm["finish"][0] / steps,
                    "n_pairs": info["n_pairs"], "pairs_per_target": info["n_pairs"] / len(tg),
                    "n_src": info["n_src"]}
            lines.append(line)
            say(json.dumps({"sweep_star20k": line}))
    mesh.close()
    return {"workload": f"star r=1+0.3cos(5t): {len(tq)} triangles (seed 20), {len(tg)} targets (seed 21), "
                        f"p={p}, eps={eps}, 1 density; step = plan + evaluation", "lines": lines}


def sweep_batched(ctx, qs, R=64):
    """The 100k-triangle star with 64 densities (seeds 1000..), far sum by
    the FMM in passes of 16 densities, far order q swept: per q the plan and
    one evaluation of all 64 densities, FP64 (plan eps 1e-13, 32 terms) and
    mixed (plan eps 1e-8, 16 terms, FP32 leaf passes)."""
    import torch
    from paper_2205_04401_amd import workloads as W
    from paper_2205_04401_amd import vp
    p, eps = 6, 1e-13
    vq, tq = W.star_mesh(n_tri=100000, n_boundary=2000, seed=30)
    vt, tt = W.star_mesh(n_tri=100000, n_boundary=2000, seed=31, staggered=True)
    nodes = vp.ref_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    FR = np.ascontiguousarray(np.stack(
        [W.sample_density(W.gaussian_sum(1000 + r, vq, tq), vq, tq, nodes) for r in range(R)], -1))
    mesh = ctx.mesh(vq, tq)
    tg_d = torch.from_numpy(tg).cuda()
    FR_d = torch.from_numpy(FR).cuda()
    u = torch.empty((len(tg), R), dtype=torch.float64, device="cuda")
    lines = []
    for q in qs:
        for mixed, eps_plan, terms in ((False, eps, 32), (True, 1e-8, 16)):
            torch.cuda.synchronize()
            ctx.profile(True)
            t0 = time.perf_counter()
            plan = ctx.plan(mesh, p, q, eps_plan, tg_d, fmm_terms=terms, fmm_leaf=FMM["fmm_leaf"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan.execute(FR_d, out=u, mixed=mixed)  # builds the 16-density tables on first use
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            plan.execute(FR_d, out=u, mixed=mixed)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            tm = ctx.timings()
            ctx.profile(False)
            info = plan.info()
            plan.close()
            line = {"q": q, "precision": "mixed" if mixed else "fp64", "plan_eps": eps_plan, "fmm_terms": terms,
                    "plan_ms": (t1 - t0) * 1e3, "execute_ms": (t3 - t2) * 1e3,
                    "evals_per_s_execute": len(tg) * R / (t3 - t2),
                    "evals_per_s_with_plan": len(tg) * R / (t3 - t2 + t1 - t0),
                    "rows_ms": tm["rows"][0], "classify_ms": tm["classify"][0], "n_pairs": info["n_pairs"],
                    "pairs_per_target": info["n_pairs"] / len(tg), "n_src": info["n_src"]}
            lines.append(line)
            say(json.dumps({"sweep_star100k_64": line}))
    mesh.close()
    return {"workload": f"star {len(tq)} triangles (seed 30), {len(tg)} targets (seed 31), p={p}, "
                        f"{R} densities (seeds 1000..{1000 + R - 1}), far sum by the FMM; FP64 (eps {eps}) and "
                        f"mixed (eps 1e-8)", "lines": lines}


def far_order_policy(ctx):
    """The far-order policy (vp_choose_q, Sec. 4.2 trade-off) on the 20k
    star, p = 6, eps = 1e-13, one density, with the direct and with the FMM
    far sum: the order it picks for a plan used once, the times it measured
    per order, and from those times the order for a plan serving 100
    evaluations."""
    import torch
    vq, tq, tg, _ = star(20000)
    mesh = ctx.mesh(vq, tq)
    tg_d = torch.from_numpy(tg).cuda()
    out = {"workload": f"star {len(tq)} triangles (seed 20), {len(tg)} targets (seed 21), p=6, eps=1e-13, "
                       f"1 density; cost = plan + n_solves x evaluation", "lines": []}
    for far, opts, qmax in (("direct", {}, 12), ("fmm", FMM, 16)):
        t0 = time.perf_counter()
        q, times = ctx.choose_q(mesh, 6, 1e-13, tg_d, q_min=4, q_max=qmax, n_solves=1, **opts)
        ok = {k: v for k, v in times.items() if math.isfinite(v[0])}
        q100 = min(ok, key=lambda k: ok[k][0] + 100 * ok[k][1])
        line = {"far": far, "q_one_solve": q, "q_100_solves": q100, "policy_s": time.perf_counter() - t0,
                "plan_ms": {k: v[0] for k, v in times.items()}, "execute_ms": {k: v[1] for k, v in times.items()}}
        out["lines"].append(line)
        say(json.dumps({"far_order_policy": {k: line[k] for k in ("far", "q_one_solve", "q_100_solves", "policy_s")}}))
    mesh.close()
    return out


def batched(ctx, R=64, steps=2):
    """64 densities per evaluation on the 20k star at q = 8, plan built once,
    direct far sum on the matrix cores (FP64 MFMA; mixed: FP32 MFMA): the
    MFMA rooflines of the far sum and of the correction apply."""
    import torch
    from paper_2205_04401_amd import vp
    from paper_2205_04401_amd import workloads as W
    p, q = 6, 8
    vq, tq, tg, _ = star(20000)
    nodes = vp.ref_nodes(p)
    FR = np.ascontiguousarray(np.stack(
        [W.sample_density(W.gaussian_sum(1000 + r, vq, tq), vq, tq, nodes) for r in range(R)], -1))
    FR_d = torch.from_numpy(FR).cuda()
    mesh = ctx.mesh(vq, tq)
    tg_d = torch.from_numpy(tg).cuda()
    out = []
    for mixed, eps_plan in ((False, 1e-13), (True, 1e-8)):
        plan = ctx.plan(mesh, p, q, eps_plan, tg_d)
        info = plan.info()
        u = torch.empty((info["n_tgt"], R), dtype=torch.float64, device="cuda:0")
        plan.execute(FR_d, out=u, mixed=mixed)
        def step():
            plan.execute(FR_d, out=u, mixed=mixed)
        dt, _, tm = timed_steps(ctx, step, steps, 0)
        info = plan.info()
        plan.close()
        far_s = tm["far"][0] / 1e3 / steps
        pair_rhs = info["n_src"] * info["n_tgt"] * R
        peak = PEAK_FP32_MFMA_TFLOPS if mixed else PEAK_FP64_MFMA_TFLOPS
        achieved = 2.0 * pair_rhs / far_s / 1e12
        line = {"precision": "mixed" if mixed else "fp64", "plan_eps": eps_plan, "n_rhs": R,
                "evals_per_s": info["n_tgt"] * R / dt, "ms_per_execute": dt * 1e3,
                "far_pair_rhs_per_s": pair_rhs / far_s,
                "far_roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                                 "frac": achieved / peak, "flops_per_pair_rhs": 2,
                                 "kernel": "k_far_mfma32<4, 4>" if mixed else "k_far_mfma64<4, 4>"},
                "corr_roofline": corr_mfma_roofline(info, tm, steps, R),
                "breakdown_ms": {k: v[0] / steps for k, v in tm.items() if v[1]}}
        out.append(line)
        say(json.dumps({"batched": line}))
    mesh.close()
    return out


def corr_mfma_roofline(info, tm, steps, R):
    """Correction apply + partial-sum join on the FP64 matrix cores (blocks
    of 16+ densities): useful flops 2 n_pairs n_p R against the FP64 MFMA
    peak; `issued_frac` counts the padded 16-target x 4k blocks the MFMA
    steps actually run, `row_fill` the share of those rows that are pairs."""
    sec = tm["finish"][0] / 1e3 / steps
    n_p, ent = info["n_p"], max(1, info["cluster_entries"])
    useful = 2.0 * info["n_pairs"] * n_p * R
    issued = 2.0 * ent * 16 * 4 * ((n_p + 3) // 4) * R
    ach = useful / sec / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP64_MFMA_TFLOPS, "issued_frac": issued / sec / 1e12 / PEAK_FP64_MFMA_TFLOPS,
            "row_fill": info["n_pairs"] / (16 * ent), "avg_ms": sec * 1e3, "kernel": f"k_corr_mfma<{info['p']}, 4>"}


def small_case(ctx, n=300):
    """The unit-square case (8x8 cells, 128 triangles, p = 4, q = 8, 1920
    targets, one density): time per evaluation issued back to back, eager
    (vp_execute, asynchronous) and as a captured HIP graph replay
    (vp_graph_*), with the size rule's far-sum shape and after the tuner
    (vp_plan_autotune)."""
    import torch
    from paper_2205_04401_amd import vp
    from paper_2205_04401_amd import workloads as W
    p, q = 4, 8
    vq, tq = W.unit_square(8, "/")
    vt, tt = W.unit_square(8, "\\")
    nodes = vp.ref_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = torch.from_numpy(W.sample_density(W.gaussian_bump, vq, tq, nodes)[:, :, None].copy()).cuda()
    mesh = ctx.mesh(vq, tq)
    plan = ctx.plan(mesh, p, q, 1e-13, tg)
    U = torch.empty((len(tg), 1), dtype=torch.float64, device="cuda")

    def per_eval_us(fn):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n * 1e6

    out = {"workload": "unit square 8x8 cells (128 triangles), p=4, q=8, 1920 targets, 1 density, FP64"}
    for label in ("size_rule", "tuned"):
        if label == "tuned":
            cfg, ms = plan.autotune(n_rhs=1, reps=5)
            out["tuned_config"] = cfg
        g = vp.Graph(plan, F, U)
        out[label] = {"far_config": plan.far_config(1),
                      "eager_us": per_eval_us(lambda: plan.execute(F, out=U, asynchronous=True)),
                      "graph_us": per_eval_us(g.launch)}
        g.close()
    plan.close()
    mesh.close()
    say(json.dumps({"small_case": out}))
    return out


def far_probe(mixed):
    """The direct line's step (graded L-shape, FP64 direct far sum) or the
    mixed line's (plan at eps = 1e-8, FP32 direct far sum), once."""
    import torch
    from paper_2205_04401_amd import vp
    p, q = 4, 4
    vq, tq, tg, F = l_shape(p)
    ctx = vp.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    mesh = ctx.mesh(vq, tq)
    plan = ctx.plan(mesh, p, q, 1e-8 if mixed else 1e-13, torch.from_numpy(tg).cuda())
    u = plan.execute(torch.from_numpy(F).cuda(), mixed=mixed)
    torch.cuda.synchronize()
    print(json.dumps({"far_probe": {"mixed": mixed, "n_src": plan.n_src, "n_tgt": plan.n_tgt, "u0": float(u[0])}}),
          flush=True)
    plan.close()
    mesh.close()
    ctx.close()


def batched_probe():
    """The 100k-star section with 64 densities at q = 8 alone (FP64 and
    mixed: plan and two evaluations each), for kernel traces."""
    import torch
    from paper_2205_04401_amd import vp
    ctx = vp.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    res = sweep_batched(ctx, [8])
    print(json.dumps({"batched_probe": res}), flush=True)
    ctx.close()


def copy_probe(n_bytes=1 << 29, reps=3):
    """A plain device-to-device copy of known size (the calibration kernel
    for the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    a = torch.empty(n_bytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n_bytes, "reps": reps}), flush=True)


# ---------------------------------------------------------------------------
# the run
# ---------------------------------------------------------------------------

def run(args, pool, n_workers):
    import torch
    from paper_2205_04401_amd import vp

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    p, q, eps = 4, 4, 1e-13
    say("C5 workload: generating the graded L-shape meshes")
    vq, tq, tg, F = l_shape(p)
    n_tgt = len(tg)
    ctx = vp.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    mesh = ctx.mesh(vq, tq)
    tg_d = torch.from_numpy(tg).to(dev)
    F_d = torch.from_numpy(F).to(dev)
    out = torch.empty((n_tgt, 1), dtype=torch.float64, device=dev)
    rng = np.random.default_rng(7)
    sample = np.unique(np.concatenate([rng.choice(n_tgt, args.cpu_sample - 8, replace=False),
                                       np.argsort(np.hypot(tg[:, 0], tg[:, 1]))[:8]]))  # 8 next to the corner
    sample_d = torch.from_numpy(sample).to(dev)

    def step_of(eps_plan=eps, mixed=False, **opts):
        def step():
            plan = ctx.plan(mesh, p, q, eps_plan, tg_d, **opts)
            plan.execute(F_d, out=out, mixed=mixed)
            info = plan.info()
            plan.close()
            return info
        return step

    # --- headline: FP64, far sum by the FMM ---------------------------------
    say(f"headline: {args.warmup} warm-up + {args.steps} timed steps")
    dt, info, tm = timed_steps(ctx, step_of(**FMM), args.steps, args.warmup)
    u_fmm = out[sample_d, 0].cpu().numpy()
    stages = stage_rooflines(info, tm, args.steps)
    timed = {k: v for k, v in stages.items() if "ms_per_step" in v}
    dom_name = max(timed, key=lambda k: timed[k]["ms_per_step"])
    dom = dict(timed[dom_name])
    digest = source_digest(ROWS_DIGEST_PARTS)
    dom["traffic"] = traffic_from("k_rows_lshape250k_q4_counters.md", digest, dom_name)
    rc = counter_summary("k_rows_lshape250k_q4_counters.md")
    vi = rc.get(f"{dom_name}_valu_instructions_per_step")
    if vi and rc.get("kernel_source_sha256_16") == digest:
        # wave64 vector instructions of the stage against one per 4 cycles on each SIMD
        dom["valu_issue"] = {"instructions_per_step": float(vi),
                             "frac": float(vi) * 64 / (dom["ms_per_step"] / 1e3) / PEAK_VALU_LANE_INSTS}
    dom["stage"] = dom_name
    result = {
        "metric": METRIC,
        "value": n_tgt / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"graded L-shape [-1,1]^2 minus [0,1]^2, h ~ r^0.5: {len(tq)} triangles (seed 50), "
                        f"staggered target mesh (seed 51) -> {n_tgt} targets; p={p} ({info['n_p']} nodes/triangle), "
                        f"q={q} collapsed Gauss ({q * q} nodes/triangle -> {info['n_src']} sources), eps={eps}, "
                        f"1 density (r^(2/3) sin(2t/3) e^(-r^2) + 10-Gaussian sum, seed 52); "
                        f"step = plan (near lists + FP64 rows + FMM tree) + evaluation; far sum by the FMM "
                        f"({FMM['fmm_terms']} terms)",
            "p": p, "q": q, "eps": eps, "n_rhs": 1, "precision": "fp64", "far": "fmm",
        },
        "roofline": dom,
        "breakdown_ms": {k: v[0] / args.steps for k, v in tm.items() if v[1]},
        "plan_ms": (tm["classify"][0] + tm["rows"][0]) / args.steps,
        "execute_ms": (tm["coef"][0] + tm["far"][0] + tm["finish"][0]) / args.steps,
        "pairs_per_target": info["n_pairs"] / n_tgt,
        "n_pairs": info["n_pairs"], "n_self": info["n_self"], "tab_pairs": info["tab_pairs"],
        "near_subtri_per_near_pair": info["near_subtri"] / max(1, info["n_pairs"] - info["n_self"]),
        "self_panels_per_self_pair": info["self_panels"] / max(1, info["n_self"]),
        "bytes_resident": info["bytes_resident"],
        "stage_rooflines": stages,
        "rows_pairs_per_s": info["n_pairs"] / (tm["rows"][0] / 1e3 / args.steps),
    }
    say(json.dumps({"headline": {k: result[k] for k in ("value", "ms_per_step", "breakdown_ms")}}))

    if args.headline_only:
        print(json.dumps(result), flush=True)
        return
    # --- the same step with the direct far sum (FP64) -------------------------
    dt_d, info_d, tm_d = timed_steps(ctx, step_of(), args.direct_steps, 1)
    u_dir = out[sample_d, 0].cpu().numpy()
    far_d = far_roofline(info_d["n_src"], n_tgt, tm_d["far"][0], tm_d["far"][1], "k_far<1, WIDE> (FP64)",
                         PEAK_FP64_VECTOR_TFLOPS)
    f64c = counter_summary("k_far_fp64_lshape250k_q4_counters.md")
    ipp = f64c.get("valu_instructions_per_pair")
    if ipp and f64c.get("kernel_source_sha256_16") == source_digest(FAR64_DIGEST_PARTS):
        far_d["valu_issue"] = {"instructions_per_pair": float(ipp),
                               "frac": float(ipp) * far_d["pairs_per_s"] / PEAK_VALU_LANE_INSTS}
    result["direct"] = {"value": n_tgt / dt_d, "unit": "evals/s", "ms_per_step": dt_d * 1e3, "steps": args.direct_steps,
                        "far_roofline": far_d,
                        "breakdown_ms": {k: v[0] / args.direct_steps for k, v in tm_d.items() if v[1]}}
    say(json.dumps({"direct": result["direct"]}))

    # --- mixed precision: FP32 direct far sum, FP64 rows at eps = 1e-8 --------
    dt_m, info_m, tm_m = timed_steps(ctx, step_of(1e-8, True), args.mixed_steps, 1)
    u_mix = out[sample_d, 0].cpu().numpy()
    far_m = far_roofline(info_m["n_src"], n_tgt, tm_m["far"][0], tm_m["far"][1], "k_far32 (FP32)", 157.3)
    f32c = counter_summary("k_far32_lshape250k_q4_counters.md")
    ipp32 = f32c.get("valu_instructions_per_pair")
    if ipp32 and f32c.get("kernel_source_sha256_16") == source_digest(FAR32_DIGEST_PARTS):
        # vector instructions retired against one wave64 instruction per 4
        # cycles and SIMD (FP32 without packed instructions)
        far_m["valu_issue"] = {"instructions_per_pair": float(ipp32),
                               "frac": float(ipp32) * far_m["pairs_per_s"] / PEAK_VALU_LANE_INSTS}
    result["mixed"] = {"value": n_tgt / dt_m, "unit": "evals/s", "ms_per_step": dt_m * 1e3, "steps": args.mixed_steps,
                       "plan_eps": 1e-8, "pairs_per_target": info_m["n_pairs"] / n_tgt, "far_roofline": far_m,
                       "breakdown_ms": {k: v[0] / args.mixed_steps for k, v in tm_m.items() if v[1]}}
    say(json.dumps({"mixed": result["mixed"]}))
    mesh.close()

    # --- secondary sections ---------------------------------------------------
    if not args.no_sweep:
        result["sweep"] = {"star20k": sweep_star(ctx, (4, 5, 6, 8, 10, 12, 16)),
                           "star100k_64rhs": sweep_batched(ctx, (8, 10, 12, 14, 16, 18, 20))}
        result["far_order_policy"] = far_order_policy(ctx)
    if not args.no_batched:
        result["batched"] = batched(ctx)
    if not args.no_small:
        result["small_case"] = small_case(ctx)
    if not args.no_serving:
        from paper_2205_04401_amd import serving
        result["serving"] = serving.run(ctx, n_requests=args.serving_requests, budget_gb=args.serving_budget_gb,
                                        q=args.serving_q)
        for s in result["serving"]:
            say(json.dumps({"serving": s}))
    ctx.close()
    result["gpu_sections_s"] = time.perf_counter() - t_start

    # --- the oracle on the host, and the error of every line against it ------
    if pool is not None:
        say(f"oracle on {len(sample)} sampled targets ({n_workers} processes)")
        ref, wall = oracle_at(pool, n_workers, vq, tq, p, q, eps, F, tg[sample])
        model, ncpu = cpu_info()
        one = min(len(sample), args.cpu_single)
        ref1, wall1 = oracle_at(pool, 1, vq, tq, p, q, eps, F, tg[sample[:one]])
        result["cpu_baseline"] = {
            "value": len(sample) / wall, "unit": "evals/s", "cores": n_workers, "kind": "oracle",
            "sample": f"{len(sample)} seeded targets of the same workload (8 next to the re-entrant corner; all "
                      f"{info['n_src']} far sources and the targets' self/near corrections), {wall:.1f} s on "
                      f"{n_workers} worker processes of one thread each",
            "single_core": {"value": one / wall1, "unit": "evals/s", "targets": one, "seconds": wall1},
            "cpu_model": model, "nproc": ncpu,
        }
        result["accuracy"] = {
            "reference": f"oracle (FP64, eps = {eps}) at the {len(sample)} cpu_baseline targets; relative L-inf",
            "fp64_fmm": rel_err(u_fmm, ref), "fp64_direct": rel_err(u_dir, ref), "mixed": rel_err(u_mix, ref),
            "bars": {"fp64": 1e-11, "mixed": 1e-6}}
        say(json.dumps({"cpu_baseline": result["cpu_baseline"], "accuracy": result["accuracy"]}))
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--direct-steps", type=int, default=2, help="timed steps of the direct-far-sum line")
    ap.add_argument("--mixed-steps", type=int, default=2, help="timed steps of the mixed-precision line")
    ap.add_argument("--cpu-sample", type=int, default=256, help="targets of the oracle timing and error checks")
    ap.add_argument("--cpu-single", type=int, default=24, help="of them, timed on one core")
    ap.add_argument("--cpu-workers", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="only the headline step (no other sections)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the unit-square latency section")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-budget-gb", type=float, default=128.0)
    ap.add_argument("--serving-q", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true", help="only run a 512 MiB device copy (counter calibration)")
    ap.add_argument("--mixed-probe", action="store_true",
                    help="only the mixed line's step, once (counter runs of the FP32 far sum)")
    ap.add_argument("--direct-probe", action="store_true",
                    help="only the direct line's step, once (counter runs of the FP64 far sum)")
    ap.add_argument("--batched-probe", action="store_true",
                    help="only the 100k star with 64 densities at q = 8 (kernel traces of the batched FMM path)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the far sum, near lists and corrections run on a single MI355X; "
              "sharding over several GPUs is a design note only (targets would split across GPUs with one "
              "all-gather of the far charges).", file=sys.stderr)
        raise SystemExit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.mixed_probe or args.direct_probe:
        far_probe(mixed=args.mixed_probe)
        return
    if args.batched_probe:
        batched_probe()
        return
    # the oracle's worker processes start before anything touches the GPU
    pool, n_workers = None, 0
    if not args.no_cpu_baseline:
        n_workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
        pool = start_pool(n_workers)
    try:
        run(args, pool, n_workers)
    finally:
        if pool is not None:
            pool.close()
            pool.join()


if __name__ == "__main__":
    main()
