"""Ablation of the paper's two structural claims on this pipeline.

The analogue of Tables near_corr and self_stag (Sec. 5.1): for each tolerance
eps, three settings of the same star problem,

  *   Bernstein-ellipse near field (Sec. 4.1), staggered target mesh (Sec. 4.3)
  +   Bernstein-ellipse near field, targets on the quadrature mesh itself
  0   naive ball near field (kappa times the centroid radius), targets on
      the quadrature mesh itself, kappa the smallest value of a grid whose
      error is within 2x of the * setting's (the paper tunes its naive
      setting to the same error in the same way)

reporting per target the near corrections c (near pairs), the near
sub-triangles s_n, per self pair the arc-length panels s_l, the time of the
correction-row precompute and the absolute error E_abs on seeded sample
targets against the library's own FP64 result at eps = 1e-15 (ellipse
model): the tolerance-dependent error, which is what the settings trade.
All evaluation work runs in libvp.
"""

import numpy as np

from . import vp
from . import workloads as W

KAPPAS = (1.0, 1.1, 1.2, 1.3, 1.4, 1.5, 1.6, 1.7, 1.8, 1.9, 2.0, 2.25, 2.5, 3.0, 4.0, 5.0, 6.0)


def problem(n_tri=5000, p=6, seed=20):
    """Star quadrature mesh, its own interpolation nodes, the staggered
    target mesh's nodes and the Gaussian-sum density."""
    vq, tq = W.star_mesh(n_tri=n_tri, n_boundary=max(200, n_tri // 10), seed=seed)
    vt, tt = W.star_mesh(n_tri=n_tri, n_boundary=max(200, n_tri // 10), seed=seed + 1, staggered=True)
    nodes = vp.ref_nodes(p)
    return dict(vq=vq, tq=tq, p=p, same=W.node_positions(vq, tq, nodes).reshape(-1, 2),
                stag=W.node_positions(vt, tt, nodes).reshape(-1, 2),
                F=W.sample_density(W.gaussian_sum(seed + 2, vq, tq), vq, tq, nodes))


def measure(ctx, mesh, prob, q, eps, targets, sample, ref, **model):
    """One plan + evaluation; counts, rows time and E_abs on the sample."""
    plan = ctx.plan(mesh, prob["p"], q, eps, targets, **model)
    info = plan.info()
    u = plan.execute(prob["F"])
    plan.close()
    n_tgt = info["n_tgt"]
    return {"c": (info["n_pairs"] - info["n_self"]) / n_tgt, "s_n": info["near_subtri"] / n_tgt,
            "s_l": info["self_panels"] / max(1, info["n_self"]), "rows_ms": info["ms_rows"],
            "pairs": info["n_pairs"], "E_abs": float(np.abs(u[sample] - ref).max())}


def reference(ctx, mesh, prob, q, targets, eps=1e-15):
    """The library's FP64 potential at eps = 1e-15 (ellipse model)."""
    plan = ctx.plan(mesh, prob["p"], q, eps, targets)
    u = plan.execute(prob["F"])
    plan.close()
    return u


def run(ctx, eps_list=(1e-8, 1e-10, 1e-12, 1e-14), q=8, n_tri=5000, n_sample=64, seed=20, kappas=KAPPAS):
    """One dict per eps in "rows", plus the problem sizes and the sample."""
    prob = problem(n_tri=n_tri, seed=seed)
    rng = np.random.default_rng(seed + 7)
    s_same = np.sort(rng.choice(len(prob["same"]), n_sample, replace=False))
    s_stag = np.sort(rng.choice(len(prob["stag"]), n_sample, replace=False))
    mesh = ctx.mesh(prob["vq"], prob["tq"])
    ref_same = reference(ctx, mesh, prob, q, prob["same"][s_same])
    ref_stag = reference(ctx, mesh, prob, q, prob["stag"][s_stag])
    out = []
    for eps in eps_list:
        star = measure(ctx, mesh, prob, q, eps, prob["stag"], s_stag, ref_stag)
        plus = measure(ctx, mesh, prob, q, eps, prob["same"], s_same, ref_same)
        zero, kappa = None, None
        for k in kappas:
            zero = measure(ctx, mesh, prob, q, eps, prob["same"], s_same, ref_same, near_model="ball",
                           ball_factor=k)
            kappa = k
            if zero["E_abs"] <= 2.0 * star["E_abs"]:
                break
        out.append({"eps": eps, "kappa": kappa, "star": star, "plus": plus, "zero": zero,
                    "c_ratio": star["c"] / zero["c"], "s_n_ratio": star["s_n"] / zero["s_n"],
                    "s_l_ratio": star["s_l"] / plus["s_l"]})
    mesh.close()
    return {"n_tri": len(prob["tq"]), "p": prob["p"], "q": q, "n_targets_same": len(prob["same"]),
            "n_targets_stag": len(prob["stag"]), "n_sample": n_sample, "sample_same": s_same,
            "sample_stag": s_stag, "problem": prob, "rows": out}


def table(res):
    """Markdown table of run()'s result."""
    lines = ["| eps | c0 | c+ | c* | c*/c0 | s_n0 | s_n+ | s_n* | s_n*/s_n0 | s_l+ | s_l* | rows ms 0/+/* | kappa "
             "| E0 | E+ | E* |", "|" + "---|" * 16]
    for r in res["rows"]:
        z, pl, st = r["zero"], r["plus"], r["star"]
        lines.append(f"| {r['eps']:.0e} | {z['c']:.2f} | {pl['c']:.2f} | {st['c']:.2f} | {r['c_ratio']:.1%} | "
                     f"{z['s_n']:.1f} | {pl['s_n']:.1f} | {st['s_n']:.1f} | {r['s_n_ratio']:.1%} | "
                     f"{pl['s_l']:.1f} | {st['s_l']:.1f} | {z['rows_ms']:.1f}/{pl['rows_ms']:.1f}/"
                     f"{st['rows_ms']:.1f} | {r['kappa']} | {z['E_abs']:.1e} | {pl['E_abs']:.1e} | "
                     f"{st['E_abs']:.1e} |")
    return "\n".join(lines)
