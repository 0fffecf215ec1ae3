"""vp_execute_noalloc (the evaluation without device allocation) through the
C ABI: two calls in a row, the second on a smaller input, each equal to
vp_execute's result on the same plan and densities (FP64 bar 1e-11 relative
L-infinity, mixed 1e-6), device memory unchanged by the calls, and a
workspace beyond the fixed device array rejected with VP_EINVAL."""

import numpy as np
import pytest

from paper_2205_04401_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = a.reshape(len(a), -1), b.reshape(len(b), -1)
    return float((np.abs(a - b).max(0) / np.abs(b).max(0)).max())


def test_noalloc_matches_execute_twice_second_smaller():
    import torch
    from paper_2205_04401_amd import vp

    assert torch.cuda.is_available()
    ctx = vp.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    # first call: a 1000-triangle star, p = 6, q = 8, two densities
    p = 6
    vq, tq = W.star_mesh(n_tri=1000, n_boundary=200, seed=80)
    vt, tt = W.star_mesh(n_tri=1000, n_boundary=200, seed=81, staggered=True)
    nodes = vp.ref_nodes(p)
    tg = W.node_positions(vt, tt, nodes).reshape(-1, 2)
    F = np.stack([W.sample_density(W.gaussian_sum(82 + r, vq, tq), vq, tq, nodes) for r in range(2)], -1)
    mesh = ctx.mesh(vq, tq)
    plan = ctx.plan(mesh, p, 8, 1e-13, tg)
    F_d = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    out = torch.zeros((len(tg), 2), dtype=torch.float64, device="cuda")
    # before any vp_execute (the plan has no workspace): the first call also
    # loads the kernels' code on the device; around the second, which repeats
    # it, the free device memory and the context's block cache stay the same
    plan.execute_noalloc(F_d, out)
    torch.cuda.synchronize()
    first = out.clone()
    free0 = torch.cuda.mem_get_info()[0]
    cached0 = ctx.cached_bytes()
    plan.execute_noalloc(F_d, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0, "vp_execute_noalloc changed the free device memory"
    assert ctx.cached_bytes() == cached0
    assert bool((out == first).all())
    u_na = out.cpu().numpy()
    u_ref = plan.execute(F_d).cpu().numpy()
    e1 = rel(u_na, u_ref)
    out_m = torch.zeros((len(tg), 1), dtype=torch.float64, device="cuda")
    plan.execute_noalloc(F_d[:, :, :1].contiguous(), out_m, mixed=True)
    e1m = rel(out_m.cpu().numpy(), u_ref[:, :1])
    # second call: the unit square (128 triangles, 1920 targets), one density
    p2 = 4
    vq2, tq2 = W.unit_square(8, "/")
    vt2, tt2 = W.unit_square(8, "\\")
    nodes2 = vp.ref_nodes(p2)
    tg2 = W.node_positions(vt2, tt2, nodes2).reshape(-1, 2)
    F2 = W.sample_density(W.gaussian_bump, vq2, tq2, nodes2)
    mesh2 = ctx.mesh(vq2, tq2)
    plan2 = ctx.plan(mesh2, p2, 8, 1e-13, tg2)
    F2_d = torch.from_numpy(F2).cuda()
    out2 = torch.zeros((len(tg2), 1), dtype=torch.float64, device="cuda")
    plan2.execute_noalloc(F2_d, out2)
    u2_na = out2.cpu().numpy()
    u2_ref = plan2.execute(F2_d).cpu().numpy().reshape(-1, 1)
    e2 = rel(u2_na, u2_ref)
    print("noalloc vs execute: star", e1, "mixed", e1m, "unit square", e2, flush=True)
    assert e1 <= 1e-11 and e2 <= 1e-11 and e1m <= 1e-6
    # a workspace beyond the device array: rejected, output untouched
    R = 200
    Fbig = torch.zeros((len(tq), plan.n_p, R), dtype=torch.float64, device="cuda")
    outbig = torch.full((len(tg), R), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(vp.VPError) as ei:
        plan.execute_noalloc(Fbig, outbig)
    assert ei.value.status == vp.VP_EINVAL and "exceeds" in str(ei.value)
    assert bool((outbig == 7.0).all())
    # host arrays are refused by the binding; through the ABI a call without
    # VP_DEVICE_PTRS is refused by the library
    lib = vp.load()
    assert lib.vp_execute_noalloc(plan.h, 1, vp._ptr(F_d), vp._ptr(out), vp.VP_FP64, 0) == vp.VP_EINVAL
    plan2.close()
    mesh2.close()
    plan.close()
    mesh.close()
    ctx.close()
