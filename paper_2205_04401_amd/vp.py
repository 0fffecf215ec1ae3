"""ctypes binding of libvp (include/vp.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy
arrays / torch tensors to pointers and raises on a non-zero status.  Loading
fails loudly (``VPError``) when ``libvp.so`` is missing: there is no fallback.

    ctx = Context()                       # device 0, default stream
    mesh = ctx.mesh(vert, tri)            # [n_vert, 2] float64, [n_tri, 3] int32
    plan = ctx.plan(mesh, p=6, q=8, eps=1e-13, targets=tgt)
    u = plan.execute(F)                   # F [n_tri, n_p] or [n_tri, n_p, R]
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvp.so")

VP_OK, VP_EINVAL, VP_ENOMEM, VP_EDEVICE, VP_ENOTSUP, VP_EBUSY, VP_EINTERNAL = range(7)
VP_FP64, VP_MIXED = 0, 1
VP_DEVICE_PTRS, VP_FAR_ONLY, VP_ASYNC = 1, 2, 4
NEAR_MODELS = {"ellipse": 0, "ball": 1}  # VP_NEAR_ELLIPSES, VP_NEAR_BALL
STATUS_NAMES = {0: "VP_OK", 1: "VP_EINVAL", 2: "VP_ENOMEM", 3: "VP_EDEVICE", 4: "VP_ENOTSUP",
                5: "VP_EBUSY", 6: "VP_EINTERNAL"}

# every symbol include/vp.h declares
EXPORTS = ["vp_ctx_create", "vp_ctx_destroy", "vp_last_error", "vp_ref_nodes", "vp_ref_rule", "vp_mesh_create",
           "vp_mesh_destroy", "vp_mesh_set_curved_sides", "vp_mesh_map_points", "vp_plan_create", "vp_plan_info", "vp_plan_pairs", "vp_plan_rows",
           "vp_plan_rows_range",
           "vp_execute", "vp_execute_noalloc", "vp_coefficients", "vp_plan_sources", "vp_plan_destroy", "vp_sync",
           "vp_ctx_profile", "vp_ctx_timings", "vp_server_create", "vp_server_destroy", "vp_submit",
           "vp_poll", "vp_wait", "vp_server_stats", "vp_interp_create", "vp_interp_destroy", "vp_interp_locate",
           "vp_interp_eval", "vp_graph_create", "vp_graph_launch", "vp_graph_destroy", "vp_plan_far_config",
           "vp_plan_set_far_config", "vp_plan_autotune", "vp_choose_q", "vp_ctx_cached_bytes", "vp_ctx_trim", "vp_ctx_memory",
           "vp_server_admission"]
FAR_SHAPES = {"wide": 0, "narrow1": 1, "narrow2": 2}
STAGES = ["classify", "rows", "coef", "far", "finish", "rows_tab", "rows_near", "rows_self"]


class VPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class PlanOpts(ctypes.Structure):
    _fields_ = [("c_n", ctypes.c_double), ("q_near", ctypes.c_int), ("n_l", ctypes.c_int),
                ("tau", ctypes.c_double), ("depth_cap", ctypes.c_int), ("dyadic_cap", ctypes.c_int),
                ("flags", ctypes.c_uint32), ("near_model", ctypes.c_int), ("ball_factor", ctypes.c_double),
                ("fmm_terms", ctypes.c_int), ("fmm_leaf", ctypes.c_int)]


class FarConfig(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("mfma_tiles", ctypes.c_int32), ("n_split", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class PlanStats(ctypes.Structure):
    _fields_ = [("n_tri", ctypes.c_int64), ("n_src", ctypes.c_int64), ("n_tgt", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_self", ctypes.c_int64), ("near_subtri", ctypes.c_int64),
                ("self_panels", ctypes.c_int64), ("capped_leaves", ctypes.c_int64),
                ("depth_first_pairs", ctypes.c_int64),
                ("bytes_resident", ctypes.c_int64), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("n_p", ctypes.c_int32), ("n_f", ctypes.c_int32), ("eps", ctypes.c_double),
                ("ms_classify", ctypes.c_double), ("ms_rows", ctypes.c_double), ("far_split", ctypes.c_int64),
                ("cluster_entries", ctypes.c_int64), ("fmm_terms", ctypes.c_int32), ("fmm_levels", ctypes.c_int32),
                ("fmm_near_pairs", ctypes.c_int64), ("fmm_m2l_pairs", ctypes.c_int64),
                ("tab_pairs", ctypes.c_int64), ("tab_leaves", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
P = ctypes.c_void_p
I64 = ctypes.c_int64
DP = ctypes.POINTER(ctypes.c_double)


def load(path=LIB_PATH):
    """Load libvp.so (once).  Raises VPError if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise VPError(VP_EDEVICE, f"{path} not found: build it with `python -m paper_2205_04401_amd.build`")
    lib = ctypes.CDLL(path)
    sig = {
        "vp_ctx_create": [ctypes.c_int, P, ctypes.c_uint64, ctypes.POINTER(P)],
        "vp_ctx_destroy": [P],
        "vp_ref_nodes": [ctypes.c_int, P, ctypes.POINTER(ctypes.c_int)],
        "vp_ref_rule": [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.POINTER(ctypes.c_int)],
        "vp_mesh_create": [P, I64, P, I64, P, ctypes.POINTER(P)],
        "vp_mesh_destroy": [P],
        "vp_mesh_set_curved_sides": [P, I64, P, P, ctypes.c_int, P],
        "vp_mesh_map_points": [P, ctypes.c_int, P, P],
        "vp_plan_create": [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double, I64, P, P, ctypes.POINTER(P)],
        "vp_plan_info": [P, ctypes.POINTER(PlanStats)],
        "vp_plan_pairs": [P, P, P, P],
        "vp_plan_rows": [P, P],
        "vp_plan_rows_range": [P, I64, I64, P],
        "vp_execute": [P, I64, P, P, ctypes.c_int, ctypes.c_uint32],
        "vp_execute_noalloc": [P, I64, P, P, ctypes.c_int, ctypes.c_uint32],
        "vp_coefficients": [P, I64, P, P, P, ctypes.c_uint32],
        "vp_plan_sources": [P, P],
        "vp_plan_destroy": [P],
        "vp_sync": [P],
        "vp_ctx_profile": [P, ctypes.c_int],
        "vp_ctx_cached_bytes": [P, ctypes.POINTER(ctypes.c_uint64)],
        "vp_ctx_trim": [P],
        "vp_ctx_timings": [P, P, P],
        "vp_server_create": [P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(P)],
        "vp_server_destroy": [P],
        "vp_submit": [P, P, I64, P, P, ctypes.c_int, ctypes.POINTER(I64)],
        "vp_poll": [P, I64, ctypes.POINTER(ctypes.c_int)],
        "vp_wait": [P, I64],
        "vp_server_stats": [P, P, P, P],
        "vp_server_admission": [P, P, P],
        "vp_ctx_memory": [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
        "vp_graph_create": [P, I64, P, P, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(P)],
        "vp_graph_launch": [P],
        "vp_graph_destroy": [P],
        "vp_plan_far_config": [P, I64, ctypes.c_int, ctypes.POINTER(FarConfig)],
        "vp_plan_set_far_config": [P, I64, ctypes.c_int, ctypes.POINTER(FarConfig)],
        "vp_plan_autotune": [P, I64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(FarConfig),
                             ctypes.POINTER(ctypes.c_double)],
        "vp_choose_q": [P, P, ctypes.c_int, ctypes.c_double, I64, P, P, ctypes.c_int, ctypes.c_int, I64,
                        ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int), P, P],
        "vp_interp_create": [P, P, ctypes.c_int, ctypes.POINTER(P)],
        "vp_interp_destroy": [P],
        "vp_interp_locate": [P, I64, P, P, P],
        "vp_interp_eval": [P, I64, P, I64, P, P, P, ctypes.c_uint32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.vp_last_error.argtypes = []
    lib.vp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status):
    if status != VP_OK:
        raise VPError(status, _lib.vp_last_error().decode())


def _ptr(a):
    """Pointer of a contiguous numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(P)
    return P(a.data_ptr())


def _is_device(a):
    return a is not None and not isinstance(a, np.ndarray) and getattr(a, "is_cuda", False)


def ref_nodes(p):
    """Reference interpolation nodes [n_p, 2] of order p."""
    lib = load()
    n = ctypes.c_int()
    _check(lib.vp_ref_nodes(p, None, ctypes.byref(n)))
    out = np.empty((n.value, 2))
    _check(lib.vp_ref_nodes(p, _ptr(out), ctypes.byref(n)))
    return out


def ref_rule(which, n):
    """Reference rule `which` (see vp_ref_rule) as (x, y, w) arrays."""
    lib = load()
    cnt = ctypes.c_int()
    _check(lib.vp_ref_rule(which, n, None, None, None, ctypes.byref(cnt)))
    x, y, w = np.zeros(cnt.value), np.zeros(cnt.value), np.zeros(cnt.value)
    _check(lib.vp_ref_rule(which, n, _ptr(x), _ptr(y), _ptr(w), ctypes.byref(cnt)))
    return x, y, w


class Context:
    def __init__(self, device=0, stream=None, hbm_budget_bytes=0):
        lib = load()
        h = P()
        sp = None if stream is None else P(int(stream))
        _check(lib.vp_ctx_create(device, sp, hbm_budget_bytes, ctypes.byref(h)))
        self.h = h
        self.device = device

    def mesh(self, vert, tri, curved=None):
        return Mesh(self, vert, tri, curved)

    def plan(self, mesh, p, q, eps, targets, **opts):
        return Plan(self, mesh, p, q, eps, targets, **opts)

    def choose_q(self, mesh, p, eps, targets, **kw):
        """The far-order policy (vp_choose_q); see choose_q()."""
        return choose_q(self, mesh, p, eps, targets, **kw)

    def interp(self, mesh, p):
        return Interp(self, mesh, p)

    def server(self, n_slots=4, max_batch_rhs=32):
        return Server(self, n_slots, max_batch_rhs)

    def sync(self):
        _check(load().vp_sync(self.h))

    def profile(self, on=True):
        """Turn stage timing on/off (resets the accumulators)."""
        _check(load().vp_ctx_profile(self.h, 1 if on else 0))

    def cached_bytes(self):
        """Device bytes held in cached blocks of destroyed plans."""
        n = ctypes.c_uint64(0)
        _check(load().vp_ctx_cached_bytes(self.h, ctypes.byref(n)))
        return int(n.value)

    def memory(self):
        """(bytes in use, bytes cached) on the device (vp_ctx_memory)."""
        a, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(load().vp_ctx_memory(self.h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def trim(self):
        """Free the cached blocks of destroyed plans."""
        _check(load().vp_ctx_trim(self.h))

    def timings(self):
        """{stage: (total ms, launches)} accumulated since profile(True)."""
        ms = np.zeros(len(STAGES))
        n = np.zeros(len(STAGES), dtype=np.int64)
        _check(load().vp_ctx_timings(self.h, _ptr(ms), _ptr(n)))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def close(self):
        if self.h:
            _check(load().vp_ctx_destroy(self.h))
            self.h = None


class Server:
    """Continuous-batching request server (vp_server_*): device tensors in
    and out, tickets to poll or wait on."""

    def __init__(self, ctx, n_slots=4, max_batch_rhs=32):
        h = P()
        _check(load().vp_server_create(ctx.h, n_slots, max_batch_rhs, ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self._keep = {}

    def submit(self, plan, F, out, mixed=False):
        """F: device tensor [n_tri, n_p, R]; out: device tensor [n_tgt, R]."""
        if not (_is_device(F) and _is_device(out)):
            raise VPError(VP_EINVAL, "submit() takes device tensors")
        R = F.shape[2] if F.dim() == 3 else 1
        t = I64()
        _check(load().vp_submit(self.h, plan.h, R, _ptr(F), _ptr(out), VP_MIXED if mixed else VP_FP64,
                                ctypes.byref(t)))
        self._keep[t.value] = (F, out)
        return t.value

    def poll(self, ticket):
        d = ctypes.c_int()
        _check(load().vp_poll(self.h, ticket, ctypes.byref(d)))
        if d.value:
            self._keep.pop(ticket, None)
        return bool(d.value)

    def wait(self, ticket):
        _check(load().vp_wait(self.h, ticket))
        self._keep.pop(ticket, None)

    def stats(self):
        a, b, c, d, e = I64(), I64(), I64(), I64(), I64()
        _check(load().vp_server_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        _check(load().vp_server_admission(self.h, ctypes.byref(d), ctypes.byref(e)))
        return {"requests_done": a.value, "batches": b.value, "columns": c.value, "budget_waits": d.value,
                "rejected": e.value}

    def close(self):
        if self.h:
            _check(load().vp_server_destroy(self.h))
            self.h = None
            self._keep.clear()


class Mesh:
    def __init__(self, ctx, vert, tri, curved=None):
        """curved = (curved_tri [n], curved_side [n], curved_pts [n, deg+1, 2])
        or None (vp_mesh_set_curved_sides)."""
        vert = np.ascontiguousarray(vert, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = P()
        _check(load().vp_mesh_create(ctx.h, vert.shape[0], _ptr(vert), tri.shape[0], _ptr(tri), ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self.n_tri = tri.shape[0]
        if curved is not None:
            self.set_curved_sides(*curved)

    def set_curved_sides(self, curved_tri, curved_side, curved_pts):
        ct = np.ascontiguousarray(curved_tri, dtype=np.int32)
        cs = np.ascontiguousarray(curved_side, dtype=np.int32)
        cp = np.ascontiguousarray(curved_pts, dtype=np.float64)
        if cp.ndim != 3 or cp.shape[0] != ct.shape[0] or cp.shape[2] != 2 or cs.shape != ct.shape:
            raise VPError(VP_EINVAL, "curved sides: tri [n], side [n], pts [n, deg+1, 2]")
        _check(load().vp_mesh_set_curved_sides(self.h, ct.shape[0], _ptr(ct), _ptr(cs), cp.shape[1] - 1, _ptr(cp)))

    def map_points(self, ref_xy):
        """[n_tri, n, 2] physical positions of the reference points on every
        triangle (vp_mesh_map_points)."""
        ref = np.ascontiguousarray(np.asarray(ref_xy, dtype=np.float64).reshape(-1, 2))
        out = np.empty((self.n_tri, ref.shape[0], 2))
        _check(load().vp_mesh_map_points(self.h, ref.shape[0], _ptr(ref), _ptr(out)))
        return out

    def close(self):
        if self.h:
            _check(load().vp_mesh_destroy(self.h))
            self.h = None


class Graph:
    """A captured evaluation (vp_graph_*) of a plan for device density and
    output tensors that stay in place; launch() replays it asynchronously."""

    def __init__(self, plan, F, out, mixed=False, far_only=False):
        if not (_is_device(F) and _is_device(out)):
            raise VPError(VP_EINVAL, "Graph needs device tensors for the density and the output")
        import torch
        F = F if F.dim() == 3 else F.unsqueeze(-1)
        if not (F.is_contiguous() and out.is_contiguous()) or F.dtype != torch.float64 or out.dtype != torch.float64:
            raise VPError(VP_EINVAL, "Graph needs contiguous float64 tensors")
        h = P()
        _check(load().vp_graph_create(plan.h, F.shape[2], _ptr(F), _ptr(out), VP_MIXED if mixed else VP_FP64,
                                      VP_FAR_ONLY if far_only else 0, ctypes.byref(h)))
        self.h = h
        self.plan = plan
        self.F, self.out = F, out

    def launch(self):
        _check(load().vp_graph_launch(self.h))

    def close(self):
        if self.h:
            _check(load().vp_graph_destroy(self.h))
            self.h = None


class Interp:
    """Interpolation of the potential over a mesh (vp_interp_*): node values
    [n_tri, n_p] or [n_tri, n_p, R] in, values anywhere out."""

    def __init__(self, ctx, mesh, p):
        h = P()
        _check(load().vp_interp_create(ctx.h, mesh.h, int(p), ctypes.byref(h)))
        self.h = h
        self.mesh = mesh
        self.p = int(p)

    def locate(self, pts):
        """(tri [n] int32, -1 outside; ref [n, 2])."""
        pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 2))
        tri = np.empty(pts.shape[0], dtype=np.int32)
        ref = np.empty((pts.shape[0], 2))
        _check(load().vp_interp_locate(self.h, pts.shape[0], _ptr(pts), _ptr(tri), _ptr(ref)))
        return tri, ref

    def eval(self, u_nodes, tri, ref):
        u = np.ascontiguousarray(np.asarray(u_nodes, dtype=np.float64))
        single = u.ndim == 2
        if single:
            u = u[:, :, None]
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        ref = np.ascontiguousarray(np.asarray(ref, dtype=np.float64).reshape(-1, 2))
        out = np.empty((tri.shape[0], u.shape[2]))
        _check(load().vp_interp_eval(self.h, u.shape[2], _ptr(u), tri.shape[0], _ptr(tri), _ptr(ref), _ptr(out), 0))
        return out[:, 0] if single else out

    def __call__(self, u_nodes, pts):
        tri, ref = self.locate(pts)
        return self.eval(u_nodes, tri, ref)

    def close(self):
        if self.h:
            _check(load().vp_interp_destroy(self.h))
            self.h = None


def _plan_args(targets, c_n=1.0, q_near=7, n_l=16, tau=1e-13, depth_cap=50, dyadic_cap=60, near_model="ellipse",
               ball_factor=2.0, fmm_terms=0, fmm_leaf=128):
    """(targets as a contiguous host array or device tensor, PlanOpts)."""
    if _is_device(targets):
        tgt = targets.contiguous()
        flags = VP_DEVICE_PTRS
    else:
        tgt = np.ascontiguousarray(np.asarray(targets, dtype=np.float64).reshape(-1, 2))
        flags = 0
    if near_model not in NEAR_MODELS:
        raise VPError(VP_EINVAL, f"near_model must be one of {sorted(NEAR_MODELS)}")
    return tgt, PlanOpts(c_n, q_near, n_l, tau, depth_cap, dyadic_cap, flags, NEAR_MODELS[near_model], ball_factor,
                         fmm_terms, fmm_leaf)


def choose_q(ctx, mesh, p, eps, targets, q_min=4, q_max=16, n_rhs=1, mixed=False, n_solves=1.0, **opts):
    """vp_choose_q: the far order with the least plan time + n_solves
    evaluations.  Returns (q, {q: (plan_ms, exec_ms)})."""
    tgt, o = _plan_args(targets, **opts)
    n = q_max - q_min + 1
    plan_ms, exec_ms = np.zeros(max(n, 1)), np.zeros(max(n, 1))
    qb = ctypes.c_int(0)
    _check(load().vp_choose_q(ctx.h, mesh.h, p, eps, tgt.shape[0], _ptr(tgt), ctypes.byref(o), q_min, q_max, n_rhs,
                              VP_MIXED if mixed else VP_FP64, float(n_solves), ctypes.byref(qb), _ptr(plan_ms),
                              _ptr(exec_ms)))
    return qb.value, {q_min + k: (float(plan_ms[k]), float(exec_ms[k])) for k in range(n)}


class Plan:
    def __init__(self, ctx, mesh, p, q, eps, targets, **opts):
        tgt, opts = _plan_args(targets, **opts)
        h = P()
        _check(load().vp_plan_create(ctx.h, mesh.h, p, q, eps, tgt.shape[0], _ptr(tgt), ctypes.byref(opts),
                                     ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self.mesh = mesh
        st = self.info()
        self.n_tri, self.n_tgt, self.n_p, self.n_src = st["n_tri"], st["n_tgt"], st["n_p"], st["n_src"]
        self.n_pairs = st["n_pairs"]

    def info(self):
        s = PlanStats()
        _check(load().vp_plan_info(self.h, ctypes.byref(s)))
        return s.as_dict()

    def far_config(self, n_rhs=1, mixed=False):
        """Launch shape of the far sum used for n_rhs densities (dict)."""
        c = FarConfig()
        _check(load().vp_plan_far_config(self.h, n_rhs, VP_MIXED if mixed else VP_FP64, ctypes.byref(c)))
        return c.as_dict()

    def set_far_config(self, shape, mfma_tiles, n_split, n_rhs=1, mixed=False):
        """Store a far-sum launch shape (shape: a FAR_SHAPES name or its value)."""
        c = FarConfig(FAR_SHAPES.get(shape, shape), mfma_tiles, n_split)
        _check(load().vp_plan_set_far_config(self.h, n_rhs, VP_MIXED if mixed else VP_FP64, ctypes.byref(c)))

    def autotune(self, n_rhs=1, mixed=False, reps=3):
        """Time the candidate far-sum shapes on the device and keep the
        fastest; returns (config dict, mean ms of far sum + partial sums)."""
        c = FarConfig()
        ms = ctypes.c_double()
        _check(load().vp_plan_autotune(self.h, n_rhs, VP_MIXED if mixed else VP_FP64, reps, ctypes.byref(c),
                                       ctypes.byref(ms)))
        return c.as_dict(), ms.value

    def pairs(self):
        """(row_ptr [n_tgt+1] int64, tri [n_pairs] int32, kind [n_pairs] uint8)."""
        st = self.info()
        rp = np.empty(st["n_tgt"] + 1, dtype=np.int64)
        tri = np.empty(st["n_pairs"], dtype=np.int32)
        kind = np.empty(st["n_pairs"], dtype=np.uint8)
        _check(load().vp_plan_pairs(self.h, _ptr(rp), _ptr(tri), _ptr(kind)))
        return rp, tri, kind

    def rows(self):
        st = self.info()
        out = np.empty((st["n_pairs"], st["n_p"]))
        _check(load().vp_plan_rows(self.h, _ptr(out)))
        return out

    def rows_range(self, first, count):
        """Rows of pairs [first, first + count): [count, n_p]."""
        out = np.empty((count, self.n_p))
        _check(load().vp_plan_rows_range(self.h, int(first), int(count), _ptr(out)))
        return out

    def sources(self):
        out = np.empty((self.n_src, 2))
        _check(load().vp_plan_sources(self.h, _ptr(out)))
        return out

    def _density(self, F):
        if _is_device(F):
            if F.dim() == 2:
                F = F.unsqueeze(-1)
            R = F.shape[2]
            return F.contiguous(), R, True
        F = np.asarray(F, dtype=np.float64)
        if F.ndim == 2:
            F = F[:, :, None]
        if F.shape[:2] != (self.n_tri, self.n_p):
            raise VPError(VP_EINVAL, f"density shape {F.shape} != ({self.n_tri}, {self.n_p}, R)")
        return np.ascontiguousarray(F), F.shape[2], False

    def execute(self, F, far_only=False, out=None, asynchronous=False, mixed=False):
        """u [n_tgt] (one density) or [n_tgt, R].  Device tensors in ->
        device tensor out (written into `out` if given)."""
        single = (F.ndim if hasattr(F, "ndim") else F.dim()) == 2
        Fc, R, dev = self._density(F)
        flags = (VP_FAR_ONLY if far_only else 0)
        if dev:
            import torch
            if out is None:
                out = torch.empty((self.n_tgt, R), dtype=torch.float64, device=Fc.device)
            flags |= VP_DEVICE_PTRS | (VP_ASYNC if asynchronous else 0)
        else:
            out = np.empty((self.n_tgt, R))
        _check(load().vp_execute(self.h, R, _ptr(Fc), _ptr(out), VP_MIXED if mixed else VP_FP64, flags))
        return out[:, 0] if single else out

    def execute_noalloc(self, F, out, far_only=False, asynchronous=False, mixed=False):
        """vp_execute_noalloc: device tensors F [n_tri, n_p(, R)] and out
        [n_tgt, R]; the workspace is the library's fixed device array."""
        if not (_is_device(F) and _is_device(out)):
            raise VPError(VP_EINVAL, "execute_noalloc() takes device tensors")
        Fc, R, _ = self._density(F)
        flags = VP_DEVICE_PTRS | (VP_FAR_ONLY if far_only else 0) | (VP_ASYNC if asynchronous else 0)
        _check(load().vp_execute_noalloc(self.h, R, _ptr(Fc), _ptr(out), VP_MIXED if mixed else VP_FP64, flags))
        return out

    def coefficients(self, F):
        """(coefficients [n_tri, n_p, R], charges [n_src, R]) as host arrays."""
        Fc, R, dev = self._density(F)
        if dev:
            raise VPError(VP_EINVAL, "coefficients() takes host arrays")
        coef = np.empty((self.n_tri, self.n_p, R))
        charge = np.empty((self.n_src, R))
        _check(load().vp_coefficients(self.h, R, _ptr(Fc), _ptr(coef), _ptr(charge), 0))
        return coef, charge

    def close(self):
        if self.h:
            _check(load().vp_plan_destroy(self.h))
            self.h = None
