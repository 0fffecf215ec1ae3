// C ABI of libvp (declared in include/vp.h): argument checks, device memory
// ownership, host rule tables, and the order in which the kernels run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "vp_internal.h"

using vp::StageTimer;

namespace {

thread_local std::string g_err;

vp_status fail(vp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

vp_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(VP_ENOMEM, "%s: out of device memory", what);
  return fail(VP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define VP_HIP(call, what)                  \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

vp_plan_opts default_opts() {
  vp_plan_opts o;
  o.c_n = 1.0;
  o.q_near = 7;
  o.n_l = 16;
  o.tau = 1e-13;
  o.depth_cap = 50;
  o.dyadic_cap = 60;
  o.flags = 0;
  o.near_model = VP_NEAR_ELLIPSES;
  o.ball_factor = 2.0;
  o.fmm_terms = 0;
  o.fmm_leaf = 128;
  return o;
}

// the execute workspace back to the context (queued work done first)
void release_workspace(vp_plan* pl) {
  void* ws[] = {pl->ws_f, pl->ws_c, pl->ws_q, pl->ws_part, pl->ws_u, pl->ws_q32};
  bool any = false;
  for (void* p : ws) any = any || p;
  if (!any) return;
  (void)hipDeviceSynchronize();
  for (void* p : ws)
    if (p) vp::ctx_release(pl->ctx, p);
  pl->ws_f = pl->ws_c = pl->ws_q = pl->ws_part = pl->ws_u = nullptr;
  pl->ws_q32 = nullptr;
  pl->ws_bytes = 0;
}

void free_plan_memory(vp_plan* pl) {
  if (!pl->allocs.empty()) {
    // kernels of the plan's build or of executes on other streams may still
    // read these blocks; the cache hands them out without a device wait
    (void)hipDeviceSynchronize();
    for (void* p : pl->allocs) vp::ctx_release(pl->ctx, p);
  }
  pl->allocs.clear();
  release_workspace(pl);
}

struct PlanGuard {
  vp_plan* pl;
  bool keep = false;
  ~PlanGuard() {
    if (!keep && pl) {
      free_plan_memory(pl);
      delete pl;
    }
  }
};

template <class T>
hipError_t upload(vp_plan* pl, T** dst, const T* src, size_t n, hipStream_t st) {
  hipError_t e = vp::plan_alloc(pl, (void**)dst, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess && n) e = hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, st);
  return e;
}

// Stage bracket: records an event pair on the context's stream when
// profiling is on.

void fold_timings(vp_ctx* ctx) {
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->ms[p.stage] += ms;
      ctx->launches[p.stage] += p.launches;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  ctx->pending.clear();
}

}  // namespace

void vp::set_last_error(const char* msg) { g_err = msg; }

extern "C" {

vp_status vp_ctx_profile(vp_ctx* ctx, int on) {
  if (!ctx) return fail(VP_EINVAL, "vp_ctx_profile: ctx is NULL");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  fold_timings(ctx);
  for (int i = 0; i < VP_N_STAGES; ++i) {
    ctx->ms[i] = 0.0;
    ctx->launches[i] = 0;
  }
  ctx->profile = on != 0;
  return VP_OK;
}

vp_status vp_ctx_timings(vp_ctx* ctx, double* ms_out, int64_t* launches_out) {
  if (!ctx) return fail(VP_EINVAL, "vp_ctx_timings: ctx is NULL");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  fold_timings(ctx);
  for (int i = 0; i < VP_N_STAGES; ++i) {
    if (ms_out) ms_out[i] = ctx->ms[i];
    if (launches_out) launches_out[i] = ctx->launches[i];
  }
  return VP_OK;
}

const char* vp_last_error(void) { return g_err.c_str(); }

vp_status vp_ctx_create(int device, void* stream, uint64_t budget, vp_ctx** out) {
  if (!out) return fail(VP_EINVAL, "vp_ctx_create: out is NULL");
  int n = 0;
  VP_HIP(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(VP_EINVAL, "vp_ctx_create: device %d of %d", device, n);
  VP_HIP(hipSetDevice(device), "hipSetDevice");
  VP_HIP(vp::noalloc_setup(device), "vp_ctx_create: address of the allocation-free workspace");
  size_t dev_free = 0, dev_total = 0;
  VP_HIP(hipMemGetInfo(&dev_free, &dev_total), "vp_ctx_create: hipMemGetInfo");
  int n_cu = 0;
  VP_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device),
         "vp_ctx_create: compute unit count");
  vp_ctx* c = new vp_ctx;
  c->cache_cap = dev_total / 4;
  c->device = device;
  c->n_cu = std::max(n_cu, 1);
  c->stream = (hipStream_t)stream;
  c->budget = budget;
  *out = c;
  return VP_OK;
}

vp_status vp_ctx_destroy(vp_ctx* ctx) {
  if (!ctx) return VP_OK;
  if (ctx->live_meshes) return fail(VP_EBUSY, "vp_ctx_destroy: %d meshes still alive", ctx->live_meshes);
  if (ctx->live_servers) return fail(VP_EBUSY, "vp_ctx_destroy: %d servers still alive", ctx->live_servers);
  (void)hipSetDevice(ctx->device);
  fold_timings(ctx);
  for (auto& kv : ctx->fmm_ops)
    for (void* x : {(void*)kv.second.m2m, (void*)kv.second.l2l, (void*)kv.second.m2l})
      if (x) (void)hipFree(x);
  vp::ctx_trim(ctx);
  delete ctx;
  return VP_OK;
}

vp_status vp_ctx_cached_bytes(const vp_ctx* ctx, uint64_t* bytes_out) {
  if (!ctx || !bytes_out) return fail(VP_EINVAL, "vp_ctx_cached_bytes: NULL argument");
  *bytes_out = ctx->cached;
  return VP_OK;
}

vp_status vp_ctx_memory(const vp_ctx* ctx, uint64_t* in_use_out, uint64_t* cached_out) {
  if (!ctx) return fail(VP_EINVAL, "vp_ctx_memory: ctx is NULL");
  if (in_use_out) *in_use_out = ctx->in_use;
  if (cached_out) *cached_out = ctx->cached;
  return VP_OK;
}

vp_status vp_ctx_trim(vp_ctx* ctx) {
  if (!ctx) return fail(VP_EINVAL, "vp_ctx_trim: ctx is NULL");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  vp::ctx_trim(ctx);
  return VP_OK;
}

vp_status vp_sync(vp_ctx* ctx) {
  if (!ctx) return fail(VP_EINVAL, "vp_sync: ctx is NULL");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  VP_HIP(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
  return VP_OK;
}

vp_status vp_ref_nodes(int p, double* xy, int* n_p) {
  if (p < 1 || p > vp::kMaxP) return fail(VP_EINVAL, "vp_ref_nodes: p = %d outside [1, %d]", p, vp::kMaxP);
  vp::Rule2D r = vp::interp_nodes(p);
  if (n_p) *n_p = (int)r.x.size();
  if (xy)
    for (size_t i = 0; i < r.x.size(); ++i) {
      xy[2 * i] = r.x[i];
      xy[2 * i + 1] = r.y[i];
    }
  return VP_OK;
}

vp_status vp_ref_rule(int which, int n, double* x, double* y, double* w, int* count) {
  if (n < 1 || n > 64) return fail(VP_EINVAL, "vp_ref_rule: n = %d outside [1, 64]", n);
  std::vector<double> rx, ry, rw;
  switch (which) {
    case 0: {
      vp::Rule1D r = vp::gauss_legendre01(n);
      rx = r.x;
      rw = r.w;
    } break;
    case 1: {
      if (n > 16) return fail(VP_EINVAL, "vp_ref_rule: log rule limited to 16 points");
      vp::Rule1D r = vp::gauss_log01(n);
      rx = r.x;
      rw = r.w;
    } break;
    case 2: {
      vp::Rule2D r = vp::collapsed_gauss(n);
      rx = r.x;
      ry = r.y;
      rw = r.w;
    } break;
    case 3: {
      if (n > vp::kMaxP) return fail(VP_EINVAL, "vp_ref_rule: order %d outside [1, %d]", n, vp::kMaxP);
      vp::radial_rule(n, rx, ry, rw);
    } break;
    case 4: {
      vp::Rule2D r = vp::collapsed_gauss(n);
      rw.resize(3);
      vp::edge_weights(r, n, rw.data());
    } break;
    case 5: {
      if (n > vp::kMaxP) return fail(VP_EINVAL, "vp_ref_rule: order %d outside [1, %d]", n, vp::kMaxP);
      vp::radial_rule_folded(n, rx, ry, rw);
    } break;
    case 6: {
      if (n > vp::kBasisLegMax)
        return fail(VP_EINVAL, "vp_ref_rule: the product basis is used up to order %d, not %d", vp::kBasisLegMax, n);
      rw = vp::basis_connection(n);
    } break;
    default:
      return fail(VP_EINVAL, "vp_ref_rule: unknown rule %d", which);
  }
  if (count) *count = (int)rw.size();
  for (size_t i = 0; i < rw.size(); ++i) {
    if (x && i < rx.size()) x[i] = rx[i];
    if (y && i < ry.size()) y[i] = ry[i];
    if (w) w[i] = rw[i];
  }
  return VP_OK;
}

vp_status vp_mesh_create(vp_ctx* ctx, int64_t n_vert, const double* vert, int64_t n_tri, const int32_t* tri,
                         vp_mesh** out) {
  if (!ctx || !out) return fail(VP_EINVAL, "vp_mesh_create: NULL argument");
  if (n_vert < 0 || n_tri < 0 || n_tri > 0x7fffffffLL) return fail(VP_EINVAL, "vp_mesh_create: bad sizes");
  if (n_tri > 0 && (!vert || !tri)) return fail(VP_EINVAL, "vp_mesh_create: NULL arrays");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  const size_t bytes = 15 * sizeof(double) * std::max<int64_t>(n_tri, 1);
  if (!vp::ctx_fits(ctx, bytes)) return fail(VP_ENOMEM, "vp_mesh_create: %zu bytes exceed the HBM budget", bytes);
  vp_mesh* m = new vp_mesh;
  m->ctx = ctx;
  m->n_tri = n_tri;
  double* base = nullptr;
  hipError_t e = hipMalloc((void**)&base, bytes);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "vp_mesh_create: hipMalloc");
  }
  const size_t T = std::max<int64_t>(n_tri, 1);
  m->geo = (double4*)base;  // first: 32-byte aligned
  m->ax = base + 8 * T;
  m->ay = base + 9 * T;
  m->bx = base + 10 * T;
  m->by = base + 11 * T;
  m->cx = base + 12 * T;
  m->cy = base + 13 * T;
  m->det = base + 14 * T;
  m->bytes = bytes;
  hipStream_t st = ctx->stream;
  double* d_vert = nullptr;
  int32_t* d_tri = nullptr;
  int* d_bad = nullptr;
  auto cleanup = [&](bool all) {
    if (d_vert) (void)hipFree(d_vert);
    if (d_tri) (void)hipFree(d_tri);
    if (d_bad) (void)hipFree(d_bad);
    if (all) {
      (void)hipFree(base);
      delete m;
    }
  };
  int bad = 0;
  if ((e = hipMalloc((void**)&d_vert, sizeof(double) * 2 * std::max<int64_t>(n_vert, 1))) != hipSuccess ||
      (e = hipMalloc((void**)&d_tri, sizeof(int32_t) * 3 * T)) != hipSuccess ||
      (e = hipMalloc((void**)&d_bad, sizeof(int))) != hipSuccess ||
      (e = hipMemsetAsync(d_bad, 0, sizeof(int), st)) != hipSuccess ||
      (n_vert && (e = hipMemcpyAsync(d_vert, vert, sizeof(double) * 2 * n_vert, hipMemcpyHostToDevice, st)) !=
                     hipSuccess) ||
      (n_tri && (e = hipMemcpyAsync(d_tri, tri, sizeof(int32_t) * 3 * n_tri, hipMemcpyHostToDevice, st)) !=
                    hipSuccess) ||
      (e = vp::launch_mesh_geom(d_vert, n_vert, d_tri, n_tri, m, d_bad, st)) != hipSuccess ||
      (e = hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    cleanup(true);
    return hip_fail(e, "vp_mesh_create");
  }
  cleanup(false);
  if (bad) {
    (void)hipFree(base);
    delete m;
    const char* why = bad == 1 ? "vertex index out of range" : bad == 2 ? "non-finite coordinate"
                                                                       : "degenerate triangle";
    return fail(VP_EINVAL, "vp_mesh_create: %s", why);
  }
  ctx->in_use += bytes;
  ctx->live_meshes++;
  *out = m;
  return VP_OK;
}

vp_status vp_mesh_destroy(vp_mesh* m) {
  if (!m) return VP_OK;
  if (m->live_plans) return fail(VP_EBUSY, "vp_mesh_destroy: %d plans still use this mesh", m->live_plans);
  (void)hipSetDevice(m->ctx->device);
  (void)hipFree(m->geo);  // the base of the mesh block
  for (void* q : {(void*)m->curve_of, (void*)m->curve_tri, (void*)m->curve_coef, (void*)m->curve_box})
    if (q) (void)hipFree(q);
  m->ctx->in_use -= m->bytes;
  m->ctx->live_meshes--;
  delete m;
  return VP_OK;
}

namespace {

// Chebyshev coefficients of the polynomial through values f_j at
// s_j = -cos(pi j / d), j = 0..d (a discrete cosine transform, long double).
void cheb_from_lobatto(const long double* f, int d, long double* c) {
  const long double pi = acosl(-1.0L);
  for (int k = 0; k <= d; ++k) {
    long double acc = 0.0L;
    for (int m = 0; m <= d; ++m) {
      // s = cos(pi m / d) is the node j = d - m
      const long double w = (m == 0 || m == d) ? 0.5L : 1.0L;
      acc += w * f[d - m] * cosl(pi * k * m / d);
    }
    c[k] = acc * 2.0L / d;
  }
  c[0] *= 0.5L;
  c[d] *= 0.5L;
}

// coefficients of d/ds of sum c_k T_k
void cheb_derivative(const long double* c, int d, long double* dc) {
  for (int k = 0; k <= d; ++k) dc[k] = 0.0L;
  if (d == 0) return;
  long double b2 = 0.0L, b1 = 0.0L;  // dc_{k+1}, dc_{k+2} from the top
  for (int k = d; k >= 1; --k) {
    const long double v = b1 + 2.0L * k * c[k];  // dc_{k-1} = dc_{k+1} + 2 k c_k
    dc[k - 1] = v;
    b1 = b2;
    b2 = v;
  }
  dc[0] *= 0.5L;
}

}  // namespace

vp_status vp_mesh_set_curved_sides(vp_mesh* m, int64_t n, const int32_t* tri, const int32_t* side, int deg,
                                   const double* pts) {
  if (!m || (n > 0 && (!tri || !side || !pts))) return fail(VP_EINVAL, "vp_mesh_set_curved_sides: NULL argument");
  if (n < 0 || n > m->n_tri) return fail(VP_EINVAL, "vp_mesh_set_curved_sides: bad count");
  if (deg < 1 || deg > vp::kCurveMax - 1)
    return fail(VP_EINVAL, "vp_mesh_set_curved_sides: degree %d outside [1, %d]", deg, vp::kCurveMax - 1);
  if (m->live_plans) return fail(VP_EBUSY, "vp_mesh_set_curved_sides: the mesh already has plans");
  if (m->n_curved) return fail(VP_EINVAL, "vp_mesh_set_curved_sides: curved sides are already set");
  if (n == 0) return VP_OK;
  VP_HIP(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t st = m->ctx->stream;
  const int64_t T = m->n_tri;
  std::vector<double> g(7 * T);
  VP_HIP(hipMemcpyAsync(g.data(), m->ax, sizeof(double) * 7 * T, hipMemcpyDeviceToHost, st), "hipMemcpy");
  VP_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
  double *ax = g.data(), *ay = ax + T, *bx = ax + 2 * T, *by = ax + 3 * T, *cx = ax + 4 * T, *cy = ax + 5 * T,
         *det = ax + 6 * T;
  std::vector<int32_t> of(T, -1), ctri(n);
  std::vector<double> coef((size_t)n * 4 * vp::kCurveMax, 0.0), box((size_t)n * 4);
  std::vector<long double> fx(deg + 1), fy(deg + 1), c(deg + 1), dc(deg + 1);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t t = tri[i];
    if (t < 0 || t >= T || side[i] < 0 || side[i] > 2)
      return fail(VP_EINVAL, "vp_mesh_set_curved_sides: entry %lld: bad triangle or side", (long long)i);
    if (of[t] >= 0) return fail(VP_EINVAL, "vp_mesh_set_curved_sides: triangle %d listed twice", t);
    const double* P = pts + (size_t)i * (deg + 1) * 2;
    for (int j = 0; j <= 2 * deg + 1; ++j)
      if (!std::isfinite(P[j])) return fail(VP_EINVAL, "vp_mesh_set_curved_sides: non-finite point");
    // the side's end points are two of the triangle's vertices
    const double vx[3] = {ax[t], bx[t], cx[t]}, vy[3] = {ay[t], by[t], cy[t]};
    const double ext = std::max(std::max(std::fabs(vx[1] - vx[0]), std::fabs(vy[1] - vy[0])),
                                std::max(std::fabs(vx[2] - vx[0]), std::fabs(vy[2] - vy[0])));
    auto vertex_at = [&](double x, double y) {
      for (int k = 0; k < 3; ++k)
        if (std::fabs(vx[k] - x) <= 1e-13 * ext && std::fabs(vy[k] - y) <= 1e-13 * ext) return k;
      return -1;
    };
    const int kb = vertex_at(P[0], P[1]), ka = vertex_at(P[2 * deg], P[2 * deg + 1]);
    if (kb < 0 || ka < 0 || ka == kb)
      return fail(VP_EINVAL, "vp_mesh_set_curved_sides: entry %lld: the side's end points are not two vertices "
                             "of triangle %d", (long long)i, t);
    const int kc = 3 - ka - kb;
    double Ax = vx[ka], Ay = vy[ka], Bx = vx[kb], By = vy[kb];
    const double Cx = vx[kc], Cy = vy[kc];
    bool rev = false;
    if ((Bx - Ax) * (Cy - Ay) - (By - Ay) * (Cx - Ax) < 0) {  // keep (A, B, C) counter-clockwise
      std::swap(Ax, Bx);
      std::swap(Ay, By);
      rev = true;
    }
    for (int j = 0; j <= deg; ++j) {
      const int jj = rev ? deg - j : j;
      fx[j] = P[2 * jj];
      fy[j] = P[2 * jj + 1];
    }
    fx[0] = Bx;
    fy[0] = By;
    fx[deg] = Ax;
    fy[deg] = Ay;
    double* cf = coef.data() + (size_t)i * 4 * vp::kCurveMax;
    cheb_from_lobatto(fx.data(), deg, c.data());
    cheb_derivative(c.data(), deg, dc.data());
    for (int k = 0; k <= deg; ++k) {
      cf[k] = (double)c[k];
      cf[2 * vp::kCurveMax + k] = (double)dc[k];
    }
    cheb_from_lobatto(fy.data(), deg, c.data());
    cheb_derivative(c.data(), deg, dc.data());
    for (int k = 0; k <= deg; ++k) {
      cf[vp::kCurveMax + k] = (double)c[k];
      cf[3 * vp::kCurveMax + k] = (double)dc[k];
    }
    // element box: the opposite vertex and 129 points of the side, padded
    double x0 = Cx, x1 = Cx, y0 = Cy, y1 = Cy;
    for (int j = 0; j <= 128; ++j) {
      const double sp = 2.0 * (j / 128.0) - 1.0;
      const double px = vp::cheb_clenshaw(cf, deg + 1, sp), py = vp::cheb_clenshaw(cf + vp::kCurveMax, deg + 1, sp);
      x0 = std::min(x0, px);
      x1 = std::max(x1, px);
      y0 = std::min(y0, py);
      y1 = std::max(y1, py);
    }
    const double pad = 0.05 * std::max(x1 - x0, y1 - y0);
    box[4 * i] = x0 - pad;
    box[4 * i + 1] = y0 - pad;
    box[4 * i + 2] = x1 + pad;
    box[4 * i + 3] = y1 + pad;
    ax[t] = Ax;
    ay[t] = Ay;
    bx[t] = Bx;
    by[t] = By;
    cx[t] = Cx;
    cy[t] = Cy;
    det[t] = (Bx - Ax) * (Cy - Ay) - (By - Ay) * (Cx - Ax);
    if (!(det[t] > 0.0)) return fail(VP_EINVAL, "vp_mesh_set_curved_sides: degenerate triangle %d", t);
    of[t] = (int32_t)i;
    ctri[i] = t;
  }
  // the packed copy of the geometry, with the curved triangles' new vertex order
  std::vector<double> gp((size_t)8 * T);
  for (int64_t t = 0; t < T; ++t) {
    double* q = gp.data() + 8 * t;
    q[0] = ax[t];
    q[1] = ay[t];
    q[2] = bx[t];
    q[3] = by[t];
    q[4] = cx[t];
    q[5] = cy[t];
    q[6] = det[t];
    q[7] = 0.0;
  }
  const size_t bytes = sizeof(int32_t) * (T + n) + sizeof(double) * (coef.size() + box.size());
  if (!vp::ctx_fits(m->ctx, bytes))
    return fail(VP_ENOMEM, "vp_mesh_set_curved_sides: %zu bytes exceed the HBM budget", bytes);
  hipError_t e;
  if ((e = hipMalloc((void**)&m->curve_of, sizeof(int32_t) * T)) != hipSuccess ||
      (e = hipMalloc((void**)&m->curve_tri, sizeof(int32_t) * n)) != hipSuccess ||
      (e = hipMalloc((void**)&m->curve_coef, sizeof(double) * coef.size())) != hipSuccess ||
      (e = hipMalloc((void**)&m->curve_box, sizeof(double) * box.size())) != hipSuccess ||
      (e = hipMemcpyAsync(m->curve_of, of.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(m->curve_tri, ctri.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(m->curve_coef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(m->curve_box, box.data(), sizeof(double) * box.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(m->ax, g.data(), sizeof(double) * 7 * T, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(m->geo, gp.data(), sizeof(double) * 8 * T, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    for (void* q : {(void*)m->curve_of, (void*)m->curve_tri, (void*)m->curve_coef, (void*)m->curve_box})
      if (q) (void)hipFree(q);
    m->curve_of = m->curve_tri = nullptr;
    m->curve_coef = m->curve_box = nullptr;
    return hip_fail(e, "vp_mesh_set_curved_sides");
  }
  m->n_curved = n;
  m->curve_deg = deg;
  m->bytes += bytes;
  m->ctx->in_use += bytes;
  return VP_OK;
}

vp_status vp_mesh_map_points(const vp_mesh* m, int n_ref, const double* ref_xy, double* out_xy) {
  if (!m || (n_ref > 0 && (!ref_xy || !out_xy))) return fail(VP_EINVAL, "vp_mesh_map_points: NULL argument");
  if (n_ref < 0 || n_ref > 4096) return fail(VP_EINVAL, "vp_mesh_map_points: n_ref outside [0, 4096]");
  for (int i = 0; i < 2 * n_ref; ++i)
    if (!std::isfinite(ref_xy[i])) return fail(VP_EINVAL, "vp_mesh_map_points: non-finite point");
  for (int i = 0; i < n_ref; ++i)
    if (!(ref_xy[2 * i] < 1.0)) return fail(VP_EINVAL, "vp_mesh_map_points: reference points need xi < 1");
  if (n_ref == 0 || m->n_tri == 0) return VP_OK;
  VP_HIP(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t st = m->ctx->stream;
  const size_t nout = (size_t)m->n_tri * n_ref * 2;
  double *d_ref = nullptr, *d_out = nullptr;
  hipError_t e;
  if ((e = hipMalloc((void**)&d_ref, sizeof(double) * 2 * n_ref)) != hipSuccess ||
      (e = hipMalloc((void**)&d_out, sizeof(double) * nout)) != hipSuccess ||
      (e = hipMemcpyAsync(d_ref, ref_xy, sizeof(double) * 2 * n_ref, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = vp::launch_map_points(m, n_ref, d_ref, d_out, st)) != hipSuccess ||
      (e = hipMemcpyAsync(out_xy, d_out, sizeof(double) * nout, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    if (d_ref) (void)hipFree(d_ref);
    if (d_out) (void)hipFree(d_out);
    return hip_fail(e, "vp_mesh_map_points");
  }
  (void)hipFree(d_ref);
  (void)hipFree(d_out);
  return VP_OK;
}

vp_status vp_plan_create(vp_ctx* ctx, const vp_mesh* mesh, int p, int q, double eps, int64_t n_tgt,
                         const double* tgt_xy, const vp_plan_opts* opts, vp_plan** out) {
  if (!ctx || !mesh || !out) return fail(VP_EINVAL, "vp_plan_create: NULL argument");
  if (mesh->ctx != ctx) return fail(VP_EINVAL, "vp_plan_create: mesh belongs to another context");
  if (p < 1 || p > vp::kMaxP) return fail(VP_EINVAL, "vp_plan_create: p = %d outside [1, %d]", p, vp::kMaxP);
  if (q < 2 || q > vp::kMaxQ) return fail(VP_EINVAL, "vp_plan_create: q = %d outside [2, %d]", q, vp::kMaxQ);
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(VP_EINVAL, "vp_plan_create: eps must be > 0");
  if (n_tgt < 0 || n_tgt > 0x7fffffffLL) return fail(VP_EINVAL, "vp_plan_create: bad n_tgt");
  if (n_tgt > 0 && !tgt_xy) return fail(VP_EINVAL, "vp_plan_create: tgt_xy is NULL");
  if ((int64_t)q * q * mesh->n_tri > 0x7fffff00LL)
    return fail(VP_EINVAL, "vp_plan_create: n_tri * q^2 = %lld far sources exceed 2^31",
                (long long)((int64_t)q * q * mesh->n_tri));
  vp_plan_opts o = opts ? *opts : default_opts();
  if (!(o.c_n > 0.0) || o.q_near < 2 || o.q_near > vp::kMaxQ || o.n_l < 2 || o.n_l > 64 || !(o.tau >= 0.0) ||
      o.depth_cap < 1 || o.depth_cap > 60 || o.dyadic_cap < 1 || o.dyadic_cap > 100 ||
      (o.near_model != VP_NEAR_ELLIPSES && o.near_model != VP_NEAR_BALL) ||
      (o.near_model == VP_NEAR_BALL && !(o.ball_factor > 0.0 && o.ball_factor <= 64.0)) ||
      (o.fmm_terms != 0 && (o.fmm_terms < 8 || o.fmm_terms > 63)) ||
      (o.fmm_terms != 0 && (o.fmm_leaf < 8 || o.fmm_leaf > 4096)))
    return fail(VP_EINVAL, "vp_plan_create: invalid options");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = ctx->stream;

  vp_plan* pl = new vp_plan;
  PlanGuard guard{pl};
  pl->ctx = ctx;
  pl->mesh = mesh;
  pl->p = p;
  pl->q = q;
  pl->n_p = vp::n_basis(p);
  pl->n_f = q * q;
  pl->eps = eps;
  pl->opts = o;
  pl->n_tri = mesh->n_tri;
  pl->n_src = mesh->n_tri * pl->n_f;
  pl->n_tgt = n_tgt;

  // host reference rules
  vp::Rule2D far = vp::collapsed_gauss(q);
  vp::Rule2D nr = vp::collapsed_gauss(o.q_near);
  vp::Rule1D gl = vp::gauss_legendre01(o.n_l);
  vp::Rule2D nodes = vp::interp_nodes(p);
  std::vector<double> rr, ra, rb, rcr, rca, rcb;
  vp::radial_rule_folded(p, rr, ra, rb);  // straight self pieces: p + 1 nodes per ray
  vp::radial_rule(2 * vp::kCurvedRadial - 3, rcr, rca, rcb);  // kCurvedRadial points per part
  vp::edge_weights(far, q, pl->far_what);
  vp::edge_weights(nr, o.q_near, pl->near_what);
  pl->n_r = (int)rr.size();

  hipError_t e;
#define UP(dst, vec) \
  if ((e = upload(pl, &(dst), (vec).data(), (vec).size(), st)) != hipSuccess) return hip_fail(e, "vp_plan_create: upload")
  UP(pl->far_x, far.x);
  UP(pl->far_y, far.y);
  UP(pl->far_w, far.w);
  UP(pl->near_x, nr.x);
  UP(pl->near_y, nr.y);
  UP(pl->near_w, nr.w);
  UP(pl->gl_s, gl.x);
  UP(pl->gl_w, gl.w);
  UP(pl->rad_r, rr);
  UP(pl->rad_a, ra);
  UP(pl->rad_b, rb);
  UP(pl->rad_c_r, rcr);
  UP(pl->rad_c_a, rca);
  UP(pl->rad_c_b, rcb);
  pl->n_rc = (int)rcr.size();
  if (p <= vp::kBasisLegMax) {
    const std::vector<double> bg = vp::basis_connection(p);
    UP(pl->basis_g, bg);
  }
#undef UP
  const int NP = pl->n_p;
  if ((e = vp::plan_alloc(pl, (void**)&pl->vinv, sizeof(double) * NP * NP)) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->efar, sizeof(double) * pl->n_f * NP)) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->wfar, sizeof(double) * pl->n_f * NP)) != hipSuccess)
    return hip_fail(e, "vp_plan_create: hipMalloc");
  // Vandermonde inverse (device, FP64)
  {
    double* scratch = nullptr;
    const size_t sbytes = sizeof(double) * (2 * NP + 2 * NP * NP) + sizeof(int) * 2;
    vp::Scratch scr(ctx, st);
    if ((e = scr.alloc((void**)&scratch, sbytes)) != hipSuccess) return hip_fail(e, "vp_plan_create: hipMalloc");
    std::vector<double> nxy(2 * NP);
    for (int i = 0; i < NP; ++i) {
      nxy[i] = nodes.x[i];
      nxy[NP + i] = nodes.y[i];
    }
    int bad = 0;
    int* d_bad = (int*)(scratch + 2 * NP + 2 * NP * NP);
    if ((e = hipMemcpyAsync(scratch, nxy.data(), sizeof(double) * 2 * NP, hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemsetAsync(d_bad, 0, sizeof(int), st)) != hipSuccess ||
        (e = vp::launch_basis_tables(pl, scratch, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "vp_plan_create: basis tables");
    if (bad) return fail(VP_EINTERNAL, "vp_plan_create: singular Vandermonde matrix");
  }
  // sources and targets
  pl->n_src_pad = ((pl->n_src + 255) / 256) * 256;
  {
    std::vector<double2> lt(vp::kLogTab + 1), lw(vp::kFarLogTab + 1);
    vp::log_table(lt.data(), vp::kLogTab);
    vp::log_table(lw.data(), vp::kFarLogTab);
    if ((e = vp::plan_alloc(pl, (void**)&pl->logtab, sizeof(double2) * lt.size())) != hipSuccess ||
        (e = vp::plan_alloc(pl, (void**)&pl->logtab_wide, sizeof(double2) * lw.size())) != hipSuccess ||
        (e = hipMemcpyAsync(pl->logtab, lt.data(), sizeof(double2) * lt.size(), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(pl->logtab_wide, lw.data(), sizeof(double2) * lw.size(), hipMemcpyHostToDevice,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "vp_plan_create: log tables");
  }
  if ((e = vp::plan_alloc(pl, (void**)&pl->sxy, sizeof(double2) * pl->n_src_pad)) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->sgrp, sizeof(double) * 3 * (pl->n_src_pad / 64))) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->soff, sizeof(float2) * pl->n_src_pad)) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->swj, sizeof(double) * pl->n_src_pad)) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->deff, sizeof(double) * std::max<int64_t>(pl->n_tri, 1))) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->xt, sizeof(double) * n_tgt)) != hipSuccess ||
      (e = vp::plan_alloc(pl, (void**)&pl->yt, sizeof(double) * n_tgt)) != hipSuccess)
    return hip_fail(e, "vp_plan_create: hipMalloc");
  if ((e = vp::launch_sources(pl, st)) != hipSuccess) return hip_fail(e, "vp_plan_create: sources");
  {
    double* d_xy = nullptr;
    int* d_bad = nullptr;
    int bad = 0;
    vp::Scratch scr(ctx, st);
    if ((e = scr.alloc((void**)&d_xy, sizeof(double) * 2 * std::max<int64_t>(n_tgt, 1))) != hipSuccess ||
        (e = scr.alloc((void**)&d_bad, sizeof(int))) != hipSuccess)
      return hip_fail(e, "vp_plan_create: hipMalloc");
    const hipMemcpyKind kind = (o.flags & VP_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((e = hipMemsetAsync(d_bad, 0, sizeof(int), st)) != hipSuccess ||
        (n_tgt && (e = hipMemcpyAsync(d_xy, tgt_xy, sizeof(double) * 2 * n_tgt, kind, st)) != hipSuccess) ||
        (e = vp::launch_split_xy(d_xy, n_tgt, pl->xt, pl->yt, d_bad, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "vp_plan_create: targets");
    if (bad) return fail(VP_EINVAL, "vp_plan_create: non-finite target coordinate");
  }
  // near-field pair list
  hipEvent_t ev0, ev1, ev2;
  VP_HIP(hipEventCreate(&ev0), "hipEventCreate");
  VP_HIP(hipEventCreate(&ev1), "hipEventCreate");
  VP_HIP(hipEventCreate(&ev2), "hipEventCreate");
  struct EvGuard {
    hipEvent_t a, b, c;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      (void)hipEventDestroy(c);
    }
  } evg{ev0, ev1, ev2};
  VP_HIP(hipEventRecord(ev0, st), "hipEventRecord");
  StageTimer tm_classify(ctx, VP_STAGE_CLASSIFY);
  {
    std::string err;
    e = vp::build_pairs(pl, st, err);
    if (e != hipSuccess) {
      if (!err.empty()) return fail(VP_ENOMEM, "vp_plan_create: %s", err.c_str());
      return hip_fail(e, "vp_plan_create: near-field list");
    }
    if (o.fmm_terms > 0 && pl->n_src > 0 && pl->n_tgt > 0) {
      pl->fmm_terms = o.fmm_terms;
      if ((e = vp::build_fmm(pl, o.fmm_leaf, st)) != hipSuccess) return hip_fail(e, "vp_plan_create: FMM tree");
    }
  }
  tm_classify.stop(1);
  VP_HIP(hipEventRecord(ev1, st), "hipEventRecord");
  StageTimer tm_rows(ctx, VP_STAGE_ROWS);
  // correction rows
  if ((e = vp::plan_alloc(pl, (void**)&pl->rows, sizeof(double) * pl->n_pairs * NP)) != hipSuccess)
    return hip_fail(e, "vp_plan_create: rows");
  {
    int* d_flag = nullptr;
    int64_t* d_stats = nullptr;
    constexpr size_t kStatBytes = sizeof(int64_t) * vp::kRowStatSlots * vp::kRowStatStride;
    vp::Scratch scr(ctx, st);
    if ((e = scr.alloc((void**)&d_flag, sizeof(int))) != hipSuccess ||
        (e = scr.alloc((void**)&d_stats, kStatBytes)) != hipSuccess)
      return hip_fail(e, "vp_plan_create: hipMalloc");
    int flag = 0;
    std::vector<int64_t> slots((size_t)vp::kRowStatSlots * vp::kRowStatStride);
    if ((e = hipMemsetAsync(d_flag, 0, sizeof(int), st)) != hipSuccess ||
        (e = hipMemsetAsync(d_stats, 0, kStatBytes, st)) != hipSuccess ||
        (e = vp::launch_rows(pl, d_flag, d_stats, st)) != hipSuccess ||
        (e = hipEventRecord(ev2, st)) != hipSuccess || (tm_rows.stop(1), false) ||
        (e = hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(slots.data(), d_stats, kStatBytes, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "vp_plan_create: correction rows");
    for (int i = 0; i < 4; ++i) {
      pl->stats[i] = 0;
      for (int sl = 0; sl < vp::kRowStatSlots; ++sl) pl->stats[i] += slots[(size_t)sl * vp::kRowStatStride + i];
    }
    pl->stats[0] += pl->tab_leaves;
    if (flag == 1) return fail(VP_EINTERNAL, "vp_plan_create: near subdivision exceeded its depth-first stack");
    if (flag) return fail(VP_EINTERNAL, "vp_plan_create: a self pair's point location on a curved triangle failed");
  }
  float ms1 = 0.f, ms2 = 0.f;
  (void)hipEventElapsedTime(&ms1, ev0, ev1);
  (void)hipEventElapsedTime(&ms2, ev1, ev2);
  pl->ms_classify = ms1;
  pl->ms_rows = ms2;
  const_cast<vp_mesh*>(mesh)->live_plans++;
  guard.keep = true;
  *out = pl;
  return VP_OK;
}

vp_status vp_plan_info(const vp_plan* pl, vp_plan_stats* out) {
  if (!pl || !out) return fail(VP_EINVAL, "vp_plan_info: NULL argument");
  out->n_tri = pl->n_tri;
  out->n_src = pl->n_src;
  out->n_tgt = pl->n_tgt;
  out->n_pairs = pl->n_pairs;
  out->n_self = pl->n_self;
  out->near_subtri = pl->stats[0];
  out->self_panels = pl->stats[1];
  out->capped_leaves = pl->stats[2];
  out->depth_first_pairs = pl->stats[3];
  out->bytes_resident = (int64_t)(pl->bytes + pl->ws_bytes);
  out->p = pl->p;
  out->q = pl->q;
  out->n_p = pl->n_p;
  out->n_f = pl->n_f;
  out->eps = pl->eps;
  out->ms_classify = pl->ms_classify;
  out->ms_rows = pl->ms_rows;
  out->far_split = vp::far_config(pl, 1, false).n_split;
  out->cluster_entries = pl->n_entries;
  out->fmm_terms = pl->fmm_terms;
  out->fmm_levels = pl->fmm_levels;
  out->fmm_near_pairs = pl->fmm_near_pairs;
  out->fmm_m2l_pairs = pl->fmm_m2l_pairs;
  out->tab_pairs = pl->tab_pairs;
  out->tab_leaves = pl->tab_leaves;
  return VP_OK;
}

vp_status vp_plan_pairs(const vp_plan* pl, int64_t* row_ptr, int32_t* tri, uint8_t* kind) {
  if (!pl) return fail(VP_EINVAL, "vp_plan_pairs: plan is NULL");
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  hipStream_t st = pl->ctx->stream;
  if (row_ptr)
    VP_HIP(hipMemcpyAsync(row_ptr, pl->row_ptr, sizeof(int64_t) * (pl->n_tgt + 1), hipMemcpyDeviceToHost, st),
           "hipMemcpy");
  if (tri && pl->n_pairs)
    VP_HIP(hipMemcpyAsync(tri, pl->pair_tri, sizeof(int32_t) * pl->n_pairs, hipMemcpyDeviceToHost, st), "hipMemcpy");
  if (kind && pl->n_pairs)
    VP_HIP(hipMemcpyAsync(kind, pl->pair_kind, pl->n_pairs, hipMemcpyDeviceToHost, st), "hipMemcpy");
  VP_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
  return VP_OK;
}

vp_status vp_plan_rows(const vp_plan* pl, double* rows) {
  if (!pl || !rows) return fail(VP_EINVAL, "vp_plan_rows: NULL argument");
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  if (pl->n_pairs)
    VP_HIP(hipMemcpyAsync(rows, pl->rows, sizeof(double) * pl->n_pairs * pl->n_p, hipMemcpyDeviceToHost,
                          pl->ctx->stream),
           "hipMemcpy");
  VP_HIP(hipStreamSynchronize(pl->ctx->stream), "hipStreamSynchronize");
  return VP_OK;
}

vp_status vp_plan_rows_range(const vp_plan* pl, int64_t first_pair, int64_t count, double* rows) {
  if (!pl || (!rows && count)) return fail(VP_EINVAL, "vp_plan_rows_range: NULL argument");
  if (first_pair < 0 || count < 0 || first_pair > pl->n_pairs || count > pl->n_pairs - first_pair)
    return fail(VP_EINVAL, "vp_plan_rows_range: pairs [%lld, %lld) outside [0, %lld)", (long long)first_pair,
                (long long)(first_pair + count), (long long)pl->n_pairs);
  if (!count) return VP_OK;
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  VP_HIP(hipMemcpyAsync(rows, pl->rows + (size_t)first_pair * pl->n_p, sizeof(double) * count * pl->n_p,
                        hipMemcpyDeviceToHost, pl->ctx->stream),
         "hipMemcpy");
  VP_HIP(hipStreamSynchronize(pl->ctx->stream), "hipStreamSynchronize");
  return VP_OK;
}

vp_status vp_plan_sources(const vp_plan* pl, double* xy) {
  if (!pl || !xy) return fail(VP_EINVAL, "vp_plan_sources: NULL argument");
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  if (pl->n_src) {
    VP_HIP(hipMemcpyAsync(xy, pl->sxy, sizeof(double2) * pl->n_src, hipMemcpyDeviceToHost, pl->ctx->stream),
           "hipMemcpy");
    VP_HIP(hipStreamSynchronize(pl->ctx->stream), "hipStreamSynchronize");
  }
  return VP_OK;
}

}  // extern "C"

// Far-sum launch shape from the sizes.  Source chunks are set so that the
// launch has about 16384 blocks on the FP64 vector ALUs (32768 for the
// shorter FP32 sum, 4096 on the matrix cores, whose blocks hold 16x more
// work per source), with chunks of at least 64 sources and at most 2^23
// blocks: many short blocks keep the last round of blocks on the device
// short, which outweighs the extra partial sums.  The chunk count is a
// multiple of 8: the blocks of one chunk then share an XCD and its L2 (with
// 2 chunks instead of 8 the matrix-core sum of the 20k-triangle star at 64
// right-hand sides runs 5% longer).
// Wide blocks for one right-hand side once they can make 4096 such blocks,
// else narrow ones (the unit-square case with 1920 targets fills only one
// wide block per chunk).
namespace {
vp_far_config far_for_shape(const vp_plan* pl, int64_t R, bool mixed, int shape, int mfma_tiles) {
  vp_far_config c;
  c.shape = shape;
  c.mfma_tiles = mfma_tiles;
  const int64_t tpb = vp::far_targets_per_block(c, R, mixed);
  const int64_t n_tb = std::max<int64_t>(1, (pl->n_tgt + tpb - 1) / tpb);
  const int64_t blocks = R >= 16 ? 4096 : mixed ? 32768 : 16384;
  int64_t want = (blocks + n_tb - 1) / n_tb;
  want = ((want + 7) / 8) * 8;
  const int64_t most = std::max<int64_t>(1, std::min<int64_t>(pl->n_src_pad / 64, (1LL << 23) / n_tb));
  c.n_split = std::max<int64_t>(1, std::min(want, most));
  return c;
}
}  // namespace

int64_t vp::far_partial_doubles(const vp_plan* pl, int64_t n_split, int64_t R) {
  return n_split * pl->n_tgt * R + fmm_workspace_doubles(pl, R);
}

vp_far_config vp::far_default(const vp_plan* pl, int64_t R, bool mixed) {
  if (pl->fmm_terms > 0) return vp_far_config{VP_FAR_WIDE, 4, 1};  // one partial sum per target
  vp_far_config wide = far_for_shape(pl, R, mixed, VP_FAR_WIDE, 4);
  vp_far_config w1 = wide;
  w1.n_split = 1;
  const int64_t tpb = far_targets_per_block(w1, 1, false);
  const int64_t n_tb = std::max<int64_t>(1, (pl->n_tgt + tpb - 1) / tpb);
  if (n_tb * std::max<int64_t>(1, pl->n_src_pad / 64) >= 4096) return wide;
  return far_for_shape(pl, R, mixed, VP_FAR_NARROW1, 4);
}

vp_far_config vp::far_config(const vp_plan* pl, int64_t R, bool mixed) {
  auto it = pl->far_tuned.find({R, mixed ? 1 : 0});
  return it != pl->far_tuned.end() ? it->second : far_default(pl, R, mixed);
}

bool vp::far_config_valid(const vp_plan* pl, const vp_far_config& c) {
  if (pl->fmm_terms > 0 && c.n_split != 1) return false;
  return c.shape >= VP_FAR_WIDE && c.shape <= VP_FAR_NARROW2 &&
         (c.mfma_tiles == 1 || c.mfma_tiles == 2 || c.mfma_tiles == 4) && c.n_split >= 1 &&
         c.n_split <= std::max<int64_t>(1, pl->n_src_pad / 64);
}

namespace {

// grow the execute workspace to n_rhs right-hand sides
// (and at least `split` far partials per target and right-hand side)
vp_status ensure_workspace(vp_plan* pl, int64_t R, int64_t split) {
  if (pl->ws_rhs >= R && pl->ws_split >= split && pl->ws_c) return VP_OK;
  R = std::max(R, pl->ws_rhs);
  split = std::max(split, pl->ws_split);
  release_workspace(pl);
  pl->ws_bytes = 0;
  pl->ws_rhs = 0;
  const size_t nF = (size_t)pl->n_tri * pl->n_p * R;
  const size_t nQ = (size_t)pl->n_src_pad * R;
  const size_t nP = (size_t)vp::far_partial_doubles(pl, split, R);
  const size_t nU = (size_t)pl->n_tgt * R;
  const size_t bytes = 8 * (2 * nF + nQ + nP + nU) + 4 * nQ + 6 * 8;
  hipError_t e;
  vp_ctx* c = pl->ctx;
  size_t got[6] = {0, 0, 0, 0, 0, 0};
  if ((e = vp::ctx_alloc(c, (void**)&pl->ws_f, 8 * std::max<size_t>(nF, 1), &got[0])) != hipSuccess ||
      (e = vp::ctx_alloc(c, (void**)&pl->ws_c, 8 * std::max<size_t>(nF, 1), &got[1])) != hipSuccess ||
      (e = vp::ctx_alloc(c, (void**)&pl->ws_q, 8 * std::max<size_t>(nQ, 1), &got[2])) != hipSuccess ||
      (e = vp::ctx_alloc(c, (void**)&pl->ws_part, 8 * std::max<size_t>(nP, 1), &got[3])) != hipSuccess ||
      (e = vp::ctx_alloc(c, (void**)&pl->ws_u, 8 * std::max<size_t>(nU, 1), &got[4])) != hipSuccess ||
      (e = vp::ctx_alloc(c, (void**)&pl->ws_q32, 4 * std::max<size_t>(nQ, 1), &got[5])) != hipSuccess ||
      (e = hipMemsetAsync(pl->ws_q, 0, 8 * std::max<size_t>(nQ, 1), pl->ctx->stream)) != hipSuccess) {
    release_workspace(pl);
    if (e == hipErrorOutOfMemory)
      return fail(VP_ENOMEM, "vp_execute: workspace of %zu bytes exceeds the device memory or the HBM budget", bytes);
    return hip_fail(e, "vp_execute: workspace");
  }
  pl->ws_rhs = R;
  pl->ws_split = split;
  pl->ws_bytes = got[0] + got[1] + got[2] + got[3] + got[4] + got[5];
  return VP_OK;
}

}  // namespace

namespace vp {

bool ctx_fits(vp_ctx* ctx, uint64_t bytes) {
  if (!ctx->budget) return true;
  if (ctx->in_use + ctx->cached + bytes > ctx->budget) ctx_trim(ctx);
  return ctx->in_use + bytes <= ctx->budget;
}

hipError_t ctx_alloc(vp_ctx* ctx, void** p, size_t bytes, size_t* got) {
  *p = nullptr;
  // sizes rounded so that blocks of nearly equal requests are interchangeable
  const size_t g = bytes >= (size_t(1) << 20) ? (size_t(2) << 20) : 256;
  const size_t r = (std::max<size_t>(bytes, 8) + g - 1) / g * g;
  auto it = ctx->cache.lower_bound(r);
  if (it != ctx->cache.end() && it->first - r <= r / 4) {
    *p = it->second;
    ctx->cached -= it->first;
    ctx->in_use += it->first;
    if (got) *got = it->first;
    ctx->cache.erase(it);
    return hipSuccess;
  }
  if (!ctx_fits(ctx, r)) return hipErrorOutOfMemory;
  hipError_t e = hipMalloc(p, r);
  if (e == hipErrorOutOfMemory && !ctx->cache.empty()) {
    (void)hipGetLastError();  // the failed attempt's error, not a later launch's
    ctx_trim(ctx);
    e = hipMalloc(p, r);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  ctx->block_size[*p] = r;
  ctx->in_use += r;
  if (got) *got = r;
  return hipSuccess;
}

void ctx_release(vp_ctx* ctx, void* p) {
  if (!p) return;
  auto it = ctx->block_size.find(p);
  if (it == ctx->block_size.end()) {
    (void)hipFree(p);
    return;
  }
  const size_t r = it->second;
  ctx->in_use -= r;
  // (with a budget, in_use + cached stays within it: the block was counted)
  if (ctx->cached + r > ctx->cache_cap) {
    ctx->block_size.erase(it);
    (void)hipFree(p);
    return;
  }
  ctx->cache.emplace(r, p);
  ctx->cached += r;
}

void ctx_trim(vp_ctx* ctx) {
  for (auto& kv : ctx->cache) {
    ctx->block_size.erase(kv.second);
    (void)hipFree(kv.second);
  }
  ctx->cache.clear();
  ctx->cached = 0;
}

hipError_t plan_alloc(vp_plan* pl, void** dst, size_t bytes) {
  size_t got = 0;
  hipError_t e = ctx_alloc(pl->ctx, dst, std::max<size_t>(bytes, 8), &got);
  if (e != hipSuccess) return e;
  pl->allocs.push_back(*dst);
  pl->bytes += got;
  return e;
}

}  // namespace vp

extern "C" {

vp_status vp_execute(vp_plan* pl, int64_t R, const double* density, double* u_out, vp_precision prec,
                     uint32_t flags) {
  if (!pl) return fail(VP_EINVAL, "vp_execute: plan is NULL");
  if (R < 1) return fail(VP_EINVAL, "vp_execute: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return fail(VP_EINVAL, "vp_execute: unknown precision %d", (int)prec);
  if ((!density && pl->n_tri) || (!u_out && pl->n_tgt)) return fail(VP_EINVAL, "vp_execute: NULL array");
  const bool dev = flags & VP_DEVICE_PTRS;
  if ((flags & VP_ASYNC) && !dev) return fail(VP_EINVAL, "vp_execute: VP_ASYNC needs VP_DEVICE_PTRS");
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  const vp_far_config cfg = vp::far_config(pl, R, prec == VP_MIXED);
  vp_status s = ensure_workspace(pl, R, cfg.n_split);
  if (s != VP_OK) return s;
  hipStream_t st = pl->ctx->stream;
  VP_HIP(vp::prepare_blocks(pl, R, st), "vp_execute: tables for blocks of 16 densities");
  const size_t nF = (size_t)pl->n_tri * pl->n_p * R;
  const double* F = density;
  if (!dev && nF) {
    VP_HIP(hipMemcpyAsync(pl->ws_f, density, 8 * nF, hipMemcpyHostToDevice, st), "vp_execute: upload");
    F = pl->ws_f;
  }
  double* U = dev ? u_out : pl->ws_u;
  vp_ctx* ctx = pl->ctx;
  {
    StageTimer tm(ctx, VP_STAGE_COEF);
    VP_HIP(vp::launch_coefficients(pl, F, R, pl->ws_c, pl->ws_q, st), "vp_execute: coefficients");
    tm.stop(2);
  }
  {
    StageTimer tm(ctx, VP_STAGE_FAR);
    int64_t nl = 0;
    VP_HIP(vp::launch_far(pl, pl->ws_q, R, cfg, pl->ws_part, st, &nl,
                          prec == VP_MIXED ? pl->ws_q32 : nullptr),
           "vp_execute: far field");
    tm.stop(nl);
  }
  {
    StageTimer tm(ctx, VP_STAGE_FINISH);
    VP_HIP(vp::launch_finish(pl, pl->ws_part, cfg.n_split, pl->ws_c, R, (flags & VP_FAR_ONLY) != 0, U, st),
           "vp_execute: corrections");
    tm.stop(1);
  }
  if (!dev && pl->n_tgt)
    VP_HIP(hipMemcpyAsync(u_out, U, 8 * (size_t)pl->n_tgt * R, hipMemcpyDeviceToHost, st), "vp_execute: download");
  if (!(flags & VP_ASYNC)) VP_HIP(hipStreamSynchronize(st), "vp_execute: synchronize");
  return VP_OK;
}

vp_status vp_coefficients(vp_plan* pl, int64_t R, const double* density, double* coef_out, double* charge_out,
                          uint32_t flags) {
  if (!pl) return fail(VP_EINVAL, "vp_coefficients: plan is NULL");
  if (R < 1) return fail(VP_EINVAL, "vp_coefficients: n_rhs must be >= 1");
  if (!density && pl->n_tri) return fail(VP_EINVAL, "vp_coefficients: NULL density");
  const bool dev = flags & VP_DEVICE_PTRS;
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  vp_status s = ensure_workspace(pl, R, 1);
  if (s != VP_OK) return s;
  hipStream_t st = pl->ctx->stream;
  const size_t nF = (size_t)pl->n_tri * pl->n_p * R;
  const double* F = density;
  if (!dev && nF) {
    VP_HIP(hipMemcpyAsync(pl->ws_f, density, 8 * nF, hipMemcpyHostToDevice, st), "vp_coefficients: upload");
    F = pl->ws_f;
  }
  VP_HIP(vp::launch_coefficients(pl, F, R, pl->ws_c, pl->ws_q, st), "vp_coefficients");
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (coef_out && nF) VP_HIP(hipMemcpyAsync(coef_out, pl->ws_c, 8 * nF, kind, st), "vp_coefficients: copy");
  if (charge_out && pl->n_src)
    VP_HIP(hipMemcpyAsync(charge_out, pl->ws_q, 8 * (size_t)pl->n_src * R, kind, st), "vp_coefficients: copy");
  if (!(flags & VP_ASYNC)) VP_HIP(hipStreamSynchronize(st), "vp_coefficients: synchronize");
  return VP_OK;
}

}  // extern "C"

struct vp_graph {
  vp_plan* plan = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double *c = nullptr, *q = nullptr, *part = nullptr;
  float* q32 = nullptr;
  size_t bytes = 0;
};

extern "C" {

vp_status vp_graph_create(vp_plan* pl, int64_t R, const double* density, double* u_out, vp_precision prec,
                          uint32_t flags, vp_graph** out) {
  if (!pl || !out) return fail(VP_EINVAL, "vp_graph_create: NULL argument");
  if (R < 1) return fail(VP_EINVAL, "vp_graph_create: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return fail(VP_EINVAL, "vp_graph_create: unknown precision");
  if (flags & ~(uint32_t)VP_FAR_ONLY) return fail(VP_EINVAL, "vp_graph_create: flags other than VP_FAR_ONLY");
  if ((!density && pl->n_tri) || (!u_out && pl->n_tgt)) return fail(VP_EINVAL, "vp_graph_create: NULL array");
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  vp_graph* g = new vp_graph;
  g->plan = pl;
  const vp_far_config cfg = vp::far_config(pl, R, prec == VP_MIXED);
  const int64_t split = cfg.n_split;
  const size_t nC = (size_t)pl->n_tri * pl->n_p * R, nQ = (size_t)pl->n_src_pad * R,
               nP = (size_t)vp::far_partial_doubles(pl, split, R);
  vp_ctx* ctx = pl->ctx;
  auto drop = [&](vp_graph* x) {
    if (x->exec) (void)hipGraphExecDestroy(x->exec);
    if (x->graph) (void)hipGraphDestroy(x->graph);
    if (x->cap) (void)hipStreamDestroy(x->cap);
    for (void* p : {(void*)x->c, (void*)x->q, (void*)x->part, (void*)x->q32})
      if (p) vp::ctx_release(ctx, p);
    delete x;
  };
  hipError_t e;
  size_t got[4] = {0, 0, 0, 0};
  if ((e = vp::ctx_alloc(ctx, (void**)&g->c, 8 * std::max<size_t>(nC, 1), &got[0])) != hipSuccess ||
      (e = vp::ctx_alloc(ctx, (void**)&g->q, 8 * std::max<size_t>(nQ, 1), &got[1])) != hipSuccess ||
      (e = vp::ctx_alloc(ctx, (void**)&g->part, 8 * std::max<size_t>(nP, 1), &got[2])) != hipSuccess ||
      (prec == VP_MIXED && (e = vp::ctx_alloc(ctx, (void**)&g->q32, 4 * std::max<size_t>(nQ, 1), &got[3])) !=
                               hipSuccess) ||
      (e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking)) != hipSuccess) {
    drop(g);
    if (e == hipErrorOutOfMemory)
      return fail(VP_ENOMEM, "vp_graph_create: workspace exceeds the device memory or the HBM budget");
    return hip_fail(e, "vp_graph_create");
  }
  g->bytes = got[0] + got[1] + got[2] + got[3];
  if ((e = vp::prepare_blocks(pl, R, pl->ctx->stream)) != hipSuccess) {
    drop(g);
    return hip_fail(e, "vp_graph_create: FMM tables");
  }
  // capture the evaluation's launches (no memsets, no host synchronisation)
  const bool prof = pl->ctx->profile;
  pl->ctx->profile = false;
  hipError_t le = hipSuccess;
  if ((e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal)) == hipSuccess) {
    if ((le = vp::launch_coefficients(pl, density, R, g->c, g->q, g->cap)) == hipSuccess &&
        (le = vp::launch_far(pl, g->q, R, cfg, g->part, g->cap, nullptr, prec == VP_MIXED ? g->q32 : nullptr)) ==
            hipSuccess)
      le = vp::launch_finish(pl, g->part, split, g->c, R, (flags & VP_FAR_ONLY) != 0, u_out, g->cap);
    e = hipStreamEndCapture(g->cap, &g->graph);
  }
  pl->ctx->profile = prof;
  if (e == hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop(g);
    return hip_fail(e, "vp_graph_create: capture");
  }
  pl->live_requests++;
  *out = g;
  return VP_OK;
}

vp_status vp_graph_launch(vp_graph* g) {
  if (!g) return fail(VP_EINVAL, "vp_graph_launch: NULL graph");
  VP_HIP(hipSetDevice(g->plan->ctx->device), "hipSetDevice");
  VP_HIP(hipGraphLaunch(g->exec, g->plan->ctx->stream), "vp_graph_launch");
  return VP_OK;
}

vp_status vp_graph_destroy(vp_graph* g) {
  if (!g) return VP_OK;
  (void)hipSetDevice(g->plan->ctx->device);
  (void)hipStreamSynchronize(g->plan->ctx->stream);
  g->plan->live_requests--;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  (void)hipStreamDestroy(g->cap);
  for (void* p : {(void*)g->c, (void*)g->q, (void*)g->part, (void*)g->q32})
    if (p) vp::ctx_release(g->plan->ctx, p);
  delete g;
  return VP_OK;
}

vp_status vp_plan_far_config(const vp_plan* pl, int64_t R, vp_precision prec, vp_far_config* out) {
  if (!pl || !out) return fail(VP_EINVAL, "vp_plan_far_config: NULL argument");
  if (R < 1) return fail(VP_EINVAL, "vp_plan_far_config: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return fail(VP_EINVAL, "vp_plan_far_config: unknown precision");
  *out = vp::far_config(pl, R, prec == VP_MIXED);
  return VP_OK;
}

vp_status vp_plan_set_far_config(vp_plan* pl, int64_t R, vp_precision prec, const vp_far_config* cfg) {
  if (!pl || !cfg) return fail(VP_EINVAL, "vp_plan_set_far_config: NULL argument");
  if (R < 1) return fail(VP_EINVAL, "vp_plan_set_far_config: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return fail(VP_EINVAL, "vp_plan_set_far_config: unknown precision");
  if (!vp::far_config_valid(pl, *cfg))
    return fail(VP_EINVAL,
                "vp_plan_set_far_config: shape %d, mfma_tiles %d, n_split %lld out of range (n_split <= %lld)",
                (int)cfg->shape, (int)cfg->mfma_tiles, (long long)cfg->n_split,
                (long long)std::max<int64_t>(1, pl->n_src_pad / 64));
  pl->far_tuned[{R, prec == VP_MIXED ? 1 : 0}] = *cfg;
  return VP_OK;
}

// The far-order policy: every candidate order is built and run, and the one
// with the least plan time plus n_solves evaluations is kept.
vp_status vp_choose_q(vp_ctx* ctx, const vp_mesh* mesh, int p, double eps, int64_t n_tgt, const double* tgt_xy,
                      const vp_plan_opts* opts, int q_min, int q_max, int64_t n_rhs, vp_precision prec,
                      double n_solves, int* q_best, double* plan_ms, double* exec_ms) {
  if (!ctx || !mesh || !q_best) return fail(VP_EINVAL, "vp_choose_q: NULL argument");
  if (q_min < 2 || q_max > vp::kMaxQ || q_min > q_max)
    return fail(VP_EINVAL, "vp_choose_q: orders [%d, %d] outside [2, %d]", q_min, q_max, vp::kMaxQ);
  if (p < 1 || p > vp::kMaxP) return fail(VP_EINVAL, "vp_choose_q: p = %d outside [1, %d]", p, vp::kMaxP);
  if (n_rhs < 1) return fail(VP_EINVAL, "vp_choose_q: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return fail(VP_EINVAL, "vp_choose_q: unknown precision");
  if (!(n_solves >= 0.0) || !std::isfinite(n_solves)) return fail(VP_EINVAL, "vp_choose_q: n_solves must be >= 0");
  VP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t st = ctx->stream;
  // zero densities: the work of an evaluation does not depend on the values
  const size_t nF = (size_t)mesh->n_tri * vp::n_basis(p) * n_rhs, nU = (size_t)std::max<int64_t>(n_tgt, 1) * n_rhs;
  void *F = nullptr, *U = nullptr;
  hipError_t e;
  if ((e = vp::ctx_alloc(ctx, &F, sizeof(double) * nF, nullptr)) != hipSuccess)
    return fail(VP_ENOMEM, "vp_choose_q: densities: %s", hipGetErrorString(e));
  if ((e = vp::ctx_alloc(ctx, &U, sizeof(double) * nU, nullptr)) != hipSuccess) {
    vp::ctx_release(ctx, F);
    return fail(VP_ENOMEM, "vp_choose_q: output: %s", hipGetErrorString(e));
  }
  struct Release {
    vp_ctx* c;
    void *a, *b;
    ~Release() {
      (void)hipStreamSynchronize(c->stream);
      vp::ctx_release(c, a);
      vp::ctx_release(c, b);
    }
  } rel{ctx, F, U};
  VP_HIP(hipMemsetAsync(F, 0, sizeof(double) * nF, st), "hipMemsetAsync");
  vp_plan_opts o = opts ? *opts : default_opts();
  typedef std::chrono::steady_clock clk;
  auto ms_since = [](clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); };
  double best = std::numeric_limits<double>::infinity();
  int qb = -1;
  for (int q = q_min; q <= q_max; ++q) {
    const int k = q - q_min;
    if (plan_ms) plan_ms[k] = std::numeric_limits<double>::quiet_NaN();
    if (exec_ms) exec_ms[k] = std::numeric_limits<double>::quiet_NaN();
    vp_plan* pl = nullptr;
    clk::time_point t0 = clk::now();
    vp_status s = vp_plan_create(ctx, mesh, p, q, eps, n_tgt, tgt_xy, &o, &pl);
    if (s == VP_ENOMEM || (s == VP_EINVAL && (int64_t)q * q * mesh->n_tri > 0x7fffff00LL)) continue;  // skipped
    if (s != VP_OK) return s;
    const double t_create = ms_since(t0);
    double t_first = 0.0, t_exec = std::numeric_limits<double>::infinity();
    for (int rep = 0; rep < 3 && s == VP_OK; ++rep) {
      clk::time_point t1 = clk::now();
      s = vp_execute(pl, n_rhs, (const double*)F, (double*)U, prec, VP_DEVICE_PTRS);
      const double t = ms_since(t1);
      if (rep == 0)
        t_first = t;
      else
        t_exec = std::min(t_exec, t);
    }
    vp_plan_destroy(pl);
    if (s == VP_ENOMEM) continue;
    if (s != VP_OK) return s;
    // tables an evaluation builds at its first call belong to the plan
    const double t_plan = t_create + std::max(0.0, t_first - t_exec);
    if (plan_ms) plan_ms[k] = t_plan;
    if (exec_ms) exec_ms[k] = t_exec;
    const double cost = t_plan + n_solves * t_exec;
    if (cost < best) {
      best = cost;
      qb = q;
    }
  }
  if (qb < 0) return fail(VP_ENOMEM, "vp_choose_q: no order in [%d, %d] fits the device or its budget", q_min, q_max);
  *q_best = qb;
  return VP_OK;
}


// Candidates: the shapes that change a launch for this n_rhs (the one-RHS
// FP64 kernel is the only one with wide blocks; the matrix-core tiles
// matter from 16 right-hand sides on), each with the size rule's split and
// 1/4, 1/2, 2 and 4 times it.  Candidates whose partial sums would exceed
// 1 GiB are dropped unless they are the size rule's own choice.
vp_status vp_plan_autotune(vp_plan* pl, int64_t R, vp_precision prec, int reps, vp_far_config* best_out,
                           double* best_ms_out) {
  if (!pl) return fail(VP_EINVAL, "vp_plan_autotune: plan is NULL");
  if (R < 1) return fail(VP_EINVAL, "vp_plan_autotune: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return fail(VP_EINVAL, "vp_plan_autotune: unknown precision");
  if (reps < 1 || reps > 1000) return fail(VP_EINVAL, "vp_plan_autotune: reps must be in [1, 1000]");
  if (pl->live_requests > 0)
    return fail(VP_EBUSY, "vp_plan_autotune: %d requests or graphs still use this plan", pl->live_requests);
  const bool mixed = prec == VP_MIXED;
  const vp_far_config def = vp::far_default(pl, R, mixed);
  if (pl->n_tgt == 0 || pl->n_src == 0) {
    pl->far_tuned[{R, mixed ? 1 : 0}] = def;
    if (best_out) *best_out = def;
    if (best_ms_out) *best_ms_out = 0.0;
    return VP_OK;
  }
  VP_HIP(hipSetDevice(pl->ctx->device), "hipSetDevice");
  const int64_t rem = R % 16;
  std::vector<int> shapes;
  if (R < 16 || rem != 0) {
    if (!mixed && rem % 2 == 1) shapes.push_back(VP_FAR_WIDE);
    shapes.push_back(VP_FAR_NARROW1);
    shapes.push_back(VP_FAR_NARROW2);
  } else {
    shapes.push_back(def.shape);
  }
  std::vector<int> tiles = R >= 16 ? std::vector<int>{1, 2, 4} : std::vector<int>{def.mfma_tiles};
  const int64_t max_split = std::max<int64_t>(1, pl->n_src_pad / 64);
  const size_t per_split_bytes = 8 * (size_t)pl->n_tgt * R;
  std::vector<vp_far_config> cand{def};
  if (pl->fmm_terms > 0) shapes.clear();  // the FMM has no shapes to choose
  for (int sh : shapes)
    for (int mt : tiles) {
      const vp_far_config base = far_for_shape(pl, R, mixed, sh, mt);  // the size rule for this shape
      for (int k = -2; k <= 2; ++k) {
        vp_far_config c = base;
        int64_t n = k < 0 ? base.n_split >> -k : base.n_split << k;
        if (n >= 8) n = n / 8 * 8;
        c.n_split = std::max<int64_t>(1, std::min<int64_t>(n, max_split));
        if (c.n_split * per_split_bytes > (size_t(1) << 30)) continue;
        bool dup = false;
        for (const vp_far_config& o : cand)
          dup = dup || (o.shape == c.shape && o.mfma_tiles == c.mfma_tiles && o.n_split == c.n_split);
        if (!dup) cand.push_back(c);
      }
    }
  int64_t need_split = 1;
  for (const vp_far_config& c : cand) need_split = std::max(need_split, c.n_split);
  vp_status s = ensure_workspace(pl, R, need_split);
  if (s != VP_OK) return s;
  hipStream_t st = pl->ctx->stream;
  VP_HIP(vp::prepare_blocks(pl, R, st), "vp_plan_autotune: tables for blocks of 16 densities");
  VP_HIP(hipMemsetAsync(pl->ws_c, 0, 8 * std::max<size_t>((size_t)pl->n_tri * pl->n_p * R, 1), st),
         "vp_plan_autotune: clear");
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  double best_ms = 0.0;
  vp_far_config best = def;
  for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
    const vp_far_config& c = cand[i];
    auto one = [&]() {
      hipError_t le = vp::launch_far(pl, pl->ws_q, R, c, pl->ws_part, st, nullptr, mixed ? pl->ws_q32 : nullptr);
      if (le == hipSuccess) le = vp::launch_finish(pl, pl->ws_part, c.n_split, pl->ws_c, R, false, pl->ws_u, st);
      return le;
    };
    if ((e = one()) != hipSuccess) break;  // warm-up
    if ((e = hipEventRecord(ev[0], st)) != hipSuccess) break;
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = one();
    if (e != hipSuccess || (e = hipEventRecord(ev[1], st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(ev[1])) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) break;
    const double avg = (double)ms / reps;
    if (i == 0 || avg < best_ms) {
      best_ms = avg;
      best = c;
    }
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(e, "vp_plan_autotune");
  pl->far_tuned[{R, mixed ? 1 : 0}] = best;
  if (best_out) *best_out = best;
  if (best_ms_out) *best_ms_out = best_ms;
  return VP_OK;
}

vp_status vp_plan_destroy(vp_plan* pl) {
  if (!pl) return VP_OK;
  if (pl->live_requests > 0)
    return fail(VP_EBUSY, "vp_plan_destroy: %d server requests still use this plan", pl->live_requests);
  (void)hipSetDevice(pl->ctx->device);
  (void)hipStreamSynchronize(pl->ctx->stream);
  const_cast<vp_mesh*>(pl->mesh)->live_plans--;
  free_plan_memory(pl);
  delete pl;
  return VP_OK;
}

}  // extern "C"
