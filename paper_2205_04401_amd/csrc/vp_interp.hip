// Interpolation of the potential over a mesh element (Sec. 3.5): given u at
// the order-p interpolation nodes of every triangle of a mesh (for instance
// the staggered target mesh whose nodes were the targets of vp_execute),
// u anywhere in the mesh is sum_k c_k K_k(rho^{-1}(x)) with c = V^{-1} u of
// the triangle that contains x; rho^{-1} is the affine inverse, or Newton's
// method on a curved triangle.
//
//   vp_interp_create   V^{-1} on the device (the hot path's Gauss-Jordan
//                      kernel) and a uniform grid of triangle boxes (cell
//                      lists built once on the host, ascending triangle
//                      index within a cell)
//   k_locate           point -> (first containing triangle, rho^{-1}(x))
//   k_ieval<P>         (triangle, reference point, RHS) -> u
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "vp_internal.h"

struct vp_interp {
  vp_ctx* ctx = nullptr;
  vp_mesh* mesh = nullptr;
  int p = 0, n_p = 0;
  double* vinv = nullptr;      // [n_p][n_p]
  double x0 = 0, y0 = 0, inv_h = 0;
  int nx = 1, ny = 1;
  int64_t* cell_ptr = nullptr; // [nx ny + 1]
  int32_t* cell_tri = nullptr;
  size_t bytes = 0;
};

namespace vp {
namespace {

constexpr int kIBlock = 256;
constexpr double kTau = 1e-13;  // barycentric tolerance of the containment test

vp_status ifail(vp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return s;
}

vp_status ihip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return ifail(VP_ENOMEM, "%s: out of device memory", what);
  return ifail(VP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

unsigned grid_for(int64_t n) {
  const int64_t nb = (n + kIBlock - 1) / kIBlock;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, 1 << 20));
}

struct LocView {
  const double *ax, *ay, *bx, *by, *cx, *cy, *det;
  CurveView cv;
  double x0, y0, inv_h;
  int nx, ny;
  const int64_t* cell_ptr;
  const int32_t* cell_tri;
};

__global__ void k_locate(LocView v, int64_t n, const double* __restrict__ pts, int32_t* __restrict__ tri_out,
                         double* __restrict__ ref_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = pts[2 * i], y = pts[2 * i + 1];
    int32_t hit = -1;
    double r1 = 0.0, r2 = 0.0;
    const double fi = (x - v.x0) * v.inv_h, fj = (y - v.y0) * v.inv_h;
    if (fi >= 0.0 && fj >= 0.0 && fi < (double)v.nx && fj < (double)v.ny) {
      const int64_t c = (int64_t)(int)fj * v.nx + (int)fi;
      for (int64_t k = v.cell_ptr[c]; k < v.cell_ptr[c + 1] && hit < 0; ++k) {
        const int32_t t = v.cell_tri[k];
        const double Ax = v.ax[t], Ay = v.ay[t], Bx = v.bx[t], By = v.by[t], Cx = v.cx[t], Cy = v.cy[t];
        const double D = v.det[t];
        const int cc = v.cv.of ? v.cv.of[t] : -1;
        double z1, z2;
        if (cc >= 0) {
          const double* b = v.cv.box + 4 * cc;
          if (!(x >= b[0] && x <= b[2] && y >= b[1] && y <= b[3])) continue;
          if (!vp_blend_inverse(Ax, Ay, Bx, By, Cx, Cy, D, v.cv.coef + (size_t)cc * 4 * kCurveMax, v.cv.deg, x, y,
                                z1, z2))
            continue;
        } else {
          const double d0 = x - Ax, d1 = y - Ay;
          z1 = (d0 * (Cy - Ay) - d1 * (Cx - Ax)) / D;
          z2 = ((Bx - Ax) * d1 - (By - Ay) * d0) / D;
        }
        if (fmin(fmin(1.0 - z1 - z2, z1), z2) >= -kTau) {
          hit = t;
          r1 = z1;
          r2 = z2;
        }
      }
    }
    tri_out[i] = hit;
    ref_out[2 * i] = r1;
    ref_out[2 * i + 1] = r2;
  }
}

template <int P>
__global__ void k_ieval(const double* __restrict__ vinv, const double* __restrict__ u, int64_t n_tri, int64_t R,
                        int64_t n, const int32_t* __restrict__ tri, const double* __restrict__ ref,
                        double* __restrict__ out) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n * R; g += stride) {
    const int64_t i = g / R, r = g - i * R;
    const int32_t t = tri[i];
    if (t < 0 || t >= n_tri) {
      out[g] = __builtin_nan("");
      continue;
    }
    double val[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) val[k] = u[((size_t)t * NP + k) * R + r];
    double s = 0.0;
    koornwinder_emit<P>(ref[2 * i], ref[2 * i + 1], [&](int k, double kv) {
      double c = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) c = fma(vinv[k * NP + j], val[j], c);
      s = fma(c, kv, s);
    });
    out[g] = s;
  }
}

}  // namespace
}  // namespace vp

using vp::ifail;
using vp::ihip;

vp_status vp_interp_create(vp_ctx* ctx, const vp_mesh* mesh, int p, vp_interp** out) {
  if (!ctx || !mesh || !out) return ifail(VP_EINVAL, "vp_interp_create: NULL argument");
  if (mesh->ctx != ctx) return ifail(VP_EINVAL, "vp_interp_create: mesh belongs to another context");
  if (p < 1 || p > vp::kMaxP) return ifail(VP_EINVAL, "vp_interp_create: p = %d outside [1, %d]", p, vp::kMaxP);
  const int64_t T = mesh->n_tri;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return ihip(e, "hipSetDevice");
  hipStream_t st = ctx->stream;
  // boxes of the triangles (and of the curved elements) on the host
  std::vector<double> g(7 * std::max<int64_t>(T, 1));
  std::vector<double> cbox(4 * std::max<int64_t>(mesh->n_curved, 1));
  std::vector<int32_t> of(mesh->curve_of ? T : 0);
  if (T > 0 && (e = hipMemcpyAsync(g.data(), mesh->ax, sizeof(double) * 7 * T, hipMemcpyDeviceToHost, st)) !=
                   hipSuccess)
    return ihip(e, "vp_interp_create");
  if (mesh->n_curved &&
      ((e = hipMemcpyAsync(cbox.data(), mesh->curve_box, sizeof(double) * 4 * mesh->n_curved,
                           hipMemcpyDeviceToHost, st)) != hipSuccess ||
       (e = hipMemcpyAsync(of.data(), mesh->curve_of, sizeof(int32_t) * T, hipMemcpyDeviceToHost, st)) !=
           hipSuccess))
    return ihip(e, "vp_interp_create");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return ihip(e, "vp_interp_create");
  const double *ax = g.data(), *ay = ax + T, *bx = ax + 2 * T, *by = ax + 3 * T, *cx = ax + 4 * T, *cy = ax + 5 * T;
  std::vector<double> box(4 * std::max<int64_t>(T, 1));
  double X0 = 1e300, Y0 = 1e300, X1 = -1e300, Y1 = -1e300, sum_ext = 0.0;
  for (int64_t t = 0; t < T; ++t) {
    double x0 = std::min({ax[t], bx[t], cx[t]}), x1 = std::max({ax[t], bx[t], cx[t]});
    double y0 = std::min({ay[t], by[t], cy[t]}), y1 = std::max({ay[t], by[t], cy[t]});
    if (!of.empty() && of[t] >= 0) {
      const double* b = cbox.data() + 4 * of[t];
      x0 = std::min(x0, b[0]);
      y0 = std::min(y0, b[1]);
      x1 = std::max(x1, b[2]);
      y1 = std::max(y1, b[3]);
    }
    const double pad = 1e-9 * std::max(x1 - x0, y1 - y0);
    box[4 * t] = x0 - pad;
    box[4 * t + 1] = y0 - pad;
    box[4 * t + 2] = x1 + pad;
    box[4 * t + 3] = y1 + pad;
    X0 = std::min(X0, box[4 * t]);
    Y0 = std::min(Y0, box[4 * t + 1]);
    X1 = std::max(X1, box[4 * t + 2]);
    Y1 = std::max(Y1, box[4 * t + 3]);
    sum_ext += std::max(x1 - x0, y1 - y0);
  }
  vp_interp* it = new vp_interp;
  it->ctx = ctx;
  it->mesh = const_cast<vp_mesh*>(mesh);
  it->p = p;
  it->n_p = vp::n_basis(p);
  // grid: cells about the mean box size, at most 4096 per side
  const double h = T > 0 ? std::max(sum_ext / T, 1e-300) : 1.0;
  it->x0 = T > 0 ? X0 : 0.0;
  it->y0 = T > 0 ? Y0 : 0.0;
  it->nx = T > 0 ? (int)std::min(4096.0, std::max(1.0, std::ceil((X1 - X0) / h))) : 1;
  it->ny = T > 0 ? (int)std::min(4096.0, std::max(1.0, std::ceil((Y1 - Y0) / h))) : 1;
  const double hx = T > 0 ? std::max((X1 - X0) / it->nx, (Y1 - Y0) / it->ny) : 1.0;
  it->inv_h = 1.0 / std::max(hx, 1e-300);
  const int64_t nc = (int64_t)it->nx * it->ny;
  std::vector<int64_t> ptr(nc + 1, 0);
  auto cells = [&](int64_t t, int& i0, int& i1, int& j0, int& j1) {
    i0 = std::max(0, std::min(it->nx - 1, (int)std::floor((box[4 * t] - it->x0) * it->inv_h)));
    i1 = std::max(0, std::min(it->nx - 1, (int)std::floor((box[4 * t + 2] - it->x0) * it->inv_h)));
    j0 = std::max(0, std::min(it->ny - 1, (int)std::floor((box[4 * t + 1] - it->y0) * it->inv_h)));
    j1 = std::max(0, std::min(it->ny - 1, (int)std::floor((box[4 * t + 3] - it->y0) * it->inv_h)));
  };
  for (int64_t t = 0; t < T; ++t) {
    int i0, i1, j0, j1;
    cells(t, i0, i1, j0, j1);
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) ++ptr[(int64_t)j * it->nx + i + 1];
  }
  for (int64_t c = 0; c < nc; ++c) ptr[c + 1] += ptr[c];
  std::vector<int32_t> ctri(std::max<int64_t>(ptr[nc], 1));
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t t = 0; t < T; ++t) {  // ascending triangle index within every cell
    int i0, i1, j0, j1;
    cells(t, i0, i1, j0, j1);
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) ctri[fill[(int64_t)j * it->nx + i]++] = (int32_t)t;
  }
  // V^{-1} on the device
  vp::Rule2D nodes = vp::interp_nodes(p);
  const int NP = it->n_p;
  std::vector<double> nxy(2 * NP);
  for (int i = 0; i < NP; ++i) {
    nxy[i] = nodes.x[i];
    nxy[NP + i] = nodes.y[i];
  }
  double* scratch = nullptr;
  int* d_bad = nullptr;
  int bad = 0;
  auto release = [&]() {
    if (scratch) (void)hipFree(scratch);
    if (d_bad) (void)hipFree(d_bad);
  };
  auto drop = [&](vp_interp* x) {
    if (x->vinv) (void)hipFree(x->vinv);
    if (x->cell_ptr) (void)hipFree(x->cell_ptr);
    if (x->cell_tri) (void)hipFree(x->cell_tri);
    delete x;
  };
  it->bytes = sizeof(double) * NP * NP + sizeof(int64_t) * (nc + 1) + sizeof(int32_t) * ctri.size();
  if (!vp::ctx_fits(ctx, it->bytes)) {
    drop(it);
    return ifail(VP_ENOMEM, "vp_interp_create: %zu bytes exceed the HBM budget", it->bytes);
  }
  if ((e = hipMalloc((void**)&it->vinv, sizeof(double) * NP * NP)) != hipSuccess ||
      (e = hipMalloc((void**)&it->cell_ptr, sizeof(int64_t) * (nc + 1))) != hipSuccess ||
      (e = hipMalloc((void**)&it->cell_tri, sizeof(int32_t) * ctri.size())) != hipSuccess ||
      (e = hipMalloc((void**)&scratch, sizeof(double) * (2 * NP + 2 * NP * NP))) != hipSuccess ||
      (e = hipMalloc((void**)&d_bad, sizeof(int))) != hipSuccess ||
      (e = hipMemsetAsync(d_bad, 0, sizeof(int), st)) != hipSuccess ||
      (e = hipMemcpyAsync(scratch, nxy.data(), sizeof(double) * 2 * NP, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(it->cell_ptr, ptr.data(), sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(it->cell_tri, ctri.data(), sizeof(int32_t) * ctri.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = vp::launch_vinv(p, scratch, scratch + NP, scratch + 2 * NP, it->vinv, d_bad, st)) != hipSuccess ||
      (e = hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    release();
    drop(it);
    return ihip(e, "vp_interp_create");
  }
  release();
  if (bad) {
    drop(it);
    return ifail(VP_EINTERNAL, "vp_interp_create: singular Vandermonde matrix");
  }
  ctx->in_use += it->bytes;
  it->mesh->live_plans++;
  *out = it;
  return VP_OK;
}

vp_status vp_interp_destroy(vp_interp* it) {
  if (!it) return VP_OK;
  (void)hipSetDevice(it->ctx->device);
  (void)hipStreamSynchronize(it->ctx->stream);
  (void)hipFree(it->vinv);
  (void)hipFree(it->cell_ptr);
  (void)hipFree(it->cell_tri);
  it->ctx->in_use -= it->bytes;
  it->mesh->live_plans--;
  delete it;
  return VP_OK;
}

vp_status vp_interp_locate(vp_interp* it, int64_t n, const double* pts_xy, int32_t* tri_out, double* ref_out) {
  if (!it || (n > 0 && (!pts_xy || !tri_out || !ref_out))) return ifail(VP_EINVAL, "vp_interp_locate: NULL argument");
  if (n < 0) return ifail(VP_EINVAL, "vp_interp_locate: n < 0");
  if (n == 0) return VP_OK;
  hipError_t e = hipSetDevice(it->ctx->device);
  if (e != hipSuccess) return ihip(e, "hipSetDevice");
  hipStream_t st = it->ctx->stream;
  const vp_mesh* m = it->mesh;
  double *d_pts = nullptr, *d_ref = nullptr;
  int32_t* d_tri = nullptr;
  auto release = [&]() {
    if (d_pts) (void)hipFree(d_pts);
    if (d_ref) (void)hipFree(d_ref);
    if (d_tri) (void)hipFree(d_tri);
  };
  vp::LocView v{m->ax, m->ay, m->bx, m->by, m->cx, m->cy, m->det, m->curves(), it->x0, it->y0, it->inv_h, it->nx,
                it->ny, it->cell_ptr, it->cell_tri};
  if ((e = hipMalloc((void**)&d_pts, sizeof(double) * 2 * n)) != hipSuccess ||
      (e = hipMalloc((void**)&d_ref, sizeof(double) * 2 * n)) != hipSuccess ||
      (e = hipMalloc((void**)&d_tri, sizeof(int32_t) * n)) != hipSuccess ||
      (e = hipMemcpyAsync(d_pts, pts_xy, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st)) != hipSuccess) {
    release();
    return ihip(e, "vp_interp_locate");
  }
  vp::k_locate<<<vp::grid_for(n), vp::kIBlock, 0, st>>>(v, n, d_pts, d_tri, d_ref);
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipMemcpyAsync(tri_out, d_tri, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(ref_out, d_ref, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    release();
    return ihip(e, "vp_interp_locate");
  }
  release();
  return VP_OK;
}

vp_status vp_interp_eval(vp_interp* it, int64_t n_rhs, const double* u_nodes, int64_t n, const int32_t* tri,
                         const double* ref_xy, double* out, uint32_t flags) {
  if (!it || (n > 0 && (!u_nodes || !tri || !ref_xy || !out))) return ifail(VP_EINVAL, "vp_interp_eval: NULL argument");
  if (n < 0 || n_rhs < 1) return ifail(VP_EINVAL, "vp_interp_eval: n < 0 or n_rhs < 1");
  if (flags & ~(uint32_t)VP_DEVICE_PTRS) return ifail(VP_EINVAL, "vp_interp_eval: unknown flags");
  if (n == 0) return VP_OK;
  hipError_t e = hipSetDevice(it->ctx->device);
  if (e != hipSuccess) return ihip(e, "hipSetDevice");
  hipStream_t st = it->ctx->stream;
  const bool dev = flags & VP_DEVICE_PTRS;
  const int64_t T = it->mesh->n_tri, NP = it->n_p;
  const size_t nu = (size_t)T * NP * n_rhs;
  double *d_u = nullptr, *d_ref = nullptr, *d_out = nullptr;
  int32_t* d_tri = nullptr;
  auto release = [&]() {
    if (!dev) {
      if (d_u) (void)hipFree(d_u);
      if (d_ref) (void)hipFree(d_ref);
      if (d_out) (void)hipFree(d_out);
      if (d_tri) (void)hipFree(d_tri);
    }
  };
  if (dev) {
    d_u = const_cast<double*>(u_nodes);
    d_ref = const_cast<double*>(ref_xy);
    d_out = out;
    d_tri = const_cast<int32_t*>(tri);
  } else if ((e = hipMalloc((void**)&d_u, sizeof(double) * std::max<size_t>(nu, 1))) != hipSuccess ||
             (e = hipMalloc((void**)&d_ref, sizeof(double) * 2 * n)) != hipSuccess ||
             (e = hipMalloc((void**)&d_out, sizeof(double) * n * n_rhs)) != hipSuccess ||
             (e = hipMalloc((void**)&d_tri, sizeof(int32_t) * n)) != hipSuccess ||
             (nu && (e = hipMemcpyAsync(d_u, u_nodes, sizeof(double) * nu, hipMemcpyHostToDevice, st)) !=
                        hipSuccess) ||
             (e = hipMemcpyAsync(d_ref, ref_xy, sizeof(double) * 2 * n, hipMemcpyHostToDevice, st)) != hipSuccess ||
             (e = hipMemcpyAsync(d_tri, tri, sizeof(int32_t) * n, hipMemcpyHostToDevice, st)) != hipSuccess) {
    release();
    return ihip(e, "vp_interp_eval");
  }
  switch (it->p) {
#define VP_IEVAL(PV)                                                                                        \
  case PV:                                                                                                  \
    vp::k_ieval<PV><<<vp::grid_for(n * n_rhs), vp::kIBlock, 0, st>>>(it->vinv, d_u, T, n_rhs, n, d_tri,    \
                                                                     d_ref, d_out);                       \
    break
    VP_IEVAL(1);
    VP_IEVAL(2);
    VP_IEVAL(3);
    VP_IEVAL(4);
    VP_IEVAL(5);
    VP_IEVAL(6);
    VP_IEVAL(7);
    VP_IEVAL(8);
    VP_IEVAL(9);
    VP_IEVAL(10);
#undef VP_IEVAL
    default:
      release();
      return ifail(VP_EINTERNAL, "vp_interp_eval: order");
  }
  if ((e = hipGetLastError()) != hipSuccess ||
      (!dev && (e = hipMemcpyAsync(out, d_out, sizeof(double) * n * n_rhs, hipMemcpyDeviceToHost, st)) !=
                   hipSuccess) ||
      (!dev && (e = hipStreamSynchronize(st)) != hipSuccess)) {
    release();
    return ihip(e, "vp_interp_eval");
  }
  release();
  return VP_OK;
}
