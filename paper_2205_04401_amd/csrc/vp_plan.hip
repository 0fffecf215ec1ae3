// Plan-time kernels: mesh geometry, basis tables, far sources and the
// near-field pair list (Def. of far/near field, Sec. 3.2; Bernstein-ellipse
// union, Sec. 4.1, eqs. rho0 and threeE; nearby-element query, App. A.5,
// replaced by a uniform grid of cells over the targets).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>

#include "vp_internal.h"

namespace vp {
namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// mesh geometry: orientation (swap local vertices 1 and 2 if clockwise),
// det = |J| = 2 area, rejection of bad input
// ---------------------------------------------------------------------------
__global__ void k_mesh_geom(const double* __restrict__ vert, int64_t n_vert, const int32_t* __restrict__ tri,
                            int64_t n_tri, double* ax, double* ay, double* bx, double* by, double* cx,
                            double* cy, double* det, double4* geo, int* bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  int32_t i0 = tri[3 * t], i1 = tri[3 * t + 1], i2 = tri[3 * t + 2];
  if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= n_vert || i1 >= n_vert || i2 >= n_vert) {
    atomicMax(bad, 1);
    return;
  }
  double x0 = vert[2 * i0], y0 = vert[2 * i0 + 1];
  double x1 = vert[2 * i1], y1 = vert[2 * i1 + 1];
  double x2 = vert[2 * i2], y2 = vert[2 * i2 + 1];
  if (!isfinite(x0) || !isfinite(y0) || !isfinite(x1) || !isfinite(y1) || !isfinite(x2) || !isfinite(y2)) {
    atomicMax(bad, 2);
    return;
  }
  double d = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0);
  if (d < 0.0) {
    double tx = x1, ty = y1;
    x1 = x2;
    y1 = y2;
    x2 = tx;
    y2 = ty;
    d = -d;
  }
  double w = fmax(fmax(x0, x1), x2) - fmin(fmin(x0, x1), x2);
  double h = fmax(fmax(y0, y1), y2) - fmin(fmin(y0, y1), y2);
  double ext = fmax(w, h);
  if (!(d > 1e-14 * ext * ext)) {
    atomicMax(bad, 3);
  }
  ax[t] = x0;
  ay[t] = y0;
  bx[t] = x1;
  by[t] = y1;
  cx[t] = x2;
  cy[t] = y2;
  det[t] = d;
  geo[2 * t] = make_double4(x0, y0, x1, y1);
  geo[2 * t + 1] = make_double4(x2, y2, d, 0.0);
}

__global__ void k_split_xy(const double* __restrict__ xy, int64_t n, double* x, double* y, int* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = xy[2 * i], b = xy[2 * i + 1];
  if (!isfinite(a) || !isfinite(b)) atomicMax(bad, 2);
  x[i] = a;
  y[i] = b;
}

// ---------------------------------------------------------------------------
// basis tables: V (Koornwinder at the interpolation nodes) inverted by
// Gauss-Jordan with partial pivoting (one workgroup), and E = Koornwinder at
// the far nodes.  Sec. 2.2: V^{-1} maps node values to coefficients.
// ---------------------------------------------------------------------------
template <int P>
__global__ void k_vandermonde_inverse(const double* __restrict__ nx, const double* __restrict__ ny,
                                      double* aug /* [NP][2 NP] */, double* vinv, int* bad) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  constexpr int W2 = 2 * NP;
  const int tid = threadIdx.x;
  for (int i = tid; i < NP; i += blockDim.x) {
    double* row = aug + (size_t)i * W2;
    koornwinder_emit<P>(nx[i], ny[i], [&](int k, double v) { row[k] = v; });
    for (int j = 0; j < NP; ++j) row[NP + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  __shared__ int piv;
  for (int c = 0; c < NP; ++c) {
    if (tid == 0) {
      int best = c;
      double bv = fabs(aug[(size_t)c * W2 + c]);
      for (int r = c + 1; r < NP; ++r) {
        double v = fabs(aug[(size_t)r * W2 + c]);
        if (v > bv) {
          bv = v;
          best = r;
        }
      }
      piv = best;
      if (!(bv > 0.0)) atomicMax(bad, 4);
    }
    __syncthreads();
    const int pr = piv;
    if (pr != c) {
      for (int j = tid; j < W2; j += blockDim.x) {
        double a = aug[(size_t)c * W2 + j];
        aug[(size_t)c * W2 + j] = aug[(size_t)pr * W2 + j];
        aug[(size_t)pr * W2 + j] = a;
      }
    }
    __syncthreads();
    const double inv = 1.0 / aug[(size_t)c * W2 + c];
    __syncthreads();
    for (int j = tid; j < W2; j += blockDim.x) aug[(size_t)c * W2 + j] *= inv;
    __syncthreads();
    for (int idx = tid; idx < NP * W2; idx += blockDim.x) {
      int r = idx / W2, j = idx % W2;
      if (r == c || j == c) continue;
      aug[idx] -= aug[(size_t)r * W2 + c] * aug[(size_t)c * W2 + j];
    }
    __syncthreads();
    for (int r = tid; r < NP; r += blockDim.x)
      if (r != c) aug[(size_t)r * W2 + c] = 0.0;
    __syncthreads();
  }
  // aug = [I | V^{-1}]; V^{-1}[k][i] maps value i to coefficient k
  for (int idx = tid; idx < NP * NP; idx += blockDim.x) {
    int k = idx / NP, i = idx % NP;
    vinv[idx] = aug[(size_t)k * W2 + NP + i];
  }
}

template <int P>
__global__ void k_basis_at(const double* __restrict__ x, const double* __restrict__ y, int n, double* out) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double* row = out + (size_t)j * NP;
  koornwinder_emit<P>(x[j], y[j], [&](int k, double v) { row[k] = v; });
}

// far sources: node j of triangle t at A + xi_1 (B-A) + xi_2 (C-A); the
// padding entries past n_tri * nf sit at the origin (their charge is 0)
// Far sources: position rho(xi_j) and weight w_j |J(xi_j)| of every far node
// of every triangle (Thm. smooth_int_jac; affine triangles have |J| = det),
// zero in the padding.
__global__ void k_sources(const double* __restrict__ ax, const double* __restrict__ ay,
                          const double* __restrict__ bx, const double* __restrict__ by,
                          const double* __restrict__ cx, const double* __restrict__ cy,
                          const double* __restrict__ det, CurveView cv, const double* __restrict__ fx,
                          const double* __restrict__ fy, const double* __restrict__ fw, int nf, int64_t n_tri,
                          int64_t n_pad, double2* sxy, double* swj) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += stride) {
    if (i >= n_tri * nf) {
      sxy[i] = make_double2(0.0, 0.0);
      swj[i] = 0.0;
      continue;
    }
    const int64_t t = i / nf;
    const int j = (int)(i - t * nf);
    const double a0 = ax[t], a1 = ay[t];
    const int c = cv.of ? cv.of[t] : -1;
    if (c >= 0) {
      double px, py;
      const double J = vp_blend_jac(a0, a1, bx[t], by[t], cx[t], cy[t], cv.coef + (size_t)c * 4 * kCurveMax, cv.deg,
                                    fx[j], fy[j], px, py);
      sxy[i] = make_double2(px, py);
      swj[i] = fw[j] * J;
    } else {
      sxy[i] = make_double2(a0 + fx[j] * (bx[t] - a0) + fy[j] * (cx[t] - a0),
                            a1 + fx[j] * (by[t] - a1) + fy[j] * (cy[t] - a1));
      swj[i] = fw[j] * det[t];
    }
  }
}

// |J| scale of the ellipse tests: det, or for a curved triangle the largest
// |J| at its far nodes (its curved side treated as straight, Sec. 4.1).
__global__ void k_deff(const double* __restrict__ det, int64_t n_tri, CurveView cv, const double* __restrict__ swj,
                       const double* __restrict__ fw, int nf, double* __restrict__ deff) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tri; t += stride) {
    if (cv.of && cv.of[t] >= 0) {
      double mx = 0.0;
      for (int j = 0; j < nf; ++j) mx = fmax(mx, swj[t * nf + j] / fw[j]);
      deff[t] = mx;
    } else {
      deff[t] = det[t];
    }
  }
}

// Physical positions of reference points on every triangle: out[t][i].
__global__ void k_map_points(const double* __restrict__ ax, const double* __restrict__ ay,
                             const double* __restrict__ bx, const double* __restrict__ by,
                             const double* __restrict__ cx, const double* __restrict__ cy, CurveView cv,
                             int64_t n_tri, int n_ref, const double* __restrict__ ref, double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_tri * n_ref; g += stride) {
    const int64_t t = g / n_ref;
    const int i = (int)(g - t * n_ref);
    const double xi = ref[2 * i], eta = ref[2 * i + 1];
    const int c = cv.of ? cv.of[t] : -1;
    double px, py;
    if (c >= 0) {
      vp_blend(ax[t], ay[t], bx[t], by[t], cx[t], cy[t], cv.coef + (size_t)c * 4 * kCurveMax, cv.deg, xi, eta, px,
               py);
    } else {
      px = ax[t] + xi * (bx[t] - ax[t]) + eta * (cx[t] - ax[t]);
      py = ay[t] + xi * (by[t] - ay[t]) + eta * (cy[t] - ay[t]);
    }
    out[2 * g] = px;
    out[2 * g + 1] = py;
  }
}

// ---------------------------------------------------------------------------
// near-field geometry per triangle: focal-sum thresholds of the three edge
// ellipses (negative when rho <= 1, i.e. empty) and an axis-aligned box that
// contains the triangle (with the self-test tolerance) and its ellipses.
// ---------------------------------------------------------------------------
__global__ void k_tri_ellipses(const double* __restrict__ ax, const double* __restrict__ ay,
                               const double* __restrict__ bx, const double* __restrict__ by,
                               const double* __restrict__ cx, const double* __restrict__ cy,
                               const double* __restrict__ det, int64_t n_tri, double w0, double w1, double w2,
                               double eps_cn, double inv_order, int ball, double kappa, CurveView cv,
                               double* thr /* [3][n_tri] */, double* box /* [n_tri][4] */) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  const double px[3] = {ax[t], bx[t], cx[t]};
  const double py[3] = {ay[t], by[t], cy[t]};
  const double wh[3] = {w0, w1, w2};
  const double D = det[t];
  double x0 = fmin(fmin(px[0], px[1]), px[2]), x1 = fmax(fmax(px[0], px[1]), px[2]);
  double y0 = fmin(fmin(py[0], py[1]), py[2]), y1 = fmax(fmax(py[0], py[1]), py[2]);
  const double ext = fmax(x1 - x0, y1 - y0);
  // the self test accepts barycentric coordinates down to -tau: pad the box
  const double pad = 1e-9 * ext;
  x0 -= pad;
  x1 += pad;
  y0 -= pad;
  y1 += pad;
  const int cc = cv.of ? cv.of[t] : -1;
  if (cc >= 0) {  // a curved element: its own box (its side may bulge out of the chord triangle)
    x0 = fmin(x0, cv.box[4 * cc]);
    y0 = fmin(y0, cv.box[4 * cc + 1]);
    x1 = fmax(x1, cv.box[4 * cc + 2]);
    y1 = fmax(y1, cv.box[4 * cc + 3]);
  }
  if (ball) {
    // naive near field: the ball of radius kappa R about the centroid (the
    // test itself is in_ball3; this is its bounding box)
    const double gx = (px[0] + px[1] + px[2]) / 3.0, gy = (py[0] + py[1] + py[2]) / 3.0;
    double R = 0.0;
    for (int e = 0; e < 3; ++e) R = fmax(R, sqrt((px[e] - gx) * (px[e] - gx) + (py[e] - gy) * (py[e] - gy)));
    const double rad = kappa * R * (1.0 + 1e-9) + pad;
    x0 = fmin(x0, gx - rad);
    x1 = fmax(x1, gx + rad);
    y0 = fmin(y0, gy - rad);
    y1 = fmax(y1, gy + rad);
    thr[t] = kappa * R;
    thr[n_tri + t] = -1.0;
    thr[2 * n_tri + t] = -1.0;
    box[4 * t] = x0;
    box[4 * t + 1] = y0;
    box[4 * t + 2] = x1;
    box[4 * t + 3] = y1;
    return;
  }
  for (int e = 0; e < 3; ++e) {
    const double Px = px[e], Py = py[e], Qx = px[(e + 1) % 3], Qy = py[(e + 1) % 3];
    const double rho = pow(wh[e] * D / eps_cn, inv_order);
    const double ell = sqrt((Qx - Px) * (Qx - Px) + (Qy - Py) * (Qy - Py));
    double s = -1.0;
    if (rho > 1.0) {
      s = 0.5 * ell * (rho + 1.0 / rho);
      const double a = 0.5 * s, c = 0.5 * ell;
      const double b = sqrt(fmax(a * a - c * c, 0.0));
      const double ux = (Qx - Px) / ell, uy = (Qy - Py) / ell;
      const double hx = sqrt(a * a * ux * ux + b * b * uy * uy) * (1.0 + 1e-9) + pad;
      const double hy = sqrt(a * a * uy * uy + b * b * ux * ux) * (1.0 + 1e-9) + pad;
      const double mx = 0.5 * (Px + Qx), my = 0.5 * (Py + Qy);
      x0 = fmin(x0, mx - hx);
      x1 = fmax(x1, mx + hx);
      y0 = fmin(y0, my - hy);
      y1 = fmax(y1, my + hy);
    }
    thr[e * n_tri + t] = s;
  }
  box[4 * t] = x0;
  box[4 * t + 1] = y0;
  box[4 * t + 2] = x1;
  box[4 * t + 3] = y1;
}

// bounding box of the targets and mean box extent: partial reductions
__global__ void k_extent_partial(const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt,
                                 const double* __restrict__ box, int64_t n_tri, double* part /* [grid][5] */) {
  __shared__ double s[5][kBlock];
  double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300, sum = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_tgt; i += stride) {
    mnx = fmin(mnx, xt[i]);
    mxx = fmax(mxx, xt[i]);
    mny = fmin(mny, yt[i]);
    mxy = fmax(mxy, yt[i]);
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_tri; i += stride) {
    sum += fmax(box[4 * i + 2] - box[4 * i], box[4 * i + 3] - box[4 * i + 1]);
  }
  const int tid = threadIdx.x;
  s[0][tid] = mnx;
  s[1][tid] = mny;
  s[2][tid] = mxx;
  s[3][tid] = mxy;
  s[4][tid] = sum;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (tid < o) {
      s[0][tid] = fmin(s[0][tid], s[0][tid + o]);
      s[1][tid] = fmin(s[1][tid], s[1][tid + o]);
      s[2][tid] = fmax(s[2][tid], s[2][tid + o]);
      s[3][tid] = fmax(s[3][tid], s[3][tid + o]);
      s[4][tid] = s[4][tid] + s[4][tid + o];
    }
    __syncthreads();
  }
  if (tid < 5) part[blockIdx.x * 5 + tid] = s[tid][0];
}

struct Grid {
  double x0, y0, inv_h;
  int nx, ny;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ bool box_cells(const Grid g, double bx0, double by0, double bx1, double by1, int& i0,
                                          int& i1, int& j0, int& j1) {
  double fx0 = (bx0 - g.x0) * g.inv_h, fx1 = (bx1 - g.x0) * g.inv_h;
  double fy0 = (by0 - g.y0) * g.inv_h, fy1 = (by1 - g.y0) * g.inv_h;
  if (fx1 < 0.0 || fy1 < 0.0 || fx0 >= (double)g.nx || fy0 >= (double)g.ny) return false;
  i0 = clampi((int)floor(fx0), 0, g.nx - 1);
  i1 = clampi((int)floor(fx1), 0, g.nx - 1);
  j0 = clampi((int)floor(fy0), 0, g.ny - 1);
  j1 = clampi((int)floor(fy1), 0, g.ny - 1);
  return true;
}

__global__ void k_cell_count(const double* __restrict__ box, int64_t n_tri, Grid g, int32_t* cnt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  int i0, i1, j0, j1;
  if (!box_cells(g, box[4 * t], box[4 * t + 1], box[4 * t + 2], box[4 * t + 3], i0, i1, j0, j1)) return;
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) atomicAdd(&cnt[(int64_t)j * g.nx + i], 1);
}

// cells covered by each triangle's box (the number of entries it emits)
__global__ void k_cell_tcount(const double* __restrict__ box, int64_t n_tri, Grid g, int32_t* tcnt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  int i0, i1, j0, j1;
  tcnt[t] = box_cells(g, box[4 * t], box[4 * t + 1], box[4 * t + 2], box[4 * t + 3], i0, i1, j0, j1)
                ? (i1 - i0 + 1) * (j1 - j0 + 1)
                : 0;
}

// (cell, triangle) entries in triangle order at the triangle's offset; a
// stable sort by cell then gives every cell's list in ascending triangle
// order, independent of the launch
__global__ void k_cell_emit(const double* __restrict__ box, int64_t n_tri, Grid g, const int64_t* __restrict__ toff,
                            int32_t* __restrict__ key, int32_t* __restrict__ val) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  int i0, i1, j0, j1;
  if (!box_cells(g, box[4 * t], box[4 * t + 1], box[4 * t + 2], box[4 * t + 3], i0, i1, j0, j1)) return;
  int64_t o = toff[t];
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      key[o] = j * g.nx + i;
      val[o] = (int32_t)t;
      ++o;
    }
}

struct TriView {
  const double *ax, *ay, *bx, *by, *cx, *cy, *det, *thr;
  int64_t n_tri;
  int ball;      // naive ball model (in_ball3)
  double kappa;  // its factor
  CurveView cv;  // curved triangles
  // near-field boxes [n_tri][4] (k_tri_ellipses); box_reject: a target
  // outside its triangle's box is far without the tests (the boxes hold the
  // self region for tau up to 1e-10)
  const double* box;
  int box_reject;
  const double4* geo;  // the geometry packed per triangle
};

// 0 = self, 1 = near, 2 = far
// kCurved: the mesh has curved triangles (the straight-only instances carry
// none of their code)
template <bool kCurved>
__device__ __forceinline__ int classify(const TriView& tv, int32_t t, double x, double y, double tau) {
  if (tv.box_reject) {
    const double4 b = *(const double4*)(tv.box + 4 * (int64_t)t);
    if (x < b.x || y < b.y || x > b.z || y > b.w) return 2;
  }
  const TriGeo tg = tri_geo(tv.geo, t);
  const double Ax = tg.ax, Ay = tg.ay, Bx = tg.bx, By = tg.by, Cx = tg.cx, Cy = tg.cy;
  const double D = tg.det;
  const double d0 = x - Ax, d1 = y - Ay;
  const double e1x = Bx - Ax, e1y = By - Ay, e2x = Cx - Ax, e2y = Cy - Ay;
  const double xi1 = (d0 * e2y - d1 * e2x) / D;
  const double xi2 = (e1x * d1 - e1y * d0) / D;
  const double lmin = fmin(fmin(1.0 - xi1 - xi2, xi1), xi2);
  const int cc = (kCurved && tv.cv.of) ? tv.cv.of[t] : -1;
  if (kCurved && cc >= 0) {
    // curved element: self if rho^{-1}(x) is in the closed simplex; a point
    // of the chord triangle outside the element is near
    const double* bx4 = tv.cv.box + 4 * cc;
    if (x >= bx4[0] && x <= bx4[2] && y >= bx4[1] && y <= bx4[3]) {
      double z1, z2;
      if (vp_blend_inverse(Ax, Ay, Bx, By, Cx, Cy, D, tv.cv.coef + (size_t)cc * 4 * kCurveMax, tv.cv.deg, x, y, z1,
                           z2) &&
          fmin(fmin(1.0 - z1 - z2, z1), z2) >= -tau)
        return 0;
    }
    if (lmin >= -tau) return 1;
  } else if (lmin >= -tau) {
    return 0;
  }
  if (tv.ball) {
    const double px[3] = {Ax, Bx, Cx}, py[3] = {Ay, By, Cy};
    return in_ball3(x, y, px, py, tv.kappa) ? 1 : 2;
  }
  // the ellipse of edge e (foci at its ends): the focal sum from the
  // target's distances to the three vertices
  const double dA = sqrt((x - Ax) * (x - Ax) + (y - Ay) * (y - Ay));
  const double dB = sqrt((x - Bx) * (x - Bx) + (y - By) * (y - By));
  const double dC = sqrt((x - Cx) * (x - Cx) + (y - Cy) * (y - Cy));
  const double s0 = tv.thr[t], s1 = tv.thr[tv.n_tri + t], s2 = tv.thr[2 * tv.n_tri + t];
  if ((s0 > 0.0 && dA + dB < s0) || (s1 > 0.0 && dB + dC < s1) || (s2 > 0.0 && dC + dA < s2)) return 1;
  return 2;
}

__device__ __forceinline__ int64_t cell_of(const Grid g, double x, double y) {
  int i = clampi((int)floor((x - g.x0) * g.inv_h), 0, g.nx - 1);
  int j = clampi((int)floor((y - g.y0) * g.inv_h), 0, g.ny - 1);
  return (int64_t)j * g.nx + i;
}

// 32-bit words of decision bits per target: one bit per triangle of its cell
__global__ void k_pair_words(const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, Grid g,
                             const int64_t* __restrict__ cptr, int32_t* __restrict__ words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_tgt) return;
  const int64_t c = cell_of(g, xt[i], yt[i]);
  words[i] = (int32_t)((cptr[c + 1] - cptr[c] + 31) / 32);
}

// Count pass, one thread per target: classifies every triangle of the
// target's cell once, keeps the decisions as bits (mk[w].x: self or near,
// mk[w].y: self; bit j of word w is the cell's triangle 32 w + j) at the
// target's word offset woff[i], and counts its pairs.
template <bool kCurved>
__global__ void k_pair_count(const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, Grid g,
                             const int64_t* __restrict__ cptr, const int32_t* __restrict__ ctri, TriView tv,
                             double tau, const int64_t* __restrict__ woff, uint2* __restrict__ mk, int32_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_tgt) return;
  const double x = xt[i], y = yt[i];
  const int64_t c = cell_of(g, x, y);
  const int64_t k0 = cptr[c], k1 = cptr[c + 1];
  uint2* out = mk + woff[i];
  int n = 0;
  for (int64_t kb = k0; kb < k1; kb += 32) {
    uint32_t pair = 0, self = 0;
    const int m = (int)min<int64_t>(32, k1 - kb);
    for (int j = 0; j < m; ++j) {
      const int kind = classify<kCurved>(tv, ctri[kb + j], x, y, tau);
      pair |= (kind < 2 ? 1u : 0u) << j;
      self |= (kind == 0 ? 1u : 0u) << j;
    }
    out[(kb - k0) >> 5] = make_uint2(pair, self);
    n += __popc(pair);
  }
  cnt[i] = n;
}

// Fill pass, 16 lanes per target (four targets per wavefront, so that the
// loads that locate a target's cell and bits overlap for four targets):
// the lanes take 16 of the cell's triangles at a time with their decision
// bits from the count pass and write the pairs among them at consecutive
// places (ballot and prefix count within the 16), so that the stores of a
// target are contiguous; the cell lists are ascending, so are the
// target's pairs.  A target whose pairs do not fill its range exactly sets
// *bad (it writes nothing beyond its range).
constexpr int kFillWaves = 4;
constexpr int kFillLanes = 16;  // lanes per target
constexpr int kFillPerWave = 64 / kFillLanes;

__global__ __launch_bounds__(kFillWaves * 64) void k_pair_fill(
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, Grid g,
    const int64_t* __restrict__ cptr, const int32_t* __restrict__ ctri, const int64_t* __restrict__ woff,
    const uint2* __restrict__ mk, const int64_t* __restrict__ row_ptr, int32_t* pair_tri, int32_t* pair_tgt,
    uint8_t* pair_kind, int32_t* self_cnt, int* bad) {
  const int lane = threadIdx.x & 63, sub = lane / kFillLanes, gl = lane % kFillLanes;
  const uint64_t gmask = ((1ull << kFillLanes) - 1) << (kFillLanes * sub);  // this target's lanes
  const uint64_t lt = ((1ull << gl) - 1) << (kFillLanes * sub);            // its lanes below this one
  const int64_t per_block = (int64_t)kFillWaves * kFillPerWave;
  for (int64_t i = (int64_t)blockIdx.x * per_block + (threadIdx.x >> 6) * kFillPerWave + sub; i < n_tgt;
       i += (int64_t)gridDim.x * per_block) {
    const int64_t c = cell_of(g, xt[i], yt[i]);
    const int64_t k0 = cptr[c], k1 = cptr[c + 1];
    const uint2* bits = mk + woff[i];
    const int64_t end = row_ptr[i + 1];
    int64_t o = row_ptr[i];
    int ns = 0;
    for (int64_t kb = k0; kb < k1; kb += kFillLanes) {
      const int64_t k = kb + gl;
      const bool in = k < k1;
      const uint2 w = in ? bits[(k - k0) >> 5] : make_uint2(0u, 0u);
      const int b = (int)((k - k0) & 31);
      const bool is_pair = in && ((w.x >> b) & 1u);
      const bool is_self = in && ((w.y >> b) & 1u);
      const uint64_t m = __ballot(is_pair) & gmask;
      ns += __popcll(__ballot(is_self) & gmask);
      const int64_t pos = o + __popcll(m & lt);
      if (is_pair && pos < end) {
        pair_tri[pos] = ctri[k];
        pair_tgt[pos] = (int32_t)i;
        pair_kind[pos] = is_self ? (uint8_t)0 : (uint8_t)1;
      }
      o += __popcll(m);
    }
    if (gl == 0) {
      self_cnt[i] = ns;
      if (o != end) atomicOr(bad, 1);
    }
  }
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts into int64 offsets (out[n] = total)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    int64_t a = (tid >= o) ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  total = sh[kBlock - 1];
  int64_t incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_tiles(const int32_t* __restrict__ in, int64_t n, int64_t* out, int64_t* tile_sums) {
  __shared__ int64_t sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t loc[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    loc[k] = (i < n) ? (int64_t)in[i] : 0;
    s += loc[k];
  }
  int64_t total;
  int64_t off = block_exclusive_scan(s, sh, total);
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = off;
    off += loc[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_sums(int64_t* tile_sums, int64_t n_tiles, int64_t* grand) {
  __shared__ int64_t sh[kBlock];
  int64_t carry = 0;
  for (int64_t b = 0; b < n_tiles; b += kBlock) {
    int64_t i = b + threadIdx.x;
    int64_t v = (i < n_tiles) ? tile_sums[i] : 0;
    int64_t total;
    int64_t ex = block_exclusive_scan(v, sh, total);
    if (i < n_tiles) tile_sums[i] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ void k_scan_add(int64_t* out, int64_t n, const int64_t* __restrict__ tile_sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int64_t add = tile_sums[blockIdx.x];
  for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
    int64_t i = base + k;
    if (i < n) out[i] += add;
  }
}

// sum of n counts into *out: a grid of at most kCountSumBlocks blocks strides
// over the array and adds one partial per block (one atomic per wavefront on
// a single address serialised the launch: 0.7 ms for 3.75M counts)
constexpr int kCountSumBlocks = 1024;

__global__ __launch_bounds__(kBlock) void k_count_sum(const int32_t* __restrict__ v, int64_t n,
                                                      unsigned long long* out) {
  __shared__ int64_t part[kBlock / 64];
  int64_t s = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += v[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t b = 0;
    for (int w = 0; w < kBlock / 64; ++w) b += part[w];
    if (b) atomicAdd(out, (unsigned long long)b);
  }
}

}  // namespace

size_t exclusive_scan_tmp_bytes(int64_t n) {
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  return (size_t)(tiles + 1) * sizeof(int64_t);
}

hipError_t exclusive_scan_i32(const int32_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t st) {
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  int64_t* sums = (int64_t*)tmp;
  if (tiles > 0) {
    k_scan_tiles<<<(unsigned)tiles, kBlock, 0, st>>>(in, n, out, sums);
  }
  k_scan_sums<<<1, kBlock, 0, st>>>(sums, tiles, out + n);
  if (tiles > 0) {
    k_scan_add<<<(unsigned)tiles, kBlock, 0, st>>>(out, n, sums);
  }
  return hipGetLastError();
}

hipError_t launch_mesh_geom(const double* vert, int64_t n_vert, const int32_t* tri, int64_t n_tri, vp_mesh* m,
                            int* d_bad, hipStream_t st) {
  if (n_tri > 0)
    k_mesh_geom<<<blocks_for(n_tri), kBlock, 0, st>>>(vert, n_vert, tri, n_tri, m->ax, m->ay, m->bx, m->by, m->cx,
                                                      m->cy, m->det, m->geo, d_bad);
  return hipGetLastError();
}

hipError_t launch_split_xy(const double* xy, int64_t n, double* x, double* y, int* d_bad, hipStream_t st) {
  if (n > 0) k_split_xy<<<blocks_for(n), kBlock, 0, st>>>(xy, n, x, y, d_bad);
  return hipGetLastError();
}

// V^{-1} of order p at the given nodes (one workgroup; aug: [n_p][2 n_p]
// scratch), for other users of the interpolation matrix.
hipError_t launch_vinv(int p, const double* nx, const double* ny, double* aug, double* vinv, int* bad,
                       hipStream_t st) {
  switch (p) {
#define VP_VINV(PV) \
  case PV: k_vandermonde_inverse<PV><<<1, 256, 0, st>>>(nx, ny, aug, vinv, bad); break
    VP_VINV(1);
    VP_VINV(2);
    VP_VINV(3);
    VP_VINV(4);
    VP_VINV(5);
    VP_VINV(6);
    VP_VINV(7);
    VP_VINV(8);
    VP_VINV(9);
    VP_VINV(10);
#undef VP_VINV
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// W = E V^{-1} [nf][n_p]: the far-node values of the interpolant straight
// from the node values, f_h(xi_j) = sum_i W_ji f_i (E_jk = K_k(xi_j))
template <int P>
static __global__ void k_fold(const double* __restrict__ efar, const double* __restrict__ vinv, int nf,
                       double* __restrict__ wfar) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nf * NP) return;
  const int j = g / NP, i = g - j * NP;
  double s = 0.0;
  for (int k = 0; k < NP; ++k) s = fma(efar[j * NP + k], vinv[k * NP + i], s);
  wfar[g] = s;
}

template <int P>
static hipError_t basis_tables_p(vp_plan* pl, double* scratch, int* d_bad, hipStream_t st) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  k_vandermonde_inverse<P><<<1, 256, 0, st>>>(scratch, scratch + pl->n_p, scratch + 2 * pl->n_p, pl->vinv, d_bad);
  k_basis_at<P><<<blocks_for(pl->n_f), kBlock, 0, st>>>(pl->far_x, pl->far_y, pl->n_f, pl->efar);
  k_fold<P><<<blocks_for((int64_t)pl->n_f * NP), kBlock, 0, st>>>(pl->efar, pl->vinv, pl->n_f, pl->wfar);
  return hipGetLastError();
}

// scratch layout: [n_p] node x, [n_p] node y, [n_p][2 n_p] augmented matrix,
// then an int flag
hipError_t launch_basis_tables(vp_plan* pl, double* scratch, hipStream_t st) {
  int* d_bad = (int*)(scratch + 2 * pl->n_p + 2 * pl->n_p * pl->n_p);
  switch (pl->p) {
    case 1: return basis_tables_p<1>(pl, scratch, d_bad, st);
    case 2: return basis_tables_p<2>(pl, scratch, d_bad, st);
    case 3: return basis_tables_p<3>(pl, scratch, d_bad, st);
    case 4: return basis_tables_p<4>(pl, scratch, d_bad, st);
    case 5: return basis_tables_p<5>(pl, scratch, d_bad, st);
    case 6: return basis_tables_p<6>(pl, scratch, d_bad, st);
    case 7: return basis_tables_p<7>(pl, scratch, d_bad, st);
    case 8: return basis_tables_p<8>(pl, scratch, d_bad, st);
    case 9: return basis_tables_p<9>(pl, scratch, d_bad, st);
    case 10: return basis_tables_p<10>(pl, scratch, d_bad, st);
  }
  return hipErrorInvalidValue;
}

// Bounding circle (centre of the bounding box, half its diagonal) of every
// group of 64 consecutive sources, and each source's offset from its
// group's centre in FP32, for the mixed far sum (padding sources at the
// origin are included: a larger circle)
static __global__ void k_src_groups(const double2* __restrict__ sxy, int64_t n_grp, double* __restrict__ grp,
                                    float2* __restrict__ soff) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_grp) return;
  double x0 = sxy[64 * g].x, x1 = x0, y0 = sxy[64 * g].y, y1 = y0;
  for (int i = 1; i < 64; ++i) {
    const double2 s = sxy[64 * g + i];
    x0 = fmin(x0, s.x);
    x1 = fmax(x1, s.x);
    y0 = fmin(y0, s.y);
    y1 = fmax(y1, s.y);
  }
  const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1);
  grp[3 * g] = cx;
  grp[3 * g + 1] = cy;
  // a hair above half the diagonal, so that the circle holds every source
  grp[3 * g + 2] = 0.5 * sqrt((x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0)) * (1.0 + 1e-12);
  for (int i = 0; i < 64; ++i) {
    const double2 s = sxy[64 * g + i];
    soff[64 * g + i] = make_float2((float)(s.x - cx), (float)(s.y - cy));
  }
}

hipError_t launch_sources(vp_plan* pl, hipStream_t st) {
  const vp_mesh* m = pl->mesh;
  int64_t n = pl->n_src_pad;
  const CurveView cv = m->curves();
  if (n > 0) {
    k_sources<<<blocks_for(n), kBlock, 0, st>>>(m->ax, m->ay, m->bx, m->by, m->cx, m->cy, m->det, cv, pl->far_x,
                                                pl->far_y, pl->far_w, pl->n_f, pl->n_tri, n, pl->sxy, pl->swj);
    k_src_groups<<<blocks_for(n / 64), kBlock, 0, st>>>(pl->sxy, n / 64, pl->sgrp, pl->soff);
  }
  if (pl->n_tri > 0)
    k_deff<<<blocks_for(pl->n_tri), kBlock, 0, st>>>(m->det, pl->n_tri, cv, pl->swj, pl->far_w, pl->n_f, pl->deff);
  return hipGetLastError();
}

hipError_t launch_map_points(const vp_mesh* m, int n_ref, const double* ref, double* out, hipStream_t st) {
  const int64_t n = m->n_tri * n_ref;
  if (n > 0)
    k_map_points<<<blocks_for(n), kBlock, 0, st>>>(m->ax, m->ay, m->bx, m->by, m->cx, m->cy, m->curves(), m->n_tri,
                                                   n_ref, ref, out);
  return hipGetLastError();
}

// Near-list construction.  Allocates the CSR arrays of the plan.
hipError_t build_pairs(vp_plan* pl, hipStream_t st, std::string& err) {
  const vp_mesh* m = pl->mesh;
  const int64_t T = pl->n_tri, NT = pl->n_tgt;
  hipError_t e;
  auto alloc = [&](void** p, size_t bytes) -> hipError_t { return plan_alloc(pl, p, bytes); };
  e = alloc((void**)&pl->row_ptr, sizeof(int64_t) * (NT + 1));
  if (e != hipSuccess) return e;
  if (NT == 0 || T == 0) {
    if ((e = hipMemsetAsync(pl->row_ptr, 0, sizeof(int64_t) * (NT + 1), st)) != hipSuccess) return e;
    pl->n_pairs = 0;
    pl->n_self = 0;
    e = alloc((void**)&pl->pair_tri, 4);
    if (e == hipSuccess) e = alloc((void**)&pl->pair_tgt, 4);
    if (e == hipSuccess) e = alloc((void**)&pl->pair_kind, 4);
    return e;
  }
  // temporaries
  Scratch tmp(pl->ctx, st);
  auto talloc = [&](void** p, size_t bytes) { return tmp.alloc(p, bytes); };
  auto cleanup = [&]() { tmp.release(); };
  double *thr = nullptr, *box = nullptr, *part = nullptr;
  const int nred = 256;
  if ((e = talloc((void**)&thr, sizeof(double) * 3 * T)) != hipSuccess ||
      (e = talloc((void**)&box, sizeof(double) * 4 * T)) != hipSuccess ||
      (e = talloc((void**)&part, sizeof(double) * 5 * nred)) != hipSuccess) {
    cleanup();
    return e;
  }
  const double eps_cn = pl->eps * pl->opts.c_n;
  const double inv_order = 1.0 / (2.0 * pl->q - 1.0);
  k_tri_ellipses<<<blocks_for(T), kBlock, 0, st>>>(m->ax, m->ay, m->bx, m->by, m->cx, m->cy, pl->deff, T,
                                                   pl->far_what[0], pl->far_what[1], pl->far_what[2], eps_cn,
                                                   inv_order, pl->opts.near_model == VP_NEAR_BALL ? 1 : 0,
                                                   pl->opts.ball_factor, m->curves(), thr, box);
  k_extent_partial<<<nred, kBlock, 0, st>>>(pl->xt, pl->yt, NT, box, T, part);
  if ((e = hipGetLastError()) != hipSuccess) {
    cleanup();
    return e;
  }
  std::vector<double> hp(5 * nred);
  if ((e = hipMemcpyAsync(hp.data(), part, sizeof(double) * 5 * nred, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    cleanup();
    return e;
  }
  double gx0 = 1e300, gy0 = 1e300, gx1 = -1e300, gy1 = -1e300, sum = 0.0;
  for (int i = 0; i < nred; ++i) {
    gx0 = std::min(gx0, hp[5 * i]);
    gy0 = std::min(gy0, hp[5 * i + 1]);
    gx1 = std::max(gx1, hp[5 * i + 2]);
    gy1 = std::max(gy1, hp[5 * i + 3]);
    sum += hp[5 * i + 4];
  }
  // cell size: a quarter of the mean extent of the triangles' near-field
  // boxes (a target tests the triangles whose boxes meet its cell: cells of
  // the boxes' size would test about 4x as many as boxes hold it), enlarged
  // if the grid would exceed 2^24 cells
  double h = std::max(0.25 * sum / (double)T, 1e-300);
  double wx = std::max(gx1 - gx0, 0.0), wy = std::max(gy1 - gy0, 0.0);
  double cells = (wx / h + 1.0) * (wy / h + 1.0);
  if (cells > 16777216.0) h *= std::sqrt(cells / 16777216.0);
  Grid g;
  g.x0 = gx0;
  g.y0 = gy0;
  g.inv_h = 1.0 / h;
  g.nx = std::max(1, (int)std::ceil(wx / h) + 1);
  g.ny = std::max(1, (int)std::ceil(wy / h) + 1);
  const int64_t nc = (int64_t)g.nx * g.ny;
  int32_t *ccnt = nullptr, *tcnt = nullptr, *ctri = nullptr, *pcnt = nullptr, *scnt = nullptr;
  int64_t *cptr = nullptr, *toff = nullptr;
  void* stmp = nullptr;
  const int64_t nscan = std::max(std::max(nc, NT), T);
  if ((e = talloc((void**)&ccnt, sizeof(int32_t) * nc)) != hipSuccess ||
      (e = talloc((void**)&tcnt, sizeof(int32_t) * T)) != hipSuccess ||
      (e = talloc((void**)&cptr, sizeof(int64_t) * (nc + 1))) != hipSuccess ||
      (e = talloc((void**)&toff, sizeof(int64_t) * (T + 1))) != hipSuccess ||
      (e = talloc(&stmp, exclusive_scan_tmp_bytes(nscan))) != hipSuccess ||
      (e = talloc((void**)&pcnt, sizeof(int32_t) * NT)) != hipSuccess ||
      (e = talloc((void**)&scnt, sizeof(int32_t) * NT)) != hipSuccess) {
    cleanup();
    return e;
  }
  if ((e = hipMemsetAsync(ccnt, 0, sizeof(int32_t) * nc, st)) != hipSuccess) {
    cleanup();
    return e;
  }
  k_cell_count<<<blocks_for(T), kBlock, 0, st>>>(box, T, g, ccnt);
  k_cell_tcount<<<blocks_for(T), kBlock, 0, st>>>(box, T, g, tcnt);
  int64_t n_entries = 0;
  if ((e = exclusive_scan_i32(ccnt, cptr, nc, stmp, st)) != hipSuccess ||
      (e = exclusive_scan_i32(tcnt, toff, T, stmp, st)) != hipSuccess ||
      (e = hipMemcpyAsync(&n_entries, cptr + nc, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    cleanup();
    return e;
  }
  if (n_entries >= (int64_t)INT_MAX) {
    err = "near-field grid: too many (cell, triangle) entries";
    cleanup();
    return hipErrorOutOfMemory;
  }
  {
    // entries in triangle order, then a stable radix sort by cell
    int32_t *key = nullptr, *key2 = nullptr, *val = nullptr;
    void* sort_tmp = nullptr;
    size_t sort_bytes = 0;
    const size_t ne = (size_t)std::max<int64_t>(n_entries, 1);
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < nc) ++bits;
    if ((e = talloc((void**)&ctri, sizeof(int32_t) * ne)) != hipSuccess ||
        (e = talloc((void**)&key, sizeof(int32_t) * ne)) != hipSuccess ||
        (e = talloc((void**)&key2, sizeof(int32_t) * ne)) != hipSuccess ||
        (e = talloc((void**)&val, sizeof(int32_t) * ne)) != hipSuccess ||
        (e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key, key2, val, ctri, (int)n_entries, 0, bits,
                                                st)) != hipSuccess ||
        (e = talloc(&sort_tmp, std::max<size_t>(sort_bytes, 16))) != hipSuccess) {
      cleanup();
      return e;
    }
    if (n_entries > 0) {
      k_cell_emit<<<blocks_for(T), kBlock, 0, st>>>(box, T, g, toff, key, val);
      if ((e = hipcub::DeviceRadixSort::SortPairs(sort_tmp, sort_bytes, key, key2, val, ctri, (int)n_entries, 0, bits,
                                                  st)) != hipSuccess) {
        cleanup();
        return e;
      }
    }
  }
  TriView tv{m->ax,
             m->ay,
             m->bx,
             m->by,
             m->cx,
             m->cy,
             m->det,
             thr,
             T,
             pl->opts.near_model == VP_NEAR_BALL ? 1 : 0,
             pl->opts.ball_factor,
             m->curves(),
             box,
             pl->opts.tau <= 1e-10 ? 1 : 0,
             m->geo};
  // decision bits of every (target, cell triangle): word offsets per target
  int32_t* wcnt = nullptr;
  int64_t* woff = nullptr;
  uint2* mk = nullptr;
  int64_t n_words = 0;
  if ((e = talloc((void**)&wcnt, sizeof(int32_t) * std::max<int64_t>(NT, 1))) != hipSuccess ||
      (e = talloc((void**)&woff, sizeof(int64_t) * (NT + 1))) != hipSuccess) {
    cleanup();
    return e;
  }
  if (NT > 0) k_pair_words<<<blocks_for(NT), kBlock, 0, st>>>(pl->xt, pl->yt, NT, g, cptr, wcnt);
  if ((e = exclusive_scan_i32(wcnt, woff, NT, stmp, st)) != hipSuccess ||
      (e = hipMemcpyAsync(&n_words, woff + NT, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess ||
      (e = talloc((void**)&mk, sizeof(uint2) * std::max<int64_t>(n_words, 1))) != hipSuccess) {
    cleanup();
    return e;
  }
  const bool curved = tv.cv.of != nullptr;
  if (curved)
    k_pair_count<true><<<blocks_for(NT), kBlock, 0, st>>>(pl->xt, pl->yt, NT, g, cptr, ctri, tv, pl->opts.tau, woff,
                                                          mk, pcnt);
  else
    k_pair_count<false><<<blocks_for(NT), kBlock, 0, st>>>(pl->xt, pl->yt, NT, g, cptr, ctri, tv, pl->opts.tau, woff,
                                                           mk, pcnt);
  if ((e = exclusive_scan_i32(pcnt, pl->row_ptr, NT, stmp, st)) != hipSuccess) {
    cleanup();
    return e;
  }
  int64_t np = 0;
  if ((e = hipMemcpyAsync(&np, pl->row_ptr + NT, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    cleanup();
    return e;
  }
  pl->n_pairs = np;
  // the plan's blocks so far are in in_use already; the pairs and rows must
  // fit beside them (cached blocks are given back for them if needed)
  if (!ctx_fits(pl->ctx, (size_t)np * (9 + 8 * (size_t)pl->n_p))) {
    err = "plan exceeds the context's HBM budget";
    cleanup();
    return hipErrorOutOfMemory;
  }
  if ((e = alloc((void**)&pl->pair_tri, sizeof(int32_t) * np)) != hipSuccess ||
      (e = alloc((void**)&pl->pair_tgt, sizeof(int32_t) * np)) != hipSuccess ||
      (e = alloc((void**)&pl->pair_kind, std::max<int64_t>(np, 1))) != hipSuccess) {
    cleanup();
    return e;
  }
  // d_sum: self pairs; d_sum[1]: a target whose fill disagreed with its count
  unsigned long long* d_sum = (unsigned long long*)part;
  if ((e = hipMemsetAsync(d_sum, 0, 2 * sizeof(unsigned long long), st)) != hipSuccess) {
    cleanup();
    return e;
  }
  if (NT > 0) {
    const int64_t nb = std::min<int64_t>((NT + kFillWaves * kFillPerWave - 1) / (kFillWaves * kFillPerWave),
                                         (int64_t)1 << 22);
    k_pair_fill<<<(unsigned)nb, kFillWaves * 64, 0, st>>>(pl->xt, pl->yt, NT, g, cptr, ctri, woff, mk, pl->row_ptr,
                                                          pl->pair_tri, pl->pair_tgt, pl->pair_kind, scnt,
                                                          (int*)(d_sum + 1));
  }
  k_count_sum<<<(unsigned)std::min<int64_t>(std::max<int64_t>(blocks_for(NT), 1), kCountSumBlocks), kBlock, 0, st>>>(
      scnt, NT, d_sum);
  unsigned long long ns[2] = {0, 0};
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipMemcpyAsync(ns, d_sum, sizeof(ns), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    cleanup();
    return e;
  }
  if (ns[1]) {
    err = "near lists: a target's pairs do not fill its range";
    cleanup();
    return hipErrorUnknown;
  }
  pl->n_self = (int64_t)ns[0];
  cleanup();
  return hipSuccess;
}

}  // namespace vp
