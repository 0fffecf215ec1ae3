// Internal declarations of libvp: host-side rule construction, device data
// of meshes and plans, kernel launchers, and the device Koornwinder basis.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vp.h"

namespace vp {

constexpr int kMaxP = 10;
constexpr int kMaxQ = 32;
constexpr int kWave = 64;

inline int n_basis(int p) { return (p + 1) * (p + 2) / 2; }

// ---------------------------------------------------------------------------
// Host-side reference rules (vp_rules.cpp).  All built in long double from
// three-term recurrences: nodes by Sturm-sequence bisection on the Jacobi
// matrix, weights as Christoffel numbers.
// ---------------------------------------------------------------------------
struct Rule1D {
  std::vector<double> x, w;
};
struct Rule2D {
  std::vector<double> x, y, w;  // reference-simplex nodes and weights
};
Rule1D gauss_legendre01(int n);
Rule1D gauss_log01(int n);                  // weight -log(r) on [0,1]
Rule2D collapsed_gauss(int q);              // q x q, node index a*q + b
void edge_weights(const Rule2D& r, int q, double out[3]);
Rule2D interp_nodes(int p);                 // interior Blyth-Pozrikidis nodes
int radial_half(int p);
// radial rule: r, alpha (multiplies log r0), beta (constant)
void radial_rule(int p, std::vector<double>& r, std::vector<double>& alpha, std::vector<double>& beta);
// the same sums on p + 1 nodes for a basis of degree <= p along each ray
// (straight self pieces)
void radial_rule_folded(int p, std::vector<double>& r, std::vector<double>& alpha, std::vector<double>& beta);
// Up to this order the row kernels accumulate in the product basis of
// basis_acc and convert to Koornwinder coefficients once per pair
// (basis_row).
constexpr int kBasisLegMax = 6;
// the conversion's coefficients for order p <= kBasisLegMax: g[i][j],
// [n_p][p + 1], for Koornwinder index i = n(n+1)/2 + m and j <= n - m
std::vector<double> basis_connection(int p);

// ---------------------------------------------------------------------------
// Device Koornwinder basis (Sec. 2.1), division-free in the collapsed
// coordinate:  K_mn(x,y) = c_mn P^{(2m+1,0)}_{n-m}(2x-1) Q_m(x,y) with
// Q_m = (1-x)^m P_m(2y/(1-x) - 1) from the scaled Legendre recurrence
//   (m+1) Q_{m+1} = (2m+1)(2y-1+x) Q_m - m (1-x)^2 Q_{m-1}.
// `emit(k, value)` is called once per basis function, k = n(n+1)/2 + m.
// ---------------------------------------------------------------------------
template <int P, class Emit>
__device__ __forceinline__ void koornwinder_emit(double x, double y, Emit&& emit) {
  const double t = 1.0 - x;
  const double s = 2.0 * y - t;
  const double tt = t * t;
  const double z = 2.0 * x - 1.0;
  double Q[P + 1];
  Q[0] = 1.0;
  if (P >= 1) Q[1] = s;
#pragma unroll
  for (int m = 1; m < P; ++m) {
    Q[m + 1] = ((2.0 * m + 1.0) * s * Q[m] - (double)m * tt * Q[m - 1]) * (1.0 / (m + 1.0));
  }
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    const double a = 2.0 * m + 1.0;
    double jm2 = 0.0, jm1 = 1.0;
#pragma unroll
    for (int k = 0; k + m <= P; ++k) {
      double jk;
      if (k == 0) {
        jk = 1.0;
      } else if (k == 1) {
        jk = 0.5 * ((a + 2.0) * z + a);
      } else {
        const double kk = (double)k;
        const double c1 = (2.0 * kk + a - 1.0);
        const double c2 = (2.0 * kk + a) * (2.0 * kk + a - 2.0);
        const double c3 = 2.0 * (kk + a - 1.0) * (kk - 1.0) * (2.0 * kk + a);
        const double inv = 1.0 / (2.0 * kk * (kk + a) * (2.0 * kk + a - 2.0));
        jk = (c1 * (c2 * z + a * a) * jm1 - c3 * jm2) * inv;
      }
      if (k >= 1) {
        jm2 = jm1;
      }
      jm1 = jk;
      const int n = m + k;
      const double cmn = __builtin_sqrt(2.0 * (2.0 * m + 1.0) * (n + 1.0));
      emit(n * (n + 1) / 2 + m, cmn * jk * Q[m]);
    }
  }
}

// acc[k] += w K_k(x, y) for every k: the same basis with the accumulation
// folded into the recurrences.  Q_m is carried as Qh_m = d_m Q_m with
// d_{m+1} = d_m (m+1)/(2m+1), which turns its recurrence into
//   Qh_{m+1} = s Qh_m - e_m (1-x)^2 Qh_{m-1},  e_m = d_{m+1} m / ((m+1) d_{m-1}),
// and each Jacobi sequence is carried already multiplied by c_mn / d_m,
// with the three-term coefficients divided accordingly (all of them
// compile-time constants), so that a basis function costs one FMA into acc
// with w Qh_m formed once per m.  About 40% fewer operations per point than
// emit + FMA; the values agree to rounding.
template <int P>
__device__ __forceinline__ void koornwinder_acc(double x, double y, double w, double* acc) {
  const double t = 1.0 - x;
  const double s = 2.0 * y - t;
  const double tt = t * t;
  const double z = 2.0 * x - 1.0;
  double d[P + 2];
  d[0] = 1.0;
  d[1] = 1.0;
#pragma unroll
  for (int m = 1; m <= P; ++m) d[m + 1] = d[m] * (m + 1.0) / (2.0 * m + 1.0);
  // m ascending, Qh_m advanced after its Jacobi sequence (two Qh live)
  double qm1 = 0.0, qm = 1.0;
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    const double wq = w * qm;
    const double a = 2.0 * m + 1.0;
    double jm2 = 0.0, jm1 = 0.0, cprev = 1.0, cprev2 = 1.0;
#pragma unroll
    for (int k = 0; k + m <= P; ++k) {
      const int n = m + k;
      const double cmn = __builtin_sqrt(2.0 * (2.0 * m + 1.0) * (n + 1.0)) / d[m];
      double jk;
      if (k == 0) {
        jk = cmn;
      } else if (k == 1) {
        jk = fma(0.5 * (a + 2.0) * cmn, z, 0.5 * a * cmn);
      } else {
        const double kk = (double)k;
        const double c1 = (2.0 * kk + a - 1.0);
        const double c2 = (2.0 * kk + a) * (2.0 * kk + a - 2.0);
        const double c3 = 2.0 * (kk + a - 1.0) * (kk - 1.0) * (2.0 * kk + a);
        const double inv = 1.0 / (2.0 * kk * (kk + a) * (2.0 * kk + a - 2.0));
        const double al = c1 * c2 * inv * (cmn / cprev), be = c1 * a * a * inv * (cmn / cprev);
        const double ga = c3 * inv * (cmn / cprev2);
        jk = fma(fma(al, z, be), jm1, -ga * jm2);
      }
      cprev2 = cprev;
      cprev = cmn;
      jm2 = jm1;
      jm1 = jk;
      acc[n * (n + 1) / 2 + m] = fma(jk, wq, acc[n * (n + 1) / 2 + m]);
    }
    if (m < P) {
      double qn;
      if (m == 0) {
        qn = s;
      } else {
        const double e = d[m + 1] * ((double)m / (m + 1.0)) / d[m - 1];
        qn = fma(s, qm, (-e * tt) * qm1);
      }
      qm1 = qm;
      qm = qn;
    }
  }
}

// The product basis of the accumulation (orders up to kBasisLegMax): for
// each m the homogeneous monic Legendre polynomial Qm_m(x, y) = (1-x)^m
// Pm_m((2y-1+x)/(1-x)) times the monic Legendre polynomials Pm_j(2x-1),
// j <= P - m, at the Koornwinder index n(n+1)/2 + m (n = m + j).  Pm_j
// follows Pm_{j+1} = z Pm_j - j^2/(4j^2-1) Pm_{j-1}, so all the z factors
// come from one recurrence shared by every m instead of one Jacobi
// sequence per m; K_{m,k} = c_mn P^{(2m+1,0)}_k Q_m is a combination of
// the Pm_j, j <= k, with the same Qm_m, which basis_finish applies to the
// accumulated sums.
template <int P>
__device__ __forceinline__ void basis_acc(double x, double y, double w, double* acc) {
  if constexpr (P > kBasisLegMax) {
    koornwinder_acc<P>(x, y, w, acc);
  } else {
    const double t = 1.0 - x;
    const double s = 2.0 * y - t;
    const double tt = t * t;
    const double z = 2.0 * x - 1.0;
    double L[P + 1];
    L[0] = 1.0;
    if (P >= 1) L[1] = z;
#pragma unroll
    for (int j = 1; j < P; ++j) L[j + 1] = fma(z, L[j], -((double)(j * j) / (4.0 * j * j - 1.0)) * L[j - 1]);
    double qm1 = 0.0, qm = 1.0;
#pragma unroll
    for (int m = 0; m <= P; ++m) {
      const double wq = w * qm;
#pragma unroll
      for (int j = 0; j + m <= P; ++j) {
        const int n = m + j;
        acc[n * (n + 1) / 2 + m] = fma(wq, L[j], acc[n * (n + 1) / 2 + m]);
      }
      if (m < P) {
        const double qn = (m == 0) ? s : fma(s, qm, -((double)(m * m) / (4.0 * m * m - 1.0)) * (tt * qm1));
        qm1 = qm;
        qm = qn;
      }
    }
  }
}

// Koornwinder coefficient i = n(n+1)/2 + m of a pair from the pair's sums
// of the product basis (sb, at the same indices): sum over j <= k = n - m
// of g[i][j] times the sum of Qm_m Pm_j; g is [n_p][P + 1]
template <int P>
__device__ __forceinline__ double basis_row(const double* sb, const double* __restrict__ g, int i) {
  int n = 0;
  while ((n + 1) * (n + 2) / 2 <= i) ++n;
  const int m = i - n * (n + 1) / 2, k = n - m;
  double r = 0.0;
  for (int j = 0; j <= k; ++j) r = fma(g[i * (P + 1) + j], sb[(m + j) * (m + j + 1) / 2 + m], r);
  return r;
}

// The naive ball test of the near-field ablation (near: within kappa R of
// the centroid c, R = the largest vertex distance from c), evaluated with
// separately rounded operations in a fixed order (no contraction into
// FMA), so that its decisions equal those of a plain IEEE evaluation of
// the same formulas: vertex = (A + xi1 (B - A)) + xi2 (C - A),
// c = ((p0 + p1) + p2) / 3, distances sqrt(dx dx + dy dy).
__device__ __forceinline__ double ball_dist(double ax, double ay, double bx, double by) {
  const double dx = __dadd_rn(ax, -bx), dy = __dadd_rn(ay, -by);
  return sqrt(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
}

__device__ __forceinline__ bool in_ball3(double x, double y, const double px[3], const double py[3], double kappa) {
  const double gx = __dadd_rn(__dadd_rn(px[0], px[1]), px[2]) / 3.0;
  const double gy = __dadd_rn(__dadd_rn(py[0], py[1]), py[2]) / 3.0;
  const double R = fmax(fmax(ball_dist(px[0], py[0], gx, gy), ball_dist(px[1], py[1], gx, gy)),
                        ball_dist(px[2], py[2], gx, gy));
  return ball_dist(x, y, gx, gy) < __dmul_rn(kappa, R);
}

// Ball test of the sub-triangle (sa, sb, ss) of triangle A + xi1 e1 + xi2 e2:
// reference vertices (sa, sb), (sa + ss, sb), (sa, sb + ss) (exact dyadic
// values), each mapped directly.
__device__ __forceinline__ bool in_ball_sub(double x, double y, double Ax, double Ay, double e1x, double e1y,
                                            double e2x, double e2y, double sa, double sb, double ss,
                                            double kappa) {
  const double r1[3] = {sa, sa + ss, sa}, r2[3] = {sb, sb, sb + ss};
  double px[3], py[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    px[i] = __dadd_rn(__dadd_rn(Ax, __dmul_rn(r1[i], e1x)), __dmul_rn(r2[i], e2x));
    py[i] = __dadd_rn(__dadd_rn(Ay, __dmul_rn(r1[i], e1y)), __dmul_rn(r2[i], e2y));
  }
  return in_ball3(x, y, px, py, kappa);
}

// ---------------------------------------------------------------------------
// Curved boundary triangles (Sec. 3.1, eq. blend).  A curved triangle
// stores A = gamma(1), B = gamma(0) (the ends of its curved side) and the
// opposite vertex C, counter-clockwise, and gamma(u), u in [0, 1], as
// Chebyshev coefficients in s = 2u - 1 (degree <= kCurveMax - 1), together
// with those of d gamma / ds.  With beta(u) = gamma(u) - (B + u (A - B)),
// the side's offset from its chord, and u = 1 - xi:
//   rho(xi, eta) = A + xi (B - A) + eta (C - A) + ((u - eta) / u) beta(u).
// ---------------------------------------------------------------------------
constexpr int kCurveMax = 33;  // coefficients per coordinate

struct CurveView {
  const int32_t* of = nullptr;  // [T] index of the triangle's curve, -1 if straight
  const double* coef = nullptr; // [n_curved][4][kCurveMax]: x, y, dx/ds, dy/ds
  const double* box = nullptr;  // [n_curved][4]: x0, y0, x1, y1 of the element (padded)
  int deg = 0;
};

__host__ __device__ __forceinline__ double cheb_clenshaw(const double* c, int n, double s) {
  // sum_{k < n} c_k T_k(s)
  double b1 = 0.0, b2 = 0.0;
  for (int k = n - 1; k >= 1; --k) {
    const double b0 = fma(2.0 * s, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(s, b1, c[0] - b2);
}

// rho(xi, eta) of a curved triangle, and when dxi/deta are given its partial
// derivatives.  Requires xi < 1 (u > 0); the vertex B itself is B.
__host__ __device__ __forceinline__ void vp_blend(double Ax, double Ay, double Bx, double By, double Cx, double Cy,
                                                  const double* cf, int deg, double xi, double eta, double& px,
                                                  double& py, double* dxi = nullptr, double* deta = nullptr) {
  const double u = 1.0 - xi, s = 2.0 * u - 1.0;
  const double bx = cheb_clenshaw(cf, deg + 1, s) - (Bx + u * (Ax - Bx));
  const double by = cheb_clenshaw(cf + kCurveMax, deg + 1, s) - (By + u * (Ay - By));
  const double f = (u - eta) / u;
  px = Ax + xi * (Bx - Ax) + eta * (Cx - Ax) + f * bx;
  py = Ay + xi * (By - Ay) + eta * (Cy - Ay) + f * by;
  if (dxi) {
    const double dbx = 2.0 * cheb_clenshaw(cf + 2 * kCurveMax, deg, s) - (Ax - Bx);
    const double dby = 2.0 * cheb_clenshaw(cf + 3 * kCurveMax, deg, s) - (Ay - By);
    const double g = eta / (u * u), h = 1.0 - eta / u;
    dxi[0] = (Bx - Ax) - g * bx - h * dbx;
    dxi[1] = (By - Ay) - g * by - h * dby;
    deta[0] = (Cx - Ax) - bx / u;
    deta[1] = (Cy - Ay) - by / u;
  }
}

__host__ __device__ __forceinline__ double vp_blend_jac(double Ax, double Ay, double Bx, double By, double Cx,
                                                        double Cy, const double* cf, int deg, double xi, double eta,
                                                        double& px, double& py) {
  double dx[2], de[2];
  vp_blend(Ax, Ay, Bx, By, Cx, Cy, cf, deg, xi, eta, px, py, dx, de);
  return dx[0] * de[1] - dx[1] * de[0];
}

// rho^{-1}(x) by Newton's method from the chord's affine inverse; false if it
// does not converge (a point far from the element).
__host__ __device__ __forceinline__ bool vp_blend_inverse(double Ax, double Ay, double Bx, double By, double Cx,
                                                          double Cy, double D, const double* cf, int deg, double x,
                                                          double y, double& xi, double& eta) {
  const double d0 = x - Ax, d1 = y - Ay;
  xi = (d0 * (Cy - Ay) - d1 * (Cx - Ax)) / D;
  eta = ((Bx - Ax) * d1 - (By - Ay) * d0) / D;
  double step = 1.0;
  for (int it = 0; it < 60; ++it) {
    xi = fmin(xi, 1.0 - 1e-12);
    double px, py, dx[2], de[2];
    vp_blend(Ax, Ay, Bx, By, Cx, Cy, cf, deg, xi, eta, px, py, dx, de);
    const double rx = px - x, ry = py - y;
    const double J = dx[0] * de[1] - dx[1] * de[0];
    const double sx = (de[1] * rx - de[0] * ry) / J, sy = (dx[0] * ry - dx[1] * rx) / J;
    xi -= sx;
    eta -= sy;
    if (!(fabs(xi) < 1e6 && fabs(eta) < 1e6)) return false;
    step = fabs(sx) + fabs(sy);
    if (step < 1e-16) return true;
  }
  return step < 1e-12;
}

// Natural logarithm of x > 0 (normal) in FP64, table-driven (Tang's
// method): x = m 2^e with m in [1/2, 1); the top eight fraction bits select
// a sub-interval of width 1/512 with centre c_i; with inv_c_i the double
// nearest 1/c_i, r = m inv_c_i - 1 = x (inv_c_i 2^-e) - 1 (|r| <= 1/512)
// comes from one FMA with the scaled table entry, and
//   log x = e ln2 - log(inv_c_i) + log1p(r),
// with log1p(r) from its Taylor series through r^5 (truncation < 1e-17).
// tab[i] = {inv_c_i, -log(inv_c_i)} for i < 256 and tab[256] = {ln2_hi,
// ln2_lo}, ln2_hi holding 32 bits so that e ln2_hi is exact.  Error: a few
// units in the last place of the result.  Subnormal x and x = 0 are not
// supported; every squared distance that reaches a logarithm carries the
// offset kR2Bias below.
constexpr int kLogTab = 256;

// Squared distances enter the kernel as r^2 + 2^-100 (in FP64 and in FP32,
// where 2^-100 is a normal number).  A source at distance 0 from a target
// then has a finite kernel value, the same in the far sum and in the far
// rule that the correction rows subtract, so the pair cancels without a
// per-pair test; for any pair that is not cancelled in this way r is far
// above 2^-50, where the offset changes nothing.
constexpr double kR2Bias = 0x1p-100;
constexpr float kR2BiasF = 0x1p-100f;

// The two parts of vp_log kept apart: log x = e ln2 + rest, e = exponent of x
// as a double.  Sums over many x can accumulate e and rest separately.
__device__ __forceinline__ void vp_log_parts(double x, const double2* tab, double& e_out, double& rest_out) {
  const unsigned hi = (unsigned)__double2hiint(x);
  const unsigned i = (hi >> 12) & 255u;
  const int neg_e = 1022 - (int)(hi >> 20);
  const double2 t = tab[i];
  // m inv_c - 1 with m = x 2^-e: scale the table entry instead of x
  const double r = fma(x, ldexp(t.x, neg_e), -1.0);
  // log1p(r) = r b(r), b = 1 - r/2 + r^2/3 - r^3/4 + r^4/5 by Horner; the
  // table term joins in the last FMA
  double b = fma(r, 0.2, -0.25);
  b = fma(r, b, 1.0 / 3.0);
  b = fma(r, b, -0.5);
  b = fma(r, b, 1.0);
  e_out = -(double)neg_e;
  rest_out = fma(b, r, t.y);
}

__device__ __forceinline__ double vp_log(double x, const double2* tab) {
  double e, rest;
  vp_log_parts(x, tab, e, rest);
  const double2 l2 = tab[kLogTab];
  return fma(e, l2.x, rest) + e * l2.y;
}

// The same method with a 4096-entry table (the top twelve fraction bits;
// |r| <= 2^-13), where log1p(r) through r^3 suffices (truncation
// <= 2^-54), and m, e from the hardware frexp.  Two FP64 operations fewer
// per logarithm than vp_log_parts; the 64 KiB table suits kernels with wide
// blocks (the direct far sum), not the one-wavefront correction rows.
constexpr int kFarLogBits = 12;
constexpr int kFarLogTab = 1 << kFarLogBits;

__device__ __forceinline__ void vp_log_wide_parts(double x, const double2* tab, double& e_out, double& rest_out) {
  const double m = __builtin_amdgcn_frexp_mant(x);  // x = m 2^e, m in [1/2, 1)
  const int e = __builtin_amdgcn_frexp_exp(x);
  const unsigned i = ((unsigned)__double2hiint(x) >> (20 - kFarLogBits)) & (unsigned)(kFarLogTab - 1);
  const double2 t = tab[i];
  const double r = fma(m, t.x, -1.0);
  // log1p(r) = r (1 - r/2 + r^2/3): three FMAs including the table term
  const double b = fma(fma(r, 1.0 / 3.0, -0.5), r, 1.0);
  e_out = (double)e;
  rest_out = fma(b, r, t.y);
}

}  // namespace vp

struct vp_ctx {
  int device = 0;
  int n_cu = 0;  // compute units of the device
  hipStream_t stream = nullptr;
  uint64_t budget = 0;
  uint64_t in_use = 0;     // device bytes held (plans, workspaces, meshes, ...), cached blocks excluded
  uint64_t cache_cap = 0;  // most bytes the block cache keeps (a quarter of the device's memory)
  // FMM translation operators per expansion order, shared by the context's
  // plans (device memory, freed with the context)
  struct FmmOps {
    double2 *m2m = nullptr, *l2l = nullptr;
    double* m2l = nullptr;
    size_t bytes = 0;
  };
  std::map<int, FmmOps> fmm_ops;
  // Device blocks of destroyed plans and outgrown plan workspaces, kept for
  // the context's later plans (freeing a block of hundreds of MB costs about
  // a millisecond of host time, and a plan holds a dozen): cache maps a
  // block's size to the idle block, block_size holds the size of every
  // block allocated this way, idle or not.
  std::multimap<size_t, void*> cache;
  std::map<void*, size_t> block_size;
  uint64_t cached = 0;
  int live_meshes = 0;
  int live_servers = 0;
  // profiling: pending event pairs per stage, folded into the totals on read
  bool profile = false;
  struct Pending {
    int stage;
    hipEvent_t a, b;
    int64_t launches;
  };
  std::vector<Pending> pending;
  double ms[VP_N_STAGES] = {};
  int64_t launches[VP_N_STAGES] = {};
};

// one triangle's packed geometry (vp_mesh::geo)
struct TriGeo {
  double ax, ay, bx, by, cx, cy, det;
};
__device__ __forceinline__ TriGeo tri_geo(const double4* __restrict__ geo, int64_t t) {
  const double4 p = geo[2 * t], q = geo[2 * t + 1];
  return TriGeo{p.x, p.y, p.z, p.w, q.x, q.y, q.z};
}

struct vp_mesh {
  vp_ctx* ctx = nullptr;
  int64_t n_tri = 0;
  // oriented geometry, SoA [n_tri] each: A, B, C, D = det[B-A, C-A] > 0
  double *ax = nullptr, *ay = nullptr, *bx = nullptr, *by = nullptr, *cx = nullptr, *cy = nullptr,
         *det = nullptr;
  // the same packed per triangle, [n_tri][2]: (Ax, Ay, Bx, By), (Cx, Cy, D, 0)
  // (the per-pair kernels read a triangle from one 64-byte line)
  double4* geo = nullptr;
  size_t bytes = 0;
  int live_plans = 0;
  // curved boundary triangles (vp_mesh_set_curved_sides): device arrays
  int64_t n_curved = 0;
  int curve_deg = 0;
  int32_t* curve_of = nullptr;   // [n_tri]
  int32_t* curve_tri = nullptr;  // [n_curved]
  double* curve_coef = nullptr;  // [n_curved][4][kCurveMax]
  double* curve_box = nullptr;   // [n_curved][4]
  vp::CurveView curves() const {
    vp::CurveView v;
    v.of = curve_of;
    v.coef = curve_coef;
    v.box = curve_box;
    v.deg = curve_deg;
    return v;
  }
};

struct vp_plan {
  vp_ctx* ctx = nullptr;
  const vp_mesh* mesh = nullptr;
  int p = 0, q = 0, n_p = 0, n_f = 0;
  double eps = 0.0;
  vp_plan_opts opts{};
  int64_t n_tri = 0, n_src = 0, n_tgt = 0, n_pairs = 0, n_self = 0;
  int64_t stats[4] = {0, 0, 0, 0};  // near leaves, self panels, capped leaves, depth-first pairs
  int64_t tab_pairs = 0, tab_leaves = 0;  // near pairs (and their leaves) of the matrix-core row path
  double ms_classify = 0.0, ms_rows = 0.0;
  // rule tables (device)
  double* vinv = nullptr;   // [n_p][n_p]
  double* efar = nullptr;   // [n_f][n_p] Koornwinder values at far nodes
  double* wfar = nullptr;   // [n_f][n_p] efar V^{-1}: interpolant at far nodes from node values
  double* far_x = nullptr;  // [n_f]
  double* far_y = nullptr;
  double* far_w = nullptr;
  double* near_x = nullptr;  // [q_near^2]
  double* near_y = nullptr;
  double* near_w = nullptr;
  double* gl_s = nullptr;  // [n_l]
  double* gl_w = nullptr;
  double* rad_r = nullptr;  // [n_r]
  double* basis_g = nullptr;  // [n_p][p + 1] basis_row's coefficients (p <= kBasisLegMax)
  double* rad_a = nullptr;
  double* rad_b = nullptr;
  int n_r = 0;
  double far_what[3] = {0, 0, 0}, near_what[3] = {0, 0, 0};
  // sources and targets (device)
  int64_t n_src_pad = 0;                // n_src rounded up to a multiple of 256
  double2* sxy = nullptr;               // [n_src_pad] source positions
  double* sgrp = nullptr;               // [n_src_pad / 64][3] centre x, y and radius of each 64-source group
  float2* soff = nullptr;               // [n_src_pad] each source's offset from its group's centre (FP32)
  double* swj = nullptr;                // [n_src_pad] source weights w_j |J(xi_j)| (0 in the padding)
  double* deff = nullptr;               // [T] |J| scale of the ellipse tests (det; the largest far-node |J| if curved)
  double* rad_c_r = nullptr;            // radial rule of curved self pieces [n_rc]
  double* rad_c_a = nullptr;
  double* rad_c_b = nullptr;
  int n_rc = 0;
  double2* logtab = nullptr;            // [kLogTab + 1] table of the FP64 logarithm
  double2* logtab_wide = nullptr;       // [kFarLogTab + 1] table of the far sum's logarithm
  double *xt = nullptr, *yt = nullptr;  // [n_tgt]
  // pair list (device)
  int64_t* row_ptr = nullptr;  // [n_tgt+1]
  int32_t* pair_tri = nullptr;  // [n_pairs]
  int32_t* pair_tgt = nullptr;  // [n_pairs]
  uint8_t* pair_kind = nullptr;  // [n_pairs]
  double* rows = nullptr;  // [n_pairs][n_p]
  // clusters of 16 consecutive targets for the matrix-core correction apply
  // (0 clusters: not built, the apply stays on the vector ALUs)
  int64_t n_cl = 0, n_entries = 0;
  bool cl_tried = false;  // clusters built (or given up) by the first evaluation of several densities
  int64_t* cl_ptr = nullptr;    // [n_cl+1] entries of each cluster
  int32_t* ent_tri = nullptr;   // [n_entries] triangle of the entry (ascending within a cluster)
  int32_t* ent_pair = nullptr;  // [n_entries][16] pair index per cluster target, -1 if absent
  // execute workspace
  int64_t ws_rhs = 0;
  int64_t ws_split = 0;
  // FMM far sum (fmm_terms > 0; built at plan creation)
  int fmm_terms = 0, fmm_levels = 0;
  double fmm_x0 = 0.0, fmm_y0 = 0.0, fmm_width = 0.0;  // root square
  int64_t fmm_off[12] = {};                           // first box of each level in the per-level arrays
  int32_t *fmm_src_perm = nullptr, *fmm_tgt_perm = nullptr;  // leaf order -> source / target index
  int64_t *fmm_src_ptr = nullptr, *fmm_tgt_ptr = nullptr;    // [4^L + 1] CSR by leaf box
  double2* fmm_sxy = nullptr;                                // source positions in leaf order
  int32_t *fmm_cnt_src = nullptr, *fmm_cnt_tgt = nullptr;    // sources / targets per box, all levels
  double2 *fmm_m2m = nullptr, *fmm_l2l = nullptr;  // translation operators (complex)
  double* fmm_m2l = nullptr;                         // M2L operators, real form [49][fmm_mp][fmm_kp]
  int fmm_mp = 0, fmm_kp = 0;
  int64_t fmm_near_pairs = 0, fmm_m2l_pairs = 0;  // work counts (plan statistics)
  // blocks of 16 densities: P2M rows [n_src][fmm_mp], L2P rows [n_tgt][fmm_kp]
  // (both in leaf order), (leaf box, first target) of every 16-target tile
  double *fmm_vsrc = nullptr, *fmm_wtgt = nullptr;
  int2* fmm_ttile = nullptr;
  int64_t fmm_n_ttiles = 0;
  int32_t* fmm_tbox = nullptr;  // [n_tgt] leaf box of each target in leaf order
  int32_t* fmm_tile_order = nullptr;  // [ceil(n_tgt / 16)] leaf-pass tiles, most direct pairs first
  std::vector<int64_t> fmm_tgt_ptr_host;  // host copy of fmm_tgt_ptr (tile list)
  // far-sum launch shapes stored for (n_rhs, precision) by the tuner or the caller
  std::map<std::pair<int64_t, int>, vp_far_config> far_tuned;
  double *ws_f = nullptr, *ws_c = nullptr, *ws_q = nullptr, *ws_part = nullptr, *ws_u = nullptr;
  float* ws_q32 = nullptr;
  size_t ws_bytes = 0;
  std::vector<void*> allocs;  // everything above except the workspace
  size_t bytes = 0;
  int live_requests = 0;  // requests of a server not yet finished
};

namespace vp {

// Device memory of plans, their workspaces, server slots and captured
// evaluations, through the context's block cache.  ctx_alloc takes an idle
// cached block of at least `bytes` (and at most a quarter more), else calls
// hipMalloc, emptying the cache and trying once more when the device is out
// of memory; the block's size (`*got`) counts in ctx->in_use until
// ctx_release, which takes a block that no queued device work uses any
// more: it joins the cache while the cache stays within ctx->cache_cap (a
// quarter of the device's memory), else it is freed.  With an HBM budget,
// in_use + cached never exceeds it: ctx_alloc empties the cache first when
// a new block would cross it, and fails with hipErrorOutOfMemory when the
// block does not fit even then.  ctx_fits makes the same check (and the same
// room) for memory allocated outside the cache (meshes, interpolation
// objects, FMM operators), whose callers add it to in_use themselves.
// ctx_trim frees every idle block.  plan_alloc allocates a block owned by
// the plan (released when the plan is destroyed).
hipError_t ctx_alloc(vp_ctx* ctx, void** p, size_t bytes, size_t* got = nullptr);
void ctx_release(vp_ctx* ctx, void* p);
void ctx_trim(vp_ctx* ctx);
bool ctx_fits(vp_ctx* ctx, uint64_t bytes);
hipError_t plan_alloc(vp_plan* pl, void** dst, size_t bytes);

// Temporaries of a plan build used on stream st only, from the context's
// block cache: release() (also run by the destructor) waits for st and hands
// them back, so a later allocation can take them without a device wait.
struct Scratch {
  vp_ctx* ctx;
  hipStream_t st;
  std::vector<void*> blocks;
  Scratch(vp_ctx* c, hipStream_t s) : ctx(c), st(s) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() { release(); }
  hipError_t alloc(void** p, size_t bytes) {
    hipError_t r = ctx_alloc(ctx, p, bytes ? bytes : 8);
    if (r == hipSuccess) blocks.push_back(*p);
    return r;
  }
  void release() {
    if (blocks.empty()) return;
    (void)hipStreamSynchronize(st);
    for (void* p : blocks) ctx_release(ctx, p);
    blocks.clear();
  }
};

// ---------------------------------------------------------------------------
// Kernel launchers (vp_*.hip).  All enqueue on `st` and return the launch
// status.
// ---------------------------------------------------------------------------
hipError_t launch_mesh_geom(const double* vert, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                            vp_mesh* m, int* d_bad, hipStream_t st);
hipError_t launch_split_xy(const double* xy, int64_t n, double* x, double* y, int* d_bad, hipStream_t st);
hipError_t launch_basis_tables(vp_plan* pl, double* scratch, hipStream_t st);
hipError_t launch_sources(vp_plan* pl, hipStream_t st);  // positions, weights and |J| scales
hipError_t launch_map_points(const vp_mesh* m, int n_ref, const double* ref, double* out, hipStream_t st);
hipError_t launch_vinv(int p, const double* nx, const double* ny, double* aug, double* vinv, int* bad,
                       hipStream_t st);
constexpr int kCurvedRadial = 12;  // points per part of the radial rule on curved self pieces
hipError_t build_pairs(vp_plan* pl, hipStream_t st, std::string& err);  // near-list construction
// Diagnostics of the correction rows (near leaves, self panels, capped
// leaves, depth-first pairs): kRowStatSlots slots of kRowStatStride int64
// (one cache line each), zeroed by the caller and summed over the slots.
constexpr int kRowStatSlots = 256;
constexpr int kRowStatStride = 16;
hipError_t launch_rows(vp_plan* pl, int* d_flag, int64_t* d_stats, hipStream_t st);
hipError_t launch_coefficients(const vp_plan* pl, const double* F, int64_t R, double* C, double* Q,
                               hipStream_t st);
// Q32 != nullptr selects the mixed-precision far sum (Q32: [n_src_pad][R]
// scratch for the FP32 charges).
hipError_t launch_far(const vp_plan* pl, const double* Q, int64_t R, const vp_far_config& cfg, double* partial,
                      hipStream_t st, int64_t* n_launches = nullptr, float* Q32 = nullptr);
hipError_t launch_finish(const vp_plan* pl, const double* partial, int64_t n_split, const double* C,
                         int64_t R, bool far_only, double* U, hipStream_t st);
hipError_t build_clusters(vp_plan* pl, hipStream_t st);  // after the pair list; allocates plan memory
// Tables that only blocks of 16 densities use (the FMM's P2M/L2P rows, the
// correction apply's target clusters), built by the first evaluation with
// R >= kMinBlockCols; without clusters (not built, or over the HBM budget)
// the correction apply stays on the vector ALUs.
hipError_t prepare_blocks(vp_plan* pl, int64_t R, hipStream_t st);
// Densities from which the blocks of 16 on the matrix cores also take a
// remainder (padded with zero columns): a padded block costs about as much
// as two single-density passes of the FMM or of the correction apply.
constexpr int64_t kMinBlockCols = 2;
// True if the tables prepare_blocks builds for R densities exist (false
// while the context's budget keeps them out).
bool blocks_ready(const vp_plan* pl, int64_t R);
// U columns [r0, min(R, r0 + 16 nt)) on the matrix cores (nt = 1, 2 or 4)
hipError_t launch_corr_mfma(const vp_plan* pl, const double* partial, int64_t n_split, const double* C, int64_t R,
                            int64_t r0, int nt, bool far_only, double* U, hipStream_t st);
// targets per block of the far-sum launch that takes the first right-hand
// side (the matrix-core kernel for n_rhs >= 16, else the vector one)
int64_t far_targets_per_block(const vp_far_config& cfg, int64_t R, bool mixed);
vp_far_config far_default(const vp_plan* pl, int64_t R, bool mixed);  // shape chosen from the sizes
vp_far_config far_config(const vp_plan* pl, int64_t R, bool mixed);   // stored shape, else far_default
bool far_config_valid(const vp_plan* pl, const vp_far_config& cfg);
// doubles of the far-sum workspace: n_split partial sums per target and RHS,
// then the FMM's expansions and leaf-ordered charges
int64_t far_partial_doubles(const vp_plan* pl, int64_t n_split, int64_t R);
int64_t fmm_boxes(int levels);
int64_t fmm_workspace_doubles(const vp_plan* pl, int64_t R);
hipError_t build_fmm(vp_plan* pl, int leaf, hipStream_t st);  // after sources and targets; plan memory
// tables of the passes of blocks of 16 densities (no-op unless an FMM
// plan, R >= kMinBlockCols and not built yet; not built when they do not fit
// the context's budget, the passes then take one density at a time); call
// before launch_far (not under graph capture)
hipError_t fmm_prepare_blocks(vp_plan* pl, int64_t R, hipStream_t st);
// Q32 (FP32 copy of Q times ln 2, or null): the leaf passes of blocks of
// densities in mixed precision
hipError_t launch_fmm(const vp_plan* pl, const double* Q, int64_t R, double* out, double* ws, hipStream_t st,
                      int64_t* n_launches, const float* Q32 = nullptr);
void set_last_error(const char* msg);
// Device time of a stage on the context's stream (when profiling is on):
// events around the stage's launches, folded into the totals on read.
struct StageTimer {
  vp_ctx* ctx;
  int stage;
  hipEvent_t a = nullptr, b = nullptr;
  explicit StageTimer(vp_ctx* c, int s) : ctx(c), stage(s) {
    if (!ctx->profile) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      ctx->profile = false;
      return;
    }
    (void)hipEventRecord(a, ctx->stream);
  }
  void stop(int64_t launches) {
    if (!a || !ctx->profile) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->pending.push_back({stage, a, b, launches});
    a = b = nullptr;
  }
  ~StageTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Records the device address of the allocation-free evaluation's workspace
// array on `device` (current), once per device.
hipError_t noalloc_setup(int device);
// dst[i][c0 + r] = src[i][r] for i < rows, r < src_cols (dst has dst_cols)
hipError_t launch_pack_columns(const double* src, int64_t rows, int64_t src_cols, double* dst, int64_t dst_cols,
                               int64_t c0, hipStream_t st);
// dst[i][r] = src[i][c0 + r] for i < rows, r < dst_cols (src has src_cols)
hipError_t launch_unpack_columns(const double* src, int64_t rows, int64_t src_cols, int64_t c0, double* dst,
                                 int64_t dst_cols, hipStream_t st);
void log_table(double2* out, int n);  // n entries + the ln 2 split
hipError_t exclusive_scan_i32(const int32_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t st);
size_t exclusive_scan_tmp_bytes(int64_t n);

}  // namespace vp
