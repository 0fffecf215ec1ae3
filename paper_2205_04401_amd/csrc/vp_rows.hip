// Correction rows (FP64), one wavefront per (target, triangle) pair.
//
// row_k = (A_k - B_k) / 2pi for k < n_p, the subtract-and-add correction of
// Sec. 3.6 against the Koornwinder basis:
//   B_k  the far rule's own contribution, sum_j w_j |J| log|x - y_j| K_k(xi_j)
//        (squared distances carry the offset kR2Bias, as in the far sums,
//        so a pair at distance exactly 0 cancels);
//   A_k  the accurate integral of log|x - y| K_k(rho^{-1} y) over the triangle:
//        near pair: adaptive subdivision (Sec. 3.3, eq. sum_near); a
//          sub-triangle is integrated by the near rule once the target lies
//          outside its three Bernstein ellipses (Sec. 4.1, eq. rho0 with the
//          weight scaled by the sub-triangle's |J|), else split in four by
//          edge midpoints; the levels are processed breadth-first with the
//          lanes testing sub-triangles and integrating leaf nodes in
//          parallel;
//        self pair: the triangle split at the target into three pieces, each
//          in radius-arc-length coordinates (Sec. 3.4, Thm. tensor_smooth_new
//          and eq. volpot_self_single) with dyadic panels in arc length
//          toward the target's foot point and the radial rule in r; the
//          lanes share the (panel, arc node, radial node) triples.
// Each lane accumulates n_p partial sums; a butterfly reduction finishes.
//
// Sub-triangles of the reference simplex are stored as (a_x, a_y, s): the
// triangle a, a + s e_1, a + s e_2.  Children of (a, s):
//   (a, s/2), (a + s e_1/2, s/2), (a + s e_2/2, s/2), (a + s (e_1+e_2)/2, -s/2)
// i.e. the three corner triangles and the inverted middle one, each with the
// vertex order that keeps its orientation and its collapse vertex.
#include <algorithm>
#include <cmath>

#include "vp_internal.h"

namespace vp {
namespace {

constexpr int kCap = 128;  // sub-triangles per level per pair
constexpr double kInv2Pi = 0.15915494309189533577;

struct RowsArgs {
  const int32_t* pair_tri;
  const int32_t* pair_tgt;
  const uint8_t* pair_kind;
  int64_t n_pairs;
  const double *xt, *yt;
  const double *ax, *ay, *bx, *by, *cx, *cy, *det;
  const double *far_x, *far_y, *far_w, *efar;
  int nf;
  const double *near_x, *near_y, *near_w;
  int nn;
  double nwhat0, nwhat1, nwhat2;
  double inv_near_order;
  const double *gl_s, *gl_w;
  int nl;
  const double *rad_r, *rad_a, *rad_b;
  int nr;
  double eps_cn, tau;
  int depth_cap, dyadic_cap;
  int ball;            // naive ball model for the near subdivision
  double ball_factor;  // its kappa
  const double2* logtab;
  const double2* sxy;   // the plan's far sources (positions) and their weights w_j |J|
  const double* swj;
  const double* deff;   // |J| scale of the ellipse tests per triangle
  CurveView cv;         // curved triangles
  const double *rad_c_r, *rad_c_a, *rad_c_b;  // radial rule of curved self pieces
  int n_rc;
  double* rows;
  int* flag;
  int64_t* stats;  // near leaves, self panels, capped leaves, depth-first pairs
};

__device__ __forceinline__ int dyadic_count(double len, double d, int cap) {
  int n = 0;
  double w = len;
  while (!(w < d) && n < cap) {
    w *= 0.5;
    ++n;
  }
  return n;
}

// Sum of C per-lane slots over the wavefront, scattered: at each offset
// (32, 16, ..., 1) a lane and its partner (lane ^ OFF) hold the same
// segment of row indices; the lane with the OFF bit clear keeps the first
// half of the slots, its partner the second half (zero-padded when C is
// odd), and each adds what the other sends.  Once one slot is left the
// remaining offsets are a plain butterfly.  base and len track the row
// index of slot 0 and the number of valid slots; the lanes that end with
// duplicates (bits of the butterfly offsets set) report len = 0.
template <int C, int OFF>
struct ReduceScatter {
  static __device__ __forceinline__ void run(double* v, int lane, int& base, int& len) {
    constexpr int H = (C + 1) / 2;
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double lo = v[i];
      const double hi = (H + i < C) ? v[H + i] : 0.0;
      const double recv = __shfl_xor(up ? lo : hi, OFF);
      v[i] = (up ? hi : lo) + recv;
    }
    if (up) {
      base += H;
      len = max(len - H, 0);
    } else {
      len = min(len, H);
    }
    ReduceScatter<H, OFF / 2>::run(v, lane, base, len);
  }
};
template <int OFF>
struct ReduceScatter<1, OFF> {
  static __device__ __forceinline__ void run(double* v, int lane, int& base, int& len) {
#pragma unroll
    for (int o = OFF; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
    if (lane & (2 * OFF - 1)) len = 0;
  }
};
template <int C>
struct ReduceScatter<C, 0> {
  static __device__ __forceinline__ void run(double*, int, int&, int&) {}
};
template <>
struct ReduceScatter<1, 0> {
  static __device__ __forceinline__ void run(double*, int, int&, int&) {}
};

// kCurved: the mesh has curved triangles (the straight-only instance carries
// none of their code).  KIND: 0 every pair, 1 near pairs only, 2 self pairs
// only (each of the two then carries only its own branch, with fewer live
// registers than both together)
template <int P, bool kCurved, int KIND>
__global__ __launch_bounds__(64, 2) void k_rows(RowsArgs a) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  __shared__ double lv[2][kCap * 3];
  __shared__ double leaf[kCap * 3];
  __shared__ double2 tab[kLogTab + 1];
  // the small rule tables in LDS (read at every node; global loads there
  // would put a cache round trip into each node's dependency chain):
  // near-rule x, y, w [nn]; Gauss-Legendre s, w [nl]; radial r, a, b [nr];
  // curved radial r, a, b [n_rc]
  extern __shared__ double rule_tabs[];
  double* const s_nx = rule_tabs;
  double* const s_ny = s_nx + a.nn;
  double* const s_nw = s_ny + a.nn;
  double* const s_gs = s_nw + a.nn;
  double* const s_gw = s_gs + a.nl;
  double* const s_rr = s_gw + a.nl;
  double* const s_ra = s_rr + a.nr;
  double* const s_rb = s_ra + a.nr;
  double* const s_cr = s_rb + a.nr;
  double* const s_ca = s_cr + a.n_rc;
  double* const s_cb = s_ca + a.n_rc;
  const int lane = threadIdx.x;
  for (int i = lane; i <= kLogTab; i += kWave) tab[i] = a.logtab[i];
  for (int i = lane; i < a.nn; i += kWave) {
    s_nx[i] = a.near_x[i];
    s_ny[i] = a.near_y[i];
    s_nw[i] = a.near_w[i];
  }
  for (int i = lane; i < a.nl; i += kWave) {
    s_gs[i] = a.gl_s[i];
    s_gw[i] = a.gl_w[i];
  }
  for (int i = lane; i < a.nr; i += kWave) {
    s_rr[i] = a.rad_r[i];
    s_ra[i] = a.rad_a[i];
    s_rb[i] = a.rad_b[i];
  }
  for (int i = lane; i < a.n_rc; i += kWave) {
    s_cr[i] = a.rad_c_r[i];
    s_ca[i] = a.rad_c_a[i];
    s_cb[i] = a.rad_c_b[i];
  }
  __syncthreads();
  // this workgroup's diagnostics (near leaves, self panels, capped leaves,
  // depth-first pairs), added to the device counters once at the end: one
  // atomic per pair on shared counters serialises the whole launch
  int64_t tot_leaves = 0, tot_panels = 0, tot_capped = 0, tot_df = 0;
  for (int64_t pr = blockIdx.x; pr < a.n_pairs; pr += gridDim.x) {
  const int32_t t = a.pair_tri[pr];
  const int32_t it = a.pair_tgt[pr];
  const int kind = a.pair_kind[pr];
  if ((KIND == 1 && kind != 1) || (KIND == 2 && kind == 1)) continue;  // the whole workgroup
  const double x = a.xt[it], y = a.yt[it];
  const double Ax = a.ax[t], Ay = a.ay[t], Bx = a.bx[t], By = a.by[t], Cx = a.cx[t], Cy = a.cy[t];
  const double D = a.det[t];
  const double e1x = Bx - Ax, e1y = By - Ay, e2x = Cx - Ax, e2y = Cy - Ay;
  const double invD = 1.0 / D;
  const int cvi = (kCurved && a.cv.of) ? a.cv.of[t] : -1;  // curve of a curved triangle, -1 if straight
  const double* cf = (kCurved && cvi >= 0) ? a.cv.coef + (size_t)cvi * 4 * kCurveMax : nullptr;
  // image of a reference point (the vertex B, where u = 0, maps to B)
  auto map_vertex = [&](double r1, double r2, double& qx, double& qy) {
    if (r1 >= 1.0) {
      qx = Bx;
      qy = By;
    } else {
      vp_blend(Ax, Ay, Bx, By, Cx, Cy, cf, a.cv.deg, r1, r2, qx, qy);
    }
  };
  // the split test of a curved sub-triangle (sa, sb, ss): ellipses of its
  // mapped vertices (edges as chords) with the level's rho, or the ball
  auto curved_split = [&](double sa, double sb, double ss, const double* rho) {
    double qx[3], qy[3];
    map_vertex(sa, sb, qx[0], qy[0]);
    map_vertex(sa + ss, sb, qx[1], qy[1]);
    map_vertex(sa, sb + ss, qx[2], qy[2]);
    if (a.ball) return in_ball3(x, y, qx, qy, a.ball_factor);
    bool sp = false;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int f2 = (e + 1) % 3;
      if (!(rho[e] > 1.0)) continue;
      const double ell = sqrt((qx[f2] - qx[e]) * (qx[f2] - qx[e]) + (qy[f2] - qy[e]) * (qy[f2] - qy[e]));
      const double fs = sqrt((x - qx[e]) * (x - qx[e]) + (y - qy[e]) * (y - qy[e])) +
                        sqrt((x - qx[f2]) * (x - qx[f2]) + (y - qy[f2]) * (y - qy[f2]));
      if (fs < 0.5 * ell * (rho[e] + 1.0 / rho[e])) sp = true;
    }
    return sp;
  };

  double acc[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = 0.0;

  // ---- B: the far rule's own contribution (subtracted) ----
  auto add_far_rule = [&]() {
    for (int j = lane; j < a.nf; j += kWave) {
      // the far sums' sources and expression, so that a pair at r = 0 cancels
      const double2 sj = a.sxy[(int64_t)t * a.nf + j];
      const double dx = x - sj.x, dy = y - sj.y;
      const double r2 = fma(dy, dy, fma(dx, dx, kR2Bias));
      const double w = -0.5 * vp_log(r2, tab) * a.swj[(int64_t)t * a.nf + j];
      const double* E = a.efar + (size_t)j * NP;
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] = fma(w, E[k], acc[k]);
    }
  };
  add_far_rule();

  int64_t n_leaves = 0, n_panels = 0, n_capped = 0;
  if (KIND == 1 || (KIND == 0 && kind == 1)) {
    // ---- A, near pair: breadth-first subdivision ----
    // The ellipses of a level-L sub-triangle (|s| = 2^-L, area 4^-L of the
    // triangle's) have rho_e = rho0_e 2^(-2L/N_n) and edges l_e 2^-L.
    const double px[3] = {Ax, Bx, Cx}, py[3] = {Ay, By, Cy};
    const double wh[3] = {a.nwhat0, a.nwhat1, a.nwhat2};
    double rho0[3], ell0[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      rho0[e] = pow(wh[e] * a.deff[t] / a.eps_cn, a.inv_near_order);
      const double ex = px[(e + 1) % 3] - px[e], ey = py[(e + 1) % 3] - py[e];
      ell0[e] = sqrt(ex * ex + ey * ey);
    }
    double* cur = lv[0];
    double* nxt = lv[1];
    if (lane == 0) {
      cur[0] = 0.0;
      cur[1] = 0.0;
      cur[2] = 1.0;
    }
    __syncthreads();
    int n_cur = 1;
    bool overflow = false;
    for (int level = 0; n_cur > 0; ++level) {
      int n_next = 0, n_leaf = 0;
      double thr[3];
      const double f = exp2(-2.0 * level * a.inv_near_order);
      {
        const double hl = ldexp(0.5, -level);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const double rho = rho0[e] * f;
          thr[e] = (rho > 1.0) ? hl * ell0[e] * (rho + 1.0 / rho) : -1.0;
        }
      }
      for (int base = 0; base < n_cur; base += kWave) {
        const int i = base + lane;
        bool valid = i < n_cur;
        double sa = 0.0, sb = 0.0, ss = 0.0;
        bool split = false;
        if (valid && cf) {
          sa = cur[3 * i];
          sb = cur[3 * i + 1];
          ss = cur[3 * i + 2];
          double rho[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) rho[e] = rho0[e] * f;
          split = (level < a.depth_cap) && curved_split(sa, sb, ss, rho);
        } else if (valid) {
          sa = cur[3 * i];
          sb = cur[3 * i + 1];
          ss = cur[3 * i + 2];
          // physical vertices of the sub-triangle
          const double p0x = Ax + sa * e1x + sb * e2x, p0y = Ay + sa * e1y + sb * e2y;
          const double p1x = p0x + ss * e1x, p1y = p0y + ss * e1y;
          const double p2x = p0x + ss * e2x, p2y = p0y + ss * e2y;
          if (a.ball) {
            split = (level < a.depth_cap) && in_ball_sub(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss,
                                                         a.ball_factor);
          } else {
            const double d0 = sqrt((x - p0x) * (x - p0x) + (y - p0y) * (y - p0y));
            const double d1 = sqrt((x - p1x) * (x - p1x) + (y - p1y) * (y - p1y));
            const double d2 = sqrt((x - p2x) * (x - p2x) + (y - p2y) * (y - p2y));
            split = (level < a.depth_cap) && (d0 + d1 < thr[0] || d1 + d2 < thr[1] || d2 + d0 < thr[2]);
          }
        }
        const bool is_leaf = valid && !split;
        const uint64_t msplit = __ballot(split);
        const uint64_t mleaf = __ballot(is_leaf);
        const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (split) {
          const int o = n_next + 4 * __popcll(msplit & lt);
          if (o + 4 <= kCap) {
            const double h = 0.5 * ss;
            double* c = nxt + 3 * o;
            c[0] = sa;          c[1] = sb;          c[2] = h;
            c[3] = sa + h;      c[4] = sb;          c[5] = h;
            c[6] = sa;          c[7] = sb + h;      c[8] = h;
            c[9] = sa + h;      c[10] = sb + h;     c[11] = -h;
          }
        }
        if (is_leaf) {
          const int o = n_leaf + __popcll(mleaf & lt);
          if (o < kCap) {
            leaf[3 * o] = sa;
            leaf[3 * o + 1] = sb;
            leaf[3 * o + 2] = ss;
          }
        }
        n_next += 4 * __popcll(msplit);
        n_leaf += __popcll(mleaf);
      }
      if (level >= a.depth_cap) n_capped += n_leaf;
      if (n_next > kCap || n_leaf > kCap) {  // a level too wide: redo depth-first below
        overflow = true;
        __syncthreads();
        break;
      }
      __syncthreads();
      n_leaves += n_leaf;
      // integrate this level's leaves with the near rule
      const int items = n_leaf * a.nn;
      for (int item = lane; item < items; item += kWave) {
        const int l = item / a.nn, nd = item - l * a.nn;
        const double sa = leaf[3 * l], sb = leaf[3 * l + 1], ss = leaf[3 * l + 2];
        const double xi1 = sa + ss * s_nx[nd], xi2 = sb + ss * s_ny[nd];
        double yx, yy, jac = D;
        if (cf) {
          jac = vp_blend_jac(Ax, Ay, Bx, By, Cx, Cy, cf, a.cv.deg, xi1, xi2, yx, yy);
        } else {
          yx = Ax + xi1 * e1x + xi2 * e2x;
          yy = Ay + xi1 * e1y + xi2 * e2y;
        }
        const double dx = x - yx, dy = y - yy;
        const double w = 0.5 * vp_log(dx * dx + dy * dy, tab) * s_nw[nd] * ss * ss * jac;
        koornwinder_acc<P>(xi1, xi2, w, acc);
      }
      __syncthreads();
      double* sw = cur;
      cur = nxt;
      nxt = sw;
      n_cur = n_next;
    }
    if (overflow) {
      ++tot_df;
      // Depth-first walk of the same subdivision, one sub-triangle at a
      // time (lanes share its near-rule nodes); the stack holds at most
      // 3 depth_cap + 1 entries, within the two level buffers.
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] = 0.0;
      n_leaves = 0;
      n_capped = 0;
      add_far_rule();
      double* stk = &lv[0][0];
      constexpr int kStack = 2 * kCap;
      if (lane == 0) {
        stk[0] = 0.0;
        stk[1] = 0.0;
        stk[2] = 1.0;
      }
      __syncthreads();
      int sp = 1;
      while (sp > 0) {
        --sp;
        const double sa = stk[3 * sp], sb = stk[3 * sp + 1], ss = stk[3 * sp + 2];
        __syncthreads();
        const int level = -ilogb(fabs(ss));
        const double f = exp2(-2.0 * level * a.inv_near_order);
        const double hl = ldexp(0.5, -level);
        bool split = false;
        if (level < a.depth_cap && cf) {
          double rho[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) rho[e] = rho0[e] * f;
          split = curved_split(sa, sb, ss, rho);
        } else if (level < a.depth_cap && a.ball) {
          split = in_ball_sub(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss, a.ball_factor);
        } else if (level < a.depth_cap) {
          const double p0x = Ax + sa * e1x + sb * e2x, p0y = Ay + sa * e1y + sb * e2y;
          const double p1x = p0x + ss * e1x, p1y = p0y + ss * e1y;
          const double p2x = p0x + ss * e2x, p2y = p0y + ss * e2y;
          const double d0 = sqrt((x - p0x) * (x - p0x) + (y - p0y) * (y - p0y));
          const double d1 = sqrt((x - p1x) * (x - p1x) + (y - p1y) * (y - p1y));
          const double d2 = sqrt((x - p2x) * (x - p2x) + (y - p2y) * (y - p2y));
          const double dd[3] = {d0 + d1, d1 + d2, d2 + d0};
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            const double rho = rho0[e] * f;
            if (rho > 1.0 && dd[e] < hl * ell0[e] * (rho + 1.0 / rho)) split = true;
          }
        }
        if (split) {
          if (sp + 4 > kStack) {
            if (lane == 0) atomicMax(a.flag, 1);
            break;
          }
          if (lane == 0) {
            const double h = 0.5 * ss;
            double* c = stk + 3 * sp;
            c[0] = sa;          c[1] = sb;          c[2] = h;
            c[3] = sa + h;      c[4] = sb;          c[5] = h;
            c[6] = sa;          c[7] = sb + h;      c[8] = h;
            c[9] = sa + h;      c[10] = sb + h;     c[11] = -h;
          }
          sp += 4;
          __syncthreads();
        } else {
          ++n_leaves;
          if (level >= a.depth_cap) ++n_capped;
          for (int nd = lane; nd < a.nn; nd += kWave) {
            const double xi1 = sa + ss * s_nx[nd], xi2 = sb + ss * s_ny[nd];
            double yx, yy, jac = D;
            if (cf) {
              jac = vp_blend_jac(Ax, Ay, Bx, By, Cx, Cy, cf, a.cv.deg, xi1, xi2, yx, yy);
            } else {
              yx = Ax + xi1 * e1x + xi2 * e2x;
              yy = Ay + xi1 * e1y + xi2 * e2y;
            }
            const double dx = x - yx, dy = y - yy;
            const double w = 0.5 * vp_log(dx * dx + dy * dy, tab) * s_nw[nd] * ss * ss * jac;
            koornwinder_acc<P>(xi1, xi2, w, acc);
          }
        }
      }
      __syncthreads();
    }
  } else {
    // ---- A, self pair: three pieces in radius-arc-length coordinates ----
    if (cf) {
      // curved triangle: the same construction in the reference simplex about
      // z = rho^{-1}(x); log|rho(y) - x| = log r + log(|rho(y) - x| / r), the
      // radial rule's log-weight nodes take log r, its Gauss-Legendre nodes
      // the smooth remainder; weights times |J|
      double z1, z2;
      if (!vp_blend_inverse(Ax, Ay, Bx, By, Cx, Cy, D, cf, a.cv.deg, x, y, z1, z2)) {
        if (lane == 0) atomicMax(a.flag, 2);
        z1 = z2 = 1.0 / 3.0;  // keeps the loops bounded; the plan reports the failure
      }
      const double rvx[3] = {0.0, 1.0, 0.0}, rvy[3] = {0.0, 0.0, 1.0};
      const int per_panel = a.nl * a.n_rc;
      for (int side = 0; side < 3; ++side) {
        const double Px = rvx[side], Py = rvy[side], Qx = rvx[(side + 1) % 3], Qy = rvy[(side + 1) % 3];
        const double sub = 0.5 * fabs((Px - z1) * (Qy - z2) - (Py - z2) * (Qx - z1));
        if (sub <= a.tau * 0.5) continue;
        const double L = sqrt((Qx - Px) * (Qx - Px) + (Qy - Py) * (Qy - Py));
        const double ux = (Qx - Px) / L, uy = (Qy - Py) / L;
        const double h = fabs((Px - z1) * (Qy - Py) - (Py - z2) * (Qx - Px)) / L;
        const double st = fmin(fmax((z1 - Px) * ux + (z2 - Py) * uy, 0.0), L);
        const double fx = Px + st * ux, fy = Py + st * uy;
        const double d = sqrt((z1 - fx) * (z1 - fx) + (z2 - fy) * (z2 - fy));
        const double rest = L - st;
        const int n1 = (st > 0.0) ? dyadic_count(st, d, a.dyadic_cap) : -1;
        const int n2 = (rest > 0.0) ? dyadic_count(rest, d, a.dyadic_cap) : -1;
        const int nleft = n1 + 1, nright = n2 + 1;
        const int np = nleft + nright;
        n_panels += np;
        const int items = np * per_panel;
        for (int item = lane; item < items; item += kWave) {
          const int ip = item / per_panel;
          const int rem = item - ip * per_panel;
          const int il = rem / a.n_rc, ir = rem - il * a.n_rc;
          double s0, s1;
          if (ip < nleft) {
            if (ip < n1) {
              s0 = (1.0 - ldexp(1.0, -ip)) * st;
              s1 = (1.0 - ldexp(1.0, -(ip + 1))) * st;
            } else {
              s0 = (1.0 - ldexp(1.0, -n1)) * st;
              s1 = st;
            }
          } else {
            const int jp = ip - nleft;
            if (jp < n2) {
              s0 = L - (1.0 - ldexp(1.0, -(jp + 1))) * rest;
              s1 = L - (1.0 - ldexp(1.0, -jp)) * rest;
            } else {
              s0 = st;
              s1 = L - (1.0 - ldexp(1.0, -n2)) * rest;
            }
          }
          const double sv = s0 + (s1 - s0) * s_gs[il];
          const double ws = (s1 - s0) * s_gw[il];
          const double gx = Px + sv * ux, gy = Py + sv * uy;
          const double rr = s_cr[ir];
          const double yr1 = z1 + rr * (gx - z1), yr2 = z2 + rr * (gy - z2);
          double qx, qy;
          const double jac = vp_blend_jac(Ax, Ay, Bx, By, Cx, Cy, cf, a.cv.deg, yr1, yr2, qx, qy);
          const double lam = 0.5 * vp_log((qx - x) * (qx - x) + (qy - y) * (qy - y), tab) - vp_log(rr, tab);
          const double w = h * ws * (s_ca[ir] * lam + s_cb[ir]) * jac;
          koornwinder_acc<P>(yr1, yr2, w, acc);
        }
      }
    } else {
    const double area = 0.5 * D;
    const double vx[3] = {Ax, Bx, Cx}, vy[3] = {Ay, By, Cy};
    for (int side = 0; side < 3; ++side) {
      const double Px = vx[side], Py = vy[side], Qx = vx[(side + 1) % 3], Qy = vy[(side + 1) % 3];
      const double sub = 0.5 * fabs((Px - x) * (Qy - y) - (Py - y) * (Qx - x));
      if (sub <= a.tau * area) continue;
      const double L = sqrt((Qx - Px) * (Qx - Px) + (Qy - Py) * (Qy - Py));
      const double ux = (Qx - Px) / L, uy = (Qy - Py) / L;
      const double h = fabs((Px - x) * (Qy - Py) - (Py - y) * (Qx - Px)) / L;
      const double st = fmin(fmax((x - Px) * ux + (y - Py) * uy, 0.0), L);
      const double fx = Px + st * ux, fy = Py + st * uy;
      const double d = sqrt((x - fx) * (x - fx) + (y - fy) * (y - fy));
      const double rest = L - st;
      const int n1 = (st > 0.0) ? dyadic_count(st, d, a.dyadic_cap) : -1;
      const int n2 = (rest > 0.0) ? dyadic_count(rest, d, a.dyadic_cap) : -1;
      const int nleft = n1 + 1, nright = n2 + 1;  // panels per side (0 if empty)
      const int np = nleft + nright;
      n_panels += np;
      // lanes over (panel, arc node); the radial nodes of the ray share the
      // ray's arc position and its log r0 term
      const int items = np * a.nl;
      for (int item = lane; item < items; item += kWave) {
        const int ip = item / a.nl;
        const int il = item - ip * a.nl;
        double s0, s1;
        if (ip < nleft) {
          if (ip < n1) {
            s0 = (1.0 - ldexp(1.0, -ip)) * st;
            s1 = (1.0 - ldexp(1.0, -(ip + 1))) * st;
          } else {
            s0 = (1.0 - ldexp(1.0, -n1)) * st;
            s1 = st;
          }
        } else {
          const int jp = ip - nleft;
          if (jp < n2) {
            s0 = L - (1.0 - ldexp(1.0, -(jp + 1))) * rest;
            s1 = L - (1.0 - ldexp(1.0, -jp)) * rest;
          } else {
            s0 = st;
            s1 = L - (1.0 - ldexp(1.0, -n2)) * rest;
          }
        }
        const double s = s0 + (s1 - s0) * s_gs[il];
        const double hws = h * (s1 - s0) * s_gw[il];
        const double gx = Px + s * ux, gy = Py + s * uy;
        const double r0sq = (gx - x) * (gx - x) + (gy - y) * (gy - y);
        const double hlog = 0.5 * vp_log(r0sq, tab);
        // the ray from x to g in reference coordinates
        const double ox = x - Ax, oy = y - Ay, gdx = gx - x, gdy = gy - y;
        const double z1 = (ox * e2y - oy * e2x) * invD, z2 = (e1x * oy - e1y * ox) * invD;
        const double d1 = (gdx * e2y - gdy * e2x) * invD, d2 = (e1x * gdy - e1y * gdx) * invD;
        for (int ir = 0; ir < a.nr; ++ir) {
          const double rr = s_rr[ir];
          const double w = hws * fma(s_ra[ir], hlog, s_rb[ir]);
          koornwinder_acc<P>(fma(rr, d1, z1), fma(rr, d2, z2), w, acc);
        }
      }
    }
    }  // straight self pair
  }

  // ---- wave reduction and store ----
  double* out = a.rows + (size_t)pr * NP;
  {
    int base = 0, len = NP;
    ReduceScatter<NP, 32>::run(acc, lane, base, len);
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (i < len) out[base + i] = acc[i] * kInv2Pi;
  }
  tot_leaves += n_leaves;
  tot_panels += n_panels;
  tot_capped += n_capped;
  __syncthreads();
  }  // pair loop
  if (lane == 0) {
    // spread over kRowStatSlots cache lines (summed on the host)
    unsigned long long* st = (unsigned long long*)(a.stats + (int64_t)(blockIdx.x & (kRowStatSlots - 1)) * kRowStatStride);
    if (tot_leaves) atomicAdd(st + 0, (unsigned long long)tot_leaves);
    if (tot_panels) atomicAdd(st + 1, (unsigned long long)tot_panels);
    if (tot_capped) atomicAdd(st + 2, (unsigned long long)tot_capped);
    if (tot_df) atomicAdd(st + 3, (unsigned long long)tot_df);
  }
}

}  // namespace

hipError_t launch_rows(vp_plan* pl, int* d_flag, int64_t* d_stats, hipStream_t st) {
  if (pl->n_pairs == 0) return hipSuccess;
  const vp_mesh* m = pl->mesh;
  RowsArgs a;
  a.pair_tri = pl->pair_tri;
  a.pair_tgt = pl->pair_tgt;
  a.pair_kind = pl->pair_kind;
  a.n_pairs = pl->n_pairs;
  a.xt = pl->xt;
  a.yt = pl->yt;
  a.ax = m->ax;
  a.ay = m->ay;
  a.bx = m->bx;
  a.by = m->by;
  a.cx = m->cx;
  a.cy = m->cy;
  a.det = m->det;
  a.far_x = pl->far_x;
  a.far_y = pl->far_y;
  a.far_w = pl->far_w;
  a.efar = pl->efar;
  a.nf = pl->n_f;
  a.near_x = pl->near_x;
  a.near_y = pl->near_y;
  a.near_w = pl->near_w;
  a.nn = pl->opts.q_near * pl->opts.q_near;
  a.nwhat0 = pl->near_what[0];
  a.nwhat1 = pl->near_what[1];
  a.nwhat2 = pl->near_what[2];
  a.inv_near_order = 1.0 / (2.0 * pl->opts.q_near - 1.0);
  a.gl_s = pl->gl_s;
  a.gl_w = pl->gl_w;
  a.nl = pl->opts.n_l;
  a.rad_r = pl->rad_r;
  a.rad_a = pl->rad_a;
  a.rad_b = pl->rad_b;
  a.nr = pl->n_r;
  a.eps_cn = pl->eps * pl->opts.c_n;
  a.tau = pl->opts.tau;
  a.depth_cap = pl->opts.depth_cap;
  a.ball = pl->opts.near_model == VP_NEAR_BALL ? 1 : 0;
  a.ball_factor = pl->opts.ball_factor;
  a.dyadic_cap = pl->opts.dyadic_cap;
  a.logtab = pl->logtab;
  a.sxy = pl->sxy;
  a.swj = pl->swj;
  a.deff = pl->deff;
  a.cv = m->curves();
  a.rad_c_r = pl->rad_c_r;
  a.rad_c_a = pl->rad_c_a;
  a.rad_c_b = pl->rad_c_b;
  a.n_rc = pl->n_rc;
  a.rows = pl->rows;
  a.flag = d_flag;
  a.stats = d_stats;
  // one 64-lane workgroup per 8 pairs (strided over the pair list), so that
  // the tables a workgroup stages in LDS serve several pairs while the
  // dispatcher still balances workgroups of uneven cost; grid-stride beyond
  // 2^25 workgroups (a launch must stay below 2^32 work-items).  A single
  // device-wide work counter instead serialises on its atomic across the XCDs.
  constexpr int64_t kPairsPerGroup = 8;
  dim3 grid((unsigned)std::min<int64_t>((pl->n_pairs + kPairsPerGroup - 1) / kPairsPerGroup, 1 << 25));
  const bool curved = m->n_curved > 0;
  const size_t lds = sizeof(double) * (3 * (size_t)a.nn + 2 * (size_t)a.nl + 3 * (size_t)a.nr + 3 * (size_t)a.n_rc);
  // Straight meshes with many self pairs (a quarter or more: fine far rules,
  // where few targets have near pairs) at tight tolerances (deep near
  // subdivisions) run near and self pairs as two launches, each sized to its
  // pairs.  Measured on the star: q = 16 at eps = 1e-13 (37% self pairs) 8%
  // faster apart; q = 8 at eps = 1e-13 (13%) and at eps = 1e-8 (46%, shallow
  // near subdivisions) 8-10% faster in one launch.
  const int64_t n_near = pl->n_pairs - pl->n_self;
  const bool split =
      !curved && pl->n_self > 0 && n_near > 0 && 4 * pl->n_self >= pl->n_pairs && pl->eps <= 1e-10;
  auto groups = [&](int64_t n) {
    return dim3((unsigned)std::min<int64_t>((n + kPairsPerGroup - 1) / kPairsPerGroup, 1 << 25));
  };
#define VP_ROWS(PV)                                                   \
  case PV:                                                            \
    if (curved) {                                                     \
      k_rows<PV, true, 0><<<grid, 64, lds, st>>>(a);                  \
    } else if (split) {                                               \
      k_rows<PV, false, 1><<<groups(n_near), 64, lds, st>>>(a);       \
      k_rows<PV, false, 2><<<groups(pl->n_self), 64, lds, st>>>(a);   \
    } else {                                                          \
      k_rows<PV, false, 0><<<grid, 64, lds, st>>>(a);                 \
    }                                                                 \
    break
  switch (pl->p) {
    VP_ROWS(1);
    VP_ROWS(2);
    VP_ROWS(3);
    VP_ROWS(4);
    VP_ROWS(5);
    VP_ROWS(6);
    VP_ROWS(7);
    VP_ROWS(8);
    VP_ROWS(9);
    VP_ROWS(10);
    default: return hipErrorInvalidValue;
  }
#undef VP_ROWS
  return hipGetLastError();
}

}  // namespace vp
