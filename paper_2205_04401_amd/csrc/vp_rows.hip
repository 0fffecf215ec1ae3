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
  const uint32_t* list;  // pairs to compute (n_list of them), or null for all n_pairs
  int64_t n_list;
  const double *xt, *yt;
  const double *ax, *ay, *bx, *by, *cx, *cy, *det;
  const double4* geo;  // the same, packed per triangle
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
  const double* basis_g;  // basis_row's coefficients (orders <= kBasisLegMax)
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

// Focal-sum thresholds of the three near-rule ellipses of a level-L
// sub-triangle (|s| = 2^-L): rho_e = rho0_e 2^(-2L/N_n), edges l_e 2^-L;
// negative for an empty ellipse (rho <= 1).
__device__ __forceinline__ void near_level_thr(const double rho0[3], const double ell0[3], int level,
                                               double inv_near_order, double thr[3]) {
  const double f = exp2(-2.0 * level * inv_near_order);
  const double hl = ldexp(0.5, -level);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const double rho = rho0[e] * f;
    thr[e] = (rho > 1.0) ? hl * ell0[e] * (rho + 1.0 / rho) : -1.0;
  }
}

// True if the target lies in one of the three ellipses of the straight
// sub-triangle (sa, sb, ss) of the triangle A + xi1 e1 + xi2 e2.
__device__ __forceinline__ bool near_sub_split(double x, double y, double Ax, double Ay, double e1x, double e1y,
                                               double e2x, double e2y, double sa, double sb, double ss,
                                               const double thr[3]) {
  const double p0x = Ax + sa * e1x + sb * e2x, p0y = Ay + sa * e1y + sb * e2y;
  const double p1x = p0x + ss * e1x, p1y = p0y + ss * e1y;
  const double p2x = p0x + ss * e2x, p2y = p0y + ss * e2y;
  const double d0 = sqrt((x - p0x) * (x - p0x) + (y - p0y) * (y - p0y));
  const double d1 = sqrt((x - p1x) * (x - p1x) + (y - p1y) * (y - p1y));
  const double d2 = sqrt((x - p2x) * (x - p2x) + (y - p2y) * (y - p2y));
  return d0 + d1 < thr[0] || d1 + d2 < thr[1] || d2 + d0 < thr[2];
}

// rho0 and edge lengths of the near rule's ellipses for a straight triangle
__device__ __forceinline__ void near_root(double Ax, double Ay, double Bx, double By, double Cx, double Cy,
                                          double deff, const double wh[3], double eps_cn, double inv_near_order,
                                          double rho0[3], double ell0[3]) {
  const double px[3] = {Ax, Bx, Cx}, py[3] = {Ay, By, Cy};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    rho0[e] = pow(wh[e] * deff / eps_cn, inv_near_order);
    const double ex = px[(e + 1) % 3] - px[e], ey = py[(e + 1) % 3] - py[e];
    ell0[e] = sqrt(ex * ex + ey * ey);
  }
}

// A pair's row from the reduced sums (lane holds acc[0 .. len) at base):
// Koornwinder sums stored as they are; the product basis's sums (orders up
// to kBasisLegMax) pass through sb (LDS, n_p doubles of the one-wavefront
// workgroup) and basis_row
template <int P>
__device__ __forceinline__ void store_row(const double* acc, int base, int len, int lane, double* sb,
                                          const double* __restrict__ g, double* out) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  if constexpr (P <= kBasisLegMax) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (i < len) sb[base + i] = acc[i];
    __syncthreads();
    if (lane < NP) out[lane] = basis_row<P>(sb, g, lane) * kInv2Pi;
    __syncthreads();
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (i < len) out[base + i] = acc[i] * kInv2Pi;
  }
}

// kCurved: the mesh has curved triangles (the straight-only instance carries
// none of their code).  KIND: 0 every pair, 1 near pairs only, 2 self pairs
// only (each of the two then carries only its own branch, with fewer live
// registers than both together)
template <int P, bool kCurved, int KIND>
__global__ __launch_bounds__(64) void k_rows(RowsArgs a) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  __shared__ double lv[2][kCap * 3];
  __shared__ double leaf[kCap * 3];
  __shared__ double2 tab[kLogTab + 1];
  __shared__ double sb[NP];  // store_row
  __shared__ double4 piece_d[3][2];  // straight self pair: its three pieces' parameters
  __shared__ int2 piece_i[3];
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
  const int64_t n_work = a.list ? a.n_list : a.n_pairs;
  for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
  const int64_t pr = a.list ? (int64_t)a.list[wi] : wi;
  const int32_t t = a.pair_tri[pr];
  const int32_t it = a.pair_tgt[pr];
  const int kind = a.pair_kind[pr];
  if ((KIND == 1 && kind != 1) || (KIND == 2 && kind == 1)) continue;  // the whole workgroup
  const double x = a.xt[it], y = a.yt[it];
  const TriGeo tg = tri_geo(a.geo, t);
  const double Ax = tg.ax, Ay = tg.ay, Bx = tg.bx, By = tg.by, Cx = tg.cx, Cy = tg.cy;
  const double D = tg.det;
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
      basis_acc<P>(a.far_x[j], a.far_y[j], w, acc);
    }
  };
  add_far_rule();

  int64_t n_leaves = 0, n_panels = 0, n_capped = 0;
  if (KIND == 1 || (KIND == 0 && kind == 1)) {
    // ---- A, near pair: breadth-first subdivision ----
    // The ellipses of a level-L sub-triangle (|s| = 2^-L, area 4^-L of the
    // triangle's) have rho_e = rho0_e 2^(-2L/N_n) and edges l_e 2^-L.
    const double wh[3] = {a.nwhat0, a.nwhat1, a.nwhat2};
    double rho0[3], ell0[3];
    near_root(Ax, Ay, Bx, By, Cx, Cy, a.deff[t], wh, a.eps_cn, a.inv_near_order, rho0, ell0);
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
      near_level_thr(rho0, ell0, level, a.inv_near_order, thr);
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
          if (a.ball) {
            split = (level < a.depth_cap) && in_ball_sub(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss,
                                                         a.ball_factor);
          } else {
            split = (level < a.depth_cap) && near_sub_split(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss, thr);
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
        basis_acc<P>(xi1, xi2, w, acc);
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
        bool split = false;
        if (level < a.depth_cap && cf) {
          double rho[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) rho[e] = rho0[e] * f;
          split = curved_split(sa, sb, ss, rho);
        } else if (level < a.depth_cap && a.ball) {
          split = in_ball_sub(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss, a.ball_factor);
        } else if (level < a.depth_cap) {
          double thr[3];
          near_level_thr(rho0, ell0, level, a.inv_near_order, thr);
          split = near_sub_split(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss, thr);
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
            basis_acc<P>(xi1, xi2, w, acc);
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
          basis_acc<P>(yr1, yr2, w, acc);
        }
      }
    } else {
    const double area = 0.5 * D;
    const double vx[3] = {Ax, Bx, Cx}, vy[3] = {Ay, By, Cy};
    // the target in reference coordinates: the apex of every ray, the
    // radial rule's node r = 0 (s_rr[0] = 0), whose weights the lanes sum
    // and whose basis values join once per pair
    const double ox = x - Ax, oy = y - Ay;
    const double z1 = (ox * e2y - oy * e2x) * invD, z2 = (e1x * oy - e1y * ox) * invD;
    double w_apex = 0.0;
    // The three pieces' parameters first (the same in every lane; lane 0
    // keeps them in LDS), then one flat loop over every (piece, panel, arc
    // node) of the pair, so that the lanes stay full across the pieces:
    // per piece its start P, direction u, height h, foot position st,
    // length L, L - st, and the dyadic panel counts n1, n2.
    int off1 = 0, off2 = 0, n_items = 0;
    for (int side = 0; side < 3; ++side) {
      const double Px = vx[side], Py = vy[side], Qx = vx[(side + 1) % 3], Qy = vy[(side + 1) % 3];
      const double sub = 0.5 * fabs((Px - x) * (Qy - y) - (Py - y) * (Qx - x));
      int np = 0;
      if (sub > a.tau * area) {
        const double L = sqrt((Qx - Px) * (Qx - Px) + (Qy - Py) * (Qy - Py));
        const double ux = (Qx - Px) / L, uy = (Qy - Py) / L;
        const double h = fabs((Px - x) * (Qy - Py) - (Py - y) * (Qx - Px)) / L;
        const double st = fmin(fmax((x - Px) * ux + (y - Py) * uy, 0.0), L);
        const double fx = Px + st * ux, fy = Py + st * uy;
        const double d = sqrt((x - fx) * (x - fx) + (y - fy) * (y - fy));
        const double rest = L - st;
        const int n1 = (st > 0.0) ? dyadic_count(st, d, a.dyadic_cap) : -1;
        const int n2 = (rest > 0.0) ? dyadic_count(rest, d, a.dyadic_cap) : -1;
        np = (n1 + 1) + (n2 + 1);  // panels toward the foot and beyond it (0 if empty)
        if (lane == 0) {
          piece_d[side][0] = make_double4(Px, Py, ux, uy);
          piece_d[side][1] = make_double4(h, st, L, rest);
          piece_i[side] = make_int2(n1, n2);
        }
      }
      n_panels += np;
      if (side == 0) off1 = np * a.nl;
      if (side == 1) off2 = off1 + np * a.nl;
      if (side == 2) n_items = off2 + np * a.nl;
    }
    __syncthreads();
    // lanes over (piece, panel, arc node); the radial nodes of the ray share
    // the ray's arc position and its log r0 term
    for (int item = lane; item < n_items; item += kWave) {
      const int side = item >= off2 ? 2 : (item >= off1 ? 1 : 0);
      const int rel = item - (side == 2 ? off2 : (side == 1 ? off1 : 0));
      const int ip = rel / a.nl;
      const int il = rel - ip * a.nl;
      const double4 pa = piece_d[side][0], pb = piece_d[side][1];
      const int2 pn = piece_i[side];
      const double Px = pa.x, Py = pa.y, ux = pa.z, uy = pa.w;
      const double h = pb.x, st = pb.y, L = pb.z, rest = pb.w;
      const int n1 = pn.x, n2 = pn.y, nleft = n1 + 1;
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
      const double gdx = gx - x, gdy = gy - y;
      const double d1 = (gdx * e2y - gdy * e2x) * invD, d2 = (e1x * gdy - e1y * gdx) * invD;
      w_apex = fma(hws, fma(s_ra[0], hlog, s_rb[0]), w_apex);
      for (int ir = 1; ir < a.nr; ++ir) {
        const double rr = s_rr[ir];
        const double w = hws * fma(s_ra[ir], hlog, s_rb[ir]);
        basis_acc<P>(fma(rr, d1, z1), fma(rr, d2, z2), w, acc);
      }
    }
    basis_acc<P>(z1, z2, w_apex, acc);
    }  // straight self pair
  }

  // ---- wave reduction and store ----
  double* out = a.rows + (size_t)pr * NP;
  {
    int base = 0, len = NP;
    ReduceScatter<NP, 32>::run(acc, lane, base, len);
    store_row<P>(acc, base, len, lane, sb, a.basis_g, out);
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

// ---------------------------------------------------------------------------
// Deeper near pairs (subdivision two or more levels deep) of straight
// triangles with the ellipse test.
//
// The same subdivision as k_rows, walked level by level with the lanes
// testing a level's sub-triangles, but the leaves of every level are only
// collected (in LDS) during the walk and integrated afterwards in one flat
// loop whose items are the far rule's own nodes (B, subtracted) and the
// (leaf, near-rule node) pairs (A): each lane takes every 64th item and adds
// its weighted logarithm times the Koornwinder basis at the item's reference
// point.  Against k_rows' integration after each level this keeps the lanes
// full over the whole pair (a deep pair has about 12 leaves of 49 nodes,
// spread over 2 to 9 levels), drops a barrier per level, and leaves out the
// self-pair, curved and depth-first code, so that fewer registers and less
// LDS are live and more wavefronts fit on a SIMD.  The near rule's rho0
// and edge lengths per triangle come from k_near_root.  A pair with a level
// wider than kDeepLv sub-triangles or more than kDeepLeaf leaves (a target
// very close to a sliver's edge) is appended to an overflow list instead;
// k_rows computes those afterwards.
// ---------------------------------------------------------------------------
constexpr int kDeepLv = 64;     // sub-triangles of one level (one per lane)
constexpr int kDeepLeaf = 128;  // leaves of one pair

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int P>
__global__ __launch_bounds__(64) void k_rows_deep(RowsArgs a, const double* __restrict__ nr, int64_t n_tri,
                                                  const uint8_t* __restrict__ cls, uint32_t* __restrict__ ovf,
                                                  uint32_t* __restrict__ n_ovf) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  __shared__ double lv[2][kDeepLv * 3];
  __shared__ double leaf[kDeepLeaf * 3];
  // the logarithm's table through the caches: without its 4 KiB in LDS a
  // fourth wavefront fits on each SIMD (the registers allow four)
  const double2* __restrict__ tab = a.logtab;
  __shared__ double sb[NP];  // store_row
  // near-rule x, y, w [nn]; far-rule x, y [nf]
  extern __shared__ double rule_tabs[];
  double* const s_nx = rule_tabs;
  double* const s_ny = s_nx + a.nn;
  double* const s_nw = s_ny + a.nn;
  double* const s_fx = s_nw + a.nn;
  double* const s_fy = s_fx + a.nf;
  const int lane = threadIdx.x;
  for (int i = lane; i < a.nn; i += kWave) {
    s_nx[i] = a.near_x[i];
    s_ny[i] = a.near_y[i];
    s_nw[i] = a.near_w[i];
  }
  for (int i = lane; i < a.nf; i += kWave) {
    s_fx[i] = a.far_x[i];
    s_fy[i] = a.far_y[i];
  }
  __syncthreads();
  const float inv_nn = 1.0f / (float)a.nn;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t tot_leaves = 0, tot_capped = 0;
  for (int64_t wi = blockIdx.x; wi < a.n_list; wi += gridDim.x) {
    const int64_t pr = (int64_t)a.list[wi];
    const int32_t t = a.pair_tri[pr];
    const int32_t it = a.pair_tgt[pr];
    const int split1 = cls[pr] >> 4;  // level-1 children that split (class pass)
    const double x = a.xt[it], y = a.yt[it];
    const TriGeo tg = tri_geo(a.geo, t);
    const double Ax = tg.ax, Ay = tg.ay;
    const double e1x = tg.bx - Ax, e1y = tg.by - Ay, e2x = tg.cx - Ax, e2y = tg.cy - Ay;
    const double D = tg.det;
    double rho0[3], ell0[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      rho0[e] = nr[16 * (int64_t)t + e];
      ell0[e] = nr[16 * (int64_t)t + 3 + e];
    }
    // the ellipse thresholds of every level at once: lane L holds level L's
    // (the depth cap is at most 60)
    double thr_l[3];
    near_level_thr(rho0, ell0, lane, a.inv_near_order, thr_l);
    // ---- the walk: leaves of every level into leaf[] ----
    // Levels 0 and 1 are known from the class pass: the triangle splits, and
    // of its children (a, s) = ((0,0), 1/2), ((1/2,0), 1/2), ((0,1/2), 1/2),
    // ((1/2,1/2), -1/2) those in split1 split again, the others are leaves.
    double* cur = lv[0];
    double* nxt = lv[1];
    const uint64_t m1 = (uint64_t)split1;
    if (lane < 4) {
      const double sa = (lane == 1 || lane == 3) ? 0.5 : 0.0, sb = (lane >= 2) ? 0.5 : 0.0;
      const double ss = (lane == 3) ? -0.5 : 0.5;
      if ((split1 >> lane) & 1) {
        const double h = 0.5 * ss;
        double* c = cur + 12 * __popcll(m1 & lt);
        c[0] = sa;          c[1] = sb;          c[2] = h;
        c[3] = sa + h;      c[4] = sb;          c[5] = h;
        c[6] = sa;          c[7] = sb + h;      c[8] = h;
        c[9] = sa + h;      c[10] = sb + h;     c[11] = -h;
      } else {
        double* c = leaf + 3 * __popcll(~m1 & 15ull & lt);
        c[0] = sa;
        c[1] = sb;
        c[2] = ss;
      }
    }
    __syncthreads();
    int n_cur = 4 * __popcll(m1), n_leaf = 4 - __popcll(m1), n_capped = 0;
    bool over = false;
    for (int level = 2; n_cur > 0; ++level) {
      double thr[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) thr[e] = readlane_f64(thr_l[e], level);
      const bool valid = lane < n_cur;
      double sa = 0.0, sb = 0.0, ss = 0.0;
      bool split = false;
      if (valid) {
        sa = cur[3 * lane];
        sb = cur[3 * lane + 1];
        ss = cur[3 * lane + 2];
        split = (level < a.depth_cap) && near_sub_split(x, y, Ax, Ay, e1x, e1y, e2x, e2y, sa, sb, ss, thr);
      }
      const bool is_leaf = valid && !split;
      const uint64_t msplit = __ballot(split);
      const uint64_t mleaf = __ballot(is_leaf);
      const int n_next = 4 * __popcll(msplit);
      if (n_next > kDeepLv || n_leaf + __popcll(mleaf) > kDeepLeaf) {
        over = true;
        break;
      }
      if (split) {
        const double h = 0.5 * ss;
        double* c = nxt + 12 * __popcll(msplit & lt);
        c[0] = sa;          c[1] = sb;          c[2] = h;
        c[3] = sa + h;      c[4] = sb;          c[5] = h;
        c[6] = sa;          c[7] = sb + h;      c[8] = h;
        c[9] = sa + h;      c[10] = sb + h;     c[11] = -h;
      }
      if (is_leaf) {
        double* c = leaf + 3 * (n_leaf + __popcll(mleaf & lt));
        c[0] = sa;
        c[1] = sb;
        c[2] = ss;
      }
      if (level >= a.depth_cap) n_capped += __popcll(mleaf);
      n_leaf += __popcll(mleaf);
      n_cur = n_next;
      __syncthreads();
      double* sw = cur;
      cur = nxt;
      nxt = sw;
    }
    if (over) {
      if (lane == 0) ovf[atomicAdd(n_ovf, 1u)] = (uint32_t)pr;
      __syncthreads();
      continue;
    }
    // ---- the integration: far-rule nodes (B) and leaf nodes (A) ----
    double acc[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = 0.0;
    const int items = a.nf + n_leaf * a.nn;
    const double2* sxy = a.sxy + (int64_t)t * a.nf;
    const double* swj = a.swj + (int64_t)t * a.nf;
    for (int item = lane; item < items; item += kWave) {
      double xi1, xi2, r2, wf;
      if (item < a.nf) {
        // the far sums' sources and expression, so that a pair at r = 0 cancels
        const double2 sj = sxy[item];
        const double dx = x - sj.x, dy = y - sj.y;
        r2 = fma(dy, dy, fma(dx, dx, kR2Bias));
        wf = -swj[item];
        xi1 = s_fx[item];
        xi2 = s_fy[item];
      } else {
        const int q = item - a.nf;
        const int l = (int)(((float)q + 0.5f) * inv_nn);
        const int nd = q - l * a.nn;
        const double sa = leaf[3 * l], sb = leaf[3 * l + 1], ss = leaf[3 * l + 2];
        xi1 = sa + ss * s_nx[nd];
        xi2 = sb + ss * s_ny[nd];
        const double dx = x - (Ax + xi1 * e1x + xi2 * e2x), dy = y - (Ay + xi1 * e1y + xi2 * e2y);
        r2 = dx * dx + dy * dy;
        wf = s_nw[nd] * ss * ss * D;
      }
      basis_acc<P>(xi1, xi2, 0.5 * vp_log(r2, tab) * wf, acc);
    }
    double* out = a.rows + (size_t)pr * NP;
    int base = 0, len = NP;
    ReduceScatter<NP, 32>::run(acc, lane, base, len);
    store_row<P>(acc, base, len, lane, sb, a.basis_g, out);
    tot_leaves += n_leaf;
    tot_capped += n_capped;
    __syncthreads();
  }
  if (lane == 0) {
    unsigned long long* st = (unsigned long long*)(a.stats + (int64_t)(blockIdx.x & (kRowStatSlots - 1)) * kRowStatStride);
    if (tot_leaves) atomicAdd(st + 0, (unsigned long long)tot_leaves);
    if (tot_capped) atomicAdd(st + 2, (unsigned long long)tot_capped);
  }
}

// ---------------------------------------------------------------------------
// Shallow near pairs on the matrix cores.
//
// A near pair whose subdivision stops at the triangle itself (depth class 0)
// or after one split into four leaves (class 1) integrates the near rule at
// nodes fixed in the reference simplex, so the Koornwinder values there are
// one table per class: with g_j the weighted logarithm at node j of the far
// rule (subtracted, B) and of the leaves (A), the row is g^T Tab.  Sixteen
// pairs at a time, g is the A operand of v_mfma_f64_16x16x4f64 (lane l: pair
// l & 15, node 4 s + (l >> 4) of step s) and the table the B operand (node
// 4 s + (l >> 4), basis function 16 n + (l & 15)); the lanes evaluate only
// logarithms.  The same holds for a pair whose subdivision splits exactly
// one level-1 child c and stops at that child's four children (class 2 + c:
// three level-1 and four level-2 leaves at fixed places).  The pairs are
// sorted by class first: 0, 1, 2..5, deeper near pairs (6, for k_rows_deep)
// and self pairs (7, for k_rows).
// ---------------------------------------------------------------------------
constexpr int kNCls = 8;
constexpr int kClsDeep = 6, kClsSelf = 7;
constexpr int kClsThreads = 256;
constexpr int kClsPer = 4;                              // pairs per thread
constexpr int kClsChunk = kClsThreads * kClsPer;        // pairs per block
constexpr int kTabNearMax = 64;                         // near-rule nodes of the table path (q_near <= 8)
constexpr int kTabSlotsMax = 2048;                      // slots of one launch's two classes (LDS: 16 bytes each)
constexpr int kTabThreads = 512;                        // 8 wavefronts share one block's LDS tables
constexpr int kTabWaves = kTabThreads / 64;
constexpr size_t kTabLdsBlock = 53248;                  // LDS of one block for 3 blocks (24 wavefronts) per CU
constexpr size_t kTabT0LdsMax = 16384;                  // class 0's Koornwinder table alone in LDS up to this size
constexpr int kTabBlocksPerCu = 12;                     // grid: 4 rounds of 3 resident blocks per CU

struct ClassArgs {
  const int32_t *pair_tri, *pair_tgt;
  const uint8_t* pair_kind;
  int64_t n_pairs, n_blk;
  const double *xt, *yt;
  const double *ax, *ay, *bx, *by, *cx, *cy, *det, *deff;
  const double4* geo;  // the same, packed per triangle
  const double* nr;  // [n_tri][16] near-rule rho0, edge lengths, thresholds of levels 0-2 (k_near_root)
  int64_t n_tri;
  double nwhat0, nwhat1, nwhat2, eps_cn, inv_near_order;
  int depth_cap;
  uint8_t* cls;     // [n_pairs] class of every pair (bits 0..2; bits 4..7: level-1 splits of a deep pair)
  int32_t* bcnt;    // [kNCls][n_blk] pairs of each class per block
  const int64_t* boff;  // [kNCls n_blk + 1] exclusive scan of bcnt (scatter pass)
  uint32_t* list;       // [n_pairs] pair indices sorted by class (scatter pass)
  int2* stt;            // [pairs of classes 0-5] their (triangle, target), in the same order
};

// depth class of near pair pr: the tests of k_rows' first levels; for a
// deep pair (class 6) the bits 4..7 hold which of the four level-1 children
// split.  The tests of levels 0-2 take their focal-sum thresholds from the
// triangle's table (k_near_root) and the target's distance to each vertex of
// the sub-triangles once: the 3 vertices and 3 edge midpoints of the triangle,
// then the 3 edge midpoints of the one child that splits.
__device__ __forceinline__ int pair_class(const ClassArgs& a, int64_t pr) {
  if (a.pair_kind[pr] != 1) return kClsSelf;
  const int32_t t = a.pair_tri[pr];
  const int32_t it = a.pair_tgt[pr];
  const double x = a.xt[it], y = a.yt[it];
  const TriGeo tg = tri_geo(a.geo, t);
  const double Ax = tg.ax, Ay = tg.ay;
  const double e1x = tg.bx - Ax, e1y = tg.by - Ay, e2x = tg.cx - Ax, e2y = tg.cy - Ay;
  const double* thr = a.nr + 16 * (int64_t)t + 6;  // thr[3 L + e]: level L, edge e
  auto T = [&](int level, int e) { return thr[3 * level + e]; };
  // distance from the target to the point (u, v) of the reference simplex
  auto dist = [&](double u, double v) {
    const double px = fma(v, e2x, fma(u, e1x, Ax)), py = fma(v, e2y, fma(u, e1y, Ay));
    return sqrt((x - px) * (x - px) + (y - py) * (y - py));
  };
  // a sub-triangle with vertex distances d0, d1, d2 (edges p0p1, p1p2, p2p0)
  auto split = [&](int level, double d0, double d1, double d2) {
    return d0 + d1 < T(level, 0) || d1 + d2 < T(level, 1) || d2 + d0 < T(level, 2);
  };
  if (!(0 < a.depth_cap)) return 0;
  const double dA = dist(0.0, 0.0), dB = dist(1.0, 0.0), dC = dist(0.0, 1.0);
  if (!split(0, dA, dB, dC)) return 0;
  if (!(1 < a.depth_cap)) return 1;
  const double dAB = dist(0.5, 0.0), dAC = dist(0.0, 0.5), dBC = dist(0.5, 0.5);
  // children (a, s): ((0,0), 1/2), ((1/2,0), 1/2), ((0,1/2), 1/2), ((1/2,1/2), -1/2)
  const int mask = (split(1, dA, dAB, dAC) ? 1 : 0) | (split(1, dAB, dB, dBC) ? 2 : 0) |
                   (split(1, dAC, dBC, dC) ? 4 : 0) | (split(1, dBC, dAC, dAB) ? 8 : 0);
  if (!mask) return 1;
  if (mask & (mask - 1)) return kClsDeep | (mask << 4);
  // one child c splits: class 2 + c if none of its four children splits
  const int c = __ffs(mask) - 1;
  if (2 < a.depth_cap) {
    const double sa = (c == 1 || c == 3) ? 0.5 : 0.0, sb = (c >= 2) ? 0.5 : 0.0, h = (c == 3) ? -0.25 : 0.25;
    // the child's vertices p0 = (sa, sb), p1 = p0 + 2h e1, p2 = p0 + 2h e2
    // and its edge midpoints
    const double q0 = c == 0 ? dA : c == 1 ? dAB : c == 2 ? dAC : dBC;
    const double q1 = c == 0 ? dAB : c == 1 ? dB : c == 2 ? dBC : dAC;
    const double q2 = c == 0 ? dAC : c == 1 ? dBC : c == 2 ? dC : dAB;
    const double m01 = dist(sa + h, sb), m02 = dist(sa, sb + h), m12 = dist(sa + h, sb + h);
    if (split(2, q0, m01, m02) || split(2, m01, q1, m12) || split(2, m02, m12, q2) || split(2, m12, m02, m01))
      return kClsDeep | (mask << 4);
  }
  return 2 + c;
}

// near-rule rho0, edge lengths and the focal-sum thresholds of levels 0-2
// of every triangle, one 128-byte line each: nr[T][e] = rho0_e, nr[T][3 + e]
// = l_e (the values k_rows computes for each pair), nr[T][6 + 3 L + e] =
// threshold of edge e at level L
__global__ void k_near_root(const double* __restrict__ ax, const double* __restrict__ ay,
                            const double* __restrict__ bx, const double* __restrict__ by,
                            const double* __restrict__ cx, const double* __restrict__ cy,
                            const double* __restrict__ deff, int64_t n_tri, double w0, double w1, double w2,
                            double eps_cn, double inv_near_order, double* __restrict__ nr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  const double wh[3] = {w0, w1, w2};
  double rho0[3], ell0[3];
  near_root(ax[t], ay[t], bx[t], by[t], cx[t], cy[t], deff[t], wh, eps_cn, inv_near_order, rho0, ell0);
  double* row = nr + 16 * t;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    row[e] = rho0[e];
    row[3 + e] = ell0[e];
  }
#pragma unroll
  for (int level = 0; level < 3; ++level) {
    double thr[3];
    near_level_thr(rho0, ell0, level, inv_near_order, thr);
#pragma unroll
    for (int e = 0; e < 3; ++e) row[6 + 3 * level + e] = thr[e];
  }
  row[15] = 0.0;
}

// count pass: class of every pair, pairs of each class per block
__global__ __launch_bounds__(kClsThreads) void k_pair_class(ClassArgs a) {
  __shared__ int cnt[kNCls];
  if (threadIdx.x < kNCls) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kClsChunk;
  int my[kNCls] = {};
#pragma unroll
  for (int i = 0; i < kClsPer; ++i) {
    const int64_t pr = base + i * kClsThreads + threadIdx.x;
    if (pr < a.n_pairs) {
      const int c = pair_class(a, pr);
      a.cls[pr] = (uint8_t)c;
#pragma unroll
      for (int k = 0; k < kNCls; ++k) my[k] += (c & 7) == k;
    }
  }
#pragma unroll
  for (int c = 0; c < kNCls; ++c) {
    int v = my[c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&cnt[c], v);
  }
  __syncthreads();
  if (threadIdx.x < kNCls) a.bcnt[threadIdx.x * a.n_blk + blockIdx.x] = cnt[threadIdx.x];
}

// scatter pass: pair indices by class, in pair order within a class
__global__ __launch_bounds__(kClsThreads) void k_pair_scatter(ClassArgs a) {
  __shared__ int wtot[kClsThreads / 64][kNCls];
  const int64_t base = (int64_t)blockIdx.x * kClsChunk;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t off[kNCls];
#pragma unroll
  for (int c = 0; c < kNCls; ++c) off[c] = a.boff[c * a.n_blk + blockIdx.x];
  for (int i = 0; i < kClsPer; ++i) {
    const int64_t pr = base + i * kClsThreads + threadIdx.x;
    const int c = pr < a.n_pairs ? (int)(a.cls[pr] & 7) : -1;
    uint64_t m[kNCls];
#pragma unroll
    for (int k = 0; k < kNCls; ++k) m[k] = __ballot(c == k);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < kNCls; ++k) wtot[w][k] = __popcll(m[k]);
    }
    __syncthreads();
    if (c >= 0) {
      int64_t o = 0;
      uint64_t mc = 0;
#pragma unroll
      for (int k = 0; k < kNCls; ++k)
        if (k == c) {
          o = off[k];
          mc = m[k];
        }
      for (int v = 0; v < w; ++v) o += wtot[v][c];
      a.list[o + __popcll(mc & lt)] = (uint32_t)pr;
      if (c < kClsDeep) a.stt[o + __popcll(mc & lt)] = make_int2(a.pair_tri[pr], a.pair_tgt[pr]);
    }
#pragma unroll
    for (int k = 0; k < kNCls; ++k)
      for (int v = 0; v < kClsThreads / 64; ++v) off[k] += wtot[v][k];
    __syncthreads();
  }
}

// Reference data of the two classes, one row per slot (far nodes first,
// padded to a multiple of 4, then the near rule's nodes): node tables
// [rows] (xi1, xi2; the centroid in padding rows) and Koornwinder tables
// [rows][NPP] scaled by half the node's weight: -w_j / 2 of the far rule,
// subtracted, or w_j s^2 / 2 of a leaf of scale s, the 1/2 of log r^2 (zero
// rows and columns as padding).
// Class 0: the near rule on the simplex; class 1: on its four children
// (a, s) = ((0,0), 1/2), ((1/2,0), 1/2), ((0,1/2), 1/2), ((1/2,1/2), -1/2).
template <int P>
__global__ void k_tab_build(const double* __restrict__ fx, const double* __restrict__ fy,
                            const double* __restrict__ fw, int nf, int nf4, const double* __restrict__ nx,
                            const double* __restrict__ ny, const double* __restrict__ nw, int nn, int nn4,
                            double2* __restrict__ nod0, double2* __restrict__ nod1, double* __restrict__ tab0,
                            double* __restrict__ tab1) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  constexpr int NPP = 16 * ((NP + 15) / 16);
  const int rows0 = nf4 + nn4, rows1 = nf4 + 4 * nn;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows0 + rows1) return;
  const bool one = g >= rows0;
  const int r = one ? g - rows0 : g;
  double* row = (one ? tab1 : tab0) + (size_t)r * NPP;
  double2* nod = (one ? nod1 : nod0) + r;
  for (int k = 0; k < NPP; ++k) row[k] = 0.0;
  double xi1 = 1.0 / 3.0, xi2 = 1.0 / 3.0, w = 0.0;
  bool live = false;
  if (r < nf) {
    xi1 = fx[r];
    xi2 = fy[r];
    w = -fw[r];
    live = true;
  } else if (r >= nf4) {
    const int j = r - nf4;
    if (!one && j < nn) {
      xi1 = nx[j];
      xi2 = ny[j];
      w = nw[j];
      live = true;
    } else if (one) {
      const int c = j / nn, i = j - c * nn;
      const double sa = (c == 1 || c == 3) ? 0.5 : 0.0, sb = (c >= 2) ? 0.5 : 0.0, ss = (c == 3) ? -0.5 : 0.5;
      xi1 = sa + ss * nx[i];
      xi2 = sb + ss * ny[i];
      w = nw[i] * ss * ss;
      live = true;
    }
  }
  *nod = make_double2(xi1, xi2);
  const double hw = 0.5 * w;  // the kernel's 1/2 of log r^2
  if (live) koornwinder_emit<P>(xi1, xi2, [&](int k, double v) { row[k] = hw * v; });
}

// The same tables for classes 2 + c (c = 0..3), rows2 slots each (far
// nodes, then 7 leaves of nn nodes, padded to a multiple of 4): the leaves
// are the level-1 children other than c, then the four children of c.
template <int P>
__global__ void k_tab_build2(const double* __restrict__ fx, const double* __restrict__ fy,
                             const double* __restrict__ fw, int nf, int nf4, const double* __restrict__ nx,
                             const double* __restrict__ ny, const double* __restrict__ nw, int nn, int rows2,
                             double2* __restrict__ nod2, double* __restrict__ tab2) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  constexpr int NPP = 16 * ((NP + 15) / 16);
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 4 * rows2) return;
  const int c = g / rows2, r = g - c * rows2;
  double* row = tab2 + (size_t)g * NPP;
  double2* nod = nod2 + g;
  for (int k = 0; k < NPP; ++k) row[k] = 0.0;
  double xi1 = 1.0 / 3.0, xi2 = 1.0 / 3.0, w = 0.0;
  bool live = false;
  if (r < nf) {
    xi1 = fx[r];
    xi2 = fy[r];
    w = -fw[r];
    live = true;
  } else if (r >= nf4 && r < nf4 + 7 * nn) {
    const int j = r - nf4, l = j / nn, i = j - l * nn;
    double sa, sb, ss;
    if (l < 3) {  // a level-1 child k != c
      const int k = l + (l >= c ? 1 : 0);
      sa = (k == 1 || k == 3) ? 0.5 : 0.0;
      sb = (k >= 2) ? 0.5 : 0.0;
      ss = (k == 3) ? -0.5 : 0.5;
    } else {  // child l - 3 of c
      const int k = l - 3;
      const double ca = (c == 1 || c == 3) ? 0.5 : 0.0, cb = (c >= 2) ? 0.5 : 0.0, h = (c == 3) ? -0.25 : 0.25;
      sa = ca + ((k == 1 || k == 3) ? h : 0.0);
      sb = cb + ((k >= 2) ? h : 0.0);
      ss = (k == 3) ? -h : h;
    }
    xi1 = sa + ss * nx[i];
    xi2 = sb + ss * ny[i];
    w = nw[i] * ss * ss;
    live = true;
  }
  *nod = make_double2(xi1, xi2);
  const double hw = 0.5 * w;
  if (live) koornwinder_emit<P>(xi1, xi2, [&](int k, double v) { row[k] = hw * v; });
}

typedef double vp_d4 __attribute__((ext_vector_type(4)));

struct TabArgs {
  const uint32_t* list;  // class 0 pairs, then class 1 pairs
  const int2* stt;       // their (triangle, target), in the same order
  int64_t n0, n1;
  const int32_t *pair_tri, *pair_tgt;
  const double *xt, *yt;
  const double *ax, *ay, *bx, *by, *cx, *cy, *det;
  const double4* geo;  // the same, packed per triangle
  int rows0, rows1;  // slots of class 0 and class 1 (multiples of 4)
  const double2 *nod0, *nod1;
  const double *tab0, *tab1;
  const double2* logtab;
  double* rows;
};

// (at most 80 registers for 6 wavefronts per SIMD at P <= 4; above, the
// larger accumulators take 5).  kLds: 2 both classes' Koornwinder tables in
// LDS, 1 class 0's only, 0 none (read through the caches).  A block's
// wavefronts take tiles in turn over the whole list, so the LDS fill of a
// block is paid once per block of a grid sized to the device.
template <int P, int kLds>
__global__ __launch_bounds__(kTabThreads, (P <= 4) ? 6 : 5) void k_rows_tab(TabArgs a) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  constexpr int NT = (NP + 15) / 16;
  constexpr int NPP = 16 * NT;
  __shared__ double2 tab[kLogTab + 1];
  // node tables [rows0 + rows1], then the Koornwinder tables in LDS:
  // class 0's [rows0][NPP] (kLds >= 1), class 1's [rows1][NPP] (kLds == 2)
  extern __shared__ double2 nod[];
  double* const sT0 = (double*)(nod + a.rows0 + a.rows1);
  double* const sT1 = sT0 + (size_t)a.rows0 * NPP;
  for (int i = threadIdx.x; i <= kLogTab; i += blockDim.x) tab[i] = a.logtab[i];
  for (int i = threadIdx.x; i < a.rows0; i += blockDim.x) nod[i] = a.nod0[i];
  for (int i = threadIdx.x; i < a.rows1; i += blockDim.x) nod[a.rows0 + i] = a.nod1[i];
  if (kLds >= 1)
    for (int i = threadIdx.x; i < a.rows0 * NPP; i += blockDim.x) sT0[i] = a.tab0[i];
  if (kLds == 2)
    for (int i = threadIdx.x; i < a.rows1 * NPP; i += blockDim.x) sT1[i] = a.tab1[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, kq = lane >> 4, col = lane & 15;
  const int64_t t0 = (a.n0 + 15) / 16, n_tiles = t0 + (a.n1 + 15) / 16;
  // the tile index is the same in every lane: kept in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int64_t tile = (int64_t)blockIdx.x * kTabWaves + wave; tile < n_tiles; tile += (int64_t)gridDim.x * kTabWaves) {
    const bool one = tile >= t0;
    const int64_t base = one ? a.n0 + (tile - t0) * 16 : tile * 16;
    const int64_t end = one ? a.n0 + a.n1 : a.n0;
    const bool valid = base + col < end;
    const int64_t at = valid ? base + col : base;
    // the pair index (for the row) and its triangle and target, side by side
    const uint32_t pr = a.list[at];
    const int2 tt = a.stt[at];
    const int32_t t = tt.x;
    const int32_t it = tt.y;
    const TriGeo tg = tri_geo(a.geo, t);
    // the target relative to the vertex A (exact for a target near A)
    const double px = a.xt[it] - tg.ax, py = a.yt[it] - tg.ay;
    const double e1x = tg.bx - tg.ax, e1y = tg.by - tg.ay, e2x = tg.cx - tg.ax, e2y = tg.cy - tg.ay;
    const double D = tg.det;
    const double2* N = one ? nod + a.rows0 : nod;
    const int n_slots = one ? a.rows1 : a.rows0;
    vp_d4 acc[NT];
    // zero accumulators made by the matrix core itself, so that they live in
    // its registers through the loop
#pragma unroll
    for (int n = 0; n < NT; ++n)
      acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(0.0, 0.0, vp_d4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
    // Every slot alike: the target's offset from the node, r^2 and its
    // logarithm.  The target of a near pair lies outside the triangle and
    // every node inside, so r^2 > 0 without the far sums' offset (which
    // would change nothing here).  The weights are in the table (negative
    // for the far rule's own contribution, which is subtracted; zero in
    // padding rows), the triangle's Jacobian scales the finished row.
    auto steps = [&](auto trow) {
      for (int s0 = 0; s0 < n_slots; s0 += 4) {
        const int slot = s0 + kq;
        const double2 xi = N[slot];
        const double dx = fma(-xi.y, e2x, fma(-xi.x, e1x, px));
        const double dy = fma(-xi.y, e2y, fma(-xi.x, e1y, py));
        const double r2 = fma(dx, dx, dy * dy);
        const double g = vp_log(r2, tab);
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, trow(slot, n), acc[n], 0, 0, 0);
      }
    };
    if (kLds == 2) {
      const double* T = one ? sT1 : sT0;
      steps([&](int slot, int n) { return T[slot * NPP + 16 * n + col]; });
    } else if (kLds == 1 && !one) {
      steps([&](int slot, int n) { return sT0[slot * NPP + 16 * n + col]; });
    } else {
      const double* T = one ? a.tab1 : a.tab0;
      steps([&](int slot, int n) { return T[(size_t)slot * NPP + 16 * n + col]; });
    }
    // element v of lane l: pair kq + 4 v of the tile, basis function 16 n + col
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rrow = kq + 4 * v;
      const uint32_t prow = (uint32_t)__shfl((int)pr, rrow);
      const double scale = __shfl(D, rrow) * kInv2Pi;
      if (base + rrow < end) {
        double* out = a.rows + (size_t)prow * NP;
#pragma unroll
        for (int n = 0; n < NT; ++n)
          if (16 * n + col < NP) out[16 * n + col] = acc[n][v] * scale;
      }
    }
  }
}

}  // namespace

// The class-sorted launches of launch_rows (straight triangles, ellipse
// model, q_near <= 8): class pass, scatter, then k_rows_tab over classes 0
// and 1 and k_rows over deeper near pairs and over self pairs.
template <int P>
hipError_t rows_by_class(vp_plan* pl, RowsArgs a, size_t lds, hipStream_t st) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  constexpr int NPP = 16 * ((NP + 15) / 16);
  const vp_mesh* m = pl->mesh;
  const int64_t n = pl->n_pairs;
  const int64_t n_blk = (n + kClsChunk - 1) / kClsChunk;
  const int nf = pl->n_f, nf4 = (nf + 3) & ~3, nn = a.nn, nn4 = (nn + 3) & ~3;
  const int rows0 = nf4 + nn4, rows1 = nf4 + 4 * nn, rows2 = (nf4 + 7 * nn + 3) & ~3;
  Scratch tmp(pl->ctx, st);
  uint8_t* cls = nullptr;
  int32_t* bcnt = nullptr;
  int64_t* boff = nullptr;
  uint32_t* list = nullptr;
  double *tab0 = nullptr, *tab1 = nullptr, *nr = nullptr, *tab2 = nullptr;
  double2 *nod0 = nullptr, *nod1 = nullptr, *nod2 = nullptr;
  void* stmp = nullptr;
  hipError_t e;
  if ((e = tmp.alloc((void**)&cls, (size_t)n)) != hipSuccess ||
      (e = tmp.alloc((void**)&nr, sizeof(double) * 16 * std::max<int64_t>(pl->n_tri, 1))) != hipSuccess ||
      (e = tmp.alloc((void**)&bcnt, sizeof(int32_t) * kNCls * n_blk)) != hipSuccess ||
      (e = tmp.alloc((void**)&boff, sizeof(int64_t) * (kNCls * n_blk + 1))) != hipSuccess ||
      (e = tmp.alloc((void**)&list, sizeof(uint32_t) * n)) != hipSuccess ||
      (e = tmp.alloc(&stmp, exclusive_scan_tmp_bytes(kNCls * n_blk))) != hipSuccess ||
      (e = tmp.alloc((void**)&nod0, sizeof(double2) * rows0)) != hipSuccess ||
      (e = tmp.alloc((void**)&nod1, sizeof(double2) * rows1)) != hipSuccess ||
      (e = tmp.alloc((void**)&tab0, sizeof(double) * rows0 * NPP)) != hipSuccess ||
      (e = tmp.alloc((void**)&tab1, sizeof(double) * rows1 * NPP)) != hipSuccess ||
      (e = tmp.alloc((void**)&nod2, sizeof(double2) * 4 * rows2)) != hipSuccess ||
      (e = tmp.alloc((void**)&tab2, sizeof(double) * 4 * rows2 * NPP)) != hipSuccess)
    return e;
  ClassArgs c;
  c.pair_tri = pl->pair_tri;
  c.pair_tgt = pl->pair_tgt;
  c.pair_kind = pl->pair_kind;
  c.n_pairs = n;
  c.n_blk = n_blk;
  c.xt = pl->xt;
  c.yt = pl->yt;
  c.ax = m->ax;
  c.ay = m->ay;
  c.bx = m->bx;
  c.by = m->by;
  c.cx = m->cx;
  c.cy = m->cy;
  c.det = m->det;
  c.geo = m->geo;
  c.deff = pl->deff;
  c.nr = nr;
  c.n_tri = pl->n_tri;
  c.nwhat0 = a.nwhat0;
  c.nwhat1 = a.nwhat1;
  c.nwhat2 = a.nwhat2;
  c.eps_cn = a.eps_cn;
  c.inv_near_order = a.inv_near_order;
  c.depth_cap = a.depth_cap;
  c.cls = cls;
  c.bcnt = bcnt;
  c.boff = boff;
  c.list = list;
  if (pl->n_tri > 0)
    k_near_root<<<(unsigned)((pl->n_tri + 255) / 256), 256, 0, st>>>(m->ax, m->ay, m->bx, m->by, m->cx, m->cy,
                                                                      pl->deff, pl->n_tri, a.nwhat0, a.nwhat1,
                                                                      a.nwhat2, a.eps_cn, a.inv_near_order, nr);
  k_pair_class<<<(unsigned)n_blk, kClsThreads, 0, st>>>(c);
  k_tab_build<P><<<(rows0 + rows1 + 127) / 128, 128, 0, st>>>(pl->far_x, pl->far_y, pl->far_w, nf, nf4,
                                                              pl->near_x, pl->near_y, pl->near_w, nn, nn4, nod0,
                                                              nod1, tab0, tab1);
  k_tab_build2<P><<<(4 * rows2 + 127) / 128, 128, 0, st>>>(pl->far_x, pl->far_y, pl->far_w, nf, nf4, pl->near_x,
                                                          pl->near_y, pl->near_w, nn, rows2, nod2, tab2);
  // first pair of each class in the sorted list, and the total
  int64_t tot[kNCls + 1] = {};
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = exclusive_scan_i32(bcnt, boff, kNCls * n_blk, stmp, st)) != hipSuccess)
    return e;
  for (int k = 0; k <= kNCls; ++k)
    if ((e = hipMemcpyAsync(&tot[k], boff + k * n_blk, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  int64_t cnt[kNCls];
  for (int k = 0; k < kNCls; ++k) cnt[k] = tot[k + 1] - tot[k];
  if (tot[kNCls] != n) return hipErrorUnknown;
  int2* stt = nullptr;
  if ((e = tmp.alloc((void**)&stt, sizeof(int2) * std::max<int64_t>(tot[kClsDeep], 1))) != hipSuccess) return e;
  c.stt = stt;
  k_pair_scatter<<<(unsigned)n_blk, kClsThreads, 0, st>>>(c);
  TabArgs ta;
  ta.pair_tri = pl->pair_tri;
  ta.pair_tgt = pl->pair_tgt;
  ta.xt = pl->xt;
  ta.yt = pl->yt;
  ta.ax = m->ax;
  ta.ay = m->ay;
  ta.bx = m->bx;
  ta.by = m->by;
  ta.cx = m->cx;
  ta.cy = m->cy;
  ta.det = m->det;
  ta.geo = m->geo;
  ta.logtab = pl->logtab;
  ta.rows = pl->rows;
  const int64_t n_tab = cnt[0] + cnt[1] + cnt[2] + cnt[3] + cnt[4] + cnt[5];
  if (n_tab > 0) {
    StageTimer tm(pl->ctx, VP_STAGE_ROWS_TAB);
    int launches = 0;
    // classes (0, 1), (2, 3) and (4, 5), two per launch: each launch holds
    // its two classes' node tables in LDS, and class 0's Koornwinder table
    // while it is small (the common class)
    for (int k = 0; k < 6; k += 2) {
      if (cnt[k] + cnt[k + 1] == 0) continue;
      ta.list = list + tot[k];
      ta.stt = stt + tot[k];
      ta.n0 = cnt[k];
      ta.n1 = cnt[k + 1];
      if (k == 0) {
        ta.rows0 = rows0;
        ta.rows1 = rows1;
        ta.nod0 = nod0;
        ta.nod1 = nod1;
        ta.tab0 = tab0;
        ta.tab1 = tab1;
      } else {
        const int c0 = k - 2;  // configurations c0 and c0 + 1 of the class-2 tables
        ta.rows0 = ta.rows1 = rows2;
        ta.nod0 = nod2 + (size_t)c0 * rows2;
        ta.nod1 = nod2 + (size_t)(c0 + 1) * rows2;
        ta.tab0 = tab2 + (size_t)c0 * rows2 * NPP;
        ta.tab1 = tab2 + (size_t)(c0 + 1) * rows2 * NPP;
      }
      const int64_t tiles = (ta.n0 + 15) / 16 + (ta.n1 + 15) / 16;
      const size_t lds = sizeof(double2) * (size_t)(ta.rows0 + ta.rows1);
      const size_t t0_bytes = sizeof(double) * (size_t)ta.rows0 * NPP;
      const size_t t1_bytes = sizeof(double) * (size_t)ta.rows1 * NPP;
      const size_t fixed = sizeof(double2) * (kLogTab + 1);
      const unsigned nb = (unsigned)std::min<int64_t>((tiles + kTabWaves - 1) / kTabWaves,
                                                      (int64_t)kTabBlocksPerCu * pl->ctx->n_cu);
      if (fixed + lds + t0_bytes + t1_bytes <= kTabLdsBlock)
        k_rows_tab<P, 2><<<nb, kTabThreads, lds + t0_bytes + t1_bytes, st>>>(ta);
      else if (t0_bytes <= kTabT0LdsMax)
        k_rows_tab<P, 1><<<nb, kTabThreads, lds + t0_bytes, st>>>(ta);
      else
        k_rows_tab<P, 0><<<nb, kTabThreads, lds, st>>>(ta);
      ++launches;
    }
    tm.stop(launches);
  }
  constexpr int64_t kPairsPerGroup = 8;
  auto groups = [&](int64_t k) {
    return dim3((unsigned)std::min<int64_t>((k + kPairsPerGroup - 1) / kPairsPerGroup, 1 << 25));
  };
  const int64_t n2 = cnt[kClsDeep], n3 = cnt[kClsSelf];
  if (n2 > 0) {
    uint32_t* ovf = nullptr;
    uint32_t* n_ovf = nullptr;
    if ((e = tmp.alloc((void**)&ovf, sizeof(uint32_t) * n2)) != hipSuccess ||
        (e = tmp.alloc((void**)&n_ovf, sizeof(uint32_t))) != hipSuccess ||
        (e = hipMemsetAsync(n_ovf, 0, sizeof(uint32_t), st)) != hipSuccess)
      return e;
    a.list = list + tot[kClsDeep];
    a.n_list = n2;
    StageTimer tm(pl->ctx, VP_STAGE_ROWS_NEAR);
    const size_t lds_deep = sizeof(double) * (3 * (size_t)nn + 2 * (size_t)nf);
    k_rows_deep<P><<<groups(n2), 64, lds_deep, st>>>(a, nr, pl->n_tri, cls, ovf, n_ovf);
    uint32_t h_ovf = 0;
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(&h_ovf, n_ovf, sizeof(uint32_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    if (h_ovf > 0) {
      a.list = ovf;
      a.n_list = h_ovf;
      k_rows<P, false, 1><<<groups(h_ovf), 64, lds, st>>>(a);
    }
    tm.stop(h_ovf > 0 ? 2 : 1);
  }
  if (n3 > 0) {
    a.list = list + tot[kClsSelf];
    a.n_list = n3;
    StageTimer tm(pl->ctx, VP_STAGE_ROWS_SELF);
    k_rows<P, false, 2><<<groups(n3), 64, lds, st>>>(a);
    tm.stop(1);
  }
  // the table path's leaves: one per class-0 pair, four per class-1 pair,
  // seven per class 2..5 pair
  pl->tab_leaves = cnt[0] + 4 * cnt[1] + 7 * (cnt[2] + cnt[3] + cnt[4] + cnt[5]);
  pl->tab_pairs = n_tab;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  tmp.release();
  return hipSuccess;
}

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
  a.geo = m->geo;
  a.far_x = pl->far_x;
  a.far_y = pl->far_y;
  a.far_w = pl->far_w;
  a.efar = pl->efar;
  a.basis_g = pl->basis_g;
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
  a.list = nullptr;
  a.n_list = 0;
  // one 64-lane workgroup per 8 pairs (strided over the pair list), so that
  // the tables a workgroup stages in LDS serve several pairs while the
  // dispatcher still balances workgroups of uneven cost; grid-stride beyond
  // 2^25 workgroups (a launch must stay below 2^32 work-items).  A single
  // device-wide work counter instead serialises on its atomic across the XCDs.
  constexpr int64_t kPairsPerGroup = 8;
  dim3 grid((unsigned)std::min<int64_t>((pl->n_pairs + kPairsPerGroup - 1) / kPairsPerGroup, 1 << 25));
  const bool curved = m->n_curved > 0;
  const size_t lds = sizeof(double) * (3 * (size_t)a.nn + 2 * (size_t)a.nl + 3 * (size_t)a.nr + 3 * (size_t)a.n_rc);
  // straight meshes with the ellipse model: pairs sorted by depth class,
  // shallow near pairs on the matrix cores, deeper near pairs and self
  // pairs by k_rows, each launch sized to its pairs
  // LDS slots of the larger launch: classes 0 and 1, or two class-2 tables
  const int nf4 = (pl->n_f + 3) & ~3, rows2 = (nf4 + 7 * a.nn + 3) & ~3;
  const int slots = std::max(2 * nf4 + ((a.nn + 3) & ~3) + 4 * a.nn, 2 * rows2);
  if (!curved && !a.ball && a.nn <= kTabNearMax && slots <= kTabSlotsMax && pl->n_pairs < ((int64_t)1 << 32)) {
    switch (pl->p) {
      case 1: return rows_by_class<1>(pl, a, lds, st);
      case 2: return rows_by_class<2>(pl, a, lds, st);
      case 3: return rows_by_class<3>(pl, a, lds, st);
      case 4: return rows_by_class<4>(pl, a, lds, st);
      case 5: return rows_by_class<5>(pl, a, lds, st);
      case 6: return rows_by_class<6>(pl, a, lds, st);
      case 7: return rows_by_class<7>(pl, a, lds, st);
      case 8: return rows_by_class<8>(pl, a, lds, st);
      case 9: return rows_by_class<9>(pl, a, lds, st);
      case 10: return rows_by_class<10>(pl, a, lds, st);
      default: return hipErrorInvalidValue;
    }
  }
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
