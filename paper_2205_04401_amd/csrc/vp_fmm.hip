// Far sum by the fast multipole method: an O(N + M) replacement of the
// direct sum of the far-rule point charges (Sec. 3.6 couples the far rule
// to an FMM as point charges; the paper uses a library FMM).  A plan option
// (vp_plan_opts.fmm_terms > 0); the direct sum stays the default.
//
// U(x) = sum_j Q_j log|x - y_j|^2 = 2 Re sum_j Q_j log(z - w_j), z = x, w_j = y_j
// as complex numbers.  Uniform quadtree over the bounding square of sources
// and targets, levels 0..L (level l: 2^l x 2^l boxes of width s_l, row-major
// box index iy 2^l + ix); every level is stored densely.  Expansions about a
// box centre c with p terms, in units of the box width s:
//   multipole  sum_k a_k (z - c)^-k + a_0 log(z - c),  stored ah_k = a_k / s^k
//   local      sum_l b_l (z - c)^l,                     stored bh_l = b_l s^l
// (Greengard-Rokhlin translation lemmas; with these scalings the M2M and L2L
// operators depend only on the child's quadrant and the M2L operator only
// on the integer offset between the boxes, so all are precomputed once per
// context and p; the one level-dependent term, a_0 log s of M2L, is added
// apart).
// Interaction list: boxes of the same level that are not adjacent but whose
// parents are; near field: the 3 x 3 adjacent leaf boxes, summed directly
// with the direct sum's kernel log(r^2 + 2^-100), so a target on a source
// still gets the value the correction rows subtract again.  The M2L bound
// for adjacent-parent, non-adjacent boxes is (sum |Q|) 0.547^p / 0.83, so p
// sets the accuracy (p = 56: ~2e-15 of sum |Q|).
//   k_fmm_bbox_partial, k_fmm_keys, k_fmm_count, k_fmm_gather2,
//   k_fmm_tbox  (plan time)
//   k_fmm_p2m   one wavefront per leaf box: multipole of its sources
//   k_fmm_m2m   one thread per (box, coefficient): the upward pass
//   k_fmm_mreal the multipoles in real row form, [row][box] per level
//   k_fmm_m2l   16 boxes per wavefront, all levels in one launch: M2L over
//               the interaction list on the FP64 matrix cores (real form of
//               the complex operators)
//   k_fmm_l2l   one thread per (box, coefficient): L2L from the parent
//   k_fmm_leaf  one wavefront per 16 targets in leaf order: the local
//               expansion plus the direct sum over the 3 x 3 adjacent boxes
#include <hipcub/hipcub.hpp>

#include <climits>
#include <cmath>
#include <vector>

#include "vp_internal.h"

namespace vp {
namespace {

constexpr int kBlock = 256;
constexpr int kFmmMaxLevels = 10;  // finest quadtree level

inline unsigned blocks_for(int64_t n, int b = kBlock) {
  const int64_t nb = (n + b - 1) / b;
  return (unsigned)(nb < (1 << 20) ? (nb > 0 ? nb : 1) : (1 << 20));
}

__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {  // a b + c
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// per-block min x, min y, max x, max y over sources and targets
__global__ void k_fmm_bbox_partial(const double2* __restrict__ sxy, int64_t n_src, const double* __restrict__ xt,
                                   const double* __restrict__ yt, int64_t n_tgt, double* __restrict__ part) {
  __shared__ double red[4][kBlock];
  double v[4] = {1e300, 1e300, -1e300, -1e300};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_src + n_tgt; i += stride) {
    const double x = i < n_src ? sxy[i].x : xt[i - n_src];
    const double y = i < n_src ? sxy[i].y : yt[i - n_src];
    v[0] = fmin(v[0], x);
    v[1] = fmin(v[1], y);
    v[2] = fmax(v[2], x);
    v[3] = fmax(v[3], y);
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + h]);
      red[1][threadIdx.x] = fmin(red[1][threadIdx.x], red[1][threadIdx.x + h]);
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + h]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[4 * blockIdx.x + k] = red[k][0];
}

__device__ __forceinline__ uint32_t leaf_of(double x, double y, double x0, double y0, double inv_s, int n) {
  int ix = (int)floor((x - x0) * inv_s), iy = (int)floor((y - y0) * inv_s);
  ix = min(max(ix, 0), n - 1);
  iy = min(max(iy, 0), n - 1);
  return (uint32_t)(iy * n + ix);
}

// leaf keys and identity values of the sources (i < n_src) and targets
__global__ void k_fmm_keys(const double2* __restrict__ sxy, int64_t n_src, const double* __restrict__ xt,
                           const double* __restrict__ yt, int64_t n_tgt, double x0, double y0, double inv_s, int n,
                           uint32_t* __restrict__ skey, int32_t* __restrict__ sval, uint32_t* __restrict__ tkey,
                           int32_t* __restrict__ tval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_src + n_tgt; i += stride) {
    if (i < n_src) {
      skey[i] = leaf_of(sxy[i].x, sxy[i].y, x0, y0, inv_s, n);
      sval[i] = (int32_t)i;
    } else {
      const int64_t t = i - n_src;
      tkey[t] = leaf_of(xt[t], yt[t], x0, y0, inv_s, n);
      tval[t] = (int32_t)t;
    }
  }
}

__global__ void k_fmm_count(const uint32_t* __restrict__ key, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) atomicAdd(&cnt[key[i]], 1);
}

// tbox[i] = the leaf box of target i in leaf order (one thread per box)
__global__ void k_fmm_tbox(const int64_t* __restrict__ tptr, int64_t nleaf, int32_t* __restrict__ tbox) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  for (int64_t i = tptr[b]; i < tptr[b + 1]; ++i) tbox[i] = (int32_t)b;
}

// Direct pairs of every 16-target tile of the one-density leaf pass (the
// adjacent boxes' sources of its first and of its last target, the larger),
// and the tile's index, as the keys and values of a descending sort: the
// pass then starts with its longest tiles.  On a graded mesh the uniform
// quadtree leaves a few boxes with thousands of sources; started last, their
// tiles kept a few wavefronts running long after the rest had finished.
__global__ void k_fmm_tile_cost(const int32_t* __restrict__ tbox, int64_t n_tgt, const int64_t* __restrict__ sptr,
                                int L, uint32_t* __restrict__ cost, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_tiles = (n_tgt + 15) / 16;
  if (i >= n_tiles) return;
  const int n = 1 << L;
  auto adj = [&](int64_t b) -> int64_t {
    const int ix = (int)(b % n), iy = (int)(b / n);
    int64_t c = 0;
    for (int jy = max(iy - 1, 0); jy <= min(iy + 1, n - 1); ++jy) {
      const int64_t row = (int64_t)jy * n;
      c += sptr[row + min(ix + 1, n - 1) + 1] - sptr[row + max(ix - 1, 0)];
    }
    return c;
  };
  const int64_t last = min(16 * i + 15, n_tgt - 1);
  const int64_t c = max(adj(tbox[16 * i]), adj(tbox[last]));
  cost[i] = (uint32_t)min<int64_t>(c, 0xffffffffll);
  idx[i] = (int32_t)i;
}

__global__ void k_fmm_gather2(const double2* __restrict__ in, const int32_t* __restrict__ perm, int64_t n,
                              double2* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[perm[i]];
}

// Multipole of every leaf box (one wavefront each).  Lane l = g + 8 sl
// sums Q t^k (t = (w - c)/s) for the powers k = g + 8 i (i = 0..7, k <= p)
// over the box's sources sl, sl + 8, ...: t^g by binary powering, then
// repeated products with t^8, so a lane holds 8 complex sums whatever p is
// and the wavefront reduces once, over the 8 source lanes, at the end (a
// wavefront sum per power and 64 sources cost more than the powers).  The
// lanes with sl = 0 then hold ah_k = -sum Q t^k / k (a_0 = sum Q).  Also
// writes the charges in leaf order (Qs) for the near-field sum.
__global__ __launch_bounds__(kBlock) void k_fmm_p2m(const double2* __restrict__ sxy_s,
                                                    const int32_t* __restrict__ perm,
                                                    const int64_t* __restrict__ ptr, const double* __restrict__ Q,
                                                    int64_t R, int64_t r, int L, double x0, double y0, double s,
                                                    int p, double2* __restrict__ M, double* __restrict__ Qs) {
  const int lane = (int)(threadIdx.x & 63), g = lane & 7, sl = lane >> 3;
  const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int n = 1 << L;
  if (b >= (int64_t)n * n) return;  // the whole wavefront
  const int ix = (int)(b % n), iy = (int)(b / n);
  const double cx = x0 + (ix + 0.5) * s, cy = y0 + (iy + 0.5) * s, inv_s = 1.0 / s;
  double2 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = make_double2(0.0, 0.0);
  const int64_t j1 = ptr[b + 1];
  for (int64_t j = ptr[b] + sl; j < j1; j += 8) {
    const double q = Q[(int64_t)perm[j] * R + r];
    if (g == 0) Qs[j] = q;
    const double2 w = sxy_s[j];
    const double2 t = make_double2((w.x - cx) * inv_s, (w.y - cy) * inv_s);
    // v = q t^g; t8 = t^8
    double2 v = make_double2(q, 0.0), t8 = t;
#pragma unroll
    for (int bit = 0; bit < 3; ++bit) {
      if ((g >> bit) & 1) v = cmul(v, t8);
      t8 = cmul(t8, t8);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      acc[i].x += v.x;
      acc[i].y += v.y;
      if (i < 7) v = cmul(v, t8);
    }
  }
  // sum over the 8 source lanes (lane bits 3..5)
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int o = 8; o < 64; o <<= 1) {
      acc[i].x += __shfl_xor(acc[i].x, o);
      acc[i].y += __shfl_xor(acc[i].y, o);
    }
  if (sl == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = g + 8 * i;
      if (k <= p) M[b * (p + 1) + k] = k == 0 ? make_double2(acc[i].x, 0.0)
                                              : make_double2(-acc[i].x / k, -acc[i].y / k);
    }
  }
}

// Upward pass at level l: the box's multipole from its 4 children's
// (level l + 1), M2M operator of each child's quadrant.
__global__ void k_fmm_m2m(const double2* __restrict__ Mc, const int32_t* __restrict__ cnt_c, int l, int p,
                          const double2* __restrict__ m2m, double2* __restrict__ Mp) {
  const int P1 = p + 1;
  const int n = 1 << l;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * n * P1) return;
  const int64_t b = g / P1;
  const int k_out = (int)(g - b * P1);
  const int ix = (int)(b % n), iy = (int)(b / n);
  double2 acc = make_double2(0.0, 0.0);
  for (int q = 0; q < 4; ++q) {
    const int64_t c = (int64_t)(2 * iy + (q >> 1)) * (2 * n) + 2 * ix + (q & 1);
    if (cnt_c[c] == 0) continue;
    const double2* a = Mc + c * P1;
    const double2* T = m2m + ((int64_t)q * P1 + k_out) * P1;
    for (int k = 0; k <= k_out; ++k) acc = cfma(T[k], a[k], acc);
  }
  Mp[g] = acc;
}

// M2L at level l on the matrix cores.  In real form an M2L operator is a
// (2 P1) x (2 P1) matrix (rows and columns: real parts of the P1
// coefficients, then imaginary parts), padded to MP rows (multiple of 16)
// and KP columns (multiple of 4) with zeros.  One wavefront takes 16
// consecutive boxes (the 16 columns of the MFMA B operand) and one 16-row
// tile of the result, and accumulates over the 40 offsets operator rows x
// [multipoles of the 16 source boxes] (v_mfma_f64_16x16x4f64); a column
// whose box does not have that offset in its interaction list, or whose
// source box holds no sources, is zero.  The operators (49 MP KP doubles,
// 2.1 MB at p = 32) are read from the L2 cache by every wavefront, with no
// staging or barrier (measured against staging each operator in LDS for 4
// wavefronts: 1.6 ms against 2.9 ms per evaluation on the 20k-triangle
// star, and against one tile per wavefront for all row tiles: 5.6 ms; the
// pass is bound by operand loads and latency, not the matrix cores).  The
// level's a_0 log s term is added by the wavefront that holds row 0.  A
// lane l holds A row 16 t + (l & 15), column 4 s + (l >> 4); B row
// 4 s + (l >> 4), box l & 15; result element v of lane l: row
// 16 t + (l >> 4) + 4 v, box l & 15.  Boxes with no targets below them get
// zeros.
typedef double vp_d4 __attribute__((ext_vector_type(4)));

// All levels of the M2L pass in one launch (a level's translations read
// only multipoles, which are complete, and write only that level's local
// expansions): wavefronts are numbered level after level, coarsest first,
// so the few long-running wavefronts of the coarse levels start at once and
// overlap the many of the finest.
struct FmmLevels {
  int l0, l1;               // the levels l0..l1
  int64_t wave_end[kFmmMaxLevels + 1];  // wavefronts of levels l0..l (cumulative)
  int64_t off[kFmmMaxLevels + 1];       // first box of level l
  double log_s[kFmmMaxLevels + 1];      // log of level l's box width
};

// The multipoles of levels l0..l1 in real row form for the M2L pass: level
// l at Mr + 2 P1 off[l], [row][box], rows 0..P1-1 the real and P1..2P1-1 the
// imaginary parts of the coefficients (16 consecutive boxes then share
// cache lines in the M2L operand loads).
__global__ void k_fmm_mreal(const double2* __restrict__ M_all, FmmLevels lv, int p, double* __restrict__ Mr_all) {
  const int P1 = p + 1;
  const int64_t first = lv.off[lv.l0], nbox = lv.off[lv.l1] + ((int64_t)1 << (2 * lv.l1)) - first;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nbox * P1) return;
  const int64_t gb = first + g / P1;
  const int k = (int)(g % P1);
  int l = lv.l0;
  while (l < lv.l1 && gb >= lv.off[l + 1]) ++l;
  const int64_t box = gb - lv.off[l], nb = (int64_t)1 << (2 * l);
  const double2 m = M_all[gb * P1 + k];
  double* Mr = Mr_all + 2 * P1 * lv.off[l];
  Mr[(int64_t)k * nb + box] = m.x;
  Mr[(int64_t)(P1 + k) * nb + box] = m.y;
}

__global__ __launch_bounds__(kBlock) void k_fmm_m2l(const double* __restrict__ Mr_all,
                                                    const int32_t* __restrict__ cnt_s_all,
                                                    const int32_t* __restrict__ cnt_t_all, FmmLevels lv, int p,
                                                    int MP, int KP, const double* __restrict__ m2l,
                                                    double2* __restrict__ Lc_all) {
  const int P1 = p + 1;
  const int64_t w_all = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w_all >= lv.wave_end[lv.l1]) return;  // the whole wavefront
  int l = lv.l0;
  while (w_all >= lv.wave_end[l]) ++l;
  const int64_t w = w_all - (l > lv.l0 ? lv.wave_end[l - 1] : 0);
  const double* __restrict__ Mr = Mr_all + 2 * P1 * lv.off[l];
  const int32_t* __restrict__ cnt_s = cnt_s_all + lv.off[l];
  const int32_t* __restrict__ cnt_t = cnt_t_all + lv.off[l];
  double2* __restrict__ Lc = Lc_all + lv.off[l] * P1;
  const double log_s = lv.log_s[l];
  const int n = 1 << l;
  const int64_t nb = (int64_t)n * n;
  const int tiles = MP / 16;
  const int lane = (int)(threadIdx.x & 63), r16 = lane & 15, kq = lane >> 4;
  const int64_t bg = w / tiles;
  const int t = (int)(w - bg * tiles);
  if (bg * 16 >= nb) return;  // the whole wavefront
  const int64_t b = bg * 16 + r16;  // this lane's B box
  const bool live = b < nb && cnt_t[b < nb ? b : 0] > 0;
  const int ix = (int)(b % n), iy = (int)(b / n);
  vp_d4 acc = vp_d4{0.0, 0.0, 0.0, 0.0};
  double a0 = 0.0;  // sum of the used source boxes' a_0 (for the log s term)
  for (int o = 0; o < 49; ++o) {
    const int dy = o / 7 - 3, dx = o % 7 - 3;
    if (abs(dx) <= 1 && abs(dy) <= 1) continue;
    const int jx = ix + dx, jy = iy + dy;
    bool use = live && jx >= 0 && jx < n && jy >= 0 && jy < n && abs((jx >> 1) - (ix >> 1)) <= 1 &&
               abs((jy >> 1) - (iy >> 1)) <= 1;
    if (use) use = cnt_s[(int64_t)jy * n + jx] > 0;
    const int64_t j = use ? (int64_t)jy * n + jx : 0;
    if (use) a0 += Mr[j];
    const int KS = KP / 4;
    const double* A = m2l + (int64_t)(o * tiles + t) * KS * 64 + lane;
    // the operands of 8 steps are loaded before their 8 MFMAs, so that one
    // cache round trip serves 8 steps (indices clamped into the operator
    // and the multipole rows past the last step; such steps are skipped)
    for (int s0 = 0; s0 < KS; s0 += 8) {
      double av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = s0 + u < KS;  // the whole wavefront alike
        const int row = min(4 * (s0 + u) + kq, 2 * P1 - 1);
        av[u] = A[(in ? s0 + u : 0) * 64];
        bv[u] = Mr[(int64_t)row * nb + j];
      }
      // empty register constraints once all 16 loads are issued: they keep
      // the loads unconditional (the compiler otherwise turns the selects
      // below into branches around them, each with a wait inside)
#pragma unroll
      for (int u = 0; u < 8; ++u) asm volatile("" : "+v"(bv[u]));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = 4 * (s0 + u) + kq;
        bv[u] = (s0 + u < KS && use && k < 2 * P1) ? bv[u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (s0 + u < KS) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
  }
  if (b < nb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + kq + 4 * v;
      double y = acc[v];
      if (row == 0) y = fma(a0, log_s, y);
      if (row < P1)
        Lc[b * P1 + row].x = live ? y : 0.0;
      else if (row < 2 * P1)
        Lc[b * P1 + row - P1].y = live ? y : 0.0;
    }
  }
}

// L2L at level l > 2: every (box, coefficient) with targets below it adds
// the parent's local expansion shifted to its centre.
__global__ void k_fmm_l2l(const int32_t* __restrict__ cnt_t, const double2* __restrict__ Lp, int l, int p,
                          const double2* __restrict__ l2l, double2* __restrict__ Lc) {
  const int P1 = p + 1;
  const int n = 1 << l;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * n * P1) return;
  const int64_t b = g / P1;
  const int m = (int)(g - b * P1);
  if (cnt_t[b] == 0) return;
  const int ix = (int)(b % n), iy = (int)(b / n);
  const int64_t pb = (int64_t)(iy >> 1) * (n >> 1) + (ix >> 1);
  const int q = (ix & 1) | ((iy & 1) << 1);
  const double2* a = Lp + pb * P1;
  const double2* T = l2l + ((int64_t)q * P1 + m) * P1;
  double2 v = Lc[g];
  for (int k = m; k < P1; ++k) v = cfma(T[k], a[k], v);
  Lc[g] = v;
}

// Leaf pass of one density: one wavefront per 16 consecutive targets in
// leaf order (across box boundaries: a box of ~17 targets would otherwise
// leave a second, nearly empty tile), 4 lanes per target that take every
// fourth source of the target's adjacent boxes, joined by a butterfly over
// the 4; the first lane of each target adds 2 Re of its box's local
// expansion (Horner).  The direct sum is Q log(r^2 + 2^-100) over the
// sources of the 3 x 3 adjacent leaf boxes (256-entry logarithm table in
// LDS, exponent part accumulated apart as in the direct far sum).
__global__ __launch_bounds__(kBlock) void k_fmm_leaf(
    const double2* __restrict__ Lc, const int32_t* __restrict__ tbox, int64_t n_tgt,
    const double2* __restrict__ sxy_s, const double* __restrict__ Qs, const int64_t* __restrict__ sptr,
    const int32_t* __restrict__ tperm, const double* __restrict__ xt, const double* __restrict__ yt, int L,
    double x0, double y0, double s, int p, const double2* __restrict__ logtab, int64_t R, int64_t r,
    const int32_t* __restrict__ order, double* __restrict__ out) {
  __shared__ double2 tab[kLogTab + 1];
  for (int i = threadIdx.x; i <= kLogTab; i += kBlock) tab[i] = logtab[i];
  __syncthreads();
  const int lane = (int)(threadIdx.x & 63), r16 = lane & 15, kq = lane >> 4;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w * 16 >= n_tgt) return;  // the whole wavefront
  const int64_t i0 = (order ? (int64_t)order[w] : w) * 16;  // tiles longest first
  const int n = 1 << L;
  const int64_t i = i0 + r16;
  const bool act = i < n_tgt;
  const int64_t b = tbox[act ? i : i0];
  const int ix = (int)(b % n), iy = (int)(b / n);
  const double cx = x0 + (ix + 0.5) * s, cy = y0 + (iy + 0.5) * s, inv_s = 1.0 / s;
  const int64_t t = act ? tperm[i] : 0;
  const double x = act ? xt[t] : cx, y = act ? yt[t] : cy;
  const double2 l2 = tab[kLogTab];
  double acc_e = 0.0, acc_r = 0.0;
  for (int dy = -1; dy <= 1; ++dy) {
    const int jy = iy + dy;
    if (!act || jy < 0 || jy >= n) continue;
    const int64_t row = (int64_t)jy * n;
    const int64_t j0 = sptr[row + max(ix - 1, 0)], j1 = sptr[row + min(ix + 1, n - 1) + 1];
    for (int64_t j = j0 + kq; j < j1; j += 4) {
      const double2 sw = sxy_s[j];
      const double q = Qs[j];
      const double ddx = x - sw.x, ddy = y - sw.y;
      const double r2 = fma(ddy, ddy, fma(ddx, ddx, kR2Bias));
      double e, rest;
      vp_log_parts(r2, tab, e, rest);
      acc_e = fma(q, e, acc_e);
      acc_r = fma(q, rest, acc_r);
    }
  }
  acc_e += __shfl_xor(acc_e, 16);
  acc_r += __shfl_xor(acc_r, 16);
  acc_e += __shfl_xor(acc_e, 32);
  acc_r += __shfl_xor(acc_r, 32);
  if (act && kq == 0) {
    const double2* lc = Lc + b * (p + 1);
    const double2 zh = make_double2((x - cx) * inv_s, (y - cy) * inv_s);
    double2 v = lc[p];
    for (int k = p - 1; k >= 0; --k) v = cfma(v, zh, lc[k]);
    out[t * R + r] = 2.0 * v.x + acc_r + fma(acc_e, l2.x, acc_e * l2.y);
  }
}

// ---------------------------------------------------------------------------
// Blocks of 16 densities.  The expansions of 16 right-hand sides are kept in
// real form, [box][row][16] with rows 0..p the real parts of the
// coefficients and p+1..2p+1 the imaginary parts (padded with zero rows),
// so that P2M, M2L, L2P and the near-field sum all become products with 16
// right-hand sides as the MFMA B-operand columns (v_mfma_f64_16x16x4f64;
// lane l: A row l & 15, column l >> 4 of the step; B row l >> 4, column
// l & 15; result element v: row (l >> 4) + 4 v, column l & 15).

// Per plan: the P2M row of every source in leaf order, vsrc[j][0..MP) =
// real and imaginary parts of (1, -t, -t^2/2, ..., -t^p/p), t = (w - c)/s
// about its leaf centre; and the L2P row of every target in leaf order,
// wtgt[i][0..KP) = 2 Re zh^l, then -2 Im zh^l (u = 2 Re sum b_l zh^l).
__global__ void k_fmm_vsrc(const double2* __restrict__ sxy_s, int64_t n_src, double x0, double y0, double s, int L,
                           int p, int MP, double* __restrict__ vsrc) {
  const int n = 1 << L, P1 = p + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_src; j += stride) {
    const double2 w = sxy_s[j];
    const uint32_t b = leaf_of(w.x, w.y, x0, y0, 1.0 / s, n);
    const double cx = x0 + ((int)(b % n) + 0.5) * s, cy = y0 + ((int)(b / n) + 0.5) * s;
    const double2 t = make_double2((w.x - cx) / s, (w.y - cy) / s);
    double* v = vsrc + j * MP;
    v[0] = 1.0;
    v[P1] = 0.0;
    double2 pw = t;
    for (int m = 1; m <= p; ++m) {
      v[m] = -pw.x / m;
      v[P1 + m] = -pw.y / m;
      pw = cmul(pw, t);
    }
    for (int r = 2 * P1; r < MP; ++r) v[r] = 0.0;
  }
}

__global__ void k_fmm_wtgt(const double* __restrict__ xt, const double* __restrict__ yt,
                           const int32_t* __restrict__ tperm, int64_t n_tgt, double x0, double y0, double s, int L,
                           int p, int KP, double* __restrict__ wtgt) {
  const int n = 1 << L, P1 = p + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_tgt; i += stride) {
    const int64_t t = tperm[i];
    const double x = xt[t], y = yt[t];
    const uint32_t b = leaf_of(x, y, x0, y0, 1.0 / s, n);
    const double cx = x0 + ((int)(b % n) + 0.5) * s, cy = y0 + ((int)(b / n) + 0.5) * s;
    const double2 z = make_double2((x - cx) / s, (y - cy) / s);
    double* w = wtgt + i * KP;
    double2 zp = make_double2(1.0, 0.0);
    for (int l = 0; l <= p; ++l) {
      w[l] = 2.0 * zp.x;
      w[P1 + l] = -2.0 * zp.y;
      zp = cmul(zp, z);
    }
    for (int r = 2 * P1; r < KP; ++r) w[r] = 0.0;
  }
}

// The passes below take NB blocks of 16 densities at once (columns
// c0 .. c0 + 16 NB - 1, C = 16 NB columns in the real-form expansions
// [box][KP][C]): every A operand (P2M rows, M2L operator rows, L2P rows,
// the generated G) then serves NB MFMA steps, one per block of columns.

// P2M: one wavefront per (leaf box, row tile): rows of the real multipole =
// sum over the box's sources of vsrc[j][row] Q[j][column].
template <int NB>
__global__ __launch_bounds__(kBlock) void k_fmmb_p2m(const double* __restrict__ vsrc, const int32_t* __restrict__ perm,
                                                     const int64_t* __restrict__ ptr, const double* __restrict__ Q,
                                                     int64_t R, int64_t c0, int64_t nleaf, int MP, int KP,
                                                     double* __restrict__ Mb) {
  // columns c0 + 16 u + r16 >= R (the padding of a last, partial pass) read 0
  constexpr int C = 16 * NB;
  const int tiles = MP / 16;
  const int lane = (int)(threadIdx.x & 63), r16 = lane & 15, kq = lane >> 4;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t b = w / tiles;
  const int t = (int)(w - b * tiles);
  if (b >= nleaf) return;  // the whole wavefront
  const int64_t j0 = ptr[b], j1 = ptr[b + 1];
  vp_d4 acc[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) acc[u] = vp_d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t js = j0; js < j1; js += 4) {
    const int64_t j = js + kq;
    const bool ok = j < j1;
    const int64_t jc = ok ? j : j0;
    // loads from clamped (in-bounds) indices, always made; invalid entries
    // are multiplied by 0 rather than selected, so no load waits in a branch
    const double av = vsrc[jc * MP + 16 * t + r16] * (ok ? 1.0 : 0.0);
    const double* q = Q + (int64_t)perm[jc] * R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int64_t col = c0 + 16 * u + r16;
      const double qv = q[col < R ? col : R - 1] * (col < R ? 1.0 : 0.0);
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, qv, acc[u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * t + kq + 4 * v;
    if (row < KP) {
#pragma unroll
      for (int u = 0; u < NB; ++u) Mb[(b * KP + row) * C + 16 * u + r16] = acc[u][v];
    }
  }
}

// M2M / L2L in real form: one thread per (box, complex coefficient m,
// column); M2M sums the 4 children (k <= m), L2L adds the parent's
// expansion (k >= m) to the box's own.
__global__ void k_fmmb_m2m(const double* __restrict__ Mc, const int32_t* __restrict__ cnt_c, int l, int p, int KP, int C,
                           const double2* __restrict__ m2m, double* __restrict__ Mp) {
  const int P1 = p + 1, n = 1 << l;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * n * P1 * C) return;
  const int col = (int)(g % C);
  const int64_t bm = g / C;
  const int64_t b = bm / P1;
  const int m = (int)(bm - b * P1);
  const int ix = (int)(b % n), iy = (int)(b / n);
  double re = 0.0, im = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int64_t c = (int64_t)(2 * iy + (q >> 1)) * (2 * n) + 2 * ix + (q & 1);
    if (cnt_c[c] == 0) continue;
    const double* a = Mc + c * KP * C + col;
    const double2* T = m2m + ((int64_t)q * P1 + m) * P1;
    for (int k = 0; k <= m; ++k) {
      const double ar = a[k * C], ai = a[(P1 + k) * C];
      re = fma(T[k].x, ar, fma(-T[k].y, ai, re));
      im = fma(T[k].y, ar, fma(T[k].x, ai, im));
    }
  }
  Mp[(b * KP + m) * C + col] = re;
  Mp[(b * KP + P1 + m) * C + col] = im;
  if (m == 0)
    for (int r = 2 * P1; r < KP; ++r) Mp[(b * KP + r) * C + col] = 0.0;
}

__global__ void k_fmmb_l2l(const int32_t* __restrict__ cnt_t, const double* __restrict__ Lp, int l, int p, int KP,
                           int C, const double2* __restrict__ l2l, double* __restrict__ Lc) {
  const int P1 = p + 1, n = 1 << l;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * n * P1 * C) return;
  const int col = (int)(g % C);
  const int64_t bm = g / C;
  const int64_t b = bm / P1;
  const int m = (int)(bm - b * P1);
  if (cnt_t[b] == 0) return;
  const int ix = (int)(b % n), iy = (int)(b / n);
  const int64_t pb = (int64_t)(iy >> 1) * (n >> 1) + (ix >> 1);
  const int q = (ix & 1) | ((iy & 1) << 1);
  const double* a = Lp + pb * KP * C + col;
  const double2* T = l2l + ((int64_t)q * P1 + m) * P1;
  double re = Lc[(b * KP + m) * C + col], im = Lc[(b * KP + P1 + m) * C + col];
  for (int k = m; k < P1; ++k) {
    const double ar = a[k * C], ai = a[(P1 + k) * C];
    re = fma(T[k].x, ar, fma(-T[k].y, ai, re));
    im = fma(T[k].y, ar, fma(T[k].x, ai, im));
  }
  Lc[(b * KP + m) * C + col] = re;
  Lc[(b * KP + P1 + m) * C + col] = im;
}

// M2L: one wavefront per (box, row tile); all columns belong to the same
// box, so a whole offset is used or skipped.  The level's a_0 log s term
// is added per column to row 0.
template <int NB>
__global__ __launch_bounds__(kBlock) void k_fmmb_m2l(const double* __restrict__ Mb_all,
                                                     const int32_t* __restrict__ cnt_s_all,
                                                     const int32_t* __restrict__ cnt_t_all, FmmLevels lv, int MP,
                                                     int KP, const double* __restrict__ m2l,
                                                     double* __restrict__ Lb_all) {
  constexpr int C = 16 * NB;
  // all levels in one launch, numbered as in k_fmm_m2l
  const int64_t w_all = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w_all >= lv.wave_end[lv.l1]) return;  // the whole wavefront
  int l = lv.l0;
  while (w_all >= lv.wave_end[l]) ++l;
  const int64_t w = w_all - (l > lv.l0 ? lv.wave_end[l - 1] : 0);
  const double* __restrict__ Mb = Mb_all + lv.off[l] * KP * C;
  const int32_t* __restrict__ cnt_s = cnt_s_all + lv.off[l];
  const int32_t* __restrict__ cnt_t = cnt_t_all + lv.off[l];
  double* __restrict__ Lb = Lb_all + lv.off[l] * KP * C;
  const double log_s = lv.log_s[l];
  const int n = 1 << l;
  const int64_t nb = (int64_t)n * n;
  const int tiles = MP / 16;
  const int lane = (int)(threadIdx.x & 63), r16 = lane & 15, kq = lane >> 4;
  const int64_t b = w / tiles;
  const int t = (int)(w - b * tiles);
  if (b >= nb) return;  // the whole wavefront
  vp_d4 acc[NB];
  double a0[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    acc[u] = vp_d4{0.0, 0.0, 0.0, 0.0};
    a0[u] = 0.0;
  }
  if (cnt_t[b] > 0) {
    const int ix = (int)(b % n), iy = (int)(b / n);
    for (int o = 0; o < 49; ++o) {
      const int dy = o / 7 - 3, dx = o % 7 - 3;
      const int jx = ix + dx, jy = iy + dy;
      if ((abs(dx) <= 1 && abs(dy) <= 1) || jx < 0 || jx >= n || jy < 0 || jy >= n ||
          abs((jx >> 1) - (ix >> 1)) > 1 || abs((jy >> 1) - (iy >> 1)) > 1)
        continue;
      const int64_t j = (int64_t)jy * n + jx;
      if (cnt_s[j] == 0) continue;
      const double* X = Mb + j * KP * C + r16;
#pragma unroll
      for (int u = 0; u < NB; ++u) a0[u] += X[16 * u];
      const double* A = m2l + (int64_t)(o * tiles + t) * (KP / 4) * 64 + lane;
      // (each A operand serves NB MFMA steps, which hide its load: batching
      // the loads of several steps here raised the registers and cost
      // occupancy instead; so did loading the next step's operands ahead,
      // 23.6 -> 26.3 ms for 64 densities on the 100k star)
      for (int s4 = 0; s4 < KP / 4; ++s4) {
        const double av = A[s4 * 64];
        const double* x = X + (int64_t)(4 * s4 + kq) * C;
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, x[16 * u], acc[u], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * t + kq + 4 * v;
    if (row < KP) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        double y = acc[u][v];
        if (row == 0) y = fma(a0[u], log_s, y);
        Lb[(b * KP + row) * C + 16 * u + r16] = y;
      }
    }
  }
}

// Leaf pass: one wavefront per (leaf box, 16 of its targets): the local
// expansion (wtgt row x the box's local expansion) plus the direct sum over
// the sources of the 3 x 3 adjacent boxes, both on the matrix cores:
// A = G[target][source] = log(r^2 + 2^-100) generated by the lanes
// (256-entry logarithm table in LDS) once for all NB blocks, B = the
// sources' charges.
template <int NB>
__global__ __launch_bounds__(kBlock) void k_fmmb_leaf(
    const double* __restrict__ Lb, const double* __restrict__ wtgt, const int2* __restrict__ ttile, int64_t n_tiles,
    const double2* __restrict__ sxy_s, const int32_t* __restrict__ sperm, const int64_t* __restrict__ sptr,
    const int32_t* __restrict__ tperm, const int64_t* __restrict__ tptr, const double* __restrict__ xt,
    const double* __restrict__ yt, int L, int KP, const double2* __restrict__ logtab, const double* __restrict__ Q,
    int64_t R, int64_t c0, double* __restrict__ out) {
  constexpr int C = 16 * NB;
  __shared__ double2 tab[kLogTab + 1];
  for (int i = threadIdx.x; i <= kLogTab; i += kBlock) tab[i] = logtab[i];
  __syncthreads();
  const int lane = (int)(threadIdx.x & 63), r16 = lane & 15, kq = lane >> 4;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= n_tiles) return;  // the whole wavefront
  const int n = 1 << L;
  const int2 tl = ttile[w];
  const int64_t b = tl.x, i0 = tl.y, i1 = tptr[b + 1];
  const int ix = (int)(b % n), iy = (int)(b / n);
  const double2 l2 = tab[kLogTab];
  // this lane's A-row target
  const int64_t ia = i0 + r16;
  const bool ta = ia < i1;
  const int64_t tg = tperm[ta ? ia : i0];
  const double x = xt[tg], y = yt[tg];
  vp_d4 acc[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) acc[u] = vp_d4{0.0, 0.0, 0.0, 0.0};
  // local expansion
  const double* Xl = Lb + b * KP * C + r16;
  const double* Wt = wtgt + (ta ? ia : i0) * KP;
  for (int s4 = 0; s4 < KP / 4; ++s4) {
    const int k = 4 * s4 + kq;
    const double av = ta ? Wt[k] : 0.0;
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xl[k * C + 16 * u], acc[u], 0, 0, 0);
  }
  // adjacent boxes, row by row (consecutive boxes: one source range)
  for (int dy = -1; dy <= 1; ++dy) {
    const int jy = iy + dy;
    if (jy < 0 || jy >= n) continue;
    const int64_t row = (int64_t)jy * n;
    const int64_t j0 = sptr[row + max(ix - 1, 0)], j1 = sptr[row + min(ix + 1, n - 1) + 1];
    if (j0 >= j1) continue;  // no sources (the pipeline's first loads need one)
    // software pipeline: the positions and permutation entries of the step
    // after next and the charges of the next step are loaded while this
    // step's logarithms are evaluated (from clamped, in-bounds indices,
    // always; invalid entries carry a factor 0)
    int64_t cols[NB];
    double cmask[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int64_t col = c0 + 16 * u + r16;
      cols[u] = col < R ? col : R - 1;
      cmask[u] = col < R ? 1.0 : 0.0;
    }
    auto idx = [&](int64_t js) { const int64_t j = js + kq; return j < j1 ? j : j0; };
    int64_t jc = idx(j0), jn = idx(j0 + 4);
    double2 sw = sxy_s[jc], swn = sxy_s[jn];
    int32_t spn = sperm[jn];
    double qv[NB];
    {
      const double* q = Q + (int64_t)sperm[jc] * R;
      const double m = (j0 + kq < j1) ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < NB; ++u) qv[u] = q[cols[u]] * (m * cmask[u]);
    }
    for (int64_t js = j0; js < j1; js += 4) {
      const int64_t jnn = idx(js + 8);
      const double2 swnn = sxy_s[jnn];
      const int32_t spnn = sperm[jnn];
      double qn[NB];
      {
        const double* q = Q + (int64_t)spn * R;
        const double m = (js + 4 + kq < j1) ? 1.0 : 0.0;
#pragma unroll
        for (int u = 0; u < NB; ++u) qn[u] = q[cols[u]] * (m * cmask[u]);
      }
      const double ddx = x - sw.x, ddy = y - sw.y;
      const double r2 = fma(ddy, ddy, fma(ddx, ddx, kR2Bias));
      double e, rest;
      vp_log_parts(r2, tab, e, rest);
      const double g = ta ? fma(e, l2.x, fma(e, l2.y, rest)) : 0.0;
#pragma unroll
      for (int u = 0; u < NB; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, qv[u], acc[u], 0, 0, 0);
      sw = swn;
      swn = swnn;
      spn = spnn;
#pragma unroll
      for (int u = 0; u < NB; ++u) qv[u] = qn[u];
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t i = i0 + kq + 4 * v;
    if (i < i1) {
      const int64_t o = (int64_t)tperm[i] * R + c0 + r16;
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (c0 + 16 * u + r16 < R) out[o + 16 * u] = acc[u][v];
    }
  }
}

// The leaf pass in mixed precision (VP_MIXED): the same two products on the
// FP32 matrix cores (v_mfma_f32_16x16x4f32, twice the FP64 rate).  The
// local expansion and the L2P rows are rounded to FP32; G = log2(r^2 +
// 2^-100) of the FP32 difference (v_log_f32) and the charges Q32 = Q ln 2
// in FP32 (the direct far sum's mixed form).  FP32 products are summed over
// tiles of up to 256 sources and each tile joins an FP64 accumulator.
// Element v of lane l of a result tile holds column l & 15 of target
// 4 (l >> 4) + v.
typedef float vp_f4 __attribute__((ext_vector_type(4)));

template <int NB>
__global__ __launch_bounds__(kBlock) void k_fmmb_leaf32(
    const double* __restrict__ Lb, const double* __restrict__ wtgt, const int2* __restrict__ ttile, int64_t n_tiles,
    const double2* __restrict__ sxy_s, const int32_t* __restrict__ sperm, const int64_t* __restrict__ sptr,
    const int32_t* __restrict__ tperm, const int64_t* __restrict__ tptr, const double* __restrict__ xt,
    const double* __restrict__ yt, int L, int KP, const float* __restrict__ Q32, int64_t R, int64_t c0,
    double* __restrict__ out) {
  constexpr int C = 16 * NB;
  const int lane = (int)(threadIdx.x & 63), r16 = lane & 15, kq = lane >> 4;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= n_tiles) return;  // the whole wavefront
  const int n = 1 << L;
  const int2 tl = ttile[w];
  const int64_t b = tl.x, i0 = tl.y, i1 = tptr[b + 1];
  const int ix = (int)(b % n), iy = (int)(b / n);
  // this lane's A-row target
  const int64_t ia = i0 + r16;
  const bool ta = ia < i1;
  const int64_t tg = tperm[ta ? ia : i0];
  const double x = xt[tg], y = yt[tg];
  vp_d4 acc[NB];
  vp_f4 tile[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    acc[u] = vp_d4{0.0, 0.0, 0.0, 0.0};
    tile[u] = vp_f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  auto flush = [&]() {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += (double)tile[u][v];
      tile[u] = vp_f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
  };
  // local expansion
  const double* Xl = Lb + b * KP * C + r16;
  const double* Wt = wtgt + (ta ? ia : i0) * KP;
  for (int s4 = 0; s4 < KP / 4; ++s4) {
    const int k = 4 * s4 + kq;
    const float av = ta ? (float)Wt[k] : 0.0f;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      tile[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, (float)Xl[k * C + 16 * u], tile[u], 0, 0, 0);
  }
  flush();
  // adjacent boxes, row by row (consecutive boxes: one source range)
  int in_tile = 0;
  for (int dy = -1; dy <= 1; ++dy) {
    const int jy = iy + dy;
    if (jy < 0 || jy >= n) continue;
    const int64_t row = (int64_t)jy * n;
    const int64_t j0 = sptr[row + max(ix - 1, 0)], j1 = sptr[row + min(ix + 1, n - 1) + 1];
    if (j0 >= j1) continue;  // no sources (the pipeline's first loads need one)
    // software pipeline as in k_fmmb_leaf
    int64_t cols[NB];
    float cmask[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int64_t col = c0 + 16 * u + r16;
      cols[u] = col < R ? col : R - 1;
      cmask[u] = col < R ? 1.0f : 0.0f;
    }
    auto idx = [&](int64_t js) { const int64_t j = js + kq; return j < j1 ? j : j0; };
    int64_t jc = idx(j0), jn = idx(j0 + 4);
    double2 sw = sxy_s[jc], swn = sxy_s[jn];
    int32_t spn = sperm[jn];
    float qv[NB];
    {
      const float* q = Q32 + (int64_t)sperm[jc] * R;
      const float m = (j0 + kq < j1) ? 1.0f : 0.0f;
#pragma unroll
      for (int u = 0; u < NB; ++u) qv[u] = q[cols[u]] * (m * cmask[u]);
    }
    for (int64_t js = j0; js < j1; js += 4) {
      const int64_t jnn = idx(js + 8);
      const double2 swnn = sxy_s[jnn];
      const int32_t spnn = sperm[jnn];
      float qn[NB];
      {
        const float* q = Q32 + (int64_t)spn * R;
        const float m = (js + 4 + kq < j1) ? 1.0f : 0.0f;
#pragma unroll
        for (int u = 0; u < NB; ++u) qn[u] = q[cols[u]] * (m * cmask[u]);
      }
      const float dx = (float)(x - sw.x), dy2 = (float)(y - sw.y);
      const float g0 = __builtin_amdgcn_logf(fmaf(dy2, dy2, fmaf(dx, dx, kR2BiasF)));
      const float g = ta ? g0 : 0.0f;
#pragma unroll
      for (int u = 0; u < NB; ++u) tile[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, qv[u], tile[u], 0, 0, 0);
      sw = swn;
      swn = swnn;
      spn = spnn;
#pragma unroll
      for (int u = 0; u < NB; ++u) qv[u] = qn[u];
      if (++in_tile == 64) {  // 256 sources
        flush();
        in_tile = 0;
      }
    }
  }
  flush();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t i = i0 + 4 * kq + v;
    if (i < i1) {
      const int64_t o = (int64_t)tperm[i] * R + c0 + r16;
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (c0 + 16 * u + r16 < R) out[o + 16 * u] = acc[u][v];
    }
  }
}

// Work counts of a plan (statistics): the direct pairs of the adjacent leaf
// boxes (cnt[0]) and the M2L translations over all levels (cnt[1]), one
// thread per box of the level.
__global__ void k_fmm_work(const int32_t* __restrict__ cs, const int32_t* __restrict__ ct, int l, int leaf,
                           unsigned long long* __restrict__ cnt) {
  const int n = 1 << l;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (int64_t)n * n || ct[b] == 0) return;
  const int ix = (int)(b % n), iy = (int)(b / n);
  unsigned long long m2l = 0, near = 0;
  for (int jy = max(iy - 3, 0); jy <= min(iy + 3, n - 1); ++jy)
    for (int jx = max(ix - 3, 0); jx <= min(ix + 3, n - 1); ++jx) {
      const int32_t c = cs[(int64_t)jy * n + jx];
      if (abs(jx - ix) <= 1 && abs(jy - iy) <= 1)
        near += (unsigned long long)c;
      else if (abs((jx >> 1) - (ix >> 1)) <= 1 && abs((jy >> 1) - (iy >> 1)) <= 1 && c > 0)
        ++m2l;
    }
  if (l >= 2) atomicAdd(&cnt[1], m2l);
  if (leaf) atomicAdd(&cnt[0], near * (unsigned long long)ct[b]);
}

// Binomial coefficients up to n = 2 p in long double.
std::vector<long double> binomials(int nmax) {
  std::vector<long double> c((size_t)(nmax + 1) * (nmax + 1), 0.0L);
  for (int i = 0; i <= nmax; ++i) {
    c[(size_t)i * (nmax + 1)] = 1.0L;
    for (int k = 1; k <= i; ++k)
      c[(size_t)i * (nmax + 1) + k] = c[(size_t)(i - 1) * (nmax + 1) + k - 1] + (k < i ? c[(size_t)(i - 1) * (nmax + 1) + k] : 0.0L);
  }
  return c;
}

struct CLD {
  long double x, y;
};
inline CLD cl_mul(CLD a, CLD b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
inline CLD cl_pow(CLD a, int k) {
  CLD r{1.0L, 0.0L};
  for (int i = 0; i < k; ++i) r = cl_mul(r, a);
  return r;
}
inline CLD cl_inv(CLD a) {
  const long double d = a.x * a.x + a.y * a.y;
  return {a.x / d, -a.y / d};
}

// Translation operators of the scaled expansions (see the file header):
//   M2M_q[l][k], child quadrant q (bit 0: +x half, bit 1: +y half), d = child
//     centre - parent centre in parent widths:  [0][0] = 1,
//     [l][0] = -d^l / l, [l][k] = 2^-k d^(l-k) C(l-1, k-1) for 1 <= k <= l
//   L2L_q[m][l] = C(l, m) d^(l-m) 2^-m for l >= m
//   M2L_o[l][k], o = (dy + 3) 7 + dx + 3, z0 = dx + i dy (source box centre -
//     target box centre in box widths):  [0][0] = log(-z0), [0][k] = (-1)^k z0^-k,
//     [l][0] = -1 / (l z0^l), [l][k] = (-1)^k C(l+k-1, k-1) z0^-(l+k)
void fmm_operators(int p, std::vector<double2>& m2m, std::vector<double2>& l2l, std::vector<double2>& m2l);

// The M2L operators in the real, padded form ([49] of MP x KP: rows Re y then
// Im y, columns Re x then Im x), stored in the A-operand order of the MFMA
// steps: entry ((o tiles + t) KS + s) 64 + lane holds row 16 t + (lane & 15),
// column 4 s + (lane >> 4), so a wavefront reads 64 consecutive doubles per
// step.  Padding rows and columns are zero.
std::vector<double> fmm_m2l_real(int p, const std::vector<double2>& m2l, int MP, int KP) {
  const int P1 = p + 1, tiles = MP / 16, KS = KP / 4;
  std::vector<double> out((size_t)49 * MP * KP, 0.0);
  auto at = [&](int o, int row, int col) -> double& {
    return out[(((size_t)o * tiles + row / 16) * KS + col / 4) * 64 + (col % 4) * 16 + row % 16];
  };
  for (int o = 0; o < 49; ++o) {
    const double2* T = m2l.data() + (size_t)o * P1 * P1;
    for (int r = 0; r < P1; ++r)
      for (int c = 0; c < P1; ++c) {
        const double2 t = T[(size_t)r * P1 + c];
        at(o, r, c) = t.x;            // Re y <- Re T Re x
        at(o, r, P1 + c) = -t.y;      //        - Im T Im x
        at(o, P1 + r, c) = t.y;       // Im y <- Im T Re x
        at(o, P1 + r, P1 + c) = t.x;  //        + Re T Im x
      }
  }
  return out;
}
void fmm_operators(int p, std::vector<double2>& m2m, std::vector<double2>& l2l, std::vector<double2>& m2l) {
  const int P1 = p + 1, nb = 2 * p + 1;
  const std::vector<long double> C = binomials(nb);
  auto bin = [&](int i, int k) { return (k < 0 || k > i) ? 0.0L : C[(size_t)i * (nb + 1) + k]; };
  m2m.assign((size_t)4 * P1 * P1, make_double2(0.0, 0.0));
  l2l.assign((size_t)4 * P1 * P1, make_double2(0.0, 0.0));
  m2l.assign((size_t)49 * P1 * P1, make_double2(0.0, 0.0));
  for (int q = 0; q < 4; ++q) {
    const CLD d{(q & 1) ? 0.25L : -0.25L, (q & 2) ? 0.25L : -0.25L};
    double2* M = m2m.data() + (size_t)q * P1 * P1;
    double2* Lm = l2l.data() + (size_t)q * P1 * P1;
    M[0] = make_double2(1.0, 0.0);
    for (int l = 1; l <= p; ++l) {
      const CLD dl = cl_pow(d, l);
      M[(size_t)l * P1] = make_double2((double)(-dl.x / l), (double)(-dl.y / l));
      for (int k = 1; k <= l; ++k) {
        const CLD v = cl_pow(d, l - k);
        const long double f = bin(l - 1, k - 1) * std::ldexp(1.0L, -k);
        M[(size_t)l * P1 + k] = make_double2((double)(v.x * f), (double)(v.y * f));
      }
    }
    for (int m = 0; m <= p; ++m)
      for (int l = m; l <= p; ++l) {
        const CLD v = cl_pow(d, l - m);
        const long double f = bin(l, m) * std::ldexp(1.0L, -m);
        Lm[(size_t)m * P1 + l] = make_double2((double)(v.x * f), (double)(v.y * f));
      }
  }
  for (int dy = -3; dy <= 3; ++dy)
    for (int dx = -3; dx <= 3; ++dx) {
      if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
      double2* T = m2l.data() + (size_t)((dy + 3) * 7 + dx + 3) * P1 * P1;
      const CLD z0{(long double)dx, (long double)dy};
      const CLD iz = cl_inv(z0);
      // log(-z0)
      T[0] = make_double2((double)(0.5L * std::log(z0.x * z0.x + z0.y * z0.y)), (double)std::atan2(-z0.y, -z0.x));
      std::vector<CLD> izp(2 * P1 + 1);
      izp[0] = {1.0L, 0.0L};
      for (int k = 1; k <= 2 * p; ++k) izp[k] = cl_mul(izp[k - 1], iz);
      for (int k = 1; k <= p; ++k) {
        const long double sg = (k & 1) ? -1.0L : 1.0L;
        T[k] = make_double2((double)(sg * izp[k].x), (double)(sg * izp[k].y));
      }
      for (int l = 1; l <= p; ++l) {
        T[(size_t)l * P1] = make_double2((double)(-izp[l].x / l), (double)(-izp[l].y / l));
        for (int k = 1; k <= p; ++k) {
          const long double f = ((k & 1) ? -1.0L : 1.0L) * bin(l + k - 1, k - 1);
          T[(size_t)l * P1 + k] = make_double2((double)(f * izp[l + k].x), (double)(f * izp[l + k].y));
        }
      }
    }
}

}  // namespace

int64_t fmm_boxes(int L) {
  int64_t n = 0;
  for (int l = 0; l <= L; ++l) n += (int64_t)1 << (2 * l);
  return n;
}

int64_t fmm_workspace_doubles(const vp_plan* pl, int64_t R) {
  if (pl->fmm_terms <= 0) return 0;
  const int64_t nbox = fmm_boxes(pl->fmm_levels);
  // one density at a time: multipole and local coefficients (complex) of
  // every box, the charges in leaf order and the multipoles in real row
  // form; passes of 16, 32 or 64
  // densities: the real-form expansions [box][KP][16 NB]; they share the
  // space; 2 for alignment
  const int64_t one = 3 * 2 * nbox * (pl->fmm_terms + 1) + pl->n_src;
  const int64_t cols = R >= 64 ? 64 : R >= 32 ? 32 : R >= kMinBlockCols ? 16 : 0;
  const int64_t blk = 2 * nbox * pl->fmm_kp * cols;
  return std::max(one, blk) + 2;
}

hipError_t build_fmm(vp_plan* pl, int leaf, hipStream_t st) {
  const int64_t NS = pl->n_src, NT = pl->n_tgt;
  const int p = pl->fmm_terms;
  auto alloc = [&](void** ptr, size_t bytes) -> hipError_t { return plan_alloc(pl, ptr, bytes); };
  hipError_t e;
  // root square
  const int nred = 256;
  double* part = nullptr;
  std::vector<double> hp(4 * nred);
  {
    Scratch tb(pl->ctx, st);
    if ((e = tb.alloc((void**)&part, sizeof(double) * 4 * nred)) != hipSuccess) return e;
    k_fmm_bbox_partial<<<nred, kBlock, 0, st>>>(pl->sxy, NS, pl->xt, pl->yt, NT, part);
    if ((e = hipGetLastError()) == hipSuccess &&
        (e = hipMemcpyAsync(hp.data(), part, sizeof(double) * 4 * nred, hipMemcpyDeviceToHost, st)) == hipSuccess)
      e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) return e;
  double x0 = 1e300, y0 = 1e300, x1 = -1e300, y1 = -1e300;
  for (int i = 0; i < nred; ++i) {
    x0 = std::min(x0, hp[4 * i]);
    y0 = std::min(y0, hp[4 * i + 1]);
    x1 = std::max(x1, hp[4 * i + 2]);
    y1 = std::max(y1, hp[4 * i + 3]);
  }
  double w = std::max(x1 - x0, y1 - y0);
  w = w > 0.0 ? w * (1.0 + 1e-12) : 1.0;
  pl->fmm_x0 = 0.5 * (x0 + x1) - 0.5 * w;
  pl->fmm_y0 = 0.5 * (y0 + y1) - 0.5 * w;
  pl->fmm_width = w;
  // levels: about `leaf` sources per leaf box of the full grid
  int L = (int)std::lround(std::log((double)std::max<int64_t>(NS, 1) / leaf) / std::log(4.0));
  L = std::min(std::max(L, 2), kFmmMaxLevels);
  pl->fmm_levels = L;
  const int n = 1 << L;
  const int64_t nleaf = (int64_t)n * n;
  // keys and stable sort by leaf box
  uint32_t *skey = nullptr, *skey2 = nullptr, *tkey = nullptr, *tkey2 = nullptr;
  int32_t *sval = nullptr, *tval = nullptr, *cnt = nullptr;
  void* tmp = nullptr;
  size_t tmp_s = 0, tmp_t = 0;
  Scratch tmps(pl->ctx, st);
  auto talloc = [&](void** ptr, size_t bytes) { return tmps.alloc(ptr, bytes); };
  auto cleanup = [&]() { tmps.release(); };
  if ((e = alloc((void**)&pl->fmm_src_perm, sizeof(int32_t) * NS)) != hipSuccess ||
      (e = alloc((void**)&pl->fmm_tgt_perm, sizeof(int32_t) * NT)) != hipSuccess ||
      (e = alloc((void**)&pl->fmm_sxy, sizeof(double2) * NS)) != hipSuccess ||
      (e = alloc((void**)&pl->fmm_src_ptr, sizeof(int64_t) * (nleaf + 1))) != hipSuccess ||
      (e = alloc((void**)&pl->fmm_tgt_ptr, sizeof(int64_t) * (nleaf + 1))) != hipSuccess ||
      (e = talloc((void**)&skey, sizeof(uint32_t) * NS)) != hipSuccess ||
      (e = talloc((void**)&skey2, sizeof(uint32_t) * NS)) != hipSuccess ||
      (e = talloc((void**)&sval, sizeof(int32_t) * NS)) != hipSuccess ||
      (e = talloc((void**)&tkey, sizeof(uint32_t) * NT)) != hipSuccess ||
      (e = talloc((void**)&tkey2, sizeof(uint32_t) * NT)) != hipSuccess ||
      (e = talloc((void**)&tval, sizeof(int32_t) * NT)) != hipSuccess ||
      (e = talloc((void**)&cnt, sizeof(int32_t) * 2 * nleaf)) != hipSuccess) {
    cleanup();
    return e;
  }
  k_fmm_keys<<<blocks_for(NS + NT), kBlock, 0, st>>>(pl->sxy, NS, pl->xt, pl->yt, NT, pl->fmm_x0, pl->fmm_y0,
                                                     (double)n / w, n, skey, sval, tkey, tval);
  const int bits = 2 * L;
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_s, skey, skey2, sval, pl->fmm_src_perm, (int)NS, 0, bits,
                                              st)) != hipSuccess ||
      (e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_t, tkey, tkey2, tval, pl->fmm_tgt_perm, (int)NT, 0, bits,
                                              st)) != hipSuccess ||
      (e = talloc(&tmp, std::max(tmp_s, tmp_t))) != hipSuccess) {
    cleanup();
    return e;
  }
  const size_t tmp_bytes = std::max(tmp_s, tmp_t);
  size_t tb = tmp_bytes;
  if ((e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, skey, skey2, sval, pl->fmm_src_perm, (int)NS, 0, bits, st)) !=
      hipSuccess) {
    cleanup();
    return e;
  }
  tb = tmp_bytes;
  if ((e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, tkey, tkey2, tval, pl->fmm_tgt_perm, (int)NT, 0, bits, st)) !=
      hipSuccess) {
    cleanup();
    return e;
  }
  // leaf counts -> CSR pointers and per-level counts (host)
  if ((e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * 2 * nleaf, st)) != hipSuccess) {
    cleanup();
    return e;
  }
  k_fmm_count<<<blocks_for(NS), kBlock, 0, st>>>(skey, NS, cnt);
  k_fmm_count<<<blocks_for(NT), kBlock, 0, st>>>(tkey, NT, cnt + nleaf);
  k_fmm_gather2<<<blocks_for(NS), kBlock, 0, st>>>(pl->sxy, pl->fmm_src_perm, NS, pl->fmm_sxy);
  std::vector<int32_t> hc(2 * nleaf);
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * 2 * nleaf, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    cleanup();
    return e;
  }
  cleanup();
  std::vector<int64_t> sp(nleaf + 1), tp(nleaf + 1);
  sp[0] = tp[0] = 0;
  for (int64_t i = 0; i < nleaf; ++i) {
    sp[i + 1] = sp[i] + hc[i];
    tp[i + 1] = tp[i] + hc[nleaf + i];
  }
  // per-level source and target counts, levels 0..L concatenated
  const int64_t nbox = fmm_boxes(L);
  std::vector<int32_t> cs(nbox), ct(nbox);
  std::vector<int64_t> off(L + 2);
  off[0] = 0;
  for (int l = 0; l <= L; ++l) off[l + 1] = off[l] + ((int64_t)1 << (2 * l));
  for (int64_t i = 0; i < nleaf; ++i) {
    cs[off[L] + i] = hc[i];
    ct[off[L] + i] = hc[nleaf + i];
  }
  for (int l = L - 1; l >= 0; --l) {
    const int m = 1 << l;
    for (int iy = 0; iy < m; ++iy)
      for (int ix = 0; ix < m; ++ix) {
        int32_t a = 0, c = 0;
        for (int q = 0; q < 4; ++q) {
          const int64_t ch = off[l + 1] + (int64_t)(2 * iy + (q >> 1)) * (2 * m) + 2 * ix + (q & 1);
          a += cs[ch];
          c += ct[ch];
        }
        cs[off[l] + (int64_t)iy * m + ix] = a;
        ct[off[l] + (int64_t)iy * m + ix] = c;
      }
  }
  for (int l = 0; l <= L; ++l) pl->fmm_off[l] = off[l];
  pl->fmm_mp = (2 * (p + 1) + 15) / 16 * 16;
  pl->fmm_kp = (2 * (p + 1) + 3) / 4 * 4;
  // the translation operators depend only on p: built once per context and
  // order (a few ms of host work) and shared by its plans
  std::vector<double2> m2m, l2l, m2l;
  std::vector<double> m2l_r;
  vp_ctx::FmmOps& ops = pl->ctx->fmm_ops[p];
  if (!ops.m2l) {
    fmm_operators(p, m2m, l2l, m2l);
    m2l_r = fmm_m2l_real(p, m2l, pl->fmm_mp, pl->fmm_kp);
    const size_t b1 = sizeof(double2) * m2m.size(), b2 = sizeof(double2) * l2l.size(),
                 b3 = sizeof(double) * m2l_r.size();
    double2 *d1 = nullptr, *d2 = nullptr;
    double* d3 = nullptr;
    if ((e = hipMalloc((void**)&d1, b1)) != hipSuccess || (e = hipMalloc((void**)&d2, b2)) != hipSuccess ||
        (e = hipMalloc((void**)&d3, b3)) != hipSuccess ||
        (e = hipMemcpyAsync(d1, m2m.data(), b1, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d2, l2l.data(), b2, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d3, m2l_r.data(), b3, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {  // before the host tables go
      (void)hipStreamSynchronize(st);
      for (void* x : {(void*)d1, (void*)d2, (void*)d3})
        if (x) (void)hipFree(x);
      pl->ctx->fmm_ops.erase(p);
      return e;
    }
    ops.m2m = d1;
    ops.l2l = d2;
    ops.m2l = d3;
    ops.bytes = b1 + b2 + b3;
    pl->ctx->in_use += ops.bytes;
  }
  pl->fmm_m2m = ops.m2m;
  pl->fmm_l2l = ops.l2l;
  pl->fmm_m2l = ops.m2l;
  if ((e = alloc((void**)&pl->fmm_cnt_src, sizeof(int32_t) * nbox)) != hipSuccess ||
      (e = alloc((void**)&pl->fmm_cnt_tgt, sizeof(int32_t) * nbox)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(pl->fmm_src_ptr, sp.data(), sizeof(int64_t) * (nleaf + 1), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(pl->fmm_tgt_ptr, tp.data(), sizeof(int64_t) * (nleaf + 1), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(pl->fmm_cnt_src, cs.data(), sizeof(int32_t) * nbox, hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(pl->fmm_cnt_tgt, ct.data(), sizeof(int32_t) * nbox, hipMemcpyHostToDevice, st)) !=
          hipSuccess)
    return e;
  // work counts (plan statistics)
  {
    unsigned long long* d_cnt = nullptr;
    unsigned long long h_cnt[2] = {0, 0};
    Scratch tc(pl->ctx, st);
    if ((e = tc.alloc((void**)&d_cnt, sizeof(h_cnt))) != hipSuccess) return e;
    e = hipMemsetAsync(d_cnt, 0, sizeof(h_cnt), st);
    for (int l = 2; l <= L && e == hipSuccess; ++l) {
      k_fmm_work<<<blocks_for((int64_t)1 << (2 * l)), kBlock, 0, st>>>(pl->fmm_cnt_src + off[l], pl->fmm_cnt_tgt + off[l],
                                                                     l, l == L ? 1 : 0, d_cnt);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h_cnt, d_cnt, sizeof(h_cnt), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    tc.release();
    if (e != hipSuccess) return e;
    pl->fmm_near_pairs = (int64_t)h_cnt[0];
    pl->fmm_m2l_pairs = (int64_t)h_cnt[1];
  }
  pl->fmm_tgt_ptr_host = tp;
  // the leaf box of every target in leaf order (the single-density leaf pass)
  if ((e = alloc((void**)&pl->fmm_tbox, sizeof(int32_t) * std::max<int64_t>(NT, 1))) != hipSuccess) return e;
  k_fmm_tbox<<<blocks_for(nleaf), kBlock, 0, st>>>(pl->fmm_tgt_ptr, nleaf, pl->fmm_tbox);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the one-density leaf pass's tiles, longest first
  const int64_t n_tiles = (NT + 15) / 16;
  if (n_tiles > 0) {
    if ((e = alloc((void**)&pl->fmm_tile_order, sizeof(int32_t) * n_tiles)) != hipSuccess) return e;
    Scratch ts(pl->ctx, st);
    uint32_t *cost = nullptr, *cost2 = nullptr;
    int32_t* idx = nullptr;
    void* stmp = nullptr;
    size_t sbytes = 0;
    if ((e = ts.alloc((void**)&cost, sizeof(uint32_t) * n_tiles)) != hipSuccess ||
        (e = ts.alloc((void**)&cost2, sizeof(uint32_t) * n_tiles)) != hipSuccess ||
        (e = ts.alloc((void**)&idx, sizeof(int32_t) * n_tiles)) != hipSuccess ||
        (e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, sbytes, cost, cost2, idx, pl->fmm_tile_order,
                                                          (int)n_tiles, 0, 32, st)) != hipSuccess ||
        (e = ts.alloc(&stmp, std::max<size_t>(sbytes, 16))) != hipSuccess)
      return e;
    k_fmm_tile_cost<<<blocks_for(n_tiles), kBlock, 0, st>>>(pl->fmm_tbox, NT, pl->fmm_src_ptr, L, cost, idx);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipcub::DeviceRadixSort::SortPairsDescending(stmp, sbytes, cost, cost2, idx, pl->fmm_tile_order,
                                                          (int)n_tiles, 0, 32, st)) != hipSuccess)
      return e;
  }
  return hipStreamSynchronize(st);  // the host vectors above go out of scope
}

// Tables of the passes of blocks of 16 densities, built at the first evaluation
// that needs them (they cost 8 (N_src MP + N_tgt KP) bytes): P2M rows of
// the sources, L2P rows of the targets, and the (leaf box, first target)
// work list of their leaf pass.  Synchronises the stream.
hipError_t fmm_prepare_blocks(vp_plan* pl, int64_t R, hipStream_t st) {
  if (pl->fmm_terms <= 0 || R < kMinBlockCols || pl->fmm_vsrc) return hipSuccess;
  const int64_t NS = pl->n_src, NT = pl->n_tgt;
  const int L = pl->fmm_levels, n = 1 << L, p = pl->fmm_terms;
  const int64_t nleaf = (int64_t)n * n;
  const std::vector<int64_t>& tp = pl->fmm_tgt_ptr_host;
  std::vector<int2> tiles;
  for (int64_t b = 0; b < nleaf; ++b)
    for (int64_t i = tp[b]; i < tp[b + 1]; i += 16) tiles.push_back(make_int2((int)b, (int)i));
  const size_t bytes =
      sizeof(double) * (NS * pl->fmm_mp + NT * pl->fmm_kp) + sizeof(int2) * std::max<size_t>(tiles.size(), 1);
  // over the context's budget: no tables (the passes then run one density
  // at a time); a later evaluation tries again
  if (!ctx_fits(pl->ctx, bytes)) return hipSuccess;
  double *vsrc = nullptr, *wtgt = nullptr;
  int2* tt = nullptr;
  hipError_t e;
  // the blocks belong to the plan from here on, also when this fails
  if ((e = plan_alloc(pl, (void**)&vsrc, sizeof(double) * NS * pl->fmm_mp)) != hipSuccess ||
      (e = plan_alloc(pl, (void**)&wtgt, sizeof(double) * NT * pl->fmm_kp)) != hipSuccess ||
      (e = plan_alloc(pl, (void**)&tt, sizeof(int2) * std::max<size_t>(tiles.size(), 1))) != hipSuccess)
    return e;
  const double sL = pl->fmm_width / n;
  k_fmm_vsrc<<<blocks_for(NS), kBlock, 0, st>>>(pl->fmm_sxy, NS, pl->fmm_x0, pl->fmm_y0, sL, L, p, pl->fmm_mp, vsrc);
  k_fmm_wtgt<<<blocks_for(NT), kBlock, 0, st>>>(pl->xt, pl->yt, pl->fmm_tgt_perm, NT, pl->fmm_x0, pl->fmm_y0, sL, L, p,
                                                pl->fmm_kp, wtgt);
  e = hipGetLastError();
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpyAsync(tt, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  pl->fmm_vsrc = vsrc;
  pl->fmm_wtgt = wtgt;
  pl->fmm_ttile = tt;
  pl->fmm_n_ttiles = (int64_t)tiles.size();
  return hipSuccess;
}

// The far sum of every right-hand side by the FMM into out[t][R] (the
// first n_tgt R doubles of `partial`); ws = the FMM workspace
// (fmm_workspace_doubles).
hipError_t launch_fmm(const vp_plan* pl, const double* Q, int64_t R, double* out, double* ws, hipStream_t st,
                      int64_t* n_launches, const float* Q32) {
  const int p = pl->fmm_terms, P1 = p + 1, L = pl->fmm_levels;
  const int64_t nbox = fmm_boxes(L);
  // 16-byte alignment of the complex arrays
  double2* Mall = (double2*)(ws + ((uintptr_t)ws % 16 ? 1 : 0));
  double2* Lall = Mall + nbox * P1;
  double* Qs = (double*)(Lall + nbox * P1);
  double* Mr = Qs + pl->n_src;  // the multipoles in real row form (one density at a time)
  const int n = 1 << L;
  const int64_t nleaf = (int64_t)n * n;
  const double sL = pl->fmm_width / n;
  // blocks of 16 densities on the matrix cores, up to 4 blocks per pass
  const int MP = pl->fmm_mp, KP = pl->fmm_kp, tiles = MP / 16;
  // the M2L launches' level table (levels 2..L): one wavefront per (box,
  // row tile) for the blocks of densities, per (16 boxes, row tile) for one
  FmmLevels lv{}, lv1{};
  lv.l0 = lv1.l0 = 2;
  lv.l1 = lv1.l1 = L;
  {
    int64_t waves = 0, waves1 = 0;
    for (int l = 2; l <= L; ++l) {
      const int64_t nbl = (int64_t)1 << (2 * l);
      waves += nbl * tiles;
      waves1 += (nbl + 15) / 16 * tiles;
      lv.wave_end[l] = waves;
      lv1.wave_end[l] = waves1;
      lv.off[l] = lv1.off[l] = pl->fmm_off[l];
      lv.log_s[l] = lv1.log_s[l] = std::log(pl->fmm_width / (double)(1 << l));
    }
  }
  int64_t c0 = 0;
  while (pl->fmm_vsrc && R - c0 >= kMinBlockCols) {
    const int nbk = R - c0 >= 64 ? 4 : R - c0 >= 32 ? 2 : 1;
    const int C = 16 * nbk;
    double* Mb = (double*)Mall;
    double* Lb = Mb + nbox * KP * C;
#define VP_FMMB(NBV)                                                                                              \
  k_fmmb_p2m<NBV><<<(unsigned)((nleaf * tiles * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(                      \
      pl->fmm_vsrc, pl->fmm_src_perm, pl->fmm_src_ptr, Q, R, c0, nleaf, MP, KP, Mb + pl->fmm_off[L] * KP * C);     \
  for (int l = L - 1; l >= 2; --l) {                                                                              \
    const int64_t nt = ((int64_t)1 << (2 * l)) * P1 * C;                                                           \
    k_fmmb_m2m<<<blocks_for(nt), kBlock, 0, st>>>(Mb + pl->fmm_off[l + 1] * KP * C,                                 \
                                                  pl->fmm_cnt_src + pl->fmm_off[l + 1], l, p, KP, C, pl->fmm_m2m,   \
                                                  Mb + pl->fmm_off[l] * KP * C);                                    \
  }                                                                                                               \
  k_fmmb_m2l<NBV><<<(unsigned)((lv.wave_end[L] * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(                    \
      Mb, pl->fmm_cnt_src, pl->fmm_cnt_tgt, lv, MP, KP, pl->fmm_m2l, Lb);                                          \
  for (int l = 3; l <= L; ++l) {                                                                                  \
    const int64_t nbl = (int64_t)1 << (2 * l);                                                                     \
    k_fmmb_l2l<<<blocks_for(nbl * P1 * C), kBlock, 0, st>>>(pl->fmm_cnt_tgt + pl->fmm_off[l],                       \
                                                           Lb + pl->fmm_off[l - 1] * KP * C, l, p, KP, C,            \
                                                           pl->fmm_l2l, Lb + pl->fmm_off[l] * KP * C);               \
  }                                                                                                               \
  if (pl->fmm_n_ttiles > 0 && Q32)                                                                               \
    k_fmmb_leaf32<NBV><<<(unsigned)((pl->fmm_n_ttiles * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(               \
        Lb + pl->fmm_off[L] * KP * C, pl->fmm_wtgt, pl->fmm_ttile, pl->fmm_n_ttiles, pl->fmm_sxy, pl->fmm_src_perm,  \
        pl->fmm_src_ptr, pl->fmm_tgt_perm, pl->fmm_tgt_ptr, pl->xt, pl->yt, L, KP, Q32, R, c0, out);                 \
  else if (pl->fmm_n_ttiles > 0)                                                                                  \
    k_fmmb_leaf<NBV><<<(unsigned)((pl->fmm_n_ttiles * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(                 \
        Lb + pl->fmm_off[L] * KP * C, pl->fmm_wtgt, pl->fmm_ttile, pl->fmm_n_ttiles, pl->fmm_sxy, pl->fmm_src_perm,  \
        pl->fmm_src_ptr, pl->fmm_tgt_perm, pl->fmm_tgt_ptr, pl->xt, pl->yt, L, KP, pl->logtab, Q, R, c0, out)
    switch (nbk) {
      case 4: VP_FMMB(4); break;
      case 2: VP_FMMB(2); break;
      default: VP_FMMB(1); break;
    }
#undef VP_FMMB
    if (n_launches) *n_launches += 2 * L - 1;
    c0 = std::min<int64_t>(R, c0 + C);
  }
  // the remaining densities one at a time
  for (int64_t r = c0; r < R; ++r) {
    k_fmm_p2m<<<(unsigned)((nleaf * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        pl->fmm_sxy, pl->fmm_src_perm, pl->fmm_src_ptr, Q, R, r, L, pl->fmm_x0, pl->fmm_y0, sL, p,
        Mall + pl->fmm_off[L] * P1, Qs);
    for (int l = L - 1; l >= 2; --l) {
      const int64_t nt = ((int64_t)1 << (2 * l)) * P1;
      k_fmm_m2m<<<blocks_for(nt), kBlock, 0, st>>>(Mall + pl->fmm_off[l + 1] * P1, pl->fmm_cnt_src + pl->fmm_off[l + 1],
                                                   l, p, pl->fmm_m2m, Mall + pl->fmm_off[l] * P1);
    }
    k_fmm_mreal<<<blocks_for((pl->fmm_off[L] + nleaf - pl->fmm_off[2]) * P1), kBlock, 0, st>>>(Mall, lv1, p, Mr);
    k_fmm_m2l<<<(unsigned)((lv1.wave_end[L] * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        Mr, pl->fmm_cnt_src, pl->fmm_cnt_tgt, lv1, p, MP, KP, pl->fmm_m2l, Lall);
    for (int l = 3; l <= L; ++l) {
      const int64_t nbl = (int64_t)1 << (2 * l);
      k_fmm_l2l<<<blocks_for(nbl * P1), kBlock, 0, st>>>(pl->fmm_cnt_tgt + pl->fmm_off[l],
                                                        Lall + pl->fmm_off[l - 1] * P1, l, p, pl->fmm_l2l,
                                                        Lall + pl->fmm_off[l] * P1);
    }
    k_fmm_leaf<<<(unsigned)(((pl->n_tgt + 15) / 16 * 64 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        Lall + pl->fmm_off[L] * P1, pl->fmm_tbox, pl->n_tgt, pl->fmm_sxy, Qs, pl->fmm_src_ptr, pl->fmm_tgt_perm,
        pl->xt, pl->yt, L, pl->fmm_x0, pl->fmm_y0, sL, p, pl->logtab, R, r, pl->fmm_tile_order, out);
    if (n_launches) *n_launches += 2 * L;
  }
  return hipGetLastError();
}

}  // namespace vp
