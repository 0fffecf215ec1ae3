// Per-solve kernels (FP64):
//   k_coef_charges  c = V^{-1} F per triangle (Sec. 2.2 interpolation matrix)
//               and, in the same launch, the far charges
//               Q_j = w_j |J(xi_j)| f_h(y_j) / (4 pi) (Sec. 3.6: every far-rule
//               node is a point charge; the 1/2 of log r = log(r^2)/2 is
//               folded in)
//   k_far       U_far(x) = sum_j Q_j log|x - y_j|^2 over all sources: a
//               direct sum, targets across threads, sources read in
//               wavefront-uniform tiles (a pair at distance 0 gets a finite
//               value that the correction rows subtract again)
//   k_finish    u = sum of the far partials + sum over the target's self/near
//               pairs of row . c(triangle)  (Sec. 3.6 subtract-and-add)
#include <cmath>

#include "vp_internal.h"

namespace vp {
namespace {

constexpr int kBlock = 256;
constexpr double kInv4Pi = 0.07957747154594766788;

// Grid of a grid-stride launch: at most 2^20 blocks, so that a launch stays
// far below 2^32 work-items.
inline unsigned blocks_for(int64_t n, int b = kBlock) {
  const int64_t nb = (n + b - 1) / b;
  return (unsigned)(nb < (1 << 20) ? (nb > 0 ? nb : 1) : (1 << 20));
}

// Coefficients and far charges in one launch, as two independent parts:
// blocks [0, nb_c) take one (triangle, rhs) each: c = V^{-1} F (F and C are
// [T][NP][R]); the remaining blocks take one (source, rhs) each: the charge
// Q_j = w_j |J| f_h(y_j) / (4 pi) with f_h(y_j) = sum_i W_ji f_i read from the
// node values (W = E V^{-1}), zero in the source padding.  Q may be null.
// With many right-hand sides (tri_charges), the coefficient thread of
// (triangle, rhs) also writes that triangle's nf charges from the node
// values it holds, so F is read once; the charge blocks then only zero the
// padding.  With few, one thread per (source, rhs) keeps the device full.
template <int P>
__global__ __launch_bounds__(kBlock) void k_coef_charges(const double* __restrict__ F, const double* __restrict__ vinv,
                               const double* __restrict__ wfar, const double* __restrict__ swj, int nf,
                               int64_t n_tri, int64_t n_src_pad, int64_t R, unsigned nb_c, int tri_charges,
                               double* __restrict__ C, double* __restrict__ Q) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  if (blockIdx.x < nb_c) {
    const int64_t stride = (int64_t)nb_c * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_tri * R; g += stride) {
      const int64_t t = g / R, r = g - t * R;
      const double* f = F + (size_t)t * NP * R + r;
      double v[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) v[i] = f[(size_t)i * R];
      double* c = C + (size_t)t * NP * R + r;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) s = fma(vinv[k * NP + i], v[i], s);
        c[(size_t)k * R] = s;
      }
      if (tri_charges && Q) {
#pragma unroll 1
        for (int j = 0; j < nf; ++j) {
          const double* W = wfar + (size_t)j * NP;
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < NP; ++i) s = fma(W[i], v[i], s);
          const int64_t src = t * nf + j;
          Q[src * R + r] = s * swj[src] * kInv4Pi;
        }
      }
    }
    return;
  }
  const int64_t n_src = n_tri * nf;
  const int64_t stride = (int64_t)(gridDim.x - nb_c) * blockDim.x;
  const int64_t g0 = tri_charges ? n_src * R : 0;  // only the padding
  for (int64_t g = g0 + (int64_t)(blockIdx.x - nb_c) * blockDim.x + threadIdx.x; g < n_src_pad * R; g += stride) {
    const int64_t src = g / R, r = g - src * R;
    double q = 0.0;
    if (src < n_src) {
      const int64_t t = src / nf;
      const int j = (int)(src - t * nf);
      const double* f = F + (size_t)t * NP * R + r;
      const double* W = wfar + (size_t)j * NP;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) s = fma(W[i], f[(size_t)i * R], s);
      q = s * swj[src] * kInv4Pi;
    }
    Q[g] = q;
  }
}

// Direct far sum.  Each thread owns TPT targets (strided by the block
// size); the sources are read with wavefront-uniform addresses (scalar
// loads), RB right-hand sides share one logarithm per pair.  A linear block
// id b takes source chunk b % n_split and target block b / n_split, so with
// n_split a multiple of 8 the blocks that share a chunk sit on one XCD and
// its L2.  Each 256-source tile is summed on its own before it joins the
// running total (two-level summation).  Chunks are whole multiples of 64
// sources and the sources are padded to a multiple of 256 with zero
// charges.  With one right-hand side the exponent part of each logarithm is
// accumulated apart (sum Q e, times ln 2 at the end).  The shapes
// (VP_FAR_* of the C interface): WIDE runs 1024-thread blocks with the
// 4096-entry table (vp_log_wide_parts), whose 64 KiB load a long source
// chunk amortises; the NARROW shapes run 256-thread blocks with the
// 256-entry table, for target sets too small to fill the device with wide
// blocks.  With several right-hand sides the logarithm is a small share of
// the work per pair and the blocks are always narrow.
template <int S, int RB>
struct FarShape {
  static constexpr bool kWide = S == VP_FAR_WIDE && RB == 1;
  static constexpr int kThreads = kWide ? 1024 : 256;
  static constexpr int kTPT = S == VP_FAR_NARROW1 ? 1 : 2;
  static constexpr int kTab = kWide ? kFarLogTab : kLogTab;
};

template <int RB, int S>
__global__ __launch_bounds__((FarShape<S, RB>::kThreads)) void k_far(
    const double2* __restrict__ sxy, const double* __restrict__ Q, int64_t n_src_pad, int64_t R, int64_t r0,
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
    int64_t n_split, const double2* __restrict__ logtab, double* __restrict__ partial) {
  using Sh = FarShape<S, RB>;
  constexpr int kB = Sh::kThreads, kTab = Sh::kTab, TPT = Sh::kTPT;
  __shared__ double2 tab[kTab + 1];
  for (int i = threadIdx.x; i <= kTab; i += kB) tab[i] = logtab[i];
  __syncthreads();
  constexpr bool kSplitExp = (RB == 1);
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  double x[TPT], y[TPT];
  int64_t t[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    t[k] = tb * (kB * TPT) + k * kB + threadIdx.x;
    const bool act = t[k] < n_tgt;
    x[k] = act ? xt[t[k]] : 0.0;
    y[k] = act ? yt[t[k]] : 0.0;
  }
  const int64_t s_begin = chunk * per_split;
  const int64_t s_end = min(n_src_pad, s_begin + per_split);
  double acc[TPT][RB], acc_e[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    acc_e[k] = 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[k][r] = 0.0;
  }
  for (int64_t j0 = s_begin; j0 < s_end; j0 += 256) {
    const int64_t j1 = min(s_end, j0 + 256);
    double tile[TPT][RB], tile_e[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      tile_e[k] = 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) tile[k][r] = 0.0;
    }
    for (int64_t j = j0; j < j1; j += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 s = sxy[j + u];
        double q[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) q[r] = Q[(j + u) * R + r0 + r];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
          const double dx = x[k] - s.x, dy = y[k] - s.y;
          const double r2 = fma(dy, dy, fma(dx, dx, kR2Bias));
          if (kSplitExp) {
            double e, rest;
            if (Sh::kWide)
              vp_log_wide_parts(r2, tab, e, rest);
            else
              vp_log_parts(r2, tab, e, rest);
            tile_e[k] = fma(q[0], e, tile_e[k]);
            tile[k][0] = fma(q[0], rest, tile[k][0]);
          } else {
            const double lg = vp_log(r2, tab);
#pragma unroll
            for (int r = 0; r < RB; ++r) tile[k][r] = fma(q[r], lg, tile[k][r]);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      acc_e[k] += tile_e[k];
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[k][r] += tile[k][r];
    }
  }
  const double2 l2 = tab[kTab];
#pragma unroll
  for (int k = 0; k < TPT; ++k)
    if (t[k] < n_tgt) {
      if (kSplitExp) acc[k][0] += fma(acc_e[k], l2.x, acc_e[k] * l2.y);
#pragma unroll
      for (int r = 0; r < RB; ++r) partial[((size_t)chunk * n_tgt + t[k]) * R + r0 + r] = acc[k][r];
    }
}

// Mixed-precision far sum (same decomposition as k_far): r^2 + 2^-100 and
// the base-2 logarithm (the hardware v_log_f32) are FP32, the charges are
// FP32 with ln 2 folded in (Q32 = Q ln 2, so Q32 log2(r^2) = Q log(r^2)),
// each 256-source tile is summed in FP32 and the tiles are summed in FP64.
// The pair difference, per group of 64 sources (centre c, radius a; each
// source's FP32 offset s - c is a plan table): when the group's circle
// lies 3a beyond the circle around the block's targets, every pair has
// r >= 2a and |x - c| <= 1.5 r, so the FP32 offset x - c (once per target
// and group) minus s - c gives the difference to a relative 3 2^-24 with
// one FP32 subtraction per coordinate.  Nearer groups (including targets
// on or next to a source) take the difference in FP64, rounded to FP32.
template <int RB, int TPT>
__global__ __launch_bounds__(kBlock) void k_far32(const double2* __restrict__ sxy, const double* __restrict__ sgrp,
                                                  const float2* __restrict__ soff,
                                                  const float* __restrict__ Q32, int64_t n_src_pad, int64_t R,
                                                  int64_t r0, const double* __restrict__ xt,
                                                  const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
                                                  int64_t n_split, double* __restrict__ partial) {
  __shared__ double red[4][kBlock / 64];
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  double x[TPT], y[TPT];
  int64_t t[TPT];
  double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    t[k] = tb * (kBlock * TPT) + k * kBlock + threadIdx.x;
    const bool act = t[k] < n_tgt;
    x[k] = act ? xt[t[k]] : 0.0;
    y[k] = act ? yt[t[k]] : 0.0;
    if (act) {
      bx0 = fmin(bx0, x[k]);
      bx1 = fmax(bx1, x[k]);
      by0 = fmin(by0, y[k]);
      by1 = fmax(by1, y[k]);
    }
  }
  // the block's target bounding box: wavefront, then block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    bx0 = fmin(bx0, __shfl_xor(bx0, o));
    bx1 = fmax(bx1, __shfl_xor(bx1, o));
    by0 = fmin(by0, __shfl_xor(by0, o));
    by1 = fmax(by1, __shfl_xor(by1, o));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = bx0;
    red[1][wv] = bx1;
    red[2][wv] = by0;
    red[3][wv] = by1;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    bx0 = fmin(bx0, red[0][w]);
    bx1 = fmax(bx1, red[1][w]);
    by0 = fmin(by0, red[2][w]);
    by1 = fmax(by1, red[3][w]);
  }
  const double ox = 0.5 * (bx0 + bx1), oy = 0.5 * (by0 + by1);
  const double rb = 0.5 * sqrt((bx1 - bx0) * (bx1 - bx0) + (by1 - by0) * (by1 - by0));
  const int64_t s_begin = chunk * per_split;
  const int64_t s_end = min(n_src_pad, s_begin + per_split);
  double acc[TPT][RB];
#pragma unroll
  for (int k = 0; k < TPT; ++k)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[k][r] = 0.0;
  for (int64_t j0 = s_begin; j0 < s_end; j0 += 256) {
    const int64_t j1 = min(s_end, j0 + 256);
    float tile[TPT][RB];
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int r = 0; r < RB; ++r) tile[k][r] = 0.0f;
    // chunks and tiles are multiples of 64 sources: whole groups
    for (int64_t jg = j0; jg < j1; jg += 64) {
      const double* G = sgrp + 3 * (jg >> 6);
      const double gdx = G[0] - ox, gdy = G[1] - oy, lim = rb + 4.0 * G[2];
      if (gdx * gdx + gdy * gdy >= lim * lim) {  // the whole block alike
        float xg[TPT], yg[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
          xg[k] = (float)(x[k] - G[0]);
          yg[k] = (float)(y[k] - G[1]);
        }
        for (int64_t j = jg; j < jg + 64; j += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float2 so = soff[j + u];
            float q[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) q[r] = Q32[(j + u) * R + r0 + r];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
              const float dx = xg[k] - so.x, dy = yg[k] - so.y;
              const float r2 = fmaf(dy, dy, fmaf(dx, dx, kR2BiasF));
              const float lg = __builtin_amdgcn_logf(r2);
#pragma unroll
              for (int r = 0; r < RB; ++r) tile[k][r] = fmaf(q[r], lg, tile[k][r]);
            }
          }
        }
      } else {
        for (int64_t j = jg; j < jg + 64; j += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double2 s = sxy[j + u];
            float q[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) q[r] = Q32[(j + u) * R + r0 + r];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
              const float dx = (float)(x[k] - s.x), dy = (float)(y[k] - s.y);
              const float r2 = fmaf(dy, dy, fmaf(dx, dx, kR2BiasF));
              const float lg = __builtin_amdgcn_logf(r2);
#pragma unroll
              for (int r = 0; r < RB; ++r) tile[k][r] = fmaf(q[r], lg, tile[k][r]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[k][r] += (double)tile[k][r];
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k)
    if (t[k] < n_tgt) {
#pragma unroll
      for (int r = 0; r < RB; ++r) partial[((size_t)chunk * n_tgt + t[k]) * R + r0 + r] = acc[k][r];
    }
}

// Far sum for 16 NT right-hand sides at once on the matrix cores: the sum
// U[t][r] = sum_j G[t][j] Q[j][r] with G[t][j] = log(r_tj^2) is a product
// of a generated matrix with the charge matrix.  Each wavefront owns 16 MT
// targets (MT = 1, 2 or 4 tiles of 16) and walks its source chunk 4 sources
// at a time (chunks are multiples of 64 sources, so every lane of the
// wavefront takes the same number of steps);
// lane l generates G for target 16 m + (l & 15) and source l >> 4 of the
// step, i.e. exactly the A operand of a 16x16x4 MFMA, and loads
// Q[source l >> 4][16 n + (l & 15)], the B operand; every pair costs one
// logarithm however many right-hand sides share it.  Element v of lane l of
// the result tile holds RHS l & 15 of target (l >> 4) + 4 v (FP64 MFMA) or
// 4 (l >> 4) + v (FP32 MFMA).  Source chunks, padding and the XCD-aware
// block order are those of k_far.
//   k_far_mfma64  FP64 G (the 4096-entry table logarithm), FP64 MFMA
//   k_far_mfma32  FP32 G (v_log_f32 of the FP32 r^2, charges times ln 2),
//                 FP32 MFMA over 256-source tiles, tiles summed in FP64
typedef double vp_d4 __attribute__((ext_vector_type(4)));
typedef float vp_f4 __attribute__((ext_vector_type(4)));

template <int NT, int MT>
__global__ __launch_bounds__(kBlock, 2) void k_far_mfma64(
    const double2* __restrict__ sxy, const double* __restrict__ Q, int64_t n_src_pad, int64_t R, int64_t r0,
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
    int64_t n_split, const double2* __restrict__ logtab, double* __restrict__ partial) {
  constexpr int kTargets = (kBlock / 64) * 16 * MT;  // per block
  __shared__ double2 tab[kFarLogTab + 1];
  for (int i = threadIdx.x; i <= kFarLogTab; i += kBlock) tab[i] = logtab[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, kk = lane >> 4, nn = lane & 15;
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  const int64_t t0 = tb * kTargets + (threadIdx.x >> 6) * (16 * MT);
  double x[MT], y[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int64_t t = t0 + 16 * m + nn;
    x[m] = t < n_tgt ? xt[t] : 0.0;
    y[m] = t < n_tgt ? yt[t] : 0.0;
  }
  const int64_t s_begin = chunk * per_split;
  const int64_t s_end = min(n_src_pad, s_begin + per_split);
  const double2 l2 = tab[kFarLogTab];
  vp_d4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = vp_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int64_t j = s_begin + kk; j < s_end; j += 4) {
    const double2 s = sxy[j];
    double q[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) q[n] = Q[j * R + r0 + 16 * n + nn];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const double dx = x[m] - s.x, dy = y[m] - s.y;
      const double r2 = fma(dy, dy, fma(dx, dx, kR2Bias));
      double e, rest;
      vp_log_wide_parts(r2, tab, e, rest);
      const double g = fma(e, l2.x, fma(e, l2.y, rest));
#pragma unroll
      for (int n = 0; n < NT; ++n) acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(g, q[n], acc[m][n], 0, 0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t t = t0 + 16 * m + kk + 4 * v;
      if (t < n_tgt) {
#pragma unroll
        for (int n = 0; n < NT; ++n) partial[((size_t)chunk * n_tgt + t) * R + r0 + 16 * n + nn] = acc[m][n][v];
      }
    }
}

template <int NT, int MT>
__global__ __launch_bounds__(kBlock, 2) void k_far_mfma32(
    const double2* __restrict__ sxy, const float* __restrict__ Q32, int64_t n_src_pad, int64_t R, int64_t r0,
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
    int64_t n_split, double* __restrict__ partial) {
  constexpr int kTargets = (kBlock / 64) * 16 * MT;  // per block
  const int lane = threadIdx.x & 63, kk = lane >> 4, nn = lane & 15;
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  const int64_t t0 = tb * kTargets + (threadIdx.x >> 6) * (16 * MT);
  double x[MT], y[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int64_t t = t0 + 16 * m + nn;
    x[m] = t < n_tgt ? xt[t] : 0.0;
    y[m] = t < n_tgt ? yt[t] : 0.0;
  }
  const int64_t s_begin = chunk * per_split;
  const int64_t s_end = min(n_src_pad, s_begin + per_split);
  vp_d4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n] = vp_d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t j0 = s_begin; j0 < s_end; j0 += 256) {
    const int64_t j1 = min(s_end, j0 + 256);
    vp_f4 tile[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) tile[m][n] = vp_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 2
    for (int64_t j = j0 + kk; j < j1; j += 4) {
      const double2 s = sxy[j];
      float q[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) q[n] = Q32[j * R + r0 + 16 * n + nn];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const float dx = (float)(x[m] - s.x), dy = (float)(y[m] - s.y);
        const float g = __builtin_amdgcn_logf(fmaf(dy, dy, fmaf(dx, dx, kR2BiasF)));
#pragma unroll
        for (int n = 0; n < NT; ++n) tile[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, q[n], tile[m][n], 0, 0, 0);
      }
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[m][n][v] += (double)tile[m][n][v];
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t t = t0 + 16 * m + 4 * kk + v;
      if (t < n_tgt) {
#pragma unroll
        for (int n = 0; n < NT; ++n) partial[((size_t)chunk * n_tgt + t) * R + r0 + 16 * n + nn] = acc[m][n][v];
      }
    }
}


__global__ void k_to_f32_ln2(const double* __restrict__ Q, int64_t n, float* __restrict__ Q32) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    Q32[i] = (float)(Q[i] * 0.69314718055994530942);
}

__global__ void k_pack(const double* __restrict__ src, int64_t rows, int64_t sc, double* __restrict__ dst,
                       int64_t dc, int64_t c0) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < rows * sc; g += stride) {
    const int64_t i = g / sc, r = g - i * sc;
    dst[i * dc + c0 + r] = src[g];
  }
}

__global__ void k_unpack(const double* __restrict__ src, int64_t rows, int64_t sc, int64_t c0,
                         double* __restrict__ dst, int64_t dc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < rows * dc; g += stride) {
    const int64_t i = g / dc, r = g - i * dc;
    dst[g] = src[i * sc + c0 + r];
  }
}

// G lanes per (target, rhs): the lanes share out the far partials and the
// target's correction rows and are summed by a butterfly over the group.
// G = 1 is one thread per (target, rhs); G = 4 or 16 serves target sets too
// small to fill the device one thread each, where the serial walk over a
// long near list would set the time.
template <int P, int G>
__global__ __launch_bounds__(kBlock) void k_finish(const double* __restrict__ partial, int64_t n_split,
                                                   int64_t n_tgt, int64_t R, int64_t r0,
                                                   const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ pair_tri,
                                                   const double* __restrict__ rows, const double* __restrict__ C,
                                                   int far_only, double* __restrict__ U) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int lane = (int)(threadIdx.x % G);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / G);
  const int64_t Rr = R - r0;  // columns r0 .. R-1
  for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; g < n_tgt * Rr; g += stride) {
    const int64_t t = g / Rr, r = r0 + (g - t * Rr);
    double u = 0.0;
#pragma unroll 8
    for (int64_t s = lane; s < n_split; s += G) u += partial[((size_t)s * n_tgt + t) * R + r];
    if (!far_only) {
      double corr = 0.0;
      for (int64_t p = row_ptr[t] + lane; p < row_ptr[t + 1]; p += G) {
        const double* row = rows + (size_t)p * NP;
        const double* c = C + (size_t)pair_tri[p] * NP * R + r;
#pragma unroll
        for (int k = 0; k < NP; ++k) corr = fma(row[k], c[(size_t)k * R], corr);
      }
      u += corr;
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) u += __shfl_xor(u, off, G);
    if (lane == 0) U[t * R + r] = u;
  }
}

// The same sum with the G lanes of a target striding over its rows as one
// flat array of pairs x n_p values, so that consecutive lanes read
// consecutive row values (coalesced): for targets with long near lists,
// where the rows' bytes set the time.
template <int P, int G>
__global__ __launch_bounds__(kBlock) void k_finish_flat(const double* __restrict__ partial, int64_t n_split,
                                                        int64_t n_tgt, int64_t R, int64_t r0,
                                                        const int64_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ pair_tri,
                                                        const double* __restrict__ rows,
                                                        const double* __restrict__ C, int far_only,
                                                        double* __restrict__ U) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int lane = (int)(threadIdx.x % G);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / G);
  const int64_t Rr = R - r0;
  for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; g < n_tgt * Rr; g += stride) {
    const int64_t t = g / Rr, r = r0 + (g - t * Rr);
    double u = 0.0;
    for (int64_t s = lane; s < n_split; s += G) u += partial[((size_t)s * n_tgt + t) * R + r];
    if (!far_only) {
      const int64_t p0 = row_ptr[t];
      // one target's values (its pairs x n_p) stay far below 2^31
      const uint32_t nv = (uint32_t)((row_ptr[t + 1] - p0) * NP);
      const double* rw = rows + (size_t)p0 * NP;
      const int32_t* tri = pair_tri + p0;
      double corr = 0.0;
#pragma unroll 4
      for (uint32_t f = lane; f < nv; f += G) {
        const uint32_t j = f / NP, k = f - j * NP;
        corr = fma(rw[f], C[((size_t)tri[j] * NP + k) * R + r], corr);
      }
      u += corr;
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) u += __shfl_xor(u, off, G);
    if (lane == 0) U[t * R + r] = u;
  }
}

}  // namespace

#define VP_DISPATCH_P(p, CALL)   \
  switch (p) {                   \
    case 1: { constexpr int P = 1; CALL; } break; \
    case 2: { constexpr int P = 2; CALL; } break; \
    case 3: { constexpr int P = 3; CALL; } break; \
    case 4: { constexpr int P = 4; CALL; } break; \
    case 5: { constexpr int P = 5; CALL; } break; \
    case 6: { constexpr int P = 6; CALL; } break; \
    case 7: { constexpr int P = 7; CALL; } break; \
    case 8: { constexpr int P = 8; CALL; } break; \
    case 9: { constexpr int P = 9; CALL; } break; \
    case 10: { constexpr int P = 10; CALL; } break; \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_pack_columns(const double* src, int64_t rows, int64_t src_cols, double* dst, int64_t dst_cols,
                               int64_t c0, hipStream_t st) {
  if (rows * src_cols == 0) return hipSuccess;
  k_pack<<<blocks_for(rows * src_cols), kBlock, 0, st>>>(src, rows, src_cols, dst, dst_cols, c0);
  return hipGetLastError();
}

hipError_t launch_unpack_columns(const double* src, int64_t rows, int64_t src_cols, int64_t c0, double* dst,
                                 int64_t dst_cols, hipStream_t st) {
  if (rows * dst_cols == 0) return hipSuccess;
  k_unpack<<<blocks_for(rows * dst_cols), kBlock, 0, st>>>(src, rows, src_cols, c0, dst, dst_cols);
  return hipGetLastError();
}

hipError_t launch_coefficients(const vp_plan* pl, const double* F, int64_t R, double* C, double* Q, hipStream_t st) {
  const int64_t T = pl->n_tri;
  if (T == 0 && !Q) return hipSuccess;
  // from 16 right-hand sides on, the coefficient threads write the charges
  const int tri = R >= 16 ? 1 : 0;
  const unsigned nb_c = T > 0 ? blocks_for(T * R) : 0;
  const unsigned nb_q = Q ? blocks_for((tri ? pl->n_src_pad - pl->n_src : pl->n_src_pad) * R) : 0;
  if (nb_c + nb_q == 0) return hipSuccess;
  VP_DISPATCH_P(pl->p, (k_coef_charges<P><<<nb_c + nb_q, kBlock, 0, st>>>(F, pl->vinv, pl->wfar, pl->swj, pl->n_f, T,
                                                                          pl->n_src_pad, R, nb_c, tri, C, Q)));
  return hipGetLastError();
}

namespace {

template <int RB, int S>
hipError_t far_valu(const vp_plan* pl, const double* Q, int64_t R, int64_t r0, int64_t per, int64_t n_split,
                    double* partial, hipStream_t st) {
  using Sh = FarShape<S, RB>;
  const int64_t NT = pl->n_tgt, tpb = (int64_t)Sh::kThreads * Sh::kTPT;
  const int64_t nb = (NT + tpb - 1) / tpb * n_split;
  if (nb * Sh::kThreads >= (1LL << 32)) return hipErrorInvalidConfiguration;
  k_far<RB, S><<<dim3((unsigned)nb), Sh::kThreads, 0, st>>>(pl->sxy, Q, pl->n_src_pad, R, r0, pl->xt, pl->yt, NT,
                                                            per, n_split, Sh::kWide ? pl->logtab_wide : pl->logtab,
                                                            partial);
  return hipSuccess;
}

template <int RB, int TPT>
hipError_t far_valu32(const vp_plan* pl, const float* Q32, int64_t R, int64_t r0, int64_t per, int64_t n_split,
                      double* partial, hipStream_t st) {
  const int64_t NT = pl->n_tgt, tpb = (int64_t)kBlock * TPT;
  const int64_t nb = (NT + tpb - 1) / tpb * n_split;
  if (nb * kBlock >= (1LL << 32)) return hipErrorInvalidConfiguration;
  k_far32<RB, TPT><<<dim3((unsigned)nb), kBlock, 0, st>>>(pl->sxy, pl->sgrp, pl->soff, Q32, pl->n_src_pad, R, r0,
                                                          pl->xt, pl->yt, NT, per, n_split, partial);
  return hipSuccess;
}

template <int NT, int MT>
hipError_t far_mfma(const vp_plan* pl, const double* Q, const float* Q32, int64_t R, int64_t r0, int64_t per,
                    int64_t n_split, double* partial, hipStream_t st) {
  const int64_t N = pl->n_tgt, tpb = (int64_t)(kBlock / 64) * 16 * MT;
  const int64_t nb = (N + tpb - 1) / tpb * n_split;
  if (nb * kBlock >= (1LL << 32)) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nb);
  if (Q32)
    k_far_mfma32<NT, MT><<<grid, kBlock, 0, st>>>(pl->sxy, Q32, pl->n_src_pad, R, r0, pl->xt, pl->yt, N, per,
                                                  n_split, partial);
  else
    k_far_mfma64<NT, MT><<<grid, kBlock, 0, st>>>(pl->sxy, Q, pl->n_src_pad, R, r0, pl->xt, pl->yt, N, per,
                                                  n_split, pl->logtab_wide, partial);
  return hipSuccess;
}

template <int NT>
hipError_t far_mfma_mt(int mt, const vp_plan* pl, const double* Q, const float* Q32, int64_t R, int64_t r0,
                       int64_t per, int64_t n_split, double* partial, hipStream_t st) {
  switch (mt) {
    case 1: return far_mfma<NT, 1>(pl, Q, Q32, R, r0, per, n_split, partial, st);
    case 2: return far_mfma<NT, 2>(pl, Q, Q32, R, r0, per, n_split, partial, st);
    default: return far_mfma<NT, 4>(pl, Q, Q32, R, r0, per, n_split, partial, st);
  }
}

template <int RB>
hipError_t far_valu_shape(int shape, const vp_plan* pl, const double* Q, const float* Q32, int64_t R, int64_t r0,
                          int64_t per, int64_t n_split, double* partial, hipStream_t st) {
  if (Q32)
    return shape == VP_FAR_NARROW1 ? far_valu32<RB, 1>(pl, Q32, R, r0, per, n_split, partial, st)
                                   : far_valu32<RB, 2>(pl, Q32, R, r0, per, n_split, partial, st);
  switch (shape) {
    case VP_FAR_NARROW1: return far_valu<RB, VP_FAR_NARROW1>(pl, Q, R, r0, per, n_split, partial, st);
    case VP_FAR_NARROW2: return far_valu<RB, VP_FAR_NARROW2>(pl, Q, R, r0, per, n_split, partial, st);
    default: return far_valu<RB, VP_FAR_WIDE>(pl, Q, R, r0, per, n_split, partial, st);
  }
}

}  // namespace

int64_t far_targets_per_block(const vp_far_config& cfg, int64_t R, bool mixed) {
  if (R >= 16) return (int64_t)(kBlock / 64) * 16 * cfg.mfma_tiles;
  const int64_t tpt = cfg.shape == VP_FAR_NARROW1 ? 1 : 2;
  const int64_t threads = (!mixed && R == 1 && cfg.shape == VP_FAR_WIDE) ? 1024 : kBlock;
  return threads * tpt;
}

hipError_t launch_far(const vp_plan* pl, const double* Q, int64_t R, const vp_far_config& cfg, double* partial,
                      hipStream_t st, int64_t* n_launches, float* Q32) {
  const int64_t NT = pl->n_tgt, NS = pl->n_src_pad;
  if (NT == 0) return hipSuccess;
  // FMM plans: one partial sum per target, the FMM's workspace after it
  // (FP64 also in mixed precision)
  if (pl->fmm_terms > 0) {
    // mixed precision: the leaf passes of blocks of densities in FP32
    if (Q32 && R >= kMinBlockCols) k_to_f32_ln2<<<blocks_for(NS * R), kBlock, 0, st>>>(Q, NS * R, Q32);
    return launch_fmm(pl, Q, R, partial, partial + NT * R, st, n_launches, R >= kMinBlockCols ? Q32 : nullptr);
  }
  const int64_t n_split = cfg.n_split;
  if (n_split < 1 || n_split > NS) return hipErrorInvalidValue;
  // chunk length: a multiple of 64 sources
  int64_t per = (NS + n_split - 1) / n_split;
  per = ((per + 63) / 64) * 64;
  if (Q32) k_to_f32_ln2<<<blocks_for(NS * R), kBlock, 0, st>>>(Q, NS * R, Q32);
  hipError_t e = hipSuccess;
  int64_t r0 = 0;
  // blocks of 16, 32 or 64 right-hand sides on the matrix cores
  while (R - r0 >= 16 && e == hipSuccess) {
    const int64_t left = R - r0;
    const int nt = left >= 64 ? 4 : left >= 32 ? 2 : 1;
    switch (nt) {
      case 4: e = far_mfma_mt<4>(cfg.mfma_tiles, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
      case 2: e = far_mfma_mt<2>(cfg.mfma_tiles, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
      default: e = far_mfma_mt<1>(cfg.mfma_tiles, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
    }
    if (n_launches) ++*n_launches;
    r0 += 16 * nt;
  }
  // the remaining right-hand sides on the vector ALUs (RB of them share each logarithm)
  while (r0 < R && e == hipSuccess) {
    const int64_t left = R - r0;
    const int rb = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    switch (rb) {
      case 8: e = far_valu_shape<8>(cfg.shape, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
      case 4: e = far_valu_shape<4>(cfg.shape, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
      case 2: e = far_valu_shape<2>(cfg.shape, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
      default: e = far_valu_shape<1>(cfg.shape, pl, Q, Q32, R, r0, per, n_split, partial, st); break;
    }
    if (n_launches) ++*n_launches;
    r0 += rb;
  }
  return e != hipSuccess ? e : hipGetLastError();
}

// Below this many clusters (8192 targets) the vector-ALU apply with lane
// groups is faster (unit square, 1920 targets, 32 right-hand sides: 44 us
// against 75 us).
constexpr int64_t kCorrMfmaMinClusters = 512;

hipError_t launch_finish(const vp_plan* pl, const double* partial, int64_t n_split, const double* C, int64_t R,
                         bool far_only, double* U, hipStream_t st) {
  const int64_t NT = pl->n_tgt;
  if (NT == 0) return hipSuccess;
  // blocks of 64, 32 or 16 right-hand sides on the matrix cores, once there
  // are enough 16-target clusters (one wavefront each) to fill the device
  int64_t r0 = 0;
  while (pl->n_cl >= kCorrMfmaMinClusters && R - r0 >= kMinBlockCols) {
    const int nt = R - r0 >= 64 ? 4 : R - r0 >= 32 ? 2 : 1;
    const hipError_t e = launch_corr_mfma(pl, partial, n_split, C, R, r0, nt, far_only, U, st);
    if (e != hipSuccess) return e;
    r0 = std::min<int64_t>(R, r0 + 16 * nt);
  }
  if (r0 == R) return hipSuccess;
  // the rest on the vector ALUs; lanes per (target, rhs): enough
  // work-items to fill the device
  const int64_t n = NT * (R - r0);
  // long near lists (8 or more pairs per target on average) at sizes that
  // fill the device: 16 lanes per (target, rhs) reading the rows flat
  if (n >= (1 << 17) && pl->n_pairs >= 8 * NT) {
    VP_DISPATCH_P(pl->p, (k_finish_flat<P, 16><<<blocks_for(n * 16), kBlock, 0, st>>>(
                              partial, n_split, NT, R, r0, pl->row_ptr, pl->pair_tri, pl->rows, C, far_only ? 1 : 0,
                              U)));
    return hipGetLastError();
  }
  const int G = n >= (1 << 17) ? 1 : n >= (1 << 15) ? 4 : 16;
#define VP_FINISH(GV)                                                                                      \
  VP_DISPATCH_P(pl->p, (k_finish<P, GV><<<blocks_for(n * GV), kBlock, 0, st>>>(                            \
                            partial, n_split, NT, R, r0, pl->row_ptr, pl->pair_tri, pl->rows, C, far_only ? 1 : 0, \
                            U)))
  switch (G) {
    case 16: VP_FINISH(16); break;
    case 4: VP_FINISH(4); break;
    default: VP_FINISH(1); break;
  }
#undef VP_FINISH
  return hipGetLastError();
}

}  // namespace vp
