// Per-solve kernels (FP64):
//   k_coef      c = V^{-1} F per triangle (Sec. 2.2 interpolation matrix)
//   k_charges   far charges Q_j = w_j |J(xi_j)| f_h(y_j) / (4 pi) (Sec. 3.6: every
//               far-rule node is a point charge; the 1/2 of log r = log(r^2)/2
//               is folded in)
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
#ifndef VP_FAR_TPT
#define VP_FAR_TPT 2
#endif
constexpr int kFarTPT = VP_FAR_TPT;  // targets per thread in the far sum

// Grid of a grid-stride launch: at most 2^20 blocks, so that a launch stays
// far below 2^32 work-items.
inline unsigned blocks_for(int64_t n, int b = kBlock) {
  const int64_t nb = (n + b - 1) / b;
  return (unsigned)(nb < (1 << 20) ? (nb > 0 ? nb : 1) : (1 << 20));
}

// one thread per (triangle, rhs); F and C are [T][NP][R]
template <int P>
__global__ void k_coef(const double* __restrict__ F, const double* __restrict__ vinv, int64_t n_tri, int64_t R,
                       double* __restrict__ C) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
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
  }
}

// one thread per (source, rhs); Q is [n_src][R]
template <int P>
__global__ void k_charges(const double* __restrict__ C, const double* __restrict__ efar,
                          const double* __restrict__ swj, int nf, int64_t n_tri, int64_t R, double* __restrict__ Q) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t n_src = n_tri * nf;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_src * R; g += stride) {
    const int64_t src = g / R, r = g - src * R;
    const int64_t t = src / nf;
    const int j = (int)(src - t * nf);
    const double* c = C + (size_t)t * NP * R + r;
    const double* E = efar + (size_t)j * NP;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) s = fma(E[k], c[(size_t)k * R], s);
    Q[g] = s * swj[src] * kInv4Pi;
  }
}

// Direct far sum.  Each thread owns TPT targets (strided by the block
// size); the sources are read with wavefront-uniform addresses (scalar
// loads), RB right-hand sides share one logarithm per pair.  A linear block
// id b takes source chunk b % n_split and target block b / n_split, so with
// n_split a multiple of 8 the blocks that share a chunk sit on one XCD and
// its L2.  Each 256-source tile is summed on its own before it joins the
// running total (two-level summation).  Sources are padded to a multiple of
// 256 with zero charges.  With one right-hand side the logarithm comes from
// the 4096-entry table (vp_log_wide_parts) in 1024-thread blocks, and its
// exponent part is accumulated apart (sum Q e, times ln 2 at the end); with
// several, the logarithm is a small share of the work per pair and the
// 256-entry table leaves room for more blocks per CU.
template <int RB>
struct FarShape {
  static constexpr int kThreads = RB == 1 ? 1024 : 256;
  static constexpr int kTab = RB == 1 ? kFarLogTab : kLogTab;
};

template <int RB, int TPT>
__global__ __launch_bounds__(FarShape<RB>::kThreads) void k_far(
    const double2* __restrict__ sxy, const double* __restrict__ Q, int64_t n_src_pad, int64_t R, int64_t r0,
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
    int64_t n_split, const double2* __restrict__ logtab, double* __restrict__ partial) {
  constexpr int kB = FarShape<RB>::kThreads, kTab = FarShape<RB>::kTab;
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
            vp_log_wide_parts(r2, tab, e, rest);
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

// Mixed-precision far sum (same decomposition as k_far): the pair
// difference is taken in FP64 and rounded to FP32, r^2 + 2^-100 and the
// base-2 logarithm (the hardware v_log_f32) are FP32, the charges are FP32
// with ln 2 folded in (Q32 = Q ln 2, so Q32 log2(r^2) = Q log(r^2)), each
// 256-source tile is summed in FP32 and the tiles are summed in FP64.
template <int RB, int TPT>
__global__ __launch_bounds__(kBlock) void k_far32(const double2* __restrict__ sxy, const float* __restrict__ Q32,
                                                  int64_t n_src_pad, int64_t R, int64_t r0,
                                                  const double* __restrict__ xt, const double* __restrict__ yt,
                                                  int64_t n_tgt, int64_t per_split, int64_t n_split,
                                                  double* __restrict__ partial) {
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  double x[TPT], y[TPT];
  int64_t t[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    t[k] = tb * (kBlock * TPT) + k * kBlock + threadIdx.x;
    const bool act = t[k] < n_tgt;
    x[k] = act ? xt[t[k]] : 0.0;
    y[k] = act ? yt[t[k]] : 0.0;
  }
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
    for (int64_t j = j0; j < j1; j += 4) {
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
// targets (MT tiles of 16) and walks its source chunk 4 sources at a time;
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
constexpr int kMfmaMT = 4;                               // 16-target tiles per wavefront
constexpr int kMfmaTargets = (kBlock / 64) * 16 * kMfmaMT;  // targets per block

template <int NT>
__global__ __launch_bounds__(kBlock, 2) void k_far_mfma64(
    const double2* __restrict__ sxy, const double* __restrict__ Q, int64_t n_src_pad, int64_t R, int64_t r0,
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
    int64_t n_split, const double2* __restrict__ logtab, double* __restrict__ partial) {
  constexpr int MT = kMfmaMT;
  __shared__ double2 tab[kFarLogTab + 1];
  for (int i = threadIdx.x; i <= kFarLogTab; i += kBlock) tab[i] = logtab[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, kk = lane >> 4, nn = lane & 15;
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  const int64_t t0 = tb * kMfmaTargets + (threadIdx.x >> 6) * (16 * MT);
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

template <int NT>
__global__ __launch_bounds__(kBlock, 2) void k_far_mfma32(
    const double2* __restrict__ sxy, const float* __restrict__ Q32, int64_t n_src_pad, int64_t R, int64_t r0,
    const double* __restrict__ xt, const double* __restrict__ yt, int64_t n_tgt, int64_t per_split,
    int64_t n_split, double* __restrict__ partial) {
  constexpr int MT = kMfmaMT;
  const int lane = threadIdx.x & 63, kk = lane >> 4, nn = lane & 15;
  const int64_t b = blockIdx.x;
  const int64_t chunk = b % n_split, tb = b / n_split;
  const int64_t t0 = tb * kMfmaTargets + (threadIdx.x >> 6) * (16 * MT);
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
    vp_f4 tile[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n) tile[m][n] = vp_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 2
    for (int64_t j = j0 + kk; j < j0 + 256; j += 4) {
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

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
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

// one thread per (target, rhs)
template <int P>
__global__ void k_finish(const double* __restrict__ partial, int64_t n_split, int64_t n_tgt, int64_t R,
                         const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pair_tri,
                         const double* __restrict__ rows, const double* __restrict__ C, int far_only,
                         double* __restrict__ U) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_tgt * R; g += stride) {
    const int64_t t = g / R, r = g - t * R;
    double u = 0.0;
    for (int64_t s = 0; s < n_split; ++s) u += partial[((size_t)s * n_tgt + t) * R + r];
    if (!far_only) {
      double corr = 0.0;
      for (int64_t p = row_ptr[t]; p < row_ptr[t + 1]; ++p) {
        const double* row = rows + (size_t)p * NP;
        const double* c = C + (size_t)pair_tri[p] * NP * R + r;
#pragma unroll
        for (int k = 0; k < NP; ++k) corr = fma(row[k], c[(size_t)k * R], corr);
      }
      u += corr;
    }
    U[g] = u;
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
  // the padding sources past n_src carry zero charge for this R (a fill
  // kernel, not a memset, so that the sequence can be captured in a graph)
  if (Q && pl->n_src_pad > pl->n_src) {
    const int64_t nz = (pl->n_src_pad - pl->n_src) * R;
    k_fill<<<blocks_for(nz), kBlock, 0, st>>>(Q + pl->n_src * R, nz, 0.0);
  }
  if (T == 0) return hipSuccess;
  VP_DISPATCH_P(pl->p, (k_coef<P><<<blocks_for(T * R), kBlock, 0, st>>>(F, pl->vinv, T, R, C)));
  if (Q) {
    VP_DISPATCH_P(pl->p, (k_charges<P><<<blocks_for(T * pl->n_f * R), kBlock, 0, st>>>(
                              C, pl->efar, pl->swj, pl->n_f, T, R, Q)));
  }
  return hipGetLastError();
}

int64_t far_targets_per_block() { return FarShape<1>::kThreads * kFarTPT; }

hipError_t launch_far(const vp_plan* pl, const double* Q, int64_t R, int64_t n_split, double* partial,
                      hipStream_t st, int64_t* n_launches, float* Q32) {
  const int64_t NT = pl->n_tgt, NS = pl->n_src_pad;
  if (NT == 0) return hipSuccess;
  int64_t per = (NS + n_split - 1) / n_split;
  per = ((per + 255) / 256) * 256;
  if (Q32) k_to_f32_ln2<<<blocks_for(NS * R), kBlock, 0, st>>>(Q, NS * R, Q32);
  int64_t r0 = 0;
  // blocks of 16, 32 or 64 right-hand sides on the matrix cores
  while (R - r0 >= 16) {
    const int64_t left = R - r0;
    const int nt = left >= 64 ? 4 : left >= 32 ? 2 : 1;
    const int64_t nb = (NT + kMfmaTargets - 1) / kMfmaTargets * n_split;
    if (nb * kBlock >= (1LL << 32)) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nb);
#define VP_FAR_MFMA(NTV)                                                                                     \
  if (Q32)                                                                                                   \
    k_far_mfma32<NTV><<<grid, kBlock, 0, st>>>(pl->sxy, Q32, NS, R, r0, pl->xt, pl->yt, NT, per, n_split,  \
                                               partial);                                                     \
  else                                                                                                       \
    k_far_mfma64<NTV><<<grid, kBlock, 0, st>>>(pl->sxy, Q, NS, R, r0, pl->xt, pl->yt, NT, per, n_split,    \
                                               pl->logtab_wide, partial)
    switch (nt) {
      case 4: VP_FAR_MFMA(4); break;
      case 2: VP_FAR_MFMA(2); break;
      default: VP_FAR_MFMA(1); break;
    }
#undef VP_FAR_MFMA
    if (n_launches) ++*n_launches;
    r0 += 16 * nt;
  }
  // the remaining right-hand sides on the vector ALUs
  while (r0 < R) {
    const int64_t left = R - r0;
    const int rb = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    const int tpt = kFarTPT;  // RB right-hand sides share each logarithm
    const int threads = (Q32 || rb > 1) ? kBlock : FarShape<1>::kThreads;
    const int64_t n_tb = (NT + threads * tpt - 1) / (threads * tpt);
    const int64_t nb = n_tb * n_split;
    if (nb * threads >= (1LL << 32)) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nb);
#define VP_FAR(RBV, TPTV)                                                                                      \
  if (Q32)                                                                                                     \
    k_far32<RBV, TPTV><<<grid, kBlock, 0, st>>>(pl->sxy, Q32, NS, R, r0, pl->xt, pl->yt, NT, per, n_split,   \
                                                partial);                                                      \
  else                                                                                                         \
    k_far<RBV, TPTV><<<grid, FarShape<RBV>::kThreads, 0, st>>>(pl->sxy, Q, NS, R, r0, pl->xt, pl->yt, NT, per, \
                                                               n_split, RBV == 1 ? pl->logtab_wide : pl->logtab, \
                                                               partial)
    switch (rb) {
      case 8: VP_FAR(8, kFarTPT); break;
      case 4: VP_FAR(4, kFarTPT); break;
      case 2: VP_FAR(2, kFarTPT); break;
      default: VP_FAR(1, kFarTPT); break;
    }
#undef VP_FAR
    if (n_launches) ++*n_launches;
    r0 += rb;
  }
  return hipGetLastError();
}

hipError_t launch_finish(const vp_plan* pl, const double* partial, int64_t n_split, const double* C, int64_t R,
                         bool far_only, double* U, hipStream_t st) {
  const int64_t NT = pl->n_tgt;
  if (NT == 0) return hipSuccess;
  VP_DISPATCH_P(pl->p, (k_finish<P><<<blocks_for(NT * R), kBlock, 0, st>>>(
                            partial, n_split, NT, R, pl->row_ptr, pl->pair_tri, pl->rows, C, far_only ? 1 : 0, U)));
  return hipGetLastError();
}

}  // namespace vp
