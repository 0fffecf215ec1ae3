// Per-solve kernels (FP64):
//   k_coef      c = V^{-1} F per triangle (Sec. 2.2 interpolation matrix)
//   k_charges   far charges Q_j = w_j |J| f_h(y_j) / (4 pi) (Sec. 3.6: every
//               far-rule node is a point charge; the 1/2 of log r = log(r^2)/2
//               is folded in)
//   k_far       U_far(x) = sum_j Q_j log|x - y_j|^2 over all sources: a
//               direct sum, targets across threads, sources staged through
//               LDS in tiles (a pair at distance 0 contributes 0)
//   k_finish    u = sum of the far partials + sum over the target's self/near
//               pairs of row . c(triangle)  (Sec. 3.6 subtract-and-add)
#include <cmath>

#include "vp_internal.h"

namespace vp {
namespace {

constexpr int kBlock = 256;
constexpr double kInv4Pi = 0.07957747154594766788;

inline unsigned blocks_for(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// one thread per (triangle, rhs); F and C are [T][NP][R]
template <int P>
__global__ void k_coef(const double* __restrict__ F, const double* __restrict__ vinv, int64_t n_tri, int64_t R,
                       double* __restrict__ C) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_tri * R) return;
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

// one thread per (source, rhs); Q is [n_src][R]
template <int P>
__global__ void k_charges(const double* __restrict__ C, const double* __restrict__ efar,
                          const double* __restrict__ far_w, const double* __restrict__ det, int nf,
                          int64_t n_tri, int64_t R, double* __restrict__ Q) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n_src = n_tri * nf;
  if (g >= n_src * R) return;
  const int64_t src = g / R, r = g - src * R;
  const int64_t t = src / nf;
  const int j = (int)(src - t * nf);
  const double* c = C + (size_t)t * NP * R + r;
  const double* E = efar + (size_t)j * NP;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) s = fma(E[k], c[(size_t)k * R], s);
  Q[g] = s * far_w[j] * det[t] * kInv4Pi;
}

// Direct far sum.  Block = 256 threads = 256 targets; grid.y splits the
// sources.  RB right-hand sides share one logarithm per pair.  Each LDS
// tile's 256 terms are summed on their own before joining the running total
// (two-level summation).
template <int RB>
__global__ __launch_bounds__(kBlock) void k_far(const double* __restrict__ xs, const double* __restrict__ ys,
                                                const double* __restrict__ Q, int64_t n_src, int64_t R, int64_t r0,
                                                const double* __restrict__ xt, const double* __restrict__ yt,
                                                int64_t n_tgt, int64_t per_split, double* __restrict__ partial) {
  __shared__ double sx[kBlock], sy[kBlock], sq[kBlock * RB];
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = t < n_tgt;
  const double x = active ? xt[t] : 0.0, y = active ? yt[t] : 0.0;
  const int64_t s_begin = (int64_t)blockIdx.y * per_split;
  const int64_t s_end = min(n_src, s_begin + per_split);
  double acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = 0.0;
  for (int64_t base = s_begin; base < s_end; base += kBlock) {
    const int64_t j = base + threadIdx.x;
    if (j < s_end) {
      sx[threadIdx.x] = xs[j];
      sy[threadIdx.x] = ys[j];
#pragma unroll
      for (int r = 0; r < RB; ++r) sq[threadIdx.x * RB + r] = (r0 + r < R) ? Q[j * R + r0 + r] : 0.0;
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kBlock, s_end - base);
    double tile[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) tile[r] = 0.0;
    for (int i = 0; i < cnt; ++i) {
      const double dx = x - sx[i], dy = y - sy[i];
      const double r2 = fma(dx, dx, dy * dy);
      const double lg = (r2 > 0.0) ? log(r2) : 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) tile[r] = fma(sq[i * RB + r], lg, tile[r]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] += tile[r];
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r0 + r < R) partial[((size_t)blockIdx.y * n_tgt + t) * R + r0 + r] = acc[r];
  }
}

// one thread per (target, rhs)
template <int P>
__global__ void k_finish(const double* __restrict__ partial, int64_t n_split, int64_t n_tgt, int64_t R,
                         const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pair_tri,
                         const double* __restrict__ rows, const double* __restrict__ C, int far_only,
                         double* __restrict__ U) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_tgt * R) return;
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

hipError_t launch_coefficients(const vp_plan* pl, const double* F, int64_t R, double* C, double* Q, hipStream_t st) {
  const int64_t T = pl->n_tri;
  if (T == 0) return hipSuccess;
  VP_DISPATCH_P(pl->p, (k_coef<P><<<blocks_for(T * R), kBlock, 0, st>>>(F, pl->vinv, T, R, C)));
  if (Q) {
    VP_DISPATCH_P(pl->p, (k_charges<P><<<blocks_for(T * pl->n_f * R), kBlock, 0, st>>>(
                              C, pl->efar, pl->far_w, pl->mesh->det, pl->n_f, T, R, Q)));
  }
  return hipGetLastError();
}

hipError_t launch_far(const vp_plan* pl, const double* Q, int64_t R, int64_t n_split, double* partial,
                      hipStream_t st) {
  const int64_t NT = pl->n_tgt, NS = pl->n_src;
  if (NT == 0) return hipSuccess;
  int64_t per = (NS + n_split - 1) / n_split;
  per = ((per + kBlock - 1) / kBlock) * kBlock;
  dim3 grid(blocks_for(NT), (unsigned)n_split);
  int64_t r0 = 0;
  while (r0 < R) {
    const int64_t left = R - r0;
    const int rb = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    switch (rb) {
      case 8: k_far<8><<<grid, kBlock, 0, st>>>(pl->xs, pl->ys, Q, NS, R, r0, pl->xt, pl->yt, NT, per, partial); break;
      case 4: k_far<4><<<grid, kBlock, 0, st>>>(pl->xs, pl->ys, Q, NS, R, r0, pl->xt, pl->yt, NT, per, partial); break;
      case 2: k_far<2><<<grid, kBlock, 0, st>>>(pl->xs, pl->ys, Q, NS, R, r0, pl->xt, pl->yt, NT, per, partial); break;
      default: k_far<1><<<grid, kBlock, 0, st>>>(pl->xs, pl->ys, Q, NS, R, r0, pl->xt, pl->yt, NT, per, partial); break;
    }
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
