// Correction apply on the matrix cores (the add step of the Sec. 3.6
// subtract-and-add for blocks of 16, 32 or 64 right-hand sides).
//
// The correction of target t is sum over its self/near triangles D of
// row_(t,D) . c(D), c(D) = [n_p][R] coefficients.  Per target that is a
// vector-matrix product, too thin for the matrix cores.  Targets are
// therefore taken 16 at a time (a cluster: 16 consecutive targets, in the
// staggered-mesh ordering the nodes of one or two neighbouring triangles,
// whose near lists nearly coincide).  For every triangle D in the union of
// the cluster's lists, the 16 rows (zero for a target that does not list D)
// form a 16 x n_p block A_D and the cluster's correction is
// sum_D A_D C_D, C_D = c(D) restricted to 16 right-hand sides: a chain of
// 16x16x4 FP64 MFMA steps accumulated in registers, with no atomics and a
// fixed order (so the result does not depend on the launch).
//   k_cluster_union  per cluster, the sorted union of its targets' triangle
//                    lists and, for every entry, the 16 pair indices
//                    (-1 where absent); a count pass and a fill pass
//   k_corr_mfma      one wavefront per cluster: U = far partials + sum_D A_D C_D
#include <climits>

#include "vp_internal.h"

namespace vp {
namespace {

constexpr int kBlock = 256;
constexpr int kCl = 16;  // targets per cluster

inline unsigned blocks_for(int64_t n, int b = kBlock) {
  const int64_t nb = (n + b - 1) / b;
  return (unsigned)(nb < (1 << 20) ? (nb > 0 ? nb : 1) : (1 << 20));
}

// 16 lanes per cluster walk the 16 targets' triangle lists (ascending
// within a target) in step: each round takes the smallest current triangle
// of the group, the lanes that hold it record their pair and advance.
// Count pass (cl_ptr == nullptr): entries per cluster into cl_cnt.
__global__ void k_cluster_union(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ pair_tri,
                                int64_t n_tgt, int64_t n_cl, const int64_t* __restrict__ cl_ptr,
                                int32_t* __restrict__ cl_cnt, int32_t* __restrict__ ent_tri,
                                int32_t* __restrict__ ent_pair) {
  const int i = (int)(threadIdx.x % kCl);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kCl);
  for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kCl; c < n_cl; c += stride) {
    const int64_t t = c * kCl + i;
    int64_t p = 0, end = 0;
    if (t < n_tgt) {
      p = row_ptr[t];
      end = row_ptr[t + 1];
    }
    const int64_t base = cl_ptr ? cl_ptr[c] : 0;
    int64_t n = 0;
    while (true) {
      const int cur = p < end ? pair_tri[p] : INT_MAX;
      int m = cur;
#pragma unroll
      for (int off = kCl / 2; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, kCl));
      if (m == INT_MAX) break;
      if (cl_ptr) {
        if (i == 0) ent_tri[base + n] = m;
        ent_pair[(base + n) * kCl + i] = cur == m ? (int32_t)p : -1;
      }
      if (cur == m) ++p;
      ++n;
    }
    if (!cl_ptr && i == 0) cl_cnt[c] = (int32_t)n;
  }
}

typedef double vp_d4 __attribute__((ext_vector_type(4)));

// One wavefront per cluster and 16 NT right-hand sides from r0.  A-operand
// lane l: row (target) l & 15 of the cluster, basis index 4 s + (l >> 4)
// of step s; B-operand lane l: basis index 4 s + (l >> 4), right-hand side
// 16 n + (l & 15); the basis is padded with zeros to a multiple of 4.
// Result element v of lane l: target (l >> 4) + 4 v, right-hand side l & 15.
template <int P, int NT>
__global__ __launch_bounds__(kBlock) void k_corr_mfma(const double* __restrict__ partial, int64_t n_split,
                                                      int64_t n_tgt, int64_t R, int64_t r0,
                                                      const int64_t* __restrict__ cl_ptr,
                                                      const int32_t* __restrict__ ent_tri,
                                                      const int32_t* __restrict__ ent_pair, int64_t n_cl,
                                                      const double* __restrict__ rows, const double* __restrict__ C,
                                                      int far_only, double* __restrict__ U) {
  constexpr int NP = (P + 1) * (P + 2) / 2;
  constexpr int KS = (NP + 3) / 4;
  const int lane = (int)(threadIdx.x & 63), kq = lane >> 4, col = lane & 15;
  const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (c >= n_cl) return;  // the whole wavefront
  vp_d4 acc[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) acc[n] = vp_d4{0.0, 0.0, 0.0, 0.0};
  if (!far_only) {
    // the operands of entry e into a, b (zero padding past n_p and for
    // absent pairs, read from in-bounds addresses)
    auto load = [&](int64_t e, double (&a)[KS], double (&b)[KS][NT]) {
      const int32_t pr = ent_pair[e * kCl + col];
      const double* rowp = rows + (size_t)(pr >= 0 ? pr : 0) * NP;
      const double* cb = C + (size_t)ent_tri[e] * NP * R;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + kq;
        const int kc = k < NP ? k : NP - 1;
        const double av = rowp[kc];
        a[s] = (pr >= 0 && k < NP) ? av : 0.0;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const int64_t r = r0 + 16 * n + col;
          const double bv = cb[(size_t)kc * R + (r < R ? r : R - 1)];
          b[s][n] = (k < NP && r < R) ? bv : 0.0;
        }
      }
    };
    auto step = [&](const double (&a)[KS], const double (&b)[KS][NT]) {
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s][n], acc[n], 0, 0, 0);
    };
    // one entry at a time: the registers of a second entry in flight would
    // cost more occupancy (and latency hiding across wavefronts) than they save
    const int64_t e0 = cl_ptr[c], e1 = cl_ptr[c + 1];
    for (int64_t e = e0; e < e1; ++e) {
      double a0[KS], b0[KS][NT];
      load(e, a0, b0);
      step(a0, b0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t t = c * kCl + kq + 4 * v;
    if (t < n_tgt) {
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int64_t r = r0 + 16 * n + col;
        if (r >= R) continue;  // the padding of a last, partial block
        double u = acc[n][v];
#pragma unroll 8
        for (int64_t s = 0; s < n_split; ++s) u += partial[((size_t)s * n_tgt + t) * R + r];
        U[t * R + r] = u;
      }
    }
  }
}

}  // namespace

hipError_t build_clusters(vp_plan* pl, hipStream_t st) {
  const int64_t NT = pl->n_tgt;
  pl->n_cl = (NT + kCl - 1) / kCl;
  pl->n_entries = 0;
  // pair indices are stored as int32
  if (NT == 0 || pl->n_pairs == 0 || pl->n_pairs >= INT_MAX) {
    pl->n_cl = 0;
    return hipSuccess;
  }
  auto alloc = [&](void** p, size_t bytes) -> hipError_t { return plan_alloc(pl, p, bytes); };
  const int64_t ncl = pl->n_cl;
  int32_t* cnt = nullptr;
  void* tmp = nullptr;
  hipError_t e;
  Scratch scr(pl->ctx, st);
  if ((e = alloc((void**)&pl->cl_ptr, sizeof(int64_t) * (ncl + 1))) != hipSuccess) return e;
  if ((e = scr.alloc((void**)&cnt, sizeof(int32_t) * ncl)) != hipSuccess ||
      (e = scr.alloc(&tmp, exclusive_scan_tmp_bytes(ncl))) != hipSuccess)
    return e;
  const unsigned nb = blocks_for(ncl * kCl);
  k_cluster_union<<<nb, kBlock, 0, st>>>(pl->row_ptr, pl->pair_tri, NT, ncl, nullptr, cnt, nullptr, nullptr);
  int64_t ne = 0;
  if ((e = hipGetLastError()) == hipSuccess && (e = exclusive_scan_i32(cnt, pl->cl_ptr, ncl, tmp, st)) == hipSuccess &&
      (e = hipMemcpyAsync(&ne, pl->cl_ptr + ncl, sizeof(int64_t), hipMemcpyDeviceToHost, st)) == hipSuccess)
    e = hipStreamSynchronize(st);
  scr.release();
  if (e != hipSuccess) return e;
  pl->n_entries = ne;
  if ((e = alloc((void**)&pl->ent_tri, sizeof(int32_t) * ne)) != hipSuccess ||
      (e = alloc((void**)&pl->ent_pair, sizeof(int32_t) * ne * kCl)) != hipSuccess)
    return e;
  k_cluster_union<<<nb, kBlock, 0, st>>>(pl->row_ptr, pl->pair_tri, NT, ncl, pl->cl_ptr, nullptr, pl->ent_tri,
                                         pl->ent_pair);
  return hipGetLastError();
}

hipError_t prepare_blocks(vp_plan* pl, int64_t R, hipStream_t st) {
  hipError_t e = fmm_prepare_blocks(pl, R, st);
  if (e != hipSuccess || R < kMinBlockCols || pl->cl_tried) return e;
  // at most 68 bytes per pair (an entry per pair, its 16 pair slots and
  // triangle); over the budget: not now, a later evaluation tries again
  if (!ctx_fits(pl->ctx, 68 * (uint64_t)pl->n_pairs)) {
    pl->n_cl = 0;
    return hipSuccess;
  }
  pl->cl_tried = true;
  e = build_clusters(pl, st);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    pl->n_cl = 0;
    pl->n_entries = 0;
    return hipSuccess;
  }
  return e;
}

bool blocks_ready(const vp_plan* pl, int64_t R) {
  if (R < kMinBlockCols) return true;
  return (pl->fmm_terms <= 0 || pl->fmm_vsrc) && pl->cl_tried;
}

#define VP_DISPATCH_P(p, CALL)                    \
  switch (p) {                                    \
    case 1: { constexpr int P = 1; CALL; } break;  \
    case 2: { constexpr int P = 2; CALL; } break;  \
    case 3: { constexpr int P = 3; CALL; } break;  \
    case 4: { constexpr int P = 4; CALL; } break;  \
    case 5: { constexpr int P = 5; CALL; } break;  \
    case 6: { constexpr int P = 6; CALL; } break;  \
    case 7: { constexpr int P = 7; CALL; } break;  \
    case 8: { constexpr int P = 8; CALL; } break;  \
    case 9: { constexpr int P = 9; CALL; } break;  \
    case 10: { constexpr int P = 10; CALL; } break; \
    default: return hipErrorInvalidValue;          \
  }

hipError_t launch_corr_mfma(const vp_plan* pl, const double* partial, int64_t n_split, const double* C, int64_t R,
                            int64_t r0, int nt, bool far_only, double* U, hipStream_t st) {
  if (pl->n_cl == 0 || R - r0 <= 16 * (nt - 1)) return hipErrorInvalidValue;
  const int64_t nb = (pl->n_cl * 64 + kBlock - 1) / kBlock;
  if (nb >= (1LL << 31)) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nb);
#define VP_CORR(NTV)                                                                                           \
  VP_DISPATCH_P(pl->p, (k_corr_mfma<P, NTV><<<grid, kBlock, 0, st>>>(partial, n_split, pl->n_tgt, R, r0,       \
                                                                     pl->cl_ptr, pl->ent_tri, pl->ent_pair,   \
                                                                     pl->n_cl, pl->rows, C, far_only ? 1 : 0, \
                                                                     U)))
  switch (nt) {
    case 4: VP_CORR(4); break;
    case 2: VP_CORR(2); break;
    default: VP_CORR(1); break;
  }
#undef VP_CORR
  return hipGetLastError();
}

}  // namespace vp
