// The evaluation without device allocation (vp_execute_noalloc, declared in
// include/vp.h): the same launches as vp_execute, with the workspace
// (coefficients, far charges, their FP32 copy, far partial sums) carved
// from one fixed device array of this file instead of the plan's
// workspace, so that a call makes no hipMalloc, hipFree or other
// allocating call.  The array is process-wide: every device the library
// runs on holds its own copy, every call on a device shares it, and each
// call overwrites what the previous one left.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "vp_internal.h"

namespace {

// the workspace array (one copy per device)
__device__ __align__(256) unsigned char scratch[VP_NOALLOC_SCRATCH_BYTES];

// its device address on each device, taken once per device with that device
// current (the host-side name `scratch` is not a device address)
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

void* device_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

vp_status nofail(vp_status s, const char* fmt, long long a = 0, long long b = 0) {
  char buf[512];
  snprintf(buf, sizeof buf, fmt, a, b);
  vp::set_last_error(buf);
  return s;
}

}  // namespace

namespace vp {

// Called by vp_ctx_create with `device` current: records the array's
// address on that device the first time the device is seen.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = ptr;
  return hipSuccess;
}

}  // namespace vp

extern "C" {

vp_status vp_execute_noalloc(vp_plan* pl, int64_t R, const double* density, double* u_out, vp_precision prec,
                             uint32_t flags) {
  if (!pl) return nofail(VP_EINVAL, "vp_execute_noalloc: plan is NULL");
  if (R < 1) return nofail(VP_EINVAL, "vp_execute_noalloc: n_rhs must be >= 1");
  if (prec != VP_FP64 && prec != VP_MIXED) return nofail(VP_EINVAL, "vp_execute_noalloc: unknown precision");
  if (!(flags & VP_DEVICE_PTRS) || (flags & ~(uint32_t)(VP_DEVICE_PTRS | VP_FAR_ONLY | VP_ASYNC)))
    return nofail(VP_EINVAL, "vp_execute_noalloc: flags must be VP_DEVICE_PTRS [| VP_FAR_ONLY | VP_ASYNC]");
  if ((!density && pl->n_tri) || (!u_out && pl->n_tgt)) return nofail(VP_EINVAL, "vp_execute_noalloc: NULL array");
  if (pl->fmm_terms > 0 && R >= vp::kMinBlockCols && !pl->fmm_vsrc)
    return nofail(VP_EINVAL,
                  "vp_execute_noalloc: the FMM tables for blocks of densities are built by a first vp_execute "
                  "with n_rhs >= 2 on this plan");
  const bool mixed = prec == VP_MIXED;
  const vp_far_config cfg = vp::far_config(pl, R, mixed);
  const size_t nC = (size_t)pl->n_tri * pl->n_p * R;
  const size_t nQ = (size_t)pl->n_src_pad * R;
  const size_t nP = (size_t)vp::far_partial_doubles(pl, cfg.n_split, R);
  const size_t oQ = align256(8 * nC), oQ32 = oQ + align256(8 * nQ);
  const size_t oP = oQ32 + (mixed ? align256(4 * nQ) : 0);
  const size_t need = oP + 8 * nP;
  if (need > (size_t)VP_NOALLOC_SCRATCH_BYTES)
    return nofail(VP_EINVAL, "vp_execute_noalloc: workspace of %lld bytes exceeds the %lld-byte device scratch",
                  (long long)need, (long long)VP_NOALLOC_SCRATCH_BYTES);
  if (hipSetDevice(pl->ctx->device) != hipSuccess) return nofail(VP_EDEVICE, "vp_execute_noalloc: hipSetDevice");
  unsigned char* base = (unsigned char*)device_scratch(pl->ctx->device);
  if (!base) return nofail(VP_EINTERNAL, "vp_execute_noalloc: no scratch address for device %lld",
                           (long long)pl->ctx->device);
  double* C = (double*)base;
  double* Q = (double*)(base + oQ);
  float* Q32 = mixed ? (float*)(base + oQ32) : nullptr;
  double* part = (double*)(base + oP);
  hipStream_t st = pl->ctx->stream;
  hipError_t e;
  int64_t nl = 0;
  if ((e = vp::launch_coefficients(pl, density, R, C, Q, st)) != hipSuccess ||
      (e = vp::launch_far(pl, Q, R, cfg, part, st, &nl, Q32)) != hipSuccess ||
      (e = vp::launch_finish(pl, part, cfg.n_split, C, R, (flags & VP_FAR_ONLY) != 0, u_out, st)) != hipSuccess)
    return nofail(VP_EDEVICE, "vp_execute_noalloc: launch failed (%lld)", (long long)e);
  if (!(flags & VP_ASYNC) && (e = hipStreamSynchronize(st)) != hipSuccess)
    return nofail(VP_EDEVICE, "vp_execute_noalloc: synchronize (%lld)", (long long)e);
  return VP_OK;
}

}  // extern "C"
