// Serving: continuous batching of evaluation requests over stream slots
// (declared in include/vp.h).  Requests wait host-side until a slot and the
// HBM budget allow them; a starting batch packs the pending requests of the
// same plan and precision along the right-hand-side axis so they share the
// far-field logarithms; batches on different slots overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <string>
#include <vector>

#include "vp_internal.h"

namespace {

vp_status serve_fail(vp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  vp::set_last_error(buf);
  return s;
}

}  // namespace

struct vp_server {
  vp_ctx* ctx = nullptr;
  int max_batch = 32;
  enum { kPending = 0, kRunning = 1, kDone = 2, kFailed = 3 };
  struct Req {
    vp_plan* plan;
    int64_t R;
    const double* F;
    double* U;
    vp_precision prec;
    int state;
    vp_status err;
    hipEvent_t ready;  // recorded on the context's stream at submit: the inputs are complete there
  };
  struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<int64_t> members;
    // workspace: F, C, Q, partial, U (double), Q32 (float)
    void* buf[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t cap[6] = {0, 0, 0, 0, 0, 0};
  };
  std::vector<Req> reqs;
  std::deque<int64_t> pending;
  std::vector<Slot> slots;
  int64_t n_done = 0, n_batches = 0, n_columns = 0, n_rejected = 0, n_budget_waits = 0;
};

namespace {

// The slot's workspace back to the context's block cache (the slot is idle).
void slot_release(vp_server* s, vp_server::Slot& sl) {
  for (int i = 0; i < 6; ++i) {
    if (sl.buf[i]) vp::ctx_release(s->ctx, sl.buf[i]);
    sl.buf[i] = nullptr;
    sl.cap[i] = 0;
  }
}

// Grow the slot's workspace for (plan, R), through the context's block
// cache.  Returns VP_ENOMEM when the device or the context's budget cannot
// hold it right now.
vp_status slot_reserve(vp_server* s, vp_server::Slot& sl, const vp_plan* pl, int64_t R, bool mixed) {
  const int64_t split = vp::far_config(pl, R, mixed).n_split;
  const size_t need[6] = {
      8 * (size_t)pl->n_tri * pl->n_p * R,  // F (packed)
      8 * (size_t)pl->n_tri * pl->n_p * R,  // C
      8 * (size_t)pl->n_src_pad * R,        // Q
      8 * (size_t)vp::far_partial_doubles(pl, split, R),  // far partials (+ FMM workspace)
      8 * (size_t)pl->n_tgt * R,            // U (packed)
      4 * (size_t)pl->n_src_pad * R,        // Q32
  };
  vp_ctx* ctx = s->ctx;
  for (int i = 0; i < 6; ++i) {
    if (need[i] <= sl.cap[i]) continue;
    if (sl.buf[i]) {
      vp::ctx_release(ctx, sl.buf[i]);
      sl.buf[i] = nullptr;
      sl.cap[i] = 0;
    }
    size_t got = 0;
    hipError_t e = vp::ctx_alloc(ctx, &sl.buf[i], std::max<size_t>(need[i], 8), &got);
    if (e != hipSuccess) {
      sl.buf[i] = nullptr;
      if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return VP_ENOMEM;
      }
      return VP_EDEVICE;
    }
    sl.cap[i] = got;
  }
  return VP_OK;
}

vp_status issue(vp_server* s, int slot_id, const std::vector<int64_t>& batch) {
  vp_server::Slot& sl = s->slots[slot_id];
  const vp_server::Req& head = s->reqs[batch[0]];
  const vp_plan* pl = head.plan;
  int64_t R = 0;
  for (int64_t id : batch) R += s->reqs[id].R;
  hipStream_t st = sl.st;
  double* F = (double*)sl.buf[0];
  double* C = (double*)sl.buf[1];
  double* Q = (double*)sl.buf[2];
  double* part = (double*)sl.buf[3];
  double* U = (double*)sl.buf[4];
  float* Q32 = (float*)sl.buf[5];
  hipError_t e = hipSuccess;
  int64_t c0 = 0;
  for (int64_t id : batch) {
    const vp_server::Req& r = s->reqs[id];
    if ((e = hipStreamWaitEvent(st, r.ready, 0)) != hipSuccess ||
        (e = vp::launch_pack_columns(r.F, pl->n_tri * pl->n_p, r.R, F, R, c0, st)) != hipSuccess)
      break;
    c0 += r.R;
  }
  const vp_far_config cfg = vp::far_config(pl, R, head.prec == VP_MIXED);
  // tables of blocks of densities (FMM rows, correction clusters): built once, on the context's stream
  if (e == hipSuccess) e = vp::prepare_blocks(const_cast<vp_plan*>(pl), R, s->ctx->stream);
  if (e == hipSuccess) e = vp::launch_coefficients(pl, F, R, C, Q, st);
  if (e == hipSuccess)
    e = vp::launch_far(pl, Q, R, cfg, part, st, nullptr, head.prec == VP_MIXED ? Q32 : nullptr);
  if (e == hipSuccess) e = vp::launch_finish(pl, part, cfg.n_split, C, R, false, U, st);
  c0 = 0;
  for (int64_t id : batch) {
    if (e != hipSuccess) break;
    const vp_server::Req& r = s->reqs[id];
    e = vp::launch_unpack_columns(U, pl->n_tgt, R, c0, r.U, r.R, st);
    c0 += r.R;
  }
  if (e == hipSuccess) e = hipEventRecord(sl.ev, st);
  if (e != hipSuccess) {
    for (int64_t id : batch) {
      s->reqs[id].state = vp_server::kFailed;
      s->reqs[id].err = VP_EDEVICE;
      s->reqs[id].plan->live_requests--;
    }
    return serve_fail(VP_EDEVICE, "vp serve: launch failed: %s", hipGetErrorString(e));
  }
  sl.busy = true;
  sl.members = batch;
  for (int64_t id : batch) s->reqs[id].state = vp_server::kRunning;
  s->n_batches++;
  s->n_columns += R;
  return VP_OK;
}

// Retire finished slots, then start pending requests on free slots.
vp_status progress(vp_server* s) {
  for (auto& sl : s->slots) {
    if (!sl.busy) continue;
    hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) continue;
    for (int64_t id : sl.members) {
      vp_server::Req& r = s->reqs[id];
      r.state = (q == hipSuccess) ? vp_server::kDone : vp_server::kFailed;
      r.err = (q == hipSuccess) ? VP_OK : VP_EDEVICE;
      r.plan->live_requests--;
      s->n_done++;
    }
    sl.members.clear();
    sl.busy = false;
  }
  // events of finished requests go back
  for (auto& r : s->reqs)
    if (r.state >= vp_server::kDone && r.ready) {
      (void)hipEventDestroy(r.ready);
      r.ready = nullptr;
    }
  while (!s->pending.empty()) {
    int free_slot = -1;
    bool any_busy = false;
    for (size_t i = 0; i < s->slots.size(); ++i) {
      if (!s->slots[i].busy && free_slot < 0) free_slot = (int)i;
      any_busy |= s->slots[i].busy;
    }
    if (free_slot < 0) break;
    // head of the queue plus every later pending request of the same plan
    // and precision, while the packed width stays within max_batch
    const int64_t head = s->pending.front();
    const vp_server::Req& h = s->reqs[head];
    std::vector<int64_t> batch{head};
    int64_t width = h.R;
    for (size_t k = 1; k < s->pending.size(); ++k) {
      const vp_server::Req& r = s->reqs[s->pending[k]];
      if (r.plan == h.plan && r.prec == h.prec && width + r.R <= s->max_batch) {
        batch.push_back(s->pending[k]);
        width += r.R;
      }
    }
    // the plan's tables for blocks of densities first (they stay with the
    // plan); when the budget keeps them out, the idle slots' workspaces make
    // room, else the batch waits for a running one (without them it would
    // run one density at a time)
    vp_plan* hp = h.plan;
    hipError_t pe = vp::prepare_blocks(hp, width, s->ctx->stream);
    if (pe == hipSuccess && !vp::blocks_ready(hp, width)) {
      for (size_t i = 0; i < s->slots.size(); ++i)
        if (!s->slots[i].busy) slot_release(s, s->slots[i]);
      pe = vp::prepare_blocks(hp, width, s->ctx->stream);
      if (pe == hipSuccess && !vp::blocks_ready(hp, width) && any_busy) {
        s->n_budget_waits++;
        break;
      }
    }
    if (pe != hipSuccess) return serve_fail(VP_EDEVICE, "vp serve: tables: %s", hipGetErrorString(pe));
    vp_status st = slot_reserve(s, s->slots[free_slot], h.plan, width, h.prec == VP_MIXED);
    if (st == VP_ENOMEM) {
      // the other idle slots' workspaces make room (they grow again when
      // used), then the context's cache (ctx_alloc empties it under a budget)
      for (size_t i = 0; i < s->slots.size(); ++i)
        if (!s->slots[i].busy && (int)i != free_slot) slot_release(s, s->slots[i]);
      st = slot_reserve(s, s->slots[free_slot], h.plan, width, h.prec == VP_MIXED);
    }
    if (st == VP_ENOMEM) {
      if (any_busy) {  // memory frees up when a running batch retires
        s->n_budget_waits++;
        break;
      }
      // even alone on an idle device the request does not fit: fail it
      s->reqs[head].state = vp_server::kFailed;
      s->reqs[head].err = VP_ENOMEM;
      s->reqs[head].plan->live_requests--;
      s->pending.pop_front();
      s->n_rejected++;
      continue;
    }
    if (st != VP_OK) return serve_fail(st, "vp serve: workspace allocation failed");
    for (int64_t id : batch) s->pending.erase(std::find(s->pending.begin(), s->pending.end(), id));
    st = issue(s, free_slot, batch);
    if (st != VP_OK) return st;
  }
  return VP_OK;
}

}  // namespace

extern "C" {

vp_status vp_server_create(vp_ctx* ctx, int n_slots, int max_batch_rhs, vp_server** out) {
  if (!ctx || !out) return serve_fail(VP_EINVAL, "vp_server_create: NULL argument");
  if (n_slots < 1 || n_slots > 16 || max_batch_rhs < 1 || max_batch_rhs > 4096)
    return serve_fail(VP_EINVAL, "vp_server_create: n_slots in [1, 16], max_batch_rhs in [1, 4096]");
  if (hipSetDevice(ctx->device) != hipSuccess) return serve_fail(VP_EDEVICE, "hipSetDevice failed");
  vp_server* s = new vp_server;
  s->ctx = ctx;
  ctx->live_servers++;
  s->max_batch = max_batch_rhs;
  s->slots.resize(n_slots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      vp_server_destroy(s);
      return serve_fail(VP_EDEVICE, "vp_server_create: stream or event creation failed");
    }
  }
  *out = s;
  return VP_OK;
}

vp_status vp_server_destroy(vp_server* s) {
  if (!s) return VP_OK;
  (void)hipSetDevice(s->ctx->device);
  while (!s->pending.empty() || std::any_of(s->slots.begin(), s->slots.end(), [](auto& x) { return x.busy; })) {
    for (auto& sl : s->slots)
      if (sl.busy) (void)hipEventSynchronize(sl.ev);
    if (progress(s) != VP_OK) break;
  }
  for (auto& sl : s->slots) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    slot_release(s, sl);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
  }
  for (auto& r : s->reqs)
    if (r.ready) (void)hipEventDestroy(r.ready);
  s->ctx->live_servers--;
  delete s;
  return VP_OK;
}

vp_status vp_submit(vp_server* s, vp_plan* pl, int64_t R, const double* F, double* U, vp_precision prec,
                    vp_ticket* ticket) {
  if (!s || !pl || !ticket) return serve_fail(VP_EINVAL, "vp_submit: NULL argument");
  if (pl->ctx != s->ctx) return serve_fail(VP_EINVAL, "vp_submit: plan belongs to another context");
  if (R < 1) return serve_fail(VP_EINVAL, "vp_submit: n_rhs must be >= 1");
  if ((!F && pl->n_tri) || (!U && pl->n_tgt)) return serve_fail(VP_EINVAL, "vp_submit: NULL array");
  if (prec != VP_FP64 && prec != VP_MIXED) return serve_fail(VP_EINVAL, "vp_submit: unknown precision");
  if (hipSetDevice(s->ctx->device) != hipSuccess) return serve_fail(VP_EDEVICE, "hipSetDevice failed");
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ready, s->ctx->stream) != hipSuccess) {
    if (ready) (void)hipEventDestroy(ready);
    return serve_fail(VP_EDEVICE, "vp_submit: event on the context's stream failed");
  }
  *ticket = (vp_ticket)s->reqs.size();
  s->reqs.push_back({pl, R, F, U, prec, vp_server::kPending, VP_OK, ready});
  pl->live_requests++;
  s->pending.push_back(*ticket);
  return progress(s);
}

vp_status vp_poll(vp_server* s, vp_ticket t, int* done) {
  if (!s || !done || t < 0 || t >= (vp_ticket)s->reqs.size()) return serve_fail(VP_EINVAL, "vp_poll: bad ticket");
  if (hipSetDevice(s->ctx->device) != hipSuccess) return serve_fail(VP_EDEVICE, "hipSetDevice failed");
  vp_status st = progress(s);
  if (st != VP_OK) return st;
  const auto& r = s->reqs[t];
  *done = r.state >= vp_server::kDone;
  if (r.state == vp_server::kFailed) return serve_fail(r.err, "vp_poll: request %lld failed", (long long)t);
  return VP_OK;
}

vp_status vp_wait(vp_server* s, vp_ticket t) {
  if (!s || t < 0 || t >= (vp_ticket)s->reqs.size()) return serve_fail(VP_EINVAL, "vp_wait: bad ticket");
  if (hipSetDevice(s->ctx->device) != hipSuccess) return serve_fail(VP_EDEVICE, "hipSetDevice failed");
  for (;;) {
    vp_status st = progress(s);
    if (st != VP_OK) return st;
    const auto& r = s->reqs[t];
    if (r.state == vp_server::kDone) return VP_OK;
    if (r.state == vp_server::kFailed) return serve_fail(r.err, "vp_wait: request %lld failed", (long long)t);
    // block on the slot running it, else on any running slot
    int target = -1;
    for (size_t i = 0; i < s->slots.size(); ++i) {
      const auto& sl = s->slots[i];
      if (!sl.busy) continue;
      if (target < 0) target = (int)i;
      if (std::find(sl.members.begin(), sl.members.end(), t) != sl.members.end()) {
        target = (int)i;
        break;
      }
    }
    if (target < 0) return serve_fail(VP_EINTERNAL, "vp_wait: request %lld cannot start", (long long)t);
    (void)hipEventSynchronize(s->slots[target].ev);
  }
}

vp_status vp_server_admission(const vp_server* s, int64_t* budget_waits, int64_t* rejected) {
  if (!s) return serve_fail(VP_EINVAL, "vp_server_admission: NULL server");
  if (budget_waits) *budget_waits = s->n_budget_waits;
  if (rejected) *rejected = s->n_rejected;
  return VP_OK;
}

vp_status vp_server_stats(const vp_server* s, int64_t* done, int64_t* batches, int64_t* columns) {
  if (!s) return serve_fail(VP_EINVAL, "vp_server_stats: NULL server");
  if (done) *done = s->n_done;
  if (batches) *batches = s->n_batches;
  if (columns) *columns = s->n_columns;
  return VP_OK;
}

}  // extern "C"
