// Serving form: continuous batching of endgame solves on one device.
//
// A batch holds up to max_slots solves, each with its own device-resident
// state (iterates, products, q_bar, node values) and its own HIP stream, and
// admits a new solve only while the bytes of all live states fit the budget.
// egt_batch_tick advances every live solve by one phase -- a saddle-gap
// evaluation when the solve is due for one, else one attempt of an EGT step --
// by first enqueueing the phase of every solve on its stream and only then
// waiting for each, so the kernels of different solves overlap on the device.
// A solve that reaches its gap target (or its iteration cap) finishes and
// keeps its result until it is retired, which frees its memory for new
// admissions.  Each solve's arithmetic is the same kernels in the same order
// as a lone egt_solve, so its result does not depend on the mix.
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "egt_internal.h"

namespace egt {
int state_create(const egt_game* g, const egt_solve_opts* o, hipStream_t s, egt_state** out);
int state_destroy(egt_state* st);
int gap_launch(egt_state* st, hipStream_t s);
int gap_finish(egt_state* st, hipStream_t s);
int step_launch(egt_state* st, int player, hipStream_t s);
int step_finish(egt_state* st, hipStream_t s, int* accepted, double* egv_out, int* stepped);
int fill_result(egt_state* st, bool converged, double seconds, egt_result* res, hipStream_t s);
int64_t state_bytes(const egt_game* g, bool mixed);
const egt_solve_opts& state_opts(const egt_state* st);
int64_t state_iters(const egt_state* st);
bool state_gap_known(const egt_state* st);
double state_gap_value(const egt_state* st);
}  // namespace egt

namespace {

enum Phase { kFree = 0, kNeedGap, kNeedStep, kDone };

struct Slot {
  Phase phase = kFree;
  bool pending = false;  // a launched phase awaits its finish
  egt_state* st = nullptr;
  hipStream_t stream = nullptr;
  int64_t bytes = 0;
  int status = EGT_OK;
  egt_result res{};
  std::chrono::steady_clock::time_point t0;
};

}  // namespace

struct egt_batch {
  int64_t budget = 0;
  int64_t used = 0;
  std::vector<Slot> slots;
};

using namespace egt;

namespace {

void finish_slot(Slot& sl, bool converged) {
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
  const int rc = fill_result(sl.st, converged, secs, &sl.res, sl.stream);
  sl.status = rc ? rc : (converged ? EGT_OK : EGT_ENOTCONV);
  sl.phase = kDone;
}

void fail_slot(Slot& sl, int rc) {
  std::memset(&sl.res, 0, sizeof(sl.res));
  sl.res.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
  sl.status = rc;
  sl.phase = kDone;
}

// After an accepted step or at admission: due for a gap test, or step on.
Phase next_phase(const egt_state* st) {
  const egt_solve_opts& op = state_opts(st);
  const int64_t t = state_iters(st);
  return (t % op.gap_every == 0 || t >= op.max_iters) ? kNeedGap : kNeedStep;
}

}  // namespace

extern "C" {

int egt_state_bytes(const egt_game* g, const egt_solve_opts* opts, int64_t* bytes) {
  if (!g || !bytes) return fail(EGT_EINVAL, "null argument");
  const bool mixed = opts && opts->precision == EGT_PRECISION_MIXED;
  *bytes = state_bytes(g, mixed);
  return EGT_OK;
}

int egt_batch_create(int64_t budget_bytes, int32_t max_slots, egt_batch** out) {
  if (!out || budget_bytes <= 0 || max_slots < 1 || max_slots > 4096)
    return fail(EGT_EINVAL, "budget must be > 0 and max_slots in 1..4096");
  egt_batch* b = new (std::nothrow) egt_batch();
  if (!b) return fail(EGT_ENOMEM, "host allocation failed");
  b->budget = budget_bytes;
  b->slots.resize((size_t)max_slots);
  *out = b;
  return EGT_OK;
}

int egt_batch_retire(egt_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size()) return fail(EGT_EINVAL, "bad batch or slot");
  Slot& sl = b->slots[(size_t)slot];
  if (sl.phase == kFree) return fail(EGT_EINVAL, "slot is free");
  int rc = EGT_OK;
  if (sl.st) rc = state_destroy(sl.st);
  if (sl.stream) {
    const hipError_t e = hipStreamDestroy(sl.stream);
    if (e != hipSuccess && rc == EGT_OK) rc = hip_fail(e, "hipStreamDestroy");
  }
  b->used -= sl.bytes;
  sl = Slot();
  return rc;
}

int egt_batch_destroy(egt_batch* b) {
  if (!b) return EGT_OK;
  int rc = EGT_OK;
  for (size_t i = 0; i < b->slots.size(); ++i)
    if (b->slots[i].phase != kFree) {
      const int r = egt_batch_retire(b, (int32_t)i);
      if (r && rc == EGT_OK) rc = r;
    }
  delete b;
  return rc;
}

int egt_batch_admit(egt_batch* b, const egt_game* g, const egt_solve_opts* opts, int32_t* slot) {
  if (!b || !g || !slot) return fail(EGT_EINVAL, "null argument");
  *slot = -1;
  const bool mixed = opts && opts->precision == EGT_PRECISION_MIXED;
  const int64_t need = state_bytes(g, mixed);
  if (b->used + need > b->budget) return fail(EGT_EBUDGET, "the solve does not fit the memory budget now");
  size_t k = 0;
  while (k < b->slots.size() && b->slots[k].phase != kFree) ++k;
  if (k == b->slots.size()) return fail(EGT_EBUDGET, "no free slot");
  Slot& sl = b->slots[k];
  sl = Slot();
  sl.t0 = std::chrono::steady_clock::now();
  EGT_HIP(hipStreamCreate(&sl.stream));  // default priority
  const int rc = state_create(g, opts, sl.stream, &sl.st);
  if (rc) {
    (void)hipStreamDestroy(sl.stream);
    sl = Slot();
    return rc;
  }
  sl.bytes = need;
  b->used += need;
  sl.phase = next_phase(sl.st);
  *slot = (int32_t)k;
  return EGT_OK;
}

int egt_batch_tick(egt_batch* b, int32_t* n_active, int32_t* n_finished) {
  if (!b) return fail(EGT_EINVAL, "null batch");
  int32_t finished = 0;
  // 1: enqueue one phase of every live solve
  for (Slot& sl : b->slots) {
    if (sl.phase != kNeedGap && sl.phase != kNeedStep) continue;
    const int rc = sl.phase == kNeedGap ? gap_launch(sl.st, sl.stream) : step_launch(sl.st, -1, sl.stream);
    if (rc) {
      fail_slot(sl, rc);
      ++finished;
      continue;
    }
    sl.pending = true;
  }
  // 2: finish them in slot order
  for (Slot& sl : b->slots) {
    if (!sl.pending) continue;
    sl.pending = false;
    if (sl.phase == kNeedGap) {
      const int rc = gap_finish(sl.st, sl.stream);
      if (rc) {
        fail_slot(sl, rc);
        ++finished;
        continue;
      }
      const egt_solve_opts& op = state_opts(sl.st);
      if (state_gap_value(sl.st) <= op.eps) {
        finish_slot(sl, true);
        ++finished;
      } else if (state_iters(sl.st) >= op.max_iters) {
        finish_slot(sl, false);
        ++finished;
      } else {
        sl.phase = kNeedStep;
      }
    } else {
      int accepted = 0;
      const int rc = step_finish(sl.st, sl.stream, &accepted, nullptr, nullptr);
      if (rc) {
        fail_slot(sl, rc);
        ++finished;
        continue;
      }
      if (accepted) sl.phase = next_phase(sl.st);
    }
  }
  int32_t active = 0;
  for (const Slot& sl : b->slots)
    if (sl.phase == kNeedGap || sl.phase == kNeedStep) ++active;
  if (n_active) *n_active = active;
  if (n_finished) *n_finished = finished;
  return EGT_OK;
}

int egt_batch_poll(egt_batch* b, int32_t slot, int32_t* done, int32_t* status, egt_result* res) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size()) return fail(EGT_EINVAL, "bad batch or slot");
  const Slot& sl = b->slots[(size_t)slot];
  if (sl.phase == kFree) return fail(EGT_EINVAL, "slot is free");
  const bool d = sl.phase == kDone;
  if (done) *done = d ? 1 : 0;
  if (status) *status = d ? sl.status : EGT_OK;
  if (res && d) *res = sl.res;
  return EGT_OK;
}

int egt_batch_usage(const egt_batch* b, int64_t* used_bytes, int32_t* n_live, int32_t* n_done) {
  if (!b) return fail(EGT_EINVAL, "null batch");
  int32_t live = 0, dn = 0;
  for (const Slot& sl : b->slots) {
    if (sl.phase == kNeedGap || sl.phase == kNeedStep) ++live;
    if (sl.phase == kDone) ++dn;
  }
  if (used_bytes) *used_bytes = b->used;
  if (n_live) *n_live = live;
  if (n_done) *n_done = dn;
  return EGT_OK;
}

}  // extern "C"
