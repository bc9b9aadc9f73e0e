// Serving form: continuous batching of endgame solves on one device.
//
// A batch reserves its device-memory budget once (one arena) plus a pinned
// host buffer and a HIP stream per slot.  Admitting a solve charges the
// bytes of its state against the budget -- it takes a first-fit range of the
// arena, or is refused (EGT_EBUDGET) until a finished solve is retired -- and
// queues it for a pool of host worker threads.  A worker creates the state in
// its arena range and runs the solve (the same loop and kernels as
// egt_solve) on the slot's stream; solves on different workers run
// concurrently, so requests that arrive while others are running start as
// soon as memory and a worker are free, and their kernels overlap on the
// device.  No step of a solve depends on the other solves, so a result is
// bitwise the same alone and in the mix.  The hot path allocates nothing:
// no hipMalloc, no host pinning and no device-wide synchronisation after the
// batch is created.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "egt_internal.h"

namespace egt {
int state_create_in(const egt_game* g, const egt_solve_opts* o, hipStream_t s, void* dev_mem, double* host_mem,
                    egt_state** out);
int state_destroy(egt_state* st);
int solve_loop(egt_state* st, hipStream_t s, const std::atomic<bool>* stop, bool* converged);
int fill_result(egt_state* st, bool converged, double seconds, egt_result* res, hipStream_t s);
int state_get(const egt_state* st, double* x, double* y, double* mu_x, double* mu_y, double* tau, int64_t* iters,
              hipStream_t s);
int64_t state_bytes(const egt_game* g, bool mixed);
size_t state_host_doubles();
int build_game_host(const egt_game_desc* d, egt_game** out);
size_t game_device_bytes(const egt_game* g);
int upload_game(egt_game* g, void* dev, bool owned, hipStream_t stream);
int free_game(egt_game* g);
}  // namespace egt

namespace {

enum Phase { kFree = 0, kQueued, kRunning, kDone };

struct Slot {
  Phase phase = kFree;
  const egt_game* g = nullptr;
  egt_game* own_game = nullptr;  // admitted by description: the batch's, tables in the arena
  std::vector<unsigned char> mx_img;  // its precision-form tables, uploaded by the worker
  size_t mx_off[2][4] = {};
  int64_t game_bytes = 0, mx_bytes = 0;  // arena bytes ahead of the state
  egt_solve_opts opts{};
  egt_state* st = nullptr;
  hipStream_t stream = nullptr;  // created with the batch, default priority
  double* host = nullptr;        // pinned, created with the batch
  int64_t off = 0, bytes = 0;    // arena range
  int status = EGT_OK;
  egt_result res{};
  std::chrono::steady_clock::time_point t0;
};

struct Range {
  int64_t off, len;
};

}  // namespace

struct egt_batch {
  int64_t budget = 0;
  int64_t used = 0;
  void* arena = nullptr;
  std::vector<Range> free_list;  // sorted by offset, coalesced
  std::vector<Slot> slots;
  std::deque<int> queue;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable work_cv, done_cv;
  std::atomic<bool> stop{false};  // set by destroy, read by the workers' solve loops
  int64_t finished_total = 0, finished_seen = 0;
  int device = 0;
};

using namespace egt;

namespace {

constexpr int64_t kAlign = 256;

bool arena_take(egt_batch* b, int64_t need, int64_t* off) {
  for (size_t i = 0; i < b->free_list.size(); ++i) {
    Range& r = b->free_list[i];
    if (r.len >= need) {
      *off = r.off;
      r.off += need;
      r.len -= need;
      if (r.len == 0) b->free_list.erase(b->free_list.begin() + (long)i);
      return true;
    }
  }
  return false;
}

void arena_give(egt_batch* b, int64_t off, int64_t len) {
  auto it = std::lower_bound(b->free_list.begin(), b->free_list.end(), off,
                             [](const Range& r, int64_t o) { return r.off < o; });
  it = b->free_list.insert(it, Range{off, len});
  // coalesce with the neighbours
  size_t i = (size_t)(it - b->free_list.begin());
  if (i + 1 < b->free_list.size() && b->free_list[i].off + b->free_list[i].len == b->free_list[i + 1].off) {
    b->free_list[i].len += b->free_list[i + 1].len;
    b->free_list.erase(b->free_list.begin() + (long)i + 1);
  }
  if (i > 0 && b->free_list[i - 1].off + b->free_list[i - 1].len == b->free_list[i].off) {
    b->free_list[i - 1].len += b->free_list[i].len;
    b->free_list.erase(b->free_list.begin() + (long)i);
  }
}

void run_slot(egt_batch* b, Slot& sl) {
  hipError_t e = hipSetDevice(b->device);
  int rc = e == hipSuccess ? EGT_OK : hip_fail(e, "hipSetDevice");
  unsigned char* base = (unsigned char*)b->arena + sl.off;
  if (rc == EGT_OK && sl.own_game) {
    // the game's tables (and precision-form tables) into the slot's arena range, on its stream
    rc = upload_game(sl.own_game, base, false, sl.stream);
    if (rc == EGT_OK && sl.mx_bytes > 0)
      rc = mixed_tables_upload(sl.own_game, sl.mx_img, sl.mx_off, base + sl.game_bytes, false, sl.stream);
  }
  egt_state* st = nullptr;
  if (rc == EGT_OK)
    rc = state_create_in(sl.g, &sl.opts, sl.stream, base + sl.game_bytes + sl.mx_bytes, sl.host, &st);
  bool converged = false;
  if (rc == EGT_OK) rc = solve_loop(st, sl.stream, &b->stop, &converged);
  egt_result res{};
  if (rc == EGT_OK) {
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
    rc = fill_result(st, converged, secs, &res, sl.stream);
    if (rc == EGT_OK && !converged) rc = EGT_ENOTCONV;
  } else {
    res.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl.t0).count();
  }
  if (st) (void)hipStreamSynchronize(sl.stream);
  std::lock_guard<std::mutex> lk(b->mu);
  sl.st = st;  // kept (in its arena range) until the slot is retired, for egt_batch_strategies
  sl.res = res;
  sl.status = rc;
  sl.phase = kDone;
  ++b->finished_total;
  b->done_cv.notify_all();
}

void worker_main(egt_batch* b) {
  for (;;) {
    int k;
    {
      std::unique_lock<std::mutex> lk(b->mu);
      b->work_cv.wait(lk, [&] { return b->stop || !b->queue.empty(); });
      if (b->stop && b->queue.empty()) return;
      k = b->queue.front();
      b->queue.pop_front();
      b->slots[(size_t)k].phase = kRunning;
    }
    run_slot(b, b->slots[(size_t)k]);
  }
}

}  // namespace

extern "C" {

int egt_state_bytes(const egt_game* g, const egt_solve_opts* opts, int64_t* bytes) {
  if (!g || !bytes) return fail(EGT_EINVAL, "null argument");
  const bool mixed = opts && opts->precision == EGT_PRECISION_MIXED;
  *bytes = (state_bytes(g, mixed) + kAlign - 1) / kAlign * kAlign;
  return EGT_OK;
}

int egt_batch_create(int64_t budget_bytes, int32_t max_slots, egt_batch** out) {
  if (!out || budget_bytes <= 0 || max_slots < 1 || max_slots > 1024)
    return fail(EGT_EINVAL, "budget must be > 0 and max_slots in 1..1024");
  *out = nullptr;
  egt_batch* b = new (std::nothrow) egt_batch();
  if (!b) return fail(EGT_ENOMEM, "host allocation failed");
  b->budget = (budget_bytes + kAlign - 1) / kAlign * kAlign;
  EGT_HIP(hipGetDevice(&b->device));
  hipError_t e = hipMalloc(&b->arena, (size_t)b->budget);
  if (e != hipSuccess) {
    delete b;
    return fail(EGT_ENOMEM, std::string("hipMalloc (batch arena): ") + hipGetErrorString(e));
  }
  b->free_list.push_back(Range{0, b->budget});
  b->slots.resize((size_t)max_slots);
  for (Slot& sl : b->slots) {
    // non-blocking: the slots' work never orders itself against the null stream
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&sl.host, sizeof(double) * state_host_doubles(), hipHostMallocDefault);
    if (e != hipSuccess) {
      egt_batch_destroy(b);
      return fail(EGT_ENOMEM, std::string("batch slot resources: ") + hipGetErrorString(e));
    }
  }
  const int n_workers = std::min<int>(max_slots, 16);
  try {
    for (int i = 0; i < n_workers; ++i) b->workers.emplace_back(worker_main, b);
  } catch (...) {
    egt_batch_destroy(b);
    return fail(EGT_ENOMEM, "could not start the batch workers");
  }
  *out = b;
  return EGT_OK;
}

int egt_batch_retire(egt_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size()) return fail(EGT_EINVAL, "bad batch or slot");
  std::lock_guard<std::mutex> lk(b->mu);
  Slot& sl = b->slots[(size_t)slot];
  if (sl.phase != kDone) return fail(EGT_EINVAL, "only a finished solve can be retired");
  if (sl.st) state_destroy(sl.st);  // its memory stays with the batch
  if (sl.own_game) free_game(sl.own_game);  // host tables only: its device tables lie in the arena
  arena_give(b, sl.off, sl.bytes);
  b->used -= sl.bytes;
  hipStream_t stream = sl.stream;
  double* host = sl.host;
  sl = Slot();
  sl.stream = stream;
  sl.host = host;
  return EGT_OK;
}

int egt_batch_destroy(egt_batch* b) {
  if (!b) return EGT_OK;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->stop = true;
    b->queue.clear();
  }
  b->work_cv.notify_all();
  for (std::thread& t : b->workers) t.join();
  int rc = EGT_OK;
  for (Slot& sl : b->slots) {
    if (sl.st) {
      state_destroy(sl.st);
      sl.st = nullptr;
    }
    if (sl.own_game) {
      free_game(sl.own_game);
      sl.own_game = nullptr;
    }
    if (sl.stream) {
      const hipError_t e = hipStreamDestroy(sl.stream);
      if (e != hipSuccess && rc == EGT_OK) rc = hip_fail(e, "hipStreamDestroy");
    }
    if (sl.host) (void)hipHostFree(sl.host);
  }
  if (b->arena) (void)hipFree(b->arena);
  delete b;
  return rc;
}

int egt_batch_admit(egt_batch* b, const egt_game* g, const egt_solve_opts* opts, int32_t* slot) {
  if (!b || !g || !slot) return fail(EGT_EINVAL, "null argument");
  *slot = -1;
  egt_solve_opts o;
  egt_default_opts(&o);
  if (opts) o = *opts;
  const bool mixed = o.precision == EGT_PRECISION_MIXED;
  const int64_t need = (state_bytes(g, mixed) + kAlign - 1) / kAlign * kAlign;
  std::unique_lock<std::mutex> lk(b->mu);
  size_t k = 0;
  while (k < b->slots.size() && b->slots[k].phase != kFree) ++k;
  if (k == b->slots.size()) return fail(EGT_EBUDGET, "no free slot");
  int64_t off = 0;
  if (b->used + need > b->budget || !arena_take(b, need, &off))
    return fail(EGT_EBUDGET, "the solve does not fit the memory budget now");
  b->used += need;
  if (mixed) {  // the game's shared precision-form tables, built once admission is certain (not on a worker)
    b->slots[k].phase = kQueued;  // hold the slot while the lock is released
    lk.unlock();
    const int rc = ensure_mixed_tables(g);
    lk.lock();
    if (rc) {
      b->slots[k].phase = kFree;
      arena_give(b, off, need);
      b->used -= need;
      return rc;
    }
  }
  Slot& sl = b->slots[k];
  sl.phase = kQueued;
  sl.g = g;
  sl.opts = o;
  sl.off = off;
  sl.bytes = need;
  sl.status = EGT_OK;
  sl.t0 = std::chrono::steady_clock::now();
  b->queue.push_back((int)k);
  b->work_cv.notify_one();
  *slot = (int32_t)k;
  return EGT_OK;
}

int egt_batch_admit_desc(egt_batch* b, const egt_game_desc* desc, const egt_solve_opts* opts, int32_t* slot) {
  if (!b || !desc || !slot) return fail(EGT_EINVAL, "null argument");
  *slot = -1;
  egt_solve_opts o;
  egt_default_opts(&o);
  if (opts) o = *opts;
  const bool mixed = o.precision == EGT_PRECISION_MIXED;
  // host work only: the betting tree, the tables and (precision form) W
  egt_game* g = nullptr;
  int rc = build_game_host(desc, &g);
  if (rc) return rc;
  std::vector<unsigned char> mx_img;
  size_t mx_off[2][4] = {};
  if (mixed && (rc = mixed_tables_image(g, mx_img, mx_off))) {
    free_game(g);
    return rc;
  }
  const int64_t gbytes = (int64_t)((game_device_bytes(g) + kAlign - 1) / kAlign * kAlign);
  const int64_t mbytes = (int64_t)((mx_img.size() + kAlign - 1) / kAlign * kAlign);
  const int64_t need = gbytes + mbytes + (state_bytes(g, mixed) + kAlign - 1) / kAlign * kAlign;
  std::lock_guard<std::mutex> lk(b->mu);
  size_t k = 0;
  while (k < b->slots.size() && b->slots[k].phase != kFree) ++k;
  int64_t off = 0;
  if (k == b->slots.size() || b->used + need > b->budget || !arena_take(b, need, &off)) {
    free_game(g);
    return fail(EGT_EBUDGET, k == b->slots.size() ? "no free slot" : "the solve does not fit the memory budget now");
  }
  Slot& sl = b->slots[k];
  sl.phase = kQueued;
  sl.g = g;
  sl.own_game = g;
  sl.mx_img.swap(mx_img);
  std::memcpy(sl.mx_off, mx_off, sizeof(mx_off));
  sl.game_bytes = gbytes;
  sl.mx_bytes = mbytes;
  sl.opts = o;
  sl.off = off;
  sl.bytes = need;
  sl.status = EGT_OK;
  sl.t0 = std::chrono::steady_clock::now();
  b->used += need;
  b->queue.push_back((int)k);
  b->work_cv.notify_one();
  *slot = (int32_t)k;
  return EGT_OK;
}

int egt_batch_tick(egt_batch* b, int32_t* n_active, int32_t* n_finished) {
  if (!b) return fail(EGT_EINVAL, "null batch");
  std::unique_lock<std::mutex> lk(b->mu);
  auto live = [&] {
    int32_t a = 0;
    for (const Slot& sl : b->slots)
      if (sl.phase == kQueued || sl.phase == kRunning) ++a;
    return a;
  };
  if (b->finished_total == b->finished_seen && live() > 0)
    b->done_cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return b->finished_total != b->finished_seen; });
  if (n_finished) *n_finished = (int32_t)(b->finished_total - b->finished_seen);
  b->finished_seen = b->finished_total;
  if (n_active) *n_active = live();
  return EGT_OK;
}

int egt_batch_poll(egt_batch* b, int32_t slot, int32_t* done, int32_t* status, egt_result* res) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size()) return fail(EGT_EINVAL, "bad batch or slot");
  std::lock_guard<std::mutex> lk(b->mu);
  const Slot& sl = b->slots[(size_t)slot];
  if (sl.phase == kFree) return fail(EGT_EINVAL, "slot is free");
  const bool d = sl.phase == kDone;
  if (done) *done = d ? 1 : 0;
  if (status) *status = d ? sl.status : EGT_OK;
  if (res && d) *res = sl.res;
  return EGT_OK;
}

int egt_batch_strategies(egt_batch* b, int32_t slot, double* x, double* y, hipStream_t stream) {
  if (!b || slot < 0 || slot >= (int32_t)b->slots.size()) return fail(EGT_EINVAL, "bad batch or slot");
  egt_state* st = nullptr;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    const Slot& sl = b->slots[(size_t)slot];
    if (sl.phase != kDone || !sl.st) return fail(EGT_EINVAL, "the slot holds no finished solve");
    st = sl.st;
  }
  const int rc = state_get(st, x, y, nullptr, nullptr, nullptr, nullptr, stream);
  if (rc) return rc;
  EGT_HIP(hipStreamSynchronize(stream));
  return EGT_OK;
}

int egt_batch_usage(const egt_batch* cb, int64_t* used_bytes, int32_t* n_live, int32_t* n_done) {
  if (!cb) return fail(EGT_EINVAL, "null batch");
  egt_batch* b = const_cast<egt_batch*>(cb);
  std::lock_guard<std::mutex> lk(b->mu);
  int32_t live = 0, dn = 0;
  for (const Slot& sl : b->slots) {
    if (sl.phase == kQueued || sl.phase == kRunning) ++live;
    if (sl.phase == kDone) ++dn;
  }
  if (used_bytes) *used_bytes = b->used;
  if (n_live) *n_live = live;
  if (n_done) *n_done = dn;
  return EGT_OK;
}

}  // extern "C"
