// extern "C" entry points of libegt (declared in include/egt.h).  Argument
// checking, the per-game scratch workspace used by the single-operation calls,
// and the translation of internal failures into status codes.
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "egt_internal.h"

namespace egt {
int build_game(const egt_game_desc* d, hipStream_t stream, egt_game** out);
int build_general_game(const egt_general_desc* d, hipStream_t stream, egt_game** out);
int free_game(egt_game* g);
const char* last_error_cstr();
int state_create(const egt_game* g, const egt_solve_opts* o, hipStream_t s, egt_state** out);
int state_destroy(egt_state* st);
int state_step(egt_state* st, int player, double* egv_out, int* stepped, hipStream_t s);
int state_get(const egt_state* st, double* x, double* y, double* mu_x, double* mu_y, double* tau,
              int64_t* iters, hipStream_t s);
int state_gap(egt_state* st, double* gap, double* brmax, double* brmin, hipStream_t s);
int state_get_products(const egt_state* st, double* ay, double* atx, hipStream_t s);
int state_set(egt_state* st, const double* x, const double* y, double mu_x, double mu_y, double tau, int64_t iters,
              const double* ay, const double* atx, hipStream_t s);
int solve(const egt_game* g, const egt_solve_opts* o, egt_result* res, egt_state** state_out, hipStream_t s);

namespace {

int ensure_workspace(const egt_game* cg) {
  egt_game* g = const_cast<egt_game*>(cg);  // the workspace is a cache owned by the game
  if (g->ws.block) return EGT_OK;
  size_t elems = 0;
  for (int p = 0; p < 2; ++p)
    elems += 2 * (size_t)g->hp[p].n_seq * g->ld + (size_t)g->hp[p].n_nodes * g->ld;
  elems += 16 + (size_t)kMaxTrees * kMaxPartials;
  void* blk = nullptr;
  hipError_t e = hipMalloc(&blk, elems * sizeof(double));
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc (workspace): ") + hipGetErrorString(e));
  double* hs = nullptr;
  e = hipHostMalloc((void**)&hs, 16 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(blk);
    return fail(EGT_ENOMEM, std::string("hipHostMalloc (workspace): ") + hipGetErrorString(e));
  }
  double* cur = (double*)blk;
  for (int p = 0; p < 2; ++p) {
    g->ws.grad[p] = cur;
    cur += (size_t)g->hp[p].n_seq * g->ld;
    g->ws.qb[p] = cur;
    cur += (size_t)g->hp[p].n_seq * g->ld;
    g->ws.v[p] = cur;
    cur += (size_t)g->hp[p].n_nodes * g->ld;
  }
  g->ws.scal = cur;
  g->ws.hscal = hs;
  g->ws.block = blk;
  return EGT_OK;
}

bool bad_player(int p) { return p != 0 && p != 1; }

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(EGT_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(EGT_EINVAL, e.what());
  } catch (...) {
    return fail(EGT_EINVAL, "unknown exception");
  }
}

}  // namespace
}  // namespace egt

using namespace egt;

extern "C" {

const char* egt_last_error(void) { return last_error_cstr(); }

void egt_default_opts(egt_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->variant = EGT_VARIANT_AS;
  o->precision = EGT_PRECISION_FP64;
  o->eps = 0.0;
  o->max_iters = 100000;
  o->mu0_x = 0.0;
  o->mu0_y = 0.0;
  o->tau0 = 0.5;
  o->gap_every = 1;
}

int egt_build_game(const egt_game_desc* desc, hipStream_t stream, egt_game** out) {
  return guarded([&]() -> int { return build_game(desc, stream, out); });
}

int egt_build_general_game(const egt_general_desc* desc, hipStream_t stream, egt_game** out) {
  return guarded([&]() -> int { return build_general_game(desc, stream, out); });
}

int egt_free_game(egt_game* game) {
  return guarded([&]() -> int { return free_game(game); });
}

int egt_game_dims(const egt_game* g, int player, int64_t* n_seq, int64_t* n_hands, int64_t* ld,
                  int64_t* n_nodes) {
  if (!g || bad_player(player)) return fail(EGT_EINVAL, "null game or bad player");
  if (n_seq) *n_seq = g->hp[player].n_seq;
  if (n_hands) *n_hands = g->n;
  if (ld) *ld = g->ld;
  if (n_nodes) *n_nodes = g->hp[player].n_nodes;
  return EGT_OK;
}

int egt_game_layout(const egt_game* g, int player, int32_t* hand_perm, char* keys, int64_t keys_cap,
                    int64_t* keys_len) {
  if (!g || bad_player(player)) return fail(EGT_EINVAL, "null game or bad player");
  return guarded([&]() -> int {
    if (hand_perm)
      for (int i = 0; i < g->n; ++i) hand_perm[i] = g->perm[i];
    std::string all;
    for (const std::string& k : g->hp[player].seq_keys) {
      all += k;
      all += '\n';
    }
    const int64_t need = (int64_t)all.size() + 1;
    if (keys_len) *keys_len = need;
    if (keys) {
      if (keys_cap < need) return fail(EGT_EINVAL, "keys buffer too small");
      std::memcpy(keys, all.c_str(), (size_t)need);
    }
    return EGT_OK;
  });
}

int egt_game_terminals(const egt_game* g, int64_t* n_fold, int64_t* n_show) {
  if (!g) return fail(EGT_EINVAL, "null game");
  if (n_fold) *n_fold = g->n_fold;
  if (n_show) *n_show = g->n_show;
  return EGT_OK;
}

int egt_gradient(const egt_game* g, int player, const double* strat_other, double* grad_out,
                 hipStream_t stream) {
  if (!g || bad_player(player) || !strat_other || !grad_out)
    return fail(EGT_EINVAL, "null argument or bad player");
  if (strat_other == grad_out) return fail(EGT_EINVAL, "grad_out must not alias strat_other");
  EGT_HIP(launch_gradient(g, player, strat_other, grad_out, stream));
  return EGT_OK;
}

int egt_smoothed_br(const egt_game* g, int player, const double* grad, double mu, double* strat_out,
                    double* value_out, hipStream_t stream) {
  if (!g || bad_player(player) || !grad) return fail(EGT_EINVAL, "null argument or bad player");
  if (!(mu > 0) || !std::isfinite(mu)) return fail(EGT_EINVAL, "mu must be finite and > 0");
  return guarded([&]() -> int {
    int rc = ensure_workspace(g);
    if (rc) return rc;
    const Workspace& w = g->ws;
    const Pass ps{player, grad, 1.0, nullptr, 0.0, mu, w.v[player], w.qb[player]};
    const Epilogue e{strat_out, nullptr, 0.0, nullptr};
    EGT_HIP(launch_passes(g, &ps, 1, &e, value_out ? w.scal + 16 : nullptr, stream));
    if (value_out) {
      EGT_HIP(launch_sum_partials(g, w.scal + 16, 1, w.scal, stream));
      EGT_HIP(hipMemcpyAsync(value_out, w.scal, sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
    return EGT_OK;
  });
}

int egt_gradient_mixed(const egt_game* g, int player, const float* strat_other, float* grad_out,
                       hipStream_t stream) {
  if (!g || bad_player(player) || !strat_other || !grad_out)
    return fail(EGT_EINVAL, "null argument or bad player");
  if ((const void*)strat_other == (const void*)grad_out) return fail(EGT_EINVAL, "grad_out must not alias strat_other");
  return guarded([&]() -> int {
    const int rc = ensure_mixed_tables(g);
    if (rc) return rc;
    EGT_HIP(launch_gradient_mixed(g, player, strat_other, grad_out, stream));
    return EGT_OK;
  });
}

int egt_smoothed_br_mixed(const egt_game* g, int player, const float* grad, double mu, float* strat_out,
                          double* value_out, hipStream_t stream) {
  if (!g || bad_player(player) || !grad) return fail(EGT_EINVAL, "null argument or bad player");
  if (!(mu > 0) || !std::isfinite(mu)) return fail(EGT_EINVAL, "mu must be finite and > 0");
  return guarded([&]() -> int {
    int rc = ensure_workspace(g);
    if (rc) return rc;
    const Workspace& w = g->ws;
    const Pass ps{player, grad, 1.0, nullptr, 0.0, mu, w.v[player], w.qb[player]};
    const Epilogue e{strat_out, nullptr, 0.0, nullptr};
    EGT_HIP(launch_passes(g, &ps, 1, &e, value_out ? w.scal + 16 : nullptr, stream, kF32));
    if (value_out) {
      EGT_HIP(launch_sum_partials(g, w.scal + 16, 1, w.scal, stream));
      EGT_HIP(hipMemcpyAsync(value_out, w.scal, sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
    return EGT_OK;
  });
}

int egt_best_response(const egt_game* g, int player, const double* grad, double* value_out,
                      hipStream_t stream) {
  if (!g || bad_player(player) || !grad || !value_out) return fail(EGT_EINVAL, "null argument or bad player");
  return guarded([&]() -> int {
    int rc = ensure_workspace(g);
    if (rc) return rc;
    const Workspace& w = g->ws;
    const Pass ps{player, grad, 1.0, nullptr, 0.0, 0.0, w.v[player], nullptr};
    EGT_HIP(launch_passes(g, &ps, 1, nullptr, w.scal + 16, stream));
    EGT_HIP(launch_sum_partials(g, w.scal + 16, 1, w.scal, stream));
    EGT_HIP(hipMemcpyAsync(value_out, w.scal, sizeof(double), hipMemcpyDeviceToDevice, stream));
    return EGT_OK;
  });
}

int egt_uniform(const egt_game* g, int player, double* strat_out, hipStream_t stream) {
  if (!g || bad_player(player) || !strat_out) return fail(EGT_EINVAL, "null argument or bad player");
  return guarded([&]() -> int {
    EGT_HIP(launch_uniform(g, player, strat_out, stream));
    return EGT_OK;
  });
}

int egt_saddle_gap(const egt_game* g, const double* x, const double* y, double* gap, double* br_max_y,
                   double* br_min_x, hipStream_t stream) {
  if (!g || !x || !y) return fail(EGT_EINVAL, "null argument");
  return guarded([&]() -> int {
    int rc = ensure_workspace(g);
    if (rc) return rc;
    const Workspace& w = g->ws;
    EGT_HIP(launch_gradient(g, 0, y, w.grad[0], stream));
    EGT_HIP(launch_gradient(g, 1, x, w.grad[1], stream));
    const Pass ps[2] = {{0, w.grad[0], 1.0, nullptr, 0.0, 0.0, w.v[0], nullptr},
                        {1, w.grad[1], -1.0, nullptr, 0.0, 0.0, w.v[1], nullptr}};
    EGT_HIP(launch_passes(g, ps, 2, nullptr, w.scal + 16, stream));
    EGT_HIP(launch_sum_partials(g, w.scal + 16, 2, w.scal, stream));
    EGT_HIP(hipMemcpyAsync(w.hscal, w.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
    EGT_HIP(hipStreamSynchronize(stream));
    // gap = max_y x^T A y - min_x x^T A y = -BR_y(-A^T x) - BR_x(A y)
    if (gap) *gap = -w.hscal[1] - w.hscal[0];
    if (br_min_x) *br_min_x = w.hscal[0];
    if (br_max_y) *br_max_y = -w.hscal[1];
    return EGT_OK;
  });
}

int egt_state_create(const egt_game* g, const egt_solve_opts* opts, hipStream_t stream, egt_state** out) {
  return guarded([&]() -> int { return state_create(g, opts, stream, out); });
}

int egt_state_destroy(egt_state* st) {
  return guarded([&]() -> int { return state_destroy(st); });
}

int egt_step(egt_state* st, int player, double* egv_out, int* player_stepped, hipStream_t stream) {
  return guarded([&]() -> int { return state_step(st, player, egv_out, player_stepped, stream); });
}

int egt_state_get(const egt_state* st, double* x, double* y, double* mu_x, double* mu_y, double* tau,
                  int64_t* iters, hipStream_t stream) {
  return guarded([&]() -> int { return state_get(st, x, y, mu_x, mu_y, tau, iters, stream); });
}

int egt_state_get_products(const egt_state* st, double* ay, double* atx, hipStream_t stream) {
  return guarded([&]() -> int { return state_get_products(st, ay, atx, stream); });
}

int egt_state_set(egt_state* st, const double* x, const double* y, double mu_x, double mu_y, double tau,
                  int64_t iters, const double* ay, const double* atx, hipStream_t stream) {
  return guarded([&]() -> int { return state_set(st, x, y, mu_x, mu_y, tau, iters, ay, atx, stream); });
}

int egt_state_gap(egt_state* st, double* gap, double* br_max_y, double* br_min_x, hipStream_t stream) {
  return guarded([&]() -> int { return state_gap(st, gap, br_max_y, br_min_x, stream); });
}

int egt_solve(const egt_game* g, const egt_solve_opts* opts, egt_result* result, egt_state** state_out,
              hipStream_t stream) {
  return guarded([&]() -> int { return solve(g, opts, result, state_out, stream); });
}

}  // extern "C"
