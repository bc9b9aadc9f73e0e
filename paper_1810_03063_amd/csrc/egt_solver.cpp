// EGT driver: device-resident iterates, the Step of Algorithm 2, the EGT/as
// Decr of Algorithm 4 and the side selection of Algorithms 1 and 3 (alternate,
// or the player with the larger mu).  Scalars (mu, tau, the EGV sign test) are
// FP64 on the host; one small device->host copy per step attempt carries the
// excessive gap value and the saddle gap of the candidate point.
//
// Notation.  G[0] = A y and G[1] = A^T x at the current iterate.  Player p
// minimises <q, sg[p] G[p]> with sg = (+1, -1): the y-focused step is the
// x-focused one on the mirrored problem min_y max_x <y, -A^T x>.
//
// Step focused on p (o = 1 - p), with the shift-free prox (the prox's shifted
// gradient  tau/((1-tau) mu_p) g3 - grad d(x_bar)  differs from
// (g1 + tau/(1-tau) g3) / mu_p only by a constant per simplex, because x_bar
// is the smoothed best response to g1; such a shift leaves the argmin
// unchanged):
//   x_bar = SBR_p(sg G[p], mu_p);         x_hat = (1-tau) x + tau x_bar
//   T1[o] = grad_o(x_hat);                y_bar = SBR_o(sg T1[o], mu_o)
//   y_+   = (1-tau) y + tau y_bar;        T1[p] = grad_p(y_bar)
//   x_+   = (1-tau) x + tau SBR_p(sg (G[p] + tau/(1-tau) T1[p]), mu_p)
//   T2[o] = grad_o(x_+);                  mu_p+ = (1-tau) mu_p
//   EGV   = V_p(sg ((1-tau) G[p] + tau T1[p]), mu_p+) + V_o(sg T2[o], mu_o)
// (grad_p at y_+ follows by linearity).  On EGV < 0 (EGT/as) tau halves and the
// step restarts from x_hat, reusing x_bar.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "egt_internal.h"

struct egt_state {
  const egt_game* g = nullptr;
  egt_solve_opts opts{};
  double mu[2] = {0, 0};
  double tau = 0.5;
  int64_t t = 0;
  int64_t products = 0;
  int64_t backtracks = 0;
  // device buffers, each [n_seq(p)][ld] (V: [n_nodes(p)][ld])
  double* X[2] = {};
  double* Xn[2] = {};
  double* Xbar[2] = {};
  double* Xhat[2] = {};
  double* G[2] = {};
  double* T1[2] = {};
  double* T2[2] = {};
  double* QB[2] = {};
  double* V[2] = {};
  double* Vb[2] = {};       // node values of the best-response passes
  double* dscal = nullptr;  // device scalars
  double* hscal = nullptr;  // pinned host mirror (also the summed tree values)
  double* dpart = nullptr;  // device root partial sums [trees][n_partials]
  double* hpart = nullptr;  // pinned host mirror
  void* block = nullptr;
  // last saddle gap of the current iterate (valid when gap_valid)
  bool gap_valid = false;
  double gap = 0, br_max_y = 0, br_min_x = 0;
  double last_egv = 0;
};

namespace egt {

namespace {

constexpr double kSg[2] = {1.0, -1.0};
constexpr double kTauFloor = 1e-30;
constexpr int kMaxDoublings = 200;

int64_t vec_elems(const egt_game* g, int p) { return (int64_t)g->hp[p].n_seq * g->ld; }

#define EGT_TRY(expr)                                            \
  do {                                                           \
    hipError_t _e = (expr);                                      \
    if (_e != hipSuccess) return ::egt::hip_fail(_e, #expr);     \
  } while (0)

// Smoothed best response of player p to cA gA + cB gB: q to q_out and the
// epilogue (1 - tau) x_prev + tau q to comb_out (either may be null).
int sbr(egt_state* st, int p, const double* gA, double cA, const double* gB, double cB, double mu,
        double* q_out, const double* x_prev, double tau, double* comb_out, hipStream_t s) {
  const Pass ps{p, gA, cA, gB, cB, mu, st->V[p], st->QB[p]};
  const Epilogue e{q_out, x_prev, tau, comb_out};
  EGT_TRY(launch_passes(st->g, &ps, 1, &e, nullptr, s));
  return EGT_OK;
}

int grad(egt_state* st, int p, const double* v_opp, double* out, hipStream_t s) {
  st->products++;
  EGT_TRY(launch_gradient(st->g, p, v_opp, out, s));
  return EGT_OK;
}

// Copies the root partial sums of `trees` trees to the host and adds each
// tree's partials in order into hscal[k].
int fetch_values(egt_state* st, int trees, hipStream_t s) {
  const int nb = n_partials(st->g);
  EGT_TRY(hipMemcpyAsync(st->hpart, st->dpart, sizeof(double) * trees * nb, hipMemcpyDeviceToHost, s));
  EGT_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < trees; ++k) {
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += st->hpart[k * nb + b];
    if (!std::isfinite(v)) return fail(EGT_ENUMERIC, "non-finite value in the EGT driver");
    st->hscal[k] = v;
  }
  return EGT_OK;
}

int fetch(egt_state* st, int count, hipStream_t s) {
  EGT_TRY(hipMemcpyAsync(st->hscal, st->dscal, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  EGT_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i)
    if (!std::isfinite(st->hscal[i])) return fail(EGT_ENUMERIC, "non-finite scalar in the EGT driver");
  return EGT_OK;
}

// EGV at (X, Y) with the state's G and mu -> hscal[0] + hscal[1] after fetch_values.
int egv_current(egt_state* st, hipStream_t s) {
  const egt_game* g = st->g;
  const Pass ps[2] = {{0, st->G[0], kSg[0], nullptr, 0.0, st->mu[0], st->V[0], nullptr},
                      {1, st->G[1], kSg[1], nullptr, 0.0, st->mu[1], st->V[1], nullptr}};
  EGT_TRY(launch_passes(g, ps, 2, nullptr, st->dpart, s));
  return EGT_OK;
}

// The two best-response passes of the saddle gap at the point whose products
// are A y = cXA gXA + cXB gXB and A^T x = cYA gYA + cYB gYB (gXB / gYB may be
// null): tree values BR_x(A y) and BR_y(-A^T x), so that
// gap = -BR_y - BR_x = max_y x^T A y - min_x x^T A y.
void gap_passes(egt_state* st, const double* gXA, double cXA, const double* gXB, double cXB, const double* gYA,
                double cYA, const double* gYB, double cYB, Pass out[2]) {
  out[0] = Pass{0, gXA, kSg[0] * cXA, gXB, kSg[0] * cXB, 0.0, st->Vb[0], nullptr};
  out[1] = Pass{1, gYA, kSg[1] * cYA, gYB, kSg[1] * cYB, 0.0, st->Vb[1], nullptr};
}

int init_point(egt_state* st, const double* atx_omega, hipStream_t s) {
  // y0 = y_{mu_y}(x_omega) = SBR_y(-A^T x_omega); x0 = x_{mu_x}(y0) = SBR_x(A y0)
  int rc;
  if ((rc = sbr(st, 1, atx_omega, kSg[1], nullptr, 0.0, st->mu[1], st->X[1], nullptr, 0.0, nullptr, s))) return rc;
  if ((rc = grad(st, 0, st->X[1], st->G[0], s))) return rc;
  if ((rc = sbr(st, 0, st->G[0], kSg[0], nullptr, 0.0, st->mu[0], st->X[0], nullptr, 0.0, nullptr, s))) return rc;
  if ((rc = grad(st, 1, st->X[0], st->G[1], s))) return rc;
  return EGT_OK;
}

}  // namespace

int state_create(const egt_game* g, const egt_solve_opts* o, hipStream_t s, egt_state** out) {
  if (!g || !out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  egt_solve_opts opts;
  egt_default_opts(&opts);
  if (o) opts = *o;
  if (opts.variant < EGT_VARIANT_ALT || opts.variant > EGT_VARIANT_AS)
    return fail(EGT_EINVAL, "unknown variant");
  if (opts.precision != EGT_PRECISION_FP64) return fail(EGT_EINVAL, "this state supports FP64 only");
  if (opts.eps <= 0) opts.eps = 1e-3 * g->pot;
  if (opts.tau0 <= 0) opts.tau0 = 0.5;
  if (!(opts.tau0 < 1.0)) return fail(EGT_EINVAL, "tau0 must be < 1");
  if (opts.gap_every < 1) opts.gap_every = 1;
  if (opts.max_iters < 0) return fail(EGT_EINVAL, "max_iters < 0");
  const bool auto_mu = !(opts.mu0_x > 0) && !(opts.mu0_y > 0);
  if (!auto_mu && (!(opts.mu0_x > 0) || !(opts.mu0_y > 0) || !std::isfinite(opts.mu0_x) ||
                   !std::isfinite(opts.mu0_y)))
    return fail(EGT_EINVAL, "mu0_x and mu0_y must both be > 0 (or both <= 0 for automatic)");

  egt_state* st = new (std::nothrow) egt_state();
  if (!st) return fail(EGT_ENOMEM, "host allocation failed");
  std::unique_ptr<egt_state, int (*)(egt_state*)> guard(st, [](egt_state* p) {
    return egt_state_destroy(p);
  });
  st->g = g;
  st->opts = opts;
  st->tau = opts.tau0;
  size_t bytes = 0;
  for (int p = 0; p < 2; ++p)
    bytes += sizeof(double) * (8 * (size_t)vec_elems(g, p) + 2 * (size_t)g->hp[p].n_nodes * g->ld);
  bytes += (64 + (size_t)kMaxTrees * kMaxPartials) * sizeof(double);
  hipError_t e = hipMalloc(&st->block, bytes);
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipHostMalloc((void**)&st->hscal, (64 + (size_t)kMaxTrees * kMaxPartials) * sizeof(double),
                    hipHostMallocDefault);
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  st->hpart = st->hscal + 64;
  double* cur = (double*)st->block;
  auto take = [&](int64_t n) {
    double* r = cur;
    cur += n;
    return r;
  };
  for (int p = 0; p < 2; ++p) {
    const int64_t n = vec_elems(g, p);
    st->X[p] = take(n);
    st->Xn[p] = take(n);
    st->Xbar[p] = take(n);
    st->Xhat[p] = take(n);
    st->G[p] = take(n);
    st->T1[p] = take(n);
    st->T2[p] = take(n);
    st->QB[p] = take(n);
    st->V[p] = take((int64_t)g->hp[p].n_nodes * g->ld);
    st->Vb[p] = take((int64_t)g->hp[p].n_nodes * g->ld);
  }
  st->dscal = take(64);
  st->dpart = take((int64_t)kMaxTrees * kMaxPartials);
  EGT_HIP(hipMemsetAsync(st->block, 0, bytes, s));

  // x_omega and A^T x_omega (kept in T2[1] for the mu search)
  int rc;
  EGT_TRY(launch_uniform_qbar(g, 0, st->QB[0], s));
  EGT_TRY(launch_top_down(g, 0, st->QB[0], st->Xbar[0], nullptr, 0.0, nullptr, s));
  if ((rc = grad(st, 1, st->Xbar[0], st->T2[1], s))) return rc;
  if (auto_mu) {
    // mu0 = 1e-3 max(|A y_omega|_inf, |A^T x_omega|_inf) / max beta, then double
    // both until the excessive gap condition holds at (x0, y0).
    EGT_TRY(launch_uniform_qbar(g, 1, st->QB[1], s));
    EGT_TRY(launch_top_down(g, 1, st->QB[1], st->Xbar[1], nullptr, 0.0, nullptr, s));
    if ((rc = grad(st, 0, st->Xbar[1], st->T2[0], s))) return rc;
    EGT_TRY(launch_max_abs(vec_elems(g, 0), st->T2[0], st->dscal, s));
    EGT_TRY(launch_max_abs(vec_elems(g, 1), st->T2[1], st->dscal + 1, s));
    if ((rc = fetch(st, 2, s))) return rc;
    const double m0 = 1e-3 * std::max(st->hscal[0], st->hscal[1]) / g->max_beta;
    if (!(m0 > 0)) return fail(EGT_ENUMERIC, "automatic mu is zero (all-zero payoffs?)");
    st->mu[0] = st->mu[1] = m0;
    for (int k = 0;; ++k) {
      if ((rc = init_point(st, st->T2[1], s))) return rc;
      if ((rc = egv_current(st, s))) return rc;
      if ((rc = fetch_values(st, 2, s))) return rc;
      if (!(st->hscal[0] + st->hscal[1] < 0.0)) break;
      if (k >= kMaxDoublings) return fail(EGT_ENOTCONV, "no initial mu satisfies the excessive gap condition");
      st->mu[0] *= 2.0;
      st->mu[1] *= 2.0;
    }
  } else {
    st->mu[0] = opts.mu0_x;
    st->mu[1] = opts.mu0_y;
    if ((rc = init_point(st, st->T2[1], s))) return rc;
    EGT_HIP(hipStreamSynchronize(s));
  }
  st->products = 0;  // count products of the iterations only
  *out = guard.release();
  return EGT_OK;
}

int state_destroy(egt_state* st) {
  if (!st) return EGT_OK;
  int rc = EGT_OK;
  if (st->block || st->hscal) {
    hipError_t e = hipDeviceSynchronize();
    if (st->block && e == hipSuccess) e = hipFree(st->block);
    if (st->hscal && e == hipSuccess) e = hipHostFree(st->hscal);
    if (e != hipSuccess) rc = hip_fail(e, "state_destroy");
  }
  delete st;
  return rc;
}

int state_gap(egt_state* st, double* gap, double* brmax, double* brmin, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  if (!st->gap_valid) {
    int rc;
    Pass ps[2];
    gap_passes(st, st->G[0], 1.0, nullptr, 0.0, st->G[1], 1.0, nullptr, 0.0, ps);
    EGT_TRY(launch_passes(st->g, ps, 2, nullptr, st->dpart, s));
    if ((rc = fetch_values(st, 2, s))) return rc;
    st->br_min_x = st->hscal[0];
    st->br_max_y = -st->hscal[1];
    st->gap = -st->hscal[1] - st->hscal[0];
    st->gap_valid = true;
  }
  if (gap) *gap = st->gap;
  if (brmax) *brmax = st->br_max_y;
  if (brmin) *brmin = st->br_min_x;
  return EGT_OK;
}

// One attempt of the step focused on p at step size tau.  first = compute
// x_bar (otherwise reuse it).  Leaves the two EGV terms and the two
// best-response values of the candidate's saddle gap as root partials (dpart).
static int attempt(egt_state* st, int p, double tau, bool first, hipStream_t s) {
  const egt_game* g = st->g;
  const int o = 1 - p;
  int rc;
  if (first) {
    if ((rc = sbr(st, p, st->G[p], kSg[p], nullptr, 0.0, st->mu[p], st->Xbar[p], st->X[p], tau,
                  st->Xhat[p], s)))
      return rc;
  } else {
    EGT_TRY(launch_axpby(vec_elems(g, p), 1.0 - tau, st->X[p], tau, st->Xbar[p], st->Xhat[p], s));
  }
  if ((rc = grad(st, o, st->Xhat[p], st->T1[o], s))) return rc;
  if ((rc = sbr(st, o, st->T1[o], kSg[o], nullptr, 0.0, st->mu[o], st->Xbar[o], st->X[o], tau, st->Xn[o], s)))
    return rc;
  if ((rc = grad(st, p, st->Xbar[o], st->T1[p], s))) return rc;
  const double r = tau / (1.0 - tau);
  if ((rc = sbr(st, p, st->G[p], kSg[p], st->T1[p], kSg[p] * r, st->mu[p], nullptr, st->X[p], tau, st->Xn[p], s)))
    return rc;
  if ((rc = grad(st, o, st->Xn[p], st->T2[o], s))) return rc;
  const double mu_new = (1.0 - tau) * st->mu[p];
  // one launch for the four value passes: EGV at (x_+, y_+) with mu_p+ and the
  // unchanged mu_o, and the two best responses of the candidate's saddle gap
  Pass ps[4];
  ps[0] = Pass{p, st->G[p], kSg[p] * (1.0 - tau), st->T1[p], kSg[p] * tau, mu_new, st->V[p], nullptr};
  ps[1] = Pass{o, st->T2[o], kSg[o], nullptr, 0.0, st->mu[o], st->V[o], nullptr};
  if (p == 0)
    gap_passes(st, st->G[0], 1.0 - tau, st->T1[0], tau, st->T2[1], 1.0, nullptr, 0.0, ps + 2);
  else
    gap_passes(st, st->T2[0], 1.0, nullptr, 0.0, st->G[1], 1.0 - tau, st->T1[1], tau, ps + 2);
  EGT_TRY(launch_passes(g, ps, 4, nullptr, st->dpart, s));
  return EGT_OK;
}

int state_step(egt_state* st, int player, double* egv_out, int* stepped, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  if (player < -1 || player > 1) return fail(EGT_EINVAL, "player must be -1, 0 or 1");
  const egt_game* g = st->g;
  const int variant = st->opts.variant;
  int p;
  double tau;
  if (variant == EGT_VARIANT_ALT) {
    tau = 2.0 / ((double)st->t + 3.0);
    p = (st->t % 2 == 0) ? 0 : 1;
  } else if (variant == EGT_VARIANT_BAL) {
    tau = 2.0 / ((double)st->t + 3.0);
    p = st->mu[0] > st->mu[1] ? 0 : 1;
  } else {
    tau = st->tau;
    p = st->mu[0] > st->mu[1] ? 0 : 1;
  }
  if (player >= 0) p = player;
  const int o = 1 - p;
  int rc;
  bool first = true;
  double egv = 0;
  for (;;) {
    if ((rc = attempt(st, p, tau, first, s))) return rc;
    first = false;
    if ((rc = fetch_values(st, 4, s))) return rc;
    egv = st->hscal[0] + st->hscal[1];
    if (variant != EGT_VARIANT_AS || !(egv < 0.0)) break;
    tau *= 0.5;
    st->backtracks++;
    if (tau < kTauFloor) return fail(EGT_ENOTCONV, "tau fell below 1e-30 in the EGT/as backtracking");
  }
  // accept: G[p] <- (1-tau) G[p] + tau T1[p] (linearity), G[o] <- T2[o]
  EGT_TRY(launch_axpby(vec_elems(g, p), 1.0 - tau, st->G[p], tau, st->T1[p], st->G[p], s));
  std::swap(st->G[o], st->T2[o]);
  std::swap(st->X[p], st->Xn[p]);
  std::swap(st->X[o], st->Xn[o]);
  st->mu[p] *= (1.0 - tau);
  if (variant == EGT_VARIANT_AS) st->tau = tau;
  st->t++;
  st->br_min_x = st->hscal[2];
  st->br_max_y = -st->hscal[3];
  st->gap = -st->hscal[3] - st->hscal[2];
  st->gap_valid = true;
  st->last_egv = egv;
  if (egv_out) *egv_out = egv;
  if (stepped) *stepped = p;
  return EGT_OK;
}

int state_get(const egt_state* st, double* x, double* y, double* mu_x, double* mu_y, double* tau, int64_t* iters,
              hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  const egt_game* g = st->g;
  if (x) EGT_HIP(hipMemcpyAsync(x, st->X[0], sizeof(double) * vec_elems(g, 0), hipMemcpyDeviceToDevice, s));
  if (y) EGT_HIP(hipMemcpyAsync(y, st->X[1], sizeof(double) * vec_elems(g, 1), hipMemcpyDeviceToDevice, s));
  if (mu_x) *mu_x = st->mu[0];
  if (mu_y) *mu_y = st->mu[1];
  if (tau) *tau = st->tau;
  if (iters) *iters = st->t;
  return EGT_OK;
}

int state_get_products(const egt_state* st, double* ay, double* atx, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  const egt_game* g = st->g;
  if (ay) EGT_HIP(hipMemcpyAsync(ay, st->G[0], sizeof(double) * vec_elems(g, 0), hipMemcpyDeviceToDevice, s));
  if (atx) EGT_HIP(hipMemcpyAsync(atx, st->G[1], sizeof(double) * vec_elems(g, 1), hipMemcpyDeviceToDevice, s));
  return EGT_OK;
}

int state_set(egt_state* st, const double* x, const double* y, double mu_x, double mu_y, double tau, int64_t iters,
              const double* ay, const double* atx, hipStream_t s) {
  if (!st || !x || !y) return fail(EGT_EINVAL, "null argument");
  if (!(mu_x > 0) || !(mu_y > 0) || !std::isfinite(mu_x) || !std::isfinite(mu_y))
    return fail(EGT_EINVAL, "mu must be finite and > 0");
  if (!(tau > 0) || !(tau < 1)) return fail(EGT_EINVAL, "tau must lie in (0, 1)");
  if (iters < 0) return fail(EGT_EINVAL, "iters < 0");
  const egt_game* g = st->g;
  EGT_HIP(hipMemcpyAsync(st->X[0], x, sizeof(double) * vec_elems(g, 0), hipMemcpyDeviceToDevice, s));
  EGT_HIP(hipMemcpyAsync(st->X[1], y, sizeof(double) * vec_elems(g, 1), hipMemcpyDeviceToDevice, s));
  int rc;
  if (ay) {
    EGT_HIP(hipMemcpyAsync(st->G[0], ay, sizeof(double) * vec_elems(g, 0), hipMemcpyDeviceToDevice, s));
  } else if ((rc = grad(st, 0, st->X[1], st->G[0], s))) {
    return rc;
  }
  if (atx) {
    EGT_HIP(hipMemcpyAsync(st->G[1], atx, sizeof(double) * vec_elems(g, 1), hipMemcpyDeviceToDevice, s));
  } else if ((rc = grad(st, 1, st->X[0], st->G[1], s))) {
    return rc;
  }
  EGT_HIP(hipStreamSynchronize(s));
  st->mu[0] = mu_x;
  st->mu[1] = mu_y;
  st->tau = tau;
  st->t = iters;
  st->gap_valid = false;
  return EGT_OK;
}

int solve(const egt_game* g, const egt_solve_opts* o, egt_result* res, egt_state** state_out, hipStream_t s) {
  if (!g || !res) return fail(EGT_EINVAL, "null argument");
  std::memset(res, 0, sizeof(*res));
  const auto t0 = std::chrono::steady_clock::now();
  egt_state* st = nullptr;
  int rc = state_create(g, o, s, &st);
  if (rc) return rc;
  const egt_solve_opts& op = st->opts;
  bool converged = false;
  for (;;) {
    const bool check = (st->t % op.gap_every == 0) || st->t >= op.max_iters;
    if (check) {
      if ((rc = state_gap(st, nullptr, nullptr, nullptr, s))) break;
      if (st->gap <= op.eps) {
        converged = true;
        break;
      }
    }
    if (st->t >= op.max_iters) break;
    if ((rc = state_step(st, -1, nullptr, nullptr, s))) break;
  }
  if (rc == EGT_OK && !st->gap_valid) rc = state_gap(st, nullptr, nullptr, nullptr, s);
  const auto t1 = std::chrono::steady_clock::now();
  res->iters = st->t;
  res->products = st->products;
  res->backtracks = st->backtracks;
  res->gap = st->gap;
  res->br_max_y = st->br_max_y;
  res->br_min_x = st->br_min_x;
  res->mu_x = st->mu[0];
  res->mu_y = st->mu[1];
  res->tau = st->tau;
  res->converged = converged ? 1 : 0;
  res->seconds = std::chrono::duration<double>(t1 - t0).count();
  if (rc == EGT_OK) {
    // value to player 1 = -(x^T A y) = -<x, G[0]>: a dot product via root sums
    // is not needed; compute it on the host from one copy of two small sums.
    double v = 0.0;
    const int64_t n0 = vec_elems(g, 0);
    double* hx = (double*)std::malloc(sizeof(double) * n0 * 2);
    if (!hx) {
      rc = fail(EGT_ENOMEM, "host allocation failed");
    } else {
      hipError_t e = hipMemcpyAsync(hx, st->X[0], sizeof(double) * n0, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(hx + n0, st->G[0], sizeof(double) * n0, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        rc = hip_fail(e, "copy of the final iterate");
      } else {
        for (int64_t i = 0; i < n0; ++i) v += hx[i] * hx[n0 + i];
        res->value_p1 = -v;
      }
      std::free(hx);
    }
  }
  if (rc == EGT_OK && !converged) rc = fail(EGT_ENOTCONV, "iteration cap reached before the target gap");
  if (state_out && (rc == EGT_OK || rc == EGT_ENOTCONV)) {
    *state_out = st;
  } else {
    state_destroy(st);
  }
  return rc;
}

}  // namespace egt
