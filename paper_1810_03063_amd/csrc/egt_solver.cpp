// EGT driver: device-resident iterates, the Step of Algorithm 2, the EGT/as
// Decr of Algorithm 4 and the side selection of Algorithms 1 and 3 (alternate,
// or the player with the larger mu).  Scalars (mu, tau, the EGV sign test) are
// FP64 on the host; one small device->host copy per step attempt carries the
// root partial sums of the excessive gap value (and, in FP64, of the
// candidate's saddle gap).
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
//
// Precision form: iterates, products and q_bar are FP32, the showdown products
// run on the BF16 matrix cores, node values and normalisers stay FP64, and the
// saddle gap is always measured with FP64 products of the (widened) iterates.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "egt_internal.h"

using egt::Prec;

struct egt_state {
  const egt_game* g = nullptr;
  egt_solve_opts opts{};
  Prec prec = egt::kF64;
  size_t esz = sizeof(double);
  double mu[2] = {0, 0};
  double tau = 0.5;
  int64_t t = 0;
  int64_t products = 0;
  int64_t backtracks = 0;
  // iterates and products in the state's precision, each [n_seq(p)][ld]
  void* X[2] = {};
  void* Xn[2] = {};
  void* Xbar[2] = {};
  void* Xhat[2] = {};
  void* G[2] = {};
  void* T1[2] = {};
  void* T2[2] = {};
  void* QB[2] = {};
  // the local strategies q_bar of the smoothed best response that opens the
  // next iteration, written by this iteration's value launch (whose EGV tree
  // of that side is the same bottom-up pass), and what they were computed
  // from: side, gradient buffer and mu (side -1: none)
  void* QN[2] = {};
  int qn_side = -1;
  const void* qn_grad = nullptr;
  double qn_mu = 0.0;
  // spares that let the next iteration run before this one is decided: on
  // acceptance X <- Xn <- Xs <- X and G <- T2 <- Gs <- G rotate, Xbar and the
  // partial-sum buffers alternate, so a rejected step still finds its x, G and
  // x_bar untouched
  void* Xs[2] = {};
  void* Gs[2] = {};
  void* Xbar2[2] = {};
  double* V[2] = {};        // node values [n_nodes(p)][ld], FP64
  double* Vb[2] = {};       // node values of the best-response passes
  double* X64[2] = {};      // FP64 iterates for the gap (precision form; else scratch aliases)
  double* G64[2] = {};      // FP64 products for the gap (precision form; else scratch aliases)
  double* dscal = nullptr;  // device scalars
  double* hscal = nullptr;  // pinned host mirror (also the summed tree values)
  double* hpart = nullptr;      // pinned root partial sums [trees][n_partials], written by the kernels
  double* hpart_dev = nullptr;  // device address of hpart
  double* hpart2 = nullptr;     // the alternate buffer
  double* hpart2_dev = nullptr;
  const double* pending_part = nullptr;  // buffer of the values awaiting finish_values
  hipEvent_t ev[2] = {nullptr, nullptr};  // end of an attempt's value launch
  void* block = nullptr;
  bool owns_memory = true;  // false: block and hscal belong to a serving batch
  // saddle gap of the current iterate (valid when gap_valid)
  bool gap_valid = false;
  double gap = 0, br_max_y = 0, br_min_x = 0;
  double last_egv = 0;
  // split launch / finish interface: the iteration in progress and the
  // value copy awaiting its finish
  bool step_open = false;
  int step_p = 0;
  double step_tau = 0;
  int pending_trees = 0;
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
int sbr(egt_state* st, int p, const void* gA, double cA, const void* gB, double cB, double mu, void* q_out,
        const void* x_prev, double tau, void* comb_out, hipStream_t s) {
  const Pass ps{p, gA, cA, gB, cB, mu, st->V[p], st->QB[p]};
  const Epilogue e{q_out, x_prev, tau, comb_out};
  EGT_TRY(launch_passes(st->g, &ps, 1, &e, nullptr, s, st->prec));
  return EGT_OK;
}

// Product of player p's gradient at the opponent's strategy, in the state's precision.
int grad(egt_state* st, int p, const void* v_opp, void* out, hipStream_t s) {
  if (st->prec == kF64)
    EGT_TRY(launch_gradient(st->g, p, (const double*)v_opp, (double*)out, s));
  else
    EGT_TRY(launch_gradient_mixed(st->g, p, (const float*)v_opp, (float*)out, s));
  return EGT_OK;
}

int axpby(egt_state* st, int p, double a, const void* X, double b, const void* Y, void* out, hipStream_t s) {
  EGT_TRY(launch_axpby(vec_elems(st->g, p), a, X, b, Y, out, s, st->prec));
  return EGT_OK;
}

// The value launch of `trees` trees writes their partial sums into pinned
// host memory (`part`, st->hpart by default); record what to read.
int enqueue_values(egt_state* st, int trees, hipStream_t, const double* part = nullptr) {
  st->pending_trees = trees;
  st->pending_part = part ? part : st->hpart;
  return EGT_OK;
}

// Waits until `done` reports completion: polls for up to kSpinSeconds (a
// blocking wait wakes up tens of microseconds late, which an iteration of
// ~100 us cannot afford), then blocks, so that many concurrent solves do not
// keep every host core busy.
template <class Query, class Block>
int wait_for(Query done, Block block) {
  constexpr double kSpinSeconds = 200e-6;
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e;
  while ((e = done()) == hipErrorNotReady &&
         std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() < kSpinSeconds) {
  }
  if (e != hipSuccess && e != hipErrorNotReady) return hip_fail(e, "query");
  EGT_TRY(block());
  return EGT_OK;
}

// Adds each pending tree's partials in order into hscal[k] (the launch has
// completed).
int read_values(egt_state* st) {
  const int nb = n_partials(st->g);
  const int trees = st->pending_trees;
  st->pending_trees = 0;
  for (int k = 0; k < trees; ++k) {
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += st->pending_part[k * nb + b];
    if (!std::isfinite(v)) return fail(EGT_ENUMERIC, "non-finite value in the EGT driver");
    st->hscal[k] = v;
  }
  return EGT_OK;
}

// Waits for the stream, then read_values.
int finish_values(egt_state* st, hipStream_t s) {
  const int rc = wait_for([&] { return hipStreamQuery(s); }, [&] { return hipStreamSynchronize(s); });
  return rc ? rc : read_values(st);
}

int fetch_values(egt_state* st, int trees, hipStream_t s) {
  int rc = enqueue_values(st, trees, s);
  return rc ? rc : finish_values(st, s);
}

int fetch(egt_state* st, int count, hipStream_t s) {
  EGT_TRY(hipMemcpyAsync(st->hscal, st->dscal, sizeof(double) * count, hipMemcpyDeviceToHost, s));
  EGT_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i)
    if (!std::isfinite(st->hscal[i])) return fail(EGT_ENUMERIC, "non-finite scalar in the EGT driver");
  return EGT_OK;
}

// EGV at (X, Y) with the state's G and mu: root partials of the two trees.
int egv_current(egt_state* st, hipStream_t s) {
  const Pass ps[2] = {{0, st->G[0], kSg[0], nullptr, 0.0, st->mu[0], st->V[0], nullptr},
                      {1, st->G[1], kSg[1], nullptr, 0.0, st->mu[1], st->V[1], nullptr}};
  EGT_TRY(launch_passes(st->g, ps, 2, nullptr, st->hpart_dev, s, st->prec));
  return EGT_OK;
}

// The two best-response passes of the saddle gap at the point whose products
// are A y = cXA gXA + cXB gXB and A^T x = cYA gYA + cYB gYB (gXB / gYB may be
// null): tree values BR_x(A y) and BR_y(-A^T x), so that
// gap = -BR_y - BR_x = max_y x^T A y - min_x x^T A y.
void gap_passes(egt_state* st, const void* gXA, double cXA, const void* gXB, double cXB, const void* gYA,
                double cYA, const void* gYB, double cYB, Pass out[2]) {
  out[0] = Pass{0, gXA, kSg[0] * cXA, gXB, kSg[0] * cXB, 0.0, st->Vb[0], nullptr};
  out[1] = Pass{1, gYA, kSg[1] * cYA, gYB, kSg[1] * cYB, 0.0, st->Vb[1], nullptr};
}

int init_point(egt_state* st, const void* atx_omega, hipStream_t s) {
  // y0 = y_{mu_y}(x_omega) = SBR_y(-A^T x_omega); x0 = x_{mu_x}(y0) = SBR_x(A y0)
  int rc;
  if ((rc = sbr(st, 1, atx_omega, kSg[1], nullptr, 0.0, st->mu[1], st->X[1], nullptr, 0.0, nullptr, s))) return rc;
  if ((rc = grad(st, 0, st->X[1], st->G[0], s))) return rc;
  if ((rc = sbr(st, 0, st->G[0], kSg[0], nullptr, 0.0, st->mu[0], st->X[0], nullptr, 0.0, nullptr, s))) return rc;
  if ((rc = grad(st, 1, st->X[0], st->G[1], s))) return rc;
  return EGT_OK;
}

// FP64 copy of a state-precision vector into dst (a plain copy in FP64).
int widen(egt_state* st, int p, const void* src, double* dst, hipStream_t s) {
  if (st->prec == kF64) {
    if (src != dst)
      EGT_TRY(hipMemcpyAsync(dst, src, sizeof(double) * vec_elems(st->g, p), hipMemcpyDeviceToDevice, s));
  } else {
    EGT_TRY(launch_convert(vec_elems(st->g, p), src, kF32, dst, s));
  }
  return EGT_OK;
}

int narrow(egt_state* st, int p, const double* src, void* dst, hipStream_t s) {
  if (st->prec == kF64)
    EGT_TRY(hipMemcpyAsync(dst, src, sizeof(double) * vec_elems(st->g, p), hipMemcpyDeviceToDevice, s));
  else
    EGT_TRY(launch_convert(vec_elems(st->g, p), src, kF64, dst, s));
  return EGT_OK;
}

}  // namespace

int64_t state_bytes(const egt_game* g, bool mixed);
size_t state_host_doubles();

int state_create_in(const egt_game* g, const egt_solve_opts* o, hipStream_t s, void* dev_mem, double* host_mem,
                    egt_state** out);

int state_create(const egt_game* g, const egt_solve_opts* o, hipStream_t s, egt_state** out) {
  return state_create_in(g, o, s, nullptr, nullptr, out);
}

// dev_mem (state_bytes(g, mixed) bytes, 256-byte aligned) and host_mem
// (pinned, state_host_doubles() doubles) may be given by the caller, who then
// keeps ownership; otherwise the state allocates them.
int state_create_in(const egt_game* g, const egt_solve_opts* o, hipStream_t s, void* dev_mem, double* host_mem,
                    egt_state** out) {
  if (!g || !out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  egt_solve_opts opts;
  egt_default_opts(&opts);
  if (o) opts = *o;
  if (opts.variant < EGT_VARIANT_ALT || opts.variant > EGT_VARIANT_AS)
    return fail(EGT_EINVAL, "unknown variant");
  if (opts.precision != EGT_PRECISION_FP64 && opts.precision != EGT_PRECISION_MIXED)
    return fail(EGT_EINVAL, "unknown precision");
  if (opts.eps <= 0) opts.eps = 1e-3 * g->pot;
  if (opts.tau0 <= 0) opts.tau0 = 0.5;
  if (!(opts.tau0 < 1.0)) return fail(EGT_EINVAL, "tau0 must be < 1");
  if (opts.gap_every < 1) opts.gap_every = 1;
  if (opts.max_iters < 0) return fail(EGT_EINVAL, "max_iters < 0");
  const bool auto_mu = !(opts.mu0_x > 0) && !(opts.mu0_y > 0);
  if (!auto_mu && (!(opts.mu0_x > 0) || !(opts.mu0_y > 0) || !std::isfinite(opts.mu0_x) ||
                   !std::isfinite(opts.mu0_y)))
    return fail(EGT_EINVAL, "mu0_x and mu0_y must both be > 0 (or both <= 0 for automatic)");
  const bool mixed = opts.precision == EGT_PRECISION_MIXED;
  if (mixed) {
    const int rc = ensure_mixed_tables(g);
    if (rc) return rc;
  }

  egt_state* st = new (std::nothrow) egt_state();
  if (!st) return fail(EGT_ENOMEM, "host allocation failed");
  std::unique_ptr<egt_state, int (*)(egt_state*)> guard(st, [](egt_state* p) {
    return egt_state_destroy(p);
  });
  st->g = g;
  st->opts = opts;
  st->tau = opts.tau0;
  st->prec = mixed ? kF32 : kF64;
  st->esz = mixed ? sizeof(float) : sizeof(double);
  const size_t bytes = (size_t)state_bytes(g, mixed);
  if (dev_mem || host_mem) {
    if (!dev_mem || !host_mem) return fail(EGT_EINVAL, "device and host state memory go together");
    st->owns_memory = false;
    st->block = dev_mem;
    st->hscal = host_mem;
  } else {
    hipError_t e = hipMalloc(&st->block, bytes);
    if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    e = hipHostMalloc((void**)&st->hscal, state_host_doubles() * sizeof(double),
                      hipHostMallocDefault);
    if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  unsigned char* cur = (unsigned char*)st->block;
  auto take = [&](size_t nbytes) {
    void* r = cur;
    cur += (nbytes + 255) / 256 * 256;
    return r;
  };
  for (int p = 0; p < 2; ++p) {
    const size_t vb = st->esz * (size_t)vec_elems(g, p);
    st->X[p] = take(vb);
    st->Xn[p] = take(vb);
    st->Xbar[p] = take(vb);
    st->Xhat[p] = take(vb);
    st->G[p] = take(vb);
    st->T1[p] = take(vb);
    st->T2[p] = take(vb);
    st->QB[p] = take(vb);
    st->Xs[p] = take(vb);
    st->Gs[p] = take(vb);
    st->Xbar2[p] = take(vb);
    st->QN[p] = take(vb);
    st->V[p] = (double*)take(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
    st->Vb[p] = (double*)take(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
    if (mixed) {
      st->X64[p] = (double*)take(sizeof(double) * (size_t)vec_elems(g, p));
      st->G64[p] = (double*)take(sizeof(double) * (size_t)vec_elems(g, p));
    }
  }
  if (!mixed) {  // FP64: the start-up scratch lives in buffers that are free then
    for (int p = 0; p < 2; ++p) {
      st->X64[p] = (double*)st->Xbar[p];
      st->G64[p] = (double*)st->Xhat[p];
    }
  }
  st->dscal = (double*)take(64 * sizeof(double));
  st->hpart = st->hscal + 64;
  st->hpart2 = st->hpart + (size_t)kMaxTrees * kMaxPartials;
  {
    void* dev = nullptr;  // device address of the pinned host scalars
    EGT_TRY(hipHostGetDevicePointer(&dev, st->hscal, 0));
    st->hpart_dev = (double*)dev + 64;
    st->hpart2_dev = st->hpart_dev + (size_t)kMaxTrees * kMaxPartials;
  }
  for (int i = 0; i < 2; ++i) EGT_TRY(hipEventCreateWithFlags(&st->ev[i], hipEventDisableTiming));
  EGT_HIP(hipMemsetAsync(st->block, 0, bytes, s));

  // x_omega and A^T x_omega with the FP64 operator: the start of Algorithms 1/3
  int rc;
  EGT_TRY(launch_uniform(g, 0, st->X64[0], s));
  EGT_TRY(launch_gradient(g, 1, st->X64[0], st->G64[1], s));
  if (auto_mu) {
    // mu0 = 1e-3 max(|A y_omega|_inf, |A^T x_omega|_inf) / max beta, then double
    // both until the excessive gap condition holds at (x0, y0).
    EGT_TRY(launch_uniform(g, 1, st->X64[1], s));
    EGT_TRY(launch_gradient(g, 0, st->X64[1], st->G64[0], s));
    EGT_TRY(launch_max_abs(vec_elems(g, 0), st->G64[0], st->dscal, s));
    EGT_TRY(launch_max_abs(vec_elems(g, 1), st->G64[1], st->dscal + 1, s));
    if ((rc = fetch(st, 2, s))) return rc;
    const double m0 = 1e-3 * std::max(st->hscal[0], st->hscal[1]) / g->max_beta;
    if (!(m0 > 0) || !std::isfinite(m0))
      return fail(EGT_ENUMERIC, "automatic mu is zero or not finite (all-zero or non-finite payoffs?)");
    st->mu[0] = st->mu[1] = m0;
  } else {
    st->mu[0] = opts.mu0_x;
    st->mu[1] = opts.mu0_y;
  }
  // A^T x_omega in the state's precision, kept in T2[1] during the mu search
  if ((rc = narrow(st, 1, st->G64[1], st->T2[1], s))) return rc;
  if (auto_mu) {
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
  for (hipEvent_t& e : st->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (st->owns_memory && (st->block || st->hscal)) {
    hipError_t e = hipDeviceSynchronize();
    if (st->block && e == hipSuccess) e = hipFree(st->block);
    if (st->hscal && e == hipSuccess) e = hipHostFree(st->hscal);
    if (e != hipSuccess) rc = hip_fail(e, "state_destroy");
  }
  delete st;
  return rc;
}

// Enqueues the saddle-gap evaluation of the current iterate (nothing when it
// is already known); gap_finish completes it.
int gap_launch(egt_state* st, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  if (st->gap_valid) return EGT_OK;
  int rc;
  Pass ps[2];
  if (st->prec == kF64) {
    gap_passes(st, st->G[0], 1.0, nullptr, 0.0, st->G[1], 1.0, nullptr, 0.0, ps);
  } else {
    // always FP64: widen the iterates, FP64 products, FP64 best responses
    if ((rc = widen(st, 0, st->X[0], st->X64[0], s))) return rc;
    if ((rc = widen(st, 1, st->X[1], st->X64[1], s))) return rc;
    EGT_TRY(launch_gradient(st->g, 0, st->X64[1], st->G64[0], s));
    EGT_TRY(launch_gradient(st->g, 1, st->X64[0], st->G64[1], s));
    gap_passes(st, st->G64[0], 1.0, nullptr, 0.0, st->G64[1], 1.0, nullptr, 0.0, ps);
  }
  EGT_TRY(launch_passes(st->g, ps, 2, nullptr, st->hpart_dev, s, kF64));
  return enqueue_values(st, 2, s);
}

int gap_finish(egt_state* st, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  if (st->gap_valid) return EGT_OK;
  int rc;
  if ((rc = finish_values(st, s))) return rc;
  st->br_min_x = st->hscal[0];
  st->br_max_y = -st->hscal[1];
  st->gap = -st->hscal[1] - st->hscal[0];
  st->gap_valid = true;
  return EGT_OK;
}

int state_gap(egt_state* st, double* gap, double* brmax, double* brmin, hipStream_t s) {
  int rc;
  if ((rc = gap_launch(st, s))) return rc;
  if ((rc = gap_finish(st, s))) return rc;
  if (gap) *gap = st->gap;
  if (brmax) *brmax = st->br_max_y;
  if (brmin) *brmin = st->br_min_x;
  return EGT_OK;
}

// The buffers one attempt reads and writes: the state's own, or those of the
// iteration after an accepted step (see Xs / Gs / Xbar2).
struct View {
  void* X[2];
  void* Xn[2];
  void* Xbar[2];
  void* G[2];
  void* T2[2];
  double* part_dev;  // where the value launch writes its partial sums
  const double* part;
};

View current_view(const egt_state* st) {
  return View{{st->X[0], st->X[1]},       {st->Xn[0], st->Xn[1]}, {st->Xbar[0], st->Xbar[1]},
              {st->G[0], st->G[1]},       {st->T2[0], st->T2[1]}, st->hpart_dev,
              st->hpart};
}

// The view the state takes once the current step is accepted.
View next_view(const egt_state* st) {
  return View{{st->Xn[0], st->Xn[1]},     {st->Xs[0], st->Xs[1]}, {st->Xbar2[0], st->Xbar2[1]},
              {st->T2[0], st->T2[1]},     {st->Gs[0], st->Gs[1]}, st->hpart2_dev,
              st->hpart2};
}

// Acceptance: x <- x_+, G <- the products at x_+ (rotating through the spares).
void accept_rotate(egt_state* st) {
  for (int q = 0; q < 2; ++q) {
    void* x = st->X[q];
    st->X[q] = st->Xn[q];
    st->Xn[q] = st->Xs[q];
    st->Xs[q] = x;
    void* gq = st->G[q];
    st->G[q] = st->T2[q];
    st->T2[q] = st->Gs[q];
    st->Gs[q] = gq;
    std::swap(st->Xbar[q], st->Xbar2[q]);
  }
  std::swap(st->hpart, st->hpart2);
  std::swap(st->hpart_dev, st->hpart2_dev);
}

void side_and_tau(const egt_state* st, int64_t t, const double mu[2], double tau_as, int* p, double* tau);

// One attempt of the step focused on p at step size tau on the buffers of v,
// with mu, as iteration t_at (the number of steps accepted before it).
// first = the iteration's first attempt (otherwise a retry with a halved
// tau).  Leaves the two EGV terms (and with with_gap the two best-response
// values of the candidate's saddle gap: dual FP64 trees in the same launch,
// or in the precision form the widened iterates through FP64 products) as
// root partials in v.part; returns the number of values.
//
// x_bar's bottom-up pass is usually already done: the EGV tree of the side
// that steps next is the bottom-up pass of exactly the smoothed best response
// that opens the next iteration (same gradient, bit for bit, since the tree
// that stores the accepted product continues with the stored values; same
// mu), so the value launch also keeps that tree's q_bar (in QN) and the next
// first attempt runs only the top-down pass on it.
static int attempt_v(egt_state* st, const View& v, int64_t t_at, int p, double tau, const double mu[2],
                     bool first, hipStream_t s, int* trees_out, bool with_gap = false) {
  const egt_game* g = st->g;
  const int o = 1 - p;
  int rc;
  // x_bar itself is needed only when the attempt fails: the first attempt
  // writes x_hat alone, a retry recomputes x_bar (the same pass on the same
  // gradient and mu, so bit for bit the same) and combines it with the new tau
  if (first) {
    if (st->qn_side == p && st->qn_grad == v.G[p] && st->qn_mu == mu[p]) {
      EGT_TRY(launch_top_down(g, p, st->QN[p], nullptr, v.X[p], tau, st->Xhat[p], s, st->prec));
    } else if ((rc = sbr(st, p, v.G[p], kSg[p], nullptr, 0.0, mu[p], nullptr, v.X[p], tau, st->Xhat[p], s))) {
      return rc;
    }
  } else {
    if ((rc = sbr(st, p, v.G[p], kSg[p], nullptr, 0.0, mu[p], v.Xbar[p], nullptr, 0.0, nullptr, s))) return rc;
    if ((rc = axpby(st, p, 1.0 - tau, v.X[p], tau, v.Xbar[p], st->Xhat[p], s))) return rc;
  }
  if ((rc = grad(st, o, st->Xhat[p], st->T1[o], s))) return rc;
  if ((rc = sbr(st, o, st->T1[o], kSg[o], nullptr, 0.0, mu[o], v.Xbar[o], v.X[o], tau, v.Xn[o], s))) return rc;
  if ((rc = grad(st, p, v.Xbar[o], st->T1[p], s))) return rc;
  const double r = tau / (1.0 - tau);
  if ((rc = sbr(st, p, v.G[p], kSg[p], st->T1[p], kSg[p] * r, mu[p], nullptr, v.X[p], tau, v.Xn[p], s))) return rc;
  if ((rc = grad(st, o, v.Xn[p], v.T2[o], s))) return rc;
  const bool fresh = st->opts.fresh_products != 0;
  if (fresh && (rc = grad(st, p, v.Xn[o], v.T2[p], s))) return rc;  // p's gradient at y_+, recomputed
  const double mu_new = (1.0 - tau) * mu[p];
  // one launch for the value passes: EGV at (x_+, y_+) with mu_p+ and the
  // unchanged mu_o, and (FP64) the two best responses of the candidate's gap
  Pass ps[2];
  if (fresh)
    ps[0] = Pass{p, v.T2[p], kSg[p], nullptr, 0.0, mu_new, st->V[p], nullptr};
  else
    ps[0] = Pass{p, v.G[p], kSg[p] * (1.0 - tau), st->T1[p], kSg[p] * tau, mu_new, st->V[p], nullptr};
  ps[1] = Pass{o, v.T2[o], kSg[o], nullptr, 0.0, mu[o], st->V[o], nullptr};
  int trees = 2;
  if (st->prec == kF64 && with_gap) {
    // the two trees are dual: each also takes the best response to its own
    // gradient (the products at (x_+, y_+)), values 2 (p) and 3 (o)
    ps[0].VB = st->Vb[p];
    ps[1].VB = st->Vb[o];
    trees = 4;
  }
  // without fresh products the value launch also writes the accepted product
  // (1-tau) G[p] + tau T1[p] of tree 0 into T2[p], so accepting the step is a
  // rotation of buffers either way
  Epilogue epi[2] = {};
  if (!fresh) {
    epi[0].g_out = v.T2[p];
    epi[0].g_scale = kSg[p];
  }
  // the side of the iteration after this one if it is accepted: its EGV tree
  // keeps q_bar for that iteration's first smoothed best response (the
  // gradient it reads then is T2 of that side: kSg * (kSg * g~) = g~ exactly)
  {
    double mu_n[2] = {mu[0], mu[1]}, tau_n;
    mu_n[p] = mu_new;
    int pn;
    side_and_tau(st, t_at + 1, mu_n, tau, &pn, &tau_n);
    ps[pn == p ? 0 : 1].QB = st->QN[pn];     // level path
    epi[pn == p ? 0 : 1].qb_out = st->QN[pn];  // single-launch path
    st->qn_side = pn;
    st->qn_grad = v.T2[pn];
    st->qn_mu = mu_n[pn];
  }
  EGT_TRY(launch_passes(g, ps, 2, epi, v.part_dev, s, st->prec));
  if (with_gap && st->prec == kF32) {
    // precision form: the candidate's saddle gap in FP64 (widened iterates,
    // FP64 products, FP64 best responses) as values 2 and 3
    if ((rc = widen(st, 0, v.Xn[0], st->X64[0], s))) return rc;
    if ((rc = widen(st, 1, v.Xn[1], st->X64[1], s))) return rc;
    EGT_TRY(launch_gradient(g, 0, st->X64[1], st->G64[0], s));
    EGT_TRY(launch_gradient(g, 1, st->X64[0], st->G64[1], s));
    Pass gp[2];
    gap_passes(st, st->G64[0], 1.0, nullptr, 0.0, st->G64[1], 1.0, nullptr, 0.0, gp);
    EGT_TRY(launch_passes(g, gp, 2, nullptr, v.part_dev + 2 * (size_t)n_partials(g), s, kF64));
    trees = 4;
  }
  *trees_out = trees;
  return EGT_OK;
}

int products_per_attempt(const egt_state* st) { return st->opts.fresh_products ? 4 : 3; }

// The saddle gap an accepted attempt focused on p carried (values 2 and 3 of
// its value launch): in FP64 the dual trees' best responses of p and of the
// other player, in the precision form those of players 1 and 2 in order.
void take_gap(egt_state* st, int p) {
  const int i0 = (st->prec == kF64 && p == 1) ? 3 : 2;  // player 1's best response
  const int i1 = 5 - i0;
  st->br_min_x = st->hscal[i0];
  st->br_max_y = -st->hscal[i1];
  st->gap = -st->hscal[i1] - st->hscal[i0];
  st->gap_valid = true;
}

// Side and step size of an iteration after t accepted steps (the variant's
// rule: alternate with 2 / (t + 3), the larger mu with 2 / (t + 3), or the
// larger mu with the shared EGT/as tau).
void side_and_tau(const egt_state* st, int64_t t, const double mu[2], double tau_as, int* p, double* tau) {
  const int variant = st->opts.variant;
  if (variant == EGT_VARIANT_ALT) {
    *tau = 2.0 / ((double)t + 3.0);
    *p = (t % 2 == 0) ? 0 : 1;
  } else if (variant == EGT_VARIANT_BAL) {
    *tau = 2.0 / ((double)t + 3.0);
    *p = mu[0] > mu[1] ? 0 : 1;
  } else {
    *tau = tau_as;
    *p = mu[0] > mu[1] ? 0 : 1;
  }
}

// Enqueues the next attempt of the current iteration, opening one (side and
// tau from the variant, or `player`) if none is open; step_finish completes it.
int step_launch(egt_state* st, int player, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  if (player < -1 || player > 1) return fail(EGT_EINVAL, "player must be -1, 0 or 1");
  bool first = false;
  if (!st->step_open) {
    int p;
    double tau;
    side_and_tau(st, st->t, st->mu, st->tau, &p, &tau);
    if (player >= 0) p = player;
    st->step_open = true;
    st->step_p = p;
    st->step_tau = tau;
    first = true;
  }
  int rc, trees = 0;
  if ((rc = attempt_v(st, current_view(st), st->t, st->step_p, st->step_tau, st->mu, first, s, &trees,
                       st->prec == kF64)))
    return rc;
  st->products += products_per_attempt(st);
  return enqueue_values(st, trees, s, st->hpart);
}

// Waits for the enqueued attempt.  EGT/as with EGV < 0: tau halves and
// *accepted = 0 (launch again).  Otherwise the step is accepted.
int step_finish(egt_state* st, hipStream_t s, int* accepted, double* egv_out, int* stepped) {
  if (!st || !st->step_open) return fail(EGT_EINVAL, "no step in progress");
  const int trees = st->pending_trees;
  int rc;
  if ((rc = finish_values(st, s))) return rc;
  const double egv = st->hscal[0] + st->hscal[1];
  const int p = st->step_p;
  double tau = st->step_tau;
  if (st->opts.variant == EGT_VARIANT_AS && egv < 0.0) {
    tau *= 0.5;
    st->backtracks++;
    if (tau < kTauFloor) return fail(EGT_ENOTCONV, "tau fell below 1e-30 in the EGT/as backtracking");
    st->step_tau = tau;
    *accepted = 0;
    return EGT_OK;
  }
  // accept: G[p] <- (1-tau) G[p] + tau T1[p] (linearity; written by the value
  // launch into T2[p]), G[o] <- T2[o], x <- x_+
  accept_rotate(st);
  st->mu[p] *= (1.0 - tau);
  if (st->opts.variant == EGT_VARIANT_AS) st->tau = tau;
  st->t++;
  if (trees == 4)
    take_gap(st, p);
  else
    st->gap_valid = false;
  st->last_egv = egv;
  st->step_open = false;
  *accepted = 1;
  if (egv_out) *egv_out = egv;
  if (stepped) *stepped = p;
  return EGT_OK;
}

int state_step(egt_state* st, int player, double* egv_out, int* stepped, hipStream_t s) {
  if (!st) return fail(EGT_EINVAL, "null state");
  if (st->step_open) return fail(EGT_EINVAL, "a split step is in progress");
  int rc, accepted = 0;
  while (!accepted) {
    if ((rc = step_launch(st, player, s))) return rc;
    if ((rc = step_finish(st, s, &accepted, egv_out, stepped))) {
      st->step_open = false;
      return rc;
    }
  }
  return EGT_OK;
}

int state_get(const egt_state* cst, double* x, double* y, double* mu_x, double* mu_y, double* tau, int64_t* iters,
              hipStream_t s) {
  if (!cst) return fail(EGT_EINVAL, "null state");
  egt_state* st = const_cast<egt_state*>(cst);
  int rc;
  if (x && (rc = widen(st, 0, st->X[0], x, s))) return rc;
  if (y && (rc = widen(st, 1, st->X[1], y, s))) return rc;
  if (mu_x) *mu_x = st->mu[0];
  if (mu_y) *mu_y = st->mu[1];
  if (tau) *tau = st->tau;
  if (iters) *iters = st->t;
  return EGT_OK;
}

int state_get_products(const egt_state* cst, double* ay, double* atx, hipStream_t s) {
  if (!cst) return fail(EGT_EINVAL, "null state");
  egt_state* st = const_cast<egt_state*>(cst);
  int rc;
  if (ay && (rc = widen(st, 0, st->G[0], ay, s))) return rc;
  if (atx && (rc = widen(st, 1, st->G[1], atx, s))) return rc;
  return EGT_OK;
}

int state_set(egt_state* st, const double* x, const double* y, double mu_x, double mu_y, double tau, int64_t iters,
              const double* ay, const double* atx, hipStream_t s) {
  if (!st || !x || !y) return fail(EGT_EINVAL, "null argument");
  if (!(mu_x > 0) || !(mu_y > 0) || !std::isfinite(mu_x) || !std::isfinite(mu_y))
    return fail(EGT_EINVAL, "mu must be finite and > 0");
  if (!(tau > 0) || !(tau < 1)) return fail(EGT_EINVAL, "tau must lie in (0, 1)");
  if (iters < 0) return fail(EGT_EINVAL, "iters < 0");
  st->qn_side = -1;  // G changes: no kept q_bar matches it
  int rc;
  if ((rc = narrow(st, 0, x, st->X[0], s))) return rc;
  if ((rc = narrow(st, 1, y, st->X[1], s))) return rc;
  if (ay) {
    if ((rc = narrow(st, 0, ay, st->G[0], s))) return rc;
  } else if ((rc = grad(st, 0, st->X[1], st->G[0], s))) {
    return rc;
  }
  if (atx) {
    if ((rc = narrow(st, 1, atx, st->G[1], s))) return rc;
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

// Fills the scalar result of a finished run (value from FP64 copies of x and
// A y: the precision form's last gap evaluation left them in X64 / G64).
int fill_result(egt_state* st, bool converged, double seconds, egt_result* res, hipStream_t s) {
  std::memset(res, 0, sizeof(*res));
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
  res->seconds = seconds;
  const int64_t n0 = vec_elems(st->g, 0);
  double* hx = (double*)std::malloc(sizeof(double) * n0 * 2);
  if (!hx) return fail(EGT_ENOMEM, "host allocation failed");
  const double* dx = st->prec == kF64 ? (const double*)st->X[0] : st->X64[0];
  const double* dg = st->prec == kF64 ? (const double*)st->G[0] : st->G64[0];
  hipError_t e = hipMemcpyAsync(hx, dx, sizeof(double) * n0, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hx + n0, dg, sizeof(double) * n0, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    std::free(hx);
    return hip_fail(e, "copy of the final iterate");
  }
  double v = 0.0;  // x^T A y = <x, A y>
  for (int64_t i = 0; i < n0; ++i) v += hx[i] * hx[n0 + i];
  res->value_p1 = -v;
  std::free(hx);
  return EGT_OK;
}

// The iteration of egt_solve, pipelined: while the host waits for the values
// of the current attempt, the device already runs the next iteration as if
// the attempt were accepted (on the rotated buffers of next_view, which leave
// x, G and x_bar of the current step untouched).  On acceptance that work is
// the next iteration; on an EGT/as rejection it is discarded and the retry is
// enqueued behind it.  The saddle gap of the iterates the loop tests (every
// gap_every-th and the last) comes with the attempt that produces them: the
// FP64 value launch always carries it, the precision form adds its FP64 gap
// evaluation to that attempt, which is then not run ahead (its FP64 copies of
// x and A y must survive a converged stop).  Every committed attempt is
// computed exactly as by state_step, so the results are bitwise those of
// stepping with a gap test before every gap_every-th iteration.
int solve_loop_pipelined(egt_state* st, hipStream_t s, const std::atomic<bool>* stop, bool* converged) {
  const egt_solve_opts& op = st->opts;
  const bool mixed = st->prec == kF32;
  auto gap_due = [&](int64_t t) { return t % op.gap_every == 0 || t >= op.max_iters; };
  *converged = false;
  int rc = EGT_OK;
  if (gap_due(st->t)) {
    if (!st->gap_valid && (rc = state_gap(st, nullptr, nullptr, nullptr, s))) return rc;
    if (st->gap <= op.eps) {
      *converged = true;
      return EGT_OK;
    }
  }
  if (st->t >= op.max_iters || (stop && stop->load(std::memory_order_relaxed))) {
    if (!st->gap_valid) rc = state_gap(st, nullptr, nullptr, nullptr, s);
    return rc;
  }
  int p, trees = 0, cur = 0;
  double tau;
  side_and_tau(st, st->t, st->mu, st->tau, &p, &tau);
  bool wg = gap_due(st->t + 1);
  if ((rc = attempt_v(st, current_view(st), st->t, p, tau, st->mu, true, s, &trees, wg))) return rc;
  EGT_TRY(hipEventRecord(st->ev[cur], s));
  for (;;) {
    // the next iteration, assuming acceptance
    bool spec = false;
    int p2 = 0, t2 = 0;
    double tau2 = 0.0;
    if (st->t + 1 < op.max_iters && !(stop && stop->load(std::memory_order_relaxed)) && !(mixed && gap_due(st->t + 2))) {
      double mu2[2] = {st->mu[0], st->mu[1]};
      mu2[p] *= (1.0 - tau);
      side_and_tau(st, st->t + 1, mu2, op.variant == EGT_VARIANT_AS ? tau : st->tau, &p2, &tau2);
      if ((rc = attempt_v(st, next_view(st), st->t + 1, p2, tau2, mu2, true, s, &t2, gap_due(st->t + 2)))) return rc;
      EGT_TRY(hipEventRecord(st->ev[1 - cur], s));
      spec = true;
    }
    // decide the current attempt
    hipEvent_t ev = st->ev[cur];
    if ((rc = wait_for([&] { return hipEventQuery(ev); }, [&] { return hipEventSynchronize(ev); }))) return rc;
    st->pending_trees = trees;
    st->pending_part = st->hpart;
    if ((rc = read_values(st))) return rc;
    st->products += products_per_attempt(st);
    const double egv = st->hscal[0] + st->hscal[1];
    if (op.variant == EGT_VARIANT_AS && egv < 0.0) {
      tau *= 0.5;
      st->backtracks++;
      if (tau < kTauFloor) return fail(EGT_ENOTCONV, "tau fell below 1e-30 in the EGT/as backtracking");
      // retry from x_hat with the halved tau, behind the discarded iteration
      if ((rc = attempt_v(st, current_view(st), st->t, p, tau, st->mu, false, s, &trees, wg))) return rc;
      EGT_TRY(hipEventRecord(st->ev[cur], s));
      continue;
    }
    accept_rotate(st);
    st->mu[p] *= (1.0 - tau);
    if (op.variant == EGT_VARIANT_AS) st->tau = tau;
    st->t++;
    if (trees == 4)
      take_gap(st, p);
    else
      st->gap_valid = false;
    st->last_egv = egv;
    if (gap_due(st->t) && st->gap_valid && st->gap <= op.eps) {
      *converged = true;
      return EGT_OK;
    }
    if (st->t >= op.max_iters || (stop && stop->load(std::memory_order_relaxed))) {
      if (!st->gap_valid) rc = state_gap(st, nullptr, nullptr, nullptr, s);
      return rc;
    }
    cur = 1 - cur;
    wg = gap_due(st->t + 1);  // (a speculated attempt ran only where the precision form tests no gap)
    if (spec) {
      p = p2;
      tau = tau2;
      trees = t2;
    } else {
      side_and_tau(st, st->t, st->mu, st->tau, &p, &tau);
      if ((rc = attempt_v(st, current_view(st), st->t, p, tau, st->mu, true, s, &trees, wg))) return rc;
      EGT_TRY(hipEventRecord(st->ev[cur], s));
    }
  }
}

// The iteration of egt_solve: gap test before every gap_every-th iteration,
// stop at gap <= eps or max_iters (or when *stop becomes true).
int solve_loop(egt_state* st, hipStream_t s, const std::atomic<bool>* stop, bool* converged) {
  if (st->step_open) return fail(EGT_EINVAL, "a split step is in progress");
  return solve_loop_pipelined(st, s, stop, converged);
}

int solve(const egt_game* g, const egt_solve_opts* o, egt_result* res, egt_state** state_out, hipStream_t s) {
  if (!g || !res) return fail(EGT_EINVAL, "null argument");
  std::memset(res, 0, sizeof(*res));
  const auto t0 = std::chrono::steady_clock::now();
  egt_state* st = nullptr;
  int rc = state_create(g, o, s, &st);
  if (rc) return rc;
  bool converged = false;
  rc = solve_loop(st, s, nullptr, &converged);
  const auto t1 = std::chrono::steady_clock::now();
  if (rc == EGT_OK) rc = fill_result(st, converged, std::chrono::duration<double>(t1 - t0).count(), res, s);
  if (rc == EGT_OK && !converged) rc = fail(EGT_ENOTCONV, "iteration cap reached before the target gap");
  if (state_out && (rc == EGT_OK || rc == EGT_ENOTCONV)) {
    *state_out = st;
  } else {
    state_destroy(st);
  }
  return rc;
}

// Bytes of device memory a state of this game and precision allocates.
int64_t state_bytes(const egt_game* g, bool mixed) {
  const size_t esz = mixed ? sizeof(float) : sizeof(double);
  size_t bytes = 0;
  for (int p = 0; p < 2; ++p) {
    bytes += esz * 11 * (size_t)vec_elems(g, p) + sizeof(double) * 2 * (size_t)g->hp[p].n_nodes * g->ld;
    if (mixed) bytes += sizeof(double) * 2 * (size_t)vec_elems(g, p);
    bytes += esz * (size_t)vec_elems(g, p);  // QN
    bytes += 16 * 256;
  }
  bytes += 64 * sizeof(double) + 256;
  return (int64_t)bytes;
}

// Pinned host doubles of a state: 64 scalars, then two buffers of root partial sums.
size_t state_host_doubles() { return 64 + 2 * (size_t)kMaxTrees * kMaxPartials; }

// Accessors for the batch engine.
const egt_solve_opts& state_opts(const egt_state* st) { return st->opts; }
int64_t state_iters(const egt_state* st) { return st->t; }
bool state_gap_known(const egt_state* st) { return st->gap_valid; }
double state_gap_value(const egt_state* st) { return st->gap; }

}  // namespace egt
