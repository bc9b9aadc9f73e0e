// Mirror prox and Chambolle-Pock with the dilated entropy, the first-order
// methods Section 8 names as likely faster than EGT, on the same kernels:
// the payoff products and the smoothed best response.
//
// Both take Bregman prox steps of the dilated entropy from a centre c,
// argmin_q <g, q> + D(q, c).  Every centre here is itself a smoothed best
// response with weight 1, c = SBR(h, 1), and then the prox is SBR(h + g, 1)
// (grad d(c) = -h up to a constant per simplex, which leaves the argmin
// unchanged; the same shift-free form EGT's prox step uses).  So each player
// keeps the gradient sum h of its centre, starting from h = 0 (the uniform
// point, the DGF's minimiser):
//   mirror prox, steps eta_x, eta_y:
//     x^ = SBR(h_x + eta_x A y, 1),         y^ = SBR(h_y - eta_y A^T x, 1),
//     h_x += eta_x A y^, x = SBR(h_x, 1),   h_y -= eta_y A^T x^, y = SBR(h_y, 1),
//     averages of x^, y^ (4 products per iteration);
//   Chambolle-Pock, steps tau (x) and sigma (y):
//     h_x += tau A y, x' = SBR(h_x, 1),
//     h_y -= sigma A^T (2 x' - x), y' = SBR(h_y, 1),
//     averages of x', y' (2 products per iteration).
// The new h and the new strategy come out of one smoothed-best-response
// launch (its epilogue writes the combined gradient back).  The averages are
// kept as sums and divided by the iteration count when read.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "egt_internal.h"

namespace egt {
int64_t vec_elems_of(const egt_game* g, int p);
}

struct egt_fom {
  const egt_game* g = nullptr;
  int method = EGT_FOM_MIRROR_PROX;
  double step[2] = {0, 0};
  int64_t t = 0;
  int64_t products = 0;
  double* H[2] = {};    // gradient sums of the centres
  double* X[2] = {};    // current strategies
  double* Xh[2] = {};   // mirror prox: extrapolated points; Chambolle-Pock: 2 x' - x
  double* S[2] = {};    // sums of the averaged points
  double* G[2] = {};    // products
  double* QB[2] = {};   // q_bar scratch of the level path
  double* V[2] = {};    // node values
  double* part = nullptr;
  double* scal = nullptr;
  double* hscal = nullptr;
  void* block = nullptr;
};

using namespace egt;

namespace {

// q = SBR(cA gA + cB gB, 1) of player p into q_out; when g_out is set, the
// combined gradient is written there too (it may be gA itself).
int prox(egt_fom* f, int p, const double* gA, double cA, const double* gB, double cB, double* q_out, double* g_out,
         hipStream_t s) {
  const Pass ps{p, gA, cA, gB, cB, 1.0, f->V[p], f->QB[p]};
  Epilogue e{q_out, nullptr, 0.0, nullptr, g_out, 1.0};
  EGT_HIP(launch_passes(f->g, &ps, 1, &e, nullptr, s));
  return EGT_OK;
}

int accumulate(egt_fom* f, const double* const src[2], hipStream_t s) {
  for (int p = 0; p < 2; ++p)
    EGT_HIP(launch_axpby(vec_elems_of(f->g, p), 1.0, f->S[p], 1.0, src[p], f->S[p], s));
  return EGT_OK;
}

int fom_iteration(egt_fom* f, hipStream_t s) {
  const egt_game* g = f->g;
  int rc;
  if (f->method == EGT_FOM_MIRROR_PROX) {
    EGT_HIP(launch_gradient(g, 0, f->X[1], f->G[0], s));
    EGT_HIP(launch_gradient(g, 1, f->X[0], f->G[1], s));
    if ((rc = prox(f, 0, f->H[0], 1.0, f->G[0], f->step[0], f->Xh[0], nullptr, s))) return rc;
    if ((rc = prox(f, 1, f->H[1], 1.0, f->G[1], -f->step[1], f->Xh[1], nullptr, s))) return rc;
    EGT_HIP(launch_gradient(g, 0, f->Xh[1], f->G[0], s));
    EGT_HIP(launch_gradient(g, 1, f->Xh[0], f->G[1], s));
    if ((rc = prox(f, 0, f->H[0], 1.0, f->G[0], f->step[0], f->X[0], f->H[0], s))) return rc;
    if ((rc = prox(f, 1, f->H[1], 1.0, f->G[1], -f->step[1], f->X[1], f->H[1], s))) return rc;
    const double* src[2] = {f->Xh[0], f->Xh[1]};
    if ((rc = accumulate(f, src, s))) return rc;
    f->products += 4;
  } else {
    EGT_HIP(launch_gradient(g, 0, f->X[1], f->G[0], s));
    // x' into Xh[0] first: 2 x' - x needs the old x
    if ((rc = prox(f, 0, f->H[0], 1.0, f->G[0], f->step[0], f->Xh[0], f->H[0], s))) return rc;
    EGT_HIP(launch_axpby(vec_elems_of(g, 0), 2.0, f->Xh[0], -1.0, f->X[0], f->X[0], s));  // 2 x' - x
    EGT_HIP(launch_gradient(g, 1, f->X[0], f->G[1], s));
    std::swap(f->X[0], f->Xh[0]);  // X[0] = x'
    if ((rc = prox(f, 1, f->H[1], 1.0, f->G[1], -f->step[1], f->X[1], f->H[1], s))) return rc;
    const double* src[2] = {f->X[0], f->X[1]};
    if ((rc = accumulate(f, src, s))) return rc;
    f->products += 2;
  }
  f->t++;
  return EGT_OK;
}

// out = S / t (the averages); with t = 0 the current strategies.
int averages(const egt_fom* f, double* out0, double* out1, hipStream_t s) {
  double* out[2] = {out0, out1};
  for (int p = 0; p < 2; ++p) {
    if (!out[p]) continue;
    if (f->t == 0)
      EGT_HIP(hipMemcpyAsync(out[p], f->X[p], sizeof(double) * (size_t)vec_elems_of(f->g, p),
                             hipMemcpyDeviceToDevice, s));
    else
      EGT_HIP(launch_axpby(vec_elems_of(f->g, p), 1.0 / (double)f->t, f->S[p], 0.0, nullptr, out[p], s));
  }
  return EGT_OK;
}

}  // namespace

extern "C" {

int egt_fom_create(const egt_game* g, int32_t method, double step_x, double step_y, hipStream_t s, egt_fom** out) {
  if (!g || !out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  if (method != EGT_FOM_MIRROR_PROX && method != EGT_FOM_CHAMBOLLE_POCK)
    return fail(EGT_EINVAL, "unknown first-order method");
  if (!(step_x > 0) || !(step_y > 0) || !std::isfinite(step_x) || !std::isfinite(step_y))
    return fail(EGT_EINVAL, "steps must be finite and > 0");
  std::unique_ptr<egt_fom> f(new (std::nothrow) egt_fom());
  if (!f) return fail(EGT_ENOMEM, "host allocation failed");
  f->g = g;
  f->method = method;
  f->step[0] = step_x;
  f->step[1] = step_y;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t bytes = 0;
  for (int p = 0; p < 2; ++p) {
    bytes += 6 * al(sizeof(double) * (size_t)vec_elems_of(g, p));
    bytes += al(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
  }
  bytes += al(sizeof(double) * 2 * kMaxPartials) + al(2 * sizeof(double));
  hipError_t e = hipMalloc(&f->block, bytes);
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc (first-order method): ") + hipGetErrorString(e));
  e = hipHostMalloc((void**)&f->hscal, 2 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(f->block);
    return fail(EGT_ENOMEM, std::string("hipHostMalloc (first-order method): ") + hipGetErrorString(e));
  }
  unsigned char* cur = (unsigned char*)f->block;
  auto take = [&](size_t nb) {
    void* r = cur;
    cur += al(nb);
    return (double*)r;
  };
  for (int p = 0; p < 2; ++p) {
    const size_t vb = sizeof(double) * (size_t)vec_elems_of(g, p);
    f->H[p] = take(vb);
    f->X[p] = take(vb);
    f->Xh[p] = take(vb);
    f->S[p] = take(vb);
    f->G[p] = take(vb);
    f->QB[p] = take(vb);
    f->V[p] = take(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
  }
  f->part = take(sizeof(double) * 2 * kMaxPartials);
  f->scal = take(2 * sizeof(double));
  // h = 0, x = the uniform point, sums = 0
  for (int p = 0; p < 2; ++p) {
    const int64_t cnt = vec_elems_of(g, p);
    EGT_HIP(launch_uniform(g, p, f->X[p], s));
    EGT_HIP(launch_axpby(cnt, 0.0, f->X[p], 0.0, nullptr, f->H[p], s));  // 0 * (finite uniform point)
    EGT_HIP(launch_axpby(cnt, 0.0, f->X[p], 0.0, nullptr, f->S[p], s));
  }
  EGT_HIP(hipStreamSynchronize(s));
  *out = f.release();
  return EGT_OK;
}

int egt_fom_destroy(egt_fom* f) {
  if (!f) return EGT_OK;
  int rc = EGT_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && f->block) e = hipFree(f->block);
  if (e == hipSuccess && f->hscal) e = hipHostFree(f->hscal);
  if (e != hipSuccess) rc = hip_fail(e, "egt_fom_destroy");
  delete f;
  return rc;
}

int egt_fom_step(egt_fom* f, int32_t iters, hipStream_t s) {
  if (!f || iters < 0) return fail(EGT_EINVAL, "null state or negative count");
  for (int32_t k = 0; k < iters; ++k) {
    const int rc = fom_iteration(f, s);
    if (rc) return rc;
  }
  return EGT_OK;
}

int egt_fom_get(const egt_fom* f, double* x_avg, double* y_avg, double* x_cur, double* y_cur, int64_t* iters,
                int64_t* products, hipStream_t s) {
  if (!f) return fail(EGT_EINVAL, "null state");
  int rc = averages(f, x_avg, y_avg, s);
  if (rc) return rc;
  double* cur[2] = {x_cur, y_cur};
  for (int p = 0; p < 2; ++p)
    if (cur[p])
      EGT_HIP(hipMemcpyAsync(cur[p], f->X[p], sizeof(double) * (size_t)vec_elems_of(f->g, p),
                             hipMemcpyDeviceToDevice, s));
  if (iters) *iters = f->t;
  if (products) *products = f->products;
  return EGT_OK;
}

int egt_fom_gap(egt_fom* f, double* gap, double* br_max_y, double* br_min_x, hipStream_t s) {
  if (!f) return fail(EGT_EINVAL, "null state");
  const egt_game* g = f->g;
  // the averages into the scratch of the extrapolated points (free between iterations)
  int rc = averages(f, f->Xh[0], f->Xh[1], s);
  if (rc) return rc;
  EGT_HIP(launch_gradient(g, 0, f->Xh[1], f->G[0], s));
  EGT_HIP(launch_gradient(g, 1, f->Xh[0], f->G[1], s));
  const Pass ps[2] = {{0, f->G[0], 1.0, nullptr, 0.0, 0.0, f->V[0], nullptr},
                      {1, f->G[1], -1.0, nullptr, 0.0, 0.0, f->V[1], nullptr}};
  EGT_HIP(launch_passes(g, ps, 2, nullptr, f->part, s));
  EGT_HIP(launch_sum_partials(g, f->part, 2, f->scal, s));
  EGT_HIP(hipMemcpyAsync(f->hscal, f->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  EGT_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(f->hscal[0]) || !std::isfinite(f->hscal[1]))
    return fail(EGT_ENUMERIC, "non-finite value in the saddle gap");
  if (gap) *gap = -f->hscal[1] - f->hscal[0];
  if (br_max_y) *br_max_y = -f->hscal[1];
  if (br_min_x) *br_min_x = f->hscal[0];
  return EGT_OK;
}

}  // extern "C"
