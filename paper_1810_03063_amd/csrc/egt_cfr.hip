// Counterfactual regret minimisation on the same payoff kernels: CFR with
// regret matching, CFR with regret matching+ and CFR+, the regret-based
// methods Section 7 compares EGT with (two gradient computations per
// iteration).
//
// Per player p and iteration, on p's loss gradient g (A y for player 1,
// -A^T x for player 2, computed by the product kernels):
//   bottom-up over the treeplex, one launch per level, one lane per
//   information set (node v, hand h) and its actions in order:
//     g~_a  = g[v, a] + sum of the values of a's child sets (betting order),
//     V[v]  = sum_a q_bar_a g~_a            (q_bar the current local strategy),
//     r_a   = V[v] - g~_a, or 0 within 1e-12 of |V[v]| + |g~_a| + S, S the
//             largest |g| entry (an exact tie, or actions no opponent mass
//             reaches, whose sign the products' rounding would otherwise
//             decide),
//     R_a  <- R_a + r_a                     (regret matching+: then max(R_a, 0)),
//     q_bar_a = max(R_a, 0) / sum_a' max(R_a', 0), or 1 / n_v when no R_a is positive;
//   top-down, x[s] = x[parent] q_bar[s] (the pass the smoothed best response uses).
// Both players update against the strategies of the same iteration (CFR,
// CFR(RM+)), or player 2 against player 1's new strategy (CFR+).  Before the
// update the current strategies join the averages, avg <- (1 - tau) avg +
// tau x_t with tau = w_t / sum_{t' <= t} w_t' (w_t = 1, or t under CFR+); the
// saddle gap of the averages is evaluated with the FP64 products and
// best-response passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "egt_internal.h"

namespace egt {

namespace {

constexpr int kLanes = 64;

struct RegretArgs {
  const void* tab;  // the player's table image (FusedTabLayout)
  int n_nodes, n_seq;
  int node0;        // first node of the level
  int n, ld;
  const double* g;  // p's gradient (times gsign)
  double gsign;
  double* V;        // node values by value slot
  double* R;        // cumulative regrets [n_seq][ld]
  double* QB;       // local strategy [n_seq][ld], read then overwritten
  const double* gscale;  // max |g| over the real hands (device scalar)
  int plus;         // regret matching+
};

// S = max |g| over p's gradient (real hands only) into *out, which holds 0.0
// beforehand; |g| >= 0, so the bit patterns order as the values do.
__global__ __launch_bounds__(256) void absmax_kernel(const double* g, int64_t count, int n, int ld,
                                                     unsigned long long* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    if ((int)(i % ld) < n) m = fmax(m, fabs(g[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  __shared__ double wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ __launch_bounds__(kLanes) void regret_level_kernel(RegretArgs a) {
  const int h = blockIdx.x * kLanes + threadIdx.x;
  if (h >= a.n) return;
  const int v = a.node0 + (int)blockIdx.y;
  const size_t ld = a.ld;
  const FusedTabLayout L = fused_tab_layout(a.n_nodes, a.n_seq);
  const unsigned char* tab = (const unsigned char*)a.tab;
  const int4 r = ((const int4*)(tab + L.rec))[v];
  const int* cbeg = (const int*)(tab + L.cbeg);
  const int s0 = r.x, na = r.y;
  double gt[kMaxActions];
  double val = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j) {
    if (j < na) {
      const size_t idx = (size_t)(s0 + j) * ld + h;
      double x = a.gsign * a.g[idx];
      const int c1 = cbeg[s0 + j + 1];
      for (int c = cbeg[s0 + j]; c < c1; ++c) x += a.V[(size_t)c * ld + h];
      gt[j] = x;
      val += a.QB[idx] * x;
    }
  }
  a.V[(size_t)r.z * ld + h] = val;
  const double S = *a.gscale;
  double pos[kMaxActions];
  double tot = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j) {
    if (j < na) {
      const size_t idx = (size_t)(s0 + j) * ld + h;
      double r = val - gt[j];
      if (fabs(r) <= 1e-12 * (fabs(val) + fabs(gt[j]) + S)) r = 0.0;  // an exact tie
      double R = a.R[idx] + r;
      if (a.plus) R = fmax(R, 0.0);
      a.R[idx] = R;
      pos[j] = fmax(R, 0.0);
      tot += pos[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j)
    if (j < na) a.QB[(size_t)(s0 + j) * ld + h] = tot > 0.0 ? pos[j] / tot : 1.0 / (double)na;
}

// Uniform local strategy: q_bar = 1 / n_v on every action (0 in the padding).
__global__ __launch_bounds__(kLanes) void uniform_local_kernel(const int* seq_nact, int n, int ld, double* QB) {
  const int h = blockIdx.x * kLanes + threadIdx.x;
  if (h >= ld) return;
  const int s = blockIdx.y;
  QB[(size_t)s * ld + h] = h < n ? 1.0 / (double)seq_nact[s] : 0.0;
}

__global__ __launch_bounds__(256) void fill_kernel(double* p, int64_t count, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

}  // namespace

int64_t vec_elems_of(const egt_game* g, int p) { return (int64_t)g->hp[p].n_seq * g->ld; }

}  // namespace egt

struct egt_cfr {
  const egt_game* g = nullptr;
  int variant = EGT_CFR_PLUS;
  int64_t t = 0;
  double wsum = 0.0;
  double* R[2] = {};
  double* QB[2] = {};
  double* X[2] = {};    // current strategies x_t, y_t
  double* AVG[2] = {};  // averages
  double* G[2] = {};    // gradient scratch
  double* V[2] = {};    // node values
  double* Vb[2] = {};   // node values of the gap's best responses
  double* part = nullptr;    // device partial sums [2][kMaxPartials]
  double* scal = nullptr;    // device sums [2]
  double* gmax = nullptr;    // device max |g| [2]
  double* hscal = nullptr;   // pinned host copy
  void* block = nullptr;
};

using namespace egt;

namespace {

int cfr_update(egt_cfr* c, int p, hipStream_t s) {
  const egt_game* g = c->g;
  const HostPlayer& hp = g->hp[p];
  const unsigned bx = (unsigned)((g->n + kLanes - 1) / kLanes);
  RegretArgs a;
  a.tab = g->dp[p].fused_tab;
  a.n_nodes = hp.n_nodes;
  a.n_seq = hp.n_seq;
  a.n = g->n;
  a.ld = g->ld;
  a.g = c->G[p];
  a.gsign = p == 0 ? 1.0 : -1.0;
  a.V = c->V[p];
  a.R = c->R[p];
  a.QB = c->QB[p];
  a.plus = c->variant != EGT_CFR_RM;
  a.gscale = c->gmax + p;
  {
    const int64_t cnt = vec_elems_of(g, p);
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, c->gmax + p, (int64_t)1, 0.0);
    const unsigned fb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cnt + 255) / 256, 2048));
    hipLaunchKernelGGL(absmax_kernel, dim3(fb), dim3(256), 0, s, (const double*)c->G[p], cnt, g->n, g->ld,
                       (unsigned long long*)(c->gmax + p));
    EGT_HIP(hipGetLastError());
  }
  for (int l = 0; l < hp.n_levels; ++l) {
    a.node0 = hp.level_begin[l];
    const int cnt = hp.level_begin[l + 1] - hp.level_begin[l];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(regret_level_kernel, dim3(bx, (unsigned)cnt), dim3(kLanes), 0, s, a);
    EGT_HIP(hipGetLastError());
  }
  EGT_HIP(launch_top_down(g, p, c->QB[p], c->X[p], nullptr, 0.0, nullptr, s));
  return EGT_OK;
}

int cfr_iteration(egt_cfr* c, hipStream_t s) {
  const egt_game* g = c->g;
  const int64_t t = c->t + 1;
  const double w = c->variant == EGT_CFR_PLUS ? (double)t : 1.0;
  c->wsum += w;
  const double tau = w / c->wsum;
  for (int p = 0; p < 2; ++p)
    EGT_HIP(launch_axpby(vec_elems_of(g, p), 1.0 - tau, c->AVG[p], tau, c->X[p], c->AVG[p], s));
  // player 1 against y_t; player 2 against x_t (simultaneous) or x_{t+1} (CFR+)
  EGT_HIP(launch_gradient(g, 0, c->X[1], c->G[0], s));
  if (c->variant != EGT_CFR_PLUS) EGT_HIP(launch_gradient(g, 1, c->X[0], c->G[1], s));
  int rc = cfr_update(c, 0, s);
  if (rc) return rc;
  if (c->variant == EGT_CFR_PLUS) EGT_HIP(launch_gradient(g, 1, c->X[0], c->G[1], s));
  rc = cfr_update(c, 1, s);
  if (rc) return rc;
  c->t = t;
  return EGT_OK;
}

// Saddle gap of the averages: FP64 products and best responses.
int cfr_gap(egt_cfr* c, double* gap, double* brmax, double* brmin, hipStream_t s) {
  const egt_game* g = c->g;
  EGT_HIP(launch_gradient(g, 0, c->AVG[1], c->G[0], s));
  EGT_HIP(launch_gradient(g, 1, c->AVG[0], c->G[1], s));
  const Pass ps[2] = {{0, c->G[0], 1.0, nullptr, 0.0, 0.0, c->Vb[0], nullptr},
                      {1, c->G[1], -1.0, nullptr, 0.0, 0.0, c->Vb[1], nullptr}};
  EGT_HIP(launch_passes(g, ps, 2, nullptr, c->part, s));
  EGT_HIP(launch_sum_partials(g, c->part, 2, c->scal, s));
  EGT_HIP(hipMemcpyAsync(c->hscal, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  EGT_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(c->hscal[0]) || !std::isfinite(c->hscal[1]))
    return fail(EGT_ENUMERIC, "non-finite value in the CFR gap");
  if (gap) *gap = -c->hscal[1] - c->hscal[0];
  if (brmax) *brmax = -c->hscal[1];
  if (brmin) *brmin = c->hscal[0];
  return EGT_OK;
}

}  // namespace

extern "C" {

int egt_cfr_create(const egt_game* g, int32_t variant, hipStream_t s, egt_cfr** out) {
  if (!g || !out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  if (variant != EGT_CFR_RM && variant != EGT_CFR_RMPLUS && variant != EGT_CFR_PLUS)
    return fail(EGT_EINVAL, "unknown CFR variant");
  std::unique_ptr<egt_cfr> c(new (std::nothrow) egt_cfr());
  if (!c) return fail(EGT_ENOMEM, "host allocation failed");
  c->g = g;
  c->variant = variant;
  size_t bytes = 0;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  for (int p = 0; p < 2; ++p) {
    bytes += 5 * al(sizeof(double) * (size_t)vec_elems_of(g, p));
    bytes += 2 * al(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
  }
  bytes += al(sizeof(double) * 2 * kMaxPartials) + 2 * al(2 * sizeof(double));
  hipError_t e = hipMalloc(&c->block, bytes);
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc (CFR state): ") + hipGetErrorString(e));
  e = hipHostMalloc((void**)&c->hscal, 2 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(c->block);
    return fail(EGT_ENOMEM, std::string("hipHostMalloc (CFR state): ") + hipGetErrorString(e));
  }
  unsigned char* cur = (unsigned char*)c->block;
  auto take = [&](size_t nb) {
    void* r = cur;
    cur += al(nb);
    return (double*)r;
  };
  for (int p = 0; p < 2; ++p) {
    const size_t vb = sizeof(double) * (size_t)vec_elems_of(g, p);
    c->R[p] = take(vb);
    c->QB[p] = take(vb);
    c->X[p] = take(vb);
    c->AVG[p] = take(vb);
    c->G[p] = take(vb);
    c->V[p] = take(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
    c->Vb[p] = take(sizeof(double) * (size_t)g->hp[p].n_nodes * g->ld);
  }
  c->part = take(sizeof(double) * 2 * kMaxPartials);
  c->scal = take(2 * sizeof(double));
  c->gmax = take(2 * sizeof(double));
  // zero regrets, uniform local strategies, x_1 = the uniform point, avg = x_1
  for (int p = 0; p < 2; ++p) {
    const int64_t cnt = vec_elems_of(g, p);
    const unsigned fb = (unsigned)std::min<int64_t>((cnt + 255) / 256, 4096);
    if (cnt > 0) hipLaunchKernelGGL(fill_kernel, dim3(fb), dim3(256), 0, s, c->R[p], cnt, 0.0);
    const unsigned bx = (unsigned)((g->ld + kLanes - 1) / kLanes);
    if (g->hp[p].n_seq > 0)
      hipLaunchKernelGGL(uniform_local_kernel, dim3(bx, (unsigned)g->hp[p].n_seq), dim3(kLanes), 0, s,
                         g->dp[p].seq_nact, g->n, g->ld, c->QB[p]);
    EGT_HIP(hipGetLastError());
    EGT_HIP(launch_uniform(g, p, c->X[p], s));
    EGT_HIP(hipMemcpyAsync(c->AVG[p], c->X[p], sizeof(double) * (size_t)cnt, hipMemcpyDeviceToDevice, s));
  }
  EGT_HIP(hipStreamSynchronize(s));
  *out = c.release();
  return EGT_OK;
}

int egt_cfr_destroy(egt_cfr* c) {
  if (!c) return EGT_OK;
  int rc = EGT_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && c->block) e = hipFree(c->block);
  if (e == hipSuccess && c->hscal) e = hipHostFree(c->hscal);
  if (e != hipSuccess) rc = hip_fail(e, "egt_cfr_destroy");
  delete c;
  return rc;
}

int egt_cfr_step(egt_cfr* c, int32_t iters, hipStream_t s) {
  if (!c || iters < 0) return fail(EGT_EINVAL, "null state or negative count");
  for (int32_t k = 0; k < iters; ++k) {
    const int rc = cfr_iteration(c, s);
    if (rc) return rc;
  }
  return EGT_OK;
}

int egt_cfr_gap(egt_cfr* c, double* gap, double* br_max_y, double* br_min_x, hipStream_t s) {
  if (!c) return fail(EGT_EINVAL, "null state");
  return cfr_gap(c, gap, br_max_y, br_min_x, s);
}

int egt_cfr_get(const egt_cfr* c, double* x_avg, double* y_avg, double* x_cur, double* y_cur, int64_t* iters,
                hipStream_t s) {
  if (!c) return fail(EGT_EINVAL, "null state");
  const egt_game* g = c->g;
  double* dst[4] = {x_avg, y_avg, x_cur, y_cur};
  const double* src[4] = {c->AVG[0], c->AVG[1], c->X[0], c->X[1]};
  for (int k = 0; k < 4; ++k)
    if (dst[k])
      EGT_HIP(hipMemcpyAsync(dst[k], src[k], sizeof(double) * (size_t)vec_elems_of(g, k % 2),
                             hipMemcpyDeviceToDevice, s));
  if (iters) *iters = c->t;
  return EGT_OK;
}

int egt_cfr_solve(const egt_game* g, int32_t variant, double eps, int64_t max_iters, int32_t gap_every,
                  egt_result* res, hipStream_t s) {
  if (!g || !res) return fail(EGT_EINVAL, "null argument");
  if (max_iters < 0) return fail(EGT_EINVAL, "max_iters < 0");
  std::memset(res, 0, sizeof(*res));
  if (eps <= 0) eps = 1e-3 * g->pot;
  if (gap_every < 1) gap_every = 1;
  const auto t0 = std::chrono::steady_clock::now();
  egt_cfr* c = nullptr;
  int rc = egt_cfr_create(g, variant, s, &c);
  if (rc) return rc;
  std::unique_ptr<egt_cfr, int (*)(egt_cfr*)> guard(c, egt_cfr_destroy);
  double gap = 0, brmax = 0, brmin = 0;
  bool converged = false;
  for (;;) {
    if ((rc = cfr_gap(c, &gap, &brmax, &brmin, s))) return rc;
    if (gap <= eps) {
      converged = true;
      break;
    }
    if (c->t >= max_iters) break;
    const int64_t k = std::min<int64_t>(gap_every, max_iters - c->t);
    if ((rc = egt_cfr_step(c, (int32_t)k, s))) return rc;
  }
  res->iters = c->t;
  res->products = 2 * c->t;
  res->gap = gap;
  res->br_max_y = brmax;
  res->br_min_x = brmin;
  res->converged = converged ? 1 : 0;
  // value of the averages: x_avg^T A y_avg with A y_avg from the last gap evaluation
  const int64_t n0 = vec_elems_of(g, 0);
  std::vector<double> hx((size_t)n0 * 2);
  EGT_HIP(hipMemcpyAsync(hx.data(), c->AVG[0], sizeof(double) * n0, hipMemcpyDeviceToHost, s));
  EGT_HIP(hipMemcpyAsync(hx.data() + n0, c->G[0], sizeof(double) * n0, hipMemcpyDeviceToHost, s));
  EGT_HIP(hipStreamSynchronize(s));
  double v = 0.0;
  for (int64_t i = 0; i < n0; ++i) v += hx[(size_t)i] * hx[(size_t)(n0 + i)];
  res->value_p1 = -v;
  res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return converged ? EGT_OK : fail(EGT_ENOTCONV, "iteration cap reached before the target gap");
}

}  // extern "C"
