// HIP kernels of the EGT hot path for gfx950 (CDNA4, 64-lane wavefronts).
//
//  * gradient_kernel  : payoff products A y / A^T x (Section 2's gradient
//    operators) on fold and showdown terminals, O(n) per terminal;
//  * bottom_up_kernel : one level of the smoothed best response (Section 4,
//    Eq. 4 and the leaf / internal-simplex derivation), or of the best
//    response when mu = 0;
//  * top_down_kernel  : rebuild the sequence form q_i = q_{p_j} q_bar_i with
//    a fused convex-combination epilogue (Algorithm 2's x_hat, y_+, x_+);
//  * small reductions and vector combinations.
//
// Every vector is double[rows][ld], hands (slots) fastest, so a wavefront's 64
// lanes read 64 consecutive doubles of one row.  Reductions use a fixed order:
// results are bitwise repeatable run to run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "egt_internal.h"

namespace egt {

namespace {

constexpr int kGradThreads = 256;
constexpr int kGradWaves = kGradThreads / 64;
constexpr int kMaxHandsPerThread = 8;  // n <= 2048
constexpr int kPassThreads = 64;       // one wavefront per (node or sequence, 64 hands)

__device__ inline double wave_inclusive_scan(double x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// ---------------------------------------------------------------------------
// Payoff product.  One block per output sequence s of `own`.  For every
// terminal z ending at s (at most a handful), the opponent's reach
// r(h') = b_o(h') v_o[sigma_o(z)][h'] is staged in LDS; then
//   fold:     sum of r over compatible h' = T - C[a] - C[b] + r(h)
//             (T total, C[c] the mass of hands holding card c; the hand's own
//             slot holds both of its cards and is added back once);
//   showdown: (compatible mass stronger) - (compatible mass weaker), from the
//             exclusive prefix sums over strength order and, per card, over
//             the strength-ordered hands holding that card; ties
//             [glo, ghi) count as neither.
// out[s][h] = b_own(h) / Z * sum_z coef(z) * op_z(h), with the showdown op
// negated for player 2 (its gradient sums over player 1's hands).
// ---------------------------------------------------------------------------
struct GradArgs {
  DPlayer own;
  const double* b_opp;
  DHands H;
  const double* v_opp;
  double* out;
  double show_sign;
};

__global__ __launch_bounds__(kGradThreads) void gradient_kernel(GradArgs a) {
  extern __shared__ double lds[];
  const int n = a.H.n, ld = a.H.ld;
  double* r = lds;                    // [ld]
  double* G = r + ld;                 // [ld + 1]
  double* Pc = G + ld + 1;            // [n_card_slots]
  int* cbeg = (int*)(Pc + a.H.n_card_slots);  // [n_cards + 1]
  int* chand = cbeg + a.H.n_cards + 1;        // [card entries]
  __shared__ double wave_total[kGradWaves];

  const int s = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tb = a.own.term_begin[s], te = a.own.term_begin[s + 1];

  double acc[kMaxHandsPerThread];
#pragma unroll
  for (int k = 0; k < kMaxHandsPerThread; ++k) acc[k] = 0.0;

  if (te > tb) {
    const int n_entries = a.H.card_begin[a.H.n_cards];
    for (int i = tid; i <= a.H.n_cards; i += kGradThreads) cbeg[i] = a.H.card_begin[i];
    for (int i = tid; i < n_entries; i += kGradThreads) chand[i] = a.H.card_hands[i];
  }
  const int chunk = (n + kGradThreads - 1) / kGradThreads;

  for (int t = tb; t < te; ++t) {
    const int opp = a.own.term_opp[t];
    const int kind = a.own.term_kind[t];
    const double coef = a.own.term_coef[t];
    const double* v = opp >= 0 ? a.v_opp + (size_t)opp * ld : nullptr;
    for (int i = tid; i < n; i += kGradThreads) r[i] = a.b_opp[i] * (v ? v[i] : 1.0);
    __syncthreads();

    // block-wide exclusive scan of r over strength order into G[0..n]
    {
      const int beg = min(tid * chunk, n), end = min(beg + chunk, n);
      double local = 0.0;
      for (int j = beg; j < end; ++j) local += r[j];
      const double incl = wave_inclusive_scan(local, lane);
      if (lane == 63) wave_total[wave] = incl;
      __syncthreads();
      double run = incl - local;
      for (int w = 0; w < wave; ++w) run += wave_total[w];
      for (int j = beg; j < end; ++j) {
        G[j] = run;
        run += r[j];
      }
      if (beg < end && end == n) G[n] = run;
      if (n == 0 && tid == 0) G[0] = 0.0;
    }
    // per-card exclusive scans: one wavefront per card
    for (int c = wave; c < a.H.n_cards; c += kGradWaves) {
      const int cb = cbeg[c], len = cbeg[c + 1] - cb, base = cb + c;
      double carry = 0.0;
      for (int k0 = 0; k0 < len; k0 += 64) {
        const int k = k0 + lane;
        const double val = k < len ? r[chand[cb + k]] : 0.0;
        const double incl = wave_inclusive_scan(val, lane);
        if (k < len) Pc[base + k] = carry + (incl - val);
        carry += __shfl(incl, 63, 64);
      }
      if (lane == 0) Pc[base + len] = carry;
    }
    __syncthreads();

    const double T = G[n];
#pragma unroll
    for (int k = 0; k < kMaxHandsPerThread; ++k) {
      const int i = tid + k * kGradThreads;
      if (i < n) {
        const int4 A = a.H.ha[i];
        double op;
        if (kind == 0) {
          op = T - Pc[A.x + A.w];
          if (a.H.cph == 2) {
            const int4 B = a.H.hb[i];
            op = op - Pc[B.x + B.w] + r[i];
          }
        } else {
          const int2 tg = a.H.tie[i];
          double weaker = G[tg.x] - Pc[A.x + A.y];
          double stronger = (T - G[tg.y]) - (Pc[A.x + A.w] - Pc[A.x + A.z]);
          if (a.H.cph == 2) {
            const int4 B = a.H.hb[i];
            weaker -= Pc[B.x + B.y];
            stronger -= Pc[B.x + B.w] - Pc[B.x + B.z];
          }
          op = a.show_sign * (stronger - weaker);
        }
        acc[k] += coef * op;
      }
    }
    __syncthreads();  // r, G and Pc are rewritten by the next terminal
  }

  double* row = a.out + (size_t)s * ld;
#pragma unroll
  for (int k = 0; k < kMaxHandsPerThread; ++k) {
    const int i = tid + k * kGradThreads;
    if (i < ld) row[i] = i < n ? acc[k] * (a.own.belief[i] * a.H.invZ) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Bottom-up pass over one level.  Block (hand block, node): each lane is one
// information set (node v, hand h) and loops over the node's actions:
//   g~_a = cA gA[v,a] + cB gB[v,a] + sum_{k in D(v,a)} V[k]
//   smoothed (temp = mu beta_v):
//     m = min_a g~_a,  w_a = exp(-(g~_a - m) / temp),  S = sum_a w_a
//     V[v] = m - temp log S + temp log n_v,  q_bar_a = w_a / S
//   best response: V[v] = min_a g~_a.
// The action with the smallest g~ has the largest q_bar (weight exactly 1), so
// V is the value g~_i + temp log q_bar_i + temp log n_v at that action, and
// every exponent is <= 0.
// ---------------------------------------------------------------------------
struct UpArgs {
  DPlayer P;
  int n, ld;
  const double* gA;
  double cA;
  const double* gB;
  double cB;
  double mu;
  double* V;
  double* QB;
  int node_begin;
};

template <bool kBR>
__global__ __launch_bounds__(kPassThreads) void bottom_up_kernel(UpArgs a) {
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  const int v = a.node_begin + blockIdx.y;
  if (h >= a.n) return;
  const int s0 = a.P.node_first_seq[v];
  const int na = a.P.node_nact[v];
  const size_t ld = a.ld;
  double gt[kMaxActions];
  double m = INFINITY;
#pragma unroll
  for (int k = 0; k < kMaxActions; ++k) {
    if (k < na) {
      const int s = s0 + k;
      double x = a.cA * a.gA[(size_t)s * ld + h];
      if (a.gB) x += a.cB * a.gB[(size_t)s * ld + h];
      const int c1 = a.P.child_begin[s + 1];
      for (int c = a.P.child_begin[s]; c < c1; ++c) x += a.V[(size_t)a.P.child[c] * ld + h];
      gt[k] = x;
      m = fmin(m, x);
    }
  }
  if (kBR) {
    a.V[(size_t)v * ld + h] = m;
    return;
  }
  const double temp = a.mu * a.P.node_beta[v];
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxActions; ++k) {
    if (k < na) {
      gt[k] = exp(-(gt[k] - m) / temp);
      sum += gt[k];
    }
  }
  a.V[(size_t)v * ld + h] = (m - temp * log(sum)) + temp * a.P.node_logn[v];
  if (a.QB) {
#pragma unroll
    for (int k = 0; k < kMaxActions; ++k)
      if (k < na) a.QB[(size_t)(s0 + k) * ld + h] = gt[k] / sum;
  }
}

// ---------------------------------------------------------------------------
// Top-down pass, fully parallel: q[s] = q_bar[root] * ... * q_bar[s] along the
// sequence's parent chain (multiplied from the root down), then the fused
// epilogue comb = (1 - tau) x_prev + tau q.  Padding slots are written 0.
// ---------------------------------------------------------------------------
struct DownArgs {
  const int* seq_parent;
  const double* QB;
  int n, ld;
  double* q_out;
  const double* x_prev;
  double tau;
  double* comb_out;
};

__global__ __launch_bounds__(kPassThreads) void top_down_kernel(DownArgs a) {
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  const int s = blockIdx.y;
  if (h >= a.ld) return;
  const size_t idx = (size_t)s * a.ld + h;
  if (h >= a.n) {
    if (a.q_out) a.q_out[idx] = 0.0;
    if (a.comb_out) a.comb_out[idx] = 0.0;
    return;
  }
  int depth = 0;
  for (int q = s; q >= 0; q = a.seq_parent[q]) ++depth;
  double val = 1.0;
  for (int j = depth - 1; j >= 0; --j) {
    int q = s;
    for (int k = 0; k < j; ++k) q = a.seq_parent[q];
    val *= a.QB[(size_t)q * a.ld + h];
  }
  if (a.q_out) a.q_out[idx] = val;
  if (a.comb_out) a.comb_out[idx] = (1.0 - a.tau) * a.x_prev[idx] + a.tau * val;
}

struct UniformArgs {
  const int* node_first_seq;
  const int* node_nact;
  int n, ld;
  double* QB;
};

__global__ __launch_bounds__(kPassThreads) void uniform_qbar_kernel(UniformArgs a) {
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  const int v = blockIdx.y;
  if (h >= a.ld) return;
  const int s0 = a.node_first_seq[v], na = a.node_nact[v];
  const double val = h < a.n ? 1.0 / (double)na : 0.0;
  for (int k = 0; k < na; ++k) a.QB[(size_t)(s0 + k) * a.ld + h] = val;
}

// ---------------------------------------------------------------------------
// Root sums: a treeplex is a Cartesian product over (root node, hand), so its
// value is the sum of the root simplexes' values.  One block, fixed order.
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 1024;

__device__ double block_sum(double x, double* scratch) {
  const int tid = threadIdx.x;
  scratch[tid] = x;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (tid < w) scratch[tid] += scratch[tid + w];
    __syncthreads();
  }
  const double r = scratch[0];
  __syncthreads();
  return r;
}

struct RootSumArgs {
  const double* VA;
  const int* rootsA;
  int nA;
  double cA;
  const double* VB;
  const int* rootsB;
  int nB;
  double cB;
  int n, ld;
  double* out;
};

__global__ __launch_bounds__(kRedThreads) void root_sum_kernel(RootSumArgs a) {
  __shared__ double scratch[kRedThreads];
  double sA = 0.0, sB = 0.0;
  const int tot_a = a.nA * a.n, tot_b = a.nB * a.n;
  for (int i = threadIdx.x; i < tot_a; i += kRedThreads)
    sA += a.VA[(size_t)a.rootsA[i / a.n] * a.ld + (i % a.n)];
  for (int i = threadIdx.x; i < tot_b; i += kRedThreads)
    sB += a.VB[(size_t)a.rootsB[i / a.n] * a.ld + (i % a.n)];
  sA = block_sum(sA, scratch);
  sB = block_sum(sB, scratch);
  if (threadIdx.x == 0) {
    a.out[0] = a.cA * sA + a.cB * sB;
    a.out[1] = sA;
    a.out[2] = sB;
  }
}

__global__ __launch_bounds__(kRedThreads) void max_abs_kernel(int64_t count, const double* X,
                                                                double* out) {
  __shared__ double scratch[kRedThreads];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kRedThreads) m = fmax(m, fabs(X[i]));
  scratch[threadIdx.x] = m;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) scratch[threadIdx.x] = fmax(scratch[threadIdx.x], scratch[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scratch[0];
}

__global__ __launch_bounds__(256) void axpby_kernel(int64_t count, double a, const double* X, double b,
                                                    const double* Y, double* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    out[i] = Y ? a * X[i] + b * Y[i] : a * X[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_gradient(const egt_game* g, int player, const double* v_opp, double* grad_out,
                           hipStream_t s) {
  GradArgs a;
  a.own = g->dp[player];
  a.b_opp = g->dp[1 - player].belief;
  a.H = g->dh;
  a.v_opp = v_opp;
  a.out = grad_out;
  a.show_sign = player == 0 ? 1.0 : -1.0;
  const int n_entries = g->dh.n_card_slots - g->dh.n_cards;  // hands x cards per hand
  const size_t lds = sizeof(double) * (size_t)(2 * g->ld + 1 + g->dh.n_card_slots) +
                     sizeof(int) * (size_t)(g->dh.n_cards + 1 + n_entries);
  hipLaunchKernelGGL(gradient_kernel, dim3(g->dp[player].n_seq), dim3(kGradThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_bottom_up(const egt_game* g, int player, const double* gA, double cA,
                            const double* gB, double cB, double mu, double* V, double* QB,
                            hipStream_t s) {
  const HostPlayer& hp = g->hp[player];
  UpArgs a;
  a.P = g->dp[player];
  a.n = g->n;
  a.ld = g->ld;
  a.gA = gA;
  a.cA = cA;
  a.gB = gB;
  a.cB = cB;
  a.mu = mu;
  a.V = V;
  a.QB = QB;
  const unsigned bx = (unsigned)((g->n + kPassThreads - 1) / kPassThreads);
  for (int l = 0; l < hp.n_levels; ++l) {
    const int nb = hp.level_begin[l], ne = hp.level_begin[l + 1];
    if (ne <= nb) continue;
    a.node_begin = nb;
    if (mu > 0.0)
      hipLaunchKernelGGL(bottom_up_kernel<false>, dim3(bx, ne - nb), dim3(kPassThreads), 0, s, a);
    else
      hipLaunchKernelGGL(bottom_up_kernel<true>, dim3(bx, ne - nb), dim3(kPassThreads), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_top_down(const egt_game* g, int player, const double* QB, double* q_out,
                           const double* x_prev, double tau, double* comb_out, hipStream_t s) {
  DownArgs a;
  a.seq_parent = g->dp[player].seq_parent;
  a.QB = QB;
  a.n = g->n;
  a.ld = g->ld;
  a.q_out = q_out;
  a.x_prev = x_prev;
  a.tau = tau;
  a.comb_out = comb_out;
  const unsigned bx = (unsigned)((g->ld + kPassThreads - 1) / kPassThreads);
  hipLaunchKernelGGL(top_down_kernel, dim3(bx, g->dp[player].n_seq), dim3(kPassThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_uniform_qbar(const egt_game* g, int player, double* QB, hipStream_t s) {
  UniformArgs a;
  a.node_first_seq = g->dp[player].node_first_seq;
  a.node_nact = g->dp[player].node_nact;
  a.n = g->n;
  a.ld = g->ld;
  a.QB = QB;
  const unsigned bx = (unsigned)((g->ld + kPassThreads - 1) / kPassThreads);
  hipLaunchKernelGGL(uniform_qbar_kernel, dim3(bx, g->dp[player].n_nodes), dim3(kPassThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_root_sum(const egt_game* g, int playerA, const double* VA, double cA, int playerB,
                           const double* VB, double cB, double* out, hipStream_t s) {
  RootSumArgs a;
  a.VA = VA;
  a.rootsA = g->dp[playerA].roots;
  a.nA = g->dp[playerA].n_roots;
  a.cA = cA;
  a.VB = playerB >= 0 ? VB : VA;
  a.rootsB = playerB >= 0 ? g->dp[playerB].roots : a.rootsA;
  a.nB = playerB >= 0 ? g->dp[playerB].n_roots : 0;
  a.cB = playerB >= 0 ? cB : 0.0;
  a.n = g->n;
  a.ld = g->ld;
  a.out = out;
  hipLaunchKernelGGL(root_sum_kernel, dim3(1), dim3(kRedThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t count, double a, const double* X, double b, const double* Y,
                        double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, a, X, b, Y, out);
  return hipGetLastError();
}

hipError_t launch_max_abs(int64_t count, const double* X, double* out, hipStream_t s) {
  hipLaunchKernelGGL(max_abs_kernel, dim3(1), dim3(kRedThreads), 0, s, count, X, out);
  return hipGetLastError();
}

}  // namespace egt
