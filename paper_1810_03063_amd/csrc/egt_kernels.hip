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

constexpr int kGroupThreads = 256;     // one wave group evaluates one terminal
constexpr int kMaxHandsPerThread = 8;  // n <= 2048 = 256 threads x 8 contiguous hands
constexpr int kPassThreads = 64;       // per-level pass: one wavefront per (node, 64 hands)
constexpr int kFusedHands = 16;        // fused pass: hands per block
constexpr int kFusedThreads = 1024;    // fused pass: 64 node slots x 16 hands
constexpr int kFusedSlots = kFusedThreads / kFusedHands;

__device__ inline double wave_inclusive_scan(double x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// ---------------------------------------------------------------------------
// Payoff product.  One block per output sequence s of `own`; the block holds
// `groups` wave groups of 256 threads and group g evaluates the terminals
// tb + g, tb + g + groups, ... of s concurrently with the others.  For a
// terminal z the opponent's reach r(h') = b_o(h') v_o[sigma_o(z)][h'] is
// staged in LDS, each thread keeping its contiguous chunk of hands in
// registers; then
//   fold:     sum of r over compatible h' = T - C[a] - C[b] + r(h)
//             (T total, C[c] the mass of hands holding card c; the hand's own
//             slot holds both of its cards and is added back once);
//   showdown: (compatible mass stronger) - (compatible mass weaker), from the
//             exclusive prefix sum over strength order (built in place over r)
//             and, per card, over the strength-ordered hands holding that card
//             (one thread walks one card's list); a tie group [glo, ghi)
//             counts as neither.
// out[s][h] = b_own(h) / Z * sum_z coef(z) * op_z(h), the showdown op negated
// for player 2 (its gradient sums over player 1's hands).  Group partial sums
// are combined in a fixed order, so the result is bitwise repeatable.
// ---------------------------------------------------------------------------
struct GradArgs {
  DPlayer own;
  const double* b_opp;
  DHands H;
  const double* v_opp;
  double* out;
  double show_sign;
  int groups;
};

__global__ __launch_bounds__(2 * kGroupThreads) void gradient_kernel(GradArgs a) {
  extern __shared__ double lds[];
  __shared__ double wave_total[2][kGroupThreads / 64];
  const int n = a.H.n, ld = a.H.ld;
  const int groups = a.groups;
  const int per_group = (n + 1) + a.H.n_card_slots;
  const int tid = threadIdx.x;
  const int grp = tid / kGroupThreads, gt = tid % kGroupThreads;
  const int lane = tid & 63, wig = gt >> 6;
  double* R = lds + (size_t)grp * per_group;  // r, then its exclusive prefix in place [n + 1]
  double* Pc = R + (n + 1);                   // per-card exclusive prefixes [n_card_slots]
  int* cbeg = (int*)(lds + (size_t)groups * per_group);
  int* chand = cbeg + a.H.n_cards + 1;

  const int s = blockIdx.x;
  const int tb = a.own.term_begin[s], te = a.own.term_begin[s + 1];
  const int chunk = (n + kGroupThreads - 1) / kGroupThreads;
  const int beg = min(gt * chunk, n), end = min(beg + chunk, n), cnt = end - beg;

  double acc[kMaxHandsPerThread];
#pragma unroll
  for (int k = 0; k < kMaxHandsPerThread; ++k) acc[k] = 0.0;

  if (te > tb) {
    const int n_entries = a.H.card_begin[a.H.n_cards];
    for (int i = tid; i <= a.H.n_cards; i += blockDim.x) cbeg[i] = a.H.card_begin[i];
    for (int i = tid; i < n_entries; i += blockDim.x) chand[i] = a.H.card_hands[i];
  }
  const int rounds = (te - tb + groups - 1) / groups;
  for (int rd = 0; rd < rounds; ++rd) {
    const int t = tb + rd * groups + grp;
    const bool active = t < te;  // uniform within a group
    int kind = 0;
    double coef = 0.0;
    if (active) {
      const int opp = a.own.term_opp[t];
      kind = a.own.term_kind[t];
      coef = a.own.term_coef[t];
      const double* v = opp >= 0 ? a.v_opp + (size_t)opp * ld : nullptr;
      for (int i = gt; i < n; i += kGroupThreads) R[i] = a.b_opp[i] * (v ? v[i] : 1.0);
    }
    __syncthreads();
    double rloc[kMaxHandsPerThread];
    if (active) {
#pragma unroll
      for (int k = 0; k < kMaxHandsPerThread; ++k) rloc[k] = k < cnt ? R[beg + k] : 0.0;
      for (int c = gt; c < a.H.n_cards; c += kGroupThreads) {
        const int cb = cbeg[c], len = cbeg[c + 1] - cb, base = cb + c;
        double run = 0.0;
        for (int k = 0; k < len; ++k) {
          Pc[base + k] = run;
          run += R[chand[cb + k]];
        }
        Pc[base + len] = run;
      }
    }
    __syncthreads();  // the card walks have finished reading r
    double local = 0.0, incl = 0.0;
    if (active) {
#pragma unroll
      for (int k = 0; k < kMaxHandsPerThread; ++k) local += rloc[k];
      incl = wave_inclusive_scan(local, lane);
      if (lane == 63) wave_total[grp][wig] = incl;
    }
    __syncthreads();
    if (active) {
      double run = incl - local;
      for (int w = 0; w < wig; ++w) run += wave_total[grp][w];
#pragma unroll
      for (int k = 0; k < kMaxHandsPerThread; ++k) {
        if (k < cnt) {
          R[beg + k] = run;
          run += rloc[k];
        }
      }
      if (cnt > 0 && end == n) R[n] = run;
    }
    __syncthreads();
    if (active) {
      const double T = R[n];
#pragma unroll
      for (int k = 0; k < kMaxHandsPerThread; ++k) {
        if (k < cnt) {
          const int i = beg + k;
          const int4 A = a.H.ha[i];
          double op;
          if (kind == 0) {
            op = T - Pc[A.x + A.w];
            if (a.H.cph == 2) {
              const int4 B = a.H.hb[i];
              op = op - Pc[B.x + B.w] + rloc[k];
            }
          } else {
            const int2 tg = a.H.tie[i];
            double weaker = R[tg.x] - Pc[A.x + A.y];
            double stronger = (T - R[tg.y]) - (Pc[A.x + A.w] - Pc[A.x + A.z]);
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
    }
    __syncthreads();  // the next round rewrites R and Pc
  }
  if (groups == 2) {
    if (grp == 1) {
#pragma unroll
      for (int k = 0; k < kMaxHandsPerThread; ++k)
        if (k < cnt) R[beg + k] = acc[k];
    }
    __syncthreads();
    if (grp == 0) {
      const double* R1 = lds + per_group;
#pragma unroll
      for (int k = 0; k < kMaxHandsPerThread; ++k)
        if (k < cnt) acc[k] += R1[beg + k];
    }
  }
  if (grp == 0) {
    double* row = a.out + (size_t)s * ld;
#pragma unroll
    for (int k = 0; k < kMaxHandsPerThread; ++k)
      if (k < cnt) row[beg + k] = acc[k] * (a.own.belief[beg + k] * a.H.invZ);
    for (int i = n + gt; i < ld; i += kGroupThreads) row[i] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Bottom-up passes.  One information set (node v, hand h) of a tree:
//   g~_a = cA gA[v,a] + cB gB[v,a] + sum_{k in D(v,a)} V[k]
//   smoothed (mu > 0, temp = mu beta_v):
//     m = min_a g~_a,  w_a = exp(-(g~_a - m) / temp),  S = sum_a w_a
//     V[v] = m - temp log S + temp log n_v,  q_bar_a = w_a / S
//   best response (mu = 0): V[v] = min_a g~_a.
// The action with the smallest g~ has the largest q_bar (weight exactly 1), so
// V is the value g~_i + temp log q_bar_i + temp log n_v at that action, and
// every exponent is <= 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void node_pass(const TreePass& t, int v, int h, size_t ld) {
  const int s0 = t.P.node_first_seq[v];
  const int na = t.P.node_nact[v];
  double gt[kMaxActions];
  double m = INFINITY;
#pragma unroll
  for (int k = 0; k < kMaxActions; ++k) {
    if (k < na) {
      const int s = s0 + k;
      double x = t.cA * t.gA[(size_t)s * ld + h];
      if (t.gB) x += t.cB * t.gB[(size_t)s * ld + h];
      const int c1 = t.P.child_begin[s + 1];
      for (int c = t.P.child_begin[s]; c < c1; ++c) x += t.V[(size_t)t.P.child[c] * ld + h];
      gt[k] = x;
      m = fmin(m, x);
    }
  }
  if (!(t.mu > 0.0)) {
    t.V[(size_t)v * ld + h] = m;
    return;
  }
  const double temp = t.mu * t.P.node_beta[v];
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxActions; ++k) {
    if (k < na) {
      gt[k] = exp(-(gt[k] - m) / temp);
      sum += gt[k];
    }
  }
  t.V[(size_t)v * ld + h] = (m - temp * log(sum)) + temp * t.P.node_logn[v];
  if (t.QB) {
#pragma unroll
    for (int k = 0; k < kMaxActions; ++k)
      if (k < na) t.QB[(size_t)(s0 + k) * ld + h] = gt[k] / sum;
  }
}

// Small trees: one launch covers every level.  Block = 16 hands x 64 node
// slots of one tree; a level's nodes are spread over the slots and a block
// barrier separates the levels (a node only needs its children's values, all
// computed by this block for these hands).
__global__ __launch_bounds__(kFusedThreads) void bottom_up_fused_kernel(PassSet a) {
  const TreePass& t = a.t[blockIdx.y];
  const int hl = threadIdx.x % kFusedHands, slot = threadIdx.x / kFusedHands;
  const int h = blockIdx.x * kFusedHands + hl;
  for (int l = 0; l < t.n_levels; ++l) {
    if (h < a.n)
      for (int v = t.level_begin[l] + slot; v < t.level_begin[l + 1]; v += kFusedSlots) node_pass(t, v, h, a.ld);
    __syncthreads();
  }
}

// Large trees: one launch per level over all trees of the set; block = one
// wavefront for (node, 64 hands).
__global__ __launch_bounds__(kPassThreads) void bottom_up_level_kernel(PassSet a) {
  int y = blockIdx.y, k = 0;
  while (k < a.count - 1 && y >= a.level_cnt[k]) {
    y -= a.level_cnt[k];
    ++k;
  }
  const TreePass& t = a.t[k];
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  if (h >= a.n) return;
  node_pass(t, t.level_begin[a.level] + y, h, a.ld);
}

// Root sums: a treeplex is a Cartesian product over (root node, hand), so its
// value is the sum of the root simplexes' values.  Block k sums tree k in a
// fixed order.
__global__ __launch_bounds__(256) void root_sums_kernel(PassSet a, double* out) {
  __shared__ double part[4];
  const TreePass& t = a.t[blockIdx.x];
  const int total = t.P.n_roots * a.n;
  double s = 0.0;
  for (int i = threadIdx.x; i < total; i += 256) {
    const int r = i / a.n, h = i - r * a.n;
    s += t.V[(size_t)t.P.roots[r] * a.ld + h];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
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

constexpr int kRedThreads = 1024;

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
  const size_t per_group = sizeof(double) * (size_t)(g->n + 1 + g->dh.n_card_slots);
  const size_t shared_ints = sizeof(int) * (size_t)(g->dh.n_cards + 1 + n_entries);
  int groups = g->hp[player].max_terms_per_seq >= 2 ? 2 : 1;
  if (groups == 2 && 2 * per_group + shared_ints > kGradLdsLimit) groups = 1;
  a.groups = groups;
  const size_t lds = groups * per_group + shared_ints;
  hipLaunchKernelGGL(gradient_kernel, dim3(g->dp[player].n_seq), dim3(kGroupThreads * groups), lds, s, a);
  return hipGetLastError();
}

static void fill_pass_set(const egt_game* g, const Pass* p, int count, PassSet& a) {
  a.count = count;
  a.n = g->n;
  a.ld = g->ld;
  a.level = 0;
  for (int k = 0; k < kMaxTrees; ++k) {
    a.level_cnt[k] = 0;
    TreePass& t = a.t[k];
    if (k >= count) {
      t = a.t[0];
      continue;
    }
    const HostPlayer& hp = g->hp[p[k].player];
    t.P = g->dp[p[k].player];
    t.gA = p[k].gA;
    t.cA = p[k].cA;
    t.gB = p[k].gB;
    t.cB = p[k].cB;
    t.mu = p[k].mu;
    t.V = p[k].V;
    t.QB = p[k].QB;
    t.n_levels = hp.n_levels;
    for (int l = 0; l <= kMaxDepth; ++l) t.level_begin[l] = hp.level_begin[std::min(l, hp.n_levels)];
  }
}

hipError_t launch_passes(const egt_game* g, const Pass* p, int count, hipStream_t s) {
  if (count < 1 || count > kMaxTrees) return hipErrorInvalidValue;
  PassSet a;
  fill_pass_set(g, p, count, a);
  if (g->fused_passes) {
    const unsigned bx = (unsigned)((g->n + kFusedHands - 1) / kFusedHands);
    hipLaunchKernelGGL(bottom_up_fused_kernel, dim3(bx, count), dim3(kFusedThreads), 0, s, a);
    return hipGetLastError();
  }
  int max_levels = 0;
  for (int k = 0; k < count; ++k) max_levels = std::max(max_levels, a.t[k].n_levels);
  const unsigned bx = (unsigned)((g->n + kPassThreads - 1) / kPassThreads);
  for (int l = 0; l < max_levels; ++l) {
    unsigned total = 0;
    for (int k = 0; k < count; ++k) {
      const TreePass& t = a.t[k];
      a.level_cnt[k] = l < t.n_levels ? t.level_begin[l + 1] - t.level_begin[l] : 0;
      total += (unsigned)a.level_cnt[k];
    }
    if (total == 0) continue;
    a.level = l;
    hipLaunchKernelGGL(bottom_up_level_kernel, dim3(bx, total), dim3(kPassThreads), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_root_sums(const egt_game* g, const Pass* p, int count, double* out, hipStream_t s) {
  if (count < 1 || count > kMaxTrees) return hipErrorInvalidValue;
  PassSet a;
  fill_pass_set(g, p, count, a);
  hipLaunchKernelGGL(root_sums_kernel, dim3(count), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

hipError_t launch_bottom_up(const egt_game* g, int player, const double* gA, double cA,
                            const double* gB, double cB, double mu, double* V, double* QB,
                            hipStream_t s) {
  const Pass p{player, gA, cA, gB, cB, mu, V, QB};
  return launch_passes(g, &p, 1, s);
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
