// HIP kernels of the EGT hot path for gfx950 (CDNA4, 64-lane wavefronts).
//
//  * sbr_fused_kernel  : for trees whose tables fit in LDS, a whole smoothed
//    best response (Section 4, Eq. 4 and the leaf / internal-simplex
//    derivation) in one launch: bottom-up over every level, root-value
//    partial sums, then the top-down rebuild q_i = q_{p_j} q_bar_i with the
//    convex-combination epilogue of Algorithm 2 (x_hat, y_+, x_+);
//    mu = 0 gives the best response;
//  * the same steps one level per launch for large trees:
//    bottom_up_leaf_pair_kernel (lowest level) or bottom_up_level_kernel
//    (its one-hand-per-lane form), bottom_up_internal_kernel (levels with
//    children, a wavefront per action, at most 8), root_sums_kernel, and
//    top_down_pair_kernel or top_down_kernel;
//  * small helpers (uniform point, a*x + b*y, max |x|).
//
// Every vector is double[rows][ld], hands (slots) fastest, so consecutive
// lanes read consecutive doubles of one row.  Reductions use fixed orders, so
// results are bitwise repeatable run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "egt_internal.h"

namespace egt {

namespace {

constexpr int kPassThreads = 64;       // per-level pass: one wavefront per (node, 64 hands)
constexpr int kInternalWaves = 8;       // level path: wavefronts per node block (4 blocks fill a CU's 32 wave slots)
constexpr int kFusedSlots = 64;        // fused pass: node slots per block (x HB hands per slot)

// The per-information-set arithmetic of Section 4's smoothed best response in
// the association of its formulas, every operation rounded on its own (the
// library is built without floating-point contraction), so that every pass
// form below rounds exactly like a plain evaluation of those formulas:
//   weight of action a   w_a = exp((m - g~_a) / (mu beta)), m = min_a g~_a,
//                        so the largest weight is exactly 1;
//   node value           V = (m - mu beta log S) + mu beta log n, S = sum_a w_a
//                        added in action order;
//   local probability    q_bar_a = w_a / S.
// The precision form takes the exponential in FP32 of the FP64 shift times
// 1/temp, keeps S, the logarithm and V in FP64, and forms q_bar with the FP32
// reciprocal of S (itemp and rsum are used by the precision form only).
template <class TG>
__device__ inline double lse_weight(double m, double g, double temp, double itemp) {
  if constexpr (std::is_same<TG, float>::value)
    return (double)expf((float)((m - g) * itemp));
  else
    return exp((m - g) / temp);
}
template <class TG>
__device__ inline double inv_or_zero(double x) {
  return std::is_same<TG, float>::value ? 1.0 / x : 0.0;
}
template <class TG>
__device__ inline double qbar(double w, double sum, double rsum) {
  if constexpr (std::is_same<TG, float>::value)
    return (double)((float)w * (float)rsum);
  else
    return w / sum;
}
__device__ inline double lse_value(double m, double temp, double sum, double logn) {
  return (m - temp * log(sum)) + temp * logn;
}
// cA a + cB b (the mixed gradient of the prox, or a single scaled gradient).
__device__ inline double lin2(double cA, double a, double cB, double b) { return cA * a + cB * b; }

// ---------------------------------------------------------------------------
// One information set (node v, hand h) of a bottom-up pass:
//   g~_a = cA gA[v,a] + cB gB[v,a] + sum_{k in D(v,a)} V[k]
//   smoothed (mu > 0, temp = mu beta_v):
//     m = min_a g~_a,  w_a = exp((m - g~_a) / temp),  S = sum_a w_a
//     V[v] = m - temp log S + temp log n_v,  q_bar_a = w_a / S
//   best response (mu = 0): V[v] = min_a g~_a.
// The action with the smallest g~ has the largest q_bar (weight exactly 1), so
// V is the value g~_i + temp log q_bar_i + temp log n_v at that action, and
// every exponent is <= 0.  Both pass forms below evaluate exactly this through
// lse_weight / lse_value, the children of an action added in betting order
// (the order of the child CSR).
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Fused pass for trees whose tables fit in LDS.  Block = (tree k, HB hands),
// 64 node slots x HB hands.
//   1. Stage in LDS, all loads in flight together: the player's table image
//      (FusedTabLayout), the combined gradient cA gA + cB gB of the block's
//      hands and, for the epilogue, x_prev.
//   2. Bottom-up, one level at a time (a block barrier after each phase):
//      (a) sequence phase (levels above the lowest): g~_s = g_s + the values
//          of the child nodes of s, read from their contiguous value slots;
//      (b) node phase: the smoothed (or plain) best response at each
//          (node, hand) from the g~ of its actions, writing the node value to
//          its slot and q_bar.  Tasks are (sequence, hand) / (node, hand)
//          pairs spread over all threads.
//   3. The block's partial root sum (the tree value is a sum over (root, hand)).
//   4. Top-down, level by level from the roots: q[s] = q[parent] * q_bar[s]
//      in place, then the epilogue (1 - tau) x_prev + tau q.  Slots h >= n
//      (the row padding) are written 0.
//
// The grid is one-dimensional over (tree, hand block) and spread so that each
// XCD (workgroups go round-robin over the 8 XCDs) gets a contiguous range of
// hand blocks: neighbouring blocks share cache lines of every row, and those
// then meet in one L2.
// ---------------------------------------------------------------------------
struct FusedArgs {
  PassSet ps;
  Epilogue epi[kMaxTrees];
  double* partial;  // [count][n_hblocks] or null (device or pinned host memory)
  int cap_tab, cap_nodes, cap_seqs;
  int n_hblocks;  // hand blocks per tree (ld / HB)
};

// Bijection of [0, total): workgroup L (on XCD L % 8) -> position, with each
// XCD's workgroups on consecutive positions.
__device__ inline int xcd_spread(int L, int total) {
  const int q = total / 8, r = total % 8;
  const int x = L % 8, j = L / 8;
  return x * q + min(x, r) + j;
}

// One (node, hand) task of the node phase: g~ of the node's actions in Gl,
// value to the node's slot in Vs, q_bar to Ql (smoothed, want_q).  Every
// action's g~ is read up front (indices clamped into the node), so the reads
// overlap.  temp = mu beta_v.
template <class TG, int HB>
__device__ __forceinline__ void fused_node(const int4* rec, const double2* prm, const double* Gl, double* Ql,
                                           double* Vs, int v, int hl, double mu, bool want_q) {
  const int4 r = rec[v];
  const int s0 = r.x, na = r.y;
  double g[kMaxActions];
#pragma unroll
  for (int k = 0; k < kMaxActions; ++k) g[k] = Gl[(s0 + min(k, na - 1)) * HB + hl];
  double m = g[0];
#pragma unroll
  for (int k = 1; k < kMaxActions; ++k)
    if (k < na) m = fmin(m, g[k]);
  if (!(mu > 0.0)) {
    Vs[r.z * HB + hl] = m;
    return;
  }
  const double2 p0 = prm[2 * v], p1 = prm[2 * v + 1];  // {beta, 1 / beta}, {log n_v, 0}
  const double temp = mu * p0.x, itemp = inv_or_zero<TG>(temp);
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxActions; ++k) {
    if (k < na) {
      g[k] = lse_weight<TG>(m, g[k], temp, itemp);
      sum += g[k];
    }
  }
  Vs[r.z * HB + hl] = lse_value(m, temp, sum, p1.x);
  if (want_q) {
    const double rs = inv_or_zero<TG>(sum);
#pragma unroll
    for (int k = 0; k < kMaxActions; ++k)
      if (k < na) Ql[(s0 + k) * HB + hl] = (double)(TG)qbar<TG>(g[k], sum, rs);
  }
}

template <int HB, class TG>
__global__ __launch_bounds__(kFusedSlots * HB) void sbr_fused_kernel(FusedArgs a) {
  constexpr int kThreads = kFusedSlots * HB;
  constexpr int kU = 4;   // gradient loads in flight per thread and batch
  constexpr int kTU = 2;  // table loads per thread in the first batch
  extern __shared__ __align__(16) unsigned char fused_lds[];
  const int nb = a.n_hblocks;
  const int P = xcd_spread((int)blockIdx.x, (int)gridDim.x);
  const int k = P / nb, hblk = P % nb;
  const TreePass& t = a.ps.t[k];
  const Epilogue& e = a.epi[k];
  const int N = t.P.n_nodes, S = t.P.n_seq;
  const FusedTabLayout L = fused_tab_layout(N, S);
  const int4* rec = (const int4*)(fused_lds + L.rec);
  const double2* prm = (const double2*)(fused_lds + L.prm);
  const int* cbeg = (const int*)(fused_lds + L.cbeg);
  const int* spar = (const int*)(fused_lds + L.spar);
  double* Gl = (double*)(fused_lds + a.cap_tab);  // [cap_seqs][HB] gradient, then g~
  double* Ql = Gl + (size_t)a.cap_seqs * HB;      // [cap_seqs][HB] q_bar, then q
  double* Xl = Ql + (size_t)a.cap_seqs * HB;      // [cap_seqs][HB] x_prev of the epilogue
  double* Vs = Xl + (size_t)a.cap_seqs * HB;      // [cap_nodes][HB] node values by slot
  // a dual tree (VB; every tree of the launch is then dual) also takes the
  // best response to the same gradient: its g~ and node values beside
  const bool dual = t.VB != nullptr && t.mu > 0.0;
  double* GBl = Vs + (size_t)a.cap_nodes * HB;  // [cap_seqs][HB] dual: gradient, then the best response's g~
  double* VBs = GBl + (size_t)a.cap_seqs * HB;  // [cap_nodes][HB] dual: best-response node values
  const int tid = threadIdx.x;
  const int h0 = hblk * HB, n = a.ps.n;
  const size_t ld = a.ps.ld;
  const int SH = S * HB;

  // 1. staging
  const uint4* tab = (const uint4*)t.P.fused_tab;
  uint4* tl = (uint4*)fused_lds;
  const int T16 = t.P.fused_tab16;
  const TG* gA = (const TG*)t.gA;
  const TG* gB = (const TG*)t.gB;
  const TG* x_prev = (const TG*)e.x_prev;
  const bool want_x = e.comb_out != nullptr;
  TG* g_out = (TG*)e.g_out;
  uint4 tb[kTU];
#pragma unroll
  for (int u = 0; u < kTU; ++u) {
    const int i = u * kThreads + tid;
    tb[u] = i < T16 ? tab[i] : make_uint4(0u, 0u, 0u, 0u);
  }
  for (int base = 0; base < SH; base += kThreads * kU) {
    double va[kU], vb[kU], vx[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = base + u * kThreads + tid;
      const int hh = h0 + i % HB;
      va[u] = vb[u] = vx[u] = 0.0;
      if (i < SH && hh < n) {
        const size_t idx = (size_t)(i / HB) * ld + hh;
        va[u] = (double)gA[idx];
        if (gB) vb[u] = (double)gB[idx];
        if (want_x) vx[u] = (double)x_prev[idx];
      }
    }
    if (base == 0) {
#pragma unroll
      for (int u = 0; u < kTU; ++u) {
        const int i = u * kThreads + tid;
        if (i < T16) tl[i] = tb[u];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = base + u * kThreads + tid;
      if (i < SH) {
        const double x = gB ? lin2(t.cA, va[u], t.cB, vb[u]) : t.cA * va[u];
        if (dual) GBl[i] = x;
        if (want_x) Xl[i] = vx[u];
        if (g_out) {
          g_out[(size_t)(i / HB) * ld + h0 + i % HB] = (TG)(x * e.g_scale);  // 0 in the padding
          Gl[i] = (double)(TG)x;  // continue with the stored gradient (g_scale = +-1)
        } else {
          Gl[i] = x;
        }
      }
    }
  }
  if (SH == 0) {
#pragma unroll
    for (int u = 0; u < kTU; ++u) {
      const int i = u * kThreads + tid;
      if (i < T16) tl[i] = tb[u];
    }
  }
  for (int i = kTU * kThreads + tid; i < T16; i += kThreads) tl[i] = tab[i];
  __syncthreads();

  // 2. bottom-up
  const bool want_q = (e.q_out || e.comb_out || e.qb_out) && t.mu > 0.0;
  const double mu = t.mu;
  for (int l = 0; l < t.n_levels; ++l) {
    if (l > 0) {
      const int sb0 = t.seq_level_begin[l], cnt = (t.seq_level_begin[l + 1] - sb0) * HB;
      for (int i = tid; i < cnt; i += kThreads) {
        const int s = sb0 + i / HB, hl = i % HB;
        const int c0 = cbeg[s], c1 = cbeg[s + 1];
        if (h0 + hl >= n || c0 == c1) continue;
        double x = Gl[s * HB + hl];
        int c = c0;
        for (; c + 4 <= c1; c += 4) {
          const double v0 = Vs[c * HB + hl], v1 = Vs[(c + 1) * HB + hl];
          const double v2 = Vs[(c + 2) * HB + hl], v3 = Vs[(c + 3) * HB + hl];
          x += v0;
          x += v1;
          x += v2;
          x += v3;
        }
        for (; c < c1; ++c) x += Vs[c * HB + hl];
        Gl[s * HB + hl] = x;
        if (dual) {  // the same additions on the best-response values
          double xb = GBl[s * HB + hl];
          int cb = c0;
          for (; cb + 4 <= c1; cb += 4) {
            const double v0 = VBs[cb * HB + hl], v1 = VBs[(cb + 1) * HB + hl];
            const double v2 = VBs[(cb + 2) * HB + hl], v3 = VBs[(cb + 3) * HB + hl];
            xb += v0;
            xb += v1;
            xb += v2;
            xb += v3;
          }
          for (; cb < c1; ++cb) xb += VBs[cb * HB + hl];
          GBl[s * HB + hl] = xb;
        }
      }
      __syncthreads();
    }
    const int nb0 = t.level_begin[l], cnt = (t.level_begin[l + 1] - nb0) * HB;
    for (int i = tid; i < cnt; i += kThreads) {
      const int v = nb0 + i / HB, hl = i % HB;
      if (h0 + hl < n) {
        fused_node<TG, HB>(rec, prm, Gl, Ql, Vs, v, hl, mu, want_q);
        if (dual) fused_node<TG, HB>(rec, prm, GBl, nullptr, VBs, v, hl, 0.0, false);  // mu = 0: the minimum
      }
    }
    __syncthreads();
  }

  // the local strategies, for a later top-down pass (0 in the padding)
  if (e.qb_out && want_q) {
    TG* qb_out = (TG*)e.qb_out;
    for (int i = tid; i < SH; i += kThreads) {
      const int hh = h0 + i % HB;
      qb_out[(size_t)(i / HB) * ld + hh] = hh < n ? (TG)Ql[i] : (TG)0;
    }
  }

  // 3. partial root sum
  if (a.partial && tid < HB) {
    double sv = 0.0;
    if (h0 + tid < n) {
      const int C = N - t.P.n_roots;
      for (int r = 0; r < t.P.n_roots; ++r) sv += Vs[(C + r) * HB + tid];
    }
#pragma unroll
    for (int off = HB / 2; off > 0; off >>= 1) sv += __shfl_down(sv, off, HB);
    if (tid == 0) a.partial[(size_t)k * nb + hblk] = sv;
  }
  if (a.partial && dual && tid < HB) {  // the best response's, after the launch's trees
    double sv = 0.0;
    if (h0 + tid < n) {
      const int C = N - t.P.n_roots;
      for (int r = 0; r < t.P.n_roots; ++r) sv += VBs[(C + r) * HB + tid];
    }
#pragma unroll
    for (int off = HB / 2; off > 0; off >>= 1) sv += __shfl_down(sv, off, HB);
    if (tid == 0) a.partial[(size_t)(a.ps.count + k) * nb + hblk] = sv;
  }

  // 4. top-down and epilogue
  if (e.q_out || e.comb_out) {
    for (int l = t.n_levels - 1; l >= 0; --l) {
      const int sb0 = t.seq_level_begin[l], cnt = (t.seq_level_begin[l + 1] - sb0) * HB;
      for (int i = tid; i < cnt; i += kThreads) {
        const int s = sb0 + i / HB, hl = i % HB;
        const int par = spar[s];
        if (h0 + hl < n && par >= 0) Ql[s * HB + hl] = (double)((TG)Ql[par * HB + hl] * (TG)Ql[s * HB + hl]);
      }
      __syncthreads();
    }
    TG* q_out = (TG*)e.q_out;
    TG* comb_out = (TG*)e.comb_out;
    const TG tau = (TG)e.tau, one_m_tau = (TG)(1.0 - e.tau);
    for (int i = tid; i < SH; i += kThreads) {
      const int hh = h0 + i % HB;
      const size_t idx = (size_t)(i / HB) * ld + hh;
      if (hh >= n) {
        if (q_out) q_out[idx] = (TG)0;
        if (comb_out) comb_out[idx] = (TG)0;
        continue;
      }
      const TG q = (TG)Ql[i];
      if (q_out) q_out[idx] = q;
      if (comb_out) comb_out[idx] = one_m_tau * (TG)Xl[i] + tau * q;
    }
  }
}

// Large trees: one launch per level over all trees of the set; block = one
// wavefront for (node, 64 hands); node values (by value slot) and q_bar in
// global memory.  The node's record and parameters come from the table image
// (block-uniform loads), a sequence's children from contiguous value slots.
// With g_out the launch also writes g_scale (cA gA + cB gB) of every sequence
// it reads.
template <class TG>
__global__ __launch_bounds__(kPassThreads) void bottom_up_level_kernel(PassSet a) {
  int y = blockIdx.y, k = 0;
  while (k < a.count - 1 && y >= a.level_cnt[k]) {
    y -= a.level_cnt[k];
    ++k;
  }
  const TreePass& t = a.t[k];
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  if (h >= a.n) return;
  const size_t ld = a.ld;
  const int v = t.level_begin[a.level] + y;
  const FusedTabLayout L = fused_tab_layout(t.P.n_nodes, t.P.n_seq);
  const unsigned char* tab = (const unsigned char*)t.P.fused_tab;
  const int4 r = ((const int4*)(tab + L.rec))[v];
  const double2 p0 = ((const double2*)(tab + L.prm))[2 * v], p1 = ((const double2*)(tab + L.prm))[2 * v + 1];
  const int* cbeg = (const int*)(tab + L.cbeg);
  const int s0 = r.x, na = r.y;
  const TG* gA = (const TG*)t.gA;
  const TG* gB = (const TG*)t.gB;
  TG* g_out = (TG*)t.g_out;
  double g[kMaxActions];
  double m = INFINITY;
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j) {
    if (j < na) {
      const size_t idx = (size_t)(s0 + j) * ld + h;
      double x = gB ? lin2(t.cA, (double)gA[idx], t.cB, (double)gB[idx]) : t.cA * (double)gA[idx];
      if (g_out) {
        g_out[idx] = (TG)(x * t.g_scale);
        x = (double)(TG)x;  // continue with the stored gradient (g_scale = +-1)
      }
      const int c1 = cbeg[s0 + j + 1];
      for (int c = cbeg[s0 + j]; c < c1; ++c) x += t.V[(size_t)c * ld + h];
      g[j] = x;
      m = fmin(m, x);
    }
  }
  if (!(t.mu > 0.0)) {
    t.V[(size_t)r.z * ld + h] = m;
    return;
  }
  // dual pass: below a node without child nodes the best response's g~ is
  // the same, so its value is the minimum
  if (t.VB) t.VB[(size_t)r.z * ld + h] = m;
  const double temp = t.mu * p0.x, itemp = inv_or_zero<TG>(temp);
  double sum = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j) {
    if (j < na) {
      g[j] = lse_weight<TG>(m, g[j], temp, itemp);
      sum += g[j];
    }
  }
  t.V[(size_t)r.z * ld + h] = lse_value(m, temp, sum, p1.x);
  if (t.QB) {
    const double rs = inv_or_zero<TG>(sum);
#pragma unroll
    for (int j = 0; j < kMaxActions; ++j)
      if (j < na) ((TG*)t.QB)[(size_t)(s0 + j) * ld + h] = (TG)qbar<TG>(g[j], sum, rs);
  }
}

// The lowest level (no node has children) with two adjacent hands per lane:
// one 16-byte access per gradient row (8 bytes in FP32), half the wavefronts.
// Used when every row pointer is aligned to two elements; per hand the
// arithmetic is the one above, and slots h >= n are not written.
template <class TG>
__device__ inline void store_pair(TG* p, double x0, double x1, bool both) {
  using V2 = typename std::conditional<std::is_same<TG, float>::value, float2, double2>::type;
  if (both) {
    V2 o;
    o.x = (TG)x0;
    o.y = (TG)x1;
    *(V2*)p = o;
  } else {
    p[0] = (TG)x0;
  }
}

template <class TG>
__global__ __launch_bounds__(kPassThreads) void bottom_up_leaf_pair_kernel(PassSet a) {
  using V2 = typename std::conditional<std::is_same<TG, float>::value, float2, double2>::type;
  int y = blockIdx.y, k = 0;
  while (k < a.count - 1 && y >= a.level_cnt[k]) {
    y -= a.level_cnt[k];
    ++k;
  }
  const TreePass& t = a.t[k];
  const int h = 2 * (blockIdx.x * kPassThreads + threadIdx.x);
  if (h >= a.n) return;
  const bool both = h + 1 < a.n;
  const size_t ld = a.ld;
  const int v = t.level_begin[a.level] + y;
  const FusedTabLayout L = fused_tab_layout(t.P.n_nodes, t.P.n_seq);
  const unsigned char* tab = (const unsigned char*)t.P.fused_tab;
  const int4 r = ((const int4*)(tab + L.rec))[v];
  const double2 p0 = ((const double2*)(tab + L.prm))[2 * v], p1 = ((const double2*)(tab + L.prm))[2 * v + 1];
  const int s0 = r.x, na = r.y;
  const TG* gA = (const TG*)t.gA;
  const TG* gB = (const TG*)t.gB;
  TG* g_out = (TG*)t.g_out;
  double g0[kMaxActions], g1[kMaxActions];
  double m0 = INFINITY, m1 = INFINITY;
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j) {
    if (j < na) {
      const size_t idx = (size_t)(s0 + j) * ld + h;
      const V2 A = *(const V2*)(gA + idx);
      double x0 = t.cA * (double)A.x, x1 = t.cA * (double)A.y;
      if (gB) {
        const V2 B = *(const V2*)(gB + idx);
        x0 = lin2(t.cA, (double)A.x, t.cB, (double)B.x);
        x1 = lin2(t.cA, (double)A.y, t.cB, (double)B.y);
      }
      if (g_out) {
        store_pair(g_out + idx, x0 * t.g_scale, x1 * t.g_scale, both);
        x0 = (double)(TG)x0;  // continue with the stored gradient (g_scale = +-1)
        x1 = (double)(TG)x1;
      }
      g0[j] = x0;
      g1[j] = x1;
      m0 = fmin(m0, x0);
      m1 = fmin(m1, x1);
    }
  }
  double* Vrow = t.V + (size_t)r.z * ld + h;
  if (!(t.mu > 0.0)) {
    store_pair(Vrow, m0, m1, both);
    return;
  }
  if (t.VB) store_pair(t.VB + (size_t)r.z * ld + h, m0, m1, both);  // dual pass: the best response's value
  const double temp = t.mu * p0.x, itemp = inv_or_zero<TG>(temp);
  double sum0 = 0.0, sum1 = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxActions; ++j) {
    if (j < na) {
      g0[j] = lse_weight<TG>(m0, g0[j], temp, itemp);
      g1[j] = lse_weight<TG>(m1, g1[j], temp, itemp);
      sum0 += g0[j];
      sum1 += g1[j];
    }
  }
  store_pair(Vrow, lse_value(m0, temp, sum0, p1.x), lse_value(m1, temp, sum1, p1.x), both);
  if (t.QB) {
    const double rs0 = inv_or_zero<TG>(sum0), rs1 = inv_or_zero<TG>(sum1);
#pragma unroll
    for (int j = 0; j < kMaxActions; ++j)
      if (j < na)
        store_pair((TG*)t.QB + (size_t)(s0 + j) * ld + h, qbar<TG>(g0[j], sum0, rs0), qbar<TG>(g1[j], sum1, rs1),
                   both);
  }
}

// Levels above the lowest (every node has child nodes): the same evaluation
// with the actions in parallel.  Block = (node, 64 x HP hands) x `blockDim.y`
// wavefronts (the level's most actions, at most kInternalWaves); wavefront j
// takes actions j, j + blockDim.y, ... for HP
// adjacent hands per lane (HP = 2 on wide levels when every row is 2-element
// aligned): its
// gradients and its children, whose value slots [cbeg[s], cbeg[s + 1]) are
// read in batches of kChildBatch so that one round trip covers them all and
// added in slot order.  The node's g~ and weights meet in LDS; the minimum,
// the weight sum and the value are then formed in the same order as above, so
// per hand the result is bitwise the one the one-wavefront form gives.
template <class TG, int HP>
__global__ __launch_bounds__(kPassThreads * kInternalWaves) void bottom_up_internal_kernel(PassSet a) {
  static_assert(HP == 1 || HP == 2, "one or two hands per lane");
  using V2 = typename std::conditional<std::is_same<TG, float>::value, float2, double2>::type;
  constexpr int kChildBatch = 8;
  constexpr int W = HP * kPassThreads;
  __shared__ double gl[kMaxActions][W];
  __shared__ double wl[kMaxActions][W];
  int y = blockIdx.y, k = 0;
  while (k < a.count - 1 && y >= a.level_cnt[k]) {
    y -= a.level_cnt[k];
    ++k;
  }
  const TreePass& t = a.t[k];
  const int lane = threadIdx.x, j = threadIdx.y;
  const int h = HP * (blockIdx.x * kPassThreads + lane);  // the lane's first hand; h + 1 < ld when HP = 2
  const bool both = HP == 2 && h + 1 < a.n;
  const size_t ld = a.ld;
  const int v = t.level_begin[a.level] + y;
  const FusedTabLayout L = fused_tab_layout(t.P.n_nodes, t.P.n_seq);
  const unsigned char* tab = (const unsigned char*)t.P.fused_tab;
  const int4 r = ((const int4*)(tab + L.rec))[v];
  const double2 p0 = ((const double2*)(tab + L.prm))[2 * v], p1 = ((const double2*)(tab + L.prm))[2 * v + 1];
  const int* cbeg = (const int*)(tab + L.cbeg);
  const int s0 = r.x, na = r.y;
  const bool live = h < a.n;
  const bool act = live && j < na;  // this wavefront owns actions j, j + blockDim.y, ...
  const int nw = (int)blockDim.y;
  auto load2 = [&](const TG* p, double& x0, double& x1) {
    if constexpr (HP == 2) {
      const V2 q = *(const V2*)p;
      x0 = (double)q.x;
      x1 = (double)q.y;
    } else {
      x0 = (double)p[0];
      x1 = 0.0;
    }
  };
  auto store2 = [&](auto* p, double x0, double x1) {
    if constexpr (HP == 2)
      store_pair(p, x0, x1, both);
    else
      p[0] = (std::remove_pointer_t<decltype(p)>)x0;
  };
  for (int jj = j; live && jj < na; jj += nw) {
    const size_t idx = (size_t)(s0 + jj) * ld + h;
    double x0, x1, b0, b1;
    load2((const TG*)t.gA + idx, x0, x1);
    if (t.gB) {
      load2((const TG*)t.gB + idx, b0, b1);
      x0 = lin2(t.cA, x0, t.cB, b0);
      x1 = lin2(t.cA, x1, t.cB, b1);
    } else {
      x0 = t.cA * x0;
      x1 = t.cA * x1;
    }
    if (t.g_out) {
      store2((TG*)t.g_out + idx, x0 * t.g_scale, x1 * t.g_scale);
      x0 = (double)(TG)x0;  // continue with the stored gradient (g_scale = +-1)
      x1 = (double)(TG)x1;
    }
    const int c0 = cbeg[s0 + jj], c1 = cbeg[s0 + jj + 1];
    for (int c = c0; c < c1; c += kChildBatch) {
      double cv0[kChildBatch], cv1[kChildBatch];
#pragma unroll
      for (int u = 0; u < kChildBatch; ++u) {
        cv0[u] = 0.0;
        cv1[u] = 0.0;
        if (c + u < c1) {
          const double* vp = t.V + (size_t)(c + u) * ld + h;
          if constexpr (HP == 2) {
            const double2 q = *(const double2*)vp;
            cv0[u] = q.x;
            cv1[u] = q.y;
          } else {
            cv0[u] = vp[0];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kChildBatch; ++u)
        if (c + u < c1) {
          x0 += cv0[u];
          x1 += cv1[u];
        }
    }
    gl[jj][lane] = x0;
    if constexpr (HP == 2) gl[jj][kPassThreads + lane] = x1;
  }
  __syncthreads();
  double m0 = INFINITY, m1 = INFINITY;
  if (act)
    for (int i = 0; i < na; ++i) {
      m0 = fmin(m0, gl[i][lane]);
      if constexpr (HP == 2) m1 = fmin(m1, gl[i][kPassThreads + lane]);
    }
  double* Vrow = t.V + (size_t)r.z * ld + h;
  if (!(t.mu > 0.0)) {
    if (act && j == 0) store2(Vrow, m0, m1);
    return;
  }
  const double temp = t.mu * p0.x, itemp = inv_or_zero<TG>(temp);
  for (int jj = j; live && jj < na; jj += nw) {
    double w1 = 0.0;
    const double w0 = lse_weight<TG>(m0, gl[jj][lane], temp, itemp);
    if constexpr (HP == 2) w1 = lse_weight<TG>(m1, gl[jj][kPassThreads + lane], temp, itemp);
    wl[jj][lane] = w0;
    if constexpr (HP == 2) wl[jj][kPassThreads + lane] = w1;
  }
  __syncthreads();
  if (act) {
    double sum0 = 0.0, sum1 = 0.0;
    for (int i = 0; i < na; ++i) {
      sum0 += wl[i][lane];
      if constexpr (HP == 2) sum1 += wl[i][kPassThreads + lane];
    }
    if (j == 0)
      store2(Vrow, lse_value(m0, temp, sum0, p1.x), HP == 2 ? lse_value(m1, temp, sum1, p1.x) : 0.0);
    if (t.QB) {
      const double rs0 = inv_or_zero<TG>(sum0), rs1 = inv_or_zero<TG>(sum1);
      for (int jj = j; jj < na; jj += nw)
        store2((TG*)t.QB + (size_t)(s0 + jj) * ld + h, qbar<TG>(wl[jj][lane], sum0, rs0),
               HP == 2 ? qbar<TG>(wl[jj][kPassThreads + lane], sum1, rs1) : 0.0);
    }
  }
}

// Root sums of the level path: block k sums tree k, roots in order (value
// slots C + r), hands strided over the threads, then a fixed-order reduction.
__global__ __launch_bounds__(256) void root_sums_kernel(PassSet a, double* out) {
  constexpr int kRootBatch = 4;                     // roots whose values are requested together
  constexpr int kHandSteps = 8;                     // hands per thread and root (n <= 2048 = 256 x 8)
  __shared__ double part[4];
  const TreePass& t = a.t[blockIdx.x];
  double s = 0.0;
  const int C = t.P.n_nodes - t.P.n_roots;  // the r-th root's value slot is C + r
  // each thread adds its hands h = tid + 256 m root by root, m ascending; the
  // loads of kRootBatch roots are issued before the first add
  for (int r0 = 0; r0 < t.P.n_roots; r0 += kRootBatch) {
    double v[kRootBatch][kHandSteps];
#pragma unroll
    for (int u = 0; u < kRootBatch; ++u) {
      const double* row = t.V + (size_t)(C + r0 + u) * a.ld;
#pragma unroll
      for (int m = 0; m < kHandSteps; ++m) {
        const int h = (int)threadIdx.x + 256 * m;
        v[u][m] = (r0 + u < t.P.n_roots && h < a.n) ? row[h] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kRootBatch; ++u)
#pragma unroll
      for (int m = 0; m < kHandSteps; ++m)
        if (r0 + u < t.P.n_roots && (int)threadIdx.x + 256 * m < a.n) s += v[u][m];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

// out[k] = sum of partial[k][0 .. nb) in order.
__global__ __launch_bounds__(64) void sum_partials_kernel(const double* partial, int count, int nb, double* out) {
  const int k = threadIdx.x;
  if (k >= count) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(size_t)k * nb + b];
  out[k] = s;
}

// ---------------------------------------------------------------------------
// Top-down pass of the level path, fully parallel: q[s] = q_bar[root] * ...
// * q_bar[s] along the sequence's path (multiplied from the root down, the
// path read from the precomputed root-first table, so every q_bar load is
// issued at once), then the epilogue comb = (1 - tau) x_prev + tau q.
// Padding slots are written 0.
// ---------------------------------------------------------------------------
struct DownArgs {
  const int* anc;
  const void* QB;
  int n, ld, n_seq;
  void* q_out;
  const void* x_prev;
  double tau;
  void* comb_out;
};

template <class TS>
__global__ __launch_bounds__(kPassThreads) void top_down_kernel(DownArgs a) {
  const TS* QB = (const TS*)a.QB;
  TS* q_out = (TS*)a.q_out;
  TS* comb_out = (TS*)a.comb_out;
  const TS* x_prev = (const TS*)a.x_prev;
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  const int s = blockIdx.y;
  if (h >= a.ld) return;
  const size_t idx = (size_t)s * a.ld + h;
  if (h >= a.n) {
    if (q_out) q_out[idx] = (TS)0;
    if (comb_out) comb_out[idx] = (TS)0;
    return;
  }
  const int* path = a.anc + (size_t)s * kMaxDepth;
  TS f[kMaxDepth];
#pragma unroll
  for (int j = 0; j < kMaxDepth; ++j) {
    const int q = path[j];
    f[j] = q >= 0 ? QB[(size_t)q * a.ld + h] : (TS)1;
  }
  TS val = (TS)1;
#pragma unroll
  for (int j = 0; j < kMaxDepth; ++j)
    if (path[j] >= 0) val *= f[j];
  const TS xp = comb_out ? x_prev[idx] : (TS)0;
  if (q_out) q_out[idx] = val;
  if (comb_out) comb_out[idx] = (TS)(1.0 - a.tau) * xp + (TS)a.tau * val;
}

// The same with two adjacent hands per lane (one 16-byte access per row for
// FP64, 8 bytes for FP32), halving the wavefronts; used when every row
// pointer is aligned to two elements.  Per hand the arithmetic is the one
// above.
template <class TS>
__global__ __launch_bounds__(kPassThreads) void top_down_pair_kernel(DownArgs a) {
  using V2 = typename std::conditional<std::is_same<TS, float>::value, float2, double2>::type;
  const TS* QB = (const TS*)a.QB;
  TS* q_out = (TS*)a.q_out;
  TS* comb_out = (TS*)a.comb_out;
  const TS* x_prev = (const TS*)a.x_prev;
  // one-dimensional grid of (hand block, sequence) pairs in hand-block-major
  // order, dealt to the XCDs in contiguous ranges: the blocks of one XCD share
  // hand blocks, so the ancestor rows each sequence multiplies along its path
  // are re-read from that XCD's L2
  const int nbx = (a.ld / 2 + kPassThreads - 1) / kPassThreads;
  const int pos = xcd_spread((int)blockIdx.x, (int)gridDim.x);
  const int s = pos % a.n_seq, hb = pos / a.n_seq;
  const int h = 2 * (hb * kPassThreads + threadIdx.x);  // ld is even: h + 1 < ld too
  if (hb >= nbx || h >= a.ld) return;
  const size_t idx = (size_t)s * a.ld + h;
  const int* path = a.anc + (size_t)s * kMaxDepth;
  V2 f[kMaxDepth];
#pragma unroll
  for (int j = 0; j < kMaxDepth; ++j) {
    const int q = path[j];
    if (q >= 0) {
      f[j] = *(const V2*)(QB + (size_t)q * a.ld + h);
    } else {
      f[j].x = (TS)1;
      f[j].y = (TS)1;
    }
  }
  TS v0 = (TS)1, v1 = (TS)1;
#pragma unroll
  for (int j = 0; j < kMaxDepth; ++j)
    if (path[j] >= 0) {
      v0 *= f[j].x;
      v1 *= f[j].y;
    }
  const bool live0 = h < a.n, live1 = h + 1 < a.n;
  if (q_out) {
    V2 o;
    o.x = live0 ? v0 : (TS)0;
    o.y = live1 ? v1 : (TS)0;
    *(V2*)(q_out + idx) = o;
  }
  if (comb_out) {
    const V2 xp = *(const V2*)(x_prev + idx);
    V2 o;
    o.x = live0 ? (TS)(1.0 - a.tau) * xp.x + (TS)a.tau * v0 : (TS)0;
    o.y = live1 ? (TS)(1.0 - a.tau) * xp.y + (TS)a.tau * v1 : (TS)0;
    *(V2*)(comb_out + idx) = o;
  }
}

// The uniform point: q[s] = q[parent] / n for every sequence s of a node with n
// actions, from the root down along the sequence's root-first path.
struct UniformArgs {
  const int* anc;
  const int* seq_nact;
  int n, ld;
  double* out;
};

__global__ __launch_bounds__(kPassThreads) void uniform_kernel(UniformArgs a) {
  const int h = blockIdx.x * kPassThreads + threadIdx.x;
  const int s = blockIdx.y;
  if (h >= a.ld) return;
  const int* path = a.anc + (size_t)s * kMaxDepth;
  double val = 1.0;
  for (int j = 0; j < kMaxDepth && path[j] >= 0; ++j) val = val / (double)a.seq_nact[path[j]];
  a.out[(size_t)s * a.ld + h] = h < a.n ? val : 0.0;
}

// max |X| into *out, which holds +0.0 beforehand.  |x| >= 0, so the bit
// patterns order as the values do; a NaN (positive after fabs) orders above
// every number and so reaches the result instead of being skipped.
__global__ __launch_bounds__(256) void max_abs_kernel(int64_t count, const double* X, unsigned long long* out) {
  __shared__ unsigned long long wmax[4];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(X[i]));
    m = b > m ? b : m;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
    atomicMax(out, m);
  }
}

__global__ __launch_bounds__(64) void zero_kernel(double* p) {
  if (threadIdx.x == 0) p[0] = 0.0;
}

template <class T>
__global__ __launch_bounds__(256) void axpby_kernel(int64_t count, double a, const T* X, double b, const T* Y,
                                                    T* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const T ta = (T)a, tb = (T)b;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    out[i] = Y ? ta * X[i] + tb * Y[i] : ta * X[i];
}

template <class TI, class TO>
__global__ __launch_bounds__(256) void convert_kernel(int64_t count, const TI* in, TO* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) out[i] = (TO)in[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

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
    t.VB = p[k].VB;
    t.QB = p[k].QB;
    t.g_out = nullptr;
    t.g_scale = 0.0;
    t.n_levels = hp.n_levels;
    t.n_child = (int)hp.child.size();
    for (int l = 0; l <= kMaxDepth; ++l) {
      const int lb = hp.level_begin[std::min(l, hp.n_levels)];
      t.level_begin[l] = lb;
      t.seq_level_begin[l] = lb < hp.n_nodes ? hp.node_first_seq[lb] : hp.n_seq;
    }
  }
}

int n_partials(const egt_game* g) { return g->fused_passes ? g->ld / g->fused_hands : 1; }

size_t fused_lds_bytes(int hands, int cap_tab_bytes, int cap_nodes, int cap_seqs) {
  return (size_t)cap_tab_bytes + sizeof(double) * (3 * (size_t)cap_seqs + (size_t)cap_nodes) * hands;
}

template <class TG>
static hipError_t passes_launch(const egt_game* g, const Pass* p, int count, const Epilogue* epi, double* partial,
                                hipStream_t s) {
  bool any_dual = false;
  for (int k = 0; k < count; ++k) any_dual = any_dual || p[k].VB != nullptr;
  const int n_epi = count;  // epilogues belong to the passes as given
  if (g->fused_passes) {
    const int cap_tab = (int)std::max(g->hp[0].fused_tab.size(), g->hp[1].fused_tab.size());
    const int cap_nodes = std::max(g->hp[0].n_nodes, g->hp[1].n_nodes);
    const int cap_seqs = std::max(g->hp[0].n_seq, g->hp[1].n_seq);
    const size_t dual_lds = sizeof(double) * (size_t)g->fused_hands * ((size_t)cap_seqs + (size_t)cap_nodes);
    // dual passes inside the kernel when every pass is dual, every one is
    // smoothed and the extra LDS fits; otherwise each becomes a second tree
    // with mu = 0 after the others
    bool all_dual = true;
    for (int k = 0; k < count; ++k) all_dual = all_dual && p[k].VB != nullptr && p[k].mu > 0.0;
    const bool in_kernel =
        any_dual && all_dual &&
        fused_lds_bytes(g->fused_hands, cap_tab, cap_nodes, cap_seqs) + dual_lds <= (size_t)g->lds_per_block;
    Pass q[kMaxTrees];
    int nq = 0;
    for (int k = 0; k < count; ++k) {
      q[nq] = p[k];
      if (!in_kernel) q[nq].VB = nullptr;
      ++nq;
    }
    for (int k = 0; any_dual && !in_kernel && k < count; ++k) {
      if (!p[k].VB) continue;
      if (nq >= kMaxTrees) return hipErrorInvalidValue;
      q[nq++] = Pass{p[k].player, p[k].gA, p[k].cA, p[k].gB, p[k].cB, 0.0, p[k].VB, nullptr};
    }
    p = q;
    count = nq;
    FusedArgs a;
    fill_pass_set(g, p, count, a.ps);
    for (int k = 0; k < kMaxTrees; ++k)
      a.epi[k] = (epi && k < n_epi) ? epi[k] : Epilogue{nullptr, nullptr, 0.0, nullptr, nullptr, 0.0};
    a.partial = partial;
    a.cap_tab = (int)std::max(g->hp[0].fused_tab.size(), g->hp[1].fused_tab.size());
    a.cap_nodes = std::max(g->hp[0].n_nodes, g->hp[1].n_nodes);
    a.cap_seqs = std::max(g->hp[0].n_seq, g->hp[1].n_seq);
    const int hb = g->fused_hands;
    const size_t lds = fused_lds_bytes(hb, a.cap_tab, a.cap_nodes, a.cap_seqs) + (in_kernel ? dual_lds : 0);
    a.n_hblocks = g->ld / hb;
    const dim3 grid((unsigned)(a.n_hblocks * count));
    if (hb == 4)
      hipLaunchKernelGGL((sbr_fused_kernel<4, TG>), grid, dim3(kFusedSlots * 4), lds, s, a);
    else
      hipLaunchKernelGGL((sbr_fused_kernel<16, TG>), grid, dim3(kFusedSlots * 16), lds, s, a);
    return hipGetLastError();
  }
  PassSet a;
  fill_pass_set(g, p, count, a);
  for (int k = 0; k < count; ++k) {
    if (epi && (epi[k].q_out || epi[k].comb_out) && !p[k].QB) return hipErrorInvalidValue;
    a.t[k].g_out = epi ? epi[k].g_out : nullptr;
    a.t[k].g_scale = epi ? epi[k].g_scale : 0.0;
  }
  int max_levels = 0;
  for (int k = 0; k < count; ++k) max_levels = std::max(max_levels, a.t[k].n_levels);
  const unsigned bx = (unsigned)((g->n + kPassThreads - 1) / kPassThreads);
  const unsigned bx_pair = (unsigned)(((g->n + 1) / 2 + kPassThreads - 1) / kPassThreads);
  // two hands per lane when every row is 2-element aligned
  bool pair = g->ld % 2 == 0;
  {
    const size_t pb = 2 * (std::is_same<TG, float>::value ? sizeof(float) : sizeof(double));
    auto ok = [&](const void* ptr) { return ((uintptr_t)ptr % pb) == 0; };
    for (int k = 0; k < count; ++k) {
      const TreePass& t = a.t[k];
      pair = pair && ok(t.gA) && ok(t.gB) && ok(t.g_out) && ok(t.QB) && ((uintptr_t)t.V % 16) == 0 &&
             ((uintptr_t)t.VB % 16) == 0;
    }
  }
  // Dual passes: the lowest level takes the best response with the smoothed
  // pass (the same minimum); above it the best responses run as trees of
  // their own (mu = 0, node values in VB, their children's values read from
  // there), after the given ones in the same launches.
  PassSet ax = a;
  if (any_dual) {
    int nx = count;
    for (int k = 0; k < count; ++k) {
      ax.t[k].VB = nullptr;
      if (!p[k].VB) continue;
      if (nx >= kMaxTrees) return hipErrorInvalidValue;
      TreePass& b = ax.t[nx++];
      b = a.t[k];
      b.mu = 0.0;
      b.V = p[k].VB;
      b.VB = nullptr;
      b.QB = nullptr;
      b.g_out = nullptr;
      b.g_scale = 0.0;
    }
    ax.count = nx;
  }
  for (int l = 0; l < max_levels; ++l) {
    PassSet& cur = l == 0 ? a : ax;
    unsigned total = 0;
    for (int k = 0; k < cur.count; ++k) {
      const TreePass& t = cur.t[k];
      cur.level_cnt[k] = l < t.n_levels ? t.level_begin[l + 1] - t.level_begin[l] : 0;
      total += (unsigned)cur.level_cnt[k];
    }
    if (total == 0) continue;
    cur.level = l;
    if (l == 0 && pair) {
      hipLaunchKernelGGL(bottom_up_leaf_pair_kernel<TG>, dim3(bx_pair, total), dim3(kPassThreads), 0, s, a);
    } else if (l == 0) {
      hipLaunchKernelGGL(bottom_up_level_kernel<TG>, dim3(bx, total), dim3(kPassThreads), 0, s, a);
    } else {
      // above the lowest level every node has children: a wavefront per action (at most kInternalWaves)
      int wa = 1;
      for (int k = 0; k < count; ++k)
        if (l < a.t[k].n_levels) wa = std::max(wa, g->hp[p[k].player].level_max_act[l]);
      wa = std::min(wa, kInternalWaves);  // a wavefront takes actions j, j + wa, ... beyond that
      // two hands per lane only where the level fills the chip several times
      // over; a narrow level is latency-bound and gains from more lanes
      if (pair && (size_t)bx * total >= 4 * (size_t)g->n_cu)
        hipLaunchKernelGGL((bottom_up_internal_kernel<TG, 2>), dim3(bx_pair, total), dim3(kPassThreads, wa), 0, s, ax);
      else
        hipLaunchKernelGGL((bottom_up_internal_kernel<TG, 1>), dim3(bx, total), dim3(kPassThreads, wa), 0, s, ax);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (partial) {
    hipLaunchKernelGGL(root_sums_kernel, dim3(ax.count), dim3(256), 0, s, ax, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int k = 0; epi && k < count; ++k) {
    if (!epi[k].q_out && !epi[k].comb_out) continue;
    const hipError_t e = launch_top_down(g, p[k].player, p[k].QB, epi[k].q_out, epi[k].x_prev, epi[k].tau,
                                         epi[k].comb_out, s, std::is_same<TG, float>::value ? kF32 : kF64);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_passes(const egt_game* g, const Pass* p, int count, const Epilogue* epi, double* partial,
                         hipStream_t s, Prec prec) {
  if (count < 1 || count > kMaxTrees) return hipErrorInvalidValue;
  return prec == kF32 ? passes_launch<float>(g, p, count, epi, partial, s)
                      : passes_launch<double>(g, p, count, epi, partial, s);
}

hipError_t launch_sum_partials(const egt_game* g, const double* partial, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, partial, count, n_partials(g), out);
  return hipGetLastError();
}

hipError_t launch_top_down(const egt_game* g, int player, const void* QB, void* q_out, const void* x_prev,
                           double tau, void* comb_out, hipStream_t s, Prec prec) {
  DownArgs a;
  a.anc = g->dp[player].anc;
  a.QB = QB;
  a.n = g->n;
  a.ld = g->ld;
  a.q_out = q_out;
  a.x_prev = x_prev;
  a.tau = tau;
  a.comb_out = comb_out;
  a.n_seq = g->dp[player].n_seq;
  if (a.n_seq == 0) return hipSuccess;
  const size_t pair_bytes = prec == kF32 ? 8 : 16;
  auto aligned = [&](const void* ptr) { return ((uintptr_t)ptr % pair_bytes) == 0; };
  if (g->ld % 2 == 0 && aligned(QB) && aligned(q_out) && aligned(x_prev) && aligned(comb_out)) {
    const dim3 grid((unsigned)((g->ld / 2 + kPassThreads - 1) / kPassThreads) * (unsigned)g->dp[player].n_seq);
    if (prec == kF32)
      hipLaunchKernelGGL(top_down_pair_kernel<float>, grid, dim3(kPassThreads), 0, s, a);
    else
      hipLaunchKernelGGL(top_down_pair_kernel<double>, grid, dim3(kPassThreads), 0, s, a);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((g->ld + kPassThreads - 1) / kPassThreads), g->dp[player].n_seq);
  if (prec == kF32)
    hipLaunchKernelGGL(top_down_kernel<float>, grid, dim3(kPassThreads), 0, s, a);
  else
    hipLaunchKernelGGL(top_down_kernel<double>, grid, dim3(kPassThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_uniform(const egt_game* g, int player, double* out, hipStream_t s) {
  UniformArgs a;
  a.anc = g->dp[player].anc;
  a.seq_nact = g->dp[player].seq_nact;
  a.n = g->n;
  a.ld = g->ld;
  a.out = out;
  if (g->dp[player].n_seq == 0) return hipSuccess;
  const unsigned bx = (unsigned)((g->ld + kPassThreads - 1) / kPassThreads);
  hipLaunchKernelGGL(uniform_kernel, dim3(bx, g->dp[player].n_seq), dim3(kPassThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t count, double a, const void* X, double b, const void* Y, void* out, hipStream_t s,
                        Prec prec) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
  if (prec == kF32)
    hipLaunchKernelGGL(axpby_kernel<float>, dim3(blocks), dim3(256), 0, s, count, a, (const float*)X, b,
                       (const float*)Y, (float*)out);
  else
    hipLaunchKernelGGL(axpby_kernel<double>, dim3(blocks), dim3(256), 0, s, count, a, (const double*)X, b,
                       (const double*)Y, (double*)out);
  return hipGetLastError();
}

hipError_t launch_convert(int64_t count, const void* in, Prec in_prec, void* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
  if (in_prec == kF32)
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(blocks), dim3(256), 0, s, count, (const float*)in,
                       (double*)out);
  else
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(blocks), dim3(256), 0, s, count, (const double*)in,
                       (float*)out);
  return hipGetLastError();
}

hipError_t launch_max_abs(int64_t count, const double* X, double* out, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, out);
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 2048));
  hipLaunchKernelGGL(max_abs_kernel, dim3(blocks), dim3(256), 0, s, count, X, (unsigned long long*)out);
  return hipGetLastError();
}

}  // namespace egt
