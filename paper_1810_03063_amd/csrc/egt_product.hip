// Payoff products A y and A^T x (Section 2's gradient operators) on the fold
// and showdown terminals of a river endgame, O(n) per terminal, for gfx950;
// for a general game, a CSR SpMV over the explicit operator.
//
// For a terminal z with opponent sequence sigma_o(z) the opponent's reach is
// r(h') = b_o(h') v_o[sigma_o(z)][h'] over the strength-ordered hands, and
//   fold:     sum of r over hands compatible with h = T - C[a] - C[b] + r(h)
//             (T the total, C[c] the mass of the hands holding card c; hand h
//             holds both of its cards, so it is removed twice and added back);
//   showdown: (compatible mass stronger) - (compatible mass weaker): the
//             weaker mass is the exclusive prefix over strength order at the
//             start of h's tie group minus, per card of h, the exclusive
//             prefix over the strength-ordered hands holding that card; the
//             stronger mass mirrors it from the end of the tie group; hands of
//             the tie group count as neither.
// out[s][h] = b_own(h) / Z * sum over the terminals z at s of u(z) op_z(h),
// the showdown op negated for player 2 (W^T = -W).
//
// A block holds one or two wave groups of 256 threads; a group evaluates one
// terminal per round.  A round:
//   1. stage: each thread writes the reach of its strided hands into R (the
//      strength order) and into the hand's two slots of E, the card lists laid
//      end to end (card c's strength-ordered hands, then one slot for its
//      total), so every card list is contiguous in LDS;
//   2. the per-card exclusive prefixes, in place in E (four lanes per card,
//      each a contiguous quarter of the list, the quarter offsets added in a
//      fixed order), and beside them the strength-order scan of the group;
//   3. the exclusive strength prefix written in place over R;
//   4. every thread evaluates its contiguous hands from its own 16-byte
//      per-hand table of indices into R and E (kept in registers).
// While a round runs, the opponent row of the group's next round is already
// being loaded into registers, and the terminal record of the round after.  When blocks loop over many sequences they walk
// work items (TermItem): two-terminal sequences whole (one terminal per group,
// the two results added), one-terminal sequences in pairs (one per group).
// Every sum is taken in a fixed order, so results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "egt_internal.h"

namespace egt {

namespace {

constexpr int kGroupThreads = 256;  // one wave group evaluates one terminal per round
constexpr int kQR = 12;             // card-list quarters up to this long stay in registers

// A double moved across lanes by a DPP control (VALU, no LDS round trip);
// lanes whose source is out of range or whose row is masked get 0.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Inclusive scan over the 64 lanes of a wavefront (every lane active): within
// each row of 16 lanes by shifts of 1, 2, 4, 8, then each row's total carried
// to the rows after it (row broadcasts of lanes 15 and 31).  The additions are
// fixed, so the result is repeatable.
__device__ inline double wave_inclusive_scan(double x) {
  x += dpp_move<0x111, 0xf>(x);  // row_shr:1
  x += dpp_move<0x112, 0xf>(x);  // row_shr:2
  x += dpp_move<0x114, 0xf>(x);  // row_shr:4
  x += dpp_move<0x118, 0xf>(x);  // row_shr:8
  x += dpp_move<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

template <class TV, class TO>
struct ProdArgs {
  DPlayer own;
  const double* b_opp;
  DHands H;
  const TV* v_opp;
  TO* out;
  double show_sign;
  int groups;
  const TermItem* items;   // work items instead of whole sequences, or null
  int n_items;
};

// HPT = hands per thread (n <= 256 HPT).  MINW = waves per SIMD the register
// allocation leaves room for (4: two blocks of two groups share a compute unit).
// TAB = the per-hand tables (index table, own prior) staged once per block in
// LDS behind the groups' arrays, which leaves the registers to the staging
// and the accumulators (used when the device's LDS per block allows it).
template <class TV, class TO, int HPT, int MINW, bool TAB>
__global__ __launch_bounds__(2 * kGroupThreads, MINW) void product_kernel(ProdArgs<TV, TO> a) {
  extern __shared__ __align__(16) double lds[];
  __shared__ double wave_total[2][kGroupThreads / 64];
  const int n = a.H.n, ld = a.H.ld, cph = a.H.cph;
  const int groups = a.groups;
  const int rlen = (n + 2) / 2 * 2;            // R: n + 1 doubles, rounded up to keep E 16-byte aligned
  const int per_group = rlen + a.H.n_card_slots;
  const int tid = threadIdx.x;
  const int grp = tid / kGroupThreads, gt = tid % kGroupThreads;
  const int lane = tid & 63, wig = gt >> 6;
  double* R = lds + (size_t)grp * per_group;
  double* E = R + rlen;

  const int MT = a.own.term_stride, n_seq = a.own.n_seq;
  const int chunk = (n + kGroupThreads - 1) / kGroupThreads;
  const int beg = min(gt * chunk, n), end = min(beg + chunk, n), cnt = end - beg;
  const TermRec none{-1, -1, 0.0};
  const bool by_items = a.items != nullptr;
  const int n_work = by_items ? a.n_items : n_seq;
  const int rounds = by_items ? 1 : (MT + groups - 1) / groups;

  // the terminal of (unit w, round rd) for this group, and the row it writes
  auto term_of = [&](int w, int rd, TermRec& t, int& so, bool& comb) {
    if (by_items) {
      const TermItem& it = a.items[w];
      t = it.t[grp];
      so = it.seq[grp];
      comb = it.seq[0] == it.seq[1];
    } else {
      const int j = rd * groups + grp;
      t = j < MT ? a.own.term_rec[(size_t)w * MT + j] : none;
      so = w;
      comb = groups == 2;
    }
  };

  // per-thread constants, kept for every round: the indices of this thread's
  // own hands (16-bit fields: E index of the card-a prefix at the tie group's
  // start and end and of card a's total, the same for card b, then the tie
  // group [glo, ghi) in R), the opponent's prior at the strided hands it
  // stages, and those hands' two slots in E
  uint4 ht[TAB ? 1 : HPT];
  double bown[TAB ? 1 : HPT];
  double bo[HPT];
  unsigned hp[HPT];
  uint4* htab_l = (uint4*)(lds + ((size_t)groups * per_group + 1) / 2 * 2);  // TAB: [n], 16-byte aligned
  double* bown_l = (double*)(htab_l + n);                      // TAB: [n]
  if constexpr (TAB) {
    for (int i = tid; i < n; i += (int)blockDim.x) {
      htab_l[i] = a.H.htab[i];
      bown_l[i] = a.own.belief[i];
    }
  } else {
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      ht[k] = k < cnt ? a.H.htab[beg + k] : make_uint4(0u, 0u, 0u, 0u);
      bown[k] = k < cnt ? a.own.belief[beg + k] : 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int i = gt + k * kGroupThreads;
    bo[k] = i < n ? a.b_opp[i] : 0.0;
    hp[k] = i < n ? a.H.hpos[i] : 0u;
  }
  // this lane's first card list (four lanes per card): start in E and length
  const int c_first = gt >> 2;
  const int cb_first = c_first < a.H.n_cards ? a.H.card_begin[c_first] : 0;
  const int len_first = c_first < a.H.n_cards ? a.H.card_begin[c_first + 1] - cb_first : 0;

  // The rounds of this block, in order: (unit w, round rd).  The terminal
  // records run two rounds ahead and the opponent rows one round ahead of
  // the round being evaluated, so neither load waits on the other.
  auto advance = [&](int& w_, int& rd_) {
    if (++rd_ >= rounds) {
      rd_ = 0;
      w_ += (int)gridDim.x;
    }
  };
  int w = blockIdx.x, rd = 0;
  TermRec tr = none;
  int s_out = -1;
  bool combine = false;
  if (w < n_work) term_of(w, 0, tr, s_out, combine);
  int w1 = w, rd1 = rd;
  advance(w1, rd1);
  TermRec tr1 = none;
  int s1 = -1;
  bool comb1 = false;
  if (w1 < n_work) term_of(w1, rd1, tr1, s1, comb1);
  double vv[HPT];
  auto load_row = [&](const TermRec& t, double* v) {
    const TV* row = t.opp >= 0 ? a.v_opp + (size_t)t.opp * ld : nullptr;
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int i = gt + k * kGroupThreads;
      v[k] = (row && i < n) ? (double)row[i] : 1.0;
    }
  };
  load_row(tr, vv);

  double acc[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) acc[k] = 0.0;
  while (w < n_work) {
    // uniform within a group
    const bool active = tr.kind >= 0;
    const int kind = tr.kind;
    const double coef = tr.coef;
    // 1. stage the reach into R (strength order) and E (card lists)
    if (active) {
#pragma unroll
      for (int k = 0; k < HPT; ++k) {
        const int i = gt + k * kGroupThreads;
        if (i < n) {
          const double r = bo[k] * vv[k];
          R[i] = r;
          E[hp[k] & 0xffffu] = r;
          if (cph == 2) E[hp[k] >> 16] = r;
        }
      }
    }
    // the next round's row, and the terminal two rounds ahead, loaded while this round runs
    load_row(tr1, vv);
    int w2 = w1, rd2 = rd1;
    advance(w2, rd2);
    TermRec tr2 = none;
    int s2 = -1;
    bool comb2 = false;
    if (w2 < n_work) term_of(w2, rd2, tr2, s2, comb2);
    __syncthreads();

    double rloc[HPT];
    double local = 0.0, incl = 0.0;
    if (active) {
      // 2a. per-card exclusive prefixes in place over each contiguous list
      const int sub = gt & 3;
      for (int c = c_first; c - c_first < a.H.n_cards; c += kGroupThreads / 4) {
        const bool valid = c < a.H.n_cards;
        const bool first = c == c_first;
        const int cb = first ? cb_first : valid ? a.H.card_begin[c] : 0;
        const int len = first ? len_first : valid ? a.H.card_begin[c + 1] - cb : 0;
        double* L = E + cb + c;
        const int qlen = (len + 3) >> 2;
        const int lo = min(sub * qlen, len), hi = min(lo + qlen, len);
        // the card's four lanes form an aligned quad: the quarter totals
        // cross lanes by DPP quad permutes
        if (qlen <= kQR) {  // uniform over the quad: the quarter stays in registers
          double v[kQR];
          double part = 0.0;
#pragma unroll
          for (int j = 0; j < kQR; ++j) v[j] = lo + j < hi ? L[lo + j] : 0.0;
#pragma unroll
          for (int j = 0; j < kQR; ++j)
            if (lo + j < hi) part += v[j];
          const double p0 = dpp_move<0x00, 0xf>(part), p1 = dpp_move<0x55, 0xf>(part), p2 = dpp_move<0xaa, 0xf>(part);
          double run = sub == 0 ? 0.0 : sub == 1 ? p0 : sub == 2 ? p0 + p1 : (p0 + p1) + p2;
#pragma unroll
          for (int j = 0; j < kQR; ++j) {
            if (lo + j < hi) {
              L[lo + j] = run;
              run += v[j];
            }
          }
          if (valid && sub == 3) L[len] = run;
        } else {  // long lists: two passes over the quarter in batches of kQ
          constexpr int kQ = 4;
          double part = 0.0;
          for (int k0 = lo; k0 < hi; k0 += kQ) {
            double v[kQ];
#pragma unroll
            for (int j = 0; j < kQ; ++j) v[j] = k0 + j < hi ? L[k0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < kQ; ++j)
              if (k0 + j < hi) part += v[j];
          }
          const double p0 = dpp_move<0x00, 0xf>(part), p1 = dpp_move<0x55, 0xf>(part), p2 = dpp_move<0xaa, 0xf>(part);
          double run = sub == 0 ? 0.0 : sub == 1 ? p0 : sub == 2 ? p0 + p1 : (p0 + p1) + p2;
          for (int k0 = lo; k0 < hi; k0 += kQ) {
            double v[kQ];
#pragma unroll
            for (int j = 0; j < kQ; ++j) v[j] = k0 + j < hi ? L[k0 + j] : 0.0;
#pragma unroll
            for (int j = 0; j < kQ; ++j) {
              if (k0 + j < hi) {
                L[k0 + j] = run;
                run += v[j];
              }
            }
          }
          if (valid && sub == 3) L[len] = run;
        }
      }
      // 2b. the strength-order scan of this thread's contiguous hands
#pragma unroll
      for (int k = 0; k < HPT; ++k) rloc[k] = k < cnt ? R[beg + k] : 0.0;
#pragma unroll
      for (int k = 0; k < HPT; ++k) local += rloc[k];
      incl = wave_inclusive_scan(local);
      if (lane == 63) wave_total[grp][wig] = incl;
    }
    __syncthreads();
    // 3. exclusive strength prefix in place over R, R[n] = total
    if (active) {
      double run = incl - local;
      for (int q = 0; q < wig; ++q) run += wave_total[grp][q];
#pragma unroll
      for (int k = 0; k < HPT; ++k) {
        if (k < cnt) {
          R[beg + k] = run;
          run += rloc[k];
        }
      }
      if (cnt > 0 && end == n) R[n] = run;
    }
    __syncthreads();
    // 4. evaluate this thread's hands
    if (active) {
      const double T = R[n];
#pragma unroll
      for (int k = 0; k < HPT; ++k) {
        if (k < cnt) {
          const uint4 t = TAB ? htab_l[beg + k] : ht[k];
          double op;
          if (kind == 0) {
            op = T - E[t.y & 0xffffu];
            if (cph == 2) op = op - E[t.z >> 16] + rloc[k];
          } else {
            double weaker = R[t.w & 0xffffu] - E[t.x & 0xffffu];
            double stronger = (T - R[t.w >> 16]) - (E[t.y & 0xffffu] - E[t.x >> 16]);
            if (cph == 2) {
              weaker -= E[t.y >> 16];
              stronger -= E[t.z >> 16] - E[t.z & 0xffffu];
            }
            op = a.show_sign * (stronger - weaker);
          }
          acc[k] += coef * op;
        }
      }
    }
    // the unit's last round: combine the two groups' results and write the row
    if (rd + 1 >= rounds) {
      if (combine) {
        __syncthreads();  // both groups are done reading their R
        if (grp == 1) {
#pragma unroll
          for (int k = 0; k < HPT; ++k)
            if (k < cnt) R[beg + k] = acc[k];
        }
        __syncthreads();
        if (grp == 0) {
          const double* R1 = lds + per_group;
#pragma unroll
          for (int k = 0; k < HPT; ++k)
            if (k < cnt) acc[k] += R1[beg + k];
        }
      }
      if ((!combine || grp == 0) && s_out >= 0) {
        TO* row = a.out + (size_t)s_out * ld;
#pragma unroll
        for (int k = 0; k < HPT; ++k)
          if (k < cnt) row[beg + k] = (TO)(acc[k] * ((TAB ? bown_l[beg + k] : bown[k]) * a.H.invZ));
        for (int i = n + gt; i < ld; i += kGroupThreads) row[i] = (TO)0;
      }
#pragma unroll
      for (int k = 0; k < HPT; ++k) acc[k] = 0.0;
    }
    __syncthreads();  // the next round rewrites R and E of both groups
    w = w1;
    rd = rd1;
    tr = tr1;
    if (rd == 0) {
      s_out = s1;
      combine = comb1;
    }
    w1 = w2;
    rd1 = rd2;
    tr1 = tr2;
    s1 = s2;
    comb1 = comb2;
  }
}

// Precision form, fold terminals only (the BF16 GEMM adds the showdown
// terminals' part afterwards), in FP32: one block per own sequence.  For each
// fold terminal of the sequence the opponent's reach r(h') is staged into the
// card lists E (each hand in the list of each of its cards), the card totals
// C[c] are summed (four lanes per list, a quarter each, the quarters added in
// a fixed order) into the list's total slot, the total T is summed (each
// thread's hands, then the wavefronts in order), and
//   op(h) = T - C[a] - C[b] + r(h)      (hand h holds cards a and b)
// is accumulated with the terminal's chips.  The row gets b_own(h)/Z times
// the sum (0 without fold terminals), its padding 0.
struct FoldArgs {
  DPlayer own;
  const double* b_opp;
  DHands H;
  const float* v_opp;
  float* out;
};

template <int HPT>
__global__ __launch_bounds__(kGroupThreads) void fold_kernel(FoldArgs a) {
  extern __shared__ __align__(16) float E[];  // [n_card_slots]
  __shared__ float wtot[kGroupThreads / 64];
  const int s = (int)blockIdx.x;
  const int n = a.H.n, ld = a.H.ld, cph = a.H.cph;
  const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int MT = a.own.term_stride;
  float bo[HPT], acc[HPT];
  unsigned hp[HPT], tot[HPT];  // the hand's E slots; E slots of its cards' totals (16 bits each)
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int i = tid + k * kGroupThreads;
    acc[k] = 0.0f;
    bo[k] = i < n ? (float)a.b_opp[i] : 0.0f;
    hp[k] = i < n ? a.H.hpos[i] : 0u;
    tot[k] = 0u;
    if (i < n) {
      const uint4 t = a.H.htab[i];
      tot[k] = (t.y & 0xffffu) | (t.z & 0xffff0000u);
    }
  }
  for (int j = 0; j < MT; ++j) {
    const TermRec tr = a.own.term_rec[(size_t)s * MT + j];  // uniform over the block
    if (tr.kind != 0) continue;
    const float* row = tr.opp >= 0 ? a.v_opp + (size_t)tr.opp * ld : nullptr;
    float r[HPT];
    float loc = 0.0f;
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int i = tid + k * kGroupThreads;
      r[k] = i < n ? bo[k] * (row ? row[i] : 1.0f) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int i = tid + k * kGroupThreads;
      if (i < n) {
        E[hp[k] & 0xffffu] = r[k];
        if (cph == 2) E[hp[k] >> 16] = r[k];
      }
      loc += r[k];
    }
    for (int off = 32; off > 0; off >>= 1) loc += __shfl_xor(loc, off, 64);
    if (lane == 0) wtot[wv] = loc;
    __syncthreads();
    // card totals into each list's total slot
    for (int c0 = 0; c0 < a.H.n_cards; c0 += kGroupThreads / 4) {
      const int c = c0 + (tid >> 2), sub = tid & 3;
      const bool valid = c < a.H.n_cards;
      const int cb = valid ? a.H.card_begin[c] : 0;
      const int len = valid ? a.H.card_begin[c + 1] - cb : 0;
      float* L = E + cb + c;
      const int qlen = (len + 3) >> 2;
      const int lo = min(sub * qlen, len), hi = min(lo + qlen, len);
      float part = 0.0f;
      for (int k = lo; k < hi; ++k) part += L[k];
      const int q0 = lane & ~3;
      const float p0 = __shfl(part, q0, 64), p1 = __shfl(part, q0 + 1, 64), p2 = __shfl(part, q0 + 2, 64),
                  p3 = __shfl(part, q0 + 3, 64);
      if (valid && sub == 0) L[len] = ((p0 + p1) + p2) + p3;  // the total slot follows the list
    }
    const float T = ((wtot[0] + wtot[1]) + wtot[2]) + wtot[3];
    __syncthreads();
    const float coef = (float)tr.coef;
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
      const int i = tid + k * kGroupThreads;
      if (i < n) {
        float op = T - E[tot[k] & 0xffffu];
        if (cph == 2) op = (op - E[tot[k] >> 16]) + r[k];
        acc[k] += coef * op;
      }
    }
    __syncthreads();  // the next terminal restages E
  }
  float* out = a.out + (size_t)s * ld;
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int i = tid + k * kGroupThreads;
    if (i < n) out[i] = acc[k] * (float)(a.own.belief[i] * a.H.invZ);
  }
  for (int i = n + tid; i < ld; i += kGroupThreads) out[i] = 0.0f;
}

size_t align2(size_t x) { return (x + 1) / 2 * 2; }

// General games (Section 6's explicit sparse operator): one wavefront per CSR
// row; lane l takes the row's entries l, l + 64, ... in column order, then a
// fixed xor butterfly (every lane ends with the same sum); the row's slot 0
// gets the sum and its padding slots 1 .. ld - 1 are written 0.
__global__ __launch_bounds__(256) void spmv_kernel(const int64_t* ptr, const int* col, const double* val,
                                                   const double* v, int ld, int n_rows, double* out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n_rows) return;
  const int64_t k0 = ptr[row], k1 = ptr[row + 1];
  double acc = 0.0;
  for (int64_t k = k0 + lane; k < k1; k += 64) acc += val[k] * v[(size_t)col[k] * ld];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  double* o = out + (size_t)row * ld;
  for (int i = lane; i < ld; i += 64) o[i] = i == 0 ? acc : 0.0;
}

}  // namespace

hipError_t launch_spmv(const egt_game* g, int player, const double* v_opp, double* grad_out, hipStream_t s) {
  const DPlayer& P = g->dp[player];
  if (!g->general || !P.sp_ptr) return hipErrorInvalidValue;
  if (P.n_seq == 0) return hipSuccess;
  hipLaunchKernelGGL(spmv_kernel, dim3((unsigned)((P.n_seq + 3) / 4)), dim3(256), 0, s, P.sp_ptr, P.sp_col, P.sp_val,
                     v_opp, g->ld, P.n_seq, grad_out);
  return hipGetLastError();
}

// Doubles of LDS one wave group of the product kernel takes.
size_t product_group_doubles(const egt_game* g) { return align2((size_t)g->n + 1) + (size_t)g->dh.n_card_slots; }
// Bytes of the per-hand tables the kernel can stage in LDS (16-byte index table, own prior).
size_t product_table_bytes(const egt_game* g) { return (16 + 8) * (size_t)g->n; }

template <class TV, class TO>
static hipError_t product_launch(const egt_game* g, int player, const TV* v_opp, TO* grad_out, hipStream_t s) {
  ProdArgs<TV, TO> a;
  a.own = g->dp[player];
  a.b_opp = g->dp[1 - player].belief;
  a.H = g->dh;
  a.v_opp = v_opp;
  a.out = grad_out;
  a.show_sign = player == 0 ? 1.0 : -1.0;
  a.items = nullptr;
  a.n_items = 0;
  // two blocks per compute unit: each takes at most half of the CU's LDS
  const size_t budget = (size_t)g->lds_per_cu / 2;
  auto lds_bytes = [&](int gr) { return sizeof(double) * align2(gr * product_group_doubles(g)); };
  int groups = g->hp[player].max_terms_per_seq >= 2 ? 2 : 1;
  if (groups == 2 && lds_bytes(2) > std::min(budget, (size_t)g->lds_per_block)) groups = 1;
  a.groups = groups;
  const bool tab = lds_bytes(groups) + product_table_bytes(g) <= std::min(budget, (size_t)g->lds_per_block);
  const size_t lds = lds_bytes(groups) + (tab ? product_table_bytes(g) : 0);
  // one block per sequence up to two blocks per compute unit; beyond that each
  // block loops over work items that keep both groups busy
  const bool looping = g->dp[player].n_seq > g->n_cu;
  if (looping && groups == 2 && g->dp[player].term_items) {
    a.items = g->dp[player].term_items;
    a.n_items = g->dp[player].n_items;
  }
  const int units = a.items ? a.n_items : g->dp[player].n_seq;
  if (units == 0) return hipSuccess;
  const int blocks = std::min(units, 2 * g->n_cu);
  const dim3 grid(blocks), block(kGroupThreads * groups);
  if (g->n <= 2 * kGroupThreads) {
    if (tab)
      hipLaunchKernelGGL((product_kernel<TV, TO, 2, 4, true>), grid, block, lds, s, a);
    else
      hipLaunchKernelGGL((product_kernel<TV, TO, 2, 4, false>), grid, block, lds, s, a);
  } else if (g->n <= 5 * kGroupThreads) {
    if (tab)
      hipLaunchKernelGGL((product_kernel<TV, TO, 5, 4, true>), grid, block, lds, s, a);
    else
      hipLaunchKernelGGL((product_kernel<TV, TO, 5, 4, false>), grid, block, lds, s, a);
  } else {
    if (tab)
      hipLaunchKernelGGL((product_kernel<TV, TO, 8, 2, true>), grid, block, lds, s, a);
    else
      hipLaunchKernelGGL((product_kernel<TV, TO, 8, 2, false>), grid, block, lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_gradient(const egt_game* g, int player, const double* v_opp, double* grad_out, hipStream_t s) {
  if (g->general) return launch_spmv(g, player, v_opp, grad_out, s);
  return product_launch<double, double>(g, player, v_opp, grad_out, s);
}

hipError_t launch_gradient_fold_f32(const egt_game* g, int player, const float* v_opp, float* grad_out,
                                    hipStream_t s) {
  if (g->general) return hipErrorInvalidValue;  // the precision form is river-only
  const DPlayer& P = g->dp[player];
  if (P.n_seq == 0) return hipSuccess;
  FoldArgs a;
  a.own = P;
  a.b_opp = g->dp[1 - player].belief;
  a.H = g->dh;
  a.v_opp = v_opp;
  a.out = grad_out;
  const size_t lds = sizeof(float) * (size_t)g->dh.n_card_slots;
  const dim3 grid((unsigned)P.n_seq), block(kGroupThreads);
  if (g->n <= 2 * kGroupThreads)
    hipLaunchKernelGGL(fold_kernel<2>, grid, block, lds, s, a);
  else if (g->n <= 5 * kGroupThreads)
    hipLaunchKernelGGL(fold_kernel<5>, grid, block, lds, s, a);
  else
    hipLaunchKernelGGL(fold_kernel<8>, grid, block, lds, s, a);
  return hipGetLastError();
}

}  // namespace egt
