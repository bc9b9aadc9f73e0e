// Internal declarations of libegt: device tables, kernel argument blocks and
// launchers.  Not part of the public ABI (include/egt.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "egt.h"

namespace egt {

constexpr int kMaxActions = 16;  // actions per decision node
constexpr int kMaxDepth = 16;    // sequences on a root-to-leaf chain of one player (and levels)
constexpr int kMaxTrees = 4;     // trees evaluated by one bottom-up launch
constexpr size_t kFusedLdsLimit = 64 * 1024;  // LDS budget of one single-launch pass block

// Table image of one player's treeplex for the single-launch pass, staged
// into LDS verbatim with 16-byte copies:
//   rec  int4[N]    {first sequence, number of actions, value slot, 0}
//   prm  double4[N] {beta, 1 / beta, log(number of actions), 0}
//   cbeg int[S + 1] child-slot range of each sequence (CSR over child nodes)
//   spar int[S]     parent sequence (-1 at a root node)
// A node's value slot is its position in the child CSR; the r-th root node
// takes slot C + r (C = number of non-root nodes), so a sequence's children
// occupy the contiguous slots [cbeg[s], cbeg[s + 1]).
struct FusedTabLayout {
  int rec, prm, cbeg, spar, bytes;
};
__host__ __device__ inline FusedTabLayout fused_tab_layout(int n_nodes, int n_seq) {
  FusedTabLayout L;
  L.rec = 0;
  L.prm = 16 * n_nodes;
  L.cbeg = 48 * n_nodes;
  L.spar = L.cbeg + 4 * ((n_seq + 1 + 3) / 4 * 4);
  L.bytes = L.spar + 4 * ((n_seq + 3) / 4 * 4);
  return L;
}
constexpr int kMaxPartials = 2048 / 4;      // root partial sums per tree (4 hands per block)

// ---------------------------------------------------------------------------
// Error plumbing: every entry point converts failures into a status code and a
// thread-local message.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define EGT_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return ::egt::hip_fail(_e, #call); \
  } while (0)

// ---------------------------------------------------------------------------
// Device-side views (passed by value to kernels).
// ---------------------------------------------------------------------------

// One player's treeplex, in level order: nodes sorted by height (height 1 =
// no own decision below), each node's sequences contiguous.
// One terminal of a sequence's fixed-stride terminal list: the opponent's
// last sequence (-1 = empty), the kind (0 fold, 1 showdown, -1 = no terminal)
// and player 2's chips there (times the sign at a showdown).
struct TermRec {
  int opp;
  int kind;
  double coef;
};

// One work item of the product kernel when its blocks loop over many
// sequences: one (sequence, terminal) pair per wave group; seq -1 = none.  A
// sequence with two terminals is one item whose two results are added (the
// same as its sequence-by-sequence evaluation); sequences with one terminal
// are paired, two output rows per item; a sequence without terminals is an
// item that writes its zero row.
struct TermItem {
  TermRec t[2];
  int seq[2];
  int pad[2];
};

struct DPlayer {
  int n_seq;
  int n_nodes;
  int n_roots;
  const int* node_first_seq;   // [n_nodes]
  const int* node_nact;        // [n_nodes]
  const double* node_beta;     // [n_nodes] dilation weight beta_j
  const double* node_logn;     // [n_nodes] log(number of actions)
  const int* seq_parent;       // [n_seq] parent sequence of the sequence's node, -1 at a root
  const int* child_begin;      // [n_seq + 1] CSR: sequence -> child nodes
  const int* child;            // child node ids
  const int* term_begin;       // [n_seq + 1] CSR: sequence -> terminals ending there
  const int* term_opp;         // opponent's last sequence at the terminal (-1 = empty)
  const int* term_kind;        // 0 fold, 1 showdown
  const double* term_coef;     // player 2's chips at the terminal (times the sign at a showdown)
  const int* roots;            // [n_roots] root node ids
  const double* belief;        // [ld] this player's prior in slot order, 0 in the padding
  const void* fused_tab;       // the single-launch pass's table image (FusedTabLayout), 16-byte units
  const int* anc;              // [n_seq][kMaxDepth] sequences on the path root -> s (s last), -1 after
  const TermRec* term_rec;     // [n_seq][term_stride] terminals of each sequence, padded with kind -1
  int term_stride;             // max terminals per sequence (>= 1)
  const TermItem* term_items;  // [n_items] when every sequence has at most two terminals, else null
  int n_items;
  int fused_tab16;             // its size in 16-byte units
  const int* seq_nact;         // [n_seq] number of actions of the sequence's decision node
  // General games: this player's rows of the payoff operator in CSR (A for
  // player 1, A^T for player 2), columns in the opponent's library order.
  const int64_t* sp_ptr;       // [n_seq + 1], or null for a river endgame
  const int* sp_col;
  const double* sp_val;
};

// Hands in strength-ascending slot order, with the card tables the O(n) leaf
// evaluation needs.  The card lists (the strength-ordered slots holding each
// card) are laid end to end, card c's at base_c = card_begin[c] + c followed
// by one slot for its total: n_card_slots slots in all.  For a hand in slot i
// with tie group [glo, ghi) (the slots of equal strength), htab[i] holds
// 16-bit fields
//   x = lo_a | hi_a << 16,  y = tot_a | lo_b << 16,  z = hi_b | tot_b << 16,
//   w = glo | ghi << 16,
// where lo_c / hi_c are the E indices of the first hand of card c's list at or
// after glo / ghi in slot order (so the exclusive per-card prefix there is the
// mass of card c's hands below the tie group / up to its end), tot_c is the E
// index of card c's total, and hpos[i] = pos_a | pos_b << 16 are the E indices
// of i's own entries in the two lists.  Card b's fields are 0 for one-card
// hands.
struct DHands {
  int n;
  int ld;
  int cph;
  int n_cards;
  int n_card_slots;            // card_begin[n_cards] + n_cards
  const int* card_begin;       // [n_cards + 1]
  const uint4* htab;           // [n]
  const unsigned* hpos;        // [n]
  double invZ;                 // 1 / sum of b1 b2 over compatible deals
};

// One bottom-up pass over one player's treeplex on the gradient
// cA gA + cB gB (gB may be null): smoothed (mu > 0, writing q_bar to QB when
// QB != null) or best response (mu == 0).  Node values go to V.
struct TreePass {
  DPlayer P;
  const void* gA;  // double or float, per the launch's precision
  double cA;
  const void* gB;
  double cB;
  double mu;
  double* V;       // node values by value slot (FusedTabLayout): always FP64
  double* VB;      // dual pass: also the best response's node values (the level path's lowest level, or the
                   // whole single-launch pass), or null
  void* QB;        // q_bar in the launch's precision
  void* g_out;     // g_scale (cA gA + cB gB), or null (the epilogue's g_out)
  double g_scale;
  int n_levels;
  int n_child;
  int level_begin[kMaxDepth + 1];
  int seq_level_begin[kMaxDepth + 1];  // first sequence of each level's nodes (n_seq past the end)
};

// Up to kMaxTrees independent passes evaluated by the same launches.
struct PassSet {
  TreePass t[kMaxTrees];
  int count;
  int n, ld;
  int level;                  // per-level kernel: the level of this launch
  int level_cnt[kMaxTrees];   // per-level kernel: nodes of each tree at `level`
};

// Top-down epilogue of a smoothed best response: q_out = q (may be null) and
// comb_out = (1 - tau) x_prev + tau q (may be null).
struct Epilogue {
  void* q_out;
  const void* x_prev;
  double tau;
  void* comb_out;
  void* g_out;     // single-launch pass only: g_scale (cA gA + cB gB) of this tree, or null
  double g_scale;
  void* qb_out = nullptr;  // single-launch pass only: the local strategies q_bar (before the top-down), or null
};

// Host description of one pass (player instead of device tables).  With VB
// the pass is dual: besides its smoothed values it yields the best response
// (mu = 0) to the same gradient, node values in VB; a launch of `count` passes
// then returns the dual passes' best-response values after the `count`
// smoothed ones, in pass order.
struct Pass {
  int player;
  const void* gA;
  double cA;
  const void* gB;
  double cB;
  double mu;
  double* V;
  void* QB;
  double* VB = nullptr;
};

// Element type of the gradients, q_bar and strategies of a launch: FP64, or
// FP32 for the precision form (node values and normalisers stay FP64).
enum Prec { kF64 = 0, kF32 = 1 };

// ---------------------------------------------------------------------------
// Host-side tables kept with a game.
// ---------------------------------------------------------------------------
struct HostPlayer {
  int n_seq = 0, n_nodes = 0, n_levels = 0, max_chain = 0, max_terms_per_seq = 0, max_level_width = 0;
  int n_show_cols = 0;  // showdown columns of the precision form (set when its tables are built)
  std::vector<int> node_first_seq, node_nact, node_level;
  std::vector<double> node_beta, node_logn;
  std::vector<int> level_begin;  // [n_levels + 1]
  std::vector<int> level_max_act;  // [n_levels] most actions of a node at each level
  std::vector<int> seq_parent, child_begin, child;
  std::vector<int> term_begin, term_opp, term_kind;
  std::vector<double> term_coef;
  std::vector<int> roots;
  std::vector<unsigned char> fused_tab;  // table image of the single-launch pass
  std::vector<TermRec> term_rec;         // [n_seq][max(1, max_terms_per_seq)]
  std::vector<TermItem> term_items;      // work items of the looping product kernel (at most two terminals each)
  std::vector<int> anc;                  // [n_seq][kMaxDepth]
  std::vector<int> seq_nact;             // [n_seq] actions of the sequence's node
  std::vector<std::string> seq_keys;
  std::vector<int64_t> sp_ptr;           // general games: CSR rows of A (player 1) or A^T (player 2)
  std::vector<int> sp_col;
  std::vector<double> sp_val;
  int64_t sp_max_row = 0;                // most entries of one row
};

struct DeviceBlock {  // one device allocation holding many tables
  void* base = nullptr;
  size_t bytes = 0;
};

// Offsets of every table in a game's upload image.
struct GameOffsets {
  struct Player {
    size_t first, nact, beta, logn, spar, cbeg, child, tbeg, topp, tkind, tcoef, roots, belief, ftab, trec, anc,
        titems, snact, sptr, scol, sval;
  } p[2];
  size_t cbeg, htab, hpos;
};

// Scratch of the single-operation entry points (egt_smoothed_br,
// egt_best_response, egt_saddle_gap): per player a gradient, a q_bar and a
// node-value buffer, plus device scalars.  Allocated on first use, owned by
// the game.
struct Workspace {
  void* block = nullptr;
  double* grad[2] = {};
  double* qb[2] = {};
  double* v[2] = {};
  double* scal = nullptr;
  double* hscal = nullptr;  // pinned host mirror of scal
};

// Precision-form tables (built on first use): W in BF16 bits over the slot
// order, padded to kpad x kpad, and per player the showdown columns.
struct MixedTables {
  void* block = nullptr;
  bool owned = true;  // false: the block lies in a serving batch's arena
  int kpad = 0;
  const unsigned short* W = nullptr;
  int L[2] = {0, 0};
  const int* col_own[2] = {nullptr, nullptr};
  const int* col_opp[2] = {nullptr, nullptr};
  const double* col_coef[2] = {nullptr, nullptr};
  const float* belief32[2] = {nullptr, nullptr};  // [ld] each player's prior in FP32
};

}  // namespace egt

struct egt_game {
  int n = 0, ld = 0, cph = 0, n_cards = 0;
  int n_cu = 256;  // compute units of the game's device
  int lds_per_block = 64 * 1024;  // the device's largest LDS allocation of one block
  int lds_per_cu = 64 * 1024;     // LDS of one compute unit
  double pot = 0, stack = 0, Z = 0;
  int64_t n_fold = 0, n_show = 0;
  egt::HostPlayer hp[2];
  std::vector<int> perm;  // slot -> caller hand index
  std::vector<int> slot_cards, slot_strength;  // cards [n * cph] and strengths [n] in slot order
  std::vector<double> hbelief[2];              // priors in slot order, [ld]
  egt::DPlayer dp[2];
  egt::DHands dh;
  egt::DeviceBlock mem;
  bool owns_mem = true;            // false: mem lies in a serving batch's arena
  std::vector<unsigned char> img;  // the tables' upload image
  egt::GameOffsets offs;
  egt::Workspace ws;
  egt::MixedTables mx;
  int device = 0;
  double max_beta = 0;
  bool general = false;       // a general game (egt_build_general_game): CSR products, one live slot
  bool fused_passes = false;  // both treeplexes' tables fit one block's LDS: single-launch passes
  int fused_hands = 4;        // hands per block of the single-launch pass (4 or 16)
};

namespace egt {

// ---------------------------------------------------------------------------
// Launchers (egt_kernels.hip).  All enqueue on `s` and return hipError_t.
// ---------------------------------------------------------------------------

// grad_out = A v_opp (player 0) or A^T v_opp (player 1); general games take
// the CSR product (launch_spmv).
hipError_t launch_spmv(const egt_game* g, int player, const double* v_opp, double* grad_out, hipStream_t s);
hipError_t launch_gradient(const egt_game* g, int player, const double* v_opp, double* grad_out,
                           hipStream_t s);

// count (1..kMaxTrees) independent passes in as few launches as possible:
// bottom-up over every level; when `partial` is not null, the tree values as
// n_partials(g) partial sums per tree (partial[k * n_partials + b], to be
// added in order of b; partial may be the device address of pinned host
// memory, read after the stream is synchronised); when epi[k] asks for it,
// the top-down rebuild of tree k's strategy with its epilogue.  On the level
// path a smoothed pass with an epilogue needs its QB buffer, and g_out is not
// produced.
hipError_t launch_passes(const egt_game* g, const Pass* p, int count, const Epilogue* epi, double* partial,
                         hipStream_t s, Prec prec = kF64);
int n_partials(const egt_game* g);
size_t fused_lds_bytes(int hands, int cap_tab_bytes, int cap_nodes, int cap_seqs);

// out[k] = sum of the n_partials(g) partials of tree k, in order.
hipError_t launch_sum_partials(const egt_game* g, const double* partial, int count, double* out, hipStream_t s);

// Top-down pass: q = product of q_bar along the sequence's chain.  Writes q to
// q_out (may be null) and (1 - tau) x_prev + tau q to comb_out (may be null).
hipError_t launch_top_down(const egt_game* g, int player, const void* QB, void* q_out, const void* x_prev,
                           double tau, void* comb_out, hipStream_t s, Prec prec = kF64);

// The uniform point x_omega: every sequence's mass is its parent's divided by
// the number of actions of its node (written 0 in the row padding).
hipError_t launch_uniform(const egt_game* g, int player, double* out, hipStream_t s);

// out = a * X + b * Y over count elements (Y may be null).
hipError_t launch_axpby(int64_t count, double a, const void* X, double b, const void* Y, void* out, hipStream_t s,
                        Prec prec = kF64);

// out = in converted FP32 -> FP64 (in_prec kF32) or FP64 -> FP32 (in_prec kF64).
hipError_t launch_convert(int64_t count, const void* in, Prec in_prec, void* out, hipStream_t s);

// Fold part of the product in FP32 for the precision form: like
// launch_gradient, but showdown terminals are skipped (their contribution is
// added by launch_show_gemm) and vectors are FP32.
hipError_t launch_gradient_fold_f32(const egt_game* g, int player, const float* v_opp, float* grad_out,
                                    hipStream_t s);

// Precision form: W and the showdown columns (once per game); the product
// fold part (FP32 O(n)) + showdown part (BF16 hi/lo MFMA GEMM, FP32 output).
int ensure_mixed_tables(const egt_game* g);
// The same tables as a host image (no device work): its size, then the upload
// into caller memory (owned = false: the memory is not the game's to free).
int mixed_tables_image(const egt_game* g, std::vector<unsigned char>& img, size_t off[2][4]);
int mixed_tables_upload(egt_game* g, const std::vector<unsigned char>& img, const size_t off[2][4], void* dev,
                        bool owned, hipStream_t s);
hipError_t launch_show_gemm(const egt_game* g, int player, const float* v_opp, float* grad_out, hipStream_t s);
hipError_t launch_gradient_mixed(const egt_game* g, int player, const float* v_opp, float* grad_out, hipStream_t s);

// out[0] = max |X| over count doubles.
hipError_t launch_max_abs(int64_t count, const double* X, double* out, hipStream_t s);

}  // namespace egt
