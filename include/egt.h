/*
 * egt.h -- C ABI of the MI355X EGT library (libegt.so).
 *
 * The library solves the bilinear saddle-point problem
 *     min_{x in X} max_{y in Y} <x, A y>                   (Section 2, Eq. 2)
 * over the sequence-form strategy polytopes (treeplexes, Section 3) of a
 * two-player poker river endgame, with the excessive gap technique and the
 * dilated entropy distance (Sections 2, 4 and 5).  x belongs to player 1, who
 * acts first and minimises; A holds player 2's payoff (= player 1's loss), with
 * chance weight pi(h1, h2) = b1(h1) b2(h2) [hands disjoint] / Z.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns an int status: EGT_OK (0) or a negative EGT_E* code.
 *   egt_last_error() returns a human-readable message for the calling
 *   thread's last failure.  No C++ exception crosses this boundary.
 * - Strategy and gradient vectors are caller-owned DEVICE pointers of doubles
 *   in the library's canonical layout  v[seq * ld + slot]:
 *     seq  : 0 .. n_seq(player)-1 in the library's sequence order (nodes sorted
 *            by height, a node's actions contiguous); egt_game_layout() gives
 *            each sequence's betting-history key;
 *     slot : 0 .. n_hands-1, hands sorted by ascending strength (ties keep the
 *            caller's order); egt_game_layout() gives slot -> caller hand index;
 *     ld   : leading dimension >= n_hands (a multiple of 32); entries
 *            n_hands .. ld-1 of every row are padding: outputs write 0 there and
 *            inputs ignore them.
 *   Pointers must be 8-byte aligned (256-byte alignment is faster).
 * - Device work is enqueued on the given HIP stream (NULL = the null stream)
 *   and runs asynchronously unless a call says it synchronises.  A game or
 *   state handle must not be used from two threads at once.
 * - Handles (egt_game, egt_state) are opaque and owned by the library.
 */
#ifndef EGT_H
#define EGT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EGT_OK = 0,
  EGT_EINVAL = -1,    /* bad argument: NULL pointer, bad player, shape, mu <= 0 ... */
  EGT_ENOMEM = -2,    /* device or host allocation failed */
  EGT_EDEVICE = -3,   /* a HIP runtime call failed */
  EGT_ENUMERIC = -4,  /* a NaN or infinity appeared in a scalar the driver uses */
  EGT_ENOTCONV = -5,  /* max_iters reached, or the step size fell below its floor */
  EGT_EBUDGET = -6    /* serving: the request does not fit the memory budget */
};

enum { EGT_VARIANT_ALT = 0, EGT_VARIANT_BAL = 1, EGT_VARIANT_AS = 2 };
enum { EGT_PRECISION_FP64 = 0, EGT_PRECISION_MIXED = 1 };

typedef struct egt_game egt_game;
typedef struct egt_state egt_state;

/* Thread-local message describing the calling thread's last error. */
const char* egt_last_error(void);

/* ------------------------------------------------------------------------ */
/* Game construction (the treeplexes of Section 3 and the terminal tables     */
/* that define A).                                                           */
/* ------------------------------------------------------------------------ */

/* Situation-dependent bet sizes: the shape Section 7 gives for the Libratus
 * river abstraction.  For acting player p (0 = player 1) once d bets or raises
 * have been made on the river (d = 0 when not facing a bet, 1 facing the
 * opening bet, 2 facing the first raise, 3 for every later raise):
 *   fracs[p][d][0 .. n_fracs[p][d])  pot fractions (bet f * pot when d = 0,
 *                                    raise to c_opp + f * (pot + to_call) else),
 *   allin[p][d]                      nonzero adds all-in there;
 * open_fold[p] nonzero lets p fold when not facing a bet.  A fold before the
 * opponent has acted gives the opponent a one-action decision "p" (pass)
 * first, so that every terminal follows a sequence of each player and the
 * payoff stays bilinear in the two treeplexes.  HOST memory, read during
 * egt_build_game only. */
typedef struct {
  int32_t n_fracs[2][4];
  const double* fracs[2][4];
  int32_t allin[2][4];
  int32_t open_fold[2];
} egt_bet_abstraction;

/* One river endgame.  All arrays are HOST memory, read during the call only.
 * hand_cards  [n_hands * cards_per_hand] card ids in [0, n_cards); two hands
 *             that share a card cannot be dealt together.
 * strength    [n_hands] larger wins a showdown, equal strengths split the pot.
 * belief[p]   [n_hands] player p's prior over its own hands (>= 0, not all 0).
 * pot         chips in the pot before the river, half from each player.
 * stack       chips each player can still bet.
 * Betting: a player not facing a bet checks or bets bet_fracs[i] * pot (plus
 * all-in if allin != 0); facing a bet it folds, calls, or raises to
 * c_opp + bet_fracs[i] * (pot + to_call) (plus all-in) while fewer than
 * max_raises raises followed the opening bet and the opponent is not all-in.
 * Amounts at or above the stack become all-in; duplicates are dropped.  Check
 * after check, or a call, is a showdown; a fold ends the hand.  With
 * abstraction != NULL the sizes (and the all-in flag) come from it per player
 * and situation instead of bet_fracs / allin; max_raises still applies. */
typedef struct {
  int32_t n_cards;
  int32_t cards_per_hand; /* 1 or 2 */
  int32_t n_hands;
  const int32_t* hand_cards;
  const int32_t* strength;
  const double* belief[2];
  double pot;
  double stack;
  int32_t n_bet_fracs;
  const double* bet_fracs;
  int32_t allin;
  int32_t max_raises;
  const egt_bet_abstraction* abstraction; /* NULL: bet_fracs and allin in every situation */
} egt_game_desc;

/* Validates the description, enumerates the betting tree, builds both
 * players' level-ordered treeplex tables, the per-sequence terminal lists and
 * the strength-sorted hand tables, and uploads them to the current device.
 * Synchronises `stream`.  EGT_EINVAL on a bad description (n_hands < 1,
 * cards_per_hand not 1 or 2, a card id out of range, a node with more than 16
 * actions, all-zero beliefs or no compatible deal). */
int egt_build_game(const egt_game_desc* desc, hipStream_t stream, egt_game** out);

/* A general two-player zero-sum extensive-form game in sequence form
 * (Section 3's treeplexes, Definition 2; Section 6's route through an
 * explicit sparse payoff matrix).  All arrays are HOST memory, read during
 * the call only.
 * n_infosets[p]         player p's information sets (simplexes), >= 1.
 * parent_seq[p][k]      the sequence leading to information set k, -1 for the
 *                       empty sequence; it must belong to an earlier set.
 * n_actions[p][k]       1 .. 16.  Player p's sequences are numbered set by
 *                       set: set k owns first_k .. first_k + n_actions - 1,
 *                       first_k = the sum of the earlier sets' n_actions.
 * a_row, a_col, a_val   nnz triples (player-1 sequence, player-2 sequence,
 *                       value) of A = player 2's expected payoff (player 1's
 *                       loss), chance folded in; repeated pairs add up.
 * scale                 payoff scale (> 0): egt_solve's default target gap
 *                       is 1e-3 * scale.
 * The game runs with one live slot per row (n_hands = 1) through every
 * FP64 entry point; the products use a CSR SpMV instead of the river
 * kernels.  The precision form and serving admission by description are
 * river-only (EGT_EINVAL).  Layout keys are the caller's sequence indices in
 * decimal.  Synchronises `stream`.  EGT_EINVAL on a bad description. */
typedef struct {
  int32_t n_infosets[2];
  const int32_t* parent_seq[2];
  const int32_t* n_actions[2];
  int64_t nnz;
  const int32_t* a_row;
  const int32_t* a_col;
  const double* a_val;
  double scale;
} egt_general_desc;

int egt_build_general_game(const egt_general_desc* desc, hipStream_t stream, egt_game** out);

/* Releases a game (synchronises the device first).  NULL is accepted. */
int egt_free_game(egt_game* game);

/* Sizes of one player's vectors: n_seq rows of ld doubles; n_hands live
 * slots; n_infosets = decision nodes x hands; n_nodes decision nodes.
 * Any output pointer may be NULL. */
int egt_game_dims(const egt_game* game, int player, int64_t* n_seq, int64_t* n_hands,
                  int64_t* ld, int64_t* n_nodes);

/* Layout export.  hand_perm[slot] (n_hands entries, may be NULL) = caller's
 * hand index at that slot.  keys (may be NULL) receives the betting-history
 * key of every sequence in library order, '\n'-terminated each; tokens are
 * joined by '/': "k" check, "f" fold, "c" call, "b<m>" bet or raise to a
 * total river contribution of m millichips, "p" the pass that follows a fold
 * made before the player acted.  *keys_len receives the bytes
 * needed (including a final NUL); EGT_EINVAL if keys_cap is too small. */
int egt_game_layout(const egt_game* game, int player, int32_t* hand_perm, char* keys,
                    int64_t keys_cap, int64_t* keys_len);

/* Total number of terminal histories (fold, showdown) of the game. */
int egt_game_terminals(const egt_game* game, int64_t* n_fold, int64_t* n_show);

/* ------------------------------------------------------------------------ */
/* Hot-path operations                                                        */
/* ------------------------------------------------------------------------ */

/* Payoff-operator product (Section 2: grad f = A y, grad phi = A^T x).
 * player 0: grad_out (player-1 layout) = A * strat_other (player-2 layout);
 * player 1: grad_out (player-2 layout) = A^T * strat_other (player-1 layout).
 * Fold terminals use per-card blocked sums (total minus the mass blocked by
 * the hand's cards); showdown terminals use strength-sorted prefix sums with a
 * per-card correction.  Overwrites all of grad_out; no host synchronisation. */
int egt_gradient(const egt_game* game, int player, const double* strat_other, double* grad_out,
                 hipStream_t stream);

/* Smoothed best response (Section 4, Eq. 4): argmin over player's treeplex of
 * <grad, q> + mu d(q), d the dilated entropy, computed bottom-up with a
 * max-shifted log-sum-exp per information set and top-down to the sequence
 * form.  Always the minimisation form (player 2 passes -A^T x).
 * strat_out (device, may be NULL = value only) receives q; value_out (device
 * pointer to one double, may be NULL) receives the optimal value.
 * mu must be finite and > 0. */
int egt_smoothed_br(const egt_game* game, int player, const double* grad, double mu,
                    double* strat_out, double* value_out, hipStream_t stream);

/* Best-response value min over player's treeplex of <grad, q> (the mu -> 0
 * limit), written to the device double *value_out. */
int egt_best_response(const egt_game* game, int player, const double* grad, double* value_out,
                      hipStream_t stream);

/* The uniform behavioural strategy x_omega (the DGF's minimiser). */
int egt_uniform(const egt_game* game, int player, double* strat_out, hipStream_t stream);

/* Saddle-point residual (Section 2): gap = max_y x^T A y - min_x x^T A y,
 * with br_max_y and br_min_x the two terms (expected chips won by player 2).
 * x, y are device vectors; results are written to HOST doubles (any may be
 * NULL).  Synchronises `stream`.  Always FP64. */
int egt_saddle_gap(const egt_game* game, const double* x, const double* y, double* gap,
                   double* br_max_y, double* br_min_x, hipStream_t stream);

/* Allocation-free saddle gap, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Computes what egt_saddle_gap computes (the same kernels, the
 * same summation order, so the same bits) but allocates nothing and does not
 * synchronise: out3 is a caller-owned DEVICE array of three doubles that
 * receives {gap, br_max_y, br_min_x} on `stream`.  Its scratch (both
 * products, both best-response node-value buffers, the root partial sums) is
 * a fixed library-owned device array of 160 MiB per device, reserved when the
 * library's code is loaded on the device and held until the process ends;
 * EGT_EINVAL when the game needs more (sum over both players of
 * (n_seq + n_nodes) * ld doubles, each part rounded up to 256 bytes, plus 8 KiB:
 * about 132 MiB for 1081 hands with eight bet sizes and four raises).  The game
 * must live on the current device.  Every call on a device uses that device's
 * one array: calls that overlap in time on one device (two streams, two
 * threads) race and must be serialised by the caller. */
int egt_saddle_gap_noalloc(const egt_game* game, const double* x, const double* y, double* out3,
                           hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Precision form (FP32 vectors in the same canonical layout)                 */
/* ------------------------------------------------------------------------ */

/* Payoff product of the precision form (same operator as egt_gradient, Section
 * 2): fold terminals by the O(n) per-card evaluation in FP32 arithmetic; all
 * showdown terminals of the player stacked into one contraction W Y on the
 * BF16 matrix cores, with W in {-1, 0, +1} (exact in BF16) over the
 * strength-ordered hands and Y = b_o * v_o split into hi + lo BF16, FP32
 * accumulation; FP32 output.  The first call on a game builds W (n x n BF16)
 * and synchronises the device.  EGT_EINVAL when a sequence ends in more than
 * one showdown terminal. */
int egt_gradient_mixed(const egt_game* game, int player, const float* strat_other, float* grad_out,
                       hipStream_t stream);

/* Smoothed best response of the precision form (Section 4, Eq. 4): FP32
 * gradient in; each exponent's shift times 1 / (mu beta) in FP64, rounded to
 * FP32 for the exponential; FP32 local strategies and strategy; FP64
 * normalisers and values.
 * strat_out / value_out as in egt_smoothed_br (value_out is a device double). */
int egt_smoothed_br_mixed(const egt_game* game, int player, const float* grad, double mu,
                          float* strat_out, double* value_out, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* EGT driver (Algorithms 1-4)                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t variant;    /* EGT_VARIANT_ALT (Alg. 1), _BAL (mu balancing), _AS (Alg. 3/4) */
  int32_t precision;  /* EGT_PRECISION_FP64, or EGT_PRECISION_MIXED: FP32 iterates and products,
                         BF16 showdown GEMM, FP64 normalisers, mu/tau and saddle gap */
  double eps;         /* target saddle gap; <= 0 means 1e-3 * pot */
  int64_t max_iters;  /* iteration cap (accepted steps) */
  double mu0_x;       /* initial mu; <= 0 (both) means automatic with doubling search */
  double mu0_y;
  double tau0;        /* EGT/as initial tau; <= 0 means 0.5 */
  int32_t gap_every;  /* test the gap every k iterations (>= 1) */
  int32_t fresh_products; /* 0 (default): the stepped player's gradient at the opponent's new
                             point is (1 - tau) A y + tau A y_bar by linearity, from products the
                             step already made (3 products per attempt); 1: it is recomputed
                             (4 per attempt, the accounting of Section 7) */
} egt_solve_opts;

typedef struct {
  int64_t iters;       /* accepted steps */
  int64_t products;    /* payoff products performed on the device */
  int64_t backtracks;  /* EGT/as tau halvings */
  double gap;          /* last measured saddle gap */
  double br_max_y;
  double br_min_x;
  double value_p1;     /* -(x^T A y): expected chips won by player 1 */
  double mu_x, mu_y, tau;
  double seconds;      /* wall time of the solve (host clock) */
  int32_t converged;   /* gap <= eps */
  int32_t reserved;
} egt_result;

/* Fills `opts` with defaults: AS, FP64, eps = 1e-3 * pot, 100000 iterations,
 * automatic mu, tau0 = 0.5, gap every iteration. */
void egt_default_opts(egt_solve_opts* opts);

/* Creates a solver state on `game` (which must outlive it): allocates the
 * device iterates and runs the start of Algorithms 1/3: y0 = SBR of -A^T x_omega,
 * x0 = SBR of A y0, with the mu search when opts asks for automatic mu.
 * Synchronises `stream`. */
int egt_state_create(const egt_game* game, const egt_solve_opts* opts, hipStream_t stream,
                     egt_state** out);
int egt_state_destroy(egt_state* state);

/* One iteration: EGT/as "Decr" (Algorithm 4) or one EGT step (Algorithm 2),
 * on the side the variant picks (player = -1) or on `player` (0 or 1).
 * Writes the excessive gap value after the step and the side stepped (host
 * pointers, may be NULL).  Synchronises `stream`. */
int egt_step(egt_state* state, int player, double* egv_out, int* player_stepped, hipStream_t stream);

/* Copies the current iterates (device -> device, canonical layout) and the
 * scalar state.  Any pointer may be NULL. */
int egt_state_get(const egt_state* state, double* x, double* y, double* mu_x, double* mu_y,
                  double* tau, int64_t* iters, hipStream_t stream);

/* Checkpoint export: the cached products A y (player-1 layout) and A^T x
 * (player-2 layout) of the current iterate (device -> device).  With
 * egt_state_get this is the whole state of the iteration. */
int egt_state_get_products(const egt_state* state, double* ay, double* atx, hipStream_t stream);

/* Checkpoint import / restart from an arbitrary point: sets the iterates
 * (device vectors, canonical layout, copied), mu_x, mu_y > 0, tau in (0, 1)
 * and the iteration counter.  ay / atx (may be NULL) are the products A y and
 * A^T x of that point; when NULL they are recomputed.  Resuming from a full
 * export (iterates, products, scalars) continues bitwise identically to the
 * run that was exported.  Synchronises `stream`. */
int egt_state_set(egt_state* state, const double* x, const double* y, double mu_x, double mu_y,
                  double tau, int64_t iters, const double* ay, const double* atx,
                  hipStream_t stream);

/* Saddle gap of the state's current iterates (host outputs; synchronises). */
int egt_state_gap(egt_state* state, double* gap, double* br_max_y, double* br_min_x,
                  hipStream_t stream);

/* Runs EGT until gap <= eps (tested before each iteration, every gap_every
 * iterations) or max_iters.  While the host decides one iteration (the
 * EGT/as accept-or-halve test) the device already runs the next one on spare
 * buffers; results are bitwise those of egt_step in a loop with the same gap
 * tests.  The final iterates stay in the state if state_out is not NULL (the
 * caller then owns it), else they are freed.  Returns EGT_OK when converged,
 * EGT_ENOTCONV at the iteration cap (result still filled); `stream` is idle
 * on return. */
int egt_solve(const egt_game* game, const egt_solve_opts* opts, egt_result* result,
              egt_state** state_out, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Counterfactual regret minimisation on the same kernels (the regret-based   */
/* methods Section 7 compares EGT with; two products per iteration)           */
/* ------------------------------------------------------------------------ */

/* EGT_CFR_RM:     regret matching, both players updated against the
 *                 strategies of the same iteration, uniform average;
 * EGT_CFR_RMPLUS: the same with regret matching+ (cumulative regrets floored
 *                 at zero after each update);
 * EGT_CFR_PLUS:   regret matching+, player 2 updated against player 1's new
 *                 strategy, average weighted by the iteration index. */
enum { EGT_CFR_RM = 0, EGT_CFR_RMPLUS = 1, EGT_CFR_PLUS = 2 };

typedef struct egt_cfr egt_cfr;

/* Creates a CFR run on `game`: zero regrets, uniform local strategies, the
 * uniform point as the first strategies and averages.  Synchronises
 * `stream`. */
int egt_cfr_create(const egt_game* game, int32_t variant, hipStream_t stream, egt_cfr** out);
int egt_cfr_destroy(egt_cfr* cfr);

/* Runs `iters` iterations on `stream` (no host synchronisation).  Iteration
 * t folds the current strategies into the averages with weight w_t, then
 * updates each player's cumulative counterfactual regrets from its product
 * (A y for player 1, -A^T x for player 2) under its current local strategy
 * and plays regret matching (or matching+) on them. */
int egt_cfr_step(egt_cfr* cfr, int32_t iters, hipStream_t stream);

/* Saddle gap of the average strategies (FP64 products and best responses;
 * host outputs, any may be NULL).  Synchronises `stream`. */
int egt_cfr_gap(egt_cfr* cfr, double* gap, double* br_max_y, double* br_min_x, hipStream_t stream);

/* Copies the averages and the current strategies (device, canonical layout;
 * any may be NULL) and the number of iterations run. */
int egt_cfr_get(const egt_cfr* cfr, double* x_avg, double* y_avg, double* x_cur, double* y_cur,
                int64_t* iters, hipStream_t stream);

/* Runs CFR until the averages' saddle gap is <= eps (<= 0 means 1e-3 * pot),
 * tested before the first iteration and every gap_every iterations, or
 * max_iters.  result: iters, products (2 per iteration), gap and its terms,
 * value_p1 of the averages, seconds; EGT_ENOTCONV at the cap. */
int egt_cfr_solve(const egt_game* game, int32_t variant, double eps, int64_t max_iters, int32_t gap_every,
                  egt_result* result, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Mirror prox and Chambolle-Pock on the same kernels (Section 8's candidate  */
/* first-order methods), with Bregman prox steps of the dilated entropy       */
/* ------------------------------------------------------------------------ */

/* EGT_FOM_MIRROR_PROX:     x^ = prox_x(eta_x A y), y^ = prox_y(-eta_y A^T x),
 *                          x = prox_x(eta_x A y^), y = prox_y(-eta_y A^T x^),
 *                          averages of x^, y^; 4 products per iteration;
 * EGT_FOM_CHAMBOLLE_POCK:  x' = prox_x(tau A y), y' = prox_y(-sigma A^T (2 x' - x)),
 *                          averages of x', y'; 2 products per iteration;
 * prox_c(g) = argmin_q <g, q> + D(q, c), D the Bregman divergence of the
 * dilated entropy; both start at its minimiser, the uniform point. */
enum { EGT_FOM_MIRROR_PROX = 0, EGT_FOM_CHAMBOLLE_POCK = 1 };

typedef struct egt_fom egt_fom;

/* step_x, step_y: eta_x, eta_y (mirror prox) or tau, sigma (Chambolle-Pock),
 * finite and > 0.  Synchronises `stream`. */
int egt_fom_create(const egt_game* game, int32_t method, double step_x, double step_y, hipStream_t stream,
                   egt_fom** out);
int egt_fom_destroy(egt_fom* fom);

/* Runs `iters` iterations on `stream` (no host synchronisation). */
int egt_fom_step(egt_fom* fom, int32_t iters, hipStream_t stream);

/* The averages (the current strategies before the first iteration) and the
 * current strategies (device, canonical layout; any may be NULL), the
 * iteration and product counts (host, may be NULL). */
int egt_fom_get(const egt_fom* fom, double* x_avg, double* y_avg, double* x_cur, double* y_cur, int64_t* iters,
                int64_t* products, hipStream_t stream);

/* Saddle gap of the averages (FP64; host outputs).  Synchronises `stream`. */
int egt_fom_gap(egt_fom* fom, double* gap, double* br_max_y, double* br_min_x, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Serving form: continuous batching of solves on one device                  */
/* ------------------------------------------------------------------------ */

typedef struct egt_batch egt_batch;

/* Device bytes a state of `game` with `opts` (precision) allocates; the
 * admission test of egt_batch_admit charges exactly this. */
int egt_state_bytes(const egt_game* game, const egt_solve_opts* opts, int64_t* bytes);

/* A batch of at most max_slots (1..1024) concurrent solves whose states
 * together stay within budget_bytes of device memory.  Reserves the budget
 * as one device arena, a non-blocking stream (default priority) and pinned
 * host scalars per slot, and starts min(max_slots, 16) host worker threads;
 * nothing is allocated on the device after this call.  EGT_ENOMEM when the reservation fails. */
int egt_batch_create(int64_t budget_bytes, int32_t max_slots, egt_batch** out);

/* Stops the workers (a running solve stops after its current iteration),
 * joins them and frees everything the batch reserved.  NULL is accepted. */
int egt_batch_destroy(egt_batch* batch);

/* Queues a solve of `game` (caller-owned; it must outlive the slot) with
 * `opts` in a free slot and returns at once: the slot's state takes a
 * first-fit range of egt_state_bytes() bytes of the arena, and a worker
 * creates it and runs the solve (the same iteration as egt_solve) on the
 * slot's stream, concurrently with the other slots.  EGT_EBUDGET when no
 * slot is free or the state does not fit the free arena; the caller retries
 * after a retire.  The precision-form tables of `game` are built here. */
int egt_batch_admit(egt_batch* batch, const egt_game* game, const egt_solve_opts* opts,
                    int32_t* slot);

/* Admission by description: like egt_batch_admit, but the batch builds the
 * game itself.  The host part (betting tree, tables, and W for the precision
 * form) runs in this call; the device tables are placed in the slot's arena
 * range ahead of the state -- their bytes are charged to the budget with the
 * state's -- and uploaded by the worker on the slot's stream, so admission
 * performs no device allocation and no synchronisation.  The game is freed
 * (host tables only) when the slot is retired.  EGT_EINVAL on a bad
 * description, EGT_EBUDGET as egt_batch_admit. */
int egt_batch_admit_desc(egt_batch* batch, const egt_game_desc* desc, const egt_solve_opts* opts,
                         int32_t* slot);

/* Waits up to about 2 ms for a solve to finish (returns at once when one
 * finished since the last tick or none is live).  n_active: queued and
 * running solves; n_finished: solves finished since the last tick.  Solves
 * advance on their own; ticking only reports.  Each result is bitwise the
 * same as a lone egt_solve with the same options. */
int egt_batch_tick(egt_batch* batch, int32_t* n_active, int32_t* n_finished);

/* done = 1 once the slot's solve has finished; then status (EGT_OK,
 * EGT_ENOTCONV or the error that stopped it) and the result are valid.
 * result->seconds counts from admission to completion. */
int egt_batch_poll(egt_batch* batch, int32_t slot, int32_t* done, int32_t* status,
                   egt_result* result);

/* Frees a finished slot and returns its bytes to the arena (EGT_EINVAL for a
 * slot that is free, queued or running). */
int egt_batch_retire(egt_batch* batch, int32_t slot);

/* Final iterates of a finished slot (canonical layout, FP64, device pointers
 * x and y of the two players; either may be NULL), e.g. to re-measure the
 * saddle gap.  The state stays in its arena range until the slot is retired.
 * Synchronises `stream`.  EGT_EINVAL unless the slot's solve has finished. */
int egt_batch_strategies(egt_batch* batch, int32_t slot, double* x, double* y, hipStream_t stream);

/* Bytes charged by live and done slots, and their counts. */
int egt_batch_usage(const egt_batch* batch, int64_t* used_bytes, int32_t* n_live, int32_t* n_done);

#ifdef __cplusplus
}
#endif

#endif /* EGT_H */
