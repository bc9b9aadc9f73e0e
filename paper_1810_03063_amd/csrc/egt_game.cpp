// Game builder: betting tree -> level-ordered treeplex tables, terminal lists
// and strength-sorted hand tables, uploaded once to the device.
//
// Treeplex notation follows Section 3 (Definition 2 and what follows): one
// simplex per information set (decision node of a player, private hand), the
// parent sequence p_j, the child simplexes D_j^i after branch i, and the
// dilation weights beta_j = 2 + sum_{k in D^j} 2 beta_k of Section 4, with D^j
// the children over all branches.  Terminal payoffs are player 2's chips:
// each player put pot/2 in before the river; a fold loses the folder's
// pot/2 + river chips; a showdown moves pot/2 + c to the stronger hand and
// nothing on a tie (Section 7's endgame structure).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <numeric>
#include <set>

#include "egt_internal.h"

namespace egt {

namespace {

thread_local std::string g_last_error;

struct Act {
  char kind;  // 'k' check, 'b' bet or raise, 'f' fold, 'c' call, 'p' pass
  double amt; // acting player's river contribution after the action
  bool raise;
};

struct RawNode {
  std::string key;
  int parent_seq;  // raw sequence index of the player's previous action, -1 = empty
  std::vector<Act> acts;
  int first_seq;   // raw index of this node's first sequence
};

struct RawTerminal {
  int kind;      // 0 fold, 1 showdown
  int seq[2];    // raw sequence index per player (-1 = empty)
  double coef;   // player 2's chips (sign of the showdown applied per deal)
};

struct Enumerator {
  double P, S;
  std::vector<double> fracs;
  bool allin;
  int max_raises;
  // situation-dependent sizes: per player and number of bets or raises so far (capped at 3)
  bool situational = false;
  std::vector<double> sfracs[2][4];
  bool sallin[2][4] = {};
  bool open_fold[2] = {false, false};
  std::vector<RawNode> nodes[2];
  std::vector<std::string> seq_key[2];
  std::vector<int> seq_node[2];
  std::vector<RawTerminal> terms;

  static std::string token(const Act& a) {
    if (a.kind == 'k') return "k";
    if (a.kind == 'f') return "f";
    if (a.kind == 'c') return "c";
    if (a.kind == 'p') return "p";
    char buf[64];
    std::snprintf(buf, sizeof buf, "b%lld", (long long)std::nearbyint(a.amt * 1000.0));
    return buf;
  }

  // pot fractions and all-in flag of player p after `bets` bets or raises on the river
  void sizes(int p, int bets, const std::vector<double>** fr, bool* ai) const {
    if (!situational) {
      *fr = &fracs;
      *ai = allin;
      return;
    }
    const int d = std::min(bets, 3);
    *fr = &sfracs[p][d];
    *ai = sallin[p][d];
  }

  std::vector<Act> actions(const double c[2], int p, int raises) const {
    const int o = 1 - p;
    const double to_call = c[o] - c[p];
    const double pot_now = P + c[0] + c[1];
    std::vector<Act> acts;
    std::vector<double> amts;
    const std::vector<double>* fr;
    bool ai;
    if (to_call == 0.0) {
      if (situational && open_fold[p]) acts.push_back({'f', c[p], false});
      acts.push_back({'k', c[p], false});
      sizes(p, 0, &fr, &ai);
      for (double f : *fr) amts.push_back(std::min(c[p] + f * pot_now, S));
      if (ai) amts.push_back(S);
      std::sort(amts.begin(), amts.end());
      amts.erase(std::unique(amts.begin(), amts.end()), amts.end());
      for (double a : amts)
        if (a > c[p]) acts.push_back({'b', a, false});
    } else {
      acts.push_back({'f', c[p], false});
      acts.push_back({'c', c[o], false});
      if (raises < max_raises && c[o] < S) {
        sizes(p, 1 + raises, &fr, &ai);  // facing the opening bet after `raises` raises
        for (double f : *fr) amts.push_back(std::min(c[o] + f * (pot_now + to_call), S));
        if (ai) amts.push_back(S);
        std::sort(amts.begin(), amts.end());
        amts.erase(std::unique(amts.begin(), amts.end()), amts.end());
        for (double a : amts)
          if (a > c[o]) acts.push_back({'b', a, true});
      }
    }
    return acts;
  }

  // A root decision of player p with the single action "p" at history hist;
  // returns the raw index of its sequence.
  int pass_node(const std::string& hist, int p, const double c[2]) {
    RawNode nd;
    nd.key = hist;
    nd.parent_seq = -1;
    nd.acts.push_back({'p', c[p], false});
    nd.first_seq = (int)seq_key[p].size();
    seq_key[p].push_back(hist + "/p");
    seq_node[p].push_back((int)nodes[p].size());
    nodes[p].push_back(nd);
    return nd.first_seq;
  }

  // hist: public history key; last[p]: raw index of p's last sequence.
  void walk(const std::string& hist, const double c[2], int p, int raises, const int last[2]) {
    RawNode nd;
    nd.key = hist;
    nd.parent_seq = last[p];
    nd.acts = actions(c, p, raises);
    nd.first_seq = (int)seq_key[p].size();
    const int node_id = (int)nodes[p].size();
    for (const Act& a : nd.acts) {
      seq_key[p].push_back(hist.empty() ? token(a) : hist + "/" + token(a));
      seq_node[p].push_back(node_id);
    }
    nodes[p].push_back(nd);
    const std::vector<Act> acts = nd.acts;  // nodes[p] may reallocate below
    const int first = nd.first_seq;
    const double half = P / 2.0;
    for (size_t i = 0; i < acts.size(); ++i) {
      const Act& a = acts[i];
      const std::string h2 = seq_key[p][first + i];
      int nl[2] = {last[0], last[1]};
      nl[p] = first + (int)i;
      if (a.kind == 'f') {
        // a fold before the opponent acted: the opponent's one-action pass first
        if (nl[1 - p] < 0) nl[1 - p] = pass_node(h2, 1 - p, c);
        terms.push_back({0, {nl[0], nl[1]}, p == 0 ? (half + c[0]) : -(half + c[1])});
      } else if (a.kind == 'c') {
        terms.push_back({1, {nl[0], nl[1]}, half + c[1 - p]});
      } else if (a.kind == 'k') {
        if (p == 0)
          walk(h2, c, 1, raises, nl);
        else
          terms.push_back({1, {nl[0], nl[1]}, half + c[0]});
      } else {
        double nc[2] = {c[0], c[1]};
        nc[p] = a.amt;
        walk(h2, nc, 1 - p, raises + (a.raise ? 1 : 0), nl);
      }
    }
  }
};

// Heights, level order and the final numbering of one player's treeplex.
int finish_player(const Enumerator& en, int p, HostPlayer& hp, std::vector<int>& raw2new) {
  const auto& nodes = en.nodes[p];
  const int nn = (int)nodes.size();
  const int ns = (int)en.seq_key[p].size();
  // children of each raw sequence
  std::vector<std::vector<int>> kids(ns);
  for (int v = 0; v < nn; ++v)
    if (nodes[v].parent_seq >= 0) kids[nodes[v].parent_seq].push_back(v);
  std::vector<int> height(nn, 0);
  std::vector<double> beta(nn, 0.0);
  // raw nodes are in pre-order, so a reverse sweep sees children first
  for (int v = nn - 1; v >= 0; --v) {
    int h = 0;
    double b = 2.0;
    for (size_t a = 0; a < nodes[v].acts.size(); ++a)
      for (int k : kids[nodes[v].first_seq + a]) {
        h = std::max(h, height[k]);
        b += 2.0 * beta[k];
      }
    height[v] = h + 1;
    beta[v] = b;
  }
  std::vector<int> order(nn);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return height[a] < height[b]; });
  std::vector<int> node_new(nn);
  for (int i = 0; i < nn; ++i) node_new[order[i]] = i;
  raw2new.assign(ns, -1);
  hp.n_nodes = nn;
  hp.n_seq = ns;
  hp.node_first_seq.resize(nn);
  hp.node_nact.resize(nn);
  hp.node_level.resize(nn);
  hp.node_beta.resize(nn);
  hp.node_logn.resize(nn);
  int next = 0;
  for (int i = 0; i < nn; ++i) {
    const RawNode& rn = nodes[order[i]];
    const int na = (int)rn.acts.size();
    if (na < 1 || na > kMaxActions) return fail(EGT_EINVAL, "a decision node needs 1 to 16 actions");
    hp.node_first_seq[i] = next;
    hp.node_nact[i] = na;
    hp.node_level[i] = height[order[i]];
    hp.node_beta[i] = beta[order[i]];
    hp.node_logn[i] = std::log((double)na);
    for (int a = 0; a < na; ++a) raw2new[rn.first_seq + a] = next + a;
    next += na;
  }
  hp.n_levels = nn ? hp.node_level[nn - 1] : 0;
  hp.level_begin.assign(hp.n_levels + 1, nn);
  for (int i = nn - 1; i >= 0; --i) hp.level_begin[hp.node_level[i] - 1] = i;
  for (int l = hp.n_levels - 1; l >= 0; --l)
    hp.level_begin[l] = std::min(hp.level_begin[l], hp.level_begin[l + 1]);
  hp.seq_keys.assign(ns, "");
  hp.seq_parent.assign(ns, -1);
  std::vector<std::vector<int>> kids_new(ns);
  for (int i = 0; i < nn; ++i) {
    const RawNode& rn = nodes[order[i]];
    const int par = rn.parent_seq >= 0 ? raw2new[rn.parent_seq] : -1;
    if (par < 0) hp.roots.push_back(i);
    for (size_t a = 0; a < rn.acts.size(); ++a) {
      const int s = hp.node_first_seq[i] + (int)a;
      hp.seq_keys[s] = en.seq_key[p][rn.first_seq + a];
      hp.seq_parent[s] = par;
    }
    if (par >= 0) kids_new[par].push_back(i);
  }
  // a sequence's children (and the roots) in betting order, the order in which
  // an action's child values are added to its gradient
  for (auto& kids : kids_new) std::sort(kids.begin(), kids.end(), [&](int a, int b) { return order[a] < order[b]; });
  std::sort(hp.roots.begin(), hp.roots.end(), [&](int a, int b) { return order[a] < order[b]; });
  hp.seq_nact.assign(ns, 0);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < hp.node_nact[i]; ++a) hp.seq_nact[hp.node_first_seq[i] + a] = hp.node_nact[i];
  hp.child_begin.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s) hp.child_begin[s + 1] = hp.child_begin[s] + (int)kids_new[s].size();
  hp.child.clear();
  for (int s = 0; s < ns; ++s) hp.child.insert(hp.child.end(), kids_new[s].begin(), kids_new[s].end());
  // longest parent chain (for the top-down pass)
  int mx = 0;
  for (int s = 0; s < ns; ++s) {
    int d = 1;
    for (int q = hp.seq_parent[s]; q >= 0; q = hp.seq_parent[q]) ++d;
    mx = std::max(mx, d);
  }
  if (mx > kMaxDepth) return fail(EGT_EINVAL, "a player's sequence chain is deeper than 16");
  hp.max_chain = mx;
  // root-first path of every sequence, for the fully parallel top-down pass
  hp.anc.assign((size_t)ns * kMaxDepth, -1);
  for (int s = 0; s < ns; ++s) {
    int path[kMaxDepth], d = 0;
    for (int q = s; q >= 0; q = hp.seq_parent[q]) path[d++] = q;
    for (int j = 0; j < d; ++j) hp.anc[(size_t)s * kMaxDepth + j] = path[d - 1 - j];
  }
  hp.max_level_width = 0;
  hp.level_max_act.assign(hp.n_levels, 0);
  for (int l = 0; l < hp.n_levels; ++l) {
    hp.max_level_width = std::max(hp.max_level_width, hp.level_begin[l + 1] - hp.level_begin[l]);
    for (int i = hp.level_begin[l]; i < hp.level_begin[l + 1]; ++i)
      hp.level_max_act[l] = std::max(hp.level_max_act[l], hp.node_nact[i]);
  }
  // table image of the single-launch pass
  const FusedTabLayout L = fused_tab_layout(nn, ns);
  hp.fused_tab.assign((size_t)L.bytes, 0);
  std::vector<int> vslot(nn, -1);
  for (size_t j = 0; j < hp.child.size(); ++j) vslot[hp.child[j]] = (int)j;
  for (size_t r = 0; r < hp.roots.size(); ++r) vslot[hp.roots[r]] = (int)(hp.child.size() + r);
  unsigned char* img = hp.fused_tab.data();
  for (int i = 0; i < nn; ++i) {
    const int rec[4] = {hp.node_first_seq[i], hp.node_nact[i], vslot[i], 0};
    const double prm[4] = {hp.node_beta[i], 1.0 / hp.node_beta[i], hp.node_logn[i], 0.0};
    std::memcpy(img + L.rec + 16 * (size_t)i, rec, sizeof(rec));
    std::memcpy(img + L.prm + 32 * (size_t)i, prm, sizeof(prm));
  }
  std::memcpy(img + L.cbeg, hp.child_begin.data(), sizeof(int) * (size_t)(ns + 1));
  if (ns) std::memcpy(img + L.spar, hp.seq_parent.data(), sizeof(int) * (size_t)ns);
  return EGT_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  return fail(EGT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
const char* last_error_cstr() { return g_last_error.c_str(); }

// The upload image of every table (one device block), the device views' sizes
// and the device attributes the launchers use.
int finish_image(egt_game* g, const std::vector<int>& card_begin, const std::vector<uint4>& htab,
                 const std::vector<unsigned>& hpos, const std::vector<double> (&b)[2]) {
  const int n = g->n, cph = g->cph, nc = g->n_cards;
  const double Z = g->Z;
  struct Piece {
    const void* src;
    size_t bytes;
    size_t off;
  };
  std::vector<Piece> pieces;
  size_t total = 0;
  auto add = [&](const void* src, size_t bytes) {
    const size_t off = total;
    pieces.push_back({src, bytes, off});
    total = align_up(total + std::max<size_t>(bytes, 1), 256);
    return off;
  };
  GameOffsets::Player* po = g->offs.p;
  for (int p = 0; p < 2; ++p) {
    HostPlayer& hp = g->hp[p];
    po[p].first = add(hp.node_first_seq.data(), hp.node_first_seq.size() * sizeof(int));
    po[p].nact = add(hp.node_nact.data(), hp.node_nact.size() * sizeof(int));
    po[p].beta = add(hp.node_beta.data(), hp.node_beta.size() * sizeof(double));
    po[p].logn = add(hp.node_logn.data(), hp.node_logn.size() * sizeof(double));
    po[p].spar = add(hp.seq_parent.data(), hp.seq_parent.size() * sizeof(int));
    po[p].cbeg = add(hp.child_begin.data(), hp.child_begin.size() * sizeof(int));
    po[p].child = add(hp.child.data(), hp.child.size() * sizeof(int));
    po[p].tbeg = add(hp.term_begin.data(), hp.term_begin.size() * sizeof(int));
    po[p].topp = add(hp.term_opp.data(), hp.term_opp.size() * sizeof(int));
    po[p].tkind = add(hp.term_kind.data(), hp.term_kind.size() * sizeof(int));
    po[p].tcoef = add(hp.term_coef.data(), hp.term_coef.size() * sizeof(double));
    po[p].roots = add(hp.roots.data(), hp.roots.size() * sizeof(int));
    po[p].belief = add(b[p].data(), b[p].size() * sizeof(double));
    po[p].ftab = add(hp.fused_tab.data(), hp.fused_tab.size());
    po[p].trec = add(hp.term_rec.data(), hp.term_rec.size() * sizeof(TermRec));
    po[p].anc = add(hp.anc.data(), hp.anc.size() * sizeof(int));
    po[p].titems = add(hp.term_items.data(), hp.term_items.size() * sizeof(TermItem));
    po[p].snact = add(hp.seq_nact.data(), hp.seq_nact.size() * sizeof(int));
    po[p].sptr = add(hp.sp_ptr.data(), hp.sp_ptr.size() * sizeof(int64_t));
    po[p].scol = add(hp.sp_col.data(), hp.sp_col.size() * sizeof(int));
    po[p].sval = add(hp.sp_val.data(), hp.sp_val.size() * sizeof(double));
  }
  g->offs.cbeg = add(card_begin.data(), card_begin.size() * sizeof(int));
  g->offs.htab = add(htab.data(), htab.size() * sizeof(uint4));
  g->offs.hpos = add(hpos.data(), hpos.size() * sizeof(unsigned));

  g->img.assign(total, 0);
  for (const Piece& pc : pieces)
    if (pc.bytes) std::memcpy(g->img.data() + pc.off, pc.src, pc.bytes);
  g->dh.n = n;
  g->dh.ld = g->ld;
  g->dh.cph = cph;
  g->dh.n_cards = nc;
  g->dh.n_card_slots = card_begin[nc] + nc;
  g->dh.invZ = 1.0 / Z;
  EGT_HIP(hipGetDevice(&g->device));
  EGT_HIP(hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, g->device));
  if (g->n_cu < 1) g->n_cu = 1;
  EGT_HIP(hipDeviceGetAttribute(&g->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device));
  EGT_HIP(hipDeviceGetAttribute(&g->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, g->device));
  if (g->lds_per_block < 64 * 1024) g->lds_per_block = 64 * 1024;
  if (g->lds_per_cu < g->lds_per_block) g->lds_per_cu = g->lds_per_block;
  return EGT_OK;
}

// Builds every table of a game on the host and lays them out as one image
// (g->img, offsets in g->offs) for a single upload; no device memory is
// touched.
int build_game_host(const egt_game_desc* d, egt_game** out) {
  if (!d || !out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  const int n = d->n_hands, cph = d->cards_per_hand, nc = d->n_cards;
  if (n < 1 || n > 2048 || (cph != 1 && cph != 2) || nc < 1 || nc > 4096)
    return fail(EGT_EINVAL, "bad n_hands (1..2048) / cards_per_hand (1 or 2) / n_cards");
  if (!d->hand_cards || !d->strength || !d->belief[0] || !d->belief[1])
    return fail(EGT_EINVAL, "null hand / strength / belief array");
  if (!(d->pot > 0) || !(d->stack >= 0) || !std::isfinite(d->pot) || !std::isfinite(d->stack))
    return fail(EGT_EINVAL, "pot must be > 0 and stack >= 0");
  if (d->n_bet_fracs < 0 || (d->n_bet_fracs > 0 && !d->bet_fracs) || d->max_raises < 0)
    return fail(EGT_EINVAL, "bad betting parameters");
  for (int i = 0; i < d->n_bet_fracs; ++i)
    if (!(d->bet_fracs[i] > 0) || !std::isfinite(d->bet_fracs[i]))
      return fail(EGT_EINVAL, "bet fractions must be finite and > 0");
  if (const egt_bet_abstraction* ab = d->abstraction) {
    for (int p = 0; p < 2; ++p)
      for (int k = 0; k < 4; ++k) {
        if (ab->n_fracs[p][k] < 0 || ab->n_fracs[p][k] > kMaxActions || (ab->n_fracs[p][k] > 0 && !ab->fracs[p][k]))
          return fail(EGT_EINVAL, "bad bet abstraction (0..16 fractions per situation)");
        for (int i = 0; i < ab->n_fracs[p][k]; ++i)
          if (!(ab->fracs[p][k][i] > 0) || !std::isfinite(ab->fracs[p][k][i]))
            return fail(EGT_EINVAL, "bet fractions must be finite and > 0");
      }
  }
  std::set<std::vector<int>> seen;
  for (int h = 0; h < n; ++h) {
    std::vector<int> cs;
    for (int j = 0; j < cph; ++j) {
      const int c = d->hand_cards[h * cph + j];
      if (c < 0 || c >= nc) return fail(EGT_EINVAL, "card id out of range");
      cs.push_back(c);
    }
    std::sort(cs.begin(), cs.end());
    if (cph == 2 && cs[0] == cs[1]) return fail(EGT_EINVAL, "a hand holds the same card twice");
    if (!seen.insert(cs).second) return fail(EGT_EINVAL, "two hands hold the same cards");
    for (int p = 0; p < 2; ++p)
      if (!(d->belief[p][h] >= 0) || !std::isfinite(d->belief[p][h]))
        return fail(EGT_EINVAL, "beliefs must be finite and >= 0");
  }

  egt_game* g = new (std::nothrow) egt_game();
  if (!g) return fail(EGT_ENOMEM, "host allocation failed");
  std::unique_ptr<egt_game> guard(g);
  g->n = n;
  g->ld = (n + 31) / 32 * 32;
  g->cph = cph;
  g->n_cards = nc;
  g->pot = d->pot;
  g->stack = d->stack;

  // ---- betting tree and treeplexes ----
  Enumerator en;
  en.P = d->pot;
  en.S = d->stack;
  en.fracs.assign(d->bet_fracs, d->bet_fracs + d->n_bet_fracs);
  en.allin = d->allin != 0;
  en.max_raises = d->max_raises;
  if (const egt_bet_abstraction* ab = d->abstraction) {
    en.situational = true;
    for (int p = 0; p < 2; ++p) {
      en.open_fold[p] = ab->open_fold[p] != 0;
      for (int k = 0; k < 4; ++k) {
        en.sfracs[p][k].assign(ab->fracs[p][k], ab->fracs[p][k] + ab->n_fracs[p][k]);
        en.sallin[p][k] = ab->allin[p][k] != 0;
      }
    }
  }
  const int none[2] = {-1, -1};
  const double c0[2] = {0.0, 0.0};
  en.walk("", c0, 0, 0, none);
  std::vector<int> raw2new[2];
  for (int p = 0; p < 2; ++p) {
    const int st = finish_player(en, p, g->hp[p], raw2new[p]);
    if (st != EGT_OK) return st;
    if (g->hp[p].n_seq > 65535) return fail(EGT_EINVAL, "more than 65535 sequences for one player");
  }
  // terminals grouped by each player's own sequence
  for (int p = 0; p < 2; ++p) {
    HostPlayer& hp = g->hp[p];
    std::vector<std::vector<int>> by(hp.n_seq);
    for (size_t t = 0; t < en.terms.size(); ++t) {
      const int s = en.terms[t].seq[p];
      if (s >= 0) by[raw2new[p][s]].push_back((int)t);
    }
    hp.term_begin.assign(hp.n_seq + 1, 0);
    for (int s = 0; s < hp.n_seq; ++s) {
      for (int t : by[s]) {
        const RawTerminal& rt = en.terms[t];
        const int os = rt.seq[1 - p];
        hp.term_opp.push_back(os >= 0 ? raw2new[1 - p][os] : -1);
        hp.term_kind.push_back(rt.kind);
        hp.term_coef.push_back(rt.coef);
      }
      hp.term_begin[s + 1] = (int)hp.term_opp.size();
      hp.max_terms_per_seq = std::max(hp.max_terms_per_seq, (int)by[s].size());
    }
    const int stride = std::max(1, hp.max_terms_per_seq);
    hp.term_rec.assign((size_t)hp.n_seq * stride, TermRec{-1, -1, 0.0});
    for (int s = 0; s < hp.n_seq; ++s)
      for (int t = hp.term_begin[s]; t < hp.term_begin[s + 1]; ++t)
        hp.term_rec[(size_t)s * stride + (t - hp.term_begin[s])] = TermRec{hp.term_opp[t], hp.term_kind[t], hp.term_coef[t]};
    // work items for blocks that loop over sequences: two-terminal sequences
    // whole, one-terminal sequences in pairs, empty sequences alone
    hp.term_items.clear();
    if (hp.max_terms_per_seq <= 2) {
      const TermRec none{-1, -1, 0.0};
      int pending = -1;
      for (int s = 0; s < hp.n_seq; ++s) {
        const int cnt = hp.term_begin[s + 1] - hp.term_begin[s];
        const TermRec* r = &hp.term_rec[(size_t)s * stride];
        if (cnt == 2) {
          hp.term_items.push_back(TermItem{{r[0], r[1]}, {s, s}, {0, 0}});
        } else if (cnt == 0) {
          hp.term_items.push_back(TermItem{{none, none}, {s, -1}, {0, 0}});
        } else if (pending < 0) {
          pending = s;
        } else {
          hp.term_items.push_back(TermItem{{hp.term_rec[(size_t)pending * stride], r[0]}, {pending, s}, {0, 0}});
          pending = -1;
        }
      }
      if (pending >= 0)
        hp.term_items.push_back(TermItem{{hp.term_rec[(size_t)pending * stride], none}, {pending, -1}, {0, 0}});
    }
  }
  // enough 4-hand blocks to spread over the chip; 16-hand blocks for tiny hand counts
  g->fused_hands = g->ld >= 512 ? 4 : 16;
  g->fused_passes =
      fused_lds_bytes(g->fused_hands, (int)std::max(g->hp[0].fused_tab.size(), g->hp[1].fused_tab.size()),
                      std::max(g->hp[0].n_nodes, g->hp[1].n_nodes),
                      std::max(g->hp[0].n_seq, g->hp[1].n_seq)) <= kFusedLdsLimit;
  for (const RawTerminal& t : en.terms) (t.kind == 0 ? g->n_fold : g->n_show)++;
  for (int p = 0; p < 2; ++p)
    for (double b : g->hp[p].node_beta) g->max_beta = std::max(g->max_beta, b);

  // ---- hands: strength order, tie groups, card lists ----
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int a, int b) { return d->strength[a] < d->strength[b]; });
  g->perm = perm;
  g->slot_cards.resize((size_t)n * cph);
  g->slot_strength.resize(n);
  for (int i = 0; i < n; ++i) {
    g->slot_strength[i] = d->strength[perm[i]];
    for (int j = 0; j < cph; ++j) g->slot_cards[(size_t)i * cph + j] = d->hand_cards[perm[i] * cph + j];
  }
  std::vector<int2> tie(n);
  for (int i = 0; i < n;) {
    int j = i;
    while (j < n && d->strength[perm[j]] == d->strength[perm[i]]) ++j;
    for (int k = i; k < j; ++k) tie[k] = make_int2(i, j);
    i = j;
  }
  std::vector<std::vector<int>> lists(nc);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < cph; ++j) lists[d->hand_cards[perm[i] * cph + j]].push_back(i);
  std::vector<int> card_begin(nc + 1, 0);
  for (int c = 0; c < nc; ++c) card_begin[c + 1] = card_begin[c] + (int)lists[c].size();
  // The product kernel's per-hand tables.  E lays the card lists end to end,
  // card c's list at base_c = card_begin[c] + c followed by one slot for its
  // total.  For the hand in slot i and each of its cards: the E index of the
  // card's exclusive prefix at the start (lo) and end (hi) of i's tie group
  // and of the card's total (len); and i's own position in the card's list
  // (where the kernel scatters its reach).  Every index fits 16 bits.
  std::vector<uint4> htab(n);
  std::vector<unsigned> hpos(n);
  for (int i = 0; i < n; ++i) {
    unsigned lo[2] = {0, 0}, hi[2] = {0, 0}, tot[2] = {0, 0}, pos[2] = {0, 0};
    for (int j = 0; j < cph; ++j) {
      const int c = d->hand_cards[perm[i] * cph + j];
      const auto& L = lists[c];
      const unsigned base = (unsigned)(card_begin[c] + c);
      lo[j] = base + (unsigned)(std::lower_bound(L.begin(), L.end(), tie[i].x) - L.begin());
      hi[j] = base + (unsigned)(std::lower_bound(L.begin(), L.end(), tie[i].y) - L.begin());
      tot[j] = base + (unsigned)L.size();
      pos[j] = base + (unsigned)(std::lower_bound(L.begin(), L.end(), i) - L.begin());
    }
    htab[i] = make_uint4(lo[0] | (hi[0] << 16), tot[0] | (lo[1] << 16), hi[1] | (tot[1] << 16),
                         (unsigned)tie[i].x | ((unsigned)tie[i].y << 16));
    hpos[i] = pos[0] | (pos[1] << 16);
  }
  if (card_begin[nc] + nc >= 65536) return fail(EGT_EINVAL, "too many card-list slots for 16-bit indices");
  // Z = sum over compatible deals of b1 b2
  std::vector<double> b[2];
  for (int p = 0; p < 2; ++p) {
    b[p].assign(g->ld, 0.0);
    for (int i = 0; i < n; ++i) b[p][i] = d->belief[p][perm[i]];
  }
  g->hbelief[0] = b[0];
  g->hbelief[1] = b[1];
  double Z = 0.0;
  for (int i = 0; i < n; ++i) {
    if (b[0][i] == 0.0) continue;
    double row = 0.0;
    for (int k = 0; k < n; ++k) {
      bool share = false;
      for (int a = 0; a < cph && !share; ++a)
        for (int c = 0; c < cph; ++c)
          if (d->hand_cards[perm[i] * cph + a] == d->hand_cards[perm[k] * cph + c]) share = true;
      if (!share) row += b[1][k];
    }
    Z += b[0][i] * row;
  }
  if (!(Z > 0) || !std::isfinite(Z)) return fail(EGT_EINVAL, "no compatible deal has positive belief");
  g->Z = Z;

  int rc = finish_image(g, card_begin, htab, hpos, b);
  if (rc) return rc;
  *out = guard.release();
  return EGT_OK;
}

// A general game (egt_general_desc) on the host: the two treeplexes through
// the same level ordering as a river endgame, the payoff operator as CSR rows
// per player, one live slot per row and no terminal or hand tables.
int build_general_host(const egt_general_desc* d, egt_game** out) {
  if (!d || !out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  if (!(d->scale > 0) || !std::isfinite(d->scale)) return fail(EGT_EINVAL, "scale must be finite and > 0");
  if (d->nnz < 0 || (d->nnz > 0 && (!d->a_row || !d->a_col || !d->a_val)))
    return fail(EGT_EINVAL, "bad payoff triples");
  Enumerator en;  // only its node and sequence lists
  for (int p = 0; p < 2; ++p) {
    const int ni = d->n_infosets[p];
    if (ni < 1 || !d->parent_seq[p] || !d->n_actions[p])
      return fail(EGT_EINVAL, "every player needs at least one information set");
    int seqs = 0;
    for (int k = 0; k < ni; ++k) {
      const int na = d->n_actions[p][k], ps = d->parent_seq[p][k];
      if (na < 1 || na > kMaxActions) return fail(EGT_EINVAL, "an information set needs 1 to 16 actions");
      if (ps < -1 || ps >= seqs)
        return fail(EGT_EINVAL, "a parent sequence must belong to an earlier information set (or be -1)");
      if (seqs > (1 << 26) - na) return fail(EGT_EINVAL, "too many sequences");
      RawNode rn;
      rn.key = std::to_string(k);
      rn.parent_seq = ps;
      rn.first_seq = seqs;
      rn.acts.assign(na, Act{'p', 0.0, false});
      en.nodes[p].push_back(rn);
      for (int a = 0; a < na; ++a) en.seq_key[p].push_back(std::to_string(seqs + a));
      seqs += na;
    }
  }
  egt_game* g = new (std::nothrow) egt_game();
  if (!g) return fail(EGT_ENOMEM, "host allocation failed");
  std::unique_ptr<egt_game> guard(g);
  g->general = true;
  g->n = 1;
  g->ld = 32;
  g->cph = 1;
  g->n_cards = 1;
  g->pot = d->scale;
  g->stack = 0.0;
  std::vector<int> raw2new[2];
  for (int p = 0; p < 2; ++p) {
    const int st = finish_player(en, p, g->hp[p], raw2new[p]);
    if (st != EGT_OK) return st;
    HostPlayer& hp = g->hp[p];
    hp.term_begin.assign(hp.n_seq + 1, 0);
    hp.max_terms_per_seq = 0;
    hp.term_rec.assign((size_t)hp.n_seq, TermRec{-1, -1, 0.0});
    hp.term_items.clear();
  }
  // payoff triples in library numbering; repeated pairs added in input order
  struct Trip {
    int r, c;
    int64_t i;
  };
  std::vector<Trip> t((size_t)d->nnz);
  for (int64_t i = 0; i < d->nnz; ++i) {
    const int r = d->a_row[i], c = d->a_col[i];
    if (r < 0 || r >= g->hp[0].n_seq || c < 0 || c >= g->hp[1].n_seq)
      return fail(EGT_EINVAL, "a payoff triple names a sequence out of range");
    if (!std::isfinite(d->a_val[i])) return fail(EGT_EINVAL, "payoff values must be finite");
    t[(size_t)i] = Trip{raw2new[0][r], raw2new[1][c], i};
  }
  for (int p = 0; p < 2; ++p) {
    HostPlayer& hp = g->hp[p];
    // this player's rows: (row, col) = (r, c) for player 1, (c, r) for player 2
    std::vector<Trip> u(t);
    if (p == 1)
      for (Trip& x : u) std::swap(x.r, x.c);
    std::stable_sort(u.begin(), u.end(), [](const Trip& a, const Trip& b) { return a.r != b.r ? a.r < b.r : a.c < b.c; });
    hp.sp_ptr.assign(hp.n_seq + 1, 0);
    hp.sp_col.clear();
    hp.sp_val.clear();
    for (size_t k = 0; k < u.size();) {
      size_t e = k;
      double v = 0.0;
      while (e < u.size() && u[e].r == u[k].r && u[e].c == u[k].c) v += d->a_val[u[e++].i];
      hp.sp_col.push_back(u[k].c);
      hp.sp_val.push_back(v);
      hp.sp_ptr[u[k].r + 1]++;
      k = e;
    }
    hp.sp_max_row = 0;
    for (int r = 0; r < hp.n_seq; ++r) {
      hp.sp_max_row = std::max(hp.sp_max_row, hp.sp_ptr[r + 1]);
      hp.sp_ptr[r + 1] += hp.sp_ptr[r];
    }
  }
  g->fused_hands = 16;
  g->fused_passes =
      fused_lds_bytes(g->fused_hands, (int)std::max(g->hp[0].fused_tab.size(), g->hp[1].fused_tab.size()),
                      std::max(g->hp[0].n_nodes, g->hp[1].n_nodes),
                      std::max(g->hp[0].n_seq, g->hp[1].n_seq)) <= kFusedLdsLimit;
  for (int p = 0; p < 2; ++p)
    for (double b : g->hp[p].node_beta) g->max_beta = std::max(g->max_beta, b);
  g->perm = {0};
  g->slot_cards = {0};
  g->slot_strength = {0};
  std::vector<double> b[2];
  for (int p = 0; p < 2; ++p) {
    b[p].assign(g->ld, 0.0);
    b[p][0] = 1.0;
    g->hbelief[p] = b[p];
  }
  g->Z = 1.0;
  const std::vector<int> card_begin = {0, 1};
  const std::vector<uint4> htab = {make_uint4(0u, 0u, 0u, 0u)};
  const std::vector<unsigned> hpos = {0u};
  const int rc = finish_image(g, card_begin, htab, hpos, b);
  if (rc) return rc;
  *out = guard.release();
  return EGT_OK;
}

size_t game_device_bytes(const egt_game* g) { return g->img.size(); }

// Copies the table image into `dev` (game_device_bytes(g) bytes, 256-byte
// aligned, owned by the caller when owned == false) on `stream` and points
// the device views at it.  The host image must stay until the copy is done.
int upload_game(egt_game* g, void* dev, bool owned, hipStream_t stream) {
  g->mem.base = dev;
  g->mem.bytes = g->img.size();
  g->owns_mem = owned;
  EGT_HIP(hipMemcpyAsync(dev, g->img.data(), g->img.size(), hipMemcpyHostToDevice, stream));
  auto at = [&](size_t off) { return (const void*)((const unsigned char*)dev + off); };
  const GameOffsets::Player* po = g->offs.p;
  for (int p = 0; p < 2; ++p) {
    HostPlayer& hp = g->hp[p];
    DPlayer& dp = g->dp[p];
    dp.n_seq = hp.n_seq;
    dp.n_nodes = hp.n_nodes;
    dp.n_roots = (int)hp.roots.size();
    dp.node_first_seq = (const int*)at(po[p].first);
    dp.node_nact = (const int*)at(po[p].nact);
    dp.node_beta = (const double*)at(po[p].beta);
    dp.node_logn = (const double*)at(po[p].logn);
    dp.seq_parent = (const int*)at(po[p].spar);
    dp.child_begin = (const int*)at(po[p].cbeg);
    dp.child = (const int*)at(po[p].child);
    dp.term_begin = (const int*)at(po[p].tbeg);
    dp.term_opp = (const int*)at(po[p].topp);
    dp.term_kind = (const int*)at(po[p].tkind);
    dp.term_coef = (const double*)at(po[p].tcoef);
    dp.roots = (const int*)at(po[p].roots);
    dp.belief = (const double*)at(po[p].belief);
    dp.fused_tab = at(po[p].ftab);
    dp.fused_tab16 = (int)(hp.fused_tab.size() / 16);
    dp.term_rec = (const TermRec*)at(po[p].trec);
    dp.anc = (const int*)at(po[p].anc);
    dp.term_stride = std::max(1, hp.max_terms_per_seq);
    dp.n_items = (int)hp.term_items.size();
    dp.term_items = dp.n_items > 0 ? (const TermItem*)at(po[p].titems) : nullptr;
    dp.seq_nact = (const int*)at(po[p].snact);
    dp.sp_ptr = hp.sp_ptr.empty() ? nullptr : (const int64_t*)at(po[p].sptr);
    dp.sp_col = (const int*)at(po[p].scol);
    dp.sp_val = (const double*)at(po[p].sval);
  }
  g->dh.card_begin = (const int*)at(g->offs.cbeg);
  g->dh.htab = (const uint4*)at(g->offs.htab);
  g->dh.hpos = (const unsigned*)at(g->offs.hpos);
  return EGT_OK;
}

namespace {

// One device block for a game built on the host, upload, synchronise.
int place_game(egt_game* g, hipStream_t stream, egt_game** out) {
  std::unique_ptr<egt_game> guard(g);
  int rc = EGT_OK;
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, game_device_bytes(g));
  if (e != hipSuccess) return fail(EGT_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  rc = upload_game(g, dev, true, stream);
  if (rc == EGT_OK) {
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) rc = hip_fail(e, "upload of game tables");
  }
  if (rc) {
    (void)hipFree(dev);
    g->mem.base = nullptr;
    return rc;
  }
  *out = guard.release();
  return EGT_OK;
}

}  // namespace

// Host tables, one device block, upload, synchronise.
int build_game(const egt_game_desc* d, hipStream_t stream, egt_game** out) {
  if (!out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  egt_game* g = nullptr;
  const int rc = build_game_host(d, &g);
  if (rc) return rc;
  return place_game(g, stream, out);
}

int build_general_game(const egt_general_desc* d, hipStream_t stream, egt_game** out) {
  if (!out) return fail(EGT_EINVAL, "null argument");
  *out = nullptr;
  egt_game* g = nullptr;
  const int rc = build_general_host(d, &g);
  if (rc) return rc;
  return place_game(g, stream, out);
}

int free_game(egt_game* g) {
  if (!g) return EGT_OK;
  int st = EGT_OK;
  const bool dev_owned = (g->mem.base && g->owns_mem) || (g->mx.block && g->mx.owned);
  if (dev_owned || g->ws.block || g->ws.hscal) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && g->mem.base && g->owns_mem) e = hipFree(g->mem.base);
    if (e == hipSuccess && g->mx.block && g->mx.owned) e = hipFree(g->mx.block);
    if (e == hipSuccess && g->ws.block) e = hipFree(g->ws.block);
    if (e == hipSuccess && g->ws.hscal) e = hipHostFree(g->ws.hscal);
    if (e != hipSuccess) st = hip_fail(e, "free_game");
  }
  delete g;
  return st;
}

}  // namespace egt
