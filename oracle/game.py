"""Oracle, part 1: the river endgame as an extensive-form game.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package; it exists to check the GPU path and is itself pinned by the
``-m "not gpu"`` tests.

What is built here, straight from the definitions:

* the public betting tree (Section 7, "Experiments": chance deals the hands,
  then the players bet; the game ends on a fold, a call, or two checks; a
  showdown splits the pot on a tie);
* for each player, the sequence-form strategy space as a treeplex
  (Section 3, Definition 2 and its notation): one simplex per information set,
  i.e. per (decision node of that player, private hand); the simplexes of all
  hands at a root node form a Cartesian product, and a simplex below is scaled
  by its parent sequence;
* the terminal list that defines the payoff matrix A of the bilinear problem
  min_x max_y <x, A y> (Section 2, Eq. 2).  A holds player 2's payoff, which is
  player 1's loss, so player 1 (x, first to act) minimises.

Betting rules used for the synthetic endgames:
  * not facing a bet: check, or bet ``f * pot`` for each bet fraction f, plus
    all-in; a bet at or above the remaining stack becomes all-in; duplicates
    are removed;
  * facing a bet of ``to_call``: fold, call, or raise to
    ``c_opp + f * (pot + to_call)`` for each f, plus all-in, while fewer than
    ``max_raises`` raises have happened after the opening bet and the opponent
    is not all-in;
  * the first player checking and the second checking back, or a call, ends in
    a showdown; a fold ends the hand (a fold before the opponent has acted
    goes through a one-action "pass" decision of the opponent, see
    ``_pass_node``).
With the symmetric rules one list of fractions and the all-in flag apply in
every situation.  With a situation-dependent abstraction (the shape Section 7
gives for Libratus' river abstraction) the fractions and the all-in flag
depend on the acting player and on how many bets or raises the river has
seen so far (0 when not facing a bet, 1 facing the opening bet, 2 facing the
first raise, 3 for every later raise), and a player not facing a bet may also
fold (the paper lets Libratus fold first and the opponent fold facing a
check).
Payoffs are net chips for player 2: each player put pot/2 in before the
river, so a fold by player 1 pays player 2 ``pot/2 + c1``, a fold by player 2
costs player 2 ``pot/2 + c2`` and a showdown pays ``(pot/2 + c)`` times the
sign of (player 2's strength - player 1's strength).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _tok_amount(c: float) -> str:
    return "b%d" % int(round(c * 1000.0))


@dataclass
class Terminal:
    kind: str  # "fold" or "show"
    history: tuple
    seq: tuple  # (player-1 sequence index or -1, player-2 sequence index or -1)
    u: float  # player 2's chips: fold -> +-(pot/2 + c_folder); show -> (pot/2 + c) (times sign)


@dataclass
class InfoNode:
    """A decision node of one player in the public tree.  Together with a
    private hand it is one information set, i.e. one simplex of the treeplex."""
    key: str
    history: tuple
    parent_seq: int  # index of the player's previous sequence, -1 = empty sequence
    first_seq: int  # sequences of this node are first_seq .. first_seq + n_act - 1
    n_act: int
    children: list = field(default_factory=list)  # per action: list of child node indices
    beta: float = 0.0
    height: int = 0


@dataclass
class Treeplex:
    player: int
    nodes: list
    seq_keys: list
    post_order: list  # node indices, every node after all of its descendants

    @property
    def n_seq(self) -> int:
        return len(self.seq_keys)

    def roots(self):
        return [i for i, v in enumerate(self.nodes) if v.parent_seq < 0]

    def seq_node(self):
        """node index owning each sequence."""
        out = np.empty(self.n_seq, dtype=np.int64)
        for i, v in enumerate(self.nodes):
            out[v.first_seq:v.first_seq + v.n_act] = i
        return out


class Game:
    def __init__(self, inst):
        self.inst = inst
        self.pot = float(inst.pot)
        self.stack = float(inst.stack)
        self.fracs = tuple(float(f) for f in inst.bet_fracs)
        self.allin = bool(inst.allin)
        self.max_raises = int(inst.max_raises)
        self.abstraction = getattr(inst, "abstraction", None)
        self._nodes = [[], []]  # raw per player: (history, parent_seq_key)
        self._seq_keys = [[], []]
        self._seq_index = [{}, {}]
        self._node_actions = [[], []]
        self.terminals_raw = []
        self._walk((), (0.0, 0.0), 0, 0, (None, None))
        self.treeplex = [self._build_treeplex(p) for p in (0, 1)]
        self.terminals = [
            Terminal(kind, hist, (self._seq_index[0].get(s0, -1) if s0 else -1,
                                  self._seq_index[1].get(s1, -1) if s1 else -1), u)
            for (kind, hist, s0, s1, u) in self.terminals_raw
        ]

    # -- betting tree ---------------------------------------------------
    def _sizes(self, player, bets_so_far):
        """(pot fractions, all-in flag) of the acting player when the river
        has seen ``bets_so_far`` bets or raises."""
        ab = self.abstraction
        if ab is None:
            return self.fracs, self.allin
        d = min(bets_so_far, 3)
        return tuple(float(f) for f in ab.fracs[player][d]), bool(ab.allin[player][d])

    def _actions(self, c, player, n_raises):
        """(token, kind, new contribution of the acting player)."""
        P, S = self.pot, self.stack
        opp = 1 - player
        to_call = c[opp] - c[player]
        pot_now = P + c[0] + c[1]
        acts = []
        if to_call == 0.0:
            if self.abstraction is not None and self.abstraction.open_fold[player]:
                acts.append(("f", "fold", c[player]))
            acts.append(("k", "check", c[player]))
            fracs, allin = self._sizes(player, 0)
            amounts = [min(c[player] + f * pot_now, S) for f in fracs]
            if allin:
                amounts.append(S)
            for a in sorted(set(a for a in amounts if a > c[player])):
                acts.append((_tok_amount(a), "bet", a))
        else:
            acts.append(("f", "fold", c[player]))
            acts.append(("c", "call", c[opp]))
            if n_raises < self.max_raises and c[opp] < S:
                # facing the opening bet after n_raises = 0 raises: 1 bet so far
                fracs, allin = self._sizes(player, 1 + n_raises)
                amounts = [min(c[opp] + f * (pot_now + to_call), S) for f in fracs]
                if allin:
                    amounts.append(S)
                for a in sorted(set(a for a in amounts if a > c[opp])):
                    acts.append((_tok_amount(a), "raise", a))
        return acts

    def _walk(self, hist, c, player, n_raises, last_seq):
        self._nodes[player].append((hist, last_seq[player]))
        acts = self._actions(c, player, n_raises)
        self._node_actions[player].append(acts)
        half = self.pot / 2.0
        # number this node's sequences contiguously before descending
        for tok, _, _ in acts:
            skey = "/".join(hist + (tok,))
            self._seq_index[player][skey] = len(self._seq_keys[player])
            self._seq_keys[player].append(skey)
        for tok, kind, newc in acts:
            h2 = hist + (tok,)
            skey = "/".join(h2)
            ls = list(last_seq)
            ls[player] = skey
            ls = tuple(ls)
            if kind == "fold":
                u = (half + c[0]) if player == 0 else -(half + c[1])
                if ls[1 - player] is None:
                    ls = self._pass_node(h2, 1 - player, c, ls)
                    h2 = h2 + ("p",)
                self.terminals_raw.append(("fold", h2, ls[0], ls[1], u))
            elif kind == "call":
                self.terminals_raw.append(("show", h2, ls[0], ls[1], half + c[1 - player]))
            elif kind == "check":
                if player == 0:
                    self._walk(h2, c, 1, n_raises, ls)
                else:
                    self.terminals_raw.append(("show", h2, ls[0], ls[1], half + c[0]))
            else:
                nc = list(c)
                nc[player] = newc
                self._walk(h2, tuple(nc), 1 - player, n_raises + (1 if kind == "raise" else 0), ls)

    def _pass_node(self, hist, player, c, last_seq):
        """A fold before ``player`` has acted would end at player's empty
        sequence, which has no coordinate in the treeplex (its value is the
        constant 1), and would add a term linear in the folder's strategy to
        the payoff.  Instead the opponent gets a decision with the single
        action "p" (pass) before the fold takes effect: its sequence always
        has mass 1, its simplex has no entropy, and the payoff stays bilinear
        in the two treeplexes."""
        self._nodes[player].append((hist, None))
        self._node_actions[player].append([("p", "pass", c[player])])
        skey = "/".join(hist + ("p",))
        self._seq_index[player][skey] = len(self._seq_keys[player])
        self._seq_keys[player].append(skey)
        ls = list(last_seq)
        ls[player] = skey
        return tuple(ls)

    # -- treeplexes -----------------------------------------------------
    def _build_treeplex(self, p):
        raw = self._nodes[p]
        acts = self._node_actions[p]
        nodes = []
        # sequences were numbered in walk order; recover each node's range
        for (hist, pkey), a in zip(raw, acts):
            first = self._seq_index[p]["/".join(hist + (a[0][0],))]
            nodes.append(InfoNode(
                key="/".join(hist), history=hist,
                parent_seq=self._seq_index[p][pkey] if pkey else -1,
                first_seq=first, n_act=len(a),
                children=[[] for _ in a]))
        for i, v in enumerate(nodes):
            if v.parent_seq >= 0:
                par = next(j for j, u in enumerate(nodes)
                           if u.first_seq <= v.parent_seq < u.first_seq + u.n_act)
                nodes[par].children[v.parent_seq - nodes[par].first_seq].append(i)
        order = []

        def visit(i):
            for ch in nodes[i].children:
                for k in ch:
                    visit(k)
            order.append(i)

        for i, v in enumerate(nodes):
            if v.parent_seq < 0:
                visit(i)
        # beta_j = 2 + sum over all child simplexes (all branches) of 2*beta_k
        # (Section 4, dilated entropy); height = 1 + max child height.
        for i in order:
            v = nodes[i]
            kids = [k for ch in v.children for k in ch]
            v.beta = 2.0 + sum(2.0 * nodes[k].beta for k in kids)
            v.height = 1 + max((nodes[k].height for k in kids), default=0)
        return Treeplex(p, nodes, list(self._seq_keys[p]), order)

    # -- summary --------------------------------------------------------
    def counts(self):
        return dict(
            nodes=[len(t.nodes) for t in self.treeplex],
            seqs=[t.n_seq for t in self.treeplex],
            roots=[len(t.roots()) for t in self.treeplex],
            fold=sum(1 for z in self.terminals if z.kind == "fold"),
            show=sum(1 for z in self.terminals if z.kind == "show"),
        )
