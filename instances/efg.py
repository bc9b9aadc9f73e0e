"""General two-player zero-sum extensive-form games in sequence form.

A game is given as each player's treeplex -- its information sets, each with
the player's parent sequence (-1 for the empty sequence) and its number of
actions, sequences numbered infoset by infoset in the order given, parents
before children -- and the payoff matrix A as triples (s1, s2, value): player
2's expected payoff (player 1's loss) over chance, for every pair of last
sequences that ends the game.  This is the input of the paper's general route
(an explicit sequence-form payoff matrix, Section 6).

Generators:
* ``leduc()``: Leduc hold'em (a six-card deck of three ranks, one private card
  each, one public card after the first betting round, raises of 2 then 4,
  at most two bets per round, antes of 1), built by walking every deal;
* ``kuhn_efg()``: Kuhn poker written as a general game (the same game as
  ``instances.endgames.kuhn``, a cross-check of the two constructions);
* ``random_efg(seed, ...)``: a seeded random game tree (random branching,
  random chance splits, random payoffs) whose terminals follow a sequence of
  each player;
* ``fig1_game(seed)``: Section 3's nine-simplex example treeplex (Fig. 1) as
  player 1's strategy space, against one two-action simplex, with seeded
  random payoffs.  The text fixes the two root simplexes (sizes 2 and 3),
  five simplexes at level 2 with the first scaled by q_1, and two at level 3;
  the figure itself is not available, so the remaining parents and sizes are
  a reading: Delta^3 (2) and Delta^4 (3) both under q_1 (a Cartesian
  product), Delta^5 (2) under q_2, Delta^6 (3) under q_3, Delta^7 (2) under
  q_5, Delta^8 (2) under Delta^3's first variable and Delta^9 (3) under
  Delta^6's first variable.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class EfgInstance:
    name: str
    infosets: tuple  # (player-1 list, player-2 list) of (parent_seq, n_actions, key)
    entries: tuple  # ((s1, s2, value), ...) with s1, s2 >= 0; repeated pairs add up
    pot: float  # scale of the payoffs (the gap target is 1e-3 * pot)
    seed: int = 0

    def n_seq(self, p):
        return sum(n for _, n, _ in self.infosets[p])


class _Builder:
    def __init__(self):
        self.sets = [[], []]
        self.index = [{}, {}]  # infoset key -> (first sequence, n_actions)
        self.n_seq = [0, 0]
        self.A = {}

    def seq(self, p, key, parent, n_act, a):
        if key not in self.index[p]:
            self.index[p][key] = (self.n_seq[p], n_act)
            self.sets[p].append((parent, n_act, key))
            self.n_seq[p] += n_act
        first, n = self.index[p][key]
        assert n == n_act, key
        return first + a

    def add(self, s1, s2, v):
        assert s1 >= 0 and s2 >= 0
        self.A[(s1, s2)] = self.A.get((s1, s2), 0.0) + v

    def instance(self, name, pot, seed=0):
        entries = tuple((s1, s2, v) for (s1, s2), v in sorted(self.A.items()) if v != 0.0)
        return EfgInstance(name, (tuple(self.sets[0]), tuple(self.sets[1])), entries, float(pot), seed)


def leduc(raises=(2.0, 4.0), max_bets=2) -> EfgInstance:
    """Leduc hold'em.  Cards 0..5, rank = card // 2; each player antes 1.  In
    round r the bet / raise size is raises[r]; at most max_bets bets or raises
    per round; a player not facing a bet checks or bets, facing one folds,
    calls or raises.  After round 1 (check-check or a call) the public card is
    dealt.  Showdown: a pair with the public card wins, else the higher rank;
    equal ranks split.  Player 2's payoff is its net chips."""
    B = _Builder()
    deals = [(c1, c2, c3) for c1 in range(6) for c2 in range(6) for c3 in range(6)
             if len({c1, c2, c3}) == 3]
    prob = 1.0 / len(deals)

    def strength(c, pub):
        return (1, c // 2) if c // 2 == pub // 2 else (0, c // 2)

    def walk(deal, rnd, hist, bets, contrib, player, last):
        c1, c2, c3 = deal
        own = deal[player] // 2
        pub = (c3 // 2,) if rnd == 1 else ()
        key = (own,) + pub + (hist,)
        facing = contrib[1 - player] > contrib[player]
        acts = (["f", "c"] + (["r"] if bets < max_bets else [])) if facing else (["k"] + (["b"] if bets < max_bets else []))
        for a_i, a in enumerate(acts):
            s = B.seq(player, key, last[player], len(acts), a_i)
            nl = list(last)
            nl[player] = s
            h2 = hist + a
            c = list(contrib)
            if a == "f":
                u2 = c[0] if player == 0 else -c[1]
                B.add(nl[0], nl[1], prob * u2)
                continue
            if a == "c":
                c[player] = c[1 - player]
            elif a in ("b", "r"):
                c[player] = c[1 - player] + raises[rnd]
            closes = a == "c" or (a == "k" and player == 1)
            if not closes:
                walk(deal, rnd, h2, bets + (1 if a in ("b", "r") else 0), tuple(c), 1 - player, tuple(nl))
            elif rnd == 0:
                walk(deal, 1, h2 + "|", 0, tuple(c), 0, tuple(nl))
            else:
                s1, s2 = strength(c1, c3), strength(c2, c3)
                u2 = c[0] if s2 > s1 else (-c[1] if s2 < s1 else 0.0)
                B.add(nl[0], nl[1], prob * u2)

    for deal in deals:
        walk(deal, 0, "", 0, (1.0, 1.0), 0, (-1, -1))
    return B.instance("leduc", pot=2.0)


def kuhn_efg() -> EfgInstance:
    """Kuhn poker (cards 0 < 1 < 2, antes of 1, one bet of 1) as a general
    game: player 1 checks or bets; after a check player 2 checks or bets;
    facing a bet a player folds or calls."""
    B = _Builder()
    deals = [(a, b) for a in range(3) for b in range(3) if a != b]
    prob = 1.0 / len(deals)
    for c1, c2 in deals:
        win2 = 1.0 if c2 > c1 else -1.0
        k1 = B.seq(0, (c1, ""), -1, 2, 0)
        b1 = B.seq(0, (c1, ""), -1, 2, 1)
        k2 = B.seq(1, (c2, "k"), -1, 2, 0)
        b2 = B.seq(1, (c2, "k"), -1, 2, 1)
        B.add(k1, k2, prob * win2 * 1.0)  # check, check: showdown for the antes
        f1 = B.seq(0, (c1, "kb"), k1, 2, 0)
        c1s = B.seq(0, (c1, "kb"), k1, 2, 1)
        B.add(f1, b2, prob * 1.0)  # player 1 folds: player 2 wins its ante
        B.add(c1s, b2, prob * win2 * 2.0)
        f2 = B.seq(1, (c2, "b"), -1, 2, 0)
        c2s = B.seq(1, (c2, "b"), -1, 2, 1)
        B.add(b1, f2, prob * -1.0)  # player 2 folds
        B.add(b1, c2s, prob * win2 * 2.0)
    return B.instance("kuhn_efg", pot=2.0)


def random_efg(seed: int, depth: int = 5, max_actions: int = 3, n_types: int = 3) -> EfgInstance:
    """A seeded random game: chance draws a private type for each player
    (n_types each, random probabilities), then the players alternate for up
    to `depth` decisions with 1 .. max_actions actions (random per public
    history), each decision ending the game with probability 0.3 after both
    have acted; payoffs uniform in [-1, 1] per (history, types)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = _Builder()
    pt = [rng.dirichlet(np.ones(n_types)) for _ in range(2)]
    shape = {}  # public history -> (n_actions, ends_after)

    def layout(hist):
        if hist not in shape:
            n_act = int(rng.integers(1, max_actions + 1))
            ends = [bool(rng.random() < 0.3) for _ in range(n_act)]
            shape[hist] = (n_act, ends)
        return shape[hist]

    payoff = {}

    def walk(types, hist, player, last, d):
        n_act, ends = layout(hist)
        key = (types[player], hist)
        for a in range(n_act):
            s = B.seq(player, key, last[player], n_act, a)
            nl = list(last)
            nl[player] = s
            h2 = hist + (a,)
            acted = nl[0] >= 0 and nl[1] >= 0
            if acted and (ends[a] or d + 1 >= depth):
                if (h2, types) not in payoff:
                    payoff[(h2, types)] = float(rng.uniform(-1.0, 1.0))
                B.add(nl[0], nl[1], pt[0][types[0]] * pt[1][types[1]] * payoff[(h2, types)])
            else:
                walk(types, h2, 1 - player, tuple(nl), d + 1)

    for t1 in range(n_types):
        for t2 in range(n_types):
            walk((t1, t2), (), 0, (-1, -1), 0)
    return B.instance(f"random{seed}", pot=2.0, seed=seed)


def fig1_game(seed: int = 0) -> EfgInstance:
    """Section 3's example treeplex (see the module docstring for the parts
    of Fig. 1 that are a reading) against a single two-action simplex."""
    # (parent sequence, size) per simplex, sequences numbered simplex by simplex:
    # D1: q0 q1 | D2: q2 q3 q4 | D3: q5 q6 | D4: q7 q8 q9 | D5: q10 q11 |
    # D6: q12 q13 q14 | D7: q15 q16 | D8: q17 q18 | D9: q19 q20 q21
    p1 = ((-1, 2, "D1"), (-1, 3, "D2"), (0, 2, "D3"), (0, 3, "D4"), (1, 2, "D5"), (2, 3, "D6"),
          (4, 2, "D7"), (5, 2, "D8"), (12, 3, "D9"))
    p2 = ((-1, 2, "E1"),)
    rng = np.random.Generator(np.random.PCG64(seed))
    entries = tuple((s1, s2, float(rng.uniform(-1.0, 1.0))) for s1 in range(22) for s2 in range(2)
                    if rng.random() < 0.7)
    return EfgInstance(f"fig1_{seed}", (p1, p2), entries, 2.0, seed)
