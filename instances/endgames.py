"""Synthetic poker river endgames with the structure of the paper's workload.

The paper (Section 7, "Experiments") solves river subgames: chance deals
each player a private hand from a prior over hands, the five board cards are
public, and the players then bet with a discrete bet abstraction.  The
Libratus priors are private, so these generators stand in with seeded
synthetic priors of the same shape:

* deck of ``n_cards`` cards numbered ``4*rank + suit``; a seeded board of
  five cards; the hands are all unordered pairs of live (non-board) cards in
  lexicographic order (Kuhn poker instead uses a three-card deck, no board and
  one-card hands);
* hand strengths: integers, larger wins, equal strengths split the pot;
* beliefs: one Dirichlet draw per player over the live hands;
* betting: pot, remaining stack, bet fractions, all-in flag and the maximum
  number of raises after the opening bet.

Every random draw goes through ``numpy.random.Generator(PCG64(seed))`` in a
fixed order (board, strengths, player-1 belief, player-2 belief).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations

import numpy as np


@dataclass(frozen=True)
class BetAbstraction:
    """Situation-dependent bet sizes (the shape of the Libratus river
    abstraction in Section 7).  ``fracs[p][d]`` lists the pot fractions player
    p may bet (d = 0, not facing a bet) or raise by (d >= 1) once d bets or
    raises have been made on the river, d capped at 3 so that ``[p][3]``
    covers every later raise; ``allin[p][d]`` adds all-in there;
    ``open_fold[p]`` lets p fold when not facing a bet."""
    fracs: tuple
    allin: tuple
    open_fold: tuple


# Section 7's description of the Libratus river abstraction, player 1
# (Libratus, first to act) then player 2.
LIBRATUS_RIVER = BetAbstraction(
    fracs=(((0.25, 0.5, 1.0, 2.0, 4.0, 8.0), (0.4, 0.7, 1.1, 2.0), (0.4, 0.7, 2.0), (0.7,)),
           ((0.5, 0.75, 1.0), (0.7, 1.1), (0.7,), (0.7,))),
    allin=((True, True, True, True), (True, True, True, True)),
    open_fold=(True, True),
)


@dataclass(frozen=True)
class Instance:
    name: str
    n_cards: int
    cards_per_hand: int
    board: np.ndarray  # int32 [n_board]
    hand_cards: np.ndarray  # int32 [n_hands, cards_per_hand]
    strength: np.ndarray  # int32 [n_hands]; larger wins, equal ties
    belief: np.ndarray  # float64 [2, n_hands]; player 1 then player 2
    pot: float
    stack: float
    bet_fracs: tuple
    allin: bool
    max_raises: int
    seed: int = 0
    abstraction: BetAbstraction | None = None  # None: bet_fracs / allin in every situation, no open fold
    meta: dict = field(default_factory=dict)

    @property
    def n_hands(self) -> int:
        return int(self.hand_cards.shape[0])


def _pairs(live_cards):
    return np.array(list(combinations(sorted(int(c) for c in live_cards), 2)), dtype=np.int32)


def _tied_ranking(rng, n, tie_prob):
    """Random ranking of ``n`` hands in which each hand joins the group of the
    hand ranked just below it with probability ``tie_prob``."""
    order = rng.permutation(n)
    merge = rng.random(n - 1) < tie_prob
    group = np.concatenate([[0], np.cumsum(~merge)]).astype(np.int32)
    strength = np.empty(n, dtype=np.int32)
    strength[order] = group
    return strength


def kuhn() -> Instance:
    """Kuhn poker as a one-street endgame: cards J<Q<K, one card each, both
    players have already put 1 chip in (pot 2), one bet of 1 chip, no raise."""
    hands = np.arange(3, dtype=np.int32).reshape(3, 1)
    return Instance(
        name="kuhn",
        n_cards=3,
        cards_per_hand=1,
        board=np.zeros(0, dtype=np.int32),
        hand_cards=hands,
        strength=np.arange(3, dtype=np.int32),
        belief=np.full((2, 3), 1.0 / 3.0),
        pot=2.0,
        stack=1.0,
        bet_fracs=(0.5,),
        allin=True,
        max_raises=0,
    )


def river(
    name: str,
    seed: int,
    n_ranks: int,
    strength_kind: str,
    alpha: float,
    pot: float,
    stack: float,
    bet_fracs,
    max_raises: int,
    allin: bool = True,
    n_board: int = 5,
    abstraction: BetAbstraction | None = None,
) -> Instance:
    rng = np.random.Generator(np.random.PCG64(seed))
    n_cards = 4 * n_ranks
    board = np.sort(rng.choice(n_cards, n_board, replace=False)).astype(np.int32)
    live = np.setdiff1d(np.arange(n_cards), board)
    hands = _pairs(live)
    n = hands.shape[0]
    if strength_kind == "int30":
        strength = rng.integers(0, 30, n).astype(np.int32)
    elif strength_kind == "ranking_ties10":
        strength = _tied_ranking(rng, n, 0.1)
    else:
        raise ValueError(strength_kind)
    b1 = rng.dirichlet(alpha * np.ones(n))
    b2 = rng.dirichlet(alpha * np.ones(n))
    return Instance(
        name=name,
        n_cards=n_cards,
        cards_per_hand=2,
        board=board,
        hand_cards=hands,
        strength=strength,
        belief=np.stack([b1, b2]),
        pot=float(pot),
        stack=float(stack),
        bet_fracs=tuple(float(f) for f in bet_fracs),
        allin=bool(allin),
        max_raises=int(max_raises),
        seed=int(seed),
        abstraction=abstraction,
    )


def micro(seed: int = 0, n_ranks: int = 2, n_board: int = 3, bet_fracs=(1.0,), max_raises: int = 1,
          pot: float = 10.0, stack: float = 20.0, alpha: float = 1.0) -> Instance:
    """A few-hand river endgame small enough for an exact LP solve."""
    return river(f"micro{seed}", seed, n_ranks, "int30", alpha, pot, stack, bet_fracs, max_raises,
                 n_board=n_board)


# Shapes of the benchmark workloads.
CONFIGS = {
    "kuhn": None,
    # 20-card deck, 105 hands, strengths uniform integers in [0, 30), Dirichlet(1).
    "c0": dict(n_ranks=5, strength_kind="int30", alpha=1.0, pot=100.0, stack=200.0,
               bet_fracs=(0.5, 1.0), max_raises=2),
    # 52-card deck, 1081 hands, random ranking with ~10% ties, Dirichlet(0.5).
    "c1": dict(n_ranks=13, strength_kind="ranking_ties10", alpha=0.5, pot=1000.0, stack=20000.0,
               bet_fracs=(0.5, 1.0, 2.0), max_raises=3),
    # Large tree: eight bet sizes (seven fractions plus all-in), four raises.
    "c3": dict(n_ranks=13, strength_kind="ranking_ties10", alpha=0.5, pot=1000.0, stack=20000.0,
               bet_fracs=(0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 3.0), max_raises=4),
}
CONFIGS["c2"] = CONFIGS["c1"]
# The Libratus-style river abstraction on a 52-card endgame with Endgame 2's
# pot (2100) and the remaining stacks of 200-big-blind play (20000 - 1050):
# 152 sequences per hand for player 1 and 153 for player 2 (its pass after
# an opening fold), 164,312 and 165,393 over 1081 hands.
CONFIGS["lib"] = dict(n_ranks=13, strength_kind="ranking_ties10", alpha=0.5, pot=2100.0, stack=18950.0,
                      bet_fracs=(), max_raises=8, abstraction=LIBRATUS_RIVER)


# The same rules on a 10-hand endgame (8-card deck, 3 board cards): small
# enough for the exact LP and for game walks deal by deal.
CONFIGS["lib_micro"] = dict(n_ranks=2, strength_kind="int30", alpha=1.0, pot=10.0, stack=20.0, bet_fracs=(),
                            max_raises=8, n_board=3, abstraction=LIBRATUS_RIVER)

# Kuhn poker where either player may also fold when not facing a bet (the
# only size is all-in): folding first, or facing a check, is never better
# than checking, so the game value is Kuhn's.
KUHN_OPEN_FOLD = BetAbstraction(fracs=(((),) * 4, ((),) * 4), allin=((True,) * 4, (True,) * 4),
                                open_fold=(True, True))


def make_instance(config: str, seed: int = 0) -> Instance:
    if config == "kuhn":
        return kuhn()
    if config == "kuhn_open_fold":
        k = kuhn()
        return Instance(**{**{f: getattr(k, f) for f in k.__dataclass_fields__}, "name": config,
                           "bet_fracs": (), "abstraction": KUHN_OPEN_FOLD})
    if config.startswith("micro"):
        return micro(seed)
    return river(config, seed, **CONFIGS[config])


def serving_trace(n_requests: int, rate: float, seed: int, shapes=("c0", "c1", "c2", "c3")):
    """Poisson request stream: exponential inter-arrival gaps of mean 1/rate
    seconds; each request's shape is a uniform choice among ``shapes`` and its
    instance seed is drawn from the same generator."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, n_requests) if rate > 0 else np.zeros(n_requests)
    arrivals = np.cumsum(gaps) - (gaps[0] if n_requests else 0.0)
    kinds = rng.integers(0, len(shapes), n_requests)
    seeds = rng.integers(0, 2**31 - 1, n_requests)
    return [(float(arrivals[i]), shapes[int(kinds[i])], int(seeds[i])) for i in range(n_requests)]
