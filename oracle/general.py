"""Oracle, part 6: general extensive-form games in sequence form (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 names the general route for games without the river structure:
write the sequence-form payoff matrix A out explicitly and apply it as a
sparse matrix.  Here a game is given by each player's information sets (the
parent sequence and the number of actions of every simplex of the treeplex,
Section 3, Definition 2) and A's nonzero entries (player 2's expected
payoff, player 1's loss, chance folded in).  The oracle assembles A densely
and applies it with a plain matrix product; every treeplex operation (the
dilated entropy, the smoothed best response, the best response, the saddle
gap) is the river oracle's own, run with a single column (one "hand"),
since nothing in those definitions depends on the hand dimension.
"""
from __future__ import annotations

import numpy as np

from .game import InfoNode, Treeplex
from .problem import Problem


def build_treeplex(player: int, infosets) -> Treeplex:
    """Treeplex of one player from (parent_seq, n_actions, key) per
    information set, sequences numbered set by set in the given order.
    beta_j = 2 + sum over the child simplexes of 2 beta_k and the height, as
    in the river oracle (Section 4's dilated entropy)."""
    nodes, first = [], 0
    owner = []  # sequence -> (node, action)
    for k, (parent, n_act, key) in enumerate(infosets):
        if not (-1 <= parent < first):
            raise ValueError("a parent sequence must belong to an earlier information set")
        if n_act < 1:
            raise ValueError("an information set needs an action")
        nodes.append(InfoNode(key=str(key), history=(), parent_seq=parent, first_seq=first, n_act=n_act,
                              children=[[] for _ in range(n_act)]))
        owner += [(k, a) for a in range(n_act)]
        first += n_act
    for i, v in enumerate(nodes):
        if v.parent_seq >= 0:
            par, a = owner[v.parent_seq]
            nodes[par].children[a].append(i)
    order = []

    def visit(i):
        for ch in nodes[i].children:
            for k in ch:
                visit(k)
        order.append(i)

    for i, v in enumerate(nodes):
        if v.parent_seq < 0:
            visit(i)
    for i in order:
        v = nodes[i]
        kids = [k for ch in v.children for k in ch]
        v.beta = 2.0 + sum(2.0 * nodes[k].beta for k in kids)
        v.height = 1 + max((nodes[k].height for k in kids), default=0)
    return Treeplex(player, nodes, [str(s) for s in range(first)], order)


class GeneralProblem(Problem):
    """Problem interface of the river oracle for a general game: vectors are
    float64[S_p, 1]."""

    def __init__(self, inst):
        self.inst = inst
        self.game = None
        self.n = 1
        self.tp = [build_treeplex(p, inst.infosets[p]) for p in (0, 1)]
        self.n_seq = [t.n_seq for t in self.tp]
        self.A = np.zeros((self.n_seq[0], self.n_seq[1]))
        for s0, s1, v in inst.entries:
            self.A[s0, s1] += v

    def grad_x(self, y):
        """A y (Section 2's gradient operator for player 1)."""
        return self.A @ y

    def grad_y(self, x):
        """A^T x (the operator for player 2)."""
        return self.A.T @ x

    def norm_A(self):
        """l1 operator norm of A = its largest absolute entry."""
        return float(np.abs(self.A).max()) if self.A.size else 0.0

    def explicit_A(self):
        return self.A.copy()
