"""Oracle, part 4: counterfactual regret minimisation on the same treeplexes (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 7 compares EGT with three regret-based methods that need two
gradient computations per iteration: CFR with regret matching (CFR(RM)), CFR
with regret matching+ (CFR(RM+)) and CFR+.  The paper cites their
definitions; they are restated here from the sequence form:

* player p's gradient g at the opponent's current strategy (A y for player 1,
  -A^T x for player 2, both losses) holds the counterfactual loss of every
  sequence with p's own reach left out;
* bottom-up over the treeplex under p's current local strategy q_bar, the
  counterfactual loss of action a at information set v is
  g~_a = g[v, a] + sum over the child sets k of V[k], and the set's loss is
  V[v] = sum_a q_bar_a g~_a;
* the instantaneous regret of a is V[v] - g~_a, taken as exactly zero when it
  is within 1e-12 of |V[v]| + |g~_a| + S, S the largest |g| entry of the
  player's gradient in this iteration (where actions tie exactly, by the
  game's symmetry or because no opponent mass reaches them, a product
  computed in another order leaves a rounding residue of the order of
  1e-16 S whose sign would flip regret matching between a uniform and a pure
  strategy); regret matching adds it to
  the cumulative regret R_a and plays q_bar_a proportional to max(R_a, 0)
  (uniform when no R_a is positive); regret matching+ floors the cumulative
  regret at zero after each addition, R_a <- max(R_a + r_a, 0);
* the sequence-form strategy follows top-down, x[s] = x[parent] q_bar[s].

Variants (reading of the cited methods):
* ``CFR``    regret matching, both players updated against the strategies
             of the same iteration, uniform average of the iterates;
* ``CFR_RMP`` the same with regret matching+;
* ``CFR_PLUS`` regret matching+, player 2 updated against player 1's new
             strategy (alternation), average weighted by the iteration index.
The average after T iterations is sum_{t<=T} w_t x_t / sum w_t over the
strategies x_1 .. x_T whose regrets were accumulated (x_1 uniform), kept as a
running convex combination avg <- (1 - tau) avg + tau x_t, tau = w_t / W_t;
its saddle gap measures convergence.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .problem import Problem

VARIANTS = ("CFR", "CFR_RMP", "CFR_PLUS")


@dataclass
class CfrTrace:
    rows: list = field(default_factory=list)
    x_avg: np.ndarray | None = None
    y_avg: np.ndarray | None = None
    iters: int = 0
    products: int = 0
    gap: float = float("nan")
    value_p2: float = float("nan")
    regrets: tuple = ()


class Cfr:
    """State of one CFR run: cumulative regrets and local strategies per
    player, the current sequence-form strategies and the running averages."""

    def __init__(self, prob: Problem, variant: str = "CFR_PLUS"):
        if variant not in VARIANTS:
            raise ValueError(variant)
        self.P = prob
        self.variant = variant
        self.plus = variant in ("CFR_RMP", "CFR_PLUS")
        self.alternate = variant == "CFR_PLUS"
        self.linear = variant == "CFR_PLUS"
        self.R = [np.zeros((t.n_seq, prob.n)) for t in prob.tp]
        self.qbar = [self._uniform_local(p) for p in (0, 1)]
        self.cur = [self.sequence_form(p, self.qbar[p]) for p in (0, 1)]
        self.avg = [self.cur[0].copy(), self.cur[1].copy()]  # before any iteration: x_1
        self.wsum = 0.0
        self.t = 0
        self.products = 0

    def weight(self, t):
        return float(t) if self.linear else 1.0

    def _uniform_local(self, p):
        t = self.P.tp[p]
        q = np.zeros((t.n_seq, self.P.n))
        for node in t.nodes:
            q[node.first_seq:node.first_seq + node.n_act] = 1.0 / node.n_act
        return q

    def sequence_form(self, p, qbar):
        """x[s] = x[parent] q_bar[s], root sequences first."""
        t = self.P.tp[p]
        x = np.zeros_like(qbar)
        for v in reversed(t.post_order):
            node = t.nodes[v]
            sl = slice(node.first_seq, node.first_seq + node.n_act)
            par = np.ones(self.P.n) if node.parent_seq < 0 else x[node.parent_seq]
            x[sl] = par[None, :] * qbar[sl]
        return x

    def regret_update(self, p, g):
        """One regret-matching update of player p on its loss gradient g."""
        t = self.P.tp[p]
        V = np.zeros((len(t.nodes), self.P.n))
        R, qbar = self.R[p], self.qbar[p]
        S = float(np.abs(g).max()) if g.size else 0.0
        for v in t.post_order:  # children first
            node = t.nodes[v]
            sl = slice(node.first_seq, node.first_seq + node.n_act)
            gt = g[sl].copy()
            for a in range(node.n_act):
                for k in node.children[a]:
                    gt[a] += V[k]
            V[v] = (qbar[sl] * gt).sum(axis=0)
            r = V[v][None, :] - gt
            # exact ties: a regret within 1e-12 of the values it is the
            # difference of, or of the gradient's scale, is zero (its sign
            # would be rounding noise)
            r = np.where(np.abs(r) <= 1e-12 * (np.abs(V[v])[None, :] + np.abs(gt) + S), 0.0, r)
            R[sl] = R[sl] + r
            if self.plus:
                R[sl] = np.maximum(R[sl], 0.0)
            pos = np.maximum(R[sl], 0.0)
            tot = pos.sum(axis=0)
            qbar[sl] = np.where(tot[None, :] > 0.0, pos / np.where(tot > 0.0, tot, 1.0)[None, :],
                                1.0 / node.n_act)
        return V

    def step(self):
        """Iteration t = self.t + 1: x_t, y_t join the averages with weight
        w_t; both players' regrets are updated (player 2 against player 1's
        new strategy under alternation) and give x_{t+1}, y_{t+1}."""
        P = self.P
        x_t, y_t = self.cur
        t = self.t + 1
        w = self.weight(t)
        self.wsum += w
        tau = w / self.wsum
        self.avg = [(1.0 - tau) * self.avg[0] + tau * x_t, (1.0 - tau) * self.avg[1] + tau * y_t]
        g1 = P.grad_x(y_t)
        self.regret_update(0, g1)
        x_new = self.sequence_form(0, self.qbar[0])
        g2 = -P.grad_y(x_new if self.alternate else x_t)
        self.regret_update(1, g2)
        y_new = self.sequence_form(1, self.qbar[1])
        self.products += 2
        self.t = t
        self.cur = [x_new, y_new]


def solve_cfr(prob: Problem, variant: str = "CFR_PLUS", iters: int = 1000, eps: float | None = None,
              gap_every: int = 1, on_iterate=None) -> CfrTrace:
    """Run `iters` iterations (or until the average's gap is <= eps, tested
    every gap_every iterations).  After t iterations the average holds
    x_1 .. x_t (x_1 before the first), weighted by w_t (1, or t under CFR+)."""
    C = Cfr(prob, variant)
    tr = CfrTrace()
    while True:
        if on_iterate is not None:
            on_iterate(C)
        if C.t % gap_every == 0 or C.t >= iters:
            gap, brmax, brmin = prob.saddle_gap(C.avg[0], C.avg[1])
            tr.rows.append(dict(t=C.t, gap=gap, br_max_y=brmax, br_min_x=brmin))
            tr.gap = gap
            if (eps is not None and gap <= eps) or C.t >= iters:
                break
        C.step()
    tr.x_avg, tr.y_avg = C.avg
    tr.iters = C.t
    tr.products = C.products
    tr.value_p2 = prob.value(C.avg[0], C.avg[1])
    tr.regrets = (C.R[0], C.R[1])
    return tr
