"""Oracle, part 3: the excessive gap technique (FP64, step by step).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method (Section 2) keeps a strategy pair (x, y) and two smoothing weights
(mu_x, mu_y) for which the excessive gap value
    EGV = [min_x <x, A y> + mu_x d_X(x)] - [max_y <x, A y> - mu_y d_Y(y)]
is non-negative; while that holds, the saddle-point residual is at most
mu_x Omega_X + mu_y Omega_Y.  Every iteration shrinks one player's weight by
the factor (1 - tau) and moves both strategies so that the condition survives.

One iteration focused on player p (Algorithm 2; o is the opponent):
  * the anchor: p's smoothed best response to the opponent's current
    strategy, an interior point of p's treeplex;
  * p's strategy mixed toward the anchor with weight tau; the opponent
    answers that mixed point with its own smoothed best response and moves
    toward the answer with the same weight;
  * p's prox step from the anchor (Section 4): the minimiser of the linear
    term tau / ((1 - tau) mu_p) <g, q> plus the Bregman divergence of d from
    the anchor, where g is p's gradient at the opponent's answer.  It is the
    smoothed best response with weight 1 to that scaled gradient minus
    grad d(anchor), grad d taken from the appendix;
  * p moves toward the prox point with weight tau, and mu_p shrinks.
The focus on y is the same iteration on the mirrored problem
min_y max_x <y, -A^T x>.  Beside the prox through grad d the oracle computes
the equivalent shift-free form, the smoothed best response with weight mu_p
to (gradient at the opponent's current strategy) + tau/(1 - tau) g, and
records the largest difference between the two.

Drivers:
* ``ALT`` (Algorithm 1): tau_t = 2 / (t + 3), focus on x at even t and on y
  at odd t, start x0 = x_{mu_x}(y0), y0 = y_{mu_y}(x_omega), stop when the
  saddle-point residual reaches eps;
* ``BAL`` (Section 5, mu balancing): as ALT but the focus goes to the player
  with the larger mu;
* ``AS`` (Algorithms 3 and 4): tau starts at 1/2, is kept between iterations,
  and is halved (redoing the iteration from the same point) for as long as
  the excessive gap value after the iteration is negative.

Readings where the paper is silent or garbled:
* Algorithm 1's first line is taken with a minus sign: x0 is player 1's
  smoothed best response to A y0, as in Algorithm 2's prox step;
* the "practically tuned" initial mu is a convention of this implementation:
  1e-3 times the largest gradient entry at the uniform point over the largest
  beta, doubled for both players until the excessive gap condition holds at
  (x0, y0);
* Algorithm 4 tests EGV at the new point with the reduced mu and the other
  player's unchanged mu, strictly "< 0", and hands back the new point, the
  reduced mu and the tau that was accepted.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .problem import Problem


@dataclass
class Trace:
    rows: list = field(default_factory=list)
    x: np.ndarray | None = None
    y: np.ndarray | None = None
    mu0: tuple = (0.0, 0.0)
    iters: int = 0
    backtracks: int = 0
    gap: float = float("nan")
    value_p2: float = float("nan")
    max_prox_diff: float = 0.0
    converged: bool = False


class EGT:
    def __init__(self, prob: Problem, literal: bool = True):
        self.P = prob
        self.literal = literal

    # the gradient each player minimises against: player 1 <x, A y>,
    # player 2 <y, -A^T x> (the mirrored problem of the y-focused step)
    def G(self, p, other):
        return self.P.grad_x(other) if p == 0 else -self.P.grad_y(other)

    def auto_mu0(self):
        xw, yw = self.P.uniform(0), self.P.uniform(1)
        gmax = max(np.abs(self.P.grad_x(yw)).max(), np.abs(self.P.grad_y(xw)).max())
        bmax = max(v.beta for t in self.P.tp for v in t.nodes)
        return 1e-3 * gmax / bmax

    def init_point(self, mu_x, mu_y):
        """Algorithm 1's start-up: y0 = y_{mu_y}(x_omega), x0 = x_{mu_x}(y0)."""
        xw = self.P.uniform(0)
        y0 = self.P.sbr(1, self.G(1, xw), mu_y)[0]
        x0 = self.P.sbr(0, self.G(0, y0), mu_x)[0]
        return x0, y0

    def egv(self, x, y, mu_x, mu_y):
        return self.P.egv(x, y, mu_x, mu_y)[0]

    def anchor(self, p, g_other, mu_p):
        """p's smoothed best response to its gradient g_other at the opponent's
        current strategy: (point, local log q_bar)."""
        q, _, lqb, _ = self.P.sbr(p, g_other, mu_p)
        return q, lqb

    def prox(self, p, anchor_lqb, g, scale):
        """Section 4's prox from an interior anchor: argmin_q scale <g, q> + D(q, anchor),
        D the Bregman divergence of the dilated entropy; the linear part of D is
        -grad d(anchor), so the minimiser is the smoothed best response with
        weight 1 to scale g - grad d(anchor) (the appendix's gradient)."""
        return self.P.sbr(p, scale * g - self.P.dgf_grad(p, anchor_lqb), 1.0)[0]

    def step(self, p, mu_p, mu_o, own, other, tau):
        """Algorithm 2 focused on player p.  Returns (mu_p+, own+, other+, prox_diff)."""
        o = 1 - p
        g_other = self.G(p, other)
        anc, anc_lqb = self.anchor(p, g_other, mu_p)
        own_mixed = (1.0 - tau) * own + tau * anc
        answer = self.P.sbr(o, self.G(o, own_mixed), mu_o)[0]
        other_next = (1.0 - tau) * other + tau * answer
        g_answer = self.G(p, answer)
        target = self.prox(p, anc_lqb, g_answer, tau / ((1.0 - tau) * mu_p))
        # shift-free form of the same prox (the anchor is the smoothed response to G(p, other))
        target_free = self.P.sbr(p, g_other + tau / (1.0 - tau) * g_answer, mu_p)[0]
        diff = float(np.max(np.abs(target - target_free)))
        if not self.literal:
            target = target_free
        own_next = (1.0 - tau) * own + tau * target
        return (1.0 - tau) * mu_p, own_next, other_next, diff


def iterate(E: EGT, variant: str, t: int, x, y, mu_x: float, mu_y: float, tau: float, side=None,
            tau_floor: float = 1e-30, record_egv: bool = True):
    """One iteration of Algorithm 1 (ALT), mu-balanced EGT (BAL) or Algorithm 3
    with the Decr of Algorithm 4 (AS), from iterate t = (x, y, mu_x, mu_y) and
    (for AS) the current tau.  ``side`` forces the player stepped.
    Returns dict(x, y, mu_x, mu_y, tau, side, egv, backtracks, prox_diff)."""
    if variant in ("ALT", "BAL"):
        tau = 2.0 / (t + 3.0)
    if side is None:
        if variant == "ALT":
            side = 0 if t % 2 == 0 else 1
        elif variant in ("BAL", "AS"):
            side = 0 if mu_x > mu_y else 1
        else:
            raise ValueError(variant)
    bt = 0
    diff = 0.0
    while True:
        if side == 0:
            mu_new, x_new, y_new, d = E.step(0, mu_x, mu_y, x, y, tau)
            mus_new = (mu_new, mu_y)
        else:
            mu_new, y_new, x_new, d = E.step(1, mu_y, mu_x, y, x, tau)
            mus_new = (mu_x, mu_new)
        diff = max(diff, d)
        if variant != "AS":
            egv = E.egv(x_new, y_new, *mus_new) if record_egv else float("nan")
            break
        egv = E.egv(x_new, y_new, *mus_new)
        if not egv < 0.0:
            break
        tau *= 0.5
        bt += 1
        if tau < tau_floor:
            raise RuntimeError("tau fell below the floor")
    return dict(x=x_new, y=y_new, mu_x=mus_new[0], mu_y=mus_new[1], tau=tau, side=side, egv=egv,
                backtracks=bt, prox_diff=diff)


def solve(prob: Problem, variant: str = "AS", eps: float | None = None, max_iters: int = 10000,
          mu0=None, tau0: float = 0.5, literal: bool = True, record_egv: bool = True,
          max_doublings: int = 200, tau_floor: float = 1e-30, on_iterate=None) -> Trace:
    """Run EGT (``ALT``), mu-balanced EGT (``BAL``) or EGT/as (``AS``).

    eps defaults to 1e-3 * pot.  mu0 = None applies the automatic rule and
    doubles both mus until the excessive gap condition holds at the start;
    an explicit (mu_x, mu_y) is used as given.  ``on_iterate(t, x, y, mu_x,
    mu_y, tau)`` is called with every iterate before its gap test."""
    E = EGT(prob, literal=literal)
    if eps is None:
        eps = 1e-3 * prob.inst.pot
    if mu0 is None:
        m = E.auto_mu0()
        mu_x = mu_y = m
        x, y = E.init_point(mu_x, mu_y)
        k = 0
        while E.egv(x, y, mu_x, mu_y) < 0.0:
            k += 1
            if k > max_doublings:
                raise RuntimeError("no initial mu satisfies the excessive gap condition")
            mu_x, mu_y = 2.0 * mu_x, 2.0 * mu_y
            x, y = E.init_point(mu_x, mu_y)
    else:
        mu_x, mu_y = float(mu0[0]), float(mu0[1])
        x, y = E.init_point(mu_x, mu_y)
    tr = Trace(mu0=(mu_x, mu_y))
    tau = tau0
    t = 0
    while True:
        if on_iterate is not None:
            on_iterate(t, x, y, mu_x, mu_y, tau)
        gap, brmax, brmin = prob.saddle_gap(x, y)
        row = dict(t=t, mu_x=mu_x, mu_y=mu_y, gap=gap, br_max_y=brmax, br_min_x=brmin)
        if gap <= eps or t >= max_iters:
            tr.rows.append(row)
            tr.converged = gap <= eps
            tr.gap = gap
            break
        r = iterate(E, variant, t, x, y, mu_x, mu_y, tau, tau_floor=tau_floor, record_egv=record_egv)
        tr.max_prox_diff = max(tr.max_prox_diff, r["prox_diff"])
        row.update(side=r["side"], tau=r["tau"], egv=r["egv"], backtracks=r["backtracks"])
        tr.rows.append(row)
        tr.backtracks += r["backtracks"]
        x, y, mu_x, mu_y = r["x"], r["y"], r["mu_x"], r["mu_y"]
        if variant == "AS":
            tau = r["tau"]
        t += 1
    tr.x, tr.y, tr.iters = x, y, t
    tr.value_p2 = prob.value(x, y)
    return tr
