"""Oracle, part 3: the excessive gap technique (FP64, step by step).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's algorithms in their own order:

* ``EGT`` (Algorithm 1): start at x0 = x_{mu_x}(y0), y0 = y_{mu_y}(x_omega);
  tau_t = 2 / (t + 3); steps alternate between x (even t) and y (odd t);
  stop when the saddle-point residual eps_sad <= eps.
* ``Step`` (Algorithm 2), for the x side:
      x_hat = (1 - tau) x + tau x_{mu_x}(y)
      y_+   = (1 - tau) y + tau y_{mu_y}(x_hat)
      x_til = grad d*( grad d(x_{mu_x}(y)) - tau / ((1 - tau) mu_x) grad f_{mu_y}(x_hat) )
      x_+   = (1 - tau) x + tau x_til
      mu_x+ = (1 - tau) mu_x
  The y side is the same step on the mirrored problem min_y max_x <y, -A^T x>.
  ``grad d*`` is computed as the prox of Section 4: the smoothed best response
  with mu = 1 of the shifted gradient  tau/((1-tau) mu_x) A y_bar - grad d(x_bar),
  with grad d from the appendix.  The equivalent shift-free form
  SBR(A y + tau/(1-tau) A y_bar, mu_x) is computed beside it and the largest
  difference is recorded.
* ``BAL`` (Section 5, mu balancing): as EGT, but step the player with the
  larger mu.
* ``AS`` (Algorithms 3 and 4, aggressive mu reduction): keep tau (initially
  1/2) across iterations; after each step test the excessive gap condition
  and, while EGV < 0, halve tau and redo the step from the same point.

Readings where the paper is silent or garbled:
* Algorithm 1's first line is taken with a minus sign, x0 = grad d*(-f'/mu_x),
  i.e. x0 is player 1's smoothed best response to A y0 (as in Algorithm 2);
* the "practically tuned" initial mu is not given: mu0 = 1e-3 times the
  largest gradient entry at the uniform point over the largest beta, doubled
  for both players until the excessive gap condition holds at (x0, y0);
* Algorithm 4 tests EGV at the new point (x+, y+) with mu+ and the other
  player's unchanged mu, strictly "< 0", and returns (mu+, x+, y+, tau).
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
    products_paper: int = 0
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

    def step(self, p, mu_p, mu_o, own, other, tau):
        """Algorithm 2 focused on player p.  Returns (mu_p+, own+, other+, prox_diff)."""
        o = 1 - p
        g1 = self.G(p, other)
        own_bar, _, lqb, _ = self.P.sbr(p, g1, mu_p)
        own_hat = (1.0 - tau) * own + tau * own_bar
        other_bar = self.P.sbr(o, self.G(o, own_hat), mu_o)[0]
        other_plus = (1.0 - tau) * other + tau * other_bar
        g3 = self.G(p, other_bar)
        shifted = tau / ((1.0 - tau) * mu_p) * g3 - self.P.dgf_grad(p, lqb)
        own_til_lit = self.P.sbr(p, shifted, 1.0)[0]
        own_til_free = self.P.sbr(p, g1 + tau / (1.0 - tau) * g3, mu_p)[0]
        diff = float(np.max(np.abs(own_til_lit - own_til_free)))
        own_til = own_til_lit if self.literal else own_til_free
        own_plus = (1.0 - tau) * own + tau * own_til
        return (1.0 - tau) * mu_p, own_plus, other_plus, diff


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
        tr.products_paper += (4 + 3 * r["backtracks"]) if variant == "AS" else 3
        x, y, mu_x, mu_y = r["x"], r["y"], r["mu_x"], r["mu_y"]
        if variant == "AS":
            tau = r["tau"]
        t += 1
    tr.x, tr.y, tr.iters = x, y, t
    tr.value_p2 = prob.value(x, y)
    return tr
