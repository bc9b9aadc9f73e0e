"""Oracle, part 5: mirror prox and Chambolle-Pock with the dilated entropy (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 8 names these first-order methods as likely faster than EGT on the
same problem.  Both need only the operations EGT uses: the products A y,
A^T x and the prox step of the dilated entropy, here the Bregman prox
    prox_c(g) = argmin_q <g, q> + D(q, c) = SBR(g - grad d(c), 1)
from a centre c, with grad d from the appendix (the same literal form the
EGT oracle uses for Algorithm 2's prox step).

* Mirror prox (Nemirovski's extragradient with a Bregman distance), step eta
  (eta_y for player 2 when given, else eta):
      x^ = prox_{x_t}(eta A y_t),          y^ = prox_{y_t}(-eta A^T x_t),
      x_{t+1} = prox_{x_t}(eta A y^),      y_{t+1} = prox_{y_t}(-eta A^T x^),
  averages of the extrapolated points x^, y^ (uniform weights); with
  eta <= 1 / L, L = ||A|| M (max |A_ij| times the largest l1 norm on the
  treeplexes, against which d is 1/M-strongly convex), the averages' saddle
  gap after T iterations is at most (Omega_X + Omega_Y) / (eta T).
* Chambolle-Pock (primal-dual hybrid gradient with Bregman proximal terms),
  steps tau, sigma:
      x_{t+1} = prox_{x_t}(tau A y_t),
      y_{t+1} = prox_{y_t}(-sigma A^T (2 x_{t+1} - x_t)),
  averages of x_{t+1}, y_{t+1} (uniform weights).
Both start at the DGF's minimiser (the uniform point).  Mirror prox makes
four products per iteration, Chambolle-Pock two.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .problem import Problem


@dataclass
class FomTrace:
    rows: list = field(default_factory=list)
    x_avg: np.ndarray | None = None
    y_avg: np.ndarray | None = None
    iters: int = 0
    products: int = 0
    gap: float = float("nan")


def bregman_prox(P: Problem, p: int, centre: np.ndarray, g: np.ndarray) -> np.ndarray:
    """argmin_q <g, q> + D(q, centre) over p's treeplex (centre interior):
    the smoothed best response with weight 1 to g - grad d(centre), grad d
    from the appendix (through the centre's local log q_bar)."""
    t = P.tp[p]
    lqb = np.zeros_like(centre)
    for node in t.nodes:
        sl = slice(node.first_seq, node.first_seq + node.n_act)
        par = np.ones(P.n) if node.parent_seq < 0 else centre[node.parent_seq]
        lqb[sl] = np.log(centre[sl] / par[None, :])
    return P.sbr(p, g - P.dgf_grad(p, lqb), 1.0)[0]


def theory_step(P: Problem) -> float:
    """1 / L with L = ||A|| max(M_X, M_Y): the mirror-prox step size of the theory."""
    return 1.0 / (P.norm_A() * max(P.max_l1(0), P.max_l1(1)))


class MirrorProx:
    def __init__(self, prob: Problem, eta: float, eta_y: float | None = None):
        self.P, self.eta = prob, float(eta)
        self.eta_y = self.eta if eta_y is None else float(eta_y)
        self.x, self.y = prob.uniform(0), prob.uniform(1)
        self.sx, self.sy = np.zeros_like(self.x), np.zeros_like(self.y)
        self.t, self.products = 0, 0

    def step(self):
        P, eta, eta_y = self.P, self.eta, self.eta_y
        xh = bregman_prox(P, 0, self.x, eta * P.grad_x(self.y))
        yh = bregman_prox(P, 1, self.y, -eta_y * P.grad_y(self.x))
        x_next = bregman_prox(P, 0, self.x, eta * P.grad_x(yh))
        y_next = bregman_prox(P, 1, self.y, -eta_y * P.grad_y(xh))
        self.x, self.y = x_next, y_next
        self.sx, self.sy = self.sx + xh, self.sy + yh
        self.t += 1
        self.products += 4

    def average(self):
        return self.sx / self.t, self.sy / self.t


class ChambollePock:
    def __init__(self, prob: Problem, tau: float, sigma: float):
        self.P, self.tau, self.sigma = prob, float(tau), float(sigma)
        self.x, self.y = prob.uniform(0), prob.uniform(1)
        self.sx, self.sy = np.zeros_like(self.x), np.zeros_like(self.y)
        self.t, self.products = 0, 0

    def step(self):
        P = self.P
        x_next = bregman_prox(P, 0, self.x, self.tau * P.grad_x(self.y))
        y_next = bregman_prox(P, 1, self.y, -self.sigma * P.grad_y(2.0 * x_next - self.x))
        self.x, self.y = x_next, y_next
        self.sx, self.sy = self.sx + x_next, self.sy + y_next
        self.t += 1
        self.products += 2

    def average(self):
        return self.sx / self.t, self.sy / self.t


def run_fom(method, iters: int, gap_every: int = 1) -> FomTrace:
    tr = FomTrace()
    P = method.P
    while method.t < iters:
        method.step()
        if method.t % gap_every == 0 or method.t == iters:
            xa, ya = method.average()
            gap, brmax, brmin = P.saddle_gap(xa, ya)
            tr.rows.append(dict(t=method.t, gap=gap, br_max_y=brmax, br_min_x=brmin))
            tr.gap = gap
    tr.x_avg, tr.y_avg = method.average()
    tr.iters, tr.products = method.t, method.products
    return tr
