"""Pins for the oracle's mirror prox and Chambolle-Pock (CPU only).

* Bregman prox of the dilated entropy: optimality against random feasible
  points (the prox objective with D computed from d and its general
  gradient), the uniform centre reducing it to the smoothed best response
  with weight 1, and the identity prox_{SBR(h, 1)}(g) = SBR(h + g, 1) on
  which a dual-averaging implementation relies.
* Mirror prox (Nemirovski): with the theory step 1 / (||A|| M) the averages'
  saddle gap is at most (Omega_X + Omega_Y) / (eta T); on Kuhn poker the
  averages approach the textbook value.
* Chambolle-Pock: the averages approach Kuhn's value and their gap shrinks.
* Gradient accounting: four products per mirror-prox iteration, two per
  Chambolle-Pock iteration.
"""
import os

import numpy as np
import pytest

from instances import make_instance
from oracle import ChambollePock, MirrorProx, Problem, bregman_prox, run_fom, theory_step


def _golden_kuhn():
    path = os.path.join(os.path.dirname(__file__), "golden", "kuhn_value.txt")
    for line in open(path):
        if line.startswith("value_player1"):
            return float(line.split("=")[1])
    raise AssertionError("fixture missing")


def _random_point(P, p, rng):
    t = P.tp[p]
    q = np.zeros((t.n_seq, P.n))
    for v in reversed(t.post_order):
        node = t.nodes[v]
        par = np.ones(P.n) if node.parent_seq < 0 else q[node.parent_seq]
        q[node.first_seq:node.first_seq + node.n_act] = par[None, :] * rng.dirichlet(np.ones(node.n_act), size=P.n).T
    return q


def _bregman(P, p, q, c):
    return P.dgf(p, q) - P.dgf(p, c) - float(np.sum(P.dgf_grad_free(p, c) * (q - c)))


@pytest.mark.parametrize("cfg,p", [("kuhn", 0), ("kuhn", 1), ("micro", 0), ("lib_micro", 1)])
def test_bregman_prox(cfg, p):
    P = Problem(make_instance(cfg, 0))
    rng = np.random.default_rng(5)
    c = _random_point(P, p, rng)
    g = rng.standard_normal(c.shape)
    q = bregman_prox(P, p, c, g)
    assert P.flow_residual(p, q) < 1e-12
    best = float(np.sum(g * q)) + _bregman(P, p, q, c)
    for _ in range(30):
        r = _random_point(P, p, rng)
        assert float(np.sum(g * r)) + _bregman(P, p, r, c) >= best - 1e-9
    # from the DGF's minimiser the prox is the smoothed best response with weight 1
    u = P.uniform(p)
    assert np.abs(bregman_prox(P, p, u, g) - P.sbr(p, g, 1.0)[0]).max() < 1e-12
    # from a smoothed best response SBR(h, 1) the prox is SBR(h + g, 1)
    h = rng.standard_normal(c.shape) * 3.0
    centre = P.sbr(p, h, 1.0)[0]
    assert np.abs(bregman_prox(P, p, centre, g) - P.sbr(p, h + g, 1.0)[0]).max() < 1e-12


def test_mirror_prox_rate_at_the_theory_step():
    P = Problem(make_instance("kuhn"))
    eta = theory_step(P)
    M = MirrorProx(P, eta)
    bound_num = P.omega(0) + P.omega(1)
    for T in (20, 100, 500):
        while M.t < T:
            M.step()
        xa, ya = M.average()
        gap, _, _ = P.saddle_gap(xa, ya)
        assert 0.0 <= gap <= bound_num / (eta * T), (T, gap, bound_num / (eta * T))
    assert M.products == 4 * 500


@pytest.mark.parametrize("cls,kw", [(MirrorProx, dict(eta=2.0)), (ChambollePock, dict(tau=2.0, sigma=2.0))])
def test_kuhn_averages_approach_the_value(cls, kw):
    P = Problem(make_instance("kuhn"))
    tr = run_fom(cls(P, **kw), 1500, gap_every=100)
    assert tr.rows[-1]["gap"] < 0.3 * tr.rows[0]["gap"]
    assert tr.gap < 0.02
    assert abs(P.value(tr.x_avg, tr.y_avg) - (-_golden_kuhn())) <= tr.gap
    assert P.flow_residual(0, tr.x_avg) < 1e-12 and P.flow_residual(1, tr.y_avg) < 1e-12
    assert tr.products == (4 if cls is MirrorProx else 2) * 1500
