"""Pins for the oracle's CFR(RM), CFR(RM+) and CFR+ (CPU only).

* Kuhn poker: the averages of every variant approach the textbook value
  (golden fixture) and their saddle gap shrinks.
* Regret decomposition (Zinkevich et al.'s bound, the basis of CFR): with
  simultaneous updates and a uniform average, the saddle gap of the average
  after T iterations equals the two players' external regrets over T, and
  each external regret is at most the sum over information sets of the
  largest positive cumulative counterfactual regret.  Regret matching+ keeps
  cumulative regrets at or above the true ones, so the bound holds for it too.
* Invariants: regret-matching+ regrets are non-negative; local strategies lie
  in their simplexes; the averages satisfy the sequence-form flow constraints.
"""
import os

import numpy as np
import pytest

from instances import make_instance
from oracle import Cfr, Problem, solve_cfr


def _golden_kuhn():
    path = os.path.join(os.path.dirname(__file__), "golden", "kuhn_value.txt")
    for line in open(path):
        if line.startswith("value_player1"):
            return float(line.split("=")[1])
    raise AssertionError("fixture missing")


@pytest.mark.parametrize("variant,bar", [("CFR", 1e-2), ("CFR_RMP", 6e-3), ("CFR_PLUS", 3e-4)])
def test_kuhn_average_converges_to_game_value(variant, bar):
    """Regret matching converges like 1/sqrt(T) (gap after 3000 iterations at
    most half of the gap after 100); CFR+ much faster on this game."""
    P = Problem(make_instance("kuhn"))
    tr = solve_cfr(P, variant, iters=3000, gap_every=100)
    assert tr.rows[-1]["gap"] < 0.5 * tr.rows[1]["gap"]
    assert tr.gap < bar
    assert abs(tr.value_p2 - (-_golden_kuhn())) <= tr.gap
    assert P.flow_residual(0, tr.x_avg) < 1e-12 and P.flow_residual(1, tr.y_avg) < 1e-12


@pytest.mark.parametrize("cfg,variant,T", [("micro", "CFR", 150), ("micro", "CFR_RMP", 150), ("c0", "CFR", 40),
                                           ("c0", "CFR_RMP", 40), ("lib_micro", "CFR", 60)])
def test_gap_equals_external_regret_and_obeys_the_decomposition(cfg, variant, T):
    P = Problem(make_instance(cfg, 0))
    C = Cfr(P, variant)
    xs, ys = [], []
    for _ in range(T):
        xs.append(C.cur[0].copy())
        ys.append(C.cur[1].copy())
        C.step()
    x_avg, y_avg = C.avg
    assert np.allclose(x_avg, sum(xs) / T, rtol=0, atol=1e-13)
    # external regrets from the definition: realised loss minus the best fixed response
    played = sum(float(np.sum(x * P.grad_x(y))) for x, y in zip(xs, ys))
    reg1 = played - T * P.br(0, P.grad_x(y_avg))
    reg2 = T * (-P.br(1, -P.grad_y(x_avg))) - played
    gap, _, _ = P.saddle_gap(x_avg, y_avg)
    assert gap == pytest.approx((reg1 + reg2) / T, rel=1e-9, abs=1e-12)
    # Zinkevich et al.: external regret <= sum over information sets of the
    # largest positive cumulative counterfactual regret
    for p, reg in ((0, reg1), (1, reg2)):
        bound = 0.0
        for node in P.tp[p].nodes:
            blk = C.R[p][node.first_seq:node.first_seq + node.n_act]
            bound += float(np.maximum(blk.max(axis=0), 0.0).sum())
        # (instantaneous regrets within 1e-12 of their terms count as ties)
        assert reg <= bound * (1 + 1e-9) + 1e-12, (p, reg, bound)


@pytest.mark.parametrize("variant", ["CFR", "CFR_RMP", "CFR_PLUS"])
def test_invariants(variant):
    P = Problem(make_instance("c0", 1))
    C = Cfr(P, variant)
    for _ in range(25):
        C.step()
        for p in (0, 1):
            t = P.tp[p]
            if variant != "CFR":
                assert np.all(C.R[p] >= 0.0)
            for node in t.nodes:
                q = C.qbar[p][node.first_seq:node.first_seq + node.n_act]
                assert np.all(q >= 0.0) and np.allclose(q.sum(axis=0), 1.0, atol=1e-14)
            assert P.flow_residual(p, C.cur[p]) < 1e-14 and P.flow_residual(p, C.avg[p]) < 1e-14
    assert C.products == 2 * 25
