"""Pins for the general-game oracle (CPU only).

* Kuhn poker written as a general game: its LP value is the textbook 1/18 to
  player 2 (golden fixture), the same as the river construction's, and the
  uniform profile is worth the same in both constructions.
* Leduc hold'em: the sequence-form value of random behavioural profiles
  equals their expected payoff computed by a separate recursive walk of the
  game's rules over histories (no sequences involved); EGT reaches its gap
  target with the LP value inside its bracket.
* Random games: the LP value lies in the EGT bracket; CFR+ converges.
* Section 3's nine-simplex treeplex: the smoothed best response attains the
  smallest objective <g, q> + mu d(q) against random feasible points and its
  value is that objective; the simplex counts and depths the text states hold.
"""
import os

import numpy as np
import pytest

from instances import make_instance
from instances.efg import fig1_game, kuhn_efg, leduc, random_efg
from oracle import GeneralProblem, Problem, solve, solve_cfr
from oracle.lp import lp_value


def _golden_kuhn():
    path = os.path.join(os.path.dirname(__file__), "golden", "kuhn_value.txt")
    for line in open(path):
        if line.startswith("value_player1"):
            return float(line.split("=")[1])
    raise AssertionError("fixture missing")


def _behavioural(P, p, rng):
    """Random local strategies and their sequence form."""
    t = P.tp[p]
    qb = np.zeros((t.n_seq, 1))
    for node in t.nodes:
        qb[node.first_seq:node.first_seq + node.n_act, 0] = rng.dirichlet(np.ones(node.n_act))
    q = np.zeros_like(qb)
    for v in reversed(t.post_order):
        node = t.nodes[v]
        par = 1.0 if node.parent_seq < 0 else q[node.parent_seq, 0]
        q[node.first_seq:node.first_seq + node.n_act, 0] = par * qb[node.first_seq:node.first_seq + node.n_act, 0]
    return qb, q


def test_kuhn_general_matches_textbook_and_river():
    G = GeneralProblem(kuhn_efg())
    v, _ = lp_value(G, G.A)
    assert abs(v - (-_golden_kuhn())) < 1e-9
    R = Problem(make_instance("kuhn"))
    vr, _ = lp_value(R)
    assert abs(v - vr) < 1e-9
    assert abs(G.value(G.uniform(0), G.uniform(1)) - R.value(R.uniform(0), R.uniform(1))) < 1e-12


def _leduc_walk(local1, local2, key_of, raises=(2.0, 4.0), max_bets=2):
    """Expected chips of player 2 in Leduc under behavioural strategies given
    as local[infoset key][action index], by recursion over histories."""
    deals = [(a, b, c) for a in range(6) for b in range(6) for c in range(6) if len({a, b, c}) == 3]
    total = 0.0

    def rank(c):
        return c // 2

    def showdown(c1, c2, pub, pot1, pot2):
        s1 = (1, rank(c1)) if rank(c1) == rank(pub) else (0, rank(c1))
        s2 = (1, rank(c2)) if rank(c2) == rank(pub) else (0, rank(c2))
        return pot1 if s2 > s1 else (-pot2 if s1 > s2 else 0.0)

    def node(deal, rnd, hist, bets, pots, player):
        c1, c2, pub = deal
        key = key_of(player, rank(deal[player]), rank(pub) if rnd == 1 else None, hist)
        probs = (local1 if player == 0 else local2)[key]
        facing = pots[1 - player] > pots[player]
        options = (["f", "c"] + (["r"] if bets < max_bets else [])) if facing else (["k"] + (["b"] if bets < max_bets else []))
        ev = 0.0
        for i, a in enumerate(options):
            pr = probs[i]
            if pr == 0.0:
                continue
            pts = list(pots)
            if a == "f":
                val = pts[0] if player == 0 else -pts[1]
            else:
                if a == "c":
                    pts[player] = pts[1 - player]
                elif a in ("b", "r"):
                    pts[player] = pts[1 - player] + raises[rnd]
                ends_round = a == "c" or (a == "k" and player == 1)
                if not ends_round:
                    val = node(deal, rnd, hist + a, bets + (a in ("b", "r")), tuple(pts), 1 - player)
                elif rnd == 0:
                    val = node(deal, 1, hist + a + "|", 0, tuple(pts), 0)
                else:
                    val = showdown(c1, c2, pub, pts[0], pts[1])
            ev += pr * val
        return ev

    for d in deals:
        total += node(d, 0, "", 0, (1.0, 1.0), 0) / len(deals)
    return total


def test_leduc_sequence_form_equals_history_walk():
    inst = leduc()
    P = GeneralProblem(inst)
    rng = np.random.default_rng(7)
    for _ in range(3):
        qb1, x = _behavioural(P, 0, rng)
        qb2, y = _behavioural(P, 1, rng)
        local = []
        for p, qb in ((0, qb1), (1, qb2)):
            d = {}
            for node, (_, n_act, key) in zip(P.tp[p].nodes, inst.infosets[p]):
                d[key] = qb[node.first_seq:node.first_seq + n_act, 0]
            local.append(d)

        def key_of(player, own, pub, hist):
            return (own,) + ((pub,) if pub is not None else ()) + (hist,)

        walk = _leduc_walk(local[0], local[1], key_of)
        assert abs(P.value(x, y) - walk) < 1e-12


@pytest.mark.parametrize("make", [leduc, lambda: random_efg(1), lambda: random_efg(2, depth=6)])
def test_egt_bracket_contains_lp_value(make):
    inst = make()
    P = GeneralProblem(inst)
    v, _ = lp_value(P, P.A)
    tr = solve(P, "AS", eps=1e-3 * inst.pot, max_iters=20000, record_egv=False)
    assert tr.converged and tr.gap <= 1e-3 * inst.pot
    last = tr.rows[-1]
    assert last["br_min_x"] - 1e-9 <= v <= last["br_max_y"] + 1e-9
    assert P.flow_residual(0, tr.x) < 1e-12 and P.flow_residual(1, tr.y) < 1e-12


def test_cfr_plus_on_random_game():
    inst = random_efg(3)
    P = GeneralProblem(inst)
    v, _ = lp_value(P, P.A)
    tr = solve_cfr(P, "CFR_PLUS", iters=3000, gap_every=100)
    assert tr.rows[-1]["gap"] < 0.05 * tr.rows[0]["gap"]
    assert tr.rows[-1]["br_min_x"] - 1e-9 <= v <= tr.rows[-1]["br_max_y"] + 1e-9


def test_fig1_treeplex_shape_and_sbr_optimality():
    inst = fig1_game(0)
    P = GeneralProblem(inst)
    t = P.tp[0]
    assert len(t.nodes) == 9 and [n.n_act for n in t.nodes[:2]] == [2, 3]
    assert sorted(i for i, n in enumerate(t.nodes) if n.parent_seq < 0) == [0, 1]
    depth = {}
    for i, n in enumerate(t.nodes):  # branchings before each simplex (b_Q^j)
        depth[i] = 0 if n.parent_seq < 0 else 1 + depth[next(j for j, m in enumerate(t.nodes)
                                                            if m.first_seq <= n.parent_seq < m.first_seq + m.n_act)]
    assert depth[0] == 0 and depth[2] == 1 and depth[7] == 2
    assert sorted(depth.values()) == [0, 0, 1, 1, 1, 1, 1, 2, 2]
    rng = np.random.default_rng(3)
    g = rng.standard_normal((t.n_seq, 1))
    for mu in (0.05, 1.0, 20.0):
        q, val, _, _ = P.sbr(0, g, mu)
        obj = float(np.sum(g * q)) + mu * P.dgf(0, q)
        assert abs(obj - val) < 1e-10 * max(1.0, abs(val))
        for _ in range(40):
            _, r = _behavioural(P, 0, rng)
            assert float(np.sum(g * r)) + mu * P.dgf(0, r) >= obj - 1e-10
