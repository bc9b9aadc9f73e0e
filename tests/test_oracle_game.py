"""Pins for the oracle's game definition and payoff operator (CPU only).

* Kuhn poker's betting tree and payoffs, written out by hand.
* Tree sizes from an independent counting recursion over the betting rules.
* The payoff operator A y / A^T x against A written entry by entry
  (Section 2, Eq. 2) and against expected payoffs obtained by walking the game
  tree with behavioural strategies, deal by deal (no sequence form at all).
"""
import numpy as np
import pytest

from instances import make_instance
from oracle import Problem
from oracle.game import Game
from oracle.lp import explicit_A


def test_kuhn_tree_is_kuhn_poker():
    g = Game(make_instance("kuhn"))
    assert g.treeplex[0].seq_keys == ["k", "b1000", "k/b1000/f", "k/b1000/c"]
    assert g.treeplex[1].seq_keys == ["k/k", "k/b1000", "b1000/f", "b1000/c"]
    got = sorted((z.history, z.kind, z.u) for z in g.terminals)
    # ante 1 each; one bet of 1; player 2's chips (times the showdown sign)
    want = sorted([
        (("k", "k"), "show", 1.0),
        (("k", "b1000", "f"), "fold", 1.0),
        (("k", "b1000", "c"), "show", 2.0),
        (("b1000", "f"), "fold", -1.0),
        (("b1000", "c"), "show", 2.0),
    ])
    assert got == want
    # player 2's two information-set kinds are both roots of its treeplex
    assert [v.parent_seq for v in g.treeplex[1].nodes] == [-1, -1]
    assert [v.parent_seq for v in g.treeplex[0].nodes] == [-1, 0]


def _count(pot, stack, fracs, allin, R):
    """Counts nodes / sequences per player and fold / showdown leaves by a
    recursion over (contributions, player to act, raises so far)."""
    nodes = [0, 0]
    seqs = [0, 0]
    leaves = {"fold": 0, "show": 0}

    def rec(c, p, r):
        nodes[p] += 1
        o = 1 - p
        pot_now = pot + c[0] + c[1]
        if c[0] == c[1]:
            amts = {min(c[p] + f * pot_now, stack) for f in fracs}
            if allin:
                amts.add(stack)
            amts = sorted(a for a in amts if a > c[p])
            seqs[p] += 1 + len(amts)
            if p == 0:
                rec(c, 1, r)
            else:
                leaves["show"] += 1
            for a in amts:
                rec((a, c[1]) if p == 0 else (c[0], a), o, r)
        else:
            to_call = c[o] - c[p]
            leaves["fold"] += 1
            leaves["show"] += 1
            amts = []
            if r < R and c[o] < stack:
                s = {min(c[o] + f * (pot_now + to_call), stack) for f in fracs}
                if allin:
                    s.add(stack)
                amts = sorted(a for a in s if a > c[o])
            seqs[p] += 2 + len(amts)
            for a in amts:
                rec((a, c[1]) if p == 0 else (c[0], a), o, r + 1)

    rec((0.0, 0.0), 0, 0)
    return nodes, seqs, leaves


@pytest.mark.parametrize("cfg", ["kuhn", "c0", "c1", "c3"])
def test_tree_sizes_match_independent_count(cfg):
    inst = make_instance(cfg, 0)
    nodes, seqs, leaves = _count(inst.pot, inst.stack, inst.bet_fracs, inst.allin, inst.max_raises)
    got = Game(inst).counts()
    assert got["nodes"] == nodes
    assert got["seqs"] == seqs
    assert got["fold"] == leaves["fold"] and got["show"] == leaves["show"]


def _count_abstraction(pot, stack, ab, R):
    """The same counts under a situation-dependent abstraction: sizes by the
    acting player and the bets or raises so far (capped at 3), open folds (a
    fold before the opponent acted adds the opponent's one-action pass node)."""
    nodes = [0, 0]
    seqs = [0, 0]
    leaves = {"fold": 0, "show": 0}

    def rec(c, p, bets, opp_acted=True):
        nodes[p] += 1
        o = 1 - p
        pot_now = pot + c[0] + c[1]
        d = min(bets, 3)
        if c[0] == c[1]:
            amts = {min(c[p] + f * pot_now, stack) for f in ab.fracs[p][0]}
            if ab.allin[p][0]:
                amts.add(stack)
            amts = sorted(a for a in amts if a > c[p])
            folds = 1 if ab.open_fold[p] else 0
            leaves["fold"] += folds
            if folds and not opp_acted:
                nodes[o] += 1
                seqs[o] += 1
            seqs[p] += folds + 1 + len(amts)
            if p == 0:
                rec(c, 1, bets)
            else:
                leaves["show"] += 1
            for a in amts:
                rec((a, c[1]) if p == 0 else (c[0], a), o, bets + 1)
        else:
            to_call = c[o] - c[p]
            leaves["fold"] += 1
            leaves["show"] += 1
            amts = []
            if bets - 1 < R and c[o] < stack:
                s = {min(c[o] + f * (pot_now + to_call), stack) for f in ab.fracs[p][d]}
                if ab.allin[p][d]:
                    s.add(stack)
                amts = sorted(a for a in s if a > c[o])
            seqs[p] += 2 + len(amts)
            for a in amts:
                rec((a, c[1]) if p == 0 else (c[0], a), o, bets + 1)

    rec((0.0, 0.0), 0, 0, opp_acted=False)
    return nodes, seqs, leaves


@pytest.mark.parametrize("cfg", ["kuhn_open_fold", "lib_micro", "lib"])
def test_abstraction_tree_sizes_match_independent_count(cfg):
    inst = make_instance(cfg, 0)
    nodes, seqs, leaves = _count_abstraction(inst.pot, inst.stack, inst.abstraction, inst.max_raises)
    got = Game(inst).counts()
    assert got["nodes"] == nodes
    assert got["seqs"] == seqs
    assert got["fold"] == leaves["fold"] and got["show"] == leaves["show"]


def test_kuhn_with_open_folds_written_out():
    """Kuhn poker where a player not facing a bet may also fold: player 1 can
    fold first, player 2 can fold facing a check.  A fold costs the folder
    its ante (pot / 2 = 1) plus its river chips."""
    g = Game(make_instance("kuhn_open_fold"))
    assert g.treeplex[0].seq_keys == ["f", "k", "b1000", "k/b1000/f", "k/b1000/c"]
    # player 2 passes (its only action) after player 1 folds first
    assert g.treeplex[1].seq_keys == ["f/p", "k/f", "k/k", "k/b1000", "b1000/f", "b1000/c"]
    got = sorted((z.history, z.kind, z.u) for z in g.terminals)
    want = sorted([
        (("f", "p"), "fold", 1.0),
        (("k", "f"), "fold", -1.0),
        (("k", "k"), "show", 1.0),
        (("k", "b1000", "f"), "fold", 1.0),
        (("k", "b1000", "c"), "show", 2.0),
        (("b1000", "f"), "fold", -1.0),
        (("b1000", "c"), "show", 2.0),
    ])
    assert got == want


def test_libratus_abstraction_sizes_per_situation():
    """Section 7's river abstraction on a pot of 2100 with 18950 behind: the
    first player's opening sizes are 0.25x to 8x pot and all-in, after fold
    and check."""
    g = Game(make_instance("lib", 0))
    root = [v for v in g.treeplex[0].nodes if v.parent_seq < 0]
    assert len(root) == 1
    keys = g.treeplex[0].seq_keys[root[0].first_seq:root[0].first_seq + root[0].n_act]
    assert keys == ["f", "k", "b525000", "b1050000", "b2100000", "b4200000", "b8400000", "b16800000", "b18950000"]
    # the second player facing a check: fold, check, 0.5x, 0.75x, 1x pot, all-in
    v = next(v for v in g.treeplex[1].nodes if v.key == "k")
    keys = g.treeplex[1].seq_keys[v.first_seq:v.first_seq + v.n_act]
    assert keys == ["k/f", "k/k", "k/b1050000", "k/b1575000", "k/b2100000", "k/b18950000"]
    # facing the opening bet of 1x pot (2100 into 2100): fold, call, raise to
    # 2100 + f * (4200 + 2100) for f = 0.7, 1.1, all-in
    v = next(v for v in g.treeplex[1].nodes if v.key == "b2100000")
    keys = g.treeplex[1].seq_keys[v.first_seq:v.first_seq + v.n_act]
    assert keys == ["b2100000/f", "b2100000/c", "b2100000/b6510000", "b2100000/b9030000", "b2100000/b18950000"]
    assert g.counts()["seqs"] == [152, 153]


def test_tree_sizes_of_the_workloads():
    # sequences per hand per player at the benchmark shapes
    assert Game(make_instance("c0", 0)).counts()["seqs"] == [22, 22]
    assert Game(make_instance("c1", 0)).counts()["seqs"] == [223, 223]
    assert Game(make_instance("c3", 0)).counts()["seqs"] == [5938, 5938]


@pytest.mark.parametrize("cfg,seed", [("kuhn", 0), ("micro", 0), ("micro", 3), ("kuhn_open_fold", 0),
                                      ("lib_micro", 1)])
def test_operator_equals_entrywise_A(cfg, seed):
    P = Problem(make_instance(cfg, seed))
    A = explicit_A(P)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((P.n_seq[1], P.n))
    x = rng.standard_normal((P.n_seq[0], P.n))
    scale = np.abs(A).sum()
    assert np.abs(A @ y.ravel() - P.grad_x(y).ravel()).max() <= 1e-14 * scale
    assert np.abs(A.T @ x.ravel() - P.grad_y(x).ravel()).max() <= 1e-14 * scale
    # adjoint identity <x, A y> = <A^T x, y>
    assert abs(np.sum(x * P.grad_x(y)) - np.sum(P.grad_y(x) * y)) <= 1e-13 * scale


def _random_behaviour(P, p, rng):
    t = P.tp[p]
    return {v: rng.dirichlet(np.ones(node.n_act), size=P.n).T for v, node in enumerate(t.nodes)}


def _seqform(P, p, beh):
    t = P.tp[p]
    q = np.zeros((t.n_seq, P.n))
    for v in reversed(t.post_order):
        node = t.nodes[v]
        par = np.ones(P.n) if node.parent_seq < 0 else q[node.parent_seq]
        q[node.first_seq:node.first_seq + node.n_act] = par[None, :] * beh[v]
    return q


def _walk_value(P, beh):
    """E[u2] by playing out every deal on the public tree; payoffs read from
    the action tokens (check 'k', bet/raise 'b<millichips>' = new total
    contribution, call 'c', fold 'f')."""
    inst = P.inst
    g = P.game
    node_of = [{node.key: v for v, node in enumerate(t.nodes)} for t in P.tp]
    cards = [set(map(int, inst.hand_cards[h])) for h in range(P.n)]
    half = inst.pot / 2.0

    def rec(hist, p, c, reach, h1, h2):
        key = "/".join(hist)
        v = node_of[p][key]
        node = P.tp[p].nodes[v]
        prob = beh[p][v][:, h1 if p == 0 else h2]
        total = 0.0
        for a in range(node.n_act):
            tok = P.tp[p].seq_keys[node.first_seq + a].split("/")[-1]
            r = reach * prob[a]
            if tok == "f":
                total += r * ((half + c[0]) if p == 0 else -(half + c[1]))
            elif tok == "c" or (tok == "k" and p == 1):
                cc = c[1 - p] if tok == "c" else c[0]
                d = int(inst.strength[h2]) - int(inst.strength[h1])
                total += r * (half + cc) * np.sign(d)
            elif tok == "k":
                total += rec(hist + (tok,), 1, c, r, h1, h2)
            else:
                nc = list(c)
                nc[p] = int(tok[1:]) / 1000.0
                total += rec(hist + (tok,), 1 - p, tuple(nc), r, h1, h2)
        return total

    num = den = 0.0
    b1, b2 = inst.belief
    for h1 in range(P.n):
        for h2 in range(P.n):
            if cards[h1] & cards[h2]:
                continue
            w = b1[h1] * b2[h2]
            den += w
            num += w * rec((), 0, (0.0, 0.0), 1.0, h1, h2)
    del g
    return num / den


@pytest.mark.parametrize("cfg,seed", [("kuhn", 0), ("micro", 1), ("c0", 2), ("kuhn_open_fold", 0), ("lib_micro", 2)])
def test_operator_matches_game_walk(cfg, seed):
    P = Problem(make_instance(cfg, seed))
    rng = np.random.default_rng(10 + seed)
    beh = [_random_behaviour(P, 0, rng), _random_behaviour(P, 1, rng)]
    x, y = _seqform(P, 0, beh[0]), _seqform(P, 1, beh[1])
    want = _walk_value(P, beh)
    assert abs(P.value(x, y) - want) <= 1e-12 * max(1.0, inst_scale(P))
    assert abs(np.sum(P.grad_y(x) * y) - want) <= 1e-12 * max(1.0, inst_scale(P))


def inst_scale(P):
    return P.inst.pot + P.inst.stack


def test_kuhn_value_of_always_bet_vs_always_call():
    """Both players always bet / call: every deal goes to a 2-chip showdown and
    the expected payoff is zero by symmetry of uniform deals."""
    P = Problem(make_instance("kuhn"))
    x = np.zeros((4, 3))
    x[1] = 1.0  # bet
    y = np.zeros((4, 3))
    y[0] = 1.0  # check back after a check (never reached)
    y[3] = 1.0  # call a bet
    assert abs(P.value(x, y)) < 1e-15
    # always check, always check back: 1-chip showdowns, again zero in total
    x = np.zeros((4, 3))
    x[0] = 1.0
    x[3] = 1.0
    y = np.zeros((4, 3))
    y[0] = 1.0
    y[3] = 1.0
    assert abs(P.value(x, y)) < 1e-15
    # player 1 always bets, player 2 always folds: player 2 loses its ante
    x = np.zeros((4, 3))
    x[1] = 1.0
    y = np.zeros((4, 3))
    y[0] = 1.0
    y[2] = 1.0
    assert abs(P.value(x, y) - (-1.0)) < 1e-15
