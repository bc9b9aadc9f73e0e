"""Pins for the oracle's dilated-entropy treeplex math (CPU only).

Section 4 and the appendix fix: the entropy DGF on a simplex, its dilation
with beta_j = 2 + sum_k 2 beta_k, the closed-form leaf solution
q_bar proportional to exp(-g / beta), the value identity, the DGF gradient
and the constant <grad d(q), q> - d(q) on the treeplex.  Each is checked
against something the oracle does not compute itself: scipy's softmax and
logsumexp, finite differences, brute force over pure strategies and random
feasible points.
"""
import itertools

import numpy as np
import pytest
from scipy.special import logsumexp, softmax

from instances import make_instance
from oracle import Problem
from oracle.lp import explicit_A


@pytest.fixture(scope="module")
def kuhn():
    return Problem(make_instance("kuhn"))


@pytest.fixture(scope="module")
def c0():
    return Problem(make_instance("c0", 1))


def _random_point(P, p, rng, alpha=1.0):
    t = P.tp[p]
    q = np.zeros((t.n_seq, P.n))
    for v in reversed(t.post_order):
        node = t.nodes[v]
        par = np.ones(P.n) if node.parent_seq < 0 else q[node.parent_seq]
        q[node.first_seq:node.first_seq + node.n_act] = par[None, :] * rng.dirichlet(
            alpha * np.ones(node.n_act), size=P.n).T
    return q


def _pure_points(P, p):
    """Every pure strategy (one action per decision node, the same for all
    hands), as sequence-form vectors."""
    t = P.tp[p]
    choices = [range(node.n_act) for node in t.nodes]
    for pick in itertools.product(*choices):
        q = np.zeros((t.n_seq, P.n))
        for v in reversed(t.post_order):
            node = t.nodes[v]
            par = np.ones(P.n) if node.parent_seq < 0 else q[node.parent_seq]
            q[node.first_seq + pick[v]] = par
        yield q


def test_sbr_on_lone_simplexes_is_softmax(kuhn):
    # player 2's treeplex in Kuhn is two root simplexes per hand, no nesting
    P = kuhn
    rng = np.random.default_rng(0)
    g = rng.standard_normal((4, 3))
    mu = 0.37
    q, val, _, _ = P.sbr(1, g, mu)
    want_val = 0.0
    for node in P.tp[1].nodes:
        sl = slice(node.first_seq, node.first_seq + node.n_act)
        tmp = mu * node.beta
        np.testing.assert_allclose(q[sl], softmax(-g[sl] / tmp, axis=0), rtol=1e-14, atol=1e-15)
        want_val += np.sum(-tmp * logsumexp(-g[sl] / tmp, axis=0) + tmp * np.log(node.n_act))
    assert abs(val - want_val) <= 1e-13 * (1 + abs(want_val))


@pytest.mark.parametrize("p", [0, 1])
def test_sbr_kkt_value_identity_and_optimality(c0, p):
    P = c0
    rng = np.random.default_rng(p)
    g = rng.standard_normal((P.n_seq[p], P.n)) * 3.0
    mu = 0.05
    q, val, lqb, V = P.sbr(p, g, mu)
    assert P.flow_residual(p, q) < 1e-14
    # KKT (Section 4): g~_i + mu beta_j log q_bar_i is the same for every i of a simplex
    t = P.tp[p]
    for node in t.nodes:
        gt = g[node.first_seq:node.first_seq + node.n_act].copy()
        for a, ch in enumerate(node.children):
            for k in ch:
                gt[a] += V[k]
        lam = gt + mu * node.beta * lqb[node.first_seq:node.first_seq + node.n_act]
        assert np.abs(lam - lam[0:1]).max() <= 1e-12 * (1 + np.abs(gt).max())
    # value identity: the propagated value equals the objective at the argmin
    obj = np.sum(g * q) + mu * P.dgf(p, q)
    assert abs(val - obj) <= 1e-12 * (1 + abs(obj))
    # optimality against random feasible points
    for _ in range(20):
        qq = _random_point(P, p, rng, alpha=0.3)
        assert val <= np.sum(g * qq) + mu * P.dgf(p, qq) + 1e-12


def test_sbr_limits(c0):
    P = c0
    rng = np.random.default_rng(5)
    g = rng.standard_normal((P.n_seq[0], P.n))
    # mu -> 0: value tends to the best-response value
    br = P.br(0, g)
    _, v_small, _, _ = P.sbr(0, g, 1e-9)
    assert abs(v_small - br) < 1e-5
    # mu -> infinity: the strategy tends to the uniform point
    q_big = P.sbr(0, g, 1e9)[0]
    assert np.abs(q_big - P.uniform(0)).max() < 1e-8


@pytest.mark.parametrize("p", [0, 1])
def test_best_response_is_min_over_pure_strategies(c0, p):
    P = c0
    rng = np.random.default_rng(7 + p)
    g = rng.standard_normal((P.n_seq[p], P.n))
    best = np.full(P.n, np.inf)
    for q in _pure_points(P, p):
        best = np.minimum(best, np.sum(g * q, axis=0))
    assert abs(P.br(p, g) - best.sum()) <= 1e-12 * (1 + np.abs(best).sum())
    q_br, v = P.br_strategy(p, g)
    assert abs(np.sum(g * q_br) - v) < 1e-12 * (1 + abs(v))


@pytest.mark.parametrize("p", [0, 1])
def test_dgf_basic_properties(c0, p):
    P = c0
    assert abs(P.dgf(p, P.uniform(p))) < 1e-12
    rng = np.random.default_rng(3)
    for _ in range(5):
        assert P.dgf(p, _random_point(P, p, rng)) >= -1e-12


@pytest.mark.parametrize("p", [0, 1])
def test_dgf_gradient_by_finite_differences(kuhn, c0, p):
    for P in (kuhn, c0):
        rng = np.random.default_rng(11)
        q = rng.uniform(0.2, 1.0, size=(P.n_seq[p], P.n))  # off the treeplex on purpose
        gr = P.dgf_grad_free(p, q)
        h = 1e-6
        for _ in range(25):
            s, j = rng.integers(P.n_seq[p]), rng.integers(P.n)
            e = np.zeros_like(q)
            e[s, j] = h
            fd = (P.dgf(p, q + e) - P.dgf(p, q - e)) / (2 * h)
            # dgf() treats a zero parent as a zero term; q here is strictly positive
            assert abs(fd - gr[s, j]) <= 1e-6 * (1 + abs(gr[s, j]))


@pytest.mark.parametrize("p", [0, 1])
def test_appendix_gradient_and_prox_shift_constant(c0, p):
    P = c0
    rng = np.random.default_rng(13)
    const = P.prox_shift_constant(p)
    for _ in range(5):
        g = rng.standard_normal((P.n_seq[p], P.n))
        q, _, lqb, _ = P.sbr(p, g, 0.3)  # an interior treeplex point with known log q_bar
        gr = P.dgf_grad(p, lqb)
        np.testing.assert_allclose(gr, P.dgf_grad_free(p, q), rtol=1e-10, atol=1e-10)
        lhs = np.sum(gr * q) - P.dgf(p, q)
        assert abs(lhs - const) <= 1e-11 * (1 + abs(const))


@pytest.mark.parametrize("p", [0, 1])
def test_diameter_and_l1_bound_by_brute_force(kuhn, c0, p):
    for P in (kuhn, c0):
        best_d = 0.0
        best_l1 = 0.0
        for q in _pure_points(P, p):
            best_d = max(best_d, P.dgf(p, q))
            best_l1 = max(best_l1, np.abs(q).sum())
        assert abs(P.omega(p) - best_d) <= 1e-10 * best_d
        assert P.max_l1(p) == pytest.approx(best_l1, rel=1e-14)


def test_beta_recursion_kuhn(kuhn):
    # player 1: the root simplex has one child simplex (after check, bet) of beta 2
    assert [v.beta for v in kuhn.tp[0].nodes] == [6.0, 2.0]
    assert [v.beta for v in kuhn.tp[1].nodes] == [2.0, 2.0]


def test_norm_A_is_largest_entry():
    P = Problem(make_instance("micro", 2))
    assert P.norm_A() == pytest.approx(np.abs(explicit_A(P)).max(), rel=1e-14)
