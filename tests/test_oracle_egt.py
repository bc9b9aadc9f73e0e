"""Pins for the oracle's EGT drivers (CPU only).

* Kuhn poker: the LP value and every EGT variant's limit equal the textbook
  game value (golden fixture).
* LP (Section 1's sequence-form LP) on tiny endgames: the best-response
  bounds of every iterate bracket the LP value; the final value is within the
  final gap of it.
* Section 2's invariants: eps_sad >= 0; the excessive gap condition implies
  eps_sad <= mu_x Omega_X + mu_y Omega_Y; EGT/as keeps EGV >= 0 at every
  accepted step; EGT started at the theory-safe mu keeps the condition and the
  O(1/T) bound.
* The literal prox of Algorithm 2 (through grad d of the appendix) equals the
  shift-free form.
* The sequence-form flow constraints hold for every iterate.
"""
import os

import numpy as np
import pytest

from instances import make_instance
from oracle import Problem, solve
from oracle.lp import lp_value


def _golden_kuhn():
    path = os.path.join(os.path.dirname(__file__), "golden", "kuhn_value.txt")
    for line in open(path):
        if line.startswith("value_player1"):
            return float(line.split("=")[1])
    raise AssertionError("fixture missing")


@pytest.fixture(scope="module")
def kuhn():
    return Problem(make_instance("kuhn"))


def test_kuhn_lp_value(kuhn):
    v, x = lp_value(kuhn)
    assert v == pytest.approx(-_golden_kuhn(), abs=1e-12)
    assert kuhn.flow_residual(0, x) < 1e-9


def test_kuhn_with_open_folds_keeps_the_value():
    """Folding when not facing a bet never beats checking, so adding those
    folds (the paper's abstraction allows them) leaves Kuhn's value."""
    P = Problem(make_instance("kuhn_open_fold"))
    v, _ = lp_value(P)
    assert v == pytest.approx(-_golden_kuhn(), abs=1e-12)
    tr = solve(P, "AS", eps=2e-4, max_iters=20000)
    assert tr.converged and abs(tr.value_p2 - (-_golden_kuhn())) <= tr.gap


@pytest.mark.parametrize("variant", ["AS", "BAL", "ALT"])
def test_kuhn_egt_converges_to_game_value(kuhn, variant):
    tr = solve(kuhn, variant, eps=2e-4, max_iters=20000)
    assert tr.converged
    assert abs(tr.value_p2 - (-_golden_kuhn())) <= tr.gap
    assert kuhn.flow_residual(0, tr.x) < 1e-13 and kuhn.flow_residual(1, tr.y) < 1e-13


@pytest.mark.parametrize("cfg,seed,eps", [("micro", 0, 1e-3), ("micro", 2, 1e-3), ("c0", 0, None),
                                          ("lib_micro", 0, 1e-3)])
def test_iterates_bracket_lp_value(cfg, seed, eps):
    """c0 is the 105-hand endgame (2310 sequences per player), solved to
    1e-3 pot; the micro endgames to 1e-3 chips."""
    P = Problem(make_instance(cfg, seed))
    v_star, _ = lp_value(P)
    tr = solve(P, "AS", eps=eps, max_iters=3000)
    for r in tr.rows:
        assert r["br_min_x"] <= v_star + 1e-10
        assert r["br_max_y"] >= v_star - 1e-10
        assert r["gap"] >= -1e-12
    assert abs(tr.value_p2 - v_star) <= tr.gap + 1e-12


@pytest.mark.parametrize("cfg,variant", [("c0", "AS"), ("micro", "AS"), ("c0", "BAL")])
def test_excessive_gap_invariants(cfg, variant):
    P = Problem(make_instance(cfg, 1))
    OX, OY = P.omega(0), P.omega(1)
    tr = solve(P, variant, max_iters=150)
    rows = tr.rows
    for prev, cur in zip(rows[:-1], rows[1:]):
        if variant == "AS":
            assert prev["egv"] >= 0.0
        if prev["egv"] >= 0.0:
            # EGV(x, y) > 0 implies eps_sad(x, y) <= mu_x Omega_X + mu_y Omega_Y
            assert cur["gap"] <= cur["mu_x"] * OX + cur["mu_y"] * OY + 1e-12
    assert tr.max_prox_diff < 1e-10
    assert P.flow_residual(0, tr.x) < 1e-12 and P.flow_residual(1, tr.y) < 1e-12


@pytest.mark.parametrize("cfg", ["kuhn", "micro"])
def test_theory_safe_start_keeps_condition_and_rate(cfg):
    """Algorithm 1 started at mu_x mu_y = ||A||^2 / (phi_X phi_Y), phi = 1/M
    (Section 4's strong-convexity modulus): EGV >= 0 at every step and
    eps_sad(x^T, y^T) <= 4 ||A|| / (T + 1) sqrt(Omega_X Omega_Y / (phi_X phi_Y))."""
    P = Problem(make_instance(cfg, 0))
    nA = P.norm_A()
    MX, MY = P.max_l1(0), P.max_l1(1)
    OX, OY = P.omega(0), P.omega(1)
    mu = nA * np.sqrt(MX * MY)
    tr = solve(P, "ALT", eps=0.0, max_iters=200, mu0=(mu, mu))
    for r in tr.rows[:-1]:
        assert r["egv"] >= 0.0
    for r in tr.rows[1:]:
        assert r["gap"] <= 4 * nA / (r["t"] + 1) * np.sqrt(OX * OY * MX * MY)


def test_gradient_accounting_counts_real_products():
    """Section 7 counts gradient computations: 3 per EGT step (A y for the
    anchor, A^T x_hat for the opponent's answer, A y_bar for the prox), 4 per
    EGT/as iteration (the excessive-gap test adds A^T x_+, while A y_+ follows
    from linearity) and 3 more per retry (the anchor's A y is kept).  The
    oracle's products are counted by wrapping grad_x / grad_y: a step makes
    exactly 3 calls; an EGT/as attempt makes 5, and the two the paper does not
    count are the reusable ones -- the gradient at y_+ equals the mixture of
    the gradients at y and y_bar, and a retry's A y equals the first
    attempt's."""
    from oracle import EGT, iterate

    P = Problem(make_instance("c0", 1))
    E = EGT(P)
    mu = E.auto_mu0()
    while True:
        x, y = E.init_point(mu, mu)
        if E.egv(x, y, mu, mu) >= 0.0:
            break
        mu *= 2.0
    log = []
    gx0, gy0 = P.grad_x, P.grad_y

    def gx(v):
        out = gx0(v)
        log.append(("x", v.copy(), out))
        return out

    def gy(v):
        out = gy0(v)
        log.append(("y", v.copy(), out))
        return out

    P.grad_x, P.grad_y = gx, gy
    try:
        E.step(0, mu, mu, x, y, 0.5)
        assert [k for k, _, _ in log] == ["x", "y", "x"]
        t, mx, my, tau = 0, mu, mu, 0.5
        seen_retry = False
        while t < 40 and not seen_retry:
            log.clear()
            r = iterate(E, "AS", t, x, y, mx, my, tau)
            attempts = 1 + r["backtracks"]
            assert len(log) == 5 * attempts
            # the last attempt: step products, then the EGV test's grad_x(y+), grad_y(x+)
            step = log[-5:-2]
            kinds = "xy"[r["side"]] + "yx"[r["side"]] + "xy"[r["side"]]
            assert "".join(k for k, _, _ in step) == kinds
            g_plus = log[-2] if log[-2][0] == "xy"[r["side"]] else log[-1]
            want = (1.0 - r["tau"]) * step[0][2] + r["tau"] * step[2][2]
            assert np.abs(g_plus[2] - want).max() <= 1e-12 * np.abs(want).max()
            if r["backtracks"]:
                seen_retry = True
                for a in range(1, attempts):
                    assert np.array_equal(log[5 * a][2], log[0][2])  # A y (or A^T x) kept across retries
            x, y, mx, my, tau = r["x"], r["y"], r["mu_x"], r["mu_y"], r["tau"]
            t += 1
        assert seen_retry
    finally:
        P.grad_x, P.grad_y = gx0, gy0


def test_oracle_rounding_sensitivity():
    """EGT/as amplifies rounding: the literal prox (through grad d) and the
    shift-free prox agree to rounding at every step, yet the trajectories part
    after a few dozen iterations.  This is why GPU parity is checked one step
    at a time from the oracle's own iterates."""
    P = Problem(make_instance("kuhn"))
    a = solve(P, "AS", eps=0.0, max_iters=100, literal=True)
    b = solve(P, "AS", eps=0.0, max_iters=100, literal=False)

    def d(t):
        return abs(a.rows[t]["gap"] - b.rows[t]["gap"])

    assert d(5) < 1e-13
    assert d(100) > 1e-6
    assert a.max_prox_diff < 1e-12 and b.max_prox_diff < 1e-12


def test_trajectory_sensitivity_to_product_rounding():
    """EGT (Algorithm 1) amplifies rounding in the products as mu shrinks:
    perturbing every product entry by at most one unit in the last place
    (relative 2.2e-16, a seeded draw) moves the 105-hand endgame's
    2000-iteration trajectory by about 1e-10 of max |x| by the end, although
    the two runs agree to 1e-15 for the first hundred iterations.  Any two
    correct FP64 evaluations of A y (e.g. the dense definition and the O(n)
    prefix-sum form) differ by at least this much per product, so whole
    2000-iteration trajectories can only be compared at a bar above it."""
    P = Problem(make_instance("c0", 0))
    Q = Problem(make_instance("c0", 0))
    rng = np.random.default_rng(1)
    gx0, gy0 = Q.grad_x, Q.grad_y
    Q.grad_x = lambda v: gx0(v) * (1.0 + rng.uniform(-1.0, 1.0, (Q.n_seq[0], Q.n)) * 2.2e-16)
    Q.grad_y = lambda v: gy0(v) * (1.0 + rng.uniform(-1.0, 1.0, (Q.n_seq[1], Q.n)) * 2.2e-16)
    xa, xb = [], []
    solve(P, "ALT", eps=0.0, max_iters=2000, on_iterate=lambda t, x, y, *r: xa.append((x.copy(), y.copy())))
    solve(Q, "ALT", eps=0.0, max_iters=2000, on_iterate=lambda t, x, y, *r: xb.append((x.copy(), y.copy())))

    def d(t):
        (x0, y0), (x1, y1) = xa[t], xb[t]
        return max(np.abs(x0 - x1).max() / np.abs(x0).max(), np.abs(y0 - y1).max() / np.abs(y0).max())

    worst = max(d(t) for t in range(len(xa)))
    print(f"  drift at t=100: {d(100):.2e}, t=2000: {d(2000):.2e}, worst {worst:.2e}")
    assert d(100) < 1e-13
    assert worst > 5e-11
