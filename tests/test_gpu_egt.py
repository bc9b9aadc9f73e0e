"""GPU parity of the EGT driver against the CPU FP64 oracle.

EGT iterations amplify rounding: the oracle disagrees with itself by 1e-13 at
t = 10 and by 1e-2 at t = 100 on Kuhn poker under EGT/as when only the
rounding of its prox changes (literal vs shift-free form; see
test_oracle_rounding_sensitivity).  So parity is checked where it is
meaningful:

* one step from the oracle's own iterate, at every (or every k-th) iterate of
  its trajectory: same side, same tau halvings, and
      max|x_gpu - x_oracle| <= 1e-10 max|x_oracle|  (same for y),
      |EGV_gpu - EGV_oracle|, |gap_gpu - gap_oracle| <= 1e-10 (|BR terms|)
  with the saddle gap of the new point measured independently by the oracle;
* whole-trajectory parity over prefixes shorter than the amplification, at
  1e-10 relative;
* full-length trajectories (2000 EGT iterations, 20 EGT/as iterations of the
  1081-hand endgame), where the bar is derived from the GPU's measured
  per-product error: the oracle re-run with product noise of that size shows
  how far such errors carry (test_full_trajectory_parity);
* complete solves: the GPU's reported final gap re-measured by the oracle at
  the GPU's final strategies, and the value within the two gaps of the
  oracle's own solve;
* bitwise repeatability and bitwise checkpoint / resume.
"""
import numpy as np
import pytest

from instances import make_instance
from oracle import EGT, Problem, iterate, solve
from tests.layout import Layout

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def egt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03063_amd import egt as mod

    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def scale_of(P, x, y):
    _, brmax, brmin = P.saddle_gap(x, y)
    return abs(brmax) + abs(brmin)


ONE_STEP = [
    ("kuhn", 0, "AS", 170, 1),
    ("kuhn", 0, "ALT", 300, 1),
    ("micro", 1, "AS", 400, 3),
    ("c0", 0, "AS", 476, 5),
    ("c0", 0, "ALT", 2000, 50),
    ("c0", 4, "BAL", 300, 10),
    ("c1", 0, "AS", 40, 13),
    ("kuhn_open_fold", 0, "AS", 150, 3),
    ("lib_micro", 0, "AS", 300, 5),
    ("lib", 0, "AS", 30, 10),
]


@pytest.mark.parametrize("cfg,seed,variant,iters,stride", ONE_STEP)
def test_one_step_parity(egt, cfg, seed, variant, iters, stride):
    inst = make_instance(cfg, seed)
    print(f"[case] one-step {cfg} seed={seed} {variant} iters={iters} stride={stride}", flush=True)
    P = Problem(inst)
    E = EGT(P)
    states = []

    def rec(t, x, y, mu_x, mu_y, tau):
        if t % stride == 0 and t < iters:
            states.append((t, x.copy(), y.copy(), mu_x, mu_y, tau))

    solve(P, variant, eps=0.0, max_iters=iters, on_iterate=rec)
    G = egt.Game(inst)
    L = Layout(G, P)
    st = egt.State(G, variant=variant, eps=0.0, max_iters=10**9)
    for t, x, y, mu_x, mu_y, tau in states:
        want = iterate(E, variant, t, x, y, mu_x, mu_y, tau)
        st.set(dev(L.to_lib(0, x)), dev(L.to_lib(1, y)), mu_x, mu_y, tau, t)
        egv, side = st.step(player=want["side"])
        got = st.get()
        gap, brmax, brmin = st.gap()
        gx, gy = L.from_lib(0, got["x"].cpu().numpy()), L.from_lib(1, got["y"].cpu().numpy())
        gap_o, brmax_o, brmin_o = P.saddle_gap(want["x"], want["y"])
        sc = abs(brmax_o) + abs(brmin_o)
        ctx = (cfg, variant, t)
        assert side == want["side"], ctx
        assert got["mu_x"] == pytest.approx(want["mu_x"], rel=1e-14), ctx
        assert got["mu_y"] == pytest.approx(want["mu_y"], rel=1e-14), ctx
        if variant == "AS":
            assert got["tau"] == want["tau"], ctx
        assert np.abs(gx - want["x"]).max() <= 1e-10 * np.abs(want["x"]).max(), ctx
        assert np.abs(gy - want["y"]).max() <= 1e-10 * np.abs(want["y"]).max(), ctx
        assert abs(egv - want["egv"]) <= 1e-10 * sc, (ctx, egv, want["egv"])
        assert abs(gap - gap_o) <= 1e-10 * sc, (ctx, gap, gap_o)
        assert abs(brmax - brmax_o) <= 1e-10 * sc and abs(brmin - brmin_o) <= 1e-10 * sc, ctx
    st.close()
    G.close()


def test_one_step_parity_large_tree(egt):
    """The 1081-hand tree with eight bet sizes and four raises: the first two
    iterations from the oracle's iterates."""
    inst = make_instance("c3", 0)
    print("[case] one-step c3 seed=0 AS", flush=True)
    P = Problem(inst)
    E = EGT(P)
    states = []
    solve(P, "AS", eps=0.0, max_iters=2,
          on_iterate=lambda t, x, y, mx, my, tau: states.append((t, x.copy(), y.copy(), mx, my, tau)))
    G = egt.Game(inst)
    L = Layout(G, P)
    st = egt.State(G, variant="AS", eps=0.0, max_iters=10**9)
    for t, x, y, mu_x, mu_y, tau in states[:2]:
        want = iterate(E, "AS", t, x, y, mu_x, mu_y, tau)
        st.set(dev(L.to_lib(0, x)), dev(L.to_lib(1, y)), mu_x, mu_y, tau, t)
        egv, side = st.step(player=want["side"])
        got = st.get()
        gx = L.from_lib(0, got["x"].cpu().numpy())
        sc = scale_of(P, want["x"], want["y"])
        assert side == want["side"] and got["tau"] == want["tau"]
        assert np.abs(gx - want["x"]).max() <= 1e-10 * np.abs(want["x"]).max()
        assert abs(egv - want["egv"]) <= 1e-10 * sc


def gpu_trajectory(egt, G, variant, eps, max_iters):
    st = egt.State(G, variant=variant, eps=eps, max_iters=max_iters)
    rows = []
    t = 0
    while True:
        gap, brmax, brmin = st.gap()
        row = dict(t=t, gap=gap)
        if gap <= eps or t >= max_iters:
            rows.append(row)
            break
        egv, side = st.step()
        row.update(side=side, egv=egv, tau=st.get()["tau"])
        rows.append(row)
        t += 1
    final = st.get()
    st.close()
    return rows, final


PREFIX = [
    ("kuhn", 0, "ALT", 1e-3, 5000),
    ("kuhn", 0, "AS", 0.0, 15),
    ("c0", 0, "AS", 0.0, 20),
    ("c0", 0, "ALT", 0.0, 500),
    ("c0", 4, "BAL", 0.0, 300),
    ("c1", 0, "AS", 0.0, 12),
    ("lib_micro", 0, "AS", 0.0, 20),
]


@pytest.mark.parametrize("cfg,seed,variant,eps,iters", PREFIX)
def test_trajectory_prefix_parity(egt, cfg, seed, variant, eps, iters):
    inst = make_instance(cfg, seed)
    print(f"[case] trajectory {cfg} seed={seed} {variant} iters<={iters}", flush=True)
    P = Problem(inst)
    tr = solve(P, variant, eps=eps, max_iters=iters)
    G = egt.Game(inst)
    L = Layout(G, P)
    rows, final = gpu_trajectory(egt, G, variant, eps, iters)
    assert len(rows) == len(tr.rows)
    for a, b in zip(rows, tr.rows):
        sc = abs(b["br_max_y"]) + abs(b["br_min_x"])
        assert abs(a["gap"] - b["gap"]) <= 1e-10 * sc, (a["t"], a["gap"], b["gap"])
        if "side" in b:
            assert a["side"] == b["side"] and abs(a["egv"] - b["egv"]) <= 1e-10 * sc, a["t"]
    assert final["mu_x"] == pytest.approx(tr.rows[-1]["mu_x"], rel=1e-12)
    x = L.from_lib(0, final["x"].cpu().numpy())
    y = L.from_lib(1, final["y"].cpu().numpy())
    assert np.abs(x - tr.x).max() <= 1e-10 * np.abs(tr.x).max()
    assert np.abs(y - tr.y).max() <= 1e-10 * np.abs(tr.y).max()


def abs_sum_bound(P, p, v_opp):
    """Per entry of p's gradient: (b_own(h)/Z) * sum over the terminals at the
    sequence of |u(z)| * sum_h' |b_opp(h') v_opp[sigma_opp(z), h']|, the sum of
    the absolute values of the terms the entry adds up."""
    o = 1 - p
    S = np.zeros(P.n_seq[p])
    for z in P.game.terminals:
        row = np.ones(P.n) if z.seq[o] < 0 else v_opp[z.seq[o]]
        S[z.seq[p]] += abs(z.u) * np.sum(np.abs(P.b[o] * row))
    return (P.b[p] / P.Z)[None, :] * S[:, None]


def oracle_trajectory(P, variant, iters, mu0=None, noise=0.0, seed=0):
    """The oracle's iterates (shift-free prox, the form the GPU computes)
    with, when noise > 0, every product entry moved by a seeded uniform draw
    of at most noise times its absolute-term sum: a model of another correct
    FP64 evaluation of A y whose per-entry error is `noise`."""
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        gx0, gy0 = P.grad_x, P.grad_y
        P.grad_x = lambda v: gx0(v) + rng.uniform(-1.0, 1.0, (P.n_seq[0], P.n)) * noise * abs_sum_bound(P, 0, v)
        P.grad_y = lambda v: gy0(v) + rng.uniform(-1.0, 1.0, (P.n_seq[1], P.n)) * noise * abs_sum_bound(P, 1, v)
    xs = []
    try:
        tr = solve(P, variant, eps=0.0, max_iters=iters, mu0=mu0, literal=False,
                   on_iterate=lambda t, x, y, *r: xs.append((x.copy(), y.copy())))
    finally:
        if noise > 0.0:
            P.grad_x, P.grad_y = gx0, gy0
    return tr, xs


def drift(a, b):
    return [max(np.abs(x0 - x1).max() / np.abs(x1).max(), np.abs(y0 - y1).max() / np.abs(y1).max())
            for (x0, y0), (x1, y1) in zip(a, b)]


FULL = [("c0", 0, "ALT", 2000), ("c1", 0, "AS", 20)]


@pytest.mark.parametrize("cfg,seed,variant,iters", FULL)
def test_full_trajectory_parity(egt, cfg, seed, variant, iters):
    """Whole trajectories: the 105-hand endgame's 2000 EGT iterations and the
    1081-hand endgame's first 20 EGT/as iterations, GPU against oracle at
    every iterate.

    EGT amplifies rounding along a trajectory roughly in proportion to the
    per-operation error (one unit in the last place of every product entry
    moves the 105-hand run by ~1e-10 of max |x| after 2000 iterations; see
    test_trajectory_sensitivity_to_product_rounding).  The GPU's smoothed best
    response follows the oracle's formulas operation by operation, but its
    O(n) products add their terms in another order than the dense
    definition.  So the test (1) measures the GPU's per-product error at
    iterates along the oracle's trajectory, (2) re-runs the oracle with
    product noise of that size, and (3) bounds the GPU's drift by
    max(1e-10, 3 x the drift that noise causes).  The GPU runs with fresh
    products at every iterate and the oracle's initial mu, like the oracle."""
    inst = make_instance(cfg, seed)
    print(f"[case] full trajectory {cfg} seed={seed} {variant} {iters}", flush=True)
    P = Problem(inst)
    tr, xs = oracle_trajectory(P, variant, iters)
    G = egt.Game(inst)
    L = Layout(G, P)
    # (1) per-product error at five iterates, relative to the absolute-term sums
    eps_prod = 0.0
    for t in np.linspace(0, iters, 5).astype(int):
        x, y = xs[t]
        ay = L.from_lib(0, egt.gradient(G, 0, dev(L.to_lib(1, y))).cpu().numpy())
        atx = L.from_lib(1, egt.gradient(G, 1, dev(L.to_lib(0, x))).cpu().numpy())
        eps_prod = max(eps_prod, (np.abs(ay - P.grad_x(y)) / np.maximum(abs_sum_bound(P, 0, y), 1e-300)).max(),
                       (np.abs(atx - P.grad_y(x)) / np.maximum(abs_sum_bound(P, 1, x), 1e-300)).max())
    # (2) the oracle's own drift under product noise of that size
    _, xn = oracle_trajectory(P, variant, iters, mu0=tr.mu0, noise=eps_prod, seed=seed + 1)
    d_noise = max(drift(xn, xs))
    # (3) the GPU trajectory
    st = egt.State(G, variant=variant, eps=0.0, max_iters=10**9, mu0=tr.mu0, fresh_products=True)
    gx = []
    for t in range(iters + 1):
        g = st.get()
        gx.append((L.from_lib(0, g["x"].cpu().numpy()), L.from_lib(1, g["y"].cpu().numpy())))
        if t < iters:
            st.step()
    st.close()
    d_gpu = drift(gx, xs)
    bar = max(1e-10, 3.0 * d_noise)
    print(f"  per-product error {eps_prod:.2e} of the absolute-term sums; oracle drift under that noise "
          f"{d_noise:.2e}; GPU drift {max(d_gpu):.2e} (t=100: {d_gpu[min(100, iters)]:.2e}); bar {bar:.2e}")
    assert eps_prod <= 1e-13
    assert d_gpu[min(10, iters)] <= 1e-12
    assert max(d_gpu) <= bar
    G.close()


@pytest.mark.parametrize("cfg,seed,with_oracle_solve", [("c0", 1, True), ("c0", 3, True), ("c1", 0, False),
                                                        ("c3", 0, False), ("lib_micro", 0, True),
                                                        ("lib", 0, False)])
def test_solve_verified_by_oracle(egt, cfg, seed, with_oracle_solve):
    inst = make_instance(cfg, seed)
    print(f"[case] egt_solve {cfg} seed={seed}", flush=True)
    P = Problem(inst)
    G = egt.Game(inst)
    L = Layout(G, P)
    r, st = egt.solve(G, keep_state=True)
    assert r["status"] == "EGT_OK" and r["converged"] == 1
    eps = 1e-3 * inst.pot
    f = st.get()
    x, y = L.from_lib(0, f["x"].cpu().numpy()), L.from_lib(1, f["y"].cpu().numpy())
    assert P.flow_residual(0, x) < 1e-12 and P.flow_residual(1, y) < 1e-12
    gap_o, brmax_o, brmin_o = P.saddle_gap(x, y)
    sc = abs(brmax_o) + abs(brmin_o)
    assert abs(r["gap"] - gap_o) <= 1e-10 * sc and gap_o <= eps * (1 + 1e-9)
    assert abs(r["br_max_y"] - brmax_o) <= 1e-10 * sc and abs(r["br_min_x"] - brmin_o) <= 1e-10 * sc
    assert r["value_p1"] == pytest.approx(-P.value(x, y), rel=1e-10, abs=1e-12)
    # the game value lies in [br_min_x, br_max_y] for every iterate
    assert brmin_o <= -r["value_p1"] + 1e-12 * sc <= brmax_o + 2e-12 * sc
    assert r["products"] == 3 * (r["iters"] + r["backtracks"])
    if with_oracle_solve:
        # the values of both solves lie within their gaps of the game value;
        # the number of EGT/as iterations to the target depends on rounding
        # (trajectories part after a few dozen iterations), so it is only
        # required to be of the same size as the oracle's
        tr = solve(P, "AS")
        assert abs(r["value_p1"] + tr.value_p2) <= r["gap"] + tr.gap
        assert 0.5 * tr.iters <= r["iters"] <= 2.0 * tr.iters, (r["iters"], tr.iters)
    st.close()


def test_repeatable_and_checkpoint_resume_bitwise(egt):
    inst = make_instance("c0", 2)
    print("[case] repeat / resume c0 seed=2", flush=True)
    G = egt.Game(inst)
    r1, s1 = egt.solve(G, keep_state=True)
    r2, s2 = egt.solve(G, keep_state=True)
    a, b = s1.get(), s2.get()
    assert torch.equal(a["x"], b["x"]) and torch.equal(a["y"], b["y"]) and r1["gap"] == r2["gap"]
    # stop after 57 iterations, export, resume in a fresh state
    st = egt.State(G, variant="AS")
    for _ in range(57):
        st.step()
    snap = st.get()
    ay, atx = st.products()
    st.close()
    st2 = egt.State(G, variant="AS")
    st2.set(snap["x"], snap["y"], snap["mu_x"], snap["mu_y"], snap["tau"], snap["iters"], ay, atx)
    while True:
        gap, _, _ = st2.gap()
        if gap <= 1e-3 * inst.pot:
            break
        st2.step()
    c = st2.get()
    assert c["iters"] == r1["iters"]
    assert torch.equal(c["x"], a["x"]) and torch.equal(c["y"], a["y"])


@pytest.mark.parametrize("cfg,variant,fresh,precision", [("c3", "AS", False, "fp64"), ("c3", "ALT", False, "fp64"),
                                                         ("c3", "AS", True, "fp64"), ("c3", "AS", False, "mixed"),
                                                         ("c1", "AS", False, "fp64"), ("c1", "ALT", False, "mixed")])
def test_kept_local_strategies_bitwise(egt, cfg, variant, fresh, precision):
    """The value launch keeps the local strategies of the next iteration's
    first smoothed best response (its EGV tree of that side is the same
    bottom-up pass, in FP64 and in the precision form), on the level path
    (c3) and on the single-launch path (c1).  Stepping with them kept, and solving
    with the pipelined loop, must give bit for bit what stepping with the full
    pass gives (a state_set before every step drops what is kept)."""
    inst = make_instance(cfg, 0)
    print(f"[case] kept q_bar {cfg} {variant} fresh={fresh} {precision}", flush=True)
    G = egt.Game(inst)
    n = 14
    # tau0 = 0.9: the first EGT/as attempts fail the excessive gap test, so
    # retries (which recompute x_bar) run between kept passes
    kw = dict(variant=variant, eps=1e-300, fresh_products=fresh, precision=precision, tau0=0.9)
    a = egt.State(G, max_iters=10**9, **kw)
    b = egt.State(G, max_iters=10**9, **kw)
    sides_a, sides_b = [], []
    for _ in range(n):
        sides_a.append(a.step()[1])
        f = b.get()
        ay, atx = b.products()
        b.set(f["x"], f["y"], f["mu_x"], f["mu_y"], f["tau"], f["iters"], ay, atx)
        sides_b.append(b.step()[1])
    r, c = egt.solve(G, keep_state=True, max_iters=n, **kw)
    assert r["status"] == "EGT_ENOTCONV" and r["iters"] == n
    assert variant != "AS" or r["backtracks"] >= 1, "EGT/as retried at least once"
    assert sides_a == sides_b and len(set(sides_a)) == 2, "both sides step, so both kinds of reuse run"
    fa, fb, fc = a.get(), b.get(), c.get()
    for f in (fb, fc):
        assert torch.equal(fa["x"], f["x"]) and torch.equal(fa["y"], f["y"])
        assert (fa["mu_x"], fa["mu_y"], fa["tau"]) == (f["mu_x"], f["mu_y"], f["tau"])
    for st in (a, b, c):
        st.close()
    G.close()


def test_iteration_cap_reports_not_converged(egt):
    inst = make_instance("c0", 0)
    G = egt.Game(inst)
    r, _ = egt.solve(G, max_iters=5)
    assert r["status"] == "EGT_ENOTCONV" and r["iters"] == 5 and r["converged"] == 0


def test_state_set_rejects_bad_scalars(egt):
    G = egt.Game(make_instance("kuhn"))
    st = egt.State(G)
    x, y = G.empty(0), G.empty(1)
    for bad in [dict(mu_x=0.0, mu_y=1.0, tau=0.5), dict(mu_x=1.0, mu_y=1.0, tau=1.0),
                dict(mu_x=1.0, mu_y=float("inf"), tau=0.5)]:
        with pytest.raises(egt.EgtError) as e:
            st.set(x, y, **bad)
        assert e.value.code == -1
