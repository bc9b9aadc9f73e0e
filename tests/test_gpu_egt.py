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
* whole-trajectory parity over prefixes shorter than the amplification;
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


@pytest.mark.parametrize("cfg,seed,with_oracle_solve", [("c0", 1, True), ("c0", 3, True), ("c1", 0, False)])
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
        tr = solve(P, "AS")
        assert abs(r["value_p1"] + tr.value_p2) <= r["gap"] + tr.gap
        assert 0.65 * tr.iters <= r["iters"] <= 1.35 * tr.iters, (r["iters"], tr.iters)
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
