"""General extensive-form games on the GPU (egt_build_general_game): the CSR
SpMV products, the smoothed best response on general treeplexes, EGT steps
and complete solves, CFR+ and mirror prox, all against the general oracle
(oracle/general.py, a dense A and the river oracle's treeplex routines).

Games: Kuhn poker written as a general game, Leduc hold'em, seeded random
game trees and Section 3's nine-simplex treeplex (Fig. 1, partly a reading)
against one two-action simplex.
"""
import numpy as np
import pytest

from instances.efg import fig1_game, kuhn_efg, leduc, random_efg
from oracle import EGT, Cfr, GeneralProblem, MirrorProx, iterate, solve
from oracle.lp import lp_value
from tests.layout import Layout

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GAMES = {
    "kuhn_efg": kuhn_efg,
    "leduc": leduc,
    "random1": lambda: random_efg(1),
    "random4": lambda: random_efg(4, depth=7, max_actions=4, n_types=5),
    "fig1": lambda: fig1_game(0),
}


@pytest.fixture(scope="module")
def egt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03063_amd import egt as mod

    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _setup(egt, name):
    inst = GAMES[name]()
    P = GeneralProblem(inst)
    G = egt.GeneralGame(inst)
    return inst, P, G, Layout(G, P)


@pytest.mark.parametrize("name", list(GAMES))
def test_spmv_and_sbr_parity(egt, name):
    print(f"[case] general products and SBR {name}", flush=True)
    inst, P, G, L = _setup(egt, name)
    assert G.n == 1 and G.n_seq == P.n_seq
    rng = np.random.default_rng(11)
    for p in (0, 1):
        other = rng.random((P.n_seq[1 - p], 1))
        want = P.grad_x(other) if p == 0 else P.grad_y(other)
        got = egt.gradient(G, p, dev(L.to_lib(1 - p, other))).cpu().numpy()
        assert np.all(got[:, 1:] == 0.0), "padding slots are written 0"
        bound = (np.abs(P.A) @ np.abs(other)) if p == 0 else (np.abs(P.A).T @ np.abs(other))
        err = np.abs(L.from_lib(p, got) - want)
        assert (err <= 1e-14 * np.maximum(bound, 1e-300) + 1e-300).all(), (name, p, err.max())
        g = rng.standard_normal((P.n_seq[p], 1))
        for mu in (1e-3, 0.3, 50.0):
            q_o, v_o, _, _ = P.sbr(p, g, mu)
            q, v = egt.smoothed_br(G, p, dev(L.to_lib(p, g)), mu)
            assert np.abs(L.from_lib(p, q.cpu().numpy()) - q_o).max() <= 1e-12, (name, p, mu)
            # the value adds terms of size mu beta log n (beta grows with the
            # treeplex below a simplex) that cancel: bound relative to them
            sc = abs(v_o) + mu * max(n.beta for n in P.tp[p].nodes) * np.log(16.0) + np.abs(g).sum()
            assert abs(float(v.item()) - v_o) <= 1e-13 * sc, (name, p, mu, float(v.item()), v_o)
        b = egt.best_response(G, p, dev(L.to_lib(p, g)))
        assert abs(float(b.item()) - P.br(p, g)) <= 1e-12 * max(1.0, abs(P.br(p, g)))
    G.close()


@pytest.mark.parametrize("name,variant,iters,stride", [("kuhn_efg", "AS", 150, 1), ("leduc", "AS", 300, 7),
                                                       ("random1", "ALT", 200, 5), ("random4", "AS", 200, 10)])
def test_one_step_parity(egt, name, variant, iters, stride):
    print(f"[case] general one-step {name} {variant} iters={iters}", flush=True)
    inst, P, G, L = _setup(egt, name)
    E = EGT(P)
    states = []

    def rec(t, x, y, mu_x, mu_y, tau):
        if t % stride == 0 and t < iters:
            states.append((t, x.copy(), y.copy(), mu_x, mu_y, tau))

    solve(P, variant, eps=0.0, max_iters=iters, on_iterate=rec)
    st = egt.State(G, variant=variant, eps=0.0, max_iters=10**9)
    for t, x, y, mu_x, mu_y, tau in states:
        want = iterate(E, variant, t, x, y, mu_x, mu_y, tau)
        st.set(dev(L.to_lib(0, x)), dev(L.to_lib(1, y)), mu_x, mu_y, tau, t)
        egv, side = st.step(player=want["side"])
        got = st.get()
        gx, gy = L.from_lib(0, got["x"].cpu().numpy()), L.from_lib(1, got["y"].cpu().numpy())
        _, brmax_o, brmin_o = P.saddle_gap(want["x"], want["y"])
        sc = abs(brmax_o) + abs(brmin_o)
        ctx = (name, variant, t)
        assert side == want["side"], ctx
        assert got["mu_x"] == pytest.approx(want["mu_x"], rel=1e-14), ctx
        assert np.abs(gx - want["x"]).max() <= 1e-10 * np.abs(want["x"]).max(), ctx
        assert np.abs(gy - want["y"]).max() <= 1e-10 * np.abs(want["y"]).max(), ctx
        assert abs(egv - want["egv"]) <= 1e-10 * sc, (ctx, egv, want["egv"])
    st.close()
    G.close()


@pytest.mark.parametrize("name,with_oracle_solve", [("kuhn_efg", True), ("leduc", False), ("random1", True),
                                                     ("random4", False)])
def test_solve_verified_by_oracle(egt, name, with_oracle_solve):
    print(f"[case] general egt_solve {name}", flush=True)
    inst, P, G, L = _setup(egt, name)
    r, st = egt.solve(G, keep_state=True)
    assert r["status"] == "EGT_OK" and r["converged"] == 1
    eps = 1e-3 * inst.pot
    f = st.get()
    x, y = L.from_lib(0, f["x"].cpu().numpy()), L.from_lib(1, f["y"].cpu().numpy())
    assert P.flow_residual(0, x) < 1e-12 and P.flow_residual(1, y) < 1e-12
    gap_o, brmax_o, brmin_o = P.saddle_gap(x, y)
    sc = abs(brmax_o) + abs(brmin_o)
    assert abs(r["gap"] - gap_o) <= 1e-10 * sc and gap_o <= eps * (1 + 1e-9)
    assert r["value_p1"] == pytest.approx(-P.value(x, y), rel=1e-10, abs=1e-12)
    # the game value (LP) lies in the GPU iterate's bracket
    v_lp, _ = lp_value(P, P.A)
    assert brmin_o - 1e-12 * sc <= v_lp <= brmax_o + 1e-12 * sc
    if with_oracle_solve:
        tr = solve(P, "AS", eps=eps, max_iters=50000, record_egv=False)
        assert 0.5 * tr.iters <= r["iters"] <= 2.0 * tr.iters + 10, (r["iters"], tr.iters)
    st.close()
    G.close()


def test_cfr_plus_and_mirror_prox_parity(egt):
    print("[case] general CFR+ and mirror prox on Leduc / Kuhn", flush=True)
    inst, P, G, L = _setup(egt, "leduc")
    C = Cfr(P, "CFR_PLUS")
    D = egt.Cfr(G, "CFR_PLUS")
    for t in range(1, 31):
        C.step()
        D.step(1)
        got = D.get()
        for p, key in ((0, "x"), (1, "y")):
            for mine, want in ((got[key], C.cur[p]), (got[key + "_avg"], C.avg[p])):
                err = np.abs(L.from_lib(p, mine.cpu().numpy()) - want).max() / np.abs(want).max()
                assert err <= 1e-10, ("CFR+", t, p, err)
    D.close()
    G.close()
    inst, P, G, L = _setup(egt, "kuhn_efg")
    O = MirrorProx(P, 1.0)
    F = egt.Fom(G, "MP", 1.0)
    for t in range(1, 101):
        O.step()
        F.step(1)
    got = F.get()
    xa, ya = O.average()
    for p, key, want in ((0, "x_avg", xa), (1, "y_avg", ya)):
        err = np.abs(L.from_lib(p, got[key].cpu().numpy()) - want).max() / np.abs(want).max()
        assert err <= 1e-10, ("MP", p, err)
    F.close()
    G.close()


def test_precision_form_is_refused(egt):
    inst, P, G, L = _setup(egt, "kuhn_efg")
    with pytest.raises(egt.EgtError):
        egt.solve(G, precision="mixed")
    G.close()
