"""CFR(RM), CFR(RM+) and CFR+ on the GPU (egt_cfr_*) against the oracle's
restatement of the same methods (oracle/cfr.py).

* Iterate parity: the current strategies and the averages after every
  iteration of a run from the same start, relative to max |x|, and the saddle
  gap of the averages against the oracle's at checkpoints.
* A complete CFR+ solve to 1e-3 pot whose final averages the oracle
  re-measures; two products per iteration.
"""
import numpy as np
import pytest

from instances import make_instance
from oracle import Cfr as OracleCfr
from oracle import Problem
from tests.layout import Layout

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def egt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03063_amd import egt as mod

    return mod


CASES = [("kuhn", 0, "CFR", 300), ("kuhn", 0, "CFR_PLUS", 300), ("c0", 0, "CFR", 100), ("c0", 0, "CFR_RMP", 100),
         ("c0", 0, "CFR_PLUS", 100), ("c1", 0, "CFR_PLUS", 12), ("lib_micro", 0, "CFR_PLUS", 100),
         ("c3", 0, "CFR_PLUS", 3)]


@pytest.mark.parametrize("cfg,seed,variant,T", CASES)
def test_cfr_iterate_parity(egt, cfg, seed, variant, T):
    inst = make_instance(cfg, seed)
    print(f"[case] CFR parity {cfg} seed={seed} {variant} T={T}", flush=True)
    P = Problem(inst)
    C = OracleCfr(P, variant)
    G = egt.Game(inst)
    L = Layout(G, P)
    D = egt.Cfr(G, variant)
    worst = 0.0
    for t in range(T + 1):
        if t > 0:
            C.step()
            D.step(1)
        got = D.get()
        assert got["iters"] == t
        for p, key in ((0, "x"), (1, "y")):
            for mine, want in ((got[key], C.cur[p]), (got[key + "_avg"], C.avg[p])):
                err = np.abs(L.from_lib(p, mine.cpu().numpy()) - want).max() / np.abs(want).max()
                worst = max(worst, err)
                assert err <= 1e-10, (cfg, variant, t, p, err)
        if t in (0, T // 2, T):
            gap, brmax, brmin = D.gap()
            gap_o, brmax_o, brmin_o = P.saddle_gap(C.avg[0], C.avg[1])
            assert abs(gap - gap_o) <= 1e-10 * (abs(brmax_o) + abs(brmin_o)), (t, gap, gap_o)
    print(f"  worst relative strategy difference over {T} iterations: {worst:.2e}")
    D.close()
    G.close()


@pytest.mark.parametrize("cfg,seed", [("c0", 2), ("lib_micro", 1)])
def test_cfr_plus_solve_verified_by_oracle(egt, cfg, seed):
    inst = make_instance(cfg, seed)
    print(f"[case] CFR+ solve {cfg} seed={seed}", flush=True)
    G = egt.Game(inst)
    eps = 1e-3 * inst.pot
    r = egt.cfr_solve(G, "CFR_PLUS", eps=eps, max_iters=20000, gap_every=10)
    assert r["status"] == "EGT_OK" and r["converged"] == 1 and r["gap"] <= eps
    assert r["products"] == 2 * r["iters"]
    # the same run stepped by hand; the oracle re-measures its averages
    D = egt.Cfr(G, "CFR_PLUS")
    D.step(r["iters"])
    got = D.get()
    P = Problem(inst)
    L = Layout(G, P)
    x, y = L.from_lib(0, got["x_avg"].cpu().numpy()), L.from_lib(1, got["y_avg"].cpu().numpy())
    gap_o, brmax, brmin = P.saddle_gap(x, y)
    print(f"  {r['iters']} iterations, gap {r['gap']:.6g}, oracle {gap_o:.6g}")
    assert abs(r["gap"] - gap_o) <= 1e-10 * (abs(brmax) + abs(brmin)) and gap_o <= eps * (1 + 1e-9)
    assert abs(-r["value_p1"] - P.value(x, y)) <= 1e-9 * (abs(brmax) + abs(brmin))
    D.close()
    G.close()
