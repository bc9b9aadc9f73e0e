"""Mirror prox and Chambolle-Pock on the GPU (egt_fom_*) against the
oracle's restatement (oracle/fom.py), which takes each Bregman prox through
the appendix's grad d of the centre, while the library carries each centre's
gradient sum (the shift-free form): the two agree up to rounding.

* Iterate parity: averages and current strategies after every iteration,
  relative to max |x|, and the averages' saddle gap at checkpoints.
* Gradient accounting: 4 products per mirror-prox iteration, 2 per
  Chambolle-Pock iteration.
"""
import numpy as np
import pytest

from instances import make_instance
from oracle import ChambollePock, MirrorProx, Problem
from tests.layout import Layout

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def egt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03063_amd import egt as mod

    return mod


CASES = [("kuhn", "MP", 1.0, 200), ("kuhn", "CP", 1.0, 200), ("c0", "MP", 0.02, 60), ("c0", "CP", 0.02, 60),
         ("lib_micro", "MP", 0.5, 60), ("c1", "CP", 0.002, 8), ("c1", "MP", 0.002, 5)]


@pytest.mark.parametrize("cfg,method,step,T", CASES)
def test_fom_iterate_parity(egt, cfg, method, step, T):
    inst = make_instance(cfg, 0)
    print(f"[case] {method} parity {cfg} step={step} T={T}", flush=True)
    P = Problem(inst)
    O = MirrorProx(P, step) if method == "MP" else ChambollePock(P, step, step)
    G = egt.Game(inst)
    L = Layout(G, P)
    D = egt.Fom(G, method, step)
    worst = 0.0
    for t in range(1, T + 1):
        O.step()
        D.step(1)
        got = D.get()
        assert got["iters"] == t and got["products"] == O.products
        xa, ya = O.average()
        for p, key, avg in ((0, "x", xa), (1, "y", ya)):
            for mine, want in ((got[key], O.x if p == 0 else O.y), (got[key + "_avg"], avg)):
                err = np.abs(L.from_lib(p, mine.cpu().numpy()) - want).max() / np.abs(want).max()
                worst = max(worst, err)
                assert err <= 1e-10, (cfg, method, t, p, err)
        if t in (1, T):
            gap, brmax, brmin = D.gap()
            gap_o, brmax_o, brmin_o = P.saddle_gap(xa, ya)
            assert abs(gap - gap_o) <= 1e-10 * (abs(brmax_o) + abs(brmin_o)), (t, gap, gap_o)
    print(f"  worst relative strategy difference over {T} iterations: {worst:.2e}; gap {gap:.6g}")
    D.close()
    G.close()
