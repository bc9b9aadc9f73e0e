"""The allocation-free saddle gap (egt_saddle_gap_noalloc) against the
allocating one (egt_saddle_gap), through the C ABI.

Both run the same kernels in the same order, so they must agree bit for bit.
Two calls in a row share the library's fixed scratch array: the first on the
1081-hand endgame, the second on a smaller one (105 hands), whose values must
not see anything the first call left behind.  A game whose scratch exceeds the
fixed array is refused before any device work."""
import numpy as np
import pytest

from instances import make_instance
from instances.endgames import Instance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def egt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_03063_amd import egt as mod

    return mod


def _point(egt, G, seed):
    """A seeded interior strategy pair: smoothed best responses to random
    gradients (every entry of both vectors is then strictly positive)."""
    rng = np.random.default_rng(seed)
    out = []
    for p in (0, 1):
        g = torch.from_numpy(rng.standard_normal((G.n_seq[p], G.ld))).to("cuda")
        q, _ = egt.smoothed_br(G, p, g, 0.3, want_value=False)
        out.append(q)
    return out


@pytest.mark.parametrize("order", [("c1", "c0")])
def test_noalloc_gap_equals_allocating_gap(egt, order):
    games = [egt.Game(make_instance(cfg, 0)) for cfg in order]
    out3 = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    for k, G in enumerate(games):
        print(f"[case] saddle_gap_noalloc call {k} on {order[k]} (n={G.n}, seqs={G.n_seq})", flush=True)
        x, y = _point(egt, G, 7 + k)
        want = egt.saddle_gap(G, x, y)
        got = egt.saddle_gap_noalloc(G, x, y, out3)
        torch.cuda.synchronize()
        got = tuple(float(v) for v in got.cpu())
        assert got == want, (order[k], got, want)
        assert want[0] >= -1e-12 * (abs(want[1]) + abs(want[2]))
    for G in games:
        G.close()


def test_noalloc_gap_refuses_a_game_beyond_its_scratch(egt):
    """2048 one-card hands with eight bet sizes and four raises need about
    260 MB of saddle-gap scratch, more than the fixed 160 MiB."""
    n = 2048
    base = make_instance("c3", 0)
    inst = Instance(name="big", n_cards=n, cards_per_hand=1, board=np.zeros(0, np.int32),
                    hand_cards=np.arange(n, dtype=np.int32).reshape(n, 1),
                    strength=np.arange(n, dtype=np.int32), belief=np.full((2, n), 1.0 / n),
                    pot=base.pot, stack=base.stack, bet_fracs=base.bet_fracs, allin=True,
                    max_raises=base.max_raises)
    print("[case] saddle_gap_noalloc refusal, 2048 hands", flush=True)
    G = egt.Game(inst)
    x, y = G.empty(0), G.empty(1)
    with pytest.raises(egt.EgtError) as e:
        egt.saddle_gap_noalloc(G, x, y)
    assert e.value.code == -1 and "scratch" in str(e.value)
    G.close()
