"""Precision form against the CPU FP64 oracle, with the error of each result
stated and bounded.

* product (BF16 hi+lo showdown GEMM with FP32 accumulation, fold terminals
  in FP32 arithmetic): on FP32 inputs, compared with the oracle applied to the
  same FP32-rounded inputs.  Bound per entry:
      |err| <= 2e-4 * (b_own(h)/Z) * sum_z |u(z)| * sum_h' |r_z(h')|
  (Y in hi+lo BF16 keeps 2^-16 of each entry; FP32 accumulation over
  2 x n_pad <= 2176 terms adds at most 2176 x 2^-24 = 1.3e-4 of the absolute
  sum, and a fold terminal's FP32 sums over at most 2048 hands at most
  2048 x 2^-24 = 1.2e-4; the observed errors are printed and are far smaller);
* smoothed best response (FP32 exponentials and strategy, FP64 normalisers
  and values): |q_err| <= 1e-5, |value_err| <= 1e-6 (|value| + sum |V|);
* one step from the oracle's iterate: strategies within 2e-3 of the oracle's
  (relative to max |x|; smoothing divides gradient errors by mu beta);
* complete solves: the FP64 saddle gap of the final strategies, re-measured by
  the oracle, reaches 1e-3 pot, and the value agrees with the FP64 path's
  within the two gaps.
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


def f32_round(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def random_point(P, p, rng, alpha=0.5):
    t = P.tp[p]
    q = np.zeros((t.n_seq, P.n))
    for v in reversed(t.post_order):
        node = t.nodes[v]
        par = np.ones(P.n) if node.parent_seq < 0 else q[node.parent_seq]
        q[node.first_seq:node.first_seq + node.n_act] = par[None, :] * rng.dirichlet(
            alpha * np.ones(node.n_act), size=P.n).T
    return q


def grad_bound(P, p, v_opp):
    o = 1 - p
    S = np.zeros(P.n_seq[p])
    for z in P.game.terminals:
        s_own, s_opp = z.seq[p], z.seq[o]
        if s_own < 0:
            continue
        row = np.ones(P.n) if s_opp < 0 else v_opp[s_opp]
        S[s_own] += abs(z.u) * np.sum(np.abs(P.b[o] * row))
    return (P.b[p] / P.Z)[None, :] * S[:, None]


@pytest.mark.parametrize("cfg,seed", [("kuhn", 0), ("c0", 0), ("c1", 0), ("c3", 0)])
def test_mixed_product_error(egt, cfg, seed):
    inst = make_instance(cfg, seed)
    print(f"[case] mixed product {cfg} seed={seed}", flush=True)
    _check_mixed_product(egt, inst, seed)


def test_mixed_product_error_ragged_k(egt):
    """The c3 betting tree (thousands of showdown columns, so the tiled GEMM)
    on a 32-card deck: 351 hands, rows padded to 352, so the last 128-row
    tile is partly outside the rows and K takes an odd number (11) of steps
    of 32."""
    from instances.endgames import CONFIGS, river
    kw = dict(CONFIGS["c3"], n_ranks=8)
    inst = river("c3_32cards", 0, **kw)
    print("[case] mixed product c3 betting, 32-card deck", flush=True)
    _check_mixed_product(egt, inst, 0)


@pytest.mark.parametrize("name", ["max-hands", "two-hands"])
def test_mixed_product_error_hand_counts(egt, name):
    """The largest hand count the library takes (2048 hands: eight per thread
    in the fold kernel, sixteen 128-row tiles of the GEMM) and two one-card
    hands (rows mostly padding)."""
    from tests.test_gpu_ops import _edge_instances
    inst = dict(_edge_instances())[name]
    print(f"[case] mixed product {name}", flush=True)
    _check_mixed_product(egt, inst, 0)


def _check_mixed_product(egt, inst, seed):
    P = Problem(inst)
    G = egt.Game(inst)
    L = Layout(G, P)
    rng = np.random.default_rng(seed + 40)
    x, y = f32_round(random_point(P, 0, rng)), f32_round(random_point(P, 1, rng))
    gx = egt.gradient_mixed(G, 0, dev32(L.to_lib(1, y)))
    gy = egt.gradient_mixed(G, 1, dev32(L.to_lib(0, x)))
    torch.cuda.synchronize()
    gx, gy = gx.double().cpu().numpy(), gy.double().cpu().numpy()
    assert np.all(gx[:, P.n:] == 0) and np.all(gy[:, P.n:] == 0)
    for p, got, want, bound in ((0, gx, P.grad_x(y), grad_bound(P, 0, y)),
                                (1, gy, P.grad_y(x), grad_bound(P, 1, x))):
        err = np.abs(L.from_lib(p, got) - want)
        rel = (err / np.maximum(bound, 1e-300)).max()
        print(f"  player {p}: max |err| / (sum of |terms|) = {rel:.3e}")
        assert np.all(err <= 2e-4 * bound + 1e-30)


@pytest.mark.parametrize("cfg,seed", [("c0", 0), ("c1", 0), ("c3", 0)])
def test_mixed_sbr_error(egt, cfg, seed):
    inst = make_instance(cfg, seed)
    print(f"[case] mixed sbr {cfg} seed={seed}", flush=True)
    P = Problem(inst)
    G = egt.Game(inst)
    L = Layout(G, P)
    rng = np.random.default_rng(seed + 50)
    for p in (0, 1):
        g = f32_round(rng.standard_normal((P.n_seq[p], P.n)) * 5.0)
        for mu in (2.0, 0.05):
            q, val = egt.smoothed_br_mixed(G, p, dev32(L.to_lib(p, g)), mu)
            torch.cuda.synchronize()
            q = q.double().cpu().numpy()
            val = float(val.cpu().numpy()[0])
            q_o, val_o, _, V = P.sbr(p, g, mu)
            qerr = np.abs(L.from_lib(p, q) - q_o).max()
            verr = abs(val - val_o) / (abs(val_o) + np.abs(V).sum())
            print(f"  player {p} mu {mu}: max |q err| = {qerr:.2e}, value rel err = {verr:.2e}")
            assert np.all(q[:, P.n:] == 0)
            assert qerr <= 1e-5 and verr <= 1e-6


@pytest.mark.parametrize("cfg,seed,stride,iters", [("c0", 0, 25, 200), ("c1", 0, 7, 21)])
def test_mixed_one_step_error(egt, cfg, seed, stride, iters):
    inst = make_instance(cfg, seed)
    print(f"[case] mixed one-step {cfg} seed={seed}", flush=True)
    P = Problem(inst)
    E = EGT(P)
    states = []

    def rec(t, x, y, mu_x, mu_y, tau):
        if t % stride == 0 and t < iters:
            states.append((t, x.copy(), y.copy(), mu_x, mu_y, tau))

    solve(P, "AS", eps=0.0, max_iters=iters, on_iterate=rec)
    G = egt.Game(inst)
    L = Layout(G, P)
    st = egt.State(G, variant="AS", eps=0.0, max_iters=10**9, precision="mixed")
    worst = 0.0
    for t, x, y, mu_x, mu_y, tau in states:
        want = iterate(E, "AS", t, x, y, mu_x, mu_y, tau)
        st.set(dev64(L.to_lib(0, x)), dev64(L.to_lib(1, y)), mu_x, mu_y, tau, t)
        egv, side = st.step(player=want["side"])
        got = st.get()
        gx = L.from_lib(0, got["x"].cpu().numpy())
        gy = L.from_lib(1, got["y"].cpu().numpy())
        ex = np.abs(gx - want["x"]).max() / np.abs(want["x"]).max()
        ey = np.abs(gy - want["y"]).max() / np.abs(want["y"]).max()
        worst = max(worst, ex, ey)
        assert ex <= 2e-3 and ey <= 2e-3, (t, ex, ey)
    print(f"  worst one-step strategy error (relative to max |x|): {worst:.2e}")
    st.close()


@pytest.mark.parametrize("cfg,seed", [("c0", 0), ("c0", 3), ("c1", 0), ("c3", 0), ("lib", 0)])
def test_mixed_solve_reaches_target(egt, cfg, seed):
    inst = make_instance(cfg, seed)
    print(f"[case] mixed solve {cfg} seed={seed}", flush=True)
    P = Problem(inst)
    G = egt.Game(inst)
    L = Layout(G, P)
    eps = 1e-3 * inst.pot
    rm, st = egt.solve(G, keep_state=True, precision="mixed", gap_every=10)
    assert rm["status"] == "EGT_OK" and rm["converged"] == 1
    f = st.get()
    x, y = L.from_lib(0, f["x"].cpu().numpy()), L.from_lib(1, f["y"].cpu().numpy())
    # FP32 iterates: every accepted step rounds (1 - tau) x + tau q to FP32
    # (2^-24 relative), so over ~10^3 iterations a simplex of up to 10 actions
    # drifts from its parent's mass by ~10 x sqrt(10^3) x 6e-8 = 2e-5
    assert P.flow_residual(0, x) < 1e-4 and P.flow_residual(1, y) < 1e-4
    gap_o, brmax, brmin = P.saddle_gap(x, y)
    assert gap_o <= eps * (1 + 1e-9)
    assert abs(rm["gap"] - gap_o) <= 1e-10 * (abs(brmax) + abs(brmin))
    rd, _ = egt.solve(G)
    assert abs(rm["value_p1"] - rd["value_p1"]) <= rm["gap"] + rd["gap"]
    print(f"  mixed: {rm['iters']} iters, gap {rm['gap']:.4g}; fp64: {rd['iters']} iters, gap {rd['gap']:.4g}; "
          f"value diff {abs(rm['value_p1'] - rd['value_p1']):.3g}")
    st.close()


def test_mixed_rejects_nothing_on_the_workload_trees(egt):
    # every benchmark tree ends each sequence in at most one showdown
    for cfg in ("kuhn", "c0", "c1", "c3"):
        G = egt.Game(make_instance(cfg, 0))
        y = G.empty(1, dtype=torch.float32)
        egt.gradient_mixed(G, 0, y)


@pytest.mark.parametrize("cfg,seed,prec,ge", [("c0", 1, "mixed", 10), ("c0", 3, "mixed", 1), ("c0", 2, "fp64", 3)])
def test_solve_equals_stepping_with_gap_tests(egt, cfg, seed, prec, ge):
    """egt_solve runs the next iteration ahead while it decides the current
    one; its result must be bitwise that of plain stepping with a gap test
    before every ge-th iteration."""
    inst = make_instance(cfg, seed)
    print(f"[case] solve vs stepping {cfg} seed={seed} {prec} gap_every={ge}", flush=True)
    G = egt.Game(inst)
    eps = 1e-3 * inst.pot
    r, st1 = egt.solve(G, keep_state=True, precision=prec, gap_every=ge)
    st2 = egt.State(G, precision=prec, gap_every=ge)
    t = 0
    while True:
        if t % ge == 0:
            gap, _, _ = st2.gap()
            if gap <= eps:
                break
        st2.step()
        t += 1
    a, b = st1.get(), st2.get()
    assert a["iters"] == b["iters"] == r["iters"]
    assert torch.equal(a["x"], b["x"]) and torch.equal(a["y"], b["y"])
    assert r["gap"] == gap
    st1.close()
    st2.close()
