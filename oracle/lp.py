"""Oracle, part 4: the explicit sequence-form payoff matrix and the LP.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``explicit_A`` writes A out entry by entry from its definition (Section 2,
  Eq. 2): for every terminal z and every pair of hands (h1, h2),
  A[(sigma_1(z), h1), (sigma_2(z), h2)] += pi(h1, h2) u2(z, h1, h2).  It uses
  plain loops and no matrix algebra, so it checks the batched operator in
  ``problem.py`` independently.
* ``lp_value`` solves the bilinear saddle-point problem as one linear program
  (Section 1: dualise the y player's best response and keep x's constraints),
  with HiGHS through ``scipy.optimize.linprog``.  Only for tiny games.

Sequence-form constraints (Section 3): for every information set (v, h),
sum_a q[(v, a), h] = q[(p_v), h], or 1 at a root.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def explicit_A(prob):
    n = prob.n
    inst = prob.inst
    S0, S1 = prob.n_seq
    cards = [set(int(c) for c in inst.hand_cards[h]) for h in range(n)]
    b1, b2 = inst.belief[0], inst.belief[1]
    Z = 0.0
    for h1 in range(n):
        for h2 in range(n):
            if not (cards[h1] & cards[h2]):
                Z += b1[h1] * b2[h2]
    A = np.zeros((S0 * n, S1 * n))
    for z in prob.game.terminals:
        s0, s1 = z.seq
        assert s0 >= 0 and s1 >= 0, "a terminal at an empty sequence has no entry in A"
        for h1 in range(n):
            for h2 in range(n):
                if cards[h1] & cards[h2]:
                    continue
                pi = b1[h1] * b2[h2] / Z
                if z.kind == "fold":
                    u = z.u
                else:
                    d = int(inst.strength[h2]) - int(inst.strength[h1])
                    u = z.u * (1 if d > 0 else (-1 if d < 0 else 0))
                A[s0 * n + h1, s1 * n + h2] += pi * u
    return A


def flow_matrix(prob, p):
    """(E, e) with E q = e the treeplex constraints, q flattened as [seq * n + h]."""
    t = prob.tp[p]
    n = prob.n
    rows, cols, vals, rhs = [], [], [], []
    r = 0
    for node in t.nodes:
        for h in range(n):
            for a in range(node.n_act):
                rows.append(r)
                cols.append((node.first_seq + a) * n + h)
                vals.append(1.0)
            if node.parent_seq >= 0:
                rows.append(r)
                cols.append(node.parent_seq * n + h)
                vals.append(-1.0)
                rhs.append(0.0)
            else:
                rhs.append(1.0)
            r += 1
    E = sp.csr_matrix((vals, (rows, cols)), shape=(r, t.n_seq * n))
    return E, np.array(rhs)


def lp_value(prob, A=None):
    """min_x max_y x^T A y.  The inner max over {y >= 0 : F y = f} has the
    dual min_v f^T v s.t. F^T v >= A^T x, so the LP is
    min_{x >= 0, v free} f^T v  s.t.  A^T x - F^T v <= 0,  E x = e.
    Returns (value, x) with x of shape [S_0, n]."""
    if A is None:
        A = explicit_A(prob)
    E, e = flow_matrix(prob, 0)
    F, f = flow_matrix(prob, 1)
    nx, nv = A.shape[0], F.shape[0]
    c = np.concatenate([np.zeros(nx), f])
    A_ub = sp.hstack([sp.csr_matrix(A.T), -F.T]).tocsr()
    b_ub = np.zeros(A.shape[1])
    A_eq = sp.hstack([E, sp.csr_matrix((E.shape[0], nv))]).tocsr()
    bounds = [(0, None)] * nx + [(None, None)] * nv
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=e, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun), res.x[:nx].reshape(prob.n_seq[0], prob.n)
