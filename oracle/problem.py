"""Oracle, part 2: payoff operator and dilated-entropy treeplex math (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is written from the plain definitions, vectorised over the
private hands (the root Cartesian product of Section 6) with NumPy:

* ``grad_x(y) = A y`` and ``grad_y(x) = A^T x`` for the sequence-form payoff
  matrix of Section 2 (Eq. 2 and the gradient operators that follow it), with
  A's entry for terminal z and hands (h1, h2) equal to
  pi(h1, h2) * u2(z, h1, h2), pi(h1, h2) = b1(h1) b2(h2) [disjoint] / Z.
  The per-terminal hand-vs-hand matrices are dense n x n (compatibility, or
  compatibility times the sign of the strength difference) and are applied
  with a matrix product: the plain O(n^2) definition, no prefix-sum trick.
* the dilated entropy DGF d(q) = sum_j beta_j q_{p_j} d_j(q^j / q_{p_j}) with
  d_j(x) = sum_i x_i log x_i + log n_j and beta_j = 2 + sum_{k in D^j} 2 beta_k
  (Section 4);
* the smoothed best response argmin_q <g, q> + mu d(q) (Section 4, Eq. 4 and
  the leaf / internal-simplex derivation after it): bottom-up, each simplex
  takes q_bar_i proportional to exp(-g~_i / (mu beta_j)) and passes up the
  value g~_i + mu beta_j log q_bar_i + mu beta_j log n_j at the i with the
  largest q_bar_i; top-down, q_i = q_{p_j} q_bar_i;
* the best response min_q <g, q> (the mu -> 0 limit);
* the DGF gradient of the appendix ("Prox shift"), the diameter
  Omega = max d - min d and the largest l1 norm M over the treeplex.

Vectors are ``float64[S_p, n]``: one row per sequence of player p in the
oracle's own sequence order, one column per hand in the instance's order.
"""
from __future__ import annotations

import numpy as np

from .game import Game


class Problem:
    def __init__(self, inst, game: Game | None = None):
        self.inst = inst
        self.game = game if game is not None else Game(inst)
        self.n = inst.n_hands
        cards = inst.hand_cards
        # C[h1, h2] = 1 if the two hands share no card
        share = np.zeros((self.n, self.n), dtype=bool)
        for i in range(cards.shape[1]):
            for j in range(cards.shape[1]):
                share |= cards[:, i][:, None] == cards[:, j][None, :]
        self.C = (~share).astype(np.float64)
        s = inst.strength.astype(np.int64)
        self.sgn = np.sign(s[None, :] - s[:, None]).astype(np.float64)  # sgn(s(h2) - s(h1))
        self.W = self.C * self.sgn
        self.b = [np.asarray(inst.belief[0], np.float64), np.asarray(inst.belief[1], np.float64)]
        self.Z = float(self.b[0] @ self.C @ self.b[1])
        self.tp = self.game.treeplex
        self.n_seq = [t.n_seq for t in self.tp]
        # the payoff is bilinear in the two treeplexes only if every terminal
        # is reached after both players acted (the game gives a one-action
        # decision to a player who would otherwise not have acted)
        assert all(z.seq[0] >= 0 and z.seq[1] >= 0 for z in self.game.terminals)
        self._by_kind = {}
        for kind in ("fold", "show"):
            zs = [z for z in self.game.terminals if z.kind == kind]
            self._by_kind[kind] = (
                np.array([z.seq[0] for z in zs], dtype=np.int64),
                np.array([z.seq[1] for z in zs], dtype=np.int64),
                np.array([z.u for z in zs], dtype=np.float64),
            )

    # ------------------------------------------------------------------
    # payoff operator
    # ------------------------------------------------------------------
    def _rows(self, v, idx):
        """rows of a strategy vector; the empty sequence (-1) has value 1."""
        out = np.ones((len(idx), self.n))
        m = idx >= 0
        out[m] = v[idx[m]]
        return out

    def grad_x(self, y):
        """A y: for each player-1 sequence s1 and hand h1,
        sum over terminals z with sigma_1(z) = s1 of
        (b1(h1)/Z) u(z) sum_{h2} M_z[h1, h2] b2(h2) y[sigma_2(z), h2]."""
        g = np.zeros((self.n_seq[0], self.n))
        for kind, M in (("fold", self.C), ("show", self.W)):
            s0, s1, u = self._by_kind[kind]
            if len(u) == 0:
                continue
            R = (self._rows(y, s1) * self.b[1][None, :]).T  # n x L
            P = (M @ R).T  # L x n
            contrib = P * u[:, None] * (self.b[0] / self.Z)[None, :]
            keep = s0 >= 0
            np.add.at(g, s0[keep], contrib[keep])
        return g

    def grad_y(self, x):
        """A^T x: for each player-2 sequence s2 and hand h2,
        sum over terminals z with sigma_2(z) = s2 of
        (b2(h2)/Z) u(z) sum_{h1} M_z[h1, h2] b1(h1) x[sigma_1(z), h1]."""
        g = np.zeros((self.n_seq[1], self.n))
        for kind, M in (("fold", self.C), ("show", self.W)):
            s0, s1, u = self._by_kind[kind]
            if len(u) == 0:
                continue
            R = (self._rows(x, s0) * self.b[0][None, :]).T  # n x L
            P = (M.T @ R).T
            contrib = P * u[:, None] * (self.b[1] / self.Z)[None, :]
            keep = s1 >= 0
            np.add.at(g, s1[keep], contrib[keep])
        return g

    def value(self, x, y):
        """<x, A y> = expected chips won by player 2."""
        return float(np.sum(x * self.grad_x(y)))

    # ------------------------------------------------------------------
    # treeplex: uniform point, flow check, DGF, gradient, constants
    # ------------------------------------------------------------------
    def _parent_rows(self, p, q, v):
        node = self.tp[p].nodes[v]
        return np.ones(self.n) if node.parent_seq < 0 else q[node.parent_seq]

    def uniform(self, p):
        """x_omega: every information set plays each action with 1/n_j."""
        t = self.tp[p]
        q = np.zeros((t.n_seq, self.n))
        for v in reversed(t.post_order):  # parents first
            node = t.nodes[v]
            q[node.first_seq:node.first_seq + node.n_act] = self._parent_rows(p, q, v)[None, :] / node.n_act
        return q

    def flow_residual(self, p, q):
        """max over information sets of |sum_a q[v,a] - q_{p_v}|."""
        t = self.tp[p]
        r = 0.0
        for v, node in enumerate(t.nodes):
            s = q[node.first_seq:node.first_seq + node.n_act].sum(0)
            r = max(r, float(np.max(np.abs(s - self._parent_rows(p, q, v)))))
        return r

    def dgf(self, p, q):
        """d(q) = sum_j beta_j q_{p_j} d_j(q^j / q_{p_j}); a simplex whose parent
        mass is zero contributes zero (the limit)."""
        t = self.tp[p]
        total = 0.0
        for v, node in enumerate(t.nodes):
            par = self._parent_rows(p, q, v)
            blk = q[node.first_seq:node.first_seq + node.n_act]
            live = par > 0
            qb = np.zeros_like(blk)
            qb[:, live] = blk[:, live] / par[None, live]
            with np.errstate(divide="ignore", invalid="ignore"):
                ent = np.where(qb > 0, qb * np.log(qb), 0.0).sum(0)
            total += float(np.sum(node.beta * par[live] * (ent[live] + np.log(node.n_act))))
        return total

    def dgf_grad_free(self, p, q):
        """Partial derivatives of d at an arbitrary positive q (flow constraints
        not assumed): for i in simplex j,
        beta_j (log(q_i/q_{p_j}) + 1) + sum_{k in D_j^i} beta_k (log n_k - sum_{i' in I_k} q_i'/q_i)."""
        t = self.tp[p]
        gr = np.zeros_like(q)
        for v, node in enumerate(t.nodes):
            par = self._parent_rows(p, q, v)
            for a in range(node.n_act):
                s = node.first_seq + a
                gr[s] += node.beta * (np.log(q[s] / par) + 1.0)
                for k in node.children[a]:
                    ch = t.nodes[k]
                    mass = q[ch.first_seq:ch.first_seq + ch.n_act].sum(0)
                    gr[s] += ch.beta * (np.log(ch.n_act) - mass / q[s])
        return gr

    def dgf_grad(self, p, logqbar):
        """The appendix's gradient on the treeplex, from the local log q_bar:
        grad_{ji} d = beta_j (log q_bar_i + 1) + sum_{k in D_j^i} beta_k (log n_k - 1)."""
        t = self.tp[p]
        gr = np.zeros_like(logqbar)
        for node in t.nodes:
            for a in range(node.n_act):
                s = node.first_seq + a
                gr[s] = node.beta * (logqbar[s] + 1.0)
                for k in node.children[a]:
                    ch = t.nodes[k]
                    gr[s] += ch.beta * (np.log(ch.n_act) - 1.0)
        return gr

    def prox_shift_constant(self, p):
        """Appendix: <grad d(q), q> - d(q) = -sum_{root j} beta_j q_{p_j} (log n_j - 1),
        with q_{p_j} = 1 at every root simplex (one per hand per root node)."""
        t = self.tp[p]
        return -float(sum(t.nodes[v].beta * (np.log(t.nodes[v].n_act) - 1.0) for v in t.roots())) * self.n

    def omega(self, p):
        """Omega = max d - min d over the treeplex; min d = 0 at x_omega and the
        max is reached by a pure strategy: Omega_v = beta_v log n_v + max_a sum_k Omega_k."""
        t = self.tp[p]
        om = {}
        for v in t.post_order:
            node = t.nodes[v]
            om[v] = node.beta * np.log(node.n_act) + max(sum(om[k] for k in ch) for ch in node.children)
        return self.n * sum(om[v] for v in t.roots())

    def max_l1(self, p):
        """M = max ||q||_1 over the treeplex (Section 4: the DGF is 1/M-strongly convex)."""
        t = self.tp[p]
        m = {}
        for v in t.post_order:
            node = t.nodes[v]
            m[v] = 1.0 + max(sum(m[k] for k in ch) for ch in node.children)
        return self.n * sum(m[v] for v in t.roots())

    def norm_A(self):
        """l1 operator norm of A = its largest absolute entry."""
        pi = self.b[0][:, None] * self.b[1][None, :] * self.C / self.Z
        umax = max(abs(z.u) for z in self.game.terminals)
        return float(pi.max() * umax)

    # ------------------------------------------------------------------
    # smoothed best response and best response
    # ------------------------------------------------------------------
    def sbr(self, p, g, mu):
        """argmin_{q in Q_p} <g, q> + mu d(q) and its value.

        Returns (q, value, logqbar, V) with V the per-(node, hand) simplex values."""
        t = self.tp[p]
        V = np.zeros((len(t.nodes), self.n))
        logqbar = np.zeros((t.n_seq, self.n))
        qbar_all = np.zeros((t.n_seq, self.n))
        for v in t.post_order:  # bottom-up
            node = t.nodes[v]
            sl = slice(node.first_seq, node.first_seq + node.n_act)
            gt = g[sl].copy()
            for a in range(node.n_act):
                for k in node.children[a]:
                    gt[a] += V[k]
            temp = mu * node.beta
            # q_bar_i proportional to exp(-g~_i / temp), shifted by the smallest g~
            # so the largest weight is exactly 1
            shift = gt.min(axis=0)
            w = np.exp(-(gt - shift[None, :]) / temp)
            tot = w.sum(axis=0)
            qbar = w / tot[None, :]
            qbar_all[sl] = qbar
            logqbar[sl] = -(gt - shift[None, :]) / temp - np.log(tot)[None, :]
            i_star = np.argmax(qbar, axis=0)
            cols = np.arange(self.n)
            V[v] = gt[i_star, cols] + temp * logqbar[sl][i_star, cols] + temp * np.log(node.n_act)
        q = np.zeros((t.n_seq, self.n))
        # top-down: the treeplex scales each simplex by its parent sequence
        # (Section 3), so a sequence's mass is the parent's mass times the local
        # probability of the action, q_i = q_{p_j} q_bar_i (Section 4)
        for v in reversed(t.post_order):
            node = t.nodes[v]
            sl = slice(node.first_seq, node.first_seq + node.n_act)
            q[sl] = self._parent_rows(p, q, v)[None, :] * qbar_all[sl]
        value = float(sum(V[v].sum() for v in t.roots()))
        return q, value, logqbar, V

    def br(self, p, g):
        """min_{q in Q_p} <g, q>: bottom-up min over actions of g + child values."""
        t = self.tp[p]
        V = np.zeros((len(t.nodes), self.n))
        for v in t.post_order:
            node = t.nodes[v]
            gt = g[node.first_seq:node.first_seq + node.n_act].copy()
            for a in range(node.n_act):
                for k in node.children[a]:
                    gt[a] += V[k]
            V[v] = gt.min(axis=0)
        return float(sum(V[v].sum() for v in t.roots()))

    def br_strategy(self, p, g):
        """A pure best response (lowest action index on ties) and its value."""
        t = self.tp[p]
        V = np.zeros((len(t.nodes), self.n))
        choice = np.zeros((len(t.nodes), self.n), dtype=np.int64)
        for v in t.post_order:
            node = t.nodes[v]
            gt = g[node.first_seq:node.first_seq + node.n_act].copy()
            for a in range(node.n_act):
                for k in node.children[a]:
                    gt[a] += V[k]
            choice[v] = np.argmin(gt, axis=0)
            V[v] = gt.min(axis=0)
        q = np.zeros((t.n_seq, self.n))
        for v in reversed(t.post_order):
            node = t.nodes[v]
            par = self._parent_rows(p, q, v)
            for a in range(node.n_act):
                q[node.first_seq + a] = par * (choice[v] == a)
        return q, float(sum(V[v].sum() for v in t.roots()))

    # ------------------------------------------------------------------
    # EGT quantities (Section 2)
    # ------------------------------------------------------------------
    def egv(self, x, y, mu_x, mu_y):
        """EGV = phi_{mu_x}(y) - f_{mu_y}(x) with
        phi_{mu_x}(y) = min_x <x, A y> + mu_x d_X(x) = SBR value of A y, and
        f_{mu_y}(x) = max_y <x, A y> - mu_y d_Y(y) = -(SBR value of -A^T x)."""
        phi = self.sbr(0, self.grad_x(y), mu_x)[1]
        f = -self.sbr(1, -self.grad_y(x), mu_y)[1]
        return phi - f, phi, f

    def saddle_gap(self, x, y):
        """eps_sad = max_y x^T A y - min_x x^T A y (both players' regrets summed)."""
        br_max_y = -self.br(1, -self.grad_y(x))
        br_min_x = self.br(0, self.grad_x(y))
        return br_max_y - br_min_x, br_max_y, br_min_x
