"""Conversions between the oracle's layout ([sequence, hand] in the oracle's
sequence order and the instance's hand order) and the library's canonical
layout ([sequence, slot] padded to ld, sequences in the library's order,
slots sorted by strength).  Sequences are matched by their betting-history
key, hands by the library's exported slot permutation."""
import numpy as np


class Layout:
    def __init__(self, game, prob):
        self.n = prob.n
        self.ld = game.ld
        self.rows = []
        self.perm = []
        for p in (0, 1):
            keys, perm = game.layout(p)
            okeys = prob.tp[p].seq_keys
            assert sorted(keys) == sorted(okeys), "library and oracle disagree on the sequences"
            idx = {k: i for i, k in enumerate(okeys)}
            self.rows.append(np.array([idx[k] for k in keys], dtype=np.int64))
            self.perm.append(np.asarray(perm, dtype=np.int64))

    def to_lib(self, p, arr):
        out = np.zeros((len(self.rows[p]), self.ld))
        out[:, :self.n] = np.asarray(arr)[self.rows[p]][:, self.perm[p]]
        return out

    def from_lib(self, p, arr):
        arr = np.asarray(arr)
        out = np.zeros((len(self.rows[p]), self.n))
        out[self.rows[p][:, None], self.perm[p][None, :]] = arr[:, :self.n]
        return out
