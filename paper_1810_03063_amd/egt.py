"""Python binding of libegt (the C ABI in include/egt.h).

Argument marshalling only: every computation runs in the HIP kernels of
libegt.so.  PyTorch provides device memory (float64 CUDA tensors) and the
current HIP stream.  Importing this module fails with ImportError when the
library has not been built (python -m paper_1810_03063_amd.build).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libegt.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_1810_03063_amd.build`")
_lib = ctypes.CDLL(_LIB_PATH)

EGT_OK = 0
ERRORS = {-1: "EGT_EINVAL", -2: "EGT_ENOMEM", -3: "EGT_EDEVICE", -4: "EGT_ENUMERIC",
          -5: "EGT_ENOTCONV", -6: "EGT_EBUDGET"}
VARIANTS = {"ALT": 0, "BAL": 1, "AS": 2}

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double


class EgtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class BetAbstraction(ctypes.Structure):
    _fields_ = [
        ("n_fracs", (_i32 * 4) * 2), ("fracs", (_p * 4) * 2), ("allin", (_i32 * 4) * 2), ("open_fold", _i32 * 2),
    ]


class GameDesc(ctypes.Structure):
    _fields_ = [
        ("n_cards", _i32), ("cards_per_hand", _i32), ("n_hands", _i32),
        ("hand_cards", _p), ("strength", _p), ("belief", _p * 2),
        ("pot", _f64), ("stack", _f64),
        ("n_bet_fracs", _i32), ("bet_fracs", _p),
        ("allin", _i32), ("max_raises", _i32),
        ("abstraction", ctypes.POINTER(BetAbstraction)),
    ]


class GeneralDesc(ctypes.Structure):
    _fields_ = [("n_infosets", ctypes.c_int32 * 2), ("parent_seq", ctypes.c_void_p * 2),
                ("n_actions", ctypes.c_void_p * 2), ("nnz", ctypes.c_int64), ("a_row", ctypes.c_void_p),
                ("a_col", ctypes.c_void_p), ("a_val", ctypes.c_void_p), ("scale", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("variant", _i32), ("precision", _i32), ("eps", _f64), ("max_iters", _i64),
        ("mu0_x", _f64), ("mu0_y", _f64), ("tau0", _f64), ("gap_every", _i32), ("fresh_products", _i32),
    ]


class SolveResult(ctypes.Structure):
    _fields_ = [
        ("iters", _i64), ("products", _i64), ("backtracks", _i64),
        ("gap", _f64), ("br_max_y", _f64), ("br_min_x", _f64), ("value_p1", _f64),
        ("mu_x", _f64), ("mu_y", _f64), ("tau", _f64), ("seconds", _f64),
        ("converged", _i32), ("reserved", _i32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def _decl(name, restype, *args):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_last_error = _decl("egt_last_error", ctypes.c_char_p)
_default_opts = _decl("egt_default_opts", None, ctypes.POINTER(SolveOpts))
_build_game = _decl("egt_build_game", ctypes.c_int, ctypes.POINTER(GameDesc), _p, ctypes.POINTER(_p))
_build_general_game = _decl("egt_build_general_game", ctypes.c_int, ctypes.POINTER(GeneralDesc), _p,
                            ctypes.POINTER(_p))
_free_game = _decl("egt_free_game", ctypes.c_int, _p)
_game_dims = _decl("egt_game_dims", ctypes.c_int, _p, ctypes.c_int, ctypes.POINTER(_i64),
                   ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_game_layout = _decl("egt_game_layout", ctypes.c_int, _p, ctypes.c_int, _p, _p, _i64, ctypes.POINTER(_i64))
_game_terminals = _decl("egt_game_terminals", ctypes.c_int, _p, ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_gradient = _decl("egt_gradient", ctypes.c_int, _p, ctypes.c_int, _p, _p, _p)
_smoothed_br = _decl("egt_smoothed_br", ctypes.c_int, _p, ctypes.c_int, _p, _f64, _p, _p, _p)
_gradient_mixed = _decl("egt_gradient_mixed", ctypes.c_int, _p, ctypes.c_int, _p, _p, _p)
_smoothed_br_mixed = _decl("egt_smoothed_br_mixed", ctypes.c_int, _p, ctypes.c_int, _p, _f64, _p, _p, _p)
_best_response = _decl("egt_best_response", ctypes.c_int, _p, ctypes.c_int, _p, _p, _p)
_uniform = _decl("egt_uniform", ctypes.c_int, _p, ctypes.c_int, _p, _p)
_saddle_gap = _decl("egt_saddle_gap", ctypes.c_int, _p, _p, _p, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                    ctypes.POINTER(_f64), _p)
_saddle_gap_noalloc = _decl("egt_saddle_gap_noalloc", ctypes.c_int, _p, _p, _p, _p, _p)
_state_create = _decl("egt_state_create", ctypes.c_int, _p, ctypes.POINTER(SolveOpts), _p, ctypes.POINTER(_p))
_state_destroy = _decl("egt_state_destroy", ctypes.c_int, _p)
_step = _decl("egt_step", ctypes.c_int, _p, ctypes.c_int, ctypes.POINTER(_f64), ctypes.POINTER(ctypes.c_int), _p)
_state_get = _decl("egt_state_get", ctypes.c_int, _p, _p, _p, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                   ctypes.POINTER(_f64), ctypes.POINTER(_i64), _p)
_state_get_products = _decl("egt_state_get_products", ctypes.c_int, _p, _p, _p, _p)
_state_set = _decl("egt_state_set", ctypes.c_int, _p, _p, _p, _f64, _f64, _f64, _i64, _p, _p, _p)
_state_gap = _decl("egt_state_gap", ctypes.c_int, _p, ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                   ctypes.POINTER(_f64), _p)
_solve = _decl("egt_solve", ctypes.c_int, _p, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveResult),
               ctypes.POINTER(_p), _p)

_cfr_create = _decl("egt_cfr_create", ctypes.c_int, _p, _i32, _p, ctypes.POINTER(_p))
_cfr_destroy = _decl("egt_cfr_destroy", ctypes.c_int, _p)
_cfr_step = _decl("egt_cfr_step", ctypes.c_int, _p, _i32, _p)
_cfr_gap = _decl("egt_cfr_gap", ctypes.c_int, _p, ctypes.POINTER(_f64), ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                 _p)
_cfr_get = _decl("egt_cfr_get", ctypes.c_int, _p, _p, _p, _p, _p, ctypes.POINTER(_i64), _p)
_cfr_solve = _decl("egt_cfr_solve", ctypes.c_int, _p, _i32, _f64, _i64, _i32, ctypes.POINTER(SolveResult), _p)

_fom_create = _decl("egt_fom_create", ctypes.c_int, _p, _i32, _f64, _f64, _p, ctypes.POINTER(_p))
_fom_destroy = _decl("egt_fom_destroy", ctypes.c_int, _p)
_fom_step = _decl("egt_fom_step", ctypes.c_int, _p, _i32, _p)
_fom_get = _decl("egt_fom_get", ctypes.c_int, _p, _p, _p, _p, _p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _p)
_fom_gap = _decl("egt_fom_gap", ctypes.c_int, _p, ctypes.POINTER(_f64), ctypes.POINTER(_f64), ctypes.POINTER(_f64),
                 _p)

_state_bytes = _decl("egt_state_bytes", ctypes.c_int, _p, ctypes.POINTER(SolveOpts), ctypes.POINTER(_i64))
_batch_create = _decl("egt_batch_create", ctypes.c_int, _i64, _i32, ctypes.POINTER(_p))
_batch_destroy = _decl("egt_batch_destroy", ctypes.c_int, _p)
_batch_admit = _decl("egt_batch_admit", ctypes.c_int, _p, _p, ctypes.POINTER(SolveOpts), ctypes.POINTER(_i32))
_batch_tick = _decl("egt_batch_tick", ctypes.c_int, _p, ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_batch_poll = _decl("egt_batch_poll", ctypes.c_int, _p, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                    ctypes.POINTER(SolveResult))
_batch_retire = _decl("egt_batch_retire", ctypes.c_int, _p, _i32)
_batch_admit_desc = _decl("egt_batch_admit_desc", ctypes.c_int, _p, ctypes.POINTER(GameDesc),
                          ctypes.POINTER(SolveOpts), ctypes.POINTER(_i32))
_batch_strategies = _decl("egt_batch_strategies", ctypes.c_int, _p, _i32, _p, _p, _p)
_batch_usage = _decl("egt_batch_usage", ctypes.c_int, _p, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                     ctypes.POINTER(_i32))

EXPORTED = [
    "egt_last_error", "egt_default_opts", "egt_build_game", "egt_free_game", "egt_game_dims",
    "egt_game_layout", "egt_game_terminals", "egt_gradient", "egt_smoothed_br", "egt_best_response",
    "egt_gradient_mixed", "egt_smoothed_br_mixed",
    "egt_uniform", "egt_saddle_gap", "egt_state_create", "egt_state_destroy", "egt_step",
    "egt_state_get", "egt_state_get_products", "egt_state_set", "egt_state_gap", "egt_solve",
    "egt_state_bytes", "egt_batch_create", "egt_batch_destroy", "egt_batch_admit", "egt_batch_tick",
    "egt_batch_poll", "egt_batch_retire", "egt_batch_usage", "egt_saddle_gap_noalloc",
    "egt_batch_strategies", "egt_cfr_create", "egt_cfr_destroy", "egt_cfr_step", "egt_cfr_gap", "egt_cfr_get",
    "egt_cfr_solve", "egt_batch_admit_desc", "egt_fom_create", "egt_fom_destroy", "egt_fom_step", "egt_fom_get", "egt_fom_gap",
    "egt_build_general_game",
]


def _check(rc, allow=()):
    if rc != EGT_OK and rc not in allow:
        raise EgtError(rc, (_last_error() or b"").decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, shape=None, dtype=torch.float64):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def game_desc(inst):
    """egt_game_desc of an instance, and the host arrays it points into (keep
    them alive while the description is in use)."""
    cards = np.ascontiguousarray(inst.hand_cards, dtype=np.int32)
    strength = np.ascontiguousarray(inst.strength, dtype=np.int32)
    b = [np.ascontiguousarray(inst.belief[p], dtype=np.float64) for p in (0, 1)]
    fr = np.ascontiguousarray(inst.bet_fracs, dtype=np.float64)
    d = GameDesc()
    d.n_cards = inst.n_cards
    d.cards_per_hand = inst.cards_per_hand
    d.n_hands = inst.n_hands
    d.hand_cards = cards.ctypes.data
    d.strength = strength.ctypes.data
    d.belief[0] = b[0].ctypes.data
    d.belief[1] = b[1].ctypes.data
    d.pot = inst.pot
    d.stack = inst.stack
    d.n_bet_fracs = len(fr)
    d.bet_fracs = fr.ctypes.data if len(fr) else None
    d.allin = 1 if inst.allin else 0
    d.max_raises = inst.max_raises
    keep = [cards, strength, b, fr]
    ab = getattr(inst, "abstraction", None)
    if ab is not None:
        a = BetAbstraction()
        for p in (0, 1):
            a.open_fold[p] = 1 if ab.open_fold[p] else 0
            for k in range(4):
                fr_k = np.ascontiguousarray(ab.fracs[p][k], dtype=np.float64)
                keep.append(fr_k)
                a.n_fracs[p][k] = len(fr_k)
                a.fracs[p][k] = fr_k.ctypes.data if len(fr_k) else None
                a.allin[p][k] = 1 if ab.allin[p][k] else 0
        keep.append(a)
        d.abstraction = ctypes.pointer(a)
    return d, keep


class Game:
    """A river endgame uploaded to the current device (egt_build_game)."""

    def __init__(self, inst, stream=None):
        self._h = None
        d, keep = game_desc(inst)
        h = _p()
        _check(_build_game(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        del keep
        self._h = h
        self.inst = inst
        self.pot = inst.pot
        dims = [self._dims(p) for p in (0, 1)]
        self.n_seq = [d_[0] for d_ in dims]
        self.n = dims[0][1]
        self.ld = dims[0][2]
        self.n_nodes = [d_[3] for d_ in dims]

    def _dims(self, p):
        a, b, c, d = _i64(), _i64(), _i64(), _i64()
        _check(_game_dims(self._h, p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    @property
    def handle(self):
        return self._h

    def layout(self, p):
        """(sequence keys in library order, slot -> instance hand index)."""
        need = _i64()
        _check(_game_layout(self._h, p, None, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        perm = np.zeros(self.n, dtype=np.int32)
        _check(_game_layout(self._h, p, ctypes.c_void_p(perm.ctypes.data), buf, need.value, ctypes.byref(need)))
        keys = buf.value.decode().split("\n")[:-1]
        return keys, perm

    def terminals(self):
        f, s = _i64(), _i64()
        _check(_game_terminals(self._h, ctypes.byref(f), ctypes.byref(s)))
        return f.value, s.value

    def empty(self, p, device="cuda", dtype=torch.float64):
        return torch.zeros((self.n_seq[p], self.ld), dtype=dtype, device=device)

    def close(self):
        if self._h is not None:
            _check(_free_game(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def general_desc(inst):
    """egt_general_desc of a general game (parents, action counts, payoff
    triples) and the host arrays it points into."""
    d = GeneralDesc()
    keep = []
    for p in (0, 1):
        sets = inst.infosets[p]
        par = np.ascontiguousarray([s_[0] for s_ in sets], dtype=np.int32)
        nact = np.ascontiguousarray([s_[1] for s_ in sets], dtype=np.int32)
        keep += [par, nact]
        d.n_infosets[p] = len(sets)
        d.parent_seq[p] = par.ctypes.data
        d.n_actions[p] = nact.ctypes.data
    e = inst.entries
    rows = np.ascontiguousarray([t[0] for t in e], dtype=np.int32)
    cols = np.ascontiguousarray([t[1] for t in e], dtype=np.int32)
    vals = np.ascontiguousarray([t[2] for t in e], dtype=np.float64)
    keep += [rows, cols, vals]
    d.nnz = len(e)
    d.a_row = rows.ctypes.data if len(e) else None
    d.a_col = cols.ctypes.data if len(e) else None
    d.a_val = vals.ctypes.data if len(e) else None
    d.scale = inst.pot
    return d, keep


class GeneralGame(Game):
    """A general extensive-form game uploaded to the current device
    (egt_build_general_game): one live slot per row; every FP64 entry point
    accepts it."""

    def __init__(self, inst, stream=None):
        self._h = None
        d, keep = general_desc(inst)
        h = _p()
        _check(_build_general_game(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        del keep
        self._h = h
        self.inst = inst
        self.pot = inst.pot
        dims = [self._dims(p) for p in (0, 1)]
        self.n_seq = [d_[0] for d_ in dims]
        self.n = dims[0][1]
        self.ld = dims[0][2]
        self.n_nodes = [d_[3] for d_ in dims]

    def seq_order(self, p):
        """library row of each of the caller's sequences."""
        keys, _ = self.layout(p)
        out = np.empty(len(keys), dtype=np.int64)
        for lib, k in enumerate(keys):
            out[int(k)] = lib
        return out


def gradient(game: Game, player: int, strat_other, out=None, stream=None):
    """A y (player 0) or A^T x (player 1) into out (allocated if None)."""
    if out is None:
        out = game.empty(player)
    _check(_gradient(game.handle, player, _dptr(strat_other, (game.n_seq[1 - player], game.ld)),
                     _dptr(out, (game.n_seq[player], game.ld)), _stream(stream)))
    return out


def smoothed_br(game: Game, player: int, grad, mu: float, strat_out=None, value_out=None, stream=None,
                want_value=True):
    """argmin_q <grad, q> + mu d(q): returns (strategy tensor, value tensor[1] or None).
    want_value=False skips the value (one launch instead of two)."""
    if strat_out is None:
        strat_out = game.empty(player)
    if value_out is None and want_value:
        value_out = torch.zeros(1, dtype=torch.float64, device=grad.device)
    _check(_smoothed_br(game.handle, player, _dptr(grad, (game.n_seq[player], game.ld)), float(mu),
                        _dptr(strat_out, (game.n_seq[player], game.ld)),
                        _dptr(value_out) if value_out is not None else None, _stream(stream)))
    return strat_out, value_out


def gradient_mixed(game: Game, player: int, strat_other, out=None, stream=None):
    """Precision-form product (FP32 in/out, BF16 hi+lo showdown GEMM)."""
    f32 = torch.float32
    if out is None:
        out = game.empty(player, dtype=f32)
    _check(_gradient_mixed(game.handle, player, _dptr(strat_other, (game.n_seq[1 - player], game.ld), f32),
                           _dptr(out, (game.n_seq[player], game.ld), f32), _stream(stream)))
    return out


def smoothed_br_mixed(game: Game, player: int, grad, mu: float, strat_out=None, value_out=None, stream=None):
    """Precision-form smoothed best response: FP32 strategy, FP64 value."""
    f32 = torch.float32
    if strat_out is None:
        strat_out = game.empty(player, dtype=f32)
    if value_out is None:
        value_out = torch.zeros(1, dtype=torch.float64, device=grad.device)
    _check(_smoothed_br_mixed(game.handle, player, _dptr(grad, (game.n_seq[player], game.ld), f32), float(mu),
                              _dptr(strat_out, (game.n_seq[player], game.ld), f32), _dptr(value_out),
                              _stream(stream)))
    return strat_out, value_out


def best_response(game: Game, player: int, grad, value_out=None, stream=None):
    if value_out is None:
        value_out = torch.zeros(1, dtype=torch.float64, device=grad.device)
    _check(_best_response(game.handle, player, _dptr(grad, (game.n_seq[player], game.ld)), _dptr(value_out),
                          _stream(stream)))
    return value_out


def uniform(game: Game, player: int, out=None, stream=None):
    if out is None:
        out = game.empty(player)
    _check(_uniform(game.handle, player, _dptr(out, (game.n_seq[player], game.ld)), _stream(stream)))
    return out


def saddle_gap(game: Game, x, y, stream=None):
    """(gap, max_y x^T A y, min_x x^T A y) as Python floats."""
    g, a, b = _f64(), _f64(), _f64()
    _check(_saddle_gap(game.handle, _dptr(x, (game.n_seq[0], game.ld)), _dptr(y, (game.n_seq[1], game.ld)),
                       ctypes.byref(g), ctypes.byref(a), ctypes.byref(b), _stream(stream)))
    return g.value, a.value, b.value


def saddle_gap_noalloc(game: Game, x, y, out3=None, stream=None):
    """egt_saddle_gap_noalloc: {gap, max_y x^T A y, min_x x^T A y} into the
    device tensor out3 (3 doubles, allocated here if None), no sync."""
    if out3 is None:
        out3 = torch.empty(3, dtype=torch.float64, device=x.device)
    _check(_saddle_gap_noalloc(game.handle, _dptr(x, (game.n_seq[0], game.ld)), _dptr(y, (game.n_seq[1], game.ld)),
                               _dptr(out3, (3,)), _stream(stream)))
    return out3


PRECISIONS = {"fp64": 0, "mixed": 1}


def make_opts(variant="AS", eps=None, max_iters=100000, mu0=None, tau0=0.5, gap_every=1, precision="fp64",
              fresh_products=False):
    o = SolveOpts()
    _default_opts(ctypes.byref(o))
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.eps = 0.0 if eps is None else float(eps)
    o.max_iters = int(max_iters)
    if mu0 is not None:
        o.mu0_x, o.mu0_y = float(mu0[0]), float(mu0[1])
    o.tau0 = float(tau0)
    o.gap_every = int(gap_every)
    o.fresh_products = 1 if fresh_products else 0
    return o


class State:
    """Device-resident EGT iterates (egt_state_create / egt_step)."""

    def __init__(self, game: Game, stream=None, handle=None, **opts):
        self.game = game
        self._h = None
        if handle is not None:
            self._h = handle
            return
        o = make_opts(**opts)
        h = _p()
        _check(_state_create(game.handle, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self._h = h

    def step(self, player=-1, stream=None):
        egv = _f64()
        side = ctypes.c_int()
        _check(_step(self._h, int(player), ctypes.byref(egv), ctypes.byref(side), _stream(stream)))
        return egv.value, side.value

    def gap(self, stream=None):
        g, a, b = _f64(), _f64(), _f64()
        _check(_state_gap(self._h, ctypes.byref(g), ctypes.byref(a), ctypes.byref(b), _stream(stream)))
        return g.value, a.value, b.value

    def get(self, stream=None):
        x = self.game.empty(0)
        y = self.game.empty(1)
        mx, my, tau = _f64(), _f64(), _f64()
        it = _i64()
        _check(_state_get(self._h, _dptr(x), _dptr(y), ctypes.byref(mx), ctypes.byref(my), ctypes.byref(tau),
                          ctypes.byref(it), _stream(stream)))
        return dict(x=x, y=y, mu_x=mx.value, mu_y=my.value, tau=tau.value, iters=it.value)

    def products(self, stream=None):
        """(A y, A^T x) cached for the current iterate."""
        ay, atx = self.game.empty(0), self.game.empty(1)
        _check(_state_get_products(self._h, _dptr(ay), _dptr(atx), _stream(stream)))
        return ay, atx

    def set(self, x, y, mu_x, mu_y, tau, iters=0, ay=None, atx=None, stream=None):
        """Restart from (x, y, mu, tau, t); products recomputed unless given."""
        g = self.game
        _check(_state_set(self._h, _dptr(x, (g.n_seq[0], g.ld)), _dptr(y, (g.n_seq[1], g.ld)), float(mu_x),
                          float(mu_y), float(tau), int(iters), _dptr(ay, (g.n_seq[0], g.ld)),
                          _dptr(atx, (g.n_seq[1], g.ld)), _stream(stream)))

    def close(self):
        if self._h is not None:
            _check(_state_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(game: Game, keep_state=False, stream=None, **opts):
    """egt_solve: returns (result dict, State or None)."""
    o = make_opts(**opts)
    res = SolveResult()
    h = _p()
    rc = _solve(game.handle, ctypes.byref(o), ctypes.byref(res), ctypes.byref(h) if keep_state else None,
                _stream(stream))
    _check(rc, allow=(-5,))
    out = res.as_dict()
    out["status"] = ERRORS.get(rc, "EGT_OK") if rc else "EGT_OK"
    st = State(game, handle=h) if keep_state and h.value else None
    return out, st


def state_bytes(game: Game, **opts):
    o = make_opts(**opts)
    b = _i64()
    _check(_state_bytes(game.handle, ctypes.byref(o), ctypes.byref(b)))
    return b.value


class Batch:
    """Continuous batching of solves (egt_batch_*): admit / tick / poll / retire."""

    def __init__(self, budget_bytes: int, max_slots: int = 64):
        h = _p()
        _check(_batch_create(int(budget_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h

    def admit(self, game: Game, **opts):
        """Slot index, or None when the solve does not fit the budget / slots now."""
        o = make_opts(**opts)
        slot = _i32()
        rc = _batch_admit(self._h, game.handle, ctypes.byref(o), ctypes.byref(slot))
        if rc == -6:
            return None
        _check(rc)
        return slot.value

    def admit_desc(self, inst, **opts):
        """Admission by description (the batch builds the game in its arena):
        slot index, or None when it does not fit the budget / slots now."""
        o = make_opts(**opts)
        d, keep = game_desc(inst)
        slot = _i32()
        rc = _batch_admit_desc(self._h, ctypes.byref(d), ctypes.byref(o), ctypes.byref(slot))
        del keep
        if rc == -6:
            return None
        _check(rc)
        return slot.value

    def tick(self):
        """(live solves, solves finished in this tick)."""
        a, f = _i32(), _i32()
        _check(_batch_tick(self._h, ctypes.byref(a), ctypes.byref(f)))
        return a.value, f.value

    def poll(self, slot: int):
        """None while running, else (status name, result dict)."""
        d, st = _i32(), _i32()
        res = SolveResult()
        _check(_batch_poll(self._h, int(slot), ctypes.byref(d), ctypes.byref(st), ctypes.byref(res)))
        if not d.value:
            return None
        return (ERRORS.get(st.value, "EGT_OK") if st.value else "EGT_OK"), res.as_dict()

    def retire(self, slot: int):
        _check(_batch_retire(self._h, int(slot)))

    def strategies(self, slot: int, game: Game, stream=None):
        """Final (x, y) of a finished slot as FP64 device tensors."""
        x, y = game.empty(0), game.empty(1)
        _check(_batch_strategies(self._h, int(slot), _dptr(x), _dptr(y), _stream(stream)))
        return x, y

    def usage(self):
        u, live, done = _i64(), _i32(), _i32()
        _check(_batch_usage(self._h, ctypes.byref(u), ctypes.byref(live), ctypes.byref(done)))
        return u.value, live.value, done.value

    def close(self):
        if self._h is not None:
            _check(_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CFR_VARIANTS = {"CFR": 0, "CFR_RMP": 1, "CFR_PLUS": 2}


class Cfr:
    """A CFR(RM) / CFR(RM+) / CFR+ run on the device (egt_cfr_*)."""

    def __init__(self, game: Game, variant="CFR_PLUS", stream=None):
        self.game = game
        self._h = None
        h = _p()
        _check(_cfr_create(game.handle, CFR_VARIANTS[variant], _stream(stream), ctypes.byref(h)))
        self._h = h

    def step(self, iters=1, stream=None):
        _check(_cfr_step(self._h, int(iters), _stream(stream)))

    def gap(self, stream=None):
        g, a, b = _f64(), _f64(), _f64()
        _check(_cfr_gap(self._h, ctypes.byref(g), ctypes.byref(a), ctypes.byref(b), _stream(stream)))
        return g.value, a.value, b.value

    def get(self, stream=None):
        G = self.game
        xa, ya, xc, yc = G.empty(0), G.empty(1), G.empty(0), G.empty(1)
        it = _i64()
        _check(_cfr_get(self._h, _dptr(xa), _dptr(ya), _dptr(xc), _dptr(yc), ctypes.byref(it), _stream(stream)))
        torch.cuda.synchronize()
        return dict(x_avg=xa, y_avg=ya, x=xc, y=yc, iters=it.value)

    def close(self):
        if self._h is not None:
            _check(_cfr_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cfr_solve(game: Game, variant="CFR_PLUS", eps=None, max_iters=100000, gap_every=10, stream=None):
    """egt_cfr_solve: result dict with status."""
    res = SolveResult()
    rc = _cfr_solve(game.handle, CFR_VARIANTS[variant], 0.0 if eps is None else float(eps), int(max_iters),
                    int(gap_every), ctypes.byref(res), _stream(stream))
    _check(rc, allow=(-5,))
    out = res.as_dict()
    out["status"] = ERRORS.get(rc, "EGT_OK") if rc else "EGT_OK"
    return out


FOM_METHODS = {"MP": 0, "CP": 1}


class Fom:
    """Mirror prox ("MP", steps eta_x, eta_y) or Chambolle-Pock ("CP", steps
    tau, sigma) on the device (egt_fom_*)."""

    def __init__(self, game: Game, method="MP", step_x=1.0, step_y=None, stream=None):
        self.game = game
        self._h = None
        h = _p()
        sy = step_x if step_y is None else step_y
        _check(_fom_create(game.handle, FOM_METHODS[method], float(step_x), float(sy), _stream(stream),
                           ctypes.byref(h)))
        self._h = h

    def step(self, iters=1, stream=None):
        _check(_fom_step(self._h, int(iters), _stream(stream)))

    def gap(self, stream=None):
        g, a, b = _f64(), _f64(), _f64()
        _check(_fom_gap(self._h, ctypes.byref(g), ctypes.byref(a), ctypes.byref(b), _stream(stream)))
        return g.value, a.value, b.value

    def get(self, stream=None):
        G = self.game
        xa, ya, xc, yc = G.empty(0), G.empty(1), G.empty(0), G.empty(1)
        it, pr = _i64(), _i64()
        _check(_fom_get(self._h, _dptr(xa), _dptr(ya), _dptr(xc), _dptr(yc), ctypes.byref(it), ctypes.byref(pr),
                        _stream(stream)))
        torch.cuda.synchronize()
        return dict(x_avg=xa, y_avg=ya, x=xc, y=yc, iters=it.value, products=pr.value)

    def close(self):
        if self._h is not None:
            _check(_fom_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
