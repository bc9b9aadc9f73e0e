"""Host-side validation of general-game descriptions (egt_build_general_game):
every malformed description is refused with EGT_EINVAL before any device
call, so these run without a GPU."""
import ctypes

import pytest

from instances.efg import EfgInstance, kuhn_efg

egt = pytest.importorskip("paper_1810_03063_amd.egt")


def _build(inst, edit=None):
    d, keep = egt.general_desc(inst)
    if edit is not None:
        keep.append(edit(d))
    h = ctypes.c_void_p()
    rc = egt._build_general_game(ctypes.byref(d), None, ctypes.byref(h))
    msg = (egt._last_error() or b"").decode()
    del keep
    assert not h.value, "no game may be returned on a refusal"
    return rc, msg


def _with(sets0=None, sets1=None, entries=None, pot=None):
    base = kuhn_efg()
    return EfgInstance("bad", (sets0 if sets0 is not None else base.infosets[0],
                               sets1 if sets1 is not None else base.infosets[1]),
                       entries if entries is not None else base.entries, base.pot if pot is None else pot)


@pytest.mark.parametrize("name,inst,fragment", [
    ("parent after the set", _with(sets0=((-1, 2, "a"), (5, 2, "b"))), "earlier information set"),
    ("parent below -1", _with(sets0=((-2, 2, "a"),)), "earlier information set"),
    ("own parent", _with(sets0=((-1, 2, "a"), (2, 2, "b"))), "earlier information set"),
    ("no actions", _with(sets1=((-1, 0, "a"),)), "1 to 16 actions"),
    ("17 actions", _with(sets1=((-1, 17, "a"),)), "1 to 16 actions"),
    ("no sets", _with(sets0=()), "at least one information set"),
    ("row out of range", _with(entries=((99, 0, 1.0),)), "out of range"),
    ("column out of range", _with(entries=((0, -1, 1.0),)), "out of range"),
    ("non-finite payoff", _with(entries=((0, 0, float("nan")),)), "finite"),
    ("zero scale", _with(pot=0.0), "scale"),
])
def test_bad_descriptions_are_refused(name, inst, fragment):
    rc, msg = _build(inst)
    assert rc == -1, (name, rc, msg)
    assert fragment in msg, (name, msg)


def test_null_triples_with_entries_are_refused():
    def edit(d):
        d.a_val = None
        return None

    rc, msg = _build(kuhn_efg(), edit)
    assert rc == -1 and "triples" in msg


def test_null_arguments():
    h = ctypes.c_void_p()
    assert egt._build_general_game(None, None, ctypes.byref(h)) == -1
    d, keep = egt.general_desc(kuhn_efg())
    assert egt._build_general_game(ctypes.byref(d), None, None) == -1
    del keep
