"""The C-ABI library loads on a machine without a GPU and exports every
function include/egt.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1810_03063_amd", "libegt.so")
HEADER = os.path.join(ROOT, "include", "egt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(egt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libegt.so is not built (python -m paper_1810_03063_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("egt_build_game", "egt_gradient", "egt_smoothed_br", "egt_step", "egt_saddle_gap",
                     "egt_solve"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1810_03063_amd import egt

    assert sorted(egt.EXPORTED) == declared_functions()


def test_default_opts_and_error_string(lib):
    from paper_1810_03063_amd import egt

    o = egt.make_opts()
    assert o.variant == egt.VARIANTS["AS"] and o.gap_every == 1 and o.tau0 == 0.5
    lib.egt_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.egt_last_error(), bytes)


def test_build_rejects_bad_descriptions_without_touching_the_device(lib):
    """Validation happens on the host before any HIP call."""
    from paper_1810_03063_amd import egt

    d = egt.GameDesc()
    d.n_hands = 0
    h = ctypes.c_void_p()
    rc = egt._build_game(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == -1 and h.value is None
    assert b"n_hands" in egt._last_error()
