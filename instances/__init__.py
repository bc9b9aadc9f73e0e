"""Seeded synthetic river-endgame instances.

This package holds input data only: decks, boards, hand lists, hand
strengths, belief vectors and betting parameters.  It contains none of the
solver's arithmetic (no payoffs, no betting-tree enumeration, no strategy
math), so both the CPU oracle and the GPU path may consume its output.
"""
from .endgames import (  # noqa: F401
    CONFIGS,
    LIBRATUS_RIVER,
    BetAbstraction,
    Instance,
    kuhn,
    make_instance,
    micro,
    river,
)
