"""CPU FP64 oracle for the excessive gap technique on poker river endgames
and on general extensive-form games in sequence form.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.  It shares
no code with the HIP implementation; the only common input is the seeded
instance generator in ``instances/``.
"""
from .game import Game  # noqa: F401,E402
from .problem import Problem  # noqa: F401,E402
from .egt import EGT, Trace, iterate, solve  # noqa: F401,E402
from .cfr import Cfr, CfrTrace, solve_cfr  # noqa: F401,E402
from .fom import ChambollePock, MirrorProx, bregman_prox, run_fom, theory_step  # noqa: F401,E402
from .general import GeneralProblem, build_treeplex  # noqa: F401,E402
