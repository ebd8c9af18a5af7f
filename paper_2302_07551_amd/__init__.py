"""Block staircase-splitting solver for Markov chain stationary vectors on
MI355X: the HIP library libstc.so (built by build.py) and its binding."""
from . import stc  # noqa: F401
from .stc import Batch, Prepared, Solver, StcError, load_library  # noqa: F401
