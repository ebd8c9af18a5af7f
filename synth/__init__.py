"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package builds block-banded Markov generators, generators of any block
pattern (CSR) and start vectors.  It holds
none of the staircase method's arithmetic: only random draws, masks, and the
generator's defining convention that each row of Q sums to zero.
"""
from .chains import (  # noqa: F401
    BlockGenerator,
    qbd,
    banded,
    skip_free,
    birth_death,
    planted_reversible,
    served_stream,
    positive_start,
    config_seed,
)
from .general import (  # noqa: F401
    SparseGenerator,
    equal_levels,
    mutual_exclusion,
    mutual_exclusion_pi,
    mutual_exclusion_states,
    localized,
    hessenberg_mmatrix,
    with_levels,
    banded_random,
    upper_hessenberg,
)
