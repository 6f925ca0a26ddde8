"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds only random draws and bookkeeping (which gate goes where,
which bits are fixed, which random complex numbers fill a tensor).  It holds
none of the method's arithmetic: no gate matrices, no contraction, no
amplitude computation.  Both ``oracle/`` and ``paper_2005_06787_amd/`` may
import it; neither imports the other.
"""

from .circuits import (  # noqa: F401
    GATE_1Q_NAMES,
    PATTERN_SEQUENCE,
    coupler_pattern,
    grid_sites,
    make_circuit,
)
from .tensors import (  # noqa: F401
    random_bitstrings,
    random_isolated_stem,
    split_open_prefix,
)
