"""Seeded synthetic circuit generators.

This module only builds circuit *text*.  It holds none of the simulation
arithmetic: no tableau, no random draws of faults, no thresholds.  Both the
sampling library and the CPU oracle read the text it writes, each with a
parser of its own.
"""

from .circuits import (  # noqa: F401
    Circuit,
    bell_example,
    fig1_example,
    repetition_memory,
    surface_memory,
    random_clifford_circuit,
    random_layered_circuit,
    batched_mix,
    serving_pool,
    format_prob,
)
