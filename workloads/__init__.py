"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This package only *describes* inputs: ring lattices as lists of element
records and Gaussian bunches drawn from a counter-based generator.  It holds
none of the tracking arithmetic (no orbit maps, no spin precession), so the
CPU oracle and the GPU path can both consume its output without sharing any
of the method's code.
"""

from .lattice import (  # noqa: F401
    KINDS, METHODS, Element, small_ring, rhic_like_ring, uniform_bend_ring,
    lattice_summary, element_table,
)
from .bunch import (  # noqa: F401
    Beam, gaussian_bunch, widened_bunch, energy_scan_gammas, energy_scan_bunches,
)
