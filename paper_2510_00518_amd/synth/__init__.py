"""Seeded synthetic inputs for the scattering-rate path.

This module produces inputs only (cells, harmonic modes, force-constant tables,
irreducible q1 sets).  It holds none of the scattering-rate arithmetic and is
the one piece shared by the HIP path and the oracle.
"""
from .cells import Cell, diamond_conventional, diamond_primitive, neighbour_shells  # noqa: F401
from .configs import (ADAPTIVE_FACTOR, NSIGMA, OMEGA_FLOOR, SEED, SIGMA, SIGMA_FLOOR,  # noqa: F401
                      adaptive_broadening, make_config, row_modes, small_config)
from .harmonic import mesh_coords, mesh_index, phonons, spring_fc2  # noqa: F401
from .ifc import build_ifc  # noqa: F401
from .qsym import irreducible_q  # noqa: F401
